// Near field P2P (Sec. 3.1, Sec. 3.6) of the regularised Biot-Savart law and
// the stretching term, Eqs. (1)-(3).  The tree path writes the near-field
// results in sorted order and a finalize kernel adds the far field and
// scatters to the caller's order (the near field runs concurrently with the
// far field on a second stream); the float64 form and the direct mode finish
// in the P2P kernel itself.
//
// Work item: one wave64 per block of <= 64 targets (one target per lane) of a
// leaf; the wave walks the leaf's P2P list.  Source particles are the same
// for every lane at a given step, so their records are read with scalar
// loads and enter the vector ALU as scalar operands: no LDS staging and no
// cross-lane traffic in the pair loop.  Per-target sums are accumulated per
// source leaf and then added to the running total (blocked summation, with an
// optional compensated add).
//
// Per pair, with r = x_i - x_j, s = |r| / (sqrt 2 sigma), x = s^2, and
// alpha~ = alpha/(4 pi) stored in the records:
//   q alpha_j       = F alpha~_j,        F = P(3/2, x) / rho^3
//   (q'/rho) alpha_j = -3 H alpha~_j,    H = P(5/2, x) / rho^5
// where P(a, x) is the regularised lower incomplete gamma function: P(3/2, x)
// is the cutoff g of Eq. (2), and P(5/2, x) = g - 4 s^3 e^{-x} / (3 sqrt pi).
//   u_i       += F (alpha~_j x r)
//   A_i       += F alpha~_j                     (alpha_i x A_i = sum q alpha_i x alpha_j)
//   T_i       += H (alpha_i . (alpha~_j x r)) r  (transpose reading of Eq. (3))
//   dalpha_i   = alpha_i x A_i - 3 T_i
// Three forms of the cutoff, chosen per source leaf from the leaf boxes:
//   full : some pair may have s < 1: Kummer series for s < 1, erfc form else;
//   mid  : every pair has s >= 1: 1 - P = e^{-x} (erfcx(s) + ...), no branch;
//   sing : the float32 cutoff is 1 for every pair (s >= 5.1): F = rho^-3.
#include "ctx.h"
#include "cutoff_fits.h"

namespace vfmm {

struct P2PConst {
    float kE;        // -log2(e) / (2 sigma^2): e^{-x} = exp2(r2 kE)
    float kS;        // 2 c / sqrt(pi), c = 1/(sqrt 2 sigma): (2/sqrt pi) s = rho kS
    float kU;        // 1/c: 1/s = rinv kU
    float t5;        // 2 c^2 / 3: (4/(3 sqrt pi)) s^3 = r2 t5 * rho kS
    float K3;        // c^3 4/(3 sqrt pi): P(3/2,x)/rho^3 -> K3 at rho = 0
    float r2_small;  // 2 sigma^2 (s < 1 <=> r2 < r2_small)
    float q[VFMM_M2_DEG + 1];  // c^5 8/(15 sqrt pi) * M2 coefficients, in powers of r2
};

struct P2PArgs {
    const float4 *__restrict__ rec;
    const int4 *__restrict__ blocks;
    const int4 *__restrict__ ent;
    int nblocks;
    int B;
    float len;
    const float *__restrict__ far_u;
    const float *__restrict__ far_da;
    int64_t n;
    const int *__restrict__ perm;
    const Bounds *__restrict__ bounds;
    float inv3V;
    int surface;
    float *ux, *uy, *uz, *dax, *day, *daz;
    float *near;  // non-null: write u and dalpha in sorted order to near[6][n] instead of finishing
};

struct Acc9 {
    float u0, u1, u2, a0, a1, a2, t0, t1, t2;
};

template <int V, int SCHEME>
__device__ __forceinline__ void pair(const P2PConst &k, float xi, float yi, float zi, float ai0, float ai1, float ai2,
                                     float4 sp, float4 sa, Acc9 &p) {
    const float dx = xi - sp.x, dy = yi - sp.y, dz = zi - sp.z;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float rinv2 = rinv * rinv;
    const float rinv3 = rinv2 * rinv;
    const float h5 = rinv3 * rinv2;
    float F = rinv3, H = h5;
    if (V <= 1) {
        const float E = __builtin_amdgcn_exp2f(r2 * k.kE);
        const float rho = r2 * rinv;
        const float ks = rho * k.kS;
        const float u = rinv * k.kU;
        float pe = VFMM_ERFCX_C[VFMM_ERFCX_DEG];
#pragma unroll
        for (int i = VFMM_ERFCX_DEG - 1; i >= 0; --i) pe = fmaf(pe, u, VFMM_ERFCX_C[i]);
        const float w3 = fmaf(u, pe, ks);                // erfcx(s) + (2/sqrt pi) s
        const float g = fmaf(-E, w3, 1.0f);              // P(3/2, x)
        const float w5 = fmaf(r2 * k.t5, ks, w3);        // + (4/(3 sqrt pi)) s^3
        const float g5 = fmaf(-E, w5, 1.0f);             // P(5/2, x)
        F = g * rinv3;
        H = g5 * h5;
        if (V == 0) {
            if (__any(r2 < k.r2_small)) {
                float q2 = k.q[VFMM_M2_DEG];
#pragma unroll
                for (int i = VFMM_M2_DEG - 1; i >= 0; --i) q2 = fmaf(q2, r2, k.q[i]);
                const float Fs = E * fmaf(r2, q2, k.K3);  // e^{-x} K3 1F1(1;5/2;x)
                const float Hs = E * q2;                  // e^{-x} K5 1F1(1;7/2;x)
                const bool sm = r2 < k.r2_small;
                F = sm ? Fs : F;
                H = sm ? Hs : H;
            }
        }
    }
    // alpha~_j x r
    const float c0 = sa.y * dz - sa.z * dy;
    const float c1 = sa.z * dx - sa.x * dz;
    const float c2 = sa.x * dy - sa.y * dx;
    p.u0 = fmaf(F, c0, p.u0);
    p.u1 = fmaf(F, c1, p.u1);
    p.u2 = fmaf(F, c2, p.u2);
    p.a0 = fmaf(F, sa.x, p.a0);
    p.a1 = fmaf(F, sa.y, p.a1);
    p.a2 = fmaf(F, sa.z, p.a2);
    if (SCHEME == VFMM_SCHEME_TRANSPOSE) {
        const float d = fmaf(ai0, c0, fmaf(ai1, c1, ai2 * c2));
        const float hd = H * d;
        p.t0 = fmaf(hd, dx, p.t0);
        p.t1 = fmaf(hd, dy, p.t1);
        p.t2 = fmaf(hd, dz, p.t2);
    } else {
        const float d = fmaf(ai0, dx, fmaf(ai1, dy, ai2 * dz));
        const float hd = H * d;
        p.t0 = fmaf(hd, c0, p.t0);
        p.t1 = fmaf(hd, c1, p.t1);
        p.t2 = fmaf(hd, c2, p.t2);
    }
}

template <int V, int SCHEME>
__device__ __forceinline__ void leaf_loop(const P2PConst &k, const float4 *__restrict__ rec, int s0, int cnt,
                                          float xi, float yi, float zi, float ai0, float ai1, float ai2, Acc9 &p) {
    const float4 *src = rec + 2 * (size_t)s0;
    int j = 0;
    for (; j + 2 <= cnt; j += 2) {
        const float4 sp0 = src[2 * j], sa0 = src[2 * j + 1];
        const float4 sp1 = src[2 * j + 2], sa1 = src[2 * j + 3];
        pair<V, SCHEME>(k, xi, yi, zi, ai0, ai1, ai2, sp0, sa0, p);
        pair<V, SCHEME>(k, xi, yi, zi, ai0, ai1, ai2, sp1, sa1, p);
    }
    if (j < cnt) pair<V, SCHEME>(k, xi, yi, zi, ai0, ai1, ai2, src[2 * j], src[2 * j + 1], p);
}

__device__ __forceinline__ void kahan_add(float &s, float &c, float v) {
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Blocks of few targets split the wave into SPLIT lane groups of 64/SPLIT
// lanes that each hold every target of the block and take every SPLIT-th
// source (the group's source is selected per lane from the SPLIT records
// fetched together); the groups' sums are added at the end.  A missing last
// source gets zero strength, which contributes exactly zero.
template <int V, int SCHEME, int SPLIT>
__device__ __forceinline__ void leaf_loop_split(const P2PConst &k, const float4 *__restrict__ rec, int s0, int cnt,
                                                int grp, float xi, float yi, float zi, float ai0, float ai1,
                                                float ai2, Acc9 &p) {
    const float4 *src = rec + 2 * (size_t)s0;
    for (int j = 0; j < cnt; j += SPLIT) {
        float4 mp = src[2 * j], ma = src[2 * j + 1];
#pragma unroll
        for (int t = 1; t < SPLIT; ++t) {
            const int jj = min(j + t, cnt - 1);
            const float4 sp = src[2 * jj];
            float4 sa = src[2 * jj + 1];
            if (j + t >= cnt) sa = make_float4(0.f, 0.f, 0.f, 0.f);
            if (grp == t) {
                mp = sp;
                ma = sa;
            }
        }
        pair<V, SCHEME>(k, xi, yi, zi, ai0, ai1, ai2, mp, ma, p);
    }
}

template <int SCHEME, bool KAHAN, int SPLIT>
__device__ __forceinline__ void p2p_block(const P2PConst &k, const P2PArgs &A, int t0, int tc, int l0, int lc) {
    const int lane = threadIdx.x & 63;
    constexpr int GL = 64 / SPLIT;  // lanes per group
    const int tl = lane % GL, grp = lane / GL;
    const bool valid = tl < tc;
    const int i = t0 + (valid ? tl : 0);
    const float4 xp = A.rec[2 * (size_t)i];
    const float4 xa = A.rec[2 * (size_t)i + 1];
    const float fp = 12.566370614359172f;  // 4 pi: stored strengths are alpha/(4 pi)
    const float ai0 = xa.x * fp, ai1 = xa.y * fp, ai2 = xa.z * fp;
    float S[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    float Cc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int W = 2 * A.B + 1;
    for (int e = 0; e < lc; ++e) {
        const int4 en = A.ent[l0 + e];
        const int s0 = __builtin_amdgcn_readfirstlane(en.x);
        const int sc = __builtin_amdgcn_readfirstlane(en.y);
        const int img = __builtin_amdgcn_readfirstlane(en.z);
        const int var = __builtin_amdgcn_readfirstlane(en.w);
        const float shx = (float)(img % W - A.B) * A.len;
        const float shy = (float)((img / W) % W - A.B) * A.len;
        const float shz = (float)(img / (W * W) - A.B) * A.len;
        const float xi = xp.x - shx, yi = xp.y - shy, zi = xp.z - shz;
        Acc9 p = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (SPLIT == 1) {
            if (var == 1)
                leaf_loop<1, SCHEME>(k, A.rec, s0, sc, xi, yi, zi, ai0, ai1, ai2, p);
            else if (var == 0)
                leaf_loop<0, SCHEME>(k, A.rec, s0, sc, xi, yi, zi, ai0, ai1, ai2, p);
            else
                leaf_loop<2, SCHEME>(k, A.rec, s0, sc, xi, yi, zi, ai0, ai1, ai2, p);
        } else {
            if (var == 1)
                leaf_loop_split<1, SCHEME, SPLIT>(k, A.rec, s0, sc, grp, xi, yi, zi, ai0, ai1, ai2, p);
            else if (var == 0)
                leaf_loop_split<0, SCHEME, SPLIT>(k, A.rec, s0, sc, grp, xi, yi, zi, ai0, ai1, ai2, p);
            else
                leaf_loop_split<2, SCHEME, SPLIT>(k, A.rec, s0, sc, grp, xi, yi, zi, ai0, ai1, ai2, p);
        }
        const float pv[9] = {p.u0, p.u1, p.u2, p.a0, p.a1, p.a2, p.t0, p.t1, p.t2};
        if (KAHAN) {
#pragma unroll
            for (int q = 0; q < 9; ++q) kahan_add(S[q], Cc[q], pv[q]);
        } else {
#pragma unroll
            for (int q = 0; q < 9; ++q) S[q] += pv[q];
        }
    }
    if (SPLIT > 1) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            if (KAHAN) S[q] -= Cc[q];
            S[q] += __shfl_xor(S[q], 32, 64);
            if (SPLIT > 2) S[q] += __shfl_xor(S[q], 16, 64);
        }
    }
    if (!valid || grp != 0) return;
    // dalpha = alpha_i x A - 3 T (transpose) or A x alpha_i - 3 T (classical)
    float d0, d1, d2;
    if (SCHEME == VFMM_SCHEME_TRANSPOSE) {
        d0 = ai1 * S[5] - ai2 * S[4];
        d1 = ai2 * S[3] - ai0 * S[5];
        d2 = ai0 * S[4] - ai1 * S[3];
    } else {
        d0 = S[4] * ai2 - S[5] * ai1;
        d1 = S[5] * ai0 - S[3] * ai2;
        d2 = S[3] * ai1 - S[4] * ai0;
    }
    d0 = fmaf(-3.0f, S[6], d0);
    d1 = fmaf(-3.0f, S[7], d1);
    d2 = fmaf(-3.0f, S[8], d2);
    float u0 = S[0], u1 = S[1], u2 = S[2];
    if (A.near) {
        A.near[i] = u0;
        A.near[A.n + i] = u1;
        A.near[2 * A.n + i] = u2;
        A.near[3 * A.n + i] = d0;
        A.near[4 * A.n + i] = d1;
        A.near[5 * A.n + i] = d2;
        return;
    }
    if (A.far_u) {
        u0 += A.far_u[i];
        u1 += A.far_u[A.n + i];
        u2 += A.far_u[2 * A.n + i];
        d0 += A.far_da[i];
        d1 += A.far_da[A.n + i];
        d2 += A.far_da[2 * A.n + i];
    }
    if (A.surface) {
        u0 -= (float)(A.bounds->sum_xa[0]) * A.inv3V;
        u1 -= (float)(A.bounds->sum_xa[1]) * A.inv3V;
        u2 -= (float)(A.bounds->sum_xa[2]) * A.inv3V;
    }
    const int o = A.perm[i];
    A.ux[o] = u0;
    A.uy[o] = u1;
    A.uz[o] = u2;
    A.dax[o] = d0;
    A.day[o] = d1;
    A.daz[o] = d2;
}

template <int SCHEME, bool KAHAN>
__global__ __launch_bounds__(256) void k_p2p(P2PConst k, P2PArgs A) {
    const int b = xcd_logical(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (b >= A.nblocks) return;
    const int4 blk = A.blocks[b];
    const int t0 = __builtin_amdgcn_readfirstlane(blk.x);
    const int tc = __builtin_amdgcn_readfirstlane(blk.y);
    const int l0 = __builtin_amdgcn_readfirstlane(blk.z);
    const int lc = __builtin_amdgcn_readfirstlane(blk.w);
    if (tc <= 16)
        p2p_block<SCHEME, KAHAN, 4>(k, A, t0, tc, l0, lc);
    else if (tc <= 32)
        p2p_block<SCHEME, KAHAN, 2>(k, A, t0, tc, l0, lc);
    else
        p2p_block<SCHEME, KAHAN, 1>(k, A, t0, tc, l0, lc);
}

// ---------------------------------------------------------------------------
// Float64 reference form: the same work blocks and lists, one lane per
// target, every quantity in double and the cutoff always in its full form:
//   F = P(3/2, x)/rho^3,  H = P(5/2, x)/rho^5,  x = c^2 rho^2,  c = 1/(sqrt 2 sigma).
// For x < 2 the power series of the lower incomplete gamma function,
//   P(a, x) = x^a e^{-x} sum_k x^k / Gamma(a + k + 1),
// divided by rho^{2a}, gives F and H without cancellation (finite at rho = 0);
// for x >= 2, 1 - P(3/2, x) = erfc(s) + (2/sqrt pi) s e^{-x}, s = sqrt x, and
// P(5/2, x) = P(3/2, x) - (4/(3 sqrt pi)) s^3 e^{-x}.
// ---------------------------------------------------------------------------
struct P2P64Args {
    const double4 *__restrict__ rec;
    const int4 *__restrict__ blocks;
    const int4 *__restrict__ ent;
    int nblocks;
    int B;
    double len, c, c2;
    const double *__restrict__ far_u;
    const double *__restrict__ far_da;
    int64_t n;
    const int *__restrict__ perm;
    const Bounds *__restrict__ bounds;
    double inv3V;
    int surface;
    float *ux, *uy, *uz, *dax, *day, *daz;
};

__device__ inline void cutoff64(double r2, double c, double c2, double &F, double &H) {
    const double x = c2 * r2;
    const double isqpi = 0.56418958354775628695;  // 1/sqrt(pi)
    const double e = exp(-x);
    if (x < 2.0) {
        double t = 4.0 / 3.0 * isqpi, u = 8.0 / 15.0 * isqpi;  // 1/Gamma(5/2), 1/Gamma(7/2)
        double st = t, su = u;
        for (int k = 1; k < 60; ++k) {
            t *= x / (k + 1.5);
            u *= x / (k + 2.5);
            st += t;
            su += u;
            if (t < 1e-18 * st) break;
        }
        F = c * c2 * e * st;
        H = c2 * c2 * c * e * su;
    } else {
        const double sx = sqrt(x);
        const double rho = sqrt(r2);
        const double q3 = erfc(sx) + 2.0 * isqpi * sx * e;
        const double g = 1.0 - q3;
        const double g5 = g - 4.0 / 3.0 * isqpi * sx * x * e;
        const double ir = 1.0 / rho, ir2 = ir * ir;
        F = g * ir * ir2;
        H = g5 * ir * ir2 * ir2;
    }
}

template <int SCHEME>
__global__ __launch_bounds__(64) void k_p2p64(P2P64Args A) {
    const int lane = threadIdx.x;
    const int b = blockIdx.x;
    if (b >= A.nblocks) return;
    const int4 blk = A.blocks[b];
    const bool valid = lane < blk.y;
    const int i = blk.x + (valid ? lane : 0);
    const double4 xp = A.rec[2 * (size_t)i];
    const double4 xa = A.rec[2 * (size_t)i + 1];
    const double fp = 12.566370614359172954;  // 4 pi
    const double ai0 = xa.x * fp, ai1 = xa.y * fp, ai2 = xa.z * fp;
    double S[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int W = 2 * A.B + 1;
    for (int e = 0; e < blk.w; ++e) {
        const int4 en = A.ent[blk.z + e];
        const double xi = xp.x - (double)(en.z % W - A.B) * A.len;
        const double yi = xp.y - (double)((en.z / W) % W - A.B) * A.len;
        const double zi = xp.z - (double)(en.z / (W * W) - A.B) * A.len;
        for (int j = en.x; j < en.x + en.y; ++j) {
            const double4 sp = A.rec[2 * (size_t)j], sa = A.rec[2 * (size_t)j + 1];
            const double dx = xi - sp.x, dy = yi - sp.y, dz = zi - sp.z;
            double F, H;
            cutoff64(dx * dx + dy * dy + dz * dz, A.c, A.c2, F, H);
            const double c0 = sa.y * dz - sa.z * dy;
            const double c1 = sa.z * dx - sa.x * dz;
            const double c2 = sa.x * dy - sa.y * dx;
            S[0] += F * c0;
            S[1] += F * c1;
            S[2] += F * c2;
            S[3] += F * sa.x;
            S[4] += F * sa.y;
            S[5] += F * sa.z;
            if (SCHEME == VFMM_SCHEME_TRANSPOSE) {
                const double hd = H * (ai0 * c0 + ai1 * c1 + ai2 * c2);
                S[6] += hd * dx;
                S[7] += hd * dy;
                S[8] += hd * dz;
            } else {
                const double hd = H * (ai0 * dx + ai1 * dy + ai2 * dz);
                S[6] += hd * c0;
                S[7] += hd * c1;
                S[8] += hd * c2;
            }
        }
    }
    if (!valid) return;
    double d0, d1, d2;
    if (SCHEME == VFMM_SCHEME_TRANSPOSE) {
        d0 = ai1 * S[5] - ai2 * S[4];
        d1 = ai2 * S[3] - ai0 * S[5];
        d2 = ai0 * S[4] - ai1 * S[3];
    } else {
        d0 = S[4] * ai2 - S[5] * ai1;
        d1 = S[5] * ai0 - S[3] * ai2;
        d2 = S[3] * ai1 - S[4] * ai0;
    }
    d0 -= 3.0 * S[6];
    d1 -= 3.0 * S[7];
    d2 -= 3.0 * S[8];
    double u0 = S[0], u1 = S[1], u2 = S[2];
    if (A.far_u) {
        u0 += A.far_u[i];
        u1 += A.far_u[A.n + i];
        u2 += A.far_u[2 * A.n + i];
        d0 += A.far_da[i];
        d1 += A.far_da[A.n + i];
        d2 += A.far_da[2 * A.n + i];
    }
    if (A.surface) {
        u0 -= A.bounds->sum_xa[0] * A.inv3V;
        u1 -= A.bounds->sum_xa[1] * A.inv3V;
        u2 -= A.bounds->sum_xa[2] * A.inv3V;
    }
    const int o = A.perm[i];
    A.ux[o] = (float)u0;
    A.uy[o] = (float)u1;
    A.uz[o] = (float)u2;
    A.dax[o] = (float)d0;
    A.day[o] = (float)d1;
    A.daz[o] = (float)d2;
}

static void launch_p2p64(Ctx &c, P2P64Args A) {
    if (A.nblocks == 0) return;
    A.c = 1.0 / (std::sqrt(2.0) * (double)c.sigma_uniform);
    A.c2 = A.c * A.c;
    if (c.prm.scheme == VFMM_SCHEME_TRANSPOSE)
        k_p2p64<VFMM_SCHEME_TRANSPOSE><<<A.nblocks, 64, 0, c.stream>>>(A);
    else
        k_p2p64<VFMM_SCHEME_CLASSICAL><<<A.nblocks, 64, 0, c.stream>>>(A);
    VFMM_LAUNCH_CHECK();
}

static P2PConst make_const(double sigma) {
    P2PConst k{};
    const double c = 1.0 / (std::sqrt(2.0) * sigma);
    const double c2 = c * c;
    const double sqpi = std::sqrt(M_PI);
    k.kE = (float)(-c2 / std::log(2.0));
    k.kS = (float)(2.0 * c / sqpi);
    k.kU = (float)(1.0 / c);
    k.t5 = (float)(2.0 * c2 / 3.0);
    k.K3 = (float)(c * c2 * 4.0 / (3.0 * sqpi));
    k.r2_small = (float)(VFMM_CUTOFF_XSPLIT / c2);
    const double K5 = c2 * c2 * c * 8.0 / (15.0 * sqpi);
    double pw = 1.0;
    for (int i = 0; i <= VFMM_M2_DEG; ++i) {
        k.q[i] = (float)(K5 * (double)VFMM_M2_C[i] * pw);
        pw *= c2;
    }
    return k;
}

template <int SCHEME, bool KAHAN>
static void launch_p2p(const P2PConst &k, const P2PArgs &A, hipStream_t s) {
    if (A.nblocks == 0) return;
    k_p2p<SCHEME, KAHAN><<<xcd_grid(cdiv(A.nblocks, 4)), 256, 0, s>>>(k, A);
    VFMM_LAUNCH_CHECK();
}

static void dispatch_p2p(Ctx &c, const P2PConst &k, const P2PArgs &A, hipStream_t s) {
    const bool kah = c.prm.kahan != 0 || c.prm.precision == VFMM_PRECISION_MIXED;
    if (c.prm.scheme == VFMM_SCHEME_TRANSPOSE) {
        if (kah) launch_p2p<VFMM_SCHEME_TRANSPOSE, true>(k, A, s);
        else launch_p2p<VFMM_SCHEME_TRANSPOSE, false>(k, A, s);
    } else {
        if (kah) launch_p2p<VFMM_SCHEME_CLASSICAL, true>(k, A, s);
        else launch_p2p<VFMM_SCHEME_CLASSICAL, false>(k, A, s);
    }
}

static P2PArgs tree_args(Ctx &c) {
    P2PArgs A{};
    A.rec = c.rec.as<float4>();
    A.blocks = c.blocks.as<int4>();
    A.ent = c.p2p_ent.as<int4>();
    A.nblocks = c.n_blocks;
    A.B = c.img_B;
    A.len = c.prm.periodic ? (float)c.prm.box_len : 0.f;
    A.n = c.n;
    A.perm = c.perm.as<int>();
    A.bounds = c.bres.as<Bounds>();
    A.surface = (c.prm.periodic && c.prm.zero_mean) ? 1 : 0;
    A.inv3V = c.prm.periodic ? (float)(1.0 / (3.0 * c.prm.box_len * c.prm.box_len * c.prm.box_len)) : 0.f;
    return A;
}

// Near field alone, on stream s, into c.near (sorted order); the far field
// runs meanwhile on the library stream and finalize_near_far adds the two.
void p2p_near(Ctx &c, hipStream_t s) {
    const P2PConst k = make_const(c.sigma_uniform);
    c.near.ensure(sizeof(float) * 6 * (size_t)c.n);
    P2PArgs A = tree_args(c);
    A.near = c.near.as<float>();
    c.record(2 * PH_P2P, s);
    dispatch_p2p(c, k, A, s);
    c.record(2 * PH_P2P + 1, s);
}

// out[perm[i]] = near[i] + far[i] (- the zero-mean surface term for u)
__global__ __launch_bounds__(256) void k_finalize(P2PArgs A, const float *__restrict__ near) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= A.n) return;
    const int64_t n = A.n;
    float u0 = near[i] + A.far_u[i], u1 = near[n + i] + A.far_u[n + i], u2 = near[2 * n + i] + A.far_u[2 * n + i];
    const float d0 = near[3 * n + i] + A.far_da[i], d1 = near[4 * n + i] + A.far_da[n + i],
                d2 = near[5 * n + i] + A.far_da[2 * n + i];
    if (A.surface) {
        u0 -= (float)(A.bounds->sum_xa[0]) * A.inv3V;
        u1 -= (float)(A.bounds->sum_xa[1]) * A.inv3V;
        u2 -= (float)(A.bounds->sum_xa[2]) * A.inv3V;
    }
    const int o = A.perm[i];
    A.ux[o] = u0;
    A.uy[o] = u1;
    A.uz[o] = u2;
    A.dax[o] = d0;
    A.day[o] = d1;
    A.daz[o] = d2;
}

void finalize_near_far(Ctx &c, float *ux, float *uy, float *uz, float *dax, float *day, float *daz) {
    P2PArgs A = tree_args(c);
    A.far_u = c.far_u.as<float>();
    A.far_da = c.far_da.as<float>();
    A.ux = ux; A.uy = uy; A.uz = uz; A.dax = dax; A.day = day; A.daz = daz;
    if (c.n == 0) return;
    k_finalize<<<cdiv(c.n, 256), 256, 0, c.stream>>>(A, c.near.as<float>());
    VFMM_LAUNCH_CHECK();
}

void p2p_and_finalize(Ctx &c, float *ux, float *uy, float *uz, float *dax, float *day, float *daz) {
    if (c.prm.precision == VFMM_PRECISION_FP64) {
        P2P64Args A{};
        A.rec = c.rec64.as<double4>();
        A.blocks = c.blocks.as<int4>();
        A.ent = c.p2p_ent.as<int4>();
        A.nblocks = c.n_blocks;
        A.B = c.img_B;
        A.len = c.prm.periodic ? c.prm.box_len : 0.0;
        A.far_u = c.far_u.as<double>();
        A.far_da = c.far_da.as<double>();
        A.n = c.n;
        A.perm = c.perm.as<int>();
        A.bounds = c.bres.as<Bounds>();
        A.surface = (c.prm.periodic && c.prm.zero_mean) ? 1 : 0;
        A.inv3V = c.prm.periodic ? 1.0 / (3.0 * c.prm.box_len * c.prm.box_len * c.prm.box_len) : 0.0;
        A.ux = ux; A.uy = uy; A.uz = uz; A.dax = dax; A.day = day; A.daz = daz;
        c.record(2 * PH_P2P);
        launch_p2p64(c, A);
        c.record(2 * PH_P2P + 1);
        return;
    }
    const P2PConst k = make_const(c.sigma_uniform);
    P2PArgs A{};
    A.rec = c.rec.as<float4>();
    A.blocks = c.blocks.as<int4>();
    A.ent = c.p2p_ent.as<int4>();
    A.nblocks = c.n_blocks;
    A.B = c.img_B;
    A.len = c.prm.periodic ? (float)c.prm.box_len : 0.f;
    A.far_u = c.far_u.as<float>();
    A.far_da = c.far_da.as<float>();
    A.n = c.n;
    A.perm = c.perm.as<int>();
    A.bounds = c.bres.as<Bounds>();
    A.surface = (c.prm.periodic && c.prm.zero_mean) ? 1 : 0;
    A.inv3V = c.prm.periodic ? (float)(1.0 / (3.0 * c.prm.box_len * c.prm.box_len * c.prm.box_len)) : 0.f;
    A.ux = ux; A.uy = uy; A.uz = uz; A.dax = dax; A.day = day; A.daz = daz;
    c.record(2 * PH_P2P);
    dispatch_p2p(c, k, A, c.stream);
    c.record(2 * PH_P2P + 1);
}

// ---------------------------------------------------------------------------
// Direct mode: every target block against all N sources (entries of 64
// sources, full cutoff form), in the caller's order, no tree, no far field.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_direct_setup64(int64_t n, const float *x, const float *y, const float *z,
                                                        const float *ax, const float *ay, const float *az,
                                                        const float *s, double4 *rec, int *perm) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double k = 0.079577471545947667884;  // 1/(4 pi)
    rec[2 * i] = make_double4(x[i], y[i], z[i], s[i]);
    rec[2 * i + 1] = make_double4((double)ax[i] * k, (double)ay[i] * k, (double)az[i] * k, 0.0);
    perm[i] = (int)i;
}

__global__ __launch_bounds__(256) void k_direct_setup(int64_t n, const float *x, const float *y, const float *z,
                                                      const float *ax, const float *ay, const float *az,
                                                      const float *s, float4 *rec, int *perm) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float k = 0.0795774715459476679f;  // 1/(4 pi)
    rec[2 * i] = make_float4(x[i], y[i], z[i], s[i]);
    rec[2 * i + 1] = make_float4(ax[i] * k, ay[i] * k, az[i] * k, 0.f);
    perm[i] = (int)i;
}

// Sources split into entries of 64 so that per-entry partial sums are blocked
// exactly as in tree mode.
__global__ __launch_bounds__(256) void k_direct_blocks(int64_t n, int nb, int4 *blocks, int4 *ent) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b < nb) {
        const int cnt = (int)min<int64_t>(64, n - (int64_t)b * 64);
        blocks[b] = make_int4(b * 64, cnt, 0, nb);
        ent[b] = make_int4(b * 64, cnt, 0, 0);
    }
}

void direct_all_pairs(Ctx &c, const float *x, const float *y, const float *z, const float *ax, const float *ay,
                      const float *az, const float *sigma, float *ux, float *uy, float *uz, float *dax, float *day,
                      float *daz) {
    const int64_t n = c.n;
    c.rec.ensure(sizeof(float4) * 2 * n);
    c.perm.ensure(sizeof(int) * n);
    const int nb = (int)cdiv(n, 64);
    c.blocks.ensure(sizeof(int4) * nb);
    c.p2p_ent.ensure(sizeof(int4) * nb);
    k_direct_setup<<<cdiv(n, 256), 256, 0, c.stream>>>(n, x, y, z, ax, ay, az, sigma, c.rec.as<float4>(),
                                                        c.perm.as<int>());
    VFMM_LAUNCH_CHECK();
    k_direct_blocks<<<cdiv(nb, 256), 256, 0, c.stream>>>(n, nb, c.blocks.as<int4>(), c.p2p_ent.as<int4>());
    VFMM_LAUNCH_CHECK();
    c.n_blocks = nb;
    c.p2p_pairs = n * n;
    if (c.prm.precision == VFMM_PRECISION_FP64) {
        c.rec64.ensure(sizeof(double4) * 2 * n);
        k_direct_setup64<<<cdiv(n, 256), 256, 0, c.stream>>>(n, x, y, z, ax, ay, az, sigma, c.rec64.as<double4>(),
                                                              c.perm.as<int>());
        VFMM_LAUNCH_CHECK();
        P2P64Args A{};
        A.rec = c.rec64.as<double4>();
        A.blocks = c.blocks.as<int4>();
        A.ent = c.p2p_ent.as<int4>();
        A.nblocks = nb;
        A.n = n;
        A.perm = c.perm.as<int>();
        A.bounds = c.bres.as<Bounds>();
        A.ux = ux; A.uy = uy; A.uz = uz; A.dax = dax; A.day = day; A.daz = daz;
        c.record(2 * PH_P2P);
        launch_p2p64(c, A);
        c.record(2 * PH_P2P + 1);
        return;
    }
    const P2PConst k = make_const(c.sigma_uniform);
    P2PArgs A{};
    A.rec = c.rec.as<float4>();
    A.blocks = c.blocks.as<int4>();
    A.ent = c.p2p_ent.as<int4>();
    A.nblocks = nb;
    A.B = 0;
    A.len = 0.f;
    A.far_u = nullptr;
    A.far_da = nullptr;
    A.n = n;
    A.perm = c.perm.as<int>();
    A.bounds = c.bres.as<Bounds>();
    A.surface = 0;
    A.ux = ux; A.uy = uy; A.uz = uz; A.dax = dax; A.day = day; A.daz = daz;
    c.n_blocks = nb;
    c.p2p_pairs = n * n;
    c.record(2 * PH_P2P);
    dispatch_p2p(c, k, A, c.stream);
    c.record(2 * PH_P2P + 1);
}

}  // namespace vfmm
