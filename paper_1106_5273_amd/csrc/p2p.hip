// Near field P2P (Sec. 3.1, Sec. 3.6) of the regularised Biot-Savart law and
// the stretching term, Eqs. (1)-(3).  The P2P kernel writes its results in
// sorted order, one buffer per part of the lists (below), and a finalize
// kernel adds the parts and the far field and scatters to the caller's order.
//
// Work item: one wave64 per part (a quarter) of the P2P list of a block of
// <= 64 targets of a leaf (one target per lane).  Source particles are the
// same for every lane at a given step, so their records are read with scalar
// loads and enter the vector ALU as scalar operands: no LDS staging and no
// cross-lane traffic in the pair loop.  Per-target sums are accumulated per
// source leaf and then added to the running total (blocked summation, with an
// optional compensated add).
//
// Scaled, leaf-local coordinates.  With c = 1/(sqrt 2 sigma) and
// lambda = log2 e, lengths are multiplied by kappa = c sqrt(lambda), so that
// e^{-x} = 2^{-r'^2} for x = (rho/(sqrt 2 sigma))^2 and the Gaussian needs no
// argument scaling.  Each particle's record holds its offset from the centre
// of its own leaf, delta' = kappa (x - c_leaf), and each list entry holds the
// offset between the two leaves, D' = kappa (c_t - c_s - image shift), so
// that r' = (delta'_i + D') - delta'_j = y_i - delta'_j is formed from small
// numbers.  Strengths are stored as ah = kappa^3 alpha/(4 pi), together with
// bh = ah x delta'.
//
// Per pair, with E = 2^{-r2'}, rho' = |r'| and a = (2/sqrt pi)/sqrt(lambda):
//   G3 = 1 - a E (rho' + (1/rho') pe(1/rho'))      = P(3/2, x)
//   G5 = G3 - a E b rho'^3,  b = 2/(3 lambda)       = P(5/2, x)
//   Fh = G3 / rho'^3,  Hh = G5 / rho'^5 = (Fh - a b E) / rho'^2
// where pe is the erfcx fit rescaled to 1/rho' and P(a, x) is the regularised
// lower incomplete gamma function (P(3/2, x) is the cutoff g of Eq. (2)).
// Then, in physical units, q alpha_j x r = Fh (ah_j x r') / kappa and
// (q'/rho)(alpha_i . (alpha_j x r)) r = -3 Hh (alpha_i . (ah_j x r')) r', and
//   transpose reading of Eq. (3):
//     Ah += Fh ah_j,  Bh += Fh bh_j,  T += Hh d r',
//     d = alpha_i . (ah_j x r') = ah_j . (y_i x alpha_i) - alpha_i . bh_j,
//     and per source leaf  U += Ah x y_i - Bh  (= sum Fh ah_j x r');
//   classical reading: U += Fh (ah_j x r'), Ah += Fh ah_j,
//     T += Hh (alpha_i . r') (ah_j x r');
//   u_i = U / kappa,  dalpha_i = alpha_i x Ah - 3 T  (or Ah x alpha_i - 3 T).
// Three forms of the cutoff, chosen per source leaf from the leaf boxes:
//   full : some pair may have s < 1: Kummer series for s < 1, the erfcx form else;
//   mid  : every pair has s >= 1: the erfcx form, no branch;
//   sing : the float32 cutoff is 1 for every pair (s >= 5.1): G3 = G5 = 1/a.
// Per-particle cores use unscaled offsets and evaluate the cutoff at
// kappa_j r with each source's kappa_j (see pair()); a list entry's source
// count covers only the sources of a leaf whose target points were moved
// behind them.
#include "ctx.h"
#include "cutoff_fits.h"

namespace vfmm {

// The launch constant that depends on the core: the strengths are
// kappa^3 alpha/(4 pi) and the velocity sum is scaled back by 1/kappa.
struct P2PConst {
    float inv_kappa; // u = U / kappa
};

// Constants of the scaled cutoff (in the scaled units every one is
// independent of sigma; the normalisation a of the cutoff is in them),
// evaluated at compile time (lam = log2 e, a = (2/sqrt pi) sqrt(ln 2)), so
// that the pair loop takes them as instruction literals (v_fmaak_f32 and the
// like) instead of reading them from registers: a constant in a vector
// register can share a register bank with another operand of the same
// instruction, which halves that instruction's issue rate.
//   a, ab      : a and a b, b = 2/(3 lam)
//   K3         : the series form's Fh at r = 0 (times E)
//   r2_small   : s < 1  <=>  r2' < r2_small
//   pe(i)      : erfcx fit in powers of 1/rho', times a
//   q(i)       : series, Hh = E sum q_k r2'^k,  Fh = E (K3 + r2' sum q_k r2'^k)
namespace cutoff_ce {
constexpr double sqrt_newton(double x) {
    double r = x > 1.0 ? x : 1.0;
    for (int i = 0; i < 200; ++i) r = 0.5 * (r + x / r);
    return r;
}
constexpr double LN2 = 0.693147180559945309417232121458;
constexpr double PI = 3.14159265358979323846264338328;
constexpr double LAM = 1.0 / LN2;
constexpr double SQRT_LAM = sqrt_newton(LAM);
constexpr double SQRT_PI = sqrt_newton(PI);
constexpr double lam_pow_half(int k) {  // lam^(k/2)
    double r = 1.0;
    for (int i = 0; i < k / 2; ++i) r *= LAM;
    return (k & 1) ? r * SQRT_LAM : r;
}
constexpr double A = 2.0 / SQRT_PI * sqrt_newton(LN2);
constexpr float a = (float)A;
constexpr float ab = (float)(A * 2.0 / (3.0 * LAM));
constexpr float K3 = (float)(4.0 / (3.0 * SQRT_PI) / lam_pow_half(3));
constexpr float r2_small = (float)((double)VFMM_CUTOFF_XSPLIT * LAM);
constexpr float pe(int i) { return (float)((double)VFMM_ERFCX_C[i] * lam_pow_half(i + 1)); }
constexpr float q(int i) { return (float)(8.0 / (15.0 * SQRT_PI) * (double)VFMM_M2_C[i] / lam_pow_half(5 + 2 * i)); }
}  // namespace cutoff_ce

struct P2PArgs {
    const float4 *__restrict__ rec;  // float4[3n] (uniform cores) or float4[4n] (per-particle cores) records
    const int4 *__restrict__ blocks;
    const int4 *__restrict__ ent;
    const float4 *__restrict__ sh;   // per entry: (D', 0)
    int nblocks;
    const float *__restrict__ far_u;
    const float *__restrict__ far_da;
    int64_t n;
    const int *__restrict__ perm;
    const Bounds *__restrict__ bounds;
    float inv3V;
    int surface;
    float *ux, *uy, *uz, *dax, *day, *daz;
    float *near;  // non-null: write u and dalpha in sorted order to near[6][n] instead of finishing
    int parts;    // 2 or 4: each block's list is taken in that many parts by neighbouring
                  // waves, part q writing to near + 6 n q (the finalize kernel adds the
                  // parts); else 1
};

struct Acc9 {
    float u0, u1, u2, a0, a1, a2, t0, t1, t2;
};

// Target-side quantities for one list entry.
struct Tgt {
    float y0, y1, y2;     // y_i = delta'_i + D'
    float w0, w1, w2;     // y_i x alpha_i (transpose reading)
    float ai0, ai1, ai2;  // alpha_i
};

// On gfx950 a run of FP32 VALU operations that read a scalar register issues
// at half the rate of ones whose operands are all vector registers (measured:
// 38.7e12 against 66-74e12 lane operations/s), and so does one whose vector
// operands share a register bank.  The loop-invariant constants of the cutoff
// are instruction literals (cutoff_ce).  The source records stay scalar
// operands: copying them into vector registers every step costs more issue
// slots than it saves.

// VAR (per-source cores): records hold unscaled leaf-local offsets, the
// strengths ah = kappa_j^3 alpha/(4 pi) and kappa_j^2, 1/kappa_j of the source
// in their fourth components.  The cutoff factors are those of the scaled form
// at r' = kappa_j r, and F ah and H (ah . (r x alpha_i)) equal the unscaled
// sums once H carries one more kappa_j^2.
// One pair in three parts, so that a loop over several sources can issue the
// transcendental instructions of all of them back to back (see leaf_loop).
struct Geo {
    float dx, dy, dz;  // r' (scaled) or r (per-source cores)
    float r2;          // |r|^2 in the units of the offsets
    float r2s;         // rho'^2
    float rinv;        // 1 / rho'
    float E;           // 2^{-rho'^2} (not for the singular form)
};

template <bool VAR>
__device__ __forceinline__ void geo_offsets(const Tgt &t, float4 sp, Geo &g) {
    g.dx = t.y0 - sp.x;
    g.dy = t.y1 - sp.y;
    g.dz = t.y2 - sp.z;
    g.r2 = fmaf(g.dx, g.dx, fmaf(g.dy, g.dy, g.dz * g.dz));
    g.r2s = VAR ? g.r2 * sp.w : g.r2;  // rho'^2
}

template <int V, bool VAR>
__device__ __forceinline__ void geo_trans(float4 sa, Geo &g) {
    const float rinv0 = __builtin_amdgcn_rsqf(g.r2);
    g.rinv = VAR ? rinv0 * sa.w : rinv0;  // 1 / rho' (rho' = kappa_j rho)
    if (V != 2) g.E = __builtin_amdgcn_exp2f(-g.r2s);
}

template <int V, int SCHEME, bool MASK, bool VAR>
__device__ __forceinline__ void pair_rest(const P2PConst &k, const Tgt &t, const Geo &g, float4 sp, float4 sa,
                                          float4 sb, bool ok, Acc9 &p) {
    const float dx = g.dx, dy = g.dy, dz = g.dz;
    const float rinv = g.rinv;
    const float rinv2 = rinv * rinv;
    float F, H;
    if (V == 2) {
        F = rinv2 * rinv;
        H = F * rinv2;
    } else {
        const float r2s = g.r2s;
        const float E = g.E;
        namespace ce = cutoff_ce;
        float pe = ce::pe(VFMM_ERFCX_DEG);
#pragma unroll
        for (int i = VFMM_ERFCX_DEG - 1; i >= 0; --i) pe = fmaf(pe, rinv, ce::pe(i));
        // G3 = 1 - a E (rho' + pe(1/rho')/rho') and G5 = G3 - a b E rho'^3, so that
        // F = G3 / rho'^3 = (1/rho' - E (a + rho'^-2 a pe)) / rho'^2 and
        // H = G5 / rho'^5 = (F - a b E) / rho'^2
        F = rinv2 * fmaf(-E, fmaf(rinv2, pe, ce::a), rinv);
        H = rinv2 * fmaf(-E, ce::ab, F);
        if (V == 0) {
            if (__any(r2s < ce::r2_small)) {
                float q2 = ce::q(VFMM_M2_DEG);
#pragma unroll
                for (int i = VFMM_M2_DEG - 1; i >= 0; --i) q2 = fmaf(q2, r2s, ce::q(i));
                const float Fs = E * fmaf(r2s, q2, ce::K3);  // 2^{-r2'} K3 1F1(1; 5/2; x)
                const float Hs = E * q2;                   // 2^{-r2'} K5 1F1(1; 7/2; x)
                const bool sm = r2s < ce::r2_small;
                F = sm ? Fs : F;
                H = sm ? Hs : H;
            }
        }
    }
    if (VAR) H *= sp.w;  // kappa_j^2
    if (MASK) {  // a padding source contributes exactly zero
        F = ok ? F : 0.f;
        H = ok ? H : 0.f;
    }
    if (SCHEME == VFMM_SCHEME_TRANSPOSE) {
        float d = fmaf(sa.x, t.w0, fmaf(sa.y, t.w1, sa.z * t.w2));
        d = fmaf(-t.ai0, sb.x, fmaf(-t.ai1, sb.y, fmaf(-t.ai2, sb.z, d)));
        p.u0 = fmaf(F, sb.x, p.u0);
        p.u1 = fmaf(F, sb.y, p.u1);
        p.u2 = fmaf(F, sb.z, p.u2);
        p.a0 = fmaf(F, sa.x, p.a0);
        p.a1 = fmaf(F, sa.y, p.a1);
        p.a2 = fmaf(F, sa.z, p.a2);
        const float hd = H * d;
        p.t0 = fmaf(hd, dx, p.t0);
        p.t1 = fmaf(hd, dy, p.t1);
        p.t2 = fmaf(hd, dz, p.t2);
    } else {
        const float c0 = sa.y * dz - sa.z * dy;
        const float c1 = sa.z * dx - sa.x * dz;
        const float c2 = sa.x * dy - sa.y * dx;
        p.u0 = fmaf(F, c0, p.u0);
        p.u1 = fmaf(F, c1, p.u1);
        p.u2 = fmaf(F, c2, p.u2);
        p.a0 = fmaf(F, sa.x, p.a0);
        p.a1 = fmaf(F, sa.y, p.a1);
        p.a2 = fmaf(F, sa.z, p.a2);
        const float d = fmaf(t.ai0, dx, fmaf(t.ai1, dy, t.ai2 * dz));
        const float hd = H * d;
        p.t0 = fmaf(hd, c0, p.t0);
        p.t1 = fmaf(hd, c1, p.t1);
        p.t2 = fmaf(hd, c2, p.t2);
    }
}

template <int V, int SCHEME, bool MASK, bool VAR>
__device__ __forceinline__ void pair(const P2PConst &k, const Tgt &t, float4 sp, float4 sa, float4 sb, bool ok,
                                     Acc9 &p) {
    Geo g;
    geo_offsets<VAR>(t, sp, g);
    geo_trans<V, VAR>(sa, g);
    pair_rest<V, SCHEME, MASK, VAR>(k, t, g, sp, sa, sb, ok, p);
}

// One group of U sources against the lane's target: the offsets of all U
// pairs, then their transcendental instructions back to back, then the rest.
// On gfx950 two waves issue their vector instructions together (about two
// clocks each) unless a scalar-register operand, a bank conflict or a nearby
// v_rsq/v_exp stops the pairing; a v_rsq/v_exp spread among the other
// instructions slows them more than the same instructions issued together.
// The scheduling barriers keep the compiler from spreading them again.
template <int V, int SCHEME, bool VAR, int U>
__device__ __forceinline__ void trip(const P2PConst &k, const Tgt &t, const float4 *sp, const float4 *sa,
                                     const float4 *sb, Acc9 &p) {
    Geo g[U];
#pragma unroll
    for (int u = 0; u < U; ++u) geo_offsets<VAR>(t, sp[u], g[u]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u) geo_trans<V, VAR>(sa[u], g[u]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u) pair_rest<V, SCHEME, false, VAR>(k, t, g[u], sp[u], sa[u], sb[u], true, p);
}

// All sources of one list entry, two per trip.  The scalar loads of the next
// trip's records are issued before the current trip is evaluated (the last
// full trip's records are loaded twice), so that their latency is covered by
// the trip's arithmetic instead of stalling the wave at the top of each trip.
// The sums are taken in source order whatever the grouping.
template <int V, int SCHEME, bool VAR>
__device__ __forceinline__ void leaf_loop(const P2PConst &k, const float4 *__restrict__ rec, int s0, int cnt,
                                          const Tgt &t, Acc9 &p) {
    constexpr int RS = VAR ? 4 : 3;  // float4 per record
    constexpr int U = 2;
    const float4 *src = rec + RS * (size_t)s0;
    int j = 0;
    if (cnt >= U) {
        const int jlast = cnt - U;
        float4 np[U], na[U], nb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            np[u] = src[RS * u];
            na[u] = src[RS * u + 1];
            nb[u] = src[RS * u + 2];
        }
        for (; j + U <= cnt; j += U) {
            float4 sp[U], sa[U], sb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                sp[u] = np[u];
                sa[u] = na[u];
                sb[u] = nb[u];
            }
            const int jn = min(j + U, jlast);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                np[u] = src[RS * (jn + u)];
                na[u] = src[RS * (jn + u) + 1];
                nb[u] = src[RS * (jn + u) + 2];
            }
            trip<V, SCHEME, VAR, U>(k, t, sp, sa, sb, p);
        }
    }
    if (j < cnt) pair<V, SCHEME, false, VAR>(k, t, src[RS * j], src[RS * j + 1], src[RS * j + 2], true, p);
}

__device__ __forceinline__ void kahan_add(float &s, float &c, float v) {
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Blocks of few targets split the wave into SPLIT lane groups of 64/SPLIT
// lanes that each hold every target of the block and take every SPLIT-th
// source of the leaf (vector loads, one address per group); the groups' sums
// are added at the end.  A group past the last source re-reads the last one
// with its cutoff factors forced to zero, which contributes exactly zero.
template <int V, int SCHEME, int SPLIT, bool VAR>
__device__ __forceinline__ void leaf_loop_split(const P2PConst &k, const float4 *__restrict__ rec, int s0, int cnt,
                                                int grp, const Tgt &t, Acc9 &p) {
    constexpr int RS = VAR ? 4 : 3;
    const float4 *src = rec + RS * (size_t)s0;
    for (int j = 0; j < cnt; j += SPLIT) {
        const bool ok = j + grp < cnt;
        const int jj = ok ? j + grp : cnt - 1;
        pair<V, SCHEME, true, VAR>(k, t, src[RS * jj], src[RS * jj + 1], src[RS * jj + 2], ok, p);
    }
}

template <int SCHEME, bool KAHAN, int SPLIT, bool VAR>
__device__ __forceinline__ void p2p_block(const P2PConst &k, const P2PArgs &A, int t0, int tc, int l0, int lc,
                                          float *near) {
    const int lane = threadIdx.x & 63;
    constexpr int GL = 64 / SPLIT;  // lanes per group
    const int tl = lane % GL, grp = lane / GL;
    const bool valid = tl < tc;
    const int i = t0 + (valid ? tl : 0);
    Tgt t;
    float4 r0;
    if (VAR) {
        r0 = A.rec[4 * (size_t)i];
        const float4 r3 = A.rec[4 * (size_t)i + 3];
        t.ai0 = r3.x;
        t.ai1 = r3.y;
        t.ai2 = r3.z;
    } else {
        r0 = A.rec[3 * (size_t)i];
        t.ai0 = r0.w;
        t.ai1 = A.rec[3 * (size_t)i + 1].w;
        t.ai2 = A.rec[3 * (size_t)i + 2].w;
    }
    float S[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    float Cc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int e = 0; e < lc; ++e) {
        const int4 en = A.ent[l0 + e];
        const float4 D = A.sh[l0 + e];
        const int s0 = __builtin_amdgcn_readfirstlane(en.x);
        const int sc = __builtin_amdgcn_readfirstlane(en.y);
        const int var = __builtin_amdgcn_readfirstlane(en.w);
        t.y0 = r0.x + D.x;
        t.y1 = r0.y + D.y;
        t.y2 = r0.z + D.z;
        if (SCHEME == VFMM_SCHEME_TRANSPOSE) {
            t.w0 = t.y1 * t.ai2 - t.y2 * t.ai1;
            t.w1 = t.y2 * t.ai0 - t.y0 * t.ai2;
            t.w2 = t.y0 * t.ai1 - t.y1 * t.ai0;
        }
        Acc9 p = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (SPLIT == 1) {
            if (var == 1)
                leaf_loop<1, SCHEME, VAR>(k, A.rec, s0, sc, t, p);
            else if (var == 0)
                leaf_loop<0, SCHEME, VAR>(k, A.rec, s0, sc, t, p);
            else
                leaf_loop<2, SCHEME, VAR>(k, A.rec, s0, sc, t, p);
        } else {
            if (var == 1)
                leaf_loop_split<1, SCHEME, SPLIT, VAR>(k, A.rec, s0, sc, grp, t, p);
            else if (var == 0)
                leaf_loop_split<0, SCHEME, SPLIT, VAR>(k, A.rec, s0, sc, grp, t, p);
            else
                leaf_loop_split<2, SCHEME, SPLIT, VAR>(k, A.rec, s0, sc, grp, t, p);
        }
        float u0 = p.u0, u1 = p.u1, u2 = p.u2;
        if (SCHEME == VFMM_SCHEME_TRANSPOSE) {  // Ah x y_i - Bh
            u0 = fmaf(p.a1, t.y2, fmaf(-p.a2, t.y1, -p.u0));
            u1 = fmaf(p.a2, t.y0, fmaf(-p.a0, t.y2, -p.u1));
            u2 = fmaf(p.a0, t.y1, fmaf(-p.a1, t.y0, -p.u2));
        }
        const float pv[9] = {u0, u1, u2, p.a0, p.a1, p.a2, p.t0, p.t1, p.t2};
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
    const float ai0 = t.ai0, ai1 = t.ai1, ai2 = t.ai2;
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
    float u0 = S[0] * k.inv_kappa, u1 = S[1] * k.inv_kappa, u2 = S[2] * k.inv_kappa;
    if (near) {
        near[i] = u0;
        near[A.n + i] = u1;
        near[2 * A.n + i] = u2;
        near[3 * A.n + i] = d0;
        near[4 * A.n + i] = d1;
        near[5 * A.n + i] = d2;
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
    if (A.bounds->stale) u0 = u1 = u2 = d0 = d1 = d2 = __builtin_nanf("");  // positions differ from the build's
    const int o = A.perm[i];
    A.ux[o] = u0;
    A.uy[o] = u1;
    A.uz[o] = u2;
    A.dax[o] = d0;
    A.day[o] = d1;
    A.daz[o] = d2;
}

template <int SCHEME, bool KAHAN, bool VAR>
__global__ __launch_bounds__(256) void k_p2p(P2PConst k, P2PArgs A) {
    const int item = xcd_logical(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    // the waves of a block's parts are neighbours (they share its target
    // records and much of its source data in the caches)
    const int np = A.parts == 4 ? 4 : (A.parts == 2 ? 2 : 1);
    const int b = item / np;
    if (b >= A.nblocks) return;
    const int4 blk = A.blocks[b];
    const int t0 = __builtin_amdgcn_readfirstlane(blk.x);
    const int tc = __builtin_amdgcn_readfirstlane(blk.y);
    int l0 = __builtin_amdgcn_readfirstlane(blk.z);
    int lc = __builtin_amdgcn_readfirstlane(blk.w);
    float *near = A.near;
    if (np > 1) {  // part q: entries [q lc / np, (q + 1) lc / np)
        const int q = item % np;
        const int e0 = (q * lc) / np, e1 = ((q + 1) * lc) / np;
        l0 += e0;
        lc = e1 - e0;
        near += 6 * A.n * q;
    }
    if (tc <= 16)
        p2p_block<SCHEME, KAHAN, 4, VAR>(k, A, t0, tc, l0, lc, near);
    else if (tc <= 32)
        p2p_block<SCHEME, KAHAN, 2, VAR>(k, A, t0, tc, l0, lc, near);
    else
        p2p_block<SCHEME, KAHAN, 1, VAR>(k, A, t0, tc, l0, lc, near);
}

// Records of the float32 near field (sorted order), one wave per leaf.
// Uniform cores (kappa the scale of the shared core):
//   rec[3i] = (kappa (x_i - c_leaf), alpha_x), rec[3i+1] = (ah_i, alpha_y),
//   rec[3i+2] = (ah_i x delta'_i, alpha_z),   ah = kappa^3 alpha/(4 pi).
// Per-source cores (kappa_j of each particle's own core):
//   rec[4i] = (x_i - c_leaf, kappa_i^2), rec[4i+1] = (ah_i, 1/kappa_i),
//   rec[4i+2] = (ah_i x delta_i, kappa_i^3), rec[4i+3] = (alpha_i, 0),  ah = kappa_i^3 alpha/(4 pi).
// Computed in float64 and rounded once.  A null cell list means one common
// origin for every particle (direct mode).
template <bool VAR>
__global__ __launch_bounds__(256) void k_p2p_records(const int *__restrict__ leaves, int nleaves,
                                                     const int *__restrict__ start, const int *__restrict__ count,
                                                     const float4 *__restrict__ geo, int64_t n, double ox, double oy,
                                                     double oz, double kappa, double sa,
                                                     const float4 *__restrict__ rec_in, float4 *__restrict__ out) {
    int64_t i0, i1;
    double cx = ox, cy = oy, cz = oz;
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (leaves) {
        if (w >= nleaves) return;
        const int cell = leaves[w];
        i0 = start[cell];
        i1 = i0 + count[cell];
        const float4 g = geo[cell];
        cx = g.x;
        cy = g.y;
        cz = g.z;
    } else {
        i0 = (int64_t)w * 64;
        i1 = min<int64_t>(i0 + 64, n);
        if (i0 >= n) return;
    }
    const double fp = 12.566370614359172954;  // 4 pi: rec_in holds alpha/(4 pi)
    for (int64_t i = i0 + (threadIdx.x & 63); i < i1; i += 64) {
        const float4 p = rec_in[2 * i], a = rec_in[2 * i + 1];
        // VAR: kappa argument = sqrt(log2 e)/sqrt(2), divided by each core
        const double kap = VAR ? kappa / (double)p.w : kappa;
        const double sc = VAR ? 1.0 : kappa;
        const double d0 = sc * ((double)p.x - cx), d1 = sc * ((double)p.y - cy), d2 = sc * ((double)p.z - cz);
        const double s3 = VAR ? kap * kap * kap : sa;
        const double h0 = s3 * a.x, h1 = s3 * a.y, h2 = s3 * a.z;
        const double b0 = h1 * d2 - h2 * d1, b1 = h2 * d0 - h0 * d2, b2 = h0 * d1 - h1 * d0;
        if (VAR) {
            out[4 * i] = make_float4((float)d0, (float)d1, (float)d2, (float)(kap * kap));
            out[4 * i + 1] = make_float4((float)h0, (float)h1, (float)h2, (float)(1.0 / kap));
            out[4 * i + 2] = make_float4((float)b0, (float)b1, (float)b2, (float)(kap * kap * kap));
            out[4 * i + 3] = make_float4((float)(fp * a.x), (float)(fp * a.y), (float)(fp * a.z), 0.f);
        } else {
            out[3 * i] = make_float4((float)d0, (float)d1, (float)d2, (float)(fp * a.x));
            out[3 * i + 1] = make_float4((float)h0, (float)h1, (float)h2, (float)(fp * a.y));
            out[3 * i + 2] = make_float4((float)b0, (float)b1, (float)b2, (float)(fp * a.z));
        }
    }
}

// ---------------------------------------------------------------------------
// Float64 reference form: the same work blocks and lists, one lane per
// target, every quantity in double and the cutoff always in its full form:
//   F = P(3/2, x)/rho^3,  H = P(5/2, x)/rho^5,  x = c^2 rho^2,  c = 1/(sqrt 2 sigma_j)
// of the source's own core (stored in the fourth component of its record).
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
    double len;
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
            const double cj = sp.w;  // 1/(sqrt 2 sigma_j), stored in the float64 records
            cutoff64(dx * dx + dy * dy + dz * dz, cj, cj * cj, F, H);
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
    if (A.bounds->stale) u0 = u1 = u2 = d0 = d1 = d2 = __builtin_nan("");  // positions differ from the build's
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
    if (c.prm.scheme == VFMM_SCHEME_TRANSPOSE)
        k_p2p64<VFMM_SCHEME_TRANSPOSE><<<A.nblocks, 64, 0, c.stream>>>(A);
    else
        k_p2p64<VFMM_SCHEME_CLASSICAL><<<A.nblocks, 64, 0, c.stream>>>(A);
    VFMM_LAUNCH_CHECK();
}

// The launch constant of the scaled form (the cutoff's constants are cutoff_ce).
static P2PConst make_const(double sigma, bool var) {
    P2PConst k{};
    k.inv_kappa = var ? 1.0f : (float)(1.0 / p2p_kappa(sigma));
    return k;
}

// Launches the float32 near-field records from the sorted records rec into
// recp (tree: one wave per leaf, offsets from the leaf centre; direct: waves of
// 64 particles, offsets from one common origin).
static void launch_records(hipStream_t s, bool var, float sigma_uniform, const int *lv, int nl, const int *start,
                           const int *count, const float4 *geo, int64_t n, const double *origin,
                           const float4 *rec, float4 *recp) {
    // uniform: kappa of the shared core and ah = kappa^3 alpha/(4 pi); per source: the
    // numerator of kappa_j (the kernel scales each strength by its own kappa_j^3)
    const double kap = var ? p2p_kappa(1.0) : p2p_kappa(sigma_uniform);
    const double sa = kap * kap * kap;
    const double o0 = origin ? origin[0] : 0.0, o1 = origin ? origin[1] : 0.0, o2 = origin ? origin[2] : 0.0;
    const unsigned grid = lv ? cdiv(nl, 4) : cdiv(cdiv(n, 64), 4);
    if (var)
        k_p2p_records<true><<<grid, 256, 0, s>>>(lv, nl, start, count, geo, n, o0, o1, o2, kap, sa, rec, recp);
    else
        k_p2p_records<false><<<grid, 256, 0, s>>>(lv, nl, start, count, geo, n, o0, o1, o2, kap, sa, rec, recp);
    VFMM_LAUNCH_CHECK();
}

// The float32 near-field records of the tree's leaves.
static void p2p_records(Ctx &c) {
    if (c.n == 0) return;
    c.recp.ensure(sizeof(float4) * (c.var_sigma ? 4 : 3) * (size_t)c.n);
    launch_records(c.stream, c.var_sigma, c.sigma_uniform, c.leaves.as<int>(), c.nleaves, c.c_start.as<int>(),
                   c.c_count.as<int>(), c.c_geo.as<float4>(), c.n, nullptr, c.rec.as<float4>(), c.recp.as<float4>());
}

void p2p_prepare(Ctx &c) { p2p_records(c); }

template <int SCHEME, bool KAHAN>
static void launch_p2p(const P2PConst &k, const P2PArgs &A, bool var, hipStream_t s) {
    if (A.nblocks == 0) return;
    const int64_t items = (int64_t)A.nblocks * (A.parts == 4 ? 4 : (A.parts == 2 ? 2 : 1));
    if (var)
        k_p2p<SCHEME, KAHAN, true><<<xcd_grid(cdiv(items, 4)), 256, 0, s>>>(k, A);
    else
        k_p2p<SCHEME, KAHAN, false><<<xcd_grid(cdiv(items, 4)), 256, 0, s>>>(k, A);
    VFMM_LAUNCH_CHECK();
}

static void dispatch_p2p(const vfmm_params &prm, bool var, const P2PConst &k, const P2PArgs &A, hipStream_t s) {
    const bool kah = prm.kahan != 0 || prm.precision == VFMM_PRECISION_MIXED;
    if (prm.scheme == VFMM_SCHEME_TRANSPOSE) {
        if (kah) launch_p2p<VFMM_SCHEME_TRANSPOSE, true>(k, A, var, s);
        else launch_p2p<VFMM_SCHEME_TRANSPOSE, false>(k, A, var, s);
    } else {
        if (kah) launch_p2p<VFMM_SCHEME_CLASSICAL, true>(k, A, var, s);
        else launch_p2p<VFMM_SCHEME_CLASSICAL, false>(k, A, var, s);
    }
}

static P2PArgs tree_args(Ctx &c) {
    P2PArgs A{};
    A.rec = c.recp.as<float4>();
    A.blocks = c.blocks.as<int4>();
    A.ent = c.p2p_ent.as<int4>();
    A.sh = c.p2p_sh.as<float4>();
    A.nblocks = c.n_blocks;
    A.n = c.n;
    A.perm = c.perm.as<int>();
    A.bounds = c.bres.as<Bounds>();
    A.surface = (c.prm.periodic && c.prm.zero_mean) ? 1 : 0;
    A.inv3V = c.prm.periodic ? (float)(1.0 / (3.0 * c.prm.box_len * c.prm.box_len * c.prm.box_len)) : 0.f;
    return A;
}

// Parts of every block's list (see p2p_near).
constexpr int P2P_PARTS = 4;
// Near field alone, on stream s, into c.near (sorted order; part q of every
// block's list in near[6 n q .. 6 n (q + 1))); the far field runs before,
// after or beside it on the library stream and finalize_near_far adds the
// parts and the far field.  Four parts per block quadruple the waves: at
// 128^3 the 32,768 one-block waves would fill every SIMD exactly four times
// over, and the uneven end of the last round costs a few percent; a
// work-group then also covers one block instead of four, so fewer target
// neighbourhoods are in flight on each XCD and more source records hit in L2.
void p2p_near(Ctx &c, hipStream_t s) {
    const P2PConst k = make_const(c.sigma_uniform, c.var_sigma);
    c.near.ensure(sizeof(float) * 6 * P2P_PARTS * (size_t)c.n);
    P2PArgs A = tree_args(c);
    A.near = c.near.as<float>();
    A.parts = P2P_PARTS;
    c.record(2 * PH_P2P, s);
    dispatch_p2p(c.prm, c.var_sigma, k, A, s);
    c.record(2 * PH_P2P + 1, s);
}

// out[perm[i]] = (sum of the near-field parts)[i] + far[i] (- the zero-mean
// surface term for u)
__global__ __launch_bounds__(256) void k_finalize(P2PArgs A, const float *__restrict__ near) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= A.n) return;
    const int64_t n = A.n;
    // the four parts in a fixed pairwise order: (p0 + p1) + (p2 + p3), then the far field
    float v[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const float *q = near + (int64_t)c * n + i;
        float a = q[0] + q[6 * n];
        a += q[12 * n] + q[18 * n];
        v[c] = a;
    }
    float u0 = v[0] + A.far_u[i], u1 = v[1] + A.far_u[n + i], u2 = v[2] + A.far_u[2 * n + i];
    float d0 = v[3] + A.far_da[i], d1 = v[4] + A.far_da[n + i], d2 = v[5] + A.far_da[2 * n + i];
    if (A.surface) {
        u0 -= (float)(A.bounds->sum_xa[0]) * A.inv3V;
        u1 -= (float)(A.bounds->sum_xa[1]) * A.inv3V;
        u2 -= (float)(A.bounds->sum_xa[2]) * A.inv3V;
    }
    if (A.bounds->stale) u0 = u1 = u2 = d0 = d1 = d2 = __builtin_nanf("");  // positions differ from the build's
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
    // the same near-field parts and finalize as the other evaluation orders,
    // so that every order gives bitwise the same results
    p2p_near(c, c.stream);
    finalize_near_far(c, ux, uy, uz, dax, day, daz);
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
    rec[2 * i] = make_double4(x[i], y[i], z[i], 0.70710678118654752440 / (double)s[i]);  // 1/(sqrt 2 sigma)
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
__global__ __launch_bounds__(256) void k_direct_blocks(int64_t n, int nb, int4 *blocks, int4 *ent, float4 *sh) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b < nb) {
        const int cnt = (int)min<int64_t>(64, n - (int64_t)b * 64);
        blocks[b] = make_int4(b * 64, cnt, 0, nb);
        ent[b] = make_int4(b * 64, cnt, 0, 0);
        if (sh) sh[b] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// The float32 (and mixed) all-pairs evaluation into caller-given buffers; the
// near-field kernel's interval is timed on ctx's events when tc is given.
static void direct_f32_impl(const Ctx &c, Ctx *tc, hipStream_t s, int64_t n, const Bounds &hb, const DirectBufs &b,
                            const float *x, const float *y, const float *z, const float *ax, const float *ay,
                            const float *az, const float *sigma, float *ux, float *uy, float *uz, float *dax,
                            float *day, float *daz) {
    if (n == 0) return;
    const int nb = (int)cdiv(n, 64);
    k_direct_setup<<<cdiv(n, 256), 256, 0, s>>>(n, x, y, z, ax, ay, az, sigma, b.rec, b.perm);
    VFMM_LAUNCH_CHECK();
    k_direct_blocks<<<cdiv(nb, 256), 256, 0, s>>>(n, nb, b.blocks, b.ent, b.sh);
    VFMM_LAUNCH_CHECK();
    // per-source cores when they differ by more than 1e-6 relative (as a build decides)
    const bool var = hb.sig_max > hb.sig_min * (1.0 + 1e-6);
    const float sig = (float)hb.sig_max;
    // one origin for every record: the centre of the bounding box
    const double org[3] = {0.5 * (hb.lo[0] + hb.hi[0]), 0.5 * (hb.lo[1] + hb.hi[1]), 0.5 * (hb.lo[2] + hb.hi[2])};
    launch_records(s, var, sig, nullptr, 0, nullptr, nullptr, nullptr, n, org, b.rec, b.recp);
    const P2PConst k = make_const(sig, var);
    P2PArgs A{};
    A.rec = b.recp;
    A.blocks = b.blocks;
    A.ent = b.ent;
    A.sh = b.sh;
    A.nblocks = nb;
    A.far_u = nullptr;
    A.far_da = nullptr;
    A.n = n;
    A.perm = b.perm;
    A.bounds = b.bounds;
    A.surface = 0;
    A.ux = ux; A.uy = uy; A.uz = uz; A.dax = dax; A.day = day; A.daz = daz;
    if (tc) tc->record(2 * PH_P2P, s);
    dispatch_p2p(c.prm, var, k, A, s);
    if (tc) tc->record(2 * PH_P2P + 1, s);
}

void direct_f32(const Ctx &c, hipStream_t s, int64_t n, const Bounds &hb, const DirectBufs &b, const float *x,
                const float *y, const float *z, const float *ax, const float *ay, const float *az,
                const float *sigma, float *ux, float *uy, float *uz, float *dax, float *day, float *daz) {
    direct_f32_impl(c, nullptr, s, n, hb, b, x, y, z, ax, ay, az, sigma, ux, uy, uz, dax, day, daz);
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
    c.n_blocks = nb;
    c.p2p_pairs = n * n;
    if (c.prm.precision == VFMM_PRECISION_FP64) {
        k_direct_setup<<<cdiv(n, 256), 256, 0, c.stream>>>(n, x, y, z, ax, ay, az, sigma, c.rec.as<float4>(),
                                                            c.perm.as<int>());
        VFMM_LAUNCH_CHECK();
        k_direct_blocks<<<cdiv(nb, 256), 256, 0, c.stream>>>(n, nb, c.blocks.as<int4>(), c.p2p_ent.as<int4>(),
                                                              nullptr);
        VFMM_LAUNCH_CHECK();
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
    c.p2p_sh.ensure(sizeof(float4) * nb);
    c.recp.ensure(sizeof(float4) * (c.var_sigma ? 4 : 3) * (size_t)n);
    DirectBufs b{c.rec.as<float4>(), c.perm.as<int>(), c.blocks.as<int4>(), c.p2p_ent.as<int4>(),
                 c.p2p_sh.as<float4>(), c.recp.as<float4>(), c.bres.as<Bounds>()};
    direct_f32_impl(c, &c, c.stream, n, c.hb, b, x, y, z, ax, ay, az, sigma, ux, uy, uz, dax, day, daz);
}

}  // namespace vfmm
