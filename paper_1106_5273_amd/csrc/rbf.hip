// Radial-basis-function reinitialisation of the particle strengths (Sec. 2.1,
// last paragraph; Sec. 2.2; Sec. 3.4).
//
// The vorticity carried by particles of strengths gamma_j and cores sigma_j is
// omega(x) = sum_j gamma_j zeta_j(x - x_j), zeta_j(r) = (2 pi sigma_j^2)^{-3/2}
// exp(-|r|^2 / (2 sigma_j^2)), the Gaussian whose enclosed mass is the cutoff
// of Eq. (2).  Reinitialising asks for the strengths that reproduce a given
// vorticity omega_i at the particles' own positions,
//     sum_j zeta_j(x_i - x_j) gamma_j = omega_i,
// one symmetric positive definite system per component (uniform cores),
// solved here by plain conjugate gradients from gamma = 0 with the
// matrix-vector product on the tree of the last build: the particles are
// reinitialised at the positions the tree was built for (Sec. 3.4).
//
// The product is a near-field pass over the build's P2P lists (the same work
// blocks of <= 64 targets, the same leaf-local scaled offsets): list entries
// whose leaf boxes are at least 7.2 sigma_max apart (the singular cutoff form
// of the Biot-Savart pass) are skipped, their Gaussians being below e^-26 of
// the peak; the pairs the traversal sent to M2L are at least sigma_gap *
// sigma_max apart and are dropped (the Gaussian mass beyond c sigma is
// 1 - g(c sigma): 1.5e-5 for c = 5, 7.5e-8 for c = 6).
//
// Per pair, with r' = kappa (x_i - x_j) (uniform cores, kappa^2 =
// log2(e) / (2 sigma^2)) or r' = kappa_j (x_i - x_j) (per-source cores):
//     w_i += 2^{-|r'|^2} (s_j gamma_j),  s_j = (2 pi sigma_j^2)^{-3/2}:
// three subtractions, three multiply-adds for |r'|^2 (one more multiply per
// source core), one exp2 and three multiply-adds.  The source records are
// scalar operands (one source per step for the whole wave), as in the P2P pass.
//
// Conjugate-gradient vectors x, r, p live in float64 in the sorted order;
// the strengths of the product are rounded to float32 once per iteration;
// every dot product is a fixed two-stage float64 reduction, so the solve is
// bit-reproducible.  One host synchronisation per iteration reads the three
// residual norms for the stopping test.
#include <cstring>

#include "ctx.h"

namespace vfmm {

static constexpr int RB_TPB = 256;
static constexpr int RB_PARTS = 1024;  // work-groups of the first reduction stage

struct GaussArgs {
    const float4 *__restrict__ pos;  // float4[n]: (r' offset from the leaf centre, kappa_j^2 or 1)
    const float4 *__restrict__ str;  // float4[n]: (s_j gamma_j, 0)
    const int4 *__restrict__ blocks;
    const int4 *__restrict__ ent;
    const float4 *__restrict__ sh;   // per entry: scaled offset between the two leaf centres
    int nblocks;
    int64_t n;
    float *__restrict__ w;           // float[3n], sorted order
};

template <bool VAR, bool MASK>
__device__ __forceinline__ void gpair(float y0, float y1, float y2, float4 sp, float4 sg, bool ok, float &w0,
                                      float &w1, float &w2) {
    const float dx = y0 - sp.x, dy = y1 - sp.y, dz = y2 - sp.z;
    float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    if (VAR) r2 *= sp.w;
    float E = __builtin_amdgcn_exp2f(-r2);
    if (MASK) E = ok ? E : 0.f;
    w0 = fmaf(E, sg.x, w0);
    w1 = fmaf(E, sg.y, w1);
    w2 = fmaf(E, sg.z, w2);
}

template <bool VAR, int SPLIT>
__device__ __forceinline__ void gauss_block(const GaussArgs &A, int t0, int tc, int l0, int lc) {
    const int lane = threadIdx.x & 63;
    constexpr int GL = 64 / SPLIT;
    const int tl = lane % GL, grp = lane / GL;
    const bool valid = tl < tc;
    const int i = t0 + (valid ? tl : 0);
    const float4 pi = A.pos[i];
    float S0 = 0.f, S1 = 0.f, S2 = 0.f;
    // the next entry's list record and shift are loaded while this one runs
    int4 en_n = lc > 0 ? A.ent[l0] : make_int4(0, 0, 0, 2);
    float4 D_n = lc > 0 ? A.sh[l0] : make_float4(0.f, 0.f, 0.f, 0.f);
    for (int e = 0; e < lc; ++e) {
        const int4 en = en_n;
        const float4 D = D_n;
        if (e + 1 < lc) {
            en_n = A.ent[l0 + e + 1];
            D_n = A.sh[l0 + e + 1];
        }
        if (__builtin_amdgcn_readfirstlane(en.w) == 2) continue;  // every pair beyond 7.2 sigma_max
        const int s0 = __builtin_amdgcn_readfirstlane(en.x);
        const int sc = __builtin_amdgcn_readfirstlane(en.y);
        const float y0 = pi.x + D.x, y1 = pi.y + D.y, y2 = pi.z + D.z;
        const float4 *sp = A.pos + s0;
        const float4 *sg = A.str + s0;
        float w0 = 0.f, w1 = 0.f, w2 = 0.f;
        if (SPLIT == 1) {
            // eight sources per batch of scalar loads: one load latency per 80 instructions
            int j = 0;
            for (; j + 8 <= sc; j += 8) {
                float4 P[8], G[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    P[q] = sp[j + q];
                    G[q] = sg[j + q];
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) gpair<VAR, false>(y0, y1, y2, P[q], G[q], true, w0, w1, w2);
            }
            for (; j < sc; ++j) gpair<VAR, false>(y0, y1, y2, sp[j], sg[j], true, w0, w1, w2);
        } else {
            // lane groups take every SPLIT-th source; a group past the end
            // re-reads the last source with its Gaussian forced to zero
            for (int j = 0; j < sc; j += SPLIT) {
                const bool ok = j + grp < sc;
                const int jj = ok ? j + grp : sc - 1;
                gpair<VAR, true>(y0, y1, y2, sp[jj], sg[jj], ok, w0, w1, w2);
            }
        }
        S0 += w0;
        S1 += w1;
        S2 += w2;
    }
    if (SPLIT > 1) {
        S0 += __shfl_xor(S0, 32, 64);
        S1 += __shfl_xor(S1, 32, 64);
        S2 += __shfl_xor(S2, 32, 64);
        if (SPLIT > 2) {
            S0 += __shfl_xor(S0, 16, 64);
            S1 += __shfl_xor(S1, 16, 64);
            S2 += __shfl_xor(S2, 16, 64);
        }
    }
    if (!valid || grp != 0) return;
    A.w[i] = S0;
    A.w[A.n + i] = S1;
    A.w[2 * A.n + i] = S2;
}

template <bool VAR>
__global__ __launch_bounds__(256) void k_gauss(GaussArgs A) {
    const int b = xcd_logical(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (b >= A.nblocks) return;
    const int4 blk = A.blocks[b];
    const int t0 = __builtin_amdgcn_readfirstlane(blk.x);
    const int tc = __builtin_amdgcn_readfirstlane(blk.y);
    const int l0 = __builtin_amdgcn_readfirstlane(blk.z);
    const int lc = __builtin_amdgcn_readfirstlane(blk.w);
    if (tc <= 16)
        gauss_block<VAR, 4>(A, t0, tc, l0, lc);
    else if (tc <= 32)
        gauss_block<VAR, 2>(A, t0, tc, l0, lc);
    else
        gauss_block<VAR, 1>(A, t0, tc, l0, lc);
}

// Particle pairs one product evaluates: per work block, its targets times the
// sources of its entries that are not skipped.
__global__ __launch_bounds__(RB_TPB) void k_gauss_pairs(const int4 *blocks, const int4 *ent, int nblocks,
                                                        unsigned long long *out) {
    unsigned long long np = 0;
    for (int b = blockIdx.x * RB_TPB + threadIdx.x; b < nblocks; b += gridDim.x * RB_TPB) {
        const int4 blk = blocks[b];
        unsigned long long s = 0;
        for (int e = 0; e < blk.w; ++e) {
            const int4 en = ent[blk.z + e];
            if (en.w != 2) s += (unsigned long long)en.y;
        }
        np += s * (unsigned long long)blk.y;
    }
    __shared__ unsigned long long sh[RB_TPB];
    sh[threadIdx.x] = np;
    __syncthreads();
    for (int o = RB_TPB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

// Offsets from each particle's leaf centre (scaled by kappa of the shared core,
// or unscaled with kappa_j^2 for per-source cores; float64, rounded once, as
// the P2P records) and the normalisation s_j of its Gaussian.  One wave per leaf.
template <bool VAR>
__global__ __launch_bounds__(256) void k_gauss_pos(const int *__restrict__ leaves, int nleaves,
                                                   const int *__restrict__ start, const int *__restrict__ count,
                                                   const float4 *__restrict__ geo, double kappa,
                                                   const float4 *__restrict__ rec, float4 *__restrict__ pos,
                                                   double *__restrict__ sfac) {
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= nleaves) return;
    const int cell = leaves[w];
    const int64_t i0 = start[cell], i1 = i0 + count[cell];
    const float4 g = geo[cell];
    const double two_pi = 6.283185307179586477;
    for (int64_t i = i0 + (threadIdx.x & 63); i < i1; i += 64) {
        const float4 p = rec[2 * i];
        const double sg = (double)p.w;
        const double sc = VAR ? 1.0 : kappa;
        const double kj = kappa / sg;  // VAR: kappa holds the numerator sqrt(log2 e) / sqrt 2
        pos[i] = make_float4((float)(sc * ((double)p.x - g.x)), (float)(sc * ((double)p.y - g.y)),
                             (float)(sc * ((double)p.z - g.z)), VAR ? (float)(kj * kj) : 1.f);
        sfac[i] = 1.0 / (two_pi * sg * sg * sqrt(two_pi * sg * sg));
    }
}

// ---- conjugate-gradient vector kernels (sorted order, SoA [3][n]) ----
struct CgVec {
    double *x, *r, *p;
    float *Ap;
    float4 *str;
    const double *sfac;
    const int *perm;
    int64_t n;
};

// block reduction of three float64 sums into part[c * RB_PARTS + blockIdx.x]
__device__ inline void reduce3(double a0, double a1, double a2, double *part) {
    __shared__ double sh[3][RB_TPB];
    sh[0][threadIdx.x] = a0;
    sh[1][threadIdx.x] = a1;
    sh[2][threadIdx.x] = a2;
    __syncthreads();
    for (int o = RB_TPB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) part[c * RB_PARTS + blockIdx.x] = sh[c][0];
}

// second stage: out[c] = sum of the partials in a fixed order
__global__ __launch_bounds__(RB_TPB) void k_sum3(const double *part, double *out) {
    const int c = blockIdx.x;
    __shared__ double sh[RB_TPB];
    double s = 0.0;
    for (int k = threadIdx.x; k < RB_PARTS; k += RB_TPB) s += part[c * RB_PARTS + k];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = RB_TPB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = sh[0];
}

// r = b (gathered from the caller's order), p = r, x = 0, strengths s p; partial b.b
__global__ __launch_bounds__(RB_TPB) void k_cg_init(CgVec V, const float *wx, const float *wy, const float *wz,
                                                     double *part) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    const int64_t n = V.n;
    for (int64_t i = (int64_t)blockIdx.x * RB_TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB_TPB) {
        const int o = V.perm[i];
        const double b0 = wx[o], b1 = wy[o], b2 = wz[o];
        V.x[i] = 0.0; V.x[n + i] = 0.0; V.x[2 * n + i] = 0.0;
        V.r[i] = b0; V.r[n + i] = b1; V.r[2 * n + i] = b2;
        V.p[i] = b0; V.p[n + i] = b1; V.p[2 * n + i] = b2;
        const double s = V.sfac[i];
        V.str[i] = make_float4((float)(s * b0), (float)(s * b1), (float)(s * b2), 0.f);
        a0 += b0 * b0;
        a1 += b1 * b1;
        a2 += b2 * b2;
    }
    reduce3(a0, a1, a2, part);
}

// partial p . Ap
__global__ __launch_bounds__(RB_TPB) void k_cg_pap(CgVec V, double *part) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    const int64_t n = V.n;
    for (int64_t i = (int64_t)blockIdx.x * RB_TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB_TPB) {
        a0 += V.p[i] * (double)V.Ap[i];
        a1 += V.p[n + i] * (double)V.Ap[n + i];
        a2 += V.p[2 * n + i] * (double)V.Ap[2 * n + i];
    }
    reduce3(a0, a1, a2, part);
}

// alpha = rr / pAp for the active components; x += alpha p, r -= alpha Ap; partial r.r
__global__ __launch_bounds__(RB_TPB) void k_cg_update(CgVec V, const double *rr, const double *pap, int active,
                                                       double *part) {
    double al[3];
    for (int c = 0; c < 3; ++c) al[c] = ((active >> c) & 1) ? rr[c] / pap[c] : 0.0;
    double a[3] = {0.0, 0.0, 0.0};
    const int64_t n = V.n;
    for (int64_t i = (int64_t)blockIdx.x * RB_TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB_TPB) {
        for (int c = 0; c < 3; ++c) {
            const int64_t k = c * n + i;
            V.x[k] += al[c] * V.p[k];
            const double rk = V.r[k] - al[c] * (double)V.Ap[k];
            V.r[k] = rk;
            a[c] += rk * rk;
        }
    }
    reduce3(a[0], a[1], a[2], part);
}

// beta = rr_new / rr for the active components; p = r + beta p; strengths s p
__global__ __launch_bounds__(RB_TPB) void k_cg_dir(CgVec V, const double *rr, const double *rrn, int active) {
    double be[3];
    for (int c = 0; c < 3; ++c) be[c] = ((active >> c) & 1) ? rrn[c] / rr[c] : 0.0;
    const int64_t n = V.n;
    for (int64_t i = (int64_t)blockIdx.x * RB_TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB_TPB) {
        double q[3];
        for (int c = 0; c < 3; ++c) {
            const int64_t k = c * n + i;
            q[c] = ((active >> c) & 1) ? V.r[k] + be[c] * V.p[k] : V.p[k];
            V.p[k] = q[c];
        }
        const double s = V.sfac[i];
        V.str[i] = make_float4((float)(s * q[0]), (float)(s * q[1]), (float)(s * q[2]), 0.f);
    }
}

// strengths s gamma of the caller's gamma (gathered into the sorted order)
__global__ __launch_bounds__(RB_TPB) void k_gauss_str(const int *perm, const double *sfac, int64_t n, const float *gx,
                                                       const float *gy, const float *gz, float4 *str) {
    const int64_t i = (int64_t)blockIdx.x * RB_TPB + threadIdx.x;
    if (i >= n) return;
    const int o = perm[i];
    const double s = sfac[i];
    str[i] = make_float4((float)(s * (double)gx[o]), (float)(s * (double)gy[o]), (float)(s * (double)gz[o]), 0.f);
}

// sorted float32 [3][n] -> the caller's order
__global__ __launch_bounds__(RB_TPB) void k_scatter3f(const int *perm, int64_t n, const float *w, float *ox, float *oy,
                                                       float *oz) {
    const int64_t i = (int64_t)blockIdx.x * RB_TPB + threadIdx.x;
    if (i >= n) return;
    const int o = perm[i];
    ox[o] = w[i];
    oy[o] = w[n + i];
    oz[o] = w[2 * n + i];
}

// sorted float64 [3][n] -> the caller's order, rounded once
__global__ __launch_bounds__(RB_TPB) void k_scatter3d(const int *perm, int64_t n, const double *x, float *ox,
                                                       float *oy, float *oz) {
    const int64_t i = (int64_t)blockIdx.x * RB_TPB + threadIdx.x;
    if (i >= n) return;
    const int o = perm[i];
    ox[o] = (float)x[i];
    oy[o] = (float)x[n + i];
    oz[o] = (float)x[2 * n + i];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static void rbf_check(const Ctx &c, int64_t n, const char *who) {
    if (c.prm.direct) throw Error{VFMM_EINVAL, std::string(who) + ": needs the tree (direct = 0)"};
    if (c.prm.precision == VFMM_PRECISION_FP64)
        throw Error{VFMM_EINVAL, std::string(who) + ": float32 and mixed forms only"};
    if (!c.built) throw Error{VFMM_ESTATE, std::string(who) + ": no fmm_build before it"};
    if (c.nprob != 1) throw Error{VFMM_EINVAL, std::string(who) + ": not after fmm_build_batched"};
    if (c.tg_n >= 0) throw Error{VFMM_EINVAL, std::string(who) + ": not after fmm_build_targets"};
    if (n != c.n) throw Error{VFMM_ESTATE, std::string(who) + ": n differs from the last fmm_build"};
}

// Buffers of the Gaussian sum and the solve (grow-only, in c.rbf):
//   pos float4[n], str float4[n], sfac double[n], w float[3n], x r p double[3n],
//   partials double[3 * RB_PARTS], scalars double[16], pair partials u64[RB_PARTS]
struct RbfBufs {
    float4 *pos, *str;
    double *sfac;
    float *w;
    double *x, *r, *p;
    double *part, *sc;
    unsigned long long *pp;
};

static size_t al256(size_t b) { return (b + 255) / 256 * 256; }

static RbfBufs rbf_bufs(Ctx &c, bool with_cg) {
    const size_t n = (size_t)c.n;
    size_t off[11];
    size_t sz[10] = {16 * n, 16 * n, 8 * n, 12 * n, with_cg ? 24 * n : 0, with_cg ? 24 * n : 0,
                     with_cg ? 24 * n : 0, 8 * 3 * RB_PARTS, 8 * 16, 8 * RB_PARTS};
    off[0] = 0;
    for (int k = 0; k < 10; ++k) off[k + 1] = off[k] + al256(sz[k]);
    c.rbf.ensure(off[10]);
    char *b = c.rbf.as<char>();
    RbfBufs B{};
    B.pos = (float4 *)(b + off[0]);
    B.str = (float4 *)(b + off[1]);
    B.sfac = (double *)(b + off[2]);
    B.w = (float *)(b + off[3]);
    B.x = with_cg ? (double *)(b + off[4]) : nullptr;
    B.r = with_cg ? (double *)(b + off[5]) : nullptr;
    B.p = with_cg ? (double *)(b + off[6]) : nullptr;
    B.part = (double *)(b + off[7]);
    B.sc = (double *)(b + off[8]);
    B.pp = (unsigned long long *)(b + off[9]);
    return B;
}

// offsets and normalisations for the tree of the last build (once per build)
static void gauss_prepare(Ctx &c, const RbfBufs &B) {
    hipStream_t s = c.stream;
    const double kap = c.var_sigma ? p2p_kappa(1.0) : p2p_kappa(c.sigma_uniform);
    const unsigned grid = cdiv(c.nleaves, 4);
    if (c.var_sigma)
        k_gauss_pos<true><<<grid, 256, 0, s>>>(c.leaves.as<int>(), c.nleaves, c.c_start.as<int>(), c.c_count.as<int>(),
                                               c.c_geo.as<float4>(), kap, c.rec.as<float4>(), B.pos, B.sfac);
    else
        k_gauss_pos<false><<<grid, 256, 0, s>>>(c.leaves.as<int>(), c.nleaves, c.c_start.as<int>(),
                                                c.c_count.as<int>(), c.c_geo.as<float4>(), kap, c.rec.as<float4>(),
                                                B.pos, B.sfac);
    VFMM_LAUNCH_CHECK();
    if (c.gauss_build_id != c.build_id) {
        k_gauss_pairs<<<RB_PARTS, RB_TPB, 0, s>>>(c.blocks.as<int4>(), c.p2p_ent.as<int4>(), c.n_blocks, B.pp);
        VFMM_LAUNCH_CHECK();
        std::vector<unsigned long long> h(RB_PARTS);
        VFMM_HIP(hipMemcpyAsync(h.data(), B.pp, sizeof(unsigned long long) * RB_PARTS, hipMemcpyDeviceToHost, s));
        VFMM_HIP(hipStreamSynchronize(s));
        unsigned long long t = 0;
        for (unsigned long long v : h) t += v;
        c.gauss_pairs = (int64_t)t;
        c.gauss_build_id = c.build_id;
    }
}

static void gauss_launch(Ctx &c, const RbfBufs &B) {
    GaussArgs A{};
    A.pos = B.pos;
    A.str = B.str;
    A.blocks = c.blocks.as<int4>();
    A.ent = c.p2p_ent.as<int4>();
    A.sh = c.p2p_sh.as<float4>();
    A.nblocks = c.n_blocks;
    A.n = c.n;
    A.w = B.w;
    if (A.nblocks == 0) return;
    const unsigned grid = xcd_grid(cdiv(A.nblocks, 4));
    if (c.var_sigma)
        k_gauss<true><<<grid, 256, 0, c.stream>>>(A);
    else
        k_gauss<false><<<grid, 256, 0, c.stream>>>(A);
    VFMM_LAUNCH_CHECK();
}

static void ensure_rbf_events(Ctx &c) {
    if (c.rbf_ev_ok) return;
    for (auto &e : c.rbf_ev) VFMM_HIP(hipEventCreate(&e));
    c.rbf_ev_ok = true;
}

static float rbf_ms(const Ctx &c, int a, int b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c.rbf_ev[a], c.rbf_ev[b]) != hipSuccess) {
        (void)hipGetLastError();
        return 0.f;
    }
    return ms;
}

void gaussian_sum_run(Ctx &c, int64_t n, const float *gx, const float *gy, const float *gz, float *wx, float *wy,
                      float *wz) {
    rbf_check(c, n, "fmm_gaussian_sum");
    ensure_rbf_events(c);
    if (n == 0) return;
    const RbfBufs B = rbf_bufs(c, false);
    gauss_prepare(c, B);
    k_gauss_str<<<cdiv(n, RB_TPB), RB_TPB, 0, c.stream>>>(c.perm.as<int>(), B.sfac, n, gx, gy, gz, B.str);
    VFMM_LAUNCH_CHECK();
    VFMM_HIP(hipEventRecord(c.rbf_ev[2], c.stream));
    gauss_launch(c, B);
    VFMM_HIP(hipEventRecord(c.rbf_ev[3], c.stream));
    k_scatter3f<<<cdiv(n, RB_TPB), RB_TPB, 0, c.stream>>>(c.perm.as<int>(), n, B.w, wx, wy, wz);
    VFMM_LAUNCH_CHECK();
    c.gauss_timed = true;
}

float gaussian_sum_ms(const Ctx &c) {
    if (!c.gauss_timed) return 0.f;
    VFMM_HIP(hipStreamSynchronize(c.stream));
    return rbf_ms(c, 2, 3);
}

void rbf_reinit_run(Ctx &c, int64_t n, const float *wx, const float *wy, const float *wz, float *gx, float *gy,
                    float *gz, double tol, int maxiter, vfmm_rbf_info *info) {
    rbf_check(c, n, "rbf_reinit");
    if (!(tol >= 0.0) || maxiter < 0) throw Error{VFMM_EINVAL, "rbf_reinit: tol must be >= 0 and maxiter >= 0"};
    // with cores that differ per particle the matrix zeta_j(x_i - x_j) is not symmetric,
    // and conjugate gradients do not apply
    if (c.var_sigma) throw Error{VFMM_EINVAL, "rbf_reinit: needs one shared core (per-particle cores give a nonsymmetric system)"};
    ensure_rbf_events(c);
    vfmm_rbf_info I;
    std::memset(&I, 0, sizeof(I));
    if (n == 0) {
        if (info) *info = I;
        return;
    }
    hipStream_t s = c.stream;
    const RbfBufs B = rbf_bufs(c, true);
    VFMM_HIP(hipEventRecord(c.rbf_ev[0], s));
    gauss_prepare(c, B);
    I.pairs = c.gauss_pairs;
    CgVec V{B.x, B.r, B.p, B.w, B.str, B.sfac, c.perm.as<int>(), n};
    double *bb = B.sc, *rrA = B.sc + 3, *rrB = B.sc + 6, *pap = B.sc + 9;
    k_cg_init<<<RB_PARTS, RB_TPB, 0, s>>>(V, wx, wy, wz, B.part);
    VFMM_LAUNCH_CHECK();
    k_sum3<<<3, RB_TPB, 0, s>>>(B.part, bb);
    VFMM_LAUNCH_CHECK();
    VFMM_HIP(hipMemcpyAsync(rrA, bb, 3 * sizeof(double), hipMemcpyDeviceToDevice, s));
    double hb[3], hr[3];
    VFMM_HIP(hipMemcpyAsync(hb, bb, sizeof(hb), hipMemcpyDeviceToHost, s));
    VFMM_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < 3; ++k) hr[k] = hb[k];
    auto active_mask = [&]() {
        int m = 0;
        for (int k = 0; k < 3; ++k)
            if (hb[k] > 0.0 && std::sqrt(hr[k]) > tol * std::sqrt(hb[k])) m |= 1 << k;
        return m;
    };
    int active = active_mask();
    double mv_ms = 0.0;
    int it = 0;
    while (active && it < maxiter) {
        double *rr = (it & 1) ? rrB : rrA, *rrn = (it & 1) ? rrA : rrB;
        VFMM_HIP(hipEventRecord(c.rbf_ev[2], s));
        gauss_launch(c, B);
        VFMM_HIP(hipEventRecord(c.rbf_ev[3], s));
        k_cg_pap<<<RB_PARTS, RB_TPB, 0, s>>>(V, B.part);
        VFMM_LAUNCH_CHECK();
        k_sum3<<<3, RB_TPB, 0, s>>>(B.part, pap);
        VFMM_LAUNCH_CHECK();
        k_cg_update<<<RB_PARTS, RB_TPB, 0, s>>>(V, rr, pap, active, B.part);
        VFMM_LAUNCH_CHECK();
        k_sum3<<<3, RB_TPB, 0, s>>>(B.part, rrn);
        VFMM_LAUNCH_CHECK();
        k_cg_dir<<<RB_PARTS, RB_TPB, 0, s>>>(V, rr, rrn, active);
        VFMM_LAUNCH_CHECK();
        double hn[3];
        VFMM_HIP(hipMemcpyAsync(hn, rrn, sizeof(hn), hipMemcpyDeviceToHost, s));
        VFMM_HIP(hipStreamSynchronize(s));
        mv_ms += rbf_ms(c, 2, 3);
        // an inactive component's r is unchanged (alpha = 0), so its new sum of
        // squares equals its old one in both buffers
        for (int k = 0; k < 3; ++k)
            if ((active >> k) & 1) {
                hr[k] = hn[k];
                ++I.iterations[k];
            }
        ++it;
        ++I.matvecs;
        active = active_mask();
    }
    k_scatter3d<<<cdiv(n, RB_TPB), RB_TPB, 0, s>>>(c.perm.as<int>(), n, B.x, gx, gy, gz);
    VFMM_LAUNCH_CHECK();
    VFMM_HIP(hipEventRecord(c.rbf_ev[1], s));
    VFMM_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < 3; ++k) I.residual[k] = hb[k] > 0.0 ? std::sqrt(hr[k] / hb[k]) : 0.0;
    I.solve_ms = rbf_ms(c, 0, 1);
    I.matvec_ms = (float)mv_ms;
    if (info) *info = I;
}

}  // namespace vfmm
