// Far field: P2M, M2M, M2L, L2L, L2P and the periodic lattice term (Sec. 3.1,
// Sec. 3.5, Sec. 3.6) for the three Laplace potentials
//   psi_m(x) = sum_j alpha_j,m / (4 pi |x - x_j|),   m = x, y, z,
// from which u = curl psi and du_l/dx_k = eps_{l n m} d_k d_n psi_m.
//
// Expansions are normalised by the cell size s (Sec. 4.2: normalised
// coefficients keep float32 in range): a cell with centre c stores
//   Mt_n^m = sum_j q_j conj(R_n^m((x_j - c)/s)),        psi = (1/s) sum Mt I_n^m((x-c)/s)
//   Lt_n^m with psi(x) = (1/s) sum Lt_n^m R_n^m((x - c)/s)
// and sums run from the highest degree to the lowest (Sec. 4.2).
#include "ctx.h"

namespace vfmm {

static constexpr int TPB = 256;

// Vector types of the compute precision R (float: the product path; double:
// the FP64 reference form of the precision parameter).
template <class R> struct VT;
template <> struct VT<float> { using V2 = float2; using V4 = float4; };
template <> struct VT<double> { using V2 = double2; using V4 = double4; };

template <class V2>
__device__ inline V2 cmul(V2 a, V2 b) { return V2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
template <class V2>
__device__ inline V2 cconj(V2 a) { return V2{a.x, -a.y}; }

__device__ inline float fmar(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline double fmar(double a, double b, double c) { return fma(a, b, c); }
__device__ inline float rsqr(float a) { return rsqrtf(a); }
__device__ inline double rsqr(double a) { return 1.0 / sqrt(a); }

// rt^e for a ratio of cell sizes (a power of two) and an integer e >= 0
__device__ inline float powr(float rt, int e) { return __builtin_amdgcn_exp2f((float)e * __log2f(rt)); }
__device__ inline double powr(double rt, int e) { return exp2((double)e * log2(rt)); }

// c_n^m for any sign of m from the m >= 0 storage: c_n^{-m} = (-1)^m conj(c_n^m).
template <class V2>
__device__ inline V2 getc(const V2 *a, int n, int m) {
    if (m >= 0) return a[CIDX(n, m)];
    const V2 v = a[CIDX(n, -m)];
    return (m & 1) ? V2{-v.x, v.y} : V2{v.x, -v.y};
}

__device__ inline void decode_nm(int t, int &n, int &m) {
    n = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
    while ((n + 1) * (n + 2) / 2 <= t) ++n;
    while (n * (n + 1) / 2 > t) --n;
    m = t - n * (n + 1) / 2;
}

// ---------------------------------------------------------------------------
// P2M: one wave per leaf, particles staged CH at a time.
// ---------------------------------------------------------------------------
template <int P, class R>
__global__ __launch_bounds__(64) void k_p2m(const int *leaves, const int *start, const int *count, const float4 *geo,
                                            const typename VT<R>::V4 *rec, typename VT<R>::V2 *Mexp) {
    using V2 = typename VT<R>::V2;
    using V4 = typename VT<R>::V4;
    constexpr int NCP = NC(P);
    // particles staged per pass: 32 (17 KB of LDS in float32) lets nine
    // one-wave work-groups share a CU; 64 (34 KB) allowed four and was slower
    constexpr int CH = 32;
    __shared__ V2 Rs[CH][NCP];
    __shared__ V4 al[CH];
    const int lane = threadIdx.x;
    const int cell = leaves[blockIdx.x];
    const float4 g = geo[cell];
    const R inv = R(1) / R(g.w);
    const int s0 = start[cell], cnt = count[cell];
    constexpr int NT = (NCP + 63) / 64;
    V2 acc[NT][3];
#pragma unroll
    for (int t = 0; t < NT; ++t)
        for (int c = 0; c < 3; ++c) acc[t][c] = V2{R(0), R(0)};
    for (int b = 0; b < cnt; b += CH) {
        if (lane < CH) {
            const int j = s0 + b + lane;
            if (b + lane < cnt) {
                const V4 p = rec[2 * j];
                V2 Rl[NCP];
                regular_harmonics<P, R, V2>((p.x - R(g.x)) * inv, (p.y - R(g.y)) * inv, (p.z - R(g.z)) * inv, Rl);
#pragma unroll
                for (int t = 0; t < NCP; ++t) Rs[lane][t] = Rl[t];
                al[lane] = rec[2 * j + 1];
            } else {
                al[lane] = V4{R(0), R(0), R(0), R(0)};
#pragma unroll
                for (int t = 0; t < NCP; ++t) Rs[lane][t] = V2{R(0), R(0)};
            }
        }
        __syncthreads();
        const int jmax = min(CH, cnt - b);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int coef = lane + 64 * t;
            if (coef < NCP) {
                for (int jj = 0; jj < jmax; ++jj) {
                    const V2 r = Rs[jj][coef];
                    const V4 a = al[jj];
                    acc[t][0].x += a.x * r.x; acc[t][0].y -= a.x * r.y;
                    acc[t][1].x += a.y * r.x; acc[t][1].y -= a.y * r.y;
                    acc[t][2].x += a.z * r.x; acc[t][2].y -= a.z * r.y;
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int coef = lane + 64 * t;
        if (coef < NCP)
            for (int c = 0; c < 3; ++c) Mexp[((size_t)cell * 3 + c) * NCP + coef] = acc[t][c];
    }
}

// ---------------------------------------------------------------------------
// M2M: one work-group per parent cell of one level, one thread per
// (potential, coefficient n >= m >= 0) of the parent.
//   Mt_n^m(P) = sum_children sum_{k,l} conj(R_k^l(d)) (s_c/s_P)^{n-k} Mt_{n-k}^{m-l}(c),
//   d = (c - P)/s_P.
// Children are staged one at a time in LDS as full-order tables (m from -n
// to n, negative orders expanded once) with the size ratio folded into the
// child's coefficients, so the inner loop is a plain complex multiply-add.
// S is the storage type of the expansions, R the arithmetic type (the mixed
// precision form keeps float storage and accumulates in double).
// ---------------------------------------------------------------------------
template <int P>
struct XferCfg {
    static constexpr int NCP = NC(P);
    static constexpr int W = 2 * P + 1;                       // full-order row width
    static constexpr int THREADS = ((3 * NCP + 63) / 64) * 64;
};

template <int P, class R, class S>
__global__ __launch_bounds__((XferCfg<P>::THREADS)) void k_m2m(int c0, int c1, const int *child, const int *nchild,
                                                               const float4 *geo, typename VT<S>::V2 *Mexp) {
    using V2 = typename VT<R>::V2;
    using C = XferCfg<P>;
    constexpr int NCP = C::NCP, W = C::W;
    __shared__ V2 Mf[3][P + 1][W];   // child multipole, scaled by (s_c/s_P)^n, full orders
    __shared__ V2 Rf[P + 1][W];      // conj R_k^l(d), full orders
    __shared__ V2 Rh[8][NCP];        // R_k^l(d) of every child, l >= 0
    const int cell = c0 + blockIdx.x;
    if (cell >= c1) return;
    const int nc = nchild[cell];
    if (nc == 0) return;
    const int f = child[cell];
    const float4 gp = geo[cell];
    const int tid = threadIdx.x;
    const bool active = tid < 3 * NCP;
    const int comp = active ? tid / NCP : 0;
    int n = 0, m = 0;
    decode_nm(active ? tid % NCP : 0, n, m);
    const R inv = R(1) / R(gp.w);
    // the regular harmonics of the eight child offsets, one lane each (the
    // recursion is serial; the children's run side by side)
    if (tid < nc) {
        const float4 gc = geo[f + tid];
        V2 Rl[NCP];
        regular_harmonics<P, R, V2>((R(gc.x) - R(gp.x)) * inv, (R(gc.y) - R(gp.y)) * inv,
                                    (R(gc.z) - R(gp.z)) * inv, Rl);
#pragma unroll
        for (int q = 0; q < NCP; ++q) Rh[tid][q] = Rl[q];
    }
    V2 acc = V2{R(0), R(0)};
    for (int k = 0; k < nc; ++k) {
        const float4 gc = geo[f + k];
        __syncthreads();
        if (tid < NCP) {
            int a, b;
            decode_nm(tid, a, b);
            const V2 v = Rh[k][tid];
            Rf[a][P + b] = V2{v.x, -v.y};                                   // conj R^b
            if (b > 0) Rf[a][P - b] = (b & 1) ? V2{-v.x, -v.y} : V2{v.x, v.y};  // conj R^{-b}
        }
        const R rt = R(gc.w) * inv;
        for (int i = tid; i < 3 * NCP; i += C::THREADS) {
            const int cc = i / NCP;
            int a, b;
            decode_nm(i % NCP, a, b);
            const auto v = Mexp[((size_t)(f + k) * 3 + cc) * NCP + i % NCP];
            const R sc = powr(rt, a);
            const R vr = sc * R(v.x), vi = sc * R(v.y);
            Mf[cc][a][P + b] = V2{vr, vi};
            if (b > 0) Mf[cc][a][P - b] = (b & 1) ? V2{-vr, vi} : V2{vr, -vi};
        }
        __syncthreads();
        if (active) {
            // sum from high source degree n - kk to low: kk from 0 up
            for (int kk = 0; kk <= n; ++kk) {
                const int nm = n - kk;
                const int lo = max(-kk, m - nm), hi = min(kk, m + nm);
                for (int l = lo; l <= hi; ++l) {
                    const V2 r = Rf[kk][P + l];
                    const V2 v = Mf[comp][nm][P + m - l];
                    acc.x = fmar(r.x, v.x, fmar(-r.y, v.y, acc.x));
                    acc.y = fmar(r.x, v.y, fmar(r.y, v.x, acc.y));
                }
            }
        }
    }
    if (active) {
        auto &dst = Mexp[((size_t)cell * 3 + comp) * NCP + CIDX(n, m)];
        dst.x = (S)acc.x;
        dst.y = (S)acc.y;
    }
}

// ---------------------------------------------------------------------------
// M2L: one work-group per target cell; each thread owns one real output row
// (Re or Im of Lt_k^l, l >= 0; (P+1)^2 rows) for all three potentials, and
// the source cells of the target's list are staged in LDS two at a time
// (Sec. 3.6: a block per target cell, source cells loaded to shared memory
// and processed sequentially).
//   Lt_k^l(A) = (-1)^{k+l} lambda^{-(k+1)} sum_{n,m} Mt_n^m(B) I_{n+k}^{m-l}((c_A - c_B)/s_B),
//   lambda = s_B/s_A.
// With I^{-mu} = (-1)^mu conj(I^mu) and Mt^{-m} = (-1)^m conj(Mt^m), the terms
// of +-m combine into Re/Im rows that read two staged tables:
//   X_N^M = (Re I_N^M, -Im I_N^M),  Y_N^M = (Im I_N^M, Re I_N^M),  |M| <= 2P.
// ---------------------------------------------------------------------------
template <int P, class R = float>
struct M2LCfg {
    static constexpr int NCP = NC(P);
    static constexpr int ROWS = (P + 1) * (P + 1);
    static constexpr int THREADS = ((ROWS + 63) / 64) * 64;
    static constexpr int Q = 2 * P;
    static constexpr int IW = 4 * P + 1;                 // M in [-2P, 2P]
    static constexpr int ISZ = (Q + 1) * IW;             // per table
    static constexpr int SB = sizeof(R) == 8 ? 1 : 2;    // sources staged at once
};

template <int P, class R>
__global__ __launch_bounds__((M2LCfg<P, R>::THREADS)) void k_m2l(int ncells, const int *off, const int2 *src,
                                                               const float4 *geo,
                                                               const typename VT<R>::V2 *__restrict__ Mexp,
                                                               typename VT<R>::V2 *__restrict__ Lexp, int B,
                                                               float len) {
    using C = M2LCfg<P, R>;
    using V2 = typename VT<R>::V2;
    __shared__ V2 Xs[C::SB][C::ISZ];
    __shared__ V2 Ys[C::SB][C::ISZ];
    __shared__ V2 Ms[C::SB][3][C::NCP];
    __shared__ R lam[C::SB];
    const int tgt = blockIdx.x;
    if (tgt >= ncells) return;
    const int o0 = off[tgt], o1 = off[tgt + 1];
    if (o0 == o1) return;
    const int tid = threadIdx.x;
    for (int i = tid; i < C::SB * C::ISZ; i += C::THREADS) {
        (&Xs[0][0])[i] = V2{R(0), R(0)};
        (&Ys[0][0])[i] = V2{R(0), R(0)};
    }
    const float4 ga = geo[tgt];
    // row of this thread
    const bool active = tid < C::ROWS;
    int k = 0, l = 0;
    bool isIm = false;
    if (active) {
        k = (int)sqrtf((float)tid);
        while ((k + 1) * (k + 1) <= tid) ++k;
        while (k * k > tid) --k;
        const int j = tid - k * k;
        l = (j + 1) / 2;
        isIm = (j > 0) && ((j & 1) == 0);
    }
    const R sig = (l & 1) ? R(-1) : R(1);
    const R sp = isIm ? -sig : sig;
    R acc[3] = {R(0), R(0), R(0)};
    const int W = 2 * B + 1;
    for (int e0 = o0; e0 < o1; e0 += C::SB) {
        __syncthreads();
        // ---- stage up to SB sources ----
        for (int s = 0; s < C::SB; ++s) {
            const int e = e0 + s;
            if (e >= o1) break;
            const int2 ent = src[e];
            const float4 gb = geo[ent.x];
            const int col = tid - s * (C::Q + 1);
            if (col >= 0 && col <= C::Q) {
                const R ix = (R)(ent.y % W - B), iy = (R)((ent.y / W) % W - B), iz = (R)(ent.y / (W * W) - B);
                const R inv = R(1) / R(gb.w);
                const R dx = (R(ga.x) - R(gb.x) - ix * R(len)) * inv;
                const R dy = (R(ga.y) - R(gb.y) - iy * R(len)) * inv;
                const R dz = (R(ga.z) - R(gb.z) - iz * R(len)) * inv;
                const R r2 = dx * dx + dy * dy + dz * dz;
                const R ir2 = R(1) / r2;
                // I_M^M by the diagonal recurrence, then upward in N
                R cr = rsqr(r2), ci = R(0);
                for (int mm = 1; mm <= col; ++mm) {
                    const R f = -(R)(2 * mm - 1) * ir2;
                    const R nr = f * (dx * cr - dy * ci);
                    const R ni = f * (dx * ci + dy * cr);
                    cr = nr;
                    ci = ni;
                }
                const int M = col;
                V2 *X = Xs[s], *Y = Ys[s];
                auto put = [&](int N, R vr, R vi) {
                    X[N * C::IW + C::Q + M] = V2{vr, -vi};
                    Y[N * C::IW + C::Q + M] = V2{vi, vr};
                    if (M > 0) {
                        // I^{-M} = (-1)^M conj(I^M)
                        const R sr = (M & 1) ? -vr : vr, si = (M & 1) ? vi : -vi;
                        X[N * C::IW + C::Q - M] = V2{sr, -si};
                        Y[N * C::IW + C::Q - M] = V2{si, sr};
                    }
                };
                put(M, cr, ci);
                R pr = cr, pi = ci;
                R qr = R(0), qi = R(0);
                if (M + 1 <= C::Q) {
                    const R a0 = (R)(2 * M + 1) * dz * ir2;
                    qr = a0 * cr;
                    qi = a0 * ci;
                    put(M + 1, qr, qi);
                }
                for (int N = M + 2; N <= C::Q; ++N) {
                    const R a = (R)(2 * N - 1) * dz;
                    const R b = (R)((N - 1) * (N - 1) - M * M);
                    const R vr = (a * qr - b * pr) * ir2;
                    const R vi = (a * qi - b * pi) * ir2;
                    put(N, vr, vi);
                    pr = qr; pi = qi; qr = vr; qi = vi;
                }
            }
            for (int i = tid; i < 3 * C::NCP; i += C::THREADS)
                Ms[s][i / C::NCP][i % C::NCP] = Mexp[(size_t)ent.x * 3 * C::NCP + i];
            if (tid == 0) lam[s] = R(ga.w) / R(gb.w);  // 1/lambda
        }
        __syncthreads();
        if (!active) continue;
        for (int s = 0; s < C::SB; ++s) {
            if (e0 + s >= o1) break;
            const V2 *Wt = isIm ? Ys[s] : Xs[s];
            R a0 = R(0), a1 = R(0), a2 = R(0);
#pragma unroll
            for (int n = P; n >= 0; --n) {
                const V2 *row = Wt + (n + k) * C::IW + C::Q;
                {
                    const R w = row[-l].x;
                    a0 += Ms[s][0][CIDX(n, 0)].x * w;
                    a1 += Ms[s][1][CIDX(n, 0)].x * w;
                    a2 += Ms[s][2][CIDX(n, 0)].x * w;
                }
#pragma unroll
                for (int m = 1; m <= n; ++m) {
                    const V2 w1 = row[m - l], w2 = row[m + l];
                    const R A1 = fmar(sp, w2.x, w1.x);
                    const R B1 = fmar(sp, w2.y, w1.y);
                    const V2 m0 = Ms[s][0][CIDX(n, m)], m1 = Ms[s][1][CIDX(n, m)], m2 = Ms[s][2][CIDX(n, m)];
                    a0 = fmar(m0.x, A1, fmar(m0.y, B1, a0));
                    a1 = fmar(m1.x, A1, fmar(m1.y, B1, a1));
                    a2 = fmar(m2.x, A1, fmar(m2.y, B1, a2));
                }
            }
            const R sc = powr(lam[s], k + 1);
            acc[0] += sc * a0;
            acc[1] += sc * a1;
            acc[2] += sc * a2;
        }
    }
    if (active) {
        const R sg = ((k + l) & 1) ? R(-1) : R(1);
        const int coef = CIDX(k, l);
        for (int c = 0; c < 3; ++c) {
            R *dst = reinterpret_cast<R *>(&Lexp[((size_t)tgt * 3 + c) * C::NCP + coef]) + (isIm ? 1 : 0);
            *dst += sg * acc[c];
        }
    }
}

// ---------------------------------------------------------------------------
// L2L: one work-group per child cell of one level, one thread per
// (potential, coefficient k >= l >= 0) of the child (storage S, arithmetic R
// as in M2M); parent expansion and R(d) staged as full-order tables.
//   Lt_k^l(c) = (s_c/s_P)^{k+1} sum_{n >= k, m} Lt_n^m(P) R_{n-k}^{m-l}(d),  d = (c - P)/s_P.
// ---------------------------------------------------------------------------
template <int P, class R, class S>
__global__ __launch_bounds__((XferCfg<P>::THREADS)) void k_l2l(int c0, int c1, const int *parent, const float4 *geo,
                                                               typename VT<S>::V2 *Lexp) {
    using V2 = typename VT<R>::V2;
    using C = XferCfg<P>;
    constexpr int NCP = C::NCP, W = C::W;
    __shared__ V2 Lf[3][P + 1][W];
    __shared__ V2 Rf[P + 1][W];
    const int cell = c0 + blockIdx.x;
    if (cell >= c1) return;
    const int par = parent[cell];
    const float4 gp = geo[par], gc = geo[cell];
    const int tid = threadIdx.x;
    const R inv = R(1) / R(gp.w);
    if (tid == 0) {
        V2 Rl[NCP];
        regular_harmonics<P, R, V2>((R(gc.x) - R(gp.x)) * inv, (R(gc.y) - R(gp.y)) * inv, (R(gc.z) - R(gp.z)) * inv,
                                    Rl);
#pragma unroll
        for (int q = 0; q < NCP; ++q) {
            int a, b;
            decode_nm(q, a, b);
            const V2 v = Rl[q];
            Rf[a][P + b] = v;
            if (b > 0) Rf[a][P - b] = (b & 1) ? V2{-v.x, v.y} : V2{v.x, -v.y};
        }
    }
    for (int i = tid; i < 3 * NCP; i += C::THREADS) {
        const int cc = i / NCP;
        int a, b;
        decode_nm(i % NCP, a, b);
        const auto v = Lexp[((size_t)par * 3 + cc) * NCP + i % NCP];
        const R vr = R(v.x), vi = R(v.y);
        Lf[cc][a][P + b] = V2{vr, vi};
        if (b > 0) Lf[cc][a][P - b] = (b & 1) ? V2{-vr, vi} : V2{vr, -vi};
    }
    __syncthreads();
    if (tid >= 3 * NCP) return;
    const int comp = tid / NCP;
    int k, l;
    decode_nm(tid % NCP, k, l);
    V2 acc = V2{R(0), R(0)};
    for (int n = P; n >= k; --n) {
        const int dn = n - k;
        const int lo = max(-n, l - dn), hi = min(n, l + dn);
        for (int m = lo; m <= hi; ++m) {
            const V2 L = Lf[comp][n][P + m];
            const V2 r = Rf[dn][P + m - l];
            acc.x = fmar(L.x, r.x, fmar(-L.y, r.y, acc.x));
            acc.y = fmar(L.x, r.y, fmar(L.y, r.x, acc.y));
        }
    }
    const R sc = powr(R(gc.w) * inv, k + 1);
    auto &dst = Lexp[((size_t)cell * 3 + comp) * NCP + tid % NCP];
    dst.x = (S)((R)dst.x + sc * acc.x);
    dst.y = (S)((R)dst.y + sc * acc.y);
}

// ---------------------------------------------------------------------------
// L2P: one wave per leaf, one lane per target.  With psi = (1/s) sum Lt R(r/s)
// and the ladder identities of the scaled harmonics
//   d_z R_n^m = R_{n-1}^m,  (d_x + i d_y) R_n^m = R_{n-1}^{m+1},  (d_x - i d_y) R_n^m = -R_{n-1}^{m-1},
// the first and second derivatives of each potential are sums of Lt_n^m
// against R_{n-1} and R_{n-2}.
// ---------------------------------------------------------------------------
template <int P, class R>
__global__ __launch_bounds__(64) void k_l2p(const int *leaves, const int *start, const int *count, const float4 *geo,
                                            const typename VT<R>::V4 *rec, const typename VT<R>::V2 *Lexp,
                                            int64_t n_all, R *far_u, R *far_da, int scheme) {
    using V2 = typename VT<R>::V2;
    using V4 = typename VT<R>::V4;
    constexpr int NCP = NC(P);
    constexpr int NR = NC(P - 1);
    __shared__ V2 Ls[3][NCP];
    const int cell = leaves[blockIdx.x];
    const int lane = threadIdx.x;
    for (int i = lane; i < 3 * NCP; i += 64) Ls[i / NCP][i % NCP] = Lexp[(size_t)cell * 3 * NCP + i];
    __syncthreads();
    const float4 g = geo[cell];
    const R inv = R(1) / R(g.w);
    const int s0 = start[cell], cnt = count[cell];
    for (int b = 0; b < cnt; b += 64) {
        if (b + lane >= cnt) continue;
        const int j = s0 + b + lane;
        const V4 p = rec[2 * j];
        V2 Rl[NR];
        regular_harmonics<P - 1, R, V2>((p.x - R(g.x)) * inv, (p.y - R(g.y)) * inv, (p.z - R(g.z)) * inv, Rl);
        R G[3][3], H[3][3][3];
        for (int c = 0; c < 3; ++c) {
            R pz = R(0), pzz = R(0);
            V2 pp = V2{R(0), R(0)}, pzp = V2{R(0), R(0)}, ppp = V2{R(0), R(0)};
#pragma unroll
            for (int n = P; n >= 1; --n) {
#pragma unroll
                for (int m = -n; m <= n; ++m) {
                    const V2 L = getc(Ls[c], n, m);
                    if (m >= -(n - 1) && m <= n - 1) pz += cmul(L, getc(Rl, n - 1, m)).x;
                    if (m + 1 >= -(n - 1) && m + 1 <= n - 1) {
                        const V2 v = cmul(L, getc(Rl, n - 1, m + 1));
                        pp.x += v.x; pp.y += v.y;
                    }
                    if (n >= 2) {
                        if (m >= -(n - 2) && m <= n - 2) pzz += cmul(L, getc(Rl, n - 2, m)).x;
                        if (m + 1 >= -(n - 2) && m + 1 <= n - 2) {
                            const V2 v = cmul(L, getc(Rl, n - 2, m + 1));
                            pzp.x += v.x; pzp.y += v.y;
                        }
                        if (m + 2 >= -(n - 2) && m + 2 <= n - 2) {
                            const V2 v = cmul(L, getc(Rl, n - 2, m + 2));
                            ppp.x += v.x; ppp.y += v.y;
                        }
                    }
                }
            }
            const R i2 = inv * inv, i3 = i2 * inv;
            G[c][0] = pp.x * i2;
            G[c][1] = pp.y * i2;
            G[c][2] = pz * i2;
            const R hzz = pzz * i3;
            const R hxx = R(0.5) * (ppp.x * i3 - hzz);
            const R hyy = R(0.5) * (-ppp.x * i3 - hzz);
            const R hxy = R(0.5) * ppp.y * i3;
            const R hxz = pzp.x * i3, hyz = pzp.y * i3;
            H[c][0][0] = hxx; H[c][0][1] = hxy; H[c][0][2] = hxz;
            H[c][1][0] = hxy; H[c][1][1] = hyy; H[c][1][2] = hyz;
            H[c][2][0] = hxz; H[c][2][1] = hyz; H[c][2][2] = hzz;
        }
        // u_l = eps_{l k c} d_k psi_c ; J_kl = eps_{l n c} d_k d_n psi_c
        const R u0 = G[2][1] - G[1][2], u1 = G[0][2] - G[2][0], u2 = G[1][0] - G[0][1];
        R J[3][3];
        for (int kk = 0; kk < 3; ++kk) {
            J[kk][0] = H[2][kk][1] - H[1][kk][2];
            J[kk][1] = H[0][kk][2] - H[2][kk][0];
            J[kk][2] = H[1][kk][0] - H[0][kk][1];
        }
        const V4 at = rec[2 * j + 1];
        const R fp = R(12.566370614359172);  // alpha_i = 4 pi * stored (alpha/4pi)
        const R a[3] = {at.x * fp, at.y * fp, at.z * fp};
        R d[3];
        if (scheme == VFMM_SCHEME_TRANSPOSE) {
            for (int kk = 0; kk < 3; ++kk) d[kk] = J[kk][0] * a[0] + J[kk][1] * a[1] + J[kk][2] * a[2];
        } else {
            for (int ll = 0; ll < 3; ++ll) d[ll] = a[0] * J[0][ll] + a[1] * J[1][ll] + a[2] * J[2][ll];
        }
        far_u[j] = u0;
        far_u[n_all + j] = u1;
        far_u[2 * n_all + j] = u2;
        far_da[j] = d[0];
        far_da[n_all + j] = d[1];
        far_da[2 * n_all + j] = d[2];
    }
}

// ---------------------------------------------------------------------------
// Periodic lattice: Lt_root += T Mt_root with the precomputed real operator T
// acting on (Re, Im) of the root coefficients, for each potential.  The
// operator and the arithmetic are in R; the expansions are stored in S.
// ---------------------------------------------------------------------------
template <int P, class R, class S>
__global__ __launch_bounds__(256) void k_lattice(const R *op, const typename VT<S>::V2 *Mexp,
                                                 typename VT<S>::V2 *Lexp) {
    constexpr int NCP = NC(P);
    constexpr int D = 2 * NCP;
    __shared__ R v[3][D];
    for (int i = threadIdx.x; i < 3 * D; i += 256) {
        const int c = i / D, r = i % D;
        const auto mm = Mexp[(size_t)c * NCP + r / 2];
        v[c][r] = (r & 1) ? R(mm.y) : R(mm.x);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * D; i += 256) {
        const int c = i / D, r = i % D;
        R acc = R(0);
        for (int q = D - 1; q >= 0; --q) acc = fmar(op[(size_t)r * D + q], v[c][q], acc);
        S *dst = reinterpret_cast<S *>(&Lexp[(size_t)c * NCP + r / 2]) + (r & 1);
        *dst = (S)((R)*dst + acc);
    }
}

// zero nw 32-bit words (any count; whole float4 stores except for the tail)
__global__ __launch_bounds__(256) void k_zero(float *p, int64_t nw) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t w = 4 * i;
    if (w + 4 <= nw) {
        reinterpret_cast<float4 *>(p)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
        for (int64_t q = w; q < nw; ++q) p[q] = 0.f;
    }
}

template <int P>
static void far_prealloc_p(Ctx &c) {
    constexpr int NCP = NC(P);
    const size_t rs = c.prm.precision == VFMM_PRECISION_FP64 ? sizeof(double) : sizeof(float);
    const size_t bytes = 2 * rs * (size_t)c.ncells * 3 * NCP;
    c.Mexp.ensure(bytes);
    c.Lexp.ensure(bytes);
    c.far_u.ensure(rs * 3 * (size_t)c.n);
    c.far_da.ensure(rs * 3 * (size_t)c.n);
    if (c.prm.precision == VFMM_PRECISION_FP64) c.rec64.ensure(sizeof(double4) * 2 * (size_t)c.n);
    else {
        c.near.ensure(sizeof(float) * 24 * (size_t)c.n);  // up to four near-field parts
        c.recp.ensure(sizeof(float4) * (c.var_sigma ? 4 : 3) * (size_t)c.n);
    }
}

void far_prealloc(Ctx &c) {
    switch (c.prm.p) {
        case 4: far_prealloc_p<4>(c); break;
        case 6: far_prealloc_p<6>(c); break;
        case 8: far_prealloc_p<8>(c); break;
        case 10: far_prealloc_p<10>(c); break;
        case 12: far_prealloc_p<12>(c); break;
        default: throw Error{VFMM_EINVAL, "unsupported expansion degree p"};
    }
}

// ---------------------------------------------------------------------------
// S: storage and arithmetic type of the expansions, P2M, M2L and L2P;
// RA: arithmetic type of M2M, L2L and the lattice operator.
//   plain float32 <float, float>, mixed <float, double>, float64 <double, double>.
// ---------------------------------------------------------------------------
template <int P, class S, class RA>
static void far_field_t(Ctx &c) {
    using V2 = typename VT<S>::V2;
    using V4 = typename VT<S>::V4;
    hipStream_t s = c.stream;
    constexpr int NCP = NC(P);
    const size_t bytes = sizeof(V2) * (size_t)c.ncells * 3 * NCP;
    c.Mexp.ensure(bytes);
    c.Lexp.ensure(bytes);
    c.far_u.ensure(sizeof(S) * 3 * (size_t)c.n);
    c.far_da.ensure(sizeof(S) * 3 * (size_t)c.n);
    const V4 *rec = (sizeof(S) == 8) ? reinterpret_cast<const V4 *>(c.rec64.ptr) : reinterpret_cast<const V4 *>(c.rec.ptr);
    c.record(2 * PH_P2M_M2M);
    // a fill kernel rather than a memset, so that the evaluation can be captured in a graph
    k_zero<<<cdiv(cdiv(bytes, 16), 256), 256, 0, s>>>(c.Lexp.as<float>(), (int64_t)(bytes / 4));
    VFMM_LAUNCH_CHECK();
    k_p2m<P, S><<<c.nleaves, 64, 0, s>>>(c.leaves.as<int>(), c.c_start.as<int>(), c.c_count.as<int>(),
                                          c.c_geo.as<float4>(), rec, c.Mexp.as<V2>());
    VFMM_LAUNCH_CHECK();
    for (int l = c.depth - 1; l >= 0; --l) {
        const int c0 = c.lvl_off[l], c1 = c.lvl_off[l + 1];
        k_m2m<P, RA, S><<<c1 - c0, XferCfg<P>::THREADS, 0, s>>>(c0, c1, c.c_child.as<int>(), c.c_nchild.as<int>(),
                                                c.c_geo.as<float4>(), c.Mexp.as<V2>());
        VFMM_LAUNCH_CHECK();
    }
    c.record(2 * PH_P2M_M2M + 1);
    c.record(2 * PH_LATTICE);
    if (c.prm.periodic && c.prm.images >= 3) {
        k_lattice<P, RA, S><<<1, 256, 0, s>>>(c.lat_op.as<RA>(), c.Mexp.as<V2>(), c.Lexp.as<V2>());
        VFMM_LAUNCH_CHECK();
    }
    c.record(2 * PH_LATTICE + 1);
    c.record(2 * PH_M2L);
    if (c.n_m2l > 0 && c.m2lb_ok && sizeof(S) == 4) {
        m2lb_run(c);
    } else if (c.n_m2l > 0) {
        k_m2l<P, S><<<c.ncells, M2LCfg<P, S>::THREADS, 0, s>>>(c.ncells, c.m2l_off.as<int>(), c.m2l_src.as<int2>(),
                                                                c.c_geo.as<float4>(), c.Mexp.as<V2>(),
                                                                c.Lexp.as<V2>(), c.img_B,
                                                                c.prm.periodic ? (float)c.prm.box_len : 0.f);
        VFMM_LAUNCH_CHECK();
    }
    c.record(2 * PH_M2L + 1);
    c.record(2 * PH_L2L_L2P);
    for (int l = 1; l <= c.depth; ++l) {
        const int c0 = c.lvl_off[l], c1 = c.lvl_off[l + 1];
        k_l2l<P, RA, S><<<c1 - c0, XferCfg<P>::THREADS, 0, s>>>(c0, c1, c.c_parent.as<int>(), c.c_geo.as<float4>(),
                                                c.Lexp.as<V2>());
        VFMM_LAUNCH_CHECK();
    }
    k_l2p<P, S><<<c.nleaves, 64, 0, s>>>(c.leaves.as<int>(), c.c_start.as<int>(), c.c_count.as<int>(),
                                          c.c_geo.as<float4>(), rec, c.Lexp.as<V2>(), c.n, c.far_u.as<S>(),
                                          c.far_da.as<S>(), c.prm.scheme);
    VFMM_LAUNCH_CHECK();
    c.record(2 * PH_L2L_L2P + 1);
}

template <int P>
static void far_field_p(Ctx &c) {
    switch (c.prm.precision) {
        case VFMM_PRECISION_FP64: far_field_t<P, double, double>(c); break;
        case VFMM_PRECISION_MIXED: far_field_t<P, float, double>(c); break;
        default: far_field_t<P, float, float>(c); break;
    }
}

void far_field(Ctx &c) {
    switch (c.prm.p) {
        case 4: far_field_p<4>(c); break;
        case 6: far_field_p<6>(c); break;
        case 8: far_field_p<8>(c); break;
        case 10: far_field_p<10>(c); break;
        case 12: far_field_p<12>(c); break;
        default: throw Error{VFMM_EINVAL, "unsupported expansion degree p"};
    }
}

}  // namespace vfmm
