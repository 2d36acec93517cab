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

__device__ inline float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// c_n^m for any sign of m from the m >= 0 storage: c_n^{-m} = (-1)^m conj(c_n^m).
__device__ inline float2 getc(const float2 *a, int n, int m) {
    if (m >= 0) return a[CIDX(n, m)];
    const float2 v = a[CIDX(n, -m)];
    return (m & 1) ? make_float2(-v.x, v.y) : make_float2(v.x, -v.y);
}

__device__ inline void decode_nm(int t, int &n, int &m) {
    n = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
    while ((n + 1) * (n + 2) / 2 <= t) ++n;
    while (n * (n + 1) / 2 > t) --n;
    m = t - n * (n + 1) / 2;
}

// ---------------------------------------------------------------------------
// P2M: one wave per leaf.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(64) void k_p2m(const int *leaves, const int *start, const int *count, const float4 *geo,
                                            const float4 *rec, float2 *Mexp) {
    constexpr int NCP = NC(P);
    __shared__ float2 Rs[64][NCP];
    __shared__ float4 al[64];
    const int lane = threadIdx.x;
    const int cell = leaves[blockIdx.x];
    const float4 g = geo[cell];
    const float inv = 1.0f / g.w;
    const int s0 = start[cell], cnt = count[cell];
    constexpr int NT = (NCP + 63) / 64;
    float2 acc[NT][3];
#pragma unroll
    for (int t = 0; t < NT; ++t)
        for (int c = 0; c < 3; ++c) acc[t][c] = make_float2(0.f, 0.f);
    for (int b = 0; b < cnt; b += 64) {
        const int j = s0 + b + lane;
        if (b + lane < cnt) {
            const float4 p = rec[2 * j];
            float2 R[NCP];
            regular_harmonics<P, float, float2>((p.x - g.x) * inv, (p.y - g.y) * inv, (p.z - g.z) * inv, R);
#pragma unroll
            for (int t = 0; t < NCP; ++t) Rs[lane][t] = R[t];
            al[lane] = rec[2 * j + 1];
        } else {
            al[lane] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int t = 0; t < NCP; ++t) Rs[lane][t] = make_float2(0.f, 0.f);
        }
        __syncthreads();
        const int jmax = min(64, cnt - b);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int coef = lane + 64 * t;
            if (coef < NCP) {
                for (int jj = 0; jj < jmax; ++jj) {
                    const float2 r = Rs[jj][coef];
                    const float4 a = al[jj];
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
// M2M: one wave per parent cell of one level.
//   Mt_n^m(P) = sum_children sum_{k,l} conj(R_k^l(d)) Mt_{n-k}^{m-l}(c) (s_c/s_P)^{n-k},
//   d = (c - P)/s_P.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(64) void k_m2m(int c0, int c1, const int *child, const int *nchild, const float4 *geo,
                                            float2 *Mexp) {
    constexpr int NCP = NC(P);
    __shared__ float2 Mc[8][3][NCP];
    __shared__ float2 Rd[8][NCP];
    __shared__ float ratio[8];
    const int cell = c0 + blockIdx.x;
    if (cell >= c1) return;
    const int nc = nchild[cell];
    if (nc == 0) return;
    const int f = child[cell];
    const float4 gp = geo[cell];
    const int lane = threadIdx.x;
    if (lane < nc) {
        const float4 gc = geo[f + lane];
        const float inv = 1.0f / gp.w;
        float2 R[NCP];
        regular_harmonics<P, float, float2>((gc.x - gp.x) * inv, (gc.y - gp.y) * inv, (gc.z - gp.z) * inv, R);
        for (int t = 0; t < NCP; ++t) Rd[lane][t] = R[t];
        ratio[lane] = gc.w * inv;
    }
    for (int i = lane; i < nc * 3 * NCP; i += 64) {
        const int k = i / (3 * NCP), r = i % (3 * NCP);
        Mc[k][r / NCP][r % NCP] = Mexp[((size_t)(f + k) * 3) * NCP + r];
    }
    __syncthreads();
    for (int t = lane; t < NCP; t += 64) {
        int n, m;
        decode_nm(t, n, m);
        float2 acc[3] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
        for (int k = 0; k < nc; ++k) {
            const float rt = ratio[k];
            // sum from high source degree nm = n - kk to low: kk from 0 up
            for (int kk = 0; kk <= n; ++kk) {
                const int nm = n - kk;
                const float sc = __builtin_amdgcn_exp2f((float)nm * __log2f(rt));
                for (int l = -kk; l <= kk; ++l) {
                    const int mm = m - l;
                    if (mm < -nm || mm > nm) continue;
                    const float2 r = cconj(getc(Rd[k], kk, l));
                    for (int c = 0; c < 3; ++c) {
                        const float2 v = cmul(r, getc(Mc[k][c], nm, mm));
                        acc[c].x += sc * v.x;
                        acc[c].y += sc * v.y;
                    }
                }
            }
        }
        for (int c = 0; c < 3; ++c) Mexp[((size_t)cell * 3 + c) * NCP + t] = acc[c];
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
template <int P>
struct M2LCfg {
    static constexpr int NCP = NC(P);
    static constexpr int ROWS = (P + 1) * (P + 1);
    static constexpr int THREADS = ((ROWS + 63) / 64) * 64;
    static constexpr int Q = 2 * P;
    static constexpr int IW = 4 * P + 1;                 // M in [-2P, 2P]
    static constexpr int ISZ = (Q + 1) * IW;             // per table
    static constexpr int SB = 2;                          // sources staged at once
};

template <int P>
__global__ __launch_bounds__(M2LCfg<P>::THREADS) void k_m2l(int ncells, const int *off, const int2 *src,
                                                            const float4 *geo, const float2 *__restrict__ Mexp,
                                                            float2 *__restrict__ Lexp, int B, float len) {
    using C = M2LCfg<P>;
    __shared__ float2 Xs[C::SB][C::ISZ];
    __shared__ float2 Ys[C::SB][C::ISZ];
    __shared__ float2 Ms[C::SB][3][C::NCP];
    __shared__ float lam[C::SB];
    const int tgt = blockIdx.x;
    if (tgt >= ncells) return;
    const int o0 = off[tgt], o1 = off[tgt + 1];
    if (o0 == o1) return;
    const int tid = threadIdx.x;
    for (int i = tid; i < C::SB * C::ISZ; i += C::THREADS) {
        (&Xs[0][0])[i] = make_float2(0.f, 0.f);
        (&Ys[0][0])[i] = make_float2(0.f, 0.f);
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
    const float sig = (l & 1) ? -1.f : 1.f;
    const float sp = isIm ? -sig : sig;
    float acc[3] = {0.f, 0.f, 0.f};
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
                const float ix = (float)(ent.y % W - B), iy = (float)((ent.y / W) % W - B),
                            iz = (float)(ent.y / (W * W) - B);
                const float inv = 1.0f / gb.w;
                const float dx = (ga.x - gb.x - ix * len) * inv;
                const float dy = (ga.y - gb.y - iy * len) * inv;
                const float dz = (ga.z - gb.z - iz * len) * inv;
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float ir2 = 1.0f / r2;
                // I_M^M by the diagonal recurrence, then upward in N
                float cr = rsqrtf(r2), ci = 0.f;
                for (int mm = 1; mm <= col; ++mm) {
                    const float f = -(float)(2 * mm - 1) * ir2;
                    const float nr = f * (dx * cr - dy * ci);
                    const float ni = f * (dx * ci + dy * cr);
                    cr = nr;
                    ci = ni;
                }
                const int M = col;
                float2 *X = Xs[s], *Y = Ys[s];
                auto put = [&](int N, float vr, float vi) {
                    X[N * C::IW + C::Q + M] = make_float2(vr, -vi);
                    Y[N * C::IW + C::Q + M] = make_float2(vi, vr);
                    if (M > 0) {
                        // I^{-M} = (-1)^M conj(I^M)
                        const float sr = (M & 1) ? -vr : vr, si = (M & 1) ? vi : -vi;
                        X[N * C::IW + C::Q - M] = make_float2(sr, -si);
                        Y[N * C::IW + C::Q - M] = make_float2(si, sr);
                    }
                };
                put(M, cr, ci);
                float pr = cr, pi = ci;
                float qr = 0.f, qi = 0.f;
                if (M + 1 <= C::Q) {
                    const float a0 = (float)(2 * M + 1) * dz * ir2;
                    qr = a0 * cr;
                    qi = a0 * ci;
                    put(M + 1, qr, qi);
                }
                for (int N = M + 2; N <= C::Q; ++N) {
                    const float a = (float)(2 * N - 1) * dz;
                    const float b = (float)((N - 1) * (N - 1) - M * M);
                    const float vr = (a * qr - b * pr) * ir2;
                    const float vi = (a * qi - b * pi) * ir2;
                    put(N, vr, vi);
                    pr = qr; pi = qi; qr = vr; qi = vi;
                }
            }
            for (int i = tid; i < 3 * C::NCP; i += C::THREADS)
                Ms[s][i / C::NCP][i % C::NCP] = Mexp[(size_t)ent.x * 3 * C::NCP + i];
            if (tid == 0) lam[s] = ga.w / gb.w;  // 1/lambda
        }
        __syncthreads();
        if (!active) continue;
        for (int s = 0; s < C::SB; ++s) {
            if (e0 + s >= o1) break;
            const float2 *Wt = isIm ? Ys[s] : Xs[s];
            float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
            for (int n = P; n >= 0; --n) {
                const float2 *row = Wt + (n + k) * C::IW + C::Q;
                {
                    const float w = row[-l].x;
                    a0 += Ms[s][0][CIDX(n, 0)].x * w;
                    a1 += Ms[s][1][CIDX(n, 0)].x * w;
                    a2 += Ms[s][2][CIDX(n, 0)].x * w;
                }
#pragma unroll
                for (int m = 1; m <= n; ++m) {
                    const float2 w1 = row[m - l], w2 = row[m + l];
                    const float A1 = fmaf(sp, w2.x, w1.x);
                    const float B1 = fmaf(sp, w2.y, w1.y);
                    const float2 m0 = Ms[s][0][CIDX(n, m)], m1 = Ms[s][1][CIDX(n, m)], m2 = Ms[s][2][CIDX(n, m)];
                    a0 = fmaf(m0.x, A1, fmaf(m0.y, B1, a0));
                    a1 = fmaf(m1.x, A1, fmaf(m1.y, B1, a1));
                    a2 = fmaf(m2.x, A1, fmaf(m2.y, B1, a2));
                }
            }
            const float sc = __builtin_amdgcn_exp2f((float)(k + 1) * __log2f(lam[s]));
            acc[0] += sc * a0;
            acc[1] += sc * a1;
            acc[2] += sc * a2;
        }
    }
    if (active) {
        const float sg = ((k + l) & 1) ? -1.f : 1.f;
        const int coef = CIDX(k, l);
        for (int c = 0; c < 3; ++c) {
            float *dst = reinterpret_cast<float *>(&Lexp[((size_t)tgt * 3 + c) * C::NCP + coef]) + (isIm ? 1 : 0);
            *dst += sg * acc[c];
        }
    }
}

// ---------------------------------------------------------------------------
// L2L: one wave per child cell of one level.
//   Lt_k^l(c) = sum_{n >= k, m} Lt_n^m(P) R_{n-k}^{m-l}(d) (s_c/s_P)^{k+1},  d = (c - P)/s_P.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(64) void k_l2l(int c0, int c1, const int *parent, const float4 *geo, float2 *Lexp) {
    constexpr int NCP = NC(P);
    __shared__ float2 Lp[3][NCP];
    __shared__ float2 Rd[NCP];
    const int cell = c0 + blockIdx.x;
    if (cell >= c1) return;
    const int par = parent[cell];
    const float4 gp = geo[par], gc = geo[cell];
    const int lane = threadIdx.x;
    const float inv = 1.0f / gp.w;
    if (lane == 0) {
        float2 R[NCP];
        regular_harmonics<P, float, float2>((gc.x - gp.x) * inv, (gc.y - gp.y) * inv, (gc.z - gp.z) * inv, R);
        for (int t = 0; t < NCP; ++t) Rd[t] = R[t];
    }
    for (int i = lane; i < 3 * NCP; i += 64) Lp[i / NCP][i % NCP] = Lexp[(size_t)par * 3 * NCP + i];
    __syncthreads();
    const float rt = gc.w * inv;
    for (int t = lane; t < NCP; t += 64) {
        int k, l;
        decode_nm(t, k, l);
        const float sc = __builtin_amdgcn_exp2f((float)(k + 1) * __log2f(rt));
        float2 acc[3] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
        for (int n = P; n >= k; --n) {
            const int dn = n - k;
            for (int m = -n; m <= n; ++m) {
                const int dm = m - l;
                if (dm < -dn || dm > dn) continue;
                const float2 r = getc(Rd, dn, dm);
                for (int c = 0; c < 3; ++c) {
                    const float2 v = cmul(getc(Lp[c], n, m), r);
                    acc[c].x += v.x;
                    acc[c].y += v.y;
                }
            }
        }
        for (int c = 0; c < 3; ++c) {
            float2 &dst = Lexp[((size_t)cell * 3 + c) * NCP + t];
            dst.x += sc * acc[c].x;
            dst.y += sc * acc[c].y;
        }
    }
}

// ---------------------------------------------------------------------------
// L2P: one wave per leaf, one lane per target.  With psi = (1/s) sum Lt R(r/s)
// and the ladder identities of the scaled harmonics
//   d_z R_n^m = R_{n-1}^m,  (d_x + i d_y) R_n^m = R_{n-1}^{m+1},  (d_x - i d_y) R_n^m = -R_{n-1}^{m-1},
// the first and second derivatives of each potential are sums of Lt_n^m
// against R_{n-1} and R_{n-2}.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(64) void k_l2p(const int *leaves, const int *start, const int *count, const float4 *geo,
                                            const float4 *rec, const float2 *Lexp, int64_t n_all, float *far_u,
                                            float *far_da, int scheme) {
    constexpr int NCP = NC(P);
    constexpr int NR = NC(P - 1);
    __shared__ float2 Ls[3][NCP];
    const int cell = leaves[blockIdx.x];
    const int lane = threadIdx.x;
    for (int i = lane; i < 3 * NCP; i += 64) Ls[i / NCP][i % NCP] = Lexp[(size_t)cell * 3 * NCP + i];
    __syncthreads();
    const float4 g = geo[cell];
    const float inv = 1.0f / g.w;
    const int s0 = start[cell], cnt = count[cell];
    for (int b = 0; b < cnt; b += 64) {
        if (b + lane >= cnt) continue;
        const int j = s0 + b + lane;
        const float4 p = rec[2 * j];
        float2 R[NR];
        regular_harmonics<P - 1, float, float2>((p.x - g.x) * inv, (p.y - g.y) * inv, (p.z - g.z) * inv, R);
        float G[3][3], H[3][3][3];
        for (int c = 0; c < 3; ++c) {
            float pz = 0.f, pzz = 0.f;
            float2 pp = make_float2(0.f, 0.f), pzp = make_float2(0.f, 0.f), ppp = make_float2(0.f, 0.f);
#pragma unroll
            for (int n = P; n >= 1; --n) {
#pragma unroll
                for (int m = -n; m <= n; ++m) {
                    const float2 L = getc(Ls[c], n, m);
                    if (m >= -(n - 1) && m <= n - 1) pz += cmul(L, getc(R, n - 1, m)).x;
                    if (m + 1 >= -(n - 1) && m + 1 <= n - 1) {
                        const float2 v = cmul(L, getc(R, n - 1, m + 1));
                        pp.x += v.x; pp.y += v.y;
                    }
                    if (n >= 2) {
                        if (m >= -(n - 2) && m <= n - 2) pzz += cmul(L, getc(R, n - 2, m)).x;
                        if (m + 1 >= -(n - 2) && m + 1 <= n - 2) {
                            const float2 v = cmul(L, getc(R, n - 2, m + 1));
                            pzp.x += v.x; pzp.y += v.y;
                        }
                        if (m + 2 >= -(n - 2) && m + 2 <= n - 2) {
                            const float2 v = cmul(L, getc(R, n - 2, m + 2));
                            ppp.x += v.x; ppp.y += v.y;
                        }
                    }
                }
            }
            const float i2 = inv * inv, i3 = i2 * inv;
            G[c][0] = pp.x * i2;
            G[c][1] = pp.y * i2;
            G[c][2] = pz * i2;
            const float hzz = pzz * i3;
            const float hxx = 0.5f * (ppp.x * i3 - hzz);
            const float hyy = 0.5f * (-ppp.x * i3 - hzz);
            const float hxy = 0.5f * ppp.y * i3;
            const float hxz = pzp.x * i3, hyz = pzp.y * i3;
            H[c][0][0] = hxx; H[c][0][1] = hxy; H[c][0][2] = hxz;
            H[c][1][0] = hxy; H[c][1][1] = hyy; H[c][1][2] = hyz;
            H[c][2][0] = hxz; H[c][2][1] = hyz; H[c][2][2] = hzz;
        }
        // u_l = eps_{l k c} d_k psi_c ; J_kl = eps_{l n c} d_k d_n psi_c
        const float u0 = G[2][1] - G[1][2], u1 = G[0][2] - G[2][0], u2 = G[1][0] - G[0][1];
        float J[3][3];
        for (int kk = 0; kk < 3; ++kk) {
            J[kk][0] = H[2][kk][1] - H[1][kk][2];
            J[kk][1] = H[0][kk][2] - H[2][kk][0];
            J[kk][2] = H[1][kk][0] - H[0][kk][1];
        }
        const float4 at = rec[2 * j + 1];
        const float fp = 12.566370614359172f;  // alpha_i = 4 pi * stored (alpha/4pi)
        const float a[3] = {at.x * fp, at.y * fp, at.z * fp};
        float d[3];
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
// acting on (Re, Im) of the root coefficients, for each potential.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_lattice(const float *op, const float2 *Mexp, float2 *Lexp) {
    constexpr int NCP = NC(P);
    constexpr int D = 2 * NCP;
    __shared__ float v[3][D];
    for (int i = threadIdx.x; i < 3 * D; i += 256) {
        const int c = i / D, r = i % D;
        const float2 mm = Mexp[(size_t)c * NCP + r / 2];
        v[c][r] = (r & 1) ? mm.y : mm.x;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * D; i += 256) {
        const int c = i / D, r = i % D;
        float acc = 0.f;
        for (int q = D - 1; q >= 0; --q) acc = fmaf(op[(size_t)r * D + q], v[c][q], acc);
        float *dst = reinterpret_cast<float *>(&Lexp[(size_t)c * NCP + r / 2]) + (r & 1);
        *dst += acc;
    }
}

// ---------------------------------------------------------------------------
template <int P>
static void far_field_p(Ctx &c) {
    hipStream_t s = c.stream;
    constexpr int NCP = NC(P);
    const size_t bytes = sizeof(float2) * (size_t)c.ncells * 3 * NCP;
    c.Mexp.ensure(bytes);
    c.Lexp.ensure(bytes);
    c.far_u.ensure(sizeof(float) * 3 * (size_t)c.n);
    c.far_da.ensure(sizeof(float) * 3 * (size_t)c.n);
    if (c.ev_ok) VFMM_HIP(hipEventRecord(c.ev[2 * PH_P2M_M2M], s));
    VFMM_HIP(hipMemsetAsync(c.Lexp.ptr, 0, bytes, s));
    k_p2m<P><<<c.nleaves, 64, 0, s>>>(c.leaves.as<int>(), c.c_start.as<int>(), c.c_count.as<int>(),
                                       c.c_geo.as<float4>(), c.rec.as<float4>(), c.Mexp.as<float2>());
    VFMM_LAUNCH_CHECK();
    for (int l = c.depth - 1; l >= 0; --l) {
        const int c0 = c.lvl_off[l], c1 = c.lvl_off[l + 1];
        k_m2m<P><<<c1 - c0, 64, 0, s>>>(c0, c1, c.c_child.as<int>(), c.c_nchild.as<int>(), c.c_geo.as<float4>(),
                                         c.Mexp.as<float2>());
        VFMM_LAUNCH_CHECK();
    }
    if (c.ev_ok) VFMM_HIP(hipEventRecord(c.ev[2 * PH_P2M_M2M + 1], s));
    if (c.ev_ok) VFMM_HIP(hipEventRecord(c.ev[2 * PH_LATTICE], s));
    if (c.prm.periodic && c.prm.images >= 3) {
        k_lattice<P><<<1, 256, 0, s>>>(c.lat_op.as<float>(), c.Mexp.as<float2>(), c.Lexp.as<float2>());
        VFMM_LAUNCH_CHECK();
    }
    if (c.ev_ok) VFMM_HIP(hipEventRecord(c.ev[2 * PH_LATTICE + 1], s));
    if (c.ev_ok) VFMM_HIP(hipEventRecord(c.ev[2 * PH_M2L], s));
    if (c.n_m2l > 0) {
        k_m2l<P><<<c.ncells, M2LCfg<P>::THREADS, 0, s>>>(c.ncells, c.m2l_off.as<int>(), c.m2l_src.as<int2>(),
                                                          c.c_geo.as<float4>(), c.Mexp.as<float2>(),
                                                          c.Lexp.as<float2>(), c.img_B,
                                                          c.prm.periodic ? (float)c.prm.box_len : 0.f);
        VFMM_LAUNCH_CHECK();
    }
    if (c.ev_ok) VFMM_HIP(hipEventRecord(c.ev[2 * PH_M2L + 1], s));
    if (c.ev_ok) VFMM_HIP(hipEventRecord(c.ev[2 * PH_L2L_L2P], s));
    for (int l = 1; l <= c.depth; ++l) {
        const int c0 = c.lvl_off[l], c1 = c.lvl_off[l + 1];
        k_l2l<P><<<c1 - c0, 64, 0, s>>>(c0, c1, c.c_parent.as<int>(), c.c_geo.as<float4>(), c.Lexp.as<float2>());
        VFMM_LAUNCH_CHECK();
    }
    k_l2p<P><<<c.nleaves, 64, 0, s>>>(c.leaves.as<int>(), c.c_start.as<int>(), c.c_count.as<int>(),
                                       c.c_geo.as<float4>(), c.rec.as<float4>(), c.Lexp.as<float2>(), c.n,
                                       c.far_u.as<float>(), c.far_da.as<float>(), c.prm.scheme);
    VFMM_LAUNCH_CHECK();
    if (c.ev_ok) VFMM_HIP(hipEventRecord(c.ev[2 * PH_L2L_L2P + 1], s));
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
