// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/vfmm.h"

namespace vfmm {

// ---------------------------------------------------------------------------
// Error plumbing: kernels and launches never abort; host code converts HIP
// failures into a status and a message stored on the context.
// ---------------------------------------------------------------------------
struct Error {
    vfmm_status st;
    std::string msg;
};

#define VFMM_HIP(call)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            throw ::vfmm::Error{VFMM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define VFMM_LAUNCH_CHECK()                                                                   \
    do {                                                                                      \
        hipError_t e_ = hipGetLastError();                                                    \
        if (e_ != hipSuccess)                                                                 \
            throw ::vfmm::Error{VFMM_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_)}; \
    } while (0)

// Grow-only device buffer.  Contents are not preserved when it grows.
struct DevBuf {
    void *ptr = nullptr;
    size_t cap = 0;
    template <class T>
    T *as() const { return static_cast<T *>(ptr); }
    void ensure(size_t bytes) {
        if (bytes <= cap) return;
        if (ptr) VFMM_HIP(hipFree(ptr));
        ptr = nullptr;
        cap = 0;
        size_t want = bytes + bytes / 8 + 256;
        if (hipMalloc(&ptr, want) != hipSuccess) {
            (void)hipGetLastError();
            ptr = nullptr;
            throw Error{VFMM_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed"};
        }
        cap = want;
    }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        cap = 0;
    }
};

inline unsigned cdiv(size_t a, size_t b) { return unsigned((a + b - 1) / b); }

// Work-groups are dispatched round-robin over the 8 XCDs (work-group i runs on
// XCD i % 8), and each XCD has its own L2.  Launch 8 * g8 work-groups for g
// logical ones (g8 = ceil(g / 8)) and map physical i to logical
// (i % 8) * g8 + i / 8: each XCD then walks one contiguous range of logical
// work, so neighbouring items (Morton-ordered targets) share its L2.  Logical
// indices >= g exit at once.
constexpr int NUM_XCD = 8;
inline unsigned xcd_grid(unsigned g) { return NUM_XCD * cdiv(g, NUM_XCD); }
__device__ inline int xcd_logical(int i, int grid) {
    const int g8 = grid / NUM_XCD;
    return (i % NUM_XCD) * g8 + i / NUM_XCD;
}

// Global reduction result of the bounds pass (device, float64 accumulators).
struct Bounds {
    double lo[3], hi[3];
    double sig_min, sig_max;
    double sum_a[3];
    double sum_xa[3];  // sum (x_j - ref) x alpha_j, ref = periodic cube centre (or 0)
    double fp;         // fingerprint of positions and cores: sum_i (1 + i mod 61)(x + 3y + 5z + 7 sigma)_i
    int nonfinite;
    int outside;       // periodic: positions outside the cube
    int stale;         // evaluation: the fingerprint differs from the build's (outputs are NaN)
    int overfull;      // build: leaves above ncrit at the key-resolution depth limit
};

// Geometry of the root cube used for Morton keys and cell centres.
struct RootBox {
    float lo[3];
    float len;
};

// ---------------------------------------------------------------------------
// Coefficient layout: complex coefficients c_n^m with 0 <= m <= n <= P are
// stored at index n(n+1)/2 + m; negative orders follow from
// c_n^{-m} = (-1)^m conj(c_n^m) (real fields).  Each cell holds 3 components
// (the Laplace potentials of alpha_x, alpha_y, alpha_z) of NC(P) float2.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int NC(int P) { return (P + 1) * (P + 2) / 2; }
__host__ __device__ constexpr int CIDX(int n, int m) { return n * (n + 1) / 2 + m; }

// Scaled regular solid harmonics R_n^m(r) = r^n P_n^m(cos t) e^{i m phi} / (n+m)!
// (associated Legendre functions with the Condon-Shortley phase), for
// 0 <= m <= n <= P, by the standard three-term recurrences:
//   R_m^m = -(x + i y) / (2m) R_{m-1}^{m-1},   R_{m+1}^m = z R_m^m,
//   R_n^m = ((2n-1) z R_{n-1}^m - r^2 R_{n-2}^m) / (n^2 - m^2).
template <int P, class T, class C>
__host__ __device__ inline void regular_harmonics(T x, T y, T z, C *R) {
    const T r2 = x * x + y * y + z * z;
    T cr = T(1), ci = T(0);  // R_m^m
    for (int m = 0; m <= P; ++m) {
        if (m > 0) {
            const T f = T(-1) / T(2 * m);
            const T nr = f * (x * cr - y * ci);
            const T ni = f * (x * ci + y * cr);
            cr = nr;
            ci = ni;
        }
        R[CIDX(m, m)] = C{cr, ci};
        if (m + 1 <= P) R[CIDX(m + 1, m)] = C{z * cr, z * ci};
        T pr = cr, pi = ci, qr = z * cr, qi = z * ci;  // R_{n-2}, R_{n-1}
        for (int n = m + 2; n <= P; ++n) {
            const T inv = T(1) / T(n * n - m * m);
            const T a = T(2 * n - 1) * z;
            const T vr = (a * qr - r2 * pr) * inv;
            const T vi = (a * qi - r2 * pi) * inv;
            R[CIDX(n, m)] = C{vr, vi};
            pr = qr; pi = qi; qr = vr; qi = vi;
        }
    }
}

// Scaled irregular solid harmonics I_n^m(r) = (n-m)! P_n^m(cos t) e^{i m phi} / r^{n+1},
// 0 <= m <= n <= Q:
//   I_m^m = -(2m-1)(x + i y)/r^2 I_{m-1}^{m-1},  I_{m+1}^m = (2m+1) z / r^2 I_m^m,
//   I_n^m = ((2n-1) z I_{n-1}^m - ((n-1)^2 - m^2) I_{n-2}^m) / r^2.
// With these, 1/|x - y| = sum_{n,m} conj(R_n^m(y)) I_n^m(x) for |y| < |x|.
template <int Q, class T, class C>
__host__ __device__ inline void irregular_harmonics(T x, T y, T z, C *I) {
    const T r2 = x * x + y * y + z * z;
    const T ir2 = T(1) / r2;
    T cr = T(1) / sqrt(r2), ci = T(0);
    for (int m = 0; m <= Q; ++m) {
        if (m > 0) {
            const T f = -T(2 * m - 1) * ir2;
            const T nr = f * (x * cr - y * ci);
            const T ni = f * (x * ci + y * cr);
            cr = nr;
            ci = ni;
        }
        I[CIDX(m, m)] = C{cr, ci};
        const T a0 = T(2 * m + 1) * z * ir2;
        if (m + 1 <= Q) I[CIDX(m + 1, m)] = C{a0 * cr, a0 * ci};
        T pr = cr, pi = ci, qr = a0 * cr, qi = a0 * ci;
        for (int n = m + 2; n <= Q; ++n) {
            const T a = T(2 * n - 1) * z;
            const T b = T((n - 1) * (n - 1) - m * m);
            const T vr = (a * qr - b * pr) * ir2;
            const T vi = (a * qi - b * pi) * ir2;
            I[CIDX(n, m)] = C{vr, vi};
            pr = qr; pi = qi; qr = vr; qi = vi;
        }
    }
}

// ---------------------------------------------------------------------------
// Host-side launch wrappers (defined in the .hip files).
// ---------------------------------------------------------------------------
struct Ctx;

}  // namespace vfmm
