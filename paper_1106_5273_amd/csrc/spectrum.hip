// Shell-binned kinetic-energy spectrum E(k) of a velocity field sampled on a
// uniform n^3 lattice (Sec. 4.3: the spectrum of the velocity induced on a
// lattice of points that are not the particles).
//
// u_hat(kappa) = (1/n^3) sum_t u(x_t) exp(-2 pi i kappa.t / n) for the integer
// wavevectors kappa of the lattice (centred, |kappa_d| <= n/2), and
//     E(k) = 1/2 sum over kappa with round(|kappa|) = k of |u_hat(kappa)|^2,
// k = 0 .. round(sqrt(3) n / 2); wavenumbers are in units of 2 pi / L, and
// sum_k E(k) = 1/2 mean |u|^2.
//
// The transform is three passes of radix-2 FFTs along the lattice axes in
// float64 (one work-group per line of n points staged in LDS, twiddles from
// sincospi), so the spectrum carries float64 rounding only.  The shell sums
// are per-work-group partial bins (LDS atomics, whose order varies in the last
// bits of float64) added across work-groups in a fixed order.
#include <cstring>

#include "ctx.h"

namespace vfmm {

static constexpr int SP_TPB = 256;
static constexpr int SP_PARTS = 512;  // work-groups of the shell-binning pass

// float32 [3][n^3] -> complex float64 [3][n^3]
__global__ __launch_bounds__(SP_TPB) void k_sp_load(int64_t N, const float *ux, const float *uy, const float *uz,
                                                     double2 *d) {
    const int64_t i = (int64_t)blockIdx.x * SP_TPB + threadIdx.x;
    if (i >= N) return;
    d[i] = make_double2((double)ux[i], 0.0);
    d[N + i] = make_double2((double)uy[i], 0.0);
    d[2 * N + i] = make_double2((double)uz[i], 0.0);
}

__device__ inline unsigned bitrev(unsigned v, int bits) { return __brev(v) >> (32 - bits); }

// In-place forward FFT of every line of n points along one axis of the three
// [n][n][n] components (index i*n*n + j*n + k).  axis 2: lines along k
// (stride 1), 1: along j (stride n), 0: along i (stride n^2).  One work-group
// of n/2 threads per line (n a power of two, 2 <= n <= 1024).
__global__ void k_sp_fft(double2 *d, int n, int logn, int axis) {
    extern __shared__ double2 line[];
    const int64_t N = (int64_t)n * n * n;
    const int64_t L = blockIdx.x;  // 0 .. 3 n^2 - 1
    const int c = (int)(L / ((int64_t)n * n));
    const int64_t r = L % ((int64_t)n * n);
    const int a = (int)(r / n), b = (int)(r % n);
    int64_t base, stride;
    if (axis == 2) {
        base = (int64_t)a * n * n + (int64_t)b * n;
        stride = 1;
    } else if (axis == 1) {
        base = (int64_t)a * n * n + b;
        stride = n;
    } else {
        base = (int64_t)a * n + b;
        stride = (int64_t)n * n;
    }
    double2 *p = d + c * N + base;
    const int h = n >> 1;
    const int t = threadIdx.x;
    // bit-reversed load
    line[bitrev(t, logn)] = p[t * stride];
    line[bitrev(t + h, logn)] = p[(t + h) * stride];
    __syncthreads();
    for (int s = 1; s <= logn; ++s) {
        const int half = 1 << (s - 1);
        const int grp = t / half, pos = t % half;
        const int i0 = grp * 2 * half + pos, i1 = i0 + half;
        double sn, cs;
        sincospi(-(double)pos / (double)half, &sn, &cs);  // exp(-2 pi i pos / (2 half))
        const double2 u = line[i0], v = line[i1];
        const double2 w = make_double2(v.x * cs - v.y * sn, v.x * sn + v.y * cs);
        __syncthreads();
        line[i0] = make_double2(u.x + w.x, u.y + w.y);
        line[i1] = make_double2(u.x - w.x, u.y - w.y);
        __syncthreads();
    }
    p[t * stride] = line[t];
    p[(t + h) * stride] = line[t + h];
}

// per-work-group partial shell sums: part[g * nbins + k]
__global__ __launch_bounds__(SP_TPB) void k_sp_shells(const double2 *d, int n, int nbins, double scale, double *part) {
    extern __shared__ double bins[];
    for (int k = threadIdx.x; k < nbins; k += SP_TPB) bins[k] = 0.0;
    __syncthreads();
    const int64_t N = (int64_t)n * n * n;
    for (int64_t i = (int64_t)blockIdx.x * SP_TPB + threadIdx.x; i < N; i += (int64_t)gridDim.x * SP_TPB) {
        int kx = (int)(i / ((int64_t)n * n)), ky = (int)((i / n) % n), kz = (int)(i % n);
        kx = kx >= (n + 1) / 2 ? kx - n : kx;  // signed wavevector (the sign does not change |kappa|)
        ky = ky >= (n + 1) / 2 ? ky - n : ky;
        kz = kz >= (n + 1) / 2 ? kz - n : kz;
        const double km = sqrt((double)((int64_t)kx * kx + (int64_t)ky * ky + (int64_t)kz * kz));
        const int sh = (int)rint(km);
        double e = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double2 v = d[c * N + i];
            e += v.x * v.x + v.y * v.y;
        }
        if (sh < nbins) atomicAdd(&bins[sh], 0.5 * e * scale);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nbins; k += SP_TPB) part[(int64_t)blockIdx.x * nbins + k] = bins[k];
}

__global__ __launch_bounds__(SP_TPB) void k_sp_sum(const double *part, int nparts, int nbins, double *E) {
    const int k = blockIdx.x * SP_TPB + threadIdx.x;
    if (k >= nbins) return;
    double s = 0.0;
    for (int g = 0; g < nparts; ++g) s += part[(int64_t)g * nbins + k];
    E[k] = s;
}

// shells 0 .. round(sqrt(3) n / 2): the lattice corner |kappa| = sqrt(3) n / 2 rounds up
int spectrum_bins(int n) { return (int)std::lrint(std::sqrt(3.0) * n / 2.0) + 1; }

void energy_spectrum_run(Ctx &c, int n, const float *ux, const float *uy, const float *uz, double *E_host) {
    int logn = 0;
    while ((1 << logn) < n) ++logn;
    if (n < 2 || n > 1024 || (1 << logn) != n)
        throw Error{VFMM_EINVAL, "vfmm_energy_spectrum: n must be a power of two in [2, 1024]"};
    const int64_t N = (int64_t)n * n * n;
    const int nbins = spectrum_bins(n);
    hipStream_t s = c.stream;
    const size_t dbytes = sizeof(double2) * 3 * (size_t)N;
    const size_t pbytes = sizeof(double) * (size_t)SP_PARTS * nbins;
    c.spec.ensure(dbytes + pbytes + sizeof(double) * nbins);
    double2 *d = c.spec.as<double2>();
    double *part = reinterpret_cast<double *>(reinterpret_cast<char *>(c.spec.ptr) + dbytes);
    double *E = part + (size_t)SP_PARTS * nbins;
    k_sp_load<<<cdiv(N, SP_TPB), SP_TPB, 0, s>>>(N, ux, uy, uz, d);
    VFMM_LAUNCH_CHECK();
    for (int axis = 2; axis >= 0; --axis) {
        k_sp_fft<<<3 * n * n, n / 2, sizeof(double2) * n, s>>>(d, n, logn, axis);
        VFMM_LAUNCH_CHECK();
    }
    const double inv = 1.0 / (double)N;
    k_sp_shells<<<SP_PARTS, SP_TPB, sizeof(double) * nbins, s>>>(d, n, nbins, inv * inv, part);
    VFMM_LAUNCH_CHECK();
    k_sp_sum<<<cdiv(nbins, SP_TPB), SP_TPB, 0, s>>>(part, SP_PARTS, nbins, E);
    VFMM_LAUNCH_CHECK();
    VFMM_HIP(hipMemcpyAsync(E_host, E, sizeof(double) * nbins, hipMemcpyDeviceToHost, s));
    VFMM_HIP(hipStreamSynchronize(s));
}

}  // namespace vfmm
