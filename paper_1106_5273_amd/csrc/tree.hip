// Tree construction on the device: bounds, Morton keys, stable LSD radix sort,
// gather into Morton order, level-synchronous octree build and cell geometry.
// Sec. 3.2 of the paper (Morton ordering of 3 x 21 coordinate bits in a 64-bit
// key; at most 21 levels).
#include "ctx.h"

#include <cstring>

namespace vfmm {

static constexpr int TPB = 256;
// work-groups of the first bounds pass (each reduces a strided share of the particles)
static constexpr int BOUNDS_MAX_PARTS = 1024;

// ---------------------------------------------------------------------------
// Exclusive scan of int32 (in-place allowed).  2048 items per block, block
// totals scanned recursively.
// ---------------------------------------------------------------------------
static constexpr int SCAN_ITEMS = 8;
static constexpr int SCAN_TILE = TPB * SCAN_ITEMS;

__global__ __launch_bounds__(TPB) void k_scan_tile(const int *in, int *out, int64_t n, int *block_sums) {
    __shared__ int wsum[TPB / 64];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)tid * SCAN_ITEMS;
    int v[SCAN_ITEMS];
    int run = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t k = base + i;
        v[i] = k < n ? in[k] : 0;
        run += v[i];
    }
    // wave inclusive scan of thread totals
    const int lane = tid & 63, w = tid >> 6;
    int incl = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int woff = 0;
    for (int i = 0; i < w; ++i) woff += wsum[i];
    int ex = woff + incl - run;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t k = base + i;
        if (k < n) out[k] = ex;
        ex += v[i];
    }
    if (tid == TPB - 1 && block_sums) block_sums[blockIdx.x] = woff + incl;
}

__global__ __launch_bounds__(TPB) void k_scan_add(int *out, int64_t n, const int *offs) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    const int add = offs[blockIdx.x];
    for (int i = threadIdx.x; i < SCAN_TILE; i += TPB) {
        const int64_t k = base + i;
        if (k < n) out[k] += add;
    }
}

// Up to SCAN_FEW_TILES tiles: reduce-then-scan in two launches, each tile's
// offset summed by its own work-group from the totals of the tiles before it.
static constexpr int SCAN_FEW_TILES = 1024;

__global__ __launch_bounds__(TPB) void k_scan_tile_sums(const int *in, int64_t n, int *block_sums) {
    __shared__ int wsum[TPB / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int run = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) run += base + i < n ? in[base + i] : 0;
    for (int o = 32; o > 0; o >>= 1) run += __shfl_xor(run, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = run;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < TPB / 64; ++w) t += wsum[w];
        block_sums[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(TPB) void k_scan_tile_offset(const int *in, int *out, int64_t n, const int *block_sums) {
    __shared__ int wsum[TPB / 64];
    __shared__ int boff;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // offset of this tile: the totals of the tiles before it (at most SCAN_FEW_TILES - 1)
    int o = 0;
    for (int i = tid; i < (int)blockIdx.x; i += TPB) o += block_sums[i];
    for (int d = 32; d > 0; d >>= 1) o += __shfl_xor(o, d, 64);
    if (lane == 0) wsum[w] = o;
    __syncthreads();
    if (tid == 0) {
        int t = 0;
        for (int i = 0; i < TPB / 64; ++i) t += wsum[i];
        boff = t;
    }
    __syncthreads();  // wsum is reused below
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)tid * SCAN_ITEMS;
    int v[SCAN_ITEMS];
    int run = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t k = base + i;
        v[i] = k < n ? in[k] : 0;
        run += v[i];
    }
    int incl = run;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int woff = boff;
    for (int i = 0; i < w; ++i) woff += wsum[i];
    int ex = woff + incl - run;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t k = base + i;
        if (k < n) out[k] = ex;
        ex += v[i];
    }
}

static void scan_rec(hipStream_t s, const int *in, int *out, int64_t n, int *scratch) {
    if (n <= 0) return;
    const unsigned nb = cdiv(n, SCAN_TILE);
    if (nb == 1) {
        k_scan_tile<<<1, TPB, 0, s>>>(in, out, n, nullptr);
        VFMM_LAUNCH_CHECK();
        return;
    }
    if (nb <= (unsigned)SCAN_FEW_TILES) {  // in may alias out: the totals are taken before any write
        k_scan_tile_sums<<<nb, TPB, 0, s>>>(in, n, scratch);
        VFMM_LAUNCH_CHECK();
        k_scan_tile_offset<<<nb, TPB, 0, s>>>(in, out, n, scratch);
        VFMM_LAUNCH_CHECK();
        return;
    }
    int *sums = scratch;
    k_scan_tile<<<nb, TPB, 0, s>>>(in, out, n, sums);
    VFMM_LAUNCH_CHECK();
    scan_rec(s, sums, sums, nb, scratch + nb);
    k_scan_add<<<nb, TPB, 0, s>>>(out, n, sums);
    VFMM_LAUNCH_CHECK();
}

void scan_excl_i32(Ctx &c, const int *in, int *out, int64_t n) {
    size_t need = 0;
    for (int64_t m = cdiv(n, SCAN_TILE); m > 1; m = cdiv(m, SCAN_TILE)) need += m;
    c.scanC.ensure((need + 64) * sizeof(int));
    scan_rec(c.stream, in, out, n, c.scanC.as<int>());
}

struct IntPtrs {
    const int *p[4];
};

__global__ __launch_bounds__(64) void k_read_ints(IntPtrs src, int n, int *out) {
    const int i = threadIdx.x;
    if (i < n) out[i] = *src.p[i];
}

int *pinned_ints(Ctx &c) {
    if (!c.hpin) VFMM_HIP(hipHostMalloc((void **)&c.hpin, 64 * sizeof(int), hipHostMallocCoherent));
    return c.hpin;
}

void sync_ints(Ctx &c, int n, int *dst) {
    VFMM_HIP(hipStreamSynchronize(c.stream));
    for (int i = 0; i < n; ++i) dst[i] = c.hpin[i];
}

__global__ __launch_bounds__(64) void k_copy_words(const int *src, int n, int *out) {
    const int i = threadIdx.x;
    if (i < n) out[i] = src[i];
}

void read_words(Ctx &c, const void *src, size_t bytes, void *dst) {
    if (bytes == 0 || bytes > 64 * sizeof(int) || bytes % sizeof(int)) throw Error{VFMM_EINVAL, "read_words: size"};
    const int n = (int)(bytes / sizeof(int));
    int *hp = pinned_ints(c);
    k_copy_words<<<1, 64, 0, c.stream>>>(static_cast<const int *>(src), n, hp);
    VFMM_LAUNCH_CHECK();
    VFMM_HIP(hipStreamSynchronize(c.stream));
    std::memcpy(dst, hp, bytes);
}

void read_ints(Ctx &c, std::initializer_list<const int *> src, int *dst) {
    if (src.size() == 0 || src.size() > 4) throw Error{VFMM_EINVAL, "read_ints: one to four values"};
    int *hp = pinned_ints(c);
    IntPtrs a{};
    int n = 0;
    for (const int *p : src) a.p[n++] = p;
    k_read_ints<<<1, 64, 0, c.stream>>>(a, n, hp);
    VFMM_LAUNCH_CHECK();
    sync_ints(c, n, dst);
}

// ---------------------------------------------------------------------------
// Bounds: min/max of positions, min/max core, float64 sums of alpha and of
// (x - ref) x alpha, non-finite and out-of-cube counts.  Deterministic two
// stage reduction.
// ---------------------------------------------------------------------------
struct BAcc {
    double lo[3], hi[3], smin, smax, sa[3], sxa[3], fp;
    int nf, out;
};

__device__ inline void bacc_init(BAcc &a) {
    for (int d = 0; d < 3; ++d) {
        a.lo[d] = 1e300; a.hi[d] = -1e300; a.sa[d] = 0; a.sxa[d] = 0;
    }
    a.smin = 1e300; a.smax = -1e300; a.fp = 0; a.nf = 0; a.out = 0;
}

__device__ inline void bacc_merge(BAcc &a, const BAcc &b) {
    for (int d = 0; d < 3; ++d) {
        a.lo[d] = fmin(a.lo[d], b.lo[d]); a.hi[d] = fmax(a.hi[d], b.hi[d]);
        a.sa[d] += b.sa[d]; a.sxa[d] += b.sxa[d];
    }
    a.smin = fmin(a.smin, b.smin); a.smax = fmax(a.smax, b.smax);
    a.fp += b.fp;
    a.nf += b.nf; a.out += b.out;
}

struct BoundsArgs {
    const float *x, *y, *z, *s, *ax, *ay, *az;
    int64_t n;
    int with_alpha, periodic;
    double ref[3];
    double plo[3], plen;
    int check_fp;  // evaluation: compare the fingerprint with fp_ref (the build's)
    double fp_ref;
};

__global__ __launch_bounds__(TPB) void k_bounds_partial(BoundsArgs A, BAcc *part) {
    __shared__ BAcc sh[TPB];
    BAcc a;
    bacc_init(a);
    for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < A.n; i += (int64_t)gridDim.x * TPB) {
        const double p[3] = {A.x[i], A.y[i], A.z[i]};
        const double sg = A.s[i];
        bool fin = isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]) && isfinite(sg) && sg > 0.0;
        double al[3] = {0, 0, 0};
        if (A.with_alpha) {
            al[0] = A.ax[i]; al[1] = A.ay[i]; al[2] = A.az[i];
            fin = fin && isfinite(al[0]) && isfinite(al[1]) && isfinite(al[2]);
        }
        a.fp += (double)(1 + i % 61) * (p[0] + 3.0 * p[1] + 5.0 * p[2] + 7.0 * sg);
        if (!fin) { a.nf++; continue; }
        for (int d = 0; d < 3; ++d) { a.lo[d] = fmin(a.lo[d], p[d]); a.hi[d] = fmax(a.hi[d], p[d]); }
        a.smin = fmin(a.smin, sg); a.smax = fmax(a.smax, sg);
        if (A.periodic || A.plen > 0.0) {  // the periodic cell, or a caller-given root cube
            for (int d = 0; d < 3; ++d)
                if (!(p[d] >= A.plo[d] && p[d] < A.plo[d] + A.plen)) { a.out++; break; }
        }
        if (A.with_alpha) {
            const double r[3] = {p[0] - A.ref[0], p[1] - A.ref[1], p[2] - A.ref[2]};
            for (int d = 0; d < 3; ++d) a.sa[d] += al[d];
            a.sxa[0] += r[1] * al[2] - r[2] * al[1];
            a.sxa[1] += r[2] * al[0] - r[0] * al[2];
            a.sxa[2] += r[0] * al[1] - r[1] * al[0];
        }
    }
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int o = TPB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) bacc_merge(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(TPB) void k_bounds_final(const BAcc *part, int np, int check_fp, double fp_ref,
                                                      Bounds *res) {
    __shared__ BAcc sh[TPB];
    BAcc a;
    bacc_init(a);
    for (int i = threadIdx.x; i < np; i += TPB) bacc_merge(a, part[i]);
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int o = TPB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) bacc_merge(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        Bounds b;
        for (int d = 0; d < 3; ++d) {
            b.lo[d] = sh[0].lo[d]; b.hi[d] = sh[0].hi[d];
            b.sum_a[d] = sh[0].sa[d]; b.sum_xa[d] = sh[0].sxa[d];
        }
        b.sig_min = sh[0].smin; b.sig_max = sh[0].smax;
        b.fp = sh[0].fp;
        b.nonfinite = sh[0].nf; b.outside = sh[0].out;
        // the two-stage sum is deterministic: equal inputs give a bitwise equal fingerprint
        b.stale = (check_fp && !(sh[0].fp == fp_ref)) ? 1 : 0;
        b.overfull = 0;
        *res = b;
    }
}

size_t bounds_scratch_bytes() { return sizeof(BAcc) * BOUNDS_MAX_PARTS; }

void launch_bounds(const Ctx &c, hipStream_t s, int64_t n, const float *x, const float *y, const float *z,
                   const float *sigma, const float *ax, const float *ay, const float *az, bool with_alpha,
                   bool check_fp, double fp_ref, void *part, Bounds *res) {
    BoundsArgs A{};
    A.x = x; A.y = y; A.z = z; A.s = sigma; A.ax = ax; A.ay = ay; A.az = az;
    A.n = n;
    A.with_alpha = with_alpha ? 1 : 0;
    A.periodic = c.prm.periodic;
    for (int d = 0; d < 3; ++d) {
        A.plo[d] = c.prm.box_lo[d];
        A.ref[d] = c.prm.periodic ? c.prm.box_lo[d] + 0.5 * c.prm.box_len : 0.0;
    }
    A.plen = c.prm.box_len;
    const int nb = (int)std::min<int64_t>(BOUNDS_MAX_PARTS, std::max<int64_t>(1, cdiv(n, TPB)));
    k_bounds_partial<<<nb, TPB, 0, s>>>(A, (BAcc *)part);
    VFMM_LAUNCH_CHECK();
    k_bounds_final<<<1, TPB, 0, s>>>((const BAcc *)part, nb, check_fp ? 1 : 0, fp_ref, res);
    VFMM_LAUNCH_CHECK();
}

void compute_bounds(Ctx &c, int64_t n, const float *x, const float *y, const float *z, const float *sigma,
                    const float *ax, const float *ay, const float *az, bool with_alpha) {
    c.bpart.ensure(bounds_scratch_bytes());
    c.bres.ensure(sizeof(Bounds));
    // an evaluation checks its positions and cores against those of the build
    launch_bounds(c, c.stream, n, x, y, z, sigma, ax, ay, az, with_alpha, with_alpha, c.build_fp, c.bpart.ptr,
                  c.bres.as<Bounds>());
}

// ---------------------------------------------------------------------------
// Morton keys: 21 bits per axis, bit 3b+2 = x bit b, 3b+1 = y bit b, 3b = z bit b.
// ---------------------------------------------------------------------------
__device__ inline uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// Batched problems: the problem id occupies the bits above 3*KL (KL key
// levels per axis), so each problem's particles stay contiguous after the
// sort and every problem gets its own root cube.
__global__ __launch_bounds__(TPB) void k_morton(const float *x, const float *y, const float *z, int64_t n,
                                                const RootBox *boxes, const int *pid, int KL, uint64_t *keys,
                                                uint32_t *vals) {
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= n) return;
    const int b = pid ? pid[i] : 0;
    const RootBox box = boxes[b];
    const float cells = (float)(1u << KL);
    const float sc = cells / box.len;
    const float p[3] = {x[i], y[i], z[i]};
    uint32_t q[3];
    for (int d = 0; d < 3; ++d) {
        float t = floorf((p[d] - box.lo[d]) * sc);
        t = fminf(fmaxf(t, 0.0f), cells - 1.0f);
        q[d] = (uint32_t)t;
    }
    keys[i] = ((uint64_t)b << (3 * KL)) | (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
    vals[i] = (uint32_t)i;
}

// problem id of every particle and per-problem bounding cubes
__global__ __launch_bounds__(TPB) void k_problem_ids(const int64_t *off, int *pid) {
    const int b = blockIdx.x;
    for (int64_t i = off[b] + threadIdx.x; i < off[b + 1]; i += TPB) pid[i] = b;
}

__global__ __launch_bounds__(TPB) void k_problem_boxes(const int64_t *off, const float *x, const float *y,
                                                       const float *z, RootBox *boxes) {
    __shared__ float lo[3][TPB], hi[3][TPB];
    const int b = blockIdx.x;
    float l[3] = {3.4e38f, 3.4e38f, 3.4e38f}, h[3] = {-3.4e38f, -3.4e38f, -3.4e38f};
    for (int64_t i = off[b] + threadIdx.x; i < off[b + 1]; i += TPB) {
        const float p[3] = {x[i], y[i], z[i]};
        for (int d = 0; d < 3; ++d) { l[d] = fminf(l[d], p[d]); h[d] = fmaxf(h[d], p[d]); }
    }
    for (int d = 0; d < 3; ++d) { lo[d][threadIdx.x] = l[d]; hi[d][threadIdx.x] = h[d]; }
    __syncthreads();
    for (int o = TPB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int d = 0; d < 3; ++d) {
                lo[d][threadIdx.x] = fminf(lo[d][threadIdx.x], lo[d][threadIdx.x + o]);
                hi[d][threadIdx.x] = fmaxf(hi[d][threadIdx.x], hi[d][threadIdx.x + o]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        float len = 0.f, c[3];
        for (int d = 0; d < 3; ++d) {
            len = fmaxf(len, hi[d][0] - lo[d][0]);
            c[d] = 0.5f * (lo[d][0] + hi[d][0]);
        }
        len = len * (1.0f + 1e-5f) + 1e-6f * fmaxf(fabsf(c[0]), fmaxf(fabsf(c[1]), fabsf(c[2]))) + 1e-30f;
        RootBox r;
        for (int d = 0; d < 3; ++d) r.lo[d] = c[d] - 0.5f * len;
        r.len = len;
        boxes[b] = r;
    }
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (uint64 key, uint32 value), 8-bit digits.
// Ranking inside a tile uses wave ballots over the digit bits, so equal
// digits keep their input order: the sort is stable and deterministic.
// ---------------------------------------------------------------------------
static constexpr int RS_ITEMS = 16;
static constexpr int RS_TILE = TPB * RS_ITEMS;

__global__ __launch_bounds__(TPB) void k_rs_hist(const uint64_t *keys, int64_t n, int shift, int *hist, int nblk) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int64_t k = base + (int64_t)i * TPB + threadIdx.x;
        if (k < n) atomicAdd(&h[(keys[k] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(TPB) void k_rs_scatter(const uint64_t *kin, const uint32_t *vin, uint64_t *kout,
                                                    uint32_t *vout, int64_t n, int shift, const int *offs,
                                                    int nblk) {
    __shared__ int base_off[256];
    __shared__ int wcnt[TPB / 64][256];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    base_off[tid] = offs[tid * nblk + blockIdx.x];
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ITEMS; ++r) {
        for (int j = 0; j < TPB / 64; ++j) wcnt[j][tid] = 0;
        const int64_t k = base + (int64_t)r * TPB + tid;
        const bool valid = k < n;
        const uint64_t key = valid ? kin[k] : 0ull;
        const uint32_t val = valid ? vin[k] : 0u;
        const int d = (int)((key >> shift) & 255);
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t mb = __ballot((d >> b) & 1);
            m &= ((d >> b) & 1) ? mb : ~mb;
        }
        const int rank = __popcll(m & lt);
        __syncthreads();
        if (valid && rank == 0) wcnt[w][d] = __popcll(m);
        __syncthreads();
        if (valid) {
            int pre = 0;
            for (int j = 0; j < w; ++j) pre += wcnt[j][d];
            const int pos = base_off[d] + pre + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        int add = 0;
        for (int j = 0; j < TPB / 64; ++j) add += wcnt[j][tid];
        base_off[tid] += add;
        __syncthreads();
    }
}

// Sorts keyA/valA (n items, significant bits [0, nbits)); result ends in keyA/valA.
static void radix_sort(Ctx &c, DevBuf &kA, DevBuf &vA, DevBuf &kB, DevBuf &vB, int64_t n, int nbits) {
    if (n <= 1) return;
    const int nblk = (int)cdiv(n, RS_TILE);
    c.hist.ensure(sizeof(int) * 256 * (size_t)nblk);
    kB.ensure(sizeof(uint64_t) * n);
    vB.ensure(sizeof(uint32_t) * n);
    const int passes = (nbits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        k_rs_hist<<<nblk, TPB, 0, c.stream>>>(kA.as<uint64_t>(), n, shift, c.hist.as<int>(), nblk);
        VFMM_LAUNCH_CHECK();
        scan_excl_i32(c, c.hist.as<int>(), c.hist.as<int>(), 256LL * nblk);
        k_rs_scatter<<<nblk, TPB, 0, c.stream>>>(kA.as<uint64_t>(), vA.as<uint32_t>(), kB.as<uint64_t>(),
                                                 vB.as<uint32_t>(), n, shift, c.hist.as<int>(), nblk);
        VFMM_LAUNCH_CHECK();
        std::swap(kA, kB);
        std::swap(vA, vB);
    }
}

void sort_pairs_u64(Ctx &c, DevBuf &kA, DevBuf &vA, DevBuf &kB, DevBuf &vB, int64_t n, int nbits) {
    radix_sort(c, kA, vA, kB, vB, n, nbits);
}

// ---------------------------------------------------------------------------
// Gather into Morton order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TPB) void k_gather_pos(const uint32_t *perm, int64_t n, const float *x, const float *y,
                                                    const float *z, const float *s, float4 *rec, int *perm_out) {
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= n) return;
    const uint32_t j = perm[i];
    rec[2 * i] = make_float4(x[j], y[j], z[j], s[j]);
    perm_out[i] = (int)j;
}

__global__ __launch_bounds__(TPB) void k_gather_alpha(const int *perm, int64_t n, const float *ax, const float *ay,
                                                      const float *az, float4 *rec) {
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= n) return;
    const int j = perm[i];
    const float k = 0.0795774715459476679f;  // 1/(4 pi): the Green's function factor of G
    rec[2 * i + 1] = make_float4(ax[j] * k, ay[j] * k, az[j] * k, 0.0f);
}

void gather_strengths(Ctx &c, const float *ax, const float *ay, const float *az, const float *) {
    if (c.n == 0) return;
    k_gather_alpha<<<cdiv(c.n, TPB), TPB, 0, c.stream>>>(c.perm.as<int>(), c.n, ax, ay, az, c.rec.as<float4>());
    VFMM_LAUNCH_CHECK();
}

// float64 records for the float64 form: positions from the sorted float32
// records (exact), c = 1/(sqrt 2 sigma) of each core, strengths from the
// caller's arrays scaled in float64
__global__ __launch_bounds__(TPB) void k_gather_rec64(const int *perm, int64_t n, const float *ax, const float *ay,
                                                      const float *az, const float4 *rec, double4 *rec64) {
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= n) return;
    const int j = perm[i];
    const double k = 0.079577471545947667884;  // 1/(4 pi)
    const float4 p = rec[2 * i];
    rec64[2 * i] = make_double4(p.x, p.y, p.z, 0.70710678118654752440 / (double)p.w);  // 1/(sqrt 2 sigma)
    rec64[2 * i + 1] = make_double4((double)ax[j] * k, (double)ay[j] * k, (double)az[j] * k, 0.0);
}

void gather_records64(Ctx &c, const float *ax, const float *ay, const float *az) {
    if (c.n == 0) return;
    c.rec64.ensure(sizeof(double4) * 2 * (size_t)c.n);
    k_gather_rec64<<<cdiv(c.n, TPB), TPB, 0, c.stream>>>(c.perm.as<int>(), c.n, ax, ay, az, c.rec.as<float4>(),
                                                         c.rec64.as<double4>());
    VFMM_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Separate target points: within every leaf the sources (caller index below
// n_src) are moved in front of the targets (a stable partition of the leaf's
// range, which leaves every cell's range unchanged), and each leaf records
// its number of sources, so that the near field never reads a target as a
// source.  One thread per leaf writes the new order of its range.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TPB) void k_leaf_partition(int nl, const int *leaves, const int *start, const int *count,
                                                        const int *perm, int64_t n_src, uint32_t *order,
                                                        int *nsrc) {
    const int l = blockIdx.x * TPB + threadIdx.x;
    if (l >= nl) return;
    const int cell = leaves[l];
    const int s0 = start[cell], cnt = count[cell];
    int w = s0;
    for (int i = s0; i < s0 + cnt; ++i)
        if (perm[i] < n_src) order[w++] = (uint32_t)i;
    nsrc[cell] = w - s0;
    for (int i = s0; i < s0 + cnt; ++i)
        if (perm[i] >= n_src) order[w++] = (uint32_t)i;
}

__global__ __launch_bounds__(TPB) void k_apply_order(int64_t n, const uint32_t *order, const int *perm_in,
                                                     const float4 *rec_in, const uint64_t *key_in, int *perm_out,
                                                     float4 *pos_out, uint64_t *key_out) {
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= n) return;
    const uint32_t j = order[i];
    perm_out[i] = perm_in[j];
    pos_out[i] = rec_in[2 * (size_t)j];
    key_out[i] = key_in[j];
}

void partition_sources(Ctx &c, int64_t n_src) {
    hipStream_t s = c.stream;
    const int64_t n = c.n;
    c.c_nsrc.ensure(sizeof(int) * (size_t)c.ncells);
    VFMM_HIP(hipMemsetAsync(c.c_nsrc.ptr, 0, sizeof(int) * (size_t)c.ncells, s));
    c.valB.ensure(sizeof(uint32_t) * n);
    c.keyB.ensure(sizeof(uint64_t) * n);
    c.part.ensure(sizeof(int) * n + 16 + sizeof(float4) * n);
    uint32_t *order = c.valB.as<uint32_t>();
    k_leaf_partition<<<cdiv(c.nleaves, TPB), TPB, 0, s>>>(c.nleaves, c.leaves.as<int>(), c.c_start.as<int>(),
                                                           c.c_count.as<int>(), c.perm.as<int>(), n_src, order,
                                                           c.c_nsrc.as<int>());
    VFMM_LAUNCH_CHECK();
    // gather into scratch, then copy back (perm, position records, keys)
    int *perm2 = c.part.as<int>();
    float4 *rec2 = reinterpret_cast<float4 *>(c.part.as<char>() + ((sizeof(int) * n + 15) / 16) * 16);
    k_apply_order<<<cdiv(n, TPB), TPB, 0, s>>>(n, order, c.perm.as<int>(), c.rec.as<float4>(), c.keyA.as<uint64_t>(),
                                                perm2, rec2, c.keyB.as<uint64_t>());
    VFMM_LAUNCH_CHECK();
    VFMM_HIP(hipMemcpyAsync(c.perm.ptr, perm2, sizeof(int) * n, hipMemcpyDeviceToDevice, s));
    VFMM_HIP(hipMemcpy2DAsync(c.rec.ptr, 2 * sizeof(float4), rec2, sizeof(float4), sizeof(float4), n,
                              hipMemcpyDeviceToDevice, s));
    VFMM_HIP(hipMemcpyAsync(c.keyA.ptr, c.keyB.ptr, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
}

// ---------------------------------------------------------------------------
// Octree, level by level.  A cell at level l holds a contiguous range of the
// sorted keys sharing their top 3l bits; it is split while it holds more than
// ncrit particles and l < 21.  Children of a cell are contiguous.
// ---------------------------------------------------------------------------
__device__ inline int octant_at(uint64_t key, int lchild, int KL) { return (int)((key >> (3 * (KL - lchild))) & 7); }

// Eight lanes per cell, one per octant o: the end of octant o's run in the
// cell's key range (the first index whose octant is > o) by a binary search;
// the octants are non-decreasing along the range, so the cell's children are
// the non-empty runs, in octant order.  The lanes of a cell are consecutive
// lanes of one wave.
__device__ inline int octant_end(const uint64_t *keys, int s, int end, int o, int lchild, int KL) {
    int a = s, b = end;
    while (a < b) {
        const int mid = (a + b) >> 1;
        if (octant_at(keys[mid], lchild, KL) <= o) a = mid + 1; else b = mid;
    }
    return a;
}

__global__ __launch_bounds__(TPB) void k_count_children(int c0, int c1, int lvl, int ncrit, int KL, const int *start,
                                                        const int *count, const uint64_t *keys, int *nchild,
                                                        Bounds *res) {
    const int g = blockIdx.x * TPB + threadIdx.x;
    const int cell = c0 + g / 8, o = g % 8;
    const bool valid = cell < c1;
    const int s = valid ? start[cell] : 0, cnt = valid ? count[cell] : 0;
    // keys resolve no finer than level KL: such a leaf keeps all its particles
    // (coincident or nearly coincident ones), which the near field handles
    if (valid && o == 0 && cnt > ncrit && lvl >= KL) atomicAdd(&res->overfull, 1);
    const bool split = valid && cnt > ncrit && lvl < KL;
    const int e = split ? octant_end(keys, s, s + cnt, o, lvl + 1, KL) : s;
    const int prev = __shfl_up(e, 1, 8);
    const bool nonempty = split && e > (o == 0 ? s : prev);
    const unsigned long long bal = __ballot(nonempty);
    const int sh = (threadIdx.x & 63) & ~7;
    if (valid && o == 0) nchild[cell - c0] = __popcll((bal >> sh) & 0xffull);
}

__global__ __launch_bounds__(TPB) void k_make_children(int c0, int c1, int lvl, int cnext, int KL, const int *start,
                                                       const int *count, const uint64_t *keys, const int *choff,
                                                       const int *nchild_l, int *c_start, int *c_count,
                                                       int *c_parent, int *c_child, int *c_nchild, int *c_level) {
    const int g = blockIdx.x * TPB + threadIdx.x;
    const int cell = c0 + g / 8, o = g % 8;
    const bool valid = cell < c1;
    const int nc = valid ? nchild_l[cell - c0] : 0;
    const int s = valid ? start[cell] : 0, end = valid ? s + count[cell] : 0;
    const int e = nc > 0 ? octant_end(keys, s, end, o, lvl + 1, KL) : s;
    const int prev = __shfl_up(e, 1, 8);
    const int lo = o == 0 ? s : prev;
    const bool nonempty = nc > 0 && e > lo;
    const unsigned long long bal = __ballot(nonempty);
    const int sh = (threadIdx.x & 63) & ~7;
    const int first = valid ? cnext + choff[cell - c0] : 0;
    if (valid && o == 0) {
        c_nchild[cell] = nc;
        c_child[cell] = nc == 0 ? -1 : first;
    }
    if (nonempty) {
        const int ch = first + __popcll((bal >> sh) & ((1ull << o) - 1));  // non-empty octants before o
        c_start[ch] = lo;
        c_count[ch] = e - lo;
        c_parent[ch] = cell;
        c_level[ch] = lvl + 1;
    }
}

// Centres from the key prefix of the first particle; leaves get their tight
// radius (max distance of a particle from the cube centre) and bounding box.
__global__ __launch_bounds__(TPB) void k_leaf_geometry(int ncell, const RootBox *boxes, int KL, const int *start,
                                                       const int *count,
                                                       const int *level, const int *nchild, const uint64_t *keys,
                                                       const float4 *rec, float4 *geo, float *rad, float4 *blo,
                                                       float4 *bhi) {
    const int cell = blockIdx.x * TPB + threadIdx.x;
    if (cell >= ncell) return;
    const int lvl = level[cell];
    const int s = start[cell];
    const uint64_t key = keys[s];
    const RootBox box = boxes[(int)(key >> (3 * KL))];
    // cell integer coordinates at this level
    uint32_t q[3] = {0, 0, 0};
    for (int b = 0; b < lvl; ++b) {
        const int o = octant_at(key, b + 1, KL);
        q[0] = (q[0] << 1) | ((o >> 2) & 1);
        q[1] = (q[1] << 1) | ((o >> 1) & 1);
        q[2] = (q[2] << 1) | (o & 1);
    }
    const double size = (double)box.len / (double)(1u << lvl);
    float4 g;
    g.x = (float)(box.lo[0] + (q[0] + 0.5) * size);
    g.y = (float)(box.lo[1] + (q[1] + 0.5) * size);
    g.z = (float)(box.lo[2] + (q[2] + 0.5) * size);
    g.w = (float)size;
    geo[cell] = g;
    if (nchild[cell] == 0) {
        float r2 = 0.f;
        float4 lo = make_float4(3.4e38f, 3.4e38f, 3.4e38f, 0.f), hi = make_float4(-3.4e38f, -3.4e38f, -3.4e38f, 0.f);
        const int cnt = count[cell];
        for (int i = s; i < s + cnt; ++i) {
            const float4 p = rec[2 * i];
            const float dx = p.x - g.x, dy = p.y - g.y, dz = p.z - g.z;
            r2 = fmaxf(r2, dx * dx + dy * dy + dz * dz);
            lo.x = fminf(lo.x, p.x); lo.y = fminf(lo.y, p.y); lo.z = fminf(lo.z, p.z);
            hi.x = fmaxf(hi.x, p.x); hi.y = fmaxf(hi.y, p.y); hi.z = fmaxf(hi.z, p.z);
            hi.w = fmaxf(hi.w, p.w);  // the cell's largest core
        }
        // round the radius up by a few ulps so float rounding never makes it short
        rad[cell] = sqrtf(r2) * (1.0f + 4.0e-7f);
        blo[cell] = lo;
        bhi[cell] = hi;
    }
}

// Internal cells, one level at a time bottom-up: radius bounded by the
// children's spheres, bounding box the union of the children's boxes, largest
// core (the box's fourth component) the largest of the children's.
__global__ __launch_bounds__(TPB) void k_internal_geometry(int c0, int c1, const int *child, const int *nchild,
                                                           const float4 *geo, float *rad, float4 *blo, float4 *bhi) {
    const int cell = c0 + blockIdx.x * TPB + threadIdx.x;
    if (cell >= c1) return;
    const int nc = nchild[cell];
    if (nc == 0) return;
    const float4 g = geo[cell];
    float r = 0.f;
    float4 lo = make_float4(3.4e38f, 3.4e38f, 3.4e38f, 0.f), hi = make_float4(-3.4e38f, -3.4e38f, -3.4e38f, 0.f);
    const int f = child[cell];
    for (int k = 0; k < nc; ++k) {
        const float4 cg = geo[f + k];
        const float dx = cg.x - g.x, dy = cg.y - g.y, dz = cg.z - g.z;
        r = fmaxf(r, sqrtf(dx * dx + dy * dy + dz * dz) + rad[f + k]);
        const float4 cl = blo[f + k], chh = bhi[f + k];
        lo.x = fminf(lo.x, cl.x); lo.y = fminf(lo.y, cl.y); lo.z = fminf(lo.z, cl.z);
        hi.x = fmaxf(hi.x, chh.x); hi.y = fmaxf(hi.y, chh.y); hi.z = fmaxf(hi.z, chh.z);
        hi.w = fmaxf(hi.w, chh.w);
    }
    rad[cell] = r * (1.0f + 4.0e-7f);
    blo[cell] = lo;
    bhi[cell] = hi;
}

__global__ __launch_bounds__(TPB) void k_leaf_flags(int ncell, const int *nchild, int *flag) {
    const int cell = blockIdx.x * TPB + threadIdx.x;
    if (cell < ncell) flag[cell] = nchild[cell] == 0 ? 1 : 0;
}

__global__ __launch_bounds__(TPB) void k_leaf_compact(int ncell, const int *nchild, const int *pos, int *leaves) {
    const int cell = blockIdx.x * TPB + threadIdx.x;
    if (cell < ncell && nchild[cell] == 0) leaves[pos[cell]] = cell;
}

__global__ __launch_bounds__(TPB) void k_roots(int nprob, const int64_t *off, int n, int *start, int *count,
                                               int *parent, int *level) {
    const int b = blockIdx.x * TPB + threadIdx.x;
    if (b >= nprob) return;
    start[b] = off ? (int)off[b] : 0;
    count[b] = off ? (int)(off[b + 1] - off[b]) : n;
    parent[b] = -1;
    level[b] = 0;
}

// grow a cell array keeping its first `used` elements
static void grow_keep(Ctx &c, DevBuf &b, size_t bytes, size_t used) {
    if (bytes <= b.cap) return;
    DevBuf nb;
    nb.ensure(bytes * 2);
    if (used) VFMM_HIP(hipMemcpyAsync(nb.ptr, b.ptr, used, hipMemcpyDeviceToDevice, c.stream));
    VFMM_HIP(hipStreamSynchronize(c.stream));
    b.release();
    b = nb;
}

void build_tree(Ctx &c, int64_t n, const float *x, const float *y, const float *z, const float *sigma) {
    hipStream_t s = c.stream;
    // ---- Morton keys and sort ----
    c.keyA.ensure(sizeof(uint64_t) * n);
    c.valA.ensure(sizeof(uint32_t) * n);
    const int nprob = c.nprob;
    int pbits = 0;
    while ((1 << pbits) < nprob) ++pbits;
    c.key_levels = nprob > 1 ? (63 - pbits) / 3 : 21;
    const int KL = c.key_levels;
    c.pbox.ensure(sizeof(RootBox) * (size_t)nprob);
    int *pid = nullptr;
    if (nprob > 1) {
        c.pid.ensure(sizeof(int) * n);
        pid = c.pid.as<int>();
        k_problem_ids<<<nprob, TPB, 0, s>>>(c.poff.as<int64_t>(), pid);
        VFMM_LAUNCH_CHECK();
        k_problem_boxes<<<nprob, TPB, 0, s>>>(c.poff.as<int64_t>(), x, y, z, c.pbox.as<RootBox>());
        VFMM_LAUNCH_CHECK();
    } else {
        VFMM_HIP(hipMemcpyAsync(c.pbox.ptr, &c.box, sizeof(RootBox), hipMemcpyHostToDevice, s));
    }
    k_morton<<<cdiv(n, TPB), TPB, 0, s>>>(x, y, z, n, c.pbox.as<RootBox>(), pid, KL, c.keyA.as<uint64_t>(),
                                           c.valA.as<uint32_t>());
    VFMM_LAUNCH_CHECK();
    radix_sort(c, c.keyA, c.valA, c.keyB, c.valB, n, 3 * KL + pbits);
    c.rec.ensure(sizeof(float4) * 2 * n);
    c.perm.ensure(sizeof(int) * n);
    k_gather_pos<<<cdiv(n, TPB), TPB, 0, s>>>(c.valA.as<uint32_t>(), n, x, y, z, sigma, c.rec.as<float4>(),
                                               c.perm.as<int>());
    VFMM_LAUNCH_CHECK();
    c.record(2 * PH_BOUNDS_SORT + 1);
    c.record(2 * PH_TREE);

    // ---- levels ----
    size_t cap = (size_t)std::max<int64_t>(64, 2 * n / std::max(1, c.prm.ncrit) + 64 + 2 * (int64_t)nprob);
    DevBuf *arrs[] = {&c.c_start, &c.c_count, &c.c_parent, &c.c_child, &c.c_nchild, &c.c_level};
    for (DevBuf *b : arrs) b->ensure(sizeof(int) * cap);
    cap = std::min(c.c_start.cap, std::min(c.c_count.cap, c.c_parent.cap)) / sizeof(int);
    for (DevBuf *b : arrs) cap = std::min(cap, b->cap / sizeof(int));
    k_roots<<<cdiv(nprob, TPB), TPB, 0, s>>>(nprob, nprob > 1 ? c.poff.as<int64_t>() : nullptr, (int)n,
                                              c.c_start.as<int>(), c.c_count.as<int>(), c.c_parent.as<int>(),
                                              c.c_level.as<int>());
    VFMM_LAUNCH_CHECK();
    c.lvl_off.assign(1, 0);
    c.lvl_off.push_back(nprob);
    int lvl = 0;
    const uint64_t *keys = c.keyA.as<uint64_t>();
    int h_tot[2];
    for (;;) {
        const int c0 = c.lvl_off[lvl], c1 = c.lvl_off[lvl + 1];
        const int nl = c1 - c0;
        c.c_tmp.ensure(sizeof(int) * (2 * (size_t)nl + 2));
        int *nch = c.c_tmp.as<int>();
        int *off = nch + nl + 1;
        k_count_children<<<cdiv(8 * (int64_t)nl, TPB), TPB, 0, s>>>(c0, c1, lvl, c.prm.ncrit, KL, c.c_start.as<int>(),
                                                        c.c_count.as<int>(), keys, nch, c.bres.as<Bounds>());
        VFMM_LAUNCH_CHECK();
        scan_excl_i32(c, nch, off, nl);
        read_ints(c, {off + nl - 1, nch + nl - 1}, h_tot);
        const int total = h_tot[0] + h_tot[1];
        if ((size_t)(c1 + total) > cap) {
            const size_t ncap = (size_t)(c1 + total) * 2;
            for (DevBuf *b : arrs) grow_keep(c, *b, sizeof(int) * ncap, sizeof(int) * (size_t)c1);
            cap = ncap;
        }
        k_make_children<<<cdiv(8 * (int64_t)nl, TPB), TPB, 0, s>>>(c0, c1, lvl, c1, KL, c.c_start.as<int>(), c.c_count.as<int>(),
                                                       keys, off, nch, c.c_start.as<int>(), c.c_count.as<int>(),
                                                       c.c_parent.as<int>(), c.c_child.as<int>(),
                                                       c.c_nchild.as<int>(), c.c_level.as<int>());
        VFMM_LAUNCH_CHECK();
        if (total == 0) break;
        c.lvl_off.push_back(c1 + total);
        ++lvl;
    }
    c.depth = lvl;
    c.ncells = c.lvl_off.back();
    const int nc = c.ncells;

    // ---- geometry ----
    c.c_geo.ensure(sizeof(float4) * nc);
    c.c_rad.ensure(sizeof(float) * nc);
    c.c_lo.ensure(sizeof(float4) * nc);
    c.c_hi.ensure(sizeof(float4) * nc);
    k_leaf_geometry<<<cdiv(nc, TPB), TPB, 0, s>>>(nc, c.pbox.as<RootBox>(), KL, c.c_start.as<int>(), c.c_count.as<int>(),
                                                   c.c_level.as<int>(), c.c_nchild.as<int>(), keys,
                                                   c.rec.as<float4>(), c.c_geo.as<float4>(), c.c_rad.as<float>(),
                                                   c.c_lo.as<float4>(), c.c_hi.as<float4>());
    VFMM_LAUNCH_CHECK();
    for (int l = c.depth - 1; l >= 0; --l) {
        const int c0 = c.lvl_off[l], c1 = c.lvl_off[l + 1];
        k_internal_geometry<<<cdiv(c1 - c0, TPB), TPB, 0, s>>>(c0, c1, c.c_child.as<int>(), c.c_nchild.as<int>(),
                                                                c.c_geo.as<float4>(), c.c_rad.as<float>(),
                                                                c.c_lo.as<float4>(), c.c_hi.as<float4>());
        VFMM_LAUNCH_CHECK();
    }
    // ---- leaf list ----
    c.c_tmp.ensure(sizeof(int) * (2 * (size_t)nc + 2));
    int *flag = c.c_tmp.as<int>();
    int *pos = flag + nc + 1;
    k_leaf_flags<<<cdiv(nc, TPB), TPB, 0, s>>>(nc, c.c_nchild.as<int>(), flag);
    VFMM_LAUNCH_CHECK();
    scan_excl_i32(c, flag, pos, nc);
    int h3[3];
    read_ints(c, {pos + nc - 1, flag + nc - 1, &c.bres.as<Bounds>()->overfull}, h3);
    h_tot[0] = h3[0];
    h_tot[1] = h3[1];
    const int h_ovf = h3[2];
    c.nleaves = h_tot[0] + h_tot[1];
    c.overfull_leaves = h_ovf;
    c.leaves.ensure(sizeof(int) * (size_t)c.nleaves);
    k_leaf_compact<<<cdiv(nc, TPB), TPB, 0, s>>>(nc, c.c_nchild.as<int>(), pos, c.leaves.as<int>());
    VFMM_LAUNCH_CHECK();
    c.record(2 * PH_TREE + 1);
}

}  // namespace vfmm
