// fmm_direct_static: the all-pairs evaluation of fmm_build + fmm_evaluate with
// direct = 1, for callers that cannot allocate device memory.  Its scratch
// space is one file-scope device array (each GPU the library runs on holds its
// own copy until the process ends); host code reaches it only through the
// address hipGetSymbolAddress returns for the current device, looked up once
// per device when a context is created.
#include <cstring>
#include <mutex>

#include "ctx.h"

namespace vfmm {

// Layout of the scratch array for VFMM_STATIC_MAX_N particles, each slice on a
// 256-byte boundary.
constexpr size_t al256(size_t b) { return (b + 255) / 256 * 256; }
constexpr int64_t SMAX = VFMM_STATIC_MAX_N;
constexpr int64_t SBLK = (SMAX + 63) / 64;
constexpr size_t S_PART = 0;                                        // bounds partial sums
constexpr size_t S_PART_BYTES = 262144;
constexpr size_t S_BOUNDS = S_PART + S_PART_BYTES;                  // Bounds
constexpr size_t S_REC = S_BOUNDS + al256(sizeof(Bounds));          // float4[2n]
constexpr size_t S_PERM = S_REC + al256(sizeof(float4) * 2 * SMAX); // int[n]
constexpr size_t S_BLK = S_PERM + al256(sizeof(int) * SMAX);        // int4[nb]
constexpr size_t S_ENT = S_BLK + al256(sizeof(int4) * SBLK);        // int4[nb]
constexpr size_t S_SH = S_ENT + al256(sizeof(int4) * SBLK);         // float4[nb]
constexpr size_t S_RECP = S_SH + al256(sizeof(float4) * SBLK);      // float4[4n]
constexpr size_t S_BYTES = S_RECP + al256(sizeof(float4) * 4 * SMAX);

static __device__ __align__(256) unsigned char scratch[S_BYTES];

static std::mutex g_scratch_mu;
static std::vector<void *> g_scratch_ptr;      // per device: the array's device address
static std::vector<std::string> g_scratch_err; // per device: why the lookup failed

// Looks up, once per device and with that device current, the device address
// of the scratch array.  Called from vfmm_create.
void resolve_static_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0) return;
    if ((int)g_scratch_ptr.size() <= device) {
        g_scratch_ptr.resize(device + 1, nullptr);
        g_scratch_err.resize(device + 1);
    }
    if (g_scratch_ptr[device]) return;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        g_scratch_err[device] = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return;
    }
    g_scratch_ptr[device] = ptr;
}

static unsigned char *static_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0 || device >= (int)g_scratch_ptr.size() || !g_scratch_ptr[device]) {
        std::string why = (device >= 0 && device < (int)g_scratch_err.size()) ? g_scratch_err[device] : "";
        throw Error{VFMM_EHIP, "fmm_direct_static: no scratch address for this device" +
                                   (why.empty() ? std::string() : " (" + why + ")")};
    }
    return static_cast<unsigned char *>(g_scratch_ptr[device]);
}

static bool ranges_overlap(const void *a, const void *b, int64_t n) {
    const char *pa = (const char *)a, *pb = (const char *)b;
    const int64_t bytes = n * (int64_t)sizeof(float);
    return pa < pb + bytes && pb < pa + bytes;
}

}  // namespace vfmm

using vfmm::Error;

vfmm_status fmm_direct_static(vfmm_ctx *ctx, int64_t n, const float *x, const float *y, const float *z,
                              const float *ax, const float *ay, const float *az, const float *sigma, float *ux,
                              float *uy, float *uz, float *dax, float *day, float *daz) {
    if (!ctx) return VFMM_EINVAL;
    vfmm::Ctx &c = ctx->c;
    try {
        if (n < 0 || n > VFMM_STATIC_MAX_N)
            throw Error{VFMM_EINVAL, "fmm_direct_static: n = " + std::to_string(n) +
                                         " is outside [0, VFMM_STATIC_MAX_N = " +
                                         std::to_string((long long)VFMM_STATIC_MAX_N) + "]"};
        if (c.prm.periodic) throw Error{VFMM_EINVAL, "fmm_direct_static: free space only (periodic = 0)"};
        if (c.prm.precision == VFMM_PRECISION_FP64)
            throw Error{VFMM_EINVAL, "fmm_direct_static: float32 and mixed forms only"};
        if (vfmm::bounds_scratch_bytes() > vfmm::S_PART_BYTES)
            throw Error{VFMM_EHIP, "fmm_direct_static: bounds scratch larger than its slice"};
        if (n == 0) {
            c.err.clear();
            return VFMM_OK;
        }
        const float *in[7] = {x, y, z, ax, ay, az, sigma};
        float *out[6] = {ux, uy, uz, dax, day, daz};
        for (const float *p : in)
            if (!p) throw Error{VFMM_EINVAL, "fmm_direct_static: null input"};
        for (int a = 0; a < 6; ++a) {
            if (!out[a]) throw Error{VFMM_EINVAL, "fmm_direct_static: null output"};
            for (const float *p : in)
                if (vfmm::ranges_overlap(out[a], p, n)) throw Error{VFMM_EINVAL, "an output aliases an input"};
            for (int b = 0; b < a; ++b)
                if (vfmm::ranges_overlap(out[a], out[b], n)) throw Error{VFMM_EINVAL, "two outputs alias"};
        }
        unsigned char *base = vfmm::static_scratch(c.device);
        vfmm::Bounds *bres = reinterpret_cast<vfmm::Bounds *>(base + vfmm::S_BOUNDS);
        vfmm::launch_bounds(c, c.stream, n, x, y, z, sigma, ax, ay, az, true, false, 0.0, base + vfmm::S_PART, bres);
        vfmm::Bounds hb;
        VFMM_HIP(hipMemcpyAsync(&hb, bres, sizeof(hb), hipMemcpyDeviceToHost, c.stream));
        VFMM_HIP(hipStreamSynchronize(c.stream));
        // the checks fmm_build applies in direct mode
        if (hb.nonfinite) throw Error{VFMM_EDOMAIN, "non-finite position or non-positive core"};
        if (c.prm.box_len > 0.0 && hb.outside)
            throw Error{VFMM_EDOMAIN, "position outside the root cube [box_lo, box_lo + box_len)"};
        double ext = 0.0;
        for (int d = 0; d < 3; ++d) ext = std::max(ext, hb.hi[d] - hb.lo[d]);
        if (ext * vfmm::p2p_kappa(hb.sig_min) >= 16777216.0)
            throw Error{VFMM_EINVAL, "cores too small for the domain: extent / sigma must stay below about 2e7"};
        vfmm::DirectBufs b{reinterpret_cast<float4 *>(base + vfmm::S_REC), reinterpret_cast<int *>(base + vfmm::S_PERM),
                           reinterpret_cast<int4 *>(base + vfmm::S_BLK), reinterpret_cast<int4 *>(base + vfmm::S_ENT),
                           reinterpret_cast<float4 *>(base + vfmm::S_SH), reinterpret_cast<float4 *>(base + vfmm::S_RECP),
                           bres};
        vfmm::direct_f32(c, c.stream, n, hb, b, x, y, z, ax, ay, az, sigma, ux, uy, uz, dax, day, daz);
        c.err.clear();
        return VFMM_OK;
    } catch (const Error &e) {
        c.err = e.msg;
        return e.st;
    } catch (const std::exception &x) {
        c.err = std::string("host: ") + x.what();
        return VFMM_EHIP;
    }
}
