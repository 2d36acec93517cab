// Autotuner: chooses the expansion degree p, the acceptance parameter theta,
// the leaf size ncrit, the core-overlap gap of the M2L test (sigma_gap), the
// precision form (float32 or mixed), the product form of the batched M2L
// (float32 products, or split bfloat16 products: six, float32-accurate, or
// three, reduced precision) and the evaluation order (one stream,
// near field on a second stream, near field first) that minimise the time of
// one build + evaluate on the caller's particles while keeping the relative
// L2 error of u and of dalpha/dt below a bound.  The error of each candidate
// is measured against the library's own high-accuracy configuration (p = 12,
// theta = 0.35, sigma_gap >= 6, mixed form) on the same input.  The paper
// fixes p and does not tune (Sec. 4.2); this is a library feature for
// choosing the accuracy/time operating point.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <fstream>
#include <new>
#include <sstream>

#include "ctx.h"

namespace vfmm {

void do_build_public(Ctx &c, int64_t n, const float *x, const float *y, const float *z, const float *sigma);
void do_evaluate_public(Ctx &c, int64_t n, const float *x, const float *y, const float *z, const float *ax,
                        const float *ay, const float *az, const float *sigma, float *ux, float *uy, float *uz,
                        float *dax, float *day, float *daz);
void set_params_public(Ctx &c, const vfmm_params &p);

// per block: sums of |a_i - b_i|^2 and |b_i|^2 over the targets i, and the
// largest |a_i - b_i|^2, for the u block and the dalpha block ([3][n] each)
__global__ __launch_bounds__(256) void k_err_partial(int64_t n, const float *a, const float *b, double *part) {
    __shared__ double s[6][256];
    double du = 0, ru = 0, dd = 0, rd = 0, mu = 0, md = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double eu = 0, qu = 0, ed = 0, qd = 0;
        for (int c = 0; c < 3; ++c) {
            const double x = a[c * n + i], y = b[c * n + i];
            const double x2 = a[(3 + c) * n + i], y2 = b[(3 + c) * n + i];
            eu += (x - y) * (x - y);
            qu += y * y;
            ed += (x2 - y2) * (x2 - y2);
            qd += y2 * y2;
        }
        du += eu; ru += qu; dd += ed; rd += qd;
        mu = fmax(mu, eu);
        md = fmax(md, ed);
    }
    s[0][threadIdx.x] = du; s[1][threadIdx.x] = ru; s[2][threadIdx.x] = dd; s[3][threadIdx.x] = rd;
    s[4][threadIdx.x] = mu; s[5][threadIdx.x] = md;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            for (int q = 0; q < 4; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + o];
            for (int q = 4; q < 6; ++q) s[q][threadIdx.x] = fmax(s[q][threadIdx.x], s[q][threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 6; ++q) part[6 * blockIdx.x + q] = s[q][0];
}

// relative L2 errors of u and dalpha, and the largest per-target error over the
// RMS per-target magnitude (wu, wd)
static void rel_errors(Ctx &c, int64_t n, const float *a, const float *b, double &eu, double &ed, double &wu,
                       double &wd) {
    const int nb = 512;
    c.tune_part.ensure(sizeof(double) * 6 * nb);
    k_err_partial<<<nb, 256, 0, c.stream>>>(n, a, b, c.tune_part.as<double>());
    VFMM_LAUNCH_CHECK();
    std::vector<double> h(6 * nb);
    VFMM_HIP(hipMemcpyAsync(h.data(), c.tune_part.ptr, sizeof(double) * 6 * nb, hipMemcpyDeviceToHost, c.stream));
    VFMM_HIP(hipStreamSynchronize(c.stream));
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; i < nb; ++i) {
        for (int q = 0; q < 4; ++q) s[q] += h[6 * i + q];
        for (int q = 4; q < 6; ++q) s[q] = std::max(s[q], h[6 * i + q]);
    }
    eu = s[1] > 0 ? std::sqrt(s[0] / s[1]) : 0.0;
    ed = s[3] > 0 ? std::sqrt(s[2] / s[3]) : 0.0;
    wu = s[1] > 0 ? std::sqrt(s[4] / (s[1] / (double)n)) : 0.0;
    wd = s[3] > 0 ? std::sqrt(s[5] / (s[3] / (double)n)) : 0.0;
}

static std::string cache_key(const Ctx &c, int64_t n, float tol, const Bounds &b) {
    std::string arch = "unknown";
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    for (char &ch : arch)
        if (ch == ' ' || ch == '|') ch = '_';
    std::ostringstream k;
    k.precision(17);
    k << "arch=" << arch << " n=" << n << " periodic=" << c.prm.periodic << " images=" << c.prm.images
      << " box_len=" << c.prm.box_len << " box_lo=" << c.prm.box_lo[0] << "," << c.prm.box_lo[1] << ","
      << c.prm.box_lo[2] << " scheme=" << c.prm.scheme << " kahan=" << c.prm.kahan << " tol=" << tol
      << " fp=" << b.fp << " sum_a=" << b.sum_a[0] << "," << b.sum_a[1] << "," << b.sum_a[2]
      << " sum_xa=" << b.sum_xa[0] << "," << b.sum_xa[1] << "," << b.sum_xa[2]
      << " sigma=" << b.sig_min << "," << b.sig_max;
    return k.str();
}

struct Trial {
    int p, ncrit;
    float theta, gap;
    int prec, form, overlap;  // precision form, M2L product form, evaluation order
    double eu, ed, ms;
    double wu, wd;  // worst target over the RMS target magnitude
    bool ok;
    int64_t tree[5];  // cells, leaves, M2L entries, P2P entries, P2P pairs of the trial's build
};

}  // namespace vfmm

using vfmm::Ctx;
using vfmm::Error;

extern "C" vfmm_status vfmm_autotune(vfmm_ctx *ctx, int64_t n, const float *x, const float *y, const float *z,
                                     const float *ax, const float *ay, const float *az, const float *sigma,
                                     float max_rel_l2, const char *cache_path, vfmm_tune_result *out) {
    if (!ctx || !out) return VFMM_EINVAL;
    Ctx &c = ctx->c;
    const vfmm_params base = c.prm;
    try {
        if (n <= 0 || !x || !y || !z || !ax || !ay || !az || !sigma)
            throw Error{VFMM_EINVAL, "autotune needs n > 0 and every input"};
        if (!(max_rel_l2 > 0.f)) throw Error{VFMM_EINVAL, "max_rel_l2 must be > 0"};
        if (c.prm.direct) throw Error{VFMM_EINVAL, "autotune applies to the tree path (direct = 0)"};
        if (c.prm.precision == VFMM_PRECISION_FP64)
            throw Error{VFMM_EINVAL, "autotune chooses between the float32 and mixed forms (precision 0 or 1)"};
        std::memset(out, 0, sizeof(*out));
        // fingerprint of the inputs for the cache key
        vfmm::compute_bounds(c, n, x, y, z, sigma, ax, ay, az, true);
        vfmm::Bounds fb;
        VFMM_HIP(hipMemcpyAsync(&fb, c.bres.ptr, sizeof(fb), hipMemcpyDeviceToHost, c.stream));
        VFMM_HIP(hipStreamSynchronize(c.stream));
        const std::string key = vfmm::cache_key(c, n, max_rel_l2, fb);
        if (cache_path) {
            std::ifstream in(cache_path);
            std::string line;
            while (std::getline(in, line)) {
                const size_t bar = line.find(" | ");
                if (bar == std::string::npos || line.substr(0, bar) != key) continue;
                std::istringstream v(line.substr(bar + 3));
                vfmm_tune_result r{};
                if (v >> r.p >> r.theta >> r.ncrit >> r.sigma_gap >> r.precision >> r.m2l_form >> r.overlap >>
                    r.err_u >> r.err_dalpha >> r.worst_u >> r.worst_dalpha >> r.ms) {
                    r.from_cache = 1;
                    *out = r;
                }
            }
            if (out->from_cache) {
                vfmm_params p = base;
                p.p = out->p;
                p.theta = out->theta;
                p.ncrit = out->ncrit;
                p.sigma_gap = out->sigma_gap;
                p.precision = out->precision;
                p.m2l_form = out->m2l_form;
                p.overlap = out->overlap;
                vfmm::set_params_public(c, p);
                return VFMM_OK;
            }
        }
        c.tune_ref.ensure(sizeof(float) * 6 * (size_t)n);
        c.tune_out.ensure(sizeof(float) * 6 * (size_t)n);
        float *R = c.tune_ref.as<float>(), *O = c.tune_out.as<float>();
        auto run = [&](int p, float theta, int ncrit, float gap, int prec, int form, int ov, float *dst, double &ms) {
            vfmm_params q = base;
            q.p = p;
            q.theta = theta;
            q.ncrit = ncrit;
            q.sigma_gap = gap;
            q.precision = prec;
            q.m2l_form = form;
            q.overlap = ov;
            q.use_graph = 0;
            vfmm::set_params_public(c, q);
            // first pass warms the buffers; the second is timed
            for (int rep = 0; rep < 2; ++rep) {
                vfmm::do_build_public(c, n, x, y, z, sigma);
                vfmm::do_evaluate_public(c, n, x, y, z, ax, ay, az, sigma, dst, dst + n, dst + 2 * n, dst + 3 * n,
                                         dst + 4 * n, dst + 5 * n);
            }
            VFMM_HIP(hipStreamSynchronize(c.stream));
            float b = 0.f, e = 0.f;
            VFMM_HIP(hipEventElapsedTime(&b, c.ev[2 * vfmm::PH_NUM], c.ev[2 * vfmm::PH_NUM + 1]));
            VFMM_HIP(hipEventElapsedTime(&e, c.ev[2 * vfmm::PH_NUM + 2], c.ev[2 * vfmm::PH_NUM + 3]));
            ms = (double)b + (double)e;
        };
        double ref_ms = 0;
        run(12, 0.35f, base.ncrit, std::max(base.sigma_gap, 6.0f), VFMM_PRECISION_MIXED, 0, 0, R, ref_ms);
        std::vector<vfmm::Trial> trials;
        auto trial = [&](int p, float theta, int ncrit, float gap, int prec, int form, int ov) {
            for (const auto &t : trials)
                if (t.p == p && t.ncrit == ncrit && std::fabs(t.theta - theta) < 1e-6f &&
                    std::fabs(t.gap - gap) < 1e-6f && t.prec == prec && t.form == form && t.overlap == ov)
                    return t;
            vfmm::Trial t{p, ncrit, theta, gap, prec, form, ov, 0, 0, 0, 0, 0, false, {0, 0, 0, 0, 0}};
            run(p, theta, ncrit, gap, prec, form, ov, O, t.ms);
            const int64_t tr[5] = {c.ncells, c.nleaves, c.n_m2l, c.n_p2p, c.p2p_pairs};
            std::copy(tr, tr + 5, t.tree);
            vfmm::rel_errors(c, n, O, R, t.eu, t.ed, t.wu, t.wd);
            // the L2 bound, and no single target off by more than fifty times it (at the L2
            // bound the largest single-target error measures 30-45 times the L2 error on the
            // turbulence-shaped lattices; the guard catches outliers, not the operating point)
            t.ok = t.eu <= max_rel_l2 && t.ed <= max_rel_l2 && t.wu <= 50.0 * max_rel_l2 && t.wd <= 50.0 * max_rel_l2;
            trials.push_back(t);
            return t;
        };
        const int ps[] = {6, 8, 10, 12};
        const float thetas[] = {0.3f, 0.4f, 0.5f, 0.6f, 0.7f};
        const int ncrits[] = {32, 64, 128, 256, 512};
        const float gaps[] = {4.0f, 5.0f, 6.0f};
        const int bprec = base.precision, bform = base.m2l_form, bov = base.overlap;
        // (theta, p) at the caller's ncrit, sigma_gap and forms: smallest feasible p per theta
        for (float th : thetas)
            for (int p : ps)
                if (trial(p, th, base.ncrit, base.sigma_gap, bprec, bform, bov).ok) break;
        // fastest feasible trial; leaf sizes that build the same tree (a lattice
        // splits into the same cells for every ncrit between two powers of 8)
        // give the same results, and among them the largest is kept: it builds
        // that tree again after the particles have moved a little, where a
        // smaller one would split the first overfull leaves
        auto best_of = [&]() {
            const vfmm::Trial *b = nullptr;
            for (const auto &t : trials)
                if (t.ok && (!b || t.ms < b->ms)) b = &t;
            if (b)
                for (const auto &t : trials)
                    if (t.ok && t.p == b->p && t.theta == b->theta && t.gap == b->gap && t.ncrit > b->ncrit &&
                        t.prec == b->prec && t.form == b->form && t.overlap == b->overlap &&
                        std::equal(t.tree, t.tree + 5, b->tree))
                        b = &t;
            return b;
        };
        const vfmm::Trial *b = best_of();
        if (!b) throw Error{VFMM_EINVAL, "no configuration reaches the requested accuracy"};
        const int bp = b->p;
        const float bth = b->theta;
        // leaf size at the best (theta, p), raising p once if accuracy drops
        for (int nc : ncrits) {
            if (nc == base.ncrit) continue;
            if (!trial(bp, bth, nc, base.sigma_gap, bprec, bform, bov).ok && bp + 2 <= 12)
                trial(bp + 2, bth, nc, base.sigma_gap, bprec, bform, bov);
        }
        // gap of the M2L core-overlap test at the best (theta, p, ncrit)
        b = best_of();
        {
            const vfmm::Trial bb = *b;
            for (float gp : gaps)
                if (std::fabs(gp - bb.gap) > 1e-6f) trial(bb.p, bb.theta, bb.ncrit, gp, bprec, bform, bov);
        }
        // forms at the best (theta, p, ncrit, gap): precision (float32, mixed),
        // M2L products (float32, split bfloat16 with six or three products),
        // evaluation order (0, 1, 2)
        b = best_of();
        {
            const vfmm::Trial bb = *b;
            for (int prec : {VFMM_PRECISION_FP32, VFMM_PRECISION_MIXED})
                for (int form : {0, 2, 3})
                    for (int ov : {0, 1, 2}) trial(bb.p, bb.theta, bb.ncrit, bb.gap, prec, form, ov);
        }
        // the neighbouring leaf sizes and acceptance parameters again with the
        // chosen forms (a cheaper M2L form moves the balance toward more
        // translations and fewer near-field pairs)
        b = best_of();
        {
            const vfmm::Trial bb = *b;
            for (int nc : {bb.ncrit / 2, bb.ncrit * 2})
                if (nc >= ncrits[0] && nc <= ncrits[4] &&
                    !trial(bb.p, bb.theta, nc, bb.gap, bb.prec, bb.form, bb.overlap).ok && bb.p + 2 <= 12)
                    trial(bb.p + 2, bb.theta, nc, bb.gap, bb.prec, bb.form, bb.overlap);
            for (float th : {bb.theta - 0.1f, bb.theta + 0.1f}) {
                if (th < thetas[0] - 1e-4f || th > thetas[4] + 1e-4f) continue;
                for (int p : ps)
                    if (p >= bb.p - 2 && trial(p, th, bb.ncrit, bb.gap, bb.prec, bb.form, bb.overlap).ok) break;
            }
        }
        b = best_of();
        out->p = b->p;
        out->theta = b->theta;
        out->ncrit = b->ncrit;
        out->sigma_gap = b->gap;
        out->precision = b->prec;
        out->m2l_form = b->form;
        out->overlap = b->overlap;
        out->worst_u = (float)b->wu;
        out->worst_dalpha = (float)b->wd;
        out->err_u = (float)b->eu;
        out->err_dalpha = (float)b->ed;
        out->ms = (float)b->ms;
        out->tried = (int)trials.size();
        out->from_cache = 0;
        vfmm_params p = base;
        p.p = b->p;
        p.theta = b->theta;
        p.ncrit = b->ncrit;
        p.sigma_gap = b->gap;
        p.precision = b->prec;
        p.m2l_form = b->form;
        p.overlap = b->overlap;
        vfmm::set_params_public(c, p);
        if (cache_path) {
            std::ofstream o(cache_path, std::ios::app);
            o << key << " | " << out->p << " " << out->theta << " " << out->ncrit << " " << out->sigma_gap << " "
              << out->precision << " " << out->m2l_form << " " << out->overlap << " " << out->err_u << " "
              << out->err_dalpha << " " << out->worst_u << " " << out->worst_dalpha << " " << out->ms << "\n";
        }
        return VFMM_OK;
    } catch (const Error &e) {
        try {
            vfmm::set_params_public(c, base);
        } catch (...) {
        }
        c.err = e.msg;
        return e.st;
    } catch (const std::exception &x) {  // a host-side failure becomes a status code
        try {
            vfmm::set_params_public(c, base);
        } catch (...) {
        }
        c.err = std::string("host: ") + x.what();
        return dynamic_cast<const std::bad_alloc *>(&x) ? VFMM_ENOMEM : VFMM_EHIP;
    }
}
