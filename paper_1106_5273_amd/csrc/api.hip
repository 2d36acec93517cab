// C ABI of the library and the host orchestration of one build / evaluate.
#include <cmath>
#include <cstring>
#include <new>
#include <stdexcept>

#include "ctx.h"

namespace vfmm {

static std::string g_create_error;

void Ctx::release_all() {
    DevBuf *bufs[] = {&bpart, &bres, &keyA, &keyB, &valA, &valB, &hist, &scanA, &scanB, &scanC, &perm, &rec, &rec64,
                      &c_start, &c_count, &c_parent, &c_child, &c_nchild, &c_level, &c_geo, &c_rad, &c_lo, &c_hi,
                      &c_tmp, &leaves, &frA, &frB, &tcnt, &m2l_raw, &p2p_raw, &lkey, &lkey2, &lval, &lval2,
                      &m2l_off, &m2l_src, &p2p_off, &p2p_ent, &p2p_sh, &recp, &tgt, &c_nsrc, &part, &blocks, &pairs64, &Mexp, &Lexp, &lat_op, &far_u,
                      &far_da, &near, &dsurf, &rk, &m2l_tgt, &mb_eq, &mb_flag, &mb_pos, &mb_kid, &mb_ukey,
                      &mb_tab, &mb_bcells, &mb_ent, &mb_groups, &mb_blk, &mb_items, &mb_mr, &mb_partial, &mb_cls, &mb_cellbs, &mb_gcnt, &mb_gid, &mb_goff, &mb_gcur, &mb_bkt, &mb_order, &mb_slots, &gpart, &pid, &pbox, &poff, &tune_ref, &tune_out, &tune_part, &rbf, &spec};
    for (DevBuf *b : bufs) b->release();
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    graph_exec = nullptr;
    graph = nullptr;
    if (ev_ok)
        for (auto &e : ev) (void)hipEventDestroy(e);
    ev_ok = false;
    if (side) {
        (void)hipStreamSynchronize(side);
        (void)hipStreamDestroy(side);
        side = nullptr;
    }
    if (rbf_ev_ok)
        for (auto &e : rbf_ev) (void)hipEventDestroy(e);
    rbf_ev_ok = false;
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    ev_fork = ev_join = nullptr;
    if (hpin) (void)hipHostFree(hpin);
    hpin = nullptr;
}

static bool supported_p(int p) { return p == 4 || p == 6 || p == 8 || p == 10 || p == 12; }

static void validate(const vfmm_params &p) {
    if (!supported_p(p.p)) throw Error{VFMM_EINVAL, "p must be one of 4, 6, 8, 10, 12"};
    if (p.ncrit < 1) throw Error{VFMM_EINVAL, "ncrit must be >= 1"};
    if (!(p.theta > 0.f && p.theta < 1.f)) throw Error{VFMM_EINVAL, "theta must be in (0, 1)"};
    if (!(p.sigma_gap >= 0.f)) throw Error{VFMM_EINVAL, "sigma_gap must be >= 0"};
    if (p.scheme != VFMM_SCHEME_TRANSPOSE && p.scheme != VFMM_SCHEME_CLASSICAL)
        throw Error{VFMM_EINVAL, "scheme must be VFMM_SCHEME_TRANSPOSE or VFMM_SCHEME_CLASSICAL"};
    if (p.m2l_mode < 0 || p.m2l_mode > 2) throw Error{VFMM_EINVAL, "m2l_mode must be 0, 1 or 2"};
    if (p.use_graph != 0 && p.use_graph != 1) throw Error{VFMM_EINVAL, "use_graph must be 0 or 1"};
    if (p.use_graph && p.direct) throw Error{VFMM_EINVAL, "use_graph needs the tree path (direct = 0)"};
    if (p.overlap < 0 || p.overlap > 2) throw Error{VFMM_EINVAL, "overlap must be 0, 1 or 2"};
    if (p.m2l_form < 0 || p.m2l_form > 3) throw Error{VFMM_EINVAL, "m2l_form must be 0, 1, 2 or 3"};
    if (p.precision < VFMM_PRECISION_FP32 || p.precision > VFMM_PRECISION_FP64)
        throw Error{VFMM_EINVAL, "precision must be VFMM_PRECISION_FP32, _MIXED or _FP64"};
    if (p.periodic) {
        if (!(p.box_len > 0.0) || !std::isfinite(p.box_len)) throw Error{VFMM_EINVAL, "periodic box_len must be > 0"};
        if (p.images < 1 || p.images > 12) throw Error{VFMM_EINVAL, "images must be in [1, 12]"};
        if (p.direct) throw Error{VFMM_EINVAL, "direct mode is free space only"};
    } else if (!(p.box_len >= 0.0) || !std::isfinite(p.box_len)) {
        throw Error{VFMM_EINVAL, "box_len must be >= 0 (free space: 0 = bounding cube of the particles)"};
    }
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(p.box_lo[d])) throw Error{VFMM_EINVAL, "box_lo must be finite"};
}

static void set_params(Ctx &c, const vfmm_params &p) {
    validate(p);
    c.prm = p;
    c.built = false;
    if (p.periodic) {
        c.img_B = p.images <= 1 ? 1 : 4;
    } else {
        c.img_B = 0;
    }
    const int W = 2 * c.img_B + 1;
    c.img_codes = W * W * W;
}

// A host-side failure (std::bad_alloc from a host vector, a stream error)
// becomes a status code: no exception crosses the C ABI.
static inline Error host_error(const std::exception &x) {
    return Error{dynamic_cast<const std::bad_alloc *>(&x) ? VFMM_ENOMEM : VFMM_EHIP, std::string("host: ") + x.what()};
}

static vfmm_status fail(const Ctx *c, const Error &e) {
    if (c) c->err = e.msg;
    return e.st;
}

static void ensure_events(Ctx &c) {
    if (c.ev_ok) return;
    for (auto &e : c.ev) VFMM_HIP(hipEventCreate(&e));
    c.ev_ok = true;
}

static float ev_ms(const Ctx &c, int a, int b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c.ev[a], c.ev[b]) != hipSuccess) {
        (void)hipGetLastError();
        return 0.f;
    }
    return ms;
}

static void upload_lattice(Ctx &c) {
    if (!c.prm.periodic || c.prm.images < 3) return;
    const int dbl = c.prm.precision != VFMM_PRECISION_FP32 ? 1 : 0;
    if (c.lat_p == c.prm.p && c.lat_K == c.prm.images && c.lat_dbl == dbl) return;
    std::vector<double> op;
    lattice_operator_host(c.prm.p, c.prm.images, op);
    if (dbl) {
        c.lat_op.ensure(sizeof(double) * op.size());
        VFMM_HIP(hipMemcpyAsync(c.lat_op.ptr, op.data(), sizeof(double) * op.size(), hipMemcpyHostToDevice,
                                c.stream));
    } else {
        std::vector<float> f(op.size());
        for (size_t i = 0; i < op.size(); ++i) f[i] = (float)op[i];
        c.lat_op.ensure(sizeof(float) * f.size());
        VFMM_HIP(hipMemcpyAsync(c.lat_op.ptr, f.data(), sizeof(float) * f.size(), hipMemcpyHostToDevice, c.stream));
    }
    VFMM_HIP(hipStreamSynchronize(c.stream));
    c.lat_p = c.prm.p;
    c.lat_K = c.prm.images;
    c.lat_dbl = dbl;
}

static void ensure_side(Ctx &c) {
    if (c.side) return;
    // non-blocking so that it overlaps the library stream even when that is the
    // legacy default stream; ordering comes from the fork/join events alone
    VFMM_HIP(hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking));
    VFMM_HIP(hipEventCreateWithFlags(&c.ev_fork, hipEventDisableTiming));
    VFMM_HIP(hipEventCreateWithFlags(&c.ev_join, hipEventDisableTiming));
}

static void do_build(Ctx &c, int64_t n, const float *x, const float *y, const float *z, const float *sigma) {
    ensure_events(c);
    c.built = false;
    hipStream_t s = c.stream;
    c.record(2 * PH_NUM);
    c.record(2 * PH_BOUNDS_SORT);
    c.n = n;
    c.overfull_leaves = 0;
    if (n == 0) {
        c.ncells = c.nleaves = c.n_p2p = c.n_blocks = 0;
        c.n_m2l = c.p2p_pairs = 0;
        c.built = true;
        return;
    }
    compute_bounds(c, n, x, y, z, sigma, nullptr, nullptr, nullptr, false);
    static_assert(sizeof(Bounds) % sizeof(int) == 0 && sizeof(Bounds) <= 256, "Bounds read through read_words");
    read_words(c, c.bres.ptr, sizeof(Bounds), &c.hb);
    c.build_fp = c.hb.fp;
    c.build_ptr[0] = x;
    c.build_ptr[1] = y;
    c.build_ptr[2] = z;
    c.build_ptr[3] = sigma;
    if (c.hb.nonfinite) throw Error{VFMM_EDOMAIN, "non-finite position or non-positive core"};
    if (c.prm.periodic && c.hb.outside) throw Error{VFMM_EDOMAIN, "position outside the periodic cube"};
    if (!c.prm.periodic && c.nprob == 1 && c.prm.box_len > 0.0 && c.hb.outside)
        throw Error{VFMM_EDOMAIN, "position outside the root cube [box_lo, box_lo + box_len)"};
    if (c.nprob > 1 && (c.prm.periodic || c.prm.direct))
        throw Error{VFMM_EINVAL, "batched problems are free space and use the tree (periodic = 0, direct = 0)"};
    // per-source cores: the separation test and the cutoff-form thresholds use
    // the largest core; the near field evaluates each pair with its source's core
    c.var_sigma = c.hb.sig_max > c.hb.sig_min * (1.0 + 1e-6);
    c.sigma_uniform = (float)c.hb.sig_max;
    {
        // the float32 near field works in lengths scaled by kappa ~ 1/sigma: keep
        // kappa x (domain extent) below 2^24 so that rho'^-5 stays a normal float
        double ext = c.prm.periodic ? c.prm.box_len : 0.0;
        for (int d = 0; d < 3; ++d) ext = std::max(ext, c.hb.hi[d] - c.hb.lo[d]);
        if (c.prm.precision != VFMM_PRECISION_FP64 && ext * p2p_kappa(c.hb.sig_min) >= 16777216.0)
            throw Error{VFMM_EINVAL, "cores too small for the domain: extent / sigma must stay below about 2e7"};
    }
    if (c.prm.direct) {
        c.built = true;
        return;
    }
    if (c.prm.periodic || (c.nprob == 1 && c.prm.box_len > 0.0)) {
        // the periodic cell, or the root cube the caller fixed for a free-space tree
        for (int d = 0; d < 3; ++d) c.box.lo[d] = (float)c.prm.box_lo[d];
        c.box.len = (float)c.prm.box_len;
    } else if (c.nprob > 1) {
        // one root cube per problem, computed on the device by the tree build
    } else {
        double len = 0.0, ctr[3];
        for (int d = 0; d < 3; ++d) {
            len = std::max(len, c.hb.hi[d] - c.hb.lo[d]);
            ctr[d] = 0.5 * (c.hb.lo[d] + c.hb.hi[d]);
        }
        len = len * (1.0 + 1e-5) + 1e-30 + 1e-6 * std::max({std::fabs(ctr[0]), std::fabs(ctr[1]), std::fabs(ctr[2])});
        if (len <= 0) len = 1.0;
        for (int d = 0; d < 3; ++d) c.box.lo[d] = (float)(ctr[d] - 0.5 * len);
        c.box.len = (float)len;
    }
    upload_lattice(c);
    build_tree(c, n, x, y, z, sigma);
    if (c.n_src_part >= 0 && c.n_src_part < n) partition_sources(c, c.n_src_part);
    c.record(2 * PH_TRAVERSE);
    traverse_and_lists(c);
    c.m2lb_ok = false;
    if (c.prm.m2l_mode != 1 && c.prm.precision != VFMM_PRECISION_FP64) m2lb_plan(c);
    if (!c.m2lb_ok && !c.m2l_csr) build_m2l_csr(c);  // the per-pair M2L runs instead
    far_prealloc(c);
    m2lb_prealloc(c);
    if (c.prm.precision != VFMM_PRECISION_FP64 && c.prm.overlap == 1) ensure_side(c);
    ++c.build_id;
    c.record(2 * PH_TRAVERSE + 1);
    c.record(2 * PH_NUM + 1);
    c.build_timed = true;
    c.built = true;
}

static void do_evaluate(Ctx &c, int64_t n, const float *x, const float *y, const float *z, const float *ax,
                        const float *ay, const float *az, const float *sigma, float *ux, float *uy, float *uz,
                        float *dax, float *day, float *daz) {
    ensure_events(c);
    hipStream_t s = c.stream;
    c.record(2 * PH_NUM + 2);
    if (n == 0) {
        c.record(2 * PH_NUM + 3);
        return;
    }
    compute_bounds(c, n, x, y, z, sigma, ax, ay, az, true);
    if (c.prm.direct) {
        direct_all_pairs(c, x, y, z, ax, ay, az, sigma, ux, uy, uz, dax, day, daz);
    } else {
        gather_strengths(c, ax, ay, az, sigma);
        if (c.prm.precision != VFMM_PRECISION_FP64) p2p_prepare(c);
        if (c.prm.precision == VFMM_PRECISION_FP64 || !c.prm.overlap) {
            if (c.prm.precision == VFMM_PRECISION_FP64) gather_records64(c, ax, ay, az);
            far_field(c);
            p2p_and_finalize(c, ux, uy, uz, dax, day, daz);
        } else if (c.prm.overlap == 2) {
            // near field first, then the far field, on the library stream
            p2p_near(c, s);
            far_field(c);
            finalize_near_far(c, ux, uy, uz, dax, day, daz);
        } else {
            // near field (VALU) on the side stream concurrently with the far
            // field (M2L on the matrix cores) on the library stream
            ensure_side(c);
            VFMM_HIP(hipEventRecord(c.ev_fork, s));
            VFMM_HIP(hipStreamWaitEvent(c.side, c.ev_fork, 0));
            p2p_near(c, c.side);
            far_field(c);
            VFMM_HIP(hipEventRecord(c.ev_join, c.side));
            VFMM_HIP(hipStreamWaitEvent(s, c.ev_join, 0));
            finalize_near_far(c, ux, uy, uz, dax, day, daz);
        }
    }
    if (!c.prm.direct) c.far_build_id = c.build_id;
    c.record(2 * PH_NUM + 3);
    c.eval_timed = true;
}

// Evaluation through a hipGraph: captured on the first call after a build (or
// when the arguments change), replayed afterwards.
static void graph_evaluate(Ctx &c, int64_t n, const float *const *in, float *const *out) {
    std::vector<const void *> args(in, in + 7);
    args.insert(args.end(), out, out + 6);
    args.push_back((const void *)(intptr_t)n);
    if (!c.graph_exec || c.graph_build_id != c.build_id || args != c.graph_args) {
        if (c.graph_exec) VFMM_HIP(hipGraphExecDestroy(c.graph_exec));
        if (c.graph) VFMM_HIP(hipGraphDestroy(c.graph));
        c.graph_exec = nullptr;
        c.graph = nullptr;
        if (c.stream == nullptr) throw Error{VFMM_EINVAL, "use_graph needs a non-default stream"};
        VFMM_HIP(hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal));
        c.capturing = true;
        try {
            do_evaluate(c, n, in[0], in[1], in[2], in[3], in[4], in[5], in[6], out[0], out[1], out[2], out[3],
                        out[4], out[5]);
        } catch (...) {
            c.capturing = false;
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(c.stream, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        c.capturing = false;
        VFMM_HIP(hipStreamEndCapture(c.stream, &c.graph));
        VFMM_HIP(hipGraphInstantiate(&c.graph_exec, c.graph, nullptr, nullptr, 0));
        c.graph_args = args;
        c.graph_build_id = c.build_id;
    }
    c.record(2 * PH_NUM + 2);
    VFMM_HIP(hipGraphLaunch(c.graph_exec, c.stream));
    if (!c.prm.direct && n > 0) c.far_build_id = c.build_id;
    c.record(2 * PH_NUM + 3);
    c.eval_timed = true;
}

static void read_timings(const Ctx &c, vfmm_timings *out) {
    std::memset(out, 0, sizeof(*out));
    if (!c.ev_ok) return;
    VFMM_HIP(hipStreamSynchronize(c.stream));
    if (c.build_timed && !c.prm.direct && c.n > 0) {
        out->bounds_sort_ms = ev_ms(c, 2 * PH_BOUNDS_SORT, 2 * PH_BOUNDS_SORT + 1);
        out->tree_ms = ev_ms(c, 2 * PH_TREE, 2 * PH_TREE + 1);
        out->traverse_ms = ev_ms(c, 2 * PH_TRAVERSE, 2 * PH_TRAVERSE + 1);
        out->build_ms = ev_ms(c, 2 * PH_NUM, 2 * PH_NUM + 1);
    }
    if (c.eval_timed && c.n > 0) {
        if (!c.prm.direct && !c.prm.use_graph) {
            out->p2m_m2m_ms = ev_ms(c, 2 * PH_P2M_M2M, 2 * PH_P2M_M2M + 1);
            out->lattice_ms = ev_ms(c, 2 * PH_LATTICE, 2 * PH_LATTICE + 1);
            out->m2l_ms = ev_ms(c, 2 * PH_M2L, 2 * PH_M2L + 1);
            out->l2l_l2p_ms = ev_ms(c, 2 * PH_L2L_L2P, 2 * PH_L2L_L2P + 1);
            out->p2p_ms = ev_ms(c, 2 * PH_P2P, 2 * PH_P2P + 1);
        } else if (c.prm.direct) {
            out->p2p_ms = ev_ms(c, 2 * PH_P2P, 2 * PH_P2P + 1);
        }
        out->evaluate_ms = ev_ms(c, 2 * PH_NUM + 2, 2 * PH_NUM + 3);
    }
}

// ---------------------------------------------------------------------------
// rk_step helpers
// ---------------------------------------------------------------------------
struct RkArgs {
    int64_t n;
    float dt, nu;
    int periodic;
    double lo[3], len;
};

// Wraps v into the periodic cube [lo, lo + len) along one axis.  The
// arithmetic is float64 against the float64 cube, and the float32 result is
// then nudged by single ulps until it passes the same float64 comparison
// lo <= v < lo + len that the bounds pass of the next build applies (a cube
// corner such as -pi is not a float32 number, so a plain float32 wrap can
// land a particle just outside the cube).
__device__ inline float wrap(float v, double lo, double len) {
    double t = (double)v - lo;
    t -= floor(t / len) * len;
    if (t >= len) t -= len;
    if (t < 0.0) t += len;
    float r = (float)(lo + t);
    for (int k = 0; k < 4 && (double)r < lo; ++k) r = nextafterf(r, INFINITY);
    for (int k = 0; k < 4 && (double)r >= lo + len; ++k) r = nextafterf(r, -INFINITY);
    return r;
}

// stage 1 predictor: xs = x + dt u1, as = a + dt da1, ss = sqrt(s^2 + 2 nu dt)
__global__ __launch_bounds__(256) void k_rk_pred(RkArgs A, const float *x, const float *y, const float *z,
                                                 const float *ax, const float *ay, const float *az, const float *s,
                                                 const float *U, float *X) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= A.n) return;
    const int64_t n = A.n;
    float p[3] = {x[i] + A.dt * U[i], y[i] + A.dt * U[n + i], z[i] + A.dt * U[2 * n + i]};
    if (A.periodic)
        for (int d = 0; d < 3; ++d) p[d] = wrap(p[d], A.lo[d], A.len);
    X[i] = p[0];
    X[n + i] = p[1];
    X[2 * n + i] = p[2];
    X[3 * n + i] = ax[i] + A.dt * U[3 * n + i];
    X[4 * n + i] = ay[i] + A.dt * U[4 * n + i];
    X[5 * n + i] = az[i] + A.dt * U[5 * n + i];
    X[6 * n + i] = sqrtf(s[i] * s[i] + 2.f * A.nu * A.dt);
}

// corrector: x += dt/2 (u1 + u2) etc.
__global__ __launch_bounds__(256) void k_rk_corr(RkArgs A, float *x, float *y, float *z, float *ax, float *ay,
                                                 float *az, float *s, const float *U, const float *U2) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= A.n) return;
    const int64_t n = A.n;
    const float h = 0.5f * A.dt;
    float p[3] = {x[i] + h * (U[i] + U2[i]), y[i] + h * (U[n + i] + U2[n + i]), z[i] + h * (U[2 * n + i] + U2[2 * n + i])};
    if (A.periodic)
        for (int d = 0; d < 3; ++d) p[d] = wrap(p[d], A.lo[d], A.len);
    x[i] = p[0];
    y[i] = p[1];
    z[i] = p[2];
    ax[i] += h * (U[3 * n + i] + U2[3 * n + i]);
    ay[i] += h * (U[4 * n + i] + U2[4 * n + i]);
    az[i] += h * (U[5 * n + i] + U2[5 * n + i]);
    s[i] = sqrtf(s[i] * s[i] + 2.f * A.nu * A.dt);
}

static void do_rk(Ctx &c, int64_t n, float dt, float nu, float *x, float *y, float *z, float *ax, float *ay, float *az,
                  float *sigma) {
    if (n == 0) return;
    c.rk.ensure(sizeof(float) * 19 * (size_t)n);
    float *U1 = c.rk.as<float>();       // 6n: u1, da1
    float *X = U1 + 6 * n;              // 7n: predictor state
    float *U2 = X + 7 * n;              // 6n: u2, da2
    RkArgs A{};
    A.n = n;
    A.dt = dt;
    A.nu = nu;
    A.periodic = c.prm.periodic;
    for (int d = 0; d < 3; ++d) A.lo[d] = c.prm.box_lo[d];
    A.len = c.prm.box_len;
    do_build(c, n, x, y, z, sigma);
    do_evaluate(c, n, x, y, z, ax, ay, az, sigma, U1, U1 + n, U1 + 2 * n, U1 + 3 * n, U1 + 4 * n, U1 + 5 * n);
    read_timings(c, &c.t_stage1);
    k_rk_pred<<<cdiv(n, 256), 256, 0, c.stream>>>(A, x, y, z, ax, ay, az, sigma, U1, X);
    VFMM_LAUNCH_CHECK();
    do_build(c, n, X, X + n, X + 2 * n, X + 6 * n);
    do_evaluate(c, n, X, X + n, X + 2 * n, X + 3 * n, X + 4 * n, X + 5 * n, X + 6 * n, U2, U2 + n, U2 + 2 * n,
                U2 + 3 * n, U2 + 4 * n, U2 + 5 * n);
    k_rk_corr<<<cdiv(n, 256), 256, 0, c.stream>>>(A, x, y, z, ax, ay, az, sigma, U1, U2);
    VFMM_LAUNCH_CHECK();
    // the tree now describes the predictor positions
    c.built = false;
    c.last_was_rk = true;
}

}  // namespace vfmm

namespace vfmm {
void do_build_public(Ctx &c, int64_t n, const float *x, const float *y, const float *z, const float *sigma) {
    c.nprob = 1;
    do_build(c, n, x, y, z, sigma);
}
void do_evaluate_public(Ctx &c, int64_t n, const float *x, const float *y, const float *z, const float *ax,
                        const float *ay, const float *az, const float *sigma, float *ux, float *uy, float *uz,
                        float *dax, float *day, float *daz) {
    do_evaluate(c, n, x, y, z, ax, ay, az, sigma, ux, uy, uz, dax, day, daz);
}
void set_params_public(Ctx &c, const vfmm_params &p) { set_params(c, p); }
}  // namespace vfmm

using vfmm::Ctx;
using vfmm::Error;

extern "C" {

void vfmm_default_params(vfmm_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->p = 10;
    p->ncrit = 64;
    p->theta = 0.5f;
    p->sigma_gap = 5.0f;
    p->periodic = 0;
    p->images = 3;
    p->box_len = 0.0;
    p->scheme = VFMM_SCHEME_TRANSPOSE;
    p->kahan = 0;
    p->zero_mean = 1;
    p->direct = 0;
    p->m2l_mode = 0;
    p->use_graph = 0;
    p->overlap = 2;
    p->m2l_form = 2;
}

vfmm_status vfmm_create(const vfmm_params *params, void *hip_stream, vfmm_ctx **out) {
    if (!out || !params) {
        vfmm::g_create_error = "null argument";
        return VFMM_EINVAL;
    }
    *out = nullptr;
    vfmm_ctx *h = nullptr;
    try {
        h = new vfmm_ctx();
        vfmm::set_params(h->c, *params);
        h->c.stream = (hipStream_t)hip_stream;
        VFMM_HIP(hipGetDevice(&h->c.device));
        // the device address of fmm_direct_static's scratch array on this device
        vfmm::resolve_static_scratch(h->c.device);
        *out = h;
        return VFMM_OK;
    } catch (const Error &e) {
        vfmm::g_create_error = e.msg;
        delete h;
        return e.st;
    } catch (const std::exception &e) {
        vfmm::g_create_error = e.what();
        delete h;
        return VFMM_ENOMEM;
    }
}

vfmm_status vfmm_set_params(vfmm_ctx *ctx, const vfmm_params *params) {
    if (!ctx || !params) return VFMM_EINVAL;
    try {
        vfmm::set_params(ctx->c, *params);
        return VFMM_OK;
    } catch (const Error &e) {
        return vfmm::fail(&ctx->c, e);
    } catch (const std::exception &x) {
        const Error e = vfmm::host_error(x);
        return vfmm::fail(&ctx->c, e);
    }
}

// [a, a + na floats) and [b, b + nb floats) intersect
static bool overlaps_ab(const void *a, int64_t na, const void *b, int64_t nb) {
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + 4 * nb && pb < pa + 4 * na;
}

static bool overlaps(const void *a, const void *b, int64_t n) {
    const char *pa = (const char *)a, *pb = (const char *)b;
    const int64_t bytes = n * (int64_t)sizeof(float);
    return pa < pb + bytes && pb < pa + bytes;
}

vfmm_status fmm_build(vfmm_ctx *ctx, int64_t n, const float *x, const float *y, const float *z, const float *sigma) {
    if (!ctx) return VFMM_EINVAL;
    Ctx &c = ctx->c;
    try {
        if (n < 0 || n >= (1LL << 31)) throw Error{VFMM_EINVAL, "n must be in [0, 2^31)"};
        if (n > 0 && (!x || !y || !z || !sigma)) throw Error{VFMM_EINVAL, "null input pointer"};
        c.err.clear();
        c.nprob = 1;
        c.last_was_rk = false;
        c.tg_n = -1;
        vfmm::do_build(c, n, x, y, z, sigma);
        return VFMM_OK;
    } catch (const Error &e) {
        c.built = false;
        return vfmm::fail(&c, e);
    } catch (const std::exception &x) {
        const Error e = vfmm::host_error(x);
        c.built = false;
        return vfmm::fail(&c, e);
    }
}

// ---------------------------------------------------------------------------
// Separate target points: the particles and the m target points share one
// tree (the targets carry zero strength, so they add nothing to any sum) and
// one evaluation; the caller's outputs are copied out of the combined ones.
// ---------------------------------------------------------------------------
namespace vfmm {
__global__ __launch_bounds__(256) void k_fill_first(int64_t m, const float *src, float *dst) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < m) dst[i] = src[0];
}

static void copy_d2d(Ctx &c, float *dst, const float *src, int64_t n) {
    if (n > 0) VFMM_HIP(hipMemcpyAsync(dst, src, sizeof(float) * n, hipMemcpyDeviceToDevice, c.stream));
}
}  // namespace vfmm

vfmm_status fmm_build_targets(vfmm_ctx *ctx, int64_t n, const float *x, const float *y, const float *z,
                              const float *sigma, int64_t m, const float *tx, const float *ty, const float *tz) {
    if (!ctx) return VFMM_EINVAL;
    Ctx &c = ctx->c;
    try {
        if (n < 1 || m < 0 || n + m >= (1LL << 31)) throw Error{VFMM_EINVAL, "need n >= 1, m >= 0, n + m < 2^31"};
        if (!x || !y || !z || !sigma || (m > 0 && (!tx || !ty || !tz))) throw Error{VFMM_EINVAL, "null input pointer"};
        c.err.clear();
        c.nprob = 1;
        c.last_was_rk = false;
        c.tg_n = -1;
        const int64_t N = n + m;
        c.tgt.ensure(sizeof(float) * 13 * (size_t)N);
        float *X = c.tgt.as<float>(), *Y = X + N, *Z = Y + N, *S = Z + N;
        copy_d2d(c, X, x, n);
        copy_d2d(c, Y, y, n);
        copy_d2d(c, Z, z, n);
        copy_d2d(c, S, sigma, n);
        copy_d2d(c, X + n, tx, m);
        copy_d2d(c, Y + n, ty, m);
        copy_d2d(c, Z + n, tz, m);
        if (m > 0) {
            vfmm::k_fill_first<<<vfmm::cdiv(m, 256), 256, 0, c.stream>>>(m, sigma, S + n);  // any particle's core
            VFMM_LAUNCH_CHECK();
        }
        c.n_src_part = n;  // the near field reads only the particles as sources
        vfmm::do_build(c, N, X, Y, Z, S);
        c.n_src_part = -1;
        c.tg_n = n;
        c.tg_m = m;
        return VFMM_OK;
    } catch (const Error &e) {
        c.built = false;
        c.tg_n = -1;
        c.n_src_part = -1;
        return vfmm::fail(&c, e);
    } catch (const std::exception &x) {
        const Error e = vfmm::host_error(x);
        c.built = false;
        c.tg_n = -1;
        c.n_src_part = -1;
        return vfmm::fail(&c, e);
    }
}

vfmm_status fmm_evaluate_targets(vfmm_ctx *ctx, int64_t n, const float *ax, const float *ay, const float *az,
                                 int64_t m, float *ux, float *uy, float *uz, float *dax, float *day, float *daz,
                                 float *tux, float *tuy, float *tuz) {
    if (!ctx) return VFMM_EINVAL;
    Ctx &c = ctx->c;
    try {
        if (!c.built || c.tg_n < 0 || n != c.tg_n || m != c.tg_m)
            throw Error{VFMM_ESTATE, "fmm_evaluate_targets needs a prior fmm_build_targets with the same n and m"};
        if (!ax || !ay || !az) throw Error{VFMM_EINVAL, "null input pointer"};
        float *op[6] = {ux, uy, uz, dax, day, daz};
        float *tp[3] = {tux, tuy, tuz};
        for (float *p : op)
            if (!p) throw Error{VFMM_EINVAL, "null output pointer"};
        for (float *p : tp)
            if (m > 0 && !p) throw Error{VFMM_EINVAL, "null output pointer"};
        const void *in[3] = {ax, ay, az};
        for (int a = 0; a < 9; ++a) {
            void *pa = a < 6 ? (void *)op[a] : (void *)tp[a - 6];
            const int64_t la = a < 6 ? n : m;
            if (la == 0) continue;
            for (int b = a + 1; b < 9; ++b) {
                void *pb = b < 6 ? (void *)op[b] : (void *)tp[b - 6];
                const int64_t lb = b < 6 ? n : m;
                if (lb > 0 && overlaps_ab(pa, la, pb, lb)) throw Error{VFMM_EINVAL, "output arrays overlap"};
            }
            for (const void *p : in)
                if (overlaps_ab(pa, la, p, n)) throw Error{VFMM_EINVAL, "an output aliases an input"};
        }
        c.err.clear();
        const int64_t N = n + m;
        float *X = c.tgt.as<float>(), *Y = X + N, *Z = Y + N, *S = Z + N;
        float *AX = S + N, *AY = AX + N, *AZ = AY + N, *O = AZ + N;
        copy_d2d(c, AX, ax, n);
        copy_d2d(c, AY, ay, n);
        copy_d2d(c, AZ, az, n);
        if (m > 0) {
            VFMM_HIP(hipMemsetAsync(AX + n, 0, sizeof(float) * m, c.stream));
            VFMM_HIP(hipMemsetAsync(AY + n, 0, sizeof(float) * m, c.stream));
            VFMM_HIP(hipMemsetAsync(AZ + n, 0, sizeof(float) * m, c.stream));
        }
        vfmm::do_evaluate(c, N, X, Y, Z, AX, AY, AZ, S, O, O + N, O + 2 * N, O + 3 * N, O + 4 * N, O + 5 * N);
        for (int k = 0; k < 6; ++k) copy_d2d(c, op[k], O + k * N, n);
        for (int k = 0; k < 3; ++k) copy_d2d(c, tp[k], O + k * N + n, m);
        return VFMM_OK;
    } catch (const Error &e) {
        return vfmm::fail(&c, e);
    } catch (const std::exception &x) {
        const Error e = vfmm::host_error(x);
        return vfmm::fail(&c, e);
    }
}

vfmm_status fmm_build_batched(vfmm_ctx *ctx, int32_t nprob, const int64_t *offsets, const float *x, const float *y,
                              const float *z, const float *sigma) {
    if (!ctx) return VFMM_EINVAL;
    Ctx &c = ctx->c;
    try {
        if (nprob < 1 || !offsets) throw Error{VFMM_EINVAL, "nprob must be >= 1 with an offsets array"};
        if (offsets[0] != 0) throw Error{VFMM_EINVAL, "offsets[0] must be 0"};
        for (int b = 0; b < nprob; ++b)
            if (offsets[b + 1] <= offsets[b]) throw Error{VFMM_EINVAL, "every problem needs at least one particle"};
        const int64_t n = offsets[nprob];
        if (n >= (1LL << 31)) throw Error{VFMM_EINVAL, "n must be in [0, 2^31)"};
        if (nprob > 1 << 20) throw Error{VFMM_EINVAL, "at most 2^20 problems"};
        if (!x || !y || !z || !sigma) throw Error{VFMM_EINVAL, "null input pointer"};
        c.err.clear();
        c.last_was_rk = false;
        c.nprob = nprob;
        c.h_poff.assign(offsets, offsets + nprob + 1);
        c.poff.ensure(sizeof(int64_t) * (nprob + 1));
        VFMM_HIP(hipMemcpyAsync(c.poff.ptr, c.h_poff.data(), sizeof(int64_t) * (nprob + 1), hipMemcpyHostToDevice,
                                c.stream));
        vfmm::do_build(c, n, x, y, z, sigma);
        return VFMM_OK;
    } catch (const Error &e) {
        c.built = false;
        c.nprob = 1;
        return vfmm::fail(&c, e);
    } catch (const std::exception &x) {
        const Error e = vfmm::host_error(x);
        c.built = false;
        c.nprob = 1;
        return vfmm::fail(&c, e);
    }
}

vfmm_status fmm_evaluate_batched(vfmm_ctx *ctx, int32_t nprob, const int64_t *offsets, const float *x, const float *y,
                                 const float *z, const float *ax, const float *ay, const float *az, const float *sigma,
                                 float *ux, float *uy, float *uz, float *dax, float *day, float *daz) {
    const vfmm_status st = fmm_build_batched(ctx, nprob, offsets, x, y, z, sigma);
    if (st != VFMM_OK) return st;
    return fmm_evaluate(ctx, offsets[nprob], x, y, z, ax, ay, az, sigma, ux, uy, uz, dax, day, daz);
}

vfmm_status fmm_evaluate(vfmm_ctx *ctx, int64_t n, const float *x, const float *y, const float *z, const float *ax,
                         const float *ay, const float *az, const float *sigma, float *ux, float *uy, float *uz,
                         float *dax, float *day, float *daz) {
    if (!ctx) return VFMM_EINVAL;
    Ctx &c = ctx->c;
    try {
        if (!c.built || n != c.n) throw Error{VFMM_ESTATE, "fmm_evaluate needs a prior fmm_build with the same n"};
        if (n > 0) {
            const void *in[] = {x, y, z, ax, ay, az, sigma};
            void *outp[] = {ux, uy, uz, dax, day, daz};
            for (const void *p : in)
                if (!p) throw Error{VFMM_EINVAL, "null input pointer"};
            for (void *p : outp)
                if (!p) throw Error{VFMM_EINVAL, "null output pointer"};
            for (int a = 0; a < 6; ++a) {
                for (int b = a + 1; b < 6; ++b)
                    if (overlaps(outp[a], outp[b], n)) throw Error{VFMM_EINVAL, "output arrays overlap"};
                for (const void *p : in)
                    if (overlaps(outp[a], p, n)) throw Error{VFMM_EINVAL, "an output aliases an input"};
            }
        }
        if (n > 0 && (x != c.build_ptr[0] || y != c.build_ptr[1] || z != c.build_ptr[2] || sigma != c.build_ptr[3])) {
            // other arrays than the build's: their contents must be the build's positions and cores
            vfmm::compute_bounds(c, n, x, y, z, sigma, ax, ay, az, true);
            vfmm::Bounds b;
            VFMM_HIP(hipMemcpyAsync(&b, c.bres.ptr, sizeof(b), hipMemcpyDeviceToHost, c.stream));
            VFMM_HIP(hipStreamSynchronize(c.stream));
            if (b.stale) throw Error{VFMM_ESTATE, "fmm_evaluate: positions or cores differ from those of the last build"};
        }
        c.err.clear();
        if (c.prm.use_graph && n > 0) {
            const float *in[7] = {x, y, z, ax, ay, az, sigma};
            float *out[6] = {ux, uy, uz, dax, day, daz};
            vfmm::graph_evaluate(c, n, in, out);
        } else {
            vfmm::do_evaluate(c, n, x, y, z, ax, ay, az, sigma, ux, uy, uz, dax, day, daz);
        }
        return VFMM_OK;
    } catch (const Error &e) {
        return vfmm::fail(&c, e);
    } catch (const std::exception &x) {
        const Error e = vfmm::host_error(x);
        return vfmm::fail(&c, e);
    }
}

vfmm_status rk_step(vfmm_ctx *ctx, int64_t n, float dt, float nu, float *x, float *y, float *z, float *ax, float *ay,
                    float *az, float *sigma) {
    if (!ctx) return VFMM_EINVAL;
    Ctx &c = ctx->c;
    try {
        if (n < 0 || n >= (1LL << 31)) throw Error{VFMM_EINVAL, "n must be in [0, 2^31)"};
        if (n > 0 && (!x || !y || !z || !ax || !ay || !az || !sigma)) throw Error{VFMM_EINVAL, "null pointer"};
        if (!std::isfinite(dt) || !std::isfinite(nu) || nu < 0.f) throw Error{VFMM_EINVAL, "bad dt or nu"};
        if (c.prm.direct && c.prm.periodic) throw Error{VFMM_EINVAL, "direct mode is free space only"};
        c.err.clear();
        c.nprob = 1;
        vfmm::do_rk(c, n, dt, nu, x, y, z, ax, ay, az, sigma);
        return VFMM_OK;
    } catch (const Error &e) {
        c.built = false;
        return vfmm::fail(&c, e);
    } catch (const std::exception &x) {
        const Error e = vfmm::host_error(x);
        c.built = false;
        return vfmm::fail(&c, e);
    }
}

vfmm_status fmm_gaussian_sum(vfmm_ctx *ctx, int64_t n, const float *gx, const float *gy, const float *gz,
                             float *wx, float *wy, float *wz) {
    if (!ctx) return VFMM_EINVAL;
    Ctx &c = ctx->c;
    try {
        if (n < 0 || n >= (1LL << 31)) throw Error{VFMM_EINVAL, "n must be in [0, 2^31)"};
        if (n > 0 && (!gx || !gy || !gz || !wx || !wy || !wz)) throw Error{VFMM_EINVAL, "null pointer"};
        const float *in[3] = {gx, gy, gz};
        float *out[3] = {wx, wy, wz};
        for (int a = 0; a < 3; ++a) {
            for (const float *p : in)
                if (overlaps_ab(out[a], n, p, n)) throw Error{VFMM_EINVAL, "an output aliases an input"};
            for (int b = 0; b < a; ++b)
                if (overlaps_ab(out[a], n, out[b], n)) throw Error{VFMM_EINVAL, "two outputs alias"};
        }
        c.err.clear();
        vfmm::gaussian_sum_run(c, n, gx, gy, gz, wx, wy, wz);
        return VFMM_OK;
    } catch (const Error &e) {
        return vfmm::fail(&c, e);
    } catch (const std::exception &x) {
        return vfmm::fail(&c, vfmm::host_error(x));
    }
}

vfmm_status rbf_reinit(vfmm_ctx *ctx, int64_t n, const float *wx, const float *wy, const float *wz, float *gx,
                       float *gy, float *gz, double tol, int32_t maxiter, vfmm_rbf_info *info) {
    if (!ctx) return VFMM_EINVAL;
    Ctx &c = ctx->c;
    try {
        if (n < 0 || n >= (1LL << 31)) throw Error{VFMM_EINVAL, "n must be in [0, 2^31)"};
        if (n > 0 && (!gx || !gy || !gz || !wx || !wy || !wz)) throw Error{VFMM_EINVAL, "null pointer"};
        const float *in[3] = {wx, wy, wz};
        float *out[3] = {gx, gy, gz};
        for (int a = 0; a < 3; ++a) {
            for (const float *p : in)
                if (overlaps_ab(out[a], n, p, n)) throw Error{VFMM_EINVAL, "an output aliases an input"};
            for (int b = 0; b < a; ++b)
                if (overlaps_ab(out[a], n, out[b], n)) throw Error{VFMM_EINVAL, "two outputs alias"};
        }
        c.err.clear();
        vfmm::rbf_reinit_run(c, n, wx, wy, wz, gx, gy, gz, tol, maxiter, info);
        return VFMM_OK;
    } catch (const Error &e) {
        return vfmm::fail(&c, e);
    } catch (const std::exception &x) {
        return vfmm::fail(&c, vfmm::host_error(x));
    }
}

vfmm_status vfmm_energy_spectrum(vfmm_ctx *ctx, int32_t n, const float *ux, const float *uy, const float *uz,
                                 double *E) {
    if (!ctx) return VFMM_EINVAL;
    Ctx &c = ctx->c;
    try {
        if (!ux || !uy || !uz || !E) throw Error{VFMM_EINVAL, "null pointer"};
        c.err.clear();
        vfmm::energy_spectrum_run(c, n, ux, uy, uz, E);
        return VFMM_OK;
    } catch (const Error &e) {
        return vfmm::fail(&c, e);
    } catch (const std::exception &x) {
        return vfmm::fail(&c, vfmm::host_error(x));
    }
}

vfmm_status vfmm_get_gaussian_ms(const vfmm_ctx *ctx, float *ms) {
    if (!ctx || !ms) return VFMM_EINVAL;
    const Ctx &c = ctx->c;
    try {
        *ms = vfmm::gaussian_sum_ms(c);
        return VFMM_OK;
    } catch (const Error &e) {
        return vfmm::fail(&c, e);
    }
}

vfmm_status vfmm_get_timings(const vfmm_ctx *ctx, vfmm_timings *out) {
    if (!ctx || !out) return VFMM_EINVAL;
    const Ctx &c = ctx->c;
    try {
        vfmm::read_timings(c, out);
        if (c.last_was_rk) {
            float *a = reinterpret_cast<float *>(out);
            const float *b = reinterpret_cast<const float *>(&c.t_stage1);
            for (size_t i = 0; i < sizeof(vfmm_timings) / sizeof(float); ++i) a[i] += b[i];
        }
        return VFMM_OK;
    } catch (const Error &e) {
        return vfmm::fail(&c, e);
    } catch (const std::exception &x) {
        const Error e = vfmm::host_error(x);
        return vfmm::fail(&c, e);
    }
}

vfmm_status vfmm_get_stats(const vfmm_ctx *ctx, vfmm_stats *out) {
    if (!ctx || !out) return VFMM_EINVAL;
    const Ctx &c = ctx->c;
    std::memset(out, 0, sizeof(*out));
    if (hipStreamSynchronize(c.stream) != hipSuccess) {
        c.err = "stream synchronisation failed";
        return VFMM_EHIP;
    }
    out->n = c.n;
    out->ncells = c.ncells;
    out->nleaves = c.nleaves;
    out->depth = c.depth;
    out->p2p_entries = c.n_p2p;
    out->p2p_pairs = c.p2p_pairs;
    out->m2l_entries = c.n_m2l;
    out->p2p_blocks = c.n_blocks;
    out->images_traversed = c.prm.periodic ? c.img_codes : 0;
    out->sigma_min = c.hb.sig_min;
    out->sigma_max = c.hb.sig_max;
    if (c.m2lb_ok) {
        out->m2l_keys = c.mb_nkeys;
        out->m2l_groups = c.mb_ngroups;
        out->m2l_items = c.mb_nitems;
        out->m2l_split = c.mb_x6 ? (c.mb_nsplit == 2 ? 2 : 1) : 0;
    }
    out->overfull_leaves = c.overfull_leaves;
    if (c.bres.ptr && c.n > 0) {
        vfmm::Bounds b;
        if (hipMemcpy(&b, c.bres.ptr, sizeof(b), hipMemcpyDeviceToHost) == hipSuccess) {
            for (int d = 0; d < 3; ++d) out->sum_alpha[d] = b.sum_a[d];
            out->stale = b.stale;
        }
    }
    return VFMM_OK;
}

vfmm_status vfmm_copy_lists(vfmm_ctx *ctx, int32_t *p2p_tgt, int32_t *p2p_src, int32_t *p2p_img, int32_t *m2l_tgt,
                            int32_t *m2l_src, int32_t *m2l_img, int32_t *cell_start, int32_t *cell_count,
                            int32_t *perm) {
    if (!ctx) return VFMM_EINVAL;
    Ctx &c = ctx->c;
    if (!c.built || c.prm.direct) {
        c.err = "no tree built";
        return VFMM_ESTATE;
    }
    try {
        VFMM_HIP(hipStreamSynchronize(c.stream));
        const int nc = c.ncells;
        if (cell_start && nc) VFMM_HIP(hipMemcpy(cell_start, c.c_start.ptr, sizeof(int) * nc, hipMemcpyDeviceToHost));
        if (cell_count && nc) VFMM_HIP(hipMemcpy(cell_count, c.c_count.ptr, sizeof(int) * nc, hipMemcpyDeviceToHost));
        if (perm && c.n) VFMM_HIP(hipMemcpy(perm, c.perm.ptr, sizeof(int) * c.n, hipMemcpyDeviceToHost));
        // lists in CSR (sorted by target) order
        std::vector<int> off(nc + 1);
        if (c.n_p2p > 0 && (p2p_tgt || p2p_src || p2p_img)) {
            VFMM_HIP(hipMemcpy(off.data(), c.p2p_off.ptr, sizeof(int) * (nc + 1), hipMemcpyDeviceToHost));
            std::vector<int4> ent(c.n_p2p);
            VFMM_HIP(hipMemcpy(ent.data(), c.p2p_ent.ptr, sizeof(int4) * c.n_p2p, hipMemcpyDeviceToHost));
            std::vector<int> st(nc);
            VFMM_HIP(hipMemcpy(st.data(), c.c_start.ptr, sizeof(int) * nc, hipMemcpyDeviceToHost));
            std::vector<int> cn(nc);
            VFMM_HIP(hipMemcpy(cn.data(), c.c_count.ptr, sizeof(int) * nc, hipMemcpyDeviceToHost));
            // map source (start, count) back to a leaf id: leaves have unique starts among leaves
            std::vector<int> leaf_of_start(c.n, -1);
            std::vector<int> nchild(nc);
            VFMM_HIP(hipMemcpy(nchild.data(), c.c_nchild.ptr, sizeof(int) * nc, hipMemcpyDeviceToHost));
            for (int i = 0; i < nc; ++i)
                if (nchild[i] == 0 && cn[i] > 0) leaf_of_start[st[i]] = i;
            for (int t = 0; t < nc; ++t)
                for (int e = off[t]; e < off[t + 1]; ++e) {
                    if (p2p_tgt) p2p_tgt[e] = t;
                    if (p2p_src) p2p_src[e] = leaf_of_start[ent[e].x];
                    if (p2p_img) p2p_img[e] = ent[e].z;
                }
        }
        if (c.n_m2l > 0 && (m2l_tgt || m2l_src || m2l_img)) {
            if (!c.m2l_csr) {  // the batched M2L works from the raw list; order it on request
                vfmm::build_m2l_csr(c);
                VFMM_HIP(hipStreamSynchronize(c.stream));
            }
            VFMM_HIP(hipMemcpy(off.data(), c.m2l_off.ptr, sizeof(int) * (nc + 1), hipMemcpyDeviceToHost));
            std::vector<int2> src(c.n_m2l);
            VFMM_HIP(hipMemcpy(src.data(), c.m2l_src.ptr, sizeof(int2) * c.n_m2l, hipMemcpyDeviceToHost));
            for (int t = 0; t < nc; ++t)
                for (int e = off[t]; e < off[t + 1]; ++e) {
                    if (m2l_tgt) m2l_tgt[e] = t;
                    if (m2l_src) m2l_src[e] = src[e].x;
                    if (m2l_img) m2l_img[e] = src[e].y;
                }
        }
        return VFMM_OK;
    } catch (const Error &e) {
        return vfmm::fail(&c, e);
    } catch (const std::exception &x) {
        const Error e = vfmm::host_error(x);
        return vfmm::fail(&c, e);
    }
}

vfmm_status vfmm_copy_expansions(vfmm_ctx *ctx, int32_t *level, int32_t *parent, int32_t *first_child,
                                 int32_t *nchild, double *geo, double *mult, double *loc, double *far_u,
                                 double *far_da) {
    if (!ctx) return VFMM_EINVAL;
    Ctx &c = ctx->c;
    if (!c.built || c.prm.direct || c.n == 0 || c.ncells == 0) {
        c.err = "no tree built";
        return VFMM_ESTATE;
    }
    if ((mult || loc || far_u || far_da) && c.far_build_id != c.build_id) {
        c.err = "no evaluation on this tree";
        return VFMM_ESTATE;
    }
    try {
        VFMM_HIP(hipStreamSynchronize(c.stream));
        const int nc = c.ncells;
        if (level) VFMM_HIP(hipMemcpy(level, c.c_level.ptr, sizeof(int) * nc, hipMemcpyDeviceToHost));
        if (parent) VFMM_HIP(hipMemcpy(parent, c.c_parent.ptr, sizeof(int) * nc, hipMemcpyDeviceToHost));
        if (first_child) VFMM_HIP(hipMemcpy(first_child, c.c_child.ptr, sizeof(int) * nc, hipMemcpyDeviceToHost));
        if (nchild) VFMM_HIP(hipMemcpy(nchild, c.c_nchild.ptr, sizeof(int) * nc, hipMemcpyDeviceToHost));
        if (geo) {
            std::vector<float4> g(nc);
            std::vector<float> r(nc);
            VFMM_HIP(hipMemcpy(g.data(), c.c_geo.ptr, sizeof(float4) * nc, hipMemcpyDeviceToHost));
            VFMM_HIP(hipMemcpy(r.data(), c.c_rad.ptr, sizeof(float) * nc, hipMemcpyDeviceToHost));
            for (int i = 0; i < nc; ++i) {
                geo[5 * i] = g[i].x;
                geo[5 * i + 1] = g[i].y;
                geo[5 * i + 2] = g[i].z;
                geo[5 * i + 3] = g[i].w;
                geo[5 * i + 4] = r[i];
            }
        }
        // expansions and far-field outputs are float64 in the float64 form, float32 otherwise
        const bool dbl = c.prm.precision == VFMM_PRECISION_FP64;
        auto copy_real = [&](const void *src, double *dst, size_t cnt) {
            if (dbl) {
                VFMM_HIP(hipMemcpy(dst, src, sizeof(double) * cnt, hipMemcpyDeviceToHost));
            } else {
                std::vector<float> t(cnt);
                VFMM_HIP(hipMemcpy(t.data(), src, sizeof(float) * cnt, hipMemcpyDeviceToHost));
                for (size_t i = 0; i < cnt; ++i) dst[i] = t[i];
            }
        };
        const size_t ncoef = (size_t)nc * 3 * vfmm::NC(c.prm.p) * 2;
        if (mult) copy_real(c.Mexp.ptr, mult, ncoef);
        if (loc) copy_real(c.Lexp.ptr, loc, ncoef);
        if (far_u) copy_real(c.far_u.ptr, far_u, 3 * (size_t)c.n);
        if (far_da) copy_real(c.far_da.ptr, far_da, 3 * (size_t)c.n);
        return VFMM_OK;
    } catch (const Error &e) {
        return vfmm::fail(&c, e);
    } catch (const std::exception &x) {
        const Error e = vfmm::host_error(x);
        return vfmm::fail(&c, e);
    }
}

const char *vfmm_last_error(const vfmm_ctx *ctx) {
    if (!ctx) return vfmm::g_create_error.c_str();
    return ctx->c.err.c_str();
}

void vfmm_destroy(vfmm_ctx *ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->c.stream);
    ctx->c.release_all();
    delete ctx;
}

}  // extern "C"
