// Library context: parameters, device buffers and host-side sizes.
#pragma once
#include <initializer_list>

#include "common.h"

namespace vfmm {

enum Phase { PH_BOUNDS_SORT = 0, PH_TREE, PH_TRAVERSE, PH_P2M_M2M, PH_LATTICE, PH_M2L, PH_L2L_L2P,
             PH_P2P, PH_NUM };

struct Ctx {
    vfmm_params prm{};
    hipStream_t stream = nullptr;
    mutable std::string err;
    int device = 0;

    // ---- state of the last build ----
    bool built = false;
    int64_t n = 0;
    Bounds hb{};
    RootBox box{};
    bool var_sigma = false;
    float sigma_uniform = 0.f;
    int depth = 0;
    std::vector<int> lvl_off;  // cells of level l are [lvl_off[l], lvl_off[l+1])
    int ncells = 0, nleaves = 0;
    int n_p2p = 0, n_blocks = 0;
    int64_t n_m2l = 0, p2p_pairs = 0;
    int img_B = 0, img_codes = 1;
    int nprob = 1;                       // independent problems in the tree (forest)
    int key_levels = 21;                 // Morton levels per axis below the problem id
    std::vector<int64_t> h_poff;         // problem offsets (host)
    int images_traversed = 0;
    double build_fp = 0.0;               // fingerprint of the build's positions and cores (Bounds::fp)
    const void *build_ptr[4] = {nullptr, nullptr, nullptr, nullptr};  // x, y, z, sigma of the build
    int overfull_leaves = 0;             // leaves above ncrit at the key-resolution depth limit

    // ---- device buffers (grow-only) ----
    DevBuf bpart, bres;                  // bounds partials / result
    DevBuf keyA, keyB, valA, valB;       // sort ping-pong (uint64 keys, uint32 values)
    DevBuf hist, scanA, scanB, scanC;    // sort histogram, scan scratch
    DevBuf perm;                         // sorted position -> caller index (int)
    DevBuf pid, pbox, poff;              // batched problems: id per particle, root cubes, offsets
    DevBuf rec;                          // float4[2n]: (x,y,z,sigma) (ax,ay,az,0)/(4 pi)
    DevBuf rec64;                        // double4[2n]: the same records, float64 form only
    DevBuf recp;                         // float4[3n]: float32 near-field records (scaled, leaf-local)
    // cells
    DevBuf c_start, c_count, c_parent, c_child, c_nchild, c_level;  // int
    DevBuf c_geo;                        // float4 (cx, cy, cz, size)
    DevBuf c_rad;                        // float tight radius
    DevBuf c_lo, c_hi;                   // float4 particle bounding box
    DevBuf c_tmp;                        // build scratch: child counts
    DevBuf leaves;                       // leaf cell ids
    // traversal
    DevBuf frA, frB;                     // frontier int4 (A, B, img, 0)
    DevBuf tcnt;                         // per-pair counts (3 ints)
    DevBuf m2l_raw, p2p_raw;             // unsorted (tgt,src,img) int4
    DevBuf lkey, lkey2, lval, lval2;     // list sort
    DevBuf m2l_off, m2l_src;             // CSR by target cell: int offsets[ncells+1], int2 (src, img)
    DevBuf m2l_tgt;                      // target cell of each CSR entry
    DevBuf p2p_off, p2p_ent;             // CSR by target cell: int offsets, int4 (start, count, img, variant)
    DevBuf p2p_sh;                       // float4 per P2P entry: scaled offset between the two leaf centres
    DevBuf blocks;                       // int4 (tgt start, tgt count, list off, list count)
    DevBuf pairs64;                      // int64 reduction scratch
    DevBuf gpart;                        // per-work-group partial pair counts of the P2P list
    int *hpin = nullptr;                 // pinned host ints written by k_read_ints (read_ints)
    // expansions
    DevBuf Mexp, Lexp;                   // float2 [ncells][3][NC(p)]
    DevBuf lat_op;                       // float [2NC x 2NC] periodic lattice operator
    int lat_p = -1, lat_K = -1, lat_dbl = -1;
    double lat_len = 0.0;
    // operator-batched M2L plan
    bool m2lb_ok = false;
    bool m2l_csr = false;                // M2L CSR by target (m2l_off/src/tgt) built for this tree
    int m2lb_lds_set = 0;                // dynamic LDS size the batched M2L kernel has been allowed
    int m2lbx_lds_set = 0;               // the same for its split-product form
    bool mb_x6 = false;                  // the plan's operator table is in the split bf16 form
    int mb_nsplit = 3;                   // bf16 parts per operand the split form multiplies (3 or 2)
    int m2lbx3_lds_set = 0;              // dynamic LDS allowed for the two-part split kernel
    int mb_nblk = 0, mb_nkeys = 0, mb_ngroups = 0, mb_nitems = 0;
    int mb_fmt[4] = {0, 0, 0, 0};
    DevBuf mb_eq, mb_flag, mb_pos, mb_kid, mb_ukey, mb_tab, mb_bcells, mb_ent, mb_groups, mb_blk, mb_items,
        mb_mr, mb_partial, mb_cls, mb_cellbs, mb_gcnt, mb_gid, mb_goff, mb_gcur, mb_bkt, mb_order, mb_slots;
    // outputs of the far field, sorted order: float [3n] each
    DevBuf far_u, far_da;
    DevBuf dsurf;                        // float[4] surface velocity term
    // rk_step stage storage
    DevBuf rk;                           // float [19 n]
    // separate target points: combined inputs/outputs x y z sigma ax ay az + 6 outputs, float[13 (n + m)]
    DevBuf tgt;
    int64_t tg_n = -1, tg_m = 0;         // particles and targets of the last fmm_build_targets (-1: none)
    int64_t n_src_part = -1;             // >= 0: callers' indices below it are sources, the rest targets
    DevBuf c_nsrc;                       // per leaf: sources in front of its targets (partitioned builds)
    DevBuf part;                         // partition scratch
    // radial-basis-function reinitialisation: Gaussian-sum and conjugate-gradient buffers
    DevBuf rbf;
    hipEvent_t rbf_ev[4] = {};           // solve start/end, Gaussian-sum kernel start/end
    bool rbf_ev_ok = false, gauss_timed = false;
    int64_t gauss_pairs = 0;             // particle pairs of one Gaussian sum on this tree
    uint64_t gauss_build_id = ~0ull;     // build the pair count belongs to
    // energy spectrum: complex float64 [3][n^3] field, partial and final shell sums
    DevBuf spec;
    // autotuner scratch
    DevBuf tune_ref, tune_out, tune_part;

    // hipGraph of one evaluation (captured once per build, then replayed)
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<const void *> graph_args;
    bool capturing = false;
    uint64_t build_id = 0, graph_build_id = 0;
    uint64_t far_build_id = ~0ull;       // build whose expansions the last evaluation computed

    // near field on a second stream, concurrent with the far field
    hipStream_t side = nullptr;          // non-blocking, default priority; created on first use
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    DevBuf near;                         // float[6][n]: P2P u and dalpha in sorted order

    // timing
    hipEvent_t ev[2 * PH_NUM + 4] = {};
    bool ev_ok = false;
    bool last_was_rk = false;            // timings then sum both RK2 stages
    vfmm_timings t_stage1{};
    bool build_timed = false, eval_timed = false;

    void release_all();
    // records timing event i (on stream s, default the library stream) unless
    // the stream is being captured into a graph
    void record(int i, hipStream_t s) {
        if (ev_ok && !capturing) {
            hipError_t e = hipEventRecord(ev[i], s);
            if (e != hipSuccess) throw Error{VFMM_EHIP, std::string("hipEventRecord: ") + hipGetErrorString(e)};
        }
    }
    void record(int i) { record(i, stream); }
};

// tree.hip
// bytes of the partial-sum buffer of the bounds pass (any n)
size_t bounds_scratch_bytes();
// the bounds pass into caller-given buffers: part (bounds_scratch_bytes()) and res;
// check_fp compares the positions' fingerprint with fp_ref (Bounds::stale)
void launch_bounds(const Ctx &c, hipStream_t s, int64_t n, const float *x, const float *y, const float *z,
                   const float *sigma, const float *ax, const float *ay, const float *az, bool with_alpha,
                   bool check_fp, double fp_ref, void *part, Bounds *res);
void compute_bounds(Ctx &c, int64_t n, const float *x, const float *y, const float *z, const float *sigma,
                    const float *ax, const float *ay, const float *az, bool with_alpha);
void build_tree(Ctx &c, int64_t n, const float *x, const float *y, const float *z, const float *sigma);
void gather_strengths(Ctx &c, const float *ax, const float *ay, const float *az, const float *sigma);
void gather_records64(Ctx &c, const float *ax, const float *ay, const float *az);
void partition_sources(Ctx &c, int64_t n_src);
void build_m2l_csr(Ctx &c);
void p2p_prepare(Ctx &c);
void p2p_near(Ctx &c, hipStream_t s);
void finalize_near_far(Ctx &c, float *ux, float *uy, float *uz, float *dax, float *day, float *daz);
void scan_excl_i32(Ctx &c, const int *in, int *out, int64_t n);  // out may alias in
// Reads up to four device ints (one each at the given device addresses) into
// dst: one small kernel writes them to pinned host memory, then the library
// stream is synchronised (no copy engine or staging blit per value).
void read_ints(Ctx &c, std::initializer_list<const int *> src, int *dst);
// The pinned host ints (64) that a kernel may write directly, and the
// synchronisation that hands their first n values to the host.
int *pinned_ints(Ctx &c);
void sync_ints(Ctx &c, int n, int *dst);
// The same for a small device struct (at most 256 bytes, whole 4-byte words).
void read_words(Ctx &c, const void *src, size_t bytes, void *dst);
// traverse.hip
void traverse_and_lists(Ctx &c);
// far.hip
void far_field(Ctx &c);
void far_prealloc(Ctx &c);
// m2lb.hip
void m2lb_plan(Ctx &c);
void m2lb_run(Ctx &c);
void m2lb_prealloc(Ctx &c);
// p2p.hip
void p2p_and_finalize(Ctx &c, float *ux, float *uy, float *uz, float *dax, float *day, float *daz);
void direct_all_pairs(Ctx &c, const float *x, const float *y, const float *z, const float *ax,
                      const float *ay, const float *az, const float *sigma, float *ux, float *uy,
                      float *uz, float *dax, float *day, float *daz);
// Device buffers of the float32 all-pairs evaluation of n particles.
struct DirectBufs {
    float4 *rec;     // float4[2n]  (x, y, z, sigma), alpha/(4 pi)
    int *perm;       // int[n]
    int4 *blocks;    // int4[ceil(n/64)]
    int4 *ent;       // int4[ceil(n/64)]
    float4 *sh;      // float4[ceil(n/64)]
    float4 *recp;    // float4[3n] (uniform cores) or float4[4n] (per-particle cores)
    Bounds *bounds;  // bounds of the n particles (already computed)
};
// float32 (and mixed) all-pairs near field of n free-space particles into the
// outputs (caller order); hb: the bounds' host copy (cores, extent).
void direct_f32(const Ctx &c, hipStream_t s, int64_t n, const Bounds &hb, const DirectBufs &b, const float *x,
                const float *y, const float *z, const float *ax, const float *ay, const float *az,
                const float *sigma, float *ux, float *uy, float *uz, float *dax, float *day, float *daz);
// Scale of the float32 near field: lengths times kappa = log2(e)^(1/2) / (sqrt 2 sigma)
// turn the Gaussian e^{-rho^2/(2 sigma^2)} into 2^{-rho'^2}; a = (2/sqrt pi) ln(2)^(1/2).
inline double p2p_kappa(double sigma) { return std::sqrt(1.0 / std::log(2.0)) / (std::sqrt(2.0) * sigma); }
inline double p2p_cutoff_a() { return 2.0 / std::sqrt(M_PI) * std::sqrt(std::log(2.0)); }
// direct_static.hip: looks up the scratch array's address on a device (once per device)
void resolve_static_scratch(int device);
// rbf.hip
void gaussian_sum_run(Ctx &c, int64_t n, const float *gx, const float *gy, const float *gz, float *wx, float *wy,
                      float *wz);
float gaussian_sum_ms(const Ctx &c);
void rbf_reinit_run(Ctx &c, int64_t n, const float *wx, const float *wy, const float *wz, float *gx, float *gy,
                    float *gz, double tol, int maxiter, vfmm_rbf_info *info);
// spectrum.hip
int spectrum_bins(int n);
void energy_spectrum_run(Ctx &c, int n, const float *ux, const float *uy, const float *uz, double *E_host);
// lattice_host.cpp
void lattice_operator_host(int p, int K, std::vector<double> &op);

}  // namespace vfmm

// the opaque handle of the C ABI
struct vfmm_ctx {
    vfmm::Ctx c;
};
