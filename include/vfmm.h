/*
 * vfmm.h -- C ABI of the MI355X (gfx950) vortex-particle FMM library.
 *
 * One call of fmm_build + fmm_evaluate computes, for N vortex particles with
 * positions x_i, strengths alpha_i and Gaussian cores sigma_i:
 *
 *   u_i       = sum_j q(rho) alpha_j x r,                  Biot-Savart law, Eq. (1)
 *   dalpha_i  = sum_j grad(alpha_j x grad G g_sigma) . alpha_i,  stretching, Eq. (3)
 *
 * with r = x_i - x_j, G = 1/(4 pi rho) and the Gaussian cutoff g_sigma of
 * Eq. (2) (Yokota, Barba, Narumi, Yasuoka, "Petascale turbulence simulation
 * using a highly parallel fast multipole method on GPUs", Sec. 2.1), using a
 * Morton-sorted octree, a dual tree traversal (Sec. 3.3, Algorithms 1-2), the
 * spherical-harmonic expansions P2M/M2M/M2L/L2L/L2P of the three Laplace
 * potentials psi_m = sum_j alpha_j,m G (Sec. 3.1) and the near-field P2P pass,
 * optionally in a periodic cube with image cells (Sec. 3.5).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Array pointers are DEVICE pointers to contiguous float32 arrays of length
 *   n (structure of arrays), owned by the caller.  The library never frees
 *   them and never keeps them past the call.
 * - All work is enqueued on the HIP stream given to vfmm_create and is
 *   asynchronous with respect to the host, except where a function says it
 *   synchronises.  fmm_build synchronises the stream a few times (it reads
 *   tree and list sizes back to size its buffers); fmm_evaluate does not.
 * - Outputs are in the caller's particle order.  Output arrays must not alias
 *   input arrays or each other (VFMM_EINVAL).
 * - Errors are reported as status codes; nothing aborts or throws across this
 *   boundary.  vfmm_last_error() returns a text description of the last
 *   failure on that context.
 * - The context owns the tree, expansions, interaction lists and scratch space
 *   in device memory, and 256 bytes of pinned host memory (hipHostMalloc) that
 *   the build reads its sizes through.  These only grow; vfmm_destroy frees
 *   them.
 * - A context is not thread safe; calls on one context must not overlap.
 * - Depth.  Morton keys hold 21 bits per axis (Sec. 3.2), so a cell is split
 *   at most 21 times (fewer in a batch, whose keys also carry the problem id).
 *   A cell that still holds more than ncrit particles at that depth (particles
 *   closer than 2^-21 of the root cube, coincident ones included) stays a leaf
 *   with all of them: its pairs go to the near field, which is exact for any
 *   count (coincident pairs take the r -> 0 limit of the cutoff), so results
 *   stay correct and only that leaf's work grows.  This is deliberate: no
 *   call returns VFMM_EDEPTH; vfmm_get_stats counts such leaves.
 */
#ifndef VFMM_H
#define VFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vfmm_ctx vfmm_ctx;

typedef enum {
    VFMM_OK = 0,
    VFMM_EINVAL = -1,  /* bad argument: null pointer, n < 0, aliasing, unsupported parameter */
    VFMM_ENOMEM = -2,  /* device allocation failed                                         */
    VFMM_EDEPTH = -3,  /* never returned (see "Depth" below); kept so that codes stay stable        */
    VFMM_EDOMAIN = -4, /* periodic: a position outside [lo, lo+len), or a non-finite input    */
    VFMM_ESTATE = -5,  /* fmm_evaluate without a matching fmm_build                            */
    VFMM_EHIP = -6     /* a HIP runtime call failed                                            */
} vfmm_status;

/* Arithmetic forms (vfmm_params.precision). */
enum { VFMM_PRECISION_FP32 = 0,  /* float32 throughout (default)                                   */
       VFMM_PRECISION_MIXED = 1, /* float32 with float64 or compensated accumulation of long sums  */
       VFMM_PRECISION_FP64 = 2   /* float64 reference form of the same tree, lists and expansions  */
};

/* Stretching readings of Eq. (3). */
enum { VFMM_SCHEME_TRANSPOSE = 0, /* (dalpha)_k = sum_l (du_l/dx_k) alpha_l : Eq. (3) as printed */
       VFMM_SCHEME_CLASSICAL = 1  /* (dalpha)_l = sum_k alpha_k du_l/dx_k : "omega . grad u"     */
};

typedef struct vfmm_params {
    int32_t p;           /* expansion degree n = 0..p (supported: 4, 6, 8, 10, 12)  default 10  */
    int32_t ncrit;       /* split a cell while it holds more than ncrit particles  default 64  */
    float theta;         /* multipole acceptance (R_A + R_B) < theta * D           default 0.5 */
    float sigma_gap;     /* M2L also requires D - R_A - R_B >= sigma_gap * sigma_max   default 5 */
    int32_t periodic;    /* 0 free space, 1 periodic cube [box_lo, box_lo + box_len)^3         */
    int32_t images;      /* periodic: K, image cells cover |n|_inf <= (3^K - 1)/2   default 3  */
    double box_lo[3];    /* periodic cube corner, or (free space, box_len > 0) root cube corner  */
    double box_len;      /* periodic cube side (> 0 when periodic).  Free space: 0 (default) =
                            the bounding cube of the particles; > 0 = the octree's root cube
                            [box_lo, box_lo + box_len)^3, which must hold every position
                            (VFMM_EDOMAIN otherwise; batched problems keep their own cubes):
                            a cube aligned with a particle lattice gives regular cells       */
    int32_t scheme;      /* VFMM_SCHEME_TRANSPOSE (default) or VFMM_SCHEME_CLASSICAL          */
    int32_t kahan;       /* 1: compensated per-target sums in P2P (default 0: blocked sums)    */
    int32_t zero_mean;   /* periodic: subtract (1/3V) sum x_j x alpha_j (default 1)           */
    int32_t direct;      /* 1: all-pairs P2P without a tree (test mode; free space only)      */
    int32_t m2l_mode;    /* 0 (default): operator-batched M2L when the tree's translations group
                            densely (at least 8 per (64-target block, offset) group), else per
                            pair; 1: per-pair M2L; 2: operator-batched whenever the offsets can be
                            keyed (falls back to per pair only when they cannot)                 */
    int32_t use_graph;   /* 1: fmm_evaluate runs as a hipGraph, captured on the first call after
                            a build (or when its pointers change) and replayed afterwards; needs
                            a non-default stream and the tree path (default 0)                */
    int32_t precision;   /* VFMM_PRECISION_FP32 (default): float32 records, expansions and sums.
                            VFMM_PRECISION_MIXED: as FP32, but compensated per-target P2P sums (as
                            kahan = 1), float64 accumulation in M2M, L2L and in the reduction of
                            the batched M2L's partial sums, float64 periodic lattice operator.
                            VFMM_PRECISION_FP64: particle records, expansions, every far-field
                            operator (M2L per pair) and P2P in float64 (cutoff always in its full
                            form), outputs rounded to float32 once; with the same tree and lists
                            as the other forms, its difference from them is their rounding error
                            (Sec. 4.2 normalises the expansions so that float32 stays in range). */
    int32_t overlap;     /* 0: one stream, the phases run one after the other (P2P last).  1:
                            the near field (P2P) runs on a second stream of the library
                            concurrently with the far field and a final kernel adds them (the
                            small far-field kernels then fill the GPU beside the P2P; the P2P
                            and far-field phase timings overlap).  2 (default): one stream, the
                            near field first, then P2M ... L2P, and the final kernel.  At 128^3,
                            p = 10 with m2l_form = 2: 27.5 ms (2), 26.8 ms (1) and 28.5 ms (0)
                            per build + evaluate.  Results are bitwise the same in all three. */
    int32_t m2l_form;    /* products of the operator-batched M2L.  0 or 1: float32 matrix-core
                            products.  2 (default; p <= 10, p = 12 uses 1): split products:
                            operator and multipole values are each split into three bfloat16
                            parts (24 significant bits) and the six leading partial products
                            run on the bfloat16 matrix cores with float32 accumulation; the
                            translations agree with form 1 to float32 rounding and the M2L
                            kernel takes 7.1-7.5 ms instead of 9.0 ms at 128^3, p = 10.
                            3: reduced-precision split products: two bfloat16 parts per
                            operand (16 significant bits) and only the three leading partial
                            products, half the matrix-core work of form 2; each translation
                            carries relative errors of order 1e-5, meant for error bounds near
                            1e-4 (the autotuner chooses it only where the bound holds).  p = 12
                            uses form 1 for 2 and 3.                                           */
} vfmm_params;

/* Per-phase device times of the last fmm_build / fmm_evaluate, in milliseconds,
 * measured with HIP events on the stream that runs each phase.  With overlap = 1
 * the P2P phase runs concurrently with P2M ... L2P, so those intervals overlap
 * and include time spent sharing the GPU; evaluate_ms is the whole call. */
typedef struct vfmm_timings {
    float bounds_sort_ms;   /* bounds, Morton keys, radix sort, gather            */
    float tree_ms;          /* octree levels, cell geometry                       */
    float traverse_ms;      /* dual traversal + interaction-list build            */
    float p2m_m2m_ms;       /* P2M at leaves, M2M up the tree                     */
    float lattice_ms;       /* periodic image lattice into the root local        */
    float m2l_ms;           /* all M2L translations                               */
    float l2l_l2p_ms;       /* L2L down the tree, L2P at leaves                   */
    float p2p_ms;           /* near field P2P, fused with the output scatter      */
    float build_ms;         /* whole fmm_build                                    */
    float evaluate_ms;      /* whole fmm_evaluate                                 */
} vfmm_timings;

/* Sizes of the current tree and lists (valid after fmm_build). */
typedef struct vfmm_stats {
    int64_t n;              /* particles                                          */
    int32_t ncells;         /* octree cells                                       */
    int32_t nleaves;        /* leaf cells                                         */
    int32_t depth;          /* deepest level (root = 0)                           */
    int32_t p2p_entries;    /* (target leaf, source leaf, image) triples          */
    int64_t p2p_pairs;      /* particle pairs evaluated by P2P (self pairs incl.) */
    int64_t m2l_entries;    /* (target cell, source cell, image) translations     */
    int32_t p2p_blocks;     /* P2P work items (<= 64 targets each)                */
    int32_t images_traversed; /* periodic image cells started in the traversal    */
    double sum_alpha[3];    /* float64 sum of alpha (set by fmm_evaluate)         */
    double sigma_min, sigma_max;
    int32_t m2l_keys;       /* batched M2L: distinct translation operators (0 if per pair) */
    int32_t m2l_groups;     /* batched M2L: (target block, operator) groups        */
    int32_t m2l_items;      /* batched M2L: work items (<= 24 groups of one block) */
    int32_t m2l_split;      /* batched M2L: 1 when it runs the split bf16 products
                               (six per product), 2 for the three-product form      */
    int32_t stale;          /* 1 when the last fmm_evaluate found positions or cores
                               that differ from the build's (its outputs are NaN)     */
    int32_t overfull_leaves;/* leaves holding more than ncrit particles because the
                               keys resolve no finer (21 levels, Sec. 3.2; fewer in a
                               batch): coincident or nearly coincident particles      */
} vfmm_stats;

/* Fill *p with the defaults listed above (free space). */
void vfmm_default_params(vfmm_params *p);

/* Create a context bound to hip_stream (a hipStream_t; NULL = default stream)
 * on the current HIP device.  *out receives the context.  The parameters are
 * copied.  Errors: VFMM_EINVAL for a null out or unsupported parameters
 * (p not in the supported set, ncrit < 1, theta not in (0, 1), periodic with
 * box_len <= 0, images < 1, direct together with periodic). */
vfmm_status vfmm_create(const vfmm_params *params, void *hip_stream, vfmm_ctx **out);

/* Replace the parameters of an existing context (same validation as
 * vfmm_create).  Invalidates the current tree. */
vfmm_status vfmm_set_params(vfmm_ctx *ctx, const vfmm_params *params);

/* Build the octree and interaction lists for n particles (Sec. 3.2-3.3).
 * x, y, z, sigma: device float32[n].  The tree depends on positions only; the
 * cores enter the separation test (sigma_gap * largest core) and the near
 * field, where every pair uses its source's own core (Eq. 2); cores may differ
 * per particle (equal cores take a faster near-field path).  n = 0 is allowed
 * (evaluate then writes nothing).  Errors: VFMM_EINVAL (null pointer, n < 0,
 * n >= 2^31, or - float32 and mixed forms, whose near field works in lengths
 * scaled by 1/sigma - cores below 1/(2e7) of the domain extent), VFMM_EDOMAIN
 * (non-finite input or non-positive core; periodic position outside the
 * cube), VFMM_ENOMEM (allocation failed, or the M2L or P2P list would exceed
 * 2^31 - 1 entries: about 4e8 particles at p = 10, theta = 0.5), VFMM_EHIP. */
vfmm_status fmm_build(vfmm_ctx *ctx, int64_t n, const float *x, const float *y, const float *z,
                      const float *sigma);

/* Evaluate u (Eq. 1) and dalpha/dt (Eq. 3, reading ctx scheme) at every
 * particle, using the tree of the last fmm_build, which must have been made
 * from the same n, positions and cores.  Inputs and outputs are device
 * float32[n].  Periodic with zero_mean: u is the zero-mean periodic field (the
 * cube-ordered image sum minus (1/3V) sum x_j x alpha_j).
 * The check that positions and cores are the build's: when x, y, z, sigma are
 * other arrays than the ones given to fmm_build, the call compares a float64
 * fingerprint of their contents with the build's before it starts
 * (synchronising the stream once) and returns VFMM_ESTATE on a difference.
 * When they are the same arrays, the call stays asynchronous; the device
 * compares the fingerprints and, if the contents changed since the build,
 * every output is NaN and vfmm_get_stats reports stale = 1.
 * Errors: VFMM_ESTATE (no build, n differs, or other arrays whose contents
 * differ), VFMM_EINVAL (null pointer, aliasing), VFMM_EHIP. */
vfmm_status fmm_evaluate(vfmm_ctx *ctx, int64_t n, const float *x, const float *y, const float *z,
                         const float *ax, const float *ay, const float *az, const float *sigma,
                         float *ux, float *uy, float *uz, float *dax, float *day, float *daz);

/* Radial-basis-function reinitialisation of the strengths (Sec. 2.1, last
 * paragraph; Sec. 2.2; Sec. 3.4).  The vorticity of particles with strengths
 * gamma_j and cores sigma_j is omega(x) = sum_j gamma_j zeta_j(x - x_j), with
 * zeta_j(r) = (2 pi sigma_j^2)^{-3/2} exp(-|r|^2 / (2 sigma_j^2)) the Gaussian
 * whose enclosed mass is the cutoff of Eq. (2).
 *
 * Both calls work on the particles (positions and cores) of the last
 * fmm_build, reusing its tree and near-field lists, as the paper reuses its
 * tree for particles reinitialised at the same positions; they need a plain
 * fmm_build (not batched, not with separate targets), the tree path
 * (direct = 0) and the float32 or mixed form.  The sum runs over the build's
 * near-field (P2P) lists only: pairs farther apart than sigma_gap * sigma_max
 * (those the traversal sends to M2L) are dropped, which leaves out the
 * Gaussian mass beyond that radius, 1 - g(c sigma) = 1.5e-5 at c = 5 and
 * 7.5e-8 at c = 6 (build with sigma_gap >= 6 for float32-level sums), and
 * leaf pairs at least 7.2 sigma_max apart are skipped (below e^-26 of the
 * peak).  Periodic builds sum over the image cells of their lists.  Arrays
 * are device float32[n] in the caller's order; n must equal the build's. */

/* w_i = sum_j zeta_j(x_i - x_j) gamma_j (each component), the matrix-vector
 * product of the reinitialisation.  Asynchronous.  Errors: VFMM_ESTATE (no
 * build, or n differs), VFMM_EINVAL (null pointer, aliasing, a build of the
 * wrong kind), VFMM_ENOMEM, VFMM_EHIP. */
vfmm_status fmm_gaussian_sum(vfmm_ctx *ctx, int64_t n, const float *gx, const float *gy, const float *gz,
                             float *wx, float *wy, float *wz);

typedef struct vfmm_rbf_info {
    int32_t iterations[3];  /* conjugate-gradient iterations of each component        */
    int32_t matvecs;        /* Gaussian sums evaluated (the largest of the three)       */
    double  residual[3];    /* final ||omega - A gamma|| / ||omega|| per component
                               (the iteration's recursive residual)                   */
    int64_t pairs;          /* particle pairs one Gaussian sum evaluates               */
    float   solve_ms;       /* the whole call, HIP events on the context stream        */
    float   matvec_ms;      /* the Gaussian-sum kernels alone, summed over iterations  */
} vfmm_rbf_info;

/* Strengths gamma that reproduce the vorticity omega = (wx, wy, wz) at the
 * particles: sum_j zeta_j(x_i - x_j) gamma_j = omega_i for every i, each
 * component solved by plain conjugate gradients from gamma = 0 (the matrix is
 * symmetric positive definite for one shared core), iterating until
 * ||omega - A gamma|| <= tol ||omega|| (recursive residual) or maxiter
 * iterations.  The iteration's vectors are float64, the Gaussian sums
 * float32; the float32 sums limit the reachable residual to about 1e-5
 * relative.  Synchronises the stream once per iteration.  info (host, may be
 * null) receives iteration counts, residuals and times.  Errors: as
 * fmm_gaussian_sum, and VFMM_EINVAL for tol < 0, maxiter < 0 or per-particle
 * cores (the system is then not symmetric; core spreading by Eq. 4 keeps one
 * shared core). */
vfmm_status rbf_reinit(vfmm_ctx *ctx, int64_t n, const float *wx, const float *wy, const float *wz, float *gx,
                       float *gy, float *gz, double tol, int32_t maxiter, vfmm_rbf_info *info);

/* Duration of the last fmm_gaussian_sum's kernel (ms, HIP events on the
 * context stream); synchronises the stream.  Errors: VFMM_EINVAL. */
vfmm_status vfmm_get_gaussian_ms(const vfmm_ctx *ctx, float *ms);

/* Kinetic-energy spectrum of a velocity field sampled on a uniform n^3
 * lattice (Sec. 4.3, the spectrum of the velocity at a lattice of probe
 * points, e.g. from fmm_evaluate_targets): with
 * u_hat(kappa) = n^-3 sum_t u(x_t) exp(-2 pi i kappa.t / n) over the lattice
 * indices t = (i, j, k) (input index i n^2 + j n + k), E[k] = 1/2 sum of
 * |u_hat(kappa)|^2 over the integer wavevectors with round(|kappa|) = k, for
 * k = 0 .. round(sqrt(3) n / 2) (wavenumbers in units of 2 pi / L; the sum
 * of E is half the mean of |u|^2).  ux, uy, uz: device float32[n^3]; E: HOST
 * float64[round(sqrt(3) n / 2) + 1].  Float64 FFTs on the GPU; synchronises.
 * Errors: VFMM_EINVAL (null pointer, n not a power of two in [2, 1024]),
 * VFMM_ENOMEM, VFMM_EHIP. */
vfmm_status vfmm_energy_spectrum(vfmm_ctx *ctx, int32_t n, const float *ux, const float *uy, const float *uz,
                                 double *E);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Computes what
 * fmm_build followed by fmm_evaluate compute on a context with direct = 1 (the
 * all-pairs near-field sum of Eqs. 1-3, free space, no tree), with the
 * context's scheme, kahan and precision (float32 or mixed), and the same
 * results bit for bit; the context's tree and lists are left as they were.
 * Inputs and outputs as in fmm_evaluate (device float32[n], caller order).
 * It allocates nothing: its scratch space is one device array of about
 * 6.7 MB compiled into the library, which every GPU that the library runs on
 * holds until the process ends, and it is limited to n <= VFMM_STATIC_MAX_N.
 * Every call on one GPU uses that GPU's one array: calls that overlap on one
 * GPU (from several contexts, streams or threads) race and give wrong
 * results; calls in sequence on one stream are safe.  It synchronises the
 * context stream once (the particles' bounds and cores decide the kernels'
 * constants).  Errors: VFMM_EINVAL (null pointer, aliasing, n < 0 or
 * n > VFMM_STATIC_MAX_N, a periodic context, the float64 form, cores below
 * 1/(2e7) of the extent), VFMM_EDOMAIN (non-finite input, non-positive core,
 * a position outside a root cube fixed by box_len), VFMM_EHIP. */
#define VFMM_STATIC_MAX_N 65536
vfmm_status fmm_direct_static(vfmm_ctx *ctx, int64_t n, const float *x, const float *y, const float *z,
                              const float *ax, const float *ay, const float *az, const float *sigma,
                              float *ux, float *uy, float *uz, float *dax, float *day, float *daz);

/* Velocity at target points that are not particles (Eq. 1 holds at any point
 * x; e.g. a probe lattice for spectra).  fmm_build_targets builds one tree
 * over the n particles and the m target points (targets carry no strength
 * and no core); fmm_evaluate_targets then evaluates, from the strengths of
 * the n particles, u and dalpha/dt at the particles (as fmm_evaluate) and u
 * at the targets.  Particle inputs are those of fmm_build / fmm_evaluate;
 * tx, ty, tz: device float32[m]; outputs: device float32[n] (ux .. daz) and
 * float32[m] (tux, tuy, tuz), all in the caller's order; m = 0 is allowed.
 * The library keeps float32[13 (n + m)] of combined inputs and outputs.  A
 * later fmm_build (or rk_step) ends the target set.  Errors: as fmm_build /
 * fmm_evaluate; VFMM_EINVAL also for n < 1; VFMM_ESTATE when the last build
 * was not fmm_build_targets with the same n and m. */
vfmm_status fmm_build_targets(vfmm_ctx *ctx, int64_t n, const float *x, const float *y, const float *z,
                              const float *sigma, int64_t m, const float *tx, const float *ty, const float *tz);
vfmm_status fmm_evaluate_targets(vfmm_ctx *ctx, int64_t n, const float *ax, const float *ay, const float *az,
                                 int64_t m, float *ux, float *uy, float *uz, float *dax, float *day, float *daz,
                                 float *tux, float *tuy, float *tuz);

/* Batched form: nprob independent free-space problems stored back to back in
 * the same arrays; problem b owns particles [offsets[b], offsets[b+1]).
 * offsets is a HOST int64 array of nprob+1 entries with offsets[0] = 0 and
 * every problem non-empty.  One forest is built (one root cube per problem;
 * Morton keys carry the problem id above 3 x floor((63 - bits(nprob))/3)
 * coordinate bits), so one fmm_evaluate(ctx, offsets[nprob], ...) evaluates
 * every problem with the same kernel launches; no pair between two problems
 * is ever formed.  Errors: VFMM_EINVAL (bad offsets, periodic or direct
 * context, more than 2^20 problems) and those of fmm_build. */
vfmm_status fmm_build_batched(vfmm_ctx *ctx, int32_t nprob, const int64_t *offsets, const float *x, const float *y,
                              const float *z, const float *sigma);

/* fmm_build_batched followed by fmm_evaluate on the concatenated arrays. */
vfmm_status fmm_evaluate_batched(vfmm_ctx *ctx, int32_t nprob, const int64_t *offsets, const float *x,
                                 const float *y, const float *z, const float *ax, const float *ay,
                                 const float *az, const float *sigma, float *ux, float *uy, float *uz,
                                 float *dax, float *day, float *daz);

/* One Heun (RK2) step of the vortex-particle system, in place:
 *   stage 1: build + evaluate at (x, alpha);  x* = x + dt u, alpha* = alpha + dt dalpha
 *   stage 2: build + evaluate at (x*, alpha*); x += dt/2 (u + u*), alpha += dt/2 (dalpha + dalpha*)
 *   sigma^2 += 2 nu dt                                                       (Eq. 4)
 * Periodic positions are wrapped back into the cube after each stage.  Both
 * stages re-sort and rebuild the tree.  Scratch for the stage values is owned
 * by the context.  Errors as fmm_build / fmm_evaluate. */
vfmm_status rk_step(vfmm_ctx *ctx, int64_t n, float dt, float nu, float *x, float *y, float *z,
                    float *ax, float *ay, float *az, float *sigma);

/* Result of vfmm_autotune. */
typedef struct vfmm_tune_result {
    int32_t p;             /* chosen expansion degree                                  */
    float theta;           /* chosen acceptance parameter                              */
    int32_t ncrit;         /* chosen leaf size                                         */
    float sigma_gap;       /* chosen core-overlap gap of the M2L test                  */
    int32_t precision;     /* chosen precision form (VFMM_PRECISION_FP32 or _MIXED)     */
    int32_t m2l_form;      /* chosen batched-M2L products (0 float32, 2 split bf16, 3
                              reduced-precision split bf16)                            */
    int32_t overlap;       /* chosen evaluation order (0, 1, 2 as in vfmm_params)       */
    float err_u, err_dalpha; /* rel-L2 of u and dalpha vs the high-accuracy reference  */
    float worst_u, worst_dalpha; /* largest single-target error over the RMS target
                                    magnitude, vs the same reference                  */
    float ms;              /* build + evaluate time of the chosen configuration        */
    int32_t tried;         /* configurations timed                                     */
    int32_t from_cache;    /* 1 when read from cache_path                              */
} vfmm_tune_result;

/* Choose p in {6,8,10,12}, theta in {0.3,...,0.7}, ncrit in {32,...,512},
 * sigma_gap in {4,5,6}, the precision form (float32 or mixed), the batched
 * M2L products (m2l_form 0, 2 or 3) and the evaluation order (overlap 0, 1, 2)
 * minimising the time of fmm_build + fmm_evaluate on these particles subject
 * to rel-L2(u) <= max_rel_l2 and rel-L2(dalpha) <= max_rel_l2, and no single
 * target's error above 50 max_rel_l2 of the RMS target magnitude (u and
 * dalpha; an outlier guard: at the L2 bound the largest single-target error is
 * typically 30-45 times the L2 error), where the errors are measured against the library's own p = 12, theta = 0.35,
 * sigma_gap = max(sigma_gap, 6), mixed-form evaluation of the same input.
 * Search: smallest feasible p for each theta at the context's ncrit,
 * sigma_gap and forms, then ncrit at the best (theta, p) (p + 2 if accuracy
 * drops), then sigma_gap at the best (theta, p, ncrit), then the 12
 * combinations of the three forms at the best (theta, p, ncrit, gap).  Every
 * candidate is built and evaluated twice on the GPU (the second is timed).
 * The chosen values are written into the context's parameters (the caller
 * builds again).  cache_path (may be NULL) is a text file of previous results
 * keyed by the device architecture, n, periodicity, images, box, scheme,
 * kahan, max_rel_l2 and a fingerprint of the inputs (float64 sums of
 * positions, cores, strengths and x_j x alpha_j, the core range); a hit skips
 * the search.
 * Synchronises.  Inputs are device float32[n] as for fmm_evaluate.  Errors:
 * VFMM_EINVAL (null pointer, n <= 0, max_rel_l2 <= 0, direct context, a
 * float64-form context, no feasible configuration) and those of
 * build/evaluate; on error the context's parameters are restored. */
vfmm_status vfmm_autotune(vfmm_ctx *ctx, int64_t n, const float *x, const float *y, const float *z,
                          const float *ax, const float *ay, const float *az, const float *sigma,
                          float max_rel_l2, const char *cache_path, vfmm_tune_result *out);

/* Copy the per-phase times of the last build/evaluate to *out.  Synchronises
 * the context stream.  Errors: VFMM_EINVAL for null arguments. */
vfmm_status vfmm_get_timings(const vfmm_ctx *ctx, vfmm_timings *out);

/* Copy the tree/list sizes of the last build to *out.  Synchronises the
 * context stream.  Errors: VFMM_EINVAL for null arguments. */
vfmm_status vfmm_get_stats(const vfmm_ctx *ctx, vfmm_stats *out);

/* Copy the interaction lists of the last build to HOST buffers, for checking
 * that the traversal covers every (target, source, image) particle pair once.
 * For each list entry k: target cell, source cell, image code
 * (code = (nx+B) + (2B+1)((ny+B) + (2B+1)(nz+B)) with B = 1 for images = 1 and
 * B = 4 otherwise; B = 0 in free space).  Cells are described by
 * cell_start/cell_count (ranges in the library's sorted order) and perm maps
 * sorted position -> caller index.  Pass NULL for any array not wanted;
 * sizes come from vfmm_get_stats (ncells, p2p_entries, m2l_entries, n).
 * Synchronises.  Errors: VFMM_ESTATE without a build. */
vfmm_status vfmm_copy_lists(vfmm_ctx *ctx, int32_t *p2p_tgt, int32_t *p2p_src, int32_t *p2p_img,
                            int32_t *m2l_tgt, int32_t *m2l_src, int32_t *m2l_img,
                            int32_t *cell_start, int32_t *cell_count, int32_t *perm);

/* Copy the tree and the expansions of the last build and evaluation to HOST
 * buffers, for checking each far-field operator (Sec. 3.1: P2M, M2M, L2L,
 * L2P) against its definition.  Pass NULL for any array not wanted; ncells,
 * n and p as in vfmm_get_stats and the parameters.  Per cell i:
 *   level[i], parent[i] (-1 at a root), first_child[i], nchild[i] (its
 *   children are first_child .. first_child + nchild - 1; 0 for a leaf);
 *   geo[5i .. 5i+4] = centre x, y, z, cube side s and the radius used by the
 *   acceptance test (float32 values widened to double).
 * mult and loc: double[ncells][3][NC][2], NC = (p+1)(p+2)/2, the coefficients
 * c_n^m (0 <= m <= n <= p at index n(n+1)/2 + m; real, imaginary part; the
 * other orders are c_n^{-m} = (-1)^m conj(c_n^m)) of the Laplace potentials
 * psi_k(x) = sum_j q_jk / |x - x_j|, q_j = alpha_j / (4 pi), k = x, y, z, with
 *   R_n^m(r) = r^n P_n^m(cos t) e^{i m phi} / (n+m)!,
 *   I_n^m(r) = (n-m)! P_n^m(cos t) e^{i m phi} / r^{n+1}
 * (associated Legendre functions with the Condon-Shortley phase):
 *   mult: Mt_n^m = sum_j q_j conj(R_n^m((x_j - c)/s)) over the cell's
 *         particles, psi = (1/s) sum_{n <= p, |m| <= n} Mt_n^m I_n^m((x - c)/s)
 *         away from the cell;
 *   loc:  psi(x) = (1/s) sum Lt_n^m R_n^m((x - c)/s) is the part of the field
 *         the far field delivers to the cell (its own translations and its
 *         ancestors', and the periodic lattice term).
 * far_u, far_da: double[3][n] in the library's sorted order (perm of
 * vfmm_copy_lists): the far-field part of u and dalpha at each particle (L2P
 * of its leaf's local expansion).  The values are the library's float32
 * numbers (float64 in the float64 form).  Synchronises.  Errors: VFMM_EINVAL
 * (null ctx), VFMM_ESTATE (no tree: no build, direct mode, n = 0, or after
 * rk_step; and for mult, loc, far_u, far_da when no evaluation has run since
 * the build). */
vfmm_status vfmm_copy_expansions(vfmm_ctx *ctx, int32_t *level, int32_t *parent, int32_t *first_child,
                                 int32_t *nchild, double *geo, double *mult, double *loc, double *far_u,
                                 double *far_da);

/* Text of the last error on ctx (never NULL; "" when none).  Valid until the
 * next call on ctx.  A NULL ctx returns the last vfmm_create failure. */
const char *vfmm_last_error(const vfmm_ctx *ctx);

/* Free every device and host resource of ctx (NULL is ignored).
 * Synchronises the context stream first. */
void vfmm_destroy(vfmm_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* VFMM_H */
