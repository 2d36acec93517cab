// Dual tree traversal (Sec. 3.3, Algorithms 1 and 2) and interaction-list
// construction ("GPU buffering", Sec. 4.4).
//
// The paper's stack of cell pairs becomes a frontier processed one
// generation at a time: each pair splits its cell of larger radius (the other
// one when that cell is a leaf) and every child pair is classified
//   M2L  if (R_A + R_B) < theta D  and  D - R_A - R_B >= sigma_gap sigma_max,
//   P2P  else if both cells are leaves,
//   push else (next generation).
// Counts, an exclusive scan and a write pass keep the output order fixed, so
// the lists (and every sum built from them) are bit-reproducible.  Periodic
// images enter as an image code on each pair: the source cell is shifted by
// n * box_len.
#include "ctx.h"
#include "cutoff_fits.h"

namespace vfmm {

static constexpr int TPB = 256;

void sort_pairs_u64(Ctx &c, DevBuf &kA, DevBuf &vA, DevBuf &kB, DevBuf &vB, int64_t n, int nbits);

struct TravArgs {
    const int *child, *nchild;
    const float4 *geo;
    const float *rad;
    float theta, gap;  // gap = sigma_gap * sigma_max
    const float4 *hi;  // per-source cores: cell boxes whose .w is the cell's largest core (else null)
    float sgap;        // sigma_gap (with hi)
    float len;         // periodic cube side (0 in free space)
    int B;             // image range |n|_inf <= B
};

__device__ inline void img_shift(int code, int B, float len, float &sx, float &sy, float &sz) {
    const int W = 2 * B + 1;
    const int ix = code % W - B;
    const int iy = (code / W) % W - B;
    const int iz = code / (W * W) - B;
    sx = ix * len;
    sy = iy * len;
    sz = iz * len;
}

// Decisions on distances and radii use a relative margin TIE_TOL: quantities
// that agree to within float32 rounding of the cell coordinates (exact ties
// are common in regular particle layouts) are decided the same way for every
// cell pair, so pairs related by a translation of the tree get equal lists.
static constexpr float TIE_TOL = 1.0f / 65536.0f;

// 0 = M2L, 1 = P2P, 2 = push
__device__ inline int interact(const TravArgs &A, int a, int b, int img) {
    float sx, sy, sz;
    img_shift(img, A.B, A.len, sx, sy, sz);
    const float4 ga = A.geo[a], gb = A.geo[b];
    const float dx = ga.x - gb.x - sx, dy = ga.y - gb.y - sy, dz = ga.z - gb.z - sz;
    const float D = sqrtf(dx * dx + dy * dy + dz * dz);
    const float ra = A.rad[a], rb = A.rad[b];
    // the MAC and the core gap, both failing on (near-)ties; with per-source
    // cores the gap is measured in the largest core of the source cell b
    const float gap = A.hi ? A.sgap * A.hi[b].w : A.gap;
    if (ra + rb < A.theta * D * (1.0f - TIE_TOL) && D - ra - rb >= gap + TIE_TOL * D) return 0;
    if (A.nchild[a] == 0 && A.nchild[b] == 0) return 1;
    return 2;
}

// Children pairs of a frontier pair (Algorithm 1): split A when its radius is
// larger (radii equal to within TIE_TOL split B), unless the chosen cell is a
// leaf.
__device__ inline void split_pair(const TravArgs &A, int a, int b, bool &splitA, int &first, int &cnt) {
    const float ra = A.rad[a], rb = A.rad[b];
    const bool la = A.nchild[a] == 0, lb = A.nchild[b] == 0;
    splitA = (ra > rb * (1.0f + TIE_TOL) && !la) || lb;
    const int s = splitA ? a : b;
    first = A.child[s];
    cnt = A.nchild[s];
}

__global__ __launch_bounds__(TPB) void k_trav_count(TravArgs A, const int4 *fr, int nf, int split, int *cnt) {
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i >= nf) return;
    const int4 pr = fr[i];
    int c[3] = {0, 0, 0};
    if (!split) {
        c[interact(A, pr.x, pr.y, pr.z)]++;
    } else {
        bool sa;
        int first, n;
        split_pair(A, pr.x, pr.y, sa, first, n);
        for (int k = 0; k < n; ++k) {
            const int a = sa ? first + k : pr.x;
            const int b = sa ? pr.y : first + k;
            c[interact(A, a, b, pr.z)]++;
        }
    }
    cnt[i] = c[0];
    cnt[nf + i] = c[1];
    cnt[2 * nf + i] = c[2];
}

__global__ void k_trav_totals(const int *cnt, const int *off, int nf, int *tot) {
    for (int k = 0; k < 3; ++k) tot[k] = off[(k + 1) * nf - 1] + cnt[(k + 1) * nf - 1] - off[k * nf];
}

__global__ __launch_bounds__(TPB) void k_trav_write(TravArgs A, const int4 *fr, int nf, int split, const int *off,
                                                    int4 *m2l, int m2l_base, int4 *p2p, int p2p_base, int4 *next) {
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i >= nf) return;
    const int4 pr = fr[i];
    int o[3] = {off[i] - off[0] + m2l_base, off[nf + i] - off[nf] + p2p_base, off[2 * nf + i] - off[2 * nf]};
    auto emit = [&](int a, int b) {
        const int k = interact(A, a, b, pr.z);
        const int4 e = make_int4(a, b, pr.z, 0);
        if (k == 0) m2l[o[0]++] = e;
        else if (k == 1) p2p[o[1]++] = e;
        else next[o[2]++] = e;
    };
    if (!split) {
        emit(pr.x, pr.y);
    } else {
        bool sa;
        int first, n;
        split_pair(A, pr.x, pr.y, sa, first, n);
        for (int k = 0; k < n; ++k) emit(sa ? first + k : pr.x, sa ? pr.y : first + k);
    }
}

// one (root, root, image) pair per problem and image code
__global__ __launch_bounds__(TPB) void k_trav_init(int4 *fr, int nroot, int ncode) {
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i < nroot * ncode) fr[i] = make_int4(i / ncode, i / ncode, i % ncode, 0);
}

// ---------------------------------------------------------------------------
// CSR by target cell.  Entries are stably sorted by target, so within a
// target they keep the traversal's (deterministic) order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TPB) void k_list_keys(const int4 *raw, int64_t n, uint64_t *key, uint32_t *val) {
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= n) return;
    key[i] = (uint64_t)(uint32_t)raw[i].x;
    val[i] = (uint32_t)i;
}

// CSR offsets from the sorted targets: off[t] = first position with target >= t
// (t = 0 .. nc), by a binary search per target: a thread per target, so a long
// run of cells without entries (the internal cells) costs no serial loop.
__global__ __launch_bounds__(TPB) void k_csr_bounds(const uint64_t *key, int64_t n, int nc, int *off) {
    const int t = blockIdx.x * TPB + threadIdx.x;
    if (t > nc) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)key[mid] < t) lo = mid + 1;
        else hi = mid;
    }
    off[t] = (int)lo;
}

__global__ __launch_bounds__(TPB) void k_m2l_gather(const int4 *raw, const uint32_t *order, int64_t n, int2 *out,
                                                    int *tgt) {
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= n) return;
    const int4 e = raw[order[i]];
    out[i] = make_int2(e.y, e.z);
    tgt[i] = e.x;
}

struct P2PEntryArgs {
    const int *start, *count;
    const float4 *lo, *hi;
    const float4 *geo;        // cell centres
    float len;
    int B;
    float r2_small, r2_sing;  // thresholds on squared distance for the cutoff branches
    int per_cell;             // per-source cores: thresholds from the source leaf's largest core (hi.w)
    double kappa;             // length scale of the float32 near field
    double len64;             // period (0: free space)
    const int *nsrc;          // partitioned builds: sources in front of each leaf's targets (else null)
    float4 *sh;               // out: kappa (c_t - c_s - image shift) per entry (null: not needed)
};

// entry = (source start, source count, image code, variant) with variant
// 0 = full cutoff (some pair may have s < 1), 1 = s >= 1 for every pair,
// 2 = cutoff equal to 1 in float32 for every pair (singular kernel).  The
// float32 near field also gets the scaled offset between the leaf centres.
__global__ __launch_bounds__(TPB) void k_p2p_gather(P2PEntryArgs A, const int4 *raw, const uint32_t *order,
                                                    int64_t n, int4 *out, unsigned long long *part) {
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    unsigned long long np = 0;
    if (i < n) {
        const int4 e = raw[order[i]];
        const int t = e.x, s = e.y;
        float sx, sy, sz;
        const int W = 2 * A.B + 1;
        sx = (e.z % W - A.B) * A.len;
        sy = ((e.z / W) % W - A.B) * A.len;
        sz = (e.z / (W * W) - A.B) * A.len;
        const float4 tl = A.lo[t], th = A.hi[t], sl = A.lo[s], sh = A.hi[s];
        const float gx = fmaxf(0.f, fmaxf(sl.x + sx - th.x, tl.x - sh.x - sx));
        const float gy = fmaxf(0.f, fmaxf(sl.y + sy - th.y, tl.y - sh.y - sy));
        const float gz = fmaxf(0.f, fmaxf(sl.z + sz - th.z, tl.z - sh.z - sz));
        const float d2 = gx * gx + gy * gy + gz * gz;
        float r2s = A.r2_small, r2g = A.r2_sing;
        if (A.per_cell) {  // every pair's source core is at most the source leaf's largest
            const float s2 = 2.0f * sh.w * sh.w;
            r2s = s2 * VFMM_CUTOFF_XSPLIT * 1.0001f;
            r2g = s2 * 26.0f;
        }
        const int variant = d2 >= r2g ? 2 : (d2 >= r2s ? 1 : 0);
        const int sc = A.nsrc ? A.nsrc[s] : A.count[s];  // only sources enter the near field
        out[i] = make_int4(A.start[s], sc, e.z, variant);
        if (A.sh) {
            const float4 ct = A.geo[t], cs = A.geo[s];
            const double L = A.len64;
            const double Dx = ((double)ct.x - (double)cs.x - (double)(e.z % W - A.B) * L) * A.kappa;
            const double Dy = ((double)ct.y - (double)cs.y - (double)((e.z / W) % W - A.B) * L) * A.kappa;
            const double Dz = ((double)ct.z - (double)cs.z - (double)(e.z / (W * W) - A.B) * L) * A.kappa;
            A.sh[i] = make_float4((float)Dx, (float)Dy, (float)Dz, 0.f);
        }
        np = (unsigned long long)A.count[t] * (unsigned long long)sc;
    }
    // block reduction of the pair count
    __shared__ unsigned long long sh[TPB];
    sh[threadIdx.x] = np;
    __syncthreads();
    for (int o = TPB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];  // summed by k_sum_u64 (no contended atomics)
}

// total of n unsigned 64-bit partial counts (one work-group)
__global__ __launch_bounds__(TPB) void k_sum_u64(const unsigned long long *part, int n, unsigned long long *out) {
    __shared__ unsigned long long sh[TPB];
    unsigned long long v = 0;
    for (int i = threadIdx.x; i < n; i += TPB) v += part[i];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = TPB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

__global__ __launch_bounds__(TPB) void k_block_counts(const int *leaves, int nl, const int *count, int *nb) {
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i < nl) nb[i] = (count[leaves[i]] + 63) / 64;
}

__global__ __launch_bounds__(TPB) void k_block_fill(const int *leaves, int nl, const int *start, const int *count,
                                                    const int *boff, const int *loff, int4 *blocks) {
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i >= nl) return;
    const int cell = leaves[i];
    const int s = start[cell], cnt = count[cell];
    const int l0 = loff[cell], l1 = loff[cell + 1];
    int b = boff[i];
    for (int k = 0; k < cnt; k += 64) blocks[b++] = make_int4(s + k, min(64, cnt - k), l0, l1 - l0);
}

static int bits_for(int64_t v) {
    int b = 1;
    while ((1LL << b) < v) ++b;
    return b;
}

static void grow_keep4(Ctx &c, DevBuf &b, size_t bytes, size_t used) {
    if (bytes <= b.cap) return;
    DevBuf nb;
    nb.ensure(bytes * 3 / 2);
    if (used) VFMM_HIP(hipMemcpyAsync(nb.ptr, b.ptr, used, hipMemcpyDeviceToDevice, c.stream));
    VFMM_HIP(hipStreamSynchronize(c.stream));
    b.release();
    b = nb;
}

// Builds CSR offsets (ncells+1) for a raw (tgt, src, img) list and the
// stable order that sorts it by target.
static void csr_by_target(Ctx &c, const int4 *raw, int64_t n, DevBuf &off) {
    hipStream_t s = c.stream;
    const int nc = c.ncells;
    off.ensure(sizeof(int) * ((size_t)nc + 1));
    if (n == 0) {
        VFMM_HIP(hipMemsetAsync(off.ptr, 0, sizeof(int) * ((size_t)nc + 1), s));
        return;
    }
    c.lkey.ensure(sizeof(uint64_t) * n);
    c.lval.ensure(sizeof(uint32_t) * n);
    k_list_keys<<<cdiv(n, TPB), TPB, 0, s>>>(raw, n, c.lkey.as<uint64_t>(), c.lval.as<uint32_t>());
    VFMM_LAUNCH_CHECK();
    sort_pairs_u64(c, c.lkey, c.lval, c.lkey2, c.lval2, n, bits_for(nc));
    k_csr_bounds<<<cdiv(nc + 1, TPB), TPB, 0, s>>>(c.lkey.as<uint64_t>(), n, nc, off.as<int>());
    VFMM_LAUNCH_CHECK();
}

// M2L list in CSR order by target cell (stable: traversal order within a
// target), for the per-pair M2L kernel and for vfmm_copy_lists.
void build_m2l_csr(Ctx &c) {
    hipStream_t s = c.stream;
    const int64_t n_m2l = c.n_m2l;
    csr_by_target(c, c.m2l_raw.as<int4>(), n_m2l, c.m2l_off);
    c.m2l_src.ensure(sizeof(int2) * (size_t)std::max<int64_t>(n_m2l, 1));
    c.m2l_tgt.ensure(sizeof(int) * (size_t)std::max<int64_t>(n_m2l, 1));
    if (n_m2l > 0) {
        k_m2l_gather<<<cdiv(n_m2l, TPB), TPB, 0, s>>>(c.m2l_raw.as<int4>(), c.lval.as<uint32_t>(), n_m2l,
                                                       c.m2l_src.as<int2>(), c.m2l_tgt.as<int>());
        VFMM_LAUNCH_CHECK();
    }
    c.m2l_csr = true;
}

void traverse_and_lists(Ctx &c) {
    hipStream_t s = c.stream;
    TravArgs A{};
    A.child = c.c_child.as<int>();
    A.nchild = c.c_nchild.as<int>();
    A.geo = c.c_geo.as<float4>();
    A.rad = c.c_rad.as<float>();
    A.theta = c.prm.theta;
    A.gap = (float)(c.prm.sigma_gap * c.hb.sig_max);
    if (c.var_sigma) {  // the core gap of each source cell's own largest core
        A.hi = c.c_hi.as<float4>();
        A.sgap = c.prm.sigma_gap;
    }
    A.len = c.prm.periodic ? (float)c.prm.box_len : 0.f;
    A.B = c.img_B;
    const int ncode = c.img_codes;
    c.images_traversed = ncode;

    int nf = ncode * c.nprob;
    c.frA.ensure(sizeof(int4) * (size_t)nf);
    k_trav_init<<<cdiv(nf, TPB), TPB, 0, s>>>(c.frA.as<int4>(), c.nprob, ncode);
    VFMM_LAUNCH_CHECK();
    int64_t n_m2l = 0, n_p2p = 0;
    c.m2l_raw.ensure(sizeof(int4) * 1024);
    c.p2p_raw.ensure(sizeof(int4) * 1024);
    int split = 0;
    int h_tot[4];
    while (nf > 0) {
        c.tcnt.ensure(sizeof(int) * 6 * (size_t)nf + 64);
        int *cnt = c.tcnt.as<int>();
        int *off = cnt + 3 * (size_t)nf;
        k_trav_count<<<cdiv(nf, TPB), TPB, 0, s>>>(A, c.frA.as<int4>(), nf, split, cnt);
        VFMM_LAUNCH_CHECK();
        scan_excl_i32(c, cnt, off, 3LL * nf);
        k_trav_totals<<<1, 1, 0, s>>>(cnt, off, nf, pinned_ints(c));  // straight to pinned host memory
        VFMM_LAUNCH_CHECK();
        sync_ints(c, 3, h_tot);
        const int tm = h_tot[0], tp = h_tot[1], tn = h_tot[2];
        // list positions and frontier counts are 32-bit on the device: refuse before the
        // write pass rather than let an offset wrap (a pair emits at most 8 of each, so
        // a frontier below 2^28 keeps this generation's own totals exact)
        if (tm < 0 || tp < 0 || tn < 0 || n_m2l + tm > INT32_MAX || n_p2p + tp > INT32_MAX || tn > (1 << 28))
            throw Error{VFMM_ENOMEM, "interaction lists exceed 2^31 entries"};
        grow_keep4(c, c.m2l_raw, sizeof(int4) * (size_t)(n_m2l + tm), sizeof(int4) * (size_t)n_m2l);
        grow_keep4(c, c.p2p_raw, sizeof(int4) * (size_t)(n_p2p + tp), sizeof(int4) * (size_t)n_p2p);
        c.frB.ensure(sizeof(int4) * (size_t)std::max(tn, 1));
        k_trav_write<<<cdiv(nf, TPB), TPB, 0, s>>>(A, c.frA.as<int4>(), nf, split, off, c.m2l_raw.as<int4>(),
                                                    (int)n_m2l, c.p2p_raw.as<int4>(), (int)n_p2p,
                                                    c.frB.as<int4>());
        VFMM_LAUNCH_CHECK();
        n_m2l += tm;
        n_p2p += tp;
        std::swap(c.frA, c.frB);
        nf = tn;
        split = 1;
    }
    c.n_m2l = n_m2l;
    c.n_p2p = (int)n_p2p;

    // ---- M2L CSR: only for the per-pair M2L (the batched plan reads the raw list) ----
    c.m2l_csr = false;
    if (!(c.prm.m2l_mode != 1 && c.prm.precision != VFMM_PRECISION_FP64)) build_m2l_csr(c);
    // ---- P2P CSR ----
    csr_by_target(c, c.p2p_raw.as<int4>(), n_p2p, c.p2p_off);
    c.p2p_ent.ensure(sizeof(int4) * (size_t)std::max<int64_t>(n_p2p, 1));
    const bool f32 = c.prm.precision != VFMM_PRECISION_FP64;
    if (f32) c.p2p_sh.ensure(sizeof(float4) * (size_t)std::max<int64_t>(n_p2p, 1));
    c.pairs64.ensure(64);
    VFMM_HIP(hipMemsetAsync(c.pairs64.ptr, 0, 8, s));
    if (n_p2p > 0) {
        P2PEntryArgs E{};
        E.start = c.c_start.as<int>();
        E.count = c.c_count.as<int>();
        E.lo = c.c_lo.as<float4>();
        E.hi = c.c_hi.as<float4>();
        E.len = A.len;
        E.B = c.img_B;
        const float s2 = 2.0f * (float)(c.hb.sig_max * c.hb.sig_max);
        E.r2_small = s2 * VFMM_CUTOFF_XSPLIT * 1.0001f;
        E.r2_sing = s2 * 26.0f;
        E.per_cell = c.var_sigma ? 1 : 0;
        E.geo = c.c_geo.as<float4>();
        E.kappa = c.var_sigma ? 1.0 : p2p_kappa(c.sigma_uniform);  // per-source cores: unscaled offsets
        E.len64 = c.prm.periodic ? c.prm.box_len : 0.0;
        E.nsrc = c.n_src_part >= 0 && c.n_src_part < c.n ? c.c_nsrc.as<int>() : nullptr;
        E.sh = f32 ? c.p2p_sh.as<float4>() : nullptr;
        const int ngb = (int)cdiv(n_p2p, TPB);
        c.gpart.ensure(sizeof(unsigned long long) * (size_t)ngb);
        k_p2p_gather<<<ngb, TPB, 0, s>>>(E, c.p2p_raw.as<int4>(), c.lval.as<uint32_t>(), n_p2p, c.p2p_ent.as<int4>(),
                                         c.gpart.as<unsigned long long>());
        VFMM_LAUNCH_CHECK();
        k_sum_u64<<<1, TPB, 0, s>>>(c.gpart.as<unsigned long long>(), ngb, c.pairs64.as<unsigned long long>());
        VFMM_LAUNCH_CHECK();
    }
    // ---- P2P work blocks (<= 64 targets each) ----
    const int nl = c.nleaves;
    c.c_tmp.ensure(sizeof(int) * (2 * (size_t)nl + 2));
    int *nb = c.c_tmp.as<int>();
    int *boff = nb + nl + 1;
    k_block_counts<<<cdiv(nl, TPB), TPB, 0, s>>>(c.leaves.as<int>(), nl, c.c_count.as<int>(), nb);
    VFMM_LAUNCH_CHECK();
    scan_excl_i32(c, nb, boff, nl);
    int h4[4];
    read_ints(c, {boff + nl - 1, nb + nl - 1, c.pairs64.as<int>(), c.pairs64.as<int>() + 1}, h4);
    h_tot[0] = h4[0];
    h_tot[1] = h4[1];
    const unsigned long long pairs = (unsigned long long)(uint32_t)h4[2] | ((unsigned long long)(uint32_t)h4[3] << 32);
    c.n_blocks = h_tot[0] + h_tot[1];
    c.p2p_pairs = (int64_t)pairs;
    c.blocks.ensure(sizeof(int4) * (size_t)std::max(c.n_blocks, 1));
    k_block_fill<<<cdiv(nl, TPB), TPB, 0, s>>>(c.leaves.as<int>(), nl, c.c_start.as<int>(), c.c_count.as<int>(),
                                                boff, c.p2p_off.as<int>(), c.blocks.as<int4>());
    VFMM_LAUNCH_CHECK();
}

}  // namespace vfmm
