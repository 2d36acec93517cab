// Operator-batched M2L (Sec. 3.1, Sec. 3.6).
//
// An M2L translation between a target cell A and a source cell B depends only
// on the level difference dl = level(B) - level(A) and on the offset
// c_B + shift - c_A in units of s_A / 2^(max(dl,0)+2) (octree centres lie on
// that grid), for the size-normalised expansions.  A uniform octree has only a
// few thousand distinct such keys, so each key's translation is built once as
// a real (P+1)^2 x (P+1)^2 matrix T acting on (Re, Im) of Mt and producing
// (Re, Im) rows of Lt:
//   Lt_k^l = (-1)^{k+l} (s_A/s_B)^{k+1} sum_{n,m} Mt_n^m I_{n+k}^{m-l}((c_A - c_B)/s_B).
// Plan (once per tree): the distinct keys are numbered and each key's matrix
// is built into an HBM table in MFMA operand order (k_m2lb_optab).  Target
// cells are cut into blocks of 64 cells of one level and one octant class
// (cells whose position in their parent, and in their grandparent where the
// level is large enough, agree), so that the 64 targets of a block share
// almost all of their keys; the translations are grouped by (block, key) by
// counting.  Evaluation: a work-group of four waves takes up to ITEM_GROUPS
// keys of one block; each wave holds its operator rows in registers, the
// group stages the source multipoles of the 64 target slots in LDS, and the
// products [rows x inputs] x [inputs x 64 targets] run on FP32 matrix-core
// instructions (v_mfma_f32_16x16x4f32).  Partial sums of the work items are
// added per block in item order, so results are bit-reproducible.  Trees
// whose groups stay sparse (irregular particle sets) use the per-pair M2L.
#include <algorithm>
#include <type_traits>
#include <utility>

#include "ctx.h"

namespace vfmm {

static constexpr int TPB = 256;
static constexpr int ITEM_GROUPS = 24;
static constexpr int TABLE_KEY_BITS = 24;  // offset keys up to this width are numbered through a direct table
static constexpr size_t MAX_TABLE_BYTES = size_t(8) << 30;  // operator table cap (else the per-pair kernel)
static constexpr int MIN_GROUP_FILL = 8;  // translations per (block, key) group below which per-pair M2L runs

void sort_pairs_u64(Ctx &c, DevBuf &kA, DevBuf &vA, DevBuf &kB, DevBuf &vB, int64_t n, int nbits);

__host__ __device__ constexpr int NR(int P) { return (P + 1) * (P + 1); }      // real rows
__host__ __device__ constexpr int NRP(int P) { return (NR(P) + 15) / 16 * 16; } // inputs padded to 16
__host__ __device__ constexpr int NRT(int P) { return (NR(P) + 15) / 16 * 16; } // rows padded to 16

// Within each chunk of 16 input rows the (e, kq) digits of a row r = 16 c + 4 e + kq
// are swapped, so that the four rows one MFMA lane needs for k steps 4c..4c+3
// are contiguous: position 16 c + 4 kq + e.  The map is its own inverse.
__host__ __device__ constexpr int kperm(int r) { return (r & ~15) | ((r & 3) << 2) | ((r >> 2) & 3); }

// real index r = k^2 + j:  j = 0 -> (l = 0, Re); j odd -> (l = (j+1)/2, Re); j even > 0 -> (l = j/2, Im)
__host__ __device__ inline void decode_row(int r, int &k, int &l, int &im) {
    k = 0;
    while ((k + 1) * (k + 1) <= r) ++k;
    const int j = r - k * k;
    l = (j + 1) / 2;
    im = (j > 0 && (j & 1) == 0) ? 1 : 0;
}

struct KeyFmt {
    int bq;       // bits per offset component
    int bdl;      // bits of the level difference
    int oq, odl;  // offsets making the packed fields non-negative
};

// Blocking of target cells: the M2L list of a cell in a uniform region is
// fixed by its position in its parent (and, more weakly, the parent's in the
// grandparent), so the 64 targets of a block are taken from one such class:
// cells of one level with equal octant digits, in Morton order.  Per level the
// mode is 0 (no class), 1 (own octant) or 2 (own and parent's octant), chosen
// from the number of cells in the level so that classes still fill blocks.
struct ClassModes {
    int m[23];
};

__global__ __launch_bounds__(TPB) void k_cell_class(int ncells, const int *level, const int *start,
                                                    const uint64_t *keys, int KL, ClassModes M, int *cls) {
    const int c = blockIdx.x * TPB + threadIdx.x;
    if (c >= ncells) return;
    const int lv = level[c];
    const int mode = M.m[lv];
    const uint64_t k = keys[start[c]];
    int v = 0;
    if (mode >= 1) v = (int)((k >> (3 * (KL - lv))) & 7);
    if (mode >= 2) v = v * 8 + (int)((k >> (3 * (KL - lv + 1))) & 7);
    cls[c] = v;
}

// Blocks from the classes on the device: a cell's bucket is 64 level + class;
// a stable sort by bucket keeps the cells of a bucket in cell (Morton) order,
// and the blocks of 64 are numbered bucket by bucket.
constexpr int NBUCKET = 64 * 23;

__global__ __launch_bounds__(TPB) void k_cell_bucket(int nc, const int *level, const int *cls, uint64_t *key,
                                                     uint32_t *val) {
    const int c = blockIdx.x * TPB + threadIdx.x;
    if (c >= nc) return;
    key[c] = (uint64_t)(64 * level[c] + cls[c]);
    val[c] = (uint32_t)c;
}

// first and one-past-last sorted position of every bucket that holds cells
__global__ __launch_bounds__(TPB) void k_bucket_ranges(int nc, const uint64_t *key, int *bstart, int *bend) {
    const int j = blockIdx.x * TPB + threadIdx.x;
    if (j >= nc) return;
    const int k = (int)key[j];
    if (j == 0 || (int)key[j - 1] != k) bstart[k] = j;
    if (j == nc - 1 || (int)key[j + 1] != k) bend[k] = j + 1;
}

// block offset of every bucket (exclusive scan of its block count) and the
// total, in one work-group of 1024 threads, two buckets per thread
__global__ __launch_bounds__(1024) void k_bucket_blocks(const int *bstart, const int *bend, int *boff, int *nblk) {
    static_assert(2 * 1024 >= NBUCKET, "two buckets per thread");
    __shared__ int wsum[16];
    const int t = threadIdx.x;
    int v[2], tot = 0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int k = 2 * t + q;
        v[q] = k < NBUCKET ? (bend[k] - bstart[k] + 63) / 64 : 0;
        tot += v[q];
    }
    int x = tot;  // inclusive scan within the wave
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if ((t & 63) >= o) x += y;
    }
    if ((t & 63) == 63) wsum[t >> 6] = x;
    __syncthreads();
    if (t < 64) {
        int w = t < 16 ? wsum[t] : 0;
        for (int o = 1; o < 16; o <<= 1) {
            const int y = __shfl_up(w, o, 64);
            if (t >= o) w += y;
        }
        if (t < 16) wsum[t] = w;
    }
    __syncthreads();
    int e = x - tot + ((t >> 6) ? wsum[(t >> 6) - 1] : 0);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int k = 2 * t + q;
        if (k < NBUCKET) boff[k] = e;
        e += v[q];
    }
    if (t == 1023) *nblk = e;
}

__global__ __launch_bounds__(TPB) void k_bucket_assign(int nc, const uint64_t *key, const uint32_t *val,
                                                       const int *bstart, const int *boff, int2 *cell_bs,
                                                       int *bcells) {
    const int j = blockIdx.x * TPB + threadIdx.x;
    if (j >= nc) return;
    const int k = (int)key[j];
    const int i = j - bstart[k];
    const int blk = boff[k] + i / 64, slot = i % 64;
    const int cell = (int)val[j];
    cell_bs[cell] = make_int2(blk, slot);
    bcells[(size_t)blk * 64 + slot] = cell;
}

// ---------------------------------------------------------------------------
// per entry: level difference and quantised offset; track the ranges
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TPB) void k_m2lb_offsets(int64_t n, const int4 *raw, const float4 *geo, const int *level,
                                                      int B, float len, int4 *eq, int *range) {
    __shared__ int red[2][TPB / 64];
    int aq = 0, adl = 0;
    const int W = 2 * B + 1;
    for (int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB) {
        const int4 r = raw[e];  // (target, source, image code, -)
        const int t = r.x;
        const int2 s = make_int2(r.y, r.z);
        const float shx = (float)(s.y % W - B) * len;
        const float shy = (float)((s.y / W) % W - B) * len;
        const float shz = (float)(s.y / (W * W) - B) * len;
        const float4 ga = geo[t], gb = geo[s.x];
        const int dl = level[s.x] - level[t];
        const float unit = ga.w * exp2f(-(float)(max(dl, 0) + 2));
        const int qx = (int)rintf((gb.x + shx - ga.x) / unit);
        const int qy = (int)rintf((gb.y + shy - ga.y) / unit);
        const int qz = (int)rintf((gb.z + shz - ga.z) / unit);
        eq[e] = make_int4(qx, qy, qz, dl);
        aq = max(aq, max(abs(qx), max(abs(qy), abs(qz))));
        adl = max(adl, abs(dl));
    }
    // block max, then one atomic per block (the grid is capped, so few atomics)
    for (int o = 32; o > 0; o >>= 1) {
        aq = max(aq, __shfl_xor(aq, o, 64));
        adl = max(adl, __shfl_xor(adl, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = aq;
        red[1][threadIdx.x >> 6] = adl;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < TPB / 64; ++w) {
            aq = max(aq, red[0][w]);
            adl = max(adl, red[1][w]);
        }
        atomicMax(&range[0], aq);
        atomicMax(&range[1], adl);
    }
}

__device__ inline uint64_t pack_key(int4 q, const KeyFmt &f) {
    return ((uint64_t)(q.w + f.odl) << (3 * f.bq)) | ((uint64_t)(q.x + f.oq) << (2 * f.bq)) |
           ((uint64_t)(q.y + f.oq) << f.bq) | (uint64_t)(q.z + f.oq);
}

__global__ __launch_bounds__(TPB) void k_m2lb_pack(int64_t n, const int4 *eq, KeyFmt f, uint64_t *key, uint32_t *val) {
    const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= n) return;
    key[e] = pack_key(eq[e], f);
    val[e] = (uint32_t)e;
}

// compact key spaces: mark the keys in use in a direct table (every writer
// stores the same value), number them by a scan, look the numbers up
__global__ __launch_bounds__(TPB) void k_key_mark(int64_t n, const int4 *eq, KeyFmt f, int *tab) {
    const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (e < n) tab[pack_key(eq[e], f)] = 1;
}

__global__ __launch_bounds__(TPB) void k_key_lookup(int64_t n, const int4 *eq, KeyFmt f, const int *pos, int *kid,
                                                    uint64_t *ukey) {
    const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= n) return;
    const uint64_t k = pack_key(eq[e], f);
    const int id = pos[k];
    kid[e] = id;
    ukey[id] = k;
}

__global__ __launch_bounds__(TPB) void k_flag_changes(int64_t n, const uint64_t *key, int *flag) {
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i < n) flag[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

// unique keys and the key id of every entry
__global__ __launch_bounds__(TPB) void k_key_ids(int64_t n, const uint64_t *key, const uint32_t *val, const int *flag,
                                                 const int *pos, int *kid, uint64_t *ukey) {
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= n) return;
    const int id = pos[i] + flag[i] - 1;
    kid[val[i]] = id;
    if (flag[i]) ukey[id] = key[i];
}

// (block, key) groups by counting: gk = block * nkeys + key indexes a dense
// table; entries are scattered to their group with an atomic cursor.  Within
// a group every entry fills a different target slot, so the order in which
// the entries land does not change any result.
__global__ __launch_bounds__(TPB) void k_gk_count(int64_t n, const int4 *raw, const int2 *cell_bs, const int *kid,
                                                  int nkeys, int *cnt) {
    const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= n) return;
    atomicAdd(&cnt[(int64_t)cell_bs[raw[e].x].x * nkeys + kid[e]], 1);
}

// occupancy only (every writer stores the same value): the split-product
// kernel needs which groups exist and their slot tables, not their entry lists
__global__ __launch_bounds__(TPB) void k_gk_mark(int64_t n, const int4 *raw, const int2 *cell_bs, const int *kid,
                                                 int nkeys, int *cnt) {
    const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= n) return;
    cnt[(int64_t)cell_bs[raw[e].x].x * nkeys + kid[e]] = 1;
}

__global__ __launch_bounds__(TPB) void k_gk_flags(int64_t T, const int *cnt, int *flag) {
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i < T) flag[i] = cnt[i] > 0 ? 1 : 0;
}

__global__ __launch_bounds__(TPB) void k_gk_groups(int64_t T, const int *cnt, const int *gid, const int *eoff, int nkeys,
                                                   int4 *groups, int *cursor) {
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= T) return;
    cursor[i] = 0;
    if (cnt[i] > 0) groups[gid[i]] = make_int4((int)(i % nkeys), eoff ? eoff[i] : 0, cnt[i], (int)(i / nkeys));
}

__global__ __launch_bounds__(TPB) void k_gk_scatter(int64_t n, const int4 *raw, const int2 *cell_bs, const int *kid,
                                                    int nkeys, const int *eoff, int *cursor, int2 *ent) {
    const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= n) return;
    const int4 r = raw[e];
    const int2 bs = cell_bs[r.x];
    const int64_t gk = (int64_t)bs.x * nkeys + kid[e];
    const int pos = eoff[gk] + atomicAdd(&cursor[gk], 1);
    ent[pos] = make_int2(r.y, bs.y);
}

// Dense slot table of every group: the source cell of each of its 64 target
// slots (filled beforehand with the zero row).  A group holds at most one
// entry per slot, so every slot is written at most once.
__global__ __launch_bounds__(TPB) void k_gk_slots(int64_t n, const int4 *raw, const int2 *cell_bs, const int *kid,
                                                  int nkeys, const int *gid, int *slots) {
    const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= n) return;
    const int4 r = raw[e];
    const int2 bs = cell_bs[r.x];
    slots[(int64_t)gid[(int64_t)bs.x * nkeys + kid[e]] * 64 + bs.y] = r.y;
}

__global__ __launch_bounds__(TPB) void k_fill_i32(int64_t n, int v, int *p) {
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i < n) p[i] = v;
}

// Launch order of the work items: by their position in their block's item
// list, then by block.  Blocks of one octant class hold nearly the same
// translation keys in the same order, so the work-groups that run together on
// one XCD (consecutive in this order) load the same operators, which their L2
// then serves once; the partial sums stay indexed by item.
__global__ __launch_bounds__(TPB) void k_item_order_keys(int nitems, const int4 *items, const int *blk_item0, int bshift,
                                                         uint64_t *key, uint32_t *val) {
    const int it = blockIdx.x * TPB + threadIdx.x;
    if (it >= nitems) return;
    const int b = items[it].x;
    key[it] = ((uint64_t)(it - blk_item0[b]) << bshift) | (uint64_t)b;
    val[it] = (uint32_t)it;
}

// group counts (from the next group's start; groups without entry lists keep
// first entry and count 0) and the per-block first group
__global__ __launch_bounds__(TPB) void k_group_counts(int ng, int64_t n, bool lists, int4 *groups, int *blk_first) {
    const int g = blockIdx.x * TPB + threadIdx.x;
    if (g >= ng) return;
    int4 gr = groups[g];
    const int next = (g + 1 < ng) ? groups[g + 1].y : (int)n;
    gr.z = lists ? next - gr.y : 0;
    groups[g] = gr;
    if (g == 0 || groups[g - 1].w != gr.w) blk_first[gr.w] = g;
}

__global__ __launch_bounds__(TPB) void k_item_flags(int ng, const int4 *groups, const int *blk_first, int *flag) {
    const int g = blockIdx.x * TPB + threadIdx.x;
    if (g >= ng) return;
    flag[g] = ((g - blk_first[groups[g].w]) % ITEM_GROUPS) == 0 ? 1 : 0;
}

// items: (block, first group, end group, 0); per block first item and item count
__global__ __launch_bounds__(TPB) void k_items(int ng, const int4 *groups, const int *flag, const int *pos,
                                               int4 *items, int *blk_item0, int *blk_nitem) {
    const int g = blockIdx.x * TPB + threadIdx.x;
    if (g >= ng || !flag[g]) return;
    const int b = groups[g].w;
    int end = g + 1;
    while (end < ng && end < g + ITEM_GROUPS && groups[end].w == b) ++end;
    const int it = pos[g];
    items[it] = make_int4(b, g, end, 0);
    if (g == 0 || groups[g - 1].w != b) blk_item0[b] = it;
    atomicAdd(&blk_nitem[b], 1);
}

// ---------------------------------------------------------------------------
// Mt in real row order, padded, k-permuted: Mr[cell][comp][NRP] (extra zero cell at the end)
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(TPB) void k_m2lb_mreal(int ncells, const float2 *Mexp, float *Mr) {
    constexpr int R = NR(P), RP = NRP(P), NCP = NC(P);
    const int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const int64_t total = (int64_t)(ncells + 1) * 3 * RP;
    if (idx >= total) return;
    const int r = kperm((int)(idx % RP));  // row held at this position
    const int64_t cc = idx / RP;           // cell*3 + comp
    float v = 0.f;
    if (r < R && cc < (int64_t)ncells * 3) {
        int n, m, im;
        decode_row(r, n, m, im);
        const float2 z = Mexp[cc * NCP + CIDX(n, m)];
        v = im ? z.y : z.x;
    }
    Mr[idx] = v;
}

// ---------------------------------------------------------------------------
// the batched translation
// ---------------------------------------------------------------------------
typedef float vf4 __attribute__((ext_vector_type(4)));

template <int P>
struct MbCfg {
    static constexpr int R = NR(P), RP = NRP(P), RT = NRT(P);
    static constexpr int Q = 2 * P, IW = 4 * P + 1;
    static constexpr int RTI = RT / 16;            // row tiles
    static constexpr int KC = RP / 16;             // chunks of four k steps
    static constexpr int RW = (RTI + 3) / 4;       // row tiles per wave (4 waves)
    static constexpr int BS = RP + 4;              // LDS column stride of the staged multipoles
    static constexpr size_t OP = (size_t)RT * RP;  // floats per operator
    static constexpr bool X6 = RP % 32 == 0;       // bf16 k blocks of 32 fit the padded inputs
    static constexpr size_t OPX = (size_t)RT * RP * 3 / 2;  // 32-bit words per operator, split form
};

// One operator per key, built once per tree.  T[r][c] (r output row
// (k, l, Re/Im), c input row (n, m, Re/Im)):
//   Lt_k^l = (-1)^{k+l} 2^{dl (k+1)} sum_{n,m} Mt_n^m I_{n+k}^{m-l}(-q 2^{min(dl,0)-2}).
// FORM 0 (float32 products): MFMA A-fragment order [key][row tile a][chunk]
// [lane][e] = T[16 a + lane % 16][16 chunk + 4 e + lane / 16], zero outside
// R x R, so a lane reads the operands of four k steps as one float4.
// FORM 1 (three-way bfloat16 split): T = T0 + T1 + T2 with T0 = bf16(T),
// T1 = bf16(T - T0), T2 = bf16(T - T0 - T1) (24 significant bits), stored
// [key][row tile a][k block kb][split s][lane][e] = Ts[16 a + lane % 16]
// [kperm(32 kb + 8 (lane / 16) + e)], e = 0..7: the input positions of a
// bf16 MFMA k block are eight consecutive positions of the k-permuted
// multipole rows.
__device__ inline uint32_t bf16_bits_rne(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;  // finite inputs only
}

template <int P, int FORM>
__global__ __launch_bounds__(256) void k_m2lb_optab(int nkeys, const uint64_t *__restrict__ ukey, KeyFmt f,
                                                    float *__restrict__ tab) {
    using C = MbCfg<P>;
    __shared__ float2 Is[(C::Q + 1) * C::IW];  // full orders M in [-Q, Q]
    __shared__ int rinfo[C::RP];
    const int key = blockIdx.x;
    if (key >= nkeys) return;
    const int tid = threadIdx.x;
    for (int r = tid; r < C::RP; r += 256) {
        int k = 0, l = 0, im = 0;
        if (r < C::R) decode_row(r, k, l, im);
        rinfo[r] = k | (l << 8) | (im << 16);
    }
    for (int i = tid; i < (C::Q + 1) * C::IW; i += 256) Is[i] = make_float2(0.f, 0.f);
    const uint64_t kv = ukey[key];
    const uint64_t mq = (1ull << f.bq) - 1;
    const int dl = (int)(kv >> (3 * f.bq)) - f.odl;
    __syncthreads();
    if (tid <= C::Q) {
        // irregular harmonics I_N^M((c_A - c_B)/s_B), (c_A - c_B)/s_B = -q 2^(min(dl,0) - 2)
        const int M = tid;
        const float sc = -ldexpf(1.0f, min(dl, 0) - 2);
        const float dx = (float)((int)((kv >> (2 * f.bq)) & mq) - f.oq) * sc;
        const float dy = (float)((int)((kv >> f.bq) & mq) - f.oq) * sc;
        const float dz = (float)((int)(kv & mq) - f.oq) * sc;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float ir2 = 1.0f / r2;
        float cr = rsqrtf(r2), ci = 0.f;
        for (int mm = 1; mm <= M; ++mm) {
            const float fc = -(float)(2 * mm - 1) * ir2;
            const float nr = fc * (dx * cr - dy * ci);
            const float ni = fc * (dx * ci + dy * cr);
            cr = nr;
            ci = ni;
        }
        auto put = [&](int N, float vr, float vi) {
            Is[N * C::IW + C::Q + M] = make_float2(vr, vi);
            if (M > 0) Is[N * C::IW + C::Q - M] = (M & 1) ? make_float2(-vr, vi) : make_float2(vr, -vi);
        };
        put(M, cr, ci);
        float pr = cr, pi = ci, qr = 0.f, qi = 0.f;
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
    __syncthreads();
    auto value = [&](int r, int c) -> float {
        float v = 0.f;
        if (r < C::R && c < C::R) {
            const int ri = rinfo[r], ci = rinfo[c];
            const int k = ri & 255, l = (ri >> 8) & 255, im = (ri >> 16) & 1;
            const int n = ci & 255, m = (ci >> 8) & 255, imc = (ci >> 16) & 1;
            const float2 x = Is[(n + k) * C::IW + C::Q + m - l];
            const float2 y = Is[(n + k) * C::IW + C::Q + m + l];
            const float sg = (l & 1) ? -1.f : 1.f;
            if (m == 0) v = im ? x.y : x.x;
            else if (!im) v = imc ? (-x.y - sg * y.y) : (x.x + sg * y.x);
            else v = imc ? (x.x - sg * y.x) : (x.y - sg * y.y);
            v *= (((k + l) & 1) ? -1.f : 1.f) * ldexpf(1.0f, dl * (k + 1));
        }
        return v;
    };
    if (FORM == 0) {
        float *T = tab + (size_t)key * C::OP;
        for (int idx = tid; idx < (int)C::OP; idx += 256) {
            const int e = idx & 3, lane = (idx >> 2) & 63;
            const int chunk = (idx >> 8) % C::KC, a = (idx >> 8) / C::KC;
            T[idx] = value(16 * a + (lane & 15), 16 * chunk + 4 * e + (lane >> 4));
        }
    } else {
        // one thread per (a, kb, lane, pair of e): two values packed per 32-bit word and split
        uint32_t *T = reinterpret_cast<uint32_t *>(tab) + (size_t)key * C::OPX;
        constexpr int KB = C::RP / 32;
        for (int idx = tid; idx < C::RTI * KB * 64 * 4; idx += 256) {
            const int ep = idx & 3, lane = (idx >> 2) & 63;
            const int kb = (idx >> 8) % KB, a = (idx >> 8) / KB;
            const int r = 16 * a + (lane & 15);
            const int p0 = 32 * kb + 8 * (lane >> 4) + 2 * ep;
            float v[2] = {value(r, kperm(p0)), value(r, kperm(p0 + 1))};
            uint32_t w[3][2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                float rem = v[h];
#pragma unroll
                for (int sp = 0; sp < 3; ++sp) {
                    w[sp][h] = bf16_bits_rne(rem);
                    rem -= __uint_as_float(w[sp][h] << 16);
                }
            }
#pragma unroll
            for (int sp = 0; sp < 3; ++sp)
                T[((((size_t)a * KB + kb) * 3 + sp) * 64 + lane) * 4 + ep] = w[sp][0] | (w[sp][1] << 16);
        }
    }
}

// A work-group of four waves takes one work item: up to ITEM_GROUPS keys of
// one block of 64 target cells.  Wave w owns row tiles w, w + 4, ... of the
// output for the three potentials; per key it loads its operator rows into
// registers, and the group stages the 64 target slots' source multipoles
// (absent slots read the zero cell) in LDS one potential at a time, double
// buffered, while the previous potential's products
// [16 rows x 4 inputs] x [4 inputs x 16 targets] run on v_mfma_f32_16x16x4f32.
template <int P>
__global__ __launch_bounds__(256) void k_m2lb(const int4 *__restrict__ items, const int *__restrict__ order,
                                              const int4 *__restrict__ groups,
                                              const int2 *__restrict__ ent, const float *__restrict__ Mr,
                                              const float *__restrict__ tab, int zero_cell, int nitems,
                                              float *__restrict__ partial) {
    using C = MbCfg<P>;
    const int li = xcd_logical(blockIdx.x, gridDim.x);
    if (li >= nitems) return;
    const int item = order[li];
    static_assert(64 * C::RP / 4 == 256 * C::KC, "one float4 per thread and chunk");
    extern __shared__ float smem[];
    float *Bs = smem;                                                // [2][64][BS]
    int *src_of = reinterpret_cast<int *>(smem + 2 * 64 * C::BS);    // [64]
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int i16 = lane & 15, kq = lane >> 4;
    const int4 it = items[item];
    const int g0 = __builtin_amdgcn_readfirstlane(it.y);
    const int g1 = __builtin_amdgcn_readfirstlane(it.z);
    vf4 acc[3][C::RW][4];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < C::RW; ++j)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[c][j][b] = vf4{0.f, 0.f, 0.f, 0.f};
    for (int g = g0; g < g1; ++g) {
        const int4 gr = groups[g];
        const int key = __builtin_amdgcn_readfirstlane(gr.x);
        const int e0 = __builtin_amdgcn_readfirstlane(gr.y);
        const int ne = __builtin_amdgcn_readfirstlane(gr.z);
        __syncthreads();  // the previous key's tiles and slots are no longer read
        if (tid < 64) src_of[tid] = zero_cell;
        __syncthreads();
        if (tid < ne) {
            const int2 en = ent[e0 + tid];
            src_of[en.y] = en.x;
        }
        // operator rows of this wave: A[j][chunk] holds k steps 4 chunk .. 4 chunk + 3
        vf4 A[C::RW][C::KC];
        const vf4 *T4 = reinterpret_cast<const vf4 *>(tab + (size_t)key * C::OP);
#pragma unroll
        for (int j = 0; j < C::RW; ++j) {
            const int a = wave + 4 * j;
#pragma unroll
            for (int ch = 0; ch < C::KC; ++ch)
                A[j][ch] = (a < C::RTI) ? T4[((size_t)a * C::KC + ch) * 64 + lane] : vf4{0.f, 0.f, 0.f, 0.f};
        }
        __syncthreads();
        // column and offset of this thread's float4 number i of a staged tile
        int scol[C::KC];
#pragma unroll
        for (int i = 0; i < C::KC; ++i) scol[i] = src_of[(tid + 256 * i) / (C::RP / 4)];
        auto src4 = [&](int i, int c) {
            return reinterpret_cast<const vf4 *>(Mr + ((size_t)scol[i] * 3 + c) * C::RP +
                                                 4 * ((tid + 256 * i) % (C::RP / 4)));
        };
        auto dst4 = [&](float *B, int i) {
            const int q = tid + 256 * i;
            return reinterpret_cast<vf4 *>(&B[(q / (C::RP / 4)) * C::BS + 4 * (q % (C::RP / 4))]);
        };
        {
            vf4 pre[C::KC];
#pragma unroll
            for (int i = 0; i < C::KC; ++i) pre[i] = *src4(i, 0);
#pragma unroll
            for (int i = 0; i < C::KC; ++i) *dst4(Bs, i) = pre[i];
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float *Bc = Bs + (c & 1) * 64 * C::BS;
            float *Bn = Bs + ((c + 1) & 1) * 64 * C::BS;
            // the next potential's tile streams in one float4 per chunk, stored a chunk later
            vf4 inflight = vf4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ch = 0; ch < C::KC; ++ch) {
                if (c < 2) {
                    if (ch > 0) *dst4(Bn, ch - 1) = inflight;
                    inflight = *src4(ch, c + 1);
                }
                vf4 Bv[4];
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    Bv[b] = *reinterpret_cast<const vf4 *>(&Bc[(16 * b + i16) * C::BS + 16 * ch + 4 * kq]);
#pragma unroll
                for (int j = 0; j < C::RW; ++j) {
                    if (wave + 4 * j >= C::RTI) continue;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
#pragma unroll
                        for (int b = 0; b < 4; ++b)
                            acc[c][j][b] =
                                __builtin_amdgcn_mfma_f32_16x16x4f32(A[j][ch][e], Bv[b][e], acc[c][j][b], 0, 0, 0);
                }
            }
            if (c < 2) {
                *dst4(Bn, C::KC - 1) = inflight;
                __syncthreads();
            }
        }
    }
    // D fragment: lane holds rows 16 a + 4 kq + v of target column 16 b + i16
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float *out = partial + ((size_t)item * 3 + c) * C::R * 64;
#pragma unroll
        for (int j = 0; j < C::RW; ++j) {
            const int a = wave + 4 * j;
            if (a >= C::RTI) continue;
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * a + 4 * kq + v;
                    if (row < C::R) out[(size_t)row * 64 + 16 * b + i16] = acc[c][j][b][v];
                }
        }
    }
}

// Split-product form of the batched translation (float32-accurate products
// on the bfloat16 matrix cores).  The operator comes from the table in three
// bf16 parts (T = T0 + T1 + T2, 24 significant bits); each staged multipole
// value is split the same way (M = M0 + M1 + M2) as it is written to LDS.
// T M is then the sum of the six products Ti Mj with i + j <= 2, each on
// v_mfma_f32_16x16x32_bf16 (exact bf16 products, float32 accumulation); the
// three dropped products and the splitting residuals are each of order
// 2^-26 |T| |M|.  With NS = 2 parts per operand (T0 + T1, M0 + M1: 16
// significant bits) only the three products T1 M0, T0 M1, T0 M0 are taken, at
// half the matrix-core work; each dropped term is then of order 2^-16 |T| |M|
// (m2l_form 3, a reduced-precision form for error bounds near 1e-4).  A
// work-group of RTI waves (eight at p = 10) takes one work item; a wave owns
// two row tiles (32 output rows) of 32 of the 64 targets, for the three
// potentials.
template <int P>
struct MbxCfg {
    using C = MbCfg<P>;
    static constexpr int KB = C::RP / 32;     // k blocks of 32 inputs
    static constexpr int WAVES = C::RTI;      // (RTI / 2 row-tile pairs) x (2 column halves)
    static constexpr int BSX = C::RP + 8;     // LDS column stride (bf16) of a split plane
    static constexpr int PLANE = 64 * BSX;    // bf16 per plane
    static constexpr int F4 = 64 * C::RP / 4 / (64 * WAVES);  // staged float4 per thread and potential
    static_assert(!C::X6 || ((64 * C::RP / 4) % (64 * WAVES) == 0 && C::RTI % 2 == 0), "tile split");
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// x = h + m + l with h, m, l in bf16 (v_cvt_pk_bf16_f32, round to nearest
// even; each residual is exact in float32); two values per word
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ inline void split4(vf4 x, u32x2 &h, u32x2 &m, u32x2 &l) {
    float r[4] = {x[0], x[1], x[2], x[3]};
    uint32_t w[3][2];
#pragma unroll
    for (int sp = 0; sp < 3; ++sp)
#pragma unroll
        for (int pr = 0; pr < 2; ++pr) {
            const bf16x2 v = {(__bf16)r[2 * pr], (__bf16)r[2 * pr + 1]};
            const uint32_t u = __builtin_bit_cast(uint32_t, v);
            w[sp][pr] = u;
            if (sp < 2) {
                r[2 * pr] -= __uint_as_float(u << 16);
                r[2 * pr + 1] -= __uint_as_float(u & 0xffff0000u);
            }
        }
    h = u32x2{w[0][0], w[0][1]};
    m = u32x2{w[1][0], w[1][1]};
    l = u32x2{w[2][0], w[2][1]};
}

__device__ __forceinline__ vf4 mfma_bf16(u32x4 a, u32x4 b, vf4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                  0, 0, 0);
}

template <int P, int NS>
__global__ __launch_bounds__(MbxCfg<P>::WAVES * 64) void k_m2lb_x6(const int4 *__restrict__ items,
                                                                  const int *__restrict__ order,
                                                                  const int4 *__restrict__ groups,
                                                                  const int *__restrict__ slots,
                                                                  const float *__restrict__ Mr,
                                                                  const uint32_t *__restrict__ tab, int nitems,
                                                                  float *__restrict__ partial) {
    using C = MbCfg<P>;
    using X = MbxCfg<P>;
    constexpr int NT = X::WAVES * 64;
    const int li = xcd_logical(blockIdx.x, gridDim.x);
    if (li >= nitems) return;
    const int item = order[li];
    extern __shared__ float smem[];
    uint16_t *Bs = reinterpret_cast<uint16_t *>(smem);                     // [2][NS][64][BSX]
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int i16 = lane & 15, kq = lane >> 4;
    constexpr int RH = C::RTI / 2;              // row-tile pairs
    const int ra0 = 2 * (wave % RH), cb0 = 2 * (wave / RH);  // this wave: row tiles ra0, ra0+1; columns cb0, cb0+1
    const int4 it = items[item];
    const int g0 = __builtin_amdgcn_readfirstlane(it.y);
    const int g1 = __builtin_amdgcn_readfirstlane(it.z);
    vf4 acc[3][2][2];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[c][j][b] = vf4{0.f, 0.f, 0.f, 0.f};
    // this wave's two row tiles of the operator: A[j][kb][split].  The first
    // group's operator is loaded here; each later group's is loaded k block
    // by k block while the group before it does its last potential, as soon as
    // that k block's products have been issued.
    u32x4 A[2][X::KB][NS];
    auto load_a = [&](int key, int kb) {
        const u32x4 *T4 = reinterpret_cast<const u32x4 *>(tab + (size_t)key * C::OPX);
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int sp = 0; sp < NS; ++sp)
                A[j][kb][sp] = T4[(((size_t)(ra0 + j) * X::KB + kb) * 3 + sp) * 64 + lane];
    };
    if (g0 < g1) {
        const int key0 = __builtin_amdgcn_readfirstlane(groups[g0].x);
#pragma unroll
        for (int kb = 0; kb < X::KB; ++kb) load_a(key0, kb);
    }
    // float4 number q = tid + NT i of a staged tile: column q / (RP/4), inputs 4 (q % (RP/4)) ..;
    // the source cell of every column of a group comes from its dense slot table (the
    // current group's until its last potential, then the next group's)
    int scol[X::F4];
    auto load_cols = [&](int g) {
#pragma unroll
        for (int i = 0; i < X::F4; ++i) scol[i] = slots[(size_t)g * 64 + (tid + NT * i) / (C::RP / 4)];
    };
    auto src4 = [&](int i, int c) {
        return reinterpret_cast<const vf4 *>(Mr + ((size_t)scol[i] * 3 + c) * C::RP +
                                             4 * ((tid + NT * i) % (C::RP / 4)));
    };
    auto put = [&](int buf, int i, vf4 x) {
        const int q = tid + NT * i;
        const int off = (q / (C::RP / 4)) * X::BSX + 4 * (q % (C::RP / 4));
        u32x2 h, m, l;
        split4(x, h, m, l);
        uint16_t *base = Bs + (size_t)buf * NS * X::PLANE + off;
        *reinterpret_cast<u32x2 *>(base) = h;
        *reinterpret_cast<u32x2 *>(base + X::PLANE) = m;
        if (NS == 3) *reinterpret_cast<u32x2 *>(base + 2 * X::PLANE) = l;
    };
    // the first potential's multipoles of a group: loaded for the first group
    // here, for each later one while the group before it does its last potential
    vf4 pre[X::F4];
    if (g0 < g1) {
        load_cols(g0);
#pragma unroll
        for (int i = 0; i < X::F4; ++i) pre[i] = *src4(i, 0);
    }
    for (int g = g0; g < g1; ++g) {
        const bool more = g + 1 < g1;
        const int nkey = more ? __builtin_amdgcn_readfirstlane(groups[g + 1].x) : 0;
        __syncthreads();  // the previous group's tiles are no longer read
#pragma unroll
        for (int i = 0; i < X::F4; ++i) put(0, i, pre[i]);
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const uint16_t *Bc = Bs + (size_t)(c & 1) * NS * X::PLANE;
            vf4 nxt[X::F4];
            if (c < 2) {
#pragma unroll
                for (int i = 0; i < X::F4; ++i) nxt[i] = *src4(i, c + 1);
            } else if (more) {
                load_cols(g + 1);
#pragma unroll
                for (int i = 0; i < X::F4; ++i) pre[i] = *src4(i, 0);
            }
#pragma unroll
            for (int kb = 0; kb < X::KB; ++kb) {
                u32x4 Bv[2][NS];
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int sp = 0; sp < NS; ++sp)
                        Bv[b][sp] = *reinterpret_cast<const u32x4 *>(
                            Bc + sp * X::PLANE + (16 * (cb0 + b) + i16) * X::BSX + 32 * kb + 8 * kq);
                // smallest products first: (2,0) (1,1) (0,2) (1,0) (0,1) (0,0); with two
                // parts per operand only the last three
                constexpr int TA[6] = {2, 1, 0, 1, 0, 0}, TB[6] = {0, 1, 2, 0, 1, 0};
                constexpr int T0 = NS == 3 ? 0 : 3;
#pragma unroll
                for (int t = T0; t < 6; ++t)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
#pragma unroll
                        for (int b = 0; b < 2; ++b)
                            acc[c][j][b] = mfma_bf16(A[j][kb][TA[t]], Bv[b][TB[t]], acc[c][j][b]);
                if (c == 2 && more) load_a(nkey, kb);  // this k block's last use in this group
            }
            if (c < 2) {
#pragma unroll
                for (int i = 0; i < X::F4; ++i) put((c + 1) & 1, i, nxt[i]);
                __syncthreads();
            }
        }
    }
    // D fragment: lane holds rows 16 a + 4 kq + v of target column 16 b + i16
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float *out = partial + ((size_t)item * 3 + c) * C::R * 64;
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * (ra0 + j) + 4 * kq + v;
                    if (row < C::R) out[(size_t)row * 64 + 16 * (cb0 + b) + i16] = acc[c][j][b][v];
                }
    }
}

template <int P, int NS>
static size_t m2lb_x6_lds_bytes() {
    using X = MbxCfg<P>;
    return sizeof(uint16_t) * 2 * NS * X::PLANE;
}

template <int P>
static size_t m2lb_lds_bytes() {
    using C = MbCfg<P>;
    return sizeof(float) * 2 * 64 * C::BS + sizeof(int) * 64;
}

// per block: sum the items' partials in item order and add to Lt.  One thread
// per (potential, row, target slot) of a block; blockIdx.y strides over blocks.
// Per target block, potential and chunk of RC rows: the items' partial sums of
// each (row, slot), in item order, staged in LDS (phase 1: a wave per row,
// lanes over the 64 slots, so the partials are read in whole rows), then
// added to each cell's local expansion with lanes over its rows (phase 2), so
// the read-modify-write of Lexp touches each cell's coefficients together.
static constexpr int RC = 64;  // rows per work-group

template <int P, typename A>
__global__ __launch_bounds__(TPB) void k_m2lb_reduce(const int *blk_item0, const int *blk_nitem, const int *blk_cells,
                                                     const float *partial, float2 *Lexp) {
    // A: accumulator type (double in the mixed precision form)
    constexpr int R = NR(P), NCP = NC(P);
    __shared__ A tile[RC][65];
    const int b = blockIdx.x, comp = blockIdx.y, r0 = blockIdx.z * RC;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ni = blk_nitem[b];
    if (ni == 0) return;
    const size_t stride = (size_t)3 * R * 64;
    for (int rr = wave; rr < RC; rr += TPB / 64) {
        const int r = r0 + rr;
        if (r >= R) break;
        const float *p = partial + ((size_t)blk_item0[b] * 3 * R + (size_t)comp * R + r) * 64 + lane;
        // up to 16 items' loads in flight, added in item order
        A acc = A(0);
        for (int i0 = 0; i0 < ni; i0 += 16) {
            float v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = i0 + u < ni ? p[(size_t)(i0 + u) * stride] : 0.f;
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (i0 + u < ni) acc += (A)v[u];
        }
        tile[rr][lane] = acc;
    }
    __syncthreads();
    const int r = r0 + lane;
    if (r >= R) return;
    int k, l, im;
    decode_row(r, k, l, im);
    for (int slot = wave; slot < 64; slot += TPB / 64) {
        const int cell = blk_cells[(size_t)b * 64 + slot];
        if (cell < 0) continue;
        float *dst = reinterpret_cast<float *>(&Lexp[((size_t)cell * 3 + comp) * NCP + CIDX(k, l)]) + im;
        *dst = (float)((A)*dst + tile[lane][slot]);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// Product form of the batched M2L: split bf16 products when asked for
// (m2l_form 2: six products, 3: three) and the padded inputs make whole k
// blocks of 32.
static bool m2lb_split_form(const Ctx &c, bool fits) { return fits && (c.prm.m2l_form == 2 || c.prm.m2l_form == 3); }

static int bits_for_range(int64_t maxabs) {
    int b = 1;
    while ((1LL << b) < 2 * maxabs + 1) ++b;
    return b;
}

template <int P>
static void m2lb_plan_p(Ctx &c) {
    hipStream_t s = c.stream;
    const int64_t n = c.n_m2l;
    c.m2lb_ok = false;
    if (n == 0) return;
    // ---- offsets and ranges ----
    c.mb_eq.ensure(sizeof(int4) * n);
    c.pairs64.ensure(64);
    VFMM_HIP(hipMemsetAsync(c.pairs64.ptr, 0, 8, s));
    k_m2lb_offsets<<<std::min<unsigned>(cdiv(n, TPB), 1024), TPB, 0, s>>>(n, c.m2l_raw.as<int4>(), c.c_geo.as<float4>(),
                                                 c.c_level.as<int>(), c.img_B,
                                                 c.prm.periodic ? (float)c.prm.box_len : 0.f, c.mb_eq.as<int4>(),
                                                 c.pairs64.as<int>());
    VFMM_LAUNCH_CHECK();
    int rng[2];
    read_ints(c, {c.pairs64.as<int>(), c.pairs64.as<int>() + 1}, rng);
    KeyFmt f{};
    f.bq = bits_for_range(rng[0]);
    f.bdl = bits_for_range(rng[1]);
    f.oq = (1 << (f.bq - 1));
    f.odl = (1 << (f.bdl - 1));
    const int kb = 3 * f.bq + f.bdl;
    if (kb > 62) return;  // offsets too spread for packed keys: generic kernel
    // ---- unique keys, numbered in increasing key order ----
    int nkeys = 0;
    int h2[2];
    if (kb <= TABLE_KEY_BITS) {
        const int64_t tsz = (int64_t)1 << kb;
        c.mb_flag.ensure(sizeof(int) * (std::max<int64_t>(n, tsz) + 1));
        c.mb_pos.ensure(sizeof(int) * (std::max<int64_t>(n, tsz) + 1));
        int *tab = c.mb_flag.as<int>(), *tpos = c.mb_pos.as<int>();
        VFMM_HIP(hipMemsetAsync(tab, 0, sizeof(int) * tsz, s));
        k_key_mark<<<cdiv(n, TPB), TPB, 0, s>>>(n, c.mb_eq.as<int4>(), f, tab);
        VFMM_LAUNCH_CHECK();
        scan_excl_i32(c, tab, tpos, tsz);
        read_ints(c, {tpos + tsz - 1, tab + tsz - 1}, h2);
        nkeys = h2[0] + h2[1];
        c.mb_kid.ensure(sizeof(int) * n);
        c.mb_ukey.ensure(sizeof(uint64_t) * nkeys);
        k_key_lookup<<<cdiv(n, TPB), TPB, 0, s>>>(n, c.mb_eq.as<int4>(), f, tpos, c.mb_kid.as<int>(),
                                                   c.mb_ukey.as<uint64_t>());
        VFMM_LAUNCH_CHECK();
    } else {
        c.lkey.ensure(sizeof(uint64_t) * n);
        c.lval.ensure(sizeof(uint32_t) * n);
        k_m2lb_pack<<<cdiv(n, TPB), TPB, 0, s>>>(n, c.mb_eq.as<int4>(), f, c.lkey.as<uint64_t>(),
                                                  c.lval.as<uint32_t>());
        VFMM_LAUNCH_CHECK();
        sort_pairs_u64(c, c.lkey, c.lval, c.lkey2, c.lval2, n, kb);
        c.mb_flag.ensure(sizeof(int) * (n + 1));
        c.mb_pos.ensure(sizeof(int) * (n + 1));
        int *flag = c.mb_flag.as<int>(), *pos = c.mb_pos.as<int>();
        k_flag_changes<<<cdiv(n, TPB), TPB, 0, s>>>(n, c.lkey.as<uint64_t>(), flag);
        VFMM_LAUNCH_CHECK();
        scan_excl_i32(c, flag, pos, n);
        read_ints(c, {pos + n - 1, flag + n - 1}, h2);
        nkeys = h2[0] + h2[1];
        c.mb_kid.ensure(sizeof(int) * n);
        c.mb_ukey.ensure(sizeof(uint64_t) * nkeys);
        k_key_ids<<<cdiv(n, TPB), TPB, 0, s>>>(n, c.lkey.as<uint64_t>(), c.lval.as<uint32_t>(), flag, pos,
                                                c.mb_kid.as<int>(), c.mb_ukey.as<uint64_t>());
        VFMM_LAUNCH_CHECK();
    }
    c.lkey.ensure(sizeof(uint64_t) * n);
    c.lval.ensure(sizeof(uint32_t) * n);
    int *flag = c.mb_flag.as<int>(), *pos = c.mb_pos.as<int>();
    // ---- blocks of 64 target cells: one level, one octant class, Morton order ----
    ClassModes cm{};
    for (int l = 0; l <= c.depth && l < 23; ++l) {
        const int cnt = c.lvl_off[l + 1] - c.lvl_off[l];
        cm.m[l] = (l >= 2 && cnt >= 64 * 64) ? 2 : (l >= 1 && cnt >= 64 * 8) ? 1 : 0;
    }
    const int nc = c.ncells;
    if (c.depth >= 23) return;  // buckets hold levels 0..22: per-pair M2L
    c.mb_cls.ensure(sizeof(int) * (size_t)nc);
    k_cell_class<<<cdiv(nc, TPB), TPB, 0, s>>>(nc, c.c_level.as<int>(), c.c_start.as<int>(), c.keyA.as<uint64_t>(),
                                               c.key_levels, cm, c.mb_cls.as<int>());
    VFMM_LAUNCH_CHECK();
    c.lkey.ensure(sizeof(uint64_t) * (size_t)nc);
    c.lval.ensure(sizeof(uint32_t) * (size_t)nc);
    k_cell_bucket<<<cdiv(nc, TPB), TPB, 0, s>>>(nc, c.c_level.as<int>(), c.mb_cls.as<int>(), c.lkey.as<uint64_t>(),
                                                c.lval.as<uint32_t>());
    VFMM_LAUNCH_CHECK();
    sort_pairs_u64(c, c.lkey, c.lval, c.lkey2, c.lval2, nc, 11);  // buckets < 2^11
    c.mb_bkt.ensure(sizeof(int) * (3 * NBUCKET + 1));
    int *bstart = c.mb_bkt.as<int>(), *bend = bstart + NBUCKET, *boff = bend + NBUCKET, *dnblk = boff + NBUCKET;
    VFMM_HIP(hipMemsetAsync(bstart, 0, sizeof(int) * 2 * NBUCKET, s));
    k_bucket_ranges<<<cdiv(nc, TPB), TPB, 0, s>>>(nc, c.lkey.as<uint64_t>(), bstart, bend);
    VFMM_LAUNCH_CHECK();
    k_bucket_blocks<<<1, 1024, 0, s>>>(bstart, bend, boff, dnblk);
    VFMM_LAUNCH_CHECK();
    int nblk = 0;
    read_ints(c, {dnblk}, &nblk);
    c.mb_nblk = nblk;
    c.mb_bcells.ensure(sizeof(int) * 64 * (size_t)nblk);
    c.mb_cellbs.ensure(sizeof(int2) * (size_t)nc);
    VFMM_HIP(hipMemsetAsync(c.mb_bcells.ptr, 0xff, sizeof(int) * 64 * (size_t)nblk, s));  // -1: empty slot
    k_bucket_assign<<<cdiv(nc, TPB), TPB, 0, s>>>(nc, c.lkey.as<uint64_t>(), c.lval.as<uint32_t>(), bstart, boff,
                                                  c.mb_cellbs.as<int2>(), c.mb_bcells.as<int>());
    VFMM_LAUNCH_CHECK();
    // ---- groups (block, key) in (block, key) order ----
    const int64_t T = (int64_t)nblk * nkeys;
    if (T > ((int64_t)1 << 28)) return;  // table too large: per-pair M2L
    c.mb_gcnt.ensure(sizeof(int) * (size_t)(T + 1));
    c.mb_gid.ensure(sizeof(int) * (size_t)(T + 1));
    c.mb_goff.ensure(sizeof(int) * (size_t)(T + 1));
    c.mb_gcur.ensure(sizeof(int) * (size_t)(T + 1));
    int *gcnt = c.mb_gcnt.as<int>(), *gid = c.mb_gid.as<int>(), *goff = c.mb_goff.as<int>(),
        *gcur = c.mb_gcur.as<int>();
    using C = MbCfg<P>;
    const bool x6 = m2lb_split_form(c, C::X6);
    VFMM_HIP(hipMemsetAsync(gcnt, 0, sizeof(int) * (size_t)T, s));
    if (x6) {
        k_gk_mark<<<cdiv(n, TPB), TPB, 0, s>>>(n, c.m2l_raw.as<int4>(), c.mb_cellbs.as<int2>(), c.mb_kid.as<int>(),
                                                nkeys, gcnt);
        VFMM_LAUNCH_CHECK();
    } else {
        k_gk_count<<<cdiv(n, TPB), TPB, 0, s>>>(n, c.m2l_raw.as<int4>(), c.mb_cellbs.as<int2>(), c.mb_kid.as<int>(),
                                                 nkeys, gcnt);
        VFMM_LAUNCH_CHECK();
        scan_excl_i32(c, gcnt, goff, T);
    }
    k_gk_flags<<<cdiv(T, TPB), TPB, 0, s>>>(T, gcnt, gcur);  // flags, then reused as cursors
    VFMM_LAUNCH_CHECK();
    scan_excl_i32(c, gcur, gid, T);
    read_ints(c, {gid + T - 1, gcur + T - 1}, h2);
    const int ng = h2[0] + h2[1];
    // A group costs a full 64-target operator product whether its targets are
    // all present or not; measured on gfx950 a group costs about as much as
    // 6-7 translations of the per-pair kernel, so sparse groups (irregular
    // trees: many offsets, few targets sharing each) go to the per-pair M2L.
    if (c.prm.m2l_mode == 0 && n < (int64_t)MIN_GROUP_FILL * ng) return;
    c.mb_groups.ensure(sizeof(int4) * ng);
    k_gk_groups<<<cdiv(T, TPB), TPB, 0, s>>>(T, gcnt, gid, x6 ? nullptr : goff, nkeys, c.mb_groups.as<int4>(), gcur);
    VFMM_LAUNCH_CHECK();
    if (x6) {  // the split-product kernel reads each group's sources from its slot table
        c.mb_slots.ensure(sizeof(int) * 64 * (size_t)ng);
        k_fill_i32<<<cdiv(64 * (int64_t)ng, TPB), TPB, 0, s>>>(64 * (int64_t)ng, nc, c.mb_slots.as<int>());
        VFMM_LAUNCH_CHECK();
        k_gk_slots<<<cdiv(n, TPB), TPB, 0, s>>>(n, c.m2l_raw.as<int4>(), c.mb_cellbs.as<int2>(), c.mb_kid.as<int>(),
                                                 nkeys, gid, c.mb_slots.as<int>());
        VFMM_LAUNCH_CHECK();
    } else {  // the float32-product kernel reads each group's entry list
        c.mb_ent.ensure(sizeof(int2) * n);
        k_gk_scatter<<<cdiv(n, TPB), TPB, 0, s>>>(n, c.m2l_raw.as<int4>(), c.mb_cellbs.as<int2>(),
                                                   c.mb_kid.as<int>(), nkeys, goff, gcur, c.mb_ent.as<int2>());
        VFMM_LAUNCH_CHECK();
    }
    c.mb_blk.ensure(sizeof(int) * 3 * (size_t)nblk);
    int *blk_first = c.mb_blk.as<int>(), *blk_item0 = blk_first + nblk, *blk_nitem = blk_item0 + nblk;
    VFMM_HIP(hipMemsetAsync(c.mb_blk.ptr, 0, sizeof(int) * 3 * (size_t)nblk, s));
    k_group_counts<<<cdiv(ng, TPB), TPB, 0, s>>>(ng, n, !x6, c.mb_groups.as<int4>(), blk_first);
    VFMM_LAUNCH_CHECK();
    k_item_flags<<<cdiv(ng, TPB), TPB, 0, s>>>(ng, c.mb_groups.as<int4>(), blk_first, flag);
    VFMM_LAUNCH_CHECK();
    scan_excl_i32(c, flag, pos, ng);
    read_ints(c, {pos + ng - 1, flag + ng - 1}, h2);
    const int nitems = h2[0] + h2[1];
    c.mb_items.ensure(sizeof(int4) * nitems);
    k_items<<<cdiv(ng, TPB), TPB, 0, s>>>(ng, c.mb_groups.as<int4>(), flag, pos, c.mb_items.as<int4>(), blk_item0,
                                           blk_nitem);
    VFMM_LAUNCH_CHECK();
    {
        const int bshift = bits_for_range(nblk);  // block ids below 2^bshift
        const int kbits = bits_for_range(nitems);  // an item's position in its block < nitems
        c.lkey.ensure(sizeof(uint64_t) * (size_t)nitems);
        c.lval.ensure(sizeof(uint32_t) * (size_t)nitems);
        k_item_order_keys<<<cdiv(nitems, TPB), TPB, 0, s>>>(nitems, c.mb_items.as<int4>(), blk_item0, bshift,
                                                            c.lkey.as<uint64_t>(), c.lval.as<uint32_t>());
        VFMM_LAUNCH_CHECK();
        sort_pairs_u64(c, c.lkey, c.lval, c.lkey2, c.lval2, nitems, bshift + kbits);
        c.mb_order.ensure(sizeof(int) * (size_t)nitems);
        VFMM_HIP(hipMemcpyAsync(c.mb_order.ptr, c.lval.ptr, sizeof(int) * (size_t)nitems, hipMemcpyDeviceToDevice, s));
    }
    // ---- one operator per key ----
    const size_t tab_bytes = (x6 ? sizeof(uint32_t) * C::OPX : sizeof(float) * C::OP) * (size_t)nkeys;
    if (tab_bytes > MAX_TABLE_BYTES) return;  // too many distinct offsets: generic kernel
    c.mb_tab.ensure(tab_bytes);
    if (x6)
        k_m2lb_optab<P, 1><<<nkeys, 256, 0, s>>>(nkeys, c.mb_ukey.as<uint64_t>(), f, c.mb_tab.as<float>());
    else
        k_m2lb_optab<P, 0><<<nkeys, 256, 0, s>>>(nkeys, c.mb_ukey.as<uint64_t>(), f, c.mb_tab.as<float>());
    VFMM_LAUNCH_CHECK();
    c.mb_x6 = x6;
    c.mb_nsplit = x6 && c.prm.m2l_form == 3 ? 2 : 3;
    c.mb_nkeys = nkeys;
    c.mb_fmt[0] = f.bq;
    c.mb_fmt[1] = f.bdl;
    c.mb_fmt[2] = f.oq;
    c.mb_fmt[3] = f.odl;
    c.mb_ngroups = ng;
    c.mb_nitems = nitems;
    c.m2lb_ok = true;
}

void m2lb_plan(Ctx &c) {
    switch (c.prm.p) {
        case 4: m2lb_plan_p<4>(c); break;
        case 6: m2lb_plan_p<6>(c); break;
        case 8: m2lb_plan_p<8>(c); break;
        case 10: m2lb_plan_p<10>(c); break;
        case 12: m2lb_plan_p<12>(c); break;
        default: throw Error{VFMM_EINVAL, "unsupported expansion degree p"};
    }
}

template <int P>
static void m2lb_prealloc_p(Ctx &c) {
    constexpr int R = NR(P), RP = NRP(P);
    c.mb_mr.ensure(sizeof(float) * (size_t)(c.ncells + 1) * 3 * RP);
    c.mb_partial.ensure(sizeof(float) * (size_t)std::max(c.mb_nitems, 1) * 3 * R * 64);
}

void m2lb_prealloc(Ctx &c) {
    if (!c.m2lb_ok) return;
    switch (c.prm.p) {
        case 4: m2lb_prealloc_p<4>(c); break;
        case 6: m2lb_prealloc_p<6>(c); break;
        case 8: m2lb_prealloc_p<8>(c); break;
        case 10: m2lb_prealloc_p<10>(c); break;
        case 12: m2lb_prealloc_p<12>(c); break;
        default: throw Error{VFMM_EINVAL, "unsupported expansion degree p"};
    }
}

template <int P>
static void m2lb_run_p(Ctx &c) {
    hipStream_t s = c.stream;
    constexpr int R = NR(P), RP = NRP(P);
    const int64_t mr_total = (int64_t)(c.ncells + 1) * 3 * RP;
    c.mb_mr.ensure(sizeof(float) * mr_total);
    k_m2lb_mreal<P><<<cdiv(mr_total, TPB), TPB, 0, s>>>(c.ncells, c.Mexp.as<float2>(), c.mb_mr.as<float>());
    VFMM_LAUNCH_CHECK();
    c.mb_partial.ensure(sizeof(float) * (size_t)c.mb_nitems * 3 * R * 64);
    if (c.mb_x6) {
        using X = MbxCfg<P>;
        auto launch = [&](auto ns) {
            constexpr int NS = decltype(ns)::value;
            const size_t lds = m2lb_x6_lds_bytes<P, NS>();
            int &set = NS == 3 ? c.m2lbx_lds_set : c.m2lbx3_lds_set;
            if (set < (int)lds) {  // once per context (a context lives on one device)
                VFMM_HIP(hipFuncSetAttribute((const void *)k_m2lb_x6<P, NS>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
                set = (int)lds;
            }
            k_m2lb_x6<P, NS><<<xcd_grid(c.mb_nitems), X::WAVES * 64, lds, s>>>(
                c.mb_items.as<int4>(), c.mb_order.as<int>(), c.mb_groups.as<int4>(), c.mb_slots.as<int>(),
                c.mb_mr.as<float>(),
                c.mb_tab.as<uint32_t>(), c.mb_nitems, c.mb_partial.as<float>());
        };
        if (c.mb_nsplit == 2)
            launch(std::integral_constant<int, 2>{});
        else
            launch(std::integral_constant<int, 3>{});
    } else {
        const size_t lds = m2lb_lds_bytes<P>();
        if (c.m2lb_lds_set < (int)lds) {  // once per context (a context lives on one device)
            VFMM_HIP(hipFuncSetAttribute((const void *)k_m2lb<P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)lds));
            c.m2lb_lds_set = (int)lds;
        }
        k_m2lb<P><<<xcd_grid(c.mb_nitems), 256, lds, s>>>(c.mb_items.as<int4>(), c.mb_order.as<int>(),
                                                           c.mb_groups.as<int4>(),
                                                           c.mb_ent.as<int2>(), c.mb_mr.as<float>(),
                                                           c.mb_tab.as<float>(), c.ncells, c.mb_nitems,
                                                           c.mb_partial.as<float>());
    }
    VFMM_LAUNCH_CHECK();
    const int nblk = c.mb_nblk;
    int *blk_item0 = c.mb_blk.as<int>() + nblk, *blk_nitem = blk_item0 + nblk;
    const dim3 rgrid(nblk, 3, cdiv(R, RC));
    if (nblk == 0) return;
    if (c.prm.precision == VFMM_PRECISION_MIXED)
        k_m2lb_reduce<P, double><<<rgrid, TPB, 0, s>>>(blk_item0, blk_nitem, c.mb_bcells.as<int>(),
                                                        c.mb_partial.as<float>(), c.Lexp.as<float2>());
    else
        k_m2lb_reduce<P, float><<<rgrid, TPB, 0, s>>>(blk_item0, blk_nitem, c.mb_bcells.as<int>(),
                                                       c.mb_partial.as<float>(), c.Lexp.as<float2>());
    VFMM_LAUNCH_CHECK();
}

void m2lb_run(Ctx &c) {
    switch (c.prm.p) {
        case 4: m2lb_run_p<4>(c); break;
        case 6: m2lb_run_p<6>(c); break;
        case 8: m2lb_run_p<8>(c); break;
        case 10: m2lb_run_p<10>(c); break;
        case 12: m2lb_run_p<12>(c); break;
        default: throw Error{VFMM_EINVAL, "unsupported expansion degree p"};
    }
}

}  // namespace vfmm
