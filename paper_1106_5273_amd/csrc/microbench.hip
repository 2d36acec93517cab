// VALU rate microbenchmarks for the roofline of the P2P and M2L kernels:
// independent chains of float32 FMA (v_fmac_f32 with vector-register
// operands only, or with one scalar-register operand; the instruction is
// written out so that the compiler cannot pick another form), v_exp_f32 and
// v_rsq_f32, FMA with a DPP row-broadcast operand and the VOP3 FMA, timed
// with HIP events.  Built into its own small library
// (libvfmm_mb.so); not part of the vfmm C ABI.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int CH = 8;  // independent chains per lane

template <int KIND>
__global__ __launch_bounds__(256) void k_rate(float *out, int iters, float a, float b) {
    float v[CH];
    for (int i = 0; i < CH; ++i) v[i] = (float)(threadIdx.x + i) * 1e-3f;
    const float sa = a;                                // kernel argument: a scalar register
    const float va = a + (float)threadIdx.x * 1e-9f;  // per-lane values
    const float vb = b + (float)threadIdx.x * 1e-9f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                if (KIND == 0) asm volatile("v_fmac_f32_e32 %0, %1, %2" : "+v"(v[i]) : "v"(va), "v"(vb));
                if (KIND == 1) asm volatile("v_fmac_f32_e32 %0, %1, %2" : "+v"(v[i]) : "s"(sa), "v"(vb));
                if (KIND == 2) v[i] = __builtin_amdgcn_exp2f(v[i]);
                if (KIND == 3) v[i] = __builtin_amdgcn_rsqf(v[i]);
                if (KIND == 4)
                    asm volatile("v_fmac_f32_dpp %0, %1, %2 row_newbcast:5 row_mask:0xf bank_mask:0xf"
                                 : "+v"(v[i]) : "v"(va), "v"(vb));
                if (KIND == 5) asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(v[i]) : "v"(va), "v"(vb));
                if (KIND == 6) asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(v[i]) : "v"(va), "s"(sa));
                if (KIND == 7) asm volatile("v_fma_f32 %0, %1, %2, %3" : "=v"(v[i]) : "v"(va), "v"(v[i]), "s"(sa));
                if (KIND == 8) asm volatile("v_mov_b32 %0, %1" : "=v"(v[i]) : "s"(sa));
            }
        }
    }
    float s = 0.f;
    for (int i = 0; i < CH; ++i) s += v[i];
    if (s == 12345.678f) out[threadIdx.x] = s;  // keep the chains live
}

// Loops written out in one asm statement with fixed registers, so that the
// register banks (register number mod 4) and the instruction order are known:
// 9: v_fmac_f32 whose accumulators share a bank with one source (v32, v36, ..
// against v20), 10: the same with the accumulators in another bank (v33, v37,
// ..), 11: seven of kind 10's FMAs and one independent v_exp_f32 in every
// eight instructions.  16 x 8 instructions per trip, as in k_rate.
#define MB_INIT                                                                                             \
    "v_mov_b32 v20, 0.5\nv_mov_b32 v22, 0.5\nv_mov_b32 v32, 0.5\nv_mov_b32 v33, 0.5\nv_mov_b32 v36, 0.5\n" \
    "v_mov_b32 v37, 0.5\nv_mov_b32 v40, 0.5\nv_mov_b32 v41, 0.5\nv_mov_b32 v44, 0.5\nv_mov_b32 v45, 0.5\n" \
    "v_mov_b32 v48, 0.5\nv_mov_b32 v49, 0.5\nv_mov_b32 v52, 0.5\nv_mov_b32 v53, 0.5\nv_mov_b32 v56, 0.5\n" \
    "v_mov_b32 v57, 0.5\nv_mov_b32 v60, 0.5\nv_mov_b32 v61, 0.5\n"
#define MB_F(r) "v_fmac_f32_e32 v" #r ", v20, v22\n"
#define MB_SAME MB_F(32) MB_F(36) MB_F(40) MB_F(44) MB_F(48) MB_F(52) MB_F(56) MB_F(60)
#define MB_OTHER MB_F(33) MB_F(37) MB_F(41) MB_F(45) MB_F(49) MB_F(53) MB_F(57) MB_F(61)
#define MB_EXP MB_F(33) MB_F(37) MB_F(41) MB_F(45) MB_F(49) MB_F(53) MB_F(57) "v_exp_f32_e32 v60, v20\n"
#define MB_X16(g) g g g g g g g g g g g g g g g g
#define MB_LOOP(g)                                                                                      \
    asm volatile(MB_INIT "s_mov_b32 s40, %0\n1:\n" MB_X16(g) "s_sub_u32 s40, s40, 1\ns_cmp_lg_u32 s40, 0\n" \
                 "s_cbranch_scc1 1b\n"                                                                  \
                 :                                                                                      \
                 : "s"(iters)                                                                           \
                 : "v20", "v22", "v32", "v33", "v36", "v37", "v40", "v41", "v44", "v45", "v48", "v49", "v52", \
                   "v53", "v56", "v57", "v60", "v61", "s40", "scc")

template <int KIND>
__global__ __launch_bounds__(256) void k_fixed(int iters) {
    if (iters < 1) return;
    if (KIND == 9) MB_LOOP(MB_SAME);
    if (KIND == 10) MB_LOOP(MB_OTHER);
    if (KIND == 11) MB_LOOP(MB_EXP);
}

}  // namespace

extern "C" {

// Runs kind (0: FMA vector operands, 1: FMA scalar operand, 2: exp2, 3: rsq,
// 4: FMA with a DPP row-broadcast operand, 5: FMA in its three-operand VOP3 form,
// 6: VOP3 FMA with a scalar register as its second operand, 7: as its addend,
// 8: v_mov_b32 from a scalar register, 9: FMA whose accumulator shares a
// register bank with a source, 10: the same FMAs without the shared bank,
// 11: seven FMAs of kind 10 and one v_exp_f32 in every eight instructions)
// on `blocks` work-groups of 256 threads for `iters` x 16 x 8 operations per
// lane (kinds 2 and 3: one per operation; kind 11 counts the exp as one).  Returns the device time in milliseconds (< 0 on error).
float vfmm_mb_rate(int kind, int blocks, int iters) {
    float *out = nullptr;
    if (hipMalloc(&out, 256 * sizeof(float)) != hipSuccess) return -1.f;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    auto launch = [&]() {
        switch (kind) {
            case 0: k_rate<0><<<blocks, 256>>>(out, iters, 0.999f, 0.9999f); break;
            case 1: k_rate<1><<<blocks, 256>>>(out, iters, 0.999f, 0.9999f); break;
            case 2: k_rate<2><<<blocks, 256>>>(out, iters, 0.999f, 0.9999f); break;
            case 4: k_rate<4><<<blocks, 256>>>(out, iters, 0.999f, 0.9999f); break;
            case 5: k_rate<5><<<blocks, 256>>>(out, iters, 0.999f, 0.9999f); break;
            case 6: k_rate<6><<<blocks, 256>>>(out, iters, 0.999f, 0.9999f); break;
            case 7: k_rate<7><<<blocks, 256>>>(out, iters, 0.999f, 0.9999f); break;
            case 8: k_rate<8><<<blocks, 256>>>(out, iters, 0.999f, 0.9999f); break;
            case 9: k_fixed<9><<<blocks, 256>>>(iters); break;
            case 10: k_fixed<10><<<blocks, 256>>>(iters); break;
            case 11: k_fixed<11><<<blocks, 256>>>(iters); break;
            default: k_rate<3><<<blocks, 256>>>(out, iters, 0.999f, 0.9999f); break;
        }
    };
    launch();
    (void)hipEventRecord(e0, nullptr);
    launch();
    (void)hipEventRecord(e1, nullptr);
    float ms = -1.f;
    if (hipEventSynchronize(e1) == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (hipGetLastError() != hipSuccess) return -1.f;
    return ms;
}
}
