// Issue-rate probe: the throughput of single vector-ALU instruction classes on
// the GPU, used to price a compute-bound kernel by its instruction mix (the
// noise pass is bound by instruction issue, and on gfx950 wave64 instructions
// of different classes occupy a SIMD for different numbers of cycles).
//
// Each class runs in its own kernel: every thread executes kIter iterations of
// eight independent dependency chains of that one instruction (written as
// inline assembly so that the compiler neither folds nor reorders them), at
// eight waves per SIMD; the only memory access is one in-bounds store per
// thread at the end.  Output, one line per class: the kernel time and the time
// per wave-level instruction per SIMD (kernel time x SIMDs / wave
// instructions), which needs no assumption about the clock.
//
// Build: done by paper_2511_10353_amd.build (hipcc --offload-arch=gfx950).
// Run:   paper_2511_10353_amd/probe/issue_probe
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

namespace {

constexpr int kIter = 16000;
constexpr int kBlock = 256;
constexpr int kClasses = 15;

const char* const kNames[kClasses] = {"v_add_u32",     "v_xor_b32",     "v_lshlrev_b32", "v_bitop3_b32",
                                      "v_mov_b32",     "v_cndmask_b32", "v_fma_f32",     "v_add_f32",
                                      "v_fma_f64",     "v_mul_f64",     "v_add_f64",     "v_rsq_f64",
                                      "v_mad_u64_u32", "v_cvt_f64_u32", "v_cvt_f32_f64"};

#define GG_CH8(S) S(a0) S(a1) S(a2) S(a3) S(a4) S(a5) S(a6) S(a7)

template <int OP>
__global__ __launch_bounds__(kBlock) void k_issue(float* out, uint32_t seed) {
    const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
    if constexpr (OP <= 7) {
        uint32_t a0 = t, a1 = t + 1, a2 = t + 2, a3 = t + 3, a4 = t + 4, a5 = t + 5, a6 = t + 6, a7 = t + 7;
        const uint32_t b = seed | 1u, c = seed ^ 0x9E3779B9u;
        const uint64_t m = 0x5555555555555555ull ^ seed;
        for (int i = 0; i < kIter; ++i) {
#define S0(x) asm volatile("v_add_u32 %0, %0, %1" : "+v"(x) : "v"(b));
#define S1(x) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(x) : "v"(b));
#define S2(x) asm volatile("v_lshlrev_b32 %0, 1, %0" : "+v"(x));
#define S3(x) asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(x) : "v"(b), "v"(c));
#define S4(x) asm volatile("v_mov_b32 %0, %0" : "+v"(x));
#define S5(x) asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(x) : "v"(b), "s"(m));
#define S6(x) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(x) : "v"(b), "v"(c));
#define S7(x) asm volatile("v_add_f32 %0, %0, %1" : "+v"(x) : "v"(b));
            if constexpr (OP == 0) { GG_CH8(S0) }
            if constexpr (OP == 1) { GG_CH8(S1) }
            if constexpr (OP == 2) { GG_CH8(S2) }
            if constexpr (OP == 3) { GG_CH8(S3) }
            if constexpr (OP == 4) { GG_CH8(S4) }
            if constexpr (OP == 5) { GG_CH8(S5) }
            if constexpr (OP == 6) { GG_CH8(S6) }
            if constexpr (OP == 7) { GG_CH8(S7) }
        }
        out[t] = (float)(a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7);
    } else if constexpr (OP <= 11) {
        double a0 = t, a1 = t + 1, a2 = t + 2, a3 = t + 3, a4 = t + 4, a5 = t + 5, a6 = t + 6, a7 = t + 7;
        const double b = 1.0 + seed * 1e-9, c = 0.5;
        for (int i = 0; i < kIter; ++i) {
#define D8(x) asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(x) : "v"(b), "v"(c));
#define D9(x) asm volatile("v_mul_f64 %0, %0, %1" : "+v"(x) : "v"(b));
#define D10(x) asm volatile("v_add_f64 %0, %0, %1" : "+v"(x) : "v"(b));
#define D11(x) asm volatile("v_rsq_f64 %0, %0" : "+v"(x));
            if constexpr (OP == 8) { GG_CH8(D8) }
            if constexpr (OP == 9) { GG_CH8(D9) }
            if constexpr (OP == 10) { GG_CH8(D10) }
            if constexpr (OP == 11) { GG_CH8(D11) }
        }
        out[t] = (float)(a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7);
    } else if constexpr (OP <= 13) {
        uint64_t a0 = t, a1 = t + 1, a2 = t + 2, a3 = t + 3, a4 = t + 4, a5 = t + 5, a6 = t + 6, a7 = t + 7;
        const uint32_t b = seed | 1u, c = 0xD2511F53u;
        for (int i = 0; i < kIter; ++i) {
#define M12(x) { uint64_t cy; asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(x), "=s"(cy) : "v"(b), "v"(c)); }
#define M13(x) asm volatile("v_cvt_f64_u32 %0, %1" : "=v"(x) : "v"((uint32_t)x));
            if constexpr (OP == 12) { GG_CH8(M12) }
            if constexpr (OP == 13) { GG_CH8(M13) }
        }
        out[t] = (float)(a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7);
    } else {
        float a0 = t, a1 = t + 1, a2 = t + 2, a3 = t + 3, a4 = t + 4, a5 = t + 5, a6 = t + 6, a7 = t + 7;
        const double b = 1.0 + seed * 1e-9;
        for (int i = 0; i < kIter; ++i) {
#define C14(x) asm volatile("v_cvt_f32_f64 %0, %1" : "=v"(x) : "v"(b));
            GG_CH8(C14)
        }
        out[t] = a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7;
    }
}

template <int OP>
float time_class(float* out, int nblk, hipEvent_t e0, hipEvent_t e1) {
    k_issue<OP><<<nblk, kBlock>>>(out, 12345u);  // warm-up
    (void)hipEventRecord(e0);
    k_issue<OP><<<nblk, kBlock>>>(out, 12345u);
    (void)hipEventRecord(e1);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return ms;
}

template <int... OPS>
void time_all(float* out, int nblk, hipEvent_t e0, hipEvent_t e1, float* ms, std::integer_sequence<int, OPS...>) {
    ((ms[OPS] = time_class<OPS>(out, nblk, e0, e1)), ...);
}

}  // namespace

int main() {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, 0) != hipSuccess) {
        fprintf(stderr, "no HIP device\n");
        return 1;
    }
    const int cus = prop.multiProcessorCount;
    const int nblk = cus * 8;  // 8 work-groups of 4 waves per CU: 8 waves per SIMD
    float* out = nullptr;
    if (hipMalloc(&out, sizeof(float) * (size_t)nblk * kBlock) != hipSuccess) return 1;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
    float ms[kClasses];
    time_all(out, nblk, e0, e1, ms, std::make_integer_sequence<int, kClasses>{});
    if (hipDeviceSynchronize() != hipSuccess) return 1;
    const double waves = (double)nblk * (kBlock / 64);
    const double winstr = waves * kIter * 8;  // wave-level instructions of the class per kernel
    const double simds = cus * 4.0;
    printf("# %d CUs, %d SIMDs, %.0f waves of 8 chains x %d iterations\n", cus, (int)simds, waves, kIter);
    printf("# class  kernel_ms  ns_per_wave_instruction_per_SIMD\n");
    for (int i = 0; i < kClasses; ++i)
        printf("%s %.4f %.4f\n", kNames[i], ms[i], ms[i] * 1e6 * simds / winstr);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return 0;
}
