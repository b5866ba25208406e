// Issue-rate probe for gfx950: SIMD cycles per wave64 instruction of the
// instructions the product sweeps are built from (v_exp_f32, v_fma_f32,
// v_cvt_pk_bf16_f32, FP32 and BF16 MFMA), alone and interleaved, so that a
// sweep's instruction counts (rocprofv3 SQ_INSTS_* counters) can be turned
// into the cycles they take.  A standalone program, not part of libmfgp.so.
//
// Each mode runs kNit iterations of a fixed instruction mix over independent
// register chains in every lane; 8 resident waves per SIMD (2048 blocks of 4
// waves on 256 CUs, one dispatch round).  Cycles per SIMD for one iteration =
// launch time x 2.4 GHz / (wave-iterations per SIMD), after about 200 ms of
// warm-up launches; a clock below 2.4 GHz under a given mix shows as more
// cycles.  Every lane writes one float (its chains' sum) so that nothing is
// optimised away.
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

constexpr int kNit = 4096;
constexpr int kBlocks = 2048;

enum Mode {
    EXP8,          // 8 v_exp_f32
    FMA8,          // 8 v_fma_f32
    EXP8_FMA8,     // both
    MF32_4,        // 4 v_mfma_f32_16x16x4_f32
    EXP8_MF32_4,   // 8 exp + 4 FP32 MFMA
    FMA8_MF32_4,   // 8 fma + 4 FP32 MFMA
    EXP8_FMA8_MF32_1,
    MBF16_4,       // 4 v_mfma_f32_32x32x16_bf16
    FMA8_MBF16_4,  // 8 fma + 4 BF16 MFMA
    EXP8_MBF16_4,  // 8 exp + 4 BF16 MFMA
    CVT8,          // 8 v_cvt_pk_bf16_f32
    kModes
};

const char* kNames[kModes] = {"8 exp",          "8 fma",          "8 exp + 8 fma",  "4 mfma_f32_16x16x4",
                              "8 exp + 4 mfma_f32", "8 fma + 4 mfma_f32", "8 exp + 8 fma + 1 mfma_f32",
                              "4 mfma_bf16_32x32x16", "8 fma + 4 mfma_bf16", "8 exp + 4 mfma_bf16",
                              "8 cvt_pk_bf16_f32"};

template <int MODE>
__global__ __launch_bounds__(256) void probe(float* __restrict__ out, float b, float c) {
    float a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = 0.5f + 1e-4f * ((threadIdx.x + k) & 63);
    f32x4 acc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
    f32x16 acc16[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < 16; ++q) acc16[k][q] = 0.f;
    const float ma = 1e-3f * (threadIdx.x & 7), mb = 1e-3f * (threadIdx.x & 3);
    bf16x8 ha, hb;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        ha[q] = static_cast<__bf16>(ma + q);
        hb[q] = static_cast<__bf16>(mb - q);
    }

    for (int it = 0; it < kNit; ++it) {
        if constexpr (MODE == EXP8 || MODE == EXP8_FMA8 || MODE == EXP8_MF32_4 || MODE == EXP8_FMA8_MF32_1 ||
                      MODE == EXP8_MBF16_4) {
#pragma unroll
            for (int k = 0; k < 8; ++k) a[k] = __builtin_amdgcn_exp2f(-a[k]);
        }
        if constexpr (MODE == FMA8 || MODE == EXP8_FMA8 || MODE == FMA8_MF32_4 || MODE == EXP8_FMA8_MF32_1 ||
                      MODE == FMA8_MBF16_4) {
#pragma unroll
            for (int k = 0; k < 8; ++k) a[k] = fmaf(a[k], b, c);
        }
        if constexpr (MODE == MF32_4 || MODE == EXP8_MF32_4 || MODE == FMA8_MF32_4) {
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(ma, mb, acc[k], 0, 0, 0);
        }
        if constexpr (MODE == EXP8_FMA8_MF32_1) acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(ma, mb, acc[0], 0, 0, 0);
        if constexpr (MODE == MBF16_4 || MODE == FMA8_MBF16_4 || MODE == EXP8_MBF16_4) {
#pragma unroll
            for (int k = 0; k < 4; ++k) acc16[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ha, hb, acc16[k], 0, 0, 0);
        }
        if constexpr (MODE == CVT8) {
            // two values per conversion; each reads the previous result's bits
            // as one of its inputs (a dependent chain per k)
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const f32x2v v = {a[k], b};
                a[k] = __builtin_bit_cast(float, __builtin_convertvector(v, bf16x2v));
            }
        }
    }

    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += a[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3] + acc16[k][0] + acc16[k][15];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

template <int M>
void launch(float* out) {
    hipLaunchKernelGGL(probe<M>, dim3(kBlocks), dim3(256), 0, 0, out, 0.999f, 1e-4f);
}

typedef void (*LaunchFn)(float*);
const LaunchFn kLaunch[kModes] = {launch<0>, launch<1>, launch<2>, launch<3>, launch<4>,
                                  launch<5>, launch<6>, launch<7>, launch<8>, launch<9>, launch<10>};

}  // namespace

int main() {
    float* out = nullptr;
    if (hipMalloc(&out, sizeof(float) * kBlocks * 256) != hipSuccess) return 1;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
    // about 200 ms of warm-up launches so that the clocks have ramped
    for (int w = 0; w < 200; ++w) kLaunch[FMA8_MF32_4](out);
    if (hipDeviceSynchronize() != hipSuccess) return 2;
    printf("%-28s %16s\n", "mix per iteration", "cycles per SIMD");
    for (int m = 0; m < kModes; ++m) {
        for (int w = 0; w < 5; ++w) kLaunch[m](out);
        const int reps = 10;
        (void)hipEventRecord(e0, 0);
        for (int r = 0; r < reps; ++r) kLaunch[m](out);
        (void)hipEventRecord(e1, 0);
        if (hipEventSynchronize(e1) != hipSuccess) return 2;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= reps;
        const double cycles = ms * 1e-3 * 2.4e9 / (static_cast<double>(kBlocks) * 4 * kNit / 1024.0);
        printf("%-28s %16.2f\n", kNames[m], cycles);
    }
    (void)hipFree(out);
    return 0;
}
