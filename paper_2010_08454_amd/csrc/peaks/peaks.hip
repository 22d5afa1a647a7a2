// peaks.hip -- micro-benchmarks of the gfx950 rates that the roofline
// fractions are priced against: FP32 and FP64 FMA, the transcendental unit
// (v_exp_f32, v_log_f32, v_sin_f32), 32-bit integer multiply-high (the
// Philox rounds), BF16 MFMA and an HBM copy.  Built as its own library
// (libppl_peaks.so) and used only to measure; nothing in libppl calls it.
//
// Each ALU kernel runs kChains independent dependency chains per lane,
// kUnroll steps per loop iteration, so a lane issues kChains * kUnroll
// instructions of the measured kind per iteration, and stores its result so
// that no chain is dead.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kThreads = 256;
constexpr int kChains = 8;
constexpr int kUnroll = 8;

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

enum {
    PEAK_FMA_F32 = 0,
    PEAK_FMA_F64 = 1,
    PEAK_EXP_F32 = 2,
    PEAK_LOG_F32 = 3,
    PEAK_SIN_F32 = 4,
    PEAK_MULHI_U32 = 5,
    PEAK_MFMA_BF16 = 6,
};

__global__ __launch_bounds__(kThreads) void fma_f32_kernel(int iters, float a, float b, float *__restrict__ out) {
    float x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = threadIdx.x * 1e-3f + k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int k = 0; k < kChains; ++k) x[k] = fmaf(x[k], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    out[blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void fma_f64_kernel(int iters, double a, double b, float *__restrict__ out) {
    double x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = threadIdx.x * 1e-3 + k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int k = 0; k < kChains; ++k) x[k] = fma(x[k], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    out[blockIdx.x * kThreads + threadIdx.x] = (float)s;
}

// One transcendental per step: x = 2^-x, x = log2 |x| or x = sin(2 pi x)
// (the negation and absolute value are source modifiers of the instruction).
template <int KIND>
__global__ __launch_bounds__(kThreads) void trans_f32_kernel(int iters, float *__restrict__ out) {
    float x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = 0.25f + 0.01f * k + threadIdx.x * 1e-4f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int k = 0; k < kChains; ++k) {
                if constexpr (KIND == PEAK_EXP_F32) x[k] = __builtin_amdgcn_exp2f(-x[k]);
                else if constexpr (KIND == PEAK_LOG_F32) x[k] = __builtin_amdgcn_logf(fabsf(x[k]));
                else x[k] = __builtin_amdgcn_sinf(x[k]);
            }
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    out[blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void mulhi_u32_kernel(int iters, uint32_t c, float *__restrict__ out) {
    uint32_t x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = 0x9E3779B9u * (threadIdx.x + 1) + 0x85EBCA6Bu * k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int k = 0; k < kChains; ++k) x[k] = __umulhi(x[k], c);
    }
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s ^= x[k];
    out[blockIdx.x * kThreads + threadIdx.x] = (float)s;
}

// v_mfma_f32_16x16x32_bf16: kChains independent accumulators per wave; each
// instruction is 16 x 16 x 32 multiply-adds (16384 FLOP) per wave.
__global__ __launch_bounds__(kThreads) void mfma_bf16_kernel(int iters, float *__restrict__ out) {
    bf16x8_t a, b;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        a[k] = (__bf16)(1e-3f * (threadIdx.x + k));
        b[k] = (__bf16)(1e-3f * (threadIdx.x - k));
    }
    floatx4_t acc[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) acc[k] = floatx4_t{0.0f, 0.0f, 0.0f, 0.0f};
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int k = 0; k < kChains; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[k], 0, 0, 0);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// HBM copy, 16 bytes per lane per step, grid-stride over n4 float4 words.
__global__ __launch_bounds__(kThreads) void copy_kernel(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                        int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n4; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" {

// Launches micro-benchmark `kind` on `blocks` workgroups of 256 threads for
// `iters` loop iterations; out holds blocks * 256 floats (device).  Returns 0,
// or -1 for an unknown kind or invalid sizes, or the HIP error code.
int peak_alu(int kind, int blocks, int iters, float *out, void *stream) {
    if (blocks < 1 || iters < 1 || !out) return -1;
    hipStream_t st = (hipStream_t)stream;
    switch (kind) {
        case PEAK_FMA_F32: hipLaunchKernelGGL(fma_f32_kernel, dim3(blocks), dim3(kThreads), 0, st, iters, 0.999f, 1e-3f, out); break;
        case PEAK_FMA_F64: hipLaunchKernelGGL(fma_f64_kernel, dim3(blocks), dim3(kThreads), 0, st, iters, 0.999, 1e-3, out); break;
        case PEAK_EXP_F32: hipLaunchKernelGGL(trans_f32_kernel<PEAK_EXP_F32>, dim3(blocks), dim3(kThreads), 0, st, iters, out); break;
        case PEAK_LOG_F32: hipLaunchKernelGGL(trans_f32_kernel<PEAK_LOG_F32>, dim3(blocks), dim3(kThreads), 0, st, iters, out); break;
        case PEAK_SIN_F32: hipLaunchKernelGGL(trans_f32_kernel<PEAK_SIN_F32>, dim3(blocks), dim3(kThreads), 0, st, iters, out); break;
        case PEAK_MULHI_U32: hipLaunchKernelGGL(mulhi_u32_kernel, dim3(blocks), dim3(kThreads), 0, st, iters, 0x9E3779B9u, out); break;
        case PEAK_MFMA_BF16: hipLaunchKernelGGL(mfma_bf16_kernel, dim3(blocks), dim3(kThreads), 0, st, iters, out); break;
        default: return -1;
    }
    return (int)hipGetLastError();
}

// Copies n4 16-byte words from src to dst (device buffers of n4 * 16 bytes).
int peak_copy(const void *src, void *dst, int64_t n4, int blocks, void *stream) {
    if (!src || !dst || n4 < 1 || blocks < 1) return -1;
    hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(kThreads), 0, (hipStream_t)stream, (const float4 *)src,
                       (float4 *)dst, n4);
    return (int)hipGetLastError();
}

// Instructions of the measured kind per lane per loop iteration.
int peak_ops_per_iter(int kind) { return (kind >= 0 && kind <= PEAK_MFMA_BF16) ? kChains * kUnroll : 0; }

}  // extern "C"
