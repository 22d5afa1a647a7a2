// mlp.h -- BF16 MFMA building blocks of the learned proposal network.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppl {

// Network shape: 64 -> 256 -> 256 -> 256, ReLU after layers 1 and 2.
constexpr int kMlpIn = 64;
constexpr int kMlpHid = 256;
constexpr int kMlpOut = 256;
constexpr int kMlpLayers = 3;

// Parameter block (device, caller-owned), in this order:
//   FP32 master copy of all parameters, Adam first and second moments (same
//   layout), then BF16 copies of each weight matrix in two layouts:
//   Wt[l] = [out][in] (row = output unit) and W[l] = [in][out].
// Per layer l the FP32 parameters are W_l as [out][in] followed by b_l[out].
struct MlpParams {
    __host__ __device__ static constexpr int in(int l) { return l == 0 ? kMlpIn : kMlpHid; }
    __host__ __device__ static constexpr int out(int l) { return l == 2 ? kMlpOut : kMlpHid; }
    __host__ __device__ static constexpr int64_t w_off(int l) {
        return l == 0 ? 0 : l == 1 ? (int64_t)kMlpIn * kMlpHid + kMlpHid
                                   : (int64_t)kMlpIn * kMlpHid + kMlpHid + (int64_t)kMlpHid * kMlpHid + kMlpHid;
    }
    __host__ __device__ static constexpr int64_t b_off(int l) { return w_off(l) + (int64_t)in(l) * out(l); }
    __host__ __device__ static constexpr int64_t count() { return b_off(2) + kMlpOut; }      // 148224
    __host__ __device__ static constexpr int64_t bf16_w_off(int l) {                         // offsets within one BF16 layout
        return l == 0 ? 0 : l == 1 ? (int64_t)kMlpIn * kMlpHid : (int64_t)kMlpIn * kMlpHid + (int64_t)kMlpHid * kMlpHid;
    }
    __host__ __device__ static constexpr int64_t bf16_count() { return bf16_w_off(2) + (int64_t)kMlpHid * kMlpOut; }
    static constexpr size_t step_off() {                                  // int64 Adam step count
        return (3 * count() * sizeof(float) + 2 * bf16_count() * sizeof(uint16_t) + 255) / 256 * 256;
    }
    // BF16 copies of both layouts in fragment order (frag_index), after the
    // step count: what the fused training pass loads
    static constexpr size_t frag_off() { return step_off() + 256; }
    static constexpr size_t bytes() { return frag_off() + (2 * bf16_count() * sizeof(uint16_t) + 255) / 256 * 256; }
};

// Position of element (n, k) of a weight matrix with rows n < 256 and KD
// columns (KD a multiple of 32) in fragment order: wave n / 64 of the fused
// training pass loads, for k-step s = k / 32 and column tile j = (n % 64) / 16,
// 64 lanes x 8 consecutive values (lane = 16 ((k % 32) / 8) + n % 16), so each
// of its load instructions reads 1 KB of consecutive bytes.
__host__ __device__ inline int64_t frag_index(int n, int k, int KD) {
    const int wave = n >> 6, j = (n >> 4) & 3, s = k >> 5, lane = ((k & 31) >> 3) * 16 + (n & 15);
    return ((((int64_t)wave * (KD >> 5) + s) * 4 + j) * 64 + lane) * 8 + (k & 7);
}

// FP32 -> BF16 bit pattern, round to nearest even (NaN stays NaN).
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf16_to_f32(uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

struct MlpView {
    float *master, *m, *v;
    uint16_t *wt, *w;        // BF16 bit patterns: [out][in] and [in][out]
    uint16_t *wtf, *wf;      // the same two in fragment order (frag_index)
    int64_t *step;           // completed Adam steps (device)
};

inline MlpView mlp_view(void *p) {
    MlpView v;
    v.master = (float *)p;
    v.m = v.master + MlpParams::count();
    v.v = v.m + MlpParams::count();
    v.wt = (uint16_t *)(v.v + MlpParams::count());
    v.w = v.wt + MlpParams::bf16_count();
    v.step = (int64_t *)((char *)p + MlpParams::step_off());
    v.wtf = (uint16_t *)((char *)p + MlpParams::frag_off());
    v.wf = v.wtf + MlpParams::bf16_count();
    return v;
}

// Epilogue of the NT GEMM C[M][N] = sum_r A[M][r] B[N][r] (+ bias[N]).
enum MlpEpi : int {
    kEpiRelu = 1,        // max(0, .)
    kEpiOutRow = 2,      // BF16 row-major [M][N] output
    kEpiOutCol = 4,      // BF16 column-major [N][M] output
    kEpiOutF32 = 8,      // FP32 row-major output
    kEpiMaskRow = 16,    // multiply by (mask[M][N] > 0), mask BF16 row-major (ReLU derivative)
    kEpiBias = 32,
    kEpiOutF32Col = 64,  // FP32 column-major [N][M] output
};

// ------------------------------------------------------------ GEMM tile --
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

constexpr int kGemmTile = 64;

__device__ __forceinline__ bf16x8_t load_frag(const uint16_t *p) { return *(const bf16x8_t *)p; }

// One 64 x 64 output tile (bx, by) of C = A B^T over R-chunk bz, four waves of
// 32 x 32 (the body of gemm_nt_kernel, also run by grouped launches).
template <int EPI>
__device__ __forceinline__ void gemm_nt_tile(const uint16_t *__restrict__ A, const uint16_t *__restrict__ B, int M,
                                             int N, int R, int lda, int ldb, const float *__restrict__ bias,
                                             const uint16_t *__restrict__ mask, uint16_t *__restrict__ out_row,
                                             uint16_t *__restrict__ out_col, float *__restrict__ out_f32, int r_chunk,
                                             int bx, int by, int bz) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = by * kGemmTile + (wave >> 1) * 32;
    const int n0 = bx * kGemmTile + (wave & 1) * 32;
    const int r_begin = bz * r_chunk;
    const int r_end = min(R, r_begin + r_chunk);
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    floatx4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    const uint16_t *a0 = A + (size_t)(m0 + fr) * lda + fk;
    const uint16_t *a1 = A + (size_t)(m0 + 16 + fr) * lda + fk;
    const uint16_t *b0 = B + (size_t)(n0 + fr) * ldb + fk;
    const uint16_t *b1 = B + (size_t)(n0 + 16 + fr) * ldb + fk;
    for (int r = r_begin; r < r_end; r += 32) {
        const bf16x8_t fa0 = load_frag(a0 + r), fa1 = load_frag(a1 + r);
        const bf16x8_t fb0 = load_frag(b0 + r), fb1 = load_frag(b1 + r);
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa0, fb0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa0, fb1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa1, fb0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa1, fb1, acc[1][1], 0, 0, 0);
    }
    // epilogue: acc[i][j][q] is C[m0 + 16 i + 4 (lane/16) + q][n0 + 16 j + lane%16]
    float *part = (EPI & kEpiOutF32) ? out_f32 + (size_t)bz * M * N : nullptr;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + 16 * j + fr;
            const int mb = m0 + 16 * i + (lane >> 4) * 4;
            const float bn = (EPI & kEpiBias) ? bias[n] : 0.0f;
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = mb + q;
                float t = acc[i][j][q] + bn;
                if (EPI & kEpiMaskRow) t = (mask[(size_t)m * N + n] & 0x7FFFu) ? t : 0.0f;
                if (EPI & kEpiRelu) t = fmaxf(t, 0.0f);
                v[q] = t;
                if (EPI & kEpiOutF32) part[(size_t)m * N + n] = t;
                if (EPI & kEpiOutRow) out_row[(size_t)m * N + n] = f32_to_bf16(t);
            }
            if (EPI & kEpiOutF32Col) *(float4 *)(out_f32 + (size_t)n * M + mb) = make_float4(v[0], v[1], v[2], v[3]);
            if (EPI & kEpiOutCol) {
                const uint32_t lo = (uint32_t)f32_to_bf16(v[0]) | ((uint32_t)f32_to_bf16(v[1]) << 16);
                const uint32_t hi = (uint32_t)f32_to_bf16(v[2]) | ((uint32_t)f32_to_bf16(v[3]) << 16);
                *(uint2 *)(out_col + (size_t)n * M + mb) = make_uint2(lo, hi);
            }
        }
    }
}

// Launch C = A B^T for BF16 operands stored with the reduction dimension
// contiguous (A: [M][R], B: [N][R]); M, N multiples of 64, R multiple of 32.
int mlp_gemm(const uint16_t *A, const uint16_t *B, int M, int N, int R, int lda, int ldb, int epi, const float *bias,
             const uint16_t *mask, uint16_t *out_row, uint16_t *out_col, float *out_f32, hipStream_t st);

// Split-R variant for weight gradients: partial[c][M][N] (FP32) over
// R-chunks of `chunk` (a multiple of 32); the consumer sums the chunks in order.
int mlp_gemm_splitr(const uint16_t *A, const uint16_t *B, int M, int N, int R, int lda, int ldb, int chunk,
                    float *partial, hipStream_t st);

// Number of R-chunks the split GEMM uses for an M x N output over R rows, and
// the chunk length (both fixed by the shape, so every call sums in one order).
void mlp_split_plan(int M, int N, int R, int *nchunks, int *chunk);

}  // namespace ppl
