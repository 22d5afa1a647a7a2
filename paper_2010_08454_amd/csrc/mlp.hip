// mlp.hip -- BF16 MFMA GEMMs of the proposal network (gfx950 v_mfma_f32_16x16x32_bf16).
//
// Every product of the network -- forward layers, input gradients and weight
// gradients -- is written as an "NT" GEMM C[M][N] = sum_r A[M][r] B[N][r]
// whose operands keep the reduction index contiguous, so each lane loads its
// MFMA fragment (8 consecutive BF16 values) with one 16-byte load.  Activations
// and gradients are therefore produced in both row- and column-major BF16
// layouts by the epilogues, and the weights are kept as [out][in] and [in][out].
//
// MFMA fragment layout (16x16x32): lane l supplies A[row l%16][k 8(l/16)..+7]
// and B[col l%16][k 8(l/16)..+7] and receives C[rows 4(l/16)..+3][col l%16].
// A workgroup of 4 waves computes a 64x64 tile, each wave a 32x32 quarter
// (2x2 MFMA blocks); accumulation is FP32.
#include "host.h"
#include "mlp.h"
#include "timing.h"

namespace ppl {

template <int EPI>
__global__ __launch_bounds__(256) void gemm_nt_kernel(const uint16_t *__restrict__ A, const uint16_t *__restrict__ B,
                                                      int M, int N, int R, int lda, int ldb,
                                                      const float *__restrict__ bias, const uint16_t *__restrict__ mask,
                                                      uint16_t *__restrict__ out_row, uint16_t *__restrict__ out_col,
                                                      float *__restrict__ out_f32, int r_chunk) {
    gemm_nt_tile<EPI>(A, B, M, N, R, lda, ldb, bias, mask, out_row, out_col, out_f32, r_chunk, blockIdx.x, blockIdx.y,
                      blockIdx.z);
}

template <int EPI>
static void launch_gemm(const uint16_t *A, const uint16_t *B, int M, int N, int R, int lda, int ldb, const float *bias,
                        const uint16_t *mask, uint16_t *orow, uint16_t *ocol, float *of32, int chunk, int nchunks,
                        hipStream_t st) {
    hipLaunchKernelGGL(gemm_nt_kernel<EPI>, dim3(N / kGemmTile, M / kGemmTile, nchunks), dim3(256), 0, st, A, B, M, N,
                       R, lda, ldb, bias, mask, orow, ocol, of32, chunk);
}

int mlp_gemm(const uint16_t *A, const uint16_t *B, int M, int N, int R, int lda, int ldb, int epi, const float *bias,
             const uint16_t *mask, uint16_t *out_row, uint16_t *out_col, float *out_f32, hipStream_t st) {
    if (M % kGemmTile || N % kGemmTile || R % 32 || M <= 0 || N <= 0 || R <= 0)
        return fail(PPL_E_ARG, "GEMM shape %d x %d x %d is not a multiple of the 64 x 64 x 32 tile", M, N, R);
    KernelTimer timer("gemm_nt_kernel", st);
    switch (epi) {
#define PPL_EPI(E) case (E): launch_gemm<(E)>(A, B, M, N, R, lda, ldb, bias, mask, out_row, out_col, out_f32, R, 1, st); break;
        PPL_EPI(kEpiBias | kEpiRelu | kEpiOutRow | kEpiOutCol)
        PPL_EPI(kEpiBias | kEpiRelu | kEpiOutRow)
        PPL_EPI(kEpiBias | kEpiOutF32Col)
        PPL_EPI(kEpiMaskRow | kEpiOutRow | kEpiOutCol)
        PPL_EPI(kEpiMaskRow | kEpiOutCol)
        PPL_EPI(kEpiOutF32)
#undef PPL_EPI
        default: return fail(PPL_E_ARG, "unsupported GEMM epilogue %d", epi);
    }
    timer.stop();
    PPL_LAUNCH_CHECK("gemm_nt_kernel");
    return PPL_OK;
}

int mlp_gemm_splitr(const uint16_t *A, const uint16_t *B, int M, int N, int R, int lda, int ldb, int chunk,
                    float *partial, hipStream_t st) {
    if (M % kGemmTile || N % kGemmTile || R % 32 || chunk % 32 || chunk <= 0 || M <= 0 || N <= 0 || R <= 0)
        return fail(PPL_E_ARG, "split GEMM shape %d x %d x %d / %d not tile-aligned", M, N, R, chunk);
    const int nchunks = (R + chunk - 1) / chunk;
    KernelTimer timer("gemm_nt_kernel", st);
    launch_gemm<kEpiOutF32>(A, B, M, N, R, lda, ldb, nullptr, nullptr, nullptr, nullptr, partial, chunk, nchunks, st);
    timer.stop();
    PPL_LAUNCH_CHECK("gemm_nt_kernel");
    return PPL_OK;
}

// About 128 workgroups per product (each chunk a multiple of 32 rows): more
// chunks spread the reduction over more compute units but write, and make the
// Adam step read, one FP32 partial of the whole matrix per chunk.
void mlp_split_plan(int M, int N, int R, int *nchunks, int *chunk) {
    const int tiles = (M / kGemmTile) * (N / kGemmTile);
    int want = (128 + tiles - 1) / tiles;
    const int max_chunks = R / 32;
    if (want > max_chunks) want = max_chunks;
    if (want < 1) want = 1;
    int c = (R + want - 1) / want;
    c = (c + 31) / 32 * 32;
    *chunk = c;
    *nchunks = (R + c - 1) / c;
}

}  // namespace ppl
