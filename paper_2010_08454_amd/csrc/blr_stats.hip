// blr_stats.hip -- Bayesian linear regression importance sampling with the
// likelihood evaluated from sufficient statistics (Sec. 3.6.2 importance
// sampling; the model of PPL_MODEL_BLR).
//
// For Gaussian observations y_d ~ Normal(x_d . w, sigma) the data enter the
// log-likelihood only through A = X^T X, b = X^T y and c = y^T y:
//   sum_d (y_d - x_d . w)^2 = c - 2 w . b + w^T A w,
// so once the statistics are formed (O(D d^2), once per call) each particle
// costs O(d^2) instead of O(D d).  The statistics and the quadratic form are
// FP64: the three terms nearly cancel near the posterior (each is about D
// times the residual variance), which FP32 could not resolve.  The latents
// are the BLR model's (same Philox words, same FP32 draw), so only the
// evaluation of the likelihood differs.
//
// Kernels:
//   blr_stats_partial_kernel: workgroup g sums rows [g R, (g + 1) R) of
//     x x^T, x y and y^2 in FP64 (one thread per statistic);
//   blr_stats_finalize_kernel: sums the workgroup partials in a fixed order,
//     one wave per statistic;
//   blr_stats_is_kernel: per particle draw, FP64 quadratic form, log-weight,
//     and the normaliser's partial record (as blr_is_kernel).
#include "blr.h"
#include "device.h"
#include "host.h"
#include "kernels.h"
#include "timing.h"

namespace ppl {

constexpr int kStatsThreads = 256;
constexpr int kStatsRows = 64;             // rows per workgroup of the statistics pass
constexpr int kSsThreads = 256;
constexpr int kSsWaves = kSsThreads / 64;
constexpr int kSsP = 4;                    // particles per thread

// Statistic e of a DIM-column problem: e < DIM^2 -> A[e / DIM][e % DIM];
// e < DIM^2 + DIM -> b[e - DIM^2]; e == DIM^2 + DIM -> c.
constexpr int ss_count(int dim) { return dim * dim + dim + 1; }

template <int DIM>
__global__ __launch_bounds__(kStatsThreads) void blr_stats_partial_kernel(const float *__restrict__ X,
                                                                        const float *__restrict__ Y, int D,
                                                                        double *__restrict__ part) {
    __shared__ float xs[kStatsRows][DIM + 1];
    __shared__ float ys[kStatsRows];
    const int r0 = blockIdx.x * kStatsRows;
    const int nr = min(kStatsRows, D - r0);
    for (int e = threadIdx.x; e < nr * DIM; e += kStatsThreads) xs[e / DIM][e % DIM] = X[(size_t)r0 * DIM + e];
    for (int r = threadIdx.x; r < nr; r += kStatsThreads) ys[r] = Y[r0 + r];
    __syncthreads();
    constexpr int NS = ss_count(DIM);
    for (int e = threadIdx.x; e < NS; e += kStatsThreads) {
        double s = 0.0;
        if (e < DIM * DIM) {
            const int i = e / DIM, j = e % DIM;
            for (int r = 0; r < nr; ++r) s = fma((double)xs[r][i], (double)xs[r][j], s);
        } else if (e < DIM * DIM + DIM) {
            const int i = e - DIM * DIM;
            for (int r = 0; r < nr; ++r) s = fma((double)xs[r][i], (double)ys[r], s);
        } else {
            for (int r = 0; r < nr; ++r) s = fma((double)ys[r], (double)ys[r], s);
        }
        part[(size_t)blockIdx.x * NS + e] = s;
    }
}

// One wave per statistic: lane l sums the partials of groups l, l + 64, ...
// in order, then a fixed DPP reduction adds the lanes (a dependent chain of
// one load per group would leave this launch latency-bound).
template <int DIM>
__global__ __launch_bounds__(kStatsThreads) void blr_stats_finalize_kernel(const double *__restrict__ part, int groups,
                                                                         double *__restrict__ stats) {
    constexpr int NS = ss_count(DIM);
    const int e = blockIdx.x * (kStatsThreads / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (e >= NS) return;                     // whole waves leave together
    double s = 0.0;
    for (int g = lane; g < groups; g += 64) s += part[(size_t)g * NS + e];
    s = wave_sum_dpp(s);
    if (lane == 0) stats[e] = s;
}

template <int P, int DIM, bool PROP>
__global__ __launch_bounds__(kSsThreads) void blr_stats_is_kernel(const double *__restrict__ stats, int D, int64_t N,
                                                                Key key, float prior_sd, double noise_sd,
                                                                const float *__restrict__ qp,
                                                                double *__restrict__ lw_out,
                                                                float *__restrict__ lat_out,
                                                                double *__restrict__ part) {
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * (kSsThreads * P);
    float w[P][DIM];
    double extra[P];
    blr_draw<P, DIM, PROP, kSsThreads>(base, tid, key, prior_sd, qp, w, extra);
    const double *A = stats, *b = stats + DIM * DIM;
    const double c = stats[DIM * DIM + DIM];
    const double var = noise_sd * noise_sd;
    const double cterm = (double)D * (-0.5 * log(2.0 * M_PI * var));
    double lw[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        // residual sum of squares c - 2 w.b + w^T A w, the quadratic form row by row
        double q = c;
#pragma unroll
        for (int r = 0; r < DIM; ++r) {
            double v = -2.0 * b[r];
#pragma unroll
            for (int k = 0; k < DIM; ++k) v = fma(A[r * DIM + k], (double)w[p][k], v);
            q = fma((double)w[p][r], v, q);
        }
        lw[p] = cterm - q / (2.0 * var) + extra[p];
    }
    blr_finish<P, DIM, kSsThreads, kSsWaves>(base, tid, N, w, lw, lw_out, lat_out, part);
}

// ---------------------------------------------------------------- host --
size_t blr_stats_ws_bytes(int dim, int64_t N, int64_t D) {
    const int64_t groups = D > 0 ? (D + kStatsRows - 1) / kStatsRows : 0;
    const int64_t blocks = (N + (int64_t)kSsThreads * kSsP - 1) / ((int64_t)kSsThreads * kSsP);
    const size_t stats = align_up((size_t)ss_count(dim) * sizeof(double), 256);
    const size_t sparts = align_up((size_t)groups * ss_count(dim) * sizeof(double), 256);
    return stats + sparts + (size_t)blocks * (4 + dim) * sizeof(double) + merge_scratch_bytes(dim);
}

template <int DIM>
static int launch_blr_stats(const IsArgs &a, hipStream_t st) {
    constexpr int P = kSsP;
    const int64_t groups = a.D > 0 ? (a.D + kStatsRows - 1) / kStatsRows : 0;
    const int64_t blocks = (a.N + (int64_t)kSsThreads * P - 1) / ((int64_t)kSsThreads * P);
    if (int rc = check_grid("blr_stats_is_kernel", blocks, kSsThreads)) return rc;
    double *stats = a.part;
    double *sparts = stats + align_up((size_t)ss_count(DIM) * sizeof(double), 256) / sizeof(double);
    double *part = sparts + align_up((size_t)groups * ss_count(DIM) * sizeof(double), 256) / sizeof(double);
    if (groups > 0) {
        hipLaunchKernelGGL(blr_stats_partial_kernel<DIM>, dim3((unsigned)groups), dim3(kStatsThreads), 0, st,
                           (const float *)a.x, (const float *)a.y, (int)a.D, sparts);
        PPL_LAUNCH_CHECK("blr_stats_partial_kernel");
    }
    constexpr int kWavesPerBlock = kStatsThreads / 64;
    hipLaunchKernelGGL(blr_stats_finalize_kernel<DIM>, dim3((ss_count(DIM) + kWavesPerBlock - 1) / kWavesPerBlock),
                       dim3(kStatsThreads), 0, st, sparts, (int)groups, stats);
    PPL_LAUNCH_CHECK("blr_stats_finalize_kernel");
    {
        KernelTimer timer("blr_stats_is_kernel", st);
        if (a.q_params)
            hipLaunchKernelGGL((blr_stats_is_kernel<P, DIM, true>), dim3((unsigned)blocks), dim3(kSsThreads), 0, st,
                               stats, (int)a.D, a.N, make_key(a.seed), (float)a.hyper[0], a.hyper[1],
                               (const float *)a.q_params, (double *)a.lw_out, (float *)a.lat_out, part);
        else
            hipLaunchKernelGGL((blr_stats_is_kernel<P, DIM, false>), dim3((unsigned)blocks), dim3(kSsThreads), 0,
                               st, stats, (int)a.D, a.N, make_key(a.seed), (float)a.hyper[0], a.hyper[1], nullptr,
                               (double *)a.lw_out, (float *)a.lat_out, part);
        timer.stop();
    }
    PPL_LAUNCH_CHECK("blr_stats_is_kernel");
    int nrec = 0;
    const double *rec = merge_partials_first<DIM>(part, blocks, part + (size_t)blocks * (4 + DIM), &nrec, st);
    PPL_LAUNCH_CHECK("partial_merge_kernel");
    hipLaunchKernelGGL(weights_finalize_kernel<DIM>, dim3(1), dim3(kFinalizeThreads), 0, st, rec, nrec, a.N,
                       (int)PPL_MODEL_BLR, a.scalars, a.summaries);
    PPL_LAUNCH_CHECK("weights_finalize_kernel");
    return PPL_OK;
}

int run_importance_blr_stats(const IsArgs &a, hipStream_t st) {
    switch (a.dim) {
        case 4: return launch_blr_stats<4>(a, st);
        case 8: return launch_blr_stats<8>(a, st);
        case 12: return launch_blr_stats<12>(a, st);
        case 16: return launch_blr_stats<16>(a, st);
    }
    return fail(PPL_E_ARG, "BLR dim must be 4, 8, 12 or 16 (got %d)", a.dim);
}

}  // namespace ppl
