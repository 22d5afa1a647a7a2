// simulate.hip -- training pairs drawn from the model's own prior, and the 64
// data summaries the proposal network reads.  One 256-thread workgroup per
// dataset: the threads stride over the data points, FP64 moment sums are
// combined by wave butterflies and a fixed-order sum of the four wave totals,
// and the per-dataset finishing work (least-squares fits, order statistics)
// runs on the first wave.
//
// Training pair of step t, pair i (Philox tag 4, counter (i, block, t, 4)):
//   POLY: block 0 word 0 -> degree n (uniform discrete); blocks 1, 2 -> eight
//         normals (two single-precision-stream Box-Muller pairs each), c_j =
//         sd z_j; block 8 + e -> points 2e, 2e + 1: x = 2u - 1 from words 0, 1
//         and the observation noise from a Box-Muller pair on words 2, 3;
//         y = poly_c(x) + noise_sd * eps.
//   GMM:  blocks 0, 1 -> Exp(1) draws E_k = -ln u_k, pi = E / sum E (a
//         Dirichlet(1) draw); blocks 2, 3 -> mu_k = mu_sd z_k; block 8 + e ->
//         the components of points 2e, 2e + 1 (inverse CDF on pi, words 0, 1)
//         and their noise (words 2, 3); latents returned in the ordered
//         unconstrained space (mu_(1), log gaps, log pi_(k) - log pi_(K)).
// Every step is in FP64 on uniforms that are exact in both precisions.
#include "adam.h"
#include "device.h"
#include "host.h"
#include "proposal.h"

namespace ppl {

constexpr uint32_t kTagTrain = 4;
constexpr int kSumThreads = 256;     // one dataset per workgroup
constexpr int kSumWaves = kSumThreads / 64;

__device__ __forceinline__ double u01(uint32_t w) { return (double)unit_f32(w); }

// Index of the first cumulative probability above u (K - 1 if none).
__device__ __forceinline__ int categorical8(double u, const double (&p)[8], int K) {
    double c = 0.0;
    int r = K - 1;
    bool found = false;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (k < K && !found) {
            c += p[k];
            if (u < c) {
                r = k;
                found = true;
            }
        }
    }
    return r;
}

__device__ __forceinline__ double pick8(const double (&v)[8], int k) {
    double r = v[0];
#pragma unroll
    for (int j = 1; j < 8; ++j) r = (k == j) ? v[j] : r;
    return r;
}

// ------------------------------------------------------------- POLY --
// Moment accumulators: [0..7] sum x^j y, [8..22] sum x^k (k = 0..14), [23] sum y^2.
constexpr int kPolyAcc = 24;

__device__ __forceinline__ void poly_acc_point(double (&a)[kPolyAcc], double x, double y) {
#pragma clang fp contract(off)
    double p = 1.0;
#pragma unroll
    for (int k = 0; k <= 14; ++k) {
        if (k < 8) a[k] += p * y;
        a[8 + k] += p;
        p *= x;
    }
    a[23] += y * y;
}

// Least-squares fit with n coefficients from the normalised moments
// (normal equations G beta = m, G_ij = mean x^(i+j), m_i = mean x^i y) by a
// Cholesky factorisation and two triangular solves.
// The diagonal's reciprocals are formed once (one division per column, then
// products): the solve's chain of dependent FP64 divisions is its latency.
__device__ void poly_ls(int n, const double *gx, const double *mxy, double (&beta)[5]) {
#pragma clang fp contract(off)
    double L[5][5], z[5], rd[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            if (i < n) {
                double s = gx[i + j];
#pragma unroll
                for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
                if (i == j) {
                    L[i][i] = sqrt(s > 1e-300 ? s : 1e-300);
                    rd[i] = 1.0 / L[i][i];
                } else {
                    L[i][j] = s * rd[j];
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        if (i < n) {
            double s = mxy[i];
#pragma unroll
            for (int k = 0; k < i; ++k) s -= L[i][k] * z[k];
            z[i] = s * rd[i];
        }
    }
#pragma unroll
    for (int i = 4; i >= 0; --i) {
        beta[i] = 0.0;
        if (i < n) {
            double s = z[i];
#pragma unroll
            for (int k = i + 1; k < 5; ++k)
                if (k < n) s -= L[k][i] * beta[k];
            beta[i] = s * rd[i];
        }
    }
}

// Sum of one double per thread over the workgroup, returned to every thread:
// wave butterflies, then the wave totals in a fixed order.  red holds
// kSumWaves doubles.
__device__ __forceinline__ double block_sum(double v, double *red) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// Reduce the thread accumulators and write the 64 POLY summaries to s[]:
//   [0..7] mean x^j y / 10; [8..21] mean x^k, k = 1..14; [22] mean y^2 / 100;
//   [23..36] least-squares coefficients for n = 2..5 / 10;
//   [37..40] log(1 + (RSS_n - RSS_5) / 2) / 10 (RSS_n the residual sum of
//   squares of the n-coefficient fit: the log-likelihood gap to the largest
//   fit, independent of the absolute noise level); [41] log D / 10; rest 0.
__device__ void poly_finish(double (&a)[kPolyAcc], int64_t D, double (*wtot)[kPolyAcc], double *tot, double *s) {
#pragma clang fp contract(off)
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
#pragma unroll
    for (int k = 0; k < kPolyAcc; ++k) a[k] = wave_sum_dpp(a[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < kPolyAcc; ++k) wtot[wv][k] = a[k];
    }
    __syncthreads();
    if (tid < kPolyAcc)
        tot[tid] = D > 0 ? ((wtot[0][tid] + wtot[1][tid]) + (wtot[2][tid] + wtot[3][tid])) / (double)D : 0.0;
    __syncthreads();
    if (wv == 0) {
        const double *mxy = tot, *gx = tot + 8;
        double v = 0.0;
        if (D > 0) {
            if (lane < 8) v = mxy[lane] / 10.0;
            else if (lane < 22) v = gx[lane - 7];
            else if (lane == 22) v = tot[23] / 100.0;
            else if (lane == 41) v = log((double)D) / 10.0;
        }
        if (lane < 23 || lane >= 41) s[lane] = v;
        double rss = 0.0;
        if (lane < 4) {
            const int n = 2 + lane;
            double beta[5];
            poly_ls(n, gx, mxy, beta);
            double fit = 0.0;
            const int o = 23 + (n - 2) * (n + 1) / 2;
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                if (j < n) {
                    s[o + j] = D > 0 ? beta[j] / 10.0 : 0.0;
                    fit += beta[j] * mxy[j];
                }
            }
            rss = tot[23] - fit;
            if (rss < 0.0) rss = 0.0;
        }
        const double rss5 = __shfl(rss, 3, 64);
        if (lane < 4) {
            double gap = (double)D * (rss - rss5) / 2.0;
            if (gap < 0.0) gap = 0.0;
            s[37 + lane] = D > 0 ? log1p(gap) / 10.0 : 0.0;
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------- GMM --
// Summaries from the data in LDS ys[D] (FP64 simulated points, or the FP32
// observed values, compared and summed in FP64):
//   [0..15] order statistics y_(floor((q + 1/2) D / 16)) / 10;
//   [16..47] counts on the unit bins of [-16, 16) (ends clamped) / D;
//   [48] mean / 10, [49] sd / 10, [50] skewness, [51] excess kurtosis / 10,
//   [52] log D / 10; rest 0.  hist holds the workgroup's 32 bin counts,
//   already filled; sum_y is the thread's sum of its points.
template <typename T>
__device__ void gmm_finish(const T *ys, int64_t D, const int *hist, double sum_y, double *red, double *s) {
#pragma clang fp contract(off)
    const int tid = threadIdx.x;
    const double m1 = D > 0 ? block_sum(sum_y, red) / (double)D : 0.0;
    double c2 = 0.0, c3 = 0.0, c4 = 0.0;
    for (int64_t d = tid; d < D; d += kSumThreads) {
        const double y = (double)ys[d];
        int64_t r = 0;
        for (int64_t e = 0; e < D; ++e) {
            const double ye = (double)ys[e];
            r += (ye < y) || (ye == y && e < d);
        }
#pragma unroll
        for (int q = 0; q < 16; ++q)
            if (r == (int64_t)floor((q + 0.5) * (double)D / 16.0)) s[q] = y / 10.0;
        const double dv = y - m1;
        c2 += dv * dv;
        c3 += dv * dv * dv;
        c4 += dv * dv * dv * dv;
    }
    c2 = block_sum(c2, red);
    c3 = block_sum(c3, red);
    c4 = block_sum(c4, red);
    if (D <= 0 && tid < 16) s[tid] = 0.0;
    if (tid < 32) s[16 + tid] = D > 0 ? (double)hist[tid] / (double)D : 0.0;
    if (tid >= 53 && tid < kSummaryDim) s[tid] = 0.0;
    if (tid == 0) {
        double v2 = 0.0, v3 = 0.0, v4 = 0.0;
        if (D > 0) {
            v2 = c2 / (double)D;
            v3 = c3 / (double)D;
            v4 = c4 / (double)D;
        }
        const double sd = sqrt(v2);
        s[48] = m1 / 10.0;
        s[49] = sd / 10.0;
        s[50] = v2 > 0 ? v3 / (v2 * sd) : 0.0;
        s[51] = v2 > 0 ? (v4 / (v2 * v2) - 3.0) / 10.0 : 0.0;
        s[52] = D > 0 ? log((double)D) / 10.0 : 0.0;
    }
    __syncthreads();
}

__device__ __forceinline__ void gmm_bin(int *hist, double y) {
    int b = (int)floor(y + 16.0);
    b = b < 0 ? 0 : (b > 31 ? 31 : b);
    atomicAdd(&hist[b], 1);
}

// -------------------------------------------------- training simulation --
// Dataset b of the batch (one workgroup).
template <int MODEL>
__device__ __forceinline__ void simulate_block(const SimSpec &sp, int B, Key key, const int64_t *__restrict__ step_ptr,
                                               uint16_t *__restrict__ x_row, uint16_t *__restrict__ x_col,
                                               double *__restrict__ theta, double *__restrict__ s64, int b) {
#pragma clang fp contract(off)
    extern __shared__ double ys[];
    __shared__ double wtot[kSumWaves][kPolyAcc];
    __shared__ double tot[kPolyAcc];
    __shared__ double s[kSummaryDim];
    __shared__ double red[kSumWaves];
    __shared__ int hist[32];
    const int tid = threadIdx.x;
    const uint32_t step = (uint32_t)*step_ptr;
    const uint32_t pair = (uint32_t)b;
    const int64_t D = sp.D;

    if constexpr (MODEL == PPL_MODEL_POLY) {
        const uint4 w0 = philox(pair, 0, step, kTagTrain, key);
        const int n = uniform_discrete(w0.x, (int)sp.hyper[1], (uint32_t)((int)sp.hyper[2] - (int)sp.hyper[1] + 1));
        // coefficient normals z_0..z_4: Box-Muller pairs 0..2 of blocks 1 and
        // 2 (pair q from words 2 (q % 2), 2 (q % 2) + 1 of block 1 + q / 2),
        // one pair per thread of the first three, shared through LDS
        __shared__ double s_z[6];
        if (tid < 3) {
            const uint4 w = philox(pair, 1 + (tid >> 1), step, kTagTrain, key);
            double za, zb;
            box_muller(u01((tid & 1) ? w.z : w.x), u01((tid & 1) ? w.w : w.y), za, zb);
            s_z[2 * tid] = za;
            s_z[2 * tid + 1] = zb;
        }
        __syncthreads();
        double c[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) c[j] = sp.hyper[0] * s_z[j];
        double a[kPolyAcc];
#pragma unroll
        for (int k = 0; k < kPolyAcc; ++k) a[k] = 0.0;
        for (int64_t e = tid; 2 * e < D; e += kSumThreads) {
            const uint4 w = philox(pair, (uint32_t)(8 + e), step, kTagTrain, key);
            double e0, e1;
            box_muller(u01(w.z), u01(w.w), e0, e1);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (2 * e + h < D) {
                    const double x = 2.0 * u01(h ? w.y : w.x) - 1.0;
                    double p = 0.0;
#pragma unroll
                    for (int j = 4; j >= 0; --j)
                        if (j < n) p = p * x + c[j];
                    const double y = p + sp.hyper[3] * (h ? e1 : e0);
                    poly_acc_point(a, x, y);
                }
            }
        }
        poly_finish(a, D, wtot, tot, s);
        if (tid < 6) theta[(size_t)b * kThetaStride + tid] = tid == 0 ? (double)n : (tid - 1 < n ? c[tid - 1] : 0.0);
    } else {
        const int K = sp.K;
        if (tid < 32) hist[tid] = 0;
        const uint4 wa = philox(pair, 0, step, kTagTrain, key), wb = philox(pair, 1, step, kTagTrain, key);
        const uint32_t ew[8] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y, wb.z, wb.w};
        double E[8], pi[8], mu[8], z[8], etot = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            E[k] = k < K ? -log(u01(ew[k])) : 0.0;
            if (k < K) etot += E[k];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) pi[k] = k < K ? E[k] / etot : 0.0;
        {
            const uint4 w2 = philox(pair, 2, step, kTagTrain, key), w3 = philox(pair, 3, step, kTagTrain, key);
            box_muller(u01(w2.x), u01(w2.y), z[0], z[1]);
            box_muller(u01(w2.z), u01(w2.w), z[2], z[3]);
            box_muller(u01(w3.x), u01(w3.y), z[4], z[5]);
            box_muller(u01(w3.z), u01(w3.w), z[6], z[7]);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) mu[k] = sp.hyper[0] * z[k];
        __syncthreads();
        double sum_y = 0.0;
        for (int64_t e = tid; 2 * e < D; e += kSumThreads) {
            const uint4 w = philox(pair, (uint32_t)(8 + e), step, kTagTrain, key);
            double e0, e1;
            box_muller(u01(w.z), u01(w.w), e0, e1);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (2 * e + h < D) {
                    const int k = categorical8(u01(h ? w.y : w.x), pi, K);
                    const double y = pick8(mu, k) + sp.hyper[1] * (h ? e1 : e0);
                    ys[2 * e + h] = y;
                    sum_y += y;
                    gmm_bin(hist, y);
                }
            }
        }
        __syncthreads();
        gmm_finish(ys, D, hist, sum_y, red, s);
        if (tid == 0) {
            // order the components by mean (insertion sort; ties keep index order)
            int ord[8] = {0, 1, 2, 3, 4, 5, 6, 7};
            for (int q = 1; q < K; ++q)
                for (int r = q; r > 0 && mu[ord[r]] < mu[ord[r - 1]]; --r) {
                    const int t = ord[r];
                    ord[r] = ord[r - 1];
                    ord[r - 1] = t;
                }
            double *u = theta + (size_t)b * kThetaStride;
            u[0] = mu[ord[0]];
            for (int q = 1; q < K; ++q) u[q] = log(mu[ord[q]] - mu[ord[q - 1]]);
            const double lk = log(pi[ord[K - 1]]);
            for (int q = 0; q < K - 1; ++q) u[K + q] = log(pi[ord[q]]) - lk;
        }
    }
    if (tid < kSummaryDim) {
        const double v = s[tid];
        const uint16_t h = f32_to_bf16((float)v);
        x_row[(size_t)b * kSummaryDim + tid] = h;
        x_col[(size_t)tid * B + b] = h;
        if (s64) s64[(size_t)b * kSummaryDim + tid] = v;
    }
}

template <int MODEL>
__global__ __launch_bounds__(kSumThreads) void simulate_kernel(SimSpec sp, int B, Key key,
                                                               const int64_t *__restrict__ step_ptr,
                                                               uint16_t *__restrict__ x_row,
                                                               uint16_t *__restrict__ x_col,
                                                               double *__restrict__ theta,
                                                               double *__restrict__ s64) {
    simulate_block<MODEL>(sp, B, key, step_ptr, x_row, x_col, theta, s64, (int)blockIdx.x);
}

// The simulation of the next step's batch (workgroups 0 .. B - 1, first, as
// the longer ones) and the Adam update of this step (the rest) in one launch:
// the simulation reads only the step count, which the step's bookkeeping has
// already advanced, and its buffers were last read by the launches before.
template <int MODEL>
__global__ __launch_bounds__(kSumThreads) void adam_simulate_kernel(MlpView w, SplitParts spl,
                                                                    const float *__restrict__ bgrad, AdamSpec ad,
                                                                    const float *__restrict__ coef, SimSpec sp, int B,
                                                                    Key key,
                                                                    const int64_t *__restrict__ step_ptr,
                                                                    uint16_t *__restrict__ x_row,
                                                                    uint16_t *__restrict__ x_col,
                                                                    double *__restrict__ theta) {
    if ((int)blockIdx.x >= B) {
        adam_unit(w, spl, bgrad, ad, coef, nullptr, (int64_t)((int)blockIdx.x - B) * kSumThreads + threadIdx.x);
        return;
    }
    simulate_block<MODEL>(sp, B, key, step_ptr, x_row, x_col, theta, nullptr, (int)blockIdx.x);
}

// ----------------------------------------------------- observed summary --
template <int MODEL>
__global__ __launch_bounds__(kSumThreads) void observed_summary_kernel(const void *__restrict__ xv,
                                                                       const void *__restrict__ yv, int64_t D,
                                                                       uint16_t *__restrict__ x_row,
                                                                       double *__restrict__ s64) {
#pragma clang fp contract(off)
    extern __shared__ float ysf[];
    __shared__ double wtot[kSumWaves][kPolyAcc];
    __shared__ double tot[kPolyAcc];
    __shared__ double s[kSummaryDim];
    __shared__ double red[kSumWaves];
    __shared__ int hist[32];
    const int tid = threadIdx.x;
    if constexpr (MODEL == PPL_MODEL_POLY) {
        const double *X = (const double *)xv, *Y = (const double *)yv;
        double a[kPolyAcc];
#pragma unroll
        for (int k = 0; k < kPolyAcc; ++k) a[k] = 0.0;
        for (int64_t d = tid; d < D; d += kSumThreads) poly_acc_point(a, X[d], Y[d]);
        poly_finish(a, D, wtot, tot, s);
    } else {
        const float *Y = (const float *)yv;
        if (tid < 32) hist[tid] = 0;
        __syncthreads();
        double sum_y = 0.0;
        for (int64_t d = tid; d < D; d += kSumThreads) {
            const float yf = Y[d];
            ysf[d] = yf;
            sum_y += (double)yf;
            gmm_bin(hist, (double)yf);
        }
        __syncthreads();
        gmm_finish(ysf, D, hist, sum_y, red, s);
    }
    // row 0 holds the summaries, rows 1..63 of the 64-row batch are cleared
    for (int e = tid; e < 64 * kSummaryDim; e += kSumThreads)
        x_row[e] = e < kSummaryDim ? f32_to_bf16((float)s[e]) : (uint16_t)0;
    if (s64 && tid < kSummaryDim) s64[tid] = s[tid];
}

// ------------------------------------------------------------------ host --
int launch_simulate(const SimSpec &sp, int B, uint64_t seed, const int64_t *step, uint16_t *x_row, uint16_t *x_col,
                    double *theta, double *s64, hipStream_t st) {
    if (B <= 0) return fail(PPL_E_ARG, "simulation batch %d is not positive", B);
    const dim3 grid((unsigned)B), block(kSumThreads);
    if (sp.model == PPL_MODEL_POLY) {
        hipLaunchKernelGGL(simulate_kernel<PPL_MODEL_POLY>, grid, block, 0, st, sp, B, make_key(seed), step, x_row,
                           x_col, theta, s64);
        PPL_LAUNCH_CHECK("simulate_kernel<POLY>");
    } else {
        if (sp.D > kGmmTrainMaxD) return fail(PPL_E_ARG, "mixture training datasets hold at most %d points", kGmmTrainMaxD);
        const size_t lds = (size_t)(sp.D > 0 ? sp.D : 1) * sizeof(double);
        hipLaunchKernelGGL(simulate_kernel<PPL_MODEL_GMM>, grid, block, lds, st, sp, B, make_key(seed), step, x_row,
                           x_col, theta, s64);
        PPL_LAUNCH_CHECK("simulate_kernel<GMM>");
    }
    return PPL_OK;
}

int launch_update_simulate(const MlpView &w, const TrainBufs &b, const AdamSpec &ad, const SimSpec &sp, int B,
                           uint64_t seed, const int64_t *step, hipStream_t st) {
    if (B <= 0) return fail(PPL_E_ARG, "simulation batch %d is not positive", B);
    const int adam_blocks = (int)((MlpParams::count() + kSumThreads - 1) / kSumThreads);
    const dim3 grid((unsigned)(adam_blocks + B)), block(kSumThreads);
    const SplitParts spl = split_parts(b);
    if (sp.model == PPL_MODEL_POLY) {
        hipLaunchKernelGGL(adam_simulate_kernel<PPL_MODEL_POLY>, grid, block, 0, st, w, spl, (const float *)b.bgrad, ad,
                           (const float *)b.coef, sp, B, make_key(seed), step, b.x_row, b.x_col, b.theta);
    } else {
        if (sp.D > kGmmTrainMaxD) return fail(PPL_E_ARG, "mixture training datasets hold at most %d points", kGmmTrainMaxD);
        const size_t lds = (size_t)(sp.D > 0 ? sp.D : 1) * sizeof(double);
        hipLaunchKernelGGL(adam_simulate_kernel<PPL_MODEL_GMM>, grid, block, lds, st, w, spl, (const float *)b.bgrad, ad,
                           (const float *)b.coef, sp, B, make_key(seed), step, b.x_row, b.x_col, b.theta);
    }
    PPL_LAUNCH_CHECK("adam_simulate_kernel");
    return PPL_OK;
}

int launch_observed_summary(int model, const void *x, const void *y, int64_t D, uint16_t *x_row, double *s64,
                            hipStream_t st) {
    if (model == PPL_MODEL_POLY) {
        hipLaunchKernelGGL(observed_summary_kernel<PPL_MODEL_POLY>, dim3(1), dim3(kSumThreads), 0, st, x, y, D, x_row,
                           s64);
    } else {
        if (D > kGmmSummaryMaxD) return fail(PPL_E_ARG, "mixture summaries take at most %d points", kGmmSummaryMaxD);
        const size_t lds = (size_t)(D > 0 ? D : 1) * sizeof(float);
        hipLaunchKernelGGL(observed_summary_kernel<PPL_MODEL_GMM>, dim3(1), dim3(kSumThreads), lds, st, x, y, D,
                           x_row, s64);
    }
    PPL_LAUNCH_CHECK("observed_summary_kernel");
    return PPL_OK;
}

}  // namespace ppl
