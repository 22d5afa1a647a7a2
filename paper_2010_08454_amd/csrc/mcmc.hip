// mcmc.hip -- lightweight Metropolis-Hastings (paper Sec. 3.6.3) on the GPU:
// many independent chains of the polynomial model, one chain per lane.
//
// A chain's trace holds the sites its execution reached: n and c_0..c_{n-1}.
// An iteration picks one site of the trace uniformly, resamples it from its
// prior and re-executes the model: when n changes, coefficients both
// executions reach keep their values, coefficients only the new execution
// reaches are drawn fresh from their prior, and those it no longer reaches
// are dropped.  With prior proposals every prior density cancels and
//     alpha = L(x') / L(x) * (n + 1) / (n' + 1)
// (likelihood ratio times the ratio of the traces' site counts).
//
// Words of iteration t of chain c (tag 8): block (c, 3t, 0) word 0 picks the
// site (uniform discrete over 0..n: 0 is n, j + 1 is c_j), word 1 the
// proposed n' (uniform discrete over n_lo..n_hi), word 2 the acceptance
// uniform v; blocks (c, 3t + 1, 0) and (c, 3t + 2, 0) give one
// double-precision Box-Muller pair each, z_0..z_3: a resampled c_j is sd z_0
// and fresh coefficients c_n, c_{n+1}, ... are sd z_1, sd z_2, sd z_3.  A
// chain starts from the importance sampler's prior draw of execution c.
// Accepted when log v < log alpha (FP64).
//
// Each lane keeps its chain's state and the post-burn-in sums in registers;
// the data points are the same for every lane and come through scalar loads.
// The sums fold into per-workgroup records in a fixed order, and one
// workgroup merges those.
#include "device.h"
#include "host.h"
#include "mcmc.h"
#include "poly.h"
#include "timing.h"

namespace ppl {

constexpr int kMcThreads = 256;
constexpr int kMcWaves = kMcThreads / 64;
constexpr int kMcNF = 30;                   // per-chain sums: 29 summary fields + accepted count
constexpr uint32_t kTagMcmc = 8;

// -1/2 sum_d (y_d - p(x_d))^2 in FP64, points in chunks of eight (one batch of
// scalar loads per chunk).
__device__ __forceinline__ double mc_loglik(const double pc[5], const double *__restrict__ X,
                                            const double *__restrict__ Y, int D) {
    double acc = 0.0;
    int d = 0;
    for (; d + 8 <= D; d += 8) {
        double xs[8], ys[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            xs[k] = X[d + k];
            ys[k] = Y[d + k];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += poly_sq_residual(pc, xs[k], ys[k]);
    }
    for (; d < D; ++d) acc += poly_sq_residual(pc, X[d], Y[d]);
    return -0.5 * acc;
}

__global__ __launch_bounds__(kMcThreads) void mcmc_poly_kernel(
    const double *__restrict__ X, const double *__restrict__ Y, int D, int64_t C, int64_t T, int64_t burn,
    Key key, double sd, int n_lo, int n_hi, double *__restrict__ state_out, int64_t *__restrict__ acc_out,
    int8_t *__restrict__ n_tr, double *__restrict__ la_tr, double *__restrict__ part) {
    __shared__ double lds[kMcWaves][kMcNF];
    const int64_t c = (int64_t)blockIdx.x * kMcThreads + threadIdx.x;
    const bool valid = c < C;
    int n;
    double pc[5];
    poly_prior_draw((uint32_t)c, key, sd, n_lo, n_hi, n, pc);
#pragma unroll
    for (int j = 0; j < 5; ++j) pc[j] = j < n ? pc[j] : 0.0;
    double ll = mc_loglik(pc, X, Y, D);
    double sums[kMcNF];
#pragma unroll
    for (int k = 0; k < kMcNF; ++k) sums[k] = 0.0;
    const uint32_t range = (uint32_t)(n_hi - n_lo + 1);
    // log(n + 1) for the trace-size ratio, n <= 5: the same values log() gives
    // per iteration, computed once
    double lsz[7];
#pragma unroll
    for (int k = 1; k <= 6; ++k) lsz[k] = log((double)k);
    lsz[0] = 0.0;
    auto log_size = [&](int k) {
        double r = lsz[1];
#pragma unroll
        for (int q = 2; q <= 6; ++q) r = k == q ? lsz[q] : r;
        return r;
    };

    for (int64_t t = 0; t < T; ++t) {
        const uint4 w = philox((uint32_t)c, (uint32_t)(3 * t), 0, kTagMcmc, key);
        const int site = uniform_discrete(w.x, 0, (uint32_t)(n + 1));
        int n2 = n;
        double c2[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) c2[j] = pc[j];
        double z[4];
        {   // z_0 (a resampled coefficient) and z_1 (the first fresh one)
            const uint4 b1 = philox((uint32_t)c, (uint32_t)(3 * t + 1), 0, kTagMcmc, key);
            box_muller(unit_f64(b1.x, b1.y), unit_f64(b1.z, b1.w), z[0], z[1]);
        }
        if (site == 0) {
            n2 = uniform_discrete(w.y, n_lo, range);
            if (n2 > n + 1) {
                const uint4 b2 = philox((uint32_t)c, (uint32_t)(3 * t + 2), 0, kTagMcmc, key);
                box_muller(unit_f64(b2.x, b2.y), unit_f64(b2.z, b2.w), z[2], z[3]);
            } else {
                z[2] = z[3] = 0.0;
            }
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                // slot j: kept (j < n and j < n2), fresh (n <= j < n2, normal z_{1 + j - n}), dropped (j >= n2)
                const int f = j - n;                 // index of the fresh normal minus one
                const double fresh = sd * (f == 0 ? z[1] : (f == 1 ? z[2] : z[3]));
                c2[j] = j >= n2 ? 0.0 : (j < n ? pc[j] : fresh);
            }
        } else {
#pragma unroll
            for (int j = 0; j < 5; ++j) c2[j] = (j == site - 1) ? sd * z[0] : pc[j];
        }
        const double ll2 = mc_loglik(c2, X, Y, D);
        const double la = (ll2 - ll) + (log_size(n + 1) - log_size(n2 + 1));
        const bool acc = log((double)unit_f32(w.z)) < la;
        if (valid && la_tr) la_tr[t * C + c] = la;
        if (acc) {
            n = n2;
#pragma unroll
            for (int j = 0; j < 5; ++j) pc[j] = c2[j];
            ll = ll2;
            sums[29] += 1.0;
        }
        if (valid && n_tr) n_tr[t * C + c] = (int8_t)n;
        if (t >= burn) {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const bool here = n == m + 2;
                sums[m] += here ? 1.0 : 0.0;
#pragma unroll
                for (int j = 0; j < 5; ++j) sums[4 + 5 * m + j] += here ? pc[j] : 0.0;
            }
#pragma unroll
            for (int j = 0; j < 5; ++j) sums[24 + j] += pc[j];
        }
    }
    if (valid) {
        if (state_out) {
            state_out[c] = (double)n;
#pragma unroll
            for (int j = 0; j < 5; ++j) state_out[(size_t)(1 + j) * C + c] = pc[j];
        }
        if (acc_out) acc_out[c] = (int64_t)sums[29];
    } else {
#pragma unroll
        for (int k = 0; k < kMcNF; ++k) sums[k] = 0.0;
    }
    // workgroup record: waves in order
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kMcNF; ++k) {
        const double v = wave_sum_dpp(sums[k]);
        if ((threadIdx.x & 63) == 0) lds[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < kMcNF) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < kMcWaves; ++w) v += lds[w][threadIdx.x];
        part[(size_t)blockIdx.x * kMcNF + threadIdx.x] = v;
    }
}

// One workgroup: the records summed in block order, then the summaries
// (as importance sampling lays them out) and {acceptance rate, kept samples,
// chains, status}.
__global__ __launch_bounds__(kMcThreads) void mcmc_finalize_kernel(const double *__restrict__ part, int64_t nblocks,
                                                                   int64_t C, int64_t T, double *__restrict__ scalars,
                                                                   double *__restrict__ summaries) {
    __shared__ double tot[kMcNF];
    if (threadIdx.x < kMcNF) {
        double v = 0.0;
        for (int64_t b = 0; b < nblocks; ++b) v += part[(size_t)b * kMcNF + threadIdx.x];
        tot[threadIdx.x] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double all = tot[0] + tot[1] + tot[2] + tot[3];
    if (summaries) {
        for (int m = 0; m < 4; ++m) {
            summaries[m] = all > 0 ? tot[m] / all : 0.0;
            for (int j = 0; j < 5; ++j) summaries[4 + 5 * m + j] = tot[m] > 0 ? tot[4 + 5 * m + j] / tot[m] : 0.0;
        }
        for (int j = 0; j < 5; ++j) summaries[24 + j] = all > 0 ? tot[24 + j] / all : 0.0;
    }
    scalars[0] = T > 0 ? tot[29] / ((double)C * (double)T) : 0.0;
    scalars[1] = all;
    scalars[2] = (double)C;
    scalars[3] = 0.0;
}

size_t mcmc_ws_bytes(int64_t chains) {
    const int64_t blocks = (chains + kMcThreads - 1) / kMcThreads;
    return 256 + align_up((size_t)blocks * kMcNF * sizeof(double), 256);
}

int run_mcmc_poly(const McmcArgs &a, hipStream_t st) {
    const int64_t blocks = (a.C + kMcThreads - 1) / kMcThreads;
    if (int rc = check_grid("mcmc_poly_kernel", blocks, kMcThreads)) return rc;
    double *part = (double *)((char *)a.ws + 256);
    {
        KernelTimer timer("mcmc_poly_kernel", st);
        hipLaunchKernelGGL(mcmc_poly_kernel, dim3((unsigned)blocks), dim3(kMcThreads), 0, st, a.x, a.y, (int)a.D, a.C,
                           a.T, a.burn, make_key(a.seed), a.hyper[0], (int)a.hyper[1], (int)a.hyper[2], a.state_out,
                           a.acc_out, a.n_trace, a.la_trace, part);
        timer.stop();
    }
    PPL_LAUNCH_CHECK("mcmc_poly_kernel");
    hipLaunchKernelGGL(mcmc_finalize_kernel, dim3(1), dim3(kMcThreads), 0, st, part, blocks, a.C, a.T, a.scalars,
                       a.summaries);
    PPL_LAUNCH_CHECK("mcmc_finalize_kernel");
    return PPL_OK;
}

}  // namespace ppl
