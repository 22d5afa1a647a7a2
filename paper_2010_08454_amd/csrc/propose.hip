// propose.hip -- importance sampling (paper Sec. 3.6.2) with a diagonal
// Gaussian-mixture proposal q -- the decoded output of the proposal network --
// in place of the prior, and prior importance sampling of the mixture model.
// Each particle draws its latents from q (Philox tag 1), and its log-weight is
// log p(latents) + log L(latents) - log q(latents); the block partials and the
// finalize step are those of the prior importance sampler.  FP64 throughout,
// except the mixture model's likelihood: FP32 per datum (hardware exp and
// log), summed in FP32 within 16-datum blocks and in FP64 across them.
//
// Proposal parameter blocks (FP64, device):
//   POLY (degrees 2..5): lognl[4], logmix[8], mean[4][8][5], lsd[4][8][5];
//        block 0 word 0 picks the degree, word 1 the component (inverse CDF),
//        blocks 1, 2 give eight normals, c_j = mean + exp(lsd) z_j for j < n.
//   GMM (K components, d = 2K - 1): logmix[8], mean[8][d], lsd[8][d]; block 0
//        word 0 picks the component, blocks 1..4 give sixteen normals, u_k =
//        mean + exp(lsd) z_k over the ordered unconstrained latents
//        u = (mu_(1), log(mu_(k) - mu_(k-1)), log pi_(k) - log pi_(K)); its
//        prior density carries the Dirichlet(1) normaliser (K-1)!, the K!
//        orderings (p and L are invariant under relabelling) and the
//        Jacobians of the gap and softmax maps.
#include "device.h"
#include "host.h"
#include "kernels.h"
#include "proposal.h"
#include "timing.h"

namespace ppl {

constexpr int kPropThreads = 256;
constexpr int kPolyNFp = 29;
constexpr int kGmmNF = 8;
constexpr double kHalfLog2PiD = 0.91893853320467274178;

__device__ __forceinline__ double u01d(uint32_t w) { return (double)unit_f32(w); }

__device__ __forceinline__ void normals4_d(uint4 w, double *z) {
    box_muller(u01d(w.x), u01d(w.y), z[0], z[1]);
    box_muller(u01d(w.z), u01d(w.w), z[2], z[3]);
}

// log Normal(v; m, exp(lsd)) given isd = exp(-lsd).
__device__ __forceinline__ double log_normal(double v, double m, double lsd, double isd) {
    const double r = (v - m) * isd;
    return -0.5 * r * r - lsd - kHalfLog2PiD;
}

// exp(lsd) and exp(-lsd) of the proposal's ns log-scales, computed once per
// workgroup into LDS (every particle of the workgroup uses the same table).
// Every thread of the workgroup must call it.
__device__ __forceinline__ void stage_scales(const double *__restrict__ lsdv, int ns, double *sdv, double *isdv) {
    for (int t = threadIdx.x; t < ns; t += kPropThreads) {
        sdv[t] = exp(lsdv[t]);
        isdv[t] = exp(-lsdv[t]);
    }
    __syncthreads();
}

template <int KMAX>
__device__ __forceinline__ int categorical_exp(double u, const double *__restrict__ logp, int K) {
    double c = 0.0;
    int r = K - 1;
    bool found = false;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        if (k < K && !found) {
            c += exp(logp[k]);
            if (u < c) {
                r = k;
                found = true;
            }
        }
    }
    return r;
}

// -------------------------------------------------------------- POLY --
__global__ __launch_bounds__(kPropThreads) void poly_mix_is_kernel(
    const double *__restrict__ X, const double *__restrict__ Y, int D, int64_t N, Key key, double sd,
    const double *__restrict__ q, double *__restrict__ lw_out, double *__restrict__ lat_out, double *__restrict__ part) {
    const int64_t i = (int64_t)blockIdx.x * kPropThreads + threadIdx.x;
    const bool live = i < N;
    const uint32_t ii = (uint32_t)i;
    const double *lnl = q, *lmix = q + 4, *mean = q + 12, *lsdv = q + 172;
    __shared__ double sdv[160], isdv[160];
    stage_scales(lsdv, 160, sdv, isdv);
    const uint4 w0 = philox(ii, 0, 0, kTagProposal, key);
    const int n = 2 + categorical_exp<4>(u01d(w0.x), lnl, 4);
    const int comp = categorical_exp<8>(u01d(w0.y), lmix, 8);
    double z[8];
    normals4_d(philox(ii, 1, 0, kTagProposal, key), z);
    normals4_d(philox(ii, 2, 0, kTagProposal, key), z + 4);
    double c[5];
    double lp = -log(4.0);
    const double lsd0 = log(sd), isd0 = exp(-lsd0);
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const int o = ((n - 2) * 8 + comp) * 5 + j;
        c[j] = j < n ? mean[o] + sdv[o] * z[j] : 0.0;
        if (j < n) lp += log_normal(c[j], 0.0, lsd0, isd0);
    }
    // log q(n, c): degree term plus the mixture over components.
    double t[8], tm = -INFINITY;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        double a = lmix[m];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const int o = ((n - 2) * 8 + m) * 5 + j;
            if (j < n) a += log_normal(c[j], mean[o], lsdv[o], isdv[o]);
        }
        t[m] = a;
        tm = fmax(tm, a);
    }
    double ts = 0.0;
#pragma unroll
    for (int m = 0; m < 8; ++m) ts += exp(t[m] - tm);
    const double lq = lnl[n - 2] + tm + log(ts);
    // Points in chunks of eight (one batch of scalar loads per chunk); the
    // sum order is unchanged.
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
        for (int k = 0; k < 8; ++k) {
            double v = c[4];
            v = fma(v, xs[k], c[3]);
            v = fma(v, xs[k], c[2]);
            v = fma(v, xs[k], c[1]);
            v = fma(v, xs[k], c[0]);
            const double r = ys[k] - v;
            acc = fma(r, r, acc);
        }
    }
    for (; d < D; ++d) {
        const double xv = X[d], yv = Y[d];
        double v = c[4];
        v = fma(v, xv, c[3]);
        v = fma(v, xv, c[2]);
        v = fma(v, xv, c[1]);
        v = fma(v, xv, c[0]);
        const double r = yv - v;
        acc = fma(r, r, acc);
    }
    const double lw = live ? lp - 0.5 * acc - lq : -INFINITY;
    if (live) {
        if (lw_out) lw_out[i] = lw;
        if (lat_out) {
            lat_out[i] = (double)n;
#pragma unroll
            for (int j = 0; j < 5; ++j) lat_out[(size_t)(1 + j) * N + i] = c[j];
        }
    }
    Partial<kPolyNFp> pp = partial_empty<kPolyNFp>();
    if (live && isnan(lw)) pp.nan = 1.0;
    pp.m = lw;
    if (lw > -INFINITY) {
        pp.s1 = 1.0;
        pp.s2 = 1.0;
        const int k = n - 2;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const double sel = s == k ? 1.0 : 0.0;
            pp.f[s] = sel;
#pragma unroll
            for (int j = 0; j < 5; ++j) pp.f[4 + 5 * s + j] = sel * c[j];
        }
#pragma unroll
        for (int j = 0; j < 5; ++j) pp.f[24 + j] = c[j];
    } else {
        pp.m = -INFINITY;
    }
    partial_block_reduce_store<kPolyNFp, kPropThreads / 64>(pp, part + (size_t)blockIdx.x * (4 + kPolyNFp));
}

// --------------------------------------------------------------- GMM --
// One datum's log-factor, log sum_k pi_k Normal(y; mu_k, sd), in FP32 with the
// max shift and the hardware exp and log, as in the batched mixture SMC;
// c[k] = log pi_k - log(sd sqrt(2 pi)).  KK components, fully unrolled.
template <int KK>
__device__ __forceinline__ float gmm_point(float y, const float (&c)[8], const float (&mu)[8], float inv_sd) {
    float t[KK];
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        const float r = (y - mu[k]) * inv_sd;
        t[k] = fmaf(-0.5f * r, r, c[k]);
    }
    float mx = t[0];
#pragma unroll
    for (int k = 1; k < KK; ++k) mx = fmaxf(mx, t[k]);
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < KK; ++k) s += __expf(t[k] - mx);
    return mx + __logf(s);
}

// Sum of the log-factors over the data: FP32 within blocks of 16 points (one
// batch of scalar loads each), FP64 across blocks.
template <int KK>
__device__ __forceinline__ double gmm_loglik(const float *__restrict__ Y, int D, const float (&c)[8],
                                             const float (&mu)[8], float isd) {
    double ll = 0.0;
    int d = 0;
    for (; d + 16 <= D; d += 16) {
        float ys[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) ys[k] = Y[d + k];
        float sb = 0.0f;
#pragma unroll 4
        for (int k = 0; k < 16; ++k) sb += gmm_point<KK>(ys[k], c, mu, isd);
        ll += (double)sb;
    }
    if (d < D) {
        float sb = 0.0f;
        for (; d < D; ++d) sb += gmm_point<KK>(Y[d], c, mu, isd);
        ll += (double)sb;
    }
    return ll;
}

// The likelihood for the run's component count K (the same for every thread).
__device__ __forceinline__ double gmm_loglik_k(const float *__restrict__ Y, int D, int K, const double (&lpi)[8],
                                               const double (&mu)[8], double inv_sd, double cst) {
    float c[8], muf[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        c[k] = k < K ? (float)(lpi[k] + cst) : 0.0f;
        muf[k] = k < K ? (float)mu[k] : 0.0f;
    }
    const float isd = (float)inv_sd;
    switch (K) {
        case 1: return gmm_loglik<1>(Y, D, c, muf, isd);
        case 2: return gmm_loglik<2>(Y, D, c, muf, isd);
        case 3: return gmm_loglik<3>(Y, D, c, muf, isd);
        case 4: return gmm_loglik<4>(Y, D, c, muf, isd);
        case 5: return gmm_loglik<5>(Y, D, c, muf, isd);
        case 6: return gmm_loglik<6>(Y, D, c, muf, isd);
        case 7: return gmm_loglik<7>(Y, D, c, muf, isd);
        default: return gmm_loglik<8>(Y, D, c, muf, isd);
    }
}

template <bool PROP>
__global__ __launch_bounds__(kPropThreads) void gmm_is_kernel(const float *__restrict__ Y, int D, int K, int64_t N,
                                                              Key key, double mu_sd, double comp_sd,
                                                              const double *__restrict__ q, double *__restrict__ lw_out,
                                                              double *__restrict__ lat_out, double *__restrict__ part) {
    const int64_t i = (int64_t)blockIdx.x * kPropThreads + threadIdx.x;
    const bool live = i < N;
    const uint32_t ii = (uint32_t)i;
    double lpi[8], mu[8], extra = 0.0;
    __shared__ double sdv[PROP ? 8 * 15 : 1], isdv[PROP ? 8 * 15 : 1];
    if constexpr (PROP) stage_scales(q + 8 + 8 * (2 * K - 1), 8 * (2 * K - 1), sdv, isdv);
    if constexpr (!PROP) {
        // Prior draws (the SMC initial particles): Dirichlet(1) weights as
        // normalised Exp(1) draws, means mu_sd z.
        const uint4 wa = philox(ii, 0, 0, kTagPrior, key), wb = philox(ii, 1, 0, kTagPrior, key);
        const uint32_t ew[8] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y, wb.z, wb.w};
        double E[8], tot = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            E[k] = k < K ? -log(u01d(ew[k])) : 0.0;
            if (k < K) tot += E[k];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) lpi[k] = k < K ? log(E[k] / tot) : -INFINITY;
        double z[8];
        normals4_d(philox(ii, 2, 0, kTagPrior, key), z);
        normals4_d(philox(ii, 3, 0, kTagPrior, key), z + 4);
#pragma unroll
        for (int k = 0; k < 8; ++k) mu[k] = mu_sd * z[k];
    } else {
        const int d = 2 * K - 1;
        const double *lmix = q, *mean = q + 8, *lsdv = q + 8 + 8 * d;
        const uint4 w0 = philox(ii, 0, 0, kTagProposal, key);
        const int comp = categorical_exp<8>(u01d(w0.x), lmix, 8);
        double z[16], u[15];
        normals4_d(philox(ii, 1, 0, kTagProposal, key), z);
        normals4_d(philox(ii, 2, 0, kTagProposal, key), z + 4);
        normals4_d(philox(ii, 3, 0, kTagProposal, key), z + 8);
        normals4_d(philox(ii, 4, 0, kTagProposal, key), z + 12);
#pragma unroll
        for (int k = 0; k < 15; ++k) u[k] = k < d ? mean[comp * d + k] + sdv[comp * d + k] * z[k] : 0.0;
        // prior density of u and the map to (log pi, mu)
        double lg[8], lgm = -INFINITY;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            lg[k] = k < K - 1 ? u[K + k < 15 ? K + k : 14] : 0.0;
            if (k < K) lgm = fmax(lgm, lg[k]);
        }
        double lgs = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k < K) lgs += exp(lg[k] - lgm);
        const double lz = lgm + log(lgs);
        double lp = lgamma((double)K) + lgamma((double)K + 1.0);
        const double lmu = log(mu_sd), imu = exp(-lmu);
        double prev = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (k < K) {
                mu[k] = k == 0 ? u[0] : prev + exp(u[k]);
                prev = mu[k];
                lpi[k] = lg[k] - lz;
                lp += log_normal(mu[k], 0.0, lmu, imu) + lpi[k];
                if (k >= 1) lp += u[k];
            } else {
                mu[k] = 0.0;
                lpi[k] = -INFINITY;
            }
        }
        // log q(u)
        double t[8], tm = -INFINITY;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            double a = lmix[m];
            for (int k = 0; k < d; ++k) a += log_normal(u[k], mean[m * d + k], lsdv[m * d + k], isdv[m * d + k]);
            t[m] = a;
            tm = fmax(tm, a);
        }
        double ts = 0.0;
#pragma unroll
        for (int m = 0; m < 8; ++m) ts += exp(t[m] - tm);
        extra = lp - (tm + log(ts));
    }
    const double cst = -kHalfLog2PiD - log(comp_sd);
    const double ll = gmm_loglik_k(Y, D, K, lpi, mu, 1.0 / comp_sd, cst);
    const double lw = live ? ll + extra : -INFINITY;
    if (live) {
        if (lw_out) lw_out[i] = lw;
        if (lat_out) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (k < K) {
                    lat_out[(size_t)k * N + i] = lpi[k];
                    lat_out[(size_t)(K + k) * N + i] = mu[k];
                }
            }
        }
    }
    // summaries: E[mu_(k)] over the means in increasing order
    double srt[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) srt[k] = k < K ? mu[k] : INFINITY;
#pragma unroll
    for (int a = 1; a < 8; ++a)
#pragma unroll
        for (int b = a; b > 0; --b) {
            const double lo = fmin(srt[b - 1], srt[b]), hi = fmax(srt[b - 1], srt[b]);
            srt[b - 1] = lo;
            srt[b] = hi;
        }
    Partial<kGmmNF> pp = partial_empty<kGmmNF>();
    if (live && isnan(lw)) pp.nan = 1.0;
    if (lw > -INFINITY) {
        pp.m = lw;
        pp.s1 = 1.0;
        pp.s2 = 1.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) pp.f[k] = k < K ? srt[k] : 0.0;
    }
    partial_block_reduce_store<kGmmNF, kPropThreads / 64>(pp, part + (size_t)blockIdx.x * (4 + kGmmNF));
}

// ---------------------------------------------------------------- host --
size_t prop_partial_bytes(int model, int64_t N) {
    const int64_t blocks = (N + kPropThreads - 1) / kPropThreads;
    const int nf = model == PPL_MODEL_POLY ? kPolyNFp : kGmmNF;
    return (size_t)blocks * (4 + nf) * sizeof(double) + merge_scratch_bytes(nf);
}

int run_importance_q(const IsArgs &a, hipStream_t st) {
    const int64_t blocks = (a.N + kPropThreads - 1) / kPropThreads;
    const char *name = a.model == PPL_MODEL_POLY ? "poly_mix_is_kernel" : (a.q_params ? "gmm_mix_is_kernel" : "gmm_is_kernel");
    if (int rc = check_grid(name, blocks, kPropThreads)) return rc;
    {
        KernelTimer timer(name, st);
        if (a.model == PPL_MODEL_POLY) {
            hipLaunchKernelGGL(poly_mix_is_kernel, dim3((unsigned)blocks), dim3(kPropThreads), 0, st,
                               (const double *)a.x, (const double *)a.y, (int)a.D, a.N, make_key(a.seed), a.hyper[0],
                               (const double *)a.q_params, (double *)a.lw_out, (double *)a.lat_out, a.part);
        } else if (a.q_params) {
            hipLaunchKernelGGL(gmm_is_kernel<true>, dim3((unsigned)blocks), dim3(kPropThreads), 0, st,
                               (const float *)a.y, (int)a.D, a.dim, a.N, make_key(a.seed), a.hyper[0], a.hyper[1],
                               (const double *)a.q_params, (double *)a.lw_out, (double *)a.lat_out, a.part);
        } else {
            hipLaunchKernelGGL(gmm_is_kernel<false>, dim3((unsigned)blocks), dim3(kPropThreads), 0, st,
                               (const float *)a.y, (int)a.D, a.dim, a.N, make_key(a.seed), a.hyper[0], a.hyper[1],
                               nullptr, (double *)a.lw_out, (double *)a.lat_out, a.part);
        }
        timer.stop();
        PPL_LAUNCH_CHECK(name);
    }
    int nrec = 0;
    if (a.model == PPL_MODEL_POLY) {
        const double *rec =
            merge_partials_first<kPolyNFp>(a.part, blocks, a.part + (size_t)blocks * (4 + kPolyNFp), &nrec, st);
        PPL_LAUNCH_CHECK("partial_merge_kernel");
        hipLaunchKernelGGL(weights_finalize_kernel<kPolyNFp>, dim3(1), dim3(kFinalizeThreads), 0, st, rec, nrec, a.N, a.model,
                           a.scalars, a.summaries);
    } else {
        const double *rec =
            merge_partials_first<kGmmNF>(a.part, blocks, a.part + (size_t)blocks * (4 + kGmmNF), &nrec, st);
        PPL_LAUNCH_CHECK("partial_merge_kernel");
        hipLaunchKernelGGL(weights_finalize_kernel<kGmmNF>, dim3(1), dim3(kFinalizeThreads), 0, st, rec, nrec, a.N, a.model,
                           a.scalars, a.summaries);
    }
    PPL_LAUNCH_CHECK("weights_finalize_kernel");
    return PPL_OK;
}

}  // namespace ppl
