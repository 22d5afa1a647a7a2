// importance.hip -- importance-sampling kernels (paper Sec. 3.6.2).
//
// Each thread owns P particles.  A particle draws its latents at the model's
// sample sites, accumulates its factors over the data, and its log-weight is
// folded into a per-block FP64 partial {max, sum e, sum e^2, sum e f}; a
// one-wave finalize kernel merges the block partials in a fixed order and
// writes log Z-hat = LSE - log N, the ESS and the posterior summaries.
//
// Data rows are the same for every lane of a wave (all lanes process the same
// datum for different particles), so they are read with scalar loads into
// SGPRs and used directly as the scalar operand of v_fma_f32; per-particle
// state stays in VGPRs for the whole data loop.
#include "blr.h"
#include "device.h"
#include "host.h"
#include "kernels.h"
#include "poly.h"
#include "timing.h"

namespace ppl {

constexpr int kIsThreads = 256;
constexpr int kIsWaves = kIsThreads / 64;
constexpr int kPolyNF = 29;     // summary fields of the polynomial model

// ------------------------------------------------------------------ BLR --
// Likelihood of one particle set: FP32 residuals r = y_d - x_d . w and squared
// sums in FP32 within consecutive 32-row blocks; block sums accumulate in FP64.
template <int P, int DIM, bool PROP>
__global__ __launch_bounds__(kIsThreads) void blr_is_kernel(
    const float *__restrict__ X, const float *__restrict__ Y, int D, int64_t N, Key key,
    float prior_sd, double noise_sd, const float *__restrict__ qp, double *__restrict__ lw_out,
    float *__restrict__ lat_out, double *__restrict__ part) {
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * (kIsThreads * P);

    float w[P][DIM];
    double extra[P];
    blr_draw<P, DIM, PROP, kIsThreads>(base, tid, key, prior_sd, qp, w, extra);

    double acc[P];
#pragma unroll
    for (int p = 0; p < P; ++p) acc[p] = 0.0;
    int d = 0;
    for (; d + 32 <= D; d += 32) {
        float s[P];
#pragma unroll
        for (int p = 0; p < P; ++p) s[p] = 0.0f;
#pragma unroll 8
        for (int dd = 0; dd < 32; ++dd) {
            const float *row = X + (size_t)(d + dd) * DIM;
            const float yv = Y[d + dd];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                float r = yv;
#pragma unroll
                for (int k = 0; k < DIM; ++k) r = fmaf(-row[k], w[p][k], r);
                s[p] = fmaf(r, r, s[p]);
            }
        }
#pragma unroll
        for (int p = 0; p < P; ++p) acc[p] += (double)s[p];
    }
    if (d < D) {
        float s[P];
#pragma unroll
        for (int p = 0; p < P; ++p) s[p] = 0.0f;
        for (; d < D; ++d) {
            const float *row = X + (size_t)d * DIM;
            const float yv = Y[d];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                float r = yv;
#pragma unroll
                for (int k = 0; k < DIM; ++k) r = fmaf(-row[k], w[p][k], r);
                s[p] = fmaf(r, r, s[p]);
            }
        }
#pragma unroll
        for (int p = 0; p < P; ++p) acc[p] += (double)s[p];
    }

    const double var = noise_sd * noise_sd;
    const double cterm = (double)D * (-0.5 * log(2.0 * M_PI * var));
    double lw[P];
#pragma unroll
    for (int p = 0; p < P; ++p) lw[p] = cterm - acc[p] / (2.0 * var) + extra[p];
    blr_finish<P, DIM, kIsThreads, kIsWaves>(base, tid, N, w, lw, lw_out, lat_out, part);
}

// ----------------------------------------------------------------- POLY --
// FP64 polynomial model.  Horner over the five coefficient slots with slots
// j >= n set to zero: 0 * x + 0 = 0 exactly, so this equals n-term Horner and
// no lane branches on the sampled degree.
template <int P>
__global__ __launch_bounds__(kIsThreads) void poly_is_kernel(
    const double *__restrict__ X, const double *__restrict__ Y, int D, int64_t N, Key key, double sd,
    int n_lo, int n_hi, double *__restrict__ lw_out, double *__restrict__ lat_out, double *__restrict__ part) {
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * (kIsThreads * P);
    double c[P][5];
    int nn[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        poly_prior_draw((uint32_t)(base + p * kIsThreads + tid), key, sd, n_lo, n_hi, nn[p], c[p]);
    }
    double pc[P][5];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int j = 0; j < 5; ++j) pc[p][j] = j < nn[p] ? c[p][j] : 0.0;

    double acc[P];
#pragma unroll
    for (int p = 0; p < P; ++p) acc[p] = 0.0;
    // Points in chunks of eight: one batch of scalar loads per chunk instead
    // of a scalar-memory round trip per point; the sum order is unchanged.
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
#pragma unroll
            for (int p = 0; p < P; ++p) {
                double v = pc[p][4];
                v = fma(v, xs[k], pc[p][3]);
                v = fma(v, xs[k], pc[p][2]);
                v = fma(v, xs[k], pc[p][1]);
                v = fma(v, xs[k], pc[p][0]);
                const double r = ys[k] - v;
                acc[p] = fma(r, r, acc[p]);
            }
        }
    }
    for (; d < D; ++d) {
        const double xv = X[d], yv = Y[d];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            double v = pc[p][4];
            v = fma(v, xv, pc[p][3]);
            v = fma(v, xv, pc[p][2]);
            v = fma(v, xv, pc[p][1]);
            v = fma(v, xv, pc[p][0]);
            const double r = yv - v;
            acc[p] = fma(r, r, acc[p]);
        }
    }

    double lw[P];
    Partial<kPolyNF> pp = partial_empty<kPolyNF>();
    double mloc = -INFINITY;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int64_t i = base + p * kIsThreads + tid;
        lw[p] = (i < N) ? -0.5 * acc[p] : -INFINITY;
        if (i < N && isnan(lw[p])) pp.nan += 1.0;
        if (lw[p] > mloc) mloc = lw[p];
        if (i < N) {
            if (lw_out) lw_out[i] = lw[p];
            if (lat_out) {
                lat_out[i] = (double)nn[p];
#pragma unroll
                for (int j = 0; j < 5; ++j) lat_out[(size_t)(1 + j) * N + i] = c[p][j];
            }
        }
    }
    pp.m = mloc;
    if (mloc > -INFINITY) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const double e = exp(lw[p] - mloc);
            pp.s1 += e;
            pp.s2 += e * e;
            const int k = nn[p] - 2;  // degree slot (n in 2..5)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const double sel = (s == k) ? e : 0.0;
                pp.f[s] += sel;
#pragma unroll
                for (int j = 0; j < 5; ++j) pp.f[4 + 5 * s + j] += sel * pc[p][j];
            }
#pragma unroll
            for (int j = 0; j < 5; ++j) pp.f[24 + j] += e * pc[p][j];
        }
    }
    partial_block_reduce_store<kPolyNF, kIsWaves>(pp, part + (size_t)blockIdx.x * (4 + kPolyNF));
}

// ---------------------------------------------------------------- host --
size_t is_partial_bytes(int model, int dim, int64_t N) {
    const int P = model == PPL_MODEL_POLY ? 1 : 4;
    const int64_t blocks = (N + (int64_t)kIsThreads * P - 1) / ((int64_t)kIsThreads * P);
    const int nf = model == PPL_MODEL_POLY ? kPolyNF : dim;
    return (size_t)blocks * (4 + nf) * sizeof(double) + merge_scratch_bytes(nf);
}

template <int DIM>
static int launch_blr(const IsArgs &a, double *part, int64_t blocks, hipStream_t st) {
    constexpr int P = 4;
    KernelTimer timer("blr_is_kernel", st);
    if (a.q_params)
        hipLaunchKernelGGL((blr_is_kernel<P, DIM, true>), dim3((unsigned)blocks), dim3(kIsThreads), 0, st,
                           (const float *)a.x, (const float *)a.y, (int)a.D, a.N, make_key(a.seed),
                           (float)a.hyper[0], a.hyper[1], (const float *)a.q_params, (double *)a.lw_out,
                           (float *)a.lat_out, part);
    else
        hipLaunchKernelGGL((blr_is_kernel<P, DIM, false>), dim3((unsigned)blocks), dim3(kIsThreads), 0, st,
                           (const float *)a.x, (const float *)a.y, (int)a.D, a.N, make_key(a.seed),
                           (float)a.hyper[0], a.hyper[1], nullptr, (double *)a.lw_out, (float *)a.lat_out, part);
    timer.stop();
    PPL_LAUNCH_CHECK("blr_is_kernel");
    int nrec = 0;
    const double *rec = merge_partials_first<DIM>(part, blocks, part + (size_t)blocks * (4 + DIM), &nrec, st);
    PPL_LAUNCH_CHECK("partial_merge_kernel");
    hipLaunchKernelGGL(weights_finalize_kernel<DIM>, dim3(1), dim3(kFinalizeThreads), 0, st, rec, nrec, a.N,
                       (int)PPL_MODEL_BLR, a.scalars, a.summaries);
    PPL_LAUNCH_CHECK("weights_finalize_kernel");
    return PPL_OK;
}

static int launch_poly(const IsArgs &a, hipStream_t st) {
    constexpr int P = 1;
    const int64_t blocks = (a.N + kIsThreads * P - 1) / (kIsThreads * P);
    if (int rc = check_grid("poly_is_kernel", blocks, kIsThreads)) return rc;
    KernelTimer timer("poly_is_kernel", st);
    hipLaunchKernelGGL((poly_is_kernel<P>), dim3((unsigned)blocks), dim3(kIsThreads), 0, st, (const double *)a.x,
                       (const double *)a.y, (int)a.D, a.N, make_key(a.seed), a.hyper[0], (int)a.hyper[1],
                       (int)a.hyper[2], (double *)a.lw_out, (double *)a.lat_out, a.part);
    timer.stop();
    PPL_LAUNCH_CHECK("poly_is_kernel");
    int nrec = 0;
    const double *rec =
        merge_partials_first<kPolyNF>(a.part, blocks, a.part + (size_t)blocks * (4 + kPolyNF), &nrec, st);
    PPL_LAUNCH_CHECK("partial_merge_kernel");
    hipLaunchKernelGGL(weights_finalize_kernel<kPolyNF>, dim3(1), dim3(kFinalizeThreads), 0, st, rec, nrec, a.N,
                       (int)PPL_MODEL_POLY, a.scalars, a.summaries);
    PPL_LAUNCH_CHECK("weights_finalize_kernel");
    return PPL_OK;
}

int run_importance(const IsArgs &a, hipStream_t st) {
    if (a.model == PPL_MODEL_POLY) {
        return launch_poly(a, st);
    }
    constexpr int P = 4;
    const int64_t blocks = (a.N + kIsThreads * P - 1) / (kIsThreads * P);
    if (int rc = check_grid("blr_is_kernel", blocks, kIsThreads)) return rc;
    switch (a.dim) {
        case 4: return launch_blr<4>(a, a.part, blocks, st);
        case 8: return launch_blr<8>(a, a.part, blocks, st);
        case 12: return launch_blr<12>(a, a.part, blocks, st);
        case 16: return launch_blr<16>(a, a.part, blocks, st);
    }
    return fail(PPL_E_ARG, "BLR dim must be 4, 8, 12 or 16 (got %d)", a.dim);
}

}  // namespace ppl
