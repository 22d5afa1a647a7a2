// blr.h -- the parts of Bayesian-linear-regression importance sampling that
// the row-by-row likelihood (importance.hip) and the sufficient-statistics
// likelihood (blr_stats.hip) share, so both see the same latents and fold
// their log-weights into the normaliser the same way.
#pragma once

#include "device.h"

namespace ppl {

// Latents of the P particles i = base + p * STRIDE + tid: d = DIM standard
// normals from Philox blocks (i, b, 0, tag), b < DIM / 4 (tag 0 prior, 1
// proposal).  Prior: w = prior_sd z, extra = 0.  Proposal (mean + L z with the
// lower Cholesky factor L, float32 parameters qp = {mean[d], L[d][d]}):
// extra = log p(w) - log q(w), whose normalising constants cancel.
template <int P, int DIM, bool PROP, int STRIDE>
__device__ __forceinline__ void blr_draw(int64_t base, int tid, Key key, float prior_sd, const float *__restrict__ qp,
                                         float (&w)[P][DIM], double (&extra)[P]) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint32_t i = (uint32_t)(base + p * STRIDE + tid);
        float z[DIM];
#pragma unroll
        for (int b = 0; b < DIM / 4; ++b) normals4(philox(i, b, 0, PROP ? kTagProposal : kTagPrior, key), z + 4 * b);
        if constexpr (PROP) {
            double zz = 0.0, ww = 0.0, logdet = 0.0;
#pragma unroll
            for (int r = 0; r < DIM; ++r) {
                float v = qp[r];
#pragma unroll
                for (int k = 0; k <= r; ++k) v = fmaf(qp[DIM + r * DIM + k], z[k], v);
                w[p][r] = v;
                zz += (double)z[r] * z[r];
                ww += (double)v * v;
                logdet += log((double)qp[DIM + r * DIM + r]);
            }
            const double s = prior_sd;
            extra[p] = (-0.5 * ww / (s * s) - DIM * log(s)) - (-0.5 * zz - logdet);
        } else {
#pragma unroll
            for (int k = 0; k < DIM; ++k) w[p][k] = prior_sd * z[k];
            extra[p] = 0.0;
        }
    }
}

// Writes the particles' log-weights and latents (slots i < N) and the
// workgroup's FP64 partial record {max, sum e, sum e^2, NaN count, sum e w}.
template <int P, int DIM, int STRIDE, int NWAVES>
__device__ __forceinline__ void blr_finish(int64_t base, int tid, int64_t N, const float (&w)[P][DIM],
                                           const double (&lw_in)[P], double *__restrict__ lw_out,
                                           float *__restrict__ lat_out, double *__restrict__ part) {
    double lw[P];
    Partial<DIM> part_p = partial_empty<DIM>();
    double mloc = -INFINITY;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int64_t i = base + p * STRIDE + tid;
        lw[p] = (i < N) ? lw_in[p] : -INFINITY;
        if (i < N && isnan(lw[p])) part_p.nan += 1.0;
        if (lw[p] > mloc) mloc = lw[p];
        if (i < N) {
            if (lw_out) lw_out[i] = lw[p];
            if (lat_out) {
#pragma unroll
                for (int k = 0; k < DIM; ++k) lat_out[(size_t)k * N + i] = w[p][k];
            }
        }
    }
    part_p.m = mloc;
    if (mloc > -INFINITY) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const double e = exp(lw[p] - mloc);
            part_p.s1 += e;
            part_p.s2 += e * e;
#pragma unroll
            for (int k = 0; k < DIM; ++k) part_p.f[k] += e * (double)w[p][k];
        }
    }
    partial_block_reduce_store<DIM, NWAVES>(part_p, part + (size_t)blockIdx.x * (4 + DIM));
}

}  // namespace ppl
