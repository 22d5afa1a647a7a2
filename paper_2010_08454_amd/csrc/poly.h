// poly.h -- the polynomial model of the paper's running example (Sec. 1.1):
// n ~ UniformDiscrete{n_lo..n_hi}, c_j ~ Normal(0, sd) for j < n,
// factor(-sum_d (y_d - sum_j c_j x_d^j)^2 / 2); shared by importance sampling
// and the Metropolis-Hastings chains (whose chains start from this draw).
#pragma once

#include "device.h"

namespace ppl {

// Prior draw of execution i (tag 0): block 0 word 0 picks n; blocks 1..3 give
// one double-precision Box-Muller pair each, c_0..c_5 (all drawn whatever n
// is, so the word table does not depend on the branch); c_j for j >= n are
// returned as they were drawn.
__device__ __forceinline__ void poly_prior_draw(uint32_t i, Key key, double sd, int n_lo, int n_hi, int &n,
                                                double c[5]) {
    const uint4 w0 = philox(i, 0, 0, kTagPrior, key);
    n = uniform_discrete(w0.x, n_lo, (uint32_t)(n_hi - n_lo + 1));
    double z[6];
#pragma unroll
    for (int b = 1; b <= 3; ++b) {
        const uint4 w = philox(i, b, 0, kTagPrior, key);
        box_muller(unit_f64(w.x, w.y), unit_f64(w.z, w.w), z[2 * (b - 1)], z[2 * (b - 1) + 1]);
    }
#pragma unroll
    for (int j = 0; j < 5; ++j) c[j] = sd * z[j];
}

// One point's contribution (y - p(x))^2 with p evaluated by Horner over the
// five coefficient slots, zero past the degree: 0 x + 0 = 0 exactly, so this
// equals n-term Horner and no lane branches on n.
__device__ __forceinline__ double poly_sq_residual(const double pc[5], double x, double y) {
    double v = pc[4];
    v = fma(v, x, pc[3]);
    v = fma(v, x, pc[2]);
    v = fma(v, x, pc[1]);
    v = fma(v, x, pc[0]);
    const double r = y - v;
    return r * r;
}

}  // namespace ppl
