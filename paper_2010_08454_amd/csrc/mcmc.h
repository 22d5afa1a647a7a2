// mcmc.h -- launch interface of the lightweight Metropolis-Hastings chains.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppl {

struct McmcArgs {
    const double *x, *y;     // data [D] (FP64)
    int64_t D;
    int64_t C, T, burn;      // chains, iterations per chain, burn-in iterations
    uint64_t seed;
    double hyper[8];         // POLY: {sd, n_lo, n_hi}
    double *state_out;       // [6][C] or null
    int64_t *acc_out;        // [C] or null
    int8_t *n_trace;         // [T][C] or null
    double *la_trace;        // [T][C] or null
    double *summaries;       // [29] or null
    double *scalars;         // [4] device
    void *ws;
};

size_t mcmc_ws_bytes(int64_t chains);
int run_mcmc_poly(const McmcArgs &a, hipStream_t st);

}  // namespace ppl
