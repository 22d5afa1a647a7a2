// smc.h -- sequential Monte Carlo launch interface (LGSSM and mixture models).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ppl.h"

namespace ppl {

struct SmcArgs {
    int model;
    const float *y;      // observations [T]
    int64_t T;
    int K;               // mixture components (GMM)
    int64_t N;
    uint64_t seed;
    uint32_t inst;       // instance id carried in Philox counter word 3
    double ess_frac;
    int move_steps;      // resample-move: MH steps per particle after each resampling (GMM)
    double move_scale;   // random-walk scale factor (0: 2.38 / sqrt(2K - 1))
    int64_t t_begin, t_end;   // factors of this call [t_begin, t_end)
    void *ckpt;          // checkpoint read when t_begin > 0, written when t_end < T
    double hyper[8];
    ppl_result out;      // caller's output pointers
    void *ws;
};

size_t smc_ws_bytes(int model, int K, int64_t N);
size_t smc_checkpoint_bytes(int model, int K, int64_t N);
int run_smc(const SmcArgs &a, hipStream_t st);
// Device scalars the run writes (the caller's d_scalars, or the workspace slot).
double *smc_scalars_ptr(const SmcArgs &a);

}  // namespace ppl
