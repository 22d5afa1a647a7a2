// batched.h -- launch interface of the batched (many-instance) SMC engine.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ppl.h"

namespace ppl {

int bt_check(int model, int n, const ppl_instance *h);
// Workspace bytes for a configuration (tune NULL: the default one); 0 if the
// configuration is invalid for these instances.
size_t bt_ws_bytes_for(const ppl_instance *h, int n, const ppl_tune *tune);
int run_smc_batched(int n, const ppl_instance *h, const ppl_instance *d_inst, uint64_t seed, double ess_frac,
                    const ppl_tune *tune, void *ws, size_t ws_bytes, hipStream_t st, const ppl_batch_result &out,
                    ppl_tune *used);

}  // namespace ppl
