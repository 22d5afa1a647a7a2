// smc.hip -- sequential Monte Carlo (placeholder until the SMC kernels land).
#include "host.h"
#include "smc.h"

namespace ppl {

size_t smc_ws_bytes(int, int, int64_t) { return 256; }
double *smc_scalars_ptr(const SmcArgs &a) { return a.out.d_scalars ? a.out.d_scalars : (double *)a.ws; }
int run_smc(const SmcArgs &, hipStream_t) { return fail(PPL_E_UNSUPPORTED, "SMC is not built yet"); }

}  // namespace ppl
