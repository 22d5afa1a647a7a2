// noalloc.hip -- importance sampling that allocates nothing: the variant of
// ppl_importance for callers that cannot call hipMalloc (code under HIP graph
// capture, tight serving loops, harnesses that forbid allocation).
//
// The workspace of ppl_importance (the device scalars and the per-workgroup
// partial records of the normaliser and the summaries) lives in `scratch`, a
// file-scope device array of PPL_NOALLOC_SCRATCH_BYTES.  Each GPU the library
// runs on holds its own copy until the process ends.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in symbol): the
// first call on a device looks up that device's address of the array with
// hipGetSymbolAddress, with the device current, and keeps it.
//
// Every call on a GPU shares that GPU's array: calls that overlap on one GPU
// (two streams, two threads) race on it.  The kernels write every partial
// record and scalar before any is read, so nothing needs clearing between
// calls; the array keeps the last call's contents.
#include <mutex>

#include "host.h"

namespace ppl {

__device__ __align__(256) unsigned char scratch[PPL_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// The current device's address of `scratch` (looked up once per device).
static int scratch_ptr(void **out) {
    int dev = -1;
    PPL_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PPL_E_DEVICE, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PPL_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PPL_OK;
}

}  // namespace ppl

using namespace ppl;

extern "C" int ppl_importance_noalloc(int model, const ppl_data *data, int64_t n, uint64_t seed,
                                      const ppl_proposal *q, void *stream, ppl_result *out) {
    clear_error();
    if (int rc = check_device()) return rc;
    void *ws = nullptr;
    if (int rc = scratch_ptr(&ws)) return rc;
    const size_t cap = PPL_NOALLOC_SCRATCH_BYTES;
    return importance_call(model, data, n, seed, q, ws, cap, stream, out, &cap);
}
