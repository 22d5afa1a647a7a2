// host.h -- host-side helpers of libppl: error state, argument checks, device check.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ppl.h"

namespace ppl {

// Records a formatted message as the thread's last error and returns `code`.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

// PPL_OK if the current HIP device is a gfx950 part, else PPL_E_DEVICE.
int check_device();

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Hyper-parameter with a model default.
inline double hyper_or(const ppl_data *d, int i, double dflt) {
    return (d && d->hyper && d->n_hyper > i) ? d->hyper[i] : dflt;
}

// Host-side launch guard: the grid must be non-empty and within HIP limits.
int check_grid(const char *kernel, int64_t blocks, int threads);

// Importance sampling of ppl_importance on workspace ws.  ws_cap non-null: a
// request whose workspace exceeds *ws_cap fails with PPL_E_UNSUPPORTED before
// anything is launched (the no-allocation entry point's fixed scratch).
int importance_call(int model, const ppl_data *data, int64_t n, uint64_t seed, const ppl_proposal *q, void *ws,
                    size_t ws_bytes, void *stream, ppl_result *out, const size_t *ws_cap);

}  // namespace ppl

#define PPL_HIP(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) return ::ppl::fail(PPL_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define PPL_LAUNCH_CHECK(name)                                                                \
    do {                                                                                      \
        hipError_t e_ = hipGetLastError();                                                    \
        if (e_ != hipSuccess) return ::ppl::fail(PPL_E_HIP, "launch of %s: %s", name, hipGetErrorString(e_)); \
    } while (0)
