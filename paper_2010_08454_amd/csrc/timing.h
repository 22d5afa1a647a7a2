// timing.h -- scoped HIP-event timer around a kernel launch (active only when
// ppl_timing_enable(1) was called).
#pragma once

#include <hip/hip_runtime.h>

namespace ppl {

class KernelTimer {
public:
    KernelTimer(const char *name, hipStream_t st);
    void stop();
    ~KernelTimer() { stop(); }

private:
    const char *name_;
    hipStream_t st_;
    hipEvent_t a_;
};

// While an instance lives on this thread, KernelTimer records nothing (used
// while a stream is being captured into a graph).
class TimingSuspend {
public:
    TimingSuspend();
    ~TimingSuspend();
};

}  // namespace ppl
