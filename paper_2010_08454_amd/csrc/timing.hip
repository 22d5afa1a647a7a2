// timing.hip -- optional per-kernel timing with HIP events on the launch stream.
//
// When enabled, launchers bracket their dominant kernels with an event pair
// recorded on the caller's stream; ppl_timing_query() waits for the pending
// pairs and returns the accumulated elapsed time per kernel name.  Disabled
// (the default) it costs one relaxed atomic load per launch.
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "host.h"
#include "timing.h"

namespace ppl {

namespace {
struct Pending {
    const char *name;
    hipEvent_t a, b;
};
std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
std::map<std::string, std::pair<double, int64_t>> g_acc;
thread_local int t_suspended = 0;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int drain_locked() {
    for (const Pending &p : g_pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(p.b) != hipSuccess || hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess)
            return fail(PPL_E_HIP, "timing event query failed");
        auto &acc = g_acc[p.name];
        acc.first += ms;
        acc.second += 1;
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    g_pending.clear();
    return PPL_OK;
}
}  // namespace

KernelTimer::KernelTimer(const char *name, hipStream_t st) : name_(name), st_(st), a_(nullptr) {
    if (!g_on.load(std::memory_order_relaxed) || t_suspended) return;
    std::lock_guard<std::mutex> lk(g_mu);
    a_ = take_event();
    if (a_ && hipEventRecord(a_, st_) != hipSuccess) {
        g_pool.push_back(a_);
        a_ = nullptr;
    }
}

void KernelTimer::stop() {
    if (!a_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t b = take_event();
    if (b && hipEventRecord(b, st_) == hipSuccess) {
        g_pending.push_back(Pending{name_, a_, b});
    } else {
        g_pool.push_back(a_);
        if (b) g_pool.push_back(b);
    }
    a_ = nullptr;
}

TimingSuspend::TimingSuspend() { ++t_suspended; }
TimingSuspend::~TimingSuspend() { --t_suspended; }

}  // namespace ppl

using namespace ppl;

extern "C" int ppl_timing_enable(int on) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_mu);
    if (int rc = drain_locked()) return rc;
    if (on) g_acc.clear();
    g_on.store(on != 0, std::memory_order_relaxed);
    return PPL_OK;
}

extern "C" int ppl_timing_query(const char *kernel, double *total_ms, int64_t *launches) {
    clear_error();
    if (!kernel || !total_ms || !launches) return fail(PPL_E_ARG, "kernel, total_ms and launches must be non-NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    if (int rc = drain_locked()) return rc;
    auto it = g_acc.find(kernel);
    *total_ms = it == g_acc.end() ? 0.0 : it->second.first;
    *launches = it == g_acc.end() ? 0 : it->second.second;
    return PPL_OK;
}
