// api.hip -- the extern "C" boundary of libppl: argument validation, workspace
// planning, device check and dispatch to the kernel launchers.  Every error a
// host can detect is returned before anything is enqueued.
#include <math.h>
#include <stdarg.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "batched.h"
#include "host.h"
#include "kernels.h"
#include "mcmc.h"
#include "proposal.h"
#include "smc.h"
#include "timing.h"

namespace ppl {

static thread_local char g_last_error[512];

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_last_error[0] = 0; }

int check_device() {
    static std::atomic<int> verdict[64];   // 0 unknown, 1 ok, 2 not gfx950
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0) {
        (void)hipGetLastError();
        return fail(PPL_E_DEVICE, "no HIP device available (%s)", hipGetErrorString(e));
    }
    if (dev < 64) {
        const int v = verdict[dev].load(std::memory_order_relaxed);
        if (v == 1) return PPL_OK;
        if (v == 2) return fail(PPL_E_DEVICE, "device %d is not a gfx950 GPU", dev);
    }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return fail(PPL_E_DEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e));
    const bool ok = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    if (dev < 64) verdict[dev].store(ok ? 1 : 2, std::memory_order_relaxed);
    if (!ok) return fail(PPL_E_DEVICE, "device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);
    return PPL_OK;
}

int check_grid(const char *kernel, int64_t blocks, int threads) {
    if (blocks < 1 || blocks > 0x7fffffffLL || threads < 1 || threads > 1024)
        return fail(PPL_E_ARG, "%s: launch shape %lld x %d out of range", kernel, (long long)blocks, threads);
    return PPL_OK;
}

static bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

static bool is_int(double v) { return isfinite(v) && v == floor(v); }

static int check_ws(void *ws, size_t ws_bytes, size_t need) {
    if (need == 0) return PPL_OK;
    if (!ws) return fail(PPL_E_WORKSPACE, "workspace is NULL (%zu bytes needed)", need);
    if (((uintptr_t)ws & 255) != 0) return fail(PPL_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < need) return fail(PPL_E_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, need);
    return PPL_OK;
}

// Validates a model's data block and fills the hyper-parameters with defaults.
static int check_model_data(int model, const ppl_data *d, double hyper[8]) {
    if (!d) return fail(PPL_E_ARG, "data is NULL");
    if (d->n_data < 0 || d->n_data > 0x7fffffffLL) return fail(PPL_E_ARG, "n_data %lld out of range", (long long)d->n_data);
    if (d->n_hyper < 0 || (d->n_hyper > 0 && !d->hyper)) return fail(PPL_E_ARG, "hyper is NULL with n_hyper > 0");
    for (int i = 0; i < 8; ++i) hyper[i] = 0.0;
    switch (model) {
        case PPL_MODEL_POLY:
            if (d->dtype != PPL_F64) return fail(PPL_E_ARG, "POLY data must be PPL_F64");
            if (d->n_data > 0 && (!d->x || !d->y)) return fail(PPL_E_ARG, "POLY needs x and y");
            hyper[0] = hyper_or(d, 0, 10.0);
            hyper[1] = hyper_or(d, 1, 2.0);
            hyper[2] = hyper_or(d, 2, 5.0);
            if (!finite_pos(hyper[0])) return fail(PPL_E_ARG, "POLY prior sd must be positive");
            if (!is_int(hyper[1]) || !is_int(hyper[2]) || hyper[1] < 1 || hyper[2] > 5 || hyper[1] > hyper[2])
                return fail(PPL_E_ARG, "POLY degree range must satisfy 1 <= n_lo <= n_hi <= 5");
            return PPL_OK;
        case PPL_MODEL_BLR:
        case PPL_MODEL_BLR_STATS:
            if (d->dtype != PPL_F32) return fail(PPL_E_ARG, "BLR data must be PPL_F32");
            if (d->dim != 4 && d->dim != 8 && d->dim != 12 && d->dim != 16)
                return fail(PPL_E_ARG, "BLR dim must be 4, 8, 12 or 16 (got %d)", d->dim);
            if (d->n_data > 0 && (!d->x || !d->y)) return fail(PPL_E_ARG, "BLR needs x and y");
            hyper[0] = hyper_or(d, 0, 1.0);
            hyper[1] = hyper_or(d, 1, 0.5);
            if (!finite_pos(hyper[0]) || !finite_pos(hyper[1])) return fail(PPL_E_ARG, "BLR sds must be positive");
            return PPL_OK;
        case PPL_MODEL_LGSSM:
            if (d->dtype != PPL_F32) return fail(PPL_E_ARG, "LGSSM data must be PPL_F32");
            if (d->n_data > 0 && !d->y) return fail(PPL_E_ARG, "LGSSM needs y");
            hyper[0] = hyper_or(d, 0, 0.9);
            hyper[1] = hyper_or(d, 1, 1.0);
            hyper[2] = hyper_or(d, 2, 0.5);
            hyper[3] = hyper_or(d, 3, 0.0);
            hyper[4] = hyper_or(d, 4, 0.0);
            if (!isfinite(hyper[0]) || !finite_pos(hyper[1]) || !finite_pos(hyper[2]) || !isfinite(hyper[3]) ||
                !isfinite(hyper[4]) || hyper[4] < 0)
                return fail(PPL_E_ARG, "LGSSM hyper-parameters must be finite with positive sds");
            return PPL_OK;
        case PPL_MODEL_GMM:
            if (d->dtype != PPL_F32) return fail(PPL_E_ARG, "GMM data must be PPL_F32");
            if (d->dim < 1 || d->dim > 8) return fail(PPL_E_ARG, "GMM K must be in 1..8 (got %d)", d->dim);
            if (d->n_data > 0 && !d->y) return fail(PPL_E_ARG, "GMM needs y");
            hyper[0] = hyper_or(d, 0, 5.0);
            hyper[1] = hyper_or(d, 1, 1.0);
            if (!finite_pos(hyper[0]) || !finite_pos(hyper[1])) return fail(PPL_E_ARG, "GMM sds must be positive");
            return PPL_OK;
    }
    return fail(PPL_E_MODEL, "unknown model id %d", model);
}

static int check_n(int64_t n) {
    if (n < 1 || n > 0x7fffffffLL) return fail(PPL_E_ARG, "particle count %lld out of range [1, 2^31)", (long long)n);
    return PPL_OK;
}

static bool is_model(int model) {
    return model == PPL_MODEL_POLY || model == PPL_MODEL_BLR || model == PPL_MODEL_BLR_STATS || model == PPL_MODEL_GMM;
}

static size_t is_ws_bytes(int model, int dim, int64_t n, int64_t D) {
    if (model == PPL_MODEL_BLR_STATS) return 256 + align_up(blr_stats_ws_bytes(dim, n, D), 256);
    size_t part = model == PPL_MODEL_GMM ? prop_partial_bytes(model, n) : is_partial_bytes(model, dim, n);
    if (model == PPL_MODEL_POLY) part = std::max(part, prop_partial_bytes(model, n));
    return 256 + align_up(part, 256);
}

// Blocks on the stream and copies the device scalars into the host fields.
static int sync_scalars(ppl_result *out, const double *d_scal, hipStream_t st) {
    double h[8];
    PPL_HIP(hipMemcpyAsync(h, d_scal, sizeof(h), hipMemcpyDeviceToHost, st));
    PPL_HIP(hipStreamSynchronize(st));
    out->log_evidence = h[0];
    out->ess = h[1];
    out->n_resample = (int64_t)h[2];
    out->status = (int32_t)h[3];
    if (out->status) return fail(out->status, "device reported status %d (%s)", out->status, ppl_status_string(out->status));
    return PPL_OK;
}

// Importance sampling behind ppl_importance and ppl_importance_noalloc.  With
// ws_cap non-null the workspace is the caller-less scratch array: a call whose
// workspace would exceed *ws_cap is rejected before anything is launched.
int importance_call(int model, const ppl_data *data, int64_t n, uint64_t seed, const ppl_proposal *q, void *ws,
                    size_t ws_bytes, void *stream, ppl_result *out, const size_t *ws_cap) {
    if (!out) return fail(PPL_E_ARG, "out is NULL");
    if (!is_model(model))
        return fail(PPL_E_MODEL, "importance sampling supports POLY, BLR, BLR_STATS and GMM (got %d)", model);
    if (int rc = check_n(n)) return rc;
    IsArgs a{};
    if (int rc = check_model_data(model, data, a.hyper)) return rc;
    bool mixture_path = model == PPL_MODEL_GMM;
    if (q && q->kind != PPL_Q_PRIOR) {
        if (!q->d_params) return fail(PPL_E_ARG, "proposal parameters are NULL");
        if (q->kind == PPL_Q_GAUSS_FULL && (model == PPL_MODEL_BLR || model == PPL_MODEL_BLR_STATS)) {
            if (q->dim != data->dim) return fail(PPL_E_ARG, "Gaussian proposal needs params of dim %d", data->dim);
        } else if (q->kind == PPL_Q_POLY_MIX && model == PPL_MODEL_POLY) {
            if (q->dim != 5) return fail(PPL_E_ARG, "POLY mixture proposal has dim 5 (got %d)", q->dim);
            if (a.hyper[1] != 2.0 || a.hyper[2] != 5.0)
                return fail(PPL_E_ARG, "the POLY mixture proposal covers degrees 2..5; the model range must be 2..5");
            mixture_path = true;
        } else if (q->kind == PPL_Q_GMM_MIX && model == PPL_MODEL_GMM) {
            if (q->dim != 2 * data->dim - 1) return fail(PPL_E_ARG, "GMM mixture proposal has dim 2K - 1 = %d", 2 * data->dim - 1);
        } else {
            return fail(PPL_E_UNSUPPORTED, "proposal kind %d is not available for model %d", q->kind, model);
        }
        a.q_params = q->d_params;
    }
    const size_t need = is_ws_bytes(model, data->dim, n, data->n_data);
    if (ws_cap && need > *ws_cap)
        return fail(PPL_E_UNSUPPORTED, "%lld particles need %zu bytes of scratch; the no-allocation entry point holds %zu",
                    (long long)n, need, *ws_cap);
    if (int rc = check_ws(ws, ws_bytes, need)) return rc;
    if (int rc = check_device()) return rc;
    a.model = model;
    a.x = data->x;
    a.y = data->y;
    a.D = data->n_data;
    a.dim = data->dim;
    a.N = n;
    a.seed = seed;
    a.lw_out = out->d_log_weights;
    a.lat_out = out->d_latents;
    a.summaries = out->d_summaries;
    a.scalars = out->d_scalars ? out->d_scalars : (double *)ws;
    a.part = (double *)((char *)ws + 256);
    hipStream_t st = (hipStream_t)stream;
    const int rc = mixture_path ? run_importance_q(a, st)
                   : model == PPL_MODEL_BLR_STATS ? run_importance_blr_stats(a, st)
                                                  : run_importance(a, st);
    if (rc) return rc;
    if (out->sync_host) return sync_scalars(out, a.scalars, st);
    return PPL_OK;
}

// Validates PPL_MODEL_HMM data; fills the argument block's sizes and host views.
static int check_hmm(const ppl_data *d, EnumArgs &a) {
    if (!d) return fail(PPL_E_ARG, "data is NULL");
    if (!d->hyper || d->n_hyper < 2) return fail(PPL_E_ARG, "the HMM needs hyper = {K, sigma, pi0, A, mu}");
    const double *h = d->hyper;
    const int K = (int)h[0];
    if (h[0] != (double)K || K < 1 || K > 8) return fail(PPL_E_ARG, "HMM K must be an integer in 1..8");
    if (d->dim != K) return fail(PPL_E_ARG, "data dim %d differs from hyper K %d", d->dim, K);
    if (d->n_hyper != 2 + 2 * K + K * K) return fail(PPL_E_ARG, "HMM hyper needs %d values (got %d)", 2 + 2 * K + K * K, d->n_hyper);
    if (d->n_data < 1 || d->n_data > 40) return fail(PPL_E_ARG, "HMM T must be in 1..40 (got %lld)", (long long)d->n_data);
    if (!d->y) return fail(PPL_E_ARG, "HMM needs y");
    if (d->dtype != PPL_F64) return fail(PPL_E_ARG, "HMM data are float64");
    if (!finite_pos(h[1])) return fail(PPL_E_ARG, "HMM sigma must be positive");
    for (int i = 2; i < 2 + K + K * K; ++i)
        if (!(h[i] >= 0.0) || !std::isfinite(h[i])) return fail(PPL_E_ARG, "HMM probabilities must be finite and >= 0");
    for (int i = 2 + K + K * K; i < 2 + 2 * K + K * K; ++i)
        if (!std::isfinite(h[i])) return fail(PPL_E_ARG, "HMM means must be finite");
    const int T = (int)d->n_data;
    if ((double)T * std::log2((double)K) > 50.0) return fail(PPL_E_UNSUPPORTED, "%d^%d paths exceed 2^50", K, T);
    a.K = K;
    a.T = T;
    a.y = (const double *)d->y;
    a.sigma = h[1];
    a.pi0 = h + 2;
    a.A = h + 2 + K;
    a.mu = h + 2 + K + K * K;
    return PPL_OK;
}

}  // namespace ppl

using namespace ppl;

extern "C" {

const char *ppl_status_string(int status) {
    switch (status) {
        case PPL_OK: return "ok";
        case PPL_E_ARG: return "invalid argument";
        case PPL_E_MODEL: return "unknown or unsupported model";
        case PPL_E_DEVICE: return "no gfx950 device";
        case PPL_E_HIP: return "HIP runtime error";
        case PPL_E_WORKSPACE: return "workspace missing or too small";
        case PPL_E_NONFINITE: return "non-finite log-weight";
        case PPL_E_ZERO_WEIGHT: return "every weight is zero";
        case PPL_E_UNSUPPORTED: return "unsupported request";
    }
    return "unknown status";
}

const char *ppl_last_error(void) { return g_last_error; }

int ppl_version(void) { return 100; }

int ppl_workspace_size(int model, const ppl_data *data, int64_t n, int algo, size_t *bytes) {
    clear_error();
    if (!bytes) return fail(PPL_E_ARG, "bytes is NULL");
    if (int rc = check_n(n)) return rc;
    switch (algo) {
        case PPL_ALGO_LSE: *bytes = align_up(lse_ws_bytes(n), 256); return PPL_OK;
        case PPL_ALGO_RESAMPLE: *bytes = align_up(resample_ws_bytes(n), 256); return PPL_OK;
        case PPL_ALGO_IS: {
            double h[8];
            if (!is_model(model))
                return fail(PPL_E_MODEL, "importance sampling supports POLY, BLR, BLR_STATS and GMM (got %d)", model);
            if (int rc = check_model_data(model, data, h)) return rc;
            *bytes = is_ws_bytes(model, data->dim, n, data->n_data);
            return PPL_OK;
        }
        case PPL_ALGO_MCMC: {
            double h[8];
            if (model != PPL_MODEL_POLY) return fail(PPL_E_MODEL, "MCMC supports POLY (got %d)", model);
            if (int rc = check_model_data(model, data, h)) return rc;
            *bytes = mcmc_ws_bytes(n);
            return PPL_OK;
        }
        case PPL_ALGO_ENUM: {
            EnumArgs a{};
            if (model != PPL_MODEL_HMM) return fail(PPL_E_MODEL, "enumeration supports HMM (got %d)", model);
            if (int rc = check_hmm(data, a)) return rc;
            *bytes = enum_ws_bytes(a.K, a.T);
            return PPL_OK;
        }
        case PPL_ALGO_SMC: {
            double h[8];
            if (model != PPL_MODEL_LGSSM && model != PPL_MODEL_GMM)
                return fail(PPL_E_MODEL, "SMC supports LGSSM and GMM (got %d)", model);
            if (int rc = check_model_data(model, data, h)) return rc;
            *bytes = smc_ws_bytes(model, data->dim, n);
            return PPL_OK;
        }
    }
    return fail(PPL_E_ARG, "unknown algo %d", algo);
}

int ppl_importance(int model, const ppl_data *data, int64_t n, uint64_t seed, const ppl_proposal *q, void *ws,
                   size_t ws_bytes, void *stream, ppl_result *out) {
    clear_error();
    return importance_call(model, data, n, seed, q, ws, ws_bytes, stream, out, nullptr);
}

int ppl_lse_ess(const void *lw, int dtype, int64_t n, double *out, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    if (!lw || !out) return fail(PPL_E_ARG, "d_lw and d_out must be non-NULL");
    if (dtype != PPL_F32 && dtype != PPL_F64) return fail(PPL_E_ARG, "dtype must be PPL_F32 or PPL_F64");
    if (int rc = check_n(n)) return rc;
    if (int rc = check_ws(ws, ws_bytes, lse_ws_bytes(n))) return rc;
    if (int rc = check_device()) return rc;
    return run_lse(lw, dtype == PPL_F64, n, out, ws, (hipStream_t)stream);
}

int ppl_resample(const void *lw, int dtype, int64_t n, uint64_t seed, uint32_t step, uint32_t inst, int32_t *anc,
                 void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    if (!lw || !anc) return fail(PPL_E_ARG, "d_lw and d_anc must be non-NULL");
    if (dtype != PPL_F32 && dtype != PPL_F64) return fail(PPL_E_ARG, "dtype must be PPL_F32 or PPL_F64");
    if (int rc = check_n(n)) return rc;
    if (inst >= (1u << 24)) return fail(PPL_E_ARG, "instance id must be < 2^24");
    if (int rc = check_ws(ws, ws_bytes, resample_ws_bytes(n))) return rc;
    if (int rc = check_device()) return rc;
    return run_resample(lw, dtype == PPL_F64, n, seed, step, inst, anc, ws, (hipStream_t)stream);
}

int ppl_resample_gather(const void *lw, int dtype, int64_t n, uint64_t seed, uint32_t step, uint32_t inst,
                        int32_t n_fields, const void *state_in, void *state_out, int32_t *anc, void *ws,
                        size_t ws_bytes, void *stream) {
    clear_error();
    if (!lw || !state_in || !state_out) return fail(PPL_E_ARG, "d_lw, d_state_in and d_state_out must be non-NULL");
    if (dtype != PPL_F32 && dtype != PPL_F64) return fail(PPL_E_ARG, "dtype must be PPL_F32 or PPL_F64");
    if (int rc = check_n(n)) return rc;
    if (n_fields < 1 || n_fields > 4096) return fail(PPL_E_ARG, "n_fields %d out of range [1, 4096]", n_fields);
    if (inst >= (1u << 24)) return fail(PPL_E_ARG, "instance id must be < 2^24");
    const uintptr_t bytes = (uintptr_t)n_fields * (uintptr_t)n * 4u;
    const uintptr_t i0 = (uintptr_t)state_in, o0 = (uintptr_t)state_out;
    if (i0 < o0 + bytes && o0 < i0 + bytes) return fail(PPL_E_ARG, "d_state_in and d_state_out overlap");
    if (int rc = check_ws(ws, ws_bytes, resample_ws_bytes(n))) return rc;
    if (int rc = check_device()) return rc;
    return run_resample_gather(lw, dtype == PPL_F64, n, seed, step, inst, n_fields, state_in, state_out, anc, ws,
                               (hipStream_t)stream);
}

int ppl_philox(uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n, uint32_t *out, void *stream) {
    clear_error();
    if (!out) return fail(PPL_E_ARG, "d_out is NULL");
    if (n < 1 || n > (1LL << 32)) return fail(PPL_E_ARG, "n %lld out of range [1, 2^32]", (long long)n);
    if (int rc = check_device()) return rc;
    return run_philox(seed, c1, c2, c3, n, out, (hipStream_t)stream);
}

int ppl_smc_ex(int model, const ppl_data *data, int64_t n, uint64_t seed, const ppl_smc_options *opt, void *ws,
               size_t ws_bytes, void *stream, ppl_result *out) {
    clear_error();
    if (!out || !opt) return fail(PPL_E_ARG, "out and opt must be non-NULL");
    if (model != PPL_MODEL_LGSSM && model != PPL_MODEL_GMM)
        return fail(PPL_E_MODEL, "SMC supports LGSSM and GMM (got %d)", model);
    if (int rc = check_n(n)) return rc;
    SmcArgs a{};
    if (int rc = check_model_data(model, data, a.hyper)) return rc;
    const double ess_frac = opt->ess_frac;
    if (!(ess_frac >= 0.0 && ess_frac <= 1.0)) return fail(PPL_E_ARG, "ess_frac must be in [0, 1]");
    if (opt->move_steps < 0 || opt->move_steps > 64) return fail(PPL_E_ARG, "move_steps must be in 0..64");
    if (opt->move_steps > 0 && model != PPL_MODEL_GMM)
        return fail(PPL_E_UNSUPPORTED, "resample-move is implemented for the mixture model");
    if (!(opt->move_scale >= 0.0) || !isfinite(opt->move_scale)) return fail(PPL_E_ARG, "move_scale must be >= 0");
    if (out->max_events < 0 || (out->max_events > 0 && !out->d_ancestors && !out->d_event_lw && !out->d_move_log_alpha))
        return fail(PPL_E_ARG, "max_events > 0 with no event record buffer");
    const int64_t T = data->n_data;
    const int64_t t_end = opt->t_end == 0 ? T : opt->t_end;
    if (opt->t_begin < 0 || opt->t_begin > t_end || t_end > T || t_end < 0)
        return fail(PPL_E_ARG, "need 0 <= t_begin <= t_end <= T (got %lld, %lld, T = %lld)", (long long)opt->t_begin,
                    (long long)opt->t_end, (long long)T);
    if ((opt->t_begin > 0 || t_end < T) && !opt->d_checkpoint)
        return fail(PPL_E_ARG, "stopping before T or resuming needs d_checkpoint");
    if (opt->d_checkpoint && ((uintptr_t)opt->d_checkpoint & 255))
        return fail(PPL_E_ARG, "d_checkpoint must be 256-byte aligned");
    if (int rc = check_ws(ws, ws_bytes, smc_ws_bytes(model, data->dim, n))) return rc;
    if (int rc = check_device()) return rc;
    a.model = model;
    a.y = (const float *)data->y;
    a.T = data->n_data;
    a.K = data->dim;
    a.N = n;
    a.seed = seed;
    a.inst = 0;
    a.ess_frac = ess_frac;
    a.move_steps = opt->move_steps;
    a.move_scale = opt->move_scale;
    a.t_begin = opt->t_begin;
    a.t_end = t_end;
    a.ckpt = opt->d_checkpoint;
    a.out = *out;
    if (a.move_steps == 0) a.out.d_move_log_alpha = nullptr;
    a.ws = ws;
    hipStream_t st = (hipStream_t)stream;
    if (int rc = run_smc(a, st)) return rc;
    if (out->sync_host) return sync_scalars(out, smc_scalars_ptr(a), st);
    return PPL_OK;
}

int ppl_smc(int model, const ppl_data *data, int64_t n, uint64_t seed, double ess_frac, void *ws, size_t ws_bytes,
            void *stream, ppl_result *out) {
    const ppl_smc_options opt{ess_frac, 0, 0, 0.0, 0, 0, nullptr};
    return ppl_smc_ex(model, data, n, seed, &opt, ws, ws_bytes, stream, out);
}

int ppl_smc_checkpoint_bytes(int model, const ppl_data *data, int64_t n, size_t *bytes) {
    clear_error();
    if (!bytes) return fail(PPL_E_ARG, "bytes is NULL");
    if (model != PPL_MODEL_LGSSM && model != PPL_MODEL_GMM)
        return fail(PPL_E_MODEL, "SMC supports LGSSM and GMM (got %d)", model);
    if (int rc = check_n(n)) return rc;
    double h[8];
    if (int rc = check_model_data(model, data, h)) return rc;
    *bytes = smc_checkpoint_bytes(model, data->dim, n);
    return PPL_OK;
}

int ppl_mcmc(int model, const ppl_data *data, int64_t n_chains, int64_t n_iters, int64_t burn_in, uint64_t seed,
             void *ws, size_t ws_bytes, void *stream, ppl_mcmc_result *out) {
    clear_error();
    if (!out) return fail(PPL_E_ARG, "out is NULL");
    if (model != PPL_MODEL_POLY) return fail(PPL_E_MODEL, "MCMC supports POLY (got %d)", model);
    if (int rc = check_n(n_chains)) return rc;
    if (n_iters < 0 || n_iters > 0x7fffffffLL / 3) return fail(PPL_E_ARG, "n_iters %lld out of range", (long long)n_iters);
    if (burn_in < 0 || burn_in > n_iters) return fail(PPL_E_ARG, "burn_in must be in [0, n_iters]");
    McmcArgs a{};
    if (int rc = check_model_data(model, data, a.hyper)) return rc;
    if ((out->d_n_trace || out->d_log_alpha) && (double)n_iters * (double)n_chains > 4e12)
        return fail(PPL_E_ARG, "trace of %lld x %lld entries is too large", (long long)n_iters, (long long)n_chains);
    if (int rc = check_ws(ws, ws_bytes, mcmc_ws_bytes(n_chains))) return rc;
    if (int rc = check_device()) return rc;
    a.x = (const double *)data->x;
    a.y = (const double *)data->y;
    a.D = data->n_data;
    a.C = n_chains;
    a.T = n_iters;
    a.burn = burn_in;
    a.seed = seed;
    a.state_out = out->d_state;
    a.acc_out = out->d_accepts;
    a.n_trace = out->d_n_trace;
    a.la_trace = out->d_log_alpha;
    a.summaries = out->d_summaries;
    a.scalars = out->d_scalars ? out->d_scalars : (double *)ws;
    a.ws = ws;
    hipStream_t st = (hipStream_t)stream;
    if (int rc = run_mcmc_poly(a, st)) return rc;
    if (out->sync_host) {
        double h[4];
        PPL_HIP(hipMemcpyAsync(h, a.scalars, sizeof(h), hipMemcpyDeviceToHost, st));
        PPL_HIP(hipStreamSynchronize(st));
        out->accept_rate = h[0];
    }
    return PPL_OK;
}

int ppl_enumerate(int model, const ppl_data *data, void *ws, size_t ws_bytes, void *stream, ppl_enum_result *out) {
    clear_error();
    if (!out) return fail(PPL_E_ARG, "out is NULL");
    if (model != PPL_MODEL_HMM) return fail(PPL_E_MODEL, "enumeration supports HMM (got %d)", model);
    EnumArgs a{};
    if (int rc = check_hmm(data, a)) return rc;
    if (int rc = check_ws(ws, ws_bytes, enum_ws_bytes(a.K, a.T))) return rc;
    if (int rc = check_device()) return rc;
    a.scalars = out->d_scalars ? out->d_scalars : (double *)ws;
    a.marginals = out->d_marginals;
    a.map = out->d_map;
    a.ws = ws;
    hipStream_t st = (hipStream_t)stream;
    if (int rc = run_enumerate_hmm(a, st)) return rc;
    if (out->sync_host) {
        double h[4];
        PPL_HIP(hipMemcpyAsync(h, a.scalars, sizeof(h), hipMemcpyDeviceToHost, st));
        PPL_HIP(hipStreamSynchronize(st));
        out->log_evidence = h[0];
        out->map_log_joint = h[2];
        out->status = (int32_t)h[3];
        if (out->status) return fail(out->status, "device reported status %d (%s)", out->status, ppl_status_string(out->status));
    }
    return PPL_OK;
}

// ------------------------------------------------------------ batched SMC --
namespace {
// Base configurations the autotuner times, each with the smallest team that
// holds the largest instance and with twice that (fewer, wider teams).
const ppl_tune kBaseCandidates[] = {
    {4, 0, 64, 0}, {4, 0, 128, 0}, {4, 0, 256, 0}, {2, 0, 64, 0}, {2, 0, 128, 0}, {8, 0, 64, 0}, {8, 0, 128, 0},
    {8, 0, 256, 0}, {1, 0, 64, 0}, {4, 0, 16, 0},
};

std::vector<ppl_tune> tuner_candidates(int n, const ppl_instance *h) {
    int64_t nmax = 1;
    for (int i = 0; i < n; ++i) nmax = std::max<int64_t>(nmax, h[i].n_particles);
    std::vector<ppl_tune> out;
    for (const ppl_tune &b : kBaseCandidates) {
        const int64_t need = (nmax + 512LL * b.particles_per_lane - 1) / (512LL * b.particles_per_lane);
        for (int64_t w : {need, 2 * need})
            if (w <= 64) out.push_back(ppl_tune{b.particles_per_lane, (int32_t)w, b.spec_block, 0});
    }
    return out;
}

struct BatchKey {
    int n;
    int64_t sum_n, sum_d, max_n, moves;    // moves: sum of move steps x data x K (resample-move work)
    bool operator<(const BatchKey &o) const {
        return std::tie(n, sum_n, sum_d, max_n, moves) < std::tie(o.n, o.sum_n, o.sum_d, o.max_n, o.moves);
    }
};
std::mutex g_tune_mu;
std::map<BatchKey, ppl_tune> g_tune_cache;
std::string g_cache_loaded_from;   // the cache file merged into g_tune_cache ("" = none yet)

BatchKey batch_key(int n, const ppl_instance *h) {
    BatchKey k{n, 0, 0, 0, 0};
    for (int i = 0; i < n; ++i) {
        k.sum_n += h[i].n_particles;
        k.sum_d += h[i].n_data * h[i].dim;
        k.max_n = std::max<int64_t>(k.max_n, h[i].n_particles);
        k.moves += (int64_t)h[i].move_steps * h[i].n_data * h[i].dim;
    }
    return k;
}

// The persisted cache: when PPL_TUNE_CACHE names a file, every autotuner
// result is appended to it as one line
//   ppl-tune <arch> <CUs> <n> <sum N> <sum D K> <max N> <sum M D K> <P> <W> <B>
// and lines for the current device (architecture and CU count) are merged
// into the in-memory cache the first time a lookup sees that file.  Lines
// that do not parse are skipped; a file that cannot be read or written is
// treated as absent (the cache only saves tuning time).
bool device_tag(std::string &arch, int &cus) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    cus = prop.multiProcessorCount;
    return true;
}

void cache_merge_file_locked() {
    const char *path = getenv("PPL_TUNE_CACHE");
    if (!path || !*path || g_cache_loaded_from == path) return;
    g_cache_loaded_from = path;
    std::string arch;
    int cus = 0;
    if (!device_tag(arch, cus)) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char line[512], a[128];
    while (fgets(line, sizeof line, f)) {
        int c = 0, n = 0, P = 0, W = 0, B = 0;
        long long sn = 0, sd = 0, mn = 0, mv = 0;
        if (sscanf(line, "ppl-tune %127s %d %d %lld %lld %lld %lld %d %d %d", a, &c, &n, &sn, &sd, &mn, &mv, &P, &W,
                   &B) != 10)
            continue;
        if (arch != a || c != cus) continue;
        g_tune_cache[BatchKey{n, sn, sd, mn, mv}] = ppl_tune{P, W, B, 0};
    }
    fclose(f);
}

void cache_store_locked(const BatchKey &k, const ppl_tune &t) {
    g_tune_cache[k] = t;
    const char *path = getenv("PPL_TUNE_CACHE");
    if (!path || !*path) return;
    std::string arch;
    int cus = 0;
    if (!device_tag(arch, cus)) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "ppl-tune %s %d %d %lld %lld %lld %lld %d %d %d\n", arch.c_str(), cus, k.n, (long long)k.sum_n,
            (long long)k.sum_d, (long long)k.max_n, (long long)k.moves, t.particles_per_lane, t.wgs_per_instance,
            t.spec_block);
    fclose(f);
}

bool cache_lookup(int n, const ppl_instance *h, ppl_tune &out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    cache_merge_file_locked();
    auto it = g_tune_cache.find(batch_key(n, h));
    if (it == g_tune_cache.end()) return false;
    out = it->second;
    return true;
}

int check_batch_args(int model, int32_t n, const ppl_instance *h, const ppl_instance *d, double ess_frac) {
    if (int rc = bt_check(model, n, h)) return rc;
    if (!d) return fail(PPL_E_ARG, "device instance table is NULL");
    if (!(ess_frac >= 0.0 && ess_frac <= 1.0)) return fail(PPL_E_ARG, "ess_frac must be in [0, 1]");
    return PPL_OK;
}
}  // namespace

int ppl_smc_batched_workspace_size(int model, int32_t n, const ppl_instance *h, const ppl_tune *tune, size_t *bytes) {
    clear_error();
    if (!bytes) return fail(PPL_E_ARG, "bytes is NULL");
    if (int rc = bt_check(model, n, h)) return rc;
    size_t need = 0;
    if (tune) {
        need = bt_ws_bytes_for(h, n, tune);
        if (!need) return fail(PPL_E_ARG, "configuration does not fit these instances");
    } else {
        need = bt_ws_bytes_for(h, n, nullptr);
        for (const ppl_tune &c : tuner_candidates(n, h)) need = std::max(need, bt_ws_bytes_for(h, n, &c));
        if (!need) return fail(PPL_E_UNSUPPORTED, "no configuration fits these instances");
    }
    *bytes = need;
    return PPL_OK;
}

int ppl_smc_batched(int model, int32_t n, const ppl_instance *h, const ppl_instance *d, uint64_t seed,
                    double ess_frac, const ppl_tune *tune, void *ws, size_t ws_bytes, void *stream,
                    ppl_batch_result *out) {
    clear_error();
    if (!out) return fail(PPL_E_ARG, "out is NULL");
    if (int rc = check_batch_args(model, n, h, d, ess_frac)) return rc;
    ppl_tune cached{};
    if (!tune && cache_lookup(n, h, cached)) tune = &cached;
    const size_t need = bt_ws_bytes_for(h, n, tune);
    if (!need) return fail(PPL_E_ARG, "configuration does not fit these instances");
    if (int rc = check_ws(ws, ws_bytes, need)) return rc;
    if (int rc = check_device()) return rc;
    return run_smc_batched(n, h, d, seed, ess_frac, tune, ws, ws_bytes, (hipStream_t)stream, *out, nullptr);
}

int ppl_smc_autotune(int model, int32_t n, const ppl_instance *h, const ppl_instance *d, uint64_t seed,
                     double ess_frac, void *ws, size_t ws_bytes, void *stream, ppl_batch_result *out,
                     ppl_tune *best) {
    clear_error();
    if (!out || !best) return fail(PPL_E_ARG, "out and best must be non-NULL");
    if (int rc = check_batch_args(model, n, h, d, ess_frac)) return rc;
    if (int rc = check_ws(ws, ws_bytes, 256)) return rc;
    if (int rc = check_device()) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    PPL_HIP(hipEventCreate(&e0));
    PPL_HIP(hipEventCreate(&e1));
    float best_ms = -1.0f;
    ppl_tune best_cfg{};
    int rc = PPL_OK;
    const std::vector<ppl_tune> cands = tuner_candidates(n, h);
    for (size_t c = 0; c < cands.size() && rc == PPL_OK; ++c) {
        const size_t need = bt_ws_bytes_for(h, n, &cands[c]);
        if (!need || need > ws_bytes) continue;
        ppl_tune used{};
        rc = run_smc_batched(n, h, d, seed, ess_frac, &cands[c], ws, ws_bytes, st, *out, &used);
        if (rc == PPL_E_UNSUPPORTED || rc == PPL_E_ARG) { rc = PPL_OK; clear_error(); continue; }   // does not fit
        if (rc) break;
        if (hipEventRecord(e0, st) != hipSuccess) { rc = fail(PPL_E_HIP, "hipEventRecord failed"); break; }
        rc = run_smc_batched(n, h, d, seed, ess_frac, &cands[c], ws, ws_bytes, st, *out, &used);
        if (rc) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = fail(PPL_E_HIP, "autotune timing failed");
            break;
        }
        if (best_ms < 0.0f || ms < best_ms) {
            best_ms = ms;
            best_cfg = used;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (best_ms < 0.0f) return fail(PPL_E_UNSUPPORTED, "no candidate configuration fits the workspace and device");
    *best = best_cfg;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    cache_store_locked(batch_key(n, h), best_cfg);
    return PPL_OK;
}

int ppl_smc_tune_lookup(int model, int32_t n, const ppl_instance *h, ppl_tune *out) {
    clear_error();
    if (!out) return fail(PPL_E_ARG, "out is NULL");
    if (int rc = bt_check(model, n, h)) return rc;
    if (int rc = check_device()) return rc;
    if (!cache_lookup(n, h, *out)) return fail(PPL_E_UNSUPPORTED, "no tuned configuration for this batch shape");
    return PPL_OK;
}

void ppl_smc_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache.clear();
    g_cache_loaded_from.clear();
}

}  // extern "C"

// ------------------------------------------------------ learned proposal --
namespace ppl {

struct TrainPlan {
    SimSpec sim;
    AdamSpec adam;
    int B;
    int64_t steps;
};

static int check_train(int model, const ppl_train_config *c, TrainPlan *p) {
    if (!c) return fail(PPL_E_ARG, "training configuration is NULL");
    if (model != PPL_MODEL_POLY && model != PPL_MODEL_GMM)
        return fail(PPL_E_MODEL, "the learned proposal supports POLY and GMM (got %d)", model);
    if (c->batch < 64 || c->batch > 65536 || c->batch % 64)
        return fail(PPL_E_ARG, "batch %d must be a multiple of 64 in [64, 65536]", c->batch);
    if (c->n_pairs < 0 || c->n_pairs % c->batch) return fail(PPL_E_ARG, "n_pairs must be a non-negative multiple of batch");
    if (c->n_pairs / c->batch > 0x7fffffffLL) return fail(PPL_E_ARG, "too many training steps");
    if (c->n_hyper < 0 || (c->n_hyper > 0 && !c->hyper)) return fail(PPL_E_ARG, "hyper is NULL with n_hyper > 0");
    auto hy = [&](int i, double d) { return (c->hyper && c->n_hyper > i) ? c->hyper[i] : d; };
    SimSpec &sp = p->sim;
    sp = SimSpec{};
    sp.model = model;
    sp.D = c->n_data;
    if (model == PPL_MODEL_POLY) {
        sp.K = 0;
        sp.hyper[0] = hy(0, 10.0);
        sp.hyper[1] = hy(1, 2.0);
        sp.hyper[2] = hy(2, 5.0);
        sp.hyper[3] = hy(3, 1.0);
        if (!finite_pos(sp.hyper[0]) || !isfinite(sp.hyper[3]) || sp.hyper[3] < 0)
            return fail(PPL_E_ARG, "POLY simulation needs sd > 0 and noise_sd >= 0");
        if (!is_int(sp.hyper[1]) || !is_int(sp.hyper[2]) || sp.hyper[1] < 2 || sp.hyper[2] > 5 || sp.hyper[1] > sp.hyper[2])
            return fail(PPL_E_ARG, "the POLY proposal head covers degrees 2..5 (need 2 <= n_lo <= n_hi <= 5)");
        if (c->n_data < 1 || c->n_data > 0x7fffffffLL) return fail(PPL_E_ARG, "n_data must be in [1, 2^31)");
    } else {
        if (c->dim < 1 || c->dim > 8) return fail(PPL_E_ARG, "GMM K must be in 1..8 (got %d)", c->dim);
        sp.K = c->dim;
        sp.hyper[0] = hy(0, 5.0);
        sp.hyper[1] = hy(1, 1.0);
        if (!finite_pos(sp.hyper[0]) || !finite_pos(sp.hyper[1])) return fail(PPL_E_ARG, "GMM sds must be positive");
        if (c->n_data < 1 || c->n_data > kGmmTrainMaxD)
            return fail(PPL_E_ARG, "GMM n_data must be in [1, %d]", kGmmTrainMaxD);
    }
    AdamSpec &ad = p->adam;
    ad.lr = (float)(c->lr != 0.0 ? c->lr : 1e-3);
    ad.b1 = (float)(c->beta1 != 0.0 ? c->beta1 : 0.9);
    ad.b2 = (float)(c->beta2 != 0.0 ? c->beta2 : 0.999);
    ad.eps = (float)(c->eps != 0.0 ? c->eps : 1e-8);
    if (!(ad.lr > 0) || !(ad.b1 >= 0 && ad.b1 < 1) || !(ad.b2 >= 0 && ad.b2 < 1) || !(ad.eps > 0))
        return fail(PPL_E_ARG, "Adam needs lr > 0, betas in [0, 1) and eps > 0");
    if (c->lr_decay_steps < 0 || !(c->lr_final_frac >= 0.0 && c->lr_final_frac <= 1.0))
        return fail(PPL_E_ARG, "lr_decay_steps must be >= 0 and lr_final_frac in [0, 1]");
    ad.decay_steps = (double)c->lr_decay_steps;
    ad.final_frac = c->lr_final_frac;
    p->B = c->batch;
    p->steps = c->n_pairs / c->batch;
    return PPL_OK;
}

static int check_weights(const void *w) {
    if (!w) return fail(PPL_E_ARG, "d_weights is NULL");
    if (((uintptr_t)w & 255) != 0) return fail(PPL_E_ARG, "d_weights must be 256-byte aligned");
    return PPL_OK;
}

// Forward, head and backward pass of one batch: fused per 32 pairs, or (with
// the environment variable PPL_TRAIN_UNFUSED=1, a checking and timing aid)
// one launch per product; both store the same bits.
static int forward_backward(int model, int K, const MlpView &w, const TrainBufs &b, const AdvanceJob &adv,
                            hipStream_t st) {
    const char *e = getenv("PPL_TRAIN_UNFUSED");
    if (!(e && e[0] == '1')) return launch_fused_pass(model, K, w, b, adv, st);
    if (int rc = launch_forward(w, b, true, st)) return rc;
    if (int rc = launch_head_backward(model, K, w, b, st)) return rc;
    return launch_advance(adv, st);
}

// The network part of one training step, on a batch already simulated into
// b: forward, loss head, backward and the step's bookkeeping, then Adam,
// grouped with the simulation of the next step's batch when there is one.
static int train_body(const TrainPlan &p, uint64_t seed, const MlpView &w, const TrainBufs &b, double *loss_trace,
                      bool next, hipStream_t st) {
    if (int rc = forward_backward(p.sim.model, p.sim.K, w, b, advance_job(w.step, b, p.adam, loss_trace), st))
        return rc;
    if (next) return launch_update_simulate(w, b, p.adam, p.sim, p.B, seed, w.step, st);
    return launch_update(w, b, p.adam, nullptr, st);
}

static int train_first_batch(const TrainPlan &p, uint64_t seed, const MlpView &w, const TrainBufs &b, hipStream_t st) {
    return launch_simulate(p.sim, p.B, seed, w.step, b.x_row, b.x_col, b.theta, nullptr, st);
}

static int train_graph(const TrainPlan &p, uint64_t seed, const MlpView &w, const TrainBufs &b, double *loss_trace,
                       hipStream_t st) {
    hipStream_t cap = nullptr;
    PPL_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int rc = PPL_OK;
    {
        TimingSuspend quiet;
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            rc = fail(PPL_E_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
        } else {
            rc = train_body(p, seed, w, b, loss_trace, true, cap);
            e = hipStreamEndCapture(cap, &graph);
            if (!rc && e != hipSuccess) rc = fail(PPL_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        }
    }
    if (!rc) {
        hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = fail(PPL_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    // the first batch, every step but the last as one graph launch (each also
    // simulating the next batch), then the last step
    if (!rc) rc = train_first_batch(p, seed, w, b, st);
    for (int64_t s = 0; !rc && s + 1 < p.steps; ++s) {
        KernelTimer timer("proposal_train_step", st);
        hipError_t e = hipGraphLaunch(exec, st);
        timer.stop();
        if (e != hipSuccess) rc = fail(PPL_E_HIP, "hipGraphLaunch: %s", hipGetErrorString(e));
    }
    if (!rc) rc = train_body(p, seed, w, b, loss_trace, false, st);
    // the executable graph is released only after its launches have finished
    if (exec) {
        hipError_t e = hipStreamSynchronize(st);
        if (!rc && e != hipSuccess) rc = fail(PPL_E_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
        (void)hipGraphExecDestroy(exec);
    }
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cap);
    return rc;
}

static size_t infer_ws_bytes(int model, int64_t n) {
    return 256 + align_up(train_ws_bytes(64), 256) + 256 * 8 /* decoded q, <= 332 doubles */ * 2 +
           align_up(prop_partial_bytes(model, n), 256);
}

}  // namespace ppl

extern "C" {

size_t ppl_proposal_weights_bytes(void) { return MlpParams::bytes(); }

int ppl_proposal_init(void *d_weights, uint64_t seed, void *stream) {
    clear_error();
    if (int rc = check_weights(d_weights)) return rc;
    if (int rc = check_device()) return rc;
    return launch_init_weights(d_weights, seed, (hipStream_t)stream);
}

int ppl_proposal_train_workspace_size(int model, const ppl_train_config *cfg, size_t *bytes) {
    clear_error();
    if (!bytes) return fail(PPL_E_ARG, "bytes is NULL");
    TrainPlan p;
    if (int rc = check_train(model, cfg, &p)) return rc;
    *bytes = train_ws_bytes(p.B);
    return PPL_OK;
}

int ppl_proposal_train(int model, const ppl_train_config *cfg, uint64_t seed, void *d_weights, double *d_loss_trace,
                       void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    TrainPlan p;
    if (int rc = check_train(model, cfg, &p)) return rc;
    if (int rc = check_weights(d_weights)) return rc;
    if (int rc = check_ws(ws, ws_bytes, train_ws_bytes(p.B))) return rc;
    if (int rc = check_device()) return rc;
    if (p.steps == 0) return PPL_OK;
    hipStream_t st = (hipStream_t)stream;
    const MlpView w = mlp_view(d_weights);
    const TrainBufs b = train_bufs(ws, p.B);
    if (int rc = launch_set_i64(b.local, 0, st)) return rc;
    if (cfg->use_graph && p.steps > 1) return train_graph(p, seed, w, b, d_loss_trace, st);
    if (int rc = train_first_batch(p, seed, w, b, st)) return rc;
    for (int64_t s = 0; s < p.steps; ++s)
        if (int rc = train_body(p, seed, w, b, d_loss_trace, s + 1 < p.steps, st)) return rc;
    return PPL_OK;
}

int ppl_proposal_gradient(int model, const ppl_train_config *cfg, uint64_t seed, uint32_t step, const void *d_weights,
                          float *d_grad, double *d_loss, double *d_summaries, double *d_latents, float *d_outputs,
                          void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    TrainPlan p;
    if (int rc = check_train(model, cfg, &p)) return rc;
    if (int rc = check_weights(d_weights)) return rc;
    if (int rc = check_ws(ws, ws_bytes, train_ws_bytes(p.B))) return rc;
    if (int rc = check_device()) return rc;
    hipStream_t st = (hipStream_t)stream;
    const MlpView w = mlp_view(const_cast<void *>(d_weights));
    const TrainBufs b = train_bufs(ws, p.B);
    if (int rc = launch_set_i64(b.local, 0, st)) return rc;
    if (int rc = launch_set_i64(b.local + 1, (int64_t)step, st)) return rc;
    if (int rc = launch_simulate(p.sim, p.B, seed, b.local + 1, b.x_row, b.x_col, b.theta, d_summaries, st)) return rc;
    if (int rc = forward_backward(model, p.sim.K, w, b, advance_job(nullptr, b, p.adam, d_loss), st)) return rc;
    if (d_grad)
        if (int rc = launch_update(w, b, p.adam, d_grad, st)) return rc;
    if (d_latents)
        PPL_HIP(hipMemcpyAsync(d_latents, b.theta, (size_t)p.B * kThetaStride * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (d_outputs)
        PPL_HIP(hipMemcpyAsync(d_outputs, b.o_col, (size_t)p.B * kMlpOut * sizeof(float), hipMemcpyDeviceToDevice, st));
    return PPL_OK;
}

int ppl_proposal_infer_workspace_size(int model, const ppl_data *data, int64_t n, size_t *bytes) {
    clear_error();
    if (!bytes) return fail(PPL_E_ARG, "bytes is NULL");
    if (model != PPL_MODEL_POLY && model != PPL_MODEL_GMM)
        return fail(PPL_E_MODEL, "the learned proposal supports POLY and GMM (got %d)", model);
    if (int rc = check_n(n)) return rc;
    double h[8];
    if (int rc = check_model_data(model, data, h)) return rc;
    *bytes = infer_ws_bytes(model, n);
    return PPL_OK;
}

int ppl_proposal_infer(int model, const ppl_data *data, const void *d_weights, int64_t n, uint64_t seed, double widen,
                       double *d_q_params, double *d_data_summaries, void *ws, size_t ws_bytes, void *stream,
                       ppl_result *out) {
    clear_error();
    if (!out) return fail(PPL_E_ARG, "out is NULL");
    if (model != PPL_MODEL_POLY && model != PPL_MODEL_GMM)
        return fail(PPL_E_MODEL, "the learned proposal supports POLY and GMM (got %d)", model);
    if (int rc = check_n(n)) return rc;
    IsArgs a{};
    if (int rc = check_model_data(model, data, a.hyper)) return rc;
    if (model == PPL_MODEL_POLY && (a.hyper[1] != 2.0 || a.hyper[2] != 5.0))
        return fail(PPL_E_ARG, "the POLY proposal covers degrees 2..5; the model range must be 2..5");
    if (model == PPL_MODEL_GMM && data->n_data > kGmmSummaryMaxD)
        return fail(PPL_E_ARG, "GMM summaries take at most %d points", kGmmSummaryMaxD);
    if (!(widen >= 1.0 && widen <= 1e3)) return fail(PPL_E_ARG, "widen must be in [1, 1000]");
    if (int rc = check_weights(d_weights)) return rc;
    if (int rc = check_ws(ws, ws_bytes, infer_ws_bytes(model, n))) return rc;
    if (int rc = check_device()) return rc;
    hipStream_t st = (hipStream_t)stream;
    char *base = (char *)ws;
    double *scal = (double *)base;
    const TrainBufs b = train_bufs(base + 256, 64);
    double *q = (double *)(base + 256 + align_up(train_ws_bytes(64), 256));
    double *part = q + 512;
    const MlpView w = mlp_view(const_cast<void *>(d_weights));
    if (int rc = launch_observed_summary(model, data->x, data->y, data->n_data, b.x_row, d_data_summaries, st)) return rc;
    if (int rc = launch_forward(w, b, false, st)) return rc;
    if (int rc = launch_decode(model, data->dim, b.o_col, 64, log(widen), q, st)) return rc;
    const int nq = model == PPL_MODEL_POLY ? kPolyQParams : gmm_q_params(data->dim);
    if (d_q_params) PPL_HIP(hipMemcpyAsync(d_q_params, q, (size_t)nq * sizeof(double), hipMemcpyDeviceToDevice, st));
    a.model = model;
    a.x = data->x;
    a.y = data->y;
    a.D = data->n_data;
    a.dim = data->dim;
    a.N = n;
    a.seed = seed;
    a.q_params = q;
    a.lw_out = out->d_log_weights;
    a.lat_out = out->d_latents;
    a.summaries = out->d_summaries;
    a.scalars = out->d_scalars ? out->d_scalars : scal;
    a.part = part;
    if (int rc = run_importance_q(a, st)) return rc;
    if (out->sync_host) return sync_scalars(out, a.scalars, st);
    return PPL_OK;
}

int ppl_proposal_pick_widen(int model, const ppl_data *data, const void *d_weights, int64_t n_pilot, uint64_t seed,
                            const double *cand, int32_t n_cand, double *best, double *ess_out, void *ws,
                            size_t ws_bytes, void *stream) {
    clear_error();
    if (!cand || !best || n_cand < 1 || n_cand > 16) return fail(PPL_E_ARG, "need 1..16 candidates and a result pointer");
    double ess[16];
    for (int c = 0; c < n_cand; ++c) {
        ppl_result r{};
        r.sync_host = 1;
        if (int rc = ppl_proposal_infer(model, data, d_weights, n_pilot, seed, cand[c], nullptr, nullptr, ws, ws_bytes,
                                        stream, &r))
            return rc;
        ess[c] = r.ess;
    }
    int k = 0;
    for (int c = 1; c < n_cand; ++c)
        if (ess[c] > ess[k]) k = c;
    *best = cand[k];
    if (ess_out)
        for (int c = 0; c < n_cand; ++c) ess_out[c] = ess[c];
    return PPL_OK;
}

}  // extern "C"
