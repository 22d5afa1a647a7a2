"""Python binding of libppl (the MI355X particle-inference library).

Argument marshalling only: every step of inference runs in the library's HIP
kernels.  PyTorch provides device memory (tensors) and streams.  The functions
keep the C names (``ppl_importance``, ``ppl_smc``, ...); outputs and the
workspace may be passed in pre-allocated (as a benchmark does) or are
allocated here with ``torch.empty`` when omitted.

The library must be built first (``__graft_entry__.build()`` or
``python paper_2010_08454_amd/build.py``); importing this module without it
raises, there is no fallback path.
"""
import ctypes
import os

import torch  # loads the HIP runtime torch ships with before libppl binds to it

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libppl.so")

PPL_OK, PPL_E_ARG, PPL_E_MODEL, PPL_E_DEVICE, PPL_E_HIP = 0, -1, -2, -3, -4
PPL_E_WORKSPACE, PPL_E_NONFINITE, PPL_E_ZERO_WEIGHT, PPL_E_UNSUPPORTED = -5, -6, -7, -8
PPL_MODEL_POLY, PPL_MODEL_BLR, PPL_MODEL_LGSSM, PPL_MODEL_GMM = 1, 2, 3, 4
PPL_MODEL_BLR_STATS = 5
PPL_MODEL_HMM = 6
PPL_F32, PPL_F64 = 1, 2
PPL_Q_PRIOR, PPL_Q_GAUSS_FULL, PPL_Q_POLY_MIX, PPL_Q_GMM_MIX = 0, 1, 2, 3
PPL_ALGO_IS, PPL_ALGO_SMC, PPL_ALGO_LSE, PPL_ALGO_RESAMPLE, PPL_ALGO_MCMC, PPL_ALGO_ENUM = 0, 1, 2, 3, 4, 5
PPL_INST_NO_RECORD = 1
PPL_NOALLOC_SCRATCH_BYTES = 16 << 20

# Exported C symbols (kept in step with include/ppl.h).
EXPORTS = ("ppl_status_string", "ppl_last_error", "ppl_version", "ppl_workspace_size",
           "ppl_importance", "ppl_importance_noalloc", "ppl_lse_ess", "ppl_resample", "ppl_resample_gather", "ppl_philox", "ppl_smc",
           "ppl_smc_ex", "ppl_smc_checkpoint_bytes", "ppl_mcmc", "ppl_enumerate",
           "ppl_timing_enable", "ppl_timing_query")

P = ctypes.c_void_p


class PplData(ctypes.Structure):
    _fields_ = [("x", P), ("y", P), ("n_data", ctypes.c_int64), ("dim", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("hyper", ctypes.POINTER(ctypes.c_double)),
                ("n_hyper", ctypes.c_int32)]


class PplResult(ctypes.Structure):
    _fields_ = [("log_evidence", ctypes.c_double), ("ess", ctypes.c_double),
                ("n_resample", ctypes.c_int64), ("status", ctypes.c_int32), ("sync_host", ctypes.c_int32),
                ("d_scalars", P), ("d_latents", P), ("d_log_weights", P), ("d_summaries", P),
                ("d_ess_trace", P), ("d_resampled", P), ("d_ancestors", P), ("max_events", ctypes.c_int64),
                ("d_event_lw", P), ("d_logz_trace", P), ("d_move_log_alpha", P)]


class PplProposal(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dim", ctypes.c_int32), ("d_params", P)]


class PplSmcOptions(ctypes.Structure):
    _fields_ = [("ess_frac", ctypes.c_double), ("move_steps", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("move_scale", ctypes.c_double), ("t_begin", ctypes.c_int64), ("t_end", ctypes.c_int64),
                ("d_checkpoint", P)]


class PplMcmcResult(ctypes.Structure):
    _fields_ = [("accept_rate", ctypes.c_double), ("sync_host", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("d_scalars", P), ("d_state", P), ("d_accepts", P), ("d_summaries", P), ("d_n_trace", P),
                ("d_log_alpha", P)]


class PplEnumResult(ctypes.Structure):
    _fields_ = [("log_evidence", ctypes.c_double), ("map_log_joint", ctypes.c_double), ("status", ctypes.c_int32),
                ("sync_host", ctypes.c_int32), ("d_scalars", P), ("d_marginals", P), ("d_map", P)]


class PplError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libppl error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, u32, u64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
    L.ppl_status_string.argtypes = [ctypes.c_int]
    L.ppl_status_string.restype = ctypes.c_char_p
    L.ppl_last_error.restype = ctypes.c_char_p
    L.ppl_version.restype = ctypes.c_int
    L.ppl_workspace_size.argtypes = [ctypes.c_int, ctypes.POINTER(PplData), i64, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    L.ppl_importance.argtypes = [ctypes.c_int, ctypes.POINTER(PplData), i64, u64, ctypes.POINTER(PplProposal),
                                 P, ctypes.c_size_t, P, ctypes.POINTER(PplResult)]
    L.ppl_lse_ess.argtypes = [P, ctypes.c_int, i64, P, P, ctypes.c_size_t, P]
    L.ppl_resample.argtypes = [P, ctypes.c_int, i64, u64, u32, u32, P, P, ctypes.c_size_t, P]
    L.ppl_resample_gather.argtypes = [P, ctypes.c_int, i64, u64, u32, u32, i32, P, P, P, P, ctypes.c_size_t, P]
    L.ppl_philox.argtypes = [u64, u32, u32, u32, i64, P, P]
    L.ppl_smc.argtypes = [ctypes.c_int, ctypes.POINTER(PplData), i64, u64, f64, P, ctypes.c_size_t, P,
                          ctypes.POINTER(PplResult)]
    L.ppl_mcmc.argtypes = [ctypes.c_int, ctypes.POINTER(PplData), i64, i64, i64, u64, P, ctypes.c_size_t, P,
                           ctypes.POINTER(PplMcmcResult)]
    L.ppl_smc_checkpoint_bytes.argtypes = [ctypes.c_int, ctypes.POINTER(PplData), i64, ctypes.POINTER(ctypes.c_size_t)]
    L.ppl_enumerate.argtypes = [ctypes.c_int, ctypes.POINTER(PplData), P, ctypes.c_size_t, P,
                                ctypes.POINTER(PplEnumResult)]
    L.ppl_smc_ex.argtypes = [ctypes.c_int, ctypes.POINTER(PplData), i64, u64, ctypes.POINTER(PplSmcOptions), P,
                             ctypes.c_size_t, P, ctypes.POINTER(PplResult)]
    L.ppl_importance_noalloc.argtypes = [ctypes.c_int, ctypes.POINTER(PplData), i64, u64,
                                         ctypes.POINTER(PplProposal), P, ctypes.POINTER(PplResult)]
    L.ppl_timing_enable.argtypes = [ctypes.c_int]
    L.ppl_timing_query.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    for name in EXPORTS:
        if name not in ("ppl_status_string", "ppl_last_error"):
            getattr(L, name).restype = ctypes.c_int
    return L


lib = _load()


def _check(rc):
    if rc != PPL_OK:
        raise PplError(rc, lib.ppl_last_error().decode())
    return rc


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_data(x, y, n_data=None, dim=0, hyper=None, dtype=None):
    """Build a ppl_data block from device tensors; the block holds references to
    x, y and the hyper array so they outlive every call that uses it."""
    if dtype is None:
        dtype = PPL_F64 if y.dtype == torch.float64 else PPL_F32
    h = None
    if hyper is not None:
        h = (ctypes.c_double * len(hyper))(*[float(v) for v in hyper])
    d = PplData(x=None if x is None else x.data_ptr(), y=None if y is None else y.data_ptr(),
                n_data=int(y.numel() if n_data is None else n_data), dim=int(dim), dtype=dtype,
                hyper=ctypes.cast(h, ctypes.POINTER(ctypes.c_double)) if h is not None else None,
                n_hyper=0 if hyper is None else len(hyper))
    d._keep = (h, x, y)
    return d


def ppl_workspace_size(model, data, n, algo):
    b = ctypes.c_size_t()
    _check(lib.ppl_workspace_size(model, ctypes.byref(data) if data is not None else None, int(n), algo, ctypes.byref(b)))
    return b.value


def workspace(nbytes, device=None):
    """Caller-owned device workspace (256-byte aligned: the allocator aligns to 512)."""
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device or "cuda")


def _q_dim(kind, data):
    if kind == PPL_Q_POLY_MIX:
        return 5
    if kind == PPL_Q_GMM_MIX:
        return 2 * data.dim - 1
    return data.dim


def ppl_importance(model, data, n, seed, q=None, ws=None, stream=None, log_weights=None, latents=None,
                   summaries=None, scalars=None, sync=False, q_kind=None):
    """Importance sampling; returns the ppl_result struct (host scalars when sync).
    q: device parameter tensor of the proposal, of kind q_kind (default: the
    BLR full Gaussian)."""
    if ws is None:
        ws = workspace(ppl_workspace_size(model, data, n, PPL_ALGO_IS))
    res = PplResult(sync_host=1 if sync else 0, d_scalars=_ptr(scalars), d_latents=_ptr(latents),
                    d_log_weights=_ptr(log_weights), d_summaries=_ptr(summaries))
    prop = None
    if q is not None:
        kind = PPL_Q_GAUSS_FULL if q_kind is None else q_kind
        prop = PplProposal(kind=kind, dim=_q_dim(kind, data), d_params=q.data_ptr())
    _check(lib.ppl_importance(model, ctypes.byref(data), int(n), int(seed) & (2 ** 64 - 1),
                              ctypes.byref(prop) if prop is not None else None, _ptr(ws), ws.numel(),
                              _stream(stream), ctypes.byref(res)))
    return res


def ppl_importance_noalloc(model, data, n, seed, q=None, stream=None, log_weights=None, latents=None,
                           summaries=None, scalars=None, sync=False, q_kind=None):
    """Importance sampling on the library's fixed scratch (no workspace argument, nothing allocated)."""
    res = PplResult(sync_host=1 if sync else 0, d_scalars=_ptr(scalars), d_latents=_ptr(latents),
                    d_log_weights=_ptr(log_weights), d_summaries=_ptr(summaries))
    prop = None
    if q is not None:
        kind = PPL_Q_GAUSS_FULL if q_kind is None else q_kind
        prop = PplProposal(kind=kind, dim=_q_dim(kind, data), d_params=q.data_ptr())
    _check(lib.ppl_importance_noalloc(model, ctypes.byref(data), int(n), int(seed) & (2 ** 64 - 1),
                                      ctypes.byref(prop) if prop is not None else None, _stream(stream),
                                      ctypes.byref(res)))
    return res


def ppl_lse_ess(lw, out=None, ws=None, stream=None):
    """FP64 {max, s1, s2, LSE, ESS} of a device log-weight vector (returns the device tensor)."""
    n = lw.numel()
    if out is None:
        out = torch.empty(5, dtype=torch.float64, device=lw.device)
    if ws is None:
        ws = workspace(ppl_workspace_size(0, None, n, PPL_ALGO_LSE), lw.device)
    dt = PPL_F64 if lw.dtype == torch.float64 else PPL_F32
    _check(lib.ppl_lse_ess(_ptr(lw), dt, n, _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def ppl_resample(lw, seed, step=0, inst=0, anc=None, ws=None, stream=None):
    """Integer-rule systematic resampling; returns the int32 ancestor tensor."""
    n = lw.numel()
    if anc is None:
        anc = torch.empty(n, dtype=torch.int32, device=lw.device)
    if ws is None:
        ws = workspace(ppl_workspace_size(0, None, n, PPL_ALGO_RESAMPLE), lw.device)
    dt = PPL_F64 if lw.dtype == torch.float64 else PPL_F32
    _check(lib.ppl_resample(_ptr(lw), dt, n, int(seed) & (2 ** 64 - 1), step, inst, _ptr(anc), _ptr(ws),
                            ws.numel(), _stream(stream)))
    return anc


def ppl_resample_gather(lw, state, seed, step=0, inst=0, out=None, anc=None, ws=None, stream=None):
    """Resampling fused with the gather of structure-of-arrays state [F][n] of
    32-bit words; returns the gathered state (and fills anc when given)."""
    n = lw.numel()
    if state.dim() != 2 or state.shape[1] != n or state.element_size() != 4 or not state.is_contiguous():
        raise ValueError("state must be a contiguous [F, n] tensor of 32-bit words")
    if out is None:
        out = torch.empty_like(state)
    if ws is None:
        ws = workspace(ppl_workspace_size(0, None, n, PPL_ALGO_RESAMPLE), lw.device)
    dt = PPL_F64 if lw.dtype == torch.float64 else PPL_F32
    _check(lib.ppl_resample_gather(_ptr(lw), dt, n, int(seed) & (2 ** 64 - 1), step, inst, state.shape[0],
                                   _ptr(state), _ptr(out), _ptr(anc), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def ppl_philox(seed, c1, c2, c3, n, out=None, stream=None):
    """Philox4x32-10 words of blocks (i, c1, c2, c3), i < n, as an int32 tensor [n, 4]."""
    if out is None:
        out = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    _check(lib.ppl_philox(int(seed) & (2 ** 64 - 1), c1, c2, c3, n, _ptr(out), _stream(stream)))
    return out


def ppl_smc(model, data, n, seed, ess_frac=0.5, ws=None, stream=None, log_weights=None, latents=None,
            scalars=None, ess_trace=None, resampled=None, ancestors=None, sync=False, event_lw=None,
            logz_trace=None, move_steps=0, move_scale=0.0, move_log_alpha=None, t_begin=0, t_end=0,
            checkpoint=None):
    """Sequential Monte Carlo (ppl_smc_ex); returns the ppl_result struct (host
    scalars when sync).  ancestors / event_lw: [max_events, n] and
    move_log_alpha: [max_events, move_steps, n] records of the first
    resampling events.  move_steps > 0: resample-move (mixture model).
    t_begin / t_end / checkpoint: run factors [t_begin, t_end) only, resuming
    from and stopping into the checkpoint (ppl_smc_checkpoint_bytes)."""
    if ws is None:
        ws = workspace(ppl_workspace_size(model, data, n, PPL_ALGO_SMC))
    rec = next((t for t in (ancestors, event_lw, move_log_alpha) if t is not None), None)
    res = PplResult(sync_host=1 if sync else 0, d_scalars=_ptr(scalars), d_latents=_ptr(latents),
                    d_log_weights=_ptr(log_weights), d_ess_trace=_ptr(ess_trace), d_resampled=_ptr(resampled),
                    d_ancestors=_ptr(ancestors), max_events=0 if rec is None else rec.shape[0],
                    d_event_lw=_ptr(event_lw), d_logz_trace=_ptr(logz_trace), d_move_log_alpha=_ptr(move_log_alpha))
    opt = PplSmcOptions(ess_frac=float(ess_frac), move_steps=int(move_steps), move_scale=float(move_scale),
                        t_begin=int(t_begin), t_end=int(t_end), d_checkpoint=_ptr(checkpoint))
    _check(lib.ppl_smc_ex(model, ctypes.byref(data), int(n), int(seed) & (2 ** 64 - 1), ctypes.byref(opt), _ptr(ws),
                          ws.numel(), _stream(stream), ctypes.byref(res)))
    return res


def ppl_smc_checkpoint_bytes(model, data, n):
    b = ctypes.c_size_t()
    _check(lib.ppl_smc_checkpoint_bytes(model, ctypes.byref(data), int(n), ctypes.byref(b)))
    return b.value


def ppl_mcmc(model, data, n_chains, n_iters, seed, burn_in=0, ws=None, stream=None, state=None, accepts=None,
             summaries=None, scalars=None, n_trace=None, log_alpha=None, sync=False):
    """Lightweight Metropolis-Hastings chains; returns the ppl_mcmc_result struct."""
    if ws is None:
        ws = workspace(ppl_workspace_size(model, data, n_chains, PPL_ALGO_MCMC))
    res = PplMcmcResult(sync_host=1 if sync else 0, d_scalars=_ptr(scalars), d_state=_ptr(state),
                        d_accepts=_ptr(accepts), d_summaries=_ptr(summaries), d_n_trace=_ptr(n_trace),
                        d_log_alpha=_ptr(log_alpha))
    _check(lib.ppl_mcmc(model, ctypes.byref(data), int(n_chains), int(n_iters), int(burn_in),
                        int(seed) & (2 ** 64 - 1), _ptr(ws), ws.numel(), _stream(stream), ctypes.byref(res)))
    return res


def hmm_data(y, pi0, A, mu, sigma=1.0):
    """ppl_data of the hidden Markov model: y a float64 device tensor [T];
    hyper = {K, sigma, pi0, A (row = previous state), mu}."""
    K = len(pi0)
    hyper = [K, sigma] + [float(v) for v in pi0] + [float(v) for row in A for v in row] + [float(v) for v in mu]
    return make_data(None, y, dim=K, hyper=hyper, dtype=PPL_F64)


def ppl_enumerate(model, data, ws=None, stream=None, scalars=None, marginals=None, map_path=None, sync=False):
    """Exact inference by enumerating every path; returns the ppl_enum_result struct."""
    if ws is None:
        ws = workspace(ppl_workspace_size(model, data, 1, PPL_ALGO_ENUM))
    res = PplEnumResult(sync_host=1 if sync else 0, d_scalars=_ptr(scalars), d_marginals=_ptr(marginals),
                        d_map=_ptr(map_path))
    _check(lib.ppl_enumerate(model, ctypes.byref(data), _ptr(ws), ws.numel(), _stream(stream), ctypes.byref(res)))
    return res


def ppl_timing_enable(on):
    """Start (clearing the accumulators) or stop event timing of the library's dominant kernels."""
    _check(lib.ppl_timing_enable(1 if on else 0))


def ppl_timing_query(kernel):
    """(total milliseconds, launches) recorded for ``kernel`` since timing was enabled."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib.ppl_timing_query(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


# ----------------------------------------------------------- batched SMC --
class PplInstance(ctypes.Structure):
    _fields_ = [("y", P), ("n_data", ctypes.c_int64), ("n_particles", ctypes.c_int64), ("dim", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("hyper", ctypes.c_double * 2), ("move_steps", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("move_scale", ctypes.c_double)]


class PplTune(ctypes.Structure):
    _fields_ = [("particles_per_lane", ctypes.c_int32), ("wgs_per_instance", ctypes.c_int32),
                ("spec_block", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class PplBatchResult(ctypes.Structure):
    _fields_ = [("d_out", P), ("d_log_weights", P), ("d_latents", P), ("d_ess_trace", P), ("d_resampled", P),
                ("d_ancestors", P), ("max_events", ctypes.c_int64), ("d_event_lw", P), ("d_logz_trace", P),
                ("d_move_log_alpha", P), ("d_counters", P)]


def _bind_batched():
    L = lib
    L.ppl_smc_batched_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int32, ctypes.POINTER(PplInstance),
                                                 ctypes.POINTER(PplTune), ctypes.POINTER(ctypes.c_size_t)]
    L.ppl_smc_batched.argtypes = [ctypes.c_int, ctypes.c_int32, ctypes.POINTER(PplInstance), P, ctypes.c_uint64,
                                  ctypes.c_double, ctypes.POINTER(PplTune), P, ctypes.c_size_t, P,
                                  ctypes.POINTER(PplBatchResult)]
    L.ppl_smc_autotune.argtypes = [ctypes.c_int, ctypes.c_int32, ctypes.POINTER(PplInstance), P, ctypes.c_uint64,
                                   ctypes.c_double, P, ctypes.c_size_t, P, ctypes.POINTER(PplBatchResult),
                                   ctypes.POINTER(PplTune)]
    L.ppl_smc_tune_lookup.argtypes = [ctypes.c_int, ctypes.c_int32, ctypes.POINTER(PplInstance),
                                      ctypes.POINTER(PplTune)]
    L.ppl_smc_tune_cache_clear.argtypes = []
    L.ppl_smc_tune_cache_clear.restype = None
    for n in ("ppl_smc_batched_workspace_size", "ppl_smc_batched", "ppl_smc_autotune", "ppl_smc_tune_lookup"):
        getattr(L, n).restype = ctypes.c_int


_bind_batched()
EXPORTS = EXPORTS + ("ppl_smc_batched_workspace_size", "ppl_smc_batched", "ppl_smc_autotune", "ppl_smc_tune_lookup",
                     "ppl_smc_tune_cache_clear")


class InstanceTable:
    """Host and device copies of a ppl_instance table (the device copy holds the same bytes)."""

    def __init__(self, ys, ks, n_particles, hypers=None, device="cuda", record=None, move_steps=0, move_scale=0.0):
        """record: optional list of instance indices whose resampling events are
        recorded (the others get PPL_INST_NO_RECORD); None records every instance.
        move_steps: resample-move steps (one value for all instances or a list)."""
        n = len(ys)
        rec = set(range(n)) if record is None else set(int(i) for i in record)
        self.host = (PplInstance * n)()
        self._ys = ys                                  # keep the device observation tensors alive
        for i, (y, k) in enumerate(zip(ys, ks)):
            h = hypers[i] if hypers is not None else (0.0, 0.0)
            np_ = n_particles[i] if hasattr(n_particles, "__len__") else n_particles
            self.host[i] = PplInstance(y=y.data_ptr() if y.numel() else None, n_data=y.numel(), n_particles=int(np_),
                                       dim=int(k), flags=0 if i in rec else PPL_INST_NO_RECORD,
                                       hyper=(ctypes.c_double * 2)(*h),
                                       move_steps=int(move_steps[i] if hasattr(move_steps, "__len__") else move_steps),
                                       move_scale=float(move_scale))
        raw = bytes(self.host)
        self.device = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)
        self.n = n

    @property
    def n_particles(self):
        return [self.host[i].n_particles for i in range(self.n)]

    @property
    def n_data(self):
        return [self.host[i].n_data for i in range(self.n)]


def _tune_ptr(tune):
    if tune is None:
        return None, None
    t = PplTune(*[int(v) for v in tune]) if not isinstance(tune, PplTune) else tune
    return ctypes.byref(t), t


def ppl_smc_batched_workspace_size(model, table, tune=None):
    b = ctypes.c_size_t()
    tp, _keep = _tune_ptr(tune)
    _check(lib.ppl_smc_batched_workspace_size(model, table.n, table.host, tp, ctypes.byref(b)))
    return b.value


def ppl_smc_batched(model, table, seed, ess_frac=0.5, tune=None, ws=None, stream=None, out=None, log_weights=None,
                    latents=None, ess_trace=None, resampled=None, ancestors=None, max_events=0, event_lw=None,
                    logz_trace=None, move_log_alpha=None, counters=None):
    """Batched SMC; returns the [n_inst, 4] FP64 device tensor (log Z, ESS, resamplings, status).
    counters (int64 [4], optional): particle-factors in first passes, particle-factors recomputed,
    speculative blocks, resampling events."""
    if ws is None:
        ws = workspace(ppl_smc_batched_workspace_size(model, table, tune))
    if out is None:
        out = torch.empty((table.n, 4), dtype=torch.float64, device=ws.device)
    res = PplBatchResult(d_out=_ptr(out), d_log_weights=_ptr(log_weights), d_latents=_ptr(latents),
                         d_ess_trace=_ptr(ess_trace), d_resampled=_ptr(resampled), d_ancestors=_ptr(ancestors),
                         max_events=int(max_events) if any(t is not None for t in (ancestors, event_lw, move_log_alpha))
                         else 0, d_event_lw=_ptr(event_lw), d_logz_trace=_ptr(logz_trace),
                         d_move_log_alpha=_ptr(move_log_alpha), d_counters=_ptr(counters))
    tp, _keep = _tune_ptr(tune)
    _check(lib.ppl_smc_batched(model, table.n, table.host, _ptr(table.device), int(seed) & (2 ** 64 - 1),
                               float(ess_frac), tp, _ptr(ws), ws.numel(), _stream(stream), ctypes.byref(res)))
    return out


def ppl_smc_autotune(model, table, seed, ess_frac=0.5, ws=None, stream=None, out=None):
    """Times the candidate configurations on this batch; returns the chosen (P, W, spec_block)."""
    if ws is None:
        ws = workspace(ppl_smc_batched_workspace_size(model, table, None))
    if out is None:
        out = torch.empty((table.n, 4), dtype=torch.float64, device=ws.device)
    res = PplBatchResult(d_out=_ptr(out))
    best = PplTune()
    _check(lib.ppl_smc_autotune(model, table.n, table.host, _ptr(table.device), int(seed) & (2 ** 64 - 1),
                                float(ess_frac), _ptr(ws), ws.numel(), _stream(stream), ctypes.byref(res),
                                ctypes.byref(best)))
    return (best.particles_per_lane, best.wgs_per_instance, best.spec_block)


def ppl_smc_tune_lookup(model, table):
    """The (P, W, spec_block) a tune=None call would use, or None if the batch shape has no tuned entry."""
    t = PplTune()
    rc = lib.ppl_smc_tune_lookup(model, table.n, table.host, ctypes.byref(t))
    if rc == PPL_E_UNSUPPORTED:
        return None
    _check(rc)
    return (t.particles_per_lane, t.wgs_per_instance, t.spec_block)


def ppl_smc_tune_cache_clear():
    lib.ppl_smc_tune_cache_clear()


# ------------------------------------------------------- learned proposal --
class PplTrainConfig(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_int64), ("batch", ctypes.c_int32), ("dim", ctypes.c_int32),
                ("n_data", ctypes.c_int64), ("lr", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double), ("hyper", ctypes.POINTER(ctypes.c_double)),
                ("n_hyper", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("lr_decay_steps", ctypes.c_int64), ("lr_final_frac", ctypes.c_double)]


def train_config(n_pairs, batch, n_data, dim=0, lr=0.0, beta1=0.0, beta2=0.0, eps=0.0, hyper=None, use_graph=False,
                 lr_decay_steps=0, lr_final_frac=0.0):
    """Build a ppl_train_config (keeps the hyper array alive)."""
    h = None
    if hyper is not None:
        h = (ctypes.c_double * len(hyper))(*[float(v) for v in hyper])
    c = PplTrainConfig(n_pairs=int(n_pairs), batch=int(batch), dim=int(dim), n_data=int(n_data), lr=float(lr),
                       beta1=float(beta1), beta2=float(beta2), eps=float(eps),
                       hyper=ctypes.cast(h, ctypes.POINTER(ctypes.c_double)) if h is not None else None,
                       n_hyper=0 if hyper is None else len(hyper), use_graph=1 if use_graph else 0,
                       lr_decay_steps=int(lr_decay_steps), lr_final_frac=float(lr_final_frac))
    c._keep = h
    return c


def _bind_proposal():
    L, i32, i64, u32, u64 = lib, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    cfg, sz = ctypes.POINTER(PplTrainConfig), ctypes.c_size_t
    L.ppl_proposal_weights_bytes.argtypes = []
    L.ppl_proposal_weights_bytes.restype = sz
    L.ppl_proposal_init.argtypes = [P, u64, P]
    L.ppl_proposal_train_workspace_size.argtypes = [ctypes.c_int, cfg, ctypes.POINTER(sz)]
    L.ppl_proposal_train.argtypes = [ctypes.c_int, cfg, u64, P, P, P, sz, P]
    L.ppl_proposal_gradient.argtypes = [ctypes.c_int, cfg, u64, u32, P, P, P, P, P, P, P, sz, P]
    L.ppl_proposal_infer_workspace_size.argtypes = [ctypes.c_int, ctypes.POINTER(PplData), i64, ctypes.POINTER(sz)]
    L.ppl_proposal_infer.argtypes = [ctypes.c_int, ctypes.POINTER(PplData), P, i64, u64, ctypes.c_double, P, P, P,
                                     sz, P, ctypes.POINTER(PplResult)]
    L.ppl_proposal_pick_widen.argtypes = [ctypes.c_int, ctypes.POINTER(PplData), P, i64, u64,
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), P, sz, P]
    for n in ("ppl_proposal_init", "ppl_proposal_train_workspace_size", "ppl_proposal_train",
              "ppl_proposal_gradient", "ppl_proposal_infer_workspace_size", "ppl_proposal_infer",
              "ppl_proposal_pick_widen"):
        getattr(L, n).restype = ctypes.c_int


_bind_proposal()
EXPORTS = EXPORTS + ("ppl_proposal_weights_bytes", "ppl_proposal_init", "ppl_proposal_train_workspace_size",
                     "ppl_proposal_train", "ppl_proposal_gradient", "ppl_proposal_infer_workspace_size",
                     "ppl_proposal_infer", "ppl_proposal_pick_widen")
N_PARAMS = 148224


def ppl_proposal_weights_bytes():
    return int(lib.ppl_proposal_weights_bytes())


def ppl_proposal_init(seed, weights=None, stream=None):
    """Initialised parameter block (a uint8 device tensor)."""
    if weights is None:
        weights = workspace(ppl_proposal_weights_bytes())
    _check(lib.ppl_proposal_init(_ptr(weights), int(seed) & (2 ** 64 - 1), _stream(stream)))
    return weights


def ppl_proposal_train_workspace_size(model, cfg):
    b = ctypes.c_size_t()
    _check(lib.ppl_proposal_train_workspace_size(model, ctypes.byref(cfg), ctypes.byref(b)))
    return b.value


def ppl_proposal_train(model, cfg, seed, weights, loss_trace=None, ws=None, stream=None):
    if ws is None:
        ws = workspace(ppl_proposal_train_workspace_size(model, cfg))
    _check(lib.ppl_proposal_train(model, ctypes.byref(cfg), int(seed) & (2 ** 64 - 1), _ptr(weights),
                                  _ptr(loss_trace), _ptr(ws), ws.numel(), _stream(stream)))
    return loss_trace


def ppl_proposal_gradient(model, cfg, seed, step, weights, grad=None, loss=None, summaries=None, latents=None,
                          outputs=None, ws=None, stream=None):
    if ws is None:
        ws = workspace(ppl_proposal_train_workspace_size(model, cfg))
    _check(lib.ppl_proposal_gradient(model, ctypes.byref(cfg), int(seed) & (2 ** 64 - 1), int(step), _ptr(weights),
                                     _ptr(grad), _ptr(loss), _ptr(summaries), _ptr(latents), _ptr(outputs),
                                     _ptr(ws), ws.numel(), _stream(stream)))


def ppl_proposal_infer_workspace_size(model, data, n):
    b = ctypes.c_size_t()
    _check(lib.ppl_proposal_infer_workspace_size(model, ctypes.byref(data), int(n), ctypes.byref(b)))
    return b.value


def ppl_proposal_infer(model, data, weights, n, seed, q_params=None, data_summaries=None, ws=None, stream=None,
                       log_weights=None, latents=None, summaries=None, scalars=None, sync=False, widen=1.0):
    """Amortised importance sampling; returns the ppl_result struct."""
    if ws is None:
        ws = workspace(ppl_proposal_infer_workspace_size(model, data, n))
    res = PplResult(sync_host=1 if sync else 0, d_scalars=_ptr(scalars), d_latents=_ptr(latents),
                    d_log_weights=_ptr(log_weights), d_summaries=_ptr(summaries))
    _check(lib.ppl_proposal_infer(model, ctypes.byref(data), _ptr(weights), int(n), int(seed) & (2 ** 64 - 1),
                                  float(widen), _ptr(q_params), _ptr(data_summaries), _ptr(ws), ws.numel(),
                                  _stream(stream), ctypes.byref(res)))
    return res



WIDEN_CANDIDATES = (1.0, 1.25, 1.5, 2.0)


def ppl_proposal_pick_widen(model, data, weights, n_pilot=1 << 14, seed=0x51, candidates=WIDEN_CANDIDATES, ws=None,
                            stream=None):
    """Returns (chosen widen, [pilot ESS per candidate])."""
    if ws is None:
        ws = workspace(ppl_proposal_infer_workspace_size(model, data, n_pilot))
    c = (ctypes.c_double * len(candidates))(*[float(v) for v in candidates])
    ess = (ctypes.c_double * len(candidates))()
    best = ctypes.c_double()
    _check(lib.ppl_proposal_pick_widen(model, ctypes.byref(data), _ptr(weights), int(n_pilot),
                                       int(seed) & (2 ** 64 - 1), c, len(candidates), ctypes.byref(best), ess,
                                       _ptr(ws), ws.numel(), _stream(stream)))
    return best.value, list(ess)
