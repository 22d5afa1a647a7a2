"""Plain FP64 CPU oracle for the particle-inference hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg are the only callers.  The product path (the HIP
library and its Python binding) never imports this package, and this package
imports nothing from the product path.

The C part (``ppl_oracle.c``) computes the sampling, scoring, importance
sampling, log-sum-exp/ESS, resampling and SMC definitions in double precision;
``closed_forms`` holds the exact answers (conjugate Gaussian posteriors,
enumeration over the polynomial degree, the Kalman filter) that pin it.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ppl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MODEL_POLY, MODEL_BLR, MODEL_LGSSM, MODEL_GMM = 1, 2, 3, 4
TAG_PRIOR, TAG_PROPOSAL, TAG_RESAMPLE = 0, 1, 2


def build(force=False):
    """Compile the oracle with gcc (FP64, no FP contraction, OpenMP over particles)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, u32, u64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
        L.or_philox.argtypes = [u32, u32, u32, u32, u64, P]
        L.or_philox_batch.argtypes = [i64, P, P, P]
        L.or_u01_single.argtypes = [u32]; L.or_u01_single.restype = f64
        L.or_u01_double.argtypes = [u32, u32]; L.or_u01_double.restype = f64
        L.or_box_muller.argtypes = [f64, f64, P, P]
        L.or_uniform_discrete.argtypes = [u32, i64, i64]; L.or_uniform_discrete.restype = i64
        L.or_lse_ess.argtypes = [P, i64, P]
        L.or_poly_draw.argtypes = [u64, i64, u32, P, P, P]
        L.or_poly_loglik.argtypes = [i32, P, P, P, i64]; L.or_poly_loglik.restype = f64
        L.or_blr_draw_std.argtypes = [u64, i64, u32, i32, P]
        L.or_blr_loglik.argtypes = [P, i32, P, P, i64, f64]; L.or_blr_loglik.restype = f64
        L.or_importance.argtypes = [i32, P, P, i64, i32, P, i64, u64, i32, P, P, P, P, P]
        L.or_importance.restype = ctypes.c_int
        L.or_particle_logweights.argtypes = [i32, P, P, i64, i32, P, u64, i32, P, i64, P, P, P]
        L.or_quant_bits.argtypes = [i64]; L.or_quant_bits.restype = i32
        L.or_resample.argtypes = [P, i64, u64, u32, u32, P, f64, P]; L.or_resample.restype = ctypes.c_int
        L.or_resample_textbook.argtypes = [P, i64, u64, u32, u32, P]; L.or_resample_textbook.restype = ctypes.c_int
        L.or_gmm_logfactor.argtypes = [i32, P, P, f64, f64]; L.or_gmm_logfactor.restype = f64
        L.or_gmm_init.argtypes = [u64, u32, i32, P, i64, P]
        L.or_smc.argtypes = [i32, P, i64, i32, P, i64, u64, u32, f64, f64, f64, i64,
                             P, P, P, P, P, P, P, P, P, i32, f64, P]
        L.or_forced_event.argtypes = [P, P, P, i64, u64, u32, u32, P, P]
        L.or_forced_event.restype = ctypes.c_int
        L.or_smc.restype = ctypes.c_int
        L.or_smc_forced.argtypes = [i32, P, i64, i32, P, i64, u64, u32, f64, f64, P, P, P, i64,
                                    P, P, P, P, P, P, P, i32, f64, P, P]
        L.or_move_scales.argtypes = [i32, i64, P, f64, P, P]
        L.or_mcmc_poly.argtypes = [P, P, i64, P, i64, i64, i64, u64, P, P, P, P, P, P, P]
        L.or_mcmc_poly.restype = ctypes.c_int
        L.or_enumerate_hmm.argtypes = [P, i64, P, P, P, P]
        L.or_enumerate_hmm.restype = ctypes.c_int
        L.or_gmm_move_population.argtypes = [i32, P, P, i64, i64, u64, u32, i32, f64, P, P]
        L.or_smc_forced.restype = ctypes.c_int
        L.or_num_threads.restype = ctypes.c_int
        L.or_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads():
    return lib().or_num_threads()


def set_num_threads(n):
    """Host threads of the oracle's particle loops (n < 1: all available)."""
    lib().or_set_num_threads(int(n))


# ------------------------------------------------------------------ streams --
def philox(ctr, seeds):
    """Philox4x32-10 blocks for rows of counters ``ctr`` [n,4] under keys ``seeds`` [n]."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    seeds = np.ascontiguousarray(np.broadcast_to(np.asarray(seeds, dtype=np.uint64), (ctr.shape[0],)))
    out = np.empty_like(ctr)
    lib().or_philox_batch(ctr.shape[0], _p(ctr), _p(seeds), _p(out))
    return out


def u01_single(w):
    return lib().or_u01_single(int(w))


def u01_double(lo, hi):
    return lib().or_u01_double(int(lo), int(hi))


def box_muller(u1, u2):
    z0, z1 = ctypes.c_double(), ctypes.c_double()
    lib().or_box_muller(float(u1), float(u2), ctypes.byref(z0), ctypes.byref(z1))
    return z0.value, z1.value


def uniform_discrete(w, lo, hi):
    return lib().or_uniform_discrete(int(w), int(lo), int(hi))


# --------------------------------------------------------------- reductions --
def lse_ess(lw):
    """{max, s1, s2, LSE, ESS} of a log-weight vector, FP64, compensated sums."""
    lw = _f64(lw)
    out = np.empty(5)
    lib().or_lse_ess(_p(lw), lw.size, _p(out))
    return dict(max=out[0], s1=out[1], s2=out[2], lse=out[3], ess=out[4])


def quant_bits(n):
    return lib().or_quant_bits(int(n))


def resample(lw, seed, step=0, inst=0, band=0.0):
    """Integer-rule systematic resampling; returns (ancestors, tie flags)."""
    lw = _f64(lw)
    anc = np.empty(lw.size, dtype=np.int32)
    tie = np.zeros(lw.size, dtype=np.uint8)
    rc = lib().or_resample(_p(lw), lw.size, seed, step, inst, _p(anc), band, _p(tie))
    if rc:
        raise ValueError(f"or_resample failed ({rc})")
    return anc, tie.astype(bool)


def resample_textbook(lw, seed, step=0, inst=0):
    lw = _f64(lw)
    anc = np.empty(lw.size, dtype=np.int32)
    rc = lib().or_resample_textbook(_p(lw), lw.size, seed, step, inst, _p(anc))
    if rc:
        raise ValueError(f"or_resample_textbook failed ({rc})")
    return anc


# ------------------------------------------------------------------- models --
POLY_HYPER = (10.0, 2.0, 5.0)
BLR_HYPER = (1.0, 0.5)
LGSSM_HYPER = (0.9, 1.0, 0.5, 0.0, 0.0)
GMM_HYPER = (5.0, 1.0)


def poly_draw(seed, i, hyper=POLY_HYPER, tag=TAG_PRIOR):
    h = _f64(hyper)
    n = ctypes.c_int32()
    c = np.empty(6)
    lib().or_poly_draw(seed, i, tag, _p(h), ctypes.byref(n), _p(c))
    return n.value, c


def poly_loglik(n, c, x, y):
    c, x, y = _f64(c), _f64(x), _f64(y)
    return lib().or_poly_loglik(int(n), _p(c), _p(x), _p(y), x.size)


def blr_draw_std(seed, i, dim=16, tag=TAG_PRIOR):
    z = np.empty(16)
    lib().or_blr_draw_std(seed, i, tag, dim, _p(z))
    return z[:dim]


def blr_loglik(w, X, y, noise_sd=0.5):
    w, X, y = _f64(w), _f64(X), _f64(y)
    return lib().or_blr_loglik(_p(w), w.size, _p(X), _p(y), y.size, noise_sd)


def gmm_logfactor(lpi, mu, sd, y):
    lpi, mu = _f64(lpi), _f64(mu)
    return lib().or_gmm_logfactor(lpi.size, _p(lpi), _p(mu), sd, y)


def gmm_init(seed, inst, K, N, hyper=GMM_HYPER):
    h = _f64(hyper)
    st = np.empty((2 * K, N))
    lib().or_gmm_init(seed, inst, K, _p(h), N, _p(st))
    return st


def _q_args(q):
    if q is None:
        return 0, None
    mean, chol = q
    return 1, _f64(np.concatenate([np.ravel(mean), np.ravel(chol)]))


def importance(model, x, y, n, seed, hyper=None, dim=0, q=None, want_lw=False, want_latents=False):
    """Importance sampling (likelihood weighting, or the Gaussian proposal ``q`` =
    (mean, lower Cholesky factor) for BLR).  Returns a dict with log_z, ess and
    model summaries (see ``ppl_oracle.c`` for the layout)."""
    if hyper is None:
        hyper = POLY_HYPER if model == MODEL_POLY else BLR_HYPER
    x = _f64(x) if x is not None else np.zeros(1)
    y = _f64(y)
    h = _f64(hyper)
    qk, qp = _q_args(q)
    D = y.size
    n_sum = 29 if model == MODEL_POLY else dim
    summ = np.empty(max(n_sum, 1))
    scal = np.empty(5)
    lw = np.empty(n) if want_lw else None
    n_lat = 6 if model == MODEL_POLY else dim
    lat = np.empty((n_lat, n)) if want_latents else None
    rc = lib().or_importance(model, _p(x), _p(y), D, dim, _p(h), n, seed, qk, _p(qp),
                             _p(lw), _p(lat), _p(summ), _p(scal))
    if rc:
        raise ValueError(f"or_importance failed ({rc})")
    out = dict(log_z=scal[0], ess=scal[1], max_lw=scal[2], s1=scal[3], s2=scal[4], summaries=summ[:n_sum])
    if want_lw:
        out["lw"] = lw
    if want_latents:
        out["latents"] = lat
    return out


def particle_logweights(model, x, y, idx, seed, hyper=None, dim=0, q=None):
    """Log-weights (and latents) of the listed particle indices, one by one."""
    if hyper is None:
        hyper = POLY_HYPER if model == MODEL_POLY else BLR_HYPER
    x = _f64(x) if x is not None else np.zeros(1)
    y = _f64(y)
    h = _f64(hyper)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    qk, qp = _q_args(q)
    lw = np.empty(idx.size)
    n_lat = 6 if model == MODEL_POLY else dim
    lat = np.empty((idx.size, n_lat))
    lib().or_particle_logweights(model, _p(x), _p(y), y.size, dim, _p(h), seed, qk, _p(qp),
                                 idx.size, _p(idx), _p(lw), _p(lat))
    return lw, lat


def smc(model, y, n, seed, ess_frac=0.5, hyper=None, K=0, inst=0, ess_band=0.0,
        anc_band=0.0, max_events=0, want_state=False, want_event_lw=False, move_steps=0, move_scale=0.0,
        want_alpha=False):
    """Sequential Monte Carlo over the factors y[0..T-1] (LGSSM or GMM); with
    move_steps > 0 (GMM) every resampling is followed by that many
    Metropolis-Hastings moves per particle (resample-move)."""
    if hyper is None:
        hyper = LGSSM_HYPER if model == MODEL_LGSSM else GMM_HYPER
    y = _f64(y)
    T = y.size
    h = _f64(hyper)
    nf = 1 if model == MODEL_LGSSM else 2 * K
    scal = np.empty(4)
    ess_tr = np.empty(max(T, 1))
    res_tr = np.zeros(max(T, 1), dtype=np.uint8)
    ess_tie = np.zeros(max(T, 1), dtype=np.uint8)
    anc = np.empty((max_events, n), dtype=np.int32) if max_events else None
    tie = np.zeros((max_events, n), dtype=np.uint8) if max_events else None
    st = np.empty((nf, n)) if want_state else None
    lw = np.empty(n) if want_state else None
    lwh = np.zeros((max_events, n)) if (want_event_lw and max_events) else None
    ah = np.zeros((max_events, move_steps, n)) if (want_alpha and max_events and move_steps) else None
    rc = lib().or_smc(model, _p(y), T, K, _p(h), n, seed, inst, ess_frac, ess_band, anc_band,
                      max_events, _p(scal), _p(ess_tr), _p(res_tr), _p(ess_tie), _p(anc), _p(tie),
                      _p(st), _p(lw), _p(lwh), int(move_steps), float(move_scale), _p(ah))
    out = dict(log_z=scal[0], ess=scal[1], n_resample=int(scal[2]), status=int(scal[3]), rc=rc,
               ess_trace=ess_tr[:T], resampled=res_tr[:T].astype(bool), ess_tie=ess_tie[:T].astype(bool))
    if max_events:
        out["ancestors"] = anc
        out["anc_tie"] = tie.astype(bool)
    if want_state:
        out["state"] = st
        out["lw"] = lw
    if lwh is not None:
        out["event_lw"] = lwh
    if ah is not None:
        out["alpha"] = ah
    return out


def move_scales(K, s, hyper=GMM_HYPER, lam=0.0):
    """Random-walk scales (h_b, h_mu) of the resample-move step after factor s."""
    hb, hm = ctypes.c_double(), ctypes.c_double()
    lib().or_move_scales(int(K), int(s), _p(_f64(hyper)), float(lam), ctypes.byref(hb), ctypes.byref(hm))
    return hb.value, hm.value


def gmm_move_population(state, K, y, s, seed, M, inst=0, hyper=GMM_HYPER, lam=0.0, want_alpha=False):
    """M resample-move MH steps (after factor s) applied to the population
    state [2K, N] (log pi_k then mu_k); returns the new state (and the log
    alphas [M, N])."""
    st = np.array(state, dtype=np.float64, order="C", copy=True)
    N = st.shape[1]
    al = np.zeros((M, N)) if want_alpha else None
    lib().or_gmm_move_population(int(K), _p(_f64(hyper)), _p(_f64(y)), int(s), N, seed, int(inst), int(M),
                                 float(lam), _p(st), _p(al))
    return (st, al) if want_alpha else st


def mcmc_poly(x, y, n_chains, n_iters, seed, burn_in=0, hyper=POLY_HYPER, want_trace=False, given_la=None):
    """Lightweight Metropolis-Hastings chains on the polynomial model (see
    ``or_mcmc_poly``).  Returns final states [6, chains], accepted counts,
    the 29 summaries, and with want_trace the per-iteration n and log alpha
    [iters, chains]; given_la forces ties to another run's decisions."""
    x, y, h = _f64(x), _f64(y), _f64(hyper)
    st = np.empty((6, n_chains))
    acc = np.empty(n_chains, dtype=np.int64)
    summ = np.empty(29)
    ntr = np.empty((n_iters, n_chains), dtype=np.int8) if want_trace else None
    latr = np.empty((n_iters, n_chains)) if want_trace else None
    g = None if given_la is None else np.ascontiguousarray(given_la, dtype=np.float64).reshape(n_iters, n_chains)
    ts = np.zeros(3, dtype=np.int64)
    rc = lib().or_mcmc_poly(_p(x), _p(y), y.size, _p(h), int(n_chains), int(n_iters), int(burn_in), seed, _p(st),
                            _p(acc), _p(summ), _p(ntr), _p(latr), _p(g), _p(ts))
    if rc:
        raise ValueError(f"or_mcmc_poly failed ({rc})")
    out = dict(state=st, accepts=acc, summaries=summ, ties=int(ts[0]), adopted=int(ts[1]), nontie_diff=int(ts[2]))
    if want_trace:
        out["n_trace"] = ntr
        out["la_trace"] = latr
    return out


def hmm_hyper(pi0, A, mu, sigma=1.0):
    """The hyper-parameter array of the hidden Markov model: {K, sigma, pi0, A, mu}."""
    pi0, A, mu = np.asarray(pi0, np.float64), np.asarray(A, np.float64), np.asarray(mu, np.float64)
    return np.concatenate([[pi0.size, sigma], pi0, A.ravel(), mu])


def enumerate_hmm(y, hyper):
    """Exact inference by enumerating every path of the hidden Markov model:
    log Z, the number of paths, P(z_t = k | y) [T, K], the MAP path and its
    log joint."""
    y, h = _f64(y), _f64(hyper)
    K = int(h[0])
    scal = np.empty(4)
    marg = np.empty((y.size, K))
    mp = np.empty(y.size, dtype=np.int32)
    rc = lib().or_enumerate_hmm(_p(y), y.size, _p(h), _p(scal), _p(marg), _p(mp))
    if rc:
        raise ValueError(f"or_enumerate_hmm failed ({rc})")
    return dict(log_z=scal[0], paths=scal[1], map_lw=scal[2], marginals=marg, map=mp)


def forced_event(lw, given_lw, given_anc, seed, step=0, inst=0):
    """One teacher-forced resampling event (``or_forced_event``): returns this
    run's ancestors with the given ones adopted at tie slots, and the event's
    statistics (ties, adopted, non-tie differences, expected ties, bands)."""
    lw = _f64(lw)
    n = lw.size
    glw = np.ascontiguousarray(given_lw, dtype=np.float32)
    ganc = np.ascontiguousarray(given_anc, dtype=np.int32)
    anc = np.empty(n, dtype=np.int32)
    st = np.zeros(8)
    rc = lib().or_forced_event(_p(lw), _p(glw), _p(ganc), n, seed, step, inst, _p(anc), _p(st))
    if rc:
        raise ValueError(f"or_forced_event failed ({rc})")
    return anc, dict(max_dlw=st[1], ties=int(st[2]), adopted=int(st[3]), nontie_diff=int(st[4]),
                     expected_ties=st[5], max_band=st[6])


def smc_forced(model, y, n, seed, given_resampled, given_ancestors, given_event_lw, ess_frac=0.5, hyper=None,
               K=0, inst=0, ess_band=0.0, want_state=False, move_steps=0, move_scale=0.0, given_alpha=None):
    """Teacher-forced SMC beside another run (see ``or_smc_forced``): adopts the
    given decision inside the ESS tie band and the given ancestor at tie slots,
    and counts every disagreement outside them.  given_ancestors /
    given_event_lw are [E, n] (the other run's first E events)."""
    if hyper is None:
        hyper = LGSSM_HYPER if model == MODEL_LGSSM else GMM_HYPER
    y = _f64(y)
    T = y.size
    h = _f64(hyper)
    nf = 1 if model == MODEL_LGSSM else 2 * K
    g_res = np.ascontiguousarray(np.asarray(given_resampled)[:T], dtype=np.uint8)
    if g_res.size < T:
        raise ValueError("given_resampled is shorter than y")
    g_anc = np.ascontiguousarray(given_ancestors, dtype=np.int32).reshape(-1, n)
    g_lw = np.ascontiguousarray(given_event_lw, dtype=np.float32).reshape(-1, n)
    E = g_anc.shape[0]
    if g_lw.shape[0] != E:
        raise ValueError("ancestor and log-weight records differ in length")
    g_al = None
    if move_steps:
        g_al = np.ascontiguousarray(given_alpha, dtype=np.float64).reshape(-1, move_steps, n)
        if g_al.shape[0] < E:
            raise ValueError("fewer move records than events")
    mv = np.zeros((max(E, 1), 4))
    scal = np.zeros(5)
    logz_inc = np.zeros(max(T, 1))
    ess_tr = np.zeros(max(T, 1))
    ev = np.zeros((max(E, 1), 8))
    dec = np.zeros(3)
    st = np.empty((nf, n)) if want_state else None
    lw = np.empty(n) if want_state else None
    rc = lib().or_smc_forced(model, _p(y), T, K, _p(h), n, seed, inst, ess_frac, ess_band, _p(g_res),
                             _p(g_anc), _p(g_lw), E, _p(scal), _p(logz_inc), _p(ess_tr), _p(ev), _p(dec),
                             _p(st), _p(lw), int(move_steps), float(move_scale), _p(g_al), _p(mv))
    n_ev = int(scal[2])
    out = dict(rc=rc, log_z=scal[0], ess=scal[1], n_resample=n_ev, status=int(scal[3]), steps=int(scal[4]),
               logz_inc=logz_inc[:T], ess_trace=ess_tr[:T],
               events=dict(step=ev[:n_ev, 0].astype(int), max_dlw=ev[:n_ev, 1], ties=ev[:n_ev, 2].astype(int),
                           adopted=ev[:n_ev, 3].astype(int), nontie_diff=ev[:n_ev, 4].astype(int),
                           expected_ties=ev[:n_ev, 5], max_band=ev[:n_ev, 6]),
               decisions=dict(adopted=int(dec[0]), differ_outside_band=int(dec[1]), in_band=int(dec[2])),
               moves=dict(ties=mv[:n_ev, 0].astype(int), adopted=mv[:n_ev, 1].astype(int),
                          nontie_diff=mv[:n_ev, 2].astype(int), max_dalpha=mv[:n_ev, 3]))
    if want_state:
        out["state"] = st
        out["lw"] = lw
    return out
