"""GPU parity of sequential Monte Carlo (persistent cooperative kernel) against
the CPU oracle, through the C ABI.

The GPU keeps FP32 state and log-weights; the oracle runs in FP64 from the
same Philox streams.  Resampling decisions and ancestor slots that the oracle
flags as ties (decision within the band that FP32 rounding of the log-weights
can move) are excused; everything else must match exactly, event by event,
until the first excused slot actually differs (after that the two runs are
different but equally valid particle systems and only statistics compare).
"""
import math

import numpy as np
import pytest

import synthetic
from forced_check import check_forced

pytestmark = pytest.mark.gpu

LW_TOL = 1e-5          # FP32 log-weight / state tolerance (mixed)
ANC_BAND = 2e-5        # CDF perturbation band for ancestor ties (2 x the log-weight tolerance)
ESS_BAND = 1e-4        # |ESS / N - ess_frac| band for decision ties


@pytest.fixture(scope="module")
def ppl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_08454_amd as p
    return p


def run_gpu(ppl, model, y, n, seed, ess_frac=0.5, K=0, max_events=0, records=False, move_steps=0):
    import torch
    dev = torch.device("cuda:0")
    dy = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).to(dev)
    data = ppl.make_data(None, dy, n_data=y.size, dim=K, dtype=ppl.PPL_F32)
    T = max(y.size, 1)
    nf = 1 if model == ppl.PPL_MODEL_LGSSM else 2 * K
    lw = torch.empty(n, dtype=torch.float32, device=dev)
    lat = torch.empty((nf, n), dtype=torch.float32, device=dev)
    scal = torch.empty(8, dtype=torch.float64, device=dev)
    ess = torch.zeros(T, dtype=torch.float64, device=dev)
    res_flag = torch.zeros(T, dtype=torch.uint8, device=dev)
    anc = torch.full((max_events, n), -7, dtype=torch.int32, device=dev) if max_events else None
    elw = torch.full((max_events, n), float("nan"), dtype=torch.float32, device=dev) if records else None
    lzt = torch.full((T,), float("nan"), dtype=torch.float64, device=dev)
    alpha = (torch.full((max_events, move_steps, n), float("nan"), dtype=torch.float64, device=dev)
             if (records and move_steps) else None)
    r = ppl.ppl_smc(model, data, n, seed, ess_frac, log_weights=lw, latents=lat, scalars=scal, ess_trace=ess,
                    resampled=res_flag, ancestors=anc, sync=True, event_lw=elw, logz_trace=lzt,
                    move_steps=move_steps, move_log_alpha=alpha)
    out = dict(log_z=r.log_evidence, ess=r.ess, n_resample=r.n_resample, lw=lw.cpu().numpy().astype(np.float64),
               state=lat.cpu().numpy().astype(np.float64), ess_trace=ess.cpu().numpy()[:y.size],
               resampled=res_flag.cpu().numpy()[:y.size].astype(bool), scalars=scal.cpu().numpy(),
               logz_trace=lzt.cpu().numpy()[:y.size])
    if max_events:
        out["ancestors"] = anc.cpu().numpy()
    if records:
        out["event_lw"] = elw.cpu().numpy()
    if alpha is not None:
        out["alpha"] = alpha[: max(r.n_resample, 1)].cpu().numpy()
    return out


def mixed_err(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b)))) if a.size else 0.0


def compare_until_divergence(g, o, n):
    """Step-by-step comparison; returns the number of resampling events compared exactly."""
    T = o["ess_trace"].size
    events = 0
    for s in range(T):
        if o["ess_tie"][s] and g["resampled"][s] != o["resampled"][s]:
            return events, "decision tie"
        assert g["resampled"][s] == o["resampled"][s], f"resampling decision differs at factor {s}"
        assert abs(g["ess_trace"][s] - o["ess_trace"][s]) <= 1e-3 * o["ess_trace"][s], s
        if o["resampled"][s]:
            ga, oa, tie = g["ancestors"][events], o["ancestors"][events], o["anc_tie"][events]
            bad = ga != oa
            assert not np.any(bad & ~tie), f"event {events} (factor {s}): {int((bad & ~tie).sum())} non-tie slots differ"
            if np.any(bad):
                return events, "ancestor tie"
            events += 1
    return events, "complete"


@pytest.mark.parametrize("n,T", [(5000, 200), (1, 30), (70_000, 64)])
def test_lgssm_no_resampling_parity(ppl, orc, n, T):
    """ess_frac = 0: sequential importance sampling; every particle's FP32 path
    and log-weight match the FP64 oracle."""
    y = synthetic.lgssm_data(T=T, seed=21)
    g = run_gpu(ppl, ppl.PPL_MODEL_LGSSM, y, n, seed=5, ess_frac=0.0)
    o = orc.smc(orc.MODEL_LGSSM, y.astype(np.float64), n, 5, ess_frac=0.0, want_state=True)
    assert g["n_resample"] == 0 and o["n_resample"] == 0
    assert mixed_err(g["state"][0], o["state"][0]) < LW_TOL
    assert mixed_err(g["lw"], o["lw"]) < LW_TOL
    assert abs(g["log_z"] - o["log_z"]) < LW_TOL * max(1.0, abs(o["log_z"]))
    assert abs(g["ess"] - o["ess"]) < 1e-3 * o["ess"]
    assert np.all(np.abs(g["ess_trace"] - o["ess_trace"]) <= 1e-3 * o["ess_trace"])


@pytest.mark.parametrize("n,T,seed", [(4096, 120, 3), (3000, 80, 8), (20_000, 40, 1)])
def test_lgssm_resampling_parity(ppl, orc, n, T, seed):
    y = synthetic.lgssm_data(T=T, seed=31)
    o = orc.smc(orc.MODEL_LGSSM, y.astype(np.float64), n, seed, ess_frac=0.5, ess_band=ESS_BAND,
                anc_band=ANC_BAND, max_events=T, want_state=True)
    g = run_gpu(ppl, ppl.PPL_MODEL_LGSSM, y, n, seed, ess_frac=0.5, max_events=T)
    assert o["n_resample"] >= 10
    events, why = compare_until_divergence(g, o, n)
    assert events >= 5, (events, why)
    if why == "complete":
        assert g["n_resample"] == o["n_resample"]
        assert mixed_err(g["state"][0], o["state"][0]) < LW_TOL
        assert mixed_err(g["lw"], o["lw"]) < LW_TOL
        assert abs(g["log_z"] - o["log_z"]) < LW_TOL * max(1.0, abs(o["log_z"]))


def test_lgssm_resample_every_step(ppl, orc):
    y = synthetic.lgssm_data(T=40, seed=4)
    n = 2048
    g = run_gpu(ppl, ppl.PPL_MODEL_LGSSM, y, n, seed=2, ess_frac=1.0, max_events=40)
    o = orc.smc(orc.MODEL_LGSSM, y.astype(np.float64), n, 2, ess_frac=1.0, anc_band=ANC_BAND, max_events=40)
    assert g["n_resample"] == y.size - 1 == o["n_resample"]
    assert not g["resampled"][-1]
    anc = g["ancestors"][: g["n_resample"]]
    assert np.all(np.diff(anc, axis=1) >= 0) and anc.min() >= 0 and anc.max() < n


def test_lgssm_degenerate_sizes(ppl):
    """T = 0: no factor, log Z = 0 and ESS = N.  T = 1: the only factor is the last,
    so there is no resampling.  N = 1: ESS is always 1."""
    g = run_gpu(ppl, ppl.PPL_MODEL_LGSSM, np.zeros(0, np.float32), 100, seed=1)
    assert g["log_z"] == 0.0 and g["ess"] == 100.0 and g["n_resample"] == 0
    g = run_gpu(ppl, ppl.PPL_MODEL_LGSSM, np.array([0.3], np.float32), 500, seed=1, ess_frac=1.0)
    assert g["n_resample"] == 0
    g = run_gpu(ppl, ppl.PPL_MODEL_LGSSM, synthetic.lgssm_data(T=20), 1, seed=1, ess_frac=1.0)
    assert g["n_resample"] == 0 and g["ess"] == 1.0


def test_lgssm_full_size_vs_kalman(ppl):
    """The measured configuration (N = 2^20, T = 1000): the SMC log-evidence over
    seeds agrees with the Kalman filter; the resampling count matches the ESS trace."""
    from oracle import closed_forms as cf
    y = synthetic.lgssm_data()
    kf = cf.kalman(y.astype(np.float64))
    est = []
    for seed in range(1, 9):
        g = run_gpu(ppl, ppl.PPL_MODEL_LGSSM, y, 1 << 20, seed)
        trig = (g["ess_trace"][:-1] < 0.5 * (1 << 20)).sum()
        assert g["n_resample"] == trig == g["resampled"].sum()
        assert np.all(np.isfinite(g["lw"]))
        est.append(g["log_z"])
    est = np.array(est)
    sd = max(est.std(ddof=1), 0.02)
    assert abs(est.mean() - kf) < 4 * sd / math.sqrt(est.size) + 0.5 * sd * sd + 0.02, (est, kf)


@pytest.mark.parametrize("K,D,n,min_events", [(5, 300, 1 << 16, 0), (1, 50, 3000, 3), (8, 120, 5000, 3),
                                               (3, 200, 1 << 16, 0), (5, 300, 4096, 3)])
def test_gmm_smc_parity(ppl, orc, K, D, n, min_events):
    """Event-by-event parity.  At N = 2^16 a few slots per event sit inside the
    FP32 rounding band, so the runs usually part at the first event: there only
    the non-tie slots of that event are required to match."""
    inst = synthetic.gmm_instances(1, seed=K * 100 + D, d_lo=math.log10(D), d_hi=math.log10(D) + 1e-9, k_lo=K, k_hi=K)[0]
    y = inst["y"][:D]
    seed = 11
    o = orc.smc(orc.MODEL_GMM, y.astype(np.float64), n, seed, K=K, ess_band=ESS_BAND, anc_band=ANC_BAND,
                max_events=D, want_state=True)
    g = run_gpu(ppl, ppl.PPL_MODEL_GMM, y, n, seed, K=K, max_events=D)
    events, why = compare_until_divergence(g, o, n)
    assert events >= min(min_events, o["n_resample"]), (events, why)
    if why == "complete":
        assert g["n_resample"] == o["n_resample"]
        assert mixed_err(g["state"], o["state"]) < LW_TOL
        assert mixed_err(g["lw"], o["lw"]) < LW_TOL
        assert abs(g["log_z"] - o["log_z"]) < LW_TOL * max(1.0, abs(o["log_z"]))


def test_gmm_no_resampling_parity(ppl, orc):
    inst = synthetic.gmm_instances(1, seed=5, d_lo=2.0, d_hi=2.0 + 1e-9, k_lo=6, k_hi=6)[0]
    y = inst["y"]
    n = 10_000
    g = run_gpu(ppl, ppl.PPL_MODEL_GMM, y, n, seed=4, ess_frac=0.0, K=6)
    o = orc.smc(orc.MODEL_GMM, y.astype(np.float64), n, 4, ess_frac=0.0, K=6, want_state=True)
    assert mixed_err(g["state"], o["state"]) < 2e-6 * 5
    assert mixed_err(g["lw"], o["lw"]) < LW_TOL
    assert abs(g["log_z"] - o["log_z"]) < LW_TOL * max(1.0, abs(o["log_z"]))


def _pick_p(n):
    """Particles per thread of the persistent SMC kernel: one 512-thread
    workgroup per CU (256 CUs) covers n with P in {1, 2, 4, 8}."""
    per_cu, p = -(-n // 256), 1
    while p < 8 and 512 * p < per_cu:
        p *= 2
    return p


@pytest.mark.parametrize("n,T,p", [((1 << 17) + 3, 200, 2), ((1 << 18) + 7, 150, 4), ((1 << 19) + 5, 100, 8),
                                   (1 << 20, 200, 8)])
def test_lgssm_teacher_forced(ppl, orc, n, T, p):
    """Teacher-forced parity over the whole run at the particle counts that
    select 2, 4 and 8 particles per thread (the galloping ancestor search and
    the incremental slot thresholds run only there; ragged last tiles), and
    at the measured N = 2^20: every non-tie ancestor at every event, the
    event log-weights, the normaliser increments, the final particles and
    log Z-hat."""
    assert _pick_p(n) == p
    y = synthetic.lgssm_data(T=T, seed=41)
    seed = 13
    g = run_gpu(ppl, ppl.PPL_MODEL_LGSSM, y, n, seed, ess_frac=0.5, max_events=T, records=True)
    E = g["n_resample"]
    assert E >= T // 3
    f = orc.smc_forced(orc.MODEL_LGSSM, y.astype(np.float64), n, seed, g["resampled"], g["ancestors"][:E],
                       g["event_lw"][:E], ess_band=ESS_BAND, want_state=True)
    print(check_forced(g, f, n, full=True, min_events=T // 3))


@pytest.mark.parametrize("K,D,n,p", [(5, 300, (1 << 17) + 3, 2), (8, 120, (1 << 19) + 5, 8)])
def test_gmm_teacher_forced(ppl, orc, K, D, n, p):
    assert _pick_p(n) == p
    inst = synthetic.gmm_instances(1, seed=K * 100 + D, d_lo=math.log10(D), d_hi=math.log10(D) + 1e-9, k_lo=K, k_hi=K)[0]
    y = inst["y"][:D]
    seed = 17
    g = run_gpu(ppl, ppl.PPL_MODEL_GMM, y, n, seed, K=K, max_events=D, records=True)
    E = g["n_resample"]
    f = orc.smc_forced(orc.MODEL_GMM, y.astype(np.float64), n, seed, g["resampled"], g["ancestors"][:E],
                       g["event_lw"][:E], K=K, ess_band=ESS_BAND, want_state=True)
    print(check_forced(g, f, n, full=True, min_events=5))


@pytest.mark.parametrize("K,D,n,M", [(3, 120, 4096, 2), (1, 60, 3000, 3), (8, 80, 20_000, 1), (5, 150, (1 << 17) + 3, 1)])
def test_gmm_resample_move_teacher_forced(ppl, orc, K, D, n, M):
    """Resample-move: after each resampling every particle takes M
    Metropolis-Hastings steps.  Teacher-forced against the oracle over the
    whole run: ancestors, event log-weights and normaliser increments as for
    plain SMC, and every accept decision outside the tie band of the two
    runs' log acceptance ratios, which agree to FP32 rounding."""
    inst = synthetic.gmm_instances(1, seed=K * 31 + D, d_lo=math.log10(D), d_hi=math.log10(D) + 1e-9, k_lo=K, k_hi=K)[0]
    y = inst["y"][:D]
    seed = 29
    g = run_gpu(ppl, ppl.PPL_MODEL_GMM, y, n, seed, K=K, max_events=D, records=True, move_steps=M)
    E = g["n_resample"]
    assert E >= 3
    f = orc.smc_forced(orc.MODEL_GMM, y.astype(np.float64), n, seed, g["resampled"], g["ancestors"][:E],
                       g["event_lw"][:E], K=K, ess_band=ESS_BAND, want_state=True, move_steps=M,
                       given_alpha=g["alpha"][:E])
    summary = check_forced(g, f, n, full=True, min_events=3)
    mv = f["moves"]
    assert np.all(mv["nontie_diff"] == 0), mv["nontie_diff"]
    assert float(mv["max_dalpha"].max()) <= 1e-5
    decisions = E * M * n
    assert mv["ties"].sum() <= 1e-3 * decisions + 10
    a = g["alpha"][:E]
    assert np.all(np.isfinite(a))
    rate = float(np.mean(np.minimum(1.0, np.exp(a))))
    assert 0.02 < rate < 0.98
    summary.update(move_ties=int(mv["ties"].sum()), move_adopted=int(mv["adopted"].sum()), accept_rate=round(rate, 3))
    print(summary)


def test_gmm_resample_move_keeps_particles_distinct(ppl):
    """Without moves the static-parameter particles collapse onto a few
    values; with moves they stay distinct (the reason for the move step).
    (A collapsed population has ESS = N, so it resamples less often.)"""
    inst = synthetic.gmm_instances(1, seed=8, d_lo=math.log10(300), d_hi=math.log10(300) + 1e-9, k_lo=4, k_hi=4)[0]
    y = inst["y"][:300]
    n = 1 << 16
    plain = run_gpu(ppl, ppl.PPL_MODEL_GMM, y, n, 3, K=4)
    moved = run_gpu(ppl, ppl.PPL_MODEL_GMM, y, n, 3, K=4, move_steps=2)
    d_plain = np.unique(plain["state"][4]).size
    d_moved = np.unique(moved["state"][4]).size
    assert d_moved > 100 * d_plain and d_moved > n // 4, (d_plain, d_moved)


@pytest.mark.parametrize("model,K,n,T", [("lgssm", 0, (1 << 20) - 5, 60), ("lgssm", 0, 3000, 80),
                                         ("gmm", 5, (1 << 17) + 3, 60)])
def test_tagged_polling_path_gives_the_same_results(ppl, monkeypatch, model, K, n, T):
    """Every word the blocks publish for each other carries its epoch or event
    tag; a reader that finds an older tag polls the word again.  With
    PPL_SMC_POLL_ALL=1 every tagged read takes that polling path: the run must
    be bitwise the same (eight particles per lane at 2^20 - 5, one per lane at
    3000, the mixture state at 2^17 + 3)."""
    print(f"tagged polling path {model} n={n}", flush=True)
    if model == "lgssm":
        y, mid = synthetic.lgssm_data(T=T), ppl.PPL_MODEL_LGSSM
    else:
        inst = synthetic.gmm_instances(1, seed=7, d_lo=math.log10(T), d_hi=math.log10(T) + 1e-9, k_lo=K, k_hi=K)[0]
        y, mid = inst["y"][:T], ppl.PPL_MODEL_GMM
    monkeypatch.delenv("PPL_SMC_POLL_ALL", raising=False)
    a = run_gpu(ppl, mid, y, n, 3, K=K, max_events=T)
    monkeypatch.setenv("PPL_SMC_POLL_ALL", "1")
    b = run_gpu(ppl, mid, y, n, 3, K=K, max_events=T)
    monkeypatch.delenv("PPL_SMC_POLL_ALL")
    assert a["n_resample"] > 0
    assert a["log_z"] == b["log_z"] and a["n_resample"] == b["n_resample"]
    assert np.array_equal(a["ancestors"], b["ancestors"])
    assert np.array_equal(a["lw"], b["lw"]) and np.array_equal(a["state"], b["state"])
