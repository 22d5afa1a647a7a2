"""Pins of the oracle's teacher-forced SMC (no GPU).

The forced run compares a second SMC run (in the GPU tests: the HIP kernels)
with the oracle's own FP64 run event by event: it draws its own ancestors from
its FP64 weights, flags as ties the slots that the other run's perturbed
weights could move to a neighbouring ancestor, adopts the other run's ancestor
only there, and counts every other difference.  These tests check, with a
simulated other run (this oracle's weights perturbed at FP32 rounding scale,
resampled by the same integer rule), that the tie bands always cover the
slots the perturbation moves, that they stay narrow, and that a planted
difference outside a band is reported."""
import math

import numpy as np
import pytest

import synthetic


def _other_run(orc, lw, sigma, seed, step, g):
    """Another run's view of the same event: FP32 log-weights perturbed by
    relative noise sigma, resampled by the integer rule."""
    lw2 = (lw + sigma * np.maximum(1.0, np.abs(lw)) * g.standard_normal(lw.size)).astype(np.float32)
    anc, _ = orc.resample(lw2.astype(np.float64), seed, step=step)
    return lw2, anc


@pytest.mark.parametrize("n", [4096, 1 << 16, (1 << 16) + 7])
@pytest.mark.parametrize("sigma", [0.0, 1e-7, 1e-6, 1e-5])
def test_forced_event_bands_cover_the_perturbation(orc, n, sigma):
    g = np.random.default_rng(n + int(sigma * 1e9))
    for trial in range(6):
        # log-weights of one epoch: a spread of a few nats, some particles far out
        lw = -0.5 * (g.standard_normal(n) * 2.0) ** 2 + 0.3 * g.standard_normal(n)
        lw[g.choice(n, size=n // 50, replace=False)] -= 40.0
        lw2, ganc = _other_run(orc, lw, sigma, seed=trial + 1, step=trial, g=g)
        anc, st = orc.forced_event(lw, lw2, ganc, seed=trial + 1, step=trial)
        assert st["nontie_diff"] == 0, (trial, st)
        assert st["adopted"] <= st["ties"]
        e = st["expected_ties"]
        assert st["ties"] <= e + 4 * math.sqrt(e) + 4, (trial, st)
        assert np.all(np.diff(anc) >= 0) and anc.min() >= 0 and anc.max() < n
        if sigma <= 1e-6:
            assert st["ties"] <= max(8, n // 100), (trial, st)          # the bands stay narrow


def test_forced_event_reports_planted_differences(orc):
    """Ancestors changed at slots away from every band are counted one by one."""
    n = 1 << 14
    g = np.random.default_rng(3)
    lw = -0.5 * (g.standard_normal(n) * 1.5) ** 2
    lw2, ganc = _other_run(orc, lw, 1e-7, seed=9, step=2, g=g)
    _, clean = orc.forced_event(lw, lw2, ganc, seed=9, step=2)
    assert clean["nontie_diff"] == 0
    bad = ganc.copy()
    slots = g.choice(n, size=40, replace=False)
    bad[slots] = np.where(bad[slots] > 0, bad[slots] - 1, bad[slots] + 1)
    _, st = orc.forced_event(lw, lw2, bad, seed=9, step=2)
    assert st["nontie_diff"] >= 40 - clean["ties"]
    assert st["nontie_diff"] <= 40


@pytest.mark.parametrize("model,K,D,n", [("lgssm", 0, 80, 3000), ("gmm", 5, 60, 2048)])
def test_forced_smc_follows_its_own_run(orc, model, K, D, n):
    """Forced with the oracle's own decisions, ancestors and (FP32-rounded) event
    log-weights, the forced run reproduces the plain run: no difference outside
    a band, the same log-evidence, increments summing to it."""
    if model == "lgssm":
        m, y = orc.MODEL_LGSSM, synthetic.lgssm_data(T=D, seed=31).astype(np.float64)
    else:
        m = orc.MODEL_GMM
        y = synthetic.gmm_instances(1, seed=7, d_lo=math.log10(D), d_hi=math.log10(D) + 1e-9,
                                    k_lo=K, k_hi=K)[0]["y"][:D].astype(np.float64)
    o = orc.smc(m, y, n, 5, K=K, max_events=D, want_state=True, want_event_lw=True)
    E = o["n_resample"]
    assert E >= 5
    f = orc.smc_forced(m, y, n, 5, o["resampled"], o["ancestors"][:E], o["event_lw"][:E].astype(np.float32),
                       K=K, ess_band=1e-4, want_state=True)
    assert f["status"] == 0 and f["steps"] == y.size and f["n_resample"] == E
    assert f["decisions"]["differ_outside_band"] == 0 and f["decisions"]["adopted"] == 0
    assert np.all(f["events"]["nontie_diff"] == 0) and np.all(f["events"]["adopted"] == 0)
    assert np.all(f["events"]["step"] == np.flatnonzero(o["resampled"]))
    assert f["log_z"] == o["log_z"]
    assert abs(f["logz_inc"].sum() - o["log_z"]) < 1e-9 * max(1.0, abs(o["log_z"]))
    assert np.array_equal(f["state"], o["state"]) and np.array_equal(f["lw"], o["lw"])


def test_forced_smc_counts_a_planted_decision(orc):
    """A decision flipped where the ESS is far from the threshold is reported,
    and the forced run follows the given decisions (its event count grows)."""
    y = synthetic.lgssm_data(T=60, seed=5).astype(np.float64)
    n = 2048
    o = orc.smc(orc.MODEL_LGSSM, y, n, 2, max_events=60, want_event_lw=True)
    far = np.flatnonzero(~o["resampled"][:-1] & (np.abs(o["ess_trace"][:-1] / n - 0.5) > 0.05))
    assert far.size
    res = o["resampled"].copy()
    res[far[0]] = True
    f = orc.smc_forced(orc.MODEL_LGSSM, y, n, 2, res, o["ancestors"][:o["n_resample"]],
                       o["event_lw"][:o["n_resample"]].astype(np.float32), ess_band=1e-4)
    assert f["decisions"]["differ_outside_band"] >= 1
    # the extra event uses up the given records one event early: the run stops there
    assert f["steps"] < y.size
