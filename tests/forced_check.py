"""Checks of a GPU SMC run against the oracle's teacher-forced run beside it
(``oracle.smc_forced``): the oracle draws its own ancestors from its FP64
weights and takes the GPU's only at slots inside the tie band that the GPU's
FP32 log-weights span, so every other difference is a parity failure."""
import math

import numpy as np

LW_TOL = 1e-5          # FP32 log-weight / state tolerance (mixed)


def mixed_err(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b)))) if a.size else 0.0


def check_forced(g, f, n, full, min_events=1):
    """g: the GPU run (resampled, logz_trace, and when full: state, lw, log_z,
    n_resample); f: the forced oracle run over the GPU's first E events.
    full: the forced run covered every event, so the final particles compare.
    Returns a short summary for the test log."""
    ev = f["events"]
    E = f["n_resample"]
    assert f["status"] == 0, f["status"]
    assert E >= min_events, E
    # decisions outside the ESS tie band agree
    assert f["decisions"]["differ_outside_band"] == 0, f["decisions"]
    # every ancestor outside a tie band is the oracle's own, at every event
    assert np.all(ev["nontie_diff"] == 0), (np.flatnonzero(ev["nontie_diff"])[:5], ev["nontie_diff"].sum())
    # the log-weights each event resampled from agree to the FP32 tolerance
    assert np.all(ev["max_dlw"] <= LW_TOL), float(ev["max_dlw"].max())
    # tie slots: no more than their expectation allows
    exp, ties = float(ev["expected_ties"].sum()), int(ev["ties"].sum())
    assert ties <= exp + 4.0 * math.sqrt(exp) + 4.0, (ties, exp)
    # the normaliser increment of each epoch (|max lw| <= |increment| + log N)
    steps = ev["step"]
    gi, fi = g["logz_trace"][steps], f["logz_inc"][steps]
    scale = np.maximum(1.0, np.abs(fi) + math.log(n))
    assert np.all(np.abs(gi - fi) <= LW_TOL * scale), float(np.max(np.abs(gi - fi) / scale))
    if full:
        T = g["resampled"].size
        assert f["steps"] == T and g["n_resample"] == E
        assert mixed_err(g["state"], f["state"]) < LW_TOL
        assert mixed_err(g["lw"], f["lw"]) < LW_TOL
        assert abs(g["log_z"] - f["log_z"]) <= LW_TOL * max(1.0, abs(f["log_z"]))
        if T:
            fin = T - 1
            assert abs(g["logz_trace"][fin] - f["logz_inc"][fin]) <= LW_TOL * max(1.0, abs(f["logz_inc"][fin]) + math.log(n))
            assert abs(np.sum(g["logz_trace"]) - g["log_z"]) <= 1e-9 * max(1.0, abs(g["log_z"]))
    return dict(events=E, ties=ties, expected_ties=round(exp, 1), adopted=int(ev["adopted"].sum()),
                max_dlw=float(ev["max_dlw"].max()) if E else 0.0,
                decisions_in_band=f["decisions"]["in_band"], decisions_adopted=f["decisions"]["adopted"])
