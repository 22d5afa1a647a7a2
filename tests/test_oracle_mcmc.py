"""Pins of the oracle's lightweight Metropolis-Hastings (no GPU).

- With no data the chains' stationary distribution is the prior: n uniform
  on {2..5} and zero-mean coefficients.  The site-count factor of the
  acceptance ratio is what makes n uniform (without it P(n) grows like n + 1).
- With data, pooled chain averages match the conjugate closed form of the
  polynomial model (P(n | y) and E[c | n, y]) within their Monte Carlo error
  across independent groups of chains (prior proposals mix slowly across n:
  chains run 20000 iterations after a burn-in of 5000).
- Traces are consistent with the final states and the accepted counts.
"""
import math

import numpy as np

from oracle import closed_forms as cf


def _data(D, seed=5):
    g = np.random.default_rng(seed)
    x = g.uniform(-1, 1, D)
    y = 0.5 - 1.2 * x + 0.8 * x ** 3 + 0.5 * g.standard_normal(D)
    return x, y


def test_no_data_samples_the_prior(orc):
    x = np.zeros(0)
    y = np.zeros(0)
    ests = []
    for seed in range(1, 9):
        o = orc.mcmc_poly(x, y, 2048, 400, seed, burn_in=50)
        ests.append(o["summaries"][:4])
    ests = np.array(ests)
    se = ests.std(0, ddof=1) / math.sqrt(len(ests))
    assert np.all(np.abs(ests.mean(0) - 0.25) < 4 * se + 2e-3), (ests.mean(0), se)
    # coefficient means are zero under the prior
    o = orc.mcmc_poly(x, y, 4096, 400, 99, burn_in=50)
    assert np.all(np.abs(o["summaries"][24:29]) < 0.5)


def test_pooled_chains_match_the_closed_form(orc):
    x, y = _data(6)
    ex = cf.poly_exact(x, y)
    ests, cmeans = [], []
    for seed in range(1, 9):
        o = orc.mcmc_poly(x, y, 512, 20000, seed, burn_in=5000)
        ests.append(o["summaries"][:4])
        cmeans.append(o["summaries"][4:24].reshape(4, 5))
    ests = np.array(ests)
    se = ests.std(0, ddof=1) / math.sqrt(len(ests))
    assert np.all(np.abs(ests.mean(0) - ex["p_n"]) < 4 * se + 5e-3), (ests.mean(0), ex["p_n"], se)
    best = int(np.argmax(ex["p_n"]))
    n = best + 2
    cm = np.array([c[best, :n] for c in cmeans])
    cse = cm.std(0, ddof=1) / math.sqrt(len(cm))
    assert np.all(np.abs(cm.mean(0) - ex["means"][best][:n]) < 4 * cse + 0.02), (cm.mean(0), ex["means"][best], cse)


def test_traces_are_consistent(orc):
    x, y = _data(10, seed=2)
    o = orc.mcmc_poly(x, y, 300, 200, 7, want_trace=True)
    assert np.array_equal(o["n_trace"][-1], o["state"][0].astype(np.int8))
    st = o["state"]
    for c in range(300):
        n = int(st[0, c])
        assert 2 <= n <= 5 and np.all(st[1 + n:, c] == 0.0)
    assert np.all(o["accepts"] >= 0) and np.all(o["accepts"] <= 200)
    assert np.all(np.isfinite(o["la_trace"]))
    # a proposal of the same n (site 0, n' = n) is always accepted: log alpha = 0
    assert np.any(o["la_trace"] == 0.0)
