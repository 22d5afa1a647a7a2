"""Pins of the oracle's enumeration (no GPU): exact inference by enumerating
every path of a hidden Markov model agrees with the textbook forward-backward
recursions (log-evidence, posterior marginals) and the Viterbi recursion (the
most probable path and its log joint), which compute the same quantities by
dynamic programming; and the forward-backward log-evidence agrees with
scipy's multivariate normal density of y when the chain has one state."""
import numpy as np
import pytest

import synthetic
from oracle import closed_forms as cf


@pytest.mark.parametrize("K,T", [(2, 3), (2, 12), (3, 9), (4, 7), (5, 6), (8, 5), (1, 6)])
def test_enumeration_matches_forward_backward(orc, K, T):
    pi0, A, mu, sigma, y, _ = synthetic.hmm_instance(K=K, T=T)
    e = orc.enumerate_hmm(y, orc.hmm_hyper(pi0, A, mu, sigma))
    lz, marg = cf.hmm_forward_backward(y, pi0, A, mu, sigma)
    assert e["paths"] == K ** T
    assert abs(e["log_z"] - lz) < 1e-10 * max(1.0, abs(lz))
    assert np.max(np.abs(e["marginals"] - marg)) < 1e-10
    assert np.allclose(e["marginals"].sum(1), 1.0, atol=1e-12)
    path, lj = cf.hmm_viterbi(y, pi0, A, mu, sigma)
    assert np.array_equal(e["map"], path)
    assert abs(e["map_lw"] - lj) < 1e-10 * max(1.0, abs(lj))


def test_forward_backward_one_state_is_the_gaussian_density():
    from scipy.stats import multivariate_normal
    y = np.array([0.3, -1.2, 2.0, 0.7])
    lz, marg = cf.hmm_forward_backward(y, [1.0], [[1.0]], [0.5], 1.3)
    assert abs(lz - multivariate_normal(np.full(4, 0.5), 1.69 * np.eye(4)).logpdf(y)) < 1e-12
    assert np.all(marg == 1.0)


def test_enumeration_rejects_bad_sizes(orc):
    pi0, A, mu, sigma, y, _ = synthetic.hmm_instance(K=3, T=5)
    with pytest.raises(ValueError):
        orc.enumerate_hmm(np.zeros(0), orc.hmm_hyper(pi0, A, mu, sigma))
