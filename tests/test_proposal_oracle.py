"""Pins for the learned-proposal oracle (no GPU): finite differences for the
network and head gradients, library densities for the mixture heads, a
library least-squares solve and histogram for the summaries, quadrature for
the ordered-mixture prior density, and the closed-form evidence for the
proposal importance weights."""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.special import logsumexp

import synthetic
from oracle import closed_forms as cf


@pytest.fixture(scope="module")
def pr(orc):
    from oracle import proposal
    return proposal


def test_network_gradient_matches_finite_differences(pr):
    """Exact FP64 network (no BF16 rounding): backward() against central differences
    of the batch loss on a sample of parameters in every tensor."""
    th, S = pr.sim_poly(3, 0, 0, 6, D=200)
    params = [p.copy() for p in pr.init_params(11)]
    params[1] += 0.05                       # non-zero biases so every ReLU path is exercised
    params[3] -= 0.02

    def loss_of(ps):
        O, _ = pr.forward(ps, S, bf=False)
        return pr.head_loss_poly(O, th)[0].mean()

    O, cache = pr.forward(params, S, bf=False)
    loss, dO = pr.head_loss_poly(O, th)
    grads = pr.backward(params, cache, dO / len(th), bf=False)
    g = np.random.default_rng(0)
    for t, (p, gr) in enumerate(zip(params, grads)):
        flat = p.ravel()
        for k in g.choice(flat.size, size=min(12, flat.size), replace=False):
            h = 1e-5 * max(1.0, abs(flat[k]))
            old = flat[k]
            flat[k] = old + h; lp = loss_of(params)
            flat[k] = old - h; lm = loss_of(params)
            flat[k] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gr.ravel()[k]) <= 1e-5 * max(1.0, abs(fd)), (t, k, fd, gr.ravel()[k])


@pytest.mark.parametrize("head", ["poly", "gmm"])
def test_head_gradient_matches_finite_differences(pr, head):
    g = np.random.default_rng(1)
    O = 0.5 * g.standard_normal((3, 256))
    if head == "poly":
        th = np.zeros((3, 6))
        th[:, 0] = [2, 4, 5]
        th[:, 1:] = 3 * g.standard_normal((3, 5))
        f = lambda o: pr.head_loss_poly(o, th)
    else:
        U = g.standard_normal((3, 9))
        f = lambda o: pr.head_loss_gmm(o, U)
    loss, dO = f(O)
    for b in range(3):
        for k in range(256):
            h = 1e-6
            Op, Om = O.copy(), O.copy()
            Op[b, k] += h; Om[b, k] -= h
            fd = (f(Op)[0][b] - f(Om)[0][b]) / (2 * h)
            assert abs(fd - dO[b, k]) < 1e-6 * max(1.0, abs(fd)), (b, k, fd, dO[b, k])


def test_poly_head_density_matches_scipy(pr):
    """q(n, c) = Cat(n) * sum_m w_m prod_j N(c_j; mu, sd): against scipy densities."""
    g = np.random.default_rng(2)
    o = 0.5 * g.standard_normal(256)
    params = pr.decode_poly(o)
    for n in (2, 3, 5):
        c = 2 * g.standard_normal(n)
        mean = params[12:172].reshape(4, 8, 5)[n - 2, :, :n]
        lsd = params[172:332].reshape(4, 8, 5)[n - 2, :, :n]
        terms = [params[4 + m] + stats.multivariate_normal(mean[m], np.diag(np.exp(2 * lsd[m]))).logpdf(c)
                 for m in range(8)]
        ref = params[n - 2] + logsumexp(terms)
        assert pr.poly_logq(params, n, c) == pytest.approx(ref, abs=1e-10)
        th = np.zeros((1, 6)); th[0, 0] = n; th[0, 1:1 + n] = c
        assert -pr.head_loss_poly(o[None, :], th)[0][0] == pytest.approx(ref, abs=1e-10)


def test_gmm_head_density_matches_scipy(pr):
    g = np.random.default_rng(3)
    o = 0.5 * g.standard_normal(256)
    K = 5
    params = pr.decode_gmm(o, K)
    u = g.standard_normal(9)
    mean, lsd = params[8:80].reshape(8, 9), params[80:152].reshape(8, 9)
    ref = logsumexp([params[m] + stats.multivariate_normal(mean[m], np.diag(np.exp(2 * lsd[m]))).logpdf(u)
                     for m in range(8)])
    assert pr.gmm_logq(params, K, u) == pytest.approx(ref, abs=1e-10)
    assert -pr.head_loss_gmm(o[None, :], u[None, :])[0][0] == pytest.approx(ref, abs=1e-10)


def test_ordered_mixture_prior_density_integrates_to_one(pr):
    """K = 2: the density of u = (mu_(1), log gap, log pi_1 - log pi_2) integrates to 1
    (quadrature); K = 1 reduces to N(0, 5^2)."""
    from scipy import integrate
    assert pr.gmm_unpack([0.7], 1)[0] == pytest.approx(stats.norm.logpdf(0.7, 0, 5), abs=1e-12)

    def f(b, a2, a1):
        return math.exp(pr.gmm_unpack([a1, a2, b], 2)[0])
    val, _ = integrate.nquad(f, [[-25, 25], [-8, 4], [-30, 30]], opts={"epsrel": 1e-6, "epsabs": 1e-9, "limit": 60})
    assert val == pytest.approx(1.0, abs=2e-3)
    lp, lpi, mu = pr.gmm_unpack([-1.0, math.log(2.0), 0.5], 2)
    assert np.allclose(mu, [-1.0, 1.0]) and np.allclose(np.exp(lpi), [1 / (1 + math.exp(-0.5)), 1 / (1 + math.exp(0.5))])


def test_poly_summaries_match_library_routines(pr):
    x, y = synthetic.poly_data(D=300, seed=4)
    s = pr.summary_poly(x, y)
    o = 23
    rss = {}
    for n in range(2, 6):
        beta = np.linalg.lstsq(np.vander(x, n, increasing=True), y, rcond=None)[0]
        assert np.allclose(s[o:o + n] * 10, beta, atol=1e-9)
        rss[n] = ((y - np.vander(x, n, increasing=True) @ beta) ** 2).sum()
        o += n
    for n in range(2, 6):
        assert s[37 + n - 2] == pytest.approx(math.log1p(max(rss[n] - rss[5], 0.0) / 2) / 10, abs=1e-7)
    assert s[40] == 0.0
    assert s[41] == pytest.approx(math.log(300) / 10) and np.all(s[42:] == 0)


def test_gmm_summaries_match_library_routines(pr):
    y = synthetic.gmm_instances(1, seed=8, d_lo=2.0, d_hi=2.0 + 1e-9)[0]["y"].astype(np.float64)
    y[3] = 40.0                                           # beyond the histogram range
    s = pr.summary_gmm(y)
    srt = np.sort(y)
    assert np.allclose(s[:16] * 10, srt[(np.floor((np.arange(16) + 0.5) * y.size / 16)).astype(int)])
    hist = np.histogram(np.clip(y, -16, 15.5), bins=32, range=(-16, 16))[0] / y.size
    assert np.allclose(s[16:48], hist)
    assert s[48] * 10 == pytest.approx(y.mean()) and s[49] * 10 == pytest.approx(y.std())
    assert s[50] == pytest.approx(stats.skew(y)) and s[51] * 10 == pytest.approx(stats.kurtosis(y))


def test_simulators_draw_from_the_prior(pr):
    th, _ = pr.sim_poly(5, 3, 0, 4000, D=2)
    n = th[:, 0].astype(int)
    assert stats.chisquare(np.bincount(n, minlength=6)[2:6]).pvalue > 1e-3
    assert stats.kstest(th[:, 1] / 10, "norm").pvalue > 1e-3
    U, _ = pr.sim_gmm(5, 3, 0, 4000, D=2)
    mus = np.array([pr.gmm_unpack(u, 5)[2] for u in U[:2000]])
    assert np.all(np.diff(mus, axis=1) > 0)
    # the smallest of five N(0, 25) draws: P(min < t) = 1 - (1 - Phi(t / 5))^5
    assert stats.kstest(mus[:, 0], lambda t: 1 - (1 - stats.norm.cdf(t / 5)) ** 5).pvalue > 1e-3


def test_poly_proposal_weights_recover_the_evidence(pr):
    """Proposal IS with a hand-built proposal near the exact posterior (degree
    probabilities and per-degree Gaussians from the closed form, inflated 1.5x)
    recovers the exact log-evidence of the D = 1000 workload."""
    x, y = synthetic.poly_data(D=1000, seed=synthetic.SEED_POLY_LEARN)
    ex = cf.poly_exact(x, y)
    params = np.zeros(332)
    params[0:4] = np.log(ex["p_n"])
    params[4:12] = np.log(np.full(8, 1 / 8))
    for k, n in enumerate(range(2, 6)):
        Phi = np.vander(x, n, increasing=True)
        cov = np.linalg.inv(np.eye(n) / 100 + Phi.T @ Phi)
        mean = np.zeros((8, 5)); lsd = np.zeros((8, 5))
        mean[:, :n] = ex["means"][k]
        lsd[:, :n] = np.log(1.5 * np.sqrt(np.diag(cov)))
        params[12 + 40 * k:52 + 40 * k] = mean.ravel()
        params[172 + 40 * k:212 + 40 * k] = lsd.ravel()
    N = 1 << 15
    lw, _ = pr.propose_poly(9, params, x, y, np.arange(N))
    m = lw.max()
    w = np.exp(lw - m)
    est = m + math.log(w.mean())
    ess = w.sum() ** 2 / (w * w).sum()
    assert ess > 0.05 * N
    assert abs(est - ex["log_z"]) < 4 * math.sqrt(1 / ess)


def test_gmm_proposal_weights_agree_with_prior_is(pr):
    """On a small instance (K = 2, D = 12) the proposal-IS estimate with a broad
    hand-built proposal and the prior-IS estimate (both oracle) agree."""
    K = 2
    g = np.random.default_rng(6)
    y = np.concatenate([g.normal(-2, 1, 6), g.normal(3, 1, 6)])
    params = np.zeros(8 + 2 * 8 * 3)
    params[0:8] = np.log(1 / 8)
    params[8:32] = np.tile([-2.0, math.log(5.0), 0.0], 8)
    params[32:56] = np.tile([math.log(1.2), math.log(0.6), math.log(1.5)], 8)
    N = 1 << 18
    lw, _ = pr.propose_gmm(4, params, K, y, np.arange(N))
    lp = pr.gmm_prior_lw(4, K, y, np.arange(N))

    def est(v):
        m = v.max(); w = np.exp(v - m)
        return m + math.log(w.mean()), w.sum() ** 2 / (w * w).sum()
    (a, ea), (b, eb) = est(lw), est(lp)
    assert ea > 1000 and eb > 100
    assert abs(a - b) < 4 * math.sqrt(1 / ea + 1 / eb)


def test_glorot_init_is_uniform_within_bounds(pr):
    """Weights are U(-a, a) with a = sqrt(6 / (in + out)) (variance 2 / (in + out)); biases zero."""
    params = pr.init_params(3)
    for l, (o, i) in enumerate(pr.SHAPES):
        W, b = params[2 * l], params[2 * l + 1]
        a = math.sqrt(6.0 / (i + o))
        assert W.shape == (o, i) and np.all(b == 0)
        assert np.all(np.abs(W) < a * (1 + 1e-6))
        assert stats.kstest(W.ravel() / a, "uniform", args=(-1, 2)).pvalue > 1e-3
        assert abs(W.var() / (2.0 / (i + o)) - 1) < 0.05


def test_adam_with_a_constant_gradient_moves_lr_per_step(pr):
    """Bias-corrected Adam under a constant gradient g: m_t / (1 - b1^t) = g and
    v_t / (1 - b2^t) = g^2 at every step, so each step moves p by lr g / (|g| + eps)."""
    g = [np.array([[3.0, -2e-3], [0.5, -7.0]]), np.array([1e-4, -40.0])]
    p = [np.zeros((2, 2)), np.zeros(2)]
    m = [np.zeros_like(x) for x in p]
    v = [np.zeros_like(x) for x in p]
    lr, eps = 1e-3, 1e-8
    for t in range(1, 6):
        p, m, v = pr.adam(p, g, m, v, t, lr=lr, eps=eps)
        for pk, gk in zip(p, g):
            np.testing.assert_allclose(pk, -t * lr * gk / (np.abs(gk) + eps), rtol=1e-10)
