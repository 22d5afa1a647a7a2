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


def test_bf16_rounding_matches_torch(pr):
    """The oracle's BF16 rounding (round to nearest, ties to even, applied where
    the GPU stores BF16) against torch's float32 -> bfloat16 conversion on the
    CPU: random values over the whole exponent range, exact halfway cases with
    an even and an odd kept bit, values just either side of a halfway point,
    subnormals, overflow to infinity, signed zeros, infinities and NaNs."""
    import torch
    g = np.random.default_rng(17)
    bits = [g.integers(0, 2 ** 32, size=200_000, dtype=np.uint64).astype(np.uint32)]
    kept = g.integers(0, 2 ** 16, size=4000, dtype=np.uint64).astype(np.uint32) << 16
    for low in (0x8000, 0x7FFF, 0x8001, 0x0000, 0xFFFF):      # halfway, just below, just above, exact, top
        bits.append(kept | np.uint32(low))
    specials = [0x00000000, 0x80000000, 0x7F800000, 0xFF800000, 0x7FC00000, 0xFFC00000, 0x7FFFFFFF,
                0x7F800001, 0x00000001, 0x00008000, 0x00018000, 0x007FFFFF, 0x00800000, 0x7F7FFFFF,
                0x7F7F8000, 0x7F7F7FFF, 0xFF7FFFFF, 0x3F808000, 0x3F818000, 0x3F7FFFFF]
    bits.append(np.array(specials, dtype=np.uint32))
    f = np.concatenate(bits).view(np.float32)
    ours = pr.bf16(f)
    ref = torch.from_numpy(f.copy()).to(torch.bfloat16).to(torch.float64).numpy()
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(ours), nan)
    assert np.array_equal(ours[~nan], ref[~nan])
    assert np.array_equal(np.signbit(ours[~nan]), np.signbit(ref[~nan]))       # -0 stays -0


def _box_muller(w1, w2):
    """Single-precision-stream uniforms ((w >> 9) + 1/2) 2^-23 and the textbook
    Box-Muller pair (written here from its definition, not taken from the oracle)."""
    u1 = ((np.asarray(w1, np.uint64) >> 9).astype(np.float64) + 0.5) * 2.0 ** -23
    u2 = ((np.asarray(w2, np.uint64) >> 9).astype(np.float64) + 0.5) * 2.0 ** -23
    r = np.sqrt(-2.0 * np.log(u1))
    return r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)


def _u01(w):
    return ((np.asarray(w, np.uint64) >> 9).astype(np.float64) + 0.5) * 2.0 ** -23


def _words(orc, seed, i, blocks, step):
    ctr = np.zeros((len(blocks), 4), dtype=np.uint32)
    ctr[:, 0] = i
    ctr[:, 1] = blocks
    ctr[:, 2] = step
    ctr[:, 3] = 4                      # training-simulation tag
    return orc.philox(ctr, seed)


def _rebuild_poly_pair(orc, seed, step, i, D, sd=10.0, noise_sd=1.0):
    """Data of one simulated polynomial pair from its stream words: block 0 word 0
    gives the degree, blocks 1-2 the coefficient normals, block 8 + e the points
    2e, 2e + 1 (x = 2u - 1 from words 0, 1; noise from the Box-Muller pair of
    words 2, 3)."""
    w0 = _words(orc, seed, i, [0, 1, 2], step)
    n = 2 + int((int(w0[0, 0]) * 4) >> 32)
    z = []
    for b in (1, 2):
        for (a, c) in ((0, 1), (2, 3)):
            z0, z1 = _box_muller(w0[b, a], w0[b, c])
            z += [float(z0), float(z1)]
    c = sd * np.array(z[:5])
    ne = (D + 1) // 2
    wd = _words(orc, seed, i, 8 + np.arange(ne), step)
    x = (2.0 * _u01(wd[:, :2]) - 1.0).ravel()[:D]
    e0, e1 = _box_muller(wd[:, 2], wd[:, 3])
    eps = np.stack([e0, e1], axis=1).ravel()[:D]
    mean = np.polynomial.polynomial.polyval(x, c[:n])
    return n, c, x, mean + noise_sd * eps, eps


def test_poly_simulator_data_rebuilt_from_the_stream(orc, pr):
    """The simulator's data (x, y) is what its documented word table says: the
    summaries of data rebuilt here from the Philox words (independently of the
    oracle's simulator) equal the summaries the simulator returns, and over many
    pairs x is uniform on [-1, 1] and the residuals (y - poly(x)) / noise_sd are
    standard normal."""
    seed, step, D, B = 23, 7, 9, 40
    th, S = pr.sim_poly(seed, step, 0, B, D=D)
    xs, res = [], []
    for i in range(B):
        n, c, x, y, eps = _rebuild_poly_pair(orc, seed, step, i, D)
        assert th[i, 0] == n
        assert np.allclose(th[i, 1:1 + n], c[:n], rtol=1e-13, atol=1e-13)
        assert np.all(th[i, 1 + n:] == 0.0)
        s = pr.summary_poly(x, y)
        assert np.max(np.abs(s - S[i]) / np.maximum(1.0, np.abs(S[i]))) < 1e-12, i
        xs.append(x)
        res.append(y - np.polynomial.polynomial.polyval(x, c[:n]))
    # distributions over a larger draw (no summaries needed)
    big_x, big_r = [], []
    for i in range(B, B + 60):
        n, c, x, y, eps = _rebuild_poly_pair(orc, seed, step, i, 200)
        big_x.append(x)
        big_r.append(y - np.polynomial.polynomial.polyval(x, c[:n]))
    big_x, big_r = np.concatenate(big_x), np.concatenate(big_r)
    assert stats.kstest((big_x + 1) / 2, "uniform").pvalue > 1e-3
    assert stats.kstest(big_r / 1.0, "norm").pvalue > 1e-3


def test_gmm_simulator_data_rebuilt_from_the_stream(orc, pr):
    """The mixture simulator: blocks 0-1 give Exp(1) draws (pi = E / sum E),
    blocks 2-3 the component means, block 8 + e the components of points 2e,
    2e + 1 (categorical on pi from words 0, 1) and their noise (words 2, 3).
    Summaries of the rebuilt data equal the simulator's; its ordered latents are
    those of the rebuilt parameters; components follow pi (chi-square) and the
    residuals are standard normal (KS)."""
    seed, step, D, K, B = 31, 4, 50, 5, 30
    U, S = pr.sim_gmm(seed, step, 0, B, D=D, K=K)
    comp_counts, comp_exp, resid = np.zeros(K), np.zeros(K), []
    for i in range(B + 200):
        w = _words(orc, seed, i, [0, 1, 2, 3], step)
        E = -np.log(_u01(np.concatenate([w[0], w[1]])[:K]))
        pi = E / E.sum()
        z = []
        for b in (2, 3):
            for (a, c) in ((0, 1), (2, 3)):
                z0, z1 = _box_muller(w[b, a], w[b, c])
                z += [float(z0), float(z1)]
        mu = 5.0 * np.array(z[:K])
        Dn = D if i < B else 200
        wd = _words(orc, seed, i, 8 + np.arange((Dn + 1) // 2), step)
        uc = _u01(wd[:, :2]).ravel()[:Dn]
        cum = np.cumsum(pi)
        k = np.minimum(np.searchsorted(cum, uc, side="right"), K - 1)   # first k with u < C_k
        e0, e1 = _box_muller(wd[:, 2], wd[:, 3])
        eps = np.stack([e0, e1], axis=1).ravel()[:Dn]
        y = mu[k] + eps
        if i < B:
            s = pr.summary_gmm(y)
            assert np.max(np.abs(s - S[i]) / np.maximum(1.0, np.abs(S[i]))) < 1e-12, i
            o = np.argsort(mu, kind="stable")
            ref = np.concatenate([[mu[o[0]]], np.log(np.diff(mu[o])), np.log(pi[o[:-1]]) - np.log(pi[o[-1]])])
            assert np.allclose(U[i], ref, rtol=1e-12, atol=1e-12), i
        else:
            comp_counts += np.bincount(k, minlength=K)
            comp_exp += pi * Dn
            resid.append(y - mu[k])
    # per-dataset weights differ, so compare the pooled counts with their pooled expectation
    chi2 = float(np.sum((comp_counts - comp_exp) ** 2 / comp_exp))
    assert stats.chi2.sf(chi2, K - 1) > 1e-4
    assert stats.kstest(np.concatenate(resid), "norm").pvalue > 1e-3
