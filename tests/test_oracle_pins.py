"""Pins for the CPU oracle: every check here compares the oracle with something
other than itself -- an independent library (rocRAND, scipy, mpmath), a closed
form that is itself checked against a library density or quadrature, a
hand-worked value, an exact special case, or an invariant of the method.
No GPU is needed."""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

import synthetic
from oracle import closed_forms as cf

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------ Philox --
@pytest.fixture(scope="module")
def rocrand_philox():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    d = tempfile.mkdtemp(prefix="rr_philox_")
    exe = os.path.join(d, "rr_philox")
    subprocess.check_call([hipcc, "--offload-host-only", "-O1", "-o", exe,
                           os.path.join(HERE, "pins", "rocrand_philox.cpp")])
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(orc, rocrand_philox):
    g = np.random.default_rng(7)
    n = 3000
    ctr = g.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:, 1] &= (1 << 29) - 1                      # the reference maps c1 into a 64-bit offset
    ctr[:20] = 0
    ctr[20:40, 0] = np.arange(20)                  # consecutive particle counters
    seeds = g.integers(0, 2 ** 63, size=n, dtype=np.uint64)
    seeds[:10] = 0
    lines = "\n".join(f"{a} {b} {c} {d} {s}" for (a, b, c, d), s in zip(ctr.tolist(), seeds.tolist()))
    out = subprocess.run([rocrand_philox], input=lines, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(v) for v in ln.split()] for ln in out.strip().splitlines()], dtype=np.uint64)
    got = orc.philox(ctr, seeds).astype(np.uint64)
    assert ref.shape == got.shape
    np.testing.assert_array_equal(got, ref)


def test_philox_words_uniform_bytes(orc):
    """Byte histogram of 2^18 words is flat (chi-square), consecutive counters differ."""
    n = 1 << 16
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n)
    w = orc.philox(ctr, 12345).ravel()
    b = w.view(np.uint8)
    counts = np.bincount(b, minlength=256)
    chi2 = ((counts - b.size / 256) ** 2 / (b.size / 256)).sum()
    assert stats.chi2.sf(chi2, 255) > 1e-4
    assert np.unique(w).size > 0.999 * w.size


# ---------------------------------------------------------------- uniforms --
def test_uniform_single_exact(orc):
    assert orc.u01_single(0) == 2.0 ** -24
    assert orc.u01_single(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert orc.u01_single(512) == 1.5 * 2.0 ** -23
    assert orc.u01_single(511) == 2.0 ** -24           # low 9 bits are dropped
    g = np.random.default_rng(1)
    for w in g.integers(0, 2 ** 32, 200):
        u = orc.u01_single(int(w))
        assert float(np.float32(u)) == u and 0.0 < u < 1.0


def test_uniform_double_exact(orc):
    assert orc.u01_double(0, 0) == 2.0 ** -53
    assert orc.u01_double(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert orc.u01_double(0, 0x80000000) == 0.5 + 2.0 ** -53
    assert orc.u01_double(1 << 12, 0) == 3 * 2.0 ** -53  # lowest kept bit of the low word


def test_uniform_discrete_exact(orc):
    assert orc.uniform_discrete(0, 2, 5) == 2
    assert orc.uniform_discrete(0xFFFFFFFF, 2, 5) == 5
    assert orc.uniform_discrete(1 << 30, 2, 5) == 3
    assert orc.uniform_discrete((1 << 30) - 1, 2, 5) == 2
    assert orc.uniform_discrete(3 << 30, 2, 5) == 5


# ------------------------------------------------------------- Box-Muller --
def test_box_muller_special_cases(orc):
    u1 = math.exp(-0.5)                                 # radius exactly 1
    z0, z1 = orc.box_muller(u1, 0.0)
    assert z0 == pytest.approx(1.0, abs=1e-15) and z1 == pytest.approx(0.0, abs=1e-15)
    z0, z1 = orc.box_muller(u1, 0.25)
    assert z0 == pytest.approx(0.0, abs=1e-15) and z1 == pytest.approx(1.0, abs=1e-15)
    z0, z1 = orc.box_muller(u1, 0.5)
    assert z0 == pytest.approx(-1.0, abs=1e-15) and z1 == pytest.approx(0.0, abs=1e-15)
    z0, z1 = orc.box_muller(math.exp(-2.0), 0.125)      # radius 2, angle pi/4
    assert z0 == pytest.approx(math.sqrt(2.0), abs=1e-14) and z1 == pytest.approx(math.sqrt(2.0), abs=1e-14)


def test_stream_normals_distribution(orc):
    """Normals of the BLR stream (single-precision uniforms) are N(0,1): KS, moments,
    no correlation between the two outputs of a pair or between pairs."""
    z = np.array([orc.blr_draw_std(99, i) for i in range(8000)])     # 128k normals
    flat = z.ravel()
    assert stats.kstest(flat, "norm").pvalue > 1e-3
    assert abs(flat.mean()) < 4 / math.sqrt(flat.size)
    assert abs(flat.var() - 1) < 4 * math.sqrt(2 / flat.size)
    for a, b in ((0, 1), (1, 2), (0, 4), (3, 15)):
        r = np.corrcoef(z[:, a], z[:, b])[0, 1]
        assert abs(r) < 4 / math.sqrt(z.shape[0])


def test_poly_prior_draws(orc):
    """Degree is uniform on {2..5} (chi-square) and coefficients are N(0, 10^2) (KS)."""
    draws = [orc.poly_draw(5, i) for i in range(20000)]
    n = np.array([d[0] for d in draws])
    counts = np.bincount(n, minlength=6)[2:6]
    assert counts.sum() == n.size
    assert stats.chisquare(counts).pvalue > 1e-3
    c = np.array([d[1] for d in draws])
    assert stats.kstest(c[:, :5].ravel() / 10.0, "norm").pvalue > 1e-3


# ------------------------------------------------------------- POLY model --
def test_poly_loglik_worked_examples(orc):
    # n = 2, c = (1, 2): p(0.5) = 2; y = 3 -> -1/2 * 1^2
    assert orc.poly_loglik(2, [1.0, 2.0], [0.5], [3.0]) == -0.5
    # n = 3, c = (1, 0, 1): p(2) = 5, p(-1) = 2; y = (5, 0) -> -1/2 * (0 + 4)
    assert orc.poly_loglik(3, [1.0, 0.0, 1.0], [2.0, -1.0], [5.0, 0.0]) == -2.0
    # n = 5, c = (0,0,0,0,1): p(x) = x^4; x = 2, y = 0 -> -128
    assert orc.poly_loglik(5, [0, 0, 0, 0, 1.0], [2.0], [0.0]) == -128.0


def test_poly_closed_form_matches_library_density():
    x, y = synthetic.poly_data(D=40, seed=3)
    ex = cf.poly_exact(x, y)
    for k, n in enumerate((2, 3, 4, 5)):
        assert ex["log_zn"][k] == pytest.approx(cf.poly_logzn_mvn(x, y, n), abs=1e-9)
    assert ex["p_n"].sum() == pytest.approx(1.0, abs=1e-14)


def test_poly_closed_form_matches_quadrature():
    """D = 2, n = 2: Z_2 as a 2-D integral of prior density times factor (scipy nquad)."""
    from scipy import integrate
    x = np.array([-0.4, 0.7])
    y = np.array([0.3, -0.2])
    s = 10.0

    def f(c1, c0):
        r = y - (c0 + c1 * x)
        return math.exp(-0.5 * (r @ r)) * stats.norm.pdf(c0, 0, s) * stats.norm.pdf(c1, 0, s)
    Z, _ = integrate.nquad(f, [[-60, 60], [-60, 60]], opts={"epsabs": 1e-14, "epsrel": 1e-10, "limit": 200})
    ex = cf.poly_exact(x, y, degrees=(2,))
    assert ex["log_zn"][0] == pytest.approx(math.log(Z), abs=1e-6)


def test_poly_importance_vs_enumeration(orc):
    """Likelihood-weighting IS on the D=100 workload against exact inference
    (conjugate evidence per degree, enumeration over the degree)."""
    x, y = synthetic.poly_data()
    ex = cf.poly_exact(x, y)
    N = 1 << 22
    r = orc.importance(orc.MODEL_POLY, x, y, N, seed=11)
    sig = math.sqrt(1.0 / r["ess"] - 1.0 / N)
    assert r["ess"] > 100
    assert abs(r["log_z"] - ex["log_z"]) < 4 * sig
    p = r["summaries"][:4]
    assert p.sum() == pytest.approx(1.0, abs=1e-12)
    se = np.sqrt(ex["p_n"] * (1 - ex["p_n"]) / r["ess"]) + 1e-3
    assert np.all(np.abs(p - ex["p_n"]) < 5 * se)
    # conditional coefficient mean for the dominant degree (n = 2)
    m2 = r["summaries"][4:6]
    A = np.eye(2) / 100 + cf.poly_design(x, 2).T @ cf.poly_design(x, 2)
    sd = np.sqrt(np.diag(np.linalg.inv(A)))
    assert np.all(np.abs(m2 - ex["means"][0]) < 5 * sd / math.sqrt(r["ess"]) + 5e-3)


def test_poly_zero_factor_special_case(orc):
    """No data: every factor is exp(0), so log Z-hat = 0 exactly and ESS = N; the
    degree posterior is the prior."""
    r = orc.importance(orc.MODEL_POLY, np.zeros(0), np.zeros(0), 4096, seed=2)
    assert r["log_z"] == 0.0 and r["ess"] == 4096.0
    assert np.all(np.abs(r["summaries"][:4] - 0.25) < 4 * math.sqrt(0.1875 / 4096))


# -------------------------------------------------------------- BLR model --
def test_blr_closed_form_matches_library_density():
    X, y, _ = synthetic.blr_data(D=60, d=16, seed=5)
    assert cf.blr_exact(X, y)["log_z"] == pytest.approx(cf.blr_logz_mvn(X, y), abs=1e-8)


def test_blr_loglik_worked_example(orc):
    # d = 4, w = (1, 0, 0, 0), rows x = (2,0,0,0) and (0,0,0,0), y = (2, 1), sigma = 0.5:
    # residuals (0, 1): 2 * (-1/2 log(2 pi 0.25)) - 1/(2*0.25)
    X = np.array([[2.0, 0, 0, 0], [0, 0, 0, 0]])
    got = orc.blr_loglik([1.0, 0, 0, 0], X, [2.0, 1.0], 0.5)
    assert got == pytest.approx(-math.log(2 * math.pi * 0.25) - 2.0, abs=1e-14)


def test_blr_prior_importance_small(orc):
    """Prior IS on a small instance (d=4, D=10) against the closed form."""
    X, y, _ = synthetic.blr_data(D=10, d=4, seed=9)
    ex = cf.blr_exact(X, y)
    N = 1 << 19
    r = orc.importance(orc.MODEL_BLR, X, y, N, seed=3, dim=4)
    sig = math.sqrt(1.0 / r["ess"] - 1.0 / N)
    assert r["ess"] > 200
    assert abs(r["log_z"] - ex["log_z"]) < 4 * sig
    se = np.sqrt(np.diag(ex["cov"]) / r["ess"])
    assert np.all(np.abs(r["summaries"] - ex["mean"]) < 5 * se)


def test_blr_posterior_proposal_full_size(orc):
    """Full D=10^4, d=16 workload with the posterior-informed Gaussian proposal
    q = N(mu, 1.2^2 Sigma): log Z-hat and the posterior mean match the closed form."""
    X, y, _ = synthetic.blr_data()
    ex = cf.blr_exact(X, y)
    L = np.linalg.cholesky(1.44 * ex["cov"])
    N = 1 << 13
    r = orc.importance(orc.MODEL_BLR, X, y, N, seed=4, dim=16, q=(ex["mean"], L))
    assert r["ess"] > 0.2 * N
    sig = math.sqrt(1.0 / r["ess"] - 1.0 / N)
    assert abs(r["log_z"] - ex["log_z"]) < 4 * sig
    se = np.sqrt(np.diag(ex["cov"]) / r["ess"])
    assert np.all(np.abs(r["summaries"] - ex["mean"]) < 5 * se)


# --------------------------------------------------- log-sum-exp and ESS --
@pytest.mark.parametrize("kind", ["normal", "spread", "equal", "dominant", "neginf", "large"])
def test_lse_ess_vs_mpmath(orc, kind):
    import mpmath
    mpmath.mp.dps = 50
    lw = synthetic.logweights(3000, kind, seed=17, scale=1e3 if kind == "spread" else 10.0).astype(np.float64)
    got = orc.lse_ess(lw)
    fin = [mpmath.mpf(float(v)) for v in lw if np.isfinite(v)]
    s1 = mpmath.fsum(mpmath.exp(v) for v in fin)
    s2 = mpmath.fsum(mpmath.exp(2 * v) for v in fin)
    lse = mpmath.log(s1)
    ess = s1 * s1 / s2
    assert abs(got["lse"] - float(lse)) <= 1e-14 * max(1.0, abs(float(lse)))
    assert abs(got["ess"] - float(ess)) <= 1e-13 * float(ess)


def test_lse_special_cases(orc):
    r = orc.lse_ess([0.0])
    assert r["lse"] == 0.0 and r["ess"] == 1.0
    r = orc.lse_ess(np.full(1024, -7.5))
    assert r["lse"] == pytest.approx(-7.5 + math.log(1024), abs=1e-14) and r["ess"] == pytest.approx(1024, rel=1e-14)
    r = orc.lse_ess(np.full(8, -np.inf))
    assert r["lse"] == -np.inf and r["ess"] == 0.0


# -------------------------------------------------------------- resampling --
@pytest.mark.parametrize("kind", ["normal", "spread", "dominant", "neginf"])
@pytest.mark.parametrize("n", [1, 7, 1000, 4096])
def test_resample_integer_rule_vs_textbook(orc, kind, n):
    """The integer rule is systematic resampling: it agrees with textbook FP64
    systematic resampling except at slots within the quantisation band of a
    boundary, and its offspring counts are floor/ceil of N W_a."""
    lw = synthetic.logweights(n, kind, seed=n + 3, scale=3.0).astype(np.float64)
    for step in range(3):
        anc, tie = orc.resample(lw, seed=21, step=step, band=4.0 * n * 2.0 ** -orc.quant_bits(n) + 1e-12)
        ref = orc.resample_textbook(lw, seed=21, step=step)
        assert np.all(np.diff(anc) >= 0) and anc.min() >= 0 and anc.max() < n
        assert np.array_equal(anc[~tie], ref[~tie])
        assert np.all(np.abs(anc[tie] - ref[tie]) <= 1)
        w = np.exp(lw - lw.max())
        w /= w.sum()
        off = np.bincount(anc, minlength=n)
        assert off.sum() == n
        assert np.all(off >= np.floor(n * w - 1e-9)) and np.all(off <= np.ceil(n * w + 1e-9))
        assert np.all(off[np.isneginf(lw)] == 0)


def test_resample_equal_weights_identity(orc):
    """Equal weights: systematic resampling returns every particle exactly once."""
    for n in (1, 5, 1024, 1 << 16):
        anc, _ = orc.resample(np.zeros(n), seed=5, step=1)
        np.testing.assert_array_equal(anc, np.arange(n))


# ------------------------------------------------------------ LGSSM / SMC --
def test_kalman_matches_library_density():
    y = synthetic.lgssm_data(T=40, seed=8)
    assert cf.kalman(y) == pytest.approx(cf.lgssm_logz_mvn(y), abs=1e-9)
    assert cf.kalman(y, m0=0.7, p0=1.3) == pytest.approx(cf.lgssm_logz_mvn(y, m0=0.7, p0=1.3), abs=1e-9)


def test_smc_lgssm_vs_kalman(orc):
    y = synthetic.lgssm_data(T=200, seed=12)
    kf = cf.kalman(y)
    est = np.array([orc.smc(orc.MODEL_LGSSM, y, 4096, seed=s)["log_z"] for s in range(1, 33)])
    sd = est.std(ddof=1)
    assert abs(est.mean() - kf) < 4 * sd / math.sqrt(est.size) + 0.5 * sd * sd + 1e-3


def test_smc_without_resampling_is_sequential_is(orc):
    """ess_frac = 0 never resamples; every final log-weight equals the sum of
    observation log-densities along that particle's own AR(1) path, rebuilt
    here from the pinned Philox and Box-Muller conversions."""
    y = synthetic.lgssm_data(T=23, seed=2)
    r = orc.smc(orc.MODEL_LGSSM, y, 64, seed=9, ess_frac=0.0, want_state=True)
    assert r["n_resample"] == 0
    for i in (0, 5, 63):
        x, lw = 0.0, 0.0
        for s in range(y.size):
            w = orc.philox([[i, 0, s >> 2, 0]], 9)[0]
            z0, z1 = orc.box_muller(orc.u01_single(w[0]), orc.u01_single(w[1]))
            z2, z3 = orc.box_muller(orc.u01_single(w[2]), orc.u01_single(w[3]))
            x = 0.9 * x + (z0, z1, z2, z3)[s & 3]
            lw += stats.norm.logpdf(float(y[s]), x, 0.5)
        assert r["state"][0, i] == pytest.approx(x, abs=1e-12)
        assert r["lw"][i] == pytest.approx(lw, rel=1e-12)
    assert r["log_z"] == pytest.approx(orc.lse_ess(r["lw"])["lse"] - math.log(64), abs=1e-12)


def test_smc_resample_every_step(orc):
    y = synthetic.lgssm_data(T=30, seed=4)
    r = orc.smc(orc.MODEL_LGSSM, y, 256, seed=3, ess_frac=1.0)
    assert r["n_resample"] == y.size - 1
    assert not r["resampled"][-1]


# ---------------------------------------------------------------- mixture --
def test_gmm_logfactor_vs_scipy(orc):
    from scipy.special import logsumexp
    g = np.random.default_rng(4)
    for K in (1, 3, 8):
        for _ in range(20):
            pi = g.dirichlet(np.ones(K))
            mu = 5 * g.standard_normal(K)
            yv = 8 * g.standard_normal()
            ref = logsumexp(np.log(pi) + stats.norm.logpdf(yv, mu, 1.0))
            assert orc.gmm_logfactor(np.log(pi), mu, 1.0, yv) == pytest.approx(ref, abs=1e-12)
    # far from every component: still finite
    assert np.isfinite(orc.gmm_logfactor(np.log([0.5, 0.5]), [0.0, 1.0], 1.0, 200.0))


def test_gmm_prior_draws(orc):
    """pi ~ Dirichlet(1_K): each pi_k ~ Beta(1, K-1); mu_k ~ N(0, 5^2)."""
    K = 5
    st = orc.gmm_init(seed=3, inst=7, K=K, N=20000)
    pi = np.exp(st[:K])
    assert np.allclose(pi.sum(0), 1.0, atol=1e-12)
    for k in range(K):
        assert stats.kstest(pi[k], stats.beta(1, K - 1).cdf).pvalue > 1e-3
        assert stats.kstest(st[K + k] / 5.0, "norm").pvalue > 1e-3


def test_gmm_smc_vs_prior_is_reference(orc):
    """SMC log Z-hat on a small-D mixture instance against brute-force prior IS
    computed with numpy's own generator (no shared code or streams)."""
    from scipy.special import logsumexp
    inst = synthetic.gmm_instances(1, seed=77, d_lo=1.3, d_hi=1.31)[0]
    y = inst["y"].astype(np.float64)
    K = inst["K"]
    g = np.random.default_rng(123)
    chunks = []
    for _ in range(8):
        n = 1 << 17
        pi = g.dirichlet(np.ones(K), size=n)
        mu = 5 * g.standard_normal((n, K))
        comp = np.log(pi)[:, None, :] + stats.norm.logpdf(y[None, :, None], mu[:, None, :], 1.0)
        chunks.append(logsumexp(comp, axis=2).sum(1))
    lw = np.concatenate(chunks)
    ref = logsumexp(lw) - math.log(lw.size)
    w = np.exp(lw - lw.max())
    ref_se = math.sqrt(1.0 / (w.sum() ** 2 / (w * w).sum()))
    est = np.array([orc.smc(orc.MODEL_GMM, y, 4096, seed=s, K=K)["log_z"] for s in range(1, 17)])
    sd = est.std(ddof=1)
    assert abs(est.mean() - ref) < 4 * math.sqrt(sd * sd / est.size + ref_se ** 2) + 0.5 * sd * sd
