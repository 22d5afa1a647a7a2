"""Exact answers that pin the oracle (TEST INFRASTRUCTURE ONLY).

Each function is the textbook closed form of a quantity the sampler estimates;
the tests check these forms against a library routine (a multivariate normal
density) or quadrature before using them to judge the oracle.

* ``poly_exact`` -- the polynomial model of the paper's running example
  (Sec. 1.1, figure "ppl-example2") is conjugate given the degree: with
  c ~ N(0, s^2 I_n) and the factor exp(-|y - Phi c|^2 / 2), the evidence of
  degree n is a Gaussian integral, and exact inference over the finite support
  of n is the enumeration of Sec. 3.6.1.
* ``blr_exact`` -- Bayesian linear regression with a Gaussian prior and
  Gaussian observations: Gaussian posterior, Gaussian marginal likelihood.
* ``kalman`` -- the exact log-evidence of the linear-Gaussian state-space model
  (Kalman filter prediction-error decomposition).
"""
import math

import numpy as np


def poly_design(x, n):
    x = np.asarray(x, dtype=np.float64)
    return np.vander(x, n, increasing=True)          # Phi_ij = x_i^j


def poly_exact(x, y, sd=10.0, degrees=(2, 3, 4, 5)):
    """Exact evidence of the polynomial model (unit-scale factor, no 2*pi constant).

    For each number of coefficients n:  A_n = I/s^2 + Phi^T Phi,
      log Z_n = -1/2 log|I + s^2 Phi^T Phi| - 1/2 (y^T y - y^T Phi A_n^{-1} Phi^T y),
      E[c | n, y] = A_n^{-1} Phi^T y.
    n is uniform on ``degrees``; log Z = log sum_n Z_n / |degrees|.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    logzn, means = [], []
    for n in degrees:
        Phi = poly_design(x, n)
        G = Phi.T @ Phi
        A = np.eye(n) / sd ** 2 + G
        b = Phi.T @ y
        mu = np.linalg.solve(A, b)
        _, logdet = np.linalg.slogdet(np.eye(n) + sd ** 2 * G)
        logzn.append(-0.5 * logdet - 0.5 * (y @ y - b @ mu))
        means.append(mu)
    logzn = np.array(logzn)
    lp = logzn - math.log(len(degrees))
    mx = lp.max()
    log_z = mx + math.log(np.exp(lp - mx).sum())
    post = np.exp(lp - log_z)
    return dict(log_z=log_z, log_zn=logzn, p_n=post, means=means)


def poly_logzn_mvn(x, y, n, sd=10.0):
    """Same Z_n through a library density: the factor is (2 pi)^{D/2} N(y; Phi c, I),
    so Z_n = (2 pi)^{D/2} N(y; 0, I + s^2 Phi Phi^T)."""
    from scipy.stats import multivariate_normal
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    Phi = poly_design(x, n)
    C = np.eye(x.size) + sd ** 2 * Phi @ Phi.T
    return 0.5 * x.size * math.log(2 * math.pi) + multivariate_normal(np.zeros(x.size), C).logpdf(y)


def blr_exact(X, y, prior_sd=1.0, noise_sd=0.5):
    """Gaussian posterior N(mu, Sigma) and log marginal likelihood of BLR.

    A = I/s^2 + X^T X / sigma^2,  mu = A^{-1} X^T y / sigma^2,  Sigma = A^{-1},
    log Z = -D/2 log(2 pi sigma^2) - 1/2 log|s^2 A| - 1/2 (y^T y / sigma^2 - mu^T A mu).
    """
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    D, d = X.shape
    s2, v = prior_sd ** 2, noise_sd ** 2
    A = np.eye(d) / s2 + X.T @ X / v
    b = X.T @ y / v
    mu = np.linalg.solve(A, b)
    Sigma = np.linalg.inv(A)
    _, logdet = np.linalg.slogdet(s2 * A)
    log_z = -0.5 * D * math.log(2 * math.pi * v) - 0.5 * logdet - 0.5 * (y @ y / v - mu @ A @ mu)
    return dict(log_z=log_z, mean=mu, cov=0.5 * (Sigma + Sigma.T))


def blr_logz_mvn(X, y, prior_sd=1.0, noise_sd=0.5):
    """Marginal likelihood through a library density: y ~ N(0, s^2 X X^T + sigma^2 I)."""
    from scipy.stats import multivariate_normal
    X = np.asarray(X, dtype=np.float64)
    C = prior_sd ** 2 * X @ X.T + noise_sd ** 2 * np.eye(X.shape[0])
    return multivariate_normal(np.zeros(X.shape[0]), C).logpdf(np.asarray(y, dtype=np.float64))


def kalman(y, a=0.9, q_sd=1.0, r_sd=0.5, m0=0.0, p0=0.0):
    """Exact log p(y_1..y_T) of x_t = a x_{t-1} + q eps, y_t = x_t + r eta, x_0 ~ N(m0, p0)."""
    m, P, log_z = m0, p0, 0.0
    q2, r2 = q_sd ** 2, r_sd ** 2
    for yt in np.asarray(y, dtype=np.float64):
        mp = a * m
        Pp = a * a * P + q2
        S = Pp + r2
        e = yt - mp
        log_z += -0.5 * math.log(2 * math.pi * S) - 0.5 * e * e / S
        K = Pp / S
        m = mp + K * e
        P = (1 - K) * Pp
    return log_z


def lgssm_logz_mvn(y, a=0.9, q_sd=1.0, r_sd=0.5, m0=0.0, p0=0.0):
    """Same evidence through a library density of the joint Gaussian of y_1..y_T."""
    from scipy.stats import multivariate_normal
    y = np.asarray(y, dtype=np.float64)
    T = y.size
    var = np.empty(T)
    v = p0
    for t in range(T):
        v = a * a * v + q_sd ** 2
        var[t] = v
    C = np.empty((T, T))
    for s in range(T):
        for t in range(T):
            lo, hi = min(s, t), max(s, t)
            C[s, t] = a ** (hi - lo) * var[lo]
    C += r_sd ** 2 * np.eye(T)
    mean = m0 * a ** np.arange(1, T + 1)
    return multivariate_normal(mean, C).logpdf(y)


def gmm1_exact(y, mu_sd=5.0, comp_sd=1.0):
    """The mixture model with one component: mu ~ N(0, mu_sd^2), y_d ~ N(mu,
    comp_sd^2) is Gaussian-conjugate.  Returns (log Z, posterior mean,
    posterior variance) of mu given y: precision 1/mu_sd^2 + D/comp_sd^2;
    y ~ N(0, comp_sd^2 I + mu_sd^2 1 1^T), whose log density uses the
    matrix-determinant lemma and the Sherman-Morrison inverse."""
    y = np.asarray(y, dtype=np.float64)
    D = y.size
    prec = 1.0 / mu_sd ** 2 + D / comp_sd ** 2
    mean = (y.sum() / comp_sd ** 2) / prec
    s2, t2 = comp_sd ** 2, mu_sd ** 2
    logdet = D * math.log(s2) + math.log1p(D * t2 / s2)
    quad = (y @ y) / s2 - (t2 / s2 ** 2) * y.sum() ** 2 / (1.0 + D * t2 / s2)
    logz = -0.5 * (D * math.log(2 * math.pi) + logdet + quad)
    return logz, mean, 1.0 / prec


def hmm_forward_backward(y, pi0, A, mu, sigma=1.0):
    """Textbook forward-backward recursions of a hidden Markov model with
    Gaussian emissions (scaled to avoid underflow): log Z and the posterior
    marginals P(z_t = k | y)."""
    y = np.asarray(y, np.float64)
    pi0, A, mu = np.asarray(pi0, np.float64), np.asarray(A, np.float64), np.asarray(mu, np.float64)
    T, K = y.size, pi0.size
    from scipy.stats import norm
    e = norm.pdf(y[:, None], mu[None, :], sigma)          # [T, K]
    alpha = np.zeros((T, K))
    c = np.zeros(T)
    a = pi0 * e[0]
    c[0] = a.sum()
    alpha[0] = a / c[0]
    for t in range(1, T):
        a = (alpha[t - 1] @ A) * e[t]
        c[t] = a.sum()
        alpha[t] = a / c[t]
    beta = np.ones((T, K))
    for t in range(T - 2, -1, -1):
        beta[t] = (A @ (e[t + 1] * beta[t + 1])) / c[t + 1]
    return float(np.log(c).sum()), alpha * beta


def hmm_viterbi(y, pi0, A, mu, sigma=1.0):
    """Textbook Viterbi recursion: the most probable path and its log joint."""
    y = np.asarray(y, np.float64)
    from scipy.stats import norm
    le = norm.logpdf(y[:, None], np.asarray(mu)[None, :], sigma)
    lA = np.log(np.asarray(A, np.float64))
    T, K = le.shape
    d = np.log(np.asarray(pi0, np.float64)) + le[0]
    back = np.zeros((T, K), dtype=int)
    for t in range(1, T):
        cand = d[:, None] + lA
        back[t] = np.argmax(cand, axis=0)
        d = cand[back[t], np.arange(K)] + le[t]
    path = np.zeros(T, dtype=int)
    path[-1] = int(np.argmax(d))
    for t in range(T - 1, 0, -1):
        path[t - 1] = back[t, path[t]]
    return path, float(d.max())
