"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the inference method: it only generates
observed data (and synthetic log-weight vectors) with numpy's own PCG64
generator, so that the HIP path and the CPU oracle receive identical inputs.
Single-precision workloads are generated in double and rounded once to
float32; both sides then read the same float32 values.

Workload recipes (sizes and distributions of the configurations measured):
  poly  : D points, x ~ U[-1, 1], y = 0.5 - 1.2 x + 0.8 x^3 + N(0, 0.1^2)   (float64)
  blr   : X ~ N(0, 1) [D x d], w* ~ N(0, I_d), y = X w* + N(0, 0.5^2)     (float32)
  lgssm : x_0 = 0, x_t = 0.9 x_{t-1} + N(0, 1), y_t = x_t + N(0, 0.5^2)     (float32)
  gmm   : per instance K ~ U{3..8}, pi* ~ Dirichlet(1_K), mu* ~ N(0, 5^2),
          D = floor(10^U[2, 5]), z_d ~ Cat(pi*), y_d = mu*_{z_d} + N(0, 1)  (float32)
  learned-proposal workloads: poly with D = 1000 (seed SEED_POLY_LEARN); one
          gmm instance with K = 5 and D = 100 (gmm_learn_data)
"""
import numpy as np

SEED_POLY, SEED_BLR, SEED_LGSSM, SEED_GMM, SEED_POLY_LEARN, SEED_GMM_LEARN = 1000, 1001, 1002, 1003, 1004, 1005
SEED_HMM = 1006


def poly_data(D=100, seed=SEED_POLY):
    g = np.random.default_rng(seed)
    x = g.uniform(-1.0, 1.0, D)
    y = 0.5 - 1.2 * x + 0.8 * x ** 3 + 0.1 * g.standard_normal(D)
    return x.astype(np.float64), y.astype(np.float64)


def blr_data(D=10_000, d=16, seed=SEED_BLR, noise_sd=0.5):
    g = np.random.default_rng(seed)
    X = g.standard_normal((D, d)).astype(np.float32)
    w = g.standard_normal(d)
    y = (X.astype(np.float64) @ w + noise_sd * g.standard_normal(D)).astype(np.float32)
    return X, y, w


def lgssm_data(T=1000, seed=SEED_LGSSM, a=0.9, q_sd=1.0, r_sd=0.5):
    g = np.random.default_rng(seed)
    x = 0.0
    y = np.empty(T)
    for t in range(T):
        x = a * x + q_sd * g.standard_normal()
        y[t] = x + r_sd * g.standard_normal()
    return y.astype(np.float32)


def gmm_instances(n_inst=256, seed=SEED_GMM, d_lo=2.0, d_hi=5.0, k_lo=3, k_hi=8, mu_sd=5.0):
    """List of instances {K, D, y (float32), pi, mu} of the batched-mixture workload."""
    g = np.random.default_rng(seed)
    out = []
    for _ in range(n_inst):
        K = int(g.integers(k_lo, k_hi + 1))
        pi = g.dirichlet(np.ones(K))
        mu = mu_sd * g.standard_normal(K)
        D = int(np.floor(10.0 ** g.uniform(d_lo, d_hi)))
        z = g.choice(K, size=D, p=pi)
        y = (mu[z] + g.standard_normal(D)).astype(np.float32)
        out.append(dict(K=K, D=D, y=y, pi=pi, mu=mu))
    return out


def gmm_learn_data(K=5, D=100, seed=SEED_GMM_LEARN, mu_sd=5.0):
    """One mixture dataset of the gmm recipe with fixed K and D (float32)."""
    g = np.random.default_rng(seed)
    pi = g.dirichlet(np.ones(K))
    mu = mu_sd * g.standard_normal(K)
    z = g.choice(K, size=D, p=pi)
    return (mu[z] + g.standard_normal(D)).astype(np.float32)


def hmm_instance(K=4, T=14, seed=SEED_HMM, sigma=1.0):
    """A hidden Markov model with K states and T observations: pi0 ~
    Dirichlet(1); transition rows ~ Dirichlet(1) plus 3 on the diagonal
    (sticky), normalised; state means spaced 2 apart with jitter; a path
    drawn from the chain and y_t = mu[z_t] + N(0, sigma^2).
    Returns (pi0, A, mu, sigma, y, z)."""
    g = np.random.default_rng(seed + 31 * K + T)
    pi0 = g.dirichlet(np.ones(K))
    A = g.dirichlet(np.ones(K), size=K) + 3.0 * np.eye(K)
    A /= A.sum(1, keepdims=True)
    mu = 2.0 * (np.arange(K) - (K - 1) / 2.0) + 0.3 * g.standard_normal(K)
    z = np.zeros(T, dtype=int)
    z[0] = g.choice(K, p=pi0)
    for t in range(1, T):
        z[t] = g.choice(K, p=A[z[t - 1]])
    y = mu[z] + sigma * g.standard_normal(T)
    return pi0, A, mu, sigma, y.astype(np.float64), z


def logweights(n, kind="normal", seed=0, scale=10.0):
    """Synthetic float32 log-weight vectors for the normaliser / resampling checks.

    kinds: normal (N(0, scale^2)), spread (uniform on [-scale, 0]), equal (all 0),
    dominant (one entry at 0, the rest at -scale - U[0,1]), neginf (normal with a
    quarter of entries -inf), large (N(-3e5, scale^2): magnitudes of real runs).
    """
    g = np.random.default_rng(seed)
    if kind == "normal":
        v = scale * g.standard_normal(n)
    elif kind == "spread":
        v = -scale * g.uniform(0.0, 1.0, n)
    elif kind == "equal":
        v = np.zeros(n)
    elif kind == "dominant":
        v = -scale - g.uniform(0.0, 1.0, n)
        v[g.integers(0, n)] = 0.0
    elif kind == "neginf":
        v = scale * g.standard_normal(n)
        v[g.uniform(size=n) < 0.25] = -np.inf
        v[g.integers(0, n)] = 0.0
    elif kind == "large":
        v = -3.0e5 + scale * g.standard_normal(n)
    else:
        raise ValueError(kind)
    return v.astype(np.float32)
