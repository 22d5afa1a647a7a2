"""GPU parity of exact inference by enumeration (every path of a hidden Markov
model) against the CPU oracle, through the C ABI.

Both sides sum every path's weight relative to the largest in FP64, in
different orders and by different routes: the oracle as exp(lw - max) with
each log-weight summed site by site, the GPU as a product of exp(lw_j + q_j -
max) and a tabulated suffix factor.  A log-weight carries an absolute
rounding error of about T u |lw| (T <= 40, |lw| <= a few hundred: ~1e-12),
which is the relative error it gives the weight, and a sequential sum of n
positive terms a relative error of at most (n - 1) u (n <= 2^24 at the
oracle's sizes: ~2e-9, typically far less), so log Z and the marginals are
compared within 2e-9.  The most probable path must be the oracle's, unless the oracle puts
the GPU's path within 1e-12 (relative) of its maximum (a rounding tie).  At
the measured size (2^40 paths) the oracle would take minutes; there log Z and
the marginals are compared with the forward-backward recursions and the path
with Viterbi, properties of the exact result that hold at any size."""
import math

import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ppl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_08454_amd as p
    return p


def run_gpu(ppl, y, pi0, A, mu, sigma, sync=True):
    import torch
    dev = torch.device("cuda:0")
    T, K = len(y), len(pi0)
    dy = torch.from_numpy(np.ascontiguousarray(y, np.float64)).to(dev)
    data = ppl.hmm_data(dy, pi0, A, mu, sigma)
    scal = torch.full((4,), 7.0, dtype=torch.float64, device=dev)
    marg = torch.full((T, K), -1.0, dtype=torch.float64, device=dev)
    mp = torch.full((T,), -1, dtype=torch.int32, device=dev)
    r = ppl.ppl_enumerate(ppl.PPL_MODEL_HMM, data, scalars=scal, marginals=marg, map_path=mp, sync=sync)
    torch.cuda.synchronize()
    return dict(res=r, scal=scal.cpu().numpy(), marg=marg.cpu().numpy(), map=mp.cpu().numpy())


def path_lw(y, pi0, A, mu, sigma, z):
    """Log joint of one path, summed in FP64 in site order (test-side)."""
    lw = math.log(pi0[z[0]])
    for t in range(len(y)):
        if t:
            lw += math.log(A[z[t - 1]][z[t]])
        r = (y[t] - mu[z[t]]) / sigma
        lw += -0.5 * math.log(2 * math.pi) - math.log(sigma) - 0.5 * r * r
    return lw


def check_against_oracle(ppl, orc, y, pi0, A, mu, sigma):
    g = run_gpu(ppl, y, pi0, A, mu, sigma)
    o = orc.enumerate_hmm(y, orc.hmm_hyper(pi0, A, mu, sigma))
    K, T = len(pi0), len(y)
    assert g["scal"][3] == 0.0 and g["res"].status == 0
    assert g["scal"][1] == float(K) ** T == o["paths"]
    assert abs(g["scal"][0] - o["log_z"]) < 2e-9, (g["scal"][0], o["log_z"])
    assert g["res"].log_evidence == g["scal"][0]
    assert np.max(np.abs(g["marg"] - o["marginals"])) < 2e-9
    assert np.allclose(g["marg"].sum(1), 1.0, atol=1e-12)
    tol = 1e-12 * max(1.0, abs(o["map_lw"]))
    if not np.array_equal(g["map"], o["map"]):
        assert abs(path_lw(y, pi0, A, mu, sigma, g["map"]) - o["map_lw"]) < tol
    assert abs(g["scal"][2] - o["map_lw"]) < tol
    return g, o


@pytest.mark.parametrize("K,T", [(1, 1), (1, 7), (2, 1), (2, 5), (2, 11), (2, 12), (2, 24), (3, 7), (3, 15),
                                 (4, 6), (4, 12), (5, 9), (6, 8), (7, 8), (8, 3), (8, 8)])
def test_enumerate_matches_oracle(ppl, orc, K, T):
    print(f"enumerate K={K} T={T}", flush=True)
    pi0, A, mu, sigma, y, _ = synthetic.hmm_instance(K, T)
    check_against_oracle(ppl, orc, y, pi0, A, mu, sigma)


def test_enumerate_sparse_transitions(ppl, orc):
    """Zero-probability starts and transitions (a left-to-right chain): paths
    through them weigh nothing and the MAP path avoids them."""
    K, T = 4, 13
    pi0, A, mu, sigma, y, _ = synthetic.hmm_instance(K, T, seed=5)
    pi0 = np.array([0.7, 0.3, 0.0, 0.0])
    A = np.triu(np.asarray(A)) + 0.0
    A /= A.sum(1, keepdims=True)
    g, o = check_against_oracle(ppl, orc, y, pi0, A, mu, sigma)
    assert np.all(np.diff(g["map"]) >= 0)
    assert g["marg"][0, 2] == 0.0 and g["marg"][0, 3] == 0.0


def test_enumerate_narrow_emissions(ppl, orc):
    """sigma = 0.05: emission log-densities far above zero and far below it."""
    pi0, A, mu, _, y, _ = synthetic.hmm_instance(3, 11, seed=8)
    check_against_oracle(ppl, orc, y, pi0, A, mu, 0.05)


def test_enumerate_exact_ties_take_the_lowest_path(ppl):
    """Identical states: every path has the same log joint, bit for bit, so the
    most probable path is index 0 and every marginal is 1/K."""
    K, T = 3, 14
    pi0 = np.full(K, 1.0 / K)
    A = np.full((K, K), 1.0 / K)
    mu = np.zeros(K)
    y = synthetic.hmm_instance(K, T, seed=2)[4]
    g = run_gpu(ppl, y, pi0, A, mu, 1.0)
    assert np.all(g["map"] == 0)
    assert np.allclose(g["marg"], 1.0 / K, atol=1e-12)
    ll = float(np.sum(-0.5 * np.log(2 * np.pi) - 0.5 * y * y))
    assert abs(g["scal"][0] - ll) < 1e-10


def test_enumerate_all_zero_weights(ppl):
    """An initial distribution of zeros: every path weighs zero."""
    import torch
    pi0, A, mu, sigma, y, _ = synthetic.hmm_instance(2, 9)
    g = run_gpu(ppl, y, [0.0, 0.0], A, mu, sigma, sync=False)
    assert g["scal"][3] == ppl.PPL_E_ZERO_WEIGHT and g["scal"][0] == -np.inf
    assert np.all(g["marg"] == 0.0)
    with pytest.raises(ppl.PplError) as e:
        run_gpu(ppl, y, [0.0, 0.0], A, mu, sigma, sync=True)
    assert e.value.code == ppl.PPL_E_ZERO_WEIGHT
    torch.cuda.synchronize()


def test_enumerate_nan_observation(ppl):
    pi0, A, mu, sigma, y, _ = synthetic.hmm_instance(3, 8)
    y = y.copy()
    y[5] = np.nan
    g = run_gpu(ppl, y, pi0, A, mu, sigma, sync=False)
    assert g["scal"][3] == ppl.PPL_E_NONFINITE and np.isnan(g["scal"][0])


def test_enumerate_full_size_against_forward_backward(ppl):
    """4 states over 20 steps (2^40 paths, the measured workload): log Z and
    the marginals agree with the forward-backward recursions, the path with
    Viterbi."""
    from oracle import closed_forms
    K, T = 4, 20
    print(f"enumerate K={K} T={T} (2^40 paths)", flush=True)
    pi0, A, mu, sigma, y, _ = synthetic.hmm_instance(K, T)
    g = run_gpu(ppl, y, pi0, A, mu, sigma)
    lz, marg = closed_forms.hmm_forward_backward(y, pi0, A, mu, sigma)
    vz, vlw = closed_forms.hmm_viterbi(y, pi0, A, mu, sigma)
    assert abs(g["scal"][0] - lz) < 2e-9, (g["scal"][0], lz)
    assert np.max(np.abs(g["marg"] - marg)) < 2e-9
    assert abs(g["scal"][2] - vlw) < 1e-12 * max(1.0, abs(vlw))
    if not np.array_equal(g["map"], vz):
        assert abs(path_lw(y, pi0, A, mu, sigma, g["map"]) - vlw) < 1e-12 * max(1.0, abs(vlw))


def test_enumerate_rejects_bad_models(ppl):
    import torch
    dev = torch.device("cuda:0")
    pi0, A, mu, sigma, y, _ = synthetic.hmm_instance(3, 8)
    dy = torch.from_numpy(y).to(dev)
    bad = [
        ([9] + [1.0] * 9, dict()),                                # K out of range
        (None, dict(sigma=-1.0)),
        (None, dict(pi0=[0.5, -0.1, 0.6])),
    ]
    for hyper, kw in bad:
        if hyper is None:
            data = ppl.hmm_data(dy, kw.get("pi0", pi0), A, mu, kw.get("sigma", sigma))
        else:
            data = ppl.make_data(None, dy, dim=hyper[0], hyper=hyper, dtype=ppl.PPL_F64)
        with pytest.raises(ppl.PplError) as e:
            ppl.ppl_enumerate(ppl.PPL_MODEL_HMM, data, ws=ppl.workspace(1 << 20))
        assert e.value.code == ppl.PPL_E_ARG
    long_y = torch.zeros(40, dtype=torch.float64, device=dev)
    data = ppl.hmm_data(long_y, pi0, A, mu, sigma)                # 3^40 > 2^50 paths
    with pytest.raises(ppl.PplError) as e:
        ppl.ppl_enumerate(ppl.PPL_MODEL_HMM, data, ws=ppl.workspace(1 << 20))
    assert e.value.code == ppl.PPL_E_UNSUPPORTED
    data = ppl.hmm_data(dy, pi0, A, mu, sigma)
    with pytest.raises(ppl.PplError) as e:
        ppl.ppl_enumerate(ppl.PPL_MODEL_HMM, data, ws=ppl.workspace(64))
    assert e.value.code == ppl.PPL_E_WORKSPACE
