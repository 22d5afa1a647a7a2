"""The no-allocation importance-sampling entry point (ppl_importance_noalloc)
against ppl_importance, through the C ABI: the same kernels on the library's
fixed scratch array instead of a caller workspace must give bit-identical
outputs, on two calls in a row (the second smaller, over the first call's
leftover scratch contents), and requests beyond the scratch are refused."""
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


def _outputs(ppl, fn, model, data, n, seed, n_lat, lat_dtype, n_sum, q=None, q_kind=None):
    import torch
    dev = torch.device("cuda:0")
    lw = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    lat = torch.full((n_lat, n), float("nan"), dtype=lat_dtype, device=dev)
    summ = torch.full((n_sum,), float("nan"), dtype=torch.float64, device=dev)
    scal = torch.full((8,), float("nan"), dtype=torch.float64, device=dev)
    r = fn(model, data, n, seed, q=q, q_kind=q_kind, log_weights=lw, latents=lat, summaries=summ, scalars=scal,
           sync=True)
    return dict(log_z=r.log_evidence, ess=r.ess, lw=lw.cpu().numpy(), lat=lat.cpu().numpy(),
                summ=summ.cpu().numpy(), scal=scal.cpu().numpy())


def _same(a, b):
    for k in ("lw", "lat", "summ", "scal"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    assert a["log_z"] == b["log_z"] and a["ess"] == b["ess"]


def test_noalloc_matches_importance_blr_then_smaller(ppl):
    import torch
    dev = torch.device("cuda:0")
    for (D, n, seed) in [(10_000, 1 << 20, 7), (1000, 5003, 8)]:
        X, y, _ = synthetic.blr_data(D=D)
        data = ppl.make_data(torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev), dim=16)
        a = _outputs(ppl, ppl.ppl_importance_noalloc, ppl.PPL_MODEL_BLR, data, n, seed, 16, torch.float32, 16)
        b = _outputs(ppl, ppl.ppl_importance, ppl.PPL_MODEL_BLR, data, n, seed, 16, torch.float32, 16)
        assert np.isfinite(a["log_z"])
        _same(a, b)


def test_noalloc_matches_importance_poly_and_mixture(ppl):
    import torch
    dev = torch.device("cuda:0")
    x, y = synthetic.poly_data()
    data = ppl.make_data(torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev))
    for n in (1 << 18, 10_000):
        a = _outputs(ppl, ppl.ppl_importance_noalloc, ppl.PPL_MODEL_POLY, data, n, 3, 6, torch.float64, 29)
        b = _outputs(ppl, ppl.ppl_importance, ppl.PPL_MODEL_POLY, data, n, 3, 6, torch.float64, 29)
        _same(a, b)
    inst = synthetic.gmm_instances(1, seed=9, d_lo=2.0, d_hi=2.0 + 1e-9, k_lo=5, k_hi=5)[0]
    dy = torch.from_numpy(inst["y"].astype(np.float32)).to(dev)
    data = ppl.make_data(None, dy, dim=5, dtype=ppl.PPL_F32)
    for n in (1 << 17, 777):
        a = _outputs(ppl, ppl.ppl_importance_noalloc, ppl.PPL_MODEL_GMM, data, n, 4, 10, torch.float64, 8)
        b = _outputs(ppl, ppl.ppl_importance, ppl.PPL_MODEL_GMM, data, n, 4, 10, torch.float64, 8)
        _same(a, b)


def test_noalloc_refuses_requests_beyond_its_scratch(ppl):
    import torch
    dev = torch.device("cuda:0")
    X, y, _ = synthetic.blr_data(D=100)
    data = ppl.make_data(torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev), dim=16)
    n_big = (1 << 31) - 1
    need = ppl.ppl_workspace_size(ppl.PPL_MODEL_BLR, data, n_big, ppl.PPL_ALGO_IS)
    assert need > ppl.PPL_NOALLOC_SCRATCH_BYTES
    with pytest.raises(ppl.PplError) as e:
        ppl.ppl_importance_noalloc(ppl.PPL_MODEL_BLR, data, n_big, 1, sync=True)
    assert e.value.code == ppl.PPL_E_UNSUPPORTED
    # the largest BLR request that fits still runs (and agrees with the workspace path)
    lo, hi = 1, n_big
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if ppl.ppl_workspace_size(ppl.PPL_MODEL_BLR, data, mid, ppl.PPL_ALGO_IS) <= ppl.PPL_NOALLOC_SCRATCH_BYTES:
            lo = mid
        else:
            hi = mid - 1
    assert lo >= 1 << 26
    r = ppl.ppl_importance_noalloc(ppl.PPL_MODEL_BLR, data, lo, 2, sync=True)
    s = ppl.ppl_importance(ppl.PPL_MODEL_BLR, data, lo, 2, sync=True)
    assert r.log_evidence == s.log_evidence and r.ess == s.ess
