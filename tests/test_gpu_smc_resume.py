"""SMC stop and resume: a run split into calls over factor ranges, each
stopping into and resuming from a device checkpoint, gives the same bits as
one call over all factors (log Z-hat, final ESS, resampling count, final
log-weights and particles, per-factor traces and recorded ancestors)."""
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


def _data(ppl, name, T, K):
    import torch
    dev = torch.device("cuda:0")
    if name == "lgssm":
        y = synthetic.lgssm_data(T=T)
        model = ppl.PPL_MODEL_LGSSM
    else:
        inst = synthetic.gmm_instances(1, seed=77, d_lo=2.0, d_hi=2.0 + 1e-9, k_lo=K, k_hi=K)[0]
        g = np.random.default_rng(5)
        z = g.choice(K, size=T, p=inst["pi"])
        y = (inst["mu"][z] + g.standard_normal(T)).astype(np.float32)
        model = ppl.PPL_MODEL_GMM
    dy = torch.from_numpy(np.ascontiguousarray(y, np.float32)).to(dev)
    return model, ppl.make_data(None, dy, n_data=T, dim=K, dtype=ppl.PPL_F32), dy


def _run(ppl, model, data, n, T, K, pieces, moves, seed=11, max_events=16):
    import torch
    dev = torch.device("cuda:0")
    nf = 1 if model == ppl.PPL_MODEL_LGSSM else 2 * K
    out = dict(lw=torch.empty(n, dtype=torch.float32, device=dev),
               lat=torch.empty((nf, n), dtype=torch.float32, device=dev),
               scal=torch.empty(8, dtype=torch.float64, device=dev),
               ess=torch.zeros(T, dtype=torch.float64, device=dev),
               res=torch.zeros(T, dtype=torch.uint8, device=dev),
               lzt=torch.zeros(T, dtype=torch.float64, device=dev),
               anc=torch.full((max_events, n), -7, dtype=torch.int32, device=dev))
    ws = ppl.workspace(ppl.ppl_workspace_size(model, data, n, ppl.PPL_ALGO_SMC), dev)
    ck = ppl.workspace(ppl.ppl_smc_checkpoint_bytes(model, data, n), dev)
    partial = []
    bounds = [0] + list(pieces) + [T]
    for t0, t1 in zip(bounds[:-1], bounds[1:]):
        r = ppl.ppl_smc(model, data, n, seed, 0.5, ws=ws, log_weights=out["lw"], latents=out["lat"],
                        scalars=out["scal"], ess_trace=out["ess"], resampled=out["res"], ancestors=out["anc"],
                        logz_trace=out["lzt"], move_steps=moves, sync=True, t_begin=t0, t_end=t1 if t1 < T else 0,
                        checkpoint=ck)
        partial.append((t1, r.log_evidence, r.n_resample))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}, partial


@pytest.mark.parametrize("name,n,T,K,pieces,moves", [
    ("lgssm", 1 << 20, 1000, 0, [500], 0),
    ("lgssm", 5000, 300, 0, [1, 77, 150, 299], 0),
    ("lgssm", (1 << 17) + 3, 200, 0, [64, 65], 0),
    ("gmm", 20_000, 200, 5, [60, 61, 130], 1),
    ("gmm", (1 << 18) + 7, 150, 3, [75], 0),
])
def test_smc_stop_and_resume_is_bitwise(ppl, name, n, T, K, pieces, moves):
    print(f"resume {name} n={n} T={T} pieces={pieces}", flush=True)
    model, data, _ = _data(ppl, name, T, K)
    full, _ = _run(ppl, model, data, n, T, K, [], moves)
    split, partial = _run(ppl, model, data, n, T, K, pieces, moves)
    for key in ("lw", "lat", "scal", "ess", "res", "lzt", "anc"):
        np.testing.assert_array_equal(split[key], full[key], err_msg=key)
    # each stop reports the log Z-hat of the resamplings so far, summed in factor order
    for t1, lz, nres in partial[:-1]:
        acc = 0.0
        for v in full["lzt"][:t1]:
            acc += v
        assert lz == acc
        assert nres == int(full["res"][:t1].sum())


def test_smc_resume_rejects_a_mismatched_checkpoint(ppl):
    import torch
    model, data, _ = _data(ppl, "lgssm", 100, 0)
    n = 4096
    dev = torch.device("cuda:0")
    ws = ppl.workspace(ppl.ppl_workspace_size(model, data, n, ppl.PPL_ALGO_SMC), dev)
    ck = ppl.workspace(ppl.ppl_smc_checkpoint_bytes(model, data, n), dev)
    ppl.ppl_smc(model, data, n, 3, ws=ws, sync=True, t_begin=0, t_end=40, checkpoint=ck)
    with pytest.raises(ppl.PplError) as e:
        ppl.ppl_smc(model, data, n, 3, ws=ws, sync=True, t_begin=30, checkpoint=ck)
    assert e.value.code == ppl.PPL_E_ARG
    # the checkpoint is intact: resuming at the stored factor works
    ppl.ppl_smc(model, data, n, 3, ws=ws, sync=True, t_begin=40, checkpoint=ck)
