"""GPU parity of the learned proposal against the CPU oracle, through the C ABI.

What is compared (same seeds, the oracle computing everything itself):
  - weight initialisation: FP32 master weights and both BF16 layouts bit-exact;
  - simulated training pairs: degrees bit-exact, latents 1e-12 mixed, the 64
    FP64 summaries 1e-8 mixed (summation order; the least-squares fits
    amplify it by the conditioning of the moment matrix);
  - network outputs and every gradient tensor at the initial weights, with the
    oracle's BF16 emulation: relative 2-norm error <= 1e-3 per tensor;
  - one Adam step: moments within the gradient tolerance, updates within
    1e-3 lr where the gradient is well away from zero;
  - polynomial mixture-proposal importance sampling (FP64): discrete draws
    bit-exact, latents 1e-12, log-weights 1e-10 mixed, log Z-hat 1e-9;
  - mixture-model importance sampling (FP64 draws and densities, FP32
    likelihood): latents 1e-12, log-weights and log Z-hat 1e-5 mixed (the FP32
    class; the FP32 per-datum error is about 1e-6 and the 16-datum FP32 block
    sums add a few 1e-6, far inside it);
  - amortised inference: the data summaries 1e-10, the decoded proposal 1e-4.
Training itself is checked by a falling loss, bit-identical results with and
without graph replay, and the gain over the prior proposal on the 1000-point
polynomial workload (the exact evidence is the closed form) and the 5-component
mixture (reference: prior importance sampling at 2^30 particles in FP64).
"""
import math

import numpy as np
import pytest

import synthetic
from oracle import closed_forms as cf

pytestmark = pytest.mark.gpu

SEED = 20240611
COUNT = 148224
BF_COUNT = 147456
BF_OFF = (0, 64 * 256, 64 * 256 + 256 * 256)
SHAPES = ((256, 64), (256, 256), (256, 256))
STEP_OFF = 2368512


@pytest.fixture(scope="module")
def ppl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_08454_amd as p
    return p


@pytest.fixture(scope="module")
def pr(orc):
    from oracle import proposal
    return proposal


def torch_():
    import torch
    return torch


def mixed_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b)))) if a.size else 0.0


def rel_norm(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def split_weights(wts):
    raw = wts.cpu().numpy()
    f = raw[:3 * COUNT * 4].view(np.float32)
    bf = raw[3 * COUNT * 4:3 * COUNT * 4 + 2 * BF_COUNT * 2].view(np.uint16)
    return {"master": f[:COUNT], "m": f[COUNT:2 * COUNT], "v": f[2 * COUNT:], "wt": bf[:BF_COUNT],
            "w": bf[BF_COUNT:], "step": int(raw[STEP_OFF:STEP_OFF + 8].view(np.int64)[0])}


def bf16_bits(x):
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint16)


def lse(v):
    v = np.asarray(v, dtype=np.float64)
    m = v.max()
    return m + math.log(np.exp(v - m).sum())


MODELS = {"poly": dict(D=1000, K=0), "gmm": dict(D=100, K=5)}


def model_id(ppl, name):
    return ppl.PPL_MODEL_POLY if name == "poly" else ppl.PPL_MODEL_GMM


def oracle_sim(pr, name, step, B):
    spec = MODELS[name]
    if name == "poly":
        return pr.sim_poly(SEED, step, 0, B, D=spec["D"])
    return pr.sim_gmm(SEED, step, 0, B, D=spec["D"], K=spec["K"])


# --------------------------------------------------------------- weights --
def test_init_weights_match_oracle(ppl, pr):
    torch = torch_()
    wts = ppl.ppl_proposal_init(SEED)
    torch.cuda.synchronize()
    got = split_weights(wts)
    params = pr.init_params(SEED)
    np.testing.assert_array_equal(got["master"], pr.flatten(params).astype(np.float32))
    assert not got["m"].any() and not got["v"].any() and got["step"] == 0
    for l, (o, i) in enumerate(SHAPES):
        bits = bf16_bits(params[2 * l])
        np.testing.assert_array_equal(got["wt"][BF_OFF[l]:BF_OFF[l] + o * i].reshape(o, i), bits)
        np.testing.assert_array_equal(got["w"][BF_OFF[l]:BF_OFF[l] + o * i].reshape(i, o), bits.T)


# ------------------------------------------------------------ simulation --
@pytest.mark.parametrize("name", ["poly", "gmm"])
def test_simulated_pairs_match_oracle(ppl, pr, name):
    torch = torch_()
    B, step = 128, 3
    spec = MODELS[name]
    cfg = ppl.train_config(B, B, spec["D"], dim=spec["K"])
    wts = ppl.ppl_proposal_init(SEED)
    S = torch.empty((B, 64), dtype=torch.float64, device="cuda")
    lat = torch.empty((B, 16), dtype=torch.float64, device="cuda")
    ppl.ppl_proposal_gradient(model_id(ppl, name), cfg, SEED, step, wts, summaries=S, latents=lat)
    torch.cuda.synchronize()
    th, So = oracle_sim(pr, name, step, B)
    S, lat = S.cpu().numpy(), lat.cpu().numpy()
    if name == "poly":
        np.testing.assert_array_equal(lat[:, 0], th[:, 0])
        assert mixed_err(lat[:, 1:6], th[:, 1:6]) <= 1e-12
        assert set(np.unique(th[:, 0])) == {2.0, 3.0, 4.0, 5.0}
    else:
        assert mixed_err(lat[:, :th.shape[1]], th) <= 1e-12
    assert mixed_err(S, So) <= 1e-8, mixed_err(S, So)


# --------------------------------------------------- forward and backward --
def oracle_grads(pr, name, params, S, th):
    O, cache = pr.forward(params, S, bf=True)
    loss, dO = (pr.head_loss_poly if name == "poly" else pr.head_loss_gmm)(O, th)
    grads = pr.backward(params, cache, dO / len(S), bf=True)
    return O, loss.mean(), grads


@pytest.mark.parametrize("name", ["poly", "gmm"])
def test_forward_and_gradient_match_oracle(ppl, pr, name):
    torch = torch_()
    B, step = 256, 5
    spec = MODELS[name]
    cfg = ppl.train_config(B, B, spec["D"], dim=spec["K"])
    wts = ppl.ppl_proposal_init(SEED)
    grad = torch.empty(COUNT, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    out = torch.empty((256, B), dtype=torch.float32, device="cuda")
    ppl.ppl_proposal_gradient(model_id(ppl, name), cfg, SEED, step, wts, grad=grad, loss=loss, outputs=out)
    torch.cuda.synchronize()
    th, So = oracle_sim(pr, name, step, B)
    params = pr.init_params(SEED)
    Oo, lo, grads = oracle_grads(pr, name, params, So, th)
    assert rel_norm(out.cpu().numpy().T, Oo) <= 1e-3
    assert abs(loss.item() - lo) <= 1e-3 * max(1.0, abs(lo))
    g = grad.cpu().numpy()
    k = 0
    for t, ref in enumerate(grads):
        part = g[k:k + ref.size].reshape(ref.shape)
        k += ref.size
        assert rel_norm(part, ref) <= 1e-3, (t, rel_norm(part, ref))


@pytest.mark.parametrize("name,B", [("poly", 512), ("gmm", 256), ("poly", 64)])
def test_fused_pass_equals_separate_launches(ppl, name, B, monkeypatch):
    """The fused forward/head/input-gradient pass stores the same bits as one
    launch per product: outputs, loss and every gradient entry are equal."""
    torch = torch_()
    spec = MODELS[name]
    cfg = ppl.train_config(B, B, spec["D"], dim=spec["K"])
    wts = ppl.ppl_proposal_init(SEED)
    res = []
    for unfused in ("0", "1"):
        monkeypatch.setenv("PPL_TRAIN_UNFUSED", unfused)
        grad = torch.empty(COUNT, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float64, device="cuda")
        out = torch.empty((256, B), dtype=torch.float32, device="cuda")
        ppl.ppl_proposal_gradient(model_id(ppl, name), cfg, SEED, 3, wts, grad=grad, loss=loss, outputs=out)
        torch.cuda.synchronize()
        res.append((grad.cpu().numpy(), loss.cpu().numpy(), out.cpu().numpy()))
    for a, b in zip(res[0], res[1]):
        np.testing.assert_array_equal(a, b)


def test_adam_step_matches_oracle(ppl, pr):
    torch = torch_()
    B = 256
    cfg = ppl.train_config(B, B, 1000)
    wts = ppl.ppl_proposal_init(SEED)
    trace = torch.empty(1, dtype=torch.float64, device="cuda")
    ppl.ppl_proposal_train(ppl.PPL_MODEL_POLY, cfg, SEED, wts, loss_trace=trace)
    torch.cuda.synchronize()
    got = split_weights(wts)
    assert got["step"] == 1
    th, So = oracle_sim(pr, "poly", 0, B)
    params = pr.init_params(SEED)
    _, lo, grads = oracle_grads(pr, "poly", params, So, th)
    assert abs(trace.item() - lo) <= 1e-3 * max(1.0, abs(lo))
    g = pr.flatten(grads)
    p0 = pr.flatten(params)
    new, m, v = pr.adam(params, grads, [np.zeros_like(p) for p in params], [np.zeros_like(p) for p in params], 1)
    k = 0
    for ref in grads:
        sl = slice(k, k + ref.size)
        k += ref.size
        assert rel_norm(got["m"][sl], 0.1 * ref) <= 1e-3
        assert rel_norm(got["v"][sl], 1e-3 * ref * ref) <= 2e-3
    lr = 1e-3
    d_gpu = got["master"].astype(np.float64) - p0
    d_or = pr.flatten(new) - p0
    assert np.max(np.abs(d_gpu)) <= 1.01 * lr
    firm = np.abs(g) > 1e-4 * np.abs(g).max()
    assert np.mean(np.abs(d_gpu - d_or)[firm] <= 1e-3 * lr) >= 0.999
    # the BF16 copies follow the FP32 master weights
    master = got["master"]
    o = 0
    for l, (on, inn) in enumerate(SHAPES):
        W = master[o:o + on * inn].reshape(on, inn)
        np.testing.assert_array_equal(got["wt"][BF_OFF[l]:BF_OFF[l] + on * inn].reshape(on, inn), bf16_bits(W))
        o += on * inn + on


@pytest.mark.parametrize("name", ["poly", "gmm"])
def test_training_loss_falls_and_graph_replay_is_identical(ppl, name):
    torch = torch_()
    B, steps = 1024, 40
    spec = MODELS[name]
    mid = model_id(ppl, name)
    traces, blocks = [], []
    for graph in (False, True):
        cfg = ppl.train_config(B * steps, B, spec["D"], dim=spec["K"], use_graph=graph)
        wts = ppl.ppl_proposal_init(SEED)
        tr = torch.empty(steps, dtype=torch.float64, device="cuda")
        ppl.ppl_proposal_train(mid, cfg, SEED, wts, loss_trace=tr)
        torch.cuda.synchronize()
        # a second call continues from the stored step count
        tr2 = torch.empty(steps, dtype=torch.float64, device="cuda")
        ppl.ppl_proposal_train(mid, cfg, SEED, wts, loss_trace=tr2)
        torch.cuda.synchronize()
        traces.append(np.concatenate([tr.cpu().numpy(), tr2.cpu().numpy()]))
        blocks.append(wts.cpu().numpy())
    np.testing.assert_array_equal(traces[0], traces[1])
    a, b = (split_weights(torch.from_numpy(blk)) for blk in blocks)
    for key in ("master", "m", "v", "wt", "w"):
        np.testing.assert_array_equal(a[key], b[key])
    assert a["step"] == b["step"] == 2 * steps
    t = traces[0]
    assert np.all(np.isfinite(t))
    assert t[-10:].mean() < t[:10].mean() - 0.5, (t[:10].mean(), t[-10:].mean())


# --------------------------------------------- proposal importance sampling --
def poly_q_random(pr, seed):
    g = np.random.default_rng(seed)
    return pr.decode_poly(0.3 * g.standard_normal(256))


@pytest.mark.parametrize("N", [4096 + 77, 1000])
def test_poly_mixture_is_matches_oracle(ppl, pr, N):
    torch = torch_()
    x, y = synthetic.poly_data(D=1000, seed=synthetic.SEED_POLY_LEARN)
    q = poly_q_random(pr, 7)
    seed = 99
    data = ppl.make_data(torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda"))
    qd = torch.tensor(q, device="cuda")
    lw = torch.empty(N, dtype=torch.float64, device="cuda")
    lat = torch.empty((6, N), dtype=torch.float64, device="cuda")
    sc = torch.empty(8, dtype=torch.float64, device="cuda")
    summ = torch.empty(29, dtype=torch.float64, device="cuda")
    ppl.ppl_importance(ppl.PPL_MODEL_POLY, data, N, seed, q=qd, q_kind=ppl.PPL_Q_POLY_MIX, log_weights=lw,
                       latents=lat, scalars=sc, summaries=summ)
    torch.cuda.synchronize()
    lwo, drawo = pr.propose_poly(seed, q, x, y, np.arange(N))
    lat = lat.cpu().numpy()
    np.testing.assert_array_equal(lat[0], drawo[:, 0])
    assert mixed_err(lat[1:].T, drawo[:, 1:]) <= 1e-12
    assert mixed_err(lw.cpu().numpy(), lwo) <= 1e-10
    logz = lse(lwo) - math.log(N)
    assert abs(sc[0].item() - logz) <= 1e-9 * max(1.0, abs(logz))
    w = np.exp(lwo - lwo.max())
    pn = np.array([w[drawo[:, 0] == n].sum() for n in range(2, 6)]) / w.sum()
    assert mixed_err(summ.cpu().numpy()[:4], pn) <= 1e-9


@pytest.mark.parametrize("K", [2, 5, 8])
@pytest.mark.parametrize("prop", [False, True])
def test_gmm_is_matches_oracle(ppl, pr, K, prop):
    torch = torch_()
    inst = synthetic.gmm_instances(1, seed=11 + K, d_lo=2.0, d_hi=2.0 + 1e-9, k_lo=K, k_hi=K)[0]
    y = inst["y"].astype(np.float32)
    N, seed = 3000, 5
    data = ppl.make_data(None, torch.tensor(y, device="cuda"), dim=K)
    lw = torch.empty(N, dtype=torch.float64, device="cuda")
    lat = torch.empty((2 * K, N), dtype=torch.float64, device="cuda")
    sc = torch.empty(8, dtype=torch.float64, device="cuda")
    if prop:
        g = np.random.default_rng(K)
        q = pr.decode_gmm(0.3 * g.standard_normal(256), K)
        ppl.ppl_importance(ppl.PPL_MODEL_GMM, data, N, seed, q=torch.tensor(q, device="cuda"),
                           q_kind=ppl.PPL_Q_GMM_MIX, log_weights=lw, latents=lat, scalars=sc)
        torch.cuda.synchronize()
        lwo, U = pr.propose_gmm(seed, q, K, y.astype(np.float64), np.arange(N))
        lat = lat.cpu().numpy()
        for r in range(0, N, 37):
            _, lpi, mu = pr.gmm_unpack(U[r], K)
            assert mixed_err(lat[:K, r], lpi) <= 1e-12 and mixed_err(lat[K:, r], mu) <= 1e-12
    else:
        ppl.ppl_importance(ppl.PPL_MODEL_GMM, data, N, seed, log_weights=lw, latents=lat, scalars=sc)
        torch.cuda.synchronize()
        lwo = pr.gmm_prior_lw(seed, K, y.astype(np.float64), np.arange(N))
        from oracle import gmm_init
        state = gmm_init(seed, 0, K, N)
        assert mixed_err(lat.cpu().numpy(), state) <= 1e-12
    assert mixed_err(lw.cpu().numpy(), lwo) <= 1e-5
    logz = lse(lwo) - math.log(N)
    assert abs(sc[0].item() - logz) <= 1e-5 * max(1.0, abs(logz))


# ---------------------------------------------------------- amortised run --
@pytest.mark.parametrize("name", ["poly", "gmm"])
def test_infer_matches_oracle_network(ppl, pr, name):
    torch = torch_()
    wts = ppl.ppl_proposal_init(SEED)
    params = pr.init_params(SEED)
    if name == "poly":
        x, y = synthetic.poly_data(D=1000, seed=synthetic.SEED_POLY_LEARN)
        data = ppl.make_data(torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda"))
        s_or = pr.summary_poly(x, y)
        nq, mid, kind = 332, ppl.PPL_MODEL_POLY, ppl.PPL_Q_POLY_MIX
    else:
        y = synthetic.gmm_instances(1, seed=21, d_lo=2.0, d_hi=2.0 + 1e-9, k_lo=5, k_hi=5)[0]["y"].astype(np.float32)
        data = ppl.make_data(None, torch.tensor(y, device="cuda"), dim=5)
        s_or = pr.summary_gmm(y.astype(np.float64))
        nq, mid, kind = 8 + 16 * 9, ppl.PPL_MODEL_GMM, ppl.PPL_Q_GMM_MIX
    N = 2048
    q = torch.empty(nq, dtype=torch.float64, device="cuda")
    s = torch.empty(64, dtype=torch.float64, device="cuda")
    lw = torch.empty(N, dtype=torch.float64, device="cuda")
    sc = torch.empty(8, dtype=torch.float64, device="cuda")
    ppl.ppl_proposal_infer(mid, data, wts, N, 3, q_params=q, data_summaries=s, log_weights=lw, scalars=sc)
    torch.cuda.synchronize()
    assert mixed_err(s.cpu().numpy(), s_or) <= 1e-10
    O = pr.forward(params, s_or[None, :], bf=True)[0][0]
    q_or = pr.decode_poly(O) if name == "poly" else pr.decode_gmm(O, 5)
    assert mixed_err(q.cpu().numpy(), q_or) <= 1e-4
    # widening raises every used log-scale by log(widen)
    qw = torch.empty(nq, dtype=torch.float64, device="cuda")
    ppl.ppl_proposal_infer(mid, data, wts, 64, 3, q_params=qw, widen=1.5)
    torch.cuda.synchronize()
    used = np.zeros(nq, dtype=bool)
    if name == "poly":
        lsd_used = np.zeros((4, 8, 5), dtype=bool)
        for n in range(2, 6):
            lsd_used[n - 2, :, :n] = True
        used[172:] = lsd_used.ravel()
    else:
        used[8 + 72:] = True
    dq = qw.cpu().numpy() - q.cpu().numpy()
    assert np.allclose(dq[used], math.log(1.5), atol=1e-12) and np.all(dq[~used] == 0)
    # the sampling stage is ppl_importance with the decoded proposal
    lw2 = torch.empty(N, dtype=torch.float64, device="cuda")
    ppl.ppl_importance(mid, data, N, 3, q=q, q_kind=kind, log_weights=lw2)
    torch.cuda.synchronize()
    assert torch.equal(lw, lw2)


# ------------------------------------------------------ gain over the prior --
RMSE_TARGET = 0.05
TRAIN = {"poly": dict(batch=512, lr=1e-3, decay=False), "gmm": dict(batch=256, lr=3e-3, decay=True)}


def train_learned(ppl, name, D, K):
    torch = torch_()
    t = TRAIN[name]
    steps = (1 << 22) // t["batch"]
    cfg = ppl.train_config(1 << 22, t["batch"], D, dim=K, lr=t["lr"], use_graph=True,
                           lr_decay_steps=steps if t["decay"] else 0, lr_final_frac=0.02)
    wts = ppl.ppl_proposal_init(SEED)
    trace = torch.empty(steps, dtype=torch.float64, device="cuda")
    ppl.ppl_proposal_train(model_id(ppl, name), cfg, SEED, wts, loss_trace=trace)
    torch.cuda.synchronize()
    tr = trace.cpu().numpy()
    assert np.all(np.isfinite(tr)) and tr[-32:].mean() < tr[:32].mean()
    return wts


def rmse_ladder(run, ref, lg_lo, lg_hi, seeds=8):
    """Smallest power-of-two N whose log Z-hat RMSE over `seeds` runs is within
    RMSE_TARGET of ref; returns (N, rmse, mean ESS, mean GPU ms per call) or the
    last rung with its RMSE."""
    torch = torch_()
    sc = torch.empty(8, dtype=torch.float64, device="cuda")
    for lg in range(lg_lo, lg_hi + 1):
        est, ess, ms = [], [], []
        for s in range(seeds):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            run(1 << lg, 100 + s, sc)
            e1.record()
            torch.cuda.synchronize()
            v = sc.cpu().numpy()
            est.append(v[0])
            ess.append(v[1])
            ms.append(e0.elapsed_time(e1))
        rmse = math.sqrt(float(np.mean((np.array(est) - ref) ** 2)))
        if rmse <= RMSE_TARGET or lg == lg_hi:
            return 1 << lg, rmse, float(np.mean(ess)), float(np.mean(ms))


def gain_check(ppl, name, data, ref, wts, lg_learned, lg_prior):
    mid = model_id(ppl, name)
    widen, pilot = ppl.ppl_proposal_pick_widen(mid, data, wts)
    ws_l = ppl.workspace(ppl.ppl_proposal_infer_workspace_size(mid, data, 1 << lg_learned[1]))
    ws_p = ppl.workspace(ppl.ppl_workspace_size(mid, data, 1 << lg_prior[1], ppl.PPL_ALGO_IS))
    learned = rmse_ladder(lambda n, s, sc: ppl.ppl_proposal_infer(mid, data, wts, n, s, ws=ws_l, scalars=sc,
                                                                  widen=widen), ref, *lg_learned)
    prior = rmse_ladder(lambda n, s, sc: ppl.ppl_importance(mid, data, n, s, ws=ws_p, scalars=sc), ref, *lg_prior)
    rate_l = learned[2] / (learned[3] / 1e3)
    rate_p = prior[2] / (prior[3] / 1e3)
    print(f"[{name}] widen {widen} (pilot ESS {[round(e, 1) for e in pilot]}); learned: N {learned[0]} rmse "
          f"{learned[1]:.4f} ESS {learned[2]:.1f} {learned[3]:.3f} ms -> {rate_l:.3g} ESS/s; prior: N {prior[0]} "
          f"rmse {prior[1]:.4f} ESS {prior[2]:.1f} {prior[3]:.3f} ms -> {rate_p:.3g} ESS/s")
    assert learned[1] <= RMSE_TARGET
    assert prior[1] > RMSE_TARGET or rate_l > rate_p
    return learned, prior


def test_learned_proposal_beats_prior_poly(ppl):
    """Trained on 2^22 pairs simulated from the prior, the learned proposal
    reaches a log-evidence RMSE of 0.05 (exact evidence: the closed form) at a
    far smaller particle count, and a higher ESS/s, than the prior proposal."""
    torch = torch_()
    x, y = synthetic.poly_data(D=1000, seed=synthetic.SEED_POLY_LEARN)
    exact = cf.poly_exact(x, y)["log_z"]
    data = ppl.make_data(torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda"))
    wts = train_learned(ppl, "poly", 1000, 0)
    learned, prior = gain_check(ppl, "poly", data, exact, wts, (10, 20), (18, 28))
    assert learned[0] * 64 <= prior[0]


def test_learned_proposal_beats_prior_gmm(ppl):
    """K = 5 mixture, D = 100: the reference is prior importance sampling at 2^34
    particles in FP64 (16 runs of 2^30 merged by log-sum-exp)."""
    torch = torch_()
    K = 5
    y = synthetic.gmm_learn_data(K=K, D=100)
    data = ppl.make_data(None, torch.tensor(y, device="cuda"), dim=K)
    chunk, nch = 1 << 30, 16
    sc = torch.empty(8, dtype=torch.float64, device="cuda")
    parts = []
    ws = ppl.workspace(ppl.ppl_workspace_size(ppl.PPL_MODEL_GMM, data, chunk, ppl.PPL_ALGO_IS))
    for c in range(nch):
        ppl.ppl_importance(ppl.PPL_MODEL_GMM, data, chunk, 1000 + c, ws=ws, scalars=sc)
        torch.cuda.synchronize()
        parts.append(sc.cpu().numpy()[4:7].copy())
    del ws
    m = max(p[0] for p in parts)
    s1 = sum(p[1] * math.exp(p[0] - m) for p in parts)
    s2 = sum(p[2] * math.exp(2 * (p[0] - m)) for p in parts)
    ref = m + math.log(s1) - math.log(chunk * nch)
    ref_ess = s1 * s1 / s2
    print(f"[gmm] reference logZ {ref:.4f} ESS {ref_ess:.0f} of 2^34")
    assert ref_ess > 2000
    wts = train_learned(ppl, "gmm", 100, K)
    learned, prior = gain_check(ppl, "gmm", data, ref, wts, (12, 22), (22, 30))
    assert learned[0] * 64 <= prior[0]


def frag_order(mat):
    """A [N][KD] BF16 matrix (N <= 256 rows, KD a multiple of 32) in the fused
    training pass's fragment order, written out from the index definition:
    wave n // 64, k-step k // 32, row tile (n % 64) // 16, lane
    16 ((k % 32) // 8) + n % 16, element k % 8."""
    N, KD = mat.shape
    out = np.zeros(N * KD, dtype=mat.dtype)
    n = np.arange(N)[:, None]
    k = np.arange(KD)[None, :]
    lane = ((k % 32) // 8) * 16 + n % 16
    idx = ((((n // 64) * (KD // 32) + k // 32) * 4 + (n % 64) // 16) * 64 + lane) * 8 + k % 8
    out[idx.ravel()] = mat.ravel()
    return out


def test_fragment_order_copies_follow_adam(ppl):
    """The parameter block's fragment-order BF16 copies hold exactly the
    [out][in] and [in][out] weights, after initialisation and after Adam
    steps; the fused pass (which reads them) then still equals the per-product
    launches (which read the plain layouts)."""
    import os
    torch = torch_()
    frag_off = STEP_OFF + 256
    wts = ppl.ppl_proposal_init(SEED)
    assert ppl.ppl_proposal_weights_bytes() == frag_off + 2 * BF_COUNT * 2
    cfg = ppl.train_config(3 * 256, 256, 1000)
    for trained in (False, True):
        if trained:
            ppl.ppl_proposal_train(ppl.PPL_MODEL_POLY, cfg, SEED, wts)
            torch.cuda.synchronize()
        raw = wts.cpu().numpy()
        parts = split_weights(wts)
        frag = raw[frag_off:frag_off + 2 * BF_COUNT * 2].view(np.uint16)
        for l, (on, inn) in enumerate(SHAPES):
            o = BF_OFF[l]
            wt = parts["wt"][o:o + on * inn].reshape(on, inn)        # [out][in]
            w = parts["w"][o:o + on * inn].reshape(inn, on)          # [in][out]
            np.testing.assert_array_equal(frag[o:o + on * inn], frag_order(wt))
            np.testing.assert_array_equal(frag[BF_COUNT + o:BF_COUNT + o + on * inn], frag_order(w))
    # fused and per-product passes agree at the trained weights
    B = 256
    gcfg = ppl.train_config(B, B, 1000)
    res = []
    for unfused in ("0", "1"):
        os.environ["PPL_TRAIN_UNFUSED"] = unfused
        try:
            grad = torch.empty(COUNT, dtype=torch.float32, device="cuda")
            ppl.ppl_proposal_gradient(ppl.PPL_MODEL_POLY, gcfg, SEED, 5, wts, grad=grad)
            torch.cuda.synchronize()
            res.append(grad.cpu().numpy())
        finally:
            del os.environ["PPL_TRAIN_UNFUSED"]
    np.testing.assert_array_equal(res[0], res[1])
