"""FP64 oracle of the learned proposal (TEST INFRASTRUCTURE ONLY).

The proposal maps data summary statistics s(y) in R^64 through an MLP
64 -> 256 -> 256 -> 256 (ReLU after the first two layers, linear output) to an
8-component diagonal Gaussian mixture over the model's latents; it is trained
on (latent, data) pairs simulated from the model's own prior by minimising
-log q(latent | s(data)) with Adam, and used as the importance-sampling
proposal (weights log p + log L - log q, the IS of paper Sec. 3.6.2 with a
proposal other than the prior).

Everything here is plain numpy in double precision.  The GPU stores BF16 at
four points -- network inputs, weights, the hidden activations fed to the next
layer, and the back-propagated gradients fed to the next product -- and this
oracle rounds to BF16 (round to nearest even) at exactly those points when
`bf16=True`; with `bf16=False` it is the exact FP64 network, which the tests
pin with central finite differences.

Output head (o = 256 network outputs):
  POLY: o[0:4] degree logits (n = 2..5), o[4:12] mixture logits (shared by all
        degrees); for degree n a block at off(n) (12, 44, 92, 156) of 8n means
        (mean = 10 o) followed by 8n log-scales (5 tanh(o / 5)).
  GMM (K components, d = 2K - 1 ordered unconstrained latents): o[0:8]
        mixture logits, o[8:8+8d] means (5 o), o[8+8d:8+16d] log-scales (5 tanh(o / 5)).
"""
import ctypes
import math

import numpy as np

from . import lib as _lib, _p, _f64

IN, HID, OUT = 64, 256, 256
SHAPES = [(HID, IN), (HID, HID), (OUT, HID)]           # [out][in] per layer
POLY_OFF = {2: 12, 3: 44, 4: 92, 5: 156}
TAG_INIT = 5


def bf16(x):
    """Round to FP32, then to BF16 with round-to-nearest-even; returns float64.
    A NaN stays a NaN (IEEE conversion of a NaN gives a NaN; carrying its low
    bits into the exponent would turn it into an infinity or a zero)."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    with np.errstate(invalid="ignore"):
        r = u.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, r)


def _round(x, on):
    return bf16(x) if on else x


# ------------------------------------------------------------- parameters --
def init_params(seed):
    """Glorot-uniform weights from the Philox stream (block (e div 4, layer, 0, tag 5),
    word e mod 4 for element e of W_l[out][in]): w = (2u - 1) * sqrt(6 / (in + out)),
    rounded to FP32; zero biases."""
    from . import philox
    params = []
    for l, (o, i) in enumerate(SHAPES):
        n = o * i
        nb = (n + 3) // 4
        ctr = np.zeros((nb, 4), dtype=np.uint32)
        ctr[:, 0] = np.arange(nb)
        ctr[:, 1] = l
        ctr[:, 3] = TAG_INIT
        words = philox(ctr, seed).ravel()[:n]
        u = ((words >> 9).astype(np.float64) + 0.5) * 2.0 ** -23
        scale = np.float32(math.sqrt(6.0 / (i + o)))
        w = (np.float32(2.0) * u.astype(np.float32) - np.float32(1.0)) * scale
        params.append(w.astype(np.float32).astype(np.float64).reshape(o, i))
        params.append(np.zeros(o))
    return params


def flatten(params):
    return np.concatenate([p.ravel() for p in params])


def unflatten(v):
    out, k = [], 0
    for (o, i) in SHAPES:
        out.append(v[k:k + o * i].reshape(o, i)); k += o * i
        out.append(v[k:k + o]); k += o
    return out


# ---------------------------------------------------------------- network --
def forward(params, S, bf=True):
    W1, b1, W2, b2, W3, b3 = params
    X = _round(S, bf)
    H1 = _round(np.maximum(X @ _round(W1, bf).T + b1, 0.0), bf)
    H2 = _round(np.maximum(H1 @ _round(W2, bf).T + b2, 0.0), bf)
    O = H2 @ _round(W3, bf).T + b3
    return O, (X, H1, H2)


def backward(params, cache, dO, bf=True):
    W1, b1, W2, b2, W3, b3 = params
    X, H1, H2 = cache
    dO = _round(dO, bf)
    dW3, db3 = dO.T @ H2, dO.sum(0)
    dH2 = _round((dO @ _round(W3, bf)) * (H2 > 0), bf)
    dW2, db2 = dH2.T @ H1, dH2.sum(0)
    dH1 = _round((dH2 @ _round(W2, bf)) * (H1 > 0), bf)
    dW1, db1 = dH1.T @ X, dH1.sum(0)
    return [dW1, db1, dW2, db2, dW3, db3]


def adam(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    out_p, out_m, out_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = b1 * mm + (1 - b1) * g
        vv = b2 * vv + (1 - b2) * g * g
        mh = mm / (1 - b1 ** t)
        vh = vv / (1 - b2 ** t)
        out_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v


# ------------------------------------------------------------------- heads --
def _logsoftmax(z):
    m = z.max(-1, keepdims=True)
    return z - m - np.log(np.exp(z - m).sum(-1, keepdims=True))


def _lsd(o):
    return 5.0 * np.tanh(o / 5.0)


def _dlsd(o):
    return 1.0 - np.tanh(o / 5.0) ** 2


def head_loss_poly(O, theta):
    """Per-sample -log q(n, c | s) and its gradient w.r.t. the 256 outputs."""
    B = O.shape[0]
    loss = np.empty(B)
    dO = np.zeros_like(O)
    for b in range(B):
        o = O[b]
        n = int(theta[b, 0])
        c = theta[b, 1:1 + n]
        lnl, lmix = _logsoftmax(o[0:4]), _logsoftmax(o[4:12])
        off = POLY_OFF[n]
        mo = o[off:off + 8 * n].reshape(8, n)
        so = o[off + 8 * n:off + 16 * n].reshape(8, n)
        mu, lsd = 10.0 * mo, _lsd(so)
        r2 = ((c[None, :] - mu) * np.exp(-lsd)) ** 2
        t = lmix + (-0.5 * r2 - lsd - 0.5 * math.log(2 * math.pi)).sum(1)
        L = t.max() + math.log(np.exp(t - t.max()).sum())
        resp = np.exp(t - L)
        loss[b] = -lnl[n - 2] - L
        g = dO[b]
        g[0:4] = np.exp(lnl)
        g[n - 2] -= 1.0
        g[4:12] = np.exp(lmix) - resp
        gm = -resp[:, None] * (c[None, :] - mu) * np.exp(-2 * lsd) * 10.0
        gs = -resp[:, None] * (r2 - 1.0) * _dlsd(so)
        g[off:off + 8 * n] = gm.ravel()
        g[off + 8 * n:off + 16 * n] = gs.ravel()
    return loss, dO


def head_loss_gmm(O, U):
    """Per-sample -log q(u | s) and its gradient w.r.t. the outputs (u: [B][2K-1])."""
    B, d = U.shape
    lmix = _logsoftmax(O[:, 0:8])
    mo = O[:, 8:8 + 8 * d].reshape(B, 8, d)
    so = O[:, 8 + 8 * d:8 + 16 * d].reshape(B, 8, d)
    mu, lsd = 5.0 * mo, _lsd(so)
    r2 = ((U[:, None, :] - mu) * np.exp(-lsd)) ** 2
    t = lmix + (-0.5 * r2 - lsd - 0.5 * math.log(2 * math.pi)).sum(2)
    tm = t.max(1, keepdims=True)
    L = (tm + np.log(np.exp(t - tm).sum(1, keepdims=True)))[:, 0]
    resp = np.exp(t - L[:, None])
    dO = np.zeros_like(O)
    dO[:, 0:8] = np.exp(lmix) - resp
    dO[:, 8:8 + 8 * d] = (-resp[:, :, None] * (U[:, None, :] - mu) * np.exp(-2 * lsd) * 5.0).reshape(B, -1)
    dO[:, 8 + 8 * d:8 + 16 * d] = (-resp[:, :, None] * (r2 - 1.0) * _dlsd(so)).reshape(B, -1)
    return -L, dO


def decode_poly(o):
    """Proposal parameters for or_propose_poly: lognl[4], logmix[8], mean[4][8][5], lsd[4][8][5]."""
    p = np.zeros(12 + 320)
    p[0:4] = _logsoftmax(o[0:4])
    p[4:12] = _logsoftmax(o[4:12])
    for n in range(2, 6):
        off = POLY_OFF[n]
        mo = o[off:off + 8 * n].reshape(8, n)
        so = o[off + 8 * n:off + 16 * n].reshape(8, n)
        mean = np.zeros((8, 5)); lsd = np.zeros((8, 5))
        mean[:, :n] = 10.0 * mo
        lsd[:, :n] = _lsd(so)
        p[12 + (n - 2) * 40:12 + (n - 1) * 40] = mean.ravel()
        p[172 + (n - 2) * 40:172 + (n - 1) * 40] = lsd.ravel()
    return p


def decode_gmm(o, K):
    d = 2 * K - 1
    return np.concatenate([_logsoftmax(o[0:8]), 5.0 * o[8:8 + 8 * d], _lsd(o[8 + 8 * d:8 + 16 * d])])


# --------------------------------------------------------- C oracle parts --
def _bind():
    L = _lib()
    P, i32, i64, u32, u64, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                  ctypes.c_uint64, ctypes.c_double)
    L.or_summary_poly.argtypes = [P, P, i64, P]
    L.or_summary_gmm.argtypes = [P, i64, P]
    L.or_sim_poly.argtypes = [u64, u32, i64, i64, i64, P, P, P]
    L.or_sim_gmm.argtypes = [u64, u32, i64, i64, i64, i32, P, P, P]
    L.or_poly_logq.argtypes = [P, ctypes.c_int, P]
    L.or_poly_logq.restype = f64
    L.or_gmm_logq.argtypes = [P, i32, P]
    L.or_gmm_logq.restype = f64
    L.or_gmm_unpack.argtypes = [P, i32, f64, P, P]
    L.or_gmm_unpack.restype = f64
    L.or_propose_poly.argtypes = [u64, P, P, P, i64, P, i64, P, P, P]
    L.or_propose_gmm.argtypes = [u64, P, i32, P, i64, P, i64, P, P, P]
    L.or_gmm_prior_lw.argtypes = [u64, i32, P, P, i64, i64, P, P]
    return L


POLY_SIM_HYPER = (10.0, 2.0, 5.0, 1.0)
GMM_HYPER = (5.0, 1.0)


def summary_poly(x, y):
    x, y = _f64(x), _f64(y)
    s = np.empty(64)
    _bind().or_summary_poly(_p(x), _p(y), x.size, _p(s))
    return s


def summary_gmm(y):
    y = _f64(y)
    s = np.empty(64)
    _bind().or_summary_gmm(_p(y), y.size, _p(s))
    return s


def sim_poly(seed, step, i0, B, D=1000, hyper=POLY_SIM_HYPER):
    th, S = np.empty((B, 6)), np.empty((B, 64))
    h = _f64(hyper)
    _bind().or_sim_poly(seed, step, i0, B, D, _p(h), _p(th), _p(S))
    return th, S


def sim_gmm(seed, step, i0, B, D=100, K=5, hyper=GMM_HYPER):
    U, S = np.empty((B, 2 * K - 1)), np.empty((B, 64))
    h = _f64(hyper)
    _bind().or_sim_gmm(seed, step, i0, B, D, K, _p(h), _p(U), _p(S))
    return U, S


def poly_logq(params, n, c):
    params, c = _f64(params), _f64(np.resize(np.asarray(c, float), 5))
    return _bind().or_poly_logq(_p(params), int(n), _p(c))


def gmm_logq(params, K, u):
    params, u = _f64(params), _f64(u)
    return _bind().or_gmm_logq(_p(params), K, _p(u))


def gmm_unpack(u, K, mu_sd=5.0):
    u = _f64(u)
    lpi, mu = np.empty(8), np.empty(8)
    lp = _bind().or_gmm_unpack(_p(u), K, mu_sd, _p(lpi), _p(mu))
    return lp, lpi[:K], mu[:K]


def propose_poly(seed, params, x, y, idx, hyper=(10.0, 2.0, 5.0)):
    params, x, y, h = _f64(params), _f64(x), _f64(y), _f64(hyper)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    lw, draw = np.empty(idx.size), np.empty((idx.size, 6))
    _bind().or_propose_poly(seed, _p(params), _p(x), _p(y), y.size, _p(h), idx.size, _p(idx), _p(lw), _p(draw))
    return lw, draw


def propose_gmm(seed, params, K, y, idx, hyper=GMM_HYPER):
    params, y, h = _f64(params), _f64(y), _f64(hyper)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    lw, draw = np.empty(idx.size), np.empty((idx.size, 2 * K - 1))
    _bind().or_propose_gmm(seed, _p(params), K, _p(y), y.size, _p(h), idx.size, _p(idx), _p(lw), _p(draw))
    return lw, draw


def gmm_prior_lw(seed, K, y, idx, hyper=GMM_HYPER):
    y, h = _f64(y), _f64(hyper)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    lw = np.empty(idx.size)
    _bind().or_gmm_prior_lw(seed, K, _p(h), _p(y), y.size, idx.size, _p(idx), _p(lw))
    return lw
