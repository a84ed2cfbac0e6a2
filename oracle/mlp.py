"""CPU oracle for the parameter-proposal network (test infrastructure only).

The network proposes, per iteration of the Schur reduction, the number of
shifts of the next sweep and the size of the next aggressive-early-deflation
window (the two tunables of the method in Section 3.2), each as one of 8 bins.
It is a plain multilayer perceptron

    x (24) -> h1 = relu(W1 (x - mu) / sd + b1) (64) -> h2 = relu(W2 h1 + b2) (64)
           -> z = W3 h2 + b3 (16);  z[0:8] scores the shift bins, z[8:16] the window bins,

trained by reward-weighted cross-entropy: for samples (x_i, a_i, c_i, w_i)

    L = (1/B) sum_i w_i (-log softmax(z_i[0:8])[a_i] - log softmax(z_i[8:16])[c_i]).

Everything here is float64 numpy written from those definitions; only the
tests may import this module.  The parameter vector is laid out as the GPU
library lays it out: mu (24), sd (24), W1 (64x24, row-major), b1 (64),
W2 (64x64), b2 (64), W3 (16x64), b3 (16).  mu and sd are fixed input
normalisation, not trained (their gradient is reported as zero).
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT, NBIN = 24, 64, 16, 8
SHAPES = [("mu", (NIN,)), ("sd", (NIN,)), ("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
          ("W3", (NOUT, NH)), ("b3", (NOUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == NPARAM
    out, off = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = theta[off:off + k].reshape(shape)
        off += k
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(theta, X):
    """Logits z (B x 16) and the intermediate activations."""
    p = unpack(theta)
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    xn = (X - p["mu"]) / p["sd"]
    a1 = xn @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ p["W3"].T + p["b3"]
    return z, {"xn": xn, "a1": a1, "h1": h1, "a2": a2, "h2": h2}


def softmax(z):
    z = np.asarray(z, dtype=np.float64)
    e = np.exp(z - z.max(axis=-1, keepdims=True))
    return e / e.sum(axis=-1, keepdims=True)


def loss(theta, X, a, c, w) -> float:
    z, _ = forward(theta, X)
    B = z.shape[0]
    pa = softmax(z[:, :NBIN])
    pc = softmax(z[:, NBIN:])
    idx = np.arange(B)
    return float(np.sum(np.asarray(w) * (-np.log(pa[idx, a]) - np.log(pc[idx, c]))) / B)


def loss_and_grad(theta, X, a, c, w):
    """Loss and its gradient with respect to theta by the chain rule (backward
    pass written out layer by layer)."""
    p = unpack(theta)
    z, act = forward(theta, X)
    B = z.shape[0]
    a = np.asarray(a)
    c = np.asarray(c)
    w = np.asarray(w, dtype=np.float64)
    idx = np.arange(B)
    pa = softmax(z[:, :NBIN])
    pc = softmax(z[:, NBIN:])
    L = float(np.sum(w * (-np.log(pa[idx, a]) - np.log(pc[idx, c]))) / B)
    # d L / d z: w_i / B (softmax - onehot) on each head
    ga = pa.copy()
    ga[idx, a] -= 1.0
    gc = pc.copy()
    gc[idx, c] -= 1.0
    dz = np.concatenate([ga, gc], axis=1) * (w / B)[:, None]
    g = {"mu": np.zeros(NIN), "sd": np.zeros(NIN)}
    g["W3"] = dz.T @ act["h2"]
    g["b3"] = dz.sum(axis=0)
    dh2 = dz @ p["W3"]
    da2 = dh2 * (act["a2"] > 0.0)
    g["W2"] = da2.T @ act["h1"]
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ p["W2"]
    da1 = dh1 * (act["a1"] > 0.0)
    g["W1"] = da1.T @ act["xn"]
    g["b1"] = da1.sum(axis=0)
    return L, pack(g)


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) of the trainable entries.  mu and sd are
    not parameters of the optimisation: they, and their moment entries, are
    left as they are.  Returns (theta, m, v)."""
    theta = np.array(theta, dtype=np.float64)
    m_in = np.asarray(m, dtype=np.float64)
    v_in = np.asarray(v, dtype=np.float64)
    m = b1 * m_in + (1.0 - b1) * grad
    v = b2 * v_in + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    step = lr * mh / (np.sqrt(vh) + eps)
    fixed = slice(0, 2 * NIN)
    step[fixed] = 0.0
    m[fixed] = m_in[fixed]
    v[fixed] = v_in[fixed]
    return theta - step, m, v


def init(seed: int = 0, mu=None, sd=None) -> np.ndarray:
    """He-style random initialisation with zero biases."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([55, int(seed)])))
    parts = {
        "mu": np.zeros(NIN) if mu is None else np.asarray(mu, dtype=np.float64),
        "sd": np.ones(NIN) if sd is None else np.asarray(sd, dtype=np.float64),
        "W1": g.standard_normal((NH, NIN)) * np.sqrt(2.0 / NIN),
        "b1": np.zeros(NH),
        "W2": g.standard_normal((NH, NH)) * np.sqrt(2.0 / NH),
        "b2": np.zeros(NH),
        "W3": g.standard_normal((NOUT, NH)) * np.sqrt(1.0 / NH),
        "b3": np.zeros(NOUT),
    }
    return pack(parts)


def quantiles(v, probs):
    """Quantiles by linear interpolation between order statistics (position
    p (k - 1) in the sorted sample of k values)."""
    s = np.sort(np.asarray(v, dtype=np.float64))
    k = s.size
    out = []
    for p in probs:
        pos = p * (k - 1)
        lo = int(np.floor(pos))
        hi = min(lo + 1, k - 1)
        out.append(s[lo] + (pos - lo) * (s[hi] - s[lo]))
    return np.array(out)


def features(H, ktop: int, kbot: int, hnorm: float, extra):
    """The 24 features of the active block [ktop, kbot] of H (definition given
    with the library's proposal interface): log m; 19 quantiles of
    log(|h(k,k-1)| / (hnorm / sqrt n)) over the subdiagonal sample
    k = ktop + 1 + floor(i (m-1) / S), i < S = min(m-1, 1024); then extra[0..3]."""
    H = np.asarray(H, dtype=np.float64)
    n = H.shape[0]
    m = kbot - ktop + 1
    cnt = m - 1
    S = min(cnt, 1024)
    scale = hnorm / np.sqrt(n) if hnorm > 0 else 1.0
    f = np.zeros(NIN)
    f[0] = np.log(m)
    if S > 0:
        ks = [ktop + 1 + (i * cnt) // S for i in range(S)]
        vals = np.array([np.log(max(abs(H[k, k - 1]), 1e-300) / scale) for k in ks])
        f[1:20] = quantiles(vals, 0.05 * np.arange(1, 20))
    f[20:24] = np.asarray(extra, dtype=np.float64)
    return f
