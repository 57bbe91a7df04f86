"""FP64 reference for the root-proposal network of the learned solve.

TEST INFRASTRUCTURE ONLY (same rules as ``ftp_oracle``).

The network is the project's addition to the method (not in the paper):
an MLP  x -> relu(W1 x + b1) -> relu(W2 . + b2) -> relu(W3 . + b3) -> W4 . + b4
whose 4H outputs are H2 = 2H (u, v) pairs; seed k is theta_k = atan2(v_k, u_k).
Weights are stored (out, in) row-major.  ``emulate_bf16`` rounds every GEMM
operand (weights and layer inputs) to bfloat16 the way the GPU kernels do,
while all accumulation stays in FP64.

Loss (a Chamfer distance on the circle between the seed vectors e_k = (u_k,
v_k) and the unit vectors r_j = (cos theta_j, sin theta_j) of the target real
roots):  L = mean_b [ (1/n_b) sum_j min_k |e_k - r_j|^2
                      + lam (1/K) sum_k min_j |e_k - r_j|^2 ].
Adam: m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
      w <- w - lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np

__all__ = ["bf16_round", "init_params", "forward", "backward", "chamfer_loss",
           "adam_step", "LAYER_NAMES"]

LAYER_NAMES = ("1", "2", "3", "4")


def bf16_round(x):
    """Round float values to the nearest bfloat16 (ties to even), returned as
    float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(d_in, width, d_out, rng, n_hidden=3):
    """He-uniform weights, zero biases, FP64."""
    dims = [d_in] + [width] * n_hidden + [d_out]
    params = {}
    for i in range(len(dims) - 1):
        lim = np.sqrt(6.0 / dims[i])
        params["W" + LAYER_NAMES[i]] = rng.uniform(-lim, lim, (dims[i + 1], dims[i]))
        params["b" + LAYER_NAMES[i]] = np.zeros(dims[i + 1])
    return params


def _r(x, emulate):
    return bf16_round(x) if emulate else np.asarray(x, dtype=np.float64)


def forward(params, X, emulate_bf16=False):
    """Returns (out, cache).  X: (B, d_in)."""
    n_layers = sum(1 for k in params if k.startswith("W"))
    h = np.asarray(X, dtype=np.float64)
    cache = {"in": [], "pre": []}
    for i in range(n_layers):
        W = _r(params["W" + LAYER_NAMES[i]], emulate_bf16)
        a = _r(h, emulate_bf16)
        z = a @ W.T + params["b" + LAYER_NAMES[i]]
        cache["in"].append(a)
        cache["pre"].append(z)
        h = np.maximum(z, 0.0) if i < n_layers - 1 else z
    return h, cache


def backward(params, cache, dout, emulate_bf16=False):
    """Gradients of sum(dout * out) w.r.t. every W and b."""
    n_layers = len(cache["in"])
    grads = {}
    g = np.asarray(dout, dtype=np.float64)
    for i in reversed(range(n_layers)):
        if i < n_layers - 1:
            g = g * (cache["pre"][i] > 0)
        gq = _r(g, emulate_bf16)
        grads["W" + LAYER_NAMES[i]] = gq.T @ cache["in"][i]
        grads["b" + LAYER_NAMES[i]] = np.sum(g, axis=0)
        if i > 0:
            W = _r(params["W" + LAYER_NAMES[i]], emulate_bf16)
            g = gq @ W
    return grads


def chamfer_loss(out, roots, nroots, lam=0.5):
    """out: (B, 2K) with (u_k, v_k) interleaved; roots: (B, R) angles, the
    first nroots[b] valid.  Returns (loss, dout)."""
    out = np.asarray(out, dtype=np.float64)
    B, twoK = out.shape
    K = twoK // 2
    e = out.reshape(B, K, 2)
    dout = np.zeros_like(e)
    total = 0.0
    for b in range(B):
        n = int(nroots[b])
        if n == 0:
            continue
        r = np.stack([np.cos(roots[b, :n]), np.sin(roots[b, :n])], axis=1)  # (n,2)
        diff = e[b][:, None, :] - r[None, :, :]  # (K, n, 2)
        d2 = np.sum(diff * diff, axis=2)  # (K, n)
        kmin = np.argmin(d2, axis=0)  # per root
        jmin = np.argmin(d2, axis=1)  # per seed
        total += np.sum(d2[kmin, np.arange(n)]) / n + lam * np.sum(d2[np.arange(K), jmin]) / K
        for j in range(n):
            dout[b, kmin[j]] += 2.0 * diff[kmin[j], j] / n
        for k in range(K):
            dout[b, k] += lam * 2.0 * diff[k, jmin[k]] / K
    return total / B, dout.reshape(B, twoK) / B


def adam_step(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015); returns new (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
