"""Pins for the FP64 reference of the root-proposal network: finite
differences for every gradient, exact bfloat16 values, and the closed form
of a first Adam step."""
import numpy as np

from oracle import mlp_oracle as M


def test_bf16_round_exact_values():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 3.0e-3, 65504.0, 0.0])
    r = M.bf16_round(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: ties go to the even mantissa (1.0)
    assert r[0] == 1.0 and r[1] == 1.0
    # 1 + 3*2^-8 is a tie between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6
    assert r[2] == 1.0 + 2.0 ** -6
    assert r[3] == -2.5 and r[6] == 0.0
    # bf16 keeps 8 significant bits
    assert abs(r[4] - 3.0e-3) <= 3.0e-3 * 2.0 ** -8
    assert r[5] == 65536.0


def _loss(params, X, roots, nr):
    out, _ = M.forward(params, X)
    L, _ = M.chamfer_loss(out, roots, nr)
    return L


def test_gradients_by_finite_differences():
    rng = np.random.default_rng(1)
    d_in, width, K = 10, 16, 3
    params = M.init_params(d_in, width, 2 * K, rng)
    for k in params:
        if k.startswith("b"):
            params[k] = 0.1 * rng.standard_normal(params[k].shape)
    X = rng.standard_normal((5, d_in))
    roots = rng.uniform(0, 2 * np.pi, (5, 4))
    nr = np.array([1, 2, 3, 4, 2])
    out, cache = M.forward(params, X)
    L, dout = M.chamfer_loss(out, roots, nr)
    grads = M.backward(params, cache, dout)
    h = 1e-6
    for name in params:
        flat = params[name].reshape(-1)
        idx = rng.choice(len(flat), size=min(6, len(flat)), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            Lp = _loss(params, X, roots, nr)
            flat[i] = old - h
            Lm = _loss(params, X, roots, nr)
            flat[i] = old
            fd = (Lp - Lm) / (2 * h)
            g = grads[name].reshape(-1)[i]
            assert abs(fd - g) < 1e-6 * max(1.0, abs(fd)), (name, i, fd, g)


def test_chamfer_loss_closed_form():
    # one root at angle 0, seeds exactly at (1,0) and (0,1): coverage 0,
    # precision (0 + 2)/2 = 1, so L = lam * 1
    out = np.array([[1.0, 0.0, 0.0, 1.0]])
    L, _ = M.chamfer_loss(out, np.array([[0.0]]), np.array([1]), lam=0.5)
    assert abs(L - 0.5) < 1e-15


def test_adam_first_step_closed_form():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    w1, m, v = M.adam_step(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-8)
    # bias-corrected first step is -lr * g / (|g| + eps)
    assert np.allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
