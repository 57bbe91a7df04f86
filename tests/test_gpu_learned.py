"""GPU checks of the learned root proposal.

* The network's forward pass and gradients (bf16 MFMA, FP32 accumulation)
  against the FP64 reference with the same bf16 rounding points.
* Training lowers the loss.
* The learned, uniform-seed and Aberth solvers give the same periodogram as
  the companion solve (every accepted frequency has all real roots, verified
  by the Sturm count; the others go to the Aberth tier, and what it leaves to
  the companion solve).
* Forcing the fallback reproduces the companion solve bit for bit.
"""
import numpy as np
import pytest

from oracle import mlp_oracle as MO
from oracle import ftp_oracle as O
from synthetic import (single_long_case, tiny_case, learned_heldout_lightcurves, large_heldout_lightcurves,
                       large_case)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ftp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2101_12348_amd as F
    F.load_library()
    return F


def _params_from_flat(w, din, width, dout):
    dims = [din, width, width, width, dout]
    p, o = {}, 0
    for l in range(4):
        n_in, n_out = dims[l], dims[l + 1]
        p["W" + MO.LAYER_NAMES[l]] = w[o: o + n_in * n_out].reshape(n_out, n_in).astype(np.float64)
        o += n_in * n_out
        p["b" + MO.LAYER_NAMES[l]] = w[o: o + n_out].astype(np.float64)
        o += n_out
    return p


def _flat(grads):
    return np.concatenate([np.r_[grads["W" + k].ravel(), grads["b" + k].ravel()] for k in MO.LAYER_NAMES])


@pytest.mark.parametrize("B,din,width,dout", [(37, 22, 32, 8), (300, 70, 256, 24)])
def test_mlp_forward_and_gradients_match_reference(ftp, B, din, width, dout):
    import torch
    rng = np.random.default_rng(B)
    w = np.concatenate([np.r_[rng.uniform(-1, 1, (n_out, n_in)).ravel() * np.sqrt(3.0 / n_in),
                              0.1 * rng.standard_normal(n_out)]
                        for n_in, n_out in [(din, width), (width, width), (width, width), (width, dout)]])
    w = w.astype(np.float32)
    net = ftp.Mlp(din, width, dout, weights=w)
    X = rng.standard_normal((B, din)).astype(np.float32)
    Xb = torch.as_tensor(X, device="cuda").to(torch.bfloat16)
    R = 6
    roots = rng.uniform(0, 2 * np.pi, (B, R)).astype(np.float32)
    nroots = rng.integers(0, R + 1, B).astype(np.int32)
    out = net.forward(Xb).cpu().numpy()
    params = _params_from_flat(w.astype(np.float64), din, width, dout)
    Xr = Xb.float().cpu().numpy().astype(np.float64)
    ref, cache = MO.forward(params, Xr, emulate_bf16=True)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(out - ref)) <= 1e-2 * scale
    loss, grads = net.loss_grad(Xb, torch.as_tensor(roots, device="cuda"),
                                torch.as_tensor(nroots, device="cuda"), lam=0.5)
    torch.cuda.synchronize()
    # reference gradients at the GPU's own output (same rounding points)
    L_ref, dout_ref = MO.chamfer_loss(out.astype(np.float64), roots.astype(np.float64), nroots, lam=0.5)
    g_ref = _flat(MO.backward(params, cache, dout_ref, emulate_bf16=True))
    g = grads.cpu().numpy().astype(np.float64)
    # the per-sample losses average to the batch loss
    assert abs(float(loss.mean().cpu()) - L_ref) <= 1e-4 * max(1.0, abs(L_ref))
    o = 0
    dims = [din, width, width, width, dout]
    for l in range(4):
        for n in (dims[l] * dims[l + 1], dims[l + 1]):
            seg_g, seg_r = g[o: o + n], g_ref[o: o + n]
            assert np.max(np.abs(seg_g - seg_r)) <= 3e-2 * max(np.max(np.abs(seg_r)), 1e-12), (l, n)
            o += n


def test_adam_steps_match_reference(ftp):
    """Two Adam steps of the GPU training kernel against the oracle's
    adam_step (bias corrections at t = 1 and t = 2), each from the gradient
    the GPU computes at the current weights (the update arithmetic alone is
    compared; FP32 on the GPU, FP64 in the reference)."""
    import torch
    rng = np.random.default_rng(11)
    din, width, dout, B, R = 22, 32, 8, 64, 6
    net = ftp.Mlp(din, width, dout, seed=3)
    Xb = torch.as_tensor(rng.standard_normal((B, din)).astype(np.float32), device="cuda").to(torch.bfloat16)
    roots = torch.as_tensor(rng.uniform(0, 2 * np.pi, (B, R)).astype(np.float32), device="cuda")
    nroots = torch.as_tensor(rng.integers(1, R + 1, B).astype(np.int32), device="cuda")
    w = net.weights().astype(np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    lrs = (3e-3, 1e-3)
    for t, lr in enumerate(lrs, start=1):
        _, g = net.loss_grad(Xb, roots, nroots, lam=0.5)
        g = g.cpu().numpy().astype(np.float64)
        assert np.count_nonzero(g) > 0.5 * g.size
        net.train_step(Xb, roots, nroots, lr=lr, lam=0.5)
        torch.cuda.synchronize()
        w, m, v = MO.adam_step(w, g, m, v, t, lr=lr)
        got = net.weights().astype(np.float64)
        err = np.abs(got - w)
        assert np.max(err - 4e-6 * np.abs(w)) <= 1e-3 * lr, (t, float(np.max(err)))
        w = got   # continue from the GPU's weights (FP32 rounding of the masters)


def test_training_reduces_loss(ftp):
    import torch
    tmpl, lc = single_long_case(n_obs=1500)
    plan = ftp.Plan(tmpl.c, tmpl.s)
    X, roots, nroots = plan.learned_dataset(lc.t, lc.y, lc.sigma, lc.df, 6000, R=32)
    assert int(nroots.min()) >= 0 and int(nroots.max()) <= 32
    assert float(nroots.float().mean()) > 2.0
    din = X.shape[1]
    net = ftp.Mlp(din, 64, 4 * tmpl.H, seed=1)
    l0, _ = net.loss_grad(X, roots, nroots)
    loss = torch.empty(2048, dtype=torch.float32, device="cuda")
    for it in range(300):
        s = (it * 2048) % (X.shape[0] - 2048)
        net.train_step(X[s: s + 2048], roots[s: s + 2048], nroots[s: s + 2048], lr=2e-3, loss=loss)
    l1, _ = net.loss_grad(X, roots, nroots)
    assert float(l1.mean()) < 0.8 * float(l0.mean())


@pytest.mark.parametrize("solver", ["uniform", "learned", "aberth"])
def test_learned_and_uniform_match_companion(ftp, solver):
    import torch
    tmpl, lc = single_long_case(n_obs=3000)
    n_f = 8000
    plain = ftp.Plan(tmpl.c, tmpl.s)
    a = {k: v.clone() for k, v in plain.periodogram(lc.t, lc.y, lc.sigma, lc.df, n_f).items()}
    if solver == "uniform":
        p2 = ftp.Plan(tmpl.c, tmpl.s, solver=ftp.FTP_SOLVER_UNIFORM)
    elif solver == "aberth":
        p2 = ftp.Plan(tmpl.c, tmpl.s, solver=ftp.FTP_SOLVER_ABERTH)
    else:
        # an untrained network seeding every frequency's first round
        p2 = ftp.Plan(tmpl.c, tmpl.s, solver=ftp.FTP_SOLVER_LEARNED, flags=ftp.FTP_FLAG_SEEDS_ALL)
        din, width, dout = 2 * (6 * tmpl.H - 1), 64, 4 * tmpl.H
        w = np.random.default_rng(3).uniform(-0.2, 0.2, ftp.mlp_param_count(din, width, dout)).astype(np.float32)
        p2.load_mlp(w, width)
    p2.stats()
    b = p2.periodogram(lc.t, lc.y, lc.sigma, lc.df, n_f)
    st = p2.stats()
    dP = float(torch.max(torch.abs(a["power"] - b["power"])))
    assert dP <= 1e-10, dP
    fb = (b["status"] & ftp.ST_FALLBACK) != 0
    fbq = (b["status"] & ftp.ST_FALLBACK_QR) != 0
    assert int(fbq.sum()) == st["n_fallback_qr"]
    if solver == "aberth":
        assert st["n_fallback"] == 0 and st["newton_iters"] == 0
        assert int(fb.sum()) == st["n_fallback_qr"]
        assert st["aberth_iters"] > 0
    else:
        assert st["n_fallback"] < n_f
        assert int(fb.sum()) == st["n_fallback"]
        assert st["n_fallback_qr"] <= st["n_fallback"]
        assert st["n_fallback_aberth"] <= st["n_fallback"]
        if solver == "learned":
            # an untrained network leaves roots unconfirmed: the later tiers run
            assert st["n_fallback"] > 0
    assert torch.equal(a["status"], b["status"] & (0xFF ^ (ftp.ST_FALLBACK | ftp.ST_FALLBACK_QR)))


def test_forced_fallback_is_the_companion_solve(ftp):
    import torch
    tmpl, lc = single_long_case(n_obs=2000)
    n_f = 5000
    plain = ftp.Plan(tmpl.c, tmpl.s)
    a = {k: v.clone() for k, v in plain.periodogram(lc.t, lc.y, lc.sigma, lc.df, n_f).items()}
    for solver in (ftp.FTP_SOLVER_UNIFORM, ftp.FTP_SOLVER_ABERTH):
        p2 = ftp.Plan(tmpl.c, tmpl.s, solver=solver, flags=ftp.FTP_FLAG_FORCE_FALLBACK)
        p2.stats()
        b = p2.periodogram(lc.t, lc.y, lc.sigma, lc.df, n_f)
        st = p2.stats()
        assert st["n_fallback_qr"] == n_f
        assert st["n_fallback"] == (n_f if solver == ftp.FTP_SOLVER_UNIFORM else 0)
        for k in ("power", "phase", "amp", "offset"):
            assert torch.equal(a[k], b[k]), k
        assert torch.all(b["status"] == (a["status"] | ftp.ST_FALLBACK | ftp.ST_FALLBACK_QR))


def test_learned_requires_a_network(ftp):
    tmpl, lc = tiny_case(1, n_obs=50, H=3, n_f=20)
    p = ftp.Plan(tmpl.c, tmpl.s, solver=ftp.FTP_SOLVER_LEARNED)
    with pytest.raises(ftp.FtpError):
        p.periodogram(lc.t, lc.y, lc.sigma, lc.df, lc.n_f)


@pytest.mark.parametrize("width", [256, 64, 48])
def test_fused_network_kernel_equals_unfused(ftp, width):
    """The fused features + four-layer kernel reproduces the separate features
    kernel and GEMM launches bit for bit (same bf16 rounding points, same
    K order of the MFMA accumulation); width 48 is not fused (not a multiple
    of 32) and takes the separate kernels either way."""
    import torch
    tmpl, lc = single_long_case(n_obs=3000)
    n_f = 8000
    din, dout = 2 * (6 * tmpl.H - 1), 4 * tmpl.H
    if width == 256:
        w, meta = ftp.load_model("single_long_h6")
    else:
        w = np.random.default_rng(width).uniform(-0.2, 0.2, ftp.mlp_param_count(din, width, dout)).astype(np.float32)
    res = []
    for fused in (1, 0):
        p = ftp.Plan(tmpl.c, tmpl.s, solver=ftp.FTP_SOLVER_LEARNED)
        p.set_tuning(mlp_fused=fused)
        p.load_mlp(w, width)
        p.stats()
        out = {k: v.clone() for k, v in p.periodogram(lc.t, lc.y, lc.sigma, lc.df, n_f).items()}
        res.append((out, p.stats()))
    (a, sa), (b, sb) = res
    for k in a:
        assert torch.equal(a[k], b[k]), k
    for k in ("n_fallback", "newton_iters", "roots_found"):
        assert sa[k] == sb[k], k


def _run_stats(plan, lcs):
    """Periodograms of the lightcurves (power, status per lightcurve) and the
    plan's statistics summed over them."""
    import torch
    plan.stats()
    outs = []
    for lc in lcs:
        o = plan.periodogram(lc.t, lc.y, lc.sigma, lc.df, lc.n_f)
        outs.append({k: v.clone() for k, v in o.items()})
    torch.cuda.synchronize()
    return outs, plan.stats()


@pytest.mark.parametrize("model", ["single_long_h6", "large_h10"])
def test_network_seeds_beat_evenly_spaced_starts_at_equal_count(ftp, model):
    """What the trained network gains over the method without it: with the
    same number of Newton starts per frequency (2H), the network's seeds leave
    fewer frequencies unconfirmed by the Sturm count than evenly spaced starts,
    on held-out lightcurves (N_obs = 2000 for the H = 6 network, a large-case
    lightcurve for the H = 10 one); both periodograms equal the companion
    solve's."""
    import torch
    w, meta = ftp.load_model(model)
    if model == "single_long_h6":
        tmpl, lcs = learned_heldout_lightcurves(n_lc=8)
    else:
        tmpl, lcs = large_heldout_lightcurves(n_lc=1)
    uni = ftp.Plan(tmpl.c, tmpl.s, solver=ftp.FTP_SOLVER_UNIFORM, flags=ftp.FTP_FLAG_2H_STARTS)
    lrn = ftp.Plan(tmpl.c, tmpl.s, solver=ftp.FTP_SOLVER_LEARNED,
                   flags=ftp.FTP_FLAG_2H_STARTS | ftp.FTP_FLAG_SEEDS_ALL)
    lrn.load_mlp(w, meta["width"])
    ou, su = _run_stats(uni, lcs)
    ol, sl = _run_stats(lrn, lcs)
    plain = ftp.Plan(tmpl.c, tmpl.s)
    op, _ = _run_stats(plain, lcs[:2])
    for a, b, c in zip(op, ou, ol):
        assert float(torch.max(torch.abs(a["power"] - b["power"]))) <= 1e-10
        assert float(torch.max(torch.abs(a["power"] - c["power"]))) <= 1e-10
    pairs = sum(lc.n_f for lc in lcs)
    print(f"{model}: unconfirmed with 2H starts: network {sl['n_fallback'] / pairs:.4f}, "
          f"evenly spaced {su['n_fallback'] / pairs:.4f}")
    assert sl["n_fallback"] < 0.75 * su["n_fallback"]


@pytest.mark.parametrize("flags", [0, 16])
def test_learned_matches_oracle_on_heldout_lightcurves(ftp, flags):
    """The learned solver (trained H = 6 network; second-round seeds, or
    seeds in every first round) on held-out lightcurves (N_obs = 2000,
    T = 1000 d) against the oracle on sampled frequencies and at the best
    frequency, and against the companion solve everywhere."""
    import torch
    w, meta = ftp.load_model("single_long_h6")
    tmpl, lcs = learned_heldout_lightcurves(n_lc=3)
    lrn = ftp.Plan(tmpl.c, tmpl.s, solver=ftp.FTP_SOLVER_LEARNED, flags=flags)
    lrn.load_mlp(w, meta["width"])
    plain = ftp.Plan(tmpl.c, tmpl.s)
    rng = np.random.default_rng(41)
    for lc in lcs:
        a = {k: v.clone() for k, v in plain.periodogram(lc.t, lc.y, lc.sigma, lc.df, lc.n_f).items()}
        b = lrn.periodogram(lc.t, lc.y, lc.sigma, lc.df, lc.n_f)
        assert float(torch.max(torch.abs(a["power"] - b["power"]))) <= 1e-10
        P = b["power"].cpu().numpy()
        top = np.argsort(P)[::-1][:5] + 1
        js = np.unique(np.r_[rng.integers(1, lc.n_f + 1, 30), top])
        ref = O.periodogram(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, lc.df, freq_index=js)
        assert np.max(np.abs(P[js - 1] - ref["power"])) <= 1e-4
        srt = np.sort(ref["power"])[::-1]
        if srt[0] - srt[1] > 1e-4:
            assert int(js[np.argmax(ref["power"])]) == int(top[0])
