"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle.

Tolerances:
* per-frequency stage fed with exact (direct) sums: |dP| <= 1e-12;
* end to end, FP64 NFFT: |dP| <= 1e-9 (NFFT error ~5e-13 of sum|g|);
* end to end, FP32 NFFT: |dP| <= 1e-4 (NFFT error ~1e-8 of sum|g|);
* phases are compared through the power the reported phase achieves at
  observation level (robust to exact ties), amplitudes/offsets through the
  least-squares fit at the reported phase.
"""
import numpy as np
import pytest

from oracle import ftp_oracle as O
from synthetic import tiny_case, small_fp64_case, single_long_case, Template, eval_template

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ftp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2101_12348_amd as F
    F.load_library()
    return F


def _np(x):
    return x.detach().cpu().numpy()


def _check_phase_fit(tmpl, lc, js, out, tol_p, tol_fit):
    """The reported (theta2, theta1, theta3) reproduce the reported power and
    the least-squares amplitude/offset at that phase."""
    for q, j in enumerate(js):
        f = j * lc.df
        P, a, b = O.direct_fit_at_phase(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, f, out["phase"][q])
        assert abs(P - out["power"][q]) <= tol_p, (j, P, out["power"][q])
        scale = max(1.0, abs(a))
        assert abs(a - out["amp"][q]) <= tol_fit * scale, (j, a, out["amp"][q])
        assert abs(b - out["offset"][q]) <= tol_fit * max(1.0, abs(b)) + tol_fit * scale


@pytest.mark.parametrize("seed,H", [(0, 1), (1, 2), (2, 3), (3, 6), (4, 10)])
def test_solve_stage_from_exact_sums(ftp, seed, H):
    tmpl, lc = tiny_case(seed, n_obs=80, H=H, n_f=60, cadence="nightly")
    js = np.arange(1, lc.n_f + 1)
    tref = 0.5 * (lc.t.min() + lc.t.max())
    Zw, Zy, ybar, YY = O.raw_sums(lc.t, lc.y, lc.sigma, lc.df, js, 2 * H, H, t_ref=tref)
    sums = np.concatenate([Zw, Zy], axis=1)
    plan = ftp.Plan(tmpl.c, tmpl.s, precision=ftp.FTP_FP64)
    out = plan.solve_sums(sums, tref, ybar, YY, lc.df)
    g = {k: _np(v) for k, v in out.items()}
    ref = O.periodogram(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, lc.df, lc.n_f)
    assert np.all(g["status"] == 0)
    assert np.max(np.abs(g["power"] - ref["power"])) <= 1e-12
    _check_phase_fit(tmpl, lc, js, g, 1e-12, 1e-8)


@pytest.mark.parametrize("solver", ["plain", "uniform", "aberth"])
@pytest.mark.parametrize("seed,H", [(5, 1), (6, 3), (7, 6), (8, 10), (9, 11)])
def test_root_solvers_from_exact_sums(ftp, solver, seed, H):
    """Every root solver (companion QR; Newton from evenly spaced starts with
    the Sturm check and the Aberth / companion tiers behind it; Aberth on
    every frequency) reproduces the oracle from exact sums, up to H = 11
    (D = 64: all lanes of a wavefront, the LDS form of the Sturm chain)."""
    tmpl, lc = tiny_case(seed, n_obs=80, H=H, n_f=60, cadence="nightly")
    js = np.arange(1, lc.n_f + 1)
    tref = 0.5 * (lc.t.min() + lc.t.max())
    Zw, Zy, ybar, YY = O.raw_sums(lc.t, lc.y, lc.sigma, lc.df, js, 2 * H, H, t_ref=tref)
    sums = np.concatenate([Zw, Zy], axis=1)
    sv = {"plain": ftp.FTP_SOLVER_PLAIN, "uniform": ftp.FTP_SOLVER_UNIFORM, "aberth": ftp.FTP_SOLVER_ABERTH}[solver]
    plan = ftp.Plan(tmpl.c, tmpl.s, precision=ftp.FTP_FP64, solver=sv)
    out = plan.solve_sums(sums, tref, ybar, YY, lc.df)
    g = {k: _np(v) for k, v in out.items()}
    ref = O.periodogram(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, lc.df, lc.n_f)
    assert np.all((g["status"] & 0x7) == 0)
    assert np.max(np.abs(g["power"] - ref["power"])) <= 1e-12
    _check_phase_fit(tmpl, lc, js, g, 1e-12, 1e-8)


@pytest.mark.parametrize("solver", ["plain", "uniform", "aberth"])
@pytest.mark.parametrize("seed,H", [(10, 2), (11, 3), (12, 6)])
def test_positive_amplitude_from_exact_sums(ftp, solver, seed, H):
    """The theta_1 > 0 variant (FTP_FLAG_POSITIVE_AMP) against the oracle's
    constrained fit, from exact sums."""
    tmpl, lc = tiny_case(seed, n_obs=80, H=H, n_f=60, cadence="nightly")
    js = np.arange(1, lc.n_f + 1)
    tref = 0.5 * (lc.t.min() + lc.t.max())
    Zw, Zy, ybar, YY = O.raw_sums(lc.t, lc.y, lc.sigma, lc.df, js, 2 * H, H, t_ref=tref)
    sums = np.concatenate([Zw, Zy], axis=1)
    sv = {"plain": ftp.FTP_SOLVER_PLAIN, "uniform": ftp.FTP_SOLVER_UNIFORM, "aberth": ftp.FTP_SOLVER_ABERTH}[solver]
    plan = ftp.Plan(tmpl.c, tmpl.s, precision=ftp.FTP_FP64, solver=sv, flags=ftp.FTP_FLAG_POSITIVE_AMP)
    g = {k: _np(v) for k, v in plan.solve_sums(sums, tref, ybar, YY, lc.df).items()}
    ref = O.periodogram(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, lc.df, lc.n_f, positive_amplitude=True)
    unc = O.periodogram(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, lc.df, lc.n_f)
    assert np.max(np.abs(g["power"] - ref["power"])) <= 1e-12
    assert np.all(g["amp"][g["power"] > 0] > 0)
    assert np.any(unc["amp"] < 0)   # the constraint is active somewhere on this grid
    _check_phase_fit(tmpl, lc, js, g, 1e-12, 1e-8)


def test_positive_amplitude_end_to_end_fp32(ftp):
    tmpl, lc = single_long_case(n_obs=3000)
    n_f = 6000
    plan = ftp.Plan(tmpl.c, tmpl.s, solver=ftp.FTP_SOLVER_UNIFORM, flags=ftp.FTP_FLAG_POSITIVE_AMP)
    g = {k: _np(v) for k, v in plan.periodogram(lc.t, lc.y, lc.sigma, lc.df, n_f).items()}
    js = np.unique(np.random.default_rng(4).integers(1, n_f + 1, 120))
    ref = O.periodogram(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, lc.df, freq_index=js, positive_amplitude=True)
    assert np.max(np.abs(g["power"][js - 1] - ref["power"])) <= 1e-4
    assert np.all(g["amp"][g["power"] > 0] > 0)


@pytest.mark.parametrize("precision,tol", [(1, 5e-12), (0, 5e-7)])
def test_nfft_sums_against_direct_sums(ftp, precision, tol):
    tmpl, lc = single_long_case(n_obs=3000)
    H = tmpl.H
    n_f = 4000
    plan = ftp.Plan(tmpl.c, tmpl.s, precision=precision)
    sums, st = plan.nfft_sums(lc.t, lc.y, lc.sigma, lc.df, n_f)
    sums = _np(sums)
    st = _np(st)
    tref = 0.5 * (lc.t.min() + lc.t.max())
    assert st[0] == tref and st[3] == 0
    rng = np.random.default_rng(0)
    js = np.unique(np.r_[1, n_f, rng.integers(1, n_f + 1, 40)])
    Zw, Zy, ybar, YY = O.raw_sums(lc.t, lc.y, lc.sigma, lc.df, js, 2 * H, H, t_ref=tref)
    assert abs(st[1] - ybar) < 1e-12 and abs(st[2] - YY) < 1e-12 * YY
    errw = np.max(np.abs(sums[js - 1, : 2 * H] - Zw))
    # the y sums are bounded by sum|w (y - ybar)| <= sqrt(YY)
    erry = np.max(np.abs(sums[js - 1, 2 * H:] - Zy)) / np.sqrt(YY)
    assert errw <= tol and erry <= tol, (errw, erry)


def test_end_to_end_small_fp64(ftp):
    tmpl, lc = small_fp64_case()
    plan = ftp.Plan(tmpl.c, tmpl.s, precision=ftp.FTP_FP64)
    out = plan.periodogram(lc.t, lc.y, lc.sigma, lc.df, lc.n_f)
    g = {k: _np(v) for k, v in out.items()}
    ref = O.periodogram(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, lc.df, lc.n_f)
    assert np.all(g["status"] == 0)
    assert np.max(np.abs(g["power"] - ref["power"])) <= 1e-9
    assert int(np.argmax(g["power"])) == int(np.argmax(ref["power"]))
    js = np.arange(1, lc.n_f + 1)
    _check_phase_fit(tmpl, lc, js[::7], {k: v[::7] for k, v in g.items()}, 1e-9, 1e-6)


def test_end_to_end_single_long_fp32_sampled(ftp):
    tmpl, lc = single_long_case()
    plan = ftp.Plan(tmpl.c, tmpl.s, precision=ftp.FTP_FP32_SUMS)
    out = plan.periodogram(lc.t, lc.y, lc.sigma, lc.df, lc.n_f)
    g = {k: _np(v) for k, v in out.items()}
    assert np.all(g["status"] == 0)
    rng = np.random.default_rng(1)
    jbest = int(np.argmax(g["power"])) + 1
    js = np.unique(np.r_[1, lc.n_f, jbest, rng.integers(1, lc.n_f + 1, 150)])
    ref = O.periodogram(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, lc.df, freq_index=js)
    assert np.max(np.abs(g["power"][js - 1] - ref["power"])) <= 1e-4
    # the injected frequency is the GPU peak
    assert abs(jbest * lc.df - lc.f0) <= 1.5 * lc.df
    _check_phase_fit(tmpl, lc, js[:40], {k: v[js[:40] - 1] for k, v in g.items()}, 1e-4, 1e-2)


def test_repeatable_bitwise(ftp):
    import torch
    tmpl, lc = single_long_case(n_obs=2000)
    plan = ftp.Plan(tmpl.c, tmpl.s)
    a = plan.periodogram(lc.t, lc.y, lc.sigma, lc.df, 5000)
    a = {k: v.clone() for k, v in a.items()}
    b = plan.periodogram(lc.t, lc.y, lc.sigma, lc.df, 5000)
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_unsorted_times_and_edge_cases(ftp):
    tmpl, lc = tiny_case(5, n_obs=90, H=3, n_f=40)
    perm = np.random.default_rng(3).permutation(len(lc.t))
    plan = ftp.Plan(tmpl.c, tmpl.s, precision=ftp.FTP_FP64)
    a = {k: _np(v) for k, v in plan.periodogram(lc.t, lc.y, lc.sigma, lc.df, lc.n_f).items()}
    b = {k: _np(v) for k, v in plan.periodogram(lc.t[perm], lc.y[perm], lc.sigma[perm], lc.df, lc.n_f).items()}
    assert np.max(np.abs(a["power"] - b["power"])) <= 1e-12
    # all sigma = 0: uniform weights (Section 2)
    r = O.periodogram(lc.t, lc.y, np.zeros(len(lc.t)), tmpl.c, tmpl.s, lc.df, lc.n_f)
    g = _np(plan.periodogram(lc.t, lc.y, np.zeros(len(lc.t)), lc.df, lc.n_f)["power"])
    assert np.max(np.abs(g - r["power"])) <= 1e-9
    # rejected inputs: mixed zero sigma, NaN, zero variance
    bad_sig = lc.sigma.copy(); bad_sig[3] = 0.0
    st = _np(plan.periodogram(lc.t, lc.y, bad_sig, lc.df, lc.n_f)["status"])
    assert np.all(st == ftp.ST_BAD_LC)
    bad_y = lc.y.copy(); bad_y[7] = np.nan
    st = _np(plan.periodogram(lc.t, bad_y, lc.sigma, lc.df, lc.n_f)["status"])
    assert np.all(st == ftp.ST_BAD_LC)
    st = _np(plan.periodogram(lc.t, np.ones(len(lc.t)), lc.sigma, lc.df, lc.n_f)["status"])
    assert np.all(st == ftp.ST_BAD_LC)
    # host-detectable errors are returned synchronously
    with pytest.raises(ftp.FtpError):
        plan.periodogram(lc.t[:2], lc.y[:2], lc.sigma[:2], lc.df, lc.n_f)
    with pytest.raises(ftp.FtpError):
        plan.periodogram(lc.t, lc.y, lc.sigma, -1.0, lc.n_f)


def test_degenerate_periodic_sampling(ftp):
    tm = Template(np.array([1.0, 0.3]), np.array([0.2, -0.5]))
    t = np.arange(60, dtype=np.float64)
    y = np.random.default_rng(5).standard_normal(60)
    df = 1.0 / 300.0
    plan = ftp.Plan(tm.c, tm.s, precision=ftp.FTP_FP64)
    g = {k: _np(v) for k, v in plan.periodogram(t, y, np.ones(60), df, 400).items()}
    ref = O.periodogram(t, y, np.ones(60), tm.c, tm.s, df, 400)
    # f = 1/day (j = 300) is degenerate: all phases coincide
    assert ref["flag"][299] == 1 and g["status"][299] == ftp.ST_DEGENERATE and g["power"][299] == 0.0
    ok = ref["flag"] == 0
    assert np.max(np.abs(g["power"][ok] - ref["power"][ok])) <= 1e-8


def test_noiseless_injection_gpu(ftp):
    rng = np.random.default_rng(21)
    H = 5
    tm = Template(rng.standard_normal(H), rng.standard_normal(H))
    t = np.sort(rng.uniform(0, 40, 300))
    df = 1.0 / (5 * (t.max() - t.min()))
    j0 = 123
    A, phi, B = 0.8, 1.3, 2.0
    y = A * eval_template(tm, 2 * np.pi * j0 * df * t - phi) + B
    plan = ftp.Plan(tm.c, tm.s, precision=ftp.FTP_FP64)
    g = {k: _np(v) for k, v in plan.periodogram(t, y, np.full(300, 0.1), df, 400).items()}
    assert int(np.argmax(g["power"])) == j0 - 1
    assert abs(g["power"][j0 - 1] - 1.0) < 1e-9
    assert abs(g["amp"][j0 - 1] - A) < 1e-7 and abs(g["offset"][j0 - 1] - B) < 1e-7
    d = (g["phase"][j0 - 1] - phi + np.pi) % (2 * np.pi) - np.pi
    assert abs(d) < 1e-7


@pytest.mark.parametrize("n_obs", [2047, 2048, 5000, 300_000])
def test_long_lightcurve_statistics(ftp, n_obs):
    # weighted mean and YY of one long lightcurve (Section 2): the many-workgroup
    # reduction against the oracle, with weights, with uniform weights, with a
    # mean far above the scatter, and the rejected inputs
    tmpl, lc = single_long_case(n_obs=min(n_obs, 10_000))
    rng = np.random.default_rng(n_obs)
    t = np.sort(rng.uniform(0.0, 1000.0, n_obs)) if n_obs > 10_000 else lc.t
    y = rng.standard_normal(n_obs) if n_obs > 10_000 else lc.y
    sig = rng.uniform(0.05, 0.2, n_obs) if n_obs > 10_000 else lc.sigma
    plan = ftp.Plan(tmpl.c, tmpl.s, precision=ftp.FTP_FP64)
    js = np.array([1, 7])
    for yy_in, ss in ((y, sig), (y + 1e6, sig), (y, np.zeros(n_obs))):
        _, st = plan.nfft_sums(t, yy_in, ss, lc.df, 8)
        st = _np(st)
        _, _, ybar, YY = O.raw_sums(t, yy_in, ss, lc.df, js, 2 * tmpl.H, tmpl.H, t_ref=st[0])
        assert st[3] == 0
        assert st[0] == 0.5 * (t.min() + t.max())
        assert abs(st[1] - ybar) <= 1e-12 * max(1.0, abs(ybar)), (st[1], ybar)
        assert abs(st[2] - YY) <= 1e-9 * YY, (st[2], YY)
    mixed = sig.copy(); mixed[n_obs // 2] = 0.0
    nan_y = y.copy(); nan_y[-1] = np.nan
    for yy_in, ss in ((y, mixed), (nan_y, sig), (np.full(n_obs, 3.0), sig)):
        _, st = plan.nfft_sums(t, yy_in, ss, lc.df, 8)
        assert _np(st)[3] != 0


def test_plan_reuse_across_inputs(ftp):
    # one plan serving lightcurves of different sizes, a batch and the
    # solve-from-sums entry in turn gives, on every call, what a fresh plan
    # gives (the plan's tables are re-sent only when they change)
    import torch
    tmpl, a = single_long_case(n_obs=2500)
    _, b = single_long_case(n_obs=400)
    n_f = 3000
    fresh = {}
    for name, lc in (("a", a), ("b", b)):
        p = ftp.Plan(tmpl.c, tmpl.s)
        fresh[name] = {k: v.clone() for k, v in p.periodogram(lc.t, lc.y, lc.sigma, lc.df, n_f).items()}
    plan = ftp.Plan(tmpl.c, tmpl.s)
    sums, st = plan.nfft_sums(a.t, a.y, a.sigma, a.df, n_f)
    stats = [float(x) for x in st.cpu()[:3]]
    ref_ss = {k: v.clone() for k, v in plan.solve_sums(sums, *stats, a.df).items()}
    for name, lc in (("a", a), ("a", a), ("b", b), ("a", a), ("b", b), ("b", b)):
        out = plan.periodogram(lc.t, lc.y, lc.sigma, lc.df, n_f)
        for k in ("power", "phase", "amp", "offset", "status"):
            assert torch.equal(out[k], fresh[name][k]), (name, k)
        s2, st2 = plan.nfft_sums(a.t, a.y, a.sigma, a.df, n_f)
        assert torch.equal(s2, sums) and torch.equal(st2, st)
        ss = plan.solve_sums(sums, *stats, a.df)
        for k in ("power", "phase", "amp", "offset", "status"):
            assert torch.equal(ss[k], ref_ss[k]), ("sums", k)
