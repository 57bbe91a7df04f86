"""Templates with H = 12..15 harmonics (degree D = 6H - 2 = 70..88 > 64): the
companion QR with two rows per lane, the Sturm chain in double-double with
two coefficients per lane, two candidates per lane in the scoring, and the
Aberth tier handing its list to the companion solve, each against the CPU
FP64 oracle (Section 2.3
puts the practical limit of the method near H = 15).

Tolerances as in test_gpu_parity: |dP| <= 1e-12 from exact sums (1e-11 here:
the companion of degree 88 has entries over a wider range), 1e-4 end to end
with FP32 sums.
"""
import numpy as np
import pytest

from oracle import ftp_oracle as O
from synthetic import tiny_case

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


def _exact_sums(tmpl, lc, H):
    js = np.arange(1, lc.n_f + 1)
    tref = 0.5 * (lc.t.min() + lc.t.max())
    Zw, Zy, ybar, YY = O.raw_sums(lc.t, lc.y, lc.sigma, lc.df, js, 2 * H, H, t_ref=tref)
    return js, np.concatenate([Zw, Zy], axis=1), tref, ybar, YY


@pytest.mark.parametrize("solver", ["plain", "uniform", "learned"])
@pytest.mark.parametrize("seed,H", [(21, 12), (22, 13), (23, 14), (24, 15)])
def test_high_h_solvers_from_exact_sums(ftp, solver, seed, H):
    print(f"[high-H exact sums] solver={solver} seed={seed} H={H}", flush=True)
    tmpl, lc = tiny_case(seed, n_obs=120, H=H, n_f=40, cadence="nightly")
    js, sums, tref, ybar, YY = _exact_sums(tmpl, lc, H)
    sv = {"plain": ftp.FTP_SOLVER_PLAIN, "uniform": ftp.FTP_SOLVER_UNIFORM,
          "learned": ftp.FTP_SOLVER_LEARNED}[solver]
    plan = ftp.Plan(tmpl.c, tmpl.s, precision=ftp.FTP_FP64, solver=sv)
    if solver == "learned":
        # an untrained network: its seeds only steer the second Newton round
        din, width, dout = 2 * (6 * H - 1), 64, 4 * H
        w = np.random.default_rng(seed).uniform(-0.2, 0.2, ftp.mlp_param_count(din, width, dout))
        plan.load_mlp(w.astype(np.float32), width)
    g = {k: _np(v) for k, v in plan.solve_sums(sums, tref, ybar, YY, lc.df).items()}
    ref = O.periodogram(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, lc.df, lc.n_f)
    assert np.all((g["status"] & 0x7) == 0)
    dP = np.abs(g["power"] - ref["power"])
    assert np.max(dP) <= 1e-11, (float(np.max(dP)), int(np.argmax(dP)))
    # the reported phase achieves the reported power at observation level
    for q in range(0, lc.n_f, 7):
        f = js[q] * lc.df
        P, _, _ = O.direct_fit_at_phase(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, f, g["phase"][q])
        assert abs(P - g["power"][q]) <= 1e-11, (q, P, g["power"][q])


@pytest.mark.parametrize("seed,H", [(25, 12), (26, 15)])
def test_high_h_sturm_count_against_companion(ftp, seed, H):
    """At D > 64 the Sturm chain runs in double-double, two coefficients per
    lane.  Its count must equal the number of real eigenvalues the companion
    QR finds wherever the chain trusts it, and the chain must trust it on
    nearly every frequency (in double precision the coefficients' spread made
    the step test refuse every chain at these degrees)."""
    print(f"[high-H root counts] seed={seed} H={H}", flush=True)
    tmpl, lc = tiny_case(seed, n_obs=150, H=H, n_f=300, cadence="nightly")
    _, sums, tref, ybar, YY = _exact_sums(tmpl, lc, H)
    plan = ftp.Plan(tmpl.c, tmpl.s, precision=ftp.FTP_FP64)
    sc, cr = (_np(x) for x in plan.root_counts(sums, tref, ybar, YY, lc.df))
    assert np.all(cr >= 0)
    trusted = sc >= 0
    assert np.all(sc[~trusted] <= -1000)
    print(f"H={H}: trusted {int(trusted.sum())} of {len(sc)}")
    assert trusted.mean() >= 0.95, trusted.mean()
    assert np.array_equal(sc[trusted], cr[trusted]), np.flatnonzero(sc[trusted] != cr[trusted])[:10]
    assert np.all(sc[trusted] % 2 == 0)


def test_high_h_aberth_refused(ftp):
    rng = np.random.default_rng(3)
    c, s = rng.standard_normal(12), rng.standard_normal(12)
    with pytest.raises(ftp.FtpError):
        ftp.Plan(c, s, solver=ftp.FTP_SOLVER_ABERTH)
    with pytest.raises(ftp.FtpError):
        ftp.Plan(rng.standard_normal(16), rng.standard_normal(16))


@pytest.mark.parametrize("solver", ["plain", "uniform"])
def test_high_h_end_to_end_fp32(ftp, solver):
    """H = 15 end to end (FP32 NFFT sums, FP64 solve) against the oracle."""
    print(f"[high-H end to end] solver={solver}", flush=True)
    H = 15
    tmpl, lc = tiny_case(27, n_obs=400, H=H, n_f=250, baseline=30.0, cadence="nightly")
    sv = ftp.FTP_SOLVER_PLAIN if solver == "plain" else ftp.FTP_SOLVER_UNIFORM
    plan = ftp.Plan(tmpl.c, tmpl.s, solver=sv)
    g = {k: _np(v) for k, v in plan.periodogram(lc.t, lc.y, lc.sigma, lc.df, lc.n_f).items()}
    ref = O.periodogram(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, lc.df, lc.n_f)
    assert np.max(np.abs(g["power"] - ref["power"])) <= 1e-4
    assert int(np.argmax(g["power"])) == int(np.argmax(ref["power"]))


@pytest.mark.parametrize("H", [12, 13, 14, 15])
def test_high_h_uniform_equals_companion_on_long_lightcurve(ftp, H):
    """The Sturm-verified Newton path against the companion solve on every
    frequency of an N_obs = 1e4 lightcurve (~5e4 frequencies; the H sweep's
    input), same FP32 sums: a count trusted wrongly would miss roots and show
    as a lower power."""
    from synthetic import h_sweep_case
    print(f"[high-H long lightcurve] H={H}", flush=True)
    tmpl, lc = h_sweep_case(H)
    outs = {}
    for name, sv in (("plain", ftp.FTP_SOLVER_PLAIN), ("uniform", ftp.FTP_SOLVER_UNIFORM)):
        plan = ftp.Plan(tmpl.c, tmpl.s, solver=sv)
        outs[name] = _np(plan.periodogram(lc.t, lc.y, lc.sigma, lc.df, lc.n_f)["power"])
    d = np.abs(outs["plain"] - outs["uniform"])
    assert np.max(d) <= 1e-9, (float(np.max(d)), int(np.argmax(d)) + 1)
