"""Shared-phase multi-band periodogram (Appendix A) through
ftp_periodogram_shared_phase, against the oracle's
shared_phase_periodogram (per-band templates, band offsets, weights
normalised over all bands).

* FP64 sums, three small bands with different templates (one of fewer
  harmonics) and offsets, every root solver that needs no network:
  |dP| <= 1e-9; the reported phase reaches the oracle's power (|dP| <= 1e-9
  at the GPU phase, observation-level least squares), amplitude and offset
  are the least-squares values at that phase.
* One band equals the single-band plan (|dP| <= 1e-10); two bands with one
  template and no offsets equal the single-band periodogram of the joined
  data.
* FP32 sums, the five-band workload: sampled |dP| <= 1e-4 against the oracle;
  the peak is the common frequency.
* Positive amplitude: amp >= 0 and P never above the unrestricted P.
* Bands mixing unit and sigma weights, or a NaN: every frequency ST_BAD_LC.
* A bands plan refuses the single-band calls (FTP_E_OPTION).
"""
import numpy as np
import pytest

from oracle import ftp_oracle as O
from synthetic import Template, cadence_nightly, eval_template, shared_phase_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ftp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2101_12348_amd as F
    F.load_library()
    return F


TMS = [Template(np.array([1.0, 0.4, 0.1]), np.array([0.2, -0.3, 0.2])),
       Template(np.array([0.7, 0.5]), np.array([-0.1, 0.3])),
       Template(np.array([1.2, 0.2, -0.2]), np.array([0.0, 0.1, 0.3]))]
LAM = np.array([0.0, 0.8, -0.5])


def _small(seed=60, ns=(70, 55, 90)):
    """Three bands on nightly cadences over 20 d, period 1.7 d."""
    rng = np.random.default_rng(seed)
    bands = []
    for k, n in enumerate(ns):
        t = cadence_nightly(rng, n, 20.0)
        sig = rng.uniform(0.05, 0.2, n)
        y = 0.9 * eval_template(TMS[k], 2 * np.pi * t / 1.7 - 0.6) + 0.3 + LAM[k] + sig * rng.standard_normal(n)
        bands.append((t, y, sig))
    return bands, 1.0 / 40.0, 120


def _fit_at_phase(bands, tms, lam, f, th):
    """Observation-level weighted least squares of y - lambda_k on
    theta_1 M_k(2 pi f t - theta_2) + theta_3 at fixed theta_2: (P, theta_1,
    theta_3) with P = 1 - chi^2 / chi^2_0."""
    w = np.concatenate([1.0 / b[2] ** 2 for b in bands])
    y = np.concatenate([b[1] - lam[k] for k, b in enumerate(bands)])
    M = np.concatenate([O.template_values(tms[k].c, tms[k].s, 2 * np.pi * f * b[0] - th)
                        for k, b in enumerate(bands)])
    A = np.stack([M, np.ones_like(M)], axis=1)
    sw = np.sqrt(w)
    coef, *_ = np.linalg.lstsq(A * sw[:, None], y * sw, rcond=None)
    chi2 = np.sum(w * (y - A @ coef) ** 2)
    ybar = np.dot(w, y) / w.sum()
    chi20 = np.sum(w * (y - ybar) ** 2)
    return 1.0 - chi2 / chi20, coef[0], coef[1]


@pytest.mark.parametrize("solver", ["PLAIN", "UNIFORM", "ABERTH"])
def test_shared_phase_small_fp64(ftp, solver):
    bands, df, n_f = _small()
    plan = ftp.BandsPlan([(tm.c, tm.s) for tm in TMS], precision=ftp.FTP_FP64,
                         solver=getattr(ftp, "FTP_SOLVER_" + solver))
    out = {k: v.cpu().numpy() for k, v in plan.periodogram_shared_phase(bands, df, n_f, offsets=LAM).items()}
    ref = O.shared_phase_periodogram(bands, [(tm.c, tm.s) for tm in TMS], df, n_f=n_f, offsets=LAM)
    assert np.max(np.abs(out["power"] - ref["power"])) <= 1e-9
    assert np.all((out["status"] & 7) == 0)
    for j in range(1, n_f + 1, 7):
        P, a, b = _fit_at_phase(bands, TMS, LAM, j * df, out["phase"][j - 1])
        assert abs(P - ref["power"][j - 1]) <= 1e-9, j
        assert abs(a - out["amp"][j - 1]) <= 1e-7 * max(1.0, abs(a)), j
        assert abs(b - out["offset"][j - 1]) <= 1e-7 * max(1.0, abs(b)), j


def test_shared_phase_reduces_to_single_band(ftp):
    bands, df, n_f = _small(61)
    tm = TMS[0]
    single = ftp.Plan(tm.c, tm.s, precision=ftp.FTP_FP64)
    one = ftp.BandsPlan([(tm.c, tm.s)], precision=ftp.FTP_FP64)
    a = one.periodogram_shared_phase(bands[:1], df, n_f)["power"].cpu().numpy()
    b = single.periodogram(*bands[0], df, n_f)["power"].cpu().numpy()
    assert np.max(np.abs(a - b)) <= 1e-10
    two = ftp.BandsPlan([(tm.c, tm.s)] * 2, precision=ftp.FTP_FP64)
    a2 = two.periodogram_shared_phase(bands[:2], df, n_f)["power"].cpu().numpy()
    cat = [np.concatenate([bd[i] for bd in bands[:2]]) for i in range(3)]
    b2 = single.periodogram(*cat, df, n_f)["power"].cpu().numpy()
    assert np.max(np.abs(a2 - b2)) <= 1e-10


def test_shared_phase_five_bands_fp32(ftp):
    tms, bands, lam, df, n_f, f0 = shared_phase_case()
    plan = ftp.BandsPlan([(tm.c, tm.s) for tm in tms], solver=ftp.FTP_SOLVER_UNIFORM)
    out = plan.periodogram_shared_phase(bands, df, n_f, offsets=lam)
    g = out["power"].cpu().numpy()
    jbest = int(np.argmax(g)) + 1
    rng = np.random.default_rng(6)
    js = np.unique(np.r_[jbest, rng.integers(1, n_f + 1, 30)])
    ref = O.shared_phase_periodogram(bands, [(tm.c, tm.s) for tm in tms], df, freq_index=js, offsets=lam)
    assert np.max(np.abs(g[js - 1] - ref["power"])) <= 1e-4
    assert abs(jbest * df - f0) <= 1.5 * df


def test_shared_phase_positive_amplitude(ftp):
    bands, df, n_f = _small(62)
    tms = [(tm.c, tm.s) for tm in TMS]
    free = ftp.BandsPlan(tms, precision=ftp.FTP_FP64)
    pos = ftp.BandsPlan(tms, precision=ftp.FTP_FP64, flags=ftp.FTP_FLAG_POSITIVE_AMP)
    a = free.periodogram_shared_phase(bands, df, n_f, offsets=LAM)
    b = pos.periodogram_shared_phase(bands, df, n_f, offsets=LAM)
    pa, pb = a["power"].cpu().numpy(), b["power"].cpu().numpy()
    assert np.all(b["amp"].cpu().numpy() >= 0.0)
    assert np.all(pb <= pa + 1e-12)
    keep = a["amp"].cpu().numpy() > 0
    assert np.max(np.abs(pa[keep] - pb[keep])) <= 1e-12


def test_shared_phase_rejected_inputs(ftp):
    bands, df, n_f = _small(63)
    plan = ftp.BandsPlan([(tm.c, tm.s) for tm in TMS], precision=ftp.FTP_FP64)
    mixed = [bands[0], (bands[1][0], bands[1][1], np.zeros_like(bands[1][2])), bands[2]]
    st = plan.periodogram_shared_phase(mixed, df, n_f)["status"].cpu().numpy()
    assert np.all(st == ftp.ST_BAD_LC)
    nan = [bands[0], bands[1], (bands[2][0], bands[2][1].copy(), bands[2][2])]
    nan[2][1][5] = np.nan
    out = plan.periodogram_shared_phase(nan, df, n_f)
    assert np.all(out["status"].cpu().numpy() == ftp.ST_BAD_LC)
    assert float(out["power"].abs().max()) == 0.0
    with pytest.raises(ftp.FtpError):
        plan.periodogram(*bands[0], df, n_f)
    with pytest.raises(ValueError):
        plan.periodogram_shared_phase(bands[:2], df, n_f)
