"""Multi-phase multi-band periodogram (Section 2.2) through
ftp_periodogram_multiband, against the oracle's combination
sum_k chi2_0,k P_k / sum_k chi2_0,k.

* FP64 sums, three small bands: |dP| <= 1e-9, chi2_0 to 1e-12 relative, and
  the band periodograms equal single-band calls bit for bit.
* FP32 sums, the five-band workload: sampled |dP| <= 1e-4; the peak is the
  common frequency.
* A rejected band (NaN) does not count.
"""
import numpy as np
import pytest

from oracle import ftp_oracle as O
from synthetic import multiband_case, tiny_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ftp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2101_12348_amd as F
    F.load_library()
    return F


def _small_bands():
    tmpl, lc0 = tiny_case(40, n_obs=90, H=3, n_f=80, cadence="nightly")
    bands = []
    for k, seed in enumerate((41, 42, 43)):
        _, lc = tiny_case(seed, n_obs=60 + 15 * k, H=3, n_f=80, cadence="nightly")
        bands.append((lc.t, lc.y, lc.sigma))
    return tmpl, bands, lc0.df, 80


def test_multiband_small_fp64(ftp):
    import torch
    tmpl, bands, df, n_f = _small_bands()
    plan = ftp.Plan(tmpl.c, tmpl.s, precision=ftp.FTP_FP64)
    out = plan.periodogram_multiband(bands, df, n_f)
    P, Pk, c0 = O.multiband_periodogram(bands, tmpl.c, tmpl.s, df, n_f=n_f)
    assert np.max(np.abs(out["power"].cpu().numpy() - P)) <= 1e-9
    assert np.max(np.abs(out["chi2_0"].cpu().numpy() / c0 - 1.0)) <= 1e-12
    for k, b in enumerate(bands):
        single = plan.periodogram(*b, df, n_f)["power"]
        assert torch.equal(single, out["band_power"][k]), k


def test_multiband_five_bands_fp32(ftp):
    tmpl, bands, df, n_f, f0 = multiband_case()
    plan = ftp.Plan(tmpl.c, tmpl.s, solver=ftp.FTP_SOLVER_UNIFORM)
    out = plan.periodogram_multiband(bands, df, n_f)
    g = out["power"].cpu().numpy()
    jbest = int(np.argmax(g)) + 1
    rng = np.random.default_rng(5)
    js = np.unique(np.r_[jbest, rng.integers(1, n_f + 1, 40)])
    P, _, _ = O.multiband_periodogram(bands, tmpl.c, tmpl.s, df, freq_index=js)
    assert np.max(np.abs(g[js - 1] - P)) <= 1e-4
    assert abs(jbest * df - f0) <= 1.5 * df


def test_multiband_rejected_band_does_not_count(ftp):
    tmpl, bands, df, n_f = _small_bands()
    plan = ftp.Plan(tmpl.c, tmpl.s, precision=ftp.FTP_FP64)
    bad = (bands[1][0], bands[1][1].copy(), bands[1][2])
    bad[1][3] = np.nan
    out = plan.periodogram_multiband([bands[0], bad, bands[2]], df, n_f)
    ref = plan.periodogram_multiband([bands[0], bands[2]], df, n_f)
    assert float(out["chi2_0"][1]) == 0.0
    assert np.max(np.abs(out["power"].cpu().numpy() - ref["power"].cpu().numpy())) <= 1e-15
