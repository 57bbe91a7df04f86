"""The Sturm count the learned and uniform solvers trust (project addition),
checked against the companion-matrix roots (Section 2: the real-phase
solutions of Eq. theta2cond are the unit-circle roots of the polynomial of
Eq. finalpoly).

* On every frequency of the single long (H = 6, ~5e4 frequencies) and large
  (H = 10, ~3e5 frequencies) workloads, from the GPU's own NFFT sums: wherever
  the Sturm chain passes its conditioning test, its count equals the number
  of real eigenvalues of the plain solver's companion QR; the test fails on
  few frequencies.
* On a sample of frequencies, from the oracle's exact sums: the Sturm count
  equals the oracle's number of unit-circle companion roots
  (unit_circle_root_count, pinned on constructed roots and on sign changes
  of R(theta) in tests/test_oracle_pins.py).
"""
import numpy as np
import pytest

from oracle import ftp_oracle as O
from synthetic import single_long_case, large_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ftp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2101_12348_amd as F
    F.load_library()
    return F


CASES = {"single_long": single_long_case, "large": large_case}


@pytest.mark.parametrize("case", ["single_long", "large"])
def test_sturm_count_equals_companion_real_roots(ftp, case):
    tmpl, lc = CASES[case]()
    plan = ftp.Plan(tmpl.c, tmpl.s, precision=ftp.FTP_FP32_SUMS)
    sums, st = plan.nfft_sums(lc.t, lc.y, lc.sigma, lc.df, lc.n_f)
    tref, ybar, yy, bad = [float(x) for x in st.cpu()]
    assert bad == 0
    sc, cr = plan.root_counts(sums, tref, ybar, yy, lc.df)
    sc, cr = sc.cpu().numpy(), cr.cpu().numpy()
    n = lc.n_f
    assert n >= 4.9e4
    active = (sc != -2) & (cr != -2)
    assert np.all((sc == -2) == (cr == -2))
    trusted = active & (sc >= 0) & (cr >= 0)
    # the conditioning test rejects few chains (those go to the fallback
    # tiers; -1000 - n carries the count such a chain reached)
    rejected = active & (sc <= -1000)
    assert np.all(active == ((sc >= 0) | rejected))
    assert np.count_nonzero(rejected) <= 0.01 * n
    mism = trusted & (sc != cr)
    assert np.count_nonzero(mism) == 0, (np.flatnonzero(mism)[:10], sc[mism][:10], cr[mism][:10])
    # real-root counts are even (roots of a real trig polynomial) and in range
    D = 6 * tmpl.H - 2
    assert np.all(sc[trusted] % 2 == 0) and np.all((sc[trusted] >= 2) & (sc[trusted] <= D))
    print(f"{case}: {np.count_nonzero(trusted)} polynomials compared, "
          f"{np.count_nonzero(rejected)} chains rejected, mean count {sc[trusted].mean():.2f}")


@pytest.mark.parametrize("case,n_sample", [("single_long", 60), ("large", 24)])
def test_sturm_count_equals_oracle_unit_circle_roots(ftp, case, n_sample):
    tmpl, lc = CASES[case]()
    H = tmpl.H
    rng = np.random.default_rng(17)
    js = np.unique(rng.integers(1, lc.n_f + 1, n_sample))
    tref = 0.5 * (lc.t.min() + lc.t.max())
    Zw, Zy, ybar, YY = O.raw_sums(lc.t, lc.y, lc.sigma, lc.df, js, 2 * H, H, t_ref=tref)
    plan = ftp.Plan(tmpl.c, tmpl.s, precision=ftp.FTP_FP64)
    sc, cr = plan.root_counts(np.concatenate([Zw, Zy], axis=1), tref, ybar, YY, lc.df)
    sc, cr = sc.cpu().numpy(), cr.cpu().numpy()
    ref = O.periodogram(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, lc.df, freq_index=js, block=4, return_details=True)
    oc = np.array([O.unit_circle_root_count(d["p"], tol=1e-6)[0] for d in ref["details"]])
    ok = sc >= 0
    assert np.count_nonzero(ok) >= 0.95 * len(js)
    assert np.array_equal(sc[ok], oc[ok]), (js[ok], sc[ok], oc[ok])
    assert np.array_equal(cr[ok], oc[ok])
