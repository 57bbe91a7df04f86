"""Pins for the CPU FP64 oracle against facts fixed by the paper and by the
mathematics, independent of the oracle's own formulas.

* H = 1 reduces to the floating-mean Lomb-Scargle power (weighted linear
  least squares on [1, cos, sin]; Section 1 model, Section 2 template).
* 0 <= P <= 1 (Cauchy-Schwarz) and P_FTP(H) <= P_MHLS(H) (nested models).
* a noiseless injected template gives P = 1 and recovers theta (Section 2).
* invariances of P = (chi2_0 - chi2)/chi2_0 (Section 1 definition).
* brute force over a dense theta_2 grid with observation-level P.
* the polynomial pieces agree with observation-level MM(theta), YM(theta)
  and with R(theta) = 2 MM dYM/dtheta - YM dMM/dtheta (Eq. theta2cond).
"""
import math

import numpy as np
import pytest

from oracle import ftp_oracle as O
from synthetic import tiny_case, small_fp64_case, eval_template, Template


def _run(tmpl, lc, **kw):
    return O.periodogram(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, lc.df, lc.n_f, **kw)


@pytest.mark.parametrize("seed", range(4))
def test_h1_equals_floating_mean_lomb_scargle(seed):
    tmpl, lc = tiny_case(seed, n_obs=60, H=1, n_f=40)
    r = _run(tmpl, lc)
    gls = np.array([O.gls_power(lc.t, lc.y, lc.sigma, j * lc.df) for j in range(1, lc.n_f + 1)])
    assert np.max(np.abs(r["power"] - gls)) < 1e-12


@pytest.mark.parametrize("seed,H", [(0, 2), (1, 3), (2, 4), (3, 6)])
def test_bounds_and_mhls(seed, H):
    tmpl, lc = tiny_case(seed, n_obs=70, H=H, n_f=40, cadence="nightly")
    r = _run(tmpl, lc)
    P = r["power"]
    assert np.all(P >= 0.0) and np.all(P <= 1.0 + 1e-13)
    mh = np.array([O.mhls_power(lc.t, lc.y, lc.sigma, j * lc.df, H) for j in range(1, lc.n_f + 1)])
    assert np.all(P <= mh + 1e-12)


@pytest.mark.parametrize("seed,H", [(0, 1), (1, 3), (2, 5)])
def test_noiseless_injection_recovers_parameters(seed, H):
    rng = np.random.default_rng(100 + seed)
    tm = Template(rng.standard_normal(H), rng.standard_normal(H))
    t = np.sort(rng.uniform(0, 20, 80))
    df = 1.0 / (5 * (t.max() - t.min()))
    j0 = 37
    f0 = j0 * df
    A, phi, B = 1.7, 2.1, -0.4
    y = A * eval_template(tm, 2 * np.pi * f0 * t - phi) + B
    sigma = rng.uniform(0.5, 2.0, len(t))
    r = O.periodogram(t, y, sigma, tm.c, tm.s, df, freq_index=[j0])
    assert abs(r["power"][0] - 1.0) < 1e-10
    if H == 1:
        # M(x + pi) = -M(x): (phi, A) and (phi + pi, -A) tie; the tie rule picks A > 0
        pass
    assert abs(r["amp"][0] - A) < 1e-8
    d = (r["phase"][0] - phi + np.pi) % (2 * np.pi) - np.pi
    assert abs(d) < 1e-8
    assert abs(r["offset"][0] - B) < 1e-8


def test_negative_amplitude_and_tie_rule():
    # H=1: the sign flip with a pi shift gives an exact tie; theta1 > 0 wins.
    rng = np.random.default_rng(7)
    tm = Template(np.array([0.3]), np.array([1.1]))
    t = np.sort(rng.uniform(0, 10, 50))
    df = 1.0 / (5 * (t.max() - t.min()))
    y = -2.0 * eval_template(tm, 2 * np.pi * 20 * df * t - 0.5) + 0.01 * rng.standard_normal(50)
    r = O.periodogram(t, y, np.ones(50), tm.c, tm.s, df, freq_index=[20])
    assert r["amp"][0] > 0
    # a template with no such symmetry keeps the negative amplitude (Section 2.1 default)
    tm2 = Template(np.array([1.0, 0.6, 0.3]), np.array([0.0, 0.5, -0.4]))
    y2 = -1.5 * eval_template(tm2, 2 * np.pi * 20 * df * t - 0.5)
    r2 = O.periodogram(t, y2, np.ones(50), tm2.c, tm2.s, df, freq_index=[20])
    assert abs(r2["power"][0] - 1.0) < 1e-10 and abs(r2["amp"][0] + 1.5) < 1e-8


@pytest.mark.parametrize("seed,H", [(0, 1), (1, 2), (2, 3), (3, 4)])
def test_brute_force_theta_grid(seed, H):
    tmpl, lc = tiny_case(seed, n_obs=45, H=H, n_f=25)
    r = _run(tmpl, lc)
    th = np.linspace(0.0, 2 * np.pi, 100_001)[:-1]
    dth = th[1] - th[0]
    for j in range(1, lc.n_f + 1):
        f = j * lc.df
        Pg = O.direct_power_at_phase(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, f, th)
        k = int(np.argmax(Pg))
        # golden-section refinement of the grid maximum
        a, b = th[k] - dth, th[k] + dth
        g = (math.sqrt(5) - 1) / 2
        for _ in range(60):
            c1, c2 = b - g * (b - a), a + g * (b - a)
            if O.direct_power_at_phase(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, f, c1) > \
               O.direct_power_at_phase(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, f, c2):
                b = c2
            else:
                a = c1
        Pref = O.direct_power_at_phase(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, f, 0.5 * (a + b))
        Pc = r["power"][j - 1]
        assert Pc >= Pg.max() - 1e-13
        assert abs(Pc - max(Pref, Pg.max())) < 1e-10
        # the reported phase reproduces the reported power at observation level
        Pd = O.direct_power_at_phase(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, f, r["phase"][j - 1])
        assert abs(Pd - Pc) < 1e-12


def test_invariances():
    tmpl, lc = tiny_case(11, n_obs=55, H=3, n_f=30, cadence="nightly")
    base = _run(tmpl, lc)
    P0 = base["power"]
    # time shift: P unchanged, theta2 shifts by w * dt
    dt = 3.25
    sh = O.periodogram(lc.t + dt, lc.y, lc.sigma, tmpl.c, tmpl.s, lc.df, lc.n_f)
    assert np.max(np.abs(sh["power"] - P0)) < 1e-11
    w = 2 * np.pi * lc.df * np.arange(1, lc.n_f + 1)
    d = (sh["phase"] - base["phase"] - w * dt + np.pi) % (2 * np.pi) - np.pi
    good = P0 > 1e-6
    assert np.max(np.abs(d[good])) < 1e-7
    # affine y, sigma scale, template scale
    r = O.periodogram(lc.t, -3.0 * lc.y + 7.0, 2.5 * lc.sigma, 4.0 * tmpl.c, 4.0 * tmpl.s, lc.df, lc.n_f)
    assert np.max(np.abs(r["power"] - P0)) < 1e-11
    # template shift M(x) -> M(x - phi): P unchanged
    phi = 0.7
    n = np.arange(1, 4)
    # M(x - phi) = sum c_n cos(n x - n phi) + s_n sin(n x - n phi)
    c2 = tmpl.c * np.cos(n * phi) - tmpl.s * np.sin(n * phi)
    s2 = tmpl.s * np.cos(n * phi) + tmpl.c * np.sin(n * phi)
    r = O.periodogram(lc.t, lc.y, lc.sigma, c2, s2, lc.df, lc.n_f)
    assert np.max(np.abs(r["power"] - P0)) < 1e-11
    # permutation of observations
    perm = np.random.default_rng(0).permutation(len(lc.t))
    r = O.periodogram(lc.t[perm], lc.y[perm], lc.sigma[perm], tmpl.c, tmpl.s, lc.df, lc.n_f)
    assert np.max(np.abs(r["power"] - P0)) < 1e-12
    # duplicating an observation == halving its variance
    i = 5
    t2 = np.append(lc.t, lc.t[i]); y2 = np.append(lc.y, lc.y[i]); s2_ = np.append(lc.sigma, lc.sigma[i])
    s3 = lc.sigma.copy(); s3[i] = lc.sigma[i] / np.sqrt(2.0)
    ra = O.periodogram(t2, y2, s2_, tmpl.c, tmpl.s, lc.df, lc.n_f)
    rb = O.periodogram(lc.t, lc.y, s3, tmpl.c, tmpl.s, lc.df, lc.n_f)
    assert np.max(np.abs(ra["power"] - rb["power"])) < 1e-12


def test_covariances_against_scalar_loops():
    tmpl, lc = tiny_case(3, n_obs=12, H=3, n_f=4)
    w = O.weights(lc.sigma)
    ybar, YY = O.moments(lc.y, w)
    freqs = np.array([2, 3], dtype=np.float64) * lc.df
    cov = O.covariances(lc.t, lc.y, w, ybar, freqs, 3)
    for q, f in enumerate(freqs):
        x = [2 * math.pi * f * ti for ti in lc.t]
        for n in range(1, 4):
            Cn = math.fsum(wi * math.cos(n * xi) for wi, xi in zip(w, x))
            Sn = math.fsum(wi * math.sin(n * xi) for wi, xi in zip(w, x))
            assert abs(cov["C"][q, n - 1] - Cn) < 1e-12 and abs(cov["S"][q, n - 1] - Sn) < 1e-12
            YCn = math.fsum(wi * (yi - ybar) * math.cos(n * xi) for wi, yi, xi in zip(w, lc.y, x))
            assert abs(cov["YC"][q, n - 1] - YCn) < 1e-12
            for m in range(1, 4):
                Cm = math.fsum(wi * math.cos(m * xi) for wi, xi in zip(w, x))
                Sm = math.fsum(wi * math.sin(m * xi) for wi, xi in zip(w, x))
                cc = math.fsum(wi * math.cos(n * xi) * math.cos(m * xi) for wi, xi in zip(w, x)) - Cn * Cm
                cs = math.fsum(wi * math.cos(n * xi) * math.sin(m * xi) for wi, xi in zip(w, x)) - Cn * Sm
                ss = math.fsum(wi * math.sin(n * xi) * math.sin(m * xi) for wi, xi in zip(w, x)) - Sn * Sm
                assert abs(cov["CC"][q, n - 1, m - 1] - cc) < 1e-12
                assert abs(cov["CS"][q, n - 1, m - 1] - cs) < 1e-12
                assert abs(cov["SS"][q, n - 1, m - 1] - ss) < 1e-12


@pytest.mark.parametrize("H", [1, 2, 4, 6])
def test_polynomial_matches_observation_level_definitions(H):
    tmpl, lc = tiny_case(20 + H, n_obs=50, H=H, n_f=10, cadence="nightly")
    w = O.weights(lc.sigma)
    ybar, YY = O.moments(lc.y, w)
    f = 7 * lc.df
    cov = O.covariances(lc.t, lc.y, w, ybar, np.array([f]), H)
    CCt, CSt, SSt = O.tilde_matrices(cov["CC"], cov["CS"], cov["SS"])
    alpha = O.alpha_from_template(tmpl.c, tmpl.s)
    MMp = O.mm_prime(alpha, CCt, CSt, SSt)[0]
    YMp = O.ym_prime(alpha, cov["YC"], cov["YS"])[0]
    p = O.final_poly(MMp, YMp)
    # leading psi^{6H-1} coefficient cancels identically
    assert abs(p[-1]) < 1e-14 * np.max(np.abs(p))
    pD = p[:-1]
    # anti-self-inversive: p_k = -conj(p_{D-k})
    assert np.max(np.abs(pD + np.conj(pD[::-1]))) < 1e-13 * np.max(np.abs(pD))
    x = 2 * np.pi * np.array([float((np.longdouble(ti) * np.longdouble(f)) % 1) for ti in lc.t])

    def direct(theta):
        M = O.template_values(tmpl.c, tmpl.s, x - theta)
        Mb = np.sum(w * M)
        MM = np.sum(w * (M - Mb) ** 2)
        YM = np.sum(w * (M - Mb) * (lc.y - ybar))
        return MM, YM

    R = O.real_trig_poly(pD)
    for theta in np.linspace(0.1, 6.0, 7):
        psi = np.exp(1j * theta)
        MMd, YMd = direct(theta)
        MMa = np.real(psi ** (-2 * H) * np.polynomial.polynomial.polyval(psi, MMp))
        YMa = np.real(psi ** (-H) * np.polynomial.polynomial.polyval(psi, YMp))
        assert abs(MMa - MMd) < 1e-12 and abs(YMa - YMd) < 1e-12
        h = 1e-5
        MMp_, YMp_ = direct(theta + h)
        MMm_, YMm_ = direct(theta - h)
        dMM = (MMp_ - MMm_) / (2 * h)
        dYM = (YMp_ - YMm_) / (2 * h)
        Rd = 2 * MMd * dYM - YMd * dMM
        assert abs(R(theta) - Rd) < 1e-7 * max(1.0, abs(Rd))


def test_degenerate_and_error_inputs():
    rng = np.random.default_rng(5)
    tm = Template(np.array([1.0, 0.3]), np.array([0.2, -0.5]))
    # strictly periodic sampling (t integer days): at f = 1/day all phases coincide
    t = np.arange(40, dtype=np.float64)
    y = rng.standard_normal(40)
    df = 1.0 / 200.0
    r = O.periodogram(t, y, np.ones(40), tm.c, tm.s, df, freq_index=[200, 37])
    assert r["flag"][0] == 1 and r["power"][0] == 0.0 and r["amp"][0] == 0.0
    assert abs(r["offset"][0] - np.mean(y)) < 1e-12
    assert r["flag"][1] == 0 and r["power"][1] > 0
    # all sigma = 0 -> uniform weights
    ra = O.periodogram(t + 0.1 * rng.random(40), y, np.zeros(40), tm.c, tm.s, df, 20)
    rb = O.periodogram(t + 0.1 * rng.random(40) * 0, y, np.ones(40), tm.c, tm.s, df, 20)
    assert np.all(np.isfinite(ra["power"])) and np.all(np.isfinite(rb["power"]))
    with pytest.raises(O.OracleError):
        O.periodogram(t, y, np.r_[0.0, np.ones(39)], tm.c, tm.s, df, 5)
    with pytest.raises(O.OracleError):
        O.periodogram(t, np.ones(40), np.ones(40), tm.c, tm.s, df, 5)
    with pytest.raises(O.OracleError):
        O.periodogram(t, y, -np.ones(40), tm.c, tm.s, df, 5)
    with pytest.raises(O.OracleError):
        O.periodogram(t, y, np.ones(40), tm.c, tm.s, -1.0, 5)


def test_small_fp64_workload_peak():
    tmpl, lc = small_fp64_case()
    r = _run(tmpl, lc)
    j = int(np.argmax(r["power"])) + 1
    assert abs(j * lc.df - 1 / 0.7) <= lc.df
    assert r["power"][j - 1] > 0.95
    assert abs(r["amp"][j - 1] - 1.0) < 0.05


def test_raw_sums_agree_with_covariance_means():
    # Z_w(k) at t_ref = 0 must equal C_k + i S_k of the covariance path, and
    # Z_y(k) must equal YC_k + i YS_k (two independent evaluations).
    tmpl, lc = tiny_case(9, n_obs=30, H=3, n_f=6)
    js = np.array([1, 4, 6])
    Zw, Zy, ybar, YY = O.raw_sums(lc.t, lc.y, lc.sigma, lc.df, js, 3, 3)
    w = O.weights(lc.sigma)
    cov = O.covariances(lc.t, lc.y, w, ybar, js * lc.df, 3)
    assert np.max(np.abs(Zw - (cov["C"] + 1j * cov["S"]))) < 1e-13
    assert np.max(np.abs(Zy - (cov["YC"] + 1j * cov["YS"]))) < 1e-13
    # shifting t_ref multiplies Z(m) by exp(2 pi i m df t_ref)
    Zw2, _, _, _ = O.raw_sums(lc.t, lc.y, lc.sigma, lc.df, js, 3, 1, t_ref=1.7)
    k = np.arange(1, 4)[None, :]
    ph = np.exp(2j * np.pi * (k * js[:, None] * lc.df * 1.7))
    assert np.max(np.abs(Zw2 * ph - Zw)) < 1e-12


def test_direct_fit_at_phase_matches_candidate():
    tmpl, lc = tiny_case(4, n_obs=50, H=3, n_f=12)
    r = _run(tmpl, lc)
    for j in (3, 8, 12):
        P, a, b = O.direct_fit_at_phase(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, j * lc.df, r["phase"][j - 1])
        assert abs(P - r["power"][j - 1]) < 1e-12
        assert abs(a - r["amp"][j - 1]) < 1e-9 * max(1, abs(a))
        assert abs(b - r["offset"][j - 1]) < 1e-9 * max(1, abs(b))


def _constrained_grid_max(lc, tmpl, f, th):
    """max over theta_2 on the grid of observation-level P restricted to a
    positive least-squares amplitude: P = Cov_w(y, M)^2 / (Var_w(y) Var_w(M)),
    the amplitude's sign being that of Cov_w(y, M) (weighted least squares on
    [M, 1], Section 1 definition of P)."""
    w = 1.0 / lc.sigma ** 2
    w = w / w.sum()
    yc = lc.y - np.dot(w, lc.y)
    M = O.template_values(tmpl.c, tmpl.s, 2 * np.pi * f * lc.t[None, :] - th[:, None])
    Mc = M - (M @ w)[:, None]
    cov = Mc @ (w * yc)
    var = (Mc ** 2) @ w
    P = cov ** 2 / (var * np.dot(w, yc ** 2))
    P = np.where(cov > 0, P, -1.0)
    return P.max()


@pytest.mark.parametrize("seed,H", [(4, 2), (5, 3), (6, 5)])
def test_positive_amplitude_brute_force(seed, H):
    """The theta_1 > 0 variant (Section 2.1's constrained remedy) against a
    dense theta_2 grid restricted to positive amplitudes; it never exceeds
    the unconstrained power and reports a positive amplitude."""
    tmpl, lc = tiny_case(seed, n_obs=45, H=H, n_f=25)
    r = _run(tmpl, lc, positive_amplitude=True)
    u = _run(tmpl, lc)
    th = np.linspace(0.0, 2 * np.pi, 40_001)[:-1]
    for j in range(1, lc.n_f + 1):
        f = j * lc.df
        Pg = _constrained_grid_max(lc, tmpl, f, th)
        Pc = r["power"][j - 1]
        assert Pc <= u["power"][j - 1] + 1e-15
        assert Pc >= Pg - 1e-13
        assert Pc - Pg < 1e-5   # grid step 1.6e-4 rad
        assert r["amp"][j - 1] > 0
        Pd, a, _ = O.direct_fit_at_phase(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, f, r["phase"][j - 1])
        assert a > 0 and abs(Pd - Pc) < 1e-12


def test_positive_amplitude_on_a_flipped_signal():
    """A noiseless flipped copy of an asymmetric template: unconstrained,
    theta_1 = -1.5 and P = 1; constrained to theta_1 > 0, P < 1."""
    rng = np.random.default_rng(9)
    tm = Template(np.array([1.0, 0.6, 0.3]), np.array([0.0, 0.5, -0.4]))
    t = np.sort(rng.uniform(0, 10, 60))
    df = 1.0 / (5 * (t.max() - t.min()))
    y = -1.5 * eval_template(tm, 2 * np.pi * 20 * df * t - 0.5)
    u = O.periodogram(t, y, np.ones(60), tm.c, tm.s, df, freq_index=[20])
    p = O.periodogram(t, y, np.ones(60), tm.c, tm.s, df, freq_index=[20], positive_amplitude=True)
    assert abs(u["power"][0] - 1.0) < 1e-10 and u["amp"][0] < 0
    assert p["amp"][0] > 0 and p["power"][0] < 0.99


def _band(seed, n, tmpl, f0, amp, phase):
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(0, 12, n))
    sig = rng.uniform(0.3, 1.0, n)
    y = amp * eval_template(tmpl, 2 * np.pi * f0 * t - phase) + 0.7 + sig * rng.standard_normal(n)
    return t, y, sig


def test_multiband_against_per_band_least_squares():
    """Multi-phase multi-band power (Section 2.2) against its definition:
    every band fitted on its own (amplitude, phase, offset) by brute force
    over theta_2, P = 1 - sum_k chi2_k / sum_k chi2_0,k with chi2 summed over
    the residuals directly."""
    tm = Template(np.array([1.0, 0.4]), np.array([0.2, -0.3]))
    df = 1.0 / 60.0
    bands = [_band(30, 40, tm, 9 * df, 1.0, 0.4), _band(31, 35, tm, 9 * df, 0.6, 1.1),
             _band(32, 50, tm, 9 * df, 0.3, 2.0)]
    js = np.array([3, 9, 14])
    P, Pk, c0 = O.multiband_periodogram(bands, tm.c, tm.s, df, freq_index=js)
    th = np.linspace(0.0, 2 * np.pi, 20_001)[:-1]
    dth = th[1] - th[0]
    g = (math.sqrt(5) - 1) / 2
    for q, j in enumerate(js):
        f = j * df
        chi_fit, chi_0 = 0.0, 0.0
        for (t, y, sig) in bands:
            Pg = O.direct_power_at_phase(t, y, sig, tm.c, tm.s, f, th)
            k = int(np.argmax(Pg))
            a, b = th[k] - dth, th[k] + dth
            for _ in range(60):
                x1, x2 = b - g * (b - a), a + g * (b - a)
                if O.direct_power_at_phase(t, y, sig, tm.c, tm.s, f, x1) > \
                   O.direct_power_at_phase(t, y, sig, tm.c, tm.s, f, x2):
                    b = x2
                else:
                    a = x1
            _, amp, off = O.direct_fit_at_phase(t, y, sig, tm.c, tm.s, f, 0.5 * (a + b))
            model = amp * O.template_values(tm.c, tm.s, 2 * np.pi * f * t - 0.5 * (a + b)) + off
            chi_fit += np.sum((y - model) ** 2 / sig ** 2)
            ybar = np.sum(y / sig ** 2) / np.sum(1 / sig ** 2)
            chi_0 += np.sum((y - ybar) ** 2 / sig ** 2)
        assert abs(P[q] - (1.0 - chi_fit / chi_0)) < 1e-9


def test_multiband_special_cases():
    """One band is the single-band periodogram; identical bands give it too."""
    tm = Template(np.array([0.8, 0.1, 0.3]), np.array([0.0, 0.5, -0.2]))
    df = 1.0 / 60.0
    b = _band(33, 45, tm, 11 * df, 0.9, 0.3)
    P1, _, _ = O.multiband_periodogram([b], tm.c, tm.s, df, n_f=20)
    r = O.periodogram(*b, tm.c, tm.s, df, 20)
    assert np.max(np.abs(P1 - r["power"])) < 1e-15
    P3, Pk, c0 = O.multiband_periodogram([b, b, b], tm.c, tm.s, df, n_f=20)
    assert np.max(np.abs(P3 - r["power"])) < 1e-15 and np.allclose(c0, c0[0])


def _sp_bands(seed, ns, templates, f0, A, phi, B, lam, noise=0.3):
    rng = np.random.default_rng(seed)
    out = []
    for k, n in enumerate(ns):
        t = np.sort(rng.uniform(0, 12, n))
        sig = rng.uniform(0.2, 0.6, n) * noise / 0.3
        y = A * eval_template(templates[k], 2 * np.pi * f0 * t - phi) + B + lam[k] + sig * rng.standard_normal(n)
        out.append((t, y, sig))
    return out


def _sp_direct(bands, templates, lam, f, th):
    """Observation-level P(theta_2) of the shared-phase model: the weighted
    correlation of y - lambda with the per-observation template, weights
    sigma^-2 normalised over all bands (Appendix A)."""
    w = np.concatenate([1.0 / b[2] ** 2 for b in bands])
    w = w / w.sum()
    y = np.concatenate([b[1] - lam[k] for k, b in enumerate(bands)])
    M = np.concatenate([O.template_values(templates[k].c, templates[k].s,
                                          2 * np.pi * f * b[0][None, :] - np.atleast_1d(th)[:, None])
                        for k, b in enumerate(bands)], axis=1)
    yc = y - np.dot(w, y)
    Mc = M - (M @ w)[:, None]
    cov = Mc @ (w * yc)
    return cov ** 2 / (((Mc ** 2) @ w) * np.dot(w, yc ** 2)), cov / ((Mc ** 2) @ w)


def test_shared_phase_brute_force():
    """Shared-phase multi-band (Appendix A) against a dense theta_2 grid of the
    observation-level definition with per-band templates and offsets."""
    tms = [Template(np.array([1.0, 0.4, 0.1]), np.array([0.2, -0.3, 0.2])),
           Template(np.array([0.7, 0.5]), np.array([-0.1, 0.3])),
           Template(np.array([1.2, 0.2, -0.2]), np.array([0.0, 0.1, 0.3]))]
    df = 1.0 / 60.0
    lam = np.array([0.0, 0.8, -0.5])
    bands = _sp_bands(50, (40, 30, 45), tms, 9 * df, 1.3, 0.7, 0.2, lam)
    js = np.array([2, 9, 13, 21])
    r = O.shared_phase_periodogram(bands, [(tm.c, tm.s) for tm in tms], df, freq_index=js, offsets=lam)
    th = np.linspace(0.0, 2 * np.pi, 20_001)[:-1]
    dth = th[1] - th[0]
    g = (math.sqrt(5) - 1) / 2
    for q, j in enumerate(js):
        f = j * df
        Pg, _ = _sp_direct(bands, tms, lam, f, th)
        k = int(np.argmax(Pg))
        a, b = th[k] - dth, th[k] + dth
        for _ in range(60):
            x1, x2 = b - g * (b - a), a + g * (b - a)
            if _sp_direct(bands, tms, lam, f, x1)[0][0] > _sp_direct(bands, tms, lam, f, x2)[0][0]:
                b = x2
            else:
                a = x1
        Pref = _sp_direct(bands, tms, lam, f, 0.5 * (a + b))[0][0]
        assert r["power"][q] >= Pg.max() - 1e-13
        assert abs(r["power"][q] - max(Pref, Pg.max())) < 1e-10
        Pd, amp = _sp_direct(bands, tms, lam, f, r["phase"][q])
        assert abs(Pd[0] - r["power"][q]) < 1e-12 and abs(amp[0] - r["amp"][q]) < 1e-9 * max(1, abs(amp[0]))


def test_shared_phase_special_cases():
    """One band, or bands sharing one template with no offsets, reduce to the
    single-band periodogram of the (concatenated) data; relative offsets
    given back through ``offsets`` cancel."""
    tm = Template(np.array([0.8, 0.1, 0.3]), np.array([0.0, 0.5, -0.2]))
    df = 1.0 / 60.0
    bands = _sp_bands(51, (40, 35), [tm, tm], 11 * df, 0.9, 0.3, 0.1, [0.0, 0.0])
    r1 = O.shared_phase_periodogram(bands[:1], [(tm.c, tm.s)], df, n_f=20)
    s1 = O.periodogram(*bands[0], tm.c, tm.s, df, 20)
    assert np.max(np.abs(r1["power"] - s1["power"])) < 1e-12
    cat = tuple(np.concatenate([b[i] for b in bands]) for i in range(3))
    r2 = O.shared_phase_periodogram(bands, [(tm.c, tm.s)] * 2, df, n_f=20)
    s2 = O.periodogram(*cat, tm.c, tm.s, df, 20)
    assert np.max(np.abs(r2["power"] - s2["power"])) < 1e-12
    assert np.max(np.abs(r2["amp"] - s2["amp"])) < 1e-9 and np.max(np.abs(r2["offset"] - s2["offset"])) < 1e-9
    lam = np.array([0.4, -1.1])
    shifted = [(b[0], b[1] + lam[k], b[2]) for k, b in enumerate(bands)]
    r3 = O.shared_phase_periodogram(shifted, [(tm.c, tm.s)] * 2, df, n_f=20, offsets=lam)
    assert np.max(np.abs(r3["power"] - r2["power"])) < 1e-12


@pytest.mark.parametrize("seed", range(3))
def test_unit_circle_root_count_on_constructed_roots(seed):
    """Roots placed by hand: m on the unit circle, the rest in pairs psi,
    1/conj(psi) off it (the root structure of an anti-self-inversive p,
    Section 2 after Eq. finalpoly).  The count must be m and the distance of
    the nearest off-circle root must be the one placed."""
    rng = np.random.default_rng(300 + seed)
    m = 2 * int(rng.integers(1, 6))
    on = np.exp(1j * np.sort(rng.uniform(0, 2 * np.pi, m)))
    radii = rng.uniform(1.05, 3.0, 4)
    phis = rng.uniform(0, 2 * np.pi, 4)
    off = np.concatenate([radii * np.exp(1j * phis), np.exp(1j * phis) / radii])
    p = np.polynomial.polynomial.polyfromroots(np.concatenate([on, off]))
    cnt, dmin, _ = O.unit_circle_root_count(p, tol=1e-6)
    assert cnt == m
    expect = np.min(np.minimum(radii - 1.0, 1.0 - 1.0 / radii))
    assert abs(dmin - expect) < 1e-8


@pytest.mark.parametrize("seed,H", [(0, 2), (1, 3), (2, 4)])
def test_unit_circle_root_count_equals_sign_changes_of_R(seed, H):
    """On the method's own polynomials the unit-circle roots are the real
    zeros of R(theta) = i e^{-i D theta / 2} p(e^{i theta}) (Eq. theta2cond):
    their number equals the sign changes of the observation-level
    R(theta) = 2 MM dYM/dtheta - YM dMM/dtheta on a dense theta grid."""
    tmpl, lc = tiny_case(seed, n_obs=50, H=H, n_f=12, cadence="nightly")
    js = [3, 7, 11]
    r = O.periodogram(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, lc.df, freq_index=js, return_details=True)
    w = O.weights(lc.sigma)
    ybar, _ = O.moments(lc.y, w)
    th = np.linspace(0.0, 2 * np.pi, 60_001)[:-1]
    h = 1e-6
    for q, j in enumerate(js):
        x = 2 * np.pi * j * lc.df * lc.t

        def mm_ym(theta):
            M = O.template_values(tmpl.c, tmpl.s, x[None, :] - theta[:, None])
            Mc = M - np.sum(w * M, axis=1, keepdims=True)
            return np.sum(w * Mc * Mc, axis=1), np.sum(w * Mc * (lc.y - ybar), axis=1)

        MM, YM = mm_ym(th)
        MMp, YMp = mm_ym(th + h)
        MMm, YMm = mm_ym(th - h)
        R = 2 * MM * (YMp - YMm) / (2 * h) - YM * (MMp - MMm) / (2 * h)
        changes = int(np.sum(np.sign(R) != np.sign(np.roll(R, 1))))
        cnt, _, _ = O.unit_circle_root_count(r["details"][q]["p"], tol=1e-6)
        assert cnt == changes
