"""Plain CPU FP64 oracle for the fast template periodogram.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no
code with the GPU library and imports nothing from it.

It follows Hoffman, Vanderplas, Hartman & Bakos, "A Fast Template
Periodogram" (arXiv:2101.12348), Section 2, in the paper's order and
notation:

1. normalised weights, weighted mean and chi^2_0 (Section 1, Eq. ``lsp``);
2. the covariances CC, CS, SS, YC, YS of Eqs. ``CCdef``-``YSdef`` and the
   plain sums C_n, S_n, evaluated directly over the observations (no NFFT);
3. the tilde matrices and the Laurent polynomials MM and YM (Section 2, the
   expansions leading to Eq. ``finalpoly``), then MM' = psi^{2H} MM,
   YM' = psi^H YM and p = 2 MM' dYM' - YM' dMM' (Eq. ``finalpoly``);
4. the roots of p as eigenvalues of its companion matrix
   (numpy.polynomial.polynomial.polyroots, the routine the paper names);
5. every root scaled onto the unit circle and scored with
   P = YM^2 / (YY MM); theta_1 = YM/MM; theta_3 = ybar - Mbar theta_1
   (Section 2, the solution for theta_1, theta_3 and the periodogram).

Readings where the paper is silent or inexact:
* the psi^{6H-1} coefficient of p cancels identically (the leading terms of
  2 MM' dYM' and YM' dMM' are both 4H a b), so the degree is 6H-2, not the
  6H-1 stated in Section 2.3; coefficients at or below 64 eps max|p| are
  trimmed from both ends and zero roots are discarded;
* every projected root is scored, not only those already on the unit
  circle (Section 2 scores all solutions of the phase condition);
* ties (equal P within 1e-12 relative) prefer theta_1 > 0, then the smallest
  theta_2 in [0, 2 pi);
* a frequency where MM <= 1e-14 sum|alpha|^2 at every candidate (all
  phases coincide) gets P = 0, theta_1 = 0, theta_3 = ybar and flag 1;
* all sigma = 0 means uniform weights; a mix of zero and non-zero sigma, or
  Var(y) = 0, is an error (Section 2, remarks before Eq. ``simpconds``).

Phases are reduced in cycles in extended precision (numpy longdouble) before
the factor 2 pi, so the direct sums stay accurate at large k*f*t.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "weights", "moments", "harmonic_matrices", "covariances", "tilde_matrices",
    "alpha_from_template", "mm_prime", "ym_prime", "final_poly", "trim_poly",
    "poly_roots", "score_phase", "periodogram", "direct_power_at_phase",
    "template_values", "gls_power", "mhls_power", "real_trig_poly",
    "unit_circle_root_count", "raw_sums", "direct_fit_at_phase", "OracleError",
]

EPS = np.finfo(np.float64).eps
TIE_REL = 1e-12
MM_DEGENERATE = 1e-14


class OracleError(ValueError):
    pass


# -------------------------------------------------------------- Section 1

def weights(sigma) -> np.ndarray:
    """w_i proportional to sigma_i^-2 with sum w = 1 (Section 1).  All sigma = 0
    gives uniform weights; mixed zero/non-zero sigma is rejected (Section 2)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    if sigma.ndim != 1 or len(sigma) == 0:
        raise OracleError("sigma must be a non-empty vector")
    if not np.all(np.isfinite(sigma)) or np.any(sigma < 0):
        raise OracleError("sigma must be finite and non-negative")
    zero = sigma == 0
    if np.all(zero):
        return np.full(len(sigma), 1.0 / len(sigma))
    if np.any(zero):
        raise OracleError("mixed zero and non-zero sigma")
    inv = 1.0 / (sigma * sigma)
    return inv / np.sum(inv)


def moments(y, w):
    """ybar = sum w y and YY = chi^2_0 = sum w (y - ybar)^2 (Section 1)."""
    y = np.asarray(y, dtype=np.float64)
    ybar = float(np.sum(w * y))
    YY = float(np.sum(w * (y - ybar) ** 2))
    if not np.isfinite(YY) or YY <= 0.0 or np.all(y == y[0]):
        raise OracleError("Var(y) = 0: the periodogram is undefined")
    return ybar, YY


# -------------------------------------------------------------- Section 2

def _unit_phasors(t, freqs):
    """exp(i 2 pi f t) for every (observation, frequency), phase reduced in
    cycles in extended precision.  Shape (N, F)."""
    tl = np.asarray(t, dtype=np.longdouble)[:, None]
    fl = np.asarray(freqs, dtype=np.longdouble)[None, :]
    cyc = tl * fl
    cyc = cyc - np.floor(cyc)
    ang = 2.0 * np.pi * cyc.astype(np.float64)
    return np.cos(ang) + 1j * np.sin(ang)


def harmonic_matrices(t, freqs, H):
    """cos(n w t_i) and sin(n w t_i), n = 1..H, shape (F, N, H) each.
    exp(i n x) is formed as the n-th power of exp(i x) (de Moivre)."""
    e1 = _unit_phasors(t, freqs).T  # (F, N)
    out = np.empty(e1.shape + (H,), dtype=np.complex128)
    cur = np.ones_like(e1)
    for n in range(H):
        cur = cur * e1
        out[..., n] = cur
    return out.real, out.imag


def covariances(t, y, w, ybar, freqs, H):
    """Eqs. CCdef-YSdef evaluated directly over the observations, plus the
    means C_n = <cos n w t>, S_n = <sin n w t>.

    Returns dict of arrays: CC, CS, SS (F, H, H); YC, YS, C, S (F, H)."""
    cosm, sinm = harmonic_matrices(t, freqs, H)
    w = np.asarray(w, dtype=np.float64)
    yc = np.asarray(y, dtype=np.float64) - ybar
    C = np.einsum("i,fin->fn", w, cosm)
    S = np.einsum("i,fin->fn", w, sinm)
    wc = cosm * w[None, :, None]
    ws = sinm * w[None, :, None]
    CC = np.matmul(np.swapaxes(wc, 1, 2), cosm) - C[:, :, None] * C[:, None, :]
    CS = np.matmul(np.swapaxes(wc, 1, 2), sinm) - C[:, :, None] * S[:, None, :]
    SS = np.matmul(np.swapaxes(ws, 1, 2), sinm) - S[:, :, None] * S[:, None, :]
    YC = np.einsum("i,fin->fn", w * yc, cosm)
    YS = np.einsum("i,fin->fn", w * yc, sinm)
    return dict(CC=CC, CS=CS, SS=SS, YC=YC, YS=YS, C=C, S=S)


def tilde_matrices(CC, CS, SS):
    """CC~ = (CC - SS) - i(CS + CS^T); CS~ = (CC + SS) + i(CS - CS^T);
    SS~ = (CC - SS) + i(CS + CS^T)  (Section 2, after the A_n B_m products)."""
    CSt = np.swapaxes(CS, -1, -2)
    CCt_ = (CC - SS) - 1j * (CS + CSt)
    CSt_ = (CC + SS) + 1j * (CS - CSt)
    SSt_ = (CC - SS) + 1j * (CS + CSt)
    return CCt_, CSt_, SSt_


def alpha_from_template(c, s):
    """alpha_n = (c_n + i s_n)/2, n = 1..H (Section 2)."""
    return (np.asarray(c, dtype=np.float64) + 1j * np.asarray(s, dtype=np.float64)) / 2.0


def mm_prime(alpha, CCt, CSt, SSt):
    """Coefficients of MM' = psi^{2H} MM, index e <-> psi^{e}, e = 0..4H.
    MM = sum_{n,m} a_n a_m CC~_nm psi^{n+m} + 2 a_n a*_m CS~_nm psi^{n-m}
         + a*_n a*_m SS~_nm psi^{-(n+m)}."""
    H = len(alpha)
    out = np.zeros(CCt.shape[:-2] + (4 * H + 1,), dtype=np.complex128)
    for n in range(1, H + 1):
        for m in range(1, H + 1):
            an, am = alpha[n - 1], alpha[m - 1]
            out[..., 2 * H + n + m] += an * am * CCt[..., n - 1, m - 1]
            out[..., 2 * H + n - m] += 2.0 * an * np.conj(am) * CSt[..., n - 1, m - 1]
            out[..., 2 * H - n - m] += np.conj(an) * np.conj(am) * SSt[..., n - 1, m - 1]
    return out


def ym_prime(alpha, YC, YS):
    """Coefficients of YM' = psi^H YM, e = 0..2H, with
    YM = sum_k a_k YC~_k psi^k + a*_k YC~*_k psi^-k and YC~_k = YC_k - i YS_k."""
    H = len(alpha)
    out = np.zeros(YC.shape[:-1] + (2 * H + 1,), dtype=np.complex128)
    for k in range(1, H + 1):
        yct = YC[..., k - 1] - 1j * YS[..., k - 1]
        out[..., H + k] = alpha[k - 1] * yct
        out[..., H - k] = np.conj(alpha[k - 1]) * np.conj(yct)
    return out


def final_poly(MMp, YMp):
    """p = 2 MM' dYM' - YM' dMM' (Eq. finalpoly), ascending coefficients,
    6H terms of which the last vanishes identically."""
    P = np.polynomial.polynomial
    return 2.0 * P.polymul(MMp, P.polyder(YMp)) - P.polymul(YMp, P.polyder(MMp))


def trim_poly(p):
    """Drop the identically-zero psi^{6H-1} coefficient, then leading and
    trailing coefficients <= 64 eps max|p|.  Returns (coeffs, n_zero_roots)."""
    p = np.asarray(p, dtype=np.complex128)
    H6 = len(p)
    p = p[: H6 - 1]  # degree 6H-2
    scale = np.max(np.abs(p)) if len(p) else 0.0
    if scale == 0.0:
        return p[:0], 0
    tol = 64.0 * EPS * scale
    hi = len(p) - 1
    while hi >= 0 and abs(p[hi]) <= tol:
        hi -= 1
    lo = 0
    while lo <= hi and abs(p[lo]) <= tol:
        lo += 1
    return p[lo: hi + 1], lo


def poly_roots(p):
    """Roots as eigenvalues of the companion matrix (Section 2 uses
    numpy.polynomial.polyroots)."""
    if len(p) < 2:
        return np.zeros(0, dtype=np.complex128)
    return np.polynomial.polynomial.polyroots(p)


def real_trig_poly(p_full):
    """R(theta) = i e^{-i D theta/2} p(e^{i theta}) for the degree-D p
    (D = 6H-2).  p is anti-self-inversive, so R is real; returns a callable."""
    p = np.asarray(p_full, dtype=np.complex128)
    D = len(p) - 1

    def R(theta):
        th = np.asarray(theta, dtype=np.float64)[..., None]
        k = np.arange(D + 1)
        return np.real(1j * np.sum(p * np.exp(1j * (k - D / 2.0) * th), axis=-1))
    return R


def _poly_val(coef, z):
    return np.polynomial.polynomial.polyval(z, coef)


def score_phase(psi, alpha, MMp, YMp, C, S, YY, ybar):
    """For unit psi = e^{i theta_2}: YM = psi^-H YM'(psi), MM = psi^-2H MM'(psi),
    P = YM^2/(YY MM), theta_1 = YM/MM, Mbar = 2 Re sum a_n psi^n (C_n - i S_n),
    theta_3 = ybar - Mbar theta_1.  Returns (P, theta1, theta3, MM)."""
    H = len(alpha)
    YM = np.real(psi ** (-H) * _poly_val(YMp, psi))
    MM = np.real(psi ** (-2 * H) * _poly_val(MMp, psi))
    n = np.arange(1, H + 1)
    Mbar = 2.0 * np.real(np.sum(alpha * psi ** n * (C - 1j * S)))
    if MM <= MM_DEGENERATE * np.sum(np.abs(alpha) ** 2):
        return 0.0, 0.0, ybar, MM
    th1 = YM / MM
    return YM * YM / (YY * MM), th1, ybar - Mbar * th1, MM


def _best_candidate(cands):
    """cands: list of (P, theta1, theta3, theta2).  Max P; within 1e-12
    relative prefer theta_1 > 0, then the smallest theta_2."""
    Pmax = max(c[0] for c in cands)
    near = [c for c in cands if c[0] >= Pmax - TIE_REL * max(Pmax, 1e-300)]
    near.sort(key=lambda c: (0 if c[1] > 0 else 1, c[3]))
    return near[0]


def periodogram(t, y, sigma, c, s, df, n_f=None, freq_index=None, block=256,
                return_details=False, positive_amplitude=False):
    """Template periodogram at f_j = j df.  Evaluate either j = 1..n_f or the
    explicit 1-based indices ``freq_index``.  Returns dict with power, phase
    (theta_2 in [0, 2 pi), relative to t = 0), amp (theta_1), offset
    (theta_3), flag (1 = degenerate MM) and, if asked, per-frequency p and
    candidate lists.

    positive_amplitude: the fit constrained to theta_1 > 0 (Section 2.1 names
    it as a remedy for negative-amplitude solutions).  theta_1 = YM/MM with
    MM > 0, so the constraint is YM > 0; P = YM^2/(YY MM) vanishes where YM = 0,
    so the constrained maximum is attained at a stationary point inside
    {YM > 0}: the best candidate with theta_1 > 0.  With no such candidate
    (YM vanishing at every candidate) the result is P = 0, theta_1 = 0,
    theta_3 = ybar, theta_2 = 0."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if len(t) < 3 or len(y) != len(t) or len(sigma) != len(t):
        raise OracleError("need matching t, y, sigma with at least 3 points")
    if not (np.all(np.isfinite(t)) and np.all(np.isfinite(y))):
        raise OracleError("non-finite t or y")
    if not (np.isfinite(df) and df > 0):
        raise OracleError("df must be positive")
    alpha = alpha_from_template(c, s)
    H = len(alpha)
    if H < 1 or np.all(alpha == 0):
        raise OracleError("template must have H >= 1 and a non-zero coefficient")
    w = weights(sigma)
    ybar, YY = moments(y, w)
    if freq_index is None:
        if n_f is None or n_f < 1:
            raise OracleError("n_f must be >= 1")
        idx = np.arange(1, n_f + 1)
    else:
        idx = np.asarray(freq_index, dtype=np.int64)
    F = len(idx)
    out = dict(power=np.zeros(F), phase=np.zeros(F), amp=np.zeros(F),
               offset=np.zeros(F), flag=np.zeros(F, dtype=np.int8))
    details = []
    for b0 in range(0, F, block):
        jj = idx[b0: b0 + block]
        freqs = jj.astype(np.longdouble) * np.longdouble(df)
        cov = covariances(t, y, w, ybar, freqs, H)
        CCt, CSt, SSt = tilde_matrices(cov["CC"], cov["CS"], cov["SS"])
        MMp = mm_prime(alpha, CCt, CSt, SSt)
        YMp = ym_prime(alpha, cov["YC"], cov["YS"])
        for q in range(len(jj)):
            p_raw = final_poly(MMp[q], YMp[q])
            p, nzero = trim_poly(p_raw)
            if len(p) >= 2:
                roots = poly_roots(p)
                roots = roots[np.isfinite(roots) & (np.abs(roots) > 1e-8)]
            else:
                roots = np.zeros(0, dtype=np.complex128)
            psis = list(roots / np.abs(roots)) if len(roots) else []
            if not psis:
                psis = [1.0 + 0j]  # p == 0: P is constant in theta; score theta = 0
            cands = []
            allmm = []
            for psi in psis:
                P, th1, th3, MM = score_phase(psi, alpha, MMp[q], YMp[q],
                                              cov["C"][q], cov["S"][q], YY, ybar)
                th2 = float(np.angle(psi)) % (2.0 * np.pi)
                cands.append((P, th1, th3, th2))
                allmm.append(MM)
            pool = [cd for cd in cands if cd[1] > 0] if positive_amplitude else cands
            best = _best_candidate(pool) if pool else (0.0, 0.0, ybar, 0.0)
            k = b0 + q
            degenerate = max(allmm) <= MM_DEGENERATE * np.sum(np.abs(alpha) ** 2)
            if degenerate:
                out["power"][k], out["amp"][k], out["offset"][k] = 0.0, 0.0, ybar
                out["phase"][k] = 0.0
                out["flag"][k] = 1
            else:
                out["power"][k], out["amp"][k], out["offset"][k], out["phase"][k] = best
            if return_details:
                details.append(dict(p=p_raw[:-1], cands=cands, MMp=MMp[q], YMp=YMp[q]))
    out["ybar"], out["YY"] = ybar, YY
    if return_details:
        out["details"] = details
    return out


# ---------------------------------------------------- Section 2.2 multi-band

def chi2_0(y, sigma):
    """The weighted sum of squared residuals of one band about its weighted
    mean, sum (y - ybar)^2 / sigma^2 (Section 2.2); unit weights when every
    sigma is 0 (Section 2)."""
    y = np.asarray(y, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    wr = np.ones_like(y) if np.all(sigma == 0) else 1.0 / sigma ** 2
    ybar = np.sum(wr * y) / np.sum(wr)
    return float(np.sum(wr * (y - ybar) ** 2))


def multiband_periodogram(bands, c, s, df, n_f=None, freq_index=None, positive_amplitude=False):
    """Multi-phase multi-band periodogram (Section 2.2, Eq.
    multibandmultiphase): P = sum_k chi2_0,k P_k / sum_k chi2_0,k over bands
    k = 1..K, each band (t, y, sigma) with its own periodogram P_k (its own
    phase, amplitude and offset) on the common grid f_j = j df.  Returns
    (P, per-band powers (K, F), chi2_0 (K,))."""
    Pk = []
    c0 = []
    for (t, y, sig) in bands:
        r = periodogram(t, y, sig, c, s, df, n_f=n_f, freq_index=freq_index,
                        positive_amplitude=positive_amplitude)
        Pk.append(r["power"])
        c0.append(chi2_0(y, sig))
    Pk = np.array(Pk)
    c0 = np.array(c0)
    return (c0[:, None] * Pk).sum(axis=0) / c0.sum(), Pk, c0


# ------------------------------------------ Appendix A shared-phase multi-band

def shared_phase_periodogram(bands, templates, df, n_f=None, freq_index=None, offsets=None):
    """Shared-phase multi-band template periodogram (Appendix A): bands k with
    templates M^(k) (c^(k), s^(k)) share theta_1, theta_2, theta_3,
    y^(k) ~ theta_1 M^(k)(w t - theta_2) + theta_3 + lambda_k with fixed
    relative offsets lambda_k (``offsets``, subtracted first); weights
    sigma^-2 normalised over all observations (Section 2 rules).  Following
    Appendix A: psi^2H MM^ = sum_i w_i (psi^H M_i)^2 and psi^H Mbar =
    sum_i w_i psi^H M_i give MM' = psi^2H MM^ - (psi^H Mbar)^2, and
    YM' = sum_i w_i y_i psi^H M_i - ybar psi^H Mbar; then Eq. finalpoly, its
    roots and the single-band scoring with the global ybar and YY.  Templates
    with fewer harmonics are padded with zeros to the largest H.  Returns dict
    with power, phase, amp, offset, flag, ybar, YY."""
    K = len(bands)
    if K < 1 or len(templates) != K:
        raise OracleError("need one template per band")
    H = max(len(np.atleast_1d(c)) for c, _ in templates)
    alphas = np.zeros((K, H), dtype=np.complex128)
    for k, (c, sv) in enumerate(templates):
        a = alpha_from_template(c, sv)
        alphas[k, : len(a)] = a
    if np.all(alphas == 0):
        raise OracleError("templates must have a non-zero coefficient")
    lam = np.zeros(K) if offsets is None else np.asarray(offsets, dtype=np.float64)
    t_all = np.concatenate([np.asarray(b[0], dtype=np.float64) for b in bands])
    y_all = np.concatenate([np.asarray(b[1], dtype=np.float64) - lam[k] for k, b in enumerate(bands)])
    sig_all = np.concatenate([np.asarray(b[2], dtype=np.float64) for b in bands])
    band = np.concatenate([np.full(len(b[0]), k) for k, b in enumerate(bands)])
    if len(t_all) < 3 or not (np.all(np.isfinite(t_all)) and np.all(np.isfinite(y_all))):
        raise OracleError("need at least 3 finite observations")
    if not (np.isfinite(df) and df > 0):
        raise OracleError("df must be positive")
    w = weights(sig_all)
    ybar, YY = moments(y_all, w)
    A = alphas[band]                                   # (N, H) template of each observation
    scale = float(np.sum(w * np.sum(np.abs(A) ** 2, axis=1)))
    if freq_index is None:
        if n_f is None or n_f < 1:
            raise OracleError("n_f must be >= 1")
        idx = np.arange(1, n_f + 1)
    else:
        idx = np.asarray(freq_index, dtype=np.int64)
    F = len(idx)
    out = dict(power=np.zeros(F), phase=np.zeros(F), amp=np.zeros(F), offset=np.zeros(F),
               flag=np.zeros(F, dtype=np.int8))
    Pn = np.polynomial.polynomial
    for q, j in enumerate(idx):
        z = _unit_phasors(t_all, np.array([np.longdouble(j) * np.longdouble(df)]))[:, 0]   # e^{i w t}
        zn = np.empty((len(t_all), H), dtype=np.complex128)
        zn[:, 0] = z
        for n in range(1, H):
            zn[:, n] = zn[:, n - 1] * z
        # psi^H M_i(w t_i - theta): coefficient of psi^{H+n} is alpha_n e^{-i n w t},
        # of psi^{H-n} conj(alpha_n) e^{i n w t}
        Q = np.zeros((len(t_all), 2 * H + 1), dtype=np.complex128)
        Q[:, H + 1:] = A * np.conj(zn)
        Q[:, H - 1:: -1] = np.conj(A) * zn
        Mbarp = w @ Q
        MMhatp = np.zeros(4 * H + 1, dtype=np.complex128)
        for a_ in range(2 * H + 1):
            for b_ in range(2 * H + 1):
                MMhatp[a_ + b_] += np.sum(w * Q[:, a_] * Q[:, b_])
        MMp = MMhatp - Pn.polymul(Mbarp, Mbarp)
        YMp = (w * y_all) @ Q - ybar * Mbarp
        p_raw = final_poly(MMp, YMp)
        p, _ = trim_poly(p_raw)
        if len(p) >= 2:
            roots = poly_roots(p)
            roots = roots[np.isfinite(roots) & (np.abs(roots) > 1e-8)]
        else:
            roots = np.zeros(0, dtype=np.complex128)
        psis = list(roots / np.abs(roots)) if len(roots) else [1.0 + 0j]
        cands, allmm = [], []
        for psi in psis:
            YM = np.real(psi ** (-H) * Pn.polyval(psi, YMp))
            MM = np.real(psi ** (-2 * H) * Pn.polyval(psi, MMp))
            Mb = np.real(psi ** (-H) * Pn.polyval(psi, Mbarp))
            allmm.append(MM)
            if MM <= MM_DEGENERATE * scale:
                cands.append((0.0, 0.0, ybar, float(np.angle(psi)) % (2 * np.pi)))
                continue
            th1 = YM / MM
            cands.append((YM * YM / (YY * MM), th1, ybar - Mb * th1, float(np.angle(psi)) % (2 * np.pi)))
        best = _best_candidate(cands)
        if max(allmm) <= MM_DEGENERATE * scale:
            out["power"][q], out["amp"][q], out["offset"][q], out["phase"][q] = 0.0, 0.0, ybar, 0.0
            out["flag"][q] = 1
        else:
            out["power"][q], out["amp"][q], out["offset"][q], out["phase"][q] = best
    out["ybar"], out["YY"] = ybar, YY
    return out


# ----------------------------------------------------- direct definitions

def template_values(c, s, x):
    """M(x) = sum_n c_n cos(n x) + s_n sin(n x) (Section 2)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for n in range(1, len(c) + 1):
        out = out + c[n - 1] * np.cos(n * x) + s[n - 1] * np.sin(n * x)
    return out


def _cycles(t, f):
    tl = np.asarray(t, dtype=np.longdouble) * np.longdouble(f)
    return (tl - np.floor(tl)).astype(np.float64)


def direct_power_at_phase(t, y, sigma, c, s, f, theta2):
    """P = 1 - chi^2/chi^2_0 from a weighted least-squares fit of y on
    [M(w t - theta2), 1] at fixed theta2, computed from the observations
    (Section 1 definition of P; Section 2 model).  Vectorised over theta2."""
    w = weights(sigma)
    y = np.asarray(y, dtype=np.float64)
    ybar, YY = moments(y, w)
    x = 2.0 * np.pi * _cycles(t, f)
    th = np.atleast_1d(np.asarray(theta2, dtype=np.float64))
    M = template_values(c, s, x[None, :] - th[:, None])  # (T, N)
    Mbar = M @ w
    dM = M - Mbar[:, None]
    MM = (dM * dM) @ w
    YM = dM @ (w * (y - ybar))
    with np.errstate(divide="ignore", invalid="ignore"):
        P = np.where(MM > 0, YM * YM / (YY * MM), 0.0)
    return P if np.ndim(theta2) else P[0]


def _wls_power(t, y, sigma, f, H):
    w = weights(sigma)
    y = np.asarray(y, dtype=np.float64)
    ybar, YY = moments(y, w)
    x = 2.0 * np.pi * _cycles(t, f)
    cols = [np.ones_like(x)]
    for n in range(1, H + 1):
        cols += [np.cos(n * x), np.sin(n * x)]
    A = np.stack(cols, axis=1)
    sw = np.sqrt(w)
    coef, *_ = np.linalg.lstsq(A * sw[:, None], y * sw, rcond=None)
    r = y - A @ coef
    chi2 = float(np.sum(w * r * r))
    return 1.0 - chi2 / YY


def gls_power(t, y, sigma, f):
    """Floating-mean Lomb-Scargle power: weighted linear least squares of y on
    [1, cos w t, sin w t] (the H = 1 model of Section 1)."""
    return _wls_power(t, y, sigma, f, 1)


def mhls_power(t, y, sigma, f, H):
    """Multi-harmonic LS power with 2H+1 free parameters (Section 1, MHLS)."""
    return _wls_power(t, y, sigma, f, H)


def unit_circle_root_count(p_full, tol=1e-6):
    """Number of companion eigenvalues of the trimmed p with ||psi| - 1| < tol,
    and the minimum distance of the other roots from the circle."""
    p, _ = trim_poly(np.concatenate([p_full, [0.0]]))
    r = poly_roots(p)
    d = np.abs(np.abs(r) - 1.0)
    on = d < tol
    off = d[~on]
    return int(np.sum(on)), (float(np.min(off)) if len(off) else np.inf), r


def raw_sums(t, y, sigma, df, freq_index, kmax_w, kmax_y, t_ref=0.0):
    """The raw trig sums behind Eqs. CCdef-YSdef, by direct summation:
    Zw[q, k-1] = sum_i w_i exp(2 pi i k j_q df (t_i - t_ref)), k = 1..kmax_w;
    Zy[q, k-1] = sum_i w_i (y_i - ybar) exp(...), k = 1..kmax_y.
    Phases are reduced in cycles in extended precision.  Returns (Zw, Zy,
    ybar, YY)."""
    w = weights(sigma)
    y = np.asarray(y, dtype=np.float64)
    ybar, YY = moments(y, w)
    d = np.asarray(t, dtype=np.longdouble) - np.longdouble(t_ref)
    js = np.asarray(freq_index, dtype=np.int64)
    Zw = np.empty((len(js), kmax_w), dtype=np.complex128)
    Zy = np.empty((len(js), kmax_y), dtype=np.complex128)
    gy = w * (y - ybar)
    for q, j in enumerate(js):
        for k in range(1, max(kmax_w, kmax_y) + 1):
            cyc = d * (np.longdouble(k * int(j)) * np.longdouble(df))
            cyc = (cyc - np.floor(cyc)).astype(np.float64)
            e = np.exp(2j * np.pi * cyc)
            if k <= kmax_w:
                Zw[q, k - 1] = np.sum(w * e)
            if k <= kmax_y:
                Zy[q, k - 1] = np.sum(gy * e)
    return Zw, Zy, ybar, YY


def direct_fit_at_phase(t, y, sigma, c, s, f, theta2):
    """Weighted least squares of y on [M(w t - theta2), 1] at a fixed phase,
    from the observations: returns (P, theta_1, theta_3) (Section 2)."""
    w = weights(sigma)
    y = np.asarray(y, dtype=np.float64)
    ybar, YY = moments(y, w)
    x = 2.0 * np.pi * _cycles(t, f)
    M = template_values(c, s, x - theta2)
    Mbar = np.sum(w * M)
    MM = np.sum(w * (M - Mbar) ** 2)
    YM = np.sum(w * (M - Mbar) * (y - ybar))
    if MM <= 0:
        return 0.0, 0.0, ybar
    th1 = YM / MM
    return YM * YM / (YY * MM), th1, ybar - Mbar * th1
