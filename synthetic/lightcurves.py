"""Seeded synthetic workloads for the fast template periodogram.

Every generator is driven by ``numpy.random.default_rng`` with an explicit
seed; batch members derive their stream from ``(seed, index)``.  Shapes and
distributions follow the workloads the method is meant for: irregular
survey cadences (nightly windows with dropped nights and observing seasons),
heteroscedastic Gaussian noise, and templates given by truncated Fourier
series M(x) = sum_n c_n cos(n x) + s_n sin(n x), n = 1..H (the paper's
template definition, Section 2).  The paper's own simulated data (uniform
times, homoskedastic noise, an eclipsing-binary template fitted to a HATNet
star) is not available, so these recipes stand in for it.

Nothing here computes sums, covariances, polynomials or powers.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED0 = 20210129

__all__ = [
    "SEED0", "Template", "LightCurve", "Batch",
    "template_random_normal", "template_sawtooth", "template_eclipsing_binary",
    "eval_template", "cadence_uniform", "cadence_nightly",
    "frequency_grid", "small_fp64_case", "single_long_case", "ragged_batch_case",
    "learned_train_lightcurves", "learned_heldout_lightcurves", "large_case", "single_long_template",
    "large_template", "large_train_lightcurves", "large_heldout_lightcurves",
    "learned_template", "h_sweep_case", "multiband_case", "shared_phase_case",
    "tiny_case", "WORKLOADS",
]


@dataclass
class Template:
    """Truncated Fourier template: c[n-1], s[n-1] for n = 1..H."""
    c: np.ndarray
    s: np.ndarray

    @property
    def H(self) -> int:
        return int(len(self.c))


@dataclass
class LightCurve:
    t: np.ndarray
    y: np.ndarray
    sigma: np.ndarray
    df: float
    n_f: int
    # injected signal (None for pure noise): frequency, amplitude, phase, offset
    f0: Optional[float] = None
    amp: Optional[float] = None
    phase: Optional[float] = None
    offset: Optional[float] = None


@dataclass
class Batch:
    template: Template
    lcs: List[LightCurve] = field(default_factory=list)


def _unit_variance(c: np.ndarray, s: np.ndarray):
    # Var over a uniform phase of sum c cos + s sin is (1/2) sum (c^2 + s^2).
    v = 0.5 * float(np.sum(c * c + s * s))
    k = 1.0 / np.sqrt(v)
    return c * k, s * k


def template_random_normal(H: int, rng) -> Template:
    c = rng.standard_normal(H)
    s = rng.standard_normal(H)
    c, s = _unit_variance(c, s)
    return Template(c, s)


def template_sawtooth(H: int, rng) -> Template:
    """Amplitudes 1/n with random phases (a sawtooth-like shape)."""
    n = np.arange(1, H + 1, dtype=np.float64)
    ph = rng.uniform(0.0, 2.0 * np.pi, H)
    a = 1.0 / n
    c, s = _unit_variance(a * np.cos(ph), a * np.sin(ph))
    return Template(c, s)


def template_eclipsing_binary(H: int = 10, width: float = 0.03,
                              depth2: float = 0.3, ngrid: int = 1 << 14) -> Template:
    """Eclipsing-binary-like shape: a primary Gaussian dip of depth 1 and
    phase width ``width`` at phase 0 and a secondary dip of depth ``depth2``
    at phase 0.5, truncated to H harmonics and scaled to unit variance."""
    ph = np.arange(ngrid) / ngrid

    def dip(center):
        d = (ph - center + 0.5) % 1.0 - 0.5
        return np.exp(-0.5 * (d / width) ** 2)

    shape = -(dip(0.0) + depth2 * dip(0.5))
    x = 2.0 * np.pi * ph
    n = np.arange(1, H + 1)[:, None]
    c = 2.0 * np.mean(shape[None, :] * np.cos(n * x[None, :]), axis=1)
    s = 2.0 * np.mean(shape[None, :] * np.sin(n * x[None, :]), axis=1)
    c, s = _unit_variance(c, s)
    return Template(c, s)


def eval_template(tmpl: Template, x: np.ndarray) -> np.ndarray:
    """M(x) = sum_n c_n cos(n x) + s_n sin(n x) (used to synthesise y)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for n in range(1, tmpl.H + 1):
        out += tmpl.c[n - 1] * np.cos(n * x) + tmpl.s[n - 1] * np.sin(n * x)
    return out


def cadence_uniform(rng, n: int, baseline: float) -> np.ndarray:
    return np.sort(rng.uniform(0.0, baseline, n))


def cadence_nightly(rng, n: int, baseline: float, p_keep: float = 0.7,
                    window: float = 1.0 / 3.0, season_len: Optional[float] = None,
                    year: float = 365.25) -> np.ndarray:
    """Clustered ground-based cadence: one observing window of ``window``
    days per night, each night kept with probability ``p_keep``; with
    ``season_len`` only nights within the first ``season_len`` days of each
    ``year`` are observable."""
    nights = np.arange(int(np.floor(baseline)))
    keep = rng.random(len(nights)) < p_keep
    if season_len is not None:
        keep &= (nights % year) < season_len
    kept = nights[keep]
    if len(kept) == 0:
        kept = nights[:1]
    which = rng.integers(0, len(kept), n)
    t = kept[which] + rng.uniform(0.0, window, n)
    return np.sort(t)


def frequency_grid(t: np.ndarray, f_max: float, oversample: float = 5.0):
    """Regular grid f_j = j*df, j = 1..n_f with df = 1/(oversample*T)."""
    T = float(np.max(t) - np.min(t))
    df = 1.0 / (oversample * T)
    n_f = int(np.floor(f_max / df))
    return df, n_f


def _lc_rng(seed: int, index: int):
    return np.random.default_rng([int(seed), int(index)])


# ---------------------------------------------------------------- workloads

def tiny_case(seed: int, n_obs: int = 40, H: int = 2, n_f: int = 30,
              baseline: float = 5.0, noise: float = 0.2, cadence: str = "uniform"):
    """Small inputs for brute-force checks."""
    rng = np.random.default_rng(seed)
    tmpl = template_random_normal(H, rng)
    if cadence == "uniform":
        t = cadence_uniform(rng, n_obs, baseline)
    else:
        t = cadence_nightly(rng, n_obs, baseline)
    f0 = 1.0 / rng.uniform(0.3, 2.0)
    phi = rng.uniform(0, 2 * np.pi)
    sigma = rng.uniform(0.5, 1.5, n_obs) * noise
    y = 0.8 * eval_template(tmpl, 2 * np.pi * f0 * t - phi) + 0.1 + sigma * rng.standard_normal(n_obs)
    T = t.max() - t.min()
    df = 1.0 / (5.0 * T)
    return tmpl, LightCurve(t, y, sigma, df, n_f, f0, 0.8, phi, 0.1)


def small_fp64_case(seed: int = SEED0 + 0):
    """N=100 uniform times over 10 d, H=3 N(0,1) template, y = M(2 pi t/0.7 - 0.3)
    + N(0, 0.1^2), sigma = 0.1, f from df to 10/day with df = 1/(5 T)."""
    rng = np.random.default_rng(seed)
    tmpl = template_random_normal(3, rng)
    t = cadence_uniform(rng, 100, 10.0)
    y = eval_template(tmpl, 2 * np.pi * t / 0.7 - 0.3) + 0.1 * rng.standard_normal(100)
    sigma = np.full(100, 0.1)
    df, n_f = frequency_grid(t, 10.0)
    return tmpl, LightCurve(t, y, sigma, df, n_f, 1 / 0.7, 1.0, 0.3, 0.0)


def _signal_lc(rng, tmpl: Template, t: np.ndarray, amp: float, period: float,
               f_max: float, oversample: float = 5.0):
    n = len(t)
    sigma = rng.uniform(0.05, 0.2, n)
    phi = rng.uniform(0.0, 2.0 * np.pi)
    f0 = 1.0 / period
    y = amp * eval_template(tmpl, 2 * np.pi * f0 * t - phi) + sigma * rng.standard_normal(n)
    df, n_f = frequency_grid(t, f_max, oversample)
    return LightCurve(t, y, sigma, df, n_f, f0, amp, phi, 0.0)


def single_long_case(seed: int = SEED0 + 1, n_obs: int = 10_000):
    """N=1e4 over 1000 d, nightly 8 h windows, 30 % of nights dropped;
    H=6 sawtooth-like template; amplitude 0.5; sigma ~ U(0.05, 0.2);
    oversample 5, f_max = 10/day (~5e4 frequencies)."""
    rng = np.random.default_rng(seed)
    tmpl = template_sawtooth(6, rng)
    t = cadence_nightly(rng, n_obs, 1000.0)
    period = float(np.exp(rng.uniform(np.log(0.2), np.log(50.0))))
    return tmpl, _signal_lc(rng, tmpl, t, 0.5, period, 10.0)


def ragged_batch_case(seed: int = SEED0 + 2, n_lc: int = 4096, H: int = 4,
                      n_min: int = 50, n_max: int = 5000,
                      base_min: float = 30.0, base_max: float = 1500.0,
                      f_max: float = 10.0) -> Batch:
    """Ragged batch: N_obs log-uniform in [50, 5000], baselines U(30, 1500) d,
    nightly cadence, one shared H=4 template; even-indexed lightcurves carry
    a signal with period log-U[0.2, 50] d at SNR U(5, 20)
    (SNR = A * std(M) * sqrt(N) / mean(sigma), std(M) = 1); odd ones are noise."""
    rng0 = np.random.default_rng(seed)
    tmpl = template_sawtooth(H, rng0)
    batch = Batch(tmpl)
    for i in range(n_lc):
        rng = _lc_rng(seed, i)
        n = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max)))))
        T = float(rng.uniform(base_min, base_max))
        t = cadence_nightly(rng, n, T)
        sigma = rng.uniform(0.05, 0.2, n)
        df, n_f = frequency_grid(t, f_max)
        y = sigma * rng.standard_normal(n)
        lc = LightCurve(t, y, sigma, df, n_f)
        if i % 2 == 0:
            period = float(np.exp(rng.uniform(np.log(0.2), np.log(50.0))))
            snr = float(rng.uniform(5.0, 20.0))
            amp = snr * float(np.mean(sigma)) / np.sqrt(n)
            phi = float(rng.uniform(0.0, 2.0 * np.pi))
            y += amp * eval_template(tmpl, 2 * np.pi * t / period - phi)
            lc.y = y
            lc.f0, lc.amp, lc.phase, lc.offset = 1.0 / period, amp, phi, 0.0
        batch.lcs.append(lc)
    return batch


def _learned_lc(seed: int, index: int, tmpl: Template, n_obs: int, baseline: float):
    rng = _lc_rng(seed, index)
    t = cadence_nightly(rng, n_obs, baseline)
    period = float(np.exp(rng.uniform(np.log(0.2), np.log(50.0))))
    return _signal_lc(rng, tmpl, t, 0.5, period, 10.0)


def single_long_template(seed: int = SEED0 + 1) -> Template:
    """The H=6 template of the single long lightcurve workload."""
    return template_sawtooth(6, np.random.default_rng(seed))


def learned_template() -> Template:
    """Template of the learned-proposal workloads: the single long
    lightcurve's, so a network trained here applies to that workload."""
    return single_long_template()


def learned_train_lightcurves(n_lc: int = 200, seed: int = SEED0 + 3, n_obs: int = 10_000,
                              baseline: float = 1000.0):
    """Lightcurves like the single long case (H=6) used to generate the
    polynomials the root-proposal network is trained on."""
    tmpl = learned_template()
    return tmpl, [_learned_lc(seed + 1000, i, tmpl, n_obs, baseline) for i in range(n_lc)]


def learned_heldout_lightcurves(n_lc: int = 1024, seed: int = SEED0 + 3, n_obs: int = 2000,
                                baseline: float = 1000.0):
    """Held-out evaluation set (disjoint seed stream): N=2000, T=1000 d."""
    tmpl = learned_template()
    return tmpl, [_learned_lc(seed + 2000, i, tmpl, n_obs, baseline) for i in range(n_lc)]


def large_template() -> Template:
    """The H=10 eclipsing-binary-like template of the large workload."""
    return template_eclipsing_binary(10)


def _large_lc(rng, tmpl: Template, n_obs: int):
    t = cadence_nightly(rng, n_obs, 3000.0, season_len=243.0)
    period = float(np.exp(rng.uniform(np.log(0.2), np.log(50.0))))
    return _signal_lc(rng, tmpl, t, 0.5, period, 20.0)


def large_case(seed: int = SEED0 + 4, n_obs: int = 100_000):
    """N=1e5 over 3000 d: nightly windows within an 8-month season per year;
    H=10 eclipsing-binary-like template; amplitude 0.5; sigma ~ U(0.05, 0.2);
    oversample 5, f_max = 20/day (~3e5 frequencies)."""
    rng = np.random.default_rng(seed)
    tmpl = large_template()
    return tmpl, _large_lc(rng, tmpl, n_obs)


def large_train_lightcurves(n_lc: int = 34, seed: int = SEED0 + 4, n_obs: int = 100_000):
    """Lightcurves drawn like the large case (own seed stream, disjoint from
    it and from the held-out set): the polynomials the H=10 root-proposal
    network is trained on (34 x ~3e5 frequencies ~ 1e7 samples)."""
    tmpl = large_template()
    return tmpl, [_large_lc(_lc_rng(seed + 1000, i), tmpl, n_obs) for i in range(n_lc)]


def large_heldout_lightcurves(n_lc: int = 8, seed: int = SEED0 + 4, n_obs: int = 100_000):
    """Held-out lightcurves drawn like the large case (disjoint seed stream)."""
    tmpl = large_template()
    return tmpl, [_large_lc(_lc_rng(seed + 2000, i), tmpl, n_obs) for i in range(n_lc)]


def multiband_case(seed: int = SEED0 + 6, n_band: int = 5, n_obs: int = 2000, baseline: float = 1000.0,
                   H: int = 6):
    """One variable observed in n_band bands (u, g, r, i, z-like): the same
    period and phase in every band, band amplitudes 0.5, 0.4, 0.35, 0.3, 0.25
    (cycled), per-band noise sigma ~ U(0.05, 0.2) times 1.0, 0.6, 0.5, 0.6,
    0.9 (cycled), each band on its own nightly cadence over the baseline;
    df from the longest band span, f_max = 10/day.  Returns (template, bands
    [(t, y, sigma)], df, n_f, f0)."""
    rng = np.random.default_rng(seed)
    tmpl = template_sawtooth(H, rng)
    period = float(np.exp(rng.uniform(np.log(0.2), np.log(50.0))))
    phi = float(rng.uniform(0.0, 2.0 * np.pi))
    amps = [0.5, 0.4, 0.35, 0.3, 0.25]
    noise = [1.0, 0.6, 0.5, 0.6, 0.9]
    bands = []
    for k in range(n_band):
        t = cadence_nightly(rng, n_obs, baseline)
        sigma = rng.uniform(0.05, 0.2, n_obs) * noise[k % 5]
        y = amps[k % 5] * eval_template(tmpl, 2 * np.pi * t / period - phi) + 0.1 * k + sigma * rng.standard_normal(n_obs)
        bands.append((t, y, sigma))
    t_all = np.concatenate([b[0] for b in bands])
    df, n_f = frequency_grid(t_all, 10.0)
    return tmpl, bands, df, n_f, 1.0 / period


def shared_phase_case(seed: int = SEED0 + 7, n_band: int = 5, n_obs: int = 2000, baseline: float = 1000.0,
                      H: int = 6):
    """One variable in n_band bands whose shapes differ per band (the model of
    the shared-phase multi-band periodogram, Appendix A): a sawtooth-like
    template per band (own harmonic phases), one period, phase and amplitude
    for all bands, band offsets lambda_k = 0.3 k - 0.5, per-band noise sigma ~
    U(0.05, 0.2) times 1.0, 0.6, 0.5, 0.6, 0.9 (cycled), nightly cadences over
    the baseline, df from the longest band span and f_max = 10/day.  Returns
    (templates, bands [(t, y, sigma)], offsets, df, n_f, f0)."""
    rng = np.random.default_rng(seed)
    templates = [template_sawtooth(H, rng) for _ in range(n_band)]
    period = float(np.exp(rng.uniform(np.log(0.2), np.log(50.0))))
    phi = float(rng.uniform(0.0, 2.0 * np.pi))
    lam = 0.3 * np.arange(n_band) - 0.5
    noise = [1.0, 0.6, 0.5, 0.6, 0.9]
    bands = []
    for k in range(n_band):
        t = cadence_nightly(rng, n_obs, baseline)
        sigma = rng.uniform(0.05, 0.2, n_obs) * noise[k % 5]
        y = 0.4 * eval_template(templates[k], 2 * np.pi * t / period - phi) + 0.2 + lam[k] + \
            sigma * rng.standard_normal(n_obs)
        bands.append((t, y, sigma))
    t_all = np.concatenate([b[0] for b in bands])
    df, n_f = frequency_grid(t_all, 10.0)
    return templates, bands, lam, df, n_f, 1.0 / period


def h_sweep_case(H: int, seed: int = SEED0 + 5, n_obs: int = 10_000):
    """Single-long-like lightcurve (N=1e4 over 1000 d, nightly cadence,
    f_max = 10/day) carrying a signal of an H-harmonic sawtooth-like
    template; one template and lightcurve per H (seed stream seed + H)."""
    rng = np.random.default_rng(seed * 100 + H)
    tmpl = template_sawtooth(H, rng)
    t = cadence_nightly(rng, n_obs, 1000.0)
    period = float(np.exp(rng.uniform(np.log(0.2), np.log(50.0))))
    return tmpl, _signal_lc(rng, tmpl, t, 0.5, period, 10.0)


WORKLOADS = {
    "small_fp64": small_fp64_case,
    "single_long": single_long_case,
    "ragged_batch": ragged_batch_case,
    "large": large_case,
    "h_sweep": h_sweep_case,
}
