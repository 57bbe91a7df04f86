"""Writes the stored expected values used by the GPU tests, from the CPU FP64
oracle only (no GPU code is imported).

    python tests/golden/make_golden.py

single_long_oracle.json: the full oracle periodogram of the single long
lightcurve workload (N_obs = 1e4, H = 6, 49 912 frequencies): best index, its
power and the five highest local maxima.

large_oracle.json: the large workload (N_obs = 1e5, H = 10, ~3e5 frequencies;
the full oracle periodogram would take about a day on one core): the oracle
on windows of frequencies around the injected frequency f0 and around 2 f0
and f0 / 2 (the indices follow from the generator's f0 and df alone), with
the best index of the windows.

    python tests/golden/make_golden.py [single_long] [large]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import ftp_oracle as O  # noqa: E402
from synthetic import single_long_case, large_case  # noqa: E402


def large():
    tmpl, lc = large_case()
    t0 = time.time()
    windows = []
    for mult, half in ((1.0, 60), (2.0, 20), (0.5, 20)):
        j0 = int(round(mult * lc.f0 / lc.df))
        windows.append(np.arange(max(1, j0 - half), min(lc.n_f, j0 + half) + 1))
    js = np.unique(np.concatenate(windows))
    r = O.periodogram(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, lc.df, freq_index=js, block=4)
    P = r["power"]
    k = int(np.argmax(P))
    out = dict(workload="large_case()", n_f=int(lc.n_f), df=float(lc.df), f0=float(lc.f0),
               indices=[int(j) for j in js], power=[float(x) for x in P], best_index=int(js[k]),
               best_power=float(P[k]), best_phase=float(r["phase"][k]), best_amp=float(r["amp"][k]),
               best_offset=float(r["offset"][k]), seconds=time.time() - t0)
    with open(os.path.join(HERE, "large_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print({k: v for k, v in out.items() if k not in ("indices", "power")})


def single_long():
    tmpl, lc = single_long_case()
    t0 = time.time()
    r = O.periodogram(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, lc.df, lc.n_f, block=128)
    P = r["power"]
    j = int(np.argmax(P)) + 1
    peaks = [k for k in range(1, len(P) - 1) if P[k] >= P[k - 1] and P[k] >= P[k + 1]]
    peaks = sorted(peaks, key=lambda k: -P[k])[:5]
    out = dict(workload="single_long_case()", n_f=int(lc.n_f), df=float(lc.df), best_index=j,
               best_power=float(P[j - 1]), best_phase=float(r["phase"][j - 1]), best_amp=float(r["amp"][j - 1]),
               best_offset=float(r["offset"][j - 1]),
               top_peaks=[dict(index=int(k + 1), power=float(P[k])) for k in peaks],
               seconds=time.time() - t0)
    with open(os.path.join(HERE, "single_long_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(out)


if __name__ == "__main__":
    which = sys.argv[1:] or ["single_long", "large"]
    if "single_long" in which:
        single_long()
    if "large" in which:
        large()
