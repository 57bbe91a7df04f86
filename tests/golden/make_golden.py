"""Writes the stored expected values used by the GPU tests, from the CPU FP64
oracle only (no GPU code is imported).

    python tests/golden/make_golden.py

single_long_oracle.json: the full oracle periodogram of the single long
lightcurve workload (N_obs = 1e4, H = 6, 49 912 frequencies): best index, its
power and the five highest local maxima.
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
from synthetic import single_long_case  # noqa: E402


def main():
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
    main()
