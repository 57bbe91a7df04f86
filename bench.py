#!/usr/bin/env python3
"""Throughput benchmark of the fast template periodogram hot path on one GPU.

Metric: (lightcurve x trial-frequency) pairs per second, reported only when
the GPU periodogram agrees with the CPU FP64 oracle to |dP| <= 1e-4 on a
sample of frequencies (FP32 NFFT sums, FP64 assembly/roots/scoring).

Workload (single long lightcurve): N_obs = 1e4 over a 1000-day baseline with
nightly 8 h windows and 30 % of nights dropped, H = 6 sawtooth-like template,
amplitude 0.5, sigma ~ U(0.05, 0.2), f_j = j df with df = 1/(5 T) up to
10/day (~5e4 frequencies).  A step is one full pass of the hot path over that
lightcurve: weights/statistics, spreading, FFTs, gather/deconvolution,
polynomial assembly, root solve and scoring, all on the device.  Inputs are
resident in HBM before the timed region starts.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--solver plain|learned]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector, published
HBM_PEAK_GBS = 8000.0


def qr_flops(H: int) -> float:
    """Algorithmic FP64 work of one companion eigenvalue solve of degree
    D = 6H - 2: ~10 D^3 flops (Golub & Van Loan's estimate for the
    eigenvalues of a general matrix by the QR algorithm)."""
    D = 6 * H - 2
    return 10.0 * D ** 3


def cpu_baseline(tmpl, lc, n_sample: int):
    """The FP64 oracle timed on the host on an evenly spaced sample of the
    workload's frequencies."""
    import numpy as np
    from oracle import ftp_oracle as O
    js = np.unique(np.linspace(1, lc.n_f, n_sample).astype(np.int64))
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    ref = O.periodogram(lc.t, lc.y, lc.sigma, tmpl.c, tmpl.s, lc.df, freq_index=js)
    dt = time.perf_counter() - t0
    return dict(value=len(js) / dt, unit="pairs/s", cores=int(threads), kind="oracle",
                sample=f"{len(js)} evenly spaced frequencies of the {lc.n_f}-frequency grid "
                       f"(N_obs={len(lc.t)}), {dt:.1f} s"), js, ref


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--solver", default="plain", choices=["plain", "learned"])
    ap.add_argument("--cpu-sample", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(lightcurves and frequency slices shard without communication; see the design notes).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2101_12348_amd as F
    from synthetic import single_long_case

    dev = torch.device("cuda:0")
    tmpl, lc = single_long_case()
    H = tmpl.H
    solver = F.FTP_SOLVER_PLAIN if args.solver == "plain" else F.FTP_SOLVER_LEARNED
    plan = F.Plan(tmpl.c, tmpl.s, precision=F.FTP_FP32_SUMS, solver=solver, flags=F.FTP_FLAG_TIME_STAGES)
    t = torch.as_tensor(lc.t, device=dev)
    y = torch.as_tensor(lc.y, device=dev)
    s = torch.as_tensor(lc.sigma, device=dev)
    out = plan.alloc_outputs(lc.n_f, dev)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        plan.periodogram(t, y, s, lc.df, lc.n_f, out=out)
    torch.cuda.synchronize()
    plan.stats()   # reset the accumulation window

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        plan.periodogram(t, y, s, lc.df, lc.n_f, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_total = ev0.elapsed_time(ev1)
    st = plan.stats()
    ms_step = ms_total / args.steps
    pairs = lc.n_f
    value = pairs / (ms_step * 1e-3)

    # accuracy gate on a sample of frequencies against the oracle
    gate = None
    cpu = None
    P = out["power"].cpu().numpy()
    if not args.no_cpu_baseline:
        cpu, js, ref = cpu_baseline(tmpl, lc, args.cpu_sample)
        dP = float(np.max(np.abs(P[js - 1] - ref["power"])))
        gate = dict(max_abs_dP=dP, n_checked=int(len(js)), pass_=bool(dP <= 1e-4))
    jbest = int(np.argmax(P)) + 1

    ms_solve = st["ms_solve"] / args.steps
    ms_nfft = st["ms_nfft"] / args.steps
    ms_roots = st["ms_roots"] / args.steps
    flops = qr_flops(H) * pairs
    achieved = flops / (ms_roots * 1e-3) / 1e12 if ms_roots > 0 else None
    line = {
        "metric": "trial-freq x lightcurve pairs/sec at |dP|<=1e-4 vs FP64 oracle",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "single long lightcurve: N_obs=1e4, T=1000 d nightly cadence, H=6, "
                               f"f_max=10/day, oversample 5, N_f={lc.n_f}, FP32 NFFT sums, FP64 solve",
                   "solver": args.solver, "H": H, "n_obs": int(len(lc.t)), "n_f": int(lc.n_f)},
        "roofline": {"bound": "alu", "kernel": "k_qr<34> (companion QR, FP64 vector)",
                     "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": (achieved / FP64_PEAK_TFLOPS) if achieved else None, "traffic": None,
                     "flops_per_pair": qr_flops(H), "ms_kernel": ms_roots, "ms_solve_stage": ms_solve,
                     "ms_nfft_stage": ms_nfft},
        "cpu_baseline": cpu,
        "accuracy": gate,
        "best_frequency": {"index": jbest, "f": jbest * lc.df, "injected_f": lc.f0},
        "stats": {k: st[k] for k in ("n_pairs", "n_fallback", "qr_sweeps")},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
