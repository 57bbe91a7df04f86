"""Ragged batches through ftp_periodogram_batch.

* A batch equals the concatenation of single-lightcurve calls bit for bit
  (same grids, same kernels; the spreading is order independent).
* Sampled outputs of batch members match the oracle (FP32 sums: |dP| <= 1e-4).
* The full ragged-batch workload (4096 lightcurves, ~1.6e8 pairs) runs in one
  call; sampled members match the oracle and the injected signals are found.
"""
import numpy as np
import pytest

from oracle import ftp_oracle as O
from synthetic import ragged_batch_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ftp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2101_12348_amd as F
    F.load_library()
    return F


def _concat(batch):
    lcs = batch.lcs
    obs_off = np.concatenate([[0], np.cumsum([len(lc.t) for lc in lcs])])
    freq_off = np.concatenate([[0], np.cumsum([lc.n_f for lc in lcs])])
    t = np.concatenate([lc.t for lc in lcs])
    y = np.concatenate([lc.y for lc in lcs])
    s = np.concatenate([lc.sigma for lc in lcs])
    df = np.array([lc.df for lc in lcs])
    return obs_off, freq_off, t, y, s, df


@pytest.mark.parametrize("solver", [0, 2])
def test_batch_equals_single_calls(ftp, solver):
    import torch
    batch = ragged_batch_case(n_lc=24)
    obs_off, freq_off, t, y, s, df = _concat(batch)
    plan = ftp.Plan(batch.template.c, batch.template.s, solver=solver)
    out = {k: v.clone() for k, v in plan.periodogram_batch(obs_off, t, y, s, df, freq_off).items()}
    for b, lc in enumerate(batch.lcs):
        single = plan.periodogram(lc.t, lc.y, lc.sigma, lc.df, lc.n_f)
        sl = slice(int(freq_off[b]), int(freq_off[b + 1]))
        for k in ("power", "phase", "amp", "offset", "status"):
            assert torch.equal(single[k], out[k][sl]), (b, k)


def test_multichunk_batch_equals_single_calls(ftp):
    """A batch of more than two solve rounds (each round's side-stream
    scoring joined before the next round rewrites the records) equals
    single-lightcurve calls (one round each) bit for bit."""
    import torch
    batch = ragged_batch_case(n_lc=240)
    obs_off, freq_off, t, y, s, df = _concat(batch)
    assert freq_off[-1] > 8.5e6   # three rounds of 2^22 pairs at H = 4
    plan = ftp.Plan(batch.template.c, batch.template.s, solver=ftp.FTP_SOLVER_UNIFORM)
    out = {k: v.clone() for k, v in plan.periodogram_batch(obs_off, t, y, s, df, freq_off).items()}
    torch.cuda.synchronize()
    for b, lc in enumerate(batch.lcs):
        single = plan.periodogram(lc.t, lc.y, lc.sigma, lc.df, lc.n_f)
        sl = slice(int(freq_off[b]), int(freq_off[b + 1]))
        for k in ("power", "phase", "amp", "offset", "status"):
            assert torch.equal(single[k], out[k][sl]), (b, k)


def test_batch_members_match_oracle(ftp):
    batch = ragged_batch_case(n_lc=24)
    obs_off, freq_off, t, y, s, df = _concat(batch)
    plan = ftp.Plan(batch.template.c, batch.template.s)
    out = {k: v.cpu().numpy() for k, v in plan.periodogram_batch(obs_off, t, y, s, df, freq_off).items()}
    rng = np.random.default_rng(0)
    for b in (0, 1, 7, 12, 23):
        lc = batch.lcs[b]
        js = np.unique(rng.integers(1, lc.n_f + 1, 25))
        ref = O.periodogram(lc.t, lc.y, lc.sigma, batch.template.c, batch.template.s, lc.df, freq_index=js)
        g = out["power"][freq_off[b] + js - 1]
        assert np.max(np.abs(g - ref["power"])) <= 1e-4, b


def test_full_ragged_batch_workload(ftp):
    import torch
    batch = ragged_batch_case()
    assert len(batch.lcs) == 4096
    obs_off, freq_off, t, y, s, df = _concat(batch)
    plan = ftp.Plan(batch.template.c, batch.template.s)
    out = plan.periodogram_batch(obs_off, t, y, s, df, freq_off)
    torch.cuda.synchronize()
    P = out["power"].cpu().numpy()
    st = out["status"].cpu().numpy()
    assert int(freq_off[-1]) > 1e8
    assert np.all(np.isfinite(P)) and np.all(P >= 0) and np.all(P <= 1 + 1e-9)
    assert np.all((st & 0x7) != 4)
    rng = np.random.default_rng(1)
    found = 0
    injected = 0
    for b in rng.choice(4096, 12, replace=False):
        lc = batch.lcs[b]
        seg = P[freq_off[b]: freq_off[b + 1]]
        jbest = int(np.argmax(seg)) + 1
        js = np.unique(np.r_[jbest, rng.integers(1, lc.n_f + 1, 12)])
        ref = O.periodogram(lc.t, lc.y, lc.sigma, batch.template.c, batch.template.s, lc.df, freq_index=js)
        assert np.max(np.abs(seg[js - 1] - ref["power"])) <= 1e-4, b
        if lc.f0 is not None and lc.amp * np.sqrt(len(lc.t)) / np.mean(lc.sigma) > 12:
            injected += 1
            # the peak sits at the injected frequency or one of its low-order aliases
            f = jbest * lc.df
            cands = [lc.f0 * k + a for k in (1, 2, 0.5) for a in (0.0, 1.0, -1.0)]
            if min(abs(f - c) for c in cands) <= 2 * lc.df:
                found += 1
    assert found >= injected - 1
