"""Launch shapes and the autotuner (the schedule of the per-frequency stage).

* Every frequency is computed by one wavefront whatever the grid and the
  queue order, and the Newton kernel's register budgets (newton_occ) compile
  the same arithmetic, so outputs are bit-identical across launch shapes.
* The autotuner returns valid shapes, applies them, stores them in its cache
  and serves the next request for the same key from there.
"""
import numpy as np
import pytest

from synthetic import single_long_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ftp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2101_12348_amd as F
    F.load_library()
    return F


@pytest.mark.parametrize("solver", [0, 2, 3])
def test_outputs_do_not_depend_on_launch_shapes(ftp, solver):
    import torch
    tmpl, lc = single_long_case(n_obs=2000)
    n_f = 6000
    plan = ftp.Plan(tmpl.c, tmpl.s, solver=solver)
    ref = {k: v.clone() for k, v in plan.periodogram(lc.t, lc.y, lc.sigma, lc.df, n_f).items()}
    for wpc, occ in ((1, 4), (3, 5), (64, 6)):
        plan.set_tuning(assemble_wpc=wpc, newton_wpc=wpc, aberth_wpc=wpc, qr_wpc=wpc, score_wpc=wpc, newton_occ=occ)
        out = plan.periodogram(lc.t, lc.y, lc.sigma, lc.df, n_f)
        for k in ref:
            assert torch.equal(ref[k], out[k]), (wpc, k)


def test_set_tuning_rejects_bad_shapes(ftp):
    tmpl, _ = single_long_case(n_obs=500)
    plan = ftp.Plan(tmpl.c, tmpl.s)
    before = plan.tuning()
    for bad in (0, 257, -3):
        with pytest.raises(ftp.FtpError):
            plan.set_tuning(qr_wpc=bad)
    with pytest.raises(ftp.FtpError):
        plan.set_tuning(mlp_fused=2)
    for bad in (0, 3, 7):
        with pytest.raises(ftp.FtpError):
            plan.set_tuning(newton_occ=bad)
    with pytest.raises(KeyError):
        plan.set_tuning(no_such_shape=4)
    assert plan.tuning() == before


def test_autotune_and_cache(ftp, tmp_path):
    import torch
    tmpl, lc = single_long_case(n_obs=2000)
    n_f = 6000
    plan = ftp.Plan(tmpl.c, tmpl.s, solver=ftp.FTP_SOLVER_UNIFORM)
    ref = {k: v.clone() for k, v in plan.periodogram(lc.t, lc.y, lc.sigma, lc.df, n_f).items()}
    cache = str(tmp_path / "tune.txt")
    shapes, cached = plan.autotune(lc.t, lc.y, lc.sigma, lc.df, n_f, cache_path=cache)
    assert not cached
    assert all(1 <= v <= 256 for k, v in shapes.items() if k not in ("mlp_fused", "newton_occ"))
    assert shapes["mlp_fused"] in (0, 1) and shapes["newton_occ"] in (4, 5, 6)
    assert plan.tuning() == shapes
    assert ftp.tune_cache_lookup(cache, plan.tune_key(n_f)) == shapes
    out = plan.periodogram(lc.t, lc.y, lc.sigma, lc.df, n_f)
    for k in ref:
        assert torch.equal(ref[k], out[k]), k
    plan2 = ftp.Plan(tmpl.c, tmpl.s, solver=ftp.FTP_SOLVER_UNIFORM)
    shapes2, cached2 = plan2.autotune(lc.t, lc.y, lc.sigma, lc.df, n_f, cache_path=cache)
    assert cached2 and shapes2 == shapes and plan2.tuning() == shapes
    key = plan.tune_key(n_f)
    assert key.endswith("/H6/p0/s2/nf12") and "cu/" in key
    # size buckets: even powers of two, clamped to 2^10 .. 2^24
    assert plan.tune_key(1).endswith("/nf10") and plan.tune_key(4095).endswith("/nf10")
    assert plan.tune_key(4096).endswith("/nf12") and plan.tune_key(299931).endswith("/nf18")
    assert plan.tune_key(1 << 30).endswith("/nf24")
    with pytest.raises(ftp.FtpError):
        plan.tune_key(0)
