"""ftp_solve_sums_noalloc (the per-frequency stage with its scratch in the
library's fixed device array, for callers that cannot allocate) against
ftp_solve_sums on the same sums: identical outputs (same kernels, per-pair
results independent of the chunking), on two calls in a row, the second with
fewer frequencies, for the solvers the entry point serves."""
import numpy as np
import pytest

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


@pytest.mark.parametrize("case,solver,sizes", [("single_long", "plain", (20000, 7000)),
                                               ("single_long", "uniform", (49912, 12345)),
                                               ("large", "aberth", (45000, 9000)),
                                               ("large", "uniform", (65000, 3001))])
def test_noalloc_matches_solve_sums(ftp, case, solver, sizes):
    import torch
    tmpl, lc = {"single_long": single_long_case, "large": large_case}[case]()
    sv = {"plain": ftp.FTP_SOLVER_PLAIN, "uniform": ftp.FTP_SOLVER_UNIFORM, "aberth": ftp.FTP_SOLVER_ABERTH}[solver]
    src = ftp.Plan(tmpl.c, tmpl.s)
    sums, st = src.nfft_sums(lc.t, lc.y, lc.sigma, lc.df, max(sizes))
    tref, ybar, yy, bad = [float(x) for x in st.cpu()]
    assert bad == 0
    ref_plan = ftp.Plan(tmpl.c, tmpl.s, solver=sv)
    na_plan = ftp.Plan(tmpl.c, tmpl.s, solver=sv)
    for n in sizes:
        s_n = torch.view_as_real(sums[:n]).contiguous()
        ref = ref_plan.solve_sums(s_n, tref, ybar, yy, lc.df)
        out = ftp.Plan.alloc_outputs(n, s_n.device)
        for v in out.values():
            v.fill_(7)
        na_plan.solve_sums_noalloc(s_n, tref, ybar, yy, lc.df, out)
        torch.cuda.synchronize()
        for k in ("power", "phase", "amp", "offset", "status"):
            assert torch.equal(out[k], ref[k]), (k, n)
        assert float(out["power"].max()) > 0.0


def test_noalloc_rejects_learned_and_bad_input(ftp):
    import torch
    tmpl, lc = single_long_case()
    plan = ftp.Plan(tmpl.c, tmpl.s, solver=ftp.FTP_SOLVER_LEARNED)
    w, meta = ftp.load_model("single_long_h6")
    plan.load_mlp(w, meta["width"])
    sums = torch.zeros((10, 3 * tmpl.H, 2), dtype=torch.float64, device="cuda")
    out = ftp.Plan.alloc_outputs(10, sums.device)
    with pytest.raises(ftp.FtpError):
        plan.solve_sums_noalloc(sums, 0.0, 0.0, 1.0, lc.df, out)
    plain = ftp.Plan(tmpl.c, tmpl.s)
    with pytest.raises(ftp.FtpError):
        plain.solve_sums_noalloc(sums, 0.0, 0.0, -1.0, lc.df, out)
