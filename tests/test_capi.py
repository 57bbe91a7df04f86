"""CPU-side checks of the C ABI: the shared library loads and exports every
function declared in include/ftp.h (no compute calls without a GPU), and the
header's constants match the Python binding."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ftp.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ftp_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_2101_12348_amd as F
    lib = F.load_library()
    names = _declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(F.EXPORTED)


def test_header_constants_match_binding():
    import paper_2101_12348_amd as F
    src = open(HEADER).read()
    consts = dict(re.findall(r"#define (FTP_[A-Z0-9_]+) (-?\d+)u?", src))
    assert int(consts["FTP_FP32_SUMS"]) == F.FTP_FP32_SUMS
    assert int(consts["FTP_FP64"]) == F.FTP_FP64
    assert int(consts["FTP_SOLVER_LEARNED"]) == F.FTP_SOLVER_LEARNED
    assert int(consts["FTP_SOLVER_UNIFORM"]) == F.FTP_SOLVER_UNIFORM
    assert int(consts["FTP_SOLVER_ABERTH"]) == F.FTP_SOLVER_ABERTH
    assert int(consts["FTP_ST_FALLBACK"]) == F.ST_FALLBACK
    assert int(consts["FTP_ST_FALLBACK_QR"]) == F.ST_FALLBACK_QR
    assert int(consts["FTP_ST_BAD_LC"]) == F.ST_BAD_LC
    assert int(consts["FTP_MAX_H"]) == F.MAX_H


def test_status_strings_and_option_defaults():
    import ctypes
    import paper_2101_12348_amd as F
    lib = F.load_library()
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10, 1, 2, 3, 4, 8, 16):
        s = lib.ftp_status_string(code).decode()
        assert s and s != "unknown code", code
    opt = F.Options()
    assert lib.ftp_options_default(ctypes.byref(opt)) == 0
    assert opt.precision == F.FTP_FP32_SUMS and opt.solver == F.FTP_SOLVER_PLAIN and opt.nfft_R == 2.0
    assert lib.ftp_options_default(None) == -1


def test_host_validation_without_device():
    """Argument checks that return before touching the device."""
    import ctypes
    import numpy as np
    import paper_2101_12348_amd as F
    lib = F.load_library()
    h = ctypes.c_void_p()
    c = np.zeros(3)
    s = np.zeros(3)
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert lib.ftp_plan_create(None, 3, vp(c), vp(s), None) == -1
    assert lib.ftp_plan_create(ctypes.byref(h), 3, vp(c), vp(s), None) == -2      # all zero
    c[0] = 1.0
    assert lib.ftp_plan_create(ctypes.byref(h), 0, vp(c), vp(s), None) == -2      # H < 1
    assert lib.ftp_plan_create(ctypes.byref(h), 16, vp(np.ones(16)), vp(np.ones(16)), None) == -2      # H > 15
    bad = np.array([np.nan, 1.0, 1.0])
    assert lib.ftp_plan_create(ctypes.byref(h), 3, vp(bad), vp(s), None) == -2
    opt = F.Options()
    lib.ftp_options_default(ctypes.byref(opt))
    opt.precision = 7
    assert lib.ftp_plan_create(ctypes.byref(h), 3, vp(c), vp(s), ctypes.byref(opt)) == -9
    lib.ftp_options_default(ctypes.byref(opt))
    opt.nfft_R = 1.0
    assert lib.ftp_plan_create(ctypes.byref(h), 3, vp(c), vp(s), ctypes.byref(opt)) == -9
    assert lib.ftp_periodogram(None, None, None, None, 10, 0.1, 10, None, None, None, None, None, None) == -1
    assert lib.ftp_plan_destroy(None) == -1
    # bands plans: band count, all-zero or non-finite templates
    cb, sb = np.zeros((2, 3)), np.zeros((2, 3))
    assert lib.ftp_plan_create_bands(ctypes.byref(h), 0, 3, vp(cb), vp(sb), None) == -9
    assert lib.ftp_plan_create_bands(ctypes.byref(h), 17, 3, vp(np.ones(51)), vp(np.ones(51)), None) == -9
    assert lib.ftp_plan_create_bands(ctypes.byref(h), 2, 3, vp(cb), vp(sb), None) == -2
    cb[1, 0] = np.inf
    assert lib.ftp_plan_create_bands(ctypes.byref(h), 2, 3, vp(cb), vp(sb), None) == -2
    assert lib.ftp_periodogram_shared_phase(None, None, None, None, None, None, 0.1, 10, None, None, None,
                                            None, None, None) == -1


def test_tuning_cache_file_round_trip(tmp_path):
    """The autotuner's cache file: lookup of a missing file or key, replace
    and append, malformed and out-of-range lines ignored, bad keys and shapes
    rejected, an unwritable path reported (host code only)."""
    import paper_2101_12348_amd as F
    F.load_library()
    p = str(tmp_path / "tune.txt")
    key = "gfx950/256cu/H6/p0/s1"
    assert F.tune_cache_lookup(p, key) is None
    shapes = dict(assemble_wpc=32, newton_wpc=16, aberth_wpc=8, qr_wpc=16, score_wpc=24, mlp_fused=0, newton_occ=5)
    F.tune_cache_store(p, key, **shapes)
    F.tune_cache_store(p, "gfx950/256cu/H4/p0/s0", **dict({k: 4 for k in shapes}, mlp_fused=1))
    assert F.tune_cache_lookup(p, "gfx950/256cu/H4/p0/s0")["newton_occ"] == 4
    assert F.tune_cache_lookup(p, key) == shapes
    shapes2 = dict(shapes, qr_wpc=48)
    F.tune_cache_store(p, key, **shapes2)
    lines = open(p).read().splitlines()
    assert sum(1 for l in lines if l.split()[0] == key) == 1 and len(lines) == 2
    assert F.tune_cache_lookup(p, key) == shapes2
    with open(p, "a") as fh:
        fh.write("garbage line\n" + key + " 1 2 3\n" + "gfx950/256cu/H3/p0/s0 0 4 4 4 4 0\n"
                 + "gfx950/256cu/H2/p0/s0 4 4 4 4 4 2\n" + "gfx950/256cu/H1/p0/s0 4 4 4 4 4 0 7\n"
                 + "gfx950/256cu/H5/p0/s0 8 8 8 8 8 1\n")
    assert F.tune_cache_lookup(p, key) == shapes2
    assert F.tune_cache_lookup(p, "gfx950/256cu/H3/p0/s0") is None
    assert F.tune_cache_lookup(p, "gfx950/256cu/H2/p0/s0") is None
    assert F.tune_cache_lookup(p, "gfx950/256cu/H1/p0/s0") is None
    # a line without the Newton occupancy (the older six-column form) reads as 4
    assert F.tune_cache_lookup(p, "gfx950/256cu/H5/p0/s0") == dict({k: 8 for k in shapes}, mlp_fused=1, newton_occ=4)
    for bad_key in ("", "has space"):
        with pytest.raises(F.FtpError):
            F.tune_cache_store(p, bad_key, **shapes)
    for bad in (dict(shapes, score_wpc=0), dict(shapes, mlp_fused=2), dict(shapes, newton_occ=3)):
        with pytest.raises(F.FtpError):
            F.tune_cache_store(p, key, **bad)
    with pytest.raises(F.FtpError):
        F.tune_cache_store(str(tmp_path / "missing_dir" / "tune.txt"), key, **shapes)
