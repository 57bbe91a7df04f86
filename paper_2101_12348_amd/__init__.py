"""Python binding of the gfx950 fast template periodogram library.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libftp.so`` (built in-tree by ``build.py``).  Tensors are torch
tensors on a ROCm device; the current torch stream is passed to the library.
There is no CPU fallback: if the library is missing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libftp.so")

FTP_FP32_SUMS = 0
FTP_FP64 = 1
FTP_SOLVER_PLAIN = 0
FTP_SOLVER_LEARNED = 1
FTP_SOLVER_UNIFORM = 2
FTP_SOLVER_ABERTH = 3
FTP_FLAG_FORCE_FALLBACK = 1
FTP_FLAG_TIME_STAGES = 2
FTP_FLAG_POSITIVE_AMP = 8
FTP_FLAG_SEEDS_ALL = 16
FTP_FLAG_2H_STARTS = 32
MAX_H = 15

ST_OK, ST_DEGENERATE, ST_CONSTANT, ST_NO_CONVERGE, ST_BAD_LC, ST_FALLBACK, ST_FALLBACK_QR = 0, 1, 2, 3, 4, 8, 16

EXPORTED = [
    "ftp_options_default", "ftp_plan_create", "ftp_plan_destroy", "ftp_periodogram",
    "ftp_periodogram_batch", "ftp_nfft_sums", "ftp_solve_sums", "ftp_plan_load_mlp",
    "ftp_last_stats", "ftp_status_string", "ftp_last_error",
    "ftp_mlp_create", "ftp_mlp_destroy", "ftp_mlp_num_params", "ftp_mlp_get_weights", "ftp_mlp_forward",
    "ftp_mlp_loss_grad", "ftp_mlp_train_step", "ftp_learned_dataset",
    "ftp_plan_get_tuning", "ftp_plan_set_tuning", "ftp_autotune", "ftp_plan_tune_key",
    "ftp_tune_cache_lookup", "ftp_tune_cache_store", "ftp_periodogram_multiband",
    "ftp_plan_create_bands", "ftp_periodogram_shared_phase", "ftp_root_counts", "ftp_solve_sums_noalloc",
]

FTP_TUNE_FORCE = 1
FTP_E_IO = -11


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("solver", ctypes.c_int), ("nfft_R", ctypes.c_double),
                ("nfft_msp", ctypes.c_int), ("solve_waves", ctypes.c_int), ("flags", ctypes.c_uint)]


class Stats(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_uint64), ("n_fallback", ctypes.c_uint64), ("n_fallback_qr", ctypes.c_uint64),
                ("qr_sweeps", ctypes.c_uint64), ("newton_iters", ctypes.c_uint64), ("roots_found", ctypes.c_uint64),
                ("aberth_iters", ctypes.c_uint64), ("ms_nfft", ctypes.c_double), ("ms_solve", ctypes.c_double),
                ("ms_roots", ctypes.c_double), ("ms_mlp", ctypes.c_double), ("ms_verify", ctypes.c_double),
                ("ms_aberth", ctypes.c_double), ("ms_fallback", ctypes.c_double), ("ms_spread", ctypes.c_double),
                ("ms_fft", ctypes.c_double), ("ms_retry", ctypes.c_double), ("n_fallback_aberth", ctypes.c_uint64)]


class Tuning(ctypes.Structure):
    """Launch shapes of the per-frequency kernels (waves per compute unit)."""
    _fields_ = [("assemble_wpc", ctypes.c_int), ("newton_wpc", ctypes.c_int), ("aberth_wpc", ctypes.c_int),
                ("qr_wpc", ctypes.c_int), ("score_wpc", ctypes.c_int), ("mlp_fused", ctypes.c_int),
                ("newton_occ", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class FtpError(RuntimeError):
    pass


_lib = None


def _init_torch_device():
    """torch ships its own HIP runtime beside the one libftp.so links; the
    first runtime to initialise in a process must be torch's, or torch can
    find no device afterwards.  Initialise it before the library's first
    call when a device is present (device_count() itself initialises
    nothing)."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.device_count() > 0:
        torch.cuda.init()


def load_library(path: Optional[str] = None):
    """Load ``libftp.so`` and declare its C signatures (raises if absent)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    _init_torch_device()
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise FtpError(f"HIP library not built: {p} (run __graft_entry__.build())")
    lib = ctypes.CDLL(p)
    vp, i64, dbl, ip = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.ftp_options_default.argtypes = [ctypes.POINTER(Options)]
    lib.ftp_plan_create.argtypes = [ctypes.POINTER(vp), ip, vp, vp, ctypes.POINTER(Options)]
    lib.ftp_plan_create_bands.argtypes = [ctypes.POINTER(vp), ip, ip, vp, vp, ctypes.POINTER(Options)]
    lib.ftp_periodogram_shared_phase.argtypes = [vp, vp, vp, vp, vp, vp, dbl, i64, vp, vp, vp, vp, vp, vp]
    lib.ftp_plan_destroy.argtypes = [vp]
    lib.ftp_periodogram.argtypes = [vp, vp, vp, vp, i64, dbl, i64, vp, vp, vp, vp, vp, vp]
    lib.ftp_periodogram_batch.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.ftp_nfft_sums.argtypes = [vp, vp, vp, vp, i64, dbl, i64, vp, vp, vp]
    lib.ftp_solve_sums.argtypes = [vp, vp, vp, dbl, i64, vp, vp, vp, vp, vp, vp]
    lib.ftp_root_counts.argtypes = [vp, vp, vp, dbl, i64, vp, vp, vp]
    lib.ftp_solve_sums_noalloc.argtypes = [vp, vp, vp, dbl, i64, vp, vp, vp, vp, vp, vp]
    lib.ftp_plan_load_mlp.argtypes = [vp, vp, i64, ip]
    lib.ftp_last_stats.argtypes = [vp, ctypes.POINTER(Stats), vp]
    lib.ftp_mlp_create.argtypes = [ctypes.POINTER(vp), ip, ip, ip, vp, ctypes.c_uint64]
    lib.ftp_mlp_destroy.argtypes = [vp]
    lib.ftp_mlp_num_params.argtypes = [vp, ctypes.POINTER(i64)]
    lib.ftp_mlp_get_weights.argtypes = [vp, vp, i64]
    lib.ftp_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
    lib.ftp_mlp_loss_grad.argtypes = [vp, vp, i64, vp, vp, ip, ctypes.c_float, vp, vp, vp]
    lib.ftp_mlp_train_step.argtypes = [vp, vp, i64, vp, vp, ip, ctypes.c_float, ctypes.c_float, vp, vp]
    lib.ftp_learned_dataset.argtypes = [vp, vp, vp, vp, i64, dbl, i64, vp, vp, vp, ip, vp]
    lib.ftp_status_string.argtypes = [ip]
    lib.ftp_periodogram_multiband.argtypes = [vp, i64, vp, vp, vp, vp, dbl, i64, vp, vp, vp, vp]
    lib.ftp_plan_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    lib.ftp_plan_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    lib.ftp_autotune.argtypes = [vp, vp, vp, vp, i64, dbl, i64, ctypes.c_char_p, ctypes.c_uint,
                                 ctypes.POINTER(Tuning), vp]
    lib.ftp_plan_tune_key.argtypes = [vp, i64, ctypes.c_char_p, ip]
    lib.ftp_tune_cache_lookup.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(Tuning)]
    lib.ftp_tune_cache_store.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(Tuning)]
    lib.ftp_status_string.restype = ctypes.c_char_p
    lib.ftp_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("ftp_status_string", "ftp_last_error"):
            getattr(lib, name).restype = ip
    if path is None:
        _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        lib = load_library()
        msg = lib.ftp_status_string(rc).decode()
        if rc == -8:
            msg += ": " + lib.ftp_last_error().decode()
        raise FtpError(f"ftp error {rc}: {msg}")


def status_string(code: int) -> str:
    return load_library().ftp_status_string(int(code)).decode()


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(x, dtype, device):
    torch = _torch()
    t = torch.as_tensor(x, dtype=dtype, device=device)
    return t.contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Plan:
    """A plan for one template (c_n, s_n, n = 1..H)."""

    def __init__(self, c, s, precision: int = FTP_FP32_SUMS, solver: int = FTP_SOLVER_PLAIN,
                 nfft_R: float = 2.0, nfft_msp: int = 0, solve_waves: int = 0, flags: int = 0):
        import numpy as np
        self.lib = load_library()
        c = np.ascontiguousarray(c, dtype=np.float64)
        s = np.ascontiguousarray(s, dtype=np.float64)
        if c.shape != s.shape or c.ndim != 1:
            raise ValueError("c and s must be 1-D arrays of equal length")
        self.H = len(c)
        self.c, self.s = c, s
        self.options = self._options(precision, solver, nfft_R, nfft_msp, solve_waves, flags)
        h = ctypes.c_void_p()
        _check(self.lib.ftp_plan_create(ctypes.byref(h), self.H, c.ctypes.data_as(ctypes.c_void_p),
                                         s.ctypes.data_as(ctypes.c_void_p), ctypes.byref(self.options)))
        self.handle = h

    def _options(self, precision, solver, nfft_R, nfft_msp, solve_waves, flags):
        opt = Options()
        self.lib.ftp_options_default(ctypes.byref(opt))
        opt.precision, opt.solver, opt.nfft_R = precision, solver, nfft_R
        opt.nfft_msp, opt.solve_waves, opt.flags = nfft_msp, solve_waves, flags
        return opt

    def close(self):
        if getattr(self, "handle", None):
            self.lib.ftp_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def periodogram(self, t, y, sigma, df: float, n_f: int, device="cuda", stream=None, out=None):
        torch = _torch()
        t = _dev(t, torch.float64, device)
        y = _dev(y, torch.float64, device)
        sigma = _dev(sigma, torch.float64, device)
        if out is None:
            out = self.alloc_outputs(n_f, t.device)
        _check(self.lib.ftp_periodogram(self.handle, _ptr(t), _ptr(y), _ptr(sigma), t.numel(), float(df),
                                        int(n_f), _ptr(out["power"]), _ptr(out["phase"]), _ptr(out["amp"]),
                                        _ptr(out["offset"]), _ptr(out["status"]), _stream_ptr(stream)))
        return out

    @staticmethod
    def alloc_outputs(n, device):
        torch = _torch()
        return dict(power=torch.empty(n, dtype=torch.float64, device=device),
                    phase=torch.empty(n, dtype=torch.float64, device=device),
                    amp=torch.empty(n, dtype=torch.float64, device=device),
                    offset=torch.empty(n, dtype=torch.float64, device=device),
                    status=torch.empty(n, dtype=torch.uint8, device=device))

    def periodogram_batch(self, obs_off, t, y, sigma, df, freq_off, device="cuda", stream=None, out=None):
        import numpy as np
        torch = _torch()
        obs_off = np.ascontiguousarray(obs_off, dtype=np.int64)
        freq_off = np.ascontiguousarray(freq_off, dtype=np.int64)
        df = np.ascontiguousarray(df, dtype=np.float64)
        n_lc = len(df)
        if len(obs_off) != n_lc + 1 or len(freq_off) != n_lc + 1:
            raise ValueError("offsets must have n_lc + 1 entries")
        t = _dev(t, torch.float64, device)
        y = _dev(y, torch.float64, device)
        sigma = _dev(sigma, torch.float64, device)
        if out is None:
            out = self.alloc_outputs(int(freq_off[-1]), t.device)
        _check(self.lib.ftp_periodogram_batch(
            self.handle, n_lc, obs_off.ctypes.data_as(ctypes.c_void_p), _ptr(t), _ptr(y), _ptr(sigma),
            df.ctypes.data_as(ctypes.c_void_p), freq_off.ctypes.data_as(ctypes.c_void_p),
            _ptr(out["power"]), _ptr(out["phase"]), _ptr(out["amp"]), _ptr(out["offset"]),
            _ptr(out["status"]), _stream_ptr(stream)))
        return out

    def nfft_sums(self, t, y, sigma, df: float, n_f: int, device="cuda", stream=None):
        """Returns (sums complex128 tensor (n_f, 3H), stats tensor [t_ref, ybar, YY, status])."""
        torch = _torch()
        t = _dev(t, torch.float64, device)
        y = _dev(y, torch.float64, device)
        sigma = _dev(sigma, torch.float64, device)
        sums = torch.empty((n_f, 3 * self.H, 2), dtype=torch.float64, device=t.device)
        st = torch.empty(4, dtype=torch.float64, device=t.device)
        _check(self.lib.ftp_nfft_sums(self.handle, _ptr(t), _ptr(y), _ptr(sigma), t.numel(), float(df),
                                      int(n_f), _ptr(sums), _ptr(st), _stream_ptr(stream)))
        return torch.view_as_complex(sums), st

    def solve_sums(self, sums, tref: float, ybar: float, yy: float, df: float, device="cuda", stream=None,
                   out=None):
        import numpy as np
        torch = _torch()
        sums = torch.as_tensor(sums, device=device)
        if sums.is_complex():
            sums = torch.view_as_real(sums.to(torch.complex128).contiguous())
        sums = sums.to(torch.float64).contiguous()
        n_f = sums.shape[0]
        if sums.shape[1] != 3 * self.H:
            raise ValueError("sums must have 3H columns")
        stats = np.array([tref, ybar, yy], dtype=np.float64)
        if out is None:
            out = self.alloc_outputs(n_f, sums.device)
        _check(self.lib.ftp_solve_sums(self.handle, _ptr(sums), stats.ctypes.data_as(ctypes.c_void_p),
                                       float(df), int(n_f), _ptr(out["power"]), _ptr(out["phase"]),
                                       _ptr(out["amp"]), _ptr(out["offset"]), _ptr(out["status"]),
                                       _stream_ptr(stream)))
        return out

    def solve_sums_noalloc(self, sums, tref: float, ybar: float, yy: float, df: float, out, stream=None):
        """ftp_solve_sums_noalloc: as solve_sums, into caller-allocated outputs
        (dict as alloc_outputs makes); sums complex128 or (n_f, 3H, 2) float64
        on the device."""
        import numpy as np
        torch = _torch()
        if sums.is_complex():
            sums = torch.view_as_real(sums)
        if sums.dtype != torch.float64 or not sums.is_contiguous() or sums.shape[1] != 3 * self.H:
            raise ValueError("sums must be contiguous float64 (n_f, 3H, 2) on the device")
        n_f = sums.shape[0]
        stats = np.array([tref, ybar, yy], dtype=np.float64)
        _check(self.lib.ftp_solve_sums_noalloc(self.handle, _ptr(sums), stats.ctypes.data_as(ctypes.c_void_p),
                                               float(df), int(n_f), _ptr(out["power"]), _ptr(out["phase"]),
                                               _ptr(out["amp"]), _ptr(out["offset"]), _ptr(out["status"]),
                                               _stream_ptr(stream)))
        return out

    def root_counts(self, sums, tref: float, ybar: float, yy: float, df: float, device="cuda", stream=None):
        """(Sturm count, real companion eigenvalues) per frequency, int32
        tensors, from sums in the layout of nfft_sums (see ftp_root_counts)."""
        import numpy as np
        torch = _torch()
        sums = torch.as_tensor(sums, device=device)
        if sums.is_complex():
            sums = torch.view_as_real(sums.to(torch.complex128).contiguous())
        sums = sums.to(torch.float64).contiguous()
        n_f = sums.shape[0]
        if sums.shape[1] != 3 * self.H:
            raise ValueError("sums must have 3H columns")
        stats = np.array([tref, ybar, yy], dtype=np.float64)
        sc = torch.empty(n_f, dtype=torch.int32, device=sums.device)
        cr = torch.empty(n_f, dtype=torch.int32, device=sums.device)
        _check(self.lib.ftp_root_counts(self.handle, _ptr(sums), stats.ctypes.data_as(ctypes.c_void_p), float(df),
                                        int(n_f), _ptr(sc), _ptr(cr), _stream_ptr(stream)))
        return sc, cr

    def load_mlp(self, weights, width: int):
        import numpy as np
        w = np.ascontiguousarray(weights, dtype=np.float32)
        _check(self.lib.ftp_plan_load_mlp(self.handle, w.ctypes.data_as(ctypes.c_void_p), w.size, int(width)))

    def periodogram_multiband(self, bands, df: float, n_f: int, device="cuda", stream=None):
        """Multi-phase multi-band periodogram of bands [(t, y, sigma), ...]
        sharing the plan's template: dict(power (n_f,), band_power
        (n_band, n_f), chi2_0 (n_band,))."""
        import numpy as np
        torch = _torch()
        obs_off = np.concatenate([[0], np.cumsum([len(b[0]) for b in bands])]).astype(np.int64)
        t = _dev(np.concatenate([np.asarray(b[0], dtype=np.float64) for b in bands]), torch.float64, device)
        y = _dev(np.concatenate([np.asarray(b[1], dtype=np.float64) for b in bands]), torch.float64, device)
        s = _dev(np.concatenate([np.asarray(b[2], dtype=np.float64) for b in bands]), torch.float64, device)
        nb = len(bands)
        power = torch.empty(n_f, dtype=torch.float64, device=t.device)
        bp = torch.empty((nb, n_f), dtype=torch.float64, device=t.device)
        c2 = torch.empty(nb, dtype=torch.float64, device=t.device)
        _check(self.lib.ftp_periodogram_multiband(self.handle, nb, obs_off.ctypes.data_as(ctypes.c_void_p), _ptr(t),
                                                  _ptr(y), _ptr(s), float(df), int(n_f), _ptr(power), _ptr(bp),
                                                  _ptr(c2), _stream_ptr(stream)))
        return dict(power=power, band_power=bp, chi2_0=c2)

    def tuning(self) -> dict:
        tu = Tuning()
        _check(self.lib.ftp_plan_get_tuning(self.handle, ctypes.byref(tu)))
        return tu.as_dict()

    def set_tuning(self, **kw):
        tu = Tuning()
        _check(self.lib.ftp_plan_get_tuning(self.handle, ctypes.byref(tu)))
        names = {k for k, _ in Tuning._fields_}
        for k, v in kw.items():
            if k not in names:
                raise KeyError(f"unknown launch shape {k!r} (one of {sorted(names)})")
            setattr(tu, k, int(v))
        _check(self.lib.ftp_plan_set_tuning(self.handle, ctypes.byref(tu)))

    def tune_key(self, n_f: int) -> str:
        buf = ctypes.create_string_buffer(256)
        _check(self.lib.ftp_plan_tune_key(self.handle, int(n_f), buf, 256))
        return buf.value.decode()

    def autotune(self, t, y, sigma, df: float, n_f: int, cache_path: Optional[str] = None, force: bool = False,
                 device="cuda", stream=None):
        """Tune the launch shapes on one lightcurve; returns (shapes, from_cache)."""
        torch = _torch()
        t = _dev(t, torch.float64, device)
        y = _dev(y, torch.float64, device)
        sigma = _dev(sigma, torch.float64, device)
        tu = Tuning()
        rc = self.lib.ftp_autotune(self.handle, _ptr(t), _ptr(y), _ptr(sigma), t.numel(), float(df), int(n_f),
                                   cache_path.encode() if cache_path else None, FTP_TUNE_FORCE if force else 0,
                                   ctypes.byref(tu), _stream_ptr(stream))
        if rc < 0:
            _check(rc)
        return tu.as_dict(), rc == 1

    def stats(self, stream=None) -> dict:
        st = Stats()
        _check(self.lib.ftp_last_stats(self.handle, ctypes.byref(st), _stream_ptr(stream)))
        return {k: getattr(st, k) for k, _ in Stats._fields_}


    def learned_dataset(self, t, y, sigma, df: float, n_f: int, R: int = 32, device="cuda", stream=None):
        """(X bf16 (n_f, d_in), roots float32 (n_f, R), nroots int32 (n_f,)) from one lightcurve."""
        torch = _torch()
        t = _dev(t, torch.float64, device)
        y = _dev(y, torch.float64, device)
        sigma = _dev(sigma, torch.float64, device)
        din = 2 * (6 * self.H - 1)
        X = torch.empty((n_f, din), dtype=torch.bfloat16, device=t.device)
        roots = torch.zeros((n_f, R), dtype=torch.float32, device=t.device)
        nroots = torch.zeros(n_f, dtype=torch.int32, device=t.device)
        _check(self.lib.ftp_learned_dataset(self.handle, _ptr(t), _ptr(y), _ptr(sigma), t.numel(), float(df),
                                            int(n_f), _ptr(X), _ptr(roots), _ptr(nroots), int(R),
                                            _stream_ptr(stream)))
        return X, roots, nroots


MODELS = os.path.join(HERE, "models")


def load_model(name: str = "single_long_h6"):
    """(FP32 parameters, description) of a trained root-proposal network."""
    import json
    import numpy as np
    base = os.path.join(MODELS, name)
    with open(base + ".json") as fh:
        meta = json.load(fh)
    w = np.fromfile(base + ".f32", dtype=np.float32)
    if w.size != mlp_param_count(meta["d_in"], meta["width"], meta["d_out"]):
        raise FtpError(f"model {name}: parameter file has the wrong size")
    return w, meta


def mlp_param_count(d_in: int, width: int, d_out: int) -> int:
    return d_in * width + width + 2 * (width * width + width) + d_out * width + d_out



class BandsPlan(Plan):
    """A plan for the shared-phase multi-band model (Appendix A): one template
    (c_n, s_n) per band, padded with zeros to the largest H."""

    def __init__(self, templates, precision: int = FTP_FP32_SUMS, solver: int = FTP_SOLVER_PLAIN,
                 nfft_R: float = 2.0, nfft_msp: int = 0, solve_waves: int = 0, flags: int = 0):
        import numpy as np
        self.lib = load_library()
        nb = len(templates)
        H = max(len(np.atleast_1d(c)) for c, _ in templates) if nb else 0
        c = np.zeros((max(nb, 1), max(H, 1)), dtype=np.float64)
        s = np.zeros_like(c)
        for k, (ck, sk) in enumerate(templates):
            ck, sk = np.atleast_1d(np.asarray(ck, dtype=np.float64)), np.atleast_1d(np.asarray(sk, dtype=np.float64))
            if ck.shape != sk.shape or ck.ndim != 1:
                raise ValueError("each template needs 1-D c and s of equal length")
            c[k, : len(ck)], s[k, : len(sk)] = ck, sk
        self.H, self.n_band = H, nb
        self.c, self.s = c, s
        self.options = self._options(precision, solver, nfft_R, nfft_msp, solve_waves, flags)
        h = ctypes.c_void_p()
        _check(self.lib.ftp_plan_create_bands(ctypes.byref(h), nb, H, c.ctypes.data_as(ctypes.c_void_p),
                                               s.ctypes.data_as(ctypes.c_void_p), ctypes.byref(self.options)))
        self.handle = h

    def periodogram_shared_phase(self, bands, df: float, n_f: int, offsets=None, device="cuda", stream=None,
                                 out=None):
        """Shared-phase periodogram of bands [(t, y, sigma), ...] (one per
        template, in order), with fixed band offsets (None = zero); returns
        the outputs of Plan.periodogram."""
        import numpy as np
        torch = _torch()
        obs_off = np.concatenate([[0], np.cumsum([len(b[0]) for b in bands])]).astype(np.int64)
        t = _dev(np.concatenate([np.asarray(b[0], dtype=np.float64) for b in bands]), torch.float64, device)
        y = _dev(np.concatenate([np.asarray(b[1], dtype=np.float64) for b in bands]), torch.float64, device)
        sg = _dev(np.concatenate([np.asarray(b[2], dtype=np.float64) for b in bands]), torch.float64, device)
        if len(bands) != self.n_band:
            raise ValueError("one band of data per template")
        off = None if offsets is None else np.ascontiguousarray(offsets, dtype=np.float64)
        if off is not None and off.shape != (self.n_band,):
            raise ValueError("one offset per band")
        if out is None:
            out = self.alloc_outputs(n_f, t.device)
        _check(self.lib.ftp_periodogram_shared_phase(
            self.handle, obs_off.ctypes.data_as(ctypes.c_void_p), _ptr(t), _ptr(y), _ptr(sg),
            off.ctypes.data_as(ctypes.c_void_p) if off is not None else ctypes.c_void_p(0), float(df), int(n_f),
            _ptr(out["power"]), _ptr(out["phase"]), _ptr(out["amp"]), _ptr(out["offset"]), _ptr(out["status"]),
            _stream_ptr(stream)))
        return out

class Mlp:
    """The root-proposal network on the device (see include/ftp.h)."""

    def __init__(self, d_in: int, width: int, d_out: int, weights=None, seed: int = 0):
        import numpy as np
        self.lib = load_library()
        self.d_in, self.width, self.d_out = d_in, width, d_out
        h = ctypes.c_void_p()
        wp = ctypes.c_void_p(0)
        if weights is not None:
            self._w = np.ascontiguousarray(weights, dtype=np.float32)
            if self._w.size != mlp_param_count(d_in, width, d_out):
                raise ValueError("weight array has the wrong size")
            wp = self._w.ctypes.data_as(ctypes.c_void_p)
        _check(self.lib.ftp_mlp_create(ctypes.byref(h), d_in, width, d_out, wp, ctypes.c_uint64(seed)))
        self.handle = h
        n = ctypes.c_int64()
        _check(self.lib.ftp_mlp_num_params(h, ctypes.byref(n)))
        self.n_params = n.value

    def close(self):
        if getattr(self, "handle", None):
            self.lib.ftp_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def weights(self):
        import numpy as np
        w = np.empty(self.n_params, dtype=np.float32)
        _check(self.lib.ftp_mlp_get_weights(self.handle, w.ctypes.data_as(ctypes.c_void_p), self.n_params))
        return w

    def forward(self, X, stream=None):
        torch = _torch()
        X = X.contiguous()
        assert X.dtype == torch.bfloat16 and X.shape[1] == self.d_in
        out = torch.empty((X.shape[0], self.d_out), dtype=torch.float32, device=X.device)
        _check(self.lib.ftp_mlp_forward(self.handle, _ptr(X), X.shape[0], _ptr(out), _stream_ptr(stream)))
        return out

    def loss_grad(self, X, roots, nroots, lam: float = 0.5, stream=None):
        torch = _torch()
        X, roots, nroots = X.contiguous(), roots.contiguous(), nroots.contiguous()
        B, R = roots.shape
        loss = torch.empty(B, dtype=torch.float32, device=X.device)
        grads = torch.empty(self.n_params, dtype=torch.float32, device=X.device)
        _check(self.lib.ftp_mlp_loss_grad(self.handle, _ptr(X), B, _ptr(roots), _ptr(nroots), R, float(lam),
                                          _ptr(loss), _ptr(grads), _stream_ptr(stream)))
        return loss, grads

    def train_step(self, X, roots, nroots, lr: float, lam: float = 0.5, stream=None, loss=None):
        B, R = roots.shape
        _check(self.lib.ftp_mlp_train_step(self.handle, _ptr(X), B, _ptr(roots), _ptr(nroots), R, float(lam),
                                           float(lr), _ptr(loss) if loss is not None else ctypes.c_void_p(0),
                                           _stream_ptr(stream)))


def tune_cache_lookup(path: str, key: str):
    """The cached launch shapes for `key` (dict), or None."""
    lib = load_library()
    tu = Tuning()
    rc = lib.ftp_tune_cache_lookup(path.encode(), key.encode(), ctypes.byref(tu))
    if rc < 0:
        _check(rc)
    return tu.as_dict() if rc == 1 else None


def tune_cache_store(path: str, key: str, **shapes):
    lib = load_library()
    tu = Tuning(**{k: int(v) for k, v in shapes.items()})
    _check(lib.ftp_tune_cache_store(path.encode(), key.encode(), ctypes.byref(tu)))
