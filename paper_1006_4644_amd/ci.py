"""Python binding of the C-ABI library ``libci.so`` (argument marshalling only).

Every step of the search runs in the library's HIP kernels; this module only
turns torch tensors into device pointers and the current torch stream into a
``hipStream_t``.  Loading fails loudly when the library has not been built:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

__all__ = [
    "load", "LibraryMissing", "CiError", "Library", "Context", "Segment",
    "TRIGGER_DTYPE", "TPARAMS_DTYPE", "FP32", "SPLIT_BF16", "SPLIT_FP16",
    "BANK_GRID", "BANK_UNIFORM", "BANK_LOGUNIFORM", "EXPORTED_SYMBOLS",
    "RUN_GRAPH",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libci.so")

OK, EINVAL, ENOMEM, EHIP, ETRUNC, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
FP32, SPLIT_BF16, SPLIT_FP16 = 0, 1, 2
BANK_GRID, BANK_UNIFORM, BANK_LOGUNIFORM = 0, 1, 2
TMPL_EMPTY = 1

EXPORTED_SYMBOLS = (
    "ci_version", "ci_last_error", "ci_ctx_create", "ci_ctx_destroy",
    "ci_set_batch", "ci_make_bank", "ci_segment_create", "ci_segment_destroy",
    "ci_gen_templates", "ci_matched_filter", "ci_find_triggers",
    "ci_segment_update", "ci_set_timing", "ci_kernel_times",
    "ci_length_classes", "ci_search_classes", "ci_get_tune", "ci_set_tune",
    "ci_autotune", "ci_chisq", "ci_td_params", "ci_td_templates",
    "ci_td_matched_filter", "ci_td_find_triggers", "ci_stream_create",
    "ci_stream_destroy", "ci_stream_push", "ci_stream_poll", "ci_stream_last",
    "ci_bank_metric", "ci_make_bank_lattice", "ci_graph_stats",
    "ci_find_triggers_noalloc", "ci_hbm_probe", "ci_merge_triggers",
)
RUN_GRAPH = 1

# ci_trigger: {int64 tmpl, int64 index, float rho2, re, im, int32 window}
TRIGGER_DTYPE = np.dtype([("tmpl", "<i8"), ("index", "<i8"), ("rho2", "<f4"),
                          ("re", "<f4"), ("im", "<f4"), ("window", "<i4")])
# ci_tparams (96 bytes)
TPARAMS_DTYPE = np.dtype([("m1", "<f8"), ("m2", "<f8"), ("x0", "<f8"),
                          ("c0", "<f8"), ("c2", "<f8"), ("c3", "<f8"),
                          ("c4", "<f8"), ("sigma2", "<f8"), ("tau", "<f8"),
                          ("scale", "<f4"), ("k_low", "<i4"),
                          ("k_high", "<i4"), ("flags", "<i4"),
                          ("reserved", "<i4", (2,))])
# ci_tdparams (176 bytes)
TDPARAMS_DTYPE = np.dtype([("m1", "<f8"), ("m2", "<f8"), ("K", "<f8"),
                           ("tau", "<f8", (4,)), ("r", "<f8", (4,)), ("P", "<f8"),
                           ("p", "<f8", (4,)), ("v_low", "<f8"), ("v_end", "<f8"),
                           ("m_lo", "<i8"), ("m_hi", "<i8"), ("k_low", "<i4"),
                           ("k_high", "<i4"), ("flags", "<i4"), ("reserved", "<i4")])
assert TRIGGER_DTYPE.itemsize == 32 and TPARAMS_DTYPE.itemsize == 96
assert TDPARAMS_DTYPE.itemsize == 176


class LibraryMissing(RuntimeError):
    pass


class CiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ci error {code}: {msg}")
        self.code = code


class ChunkFailure(RuntimeError):
    """Raised by Context.search_bank_chunked's failure injection."""


class _Template(ctypes.Structure):
    _fields_ = [("m1", ctypes.c_double), ("m2", ctypes.c_double)]


class _BankSpec(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("m_min", ctypes.c_double), ("m_max", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class _KernelTime(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("templates", ctypes.c_int64),
                ("ms", ctypes.c_double)]


class _SegSpec(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("fs", ctypes.c_double),
                ("f_low", ctypes.c_double)]


class _ClassJob(ctypes.Structure):
    _fields_ = [("seg", ctypes.c_void_p), ("d_params", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("j_lo", ctypes.c_int64),
                ("j_hi", ctypes.c_int64), ("d_peaks", ctypes.c_void_p),
                ("d_trig", ctypes.c_void_p), ("cap", ctypes.c_int64),
                ("d_count", ctypes.c_void_p)]


class _Tune(ctypes.Structure):
    _fields_ = [("log2n", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("tile_c", ctypes.c_int32), ("tile_j", ctypes.c_int32),
                ("p2_per_cu", ctypes.c_int32), ("tuned", ctypes.c_int32),
                ("batch", ctypes.c_int64), ("ms", ctypes.c_double),
                ("candidates", ctypes.c_int32), ("rejected", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("p2_wave", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp, _i32, _i64, _f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float


class _LatticeSpec(ctypes.Structure):
    _fields_ = [("m_min", ctypes.c_double), ("m_max", ctypes.c_double),
                ("min_match", ctypes.c_double)]


class _StreamSpec(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("fs", ctypes.c_double), ("f_low", ctypes.c_double),
                ("psd_half_width", ctypes.c_int32), ("snr_threshold", ctypes.c_float),
                ("window", ctypes.c_int64), ("cap", ctypes.c_int64),
                ("psd_segments", ctypes.c_int32), ("precision", ctypes.c_int32)]

_SIGS = {
    "ci_version": (ctypes.c_char_p, []),
    "ci_last_error": (ctypes.c_char_p, [_vp]),
    "ci_ctx_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp)]),
    "ci_ctx_destroy": (ctypes.c_int, [_vp]),
    "ci_set_batch": (ctypes.c_int, [_vp, _i64]),
    "ci_make_bank": (ctypes.c_int, [ctypes.POINTER(_BankSpec), _i64, _vp]),
    "ci_segment_create": (ctypes.c_int, [_vp, ctypes.POINTER(_SegSpec), _vp,
                                         _vp, _vp, ctypes.POINTER(_vp)]),
    "ci_segment_destroy": (ctypes.c_int, [_vp]),
    "ci_segment_update": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "ci_set_timing": (ctypes.c_int, [_vp, _i32]),
    "ci_kernel_times": (ctypes.c_int, [_vp, ctypes.POINTER(_KernelTime),
                                       ctypes.POINTER(_KernelTime)]),
    "ci_gen_templates": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _vp, _vp]),
    "ci_matched_filter": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _vp, _vp]),
    "ci_find_triggers": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _f32, _i64,
                                        _i64, _i64, _vp, _vp, _i64, _vp, _i32,
                                        _vp]),
    "ci_find_triggers_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _f32, _i64,
                                                _i64, _i64, _vp, _vp, _i64, _vp, _i32,
                                                _vp]),
    "ci_length_classes": (ctypes.c_int, [_vp, _i64, ctypes.c_double,
                                         ctypes.c_double, _vp, _i32, _vp]),
    "ci_search_classes": (ctypes.c_int, [_vp, ctypes.POINTER(_ClassJob), _i32,
                                         _i32, _f32, _i64, _i32, _i32, _vp]),
    "ci_graph_stats": (ctypes.c_int, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "ci_hbm_probe": (ctypes.c_int, [_vp, _i32, _vp, _i64, _i32,
                                    ctypes.POINTER(ctypes.c_double)]),
    "ci_merge_triggers": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _vp, _i64, _i64, _i64,
                                         _vp, _i64, _vp, _vp]),
    "ci_get_tune": (ctypes.c_int, [_vp, _i32, _i32, ctypes.POINTER(_Tune)]),
    "ci_set_tune": (ctypes.c_int, [_vp, ctypes.POINTER(_Tune)]),
    "ci_autotune": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _f32, _i64,
                                   ctypes.POINTER(_Tune), _vp]),
    "ci_chisq": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _i64, _i32, _vp, _vp]),
    "ci_stream_create": (ctypes.c_int, [_vp, ctypes.POINTER(_StreamSpec), _vp, _i64,
                                        ctypes.POINTER(_vp)]),
    "ci_stream_destroy": (ctypes.c_int, [_vp]),
    "ci_bank_metric": (ctypes.c_int, [_vp, _i64, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, _vp]),
    "ci_make_bank_lattice": (ctypes.c_int, [ctypes.POINTER(_LatticeSpec), _vp, _i64,
                                            ctypes.c_double, ctypes.c_double, _vp, _i64,
                                            ctypes.POINTER(_i64)]),
    "ci_stream_push": (ctypes.c_int, [_vp, _vp, _i64]),
    "ci_stream_poll": (ctypes.c_int, [_vp, _i32, _vp, _i64, ctypes.POINTER(_i64),
                                      ctypes.POINTER(_i64), ctypes.POINTER(_i32)]),
    "ci_stream_last": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(_i64)]),
    "ci_td_params": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _vp]),
    "ci_td_templates": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp]),
    "ci_td_matched_filter": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _vp]),
    "ci_td_find_triggers": (ctypes.c_int, [_vp, _vp, _vp, _i64, _f32, _i64, _i64, _i64,
                                           _vp, _vp, _i64, _vp, _i32, _vp]),
}

_LIB = None


def load(path: str | None = None) -> "Library":
    """Load libci.so (built in-tree by ``paper_1006_4644_amd.build``)."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise LibraryMissing(
            f"{p} not found: build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = Library(ctypes.CDLL(p))
    if path is None:
        _LIB = lib
    return lib


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Library:
    """Thin wrapper over the exported C functions."""

    def __init__(self, dll):
        self.dll = dll
        for name, (res, args) in _SIGS.items():
            f = getattr(dll, name)
            f.restype = res
            f.argtypes = args

    def version(self) -> str:
        return self.dll.ci_version().decode()

    def check(self, rc, ctx=None):
        if rc != OK:
            msg = self.dll.ci_last_error(ctx)
            raise CiError(rc, msg.decode() if msg else "")

    def make_bank(self, kind: int, m_min: float, m_max: float, seed: int,
                  n: int) -> np.ndarray:
        out = np.empty((n, 2), dtype=np.float64)
        spec = _BankSpec(kind, 0, m_min, m_max, seed)
        rc = self.dll.ci_make_bank(ctypes.byref(spec), n,
                                   out.ctypes.data if n else None)
        self.check(rc)
        return out

    def bank_metric(self, psd, n: int, fs: float, f_low: float, m1: float, m2: float):
        """Metric gamma (2 x 2) in (tau_0, tau_3) at (m1, m2) (host only)."""
        psd = np.ascontiguousarray(np.asarray(psd, dtype=np.float64))
        g = np.zeros(3)
        self.check(self.dll.ci_bank_metric(psd.ctypes.data, n, fs, f_low, m1, m2, g.ctypes.data))
        return np.array([[g[0], g[1]], [g[1], g[2]]])

    def make_bank_lattice(self, m_min: float, m_max: float, min_match: float, psd, n: int,
                          fs: float, f_low: float) -> np.ndarray:
        """(count, 2) float64 bank of (m1, m2) covering the mass range at
        min_match (host only)."""
        psd = np.ascontiguousarray(np.asarray(psd, dtype=np.float64))
        spec = _LatticeSpec(m_min, m_max, min_match)
        cnt = _i64()
        self.check(self.dll.ci_make_bank_lattice(ctypes.byref(spec), psd.ctypes.data, n, fs,
                                                 f_low, None, 0, ctypes.byref(cnt)))
        out = np.zeros((max(cnt.value, 1), 2))
        self.check(self.dll.ci_make_bank_lattice(ctypes.byref(spec), psd.ctypes.data, n, fs,
                                                 f_low, out.ctypes.data, cnt.value,
                                                 ctypes.byref(cnt)))
        return out[:cnt.value]

    def length_classes(self, bank, fs: float, f_low: float, classes) -> np.ndarray:
        """Class index per template: the shortest of `classes` (increasing
        powers of two) whose duration covers the 2PN chirp from f_low."""
        bank = np.ascontiguousarray(np.asarray(bank, dtype=np.float64).reshape(-1, 2))
        cl = np.ascontiguousarray(np.asarray(classes, dtype=np.int64))
        out = np.empty(bank.shape[0], dtype=np.int32)
        rc = self.dll.ci_length_classes(
            bank.ctypes.data if len(bank) else None, len(bank), fs, f_low,
            cl.ctypes.data, len(cl), out.ctypes.data if len(bank) else None)
        self.check(rc)
        return out

    def context(self, device: int = 0) -> "Context":
        return Context(self, device)


class Segment:
    def __init__(self, ctx: "Context", handle: int, n: int, fs: float,
                 f_low: float):
        self.ctx, self.handle, self.n, self.fs, self.f_low = ctx, handle, n, fs, f_low

    def close(self):
        if self.handle:
            self.ctx.lib.dll.ci_segment_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Stream:
    """A ci_stream: overlap-save search of a continuous float32 strain
    stream (segments of n samples, stride n/2, valid half searched)."""

    def __init__(self, ctx: "Context", handle: int, spec):
        self.ctx, self.handle, self.spec = ctx, handle, spec

    def push(self, x):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float32).reshape(-1))
        self.ctx._chk(self.ctx.lib.dll.ci_stream_push(self.handle, x.ctypes.data, x.size))

    def poll(self, wait: bool = False, cap: int = 1 << 16):
        """(structured trigger array, segments collected, flags)."""
        out = np.zeros(max(cap, 1), dtype=TRIGGER_DTYPE)
        k, segs, fl = _i64(), _i64(), _i32()
        self.ctx._chk(self.ctx.lib.dll.ci_stream_poll(
            self.handle, 1 if wait else 0, out.ctypes.data, cap, ctypes.byref(k),
            ctypes.byref(segs), ctypes.byref(fl)))
        return out[:k.value].copy(), segs.value, fl.value

    def last(self):
        """(spectrum complex64 [n/2+1], PSD float64 [n/2+1], segment index)
        of the last segment processed (blocking)."""
        import torch
        m = self.spec.n // 2 + 1
        dev = torch.device("cuda", self.ctx.device)
        xt = torch.empty(m, dtype=torch.complex64, device=dev)
        ps = torch.empty(m, dtype=torch.float64, device=dev)
        seg = _i64()
        self.ctx._chk(self.ctx.lib.dll.ci_stream_last(self.handle, _ptr(xt), _ptr(ps),
                                                      ctypes.byref(seg)))
        return xt.cpu().numpy(), ps.cpu().numpy(), seg.value

    def close(self):
        if self.handle:
            self.ctx.lib.dll.ci_stream_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """A ci_ctx; device memory comes from torch tensors on `cuda:device`."""

    def __init__(self, lib: Library, device: int = 0):
        self.lib = lib
        self.device = device
        h = _vp()
        lib.check(lib.dll.ci_ctx_create(device, ctypes.byref(h)))
        self.handle = h.value

    def close(self):
        if self.handle:
            self.lib.dll.ci_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        self.lib.check(rc, self.handle)

    def set_batch(self, b: int):
        self._chk(self.lib.dll.ci_set_batch(self.handle, b))

    def segment(self, xtilde, psd, n: int, fs: float, f_low: float,
                stream=None) -> Segment:
        """xtilde: complex64 CUDA tensor [n/2+1]; psd: float64 CUDA [n/2+1]."""
        import torch
        assert xtilde.dtype == torch.complex64 and xtilde.is_cuda
        assert psd.dtype == torch.float64 and psd.is_cuda
        assert xtilde.numel() == n // 2 + 1 and psd.numel() == n // 2 + 1
        xtilde = xtilde.contiguous()
        psd = psd.contiguous()
        spec = _SegSpec(n, fs, f_low)
        h = _vp()
        self._chk(self.lib.dll.ci_segment_create(
            self.handle, ctypes.byref(spec), _ptr(xtilde), _ptr(psd),
            _stream(stream), ctypes.byref(h)))
        return Segment(self, h.value, n, fs, f_low)

    def segment_update(self, seg: Segment, xtilde, psd, stream=None):
        """Recompute `seg` in place from new data (same grid)."""
        self._chk(self.lib.dll.ci_segment_update(
            seg.handle, _ptr(xtilde), _ptr(psd), _stream(stream)))

    def set_timing(self, on: bool):
        self._chk(self.lib.dll.ci_set_timing(self.handle, 1 if on else 0))

    def kernel_times(self):
        """{'pass1': (launches, templates, ms), 'pass2': (...)} since the
        last call; waits for the recorded events."""
        a, b = _KernelTime(), _KernelTime()
        self._chk(self.lib.dll.ci_kernel_times(self.handle, ctypes.byref(a),
                                               ctypes.byref(b)))
        return {"pass1": (a.launches, a.templates, a.ms),
                "pass2": (b.launches, b.templates, b.ms)}

    def gen_templates(self, seg: Segment, bank, htilde: bool = False,
                      stream=None, out=None):
        """Generator constants (uint8 CUDA tensor [n, 96]) for a (n, 2)
        bank; with htilde=True also the templates (complex64 [n, N/2+1])."""
        import torch
        bank = np.ascontiguousarray(np.asarray(bank, dtype=np.float64).reshape(-1, 2))
        n = bank.shape[0]
        dev = torch.device("cuda", self.device)
        params = out if out is not None else torch.empty(
            (max(n, 1), 96), dtype=torch.uint8, device=dev)
        ht = None
        if htilde:
            ht = torch.empty((max(n, 1), seg.n // 2 + 1), dtype=torch.complex64,
                             device=dev)
        self._chk(self.lib.dll.ci_gen_templates(
            self.handle, seg.handle, bank.ctypes.data if n else None, n,
            _ptr(params), _ptr(ht), _stream(stream)))
        return (params, ht) if htilde else params

    def matched_filter(self, seg: Segment, params, n: int | None = None,
                       precision: int = FP32, out=None, stream=None):
        """Complex SNR series z/sigma, complex64 [n, N]."""
        import torch
        n = params.shape[0] if n is None else n
        if out is None:
            out = torch.empty((max(n, 1), seg.n), dtype=torch.complex64,
                              device=params.device)
        self._chk(self.lib.dll.ci_matched_filter(
            self.handle, seg.handle, _ptr(params), n, precision, _ptr(out),
            _stream(stream)))
        return out

    def find_triggers(self, seg: Segment, params, thr: float, window: int,
                      n: int | None = None, j_lo: int = 0, j_hi: int = 0,
                      cap: int = 1 << 16, merge: bool = False,
                      precision: int = FP32, peaks=None, trig=None,
                      count=None, stream=None):
        """Enqueue the search; returns the device tensors (peaks [n, 4] int64
        rows of ci_trigger, trig [cap, 4], count [1] int64)."""
        import torch
        n = params.shape[0] if n is None else n
        dev = params.device
        if peaks is None:
            peaks = torch.empty((max(n, 1), 4), dtype=torch.int64, device=dev)
        if trig is None:
            trig = torch.empty((max(cap, 1), 4), dtype=torch.int64, device=dev)
        if count is None:
            count = torch.zeros(1, dtype=torch.int64, device=dev)
        self._chk(self.lib.dll.ci_find_triggers(
            self.handle, seg.handle, _ptr(params), n, precision, float(thr),
            window, j_lo, j_hi, _ptr(peaks), _ptr(trig), cap, _ptr(count),
            1 if merge else 0, _stream(stream)))
        return peaks, trig, count


    def find_triggers_noalloc(self, seg: Segment, params, thr: float, window: int,
                              peaks, trig, count, n: int | None = None, j_lo: int = 0,
                              j_hi: int = 0, merge: bool = False, precision: int = FP32,
                              stream=None):
        """The search without allocation (the library's fixed scratch): the
        caller passes every output tensor; returns them."""
        n = params.shape[0] if n is None else n
        cap = trig.shape[0]
        self._chk(self.lib.dll.ci_find_triggers_noalloc(
            self.handle, seg.handle, _ptr(params), n, precision, float(thr),
            window, j_lo, j_hi, _ptr(peaks), _ptr(trig), cap, _ptr(count),
            1 if merge else 0, _stream(stream)))
        return peaks, trig, count

    def get_tune(self, log2n: int, precision: int = FP32) -> dict:
        t = _Tune()
        self._chk(self.lib.dll.ci_get_tune(self.handle, log2n, precision,
                                           ctypes.byref(t)))
        return t.as_dict()

    def set_tune(self, log2n: int, precision: int = FP32, tile_c: int = 8,
                 tile_j: int = 4, p2_per_cu: int = 2, batch: int = 0, streams: int = 2,
                 p2_wave: int = 0):
        t = _Tune(log2n, precision, tile_c, tile_j, p2_per_cu, 0, batch)
        t.streams = streams
        t.p2_wave = p2_wave
        self._chk(self.lib.dll.ci_set_tune(self.handle, ctypes.byref(t)))

    def autotune(self, seg: Segment, params, thr: float, window: int,
                 n: int | None = None, precision: int = FP32, stream=None) -> dict:
        """Choose and store the fastest launch configuration for the
        segment's length (blocking); returns it."""
        n = params.shape[0] if n is None else n
        t = _Tune()
        self._chk(self.lib.dll.ci_autotune(
            self.handle, seg.handle, _ptr(params), n, precision, float(thr),
            window, ctypes.byref(t), _stream(stream)))
        return t.as_dict()

    def chisq(self, seg: Segment, params, trig, n_trig: int | None = None,
              bands: int = 16, n: int | None = None, out=None, stream=None):
        """Chi-squared veto at trigger samples: trig is a (m, 4) int64 device
        tensor of ci_trigger rows; returns float64 [n_trig] (NaN for an
        invalid or empty entry)."""
        import torch
        n = params.shape[0] if n is None else n
        n_trig = trig.shape[0] if n_trig is None else n_trig
        if out is None:
            out = torch.empty(max(n_trig, 1), dtype=torch.float64, device=trig.device)
        self._chk(self.lib.dll.ci_chisq(
            self.handle, seg.handle, _ptr(params), n, _ptr(trig), n_trig, bands,
            _ptr(out), _stream(stream)))
        return out[:n_trig]

    def stream(self, bank, n: int, fs: float, f_low: float, thr: float, window: int,
               psd_half_width: int = 16, cap: int = 1 << 12, psd_segments: int = 1,
               precision: int = FP32) -> Stream:
        bank = np.ascontiguousarray(np.asarray(bank, dtype=np.float64).reshape(-1, 2))
        spec = _StreamSpec(n, fs, f_low, psd_half_width, thr, window, cap, psd_segments,
                           precision)
        h = _vp()
        self._chk(self.lib.dll.ci_stream_create(self.handle, ctypes.byref(spec),
                                                bank.ctypes.data, bank.shape[0],
                                                ctypes.byref(h)))
        return Stream(self, h.value, spec)

    # --- the paper's two-polarization (time-domain) template form ---------

    def td_params(self, seg: Segment, bank, stream=None, out=None):
        """Time-domain template constants (uint8 CUDA tensor [n, 176]) for a
        (n, 2) bank."""
        import torch
        bank = np.ascontiguousarray(np.asarray(bank, dtype=np.float64).reshape(-1, 2))
        n = bank.shape[0]
        dev = torch.device("cuda", self.device)
        tdp = out if out is not None else torch.empty(
            (max(n, 1), TDPARAMS_DTYPE.itemsize), dtype=torch.uint8, device=dev)
        self._chk(self.lib.dll.ci_td_params(
            self.handle, seg.handle, bank.ctypes.data, n, _ptr(tdp), _stream(stream)))
        return tdp

    def td_templates(self, seg: Segment, tdp, n: int | None = None, u: bool = True,
                     hf: bool = True, sigma2: bool = True, stream=None):
        """(u [n, N] complex64 or None, hf [n, 2, N/2+1] complex64 or None,
        sigma2 [n, 2] float64 or None)."""
        import torch
        n = tdp.shape[0] if n is None else n
        dev = tdp.device
        N = seg.n
        ou = torch.empty((max(n, 1), N), dtype=torch.complex64, device=dev) if u else None
        oh = torch.empty((max(n, 1), 2, N // 2 + 1), dtype=torch.complex64,
                         device=dev) if hf else None
        os_ = torch.empty((max(n, 1), 2), dtype=torch.float64, device=dev) if sigma2 else None
        self._chk(self.lib.dll.ci_td_templates(
            self.handle, seg.handle, _ptr(tdp), n, _ptr(ou) if u else None,
            _ptr(oh) if hf else None, _ptr(os_) if sigma2 else None, _stream(stream)))
        return ou, oh, os_

    def td_matched_filter(self, seg: Segment, tdp, n: int | None = None, out=None,
                          stream=None):
        """c_+ + i c_x per template, complex64 [n, N]."""
        import torch
        n = tdp.shape[0] if n is None else n
        if out is None:
            out = torch.empty((max(n, 1), seg.n), dtype=torch.complex64, device=tdp.device)
        self._chk(self.lib.dll.ci_td_matched_filter(
            self.handle, seg.handle, _ptr(tdp), n, _ptr(out), _stream(stream)))
        return out

    def td_find_triggers(self, seg: Segment, tdp, thr: float, window: int,
                         n: int | None = None, j_lo: int = 0, j_hi: int = 0,
                         cap: int = 1 << 16, merge: bool = False, peaks=None, trig=None,
                         count=None, stream=None):
        """Search with the two-polarization statistic; returns (peaks, trig,
        count) device tensors as find_triggers."""
        import torch
        n = tdp.shape[0] if n is None else n
        dev = tdp.device
        if peaks is None:
            peaks = torch.empty((max(n, 1), 4), dtype=torch.int64, device=dev)
        if trig is None:
            trig = torch.empty((max(cap, 1), 4), dtype=torch.int64, device=dev)
        if count is None:
            count = torch.zeros(1, dtype=torch.int64, device=dev)
        self._chk(self.lib.dll.ci_td_find_triggers(
            self.handle, seg.handle, _ptr(tdp), n, float(thr), window, j_lo, j_hi,
            _ptr(peaks), _ptr(trig), cap, _ptr(count), 1 if merge else 0, _stream(stream)))
        return peaks, trig, count

    def search_classes(self, jobs, thr: float, window: int, merge: bool = False,
                       precision: int = FP32, graph: bool = False, stream=None):
        """Multi-class search.  jobs: list of dicts with keys seg, params
        and optionally n, j_lo, j_hi, cap, peaks, trig, count (device
        tensors are allocated when absent).  Returns [(peaks, trig, count)]
        per job."""
        import torch
        arr = (_ClassJob * max(len(jobs), 1))()
        outs = []
        for i, jb in enumerate(jobs):
            params = jb["params"]
            n = jb.get("n", params.shape[0])
            cap = jb.get("cap", 1 << 16)
            dev = params.device
            peaks = jb.get("peaks")
            if peaks is None:
                peaks = torch.empty((max(n, 1), 4), dtype=torch.int64, device=dev)
            trig = jb.get("trig")
            if trig is None:
                trig = torch.empty((max(cap, 1), 4), dtype=torch.int64, device=dev)
            count = jb.get("count")
            if count is None:
                count = torch.zeros(1, dtype=torch.int64, device=dev)
            arr[i] = _ClassJob(jb["seg"].handle, _ptr(params), n, jb.get("j_lo", 0),
                               jb.get("j_hi", 0), _ptr(peaks), _ptr(trig), cap,
                               _ptr(count))
            outs.append((peaks, trig, count))
        self._chk(self.lib.dll.ci_search_classes(
            self.handle, arr, len(jobs), precision, float(thr), window,
            1 if merge else 0, RUN_GRAPH if graph else 0, _stream(stream)))
        return outs

    def merge_triggers(self, a, count_a, b, count_b, nwin: int, tmpl_offset_b: int = 0,
                       out=None, count=None, stream=None):
        """Merge two per-window trigger lists (rows of ci_trigger, device)
        into out (default: a new tensor of nwin rows); returns (out, count)."""
        import torch
        if out is None:
            out = torch.empty((max(nwin, 1), 4), dtype=torch.int64, device=a.device)
        if count is None:
            count = torch.zeros(1, dtype=torch.int64, device=a.device)
        self._chk(self.lib.dll.ci_merge_triggers(
            self.handle, _ptr(a), _ptr(count_a), a.shape[0], _ptr(b), _ptr(count_b),
            b.shape[0], tmpl_offset_b, nwin, _ptr(out), out.shape[0], _ptr(count),
            _stream(stream)))
        return out, count

    def search_bank_chunked(self, seg: "Segment", bank, thr: float, window: int, chunk: int,
                            checkpoint: str | None = None, precision: int = FP32,
                            fail_after: int | None = None):
        """The whole bank searched in chunks of `chunk` templates with a
        resumable cursor: per chunk its generator constants, the merged
        search (peaks with bank-wide template ids) and the device merge
        into the running per-window list.  With `checkpoint`, the cursor,
        the peaks so far and the merged list are written after every chunk
        (npz, replaced atomically), and a call that finds the file resumes
        after its cursor.  fail_after=k raises ChunkFailure after k chunks
        of this call (tests of the resume).  Returns (peaks [nt, 4], merged
        [nwin, 4], count [1]) as device tensors; the same results as one
        ci_find_triggers call over the bank with merging."""
        import torch
        if chunk < 1:
            raise ValueError(f"chunk must be >= 1 (got {chunk})")
        bank = np.ascontiguousarray(bank, dtype=np.float64)
        nt, n = len(bank), seg.n
        nwin = (n + window - 1) // window
        dev = torch.device("cuda", self.device)
        i64 = torch.int64
        peaks = torch.empty((max(nt, 1), 4), dtype=i64, device=dev)
        merged = torch.empty((nwin, 4), dtype=i64, device=dev)
        mcount = torch.zeros(1, dtype=i64, device=dev)
        cursor = 0
        meta = np.array([n, nt, window, chunk, precision, seg.fs, seg.f_low, thr],
                        dtype=np.float64)
        if checkpoint and os.path.exists(checkpoint):
            with np.load(checkpoint, allow_pickle=False) as z:
                if not np.array_equal(z["meta"], meta):
                    raise ValueError(f"{checkpoint} belongs to another search")
                cursor = int(z["cursor"])
                if cursor > 0:
                    peaks[:cursor] = torch.from_numpy(z["peaks"][:cursor]).to(dev)
                m = z["merged"]
                if len(m):
                    merged[:len(m)] = torch.from_numpy(m).to(dev)
                mcount.fill_(len(m))
        params = torch.empty((max(min(chunk, nt), 1), 96), dtype=torch.uint8, device=dev)
        ctrig = torch.empty((nwin, 4), dtype=i64, device=dev)
        ccount = torch.zeros(1, dtype=i64, device=dev)
        done = 0
        for c0 in range(cursor, nt, chunk):
            c1 = min(nt, c0 + chunk)
            m = c1 - c0
            self.gen_templates(seg, bank[c0:c1], out=params[:m])
            self.find_triggers(seg, params, thr, window, n=m, cap=nwin, merge=True,
                               peaks=peaks[c0:c1], trig=ctrig, count=ccount,
                               precision=precision)
            peaks[c0:c1, 0] += c0   # template ids of the chunk -> bank indices
            self.merge_triggers(merged, mcount, ctrig, ccount, nwin, tmpl_offset_b=c0,
                                out=merged, count=mcount)
            done += 1
            if checkpoint:
                torch.cuda.synchronize(dev)
                k = int(mcount.cpu()[0])
                tmp = f"{checkpoint}.tmp{os.getpid()}.npz"
                np.savez(tmp, meta=meta, cursor=np.int64(c1),
                         peaks=peaks[:c1].cpu().numpy(), merged=merged[:k].cpu().numpy())
                os.replace(tmp, checkpoint)
            if fail_after is not None and done >= fail_after and c1 < nt:
                raise ChunkFailure(f"injected failure after {done} chunks (cursor {c1})")
        return peaks[:nt], merged, mcount

    def hbm_probe(self, kind: int, buf, nbytes: int, reps: int = 10) -> float:
        """Streaming bandwidth in GB/s: kind 0 write, 1 read, 2 copy (buf holds
        2 x nbytes for a copy)."""
        g = ctypes.c_double(0.0)
        self._chk(self.lib.dll.ci_hbm_probe(self.handle, kind, _ptr(buf), nbytes, reps,
                                            ctypes.byref(g)))
        return float(g.value)

    def graph_stats(self):
        """(graphs captured, graph launches) of CI_RUN_GRAPH searches."""
        c, n = _i64(0), _i64(0)
        self._chk(self.lib.dll.ci_graph_stats(self.handle, ctypes.byref(c), ctypes.byref(n)))
        return int(c.value), int(n.value)


# --- launch-configuration cache ------------------------------------------------
# Autotuned launch configurations as JSON, keyed by the device they were
# tuned on, the transform length and the precision:
#   {"entries": {"<device key>/<log2 n>/<precision>": {tile_c, tile_j, ...}}}
TUNE_FIELDS = ("tile_c", "tile_j", "p2_per_cu", "batch", "streams", "p2_wave")


def device_key(device: int = 0) -> str:
    """Identity of a GPU for the cache: name, architecture, compute units."""
    import torch
    p = torch.cuda.get_device_properties(device)
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|{p.multi_processor_count}"


def save_tune_cache(ctx, path: str, key: str, lengths=range(16, 22),
                    precisions=(FP32, SPLIT_BF16, SPLIT_FP16)) -> int:
    """Merge ctx's autotuned configurations into the cache file (written
    atomically); returns the number of entries written for `key`."""
    data = {"entries": {}}
    if os.path.exists(path):
        with open(path) as fh:
            data = json.load(fh)
        data.setdefault("entries", {})
    n = 0
    for l2 in lengths:
        for p in precisions:
            t = ctx.get_tune(l2, p)
            if t["tuned"]:
                data["entries"][f"{key}/{l2}/{p}"] = {f: int(t[f]) for f in TUNE_FIELDS}
                n += 1
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return n


def load_tune_cache(ctx, path: str, key: str) -> list:
    """Apply the cached configurations recorded for `key` to ctx; returns
    the (log2 n, precision) pairs applied (none if the file is absent)."""
    if not os.path.exists(path):
        return []
    with open(path) as fh:
        data = json.load(fh)
    done = []
    for k, cfg in sorted(data.get("entries", {}).items()):
        dk, l2, p = k.rsplit("/", 2)
        if dk != key:
            continue
        ctx.set_tune(int(l2), int(p), cfg["tile_c"], cfg["tile_j"], cfg["p2_per_cu"],
                     cfg["batch"], streams=cfg["streams"], p2_wave=cfg.get("p2_wave", 0))
        done.append((int(l2), int(p)))
    return done


def triggers_to_numpy(t, count: int | None = None) -> np.ndarray:
    """View ci_trigger rows of a (m, 4) int64 tensor as a structured array."""
    a = t.detach().cpu().numpy().view(TRIGGER_DTYPE).reshape(-1)
    return a if count is None else a[:count]


def params_to_numpy(p) -> np.ndarray:
    return p.detach().cpu().numpy().view(TPARAMS_DTYPE).reshape(-1)


def tdparams_to_numpy(p) -> np.ndarray:
    return p.detach().cpu().numpy().view(TDPARAMS_DTYPE).reshape(-1)
