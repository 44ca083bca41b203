"""Python binding of the MI355X Fourier-domain acceleration search library.

Argument marshalling only: every step of the search runs in the HIP kernels of
libfdas.so (built in-tree by ``paper_1912_12807_amd.build``). PyTorch provides
device memory and the current stream. There is no fallback: if the library
is missing, ``load()`` raises.

    import paper_1912_12807_amd as fdas
    cands = fdas.search(x, tsamp, zmax, dz, numharm, sigma)   # x: cuda float32 [B][N]
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdas.so")

FDAS_OK, FDAS_E_INVAL, FDAS_E_NOMEM, FDAS_E_DEVICE, FDAS_E_TRUNC, FDAS_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
NORM_MEDIAN, NORM_FIXED, NORM_LOCAL = 0, 1, 2

EXPORTED = (
    "fdas_plan_opts_default", "fdas_plan_create", "fdas_plan_destroy", "fdas_search", "fdas_plane",
    "fdas_harmsum", "fdas_spectrum", "fdas_geometry", "fdas_threshold", "fdas_sigma",
    "fdas_template_taps", "fdas_status_string", "fdas_last_error", "fdas_profile_read",
    "fdas_plan_get_info", "fdas_search_ragged", "fdas_tuning_export", "fdas_tuning_import",
    "fdas_refine_eval", "fdas_refine_grad", "fdas_refine", "fdas_refine_window", "fdas_dedisperse",
    "fdas_sift", "fdas_spectrum_noalloc",
)
PHASES = ("rfft", "normalise", "plane", "harmsum", "compact", "sigma", "copyout", "refine", "dedisperse")


class PlanOpts(ctypes.Structure):
    _fields_ = [("flo_hz", ctypes.c_double), ("K", ctypes.c_int32), ("norm", ctypes.c_int32),
                ("fixed_var", ctypes.c_double), ("max_workspace_bytes", ctypes.c_int64),
                ("max_candidates", ctypes.c_int64), ("seg_len", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("harm_order", ctypes.c_int32),
                ("harm_bound", ctypes.c_int32), ("harm_block", ctypes.c_int32),
                ("harm_pair", ctypes.c_int32), ("autotune", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("fail_alloc", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("seg_len", ctypes.c_int32), ("mseg", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("chunk_series", ctypes.c_int32), ("workspace_bytes", ctypes.c_int64),
                ("harm_blocks", ctypes.c_int32), ("harm_pair", ctypes.c_int32)]


CAND_DTYPE = np.dtype([("series", "<i4"), ("harm", "<i4"), ("r_idx", "<i8"), ("z_idx", "<i4"),
                       ("power", "<f4"), ("sigma", "<f8"), ("r_fund", "<f8"), ("z_fund", "<f8"),
                       ("f_hz", "<f8"), ("fdot_hz_s", "<f8")], align=True)
assert CAND_DTYPE.itemsize == 64
SIFTED_DTYPE = np.dtype([("index", "<i8"), ("hits", "<i4"), ("series_lo", "<i4"), ("series_hi", "<i4"),
                         ("reserved", "<i4")])
assert SIFTED_DTYPE.itemsize == 24
DM_RANGE_DTYPE = np.dtype([("dm_start", "<f8"), ("dm_step", "<f8"), ("ndm", "<i4"), ("downsamp", "<i4")])
assert DM_RANGE_DTYPE.itemsize == 24
REFINE_DTYPE = np.dtype([("series", "<i4"), ("m", "<i4"), ("k0", "<i8"), ("r", "<f8"), ("z", "<f8")])
assert REFINE_DTYPE.itemsize == 32


class FdasError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


_lib = None


def load(path: Optional[str] = None):
    """Load libfdas.so (raises if it has not been built) and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("FDAS_LIB_PATH") or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1912_12807_amd.build.build()")
    lib = ctypes.CDLL(path)
    c = ctypes
    P = c.c_void_p
    lib.fdas_plan_opts_default.argtypes = [c.POINTER(PlanOpts)]
    lib.fdas_plan_opts_default.restype = None
    lib.fdas_plan_create.argtypes = [c.POINTER(P), c.c_int64, c.c_int32, c.c_double, c.c_double,
                                     c.c_int32, c.POINTER(PlanOpts)]
    lib.fdas_plan_create.restype = c.c_int
    lib.fdas_plan_destroy.argtypes = [P]
    lib.fdas_plan_destroy.restype = None
    search_args = [P, P, c.c_int64, c.c_int32, c.c_double, c.c_double, c.c_double, c.c_int32,
                   c.c_double, P, c.c_int64, c.POINTER(c.c_int64), P]
    lib.fdas_search.argtypes = search_args
    lib.fdas_search.restype = c.c_int
    lib.fdas_harmsum.argtypes = search_args
    lib.fdas_harmsum.restype = c.c_int
    lib.fdas_plane.argtypes = [P, P, c.c_int64, c.c_int32, c.c_double, c.c_double, c.c_double, P,
                               c.c_int64, P]
    lib.fdas_plane.restype = c.c_int
    lib.fdas_spectrum.argtypes = [P, P, c.c_int64, c.c_int32, P, c.POINTER(c.c_double), P]
    lib.fdas_spectrum.restype = c.c_int
    lib.fdas_geometry.argtypes = [c.c_int64, c.c_double, c.c_double, c.c_double, c.POINTER(PlanOpts),
                                  c.POINTER(c.c_int64), c.POINTER(c.c_int64), c.POINTER(c.c_int32)]
    lib.fdas_geometry.restype = c.c_int
    lib.fdas_threshold.argtypes = [c.c_int32, c.c_double]
    lib.fdas_threshold.restype = c.c_double
    lib.fdas_sigma.argtypes = [c.c_int32, c.c_double]
    lib.fdas_sigma.restype = c.c_double
    lib.fdas_template_taps.argtypes = [c.c_double, c.c_int32, c.c_int32, c.POINTER(c.c_double),
                                       c.POINTER(c.c_double), c.c_int32, c.POINTER(c.c_int32),
                                       c.POINTER(c.c_int32)]
    lib.fdas_template_taps.restype = c.c_int
    lib.fdas_status_string.argtypes = [c.c_int]
    lib.fdas_status_string.restype = c.c_char_p
    lib.fdas_last_error.argtypes = [P]
    lib.fdas_last_error.restype = c.c_char_p
    lib.fdas_profile_read.argtypes = [P, c.POINTER(c.c_double), c.POINTER(c.c_int64), c.c_int32]
    lib.fdas_profile_read.restype = c.c_int
    lib.fdas_plan_get_info.argtypes = [P, c.POINTER(PlanInfo)]
    lib.fdas_plan_get_info.restype = c.c_int
    lib.fdas_search_ragged.argtypes = [P, P, c.POINTER(c.c_int64), c.POINTER(c.c_int64),
                                       c.POINTER(c.c_double), c.POINTER(c.c_double), c.c_int32,
                                       c.c_double, c.c_int32, c.c_double, P, c.c_int64,
                                       c.POINTER(c.c_int64), P]
    lib.fdas_search_ragged.restype = c.c_int
    lib.fdas_tuning_export.argtypes = [P, c.c_char_p, c.c_int64, c.POINTER(c.c_int64)]
    lib.fdas_tuning_export.restype = c.c_int
    lib.fdas_tuning_import.argtypes = [P, c.c_char_p]
    lib.fdas_tuning_import.restype = c.c_int
    lib.fdas_refine_eval.argtypes = [P, c.c_int64, c.c_int64, c.c_int32, P, P, c.c_int64, c.c_int32, P, P, P, P]
    lib.fdas_refine_eval.restype = c.c_int
    lib.fdas_refine_grad.argtypes = [P, c.c_int64, c.c_int64, c.c_int32, P, P, c.c_int64, c.c_int32, P, P, P, P,
                                     P]
    lib.fdas_refine_grad.restype = c.c_int
    lib.fdas_refine.argtypes = [P, P, c.c_int64, c.c_int32, c.c_double, c.c_int32, P, P, c.c_int64, P]
    lib.fdas_refine.restype = c.c_int
    lib.fdas_refine_window.argtypes = [c.c_double, c.c_double, c.c_double, c.c_int32, c.POINTER(c.c_int64),
                                       c.POINTER(c.c_int32)]
    lib.fdas_refine_window.restype = c.c_int
    lib.fdas_dedisperse.argtypes = [P, P, c.c_int64, c.c_int32, c.c_double, c.c_double, c.c_double, P, c.c_int32,
                                    P, c.c_int64, P]
    lib.fdas_dedisperse.restype = c.c_int
    lib.fdas_sift.argtypes = [P, c.c_int64, c.c_double, c.c_int32, P, c.c_int64, c.POINTER(c.c_int64)]
    lib.fdas_sift.restype = c.c_int
    lib.fdas_spectrum_noalloc.argtypes = [P, c.c_int64, c.c_int32, P, c.POINTER(c.c_double), P]
    lib.fdas_spectrum_noalloc.restype = c.c_int
    _lib = lib
    return lib


def default_opts(**kw) -> PlanOpts:
    o = PlanOpts()
    load().fdas_plan_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "norm" and isinstance(v, str):
            v = {"median": NORM_MEDIAN, "fixed": NORM_FIXED, "local": NORM_LOCAL}[v]
        setattr(o, k, v)
    return o


def _stream_handle(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check_series(t):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
        raise TypeError("series must be a CUDA float32 tensor")
    if t.dim() == 1:
        t = t.unsqueeze(0)
    if t.dim() != 2 or not t.is_contiguous():
        raise ValueError("series must be a contiguous [nseries][nsamp] tensor")
    return t


class Plan:
    """A device plan: template bank and workspace for series up to max_nsamp."""

    def __init__(self, max_nsamp: int, max_series: int, zmax: float, dz: float, numharm: int, **opts):
        self.lib = load()
        self.opts = default_opts(**opts)
        self.handle = ctypes.c_void_p()
        st = self.lib.fdas_plan_create(ctypes.byref(self.handle), int(max_nsamp), int(max_series),
                                       float(zmax), float(dz), int(numharm), ctypes.byref(self.opts))
        if st != FDAS_OK:
            raise FdasError(st, f"fdas_plan_create: {self.lib.fdas_status_string(st).decode()}")
        self.max_nsamp, self.max_series, self.zmax, self.dz, self.numharm = (
            max_nsamp, max_series, zmax, dz, numharm)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.fdas_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st, what):
        msg = self.lib.fdas_last_error(self.handle).decode()
        raise FdasError(st, f"{what}: {self.lib.fdas_status_string(st).decode()}: {msg}")

    def geometry(self, nsamp: int, tsamp: float, zmax: float = None, dz: float = None):
        return geometry(nsamp, tsamp, self.zmax if zmax is None else zmax,
                        self.dz if dz is None else dz, self.opts)

    @staticmethod
    def _records(cap: int):
        """Fresh, uninitialised host array for up to cap records. The library's
        host threads write the records straight into it and the caller gets a
        view of the written prefix: no copy, and pages past it are never
        touched (a long list costs its page faults once, spread over those
        threads, instead of a fault-and-copy pass on one)."""
        cap = int(cap)
        if cap < 0:
            raise ValueError("cap must be >= 0")
        return np.empty(max(cap, 1), dtype=CAND_DTYPE)[:cap]

    def search(self, t, tsamp: float, zmax: float = None, dz: float = None, numharm: int = None,
               sigma: float = 6.0, cap: int = 1 << 16, stream=None, allow_trunc: bool = False):
        """Candidates (structured numpy array, CAND_DTYPE) sorted by (series, harm, r_idx).
        With allow_trunc, (the first min(cap, total) records, total) instead, also
        when the list was cut at cap."""
        t = _check_series(t)
        zmax = self.zmax if zmax is None else zmax
        dz = self.dz if dz is None else dz
        numharm = self.numharm if numharm is None else numharm
        out = self._records(cap)
        n = ctypes.c_int64(0)
        st = self.lib.fdas_search(self.handle, ctypes.c_void_p(t.data_ptr()), t.shape[1], t.shape[0],
                                  float(tsamp), float(zmax), float(dz), int(numharm), float(sigma),
                                  out.ctypes.data_as(ctypes.c_void_p), int(cap), ctypes.byref(n),
                                  _stream_handle(stream))
        if allow_trunc and st in (FDAS_OK, FDAS_E_TRUNC):
            return out[:min(int(cap), int(n.value))], int(n.value)
        if st != FDAS_OK:
            self._raise(st, "fdas_search")
        return out[:n.value]

    def search_ragged(self, buf, offsets, nsamp, tsamp, zmax, dz: float = None, numharm: int = None,
                      sigma: float = 6.0, cap: int = 1 << 16, stream=None, allow_trunc: bool = False):
        """Search a ragged batch packed in one CUDA float32 buffer: series i is
        buf[offsets[i] : offsets[i] + nsamp[i]] (offsets even), sampled every
        tsamp[i] s, searched to drift zmax[i]. Candidates as ``search`` with
        ``series`` = i."""
        import torch
        if not (isinstance(buf, torch.Tensor) and buf.is_cuda and buf.dtype == torch.float32
                and buf.is_contiguous()):
            raise TypeError("buf must be a contiguous CUDA float32 tensor")
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        nsamp = np.ascontiguousarray(nsamp, dtype=np.int64)
        nser = len(offsets)
        tsamp = np.ascontiguousarray(np.broadcast_to(np.asarray(tsamp, dtype=np.float64), (nser,)))
        zmax = np.ascontiguousarray(np.broadcast_to(np.asarray(zmax, dtype=np.float64), (nser,)))
        if len(nsamp) != nser:
            raise ValueError("offsets and nsamp differ in length")
        if nser and (np.any(offsets < 0) or np.any(offsets + nsamp > buf.numel())):
            raise ValueError("a series lies outside the buffer")
        dz = self.dz if dz is None else dz
        numharm = self.numharm if numharm is None else numharm
        out = self._records(cap)
        n = ctypes.c_int64(0)
        i64 = ctypes.POINTER(ctypes.c_int64)
        f64 = ctypes.POINTER(ctypes.c_double)
        st = self.lib.fdas_search_ragged(self.handle, ctypes.c_void_p(buf.data_ptr()),
                                         offsets.ctypes.data_as(i64), nsamp.ctypes.data_as(i64),
                                         tsamp.ctypes.data_as(f64), zmax.ctypes.data_as(f64), nser,
                                         float(dz), int(numharm), float(sigma),
                                         out.ctypes.data_as(ctypes.c_void_p), int(cap), ctypes.byref(n),
                                         _stream_handle(stream))
        if allow_trunc and st in (FDAS_OK, FDAS_E_TRUNC):
            return out[:min(int(cap), int(n.value))], int(n.value)
        if st != FDAS_OK:
            self._raise(st, "fdas_search_ragged")
        return out[:n.value]

    def tuning(self) -> str:
        """The autotuner's choices as text (one line per shape)."""
        n = ctypes.c_int64(0)
        self.lib.fdas_tuning_export(self.handle, None, 0, ctypes.byref(n))
        buf = ctypes.create_string_buffer(int(n.value) + 1)
        st = self.lib.fdas_tuning_export(self.handle, buf, len(buf), ctypes.byref(n))
        if st != FDAS_OK:
            self._raise(st, "fdas_tuning_export")
        return buf.value.decode()

    def load_tuning(self, text: str):
        st = self.lib.fdas_tuning_import(self.handle, text.encode())
        if st != FDAS_OK:
            self._raise(st, "fdas_tuning_import")

    def dedisperse(self, fil, tsamp: float, f0_mhz: float, df_mhz: float, ranges, stream=None):
        """Dedisperse a CUDA uint8 [nsamp][nchan] filterbank for DM plan ranges
        (dm_start, dm_step, ndm, downsamp). Returns (buf, series): buf is the packed
        CUDA float32 output, series a list of per-range [ndm][nsamp/D] views of it."""
        import torch
        if not (isinstance(fil, torch.Tensor) and fil.is_cuda and fil.dtype == torch.uint8 and fil.dim() == 2
                and fil.is_contiguous()):
            raise TypeError("fil must be a contiguous CUDA uint8 [nsamp][nchan] tensor")
        rg = np.zeros(len(ranges), dtype=DM_RANGE_DTYPE)
        for i, (a, s_, n, d) in enumerate(ranges):
            rg[i] = (a, s_, n, d)
        nsamp, nchan = fil.shape
        sizes = [int(n) * (nsamp // int(d)) if int(d) > 0 else 0 for _, _, n, d in ranges]
        buf = torch.empty(max(1, sum(sizes)), dtype=torch.float32, device=fil.device)
        st = self.lib.fdas_dedisperse(self.handle, ctypes.c_void_p(fil.data_ptr()), nsamp, nchan, float(tsamp),
                                      float(f0_mhz), float(df_mhz), rg.ctypes.data_as(ctypes.c_void_p), len(rg),
                                      ctypes.c_void_p(buf.data_ptr()), buf.numel(), _stream_handle(stream))
        if st != FDAS_OK:
            self._raise(st, "fdas_dedisperse")
        out, o = [], 0
        for (_, _, n, d), sz in zip(ranges, sizes):
            out.append(buf[o:o + sz].view(int(n), nsamp // int(d)))
            o += sz
        return buf, out

    def refine(self, t, r0, z0, series=None, dz: float = None, iters: int = 20, stream=None):
        """Refine start points (r0, z0) [bins] of series ``series`` of the CUDA float32
        [B][N] batch t; returns (r, z, power) as float64, float64, float32 arrays."""
        t = _check_series(t)
        r0 = np.atleast_1d(np.asarray(r0, dtype=np.float64))
        n = r0.shape[0]
        pts = np.zeros(n, dtype=REFINE_DTYPE)
        pts["r"] = r0
        pts["z"] = np.broadcast_to(np.asarray(z0, dtype=np.float64), (n,))
        pts["series"] = 0 if series is None else np.broadcast_to(np.asarray(series, dtype=np.int32), (n,))
        power = np.zeros(n, dtype=np.float32)
        dz = self.dz if dz is None else dz
        st = self.lib.fdas_refine(self.handle, ctypes.c_void_p(t.data_ptr()), t.shape[1], t.shape[0], float(dz),
                                  int(iters), pts.ctypes.data_as(ctypes.c_void_p),
                                  power.ctypes.data_as(ctypes.c_void_p), n, _stream_handle(stream))
        if st != FDAS_OK:
            self._raise(st, "fdas_refine")
        return pts["r"].copy(), pts["z"].copy(), power

    def harmsum(self, plane, nsamp: int, tsamp: float, zmax: float = None, dz: float = None,
                numharm: int = None, sigma: float = 6.0, cap: int = 1 << 16, stream=None):
        """Candidates of a caller-built plane (CUDA float32 [B][NZ][NR])."""
        import torch
        if not (isinstance(plane, torch.Tensor) and plane.is_cuda and plane.dtype == torch.float32
                and plane.is_contiguous() and plane.dim() == 3):
            raise TypeError("plane must be a contiguous CUDA float32 [B][NZ][NR] tensor")
        zmax = self.zmax if zmax is None else zmax
        dz = self.dz if dz is None else dz
        numharm = self.numharm if numharm is None else numharm
        out = self._records(cap)
        n = ctypes.c_int64(0)
        st = self.lib.fdas_harmsum(self.handle, ctypes.c_void_p(plane.data_ptr()), int(nsamp),
                                   plane.shape[0], float(tsamp), float(zmax), float(dz), int(numharm),
                                   float(sigma), out.ctypes.data_as(ctypes.c_void_p), int(cap),
                                   ctypes.byref(n), _stream_handle(stream))
        if st != FDAS_OK:
            self._raise(st, "fdas_harmsum")
        return out[:n.value]

    def plane(self, t, tsamp: float, zmax: float = None, dz: float = None, stream=None):
        """Normalised power plane, CUDA float32 [B][NZ][NR] (column c is R = c + 2 rlo)."""
        import torch
        t = _check_series(t)
        zmax = self.zmax if zmax is None else zmax
        dz = self.dz if dz is None else dz
        rlo, nr, nz = self.geometry(t.shape[1], tsamp, zmax, dz)
        out = torch.empty((t.shape[0], nz, nr), dtype=torch.float32, device=t.device)
        st = self.lib.fdas_plane(self.handle, ctypes.c_void_p(t.data_ptr()), t.shape[1], t.shape[0],
                                 float(tsamp), float(zmax), float(dz), ctypes.c_void_p(out.data_ptr()),
                                 out.numel(), _stream_handle(stream))
        if st != FDAS_OK:
            self._raise(st, "fdas_plane")
        return out

    def info(self) -> dict:
        """Segment length, half-width, z rows, series per chunk and workspace of the plan."""
        i = PlanInfo()
        self.lib.fdas_plan_get_info(self.handle, ctypes.byref(i))
        return {k: getattr(i, k) for k, _ in PlanInfo._fields_}

    def profile(self, reset: bool = False):
        """{phase: (summed device ms, launches)} since the last reset (plans made with profile=1)."""
        ms = (ctypes.c_double * len(PHASES))()
        n = (ctypes.c_int64 * len(PHASES))()
        self.lib.fdas_profile_read(self.handle, ms, n, 1 if reset else 0)
        return {k: (ms[i], n[i]) for i, k in enumerate(PHASES)}

    def spectrum(self, t, stream=None):
        """(A, norm): CUDA complex64 [B][N/2+1] un-normalised spectra and float64 norms."""
        import torch
        t = _check_series(t)
        B, N = t.shape
        out = torch.empty((B, N // 2 + 1, 2), dtype=torch.float32, device=t.device)
        norm = (ctypes.c_double * B)()
        st = self.lib.fdas_spectrum(self.handle, ctypes.c_void_p(t.data_ptr()), N, B,
                                    ctypes.c_void_p(out.data_ptr()), norm, _stream_handle(stream))
        if st != FDAS_OK:
            self._raise(st, "fdas_spectrum")
        return torch.view_as_complex(out), np.array(norm[:], dtype=np.float64)


def spectrum_noalloc(t, out=None, stream=None):
    """(A, norm) as Plan.spectrum with the median normalisation, through the entry
    point that allocates nothing (fixed per-GPU scratch). out: optional CUDA float32
    [B][N/2+1][2] to write into (the caller's allocation)."""
    import torch
    lib = load()
    t = _check_series(t)
    B, N = t.shape
    if out is None:
        out = torch.empty((B, N // 2 + 1, 2), dtype=torch.float32, device=t.device)
    elif out.shape != (B, N // 2 + 1, 2) or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 [B][N/2+1][2] tensor")
    norm = (ctypes.c_double * B)()
    st = lib.fdas_spectrum_noalloc(ctypes.c_void_p(t.data_ptr()), N, B, ctypes.c_void_p(out.data_ptr()), norm,
                                   _stream_handle(stream))
    if st != FDAS_OK:
        raise FdasError(st, f"fdas_spectrum_noalloc: {lib.fdas_status_string(st).decode()}")
    return torch.view_as_complex(out), np.array(norm[:], dtype=np.float64)


def geometry(nsamp: int, tsamp: float, zmax: float, dz: float, opts: Optional[PlanOpts] = None):
    """(rlo, NR, NZ) of a search."""
    lib = load()
    rlo, nr, nz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    st = lib.fdas_geometry(int(nsamp), float(tsamp), float(zmax), float(dz),
                           ctypes.byref(opts) if opts is not None else None,
                           ctypes.byref(rlo), ctypes.byref(nr), ctypes.byref(nz))
    if st != FDAS_OK:
        raise FdasError(st, f"fdas_geometry: {lib.fdas_status_string(st).decode()}")
    return rlo.value, nr.value, nz.value


def threshold(harm: int, sigma: float) -> float:
    return load().fdas_threshold(int(harm), float(sigma))


def sigma_of(harm: int, power: float) -> float:
    return load().fdas_sigma(int(harm), float(power))


def template_taps(z: float, parity: int, K: int = 16):
    """(d0, taps): the library's host FP64 unit-energy taps for offsets d0, d0+1, ..."""
    lib = load()
    cap = 4 * (int(abs(z)) // 2 + K + 2) + 8
    re = (ctypes.c_double * cap)()
    im = (ctypes.c_double * cap)()
    n, d0 = ctypes.c_int32(), ctypes.c_int32()
    st = lib.fdas_template_taps(float(z), int(parity), int(K), re, im, cap, ctypes.byref(n), ctypes.byref(d0))
    if st != FDAS_OK:
        raise FdasError(st, "fdas_template_taps")
    return d0.value, np.array(re[:n.value]) + 1j * np.array(im[:n.value])


def search(t, tsamp: float, zmax: float, dz: float, numharm: int, sigma: float = 6.0,
           cap: int = 1 << 16, stream=None, **opts):
    """One-shot search of a CUDA float32 [B][N] tensor (builds a plan for it)."""
    t = _check_series(t)
    plan = Plan(t.shape[1], t.shape[0], zmax, dz, numharm, **opts)
    try:
        return plan.search(t, tsamp, zmax, dz, numharm, sigma, cap=cap, stream=stream)
    finally:
        plan.close()


def refine_window(r0: float, z0: float, dz: float, K: int = 16):
    """(k0, m): the refinement window the library uses for a start (r0, z0)."""
    k0, m = ctypes.c_int64(), ctypes.c_int32()
    st = load().fdas_refine_window(float(r0), float(z0), float(dz), int(K), ctypes.byref(k0), ctypes.byref(m))
    if st != FDAS_OK:
        raise FdasError(st, "fdas_refine_window: window out of range")
    return k0.value, m.value


def _refine_points(series, k0, m, r, z):
    """Pack per-point fields (CUDA tensors) into the library's 32-byte point records."""
    import torch
    n = r.shape[0]
    pts = torch.empty((n, 4), dtype=torch.int64, device=r.device)
    pts[:, 0] = (m.to(torch.int64) << 32) | (series.to(torch.int64) & 0xFFFFFFFF)
    pts[:, 1] = k0.to(torch.int64)
    pts[:, 2] = r.to(torch.float64).contiguous().view(torch.int64)
    pts[:, 3] = z.to(torch.float64).contiguous().view(torch.int64)
    return pts


def _refine_autograd():
    import torch

    class RefinePower(torch.autograd.Function):
        """P(r, z) of the refinement objective with hand-written backward kernels."""

        @staticmethod
        def forward(ctx, spec, r, z, series, k0, m, max_m):
            lib = load()
            spec = spec.contiguous()
            pts = _refine_points(series, k0, m, r, z)
            n = r.shape[0]
            power = torch.empty(n, dtype=torch.float32, device=r.device)
            st = lib.fdas_refine_eval(ctypes.c_void_p(spec.data_ptr()), spec.shape[1], spec.shape[1] - 1,
                                      spec.shape[0], None, ctypes.c_void_p(pts.data_ptr()), n, int(max_m),
                                      ctypes.c_void_p(power.data_ptr()), None, None, _stream_handle())
            if st != FDAS_OK:
                raise FdasError(st, f"fdas_refine_eval: {lib.fdas_status_string(st).decode()}")
            ctx.save_for_backward(spec, pts)
            ctx.max_m = int(max_m)
            ctx.rdtype, ctx.zdtype = r.dtype, z.dtype
            return power

        @staticmethod
        def backward(ctx, grad_power):
            lib = load()
            spec, pts = ctx.saved_tensors
            n = pts.shape[0]
            g = grad_power.to(torch.float32).contiguous()
            gr = torch.empty(n, dtype=torch.float32, device=g.device)
            gz = torch.empty(n, dtype=torch.float32, device=g.device)
            gs = torch.zeros_like(spec) if ctx.needs_input_grad[0] else None
            st = lib.fdas_refine_grad(ctypes.c_void_p(spec.data_ptr()), spec.shape[1], spec.shape[1] - 1,
                                      spec.shape[0], None, ctypes.c_void_p(pts.data_ptr()), n, ctx.max_m,
                                      ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(gr.data_ptr()),
                                      ctypes.c_void_p(gz.data_ptr()),
                                      ctypes.c_void_p(gs.data_ptr()) if gs is not None else None,
                                      _stream_handle())
            if st != FDAS_OK:
                raise FdasError(st, f"fdas_refine_grad: {lib.fdas_status_string(st).decode()}")
            return gs, gr.to(ctx.rdtype), gz.to(ctx.zdtype), None, None, None, None

    return RefinePower


_REFINE_FN = None


def refine_power(spec, r, z, series, k0, m, max_m: int = None):
    """Differentiable refinement objective on the GPU.

    spec: CUDA complex64 [B][N/2+1] normalised spectra (bins 0..N/2; DC and
    Nyquist are not read); r, z: CUDA float64 [n] points (bins); series, k0, m:
    CUDA integer [n] window of each point. Returns P (float32 [n]); gradients
    flow to spec, r and z through the library's backward kernel."""
    global _REFINE_FN
    if _REFINE_FN is None:
        _REFINE_FN = _refine_autograd()
    import torch
    if not (isinstance(spec, torch.Tensor) and spec.is_cuda and spec.dtype == torch.complex64 and spec.dim() == 2):
        raise TypeError("spec must be a CUDA complex64 [B][N/2+1] tensor")
    if max_m is None:
        max_m = int(m.max().item()) if m.numel() else 0
    return _REFINE_FN.apply(torch.view_as_real(spec.contiguous()), r, z, series, k0, m, max_m)


def sift(cands, tol_bins: float = 1.1, max_ratio: int = 16):
    """Sift a candidate list (CAND_DTYPE array): duplicates by fundamental frequency,
    then integer harmonics of stronger survivors. Returns SIFTED_DTYPE records
    (index into cands, hits, series range) in sifted order (host only)."""
    lib = load()
    cands = np.ascontiguousarray(cands, dtype=CAND_DTYPE)
    out = np.zeros(max(1, len(cands)), dtype=SIFTED_DTYPE)
    n = ctypes.c_int64(0)
    st = lib.fdas_sift(cands.ctypes.data_as(ctypes.c_void_p), len(cands), float(tol_bins), int(max_ratio),
                       out.ctypes.data_as(ctypes.c_void_p), len(out), ctypes.byref(n))
    if st != FDAS_OK:
        raise FdasError(st, f"fdas_sift: {lib.fdas_status_string(st).decode()}")
    return out[:n.value].copy()
