"""MI355X Fisher Information Field: Python binding of libfif.so.

Argument marshalling only: every step of the field build, the pose queries,
their gradients and the point-cloud brute force runs in the HIP kernels of
libfif.so (see include/fif.h).  PyTorch supplies device memory and streams.
There is no CPU fallback: importing the binding on a machine without the built
library raises.

Method: Zhang & Scaramuzza, "Fisher Information Field: an Efficient and
Differentiable Map for Perception-aware Planning", arXiv 2008.03324.
"""
from __future__ import annotations

import contextlib
import ctypes
import functools
import math
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfif.so")

FP32_NAIVE, FP32_COMP, FP64 = 0, 1, 2
KIND_INFO, KIND_TRACE, KIND_TRACE_CELLS = 0, 1, 2
TRACE, LMIN, LOGDET, FIM21 = 1, 2, 4, 8
TRILINEAR, NEAREST = 0, 1
FLAG_CLAMPED, FLAG_NOT_PD, FLAG_LMIN_TIE = 1, 2, 4
STATUS = {0: "FIF_OK", -1: "FIF_EINVAL", -2: "FIF_ENOMEM", -3: "FIF_EDEVICE",
          -4: "FIF_EUNSUPPORTED"}


class FifError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {detail}")
        self.status = status


class CGrid(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("h", ctypes.c_double),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class CVis(ctypes.Structure):
    _fields_ = [("half_fov", ctypes.c_double), ("v_alpha", ctypes.c_double),
                ("sigma_bearing", ctypes.c_double), ("r_min", ctypes.c_double),
                ("r_max", ctypes.c_double)]


class CPinhole(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double), ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class CField(ctypes.Structure):
    _fields_ = [("grid", CGrid), ("vis", CVis), ("prec", ctypes.c_int32),
                ("kind", ctypes.c_int32), ("data", ctypes.c_void_p)]


class CGP(ctypes.Structure):
    _fields_ = [("n_s", ctypes.c_int32), ("reserved", ctypes.c_int32), ("k_s", ctypes.c_double),
                ("length", ctypes.c_double), ("noise", ctypes.c_double),
                ("axes", ctypes.c_void_p), ("kinv", ctypes.c_void_p)]


class CGPField(ctypes.Structure):
    _fields_ = [("grid", CGrid), ("vis", CVis), ("gp", CGP), ("prec", ctypes.c_int32),
                ("kind", ctypes.c_int32), ("data", ctypes.c_void_p)]


class CServeRequest(ctypes.Structure):
    _fields_ = [("arrival", ctypes.c_double), ("field", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("m", ctypes.c_int64), ("t", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("grad_t", ctypes.c_void_p),
                ("grad_phi", ctypes.c_void_p), ("weights", ctypes.c_double * 3),
                ("admitted", ctypes.c_double), ("done", ctypes.c_double)]


class CServeConfig(ctypes.Structure):
    _fields_ = [("n_streams", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("hbm_budget", ctypes.c_int64), ("max_batch", ctypes.c_int64),
                ("co_batch", ctypes.c_int32), ("realtime", ctypes.c_int32)]


EXPORTS = {
    "fif_field_bytes": (ctypes.c_size_t, [ctypes.POINTER(CGrid), ctypes.c_int32, ctypes.c_int32]),
    "fif_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(CGrid), ctypes.c_int64, ctypes.c_int32]),
    "fif_build": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(CField),
                                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "fif_build_noalloc": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.POINTER(CField), ctypes.c_void_p]),
    "fif_update": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.POINTER(CField), ctypes.c_void_p, ctypes.c_size_t,
                                    ctypes.c_void_p]),
    "fif_query": (ctypes.c_int32, [ctypes.POINTER(CField), ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int64, ctypes.c_uint32, ctypes.c_int32,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fif_query_grad": (ctypes.c_int32, [ctypes.POINTER(CField), ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "pc_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32]),
    "pc_query": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(CVis),
                                  ctypes.POINTER(CPinhole), ctypes.c_int32, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.c_void_p]),
    "fif_view_sweep": (ctypes.c_int32, [ctypes.POINTER(CField), ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32,
                                        ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "fif_field_export": (ctypes.c_int32, [ctypes.POINTER(CField), ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "fif_gp_field_bytes": (ctypes.c_size_t, [ctypes.POINTER(CGrid), ctypes.c_int32,
                                             ctypes.c_int32, ctypes.c_int32]),
    "fif_gp_setup": (ctypes.c_int32, [ctypes.POINTER(CGP), ctypes.c_void_p]),
    "fif_gp_evidence": (ctypes.c_int32, [ctypes.POINTER(CGP), ctypes.c_double, ctypes.c_void_p,
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "fif_gp_build": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(CGPField),
                                      ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "fif_gp_query": (ctypes.c_int32, [ctypes.POINTER(CGPField), ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_int64, ctypes.c_uint32, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fif_gp_export": (ctypes.c_int32, [ctypes.POINTER(CGPField), ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "fif_serve_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(CServeConfig)]),
    "fif_serve_run": (ctypes.c_int32, [ctypes.POINTER(CField), ctypes.c_int32,
                                       ctypes.POINTER(CServeRequest), ctypes.c_int64,
                                       ctypes.POINTER(CServeConfig), ctypes.c_void_p,
                                       ctypes.c_size_t, ctypes.POINTER(ctypes.c_double)]),
    "fif_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "fif_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load libfif.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2008_03324_amd.buildlib` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != 0:
        raise FifError(status, where, lib().fif_last_error().decode())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _on_stream(fn):
    """A call given `stream` runs with that stream current, so that every tensor
    it allocates (outputs, temporaries, workspaces) belongs to the stream its
    kernels are enqueued on: the caching allocator then does not hand that
    memory to another stream while the kernels may still use it."""
    @functools.wraps(fn)
    def wrap(*args, stream=None, **kw):
        ctx = torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()
        with ctx:
            return fn(*args, stream=stream, **kw)
    return wrap


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t: torch.Tensor, dtype, name, shape_last=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_last is not None and (t.dim() != 2 or t.shape[1] != shape_last):
        raise ValueError(f"{name} must have shape [n, {shape_last}]")
    return t


def ncols(metrics: int) -> int:
    return bool(metrics & 1) + bool(metrics & 2) + bool(metrics & 4) + (21 if metrics & 8 else 0)


@dataclass(frozen=True)
class Grid:
    origin: tuple
    h: float
    shape: tuple

    def c(self) -> CGrid:
        g = CGrid()
        for i in range(3):
            g.origin[i] = float(self.origin[i])
        g.h = float(self.h)
        g.nx, g.ny, g.nz = (int(s) for s in self.shape)
        g.reserved = 0
        return g

    @property
    def n_voxels(self) -> int:
        return int(self.shape[0]) * int(self.shape[1]) * int(self.shape[2])


@dataclass(frozen=True)
class Vis:
    half_fov: float = math.pi / 4
    v_alpha: float = 0.8
    sigma: float = 1.0 / 300.0
    r_min: float = 0.0
    r_max: float = math.inf

    def c(self) -> CVis:
        return CVis(self.half_fov, self.v_alpha, self.sigma, self.r_min, self.r_max)


def field_bytes(grid: Grid, prec: int, kind: int = KIND_INFO) -> int:
    return int(lib().fif_field_bytes(ctypes.byref(grid.c()), prec, kind))


class Field:
    """A field resident in HBM: the buffer (a torch uint8 tensor) plus its header."""

    def __init__(self, grid: Grid, vis: Vis, prec: int = FP32_COMP, kind: int = KIND_INFO,
                 device=None):
        nbytes = field_bytes(grid, prec, kind)
        if nbytes == 0:
            raise ValueError("invalid grid, precision or kind")
        self.grid, self.vis, self.prec, self.kind = grid, vis, prec, kind
        self.buffer = torch.empty(nbytes, dtype=torch.uint8, device=device or "cuda")
        self.cstruct = CField(grid.c(), vis.c(), prec, kind, self.buffer.data_ptr())

    @property
    def pose_dtype(self):
        return torch.float64 if self.prec == FP64 else torch.float32

    @property
    def nbytes(self) -> int:
        return self.buffer.numel()

    def with_vis(self, vis: Vis) -> "Field":
        """Same buffer, other visibility parameters.  The stored moments do not
        depend on the visibility or on sigma, but they do depend on the range
        bounds, which must be unchanged."""
        if (vis.r_min, vis.r_max) != (self.vis.r_min, self.vis.r_max):
            raise ValueError("the range bounds are baked into the field")
        f = object.__new__(Field)
        f.grid, f.vis, f.prec, f.kind, f.buffer = self.grid, vis, self.prec, self.kind, self.buffer
        f.cstruct = CField(self.grid.c(), vis.c(), self.prec, self.kind, self.buffer.data_ptr())
        return f


_WORKSPACE = {}
_PC_WORKSPACE = {}


def _cached_workspace(cache: dict, nbytes: int, device) -> torch.Tensor:
    """One scratch buffer per (device, current stream), grown on demand.  Calls
    enqueued on one stream run in order, so they can share it; calls on
    different streams get different buffers."""
    key = (str(device), torch.cuda.current_stream(device).cuda_stream)
    ws = cache.get(key)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        cache[key] = ws
    return ws


def workspace(grid: Grid, n_landmarks: int, prec: int, device) -> torch.Tensor | None:
    """Scratch for the spatially sorted build (see _cached_workspace)."""
    nbytes = int(lib().fif_workspace_bytes(ctypes.byref(grid.c()), int(n_landmarks), prec))
    if nbytes == 0:
        return None
    return _cached_workspace(_WORKSPACE, nbytes, device)


def release_workspaces() -> None:
    """Drop the cached build and point-cloud workspaces (one per device and
    stream used so far).  The memory returns to torch's caching allocator,
    which reuses it in stream order, so calls still in flight are not
    disturbed."""
    _WORKSPACE.clear()
    _PC_WORKSPACE.clear()


@_on_stream
def build(landmarks: torch.Tensor, grid: Grid, vis: Vis, prec: int = FP32_COMP,
          kind: int = KIND_INFO, field: Field | None = None, sort: bool = True,
          stream=None) -> Field:
    """Build a field.  With sort (the default) the landmarks are first ordered
    spatially in a workspace so that whole landmark batches out of range of a
    voxel tile are skipped; without it every pair is tested in input order."""
    lm = _dev(landmarks, torch.float64, "landmarks", 3)
    if field is None:
        field = Field(grid, vis, prec, kind, device=lm.device)
    ws = workspace(grid, lm.shape[0], prec, lm.device) if sort else None
    _check(lib().fif_build(_ptr(lm), lm.shape[0], ctypes.byref(field.cstruct), _ptr(ws),
                           ws.numel() if ws is not None else 0, _stream(stream)), "fif_build")
    return field


@_on_stream
def build_noalloc(landmarks: torch.Tensor, grid: Grid, vis: Vis, prec: int = FP32_COMP,
                  kind: int = KIND_INFO, field: Field | None = None, stream=None) -> Field:
    """Build a field with the sorted, batch-culled path and the library's static
    scratch instead of a workspace (fif_build_noalloc; the same field as
    build(sort=True)).  Pass `field` to keep the call free of allocations."""
    lm = _dev(landmarks, torch.float64, "landmarks", 3)
    if field is None:
        field = Field(grid, vis, prec, kind, device=lm.device)
    _check(lib().fif_build_noalloc(_ptr(lm), lm.shape[0], ctypes.byref(field.cstruct),
                                   _stream(stream)), "fif_build_noalloc")
    return field


@_on_stream
def update(field: Field, landmarks: torch.Tensor, sign: int, sort: bool = True,
           stream=None) -> Field:
    """Add (sign +1) or remove (sign -1) landmarks.  With sort (the default) the
    added landmarks are ordered spatially in a workspace so that voxel tiles out
    of range of a whole batch of them skip it."""
    lm = _dev(landmarks, torch.float64, "landmarks", 3)
    ws = workspace(field.grid, lm.shape[0], field.prec, lm.device) if sort else None
    _check(lib().fif_update(_ptr(lm), lm.shape[0], int(sign), ctypes.byref(field.cstruct),
                            _ptr(ws), ws.numel() if ws is not None else 0, _stream(stream)),
           "fif_update")
    return field


@_on_stream
def query(field: Field, t: torch.Tensor, q: torch.Tensor, metrics: int = TRACE | LMIN | LOGDET,
          interp: int = TRILINEAR, out: torch.Tensor | None = None,
          flags: torch.Tensor | None = None, want_flags: bool = False, stream=None):
    dt = field.pose_dtype
    t = _dev(t, dt, "t", 3)
    q = _dev(q, dt, "q", 4)
    m = t.shape[0]
    if q.shape[0] != m:
        raise ValueError("t and q differ in length")
    if out is None:
        out = torch.empty((m, ncols(metrics)), dtype=torch.float64, device=t.device)
    if flags is None and want_flags:
        flags = torch.empty(m, dtype=torch.uint8, device=t.device)
    _check(lib().fif_query(ctypes.byref(field.cstruct), _ptr(t), _ptr(q), m, metrics, interp,
                           _ptr(out), _ptr(flags), _stream(stream)), "fif_query")
    return (out, flags) if want_flags else out


@_on_stream
def query_grad(field: Field, t: torch.Tensor, q: torch.Tensor, metrics: int,
               dL_dout: torch.Tensor, want_out: bool = False, stream=None):
    dt = field.pose_dtype
    t = _dev(t, dt, "t", 3)
    q = _dev(q, dt, "q", 4)
    m = t.shape[0]
    nm = ncols(metrics & 7)
    up = _dev(dL_dout.reshape(m, nm).contiguous(), torch.float64, "dL_dout")
    gt = torch.empty((m, 3), dtype=dt, device=t.device)
    gphi = torch.empty((m, 3), dtype=dt, device=t.device)
    out = torch.empty((m, nm), dtype=torch.float64, device=t.device) if want_out else None
    _check(lib().fif_query_grad(ctypes.byref(field.cstruct), _ptr(t), _ptr(q), m, metrics,
                                _ptr(up), _ptr(gt), _ptr(gphi), _ptr(out), _stream(stream)),
           "fif_query_grad")
    return (gt, gphi, out) if want_out else (gt, gphi)


@_on_stream
def view_sweep(field: Field, t: torch.Tensor, dirs: torch.Tensor, metric: int = LOGDET,
               interp: int = TRILINEAR, want_values: bool = True, stream=None):
    """Metric of every candidate optical axis (dirs [n_dir, 3], float64) at every
    position (t [n_pos, 3]) and the index of the best axis per position.
    Returns (values [n_pos, n_dir] float64 or None, best [n_pos] int64)."""
    t = _dev(t, field.pose_dtype, "t", 3)
    dirs = _dev(dirs, torch.float64, "dirs", 3)
    n, nd = t.shape[0], dirs.shape[0]
    values = (torch.empty((n, nd), dtype=torch.float64, device=t.device) if want_values
              else None)
    best = torch.empty(n, dtype=torch.int64, device=t.device)
    _check(lib().fif_view_sweep(ctypes.byref(field.cstruct), _ptr(t), n, _ptr(dirs), nd,
                                metric, interp, _ptr(values), _ptr(best), _stream(stream)),
           "fif_view_sweep")
    return values, best


@_on_stream
def pc_query(landmarks: torch.Tensor, vis: Vis, t: torch.Tensor, q: torch.Tensor,
             metrics: int = TRACE | LMIN | LOGDET, prec: int = FP32_COMP, pinhole=None,
             out: torch.Tensor | None = None, sort: bool = True, stream=None):
    """Point-cloud FIMs.  With sort (the default) landmarks and poses are
    ordered spatially in a workspace and landmark batches out of range of a
    group of poses are skipped; without it every pair is tested in input
    order."""
    lm = _dev(landmarks, torch.float64, "landmarks", 3)
    dt = torch.float64 if prec == FP64 else torch.float32
    t = _dev(t, dt, "t", 3)
    q = _dev(q, dt, "q", 4)
    m = t.shape[0]
    if out is None:
        out = torch.empty((m, ncols(metrics)), dtype=torch.float64, device=t.device)
    cam = None
    if pinhole is not None:
        fx, fy, cx, cy, W, H = pinhole
        cam = ctypes.byref(CPinhole(fx, fy, cx, cy, int(W), int(H)))
    ws = None
    if sort and lm.shape[0] > 0 and m > 0 and math.isfinite(vis.r_max):
        nbytes = int(lib().pc_workspace_bytes(lm.shape[0], m, prec))
        ws = _cached_workspace(_PC_WORKSPACE, nbytes, lm.device) if nbytes else None
    _check(lib().pc_query(_ptr(lm), lm.shape[0], ctypes.byref(vis.c()), cam, prec, _ptr(t),
                          _ptr(q), m, metrics, _ptr(out), _ptr(ws),
                          ws.numel() if ws is not None else 0, _stream(stream)), "pc_query")
    return out


@_on_stream
def export_blocks(field: Field, voxel_ids: torch.Tensor, stream=None) -> torch.Tensor:
    ids = _dev(voxel_ids, torch.int64, "voxel_ids")
    n = ids.numel()
    shape = (n, 10, 21) if field.kind == KIND_INFO else (n, 10)
    out = torch.empty(shape, dtype=torch.float64, device=ids.device)
    _check(lib().fif_field_export(ctypes.byref(field.cstruct), _ptr(ids), n, _ptr(out),
                                  _stream(stream)), "fif_field_export")
    return out


# ------------------------------------------------------------ GP visibility fields

class GPModel:
    """GP visibility model (Sec. V-B): sample axes [n_s, 3] (float64, device),
    sigmoid slope k_s, SE length scale and noise; holds (K^s + noise I)^-1."""

    def __init__(self, axes: torch.Tensor, k_s: float = 15.0, length: float | None = None,
                 noise: float = 1e-10):
        self.axes = _dev(axes, torch.float64, "axes", 3)
        self.n_s = int(self.axes.shape[0])
        self.k_s, self.noise = float(k_s), float(noise)
        self.kinv = torch.empty((self.n_s, self.n_s), dtype=torch.float64, device=self.axes.device)
        self.length = None
        if length is not None:
            self.set_length(length)

    def c(self) -> CGP:
        return CGP(self.n_s, 0, self.k_s, float(self.length or 0.0), self.noise,
                   self.axes.data_ptr(), self.kinv.data_ptr())

    @_on_stream
    def set_length(self, length: float, stream=None) -> "GPModel":
        self.length = float(length)
        _check(lib().fif_gp_setup(ctypes.byref(self.c()), _stream(stream)), "fif_gp_setup")
        return self

    @_on_stream
    def evidence(self, half_fov: float, train_u: torch.Tensor, lengths: torch.Tensor,
                 stream=None) -> torch.Tensor:
        u = _dev(train_u, torch.float64, "train_u", 3)
        ls = _dev(lengths.reshape(-1).contiguous(), torch.float64, "lengths")
        out = torch.empty(ls.numel(), dtype=torch.float64, device=ls.device)
        _check(lib().fif_gp_evidence(ctypes.byref(self.c()), float(half_fov), _ptr(u), u.shape[0],
                                     _ptr(ls), ls.numel(), _ptr(out), _stream(stream)),
               "fif_gp_evidence")
        return out

    def fit_length(self, half_fov: float, train_u: torch.Tensor, lo: float = 0.05,
                   hi: float = 3.0, n: int = 64, rounds: int = 4) -> float:
        """ML-II length scale (Sec. V-B): the evidence of a log-spaced grid of
        candidates is evaluated on the device, and the grid is narrowed around
        the best one each round; then the model is set up with it."""
        a, b = math.log(lo), math.log(hi)
        best = None
        for _ in range(rounds):
            ls = torch.exp(torch.linspace(a, b, n, dtype=torch.float64, device=self.axes.device))
            ev = self.evidence(half_fov, train_u, ls).cpu()
            i = int(torch.argmax(ev))
            best = float(ls[i])
            step = (b - a) / (n - 1)
            a, b = math.log(best) - step, math.log(best) + step
        self.set_length(best)
        return best


def gp_field_bytes(grid: Grid, n_s: int, prec: int, kind: int = KIND_INFO) -> int:
    return int(lib().fif_gp_field_bytes(ctypes.byref(grid.c()), int(n_s), prec, kind))


class GPField:
    """A GP field resident in HBM (buffer + header) with its model."""

    def __init__(self, grid: Grid, vis: Vis, model: GPModel, prec: int = FP32_COMP,
                 kind: int = KIND_INFO, device=None):
        nbytes = gp_field_bytes(grid, model.n_s, prec, kind)
        if nbytes == 0:
            raise ValueError("invalid grid, n_s, precision or kind")
        self.grid, self.vis, self.model, self.prec, self.kind = grid, vis, model, prec, kind
        self.buffer = torch.empty(nbytes, dtype=torch.uint8, device=device or model.axes.device)

    @property
    def cstruct(self) -> CGPField:
        return CGPField(self.grid.c(), self.vis.c(), self.model.c(), self.prec, self.kind,
                        self.buffer.data_ptr())

    @property
    def pose_dtype(self):
        return torch.float64 if self.prec == FP64 else torch.float32

    @property
    def nbytes(self) -> int:
        return self.buffer.numel()


@_on_stream
def gp_build(landmarks: torch.Tensor, grid: Grid, vis: Vis, model: GPModel,
             prec: int = FP32_COMP, kind: int = KIND_INFO, field: GPField | None = None,
             sort: bool = True, stream=None) -> GPField:
    lm = _dev(landmarks, torch.float64, "landmarks", 3)
    if field is None:
        field = GPField(grid, vis, model, prec, kind, device=lm.device)
    ws = workspace(grid, lm.shape[0], prec, lm.device) if sort else None
    cs = field.cstruct
    _check(lib().fif_gp_build(_ptr(lm), lm.shape[0], ctypes.byref(cs), _ptr(ws),
                              ws.numel() if ws is not None else 0, _stream(stream)), "fif_gp_build")
    return field


@_on_stream
def gp_query(field: GPField, t: torch.Tensor, q: torch.Tensor,
             metrics: int = TRACE | LMIN | LOGDET, interp: int = TRILINEAR,
             out: torch.Tensor | None = None, want_flags: bool = False, stream=None):
    dt = field.pose_dtype
    t = _dev(t, dt, "t", 3)
    q = _dev(q, dt, "q", 4)
    m = t.shape[0]
    if q.shape[0] != m:
        raise ValueError("t and q differ in length")
    if out is None:
        out = torch.empty((m, ncols(metrics)), dtype=torch.float64, device=t.device)
    flags = torch.empty(m, dtype=torch.uint8, device=t.device) if want_flags else None
    cs = field.cstruct
    _check(lib().fif_gp_query(ctypes.byref(cs), _ptr(t), _ptr(q), m, metrics, interp, _ptr(out),
                              _ptr(flags), _stream(stream)), "fif_gp_query")
    return (out, flags) if want_flags else out


@_on_stream
def gp_export(field: GPField, voxel_ids: torch.Tensor, stream=None) -> torch.Tensor:
    ids = _dev(voxel_ids, torch.int64, "voxel_ids")
    n, ns = ids.numel(), field.model.n_s
    shape = (n, ns, 21) if field.kind == KIND_INFO else (n, ns)
    out = torch.empty(shape, dtype=torch.float64, device=ids.device)
    cs = field.cstruct
    _check(lib().fif_gp_export(ctypes.byref(cs), _ptr(ids), n, _ptr(out), _stream(stream)),
           "fif_gp_export")
    return out


def _quat_mul(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    aw, ax, ay, az = a.unbind(-1)
    bw, bx, by, bz = b.unbind(-1)
    return torch.stack([aw * bw - ax * bx - ay * by - az * bz,
                        aw * bx + ax * bw + ay * bz - az * by,
                        aw * by - ax * bz + ay * bw + az * bx,
                        aw * bz + ax * by - ay * bx + az * bw], -1)


class FIFQuery(torch.autograd.Function):
    """Differentiable field query: metrics (trace / lmin / logdet) of each pose.

    Forward and backward both run in libfif (fif_query_grad).  The kernel gives
    the gradient w.r.t. the left so(3) perturbation phi; for the quaternion
    input it is carried over by the chain rule of q' = (1, phi/2) (x) q / |q|.
    """

    @staticmethod
    def forward(ctx, t, q, field: Field, metrics: int):
        ctx.field, ctx.metrics = field, metrics
        ctx.save_for_backward(t, q)
        return query(field, t.detach().contiguous(), q.detach().contiguous(), metrics)

    @staticmethod
    def backward(ctx, grad_out):
        t, q = ctx.saved_tensors
        gt, gphi = query_grad(ctx.field, t.detach().contiguous(), q.detach().contiguous(),
                              ctx.metrics, grad_out.to(torch.float64).contiguous())
        gq = None
        if ctx.needs_input_grad[1]:
            qn = q.detach() / q.detach().norm(dim=1, keepdim=True)
            pure = torch.cat([torch.zeros_like(gphi[:, :1]), gphi], dim=1)
            gq = 2.0 * _quat_mul(pure, qn) / q.detach().norm(dim=1, keepdim=True)
        return gt, gq, None, None


def fif_query_autograd(field: Field, t: torch.Tensor, q: torch.Tensor,
                       metrics: int = TRACE | LMIN | LOGDET) -> torch.Tensor:
    return FIFQuery.apply(t, q, field, metrics)
