"""FP64 CPU oracle for the Fisher Information Field hot path (ctypes binding).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product package never does.
The C source (``fif_oracle.c``) follows Zhang & Scaramuzza, arXiv 2008.03324,
step by step in FP64; see the comment of each C function for the passage.

Parity status: every function here is pinned by ``tests/test_oracle_pins.py``
(finite-difference Jacobians of the bearing model, closed forms, LAPACK
eigen-solvers, brute force on tiny inputs); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fif_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

TRACE, LMIN, LOGDET, FIM = 1, 2, 4, 8


def compile_oracle() -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("h", ctypes.c_double),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32)]


class _Pinhole(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            compile_oracle()
        _lib = ctypes.CDLL(_LIB)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _grid(origin, h, shape):
    g = _Grid()
    for c in range(3):
        g.origin[c] = float(origin[c])
    g.h = float(h)
    g.nx, g.ny, g.nz = (int(s) for s in shape)
    return g


def _f64(a, shape_last=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape_last is not None:
        a = a.reshape(-1, shape_last)
    return a


def ncols(metrics: int) -> int:
    return bool(metrics & 1) + bool(metrics & 2) + bool(metrics & 4) + (21 if metrics & 8 else 0)


# ------------------------------------------------------------ visibility

def quad_coeffs(alpha: float, v_alpha: float) -> np.ndarray:
    """(k2, k1, k0) from eq:quadratic_conditions."""
    k = np.zeros(3)
    lib().oracle_quad_coeffs(ctypes.c_double(alpha), ctypes.c_double(v_alpha), _p(k))
    return k


def vr(k, z) -> np.ndarray:
    out = np.zeros(10)
    lib().oracle_vr(_p(_f64(k)), _p(_f64(z)), _p(out))
    return out


def vp(u) -> np.ndarray:
    out = np.zeros(10)
    lib().oracle_vp(_p(_f64(u)), _p(out))
    return out


def in_range(p, t, r_min, r_max) -> bool:
    f = lib().oracle_in_range
    f.restype = ctypes.c_int
    return bool(f(_p(_f64(p)), _p(_f64(t)), ctypes.c_double(r_min), ctypes.c_double(r_max)))


def quat_to_R(q) -> np.ndarray:
    R = np.zeros(9)
    lib().oracle_quat_to_R(_p(_f64(q)), _p(R))
    return R.reshape(3, 3)


# ------------------------------------------------------------ FIM pieces

def landmark_fim(p, t, R_wc, sigma) -> np.ndarray:
    out = np.zeros(36)
    lib().oracle_landmark_fim(_p(_f64(p)), _p(_f64(t)), _p(_f64(R_wc)),
                              ctypes.c_double(sigma), _p(out))
    return out.reshape(6, 6)


def info_factor(landmarks, t, sigma, r_min=0.0, r_max=np.inf) -> np.ndarray:
    """C_I at position t: (10, 6, 6)."""
    lm = _f64(landmarks, 3)
    out = np.zeros(360)
    lib().oracle_info_factor(_p(lm), ctypes.c_int64(lm.shape[0]), _p(_f64(t)),
                             ctypes.c_double(sigma), ctypes.c_double(r_min),
                             ctypes.c_double(r_max), _p(out))
    return out.reshape(10, 6, 6)


def trace_factor(landmarks, t, sigma, r_min=0.0, r_max=np.inf) -> np.ndarray:
    lm = _f64(landmarks, 3)
    out = np.zeros(10)
    lib().oracle_trace_factor(_p(lm), ctypes.c_int64(lm.shape[0]), _p(_f64(t)),
                              ctypes.c_double(sigma), ctypes.c_double(r_min),
                              ctypes.c_double(r_max), _p(out))
    return out


def trace_build(landmarks, origin, h, shape, sigma, r_min=0.0, r_max=np.inf,
                voxel_ids=None) -> np.ndarray:
    """Trace factors C_Tr of the listed voxels (all when voxel_ids is None): (n, 10)."""
    lm = _f64(landmarks, 3)
    g = _grid(origin, h, shape)
    if voxel_ids is None:
        n = int(np.prod(shape))
        ids = None
    else:
        ids = np.ascontiguousarray(voxel_ids, dtype=np.int64)
        n = ids.shape[0]
    out = np.zeros((n, 10))
    lib().oracle_trace_build(_p(lm), ctypes.c_int64(lm.shape[0]), ctypes.byref(g),
                             ctypes.c_double(sigma), ctypes.c_double(r_min),
                             ctypes.c_double(r_max), _p(ids), ctypes.c_int64(n), _p(out))
    return out


def build(landmarks, origin, h, shape, sigma, r_min=0.0, r_max=np.inf,
          voxel_ids=None) -> np.ndarray:
    """Factors of the listed voxels (all when voxel_ids is None): (n, 10, 6, 6)."""
    lm = _f64(landmarks, 3)
    g = _grid(origin, h, shape)
    if voxel_ids is None:
        n = int(np.prod(shape))
        ids = None
    else:
        ids = np.ascontiguousarray(voxel_ids, dtype=np.int64)
        n = ids.shape[0]
    out = np.zeros((n, 360))
    lib().oracle_build(_p(lm), ctypes.c_int64(lm.shape[0]), ctypes.byref(g),
                       ctypes.c_double(sigma), ctypes.c_double(r_min), ctypes.c_double(r_max),
                       _p(ids), ctypes.c_int64(n), _p(out))
    return out.reshape(n, 10, 6, 6)


def voxel_centre(origin, h, shape, v) -> np.ndarray:
    t = np.zeros(3)
    lib().oracle_voxel_centre(ctypes.byref(_grid(origin, h, shape)), ctypes.c_int64(v), _p(t))
    return t


# ------------------------------------------------------------ metrics

def jacobi6(F):
    w = np.zeros(6)
    V = np.zeros(36)
    lib().oracle_jacobi6(_p(_f64(F).reshape(-1)), _p(w), _p(V))
    return w, V.reshape(6, 6)


def logdet6(F, want_inv=False):
    f = lib().oracle_logdet6
    f.restype = ctypes.c_double
    inv = np.zeros(36) if want_inv else None
    ld = f(_p(_f64(F).reshape(-1)), _p(inv))
    return (ld, inv.reshape(6, 6)) if want_inv else ld


def metrics(F, which: int) -> np.ndarray:
    out = np.zeros(ncols(which))
    lib().oracle_metrics(_p(_f64(F).reshape(-1)), ctypes.c_uint32(which), _p(out))
    return out


# ------------------------------------------------------------ queries

class Field:
    """A factor field held by the oracle: all voxels, or a sparse subset."""

    def __init__(self, C, origin, h, shape, voxel_ids=None):
        self.C = np.ascontiguousarray(C, dtype=np.float64).reshape(-1, 360)
        self.origin, self.h, self.shape = tuple(origin), float(h), tuple(int(s) for s in shape)
        if voxel_ids is not None:
            order = np.argsort(voxel_ids, kind="stable")
            self.ids = np.ascontiguousarray(np.asarray(voxel_ids, np.int64)[order])
            self.C = np.ascontiguousarray(self.C[order])
        else:
            self.ids = None
        self.grid = _grid(self.origin, self.h, self.shape)

    def _args(self):
        n = self.ids.shape[0] if self.ids is not None else self.C.shape[0]
        return _p(self.C), _p(self.ids), ctypes.c_int64(n), ctypes.byref(self.grid)


def query(field: Field, alpha, v_alpha, t, q, metrics_mask, interp=0):
    t = _f64(t, 3)
    q = _f64(q, 4)
    m = t.shape[0]
    out = np.zeros((m, ncols(metrics_mask)))
    flags = np.zeros(m, np.uint8)
    rc = lib().oracle_query(*field._args(), ctypes.c_double(alpha), ctypes.c_double(v_alpha),
                            _p(t), _p(q), ctypes.c_int64(m), ctypes.c_uint32(metrics_mask),
                            ctypes.c_int(interp), _p(out), _p(flags))
    if rc != 0:
        raise KeyError("oracle field is missing a voxel the query needs")
    return out, flags


class TraceField:
    """A trace-factor field (eq:general_trace_pif) held by the oracle."""

    def __init__(self, CT, origin, h, shape, voxel_ids=None):
        self.C = np.ascontiguousarray(CT, dtype=np.float64).reshape(-1, 10)
        self.origin, self.h, self.shape = tuple(origin), float(h), tuple(int(s) for s in shape)
        if voxel_ids is not None:
            order = np.argsort(voxel_ids, kind="stable")
            self.ids = np.ascontiguousarray(np.asarray(voxel_ids, np.int64)[order])
            self.C = np.ascontiguousarray(self.C[order])
        else:
            self.ids = None
        self.grid = _grid(self.origin, self.h, self.shape)


def trace_query(field: TraceField, alpha, v_alpha, t, q, interp=0):
    """Trace of the FIM from a trace field: (traces [m], flags [m])."""
    t = _f64(t, 3)
    q = _f64(q, 4)
    m = t.shape[0]
    out = np.zeros(m)
    flags = np.zeros(m, np.uint8)
    n = field.ids.shape[0] if field.ids is not None else field.C.shape[0]
    rc = lib().oracle_trace_query(_p(field.C), _p(field.ids), ctypes.c_int64(n),
                                  ctypes.byref(field.grid), ctypes.c_double(alpha),
                                  ctypes.c_double(v_alpha), _p(t), _p(q), ctypes.c_int64(m),
                                  ctypes.c_int(interp), _p(out), _p(flags))
    if rc != 0:
        raise KeyError("oracle trace field is missing a voxel the query needs")
    return out, flags


def query_fim(field: Field, alpha, v_alpha, t, q, interp=0):
    t = _f64(t, 3)
    q = _f64(q, 4)
    m = t.shape[0]
    F = np.zeros((m, 36))
    rc = lib().oracle_query_fim(*field._args(), ctypes.c_double(alpha), ctypes.c_double(v_alpha),
                                _p(t), _p(q), ctypes.c_int64(m), ctypes.c_int(interp), _p(F))
    if rc != 0:
        raise KeyError("oracle field is missing a voxel the query needs")
    return F.reshape(m, 6, 6)


def query_grad(field: Field, alpha, v_alpha, t, q, metrics_mask, dL_dout):
    t = _f64(t, 3)
    q = _f64(q, 4)
    m = t.shape[0]
    nc = bool(metrics_mask & 1) + bool(metrics_mask & 2) + bool(metrics_mask & 4)
    up = _f64(dL_dout).reshape(m, nc)
    gt = np.zeros((m, 3))
    gphi = np.zeros((m, 3))
    rc = lib().oracle_query_grad(*field._args(), ctypes.c_double(alpha),
                                 ctypes.c_double(v_alpha), _p(t), _p(q), ctypes.c_int64(m),
                                 ctypes.c_uint32(metrics_mask), _p(up), _p(gt), _p(gphi))
    if rc != 0:
        raise KeyError("oracle field is missing a voxel the query needs")
    return gt, gphi


def view_sweep(field: Field, alpha, v_alpha, t, dirs, metric, interp=0):
    """Metric of every candidate optical axis at every position, and the index
    of the best axis per position (first among equal values; -1 if all NaN)."""
    t = _f64(t, 3)
    dirs = _f64(dirs, 3)
    n, nd = t.shape[0], dirs.shape[0]
    values = np.zeros((n, nd))
    best = np.zeros(n, np.int64)
    rc = lib().oracle_view_sweep(*field._args(), ctypes.c_double(alpha),
                                 ctypes.c_double(v_alpha), _p(t), ctypes.c_int64(n),
                                 _p(dirs), ctypes.c_int64(nd), ctypes.c_uint32(metric),
                                 ctypes.c_int(interp), _p(values), _p(best))
    if rc != 0:
        raise KeyError("oracle field is missing a voxel the sweep needs")
    return values, best


# ------------------------------------------------------------ GP visibility

def sigmoid_vis(ks, alpha, cos_theta) -> float:
    f = lib().oracle_sigmoid_vis
    f.restype = ctypes.c_double
    return f(ctypes.c_double(ks), ctypes.c_double(alpha), ctypes.c_double(cos_theta))


def gp_inverse(Z, length, noise) -> np.ndarray:
    Z = _f64(Z, 3)
    ns = Z.shape[0]
    A = np.zeros((ns, ns))
    if lib().oracle_gp_inverse(ctypes.c_int(ns), _p(Z), ctypes.c_double(length),
                               ctypes.c_double(noise), _p(A)) != 0:
        raise np.linalg.LinAlgError("K^s + noise I is not positive definite")
    return A


def gp_vr(Z, length, z) -> np.ndarray:
    Z = _f64(Z, 3)
    out = np.zeros(Z.shape[0])
    lib().oracle_gp_vr(ctypes.c_int(Z.shape[0]), _p(Z), ctypes.c_double(length),
                       _p(_f64(z).reshape(3)), _p(out))
    return out


def gp_vp(Z, ks, alpha, Ainv, u) -> np.ndarray:
    Z = _f64(Z, 3)
    out = np.zeros(Z.shape[0])
    lib().oracle_gp_vp(ctypes.c_int(Z.shape[0]), _p(Z), ctypes.c_double(ks), ctypes.c_double(alpha),
                       _p(_f64(Ainv)), _p(_f64(u).reshape(3)), _p(out))
    return out


def gp_build(landmarks, origin, h, shape, sigma, Z, ks, alpha, Ainv, r_min=0.0, r_max=np.inf,
             trace=False, voxel_ids=None) -> np.ndarray:
    """GP factors: [n_vox][ns][6][6] (information) or [n_vox][ns] (trace)."""
    lm = _f64(landmarks, 3)
    Z = _f64(Z, 3)
    ns = Z.shape[0]
    g = _grid(origin, h, shape)
    if voxel_ids is None:
        ids = None
        n = int(np.prod(shape))
    else:
        ids = np.ascontiguousarray(voxel_ids, dtype=np.int64)
        n = ids.shape[0]
    per = ns if trace else ns * 36
    C = np.zeros((n, per))
    lib().oracle_gp_build(_p(lm), ctypes.c_int64(lm.shape[0]), ctypes.byref(g),
                          ctypes.c_double(sigma), ctypes.c_double(r_min), ctypes.c_double(r_max),
                          ctypes.c_int(ns), _p(Z), ctypes.c_double(ks), ctypes.c_double(alpha),
                          _p(_f64(Ainv)), ctypes.c_int(1 if trace else 0), _p(ids),
                          ctypes.c_int64(n), _p(C))
    return C.reshape(n, ns) if trace else C.reshape(n, ns, 6, 6)


class GPField:
    """A GP factor field held by the oracle (all voxels, or a sparse subset)."""

    def __init__(self, C, origin, h, shape, Z, length, trace=False, voxel_ids=None):
        self.Z = _f64(Z, 3)
        self.ns = self.Z.shape[0]
        self.trace = bool(trace)
        per = self.ns if trace else self.ns * 36
        self.C = np.ascontiguousarray(C, dtype=np.float64).reshape(-1, per)
        self.origin, self.h, self.shape = tuple(origin), float(h), tuple(int(s) for s in shape)
        self.length = float(length)
        if voxel_ids is not None:
            order = np.argsort(voxel_ids, kind="stable")
            self.ids = np.ascontiguousarray(np.asarray(voxel_ids, np.int64)[order])
            self.C = np.ascontiguousarray(self.C[order])
        else:
            self.ids = None
        self.grid = _grid(self.origin, self.h, self.shape)


def gp_query(field: GPField, t, q, metrics_mask=7, interp=0, want_fim=False):
    t = _f64(t, 3)
    q = _f64(q, 4)
    m = t.shape[0]
    nc = 1 if field.trace else ncols(metrics_mask)
    out = np.zeros((m, nc))
    flags = np.zeros(m, np.uint8)
    F = np.zeros((m, 36)) if (want_fim and not field.trace) else None
    n = field.ids.shape[0] if field.ids is not None else field.C.shape[0]
    rc = lib().oracle_gp_query(_p(field.C), _p(field.ids), ctypes.c_int64(n),
                               ctypes.byref(field.grid), ctypes.c_int(field.ns),
                               ctypes.c_int(1 if field.trace else 0), _p(field.Z),
                               ctypes.c_double(field.length), _p(t), _p(q), ctypes.c_int64(m),
                               ctypes.c_uint32(metrics_mask), ctypes.c_int(interp), _p(out),
                               _p(flags), _p(F))
    if rc != 0:
        raise KeyError("oracle GP field is missing a voxel the query needs")
    if want_fim and F is not None:
        return out, flags, F.reshape(m, 6, 6)
    return out, flags


def gp_pc_fim(landmarks, sigma, r_min, r_max, Z, ks, alpha, length, Ainv, t, q) -> np.ndarray:
    lm = _f64(landmarks, 3)
    Z = _f64(Z, 3)
    t = _f64(t, 3)
    q = _f64(q, 4)
    m = t.shape[0]
    F = np.zeros((m, 36))
    lib().oracle_gp_pc_fim(_p(lm), ctypes.c_int64(lm.shape[0]), ctypes.c_double(sigma),
                           ctypes.c_double(r_min), ctypes.c_double(r_max), ctypes.c_int(Z.shape[0]),
                           _p(Z), ctypes.c_double(ks), ctypes.c_double(alpha),
                           ctypes.c_double(length), _p(_f64(Ainv)), _p(t), _p(q),
                           ctypes.c_int64(m), _p(F))
    return F.reshape(m, 6, 6)


def gp_lml(Z, ks, alpha, length, noise, U) -> float:
    f = lib().oracle_gp_lml
    f.restype = ctypes.c_double
    Z = _f64(Z, 3)
    U = _f64(U, 3)
    return f(ctypes.c_int(Z.shape[0]), _p(Z), ctypes.c_double(ks), ctypes.c_double(alpha),
             ctypes.c_double(length), ctypes.c_double(noise), _p(U), ctypes.c_int(U.shape[0]))


def gp_fit_length(Z, ks, alpha, noise, U, lo=0.05, hi=3.0, iters=60) -> float:
    """ML-II length scale (Sec. V-B): golden-section search of gp_lml over
    log l in [lo, hi] (the evidence is unimodal in l for these data)."""
    a, b = np.log(lo), np.log(hi)
    gr = (np.sqrt(5.0) - 1.0) / 2.0
    c, d = b - gr * (b - a), a + gr * (b - a)
    fc, fd = gp_lml(Z, ks, alpha, np.exp(c), noise, U), gp_lml(Z, ks, alpha, np.exp(d), noise, U)
    for _ in range(iters):
        if fc > fd:
            b, d, fd = d, c, fc
            c = b - gr * (b - a)
            fc = gp_lml(Z, ks, alpha, np.exp(c), noise, U)
        else:
            a, c, fc = c, d, fd
            d = a + gr * (b - a)
            fd = gp_lml(Z, ks, alpha, np.exp(d), noise, U)
    return float(np.exp((a + b) / 2))


def corner_voxels(origin, h, shape, t) -> np.ndarray:
    """Voxel ids the trilinear query of each position reads (for sparse builds)."""
    t = _f64(t, 3)
    n = np.array(shape)
    g = (t - np.asarray(origin)) / h
    i0 = np.clip(np.floor(g), 0, np.maximum(n - 2, 0)).astype(np.int64)
    ids = []
    for j in range(8):
        b = np.array([j & 1, (j >> 1) & 1, (j >> 2) & 1])
        idx = np.minimum(i0 + b * (n > 1), n - 1)
        ids.append(idx[:, 0] + n[0] * (idx[:, 1] + n[1] * idx[:, 2]))
    ni = np.clip(np.floor(g + 0.5), 0, n - 1).astype(np.int64)
    ids.append(ni[:, 0] + n[0] * (ni[:, 1] + n[1] * ni[:, 2]))
    return np.unique(np.concatenate(ids))


# ------------------------------------------------------------ point cloud

def pc_query(landmarks, alpha, v_alpha, sigma, r_min, r_max, t, q, metrics_mask,
             pinhole=None, want_fim=False, want_margin=False):
    lm = _f64(landmarks, 3)
    t = _f64(t, 3)
    q = _f64(q, 4)
    m = t.shape[0]
    out = np.zeros((m, ncols(metrics_mask)))
    F = np.zeros((m, 36)) if want_fim else None
    margin = np.zeros(m) if want_margin else None
    cam = None
    if pinhole is not None:
        cam = _Pinhole(*[float(x) for x in pinhole[:4]], int(pinhole[4]), int(pinhole[5]))
    lib().oracle_pc_query(_p(lm), ctypes.c_int64(lm.shape[0]), ctypes.c_double(alpha),
                          ctypes.c_double(v_alpha), ctypes.c_double(sigma),
                          ctypes.c_double(r_min), ctypes.c_double(r_max),
                          ctypes.byref(cam) if cam is not None else None, _p(t), _p(q),
                          ctypes.c_int64(m), ctypes.c_uint32(metrics_mask), _p(out), _p(F),
                          _p(margin))
    res = [out]
    if want_fim:
        res.append(F.reshape(m, 6, 6))
    if want_margin:
        res.append(margin)
    return res[0] if len(res) == 1 else tuple(res)


def num_threads() -> int:
    f = lib().oracle_num_threads
    f.restype = ctypes.c_int
    return int(f())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from here on."""
    lib().oracle_set_num_threads(ctypes.c_int(int(n)))
