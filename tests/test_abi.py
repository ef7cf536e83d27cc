"""The C-ABI library loads and exports every symbol of include/fif.h (CPU only).

Only calls that return before touching the GPU are made: sizes, status strings
and host-side argument validation.
"""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fif.h")


def _lib():
    import paper_2008_03324_amd as fif
    if not os.path.exists(fif.LIB_PATH):
        from paper_2008_03324_amd import buildlib
        buildlib.build()
    return fif, fif.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("fif_", "pc_"))))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("fif_build", "fif_query", "fif_query_grad", "pc_query", "fif_field_bytes",
                 "fif_workspace_bytes", "fif_update", "fif_field_export", "fif_status_string",
                 "fif_last_error"):
        assert want in names


def test_library_exports_every_declared_symbol():
    fif, L = _lib()
    for name in declared_functions():
        assert hasattr(L, name), f"libfif.so does not export {name}"
        assert name in fif.EXPORTS, f"binding does not bind {name}"


def test_field_bytes_and_status_strings():
    fif, L = _lib()
    g = fif.Grid((0.0, 0.0, 0.0), 0.5, (20, 20, 6))
    assert fif.field_bytes(g, fif.FP32_COMP) == 2400 * 80 * 4
    assert fif.field_bytes(g, fif.FP64) == 2400 * 80 * 8
    assert fif.field_bytes(g, fif.FP32_NAIVE, fif.KIND_TRACE) == 2400 * 12 * 4
    bad = fif.Grid((0.0, 0.0, 0.0), -1.0, (20, 20, 6))
    assert fif.field_bytes(bad, fif.FP64) == 0
    assert fif.field_bytes(fif.Grid((0, 0, 0), 0.5, (0, 1, 1)), fif.FP64) == 0
    assert fif.field_bytes(g, 7) == 0
    for s in (0, -1, -2, -3, -4):
        assert L.fif_status_string(s).decode().startswith(fif.STATUS[s])
    assert L.fif_workspace_bytes(ctypes.byref(g.c()), 0, fif.FP32_COMP) == 0
    assert L.fif_workspace_bytes(ctypes.byref(bad.c()), 1000, fif.FP32_COMP) == 0


def test_host_side_validation_returns_einval():
    """Every check below fails before anything is enqueued (no GPU needed)."""
    fif, L = _lib()
    g = fif.Grid((0.0, 0.0, 0.0), 0.5, (4, 4, 4))
    vis = fif.Vis()
    f = fif.CField(g.c(), vis.c(), fif.FP64, fif.KIND_INFO, None)  # NULL data
    assert L.fif_build(None, 10, ctypes.byref(f), None, 0, None) == -1
    assert b"NULL" in L.fif_last_error()
    f.data = 4096
    assert L.fif_build(None, 10, ctypes.byref(f), None, 0, None) == -1  # NULL landmarks
    assert L.fif_build(None, -1, ctypes.byref(f), None, 0, None) == -1
    assert L.fif_update(None, 1, 2, ctypes.byref(f), None, 0, None) == -1  # bad sign
    assert L.fif_query(ctypes.byref(f), None, None, 5, 0, 0, None, None, None) == -1  # no metric
    assert L.fif_query(ctypes.byref(f), None, None, 5, 1, 3, None, None, None) == -1  # interp
    assert L.fif_query(ctypes.byref(f), None, None, 5, 1, 0, None, None, None) == -1  # NULL t
    assert L.fif_query(ctypes.byref(f), None, None, 0, 1, 0, None, None, None) == 0   # m = 0
    assert L.fif_query_grad(ctypes.byref(f), None, None, 5, 8, None, None, None, None,
                            None) == -1  # FIM21 has no gradient
    ftr = fif.CField(g.c(), vis.c(), fif.FP64, fif.KIND_TRACE, 4096)
    assert L.fif_query(ctypes.byref(ftr), None, None, 5, 2, 0, None, None, None) == -1
    assert L.fif_query_grad(ctypes.byref(ftr), None, None, 5, 1, None, None, None, None,
                            None) == -4
    badvis = fif.Vis(sigma=0.0)
    assert L.pc_query(None, 0, ctypes.byref(badvis.c()), None, 2, None, None, 1, 1, None,
                      None, 0, None) == -1
    cam = fif.CPinhole(-1.0, 300.0, 300.0, 300.0, 600, 600)
    assert L.pc_query(None, 0, ctypes.byref(vis.c()), ctypes.byref(cam), 2, None, None, 1, 1,
                      None, None, 0, None) == -1
    # a misaligned point-cloud workspace is refused before anything runs
    vis15 = fif.Vis(r_max=15.0)
    assert L.pc_query(4096, 10, ctypes.byref(vis15.c()), None, 2, 4096, 4096, 1, 1, 4096, 4100,
                      1 << 20, None) == -1
    assert b"aligned" in L.fif_last_error()
    assert L.pc_workspace_bytes(0, 10, 1) == 0 and L.pc_workspace_bytes(10, 0, 1) == 0
    assert L.pc_workspace_bytes(10, 10, 7) == 0
    assert L.fif_field_export(ctypes.byref(f), None, 3, None, None) == -1
    # view sweep: exactly one metric, information fields, valid interp, t/dirs
    assert L.fif_view_sweep(ctypes.byref(f), None, 4, None, 8, 3, 0, None, None, None) == -1
    assert L.fif_view_sweep(ctypes.byref(f), None, 4, None, 8, 8, 0, None, None, None) == -1
    assert L.fif_view_sweep(ctypes.byref(f), None, 4, None, 8, 1, 2, None, None, None) == -1
    assert L.fif_view_sweep(ctypes.byref(f), None, 4, None, 8, 1, 0, None, None, None) == -1
    assert L.fif_view_sweep(ctypes.byref(f), None, -1, None, 8, 1, 0, None, None, None) == -1
    assert L.fif_view_sweep(ctypes.byref(f), None, 0, None, 8, 4, 0, None, None, None) == 0
    assert L.fif_view_sweep(ctypes.byref(ftr), None, 4, None, 8, 1, 0, None, None,
                            None) == -4
    gb = g.c()
    gb.reserved = 1
    fb = fif.CField(gb, vis.c(), fif.FP64, fif.KIND_INFO, 4096)
    assert L.fif_query(ctypes.byref(fb), None, None, 1, 1, 0, None, None, None) == -1
    # grids one build launch cannot cover: unsupported, refused before any launch
    for shape in ((1 << 28, 1, 1), (1, 600_000, 1), (1, 1, 300_000)):
        fw = fif.CField(fif.Grid((0.0, 0.0, 0.0), 0.5, shape).c(), vis.c(), fif.FP32_COMP,
                        fif.KIND_INFO, 4096)
        assert L.fif_build(None, 0, ctypes.byref(fw), None, 0, None) == -4, shape
        assert L.fif_update(None, 5, 1, ctypes.byref(fw), None, 0, None) == -1  # NULL landmarks


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_2008_03324_amd as fif
    monkeypatch.setattr(fif, "_lib", None)
    monkeypatch.setattr(fif, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        fif.lib()


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2008_03324_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "oracle/" not in text, fn
                assert "fif_oracle" not in text, fn


def test_gp_host_side_validation():
    """GP entry points reject bad models and arguments before enqueuing anything."""
    fif, L = _lib()
    g = fif.Grid((0.0, 0.0, 0.0), 0.5, (4, 4, 4))
    vis = fif.Vis()
    gp = fif.CGP(30, 0, 15.0, 0.9, 1e-10, 4096, 8192)
    assert L.fif_gp_field_bytes(ctypes.byref(g.c()), 30, fif.FP32_COMP, fif.KIND_INFO) == 64 * 30 * 16 * 4
    assert L.fif_gp_field_bytes(ctypes.byref(g.c()), 30, fif.FP64, fif.KIND_TRACE) == 64 * 30 * 8
    # trace rows hold N_s factors rounded up to an even count
    assert L.fif_gp_field_bytes(ctypes.byref(g.c()), 31, fif.FP32_COMP, fif.KIND_TRACE) == 64 * 32 * 4
    assert L.fif_gp_field_bytes(ctypes.byref(g.c()), 0, fif.FP64, fif.KIND_INFO) == 0
    assert L.fif_gp_field_bytes(ctypes.byref(g.c()), 161, fif.FP64, fif.KIND_INFO) == 0
    for bad in (fif.CGP(0, 0, 15.0, 0.9, 1e-10, 4096, 8192),      # no axes
                fif.CGP(200, 0, 15.0, 0.9, 1e-10, 4096, 8192),    # too many axes
                fif.CGP(30, 1, 15.0, 0.9, 1e-10, 4096, 8192),     # reserved
                fif.CGP(30, 0, -1.0, 0.9, 1e-10, 4096, 8192),     # k_s
                fif.CGP(30, 0, 15.0, 0.0, 1e-10, 4096, 8192),     # length
                fif.CGP(30, 0, 15.0, 0.9, -1.0, 4096, 8192),      # noise
                fif.CGP(30, 0, 15.0, 0.9, 1e-10, None, 8192),     # axes NULL
                fif.CGP(30, 0, 15.0, 0.9, 1e-10, 4096, None)):    # kinv NULL
        assert L.fif_gp_setup(ctypes.byref(bad), None) == -1
    assert L.fif_gp_evidence(ctypes.byref(gp), 0.0, None, 0, None, 1, None, None) == -1  # fov
    assert L.fif_gp_evidence(ctypes.byref(gp), 0.7, None, 10, None, 1, None, None) == -1  # NULL
    assert L.fif_gp_evidence(ctypes.byref(gp), 0.7, None, 0, None, 0, None, None) == 0   # nothing
    f = fif.CGPField(g.c(), vis.c(), gp, fif.FP32_COMP, fif.KIND_INFO, None)        # NULL data
    assert L.fif_gp_build(None, 10, ctypes.byref(f), None, 0, None) == -1
    f.data = 4096
    assert L.fif_gp_build(None, 10, ctypes.byref(f), None, 0, None) == -1               # NULL landmarks
    assert L.fif_gp_build(None, -1, ctypes.byref(f), None, 0, None) == -1
    assert L.fif_gp_query(ctypes.byref(f), None, None, 5, 0, 0, None, None, None) == -1  # no metric
    assert L.fif_gp_query(ctypes.byref(f), None, None, 5, 1, 2, None, None, None) == -1  # interp
    assert L.fif_gp_query(ctypes.byref(f), None, None, 5, 1, 0, None, None, None) == -1  # NULL t
    assert L.fif_gp_query(ctypes.byref(f), None, None, 0, 7, 0, None, None, None) == 0   # m = 0
    ft = fif.CGPField(g.c(), vis.c(), gp, fif.FP32_COMP, fif.KIND_TRACE, 4096)
    assert L.fif_gp_query(ctypes.byref(ft), None, None, 5, 2, 0, None, None, None) == -1
    assert L.fif_gp_export(ctypes.byref(f), None, 3, None, None) == -1
    assert L.fif_gp_export(ctypes.byref(f), None, 0, None, None) == 0


def test_serve_host_side_validation():
    """fif_serve_run refuses bad configurations, fields and requests before it
    creates a stream or enqueues anything."""
    fif, L = _lib()
    g = fif.Grid((0.0, 0.0, 0.0), 0.5, (4, 4, 4))
    vis = fif.Vis()
    ok = fif.CServeConfig(2, 8, 1 << 20, 1024, 1, 0)
    assert L.fif_serve_workspace_bytes(ctypes.byref(ok)) > 0
    for bad in (fif.CServeConfig(0, 8, 1 << 20, 1024, 1, 0), fif.CServeConfig(17, 8, 1 << 20, 1024, 1, 0),
                fif.CServeConfig(2, 0, 1 << 20, 1024, 1, 0), fif.CServeConfig(2, 8, 0, 1024, 1, 0),
                fif.CServeConfig(2, 8, 1 << 20, 0, 1, 0)):
        assert L.fif_serve_workspace_bytes(ctypes.byref(bad)) == 0
    fields = (fif.CField * 1)(fif.CField(g.c(), vis.c(), fif.FP32_COMP, fif.KIND_INFO, 4096))
    el = ctypes.c_double()
    ones = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    req = (fif.CServeRequest * 1)(fif.CServeRequest(0.0, 0, 0, 10, 4096, 4096, 4096, None, None,
                                                    ones, 0.0, 0.0))
    run = lambda f, nf, r, n, c, ws, nb: L.fif_serve_run(f, nf, r, n, ctypes.byref(c), ws, nb,
                                                         ctypes.byref(el))
    bad_cfg = fif.CServeConfig(0, 8, 1 << 20, 1024, 1, 0)
    assert run(fields, 1, req, 1, bad_cfg, 4096, 1 << 30) == -1
    assert run(fields, 0, req, 1, ok, 4096, 1 << 30) == -1
    trace = (fif.CField * 1)(fif.CField(g.c(), vis.c(), fif.FP32_COMP, fif.KIND_TRACE, 4096))
    assert run(trace, 1, req, 1, ok, 4096, 1 << 30) == -1  # serving needs information fields
    for fld, kind, m in ((1, 0, 10), (0, 2, 10), (0, 0, 0), (0, 0, 2048), (0, 1, 10)):
        # field index, kind, m < 1, m > max_batch, gradient buffers missing
        r = (fif.CServeRequest * 1)(fif.CServeRequest(0.0, fld, kind, m, 4096, 4096, 4096, None,
                                                      None, ones, 0.0, 0.0))
        assert run(fields, 1, r, 1, ok, 4096, 1 << 30) == -1, (fld, kind, m)
    nan_w = (ctypes.c_double * 3)(1.0, float("nan"), 1.0)
    r = (fif.CServeRequest * 1)(fif.CServeRequest(0.0, 0, 1, 10, 4096, 4096, 4096, 4096, 4096,
                                                  nan_w, 0.0, 0.0))
    assert run(fields, 1, r, 1, ok, 4096, 1 << 30) == -1
    assert b"weights" in L.fif_last_error()
    small = fif.CServeConfig(2, 8, 100, 1024, 1, 0)  # 10 poses need 240 B
    assert run(fields, 1, req, 1, small, 4096, 1 << 30) == -1
    assert b"budget" in L.fif_last_error()
    need = L.fif_serve_workspace_bytes(ctypes.byref(ok))
    assert run(fields, 1, req, 1, ok, 4096, need - 1) == -2
    assert run(fields, 1, req, 0, ok, 4096, need) == 0  # nothing to serve
