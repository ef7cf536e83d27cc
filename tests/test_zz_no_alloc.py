"""fif_build_noalloc (the build with the library's static scratch instead of a
workspace) against fif_build given a workspace: the same field bit for bit on
two calls in a row, the second with fewer landmarks, for an information field
in FP32-compensated and FP64 and a trace field; an empty landmark set; a
landmark count whose sort needs more than the static scratch is refused on the
host before anything is enqueued.  Calls go through the C ABI."""
import ctypes

import numpy as np
import pytest

import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _noalloc(fif, lm_d, n, field):
    L = fif.lib()
    st = L.fif_build_noalloc(ctypes.c_void_p(lm_d.data_ptr()), n, ctypes.byref(field.cstruct),
                             None)
    return st


def _workspace_build(fif, lm_d, n, field):
    L = fif.lib()
    nbytes = L.fif_workspace_bytes(ctypes.byref(field.grid.c()), n, field.prec)
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")
    st = L.fif_build(ctypes.c_void_p(lm_d.data_ptr()), n, ctypes.byref(field.cstruct),
                     ctypes.c_void_p(ws.data_ptr()) if nbytes else None, nbytes, None)
    torch.cuda.synchronize()
    return st


def test_noalloc_build_equals_workspace_build():
    import paper_2008_03324_amd as fif
    print("case: fif_build_noalloc vs fif_build with a workspace, building scene", flush=True)
    lm, g, v = scenes.building_scene()
    grid = fif.Grid(g.origin, g.h, g.shape)
    vis = fif.Vis(v.half_fov, v.v_alpha, v.sigma, v.r_min, v.r_max)
    lm_d = torch.tensor(lm, dtype=torch.float64, device="cuda")
    L = fif.lib()
    for n in (1000, 100_000, 900_000):
        print("workspace bytes for", n, "landmarks:",
              L.fif_workspace_bytes(ctypes.byref(grid.c()), n, fif.FP32_COMP), flush=True)
    for prec, kind in ((fif.FP32_COMP, fif.KIND_INFO), (fif.FP64, fif.KIND_INFO),
                       (fif.FP32_COMP, fif.KIND_TRACE)):
        for n in (100_000, 37_001):  # two calls in a row, the second smaller
            a = fif.Field(grid, vis, prec, kind)
            b = fif.Field(grid, vis, prec, kind)
            a.buffer.fill_(7)
            b.buffer.fill_(9)
            assert _noalloc(fif, lm_d, n, a) == 0, L.fif_last_error()
            torch.cuda.synchronize()
            assert _workspace_build(fif, lm_d, n, b) == 0
            same = torch.equal(a.buffer, b.buffer)
            print(prec, kind, n, "bitwise equal" if same else "DIFFERENT", flush=True)
            assert same
    # the Python binding of the same entry point
    c = fif.build_noalloc(lm_d[:5000], grid, vis, prec=fif.FP32_COMP)
    d = fif.build(lm_d[:5000], grid, vis, prec=fif.FP32_COMP, sort=True)
    torch.cuda.synchronize()
    assert torch.equal(c.buffer, d.buffer)


def test_noalloc_empty_and_limits():
    import paper_2008_03324_amd as fif
    print("case: fif_build_noalloc, empty input and the scratch limit", flush=True)
    L = fif.lib()
    grid = fif.Grid((-1.0, -1.0, -0.5), 0.25, (9, 9, 5))
    vis = fif.Vis()
    rng = np.random.default_rng(5)
    lm_d = torch.from_numpy(rng.uniform(-2, 2, (2_000_000, 3))).cuda()
    a = fif.Field(grid, vis, fif.FP64)
    a.buffer.fill_(3)
    assert _noalloc(fif, lm_d, 0, a) == 0
    torch.cuda.synchronize()
    assert int(a.buffer.count_nonzero()) == 0
    # 2M landmarks need about 144 MB of scratch: refused, nothing enqueued
    a.buffer.fill_(3)
    assert _noalloc(fif, lm_d, 2_000_000, a) == -1
    assert b"static scratch" in L.fif_last_error()
    torch.cuda.synchronize()
    assert bool((a.buffer == 3).all())
    # a small build after the refusal still matches
    b = fif.Field(grid, vis, fif.FP64)
    assert _noalloc(fif, lm_d, 3000, a) == 0
    assert _workspace_build(fif, lm_d, 3000, b) == 0
    assert torch.equal(a.buffer, b.buffer)
