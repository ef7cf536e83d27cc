"""Inputs longer than one launch can cover.  A dispatch holds its grid size in
work-items as a 32-bit number, so the one-lane-per-item kernels are launched
on slices of at most 2^30 items; these tests run 2^30 + 1000 poses (and
correspondingly many sweep positions and GP export items) and check the items
on both sides of every slice boundary against the same items computed in a
small call of their own (bitwise)."""
import numpy as np
import pytest

import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SLICE = 1 << 30


@pytest.fixture(scope="module")
def fif():
    import paper_2008_03324_amd as fif
    fif.lib()
    return fif


@pytest.fixture(scope="module")
def big_poses():
    print("case: 2^30 + 1000 poses (30 GB of FP32 poses)", flush=True)
    lm, g, v = scenes.building_scene(n_landmarks=20_000, shape=(64, 64, 32))
    m = SLICE + 1000
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2101)
    lo = torch.tensor(g.hull_lo, dtype=torch.float32, device="cuda")
    hi = torch.tensor(g.hull_hi, dtype=torch.float32, device="cuda")
    t = lo + (hi - lo) * torch.rand((m, 3), generator=gen, device="cuda", dtype=torch.float32)
    q = torch.randn((m, 4), generator=gen, device="cuda", dtype=torch.float32)
    torch.cuda.synchronize()
    yield lm, g, v, t, q
    del t, q
    torch.cuda.empty_cache()


def _probe_rows():
    return np.concatenate([np.arange(0, 3), np.arange(SLICE - 3, SLICE + 5),
                           np.arange(SLICE + 995, SLICE + 1000)])


def _check_rows(big_out, fn, t, q):
    rows = torch.from_numpy(_probe_rows()).cuda()
    small = fn(t[rows].contiguous(), q[rows].contiguous())
    assert torch.equal(big_out[rows].nan_to_num(7.0), small.nan_to_num(7.0))


def test_trace_query_and_point_cloud_past_one_launch(fif, big_poses):
    lm, g, v, t, q = big_poses
    grid = fif.Grid(g.origin, g.h, g.shape)
    vis = fif.Vis(v.half_fov, v.v_alpha, v.sigma, v.r_min, v.r_max)
    lm_d = torch.tensor(lm, dtype=torch.float64, device="cuda")
    tf = fif.build(lm_d, grid, vis, prec=fif.FP32_COMP, kind=fif.KIND_TRACE)
    out = fif.query(tf, t, q, fif.TRACE)
    assert bool(torch.isfinite(out).all())
    _check_rows(out, lambda a, b: fif.query(tf, a, b, fif.TRACE), t, q)
    del out
    few = lm_d[:50].contiguous()
    for sort in (True, False):  # poses sorted in passes of 2^26, and the plain pass
        pc = fif.pc_query(few, vis, t, q, fif.TRACE, prec=fif.FP32_COMP, sort=sort)
        _check_rows(pc, lambda a, b: fif.pc_query(few, vis, a, b, fif.TRACE,
                                                  prec=fif.FP32_COMP, sort=sort), t, q)
        del pc


def test_gp_trace_query_and_export_past_one_launch(fif, big_poses):
    lm, g, v, t, q = big_poses
    grid = fif.Grid(g.origin, g.h, g.shape)
    vis = fif.Vis(v.half_fov, v.v_alpha, v.sigma, v.r_min, v.r_max)
    ns = 30
    axes = torch.from_numpy(scenes.sphere_axes(ns)).cuda()
    model = fif.GPModel(axes, 15.0, scenes.GP_LENGTH[ns], 1e-10)
    lm_d = torch.tensor(lm, dtype=torch.float64, device="cuda")
    gf = fif.gp_build(lm_d, grid, vis, model, kind=fif.KIND_TRACE)
    out = fif.gp_query(gf, t, q, fif.TRACE)
    _check_rows(out, lambda a, b: fif.gp_query(gf, a, b, fif.TRACE), t, q)
    del out
    # export: n ids x n_s items past one launch (ids cycle through the grid)
    n = SLICE // ns + 100
    ids = torch.arange(n, device="cuda", dtype=torch.int64) % grid.n_voxels
    ex = fif.gp_export(gf, ids)
    per = SLICE // ns  # ids per launch
    rows = torch.from_numpy(np.array([0, 1, per - 2, per - 1, per, per + 1, n - 1])).cuda()
    assert torch.equal(ex[rows], fif.gp_export(gf, ids[rows].contiguous()))


def test_view_sweep_past_one_launch(fif):
    print("case: view sweep over 2^22 + 100 positions", flush=True)
    lm, g, v = scenes.building_scene(n_landmarks=20_000, shape=(64, 64, 32))
    grid = fif.Grid(g.origin, g.h, g.shape)
    vis = fif.Vis(v.half_fov, v.v_alpha, v.sigma, v.r_min, v.r_max)
    field = fif.build(torch.tensor(lm, dtype=torch.float64, device="cuda"), grid, vis,
                      prec=fif.FP32_COMP)
    per = SLICE // 512  # positions per launch (one 512-lane workgroup each)
    n = 2 * per + 100
    rng = np.random.default_rng(2102)
    t = torch.from_numpy(scenes.uniform_in_hull(rng, g, n).astype(np.float32)).cuda()
    dirs = torch.from_numpy(scenes.sphere_axes(4)).cuda()
    vals, best = fif.view_sweep(field, t, dirs, fif.LOGDET)
    rows = torch.from_numpy(np.array([0, per - 2, per - 1, per, per + 1, 2 * per - 1, 2 * per,
                                      n - 1])).cuda()
    v2, b2 = fif.view_sweep(field, t[rows].contiguous(), dirs, fif.LOGDET)
    assert torch.equal(vals[rows].nan_to_num(7.0), v2.nan_to_num(7.0))
    assert torch.equal(best[rows], b2)
