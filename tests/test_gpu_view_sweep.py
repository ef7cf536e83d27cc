"""GPU parity of the optimal-view sweep (fif_view_sweep) against the FP64 oracle.

Values are compared element by element; the best index is checked for validity
(the oracle's value at the GPU's choice is within the tolerance of the oracle's
maximum, and the GPU's choice is the first maximiser of its own values), since
near-ties may legitimately resolve differently under rounding.
"""
import numpy as np
import pytest

import oracle
import scenes
from fifcheck import metric_errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

METRICS = {"trace": 1, "lmin": 2, "logdet": 4}


@pytest.fixture(scope="module")
def fif():
    import paper_2008_03324_amd as fif
    fif.lib()
    return fif


@pytest.fixture(scope="module")
def tiny():
    lm, g, v = scenes.tiny_scene()
    C = oracle.build(lm, g.origin, g.h, g.shape, v.sigma)
    ofield = oracle.Field(C, g.origin, g.h, g.shape)
    rng = np.random.default_rng(70)
    t = rng.uniform(-5.5, 5.5, (40, 3)) * np.array([1, 1, 0.4])   # some outside: clamped
    dirs = scenes.sphere_axes(300)
    dirs = np.concatenate([dirs, dirs[17:18], np.zeros((1, 3)), 2.5 * dirs[40:41]])
    return dict(lm=lm, g=g, v=v, ofield=ofield, t=t, dirs=dirs)


def _field(fif, lm, g, v, prec):
    grid = fif.Grid(g.origin, g.h, g.shape)
    vis = fif.Vis(v.half_fov, v.v_alpha, v.sigma, v.r_min, v.r_max)
    return fif.build(torch.tensor(lm, dtype=torch.float64, device="cuda"), grid, vis, prec=prec)


def _check_best(best, values, ref_values, tol_of):
    """best: GPU indices; values: GPU values; ref_values: oracle values."""
    for a in range(values.shape[0]):
        row, ref = values[a], ref_values[a]
        if np.isnan(row).all():
            assert best[a] == -1
            continue
        first = int(np.nanargmax(row))
        assert best[a] == first, (a, best[a], first)
        assert ref[best[a]] >= np.nanmax(ref) - tol_of(ref), a


@pytest.mark.parametrize("interp", [0, 1])
@pytest.mark.parametrize("metric", ["trace", "lmin", "logdet"])
def test_sweep_fp64_matches_oracle(fif, tiny, metric, interp):
    print(f"case: tiny view sweep FP64 {metric} interp={interp}", flush=True)
    field = _field(fif, tiny["lm"], tiny["g"], tiny["v"], fif.FP64)
    m = METRICS[metric]
    t_d = torch.tensor(tiny["t"], dtype=torch.float64, device="cuda")
    d_d = torch.tensor(tiny["dirs"], dtype=torch.float64, device="cuda")
    vals, best = fif.view_sweep(field, t_d, d_d, m, interp=interp)
    vals, best = vals.cpu().numpy(), best.cpu().numpy()
    v = tiny["v"]
    ref, rbest = oracle.view_sweep(tiny["ofield"], v.half_fov, v.v_alpha, tiny["t"],
                                   tiny["dirs"], m, interp)
    assert np.array_equal(np.isnan(vals), np.isnan(ref))
    ok = ~np.isnan(ref)
    scale = np.nanmax(np.abs(ref), axis=1, keepdims=True)
    if metric == "logdet":
        err = np.abs(vals - ref)[ok]
        assert err.max() <= 1e-8, err.max()
        tol_of = lambda r: 1e-8  # noqa: E731
    else:
        err = (np.abs(vals - ref) / scale)[ok]
        assert err.max() <= 1e-10, err.max()
        tol_of = lambda r: 1e-10 * np.nanmax(np.abs(r))  # noqa: E731
    assert np.isnan(vals[:, 301]).all()                     # the zero axis
    assert (vals[:, 300] == vals[:, 17]).all()               # exact duplicate
    _check_best(best, vals, ref, tol_of)
    # the sweep equals plain queries whose orientation looks along each axis
    q = np.stack([scenes.rotation_to_quaternion(_axis_rotation(d)) for d in tiny["dirs"][:64]])
    tq = np.repeat(tiny["t"][:3], 64, 0)
    qq = np.tile(q, (3, 1))
    out = fif.query(field, torch.tensor(tq, device="cuda"), torch.tensor(qq, device="cuda"), m,
                    interp=interp).cpu().numpy()[:, 0].reshape(3, 64)
    dq = np.abs(out - vals[:3, :64])
    if metric == "logdet":
        assert dq.max() <= 1e-8
    else:
        assert (dq / scale[:3]).max() <= 1e-10


def _axis_rotation(z):
    z = np.asarray(z, float) / np.linalg.norm(z)
    a = np.array([1.0, 0, 0]) if abs(z[0]) < 0.9 else np.array([0, 1.0, 0])
    x = np.cross(a, z)
    x /= np.linalg.norm(x)
    return np.stack([x, np.cross(z, x), z], axis=1)


def test_sweep_fp32_field_within_bar(fif, tiny):
    print("case: tiny view sweep FP32_COMP, three metrics", flush=True)
    field = _field(fif, tiny["lm"], tiny["g"], tiny["v"], fif.FP32_COMP)
    t32 = tiny["t"].astype(np.float32)
    t_d = torch.tensor(t32, device="cuda")
    dirs = tiny["dirs"][:300]
    d_d = torch.tensor(dirs, dtype=torch.float64, device="cuda")
    v = tiny["v"]
    cols = []
    refs = []
    for name in ("trace", "lmin", "logdet"):
        vals, best = fif.view_sweep(field, t_d, d_d, METRICS[name])
        cols.append(vals.cpu().numpy().reshape(-1))
        ref, _ = oracle.view_sweep(tiny["ofield"], v.half_fov, v.v_alpha,
                                   t32.astype(np.float64), dirs, METRICS[name])
        refs.append(ref.reshape(-1))
    # full FIMs of the same poses scale the lambda_min measure
    q = np.stack([scenes.rotation_to_quaternion(_axis_rotation(d)) for d in dirs])
    tq = np.repeat(t32.astype(np.float64), len(dirs), 0)
    F = oracle.query_fim(tiny["ofield"], v.half_fov, v.v_alpha, tq, np.tile(q, (len(t32), 1)))
    iu = np.triu_indices(6)
    err = metric_errors(np.stack(cols, 1), np.stack(refs, 1), F[:, iu[0], iu[1]])
    print({k: float(np.nanmax(e)) for k, e in err.items()})
    nan_mismatch = np.mean(np.isnan(cols[2]) != np.isnan(refs[2]))
    assert nan_mismatch <= 1e-3, nan_mismatch        # only borderline-PD FIMs may differ
    assert err["trace_rel"].max() <= 1e-3
    assert err["lmin_weyl"].max() <= 1e-3
    assert np.nanmax(err["logdet_abs"]) <= 1e-3


def test_sweep_building_200_positions_sampled(fif):
    """The optimal-view workload at full size: 200 positions of the building
    scene, 4096 axes, FP32 field; 12 positions checked against the oracle."""
    print("case: building view sweep 200 x 4096, FP32_COMP", flush=True)
    lm, g, v = scenes.building_scene()
    field = _field(fif, lm, g, v, fif.FP32_COMP)
    t = scenes.sweep_positions(g, 200)
    dirs = scenes.sphere_axes(4096)
    vals, best = fif.view_sweep(field, torch.tensor(t, device="cuda"),
                                torch.tensor(dirs, device="cuda"), METRICS["logdet"])
    vals, best = vals.cpu().numpy(), best.cpu().numpy()
    assert np.isfinite(vals).all()
    pick = np.random.default_rng(71).choice(200, 12, replace=False)
    t64 = t[pick].astype(np.float64)
    ids = oracle.corner_voxels(g.origin, g.h, g.shape, t64)
    C = oracle.build(lm, g.origin, g.h, g.shape, v.sigma, v.r_min, v.r_max, voxel_ids=ids)
    of = oracle.Field(C, g.origin, g.h, g.shape, voxel_ids=ids)
    ref, rbest = oracle.view_sweep(of, v.half_fov, v.v_alpha, t64, dirs, METRICS["logdet"])
    err = np.abs(vals[pick] - ref)
    print("logdet abs err max", float(err.max()))
    assert err.max() <= 1e-3
    _check_best(best[pick], vals[pick], ref, lambda r: 2e-3)


def test_sweep_edge_cases(fif, tiny):
    print("case: view sweep edge cases", flush=True)
    field = _field(fif, tiny["lm"], tiny["g"], tiny["v"], fif.FP64)
    t_d = torch.tensor(tiny["t"][:5], dtype=torch.float64, device="cuda")
    empty = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    vals, best = fif.view_sweep(field, t_d, empty, 1)
    assert vals.shape == (5, 0) and (best.cpu() == -1).all()
    vals, best = fif.view_sweep(field, empty, torch.ones((3, 3), dtype=torch.float64,
                                                         device="cuda"), 1)
    assert vals.shape == (0, 3) and best.shape == (0,)
    # values not wanted: best alone
    d_d = torch.tensor(tiny["dirs"][:300], dtype=torch.float64, device="cuda")
    v1, b1 = fif.view_sweep(field, t_d, d_d, 4)
    v2, b2 = fif.view_sweep(field, t_d, d_d, 4, want_values=False)
    assert v2 is None and torch.equal(b1, b2)
    with pytest.raises(fif.FifError):
        fif.view_sweep(field, t_d, d_d, 3)
    grid = fif.Grid(tiny["g"].origin, tiny["g"].h, tiny["g"].shape)
    vis = fif.Vis(tiny["v"].half_fov, tiny["v"].v_alpha, tiny["v"].sigma)
    ftr = fif.build(torch.tensor(tiny["lm"], device="cuda"), grid, vis, prec=fif.FP64,
                    kind=fif.KIND_TRACE)
    with pytest.raises(fif.FifError):
        fif.view_sweep(ftr, t_d, d_d, 1)
