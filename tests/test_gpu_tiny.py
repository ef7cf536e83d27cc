"""GPU parity on the tiny scene (2,000 landmarks, 20x20x6 voxels, 1,000 poses).

Every output of the HIP path is compared element by element with the FP64
oracle on the same seeded inputs.  FP64 fields: blocks within 1e-10 relative,
queries within 1e-9 (trace), 1e-10 lambda_max (lmin), 1e-8 nats (logdet).
FP32 fields: 1e-3 per the measures of tests/fifcheck.py.
"""
import math

import numpy as np
import pytest

import oracle
import scenes
from fifcheck import block_rel_err, e_fim, metric_errors, upper21

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

M7 = 7


@pytest.fixture(scope="module")
def fif():
    import paper_2008_03324_amd as fif
    fif.lib()
    return fif


@pytest.fixture(scope="module")
def tiny():
    lm, g, v = scenes.tiny_scene()
    t, q = scenes.tiny_poses(g)
    C = oracle.build(lm, g.origin, g.h, g.shape, v.sigma)
    ofield = oracle.Field(C, g.origin, g.h, g.shape)
    return dict(lm=lm, g=g, v=v, t=t, q=q, C=C, ofield=ofield)


def _grid_vis(fif, g, v, v_alpha=None):
    return (fif.Grid(g.origin, g.h, g.shape),
            fif.Vis(v.half_fov, v.v_alpha if v_alpha is None else v_alpha, v.sigma, v.r_min,
                    v.r_max))


def _cuda(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def test_build_fp64_blocks_match_oracle(fif, tiny):
    print("case: tiny build FP64, all 2400 voxels", flush=True)
    grid, vis = _grid_vis(fif, tiny["g"], tiny["v"])
    field = fif.build(_cuda(tiny["lm"]), grid, vis, prec=fif.FP64)
    ids = torch.arange(grid.n_voxels, device="cuda", dtype=torch.int64)
    blocks = fif.export_blocks(field, ids).cpu().numpy()
    err = block_rel_err(blocks, tiny["C"])
    assert err.max() <= 1e-10, err.max()


@pytest.mark.parametrize("prec,tol", [("FP32_COMP", 1e-3), ("FP32_NAIVE", 1e-3)])
def test_build_fp32_blocks_match_oracle(fif, tiny, prec, tol):
    """FP32 build bar: 1e-3 relative per voxel (the FP32-build target)."""
    print(f"case: tiny build {prec}", flush=True)
    grid, vis = _grid_vis(fif, tiny["g"], tiny["v"])
    field = fif.build(_cuda(tiny["lm"]), grid, vis, prec=getattr(fif, prec))
    ids = torch.arange(grid.n_voxels, device="cuda", dtype=torch.int64)
    blocks = fif.export_blocks(field, ids).cpu().numpy()
    err = block_rel_err(blocks, tiny["C"])
    print(f"block rel err {prec}: max {err.max():.3e} median {np.median(err):.3e}")
    assert err.max() <= tol, err.max()


@pytest.mark.parametrize("interp", [0, 1])
def test_query_fp64_matches_oracle(fif, tiny, interp):
    print(f"case: tiny query FP64 interp={interp}", flush=True)
    grid, vis = _grid_vis(fif, tiny["g"], tiny["v"])
    field = fif.build(_cuda(tiny["lm"]), grid, vis, prec=fif.FP64)
    t, q = tiny["t"], tiny["q"]
    out, flags = fif.query(field, _cuda(t), _cuda(q), M7 | 8, interp=interp, want_flags=True)
    out = out.cpu().numpy()
    ref, rflags = oracle.query(tiny["ofield"], tiny["v"].half_fov, tiny["v"].v_alpha, t, q,
                               M7 | 8, interp)
    err = metric_errors(out[:, :3], ref[:, :3], ref[:, 3:])
    assert err["trace_rel"].max() <= 1e-9
    assert err["lmin_weyl"].max() <= 1e-10
    assert err["logdet_abs"].max() <= 1e-8
    assert e_fim(out[:, 3:], ref[:, 3:]).max() <= 1e-10
    np.testing.assert_array_equal(flags.cpu().numpy() & 3, rflags & 3)


def test_query_fp32_fields_match_oracle(fif, tiny):
    grid, vis = _grid_vis(fif, tiny["g"], tiny["v"])
    t32 = tiny["t"].astype(np.float32)
    q32 = tiny["q"].astype(np.float32)
    ref, _ = oracle.query(tiny["ofield"], tiny["v"].half_fov, tiny["v"].v_alpha,
                          t32.astype(np.float64), q32.astype(np.float64), M7 | 8, 0)
    for prec in (fif.FP32_COMP, fif.FP32_NAIVE):
        print(f"case: tiny query FP32 prec={prec}", flush=True)
        field = fif.build(_cuda(tiny["lm"]), grid, vis, prec=prec)
        out = fif.query(field, _cuda(t32, torch.float32), _cuda(q32, torch.float32),
                        M7 | 8).cpu().numpy()
        err = metric_errors(out[:, :3], ref[:, :3], ref[:, 3:])
        assert err["trace_rel"].max() <= 1e-3
        assert err["lmin_weyl"].max() <= 1e-3
        assert err["lmin_rel"].max() <= 1e-3
        assert err["logdet_abs"].max() <= 1e-3
        assert e_fim(out[:, 3:], ref[:, 3:]).max() <= 1e-3


def test_gradient_fp64_matches_oracle(fif, tiny):
    print("case: tiny gradient FP64", flush=True)
    grid, vis = _grid_vis(fif, tiny["g"], tiny["v"])
    field = fif.build(_cuda(tiny["lm"]), grid, vis, prec=fif.FP64)
    t, q = tiny["t"], tiny["q"]
    rng = np.random.default_rng(5)
    up = rng.standard_normal((t.shape[0], 3))
    gt, gphi, out = fif.query_grad(field, _cuda(t), _cuda(q), M7, _cuda(up), want_out=True)
    rgt, rgphi = oracle.query_grad(tiny["ofield"], tiny["v"].half_fov, tiny["v"].v_alpha, t, q,
                                   M7, up)
    # exclude repeated smallest eigenvalues (gradient undefined) and cell faces
    ref, rflags = oracle.query(tiny["ofield"], tiny["v"].half_fov, tiny["v"].v_alpha, t, q, M7, 0)
    g = (t - np.asarray(tiny["g"].origin)) / tiny["g"].h
    fr = g - np.floor(g)
    ok = ((fr > 1e-6) & (fr < 1 - 1e-6)).all(axis=1)
    gt, gphi = gt.cpu().numpy(), gphi.cpu().numpy()
    for a, b in ((gt, rgt), (gphi, rgphi)):
        scale = np.abs(b[ok]).max(axis=1, keepdims=True)
        rel = np.abs(a[ok] - b[ok]) / scale
        assert rel.max() <= 1e-7, rel.max()
    np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("prec", ["FP64", "FP32_COMP", "FP32_NAIVE"])
def test_pc_quadratic_matches_oracle(fif, tiny, prec):
    print(f"case: tiny pc quadratic {prec}", flush=True)
    grid, vis = _grid_vis(fif, tiny["g"], tiny["v"])
    p = getattr(fif, prec)
    dt = torch.float64 if p == fif.FP64 else torch.float32
    npd = np.float64 if p == fif.FP64 else np.float32
    t = tiny["t"][:256].astype(npd)
    q = tiny["q"][:256].astype(npd)
    out = fif.pc_query(_cuda(tiny["lm"]), vis, _cuda(t, dt), _cuda(q, dt), M7 | 8,
                       prec=p).cpu().numpy()
    v = tiny["v"]
    ref = oracle.pc_query(tiny["lm"], v.half_fov, v.v_alpha, v.sigma, v.r_min, v.r_max,
                          t.astype(np.float64), q.astype(np.float64), M7 | 8)
    err = metric_errors(out[:, :3], ref[:, :3], ref[:, 3:])
    tol = 1e-9 if p == fif.FP64 else 1e-4
    assert err["trace_rel"].max() <= tol
    assert err["lmin_weyl"].max() <= tol
    assert err["logdet_abs"].max() <= (1e-8 if p == fif.FP64 else 1e-3)
    assert e_fim(out[:, 3:], ref[:, 3:]).max() <= tol


@pytest.mark.parametrize("prec", ["FP64", "FP32_COMP"])
def test_pc_exact_matches_oracle(fif, tiny, prec):
    print(f"case: tiny pc exact {prec}", flush=True)
    grid, vis = _grid_vis(fif, tiny["g"], tiny["v"])
    p = getattr(fif, prec)
    dt = torch.float64 if p == fif.FP64 else torch.float32
    npd = np.float64 if p == fif.FP64 else np.float32
    t = tiny["t"][:256].astype(npd)
    q = tiny["q"][:256].astype(npd)
    out = fif.pc_query(_cuda(tiny["lm"]), vis, _cuda(t, dt), _cuda(q, dt), 1 | 8, prec=p,
                       pinhole=scenes.PINHOLE).cpu().numpy()
    v = tiny["v"]
    ref, margin = oracle.pc_query(tiny["lm"], v.half_fov, v.v_alpha, v.sigma, v.r_min, v.r_max,
                                  t.astype(np.float64), q.astype(np.float64), 1 | 8,
                                  pinhole=scenes.PINHOLE, want_margin=True)
    ok = margin > (1e-6 if p == fif.FP64 else 1e-2)
    assert ok.mean() > 0.9
    err = e_fim(out[ok, 1:], ref[ok, 1:])
    assert err.max() <= (1e-9 if p == fif.FP64 else 1e-4), err.max()


def test_field_at_voxel_centres_equals_gpu_point_cloud(fif, tiny):
    """eq:fim_separation on the GPU: nearest-voxel query at a centre == PC sum."""
    grid, vis = _grid_vis(fif, tiny["g"], tiny["v"])
    field = fif.build(_cuda(tiny["lm"]), grid, vis, prec=fif.FP64)
    rng = np.random.default_rng(3)
    ids = rng.choice(grid.n_voxels, 200, replace=False)
    g = tiny["g"]
    t = np.stack([oracle.voxel_centre(g.origin, g.h, g.shape, v) for v in ids])
    q = scenes.haar_quaternions(rng, 200)
    f_out = fif.query(field, _cuda(t), _cuda(q), 8, interp=1).cpu().numpy()
    pc_out = fif.pc_query(_cuda(tiny["lm"]), vis, _cuda(t), _cuda(q), 8,
                          prec=fif.FP64).cpu().numpy()
    assert e_fim(f_out, pc_out).max() <= 1e-10


def test_gradient_fp32_matches_oracle(fif, tiny):
    """FP32 compensated field (the persistent one-pose-per-lane gradient
    kernel): gradients against the oracle's on the oracle's FP64 factors at
    the FP32 bar, on ragged sizes (a single pose, one short of a batch, one
    past it, and all 1,000), and the forward values bitwise those of the
    forward query."""
    print("case: tiny gradient FP32 compensated, ragged sizes", flush=True)
    grid, vis = _grid_vis(fif, tiny["g"], tiny["v"])
    field = fif.build(_cuda(tiny["lm"]), grid, vis, prec=fif.FP32_COMP)
    # the poses as the FP32 field's kernels see them
    t = tiny["t"].astype(np.float32).astype(np.float64)
    q = tiny["q"].astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(6)
    up = rng.standard_normal((t.shape[0], 3))
    rgt, rgphi = oracle.query_grad(tiny["ofield"], tiny["v"].half_fov, tiny["v"].v_alpha, t, q,
                                   M7, up)
    ref, rflags = oracle.query(tiny["ofield"], tiny["v"].half_fov, tiny["v"].v_alpha, t, q, M7, 0)
    g = (t - np.asarray(tiny["g"].origin)) / tiny["g"].h
    fr = g - np.floor(g)
    ok_all = ((fr > 1e-6) & (fr < 1 - 1e-6)).all(axis=1) & ((rflags & 4) == 0)
    for m in (1, 63, 65, t.shape[0]):
        tf, qf = _cuda(t[:m], torch.float32), _cuda(q[:m], torch.float32)
        gt, gphi, out = fif.query_grad(field, tf, qf, M7, _cuda(up[:m]), want_out=True)
        assert torch.equal(out.nan_to_num(7.0), fif.query(field, tf, qf, M7).nan_to_num(7.0)), m
        ok = ok_all[:m]
        for a, b in ((gt.cpu().numpy(), rgt[:m]), (gphi.cpu().numpy(), rgphi[:m])):
            scale = np.abs(b[ok]).max(axis=1, keepdims=True)
            rel = np.abs(a[ok] - b[ok]) / scale
            print(m, "fp32 grad rel err max", rel.max(), "median", np.median(rel))
            assert rel.max() <= 1e-3, (m, rel.max())
            assert rel.max() <= 2e-4, (m, rel.max())  # a guard well inside the bar


def test_v05_gradient_fp32_with_zero_logdet_weight(fif, tiny):
    """v_alpha = 0.5 on an FP32 compensated field: with weight 0 on the log-det
    the gradient is finite everywhere and matches the oracle's at the FP32 bar;
    with weight 1 it is NaN on the poses whose FIM is clearly indefinite and
    finite on those clearly positive definite."""
    print("case: tiny gradient FP32 compensated, v_alpha 0.5", flush=True)
    grid, vis = _grid_vis(fif, tiny["g"], tiny["v"], v_alpha=0.5)
    field = fif.build(_cuda(tiny["lm"]), grid, vis, prec=fif.FP32_COMP)
    t = tiny["t"].astype(np.float32).astype(np.float64)
    q = tiny["q"].astype(np.float32).astype(np.float64)
    tf, qf = _cuda(t, torch.float32), _cuda(q, torch.float32)
    g = (t - np.asarray(tiny["g"].origin)) / tiny["g"].h
    fr = g - np.floor(g)
    ok = ((fr > 1e-6) & (fr < 1 - 1e-6)).all(axis=1)
    ref, rflags = oracle.query(tiny["ofield"], tiny["v"].half_fov, 0.5, t, q, M7 | 8, 0)
    ok &= (rflags & 4) == 0
    up = np.tile([1.0, 0.5, 0.0], (t.shape[0], 1))
    gt, gphi = fif.query_grad(field, tf, qf, M7, _cuda(up))
    gt, gphi = gt.cpu().numpy(), gphi.cpu().numpy()
    assert np.isfinite(gt).all() and np.isfinite(gphi).all()
    rgt, rgphi = oracle.query_grad(tiny["ofield"], tiny["v"].half_fov, 0.5, t, q, M7, up)
    for a, b in ((gt, rgt), (gphi, rgphi)):
        scale = np.abs(b[ok]).max(axis=1, keepdims=True)
        rel = (np.abs(a[ok] - b[ok]) / scale).max()
        print("fp32 v05 grad rel err max", rel)
        assert rel <= 1e-3
    lam = np.linalg.eigvalsh(_sym21(ref[:, 3:]))
    lmax = np.abs(lam).max(axis=1)
    indef = lam[:, 0] < -1e-6 * lmax
    posdef = lam[:, 0] > 1e-6 * lmax
    assert indef.any() and posdef.any()
    gt1, _ = fif.query_grad(field, tf, qf, M7, _cuda(np.ones_like(up)))
    gt1 = gt1.cpu().numpy()
    assert np.isnan(gt1[indef]).all() and np.isfinite(gt1[posdef]).all()


def _sym21(v):
    iu = np.triu_indices(6)
    F = np.zeros(v.shape[:-1] + (6, 6))
    F[..., iu[0], iu[1]] = v
    F[..., iu[1], iu[0]] = v
    return F


def test_v05_indefinite_parity(fif, tiny):
    """v_alpha = 0.5 (negative visibility weights): signed lmin, NaN logdet."""
    grid, vis = _grid_vis(fif, tiny["g"], tiny["v"], v_alpha=0.5)
    field = fif.build(_cuda(tiny["lm"]), grid, vis, prec=fif.FP64)
    t, q = tiny["t"], tiny["q"]
    out, flags = fif.query(field, _cuda(t), _cuda(q), M7 | 8, want_flags=True)
    out, flags = out.cpu().numpy(), flags.cpu().numpy()
    ref, rflags = oracle.query(tiny["ofield"], tiny["v"].half_fov, 0.5, t, q, M7 | 8, 0)
    err = metric_errors(out[:, :3], ref[:, :3], ref[:, 3:])
    assert err["trace_rel"].max() <= 1e-9
    assert err["lmin_weyl"].max() <= 1e-10
    assert err["logdet_abs"].max() <= 1e-8
    assert (ref[:, 1] < 0).any() and np.isnan(ref[:, 2]).any()
    np.testing.assert_array_equal(flags & 2, rflags & 2)


def test_v05_gradient_with_zero_logdet_weight(fif, tiny):
    """v_alpha = 0.5: indefinite FIMs have no log-det.  With weight 0 on the
    log-det the gradient is that of the other metrics (finite, equal to the
    oracle's); with weight 1 it is NaN exactly on the poses whose FIM is not
    positive definite."""
    print("case: tiny gradient FP64, v_alpha 0.5, zero log-det weight", flush=True)
    grid, vis = _grid_vis(fif, tiny["g"], tiny["v"], v_alpha=0.5)
    field = fif.build(_cuda(tiny["lm"]), grid, vis, prec=fif.FP64)
    t, q = tiny["t"], tiny["q"]
    g = (t - np.asarray(tiny["g"].origin)) / tiny["g"].h
    fr = g - np.floor(g)
    ok = ((fr > 1e-6) & (fr < 1 - 1e-6)).all(axis=1)
    ref, rflags = oracle.query(tiny["ofield"], tiny["v"].half_fov, 0.5, t, q, M7, 0)
    ok &= (rflags & 4) == 0
    up = np.tile([1.0, 0.5, 0.0], (t.shape[0], 1))
    gt, gphi = fif.query_grad(field, _cuda(t), _cuda(q), M7, _cuda(up))
    gt, gphi = gt.cpu().numpy(), gphi.cpu().numpy()
    assert np.isfinite(gt).all() and np.isfinite(gphi).all()
    rgt, rgphi = oracle.query_grad(tiny["ofield"], tiny["v"].half_fov, 0.5, t, q, M7, up)
    for a, b in ((gt, rgt), (gphi, rgphi)):
        scale = np.abs(b[ok]).max(axis=1, keepdims=True)
        assert (np.abs(a[ok] - b[ok]) / scale).max() <= 1e-7
    npd = np.isnan(ref[:, 2])
    assert npd.any()
    gt1, _ = fif.query_grad(field, _cuda(t), _cuda(q), M7, _cuda(np.ones_like(up)))
    gt1 = gt1.cpu().numpy()
    assert np.isnan(gt1[npd]).all() and np.isfinite(gt1[~npd]).all()
