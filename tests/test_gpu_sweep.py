"""Precision sweep: the building scene at 1M landmarks built in FP32 naive, FP32
compensated and FP64 on the full 2M-voxel grid; per-voxel block error against
the FP64 oracle on sampled voxels, and query-metric errors against the oracle on
sampled building poses (oracle factors of their corner voxels)."""
import numpy as np
import pytest

import oracle
import scenes
from fifcheck import block_rel_err, metric_errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_precision_sweep_1M_landmarks():
    import paper_2008_03324_amd as fif
    print("case: 1M-landmark precision sweep", flush=True)
    lm, g, v = scenes.building_scene(n_landmarks=1_000_000)
    grid = fif.Grid(g.origin, g.h, g.shape)
    vis = fif.Vis(v.half_fov, v.v_alpha, v.sigma, v.r_min, v.r_max)
    lm_d = torch.tensor(lm, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(41)
    ids = np.sort(rng.choice(grid.n_voxels, 48, replace=False))
    C = oracle.build(lm, g.origin, g.h, g.shape, v.sigma, v.r_min, v.r_max, voxel_ids=ids)
    ids_d = torch.from_numpy(ids).cuda()
    # 64 building poses: oracle factors of their corner voxels from all 1M landmarks
    t, q = scenes.building_poses(g, 64, seed=42)
    t64, q64 = t.astype(np.float64), q.astype(np.float64)
    cids = oracle.corner_voxels(g.origin, g.h, g.shape, t64)
    CQ = oracle.build(lm, g.origin, g.h, g.shape, v.sigma, v.r_min, v.r_max, voxel_ids=cids)
    of = oracle.Field(CQ, g.origin, g.h, g.shape, voxel_ids=cids)
    ref, _ = oracle.query(of, v.half_fov, v.v_alpha, t64, q64, 7 | 8)
    errs, qerrs = {}, {}
    for prec in (fif.FP32_NAIVE, fif.FP32_COMP, fif.FP64):
        f = fif.build(lm_d, grid, vis, prec=prec)
        errs[prec] = block_rel_err(fif.export_blocks(f, ids_d).cpu().numpy(), C)
        dt = torch.float64 if prec == fif.FP64 else torch.float32
        out = fif.query(f, torch.from_numpy(t64).to("cuda", dt),
                        torch.from_numpy(q64).to("cuda", dt), 7).cpu().numpy()
        assert np.array_equal(np.isnan(out), np.isnan(ref[:, :3])), prec
        qerrs[prec] = {k: float(x.max()) for k, x in
                       metric_errors(out, ref[:, :3], ref[:, 3:]).items()}
        del f
        torch.cuda.empty_cache()
    print({p: (float(e.max()), float(np.median(e))) for p, e in errs.items()})
    print("query errors vs oracle:", qerrs)
    # FP32 bar of 1e-3 on queries for the compensated build; FP64 to rounding
    for k in ("trace_rel", "lmin_weyl", "lmin_rel", "logdet_abs"):
        assert qerrs[fif.FP32_COMP][k] <= 1e-3, k
        assert qerrs[fif.FP32_COMP][k] <= 1e-4, k  # measured ~1e-6
        assert qerrs[fif.FP64][k] <= 1e-8, k
    # the naive build's summation error over ~280k terms per voxel is reported,
    # not held to the bar (its queries miss 1e-3 at this landmark count)
    assert qerrs[fif.FP32_NAIVE]["trace_rel"] <= 3e-2
    assert errs[fif.FP64].max() <= 1e-10
    assert errs[fif.FP32_COMP].max() <= 1e-3
    # the compensated build takes the offsets of landmarks very close to a voxel
    # centre from their FP64 coordinates: its worst voxel stays near FP32
    # rounding (measured 1.1e-6) instead of ~1e-4
    assert errs[fif.FP32_COMP].max() <= 1e-5
    assert errs[fif.FP32_NAIVE].max() <= 1e-3
    assert np.median(errs[fif.FP32_COMP]) <= np.median(errs[fif.FP32_NAIVE])
