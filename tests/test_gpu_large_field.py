"""A field larger than 4 GiB: 512 x 512 x 72 voxels at 0.2 m (18.9M voxels,
6.0 GB in FP32), so the main records of the top 8 z-layers and every cell side
record lie past byte offset 2^32 of the field buffer.  Blocks, trilinear and
nearest queries, the trace field and the gradient kernel are compared with the
oracle (or with each other) at voxels and poses on both sides of that offset.
"""
import numpy as np
import pytest

import oracle
import scenes
from fifcheck import block_rel_err, e_fim, metric_errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

M7 = 7
SHAPE = (512, 512, 72)
N_LANDMARKS = 20_000


@pytest.fixture(scope="module")
def fif():
    import paper_2008_03324_amd as fif
    fif.lib()
    return fif


@pytest.fixture(scope="module")
def big(fif):
    print("case: 512x512x72 grid (6.0 GB FP32 field), 20k landmarks", flush=True)
    lm, g, v = scenes.building_scene(n_landmarks=N_LANDMARKS, shape=SHAPE)
    grid = fif.Grid(g.origin, g.h, g.shape)
    vis = fif.Vis(v.half_fov, v.v_alpha, v.sigma, v.r_min, v.r_max)
    lm_d = torch.tensor(lm, dtype=torch.float64, device="cuda")
    field = fif.build(lm_d, grid, vis, prec=fif.FP32_COMP)
    assert field.nbytes > 4 * 2**30
    rng = np.random.default_rng(41)
    # poses: half in the top 8 z-layers (main records past 2^32 bytes), half anywhere
    m = 512
    t = scenes.uniform_in_hull(rng, g, m)
    z_hi = g.origin[2] + (SHAPE[2] - 1) * g.h
    t[: m // 2, 2] = rng.uniform(z_hi - 7 * g.h, z_hi, m // 2)
    q = scenes.haar_quaternions(rng, m)
    t32, q32 = t.astype(np.float32), q.astype(np.float32)
    torch.cuda.synchronize()
    yield dict(lm=lm, g=g, v=v, grid=grid, vis=vis, lm_d=lm_d, field=field,
               t=t32, q=q32, t_d=torch.from_numpy(t32).cuda(), q_d=torch.from_numpy(q32).cuda())
    del field
    torch.cuda.empty_cache()


def _oracle_field(b, t64):
    g, v = b["g"], b["v"]
    ids = oracle.corner_voxels(g.origin, g.h, g.shape, t64)
    C = oracle.build(b["lm"], g.origin, g.h, g.shape, v.sigma, v.r_min, v.r_max, voxel_ids=ids)
    return oracle.Field(C, g.origin, g.h, g.shape, voxel_ids=ids)


def test_blocks_past_4gib_match_oracle(fif, big):
    rng = np.random.default_rng(42)
    n = big["grid"].n_voxels
    first_far = 2**32 // 256  # first voxel whose main record starts at byte 2^32
    ids = np.unique(np.concatenate([rng.integers(first_far, n, 96), rng.integers(0, n, 32),
                                    [0, first_far - 1, first_far, n - 1]]))
    g, v = big["g"], big["v"]
    C = oracle.build(big["lm"], g.origin, g.h, g.shape, v.sigma, v.r_min, v.r_max, voxel_ids=ids)
    blocks = fif.export_blocks(big["field"], torch.from_numpy(ids).cuda()).cpu().numpy()
    err = block_rel_err(blocks, C)
    print("blocks err max", err.max())
    assert err.max() <= 1e-3


@pytest.mark.parametrize("interp", [0, 1])
def test_queries_past_4gib_match_oracle(fif, big, interp):
    t64, q64 = big["t"].astype(np.float64), big["q"].astype(np.float64)
    of = _oracle_field(big, t64)
    v = big["v"]
    ref, rflags = oracle.query(of, v.half_fov, v.v_alpha, t64, q64, M7 | 8, interp)
    out, flags = fif.query(big["field"], big["t_d"], big["q_d"], M7 | 8, interp=interp,
                           want_flags=True)
    out = out.cpu().numpy()
    err = metric_errors(out[:, :3], ref[:, :3], ref[:, 3:])
    print(interp, {k: float(np.max(x)) for k, x in err.items()})
    assert err["trace_rel"].max() <= 1e-3
    assert err["lmin_weyl"].max() <= 1e-3
    assert err["logdet_abs"].max() <= 1e-3
    assert e_fim(out[:, 3:], ref[:, 3:]).max() <= 1e-3
    np.testing.assert_array_equal(flags.cpu().numpy() & 3, rflags & 3)


def test_gradient_kernel_and_trace_field_past_4gib(fif, big):
    """The gradient kernel's forward values equal the forward query's, and the
    trace field (0.9 GB) gives the information field's trace."""
    f = big["field"]
    out = fif.query(f, big["t_d"], big["q_d"], M7)
    m = out.shape[0]
    gt, gphi, out_g = fif.query_grad(f, big["t_d"], big["q_d"], M7,
                                     torch.ones((m, 3), dtype=torch.float64, device="cuda"),
                                     want_out=True)
    a, b = out.cpu().numpy(), out_g.cpu().numpy()
    assert np.array_equal(np.isnan(a), np.isnan(b))
    ok = ~np.isnan(a)
    assert np.array_equal(a[ok], b[ok])
    assert bool(torch.isfinite(gt).all()) and bool(torch.isfinite(gphi).all())
    tf = fif.build(big["lm_d"], big["grid"], big["vis"], prec=fif.FP32_COMP, kind=fif.KIND_TRACE)
    tr = fif.query(tf, big["t_d"], big["q_d"], fif.TRACE)[:, 0]
    rel = ((tr - out[:, 0]).abs() / out[:, 0].abs()).max().item()
    assert rel <= 1e-3, rel
