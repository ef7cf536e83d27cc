"""Calls given an explicit stream: builds on two streams at once (each stream
gets its own sorting workspace) and queries whose outputs are allocated on the
call's stream give bitwise the results of the same calls on the default
stream."""
import pytest

import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fif():
    import paper_2008_03324_amd as fif
    fif.lib()
    return fif


def test_side_streams_match_default_stream(fif):
    print("case: builds and queries on two side streams", flush=True)
    lm, g, v = scenes.building_scene(n_landmarks=20_000, shape=(64, 64, 32))
    grid = fif.Grid(g.origin, g.h, g.shape)
    vis = fif.Vis(v.half_fov, v.v_alpha, v.sigma, v.r_min, v.r_max)
    lm_d = torch.tensor(lm, dtype=torch.float64, device="cuda")
    halves = (lm_d[:10_000].contiguous(), lm_d[10_000:].contiguous())
    ref = [fif.build(h, grid, vis, prec=fif.FP32_COMP) for h in halves]
    t, q = scenes.building_poses(g, 100_000)
    t_d, q_d = torch.from_numpy(t).cuda(), torch.from_numpy(q).cuda()
    ref_out = [fif.query(f, t_d, q_d, 7) for f in ref]
    torch.cuda.synchronize()

    streams = (torch.cuda.Stream(), torch.cuda.Stream())
    fields = [fif.Field(grid, vis, fif.FP32_COMP) for _ in halves]
    torch.cuda.synchronize()
    outs = [None, None]
    for _ in range(3):  # repeated, so a shared workspace would be raced over
        for i, s in enumerate(streams):
            fif.build(halves[i], grid, vis, field=fields[i], stream=s)
        for i, s in enumerate(streams):
            outs[i] = fif.query(fields[i], t_d, q_d, 7, stream=s)
    torch.cuda.synchronize()
    for i in range(2):
        assert torch.equal(fields[i].buffer, ref[i].buffer)
        assert torch.equal(outs[i].nan_to_num(7.0), ref_out[i].nan_to_num(7.0))
    # dropping the cached workspaces while builds are in flight on the side
    # streams does not disturb them, and later builds get fresh ones
    for i, s in enumerate(streams):
        fif.build(halves[i], grid, vis, field=fields[i], stream=s)
    fif.release_workspaces()
    again = fif.build(halves[0], grid, vis, prec=fif.FP32_COMP)
    torch.cuda.synchronize()
    for i in range(2):
        assert torch.equal(fields[i].buffer, ref[i].buffer)
    assert torch.equal(again.buffer, ref[0].buffer)
