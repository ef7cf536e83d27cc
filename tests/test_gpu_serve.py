"""Serving loop: results are bitwise the same alone and in the mix; admission
by HBM budget and slots; the one-request-per-launch mode agrees too."""
import numpy as np
import pytest

import oracle
import scenes
from fifcheck import metric_errors, sym_from21

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import paper_2008_03324_amd as fif
    from paper_2008_03324_amd import serve
    print("case: serving loop on two small fields", flush=True)
    fields, pools = [], []
    for lm, g, v in _field_scenes():
        grid = fif.Grid(g.origin, g.h, g.shape)
        vis = fif.Vis(v.half_fov, v.v_alpha, v.sigma, v.r_min, v.r_max)
        fields.append(fif.build(torch.tensor(lm, device="cuda"), grid, vis, prec=fif.FP32_COMP))
        i = len(fields) - 1
        pt, pq = scenes.building_poses(g, 20_000, seed=90 + i)
        tt, tq = scenes.trajectories(g, 128, 64, seed=95 + i)
        pools.append({"plan": (torch.from_numpy(pt).cuda(), torch.from_numpy(pq).cuda()),
                      "opt": (torch.from_numpy(tt.reshape(-1, 3)).cuda(),
                              torch.from_numpy(tq.reshape(-1, 4)).cuda())})
    specs = scenes.request_stream(2, 2000.0, 150, 20_000, 128, seed=99)
    torch.cuda.synchronize()
    return fif, serve, fields, pools, specs


def _field_scenes():
    """The two served fields' scenes (seeded, so the oracle sees the same
    landmarks and grids as the GPU fields)."""
    return [scenes.building_scene(n_landmarks=4000, seed=77 + i, shape=shape, h=0.25, r_max=6.0)
            for i, shape in enumerate(((24, 24, 12), (40, 30, 10)))]


def _check_vs_oracle(reqs, n_each=6, rows=48):
    """Served outputs and gradients of a sample of requests (n_each of each
    kind, up to `rows` poses of each) against the FP64 oracle on oracle-built
    factors of the poses' corner voxels, at the FP32-field bar of 1e-3:
    trace relative, lambda_min / lambda_max, log-det in nats; gradients
    |dg| / max|g| per pose (dL/dout = the request's weights), poses within 1e-3 of
    a cell face or with a near-repeated lambda_min left out (one-sided or
    undefined derivative)."""
    worst = {"out": 0.0, "grad": 0.0}
    scns = _field_scenes()
    n_opt = 0
    for kind in ("plan", "opt"):
        sample = [r for r in reqs if r.kind == kind][:n_each]
        assert len(sample) == n_each
        for r in sample:
            lm, g, v = scns[r.field]
            sel = np.linspace(0, r.m - 1, min(rows, r.m)).astype(np.int64)
            t64 = r.t.cpu().numpy()[sel].astype(np.float64)
            q64 = r.q.cpu().numpy()[sel].astype(np.float64)
            ids = oracle.corner_voxels(g.origin, g.h, g.shape, t64)
            C = oracle.build(lm, g.origin, g.h, g.shape, v.sigma, v.r_min, v.r_max,
                             voxel_ids=ids)
            of = oracle.Field(C, g.origin, g.h, g.shape, voxel_ids=ids)
            ref, _ = oracle.query(of, v.half_fov, v.v_alpha, t64, q64, 7 | 8)
            got = r.out.cpu().numpy()[sel]
            err = metric_errors(got, ref[:, :3], ref[:, 3:])
            e = max(err["trace_rel"].max(), err["lmin_weyl"].max(), err["logdet_abs"].max())
            worst["out"] = max(worst["out"], e)
            assert e <= 1e-3, (r.rid, err)
            if kind == "opt":
                n_opt += 1
                rgt, rgphi = oracle.query_grad(of, v.half_fov, v.v_alpha, t64, q64, 7,
                                               np.tile(np.asarray(r.weights), (len(sel), 1)))
                gg = (t64 - np.asarray(g.origin)) / g.h
                fr = gg - np.floor(gg)
                ev = np.linalg.eigvalsh(sym_from21(ref[:, 3:]))
                ok = ((fr > 1e-3) & (fr < 1 - 1e-3)).all(axis=1)
                if r.weights[1]:
                    ok &= (ev[:, 1] - ev[:, 0]) > 1e-6 * np.abs(ev).max(axis=1)
                assert ok.sum() >= len(sel) // 2
                for a, b in ((r.grad_t.cpu().numpy()[sel], rgt),
                             (r.grad_phi.cpu().numpy()[sel], rgphi)):
                    rel = np.abs(a[ok] - b[ok]) / np.abs(b[ok]).max(axis=1, keepdims=True)
                    worst["grad"] = max(worst["grad"], rel.max())
                    assert rel.max() <= 1e-3, r.rid
    assert n_opt == n_each
    assert len({r.weights for r in reqs if r.kind == "opt"}) == len(_WEIGHTS)
    return worst


@pytest.mark.parametrize("loop", ["native", "python"])
def test_served_requests_vs_oracle(setup, loop):
    """A sample of served requests, planner (queries) and optimizer (queries
    and gradients), in the mix of the realtime stream, against the oracle."""
    fif, serve, fields, pools, specs = setup
    print(f"case: served requests vs oracle, {loop} loop", flush=True)
    reqs = _make(serve, pools, specs)
    if loop == "native":
        srv = serve.NativeServer(fields, n_streams=3, co_batch=True, max_batch=16384)
        srv.run(reqs, realtime=True)
    else:
        srv = serve.Server(fields, n_streams=3, use_graphs=True, co_batch=True, max_batch=16384)
        srv.warmup()
        srv.run(reqs, realtime=True)
        assert all(r.status == "done" for r in reqs)
    worst = _check_vs_oracle(reqs)
    print(loop, "served vs oracle, worst", worst)


# optimizer requests' metric weights (trace, lambda_min, log-det), in turn:
# all three, log-det left out, lambda_min left out, lambda_min alone
_WEIGHTS = ((1.0, 1.0, 1.0), (1.0, 1.0, 0.0), (0.5, 0.0, 2.0), (0.0, 1.0, 0.0))


def _make(serve, pools, specs):
    reqs = []
    for sp in specs:
        t, q = pools[sp.field][sp.kind]
        reqs.append(serve.Request(sp.rid, sp.arrival, sp.field, sp.kind,
                                  t[sp.offset:sp.offset + sp.m], q[sp.offset:sp.offset + sp.m],
                                  weights=_WEIGHTS[sp.rid % len(_WEIGHTS)]))
    return reqs


def _alone(fif, fields, r):
    f = fields[r.field]
    if r.kind == "plan":
        return fif.query(f, r.t.contiguous(), r.q.contiguous(), 7), None, None
    up = torch.tensor(r.weights, dtype=torch.float64, device="cuda").expand(r.m, 3).contiguous()
    gt, gphi, out = fif.query_grad(f, r.t.contiguous(), r.q.contiguous(), 7, up, want_out=True)
    return out, gt, gphi


@pytest.mark.parametrize("mode", ["batched_graphs", "batched_eager", "one_per_launch"])
def test_results_identical_alone_and_in_mix(setup, mode):
    fif, serve, fields, pools, specs = setup
    kw = {"batched_graphs": dict(n_streams=3, use_graphs=True, co_batch=True, max_batch=16384),
          "batched_eager": dict(n_streams=2, use_graphs=False, co_batch=True, max_batch=4096),
          "one_per_launch": dict(n_streams=1, use_graphs=False, co_batch=False,
                                 max_inflight=1)}[mode]
    srv = serve.Server(fields, **kw)
    srv.warmup()
    reqs = _make(serve, pools, specs)
    srv.run(reqs, realtime=True)
    assert all(r.status == "done" for r in reqs)
    assert srv.reserved == 0 and not srv.inflight
    for r in reqs:
        out, gt, gphi = _alone(fif, fields, r)
        assert torch.equal(r.out, out), (mode, r.rid)
        if r.kind == "opt":
            assert torch.equal(r.grad_t, gt) and torch.equal(r.grad_phi, gphi), (mode, r.rid)
    st = serve.latency_stats(reqs)
    assert st["n"] == len(reqs) and st["p99_ms"] >= st["p50_ms"] >= 0


def test_admission_by_budget(setup):
    fif, serve, fields, pools, specs = setup
    reqs = _make(serve, pools, specs)
    big = max(r.bytes_needed() for r in reqs)
    srv = serve.Server(fields, n_streams=2, use_graphs=False, hbm_budget=big)
    srv.run(reqs, realtime=False)
    assert all(r.status == "done" for r in reqs) and srv.reserved == 0
    tiny = serve.Server(fields, n_streams=1, use_graphs=False, hbm_budget=big - 1)
    with pytest.raises(serve.AdmissionError):
        tiny.run(_make(serve, pools, specs), realtime=False)


@pytest.mark.parametrize("mode", ["packed", "packed_tight", "one_per_launch"])
def test_native_results_identical_alone_and_in_mix(setup, mode):
    """fif_serve_run (the loop in C++): every request's results equal the
    direct query / gradient call on it alone, whatever was packed with it."""
    fif, serve, fields, pools, specs = setup
    reqs = _make(serve, pools, specs)
    biggest = max(r.m for r in reqs)
    kw = {"packed": dict(n_streams=3, co_batch=True, max_batch=16384),
          "packed_tight": dict(n_streams=2, co_batch=True, max_batch=biggest, max_inflight=6),
          "one_per_launch": dict(n_streams=1, co_batch=False, max_inflight=1,
                                 max_batch=biggest)}[mode]
    print(f"case: native serving loop, {mode}", flush=True)
    srv = serve.NativeServer(fields, **kw)
    elapsed = srv.run(reqs, realtime=True)
    assert elapsed > 0
    for r in reqs:
        assert r.arrival <= r.admitted + 1e-9 and r.admitted <= r.done, (mode, r.rid)
        out, gt, gphi = _alone(fif, fields, r)
        assert torch.equal(r.out, out), (mode, r.rid)
        if r.kind == "opt":
            assert torch.equal(r.grad_t, gt) and torch.equal(r.grad_phi, gphi), (mode, r.rid)
    st = serve.latency_stats(reqs)
    assert st["n"] == len(reqs) and st["p99_ms"] >= st["p50_ms"] >= 0


def test_native_admission_and_errors(setup):
    import ctypes
    fif, serve, fields, pools, specs = setup
    reqs = _make(serve, pools, specs)
    big = max(r.bytes_needed() for r in reqs)
    srv = serve.NativeServer(fields, n_streams=2, hbm_budget=big)
    srv.run(reqs, realtime=False)
    assert all(r.done == r.done for r in reqs)  # not NaN
    # a request larger than the budget is refused before anything runs
    tiny = serve.NativeServer(fields, n_streams=1, hbm_budget=big - 1)
    with pytest.raises(fif.FifError, match="HBM budget"):
        tiny.run(_make(serve, pools, specs), realtime=False)
    with pytest.raises(ValueError):
        serve.NativeServer(fields, n_streams=0)
    # a workspace smaller than fif_serve_workspace_bytes() is refused
    cfg = fif.CServeConfig(1, 4, 1 << 30, 1024, 1, 0)
    need = fif.lib().fif_serve_workspace_bytes(ctypes.byref(cfg))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    one = (fif.CServeRequest * 1)()
    r0 = reqs[0]
    r0.out = torch.empty((r0.m, 3), dtype=torch.float64, device="cuda")
    w = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    one[0] = fif.CServeRequest(0.0, r0.field, 0, r0.m, r0.t.data_ptr(), r0.q.data_ptr(),
                               r0.out.data_ptr(), None, None, w, 0.0, 0.0)
    cf = (fif.CField * len(fields))(*[f.cstruct for f in fields])
    el = ctypes.c_double()
    L = fif.lib()
    assert L.fif_serve_run(cf, len(fields), one, 1, ctypes.byref(cfg),
                           ctypes.c_void_p(ws.data_ptr()), need - 1, ctypes.byref(el)) == -2
    bad = fif.CServeRequest(0.0, 7, 0, r0.m, r0.t.data_ptr(), r0.q.data_ptr(),
                            r0.out.data_ptr(), None, None, w, 0.0, 0.0)
    one[0] = bad
    assert L.fif_serve_run(cf, len(fields), one, 1, ctypes.byref(cfg),
                           ctypes.c_void_p(ws.data_ptr()), need, ctypes.byref(el)) == -1
    assert b"field index" in L.fif_last_error()


def test_native_fp64_fields():
    """fif_serve_run on FP64 fields: poses, gradients and results move as doubles
    through the pack and unpack kernels; every request equals its direct call."""
    import paper_2008_03324_amd as fif
    from paper_2008_03324_amd import serve
    print("case: native serving loop on two FP64 fields", flush=True)
    fields, pools = [], []
    for i, shape in enumerate(((20, 20, 10), (32, 24, 8))):
        lm, g, v = scenes.building_scene(n_landmarks=3000, seed=81 + i, shape=shape, h=0.25,
                                         r_max=6.0)
        grid = fif.Grid(g.origin, g.h, g.shape)
        vis = fif.Vis(v.half_fov, v.v_alpha, v.sigma, v.r_min, v.r_max)
        fields.append(fif.build(torch.tensor(lm, device="cuda"), grid, vis, prec=fif.FP64))
        pt, pq = scenes.building_poses(g, 4000, seed=84 + i, dtype=np.float64)
        tt, tq = scenes.trajectories(g, 80, 64, seed=86 + i)
        pools.append({"plan": (torch.from_numpy(pt).cuda(), torch.from_numpy(pq).cuda()),
                      "opt": (torch.from_numpy(tt.reshape(-1, 3).astype(np.float64)).cuda(),
                              torch.from_numpy(tq.reshape(-1, 4).astype(np.float64)).cuda())})
    specs = scenes.request_stream(2, 2000.0, 40, 4000, 80, seed=88)
    reqs = _make(serve, pools, specs)
    assert {r.kind for r in reqs} == {"plan", "opt"}
    srv = serve.NativeServer(fields, n_streams=2, co_batch=True, max_batch=8192, max_inflight=8)
    assert srv.run(reqs, realtime=False) > 0
    for r in reqs:
        assert r.out.dtype == torch.float64 and r.t.dtype == torch.float64
        out, gt, gphi = _alone(fif, fields, r)
        assert torch.equal(r.out.nan_to_num(7.0), out.nan_to_num(7.0)), r.rid
        if r.kind == "opt":
            assert r.grad_t.dtype == torch.float64
            assert torch.equal(r.grad_t, gt) and torch.equal(r.grad_phi, gphi), r.rid
