"""Pins of the FP64 oracle to facts other than itself (CPU only).

Each test checks the oracle against what the paper and the mathematics fix:
finite-difference Jacobians of the bearing measurement model, closed forms,
LAPACK eigen-solvers, brute force on tiny inputs, and the invariants the paper
states (rotation invariance, separation, additivity, trace factors).
"""
import math
import os

import numpy as np
import pytest

import oracle
import scenes

SIG = 1.0 / 300.0
ALPHA = math.pi / 4


# ------------------------------------------------------------ helpers (tests only)

def skew(v):
    return np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]], float)


def so3_exp(phi):
    th = np.linalg.norm(phi)
    K = skew(phi)
    if th < 1e-12:
        return np.eye(3) + K
    return np.eye(3) + math.sin(th) / th * K + (1 - math.cos(th)) / th ** 2 * K @ K


def se3_left(xi, R, t):
    """exp(xi^) T_wc with xi = [rho; phi] (exact SE(3) exponential)."""
    rho, phi = xi[:3], xi[3:]
    th = np.linalg.norm(phi)
    K = skew(phi)
    if th < 1e-12:
        V = np.eye(3) + 0.5 * K
    else:
        V = np.eye(3) + (1 - math.cos(th)) / th ** 2 * K + (th - math.sin(th)) / th ** 3 * K @ K
    E = so3_exp(phi)
    return E @ R, E @ t + V @ rho


def bearing(R_wc, t, p):
    pc = R_wc.T @ (p - t)
    return pc / np.linalg.norm(pc)


def fd_jacobian(R, t, p, h=1e-6):
    """Central FD of the bearing w.r.t. the global perturbation (eq:deriv_se3, first form)."""
    J = np.zeros((3, 6))
    for c in range(6):
        e = np.zeros(6)
        e[c] = h
        Rp, tp = se3_left(e, R, t)
        Rm, tm = se3_left(-e, R, t)
        J[:, c] = (bearing(Rp, tp, p) - bearing(Rm, tm, p)) / (2 * h)
    return J


def random_rotation(rng):
    q = rng.standard_normal(4)
    return oracle.quat_to_R(q / np.linalg.norm(q))


def k_closed(alpha, va):
    # our algebra from the three conditions (independent of the linear solve)
    k2 = ((1 + math.cos(alpha)) / 2 - va) / math.sin(alpha) ** 2
    return np.array([k2, 0.5, 0.5 - k2])


# ------------------------------------------------------------ visibility

@pytest.mark.parametrize("alpha,va", [(math.pi / 4, 0.5), (math.pi / 4, 0.8),
                                      (math.pi / 6, 0.3), (1.2, 0.9)])
def test_quadratic_conditions(alpha, va):
    k = oracle.quad_coeffs(alpha, va)
    v = lambda c: k[0] * c * c + k[1] * c + k[2]
    assert v(1.0) == pytest.approx(1.0, abs=1e-14)
    assert v(-1.0) == pytest.approx(0.0, abs=1e-14)
    assert v(math.cos(alpha)) == pytest.approx(va, abs=1e-14)
    np.testing.assert_allclose(k, k_closed(alpha, va), atol=1e-14)


def test_linear_case_golden():
    """Sec. V-B: the p=1 model is fixed to k0 = k1 = 0.5 by the first two conditions."""
    path = os.path.join(os.path.dirname(__file__), "golden", "linear_visibility.txt")
    k1, k0 = np.loadtxt(path)
    for alpha in (math.pi / 4, math.pi / 3, 1.0):
        k = oracle.quad_coeffs(alpha, (1 + math.cos(alpha)) / 2)
        assert abs(k[0]) < 1e-15
        assert k[1] == pytest.approx(k1, abs=1e-15)
        assert k[2] == pytest.approx(k0, abs=1e-15)


def test_v05_has_negative_values_and_psd_threshold():
    """Fig. sim_quad_vis caption: v_alpha = 0.5 at 90 deg FoV takes negative values."""
    c = np.linspace(-1, 1, 20001)
    k = oracle.quad_coeffs(ALPHA, 0.5)
    v = k[0] * c * c + k[1] * c + k[2]
    assert v.min() < -0.29
    assert v.min() == pytest.approx(-0.2955, abs=1e-3)
    k = oracle.quad_coeffs(ALPHA, 0.8)
    assert (k[0] * c * c + k[1] * c + k[2]).min() >= 0.0
    # v >= 0 on [-1, 1] iff k2 <= 1/4 (vertex value k0 - k1^2/(4 k2) >= 0)
    va_star = (1 + math.cos(ALPHA)) / 2 - 0.25 * math.sin(ALPHA) ** 2
    assert va_star == pytest.approx(0.72855, abs=1e-5)


def test_vr_vp_dot_is_quadratic_visibility():
    rng = np.random.default_rng(1)
    k = oracle.quad_coeffs(ALPHA, 0.8)
    for _ in range(20):
        z = rng.standard_normal(3); z /= np.linalg.norm(z)
        u = rng.standard_normal(3); u /= np.linalg.norm(u)
        c = z @ u
        assert oracle.vr(k, z) @ oracle.vp(u) == pytest.approx(k[0] * c * c + k[1] * c + k[2],
                                                               abs=1e-14)


# ------------------------------------------------------------ per-landmark FIM

def test_landmark_fim_matches_fd_jacobian():
    """eq:jac_pose_global vs central FD of the bearing under exp(xi^) T_wc."""
    rng = np.random.default_rng(2)
    for _ in range(10):
        R = random_rotation(rng)
        t = rng.uniform(-3, 3, 3)
        p = rng.uniform(-5, 5, 3)
        J = fd_jacobian(R, t, p)
        I_fd = J.T @ J / SIG ** 2
        I_or = oracle.landmark_fim(p, t, R.reshape(-1), SIG)
        np.testing.assert_allclose(I_or, I_fd, rtol=0, atol=1e-7 * np.abs(I_fd).max())


def test_landmark_fim_structure():
    rng = np.random.default_rng(3)
    for _ in range(10):
        p = rng.uniform(-5, 5, 3)
        t = rng.uniform(-3, 3, 3)
        R = random_rotation(rng)
        I = oracle.landmark_fim(p, t, R.reshape(-1), SIG)
        ev = np.linalg.eigvalsh(I)
        assert np.allclose(I, I.T, atol=1e-9 * np.abs(I).max())
        assert ev.min() > -1e-9 * ev.max()
        assert np.sum(ev > 1e-9 * ev.max()) == 2  # rank 2
        d = p - t
        n = np.linalg.norm(d)
        u = d / n
        # null vectors [p x w + a u; w]
        for _ in range(3):
            w = rng.standard_normal(3)
            a = rng.standard_normal()
            x = np.concatenate([np.cross(p, w) + a * u, w])
            assert np.linalg.norm(I @ x) < 1e-9 * np.abs(I).max() * np.linalg.norm(x)
        # trace closed form (2 + |p|^2 + (u.p)^2) / (sigma^2 n^2)
        assert np.trace(I) == pytest.approx((2 + p @ p + (u @ p) ** 2) / (SIG ** 2 * n * n),
                                            rel=1e-12)


def test_rotation_invariance():
    """eq:global_fim_eq: I_i does not change when R_wc -> R_wc R_cc'."""
    rng = np.random.default_rng(4)
    p = rng.uniform(-5, 5, 3)
    t = rng.uniform(-3, 3, 3)
    R = random_rotation(rng)
    I0 = oracle.landmark_fim(p, t, R.reshape(-1), SIG)
    for _ in range(5):
        R2 = R @ random_rotation(rng)
        I2 = oracle.landmark_fim(p, t, R2.reshape(-1), SIG)
        assert np.abs(I2 - I0).max() <= 1e-12 * np.abs(I0).max()


# ------------------------------------------------------------ range predicate

def test_range_predicate_fp32():
    rng = np.random.default_rng(5)
    for _ in range(2000):
        p = rng.uniform(-20, 20, 3)
        t = rng.uniform(-20, 20, 3)
        d = p.astype(np.float32) - t.astype(np.float32)
        n2 = np.float32(d[0] * d[0])
        n2 = np.float32(np.float64(d[1]) * d[1] + n2)   # exact fma then one rounding
        n2 = np.float32(np.float64(d[2]) * d[2] + n2)
        want = (n2 >= np.float32(1e-12)) and (n2 <= np.float32(15.0 * 15.0))
        assert oracle.in_range(p, t, 0.0, 15.0) == want
    assert oracle.in_range([1, 2, 3], [1, 2, 3], 0.0, math.inf) is False  # coincident
    assert oracle.in_range([100, 0, 0], [0, 0, 0], 0.0, math.inf) is True


# ------------------------------------------------------------ separation

def brute_force_fim(landmarks, R, t, k):
    """sum_i v(z.u_i) J_i^T J_i / sigma^2 with FD Jacobians (tiny inputs only)."""
    z = R[:, 2]
    F = np.zeros((6, 6))
    for p in landmarks:
        d = p - t
        u = d / np.linalg.norm(d)
        c = z @ u
        J = fd_jacobian(R, t, p)
        F += (k[0] * c * c + k[1] * c + k[2]) * (J.T @ J) / SIG ** 2
    return F


def test_field_at_voxel_centre_equals_point_cloud_bruteforce():
    """eq:fim_separation: at a voxel centre the field equals the PC sum under the
    same quadratic visibility (tiny brute force with FD Jacobians)."""
    rng = np.random.default_rng(6)
    lm = rng.uniform(-2, 2, (8, 3))
    origin, h, shape = (-0.5, -0.5, -0.5), 1.0, (2, 2, 2)
    k = oracle.quad_coeffs(ALPHA, 0.8)
    C = oracle.build(lm, origin, h, shape, SIG)
    field = oracle.Field(C, origin, h, shape)
    for v in range(8):
        t = oracle.voxel_centre(origin, h, shape, v)
        for _ in range(3):
            R = random_rotation(rng)
            q = scenes.rotation_to_quaternion(R)
            F_bf = brute_force_fim(lm, R, t, k)
            F_tri = oracle.query_fim(field, ALPHA, 0.8, t[None], q[None], interp=0)[0]
            F_nn = oracle.query_fim(field, ALPHA, 0.8, t[None], q[None], interp=1)[0]
            scale = np.abs(F_bf).max()
            assert np.abs(F_tri - F_bf).max() < 1e-7 * scale
            assert np.abs(F_nn - F_bf).max() < 1e-7 * scale


def test_field_at_voxel_centre_equals_pc_tiny_scene():
    lm, grid, vis = scenes.tiny_scene(n_landmarks=300)
    ids = np.array([0, 57, 1234, 2399])
    C = oracle.build(lm, grid.origin, grid.h, grid.shape, vis.sigma, voxel_ids=ids)
    field = oracle.Field(C, grid.origin, grid.h, grid.shape, voxel_ids=ids)
    rng = np.random.default_rng(7)
    for a, v in enumerate(ids):
        t = oracle.voxel_centre(grid.origin, grid.h, grid.shape, v)
        q = scenes.haar_quaternions(rng, 4)
        tt = np.repeat(t[None], 4, 0)
        F_field = oracle.query_fim(field, vis.half_fov, vis.v_alpha, tt, q, interp=1)
        _, F_pc = oracle.pc_query(lm, vis.half_fov, vis.v_alpha, vis.sigma, vis.r_min,
                                  vis.r_max, tt, q, 1, want_fim=True)
        for i in range(4):
            assert np.abs(F_field[i] - F_pc[i]).max() <= 1e-12 * np.abs(F_pc[i]).max()
        # roll about the optical axis leaves the approximated FIM unchanged
        R = oracle.quat_to_R(q[0])
        roll = R @ so3_exp(np.array([0, 0, 0.7]))
        q2 = scenes.rotation_to_quaternion(roll)
        _, F_roll = oracle.pc_query(lm, vis.half_fov, vis.v_alpha, vis.sigma, vis.r_min,
                                    vis.r_max, t[None], q2[None], 1, want_fim=True)
        assert np.abs(F_roll[0] - F_pc[0]).max() <= 1e-9 * np.abs(F_pc[0]).max()


def test_separation_with_range_cutoff():
    lm, grid, vis = scenes.building_scene(n_landmarks=3000, shape=(40, 40, 10), h=0.5)
    rng = np.random.default_rng(8)
    ids = rng.choice(grid.n_voxels, 5, replace=False)
    C = oracle.build(lm, grid.origin, grid.h, grid.shape, vis.sigma, vis.r_min, vis.r_max,
                     voxel_ids=ids)
    field = oracle.Field(C, grid.origin, grid.h, grid.shape, voxel_ids=ids)
    for v in ids:
        t = oracle.voxel_centre(grid.origin, grid.h, grid.shape, v)
        q = scenes.haar_quaternions(rng, 1)
        F_f = oracle.query_fim(field, vis.half_fov, vis.v_alpha, t[None], q, interp=1)[0]
        _, F_pc = oracle.pc_query(lm, vis.half_fov, vis.v_alpha, vis.sigma, vis.r_min,
                                  vis.r_max, t[None], q, 1, want_fim=True)
        assert np.abs(F_f - F_pc[0]).max() <= 1e-12 * np.abs(F_pc[0]).max()


# ------------------------------------------------------------ interpolation

def test_interpolation_properties():
    rng = np.random.default_rng(9)
    origin, h, shape = (0.0, 0.0, 0.0), 0.5, (3, 4, 2)
    C = rng.standard_normal((24, 10, 6, 6))
    C = C + C.transpose(0, 1, 3, 2)
    field = oracle.Field(C, origin, h, shape)
    q = scenes.haar_quaternions(rng, 1)
    k = oracle.quad_coeffs(ALPHA, 0.8)
    R = oracle.quat_to_R(q[0])
    vr = oracle.vr(k, R[:, 2])
    # centres reproduce voxel values
    for v in range(24):
        t = oracle.voxel_centre(origin, h, shape, v)
        F = oracle.query_fim(field, ALPHA, 0.8, t[None], q)[0]
        np.testing.assert_allclose(F, np.einsum("k,kij->ij", vr, C[v]), atol=1e-12)
    # linear along an x edge
    a = oracle.voxel_centre(origin, h, shape, 3)  # (0, 1, 0)
    b = oracle.voxel_centre(origin, h, shape, 4)  # (1, 1, 0)
    Fa = oracle.query_fim(field, ALPHA, 0.8, a[None], q)[0]
    Fb = oracle.query_fim(field, ALPHA, 0.8, b[None], q)[0]
    for s in (0.1, 0.37, 0.9):
        F = oracle.query_fim(field, ALPHA, 0.8, ((1 - s) * a + s * b)[None], q)[0]
        np.testing.assert_allclose(F, (1 - s) * Fa + s * Fb, atol=1e-12)
    # trilinear in a cell interior = explicit tensor-product formula
    f = np.array([0.3, 0.6, 0.25])
    t = np.asarray(origin) + (np.array([1, 2, 0]) + f) * h
    F = oracle.query_fim(field, ALPHA, 0.8, t[None], q)[0]
    want = np.zeros((6, 6))
    for j in range(8):
        bx, by, bz = j & 1, (j >> 1) & 1, (j >> 2) & 1
        w = (f[0] if bx else 1 - f[0]) * (f[1] if by else 1 - f[1]) * (f[2] if bz else 1 - f[2])
        v = (1 + bx) + 3 * ((2 + by) + 4 * bz)
        want += w * np.einsum("k,kij->ij", vr, C[v])
    np.testing.assert_allclose(F, want, atol=1e-12)
    # constant field -> constant query
    Cc = np.repeat(C[:1], 24, 0)
    fc = oracle.Field(Cc, origin, h, shape)
    tt = rng.uniform(-0.5, 1.5, (10, 3))
    Fs = oracle.query_fim(fc, ALPHA, 0.8, tt, np.repeat(q, 10, 0))
    np.testing.assert_allclose(Fs, np.repeat(Fs[:1], 10, 0), atol=1e-12)


def _random_sym_field(rng, n):
    C = rng.standard_normal((n, 10, 6, 6))
    return C + C.transpose(0, 1, 3, 2)


def test_nearest_rule_off_centre():
    """Sec. VI-A retrieves a factor by nearest neighbour or by interpolation;
    the nearest voxel is read as round-half-up per axis.  Off the voxel centres
    (a grid spacing that is not a binary fraction, an origin off zero): 0.4 h
    from a centre keeps that voxel, 0.6 h takes the neighbour, on every axis and
    on several axes at once; on a grid where the midpoints are exact, +0.5 h
    takes the upper voxel and -0.5 h keeps the centre's own."""
    rng = np.random.default_rng(14)
    k = oracle.quad_coeffs(ALPHA, 0.8)
    q = scenes.haar_quaternions(rng, 1)
    vr = oracle.vr(k, oracle.quat_to_R(q[0])[:, 2])

    def check(origin, h, shape, cases):
        n = int(np.prod(shape))
        C = _random_sym_field(rng, n)
        field = oracle.Field(C, origin, h, shape)
        for ijk, s, want in cases:
            t = np.asarray(origin) + (np.asarray(ijk) + np.asarray(s)) * h
            v = want[0] + shape[0] * (want[1] + shape[1] * want[2])
            F = oracle.query_fim(field, ALPHA, 0.8, t[None], q, interp=1)[0]
            ref = np.einsum("k,kij->ij", vr, C[v])
            assert np.abs(F - ref).max() <= 1e-13 * np.abs(ref).max(), (ijk, s, want)

    origin, h, shape = (0.13, -0.71, 0.37), 0.3, (5, 4, 3)
    cases = []
    for ijk in ((2, 1, 1), (1, 2, 1), (3, 2, 1)):
        for ax in range(3):
            for s, di in ((-0.6, -1), (-0.4, 0), (0.4, 0), (0.6, 1)):
                off = [0.0, 0.0, 0.0]
                off[ax] = s
                want = list(ijk)
                want[ax] += di
                cases.append((ijk, off, want))
        cases.append((ijk, (0.4, -0.6, 0.6), (ijk[0], ijk[1] - 1, ijk[2] + 1)))
        cases.append((ijk, (-0.45, 0.55, -0.3), (ijk[0], ijk[1] + 1, ijk[2])))
    check(origin, h, shape, cases)
    # exact midpoints: h and the origin are binary fractions
    origin, h, shape = (0.25, -0.5, 1.0), 0.5, (4, 4, 3)
    ties = []
    for ax in range(3):
        up_, down = [0.0] * 3, [0.0] * 3
        up_[ax], down[ax] = 0.5, -0.5
        want = [1, 1, 1]
        want[ax] = 2
        ties.append(((1, 1, 1), up_, want))
        ties.append(((1, 1, 1), down, (1, 1, 1)))
    ties.append(((1, 2, 0), (0.5, -0.5, 0.5), (2, 2, 1)))
    check(origin, h, shape, ties)


def test_hull_clamp_is_constant_extension():
    """Reading of the grid boundary (the paper is silent): a position outside
    the hull of voxel centres takes the value at its projection onto the hull
    (constant extension), for interpolation and nearest retrieval, on a field
    that is not constant.  On a field linear in the voxel index a linear
    extrapolation would differ from the hull value; the oracle returns the
    hull value."""
    rng = np.random.default_rng(15)
    origin, h, shape = (-0.4, 0.2, 0.05), 0.35, (4, 3, 3)
    n = int(np.prod(shape))
    C = _random_sym_field(rng, n)
    field = oracle.Field(C, origin, h, shape)
    lo = np.asarray(origin)
    hi = lo + (np.asarray(shape) - 1) * h
    t = rng.uniform(lo - 2 * h, hi + 2 * h, (400, 3))
    out = ((t < lo) | (t > hi)).any(axis=1)
    t = t[out]
    assert t.shape[0] > 100
    q = scenes.haar_quaternions(rng, t.shape[0])
    tc = np.clip(t, lo, hi)
    for interp in (0, 1):
        F = oracle.query_fim(field, ALPHA, 0.8, t, q, interp=interp)
        Fc = oracle.query_fim(field, ALPHA, 0.8, tc, q, interp=interp)
        scale = np.abs(Fc).max(axis=(1, 2))
        assert (np.abs(F - Fc).max(axis=(1, 2)) <= 1e-12 * scale).all(), interp
        _, fl = oracle.query(field, ALPHA, 0.8, t, q, 1, interp)
        assert (fl & 1).all()
    # linear in the x index: C_v = A + i_x B.  Beyond the upper x face (y, z
    # inside) the value is A + (nx - 1) B, not A + g_x B with g_x > nx - 1.
    A, B = _random_sym_field(rng, 2)
    ix = np.arange(n) % shape[0]
    CL = A[None] + ix[:, None, None, None] * B[None]
    fl_ = oracle.Field(CL, origin, h, shape)
    k = oracle.quad_coeffs(ALPHA, 0.8)
    for dx in (0.3 * h, 1.7 * h):
        tt = np.array([[hi[0] + dx, lo[1] + 0.37 * h, lo[2] + 1.2 * h]])
        qq = scenes.haar_quaternions(rng, 1)
        vr = oracle.vr(k, oracle.quat_to_R(qq[0])[:, 2])
        want = np.einsum("k,kij->ij", vr, A + (shape[0] - 1) * B)
        extrap = np.einsum("k,kij->ij", vr, A + (shape[0] - 1 + dx / h) * B)
        for interp in (0, 1):
            F = oracle.query_fim(fl_, ALPHA, 0.8, tt, qq, interp=interp)[0]
            assert np.abs(F - want).max() <= 1e-12 * np.abs(want).max()
            assert np.abs(F - extrap).max() > 1e-3 * np.abs(want).max()


def test_clamp_and_nearest_flags():
    origin, h, shape = (0.0, 0.0, 0.0), 1.0, (3, 3, 3)
    C = np.ones((27, 10, 6, 6))
    field = oracle.Field(C, origin, h, shape)
    q = np.array([[1.0, 0, 0, 0]] * 3)
    t = np.array([[1.0, 1.0, 1.0], [-0.5, 1.0, 1.0], [1.0, 1.0, 2.2]])
    _, flags = oracle.query(field, ALPHA, 0.8, t, q, 1)
    assert list(flags & 1) == [0, 1, 1]


# ------------------------------------------------------------ metrics

def test_metrics_match_lapack():
    rng = np.random.default_rng(10)
    for _ in range(50):
        A = rng.standard_normal((6, 6))
        F = A @ A.T + 1e-3 * np.eye(6)
        F *= 10 ** rng.uniform(-3, 8)
        out = oracle.metrics(F, 7)
        ev = np.linalg.eigvalsh(F)
        assert out[0] == pytest.approx(np.trace(F), rel=1e-13)
        assert abs(out[1] - ev[0]) <= 1e-13 * ev[-1]
        assert out[2] == pytest.approx(np.linalg.slogdet(F)[1], abs=1e-10)
        w, V = oracle.jacobi6(F)
        np.testing.assert_allclose(F @ V, V * w, atol=1e-12 * ev[-1])
        ld, inv = oracle.logdet6(F, want_inv=True)
        np.testing.assert_allclose(inv @ F, np.eye(6), atol=1e-8)
    # indefinite: lmin negative, logdet NaN
    F = np.diag([1.0, 2, 3, 4, 5, -1])
    out = oracle.metrics(F, 7)
    assert out[1] == pytest.approx(-1.0)
    assert math.isnan(out[2])
    out = oracle.metrics(F, 8)
    iu = np.triu_indices(6)
    np.testing.assert_array_equal(out, F[iu])


# ------------------------------------------------------------ field properties

def test_additivity_and_trace_factor():
    """Sec. VI-A: factors are sums of per-landmark parts; Sec. VII-A: the trace
    factor gives the same trace as the information factor."""
    rng = np.random.default_rng(11)
    lm = rng.uniform(-3, 3, (40, 3))
    t = np.array([0.2, -0.4, 0.1])
    C1 = oracle.info_factor(lm[:17], t, SIG)
    C2 = oracle.info_factor(lm[17:], t, SIG)
    C = oracle.info_factor(lm, t, SIG)
    assert np.abs(C - (C1 + C2)).max() <= 1e-12 * np.abs(C).max()
    CT = oracle.trace_factor(lm, t, SIG)
    np.testing.assert_allclose(CT, np.trace(C, axis1=1, axis2=2), rtol=1e-12)
    k = oracle.quad_coeffs(ALPHA, 0.8)
    for _ in range(5):
        z = rng.standard_normal(3); z /= np.linalg.norm(z)
        vr = oracle.vr(k, z)
        assert vr @ CT == pytest.approx(np.trace(np.einsum("k,kij->ij", vr, C)), rel=1e-12)


def test_trace_field_query_equals_information_trace():
    """eq:general_trace_pif: the trace field gives the trace of the FIM that the
    information field gives, for interpolated and nearest retrieval, inside
    and outside the hull; the built trace factors are the traces of the built
    information factors."""
    lm, grid, vis = scenes.tiny_scene(n_landmarks=300)
    rng = np.random.default_rng(16)
    t, q = scenes.tiny_poses(grid, 64, seed=78)
    t[:8] += rng.uniform(-2.0, 2.0, (8, 3))  # some outside the hull
    ids = oracle.corner_voxels(grid.origin, grid.h, grid.shape, t)
    C = oracle.build(lm, grid.origin, grid.h, grid.shape, vis.sigma, voxel_ids=ids)
    CT = oracle.trace_build(lm, grid.origin, grid.h, grid.shape, vis.sigma, voxel_ids=ids)
    np.testing.assert_allclose(CT, np.trace(C, axis1=2, axis2=3), rtol=1e-12)
    f = oracle.Field(C, grid.origin, grid.h, grid.shape, voxel_ids=ids)
    tf = oracle.TraceField(CT, grid.origin, grid.h, grid.shape, voxel_ids=ids)
    for interp in (0, 1):
        ref, rfl = oracle.query(f, vis.half_fov, vis.v_alpha, t, q, 1, interp)
        tr, fl = oracle.trace_query(tf, vis.half_fov, vis.v_alpha, t, q, interp)
        np.testing.assert_allclose(tr, ref[:, 0], rtol=1e-12)
        np.testing.assert_array_equal(fl & 1, rfl & 1)


def test_zero_weight_metric_leaves_gradient_finite():
    """The gradient of L = sum_c w_c s_c: a metric with w_c = 0 is not part of
    L.  With v_alpha = 0.5 some FIMs are indefinite (log-det NaN); weights
    (1, 1, 0) on (trace, lmin, logdet) give the finite gradient of trace +
    lmin, the same as asking for those two metrics alone, while a nonzero
    log-det weight on such a pose gives NaN."""
    lm, grid, vis = scenes.tiny_scene(n_landmarks=200)
    C = oracle.build(lm, grid.origin, grid.h, grid.shape, vis.sigma)
    field = oracle.Field(C, grid.origin, grid.h, grid.shape)
    t, q = scenes.tiny_poses(grid, 48, seed=79)
    out, fl = oracle.query(field, ALPHA, 0.5, t, q, 7)
    npd = np.isnan(out[:, 2])
    assert npd.any() and (~npd).any()
    up3 = np.tile([1.0, 1.0, 0.0], (t.shape[0], 1))
    gt, gphi = oracle.query_grad(field, ALPHA, 0.5, t, q, 7, up3)
    gt2, gphi2 = oracle.query_grad(field, ALPHA, 0.5, t, q, 3, up3[:, :2])
    assert np.isfinite(gt).all() and np.isfinite(gphi).all()
    np.testing.assert_array_equal(gt, gt2)
    np.testing.assert_array_equal(gphi, gphi2)
    gt3, _ = oracle.query_grad(field, ALPHA, 0.5, t, q, 7, np.ones((t.shape[0], 3)))
    assert np.isnan(gt3[npd]).all() and np.isfinite(gt3[~npd]).all()


def test_psd_for_nonnegative_visibility_and_indefinite_for_v05():
    lm, grid, vis = scenes.tiny_scene(n_landmarks=200)
    t, q = scenes.tiny_poses(grid, 40)
    _, F8 = oracle.pc_query(lm, ALPHA, 0.8, SIG, 0, math.inf, t, q, 1, want_fim=True)
    for F in F8:
        ev = np.linalg.eigvalsh(F)
        assert ev.min() >= -1e-10 * ev.max()
    _, F5 = oracle.pc_query(lm, ALPHA, 0.5, SIG, 0, math.inf, t, q, 1, want_fim=True)
    assert min(np.linalg.eigvalsh(F).min() for F in F5) < 0


def test_logdet_origin_invariance():
    """A shift of the world origin is a unimodular congruence of the FIM."""
    lm, grid, vis = scenes.tiny_scene(n_landmarks=200)
    t, q = scenes.tiny_poses(grid, 10)
    shift = np.array([25.0, -13.0, 4.0])
    a = oracle.pc_query(lm, ALPHA, 0.8, SIG, 0, math.inf, t, q, 7)
    b = oracle.pc_query(lm + shift, ALPHA, 0.8, SIG, 0, math.inf, t + shift, q, 7)
    np.testing.assert_allclose(a[:, 2], b[:, 2], atol=1e-7)
    assert np.abs(a[:, 0] - b[:, 0]).max() > 1.0  # trace depends on the origin


# ------------------------------------------------------------ exact point cloud

def test_exact_pc_matches_pinhole_bruteforce():
    rng = np.random.default_rng(12)
    lm = rng.uniform(-4, 4, (60, 3))
    fx, fy, cx, cy, W, H = scenes.PINHOLE
    for _ in range(10):
        t = rng.uniform(-1, 1, 3)
        R = random_rotation(rng)
        q = scenes.rotation_to_quaternion(R)
        F = np.zeros((6, 6))
        for p in lm:
            pc = R.T @ (p - t)
            if pc[2] <= 0:
                continue
            u, v = fx * pc[0] / pc[2] + cx, fy * pc[1] / pc[2] + cy
            if 0 <= u < W and 0 <= v < H:
                J = fd_jacobian(R, t, p)
                F += J.T @ J / SIG ** 2
        _, Fo = oracle.pc_query(lm, ALPHA, 0.8, SIG, 0, math.inf, t[None], q[None], 1,
                                pinhole=scenes.PINHOLE, want_fim=True)
        assert np.abs(Fo[0] - F).max() <= 1e-6 * max(np.abs(F).max(), 1.0)


# ------------------------------------------------------------ gradient

def test_gradient_matches_central_fd():
    lm, grid, vis = scenes.tiny_scene(n_landmarks=150)
    C = oracle.build(lm, grid.origin, grid.h, grid.shape, vis.sigma)
    field = oracle.Field(C, grid.origin, grid.h, grid.shape)
    rng = np.random.default_rng(13)
    t, q = scenes.tiny_poses(grid, 12, seed=77)
    # keep away from cell faces (one-sided derivative there)
    g = (t - np.asarray(grid.origin)) / grid.h
    fr = g - np.floor(g)
    keep = ((fr > 0.05) & (fr < 0.95)).all(axis=1)
    t, q = t[keep], q[keep]
    up = rng.standard_normal((t.shape[0], 3))
    gt, gphi = oracle.query_grad(field, ALPHA, 0.8, t, q, 7, up)
    hh = 1e-5

    def L(tt, qq):
        out, _ = oracle.query(field, ALPHA, 0.8, tt, qq, 7)
        return (out * up).sum(axis=1)

    for c in range(3):
        e = np.zeros(3); e[c] = hh
        fd = (L(t + e, q) - L(t - e, q)) / (2 * hh)
        np.testing.assert_allclose(gt[:, c], fd, rtol=2e-5, atol=1e-6 * np.abs(fd).max())
    for c in range(3):
        e = np.zeros(3); e[c] = hh
        qp, qm = [], []
        for qi in q:
            R = oracle.quat_to_R(qi)
            qp.append(scenes.rotation_to_quaternion(so3_exp(e) @ R))
            qm.append(scenes.rotation_to_quaternion(so3_exp(-e) @ R))
        fd = (L(t, np.array(qp)) - L(t, np.array(qm))) / (2 * hh)
        np.testing.assert_allclose(gphi[:, c], fd, rtol=2e-5, atol=1e-6 * np.abs(fd).max())


# ------------------------------------------------------------ optimal-view sweep

def axis_rotation(z):
    """A rotation R_wc whose optical axis R e3 is the unit vector along z."""
    z = np.asarray(z, float) / np.linalg.norm(z)
    a = np.array([1.0, 0, 0]) if abs(z[0]) < 0.9 else np.array([0, 1.0, 0])
    x = np.cross(a, z)
    x /= np.linalg.norm(x)
    return np.stack([x, np.cross(z, x), z], axis=1)


def test_view_sweep_equals_pc_bruteforce_at_voxel_centres():
    """Sec. VII-A relative measures: every swept value equals the point-cloud sum
    (eq:vis_fim under the quadratic visibility) of the pose that looks along that
    axis, at voxel centres where the interpolation is exact; the best index is
    the first maximiser."""
    lm, grid, vis = scenes.tiny_scene(n_landmarks=300)
    ids = np.array([0, 57, 1234, 2399])
    C = oracle.build(lm, grid.origin, grid.h, grid.shape, vis.sigma, voxel_ids=ids)
    field = oracle.Field(C, grid.origin, grid.h, grid.shape, voxel_ids=ids)
    rng = np.random.default_rng(60)
    dirs = rng.standard_normal((24, 3))
    dirs[5] = dirs[2]                  # an exact tie
    dirs[7] = dirs[1] * 3.0            # same axis, unnormalised
    t = np.stack([oracle.voxel_centre(grid.origin, grid.h, grid.shape, v) for v in ids])
    for metric in (oracle.TRACE, oracle.LMIN, oracle.LOGDET):
        values, best = oracle.view_sweep(field, vis.half_fov, vis.v_alpha, t, dirs, metric,
                                         interp=1)
        for a in range(len(ids)):
            q = np.stack([scenes.rotation_to_quaternion(axis_rotation(d)) for d in dirs])
            ref = oracle.pc_query(lm, vis.half_fov, vis.v_alpha, vis.sigma, vis.r_min,
                                  vis.r_max, np.repeat(t[a:a + 1], len(dirs), 0), q, metric)[:, 0]
            scale = np.abs(ref).max()
            assert np.abs(values[a] - ref).max() <= 1e-9 * scale
            assert values[a, 5] == values[a, 2]
            assert abs(values[a, 7] - values[a, 1]) <= 1e-12 * scale
            assert best[a] == int(np.argmax(values[a]))


def test_view_sweep_roll_invariance_and_nan_rules():
    """The swept value depends on the axis only (eq:quad_vis_component): a query
    with any roll about that axis gives the same FIM metric; NaN axes never win,
    and a position where every axis is NaN gets -1."""
    lm, grid, vis = scenes.tiny_scene(n_landmarks=300)
    C = oracle.build(lm, grid.origin, grid.h, grid.shape, vis.sigma)
    field = oracle.Field(C, grid.origin, grid.h, grid.shape)
    rng = np.random.default_rng(61)
    dirs = rng.standard_normal((10, 3))
    t = rng.uniform(-3, 3, (3, 3)) * np.array([1, 1, 0.3])
    values, best = oracle.view_sweep(field, vis.half_fov, vis.v_alpha, t, dirs, oracle.LOGDET)
    for a in range(3):
        for d in range(10):
            R = axis_rotation(dirs[d]) @ so3_exp(np.array([0, 0, rng.uniform(-3, 3)]))
            q = scenes.rotation_to_quaternion(R)
            ref, _ = oracle.query(field, vis.half_fov, vis.v_alpha, t[a:a + 1], q[None],
                                  oracle.LOGDET)
            assert abs(values[a, d] - ref[0, 0]) <= 1e-9 * max(1.0, abs(ref[0, 0]))
    dz = np.concatenate([np.zeros((1, 3)), dirs[:3]])      # the zero axis gives NaN
    v2, b2 = oracle.view_sweep(field, vis.half_fov, vis.v_alpha, t, dz, oracle.TRACE)
    assert np.isnan(v2[:, 0]).all()
    assert (b2 == 1 + np.argmax(v2[:, 1:], axis=1)).all()
    v3, b3 = oracle.view_sweep(field, vis.half_fov, vis.v_alpha, t, np.zeros((2, 3)),
                               oracle.TRACE)
    assert np.isnan(v3).all() and (b3 == -1).all()


# ------------------------------------------------------------ GP visibility (f2)

KS = 15.0
NOISE = 1e-10


def _unit(rng, n):
    u = rng.standard_normal((n, 3))
    return u / np.linalg.norm(u, axis=1, keepdims=True)


def _np_gp(Z, length):
    """numpy reference pieces: K^s + noise I and its solve (library routines)."""
    K = np.exp(-((Z[:, None, :] - Z[None, :, :]) ** 2).sum(-1) / (2 * length * length))
    return K + NOISE * np.eye(len(Z))


def _np_vgp(Z, length, z, u):
    """v_gp(z, u) = K_z (K^s + noise I)^-1 v^s(u) with numpy's solver."""
    Ky = _np_gp(Z, length)
    kz = np.exp(-((z[None, :] - Z) ** 2).sum(-1) / (2 * length * length))
    vs = 1.0 / (1.0 + np.exp(-KS * (Z @ u - math.cos(ALPHA))))
    return kz @ np.linalg.solve(Ky, vs)


@pytest.fixture(scope="module")
def gp30():
    Z = scenes.sphere_axes(30)
    U = _unit(np.random.default_rng(90), 200)
    length = oracle.gp_fit_length(Z, KS, ALPHA, NOISE, U)
    return Z, U, length, oracle.gp_inverse(Z, length, NOISE)


def test_gp_sigmoid_and_inverse(gp30):
    Z, U, length, A = gp30
    # eq:sigmoid_vis_func: 1/2 at the FoV boundary, -> 1 on axis, -> 0 behind
    assert abs(oracle.sigmoid_vis(KS, ALPHA, math.cos(ALPHA)) - 0.5) < 1e-15
    assert oracle.sigmoid_vis(KS, ALPHA, 1.0) > 0.98 and oracle.sigmoid_vis(KS, ALPHA, -1.0) < 1e-10
    Ky = _np_gp(Z, length)
    assert np.abs(A @ Ky - np.eye(len(Z))).max() < 1e-8
    assert np.abs(A - np.linalg.inv(Ky)).max() <= 1e-9 * np.abs(A).max()


def test_gp_lml_and_ml2_length(gp30):
    """Evidence vs numpy (slogdet, solve); the fitted length maximises it over
    a dense grid (brute force)."""
    Z, U, length, _ = gp30
    Ky = _np_gp(Z, length)
    Y = 1.0 / (1.0 + np.exp(-KS * (U @ Z.T - math.cos(ALPHA))))
    ref = (-0.5 * np.einsum("tg,tg->", Y, np.linalg.solve(Ky, Y.T).T)
           - 0.5 * len(U) * np.linalg.slogdet(Ky)[1] - 0.5 * len(U) * len(Z) * math.log(2 * math.pi))
    got = oracle.gp_lml(Z, KS, ALPHA, length, NOISE, U)
    assert abs(got - ref) <= 1e-9 * abs(ref)
    grid = np.geomspace(0.1, 2.5, 200)
    vals = [oracle.gp_lml(Z, KS, ALPHA, l, NOISE, U) for l in grid]
    assert got >= max(vals) - 1e-6 * abs(got)
    assert 0.5 < length < 1.5


def test_gp_visibility_interpolates_and_approximates(gp30):
    """The GP mean reproduces the training values at the sample axes and
    approximates the sigmoid between them, better with more samples."""
    Z, U, length, A = gp30
    rng = np.random.default_rng(91)
    for u in _unit(rng, 5):
        vp = oracle.gp_vp(Z, KS, ALPHA, A, u)
        for g in (0, 7, 29):
            v = oracle.gp_vr(Z, length, Z[g]) @ vp
            assert abs(v - oracle.sigmoid_vis(KS, ALPHA, Z[g] @ u)) < 1e-4
        z = _unit(rng, 1)[0]
        assert abs(oracle.gp_vr(Z, length, z) @ vp - _np_vgp(Z, length, z, u)) < 1e-8
    errs = {}
    for ns in (30, 150):
        Zn = scenes.sphere_axes(ns)
        ln = oracle.gp_fit_length(Zn, KS, ALPHA, NOISE, U)
        An = oracle.gp_inverse(Zn, ln, NOISE)
        e = 0.0
        for u, z in zip(_unit(rng, 40), _unit(rng, 40)):
            v = oracle.gp_vr(Zn, ln, z) @ oracle.gp_vp(Zn, KS, ALPHA, An, u)
            e = max(e, abs(v - oracle.sigmoid_vis(KS, ALPHA, z @ u)))
        errs[ns] = e
    assert errs[150] < errs[30] and errs[150] < 0.15


def test_gp_field_at_voxel_centre_equals_bruteforce(gp30):
    """eq:fim_separation with the GP model: at a voxel centre the field equals
    sum_i v_gp(z, u_i) J_i^T J_i / sigma^2 with FD Jacobians and numpy's GP."""
    Z, U, length, A = gp30
    rng = np.random.default_rng(92)
    lm = rng.uniform(-2, 2, (8, 3))
    origin, h, shape = (-0.5, -0.5, -0.5), 1.0, (2, 2, 2)
    C = oracle.gp_build(lm, origin, h, shape, SIG, Z, KS, ALPHA, A)
    field = oracle.GPField(C, origin, h, shape, Z, length)
    for v in (0, 5):
        t = oracle.voxel_centre(origin, h, shape, v)
        for _ in range(2):
            R = random_rotation(rng)
            q = scenes.rotation_to_quaternion(R)
            F_bf = np.zeros((6, 6))
            for p in lm:
                u = (p - t) / np.linalg.norm(p - t)
                J = fd_jacobian(R, t, p)
                F_bf += _np_vgp(Z, length, R[:, 2], u) * (J.T @ J) / SIG ** 2
            for interp in (0, 1):
                _, _, F = oracle.gp_query(field, t[None], q[None], 7, interp, want_fim=True)
                assert np.abs(F[0] - F_bf).max() < 1e-6 * np.abs(F_bf).max()
            F_pc = oracle.gp_pc_fim(lm, SIG, 0.0, np.inf, Z, KS, ALPHA, length, A, t[None],
                                    q[None])[0]
            assert np.abs(F_pc - F_bf).max() < 1e-6 * np.abs(F_bf).max()
            # roll about the optical axis leaves the GP FIM unchanged
            q2 = scenes.rotation_to_quaternion(R @ so3_exp(np.array([0, 0, 1.1])))
            _, _, F2 = oracle.gp_query(field, t[None], q2[None], 7, 0, want_fim=True)
            assert np.abs(F2[0] - F_bf).max() < 1e-6 * np.abs(F_bf).max()


def test_gp_trace_factor_is_trace_of_information_factor(gp30):
    Z, U, length, A = gp30
    lm, grid, vis = scenes.tiny_scene(n_landmarks=200)
    ids = np.array([3, 777, 2000])
    CI = oracle.gp_build(lm, grid.origin, grid.h, grid.shape, vis.sigma, Z, KS, ALPHA, A,
                         voxel_ids=ids)
    CT = oracle.gp_build(lm, grid.origin, grid.h, grid.shape, vis.sigma, Z, KS, ALPHA, A,
                         trace=True, voxel_ids=ids)
    tr = np.trace(CI, axis1=2, axis2=3)
    assert np.abs(CT - tr).max() <= 1e-12 * np.abs(tr).max()
    fi = oracle.GPField(CI, grid.origin, grid.h, grid.shape, Z, length, voxel_ids=ids)
    ft = oracle.GPField(CT, grid.origin, grid.h, grid.shape, Z, length, trace=True, voxel_ids=ids)
    t = np.stack([oracle.voxel_centre(grid.origin, grid.h, grid.shape, v) for v in ids])
    q = scenes.haar_quaternions(np.random.default_rng(93), 3)
    a, _ = oracle.gp_query(fi, t, q, 1, interp=1)
    b, _ = oracle.gp_query(ft, t, q, 1, interp=1)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_gp_length_inputs_are_the_ml2_fit():
    """The length scales the GP workloads use are the oracle's ML-II fit on the
    stated training bearings (to the 4 digits stored)."""
    U = scenes.gp_training_directions()
    for ns, l in scenes.GP_LENGTH.items():
        fit = oracle.gp_fit_length(scenes.sphere_axes(ns), KS, ALPHA, NOISE, U)
        assert abs(fit - l) < 1e-4, (ns, fit, l)
