"""Seeded synthetic inputs for the Fisher Information Field workloads.

This module only samples geometry (landmarks, grids, poses, trajectories,
request streams).  It holds none of the method's arithmetic, so both the HIP
path and the CPU oracle can take their inputs from it.

Scenes are centred on the world origin: the paper's global se(3) perturbation
(Sec. V-A, eq:jac_pose_global) is taken about the world origin, so trace and
smallest eigenvalue depend on where the scene sits; centring fixes that choice.

Workloads (shapes follow Sec. VII-A of the paper, scaled as stated):
  tiny     2,000 landmarks uniform in 10x10x5 m, 0.5 m voxels over 10x10x3 m
           (20x20x6), 1,000 poses, r_max = inf (all landmarks, as in Sec. VII-A)
  building 100k landmarks (70 % on 12 noisy vertical walls, 30 % clutter) in
           40x40x10 m, 0.2 m voxels (200x200x50), r_max = 15 m, 10M poses
  sweep    the building scene at 1M landmarks
  traj     4,096 B-spline trajectories x 64 poses, 5 m long, smooth yaw/pitch
  serve    four building-like fields of 64^3, 128x128x32, 200x200x50,
           256x256x64 voxels and a Poisson request stream
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_SCENE = 1000
SEED_POSES = 2000


@dataclasses.dataclass(frozen=True)
class Grid:
    origin: tuple  # centre of voxel (0, 0, 0), metres
    h: float
    shape: tuple  # (nx, ny, nz), x fastest

    @property
    def n_voxels(self) -> int:
        return int(np.prod(self.shape))

    @property
    def hull_lo(self) -> np.ndarray:
        return np.asarray(self.origin, dtype=np.float64)

    @property
    def hull_hi(self) -> np.ndarray:
        return self.hull_lo + (np.asarray(self.shape) - 1) * self.h


@dataclasses.dataclass(frozen=True)
class Vis:
    half_fov: float = math.pi / 4  # alpha: 90 deg horizontal FoV
    v_alpha: float = 0.8           # quadratic boundary value
    sigma: float = 1.0 / 300.0     # bearing noise: 1 px at f = 300 px
    r_min: float = 0.0
    r_max: float = math.inf


PINHOLE = (300.0, 300.0, 300.0, 300.0, 600, 600)  # fx, fy, cx, cy, W, H (90 deg FoV)


def haar_quaternions(rng: np.random.Generator, m: int) -> np.ndarray:
    """Uniform rotations as unit quaternions (w, x, y, z) (normalised Gaussians)."""
    q = rng.standard_normal((m, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def uniform_in_hull(rng: np.random.Generator, grid: Grid, m: int) -> np.ndarray:
    return rng.uniform(grid.hull_lo, grid.hull_hi, size=(m, 3))


# ---------------------------------------------------------------- tiny

def tiny_scene(seed: int = SEED_SCENE + 1, n_landmarks: int = 2000):
    rng = np.random.default_rng(seed)
    lm = rng.uniform([-5.0, -5.0, -2.5], [5.0, 5.0, 2.5], size=(n_landmarks, 3))
    grid = Grid(origin=(-4.75, -4.75, -1.25), h=0.5, shape=(20, 20, 6))
    return lm, grid, Vis()


def tiny_poses(grid: Grid, m: int = 1000, seed: int = SEED_POSES + 1):
    rng = np.random.default_rng(seed)
    return uniform_in_hull(rng, grid, m), haar_quaternions(rng, m)


# ------------------------------------------------------------ building

def _walls_and_clutter(rng, n, box_lo, box_hi, n_walls=12, wall_frac=0.7,
                       length=(5.0, 20.0), margin=2.0, noise=0.05):
    box_lo = np.asarray(box_lo, np.float64)
    box_hi = np.asarray(box_hi, np.float64)
    n_wall = int(round(wall_frac * n))
    n_clut = n - n_wall
    az = rng.uniform(0.0, math.pi, n_walls)
    cx = rng.uniform(box_lo[0] + margin, box_hi[0] - margin, n_walls)
    cy = rng.uniform(box_lo[1] + margin, box_hi[1] - margin, n_walls)
    ln = rng.uniform(length[0], length[1], n_walls)
    # equal area per wall (full height) -> landmarks in proportion to length
    which = rng.choice(n_walls, size=n_wall, p=ln / ln.sum())
    dirx, diry = np.cos(az[which]), np.sin(az[which])
    wall = np.zeros((n_wall, 3))
    todo = np.arange(n_wall)
    for _ in range(64):  # walls are cut by the box: redraw points that fall outside
        if todo.size == 0:
            break
        w = which[todo]
        s = rng.uniform(-0.5, 0.5, todo.size) * ln[w]
        off = rng.normal(0.0, noise, todo.size)
        wall[todo, 0] = cx[w] + s * dirx[todo] - off * diry[todo]
        wall[todo, 1] = cy[w] + s * diry[todo] + off * dirx[todo]
        wall[todo, 2] = rng.uniform(box_lo[2], box_hi[2], todo.size)
        inside = ((wall[todo] >= box_lo) & (wall[todo] <= box_hi)).all(axis=1)
        todo = todo[~inside]
    wall[todo] = np.clip(wall[todo], box_lo, box_hi)
    clutter = rng.uniform(box_lo, box_hi, size=(n_clut, 3))
    lm = np.concatenate([wall, clutter], axis=0)
    return lm[rng.permutation(n)]


def building_scene(n_landmarks: int = 100_000, seed: int = SEED_SCENE + 2,
                   shape=(200, 200, 50), h: float = 0.2, r_max: float = 15.0):
    """Walls + clutter in the box [-20,20]^2 x [-5,5] (or the box of `shape`)."""
    rng = np.random.default_rng(seed)
    half = np.asarray(shape, np.float64) * h / 2.0
    lm = _walls_and_clutter(rng, n_landmarks, -half, half)
    origin = tuple(float(x) for x in (-half + h / 2.0))
    grid = Grid(origin=origin, h=h, shape=tuple(int(s) for s in shape))
    return lm, grid, Vis(r_max=r_max)


def wall_patch(n: int = 1000, seed: int = SEED_SCENE + 8, centre=(3.0, -2.0, 0.0),
               size: float = 2.0, noise: float = 0.05) -> np.ndarray:
    """A newly observed piece of wall for incremental updates: n landmarks on a
    vertical size x size square at `centre` with a random azimuth, offset along
    its normal by N(0, noise^2)."""
    rng = np.random.default_rng(seed)
    az = rng.uniform(0.0, math.pi)
    s = rng.uniform(-0.5, 0.5, n) * size
    zz = rng.uniform(-0.5, 0.5, n) * size
    off = rng.normal(0.0, noise, n)
    c = np.asarray(centre, np.float64)
    return np.stack([c[0] + s * math.cos(az) - off * math.sin(az),
                     c[1] + s * math.sin(az) + off * math.cos(az),
                     c[2] + zz], axis=1)


def building_poses(grid: Grid, m: int, seed: int = SEED_POSES + 2, dtype=np.float32):
    rng = np.random.default_rng(seed)
    t = uniform_in_hull(rng, grid, m)
    q = haar_quaternions(rng, m)
    return t.astype(dtype), q.astype(dtype)


# --------------------------------------------------------- trajectories

def _bspline_eval(ctrl: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Uniform cubic B-spline through control points ctrl[..., n, d] at s in [0, 1]."""
    n = ctrl.shape[-2]
    nseg = n - 3
    x = np.clip(s, 0.0, 1.0) * nseg
    seg = np.minimum(np.floor(x).astype(np.int64), nseg - 1)
    u = x - seg
    b0 = (1 - u) ** 3 / 6.0
    b1 = (3 * u ** 3 - 6 * u ** 2 + 4) / 6.0
    b2 = (-3 * u ** 3 + 3 * u ** 2 + 3 * u + 1) / 6.0
    b3 = u ** 3 / 6.0
    out = 0.0
    for i, b in enumerate((b0, b1, b2, b3)):
        out = out + b[..., None] * np.take_along_axis(
            ctrl, (seg + i)[..., None].repeat(ctrl.shape[-1], -1), axis=-2)
    return out


def rotation_to_quaternion(R: np.ndarray) -> np.ndarray:
    """(w, x, y, z) of rotation matrices R[..., 3, 3] (Shepperd's method)."""
    R = np.asarray(R, np.float64)
    tr = R[..., 0, 0] + R[..., 1, 1] + R[..., 2, 2]
    cands = np.stack([
        np.stack([1 + tr, R[..., 2, 1] - R[..., 1, 2], R[..., 0, 2] - R[..., 2, 0],
                  R[..., 1, 0] - R[..., 0, 1]], -1),
        np.stack([R[..., 2, 1] - R[..., 1, 2], 1 + 2 * R[..., 0, 0] - tr,
                  R[..., 0, 1] + R[..., 1, 0], R[..., 0, 2] + R[..., 2, 0]], -1),
        np.stack([R[..., 0, 2] - R[..., 2, 0], R[..., 0, 1] + R[..., 1, 0],
                  1 + 2 * R[..., 1, 1] - tr, R[..., 1, 2] + R[..., 2, 1]], -1),
        np.stack([R[..., 1, 0] - R[..., 0, 1], R[..., 0, 2] + R[..., 2, 0],
                  R[..., 1, 2] + R[..., 2, 1], 1 + 2 * R[..., 2, 2] - tr], -1)], -2)
    diag = np.stack([tr, R[..., 0, 0], R[..., 1, 1], R[..., 2, 2]], -1)
    pick = np.argmax(diag, axis=-1)
    q = np.take_along_axis(cands, pick[..., None, None].repeat(4, -1), axis=-2)[..., 0, :]
    q /= np.linalg.norm(q, axis=-1, keepdims=True)
    return q


def trajectories(grid: Grid, n_traj: int = 4096, n_poses: int = 64, length: float = 5.0,
                 seed: int = SEED_POSES + 4, n_ctrl: int = 7, dtype=np.float32):
    """Smooth camera trajectories inside the voxel-centre hull.

    Positions: uniform cubic B-spline through random control points, rescaled
    to `length` metres of arc, started uniformly in the hull (rejected and
    redrawn if any sample leaves it).  Yaw: B-spline over U[-pi, pi]; pitch:
    B-spline within +-30 deg.  Optical axis z = [cp cy, cp sy, sp]; the camera
    x axis is horizontal (x = z x up / |.|), y = z x x; R_wc = [x y z].
    Returns t[n_traj, n_poses, 3], q[n_traj, n_poses, 4].
    """
    rng = np.random.default_rng(seed)
    lo, hi = grid.hull_lo, grid.hull_hi
    s = np.linspace(0.0, 1.0, n_poses)
    fine = np.linspace(0.0, 1.0, 8 * n_poses)
    out_t = np.zeros((n_traj, n_poses, 3))
    done = np.zeros(n_traj, bool)
    while not done.all():
        idx = np.nonzero(~done)[0]
        k = idx.shape[0]
        ctrl = rng.normal(0.0, 1.0, (k, n_ctrl, 3))
        ctrl[..., 2] *= 0.3
        pts = _bspline_eval(ctrl, np.broadcast_to(fine, (k, fine.shape[0])))
        arc = np.linalg.norm(np.diff(pts, axis=1), axis=-1).sum(-1)
        scale = length / np.maximum(arc, 1e-9)
        ctrl = ctrl * scale[:, None, None]
        p = _bspline_eval(ctrl, np.broadcast_to(s, (k, n_poses)))
        p = p - p[:, :1, :]
        start = rng.uniform(lo, hi, size=(k, 1, 3))
        p = p + start
        ok = ((p >= lo) & (p <= hi)).all(axis=(1, 2))
        out_t[idx[ok]] = p[ok]
        done[idx[ok]] = True
    yaw_c = rng.uniform(-math.pi, math.pi, (n_traj, n_ctrl, 1))
    pitch_c = rng.uniform(-math.radians(30), math.radians(30), (n_traj, n_ctrl, 1))
    yaw = _bspline_eval(yaw_c, np.broadcast_to(s, (n_traj, n_poses)))[..., 0]
    pitch = _bspline_eval(pitch_c, np.broadcast_to(s, (n_traj, n_poses)))[..., 0]
    z = np.stack([np.cos(pitch) * np.cos(yaw), np.cos(pitch) * np.sin(yaw), np.sin(pitch)], -1)
    up = np.array([0.0, 0.0, 1.0])
    x = np.cross(z, up)
    x /= np.linalg.norm(x, axis=-1, keepdims=True)
    y = np.cross(z, x)
    R = np.stack([x, y, z], axis=-1)  # columns
    q = rotation_to_quaternion(R)
    return out_t.astype(dtype), q.astype(dtype)


# ------------------------------------------------------------- serving

SERVE_SHAPES = ((64, 64, 64), (128, 128, 32), (200, 200, 50), (256, 256, 64))


def serve_scenes(n_landmarks: int = 100_000, seed: int = SEED_SCENE + 5, h: float = 0.2):
    """Four building-like scenes, one per field shape, each in its own box."""
    out = []
    for i, shape in enumerate(SERVE_SHAPES):
        frac = np.prod(shape) / np.prod((200, 200, 50))
        n = max(1000, int(n_landmarks * frac))
        out.append(building_scene(n, seed=seed + i, shape=shape, h=h))
    return out


@dataclasses.dataclass(frozen=True)
class RequestSpec:
    rid: int
    arrival: float  # seconds from stream start
    field: int
    kind: str       # "plan" (queries only) or "opt" (queries + gradients)
    offset: int     # first pose in the field's pool for this kind
    m: int          # number of poses


def request_stream(n_fields: int, rate_hz: float, n_requests: int, plan_pool: int,
                   traj_pool: int, n_poses_traj: int = 64, seed: int = SEED_POSES + 5):
    """Poisson arrivals at `rate_hz`; half planner batches of 1-256 random poses,
    half optimizer batches of 8-64 trajectories x `n_poses_traj` poses; the
    field is chosen uniformly.  Poses are slices of per-field pools: the
    planner pool holds `plan_pool` random poses, the trajectory pool
    `traj_pool` whole trajectories."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for rid in range(n_requests):
        f = int(rng.integers(n_fields))
        if rng.random() < 0.5:
            m = int(rng.integers(1, 257))
            off = int(rng.integers(0, plan_pool - m + 1))
            out.append(RequestSpec(rid, float(arrivals[rid]), f, "plan", off, m))
        else:
            ntr = int(rng.integers(8, 65))
            first = int(rng.integers(0, traj_pool - ntr + 1))
            out.append(RequestSpec(rid, float(arrivals[rid]), f, "opt", first * n_poses_traj,
                                   ntr * n_poses_traj))
    return out


def sphere_axes(n: int) -> np.ndarray:
    """n unit vectors spread evenly over the sphere (Fibonacci lattice): the
    candidate optical axes of a dense view sweep."""
    i = np.arange(n, dtype=np.float64) + 0.5
    zc = 1.0 - 2.0 * i / n
    r = np.sqrt(np.maximum(0.0, 1.0 - zc * zc))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), zc], axis=1)


def sweep_positions(grid: Grid, n: int = 200, seed: int = 2006,
                    dtype=np.float32) -> np.ndarray:
    """n positions for an optimal-view sweep (200 in Sec. VII-A), uniform in the
    hull of the voxel centres like the building poses."""
    rng = np.random.default_rng(seed)
    return uniform_in_hull(rng, grid, n).astype(dtype)


def gp_training_directions(n: int = 200, seed: int = 2007) -> np.ndarray:
    """Unit bearings of random landmarks: the training inputs of the GP length
    scale fit (Sec. V-B, hyperparameters)."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((n, 3))
    return u / np.linalg.norm(u, axis=1, keepdims=True)


# SE length scales for the GP visibility at N_s sphere-lattice axes (k_s = 15,
# alpha = 45 deg, noise 1e-10): the maximiser of the evidence over the 200
# training bearings above, rounded to 4 digits.  They are inputs of the GP
# workloads; the test suite checks each against the oracle's own fit.
GP_LENGTH = {30: 0.8927, 70: 0.6127, 150: 0.4448}
