"""Seeded synthetic point-cloud pairs shaped like the paper's three workloads.

This module only builds inputs: scenes, sensor sampling, noise, outliers and the
ground-truth rigid motion.  It contains none of the registration arithmetic and
is shared by the GPU tests, the oracle tests and the benchmark.  Everything is
generated in float64 and rounded once to float32 at the end.

Stand-ins (the paper's datasets are not used):
  * range_scanner_pair  -- object scans of Sec. 4.1/4.2 (about 3.5k points)
  * rgbd_pair           -- the indoor RGBD frames of Sec. 4.3
  * lidar_pair          -- the street LiDAR scans of Sec. 4.4
Seeds: numpy.random.default_rng([210315039, workload, trial]).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 210315039


@dataclass
class Pair:
    X: np.ndarray        # (N, 3) float32 source
    Y: np.ndarray        # (M, 3) float32 target
    R_gt: np.ndarray     # (3, 3) float64, g_gt(x) = R_gt x + t_gt maps source -> target
    t_gt: np.ndarray     # (3,)  float64
    name: str = ""


def rng_for(workload: int, trial: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE, int(workload), int(trial)])


def rot_axis_angle(axis, angle):
    """Rotation matrix about a unit axis (Rodrigues), float64."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def random_unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def random_rotation(rng, angle):
    return rot_axis_angle(random_unit(rng), angle)


# ---------------------------------------------------------------------------
# Workload 0: range-scanner stand-in (box surface + sphere)
# ---------------------------------------------------------------------------

def _sample_box_sphere(rng, n):
    """n points uniform by area on the surface of the cube [-0.5, 0.5]^3 and a
    sphere of radius 0.3 centred at (0, 0, 0.8)."""
    a_box, a_sph = 6.0, 4 * math.pi * 0.09
    nb = rng.binomial(n, a_box / (a_box + a_sph))
    face = rng.integers(0, 6, size=nb)
    uv = rng.uniform(-0.5, 0.5, size=(nb, 2))
    P = np.empty((nb, 3))
    ax = face // 2
    sign = np.where(face % 2 == 0, -0.5, 0.5)
    for k in range(3):
        sel = ax == k
        o = [c for c in range(3) if c != k]
        P[sel, k] = sign[sel]
        P[sel, o[0]] = uv[sel, 0]
        P[sel, o[1]] = uv[sel, 1]
    S = rng.normal(size=(n - nb, 3))
    S = 0.3 * S / np.linalg.norm(S, axis=1, keepdims=True) + np.array([0, 0, 0.8])
    Q = np.vstack([P, S])
    return Q[rng.permutation(n)]


def range_scanner_pair(trial=0, M=2000, N=2000, angle_deg=30.0, noise=0.005,
                       trans=0.1):
    """Target: M points on the box+sphere surface.  Source: an independent
    N-point resample, rotated about a random axis by angle_deg, translated by
    U(-trans, trans)^3, plus N(0, noise^2) per coordinate."""
    rng = rng_for(0, trial)
    Y = _sample_box_sphere(rng, M)
    S = _sample_box_sphere(rng, N)
    Ra = random_rotation(rng, math.radians(angle_deg))
    ta = rng.uniform(-trans, trans, size=3)
    X = S @ Ra.T + ta + rng.normal(scale=noise, size=S.shape)
    # source = Ra s + ta  =>  g_gt(x) = Ra^T (x - ta)
    return Pair(X=X.astype(np.float32), Y=Y.astype(np.float32), R_gt=Ra.T.copy(),
                t_gt=-(Ra.T @ ta), name=f"range_scanner_{M}x{N}")


# ---------------------------------------------------------------------------
# Ray casting helpers (numpy, vectorised over rays)
# ---------------------------------------------------------------------------

def _hit_box(o, d, R, c, h):
    """Ray parameter of the first hit of rays (o, d) with an oriented box
    (rotation R, centre c, half extents h) seen from outside; inf on a miss."""
    ol = (o - c) @ R
    dl = d @ R
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (-h - ol) / dl
        t2 = (h - ol) / dl
    tmin = np.nanmax(np.minimum(t1, t2), axis=1)
    tmax = np.nanmin(np.maximum(t1, t2), axis=1)
    hit = (tmax >= tmin) & (tmin > 1e-6)
    return np.where(hit, tmin, np.inf)


def _hit_room(o, d, lo, hi):
    """Ray parameter of the exit point of rays starting inside an axis-aligned
    room [lo, hi]."""
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (lo - o) / d
        t2 = (hi - o) / d
    tt = np.maximum(t1, t2)
    tt = np.where(np.isfinite(tt) & (tt > 0), tt, np.inf)
    return tt.min(axis=1)


def _hit_quad(o, d, c, u, v, hu, hv):
    """Ray hits with a finite rectangle centred at c spanned by unit u, v."""
    nrm = np.cross(u, v)
    den = d @ nrm
    with np.errstate(divide="ignore", invalid="ignore"):
        t = ((c - o) @ nrm) / den
    p = o + t[:, None] * d
    q = p - c
    ok = (t > 1e-6) & (np.abs(q @ u) <= hu) & (np.abs(q @ v) <= hv)
    return np.where(ok, t, np.inf)


def _hit_cylinder(o, d, cx, cy, r, height):
    """Vertical cylinder (axis along z from z=0 to height) outer surface."""
    ox, oy = o[:, 0] - cx, o[:, 1] - cy
    a = d[:, 0] ** 2 + d[:, 1] ** 2
    b = 2 * (ox * d[:, 0] + oy * d[:, 1])
    cc = ox ** 2 + oy ** 2 - r * r
    disc = b * b - 4 * a * cc
    with np.errstate(invalid="ignore", divide="ignore"):
        t = (-b - np.sqrt(disc)) / (2 * a)
    z = o[:, 2] + t * d[:, 2]
    ok = (disc >= 0) & (t > 1e-6) & (z >= 0) & (z <= height)
    return np.where(ok, t, np.inf)


# ---------------------------------------------------------------------------
# Workload 1: RGBD stand-in (room with boxes and tilted planes, 160 x 125)
# ---------------------------------------------------------------------------

_W, _H, _F, _CX, _CY = 160, 125, 140.0, 79.5, 62.0


def _room_scene(rng):
    lo = np.array([-2.5, -1.4, -0.5])
    hi = np.array([2.5, 1.4, 6.0])
    boxes = []
    for _ in range(int(rng.integers(3, 7))):
        h = rng.uniform(0.1, 0.4, size=3)
        c = np.array([rng.uniform(-1.8, 1.8), lo[1] + h[1], rng.uniform(2.0, 5.0)])
        boxes.append((rot_axis_angle([0, 1, 0], rng.uniform(0, math.pi)), c, h))
    quads = []
    for _ in range(2):
        c = np.array([rng.uniform(-1.5, 1.5), rng.uniform(-0.5, 0.8), rng.uniform(2.5, 5.0)])
        Rq = random_rotation(rng, rng.uniform(0.2, 0.9))
        quads.append((c, Rq[:, 0], Rq[:, 1], rng.uniform(0.3, 0.6), rng.uniform(0.3, 0.6)))
    return lo, hi, boxes, quads


def _render_depth(rng, scene, Rc, tc, noise=(0.0, 0.002, 0.0)):
    """Render the scene from a pinhole camera (camera-to-world Rc, tc; camera
    looks along +z).  Returns camera-frame points, one per pixel, with depth
    noise N(0, s(z)^2), s(z) = noise[0] + noise[1] z + noise[2] z^2."""
    lo, hi, boxes, quads = scene
    u, v = np.meshgrid(np.arange(_W), np.arange(_H))
    dc = np.stack([(u.ravel() - _CX) / _F, (v.ravel() - _CY) / _F, np.ones(u.size)], axis=1)
    dw = dc @ Rc.T
    o = np.broadcast_to(tc, dw.shape)
    t = _hit_room(o, dw, lo, hi)
    for (Rb, c, h) in boxes:
        t = np.minimum(t, _hit_box(o, dw, Rb, c, h))
    for (c, uu, vv, hu, hv) in quads:
        t = np.minimum(t, _hit_quad(o, dw, c, uu, vv, hu, hv))
    z = t  # dc has unit z component, so the ray parameter is the depth
    z = z + rng.normal(size=z.shape) * (noise[0] + noise[1] * z + noise[2] * z * z)
    return dc * z[:, None]


def rgbd_pair(trial=0, outlier_frac=0.05, angle_deg=15.0, trans=0.05):
    """Two 160x125 depth frames of one random room, back-projected (20,000
    points each), depth noise N(0, (0.002 z)^2), 5 % of the points replaced by
    uniform samples in the cloud's box.  Second camera: 15 deg about a random
    axis and 0.05 m in a random direction from the first."""
    rng = rng_for(1, trial)
    scene = _room_scene(rng)
    R1 = np.eye(3)
    t1 = np.array([0.0, 0.0, 0.0])
    R2 = random_rotation(rng, math.radians(angle_deg)) @ R1
    t2 = t1 + trans * random_unit(rng)
    clouds = []
    for (Rc, tc) in ((R1, t1), (R2, t2)):
        P = _render_depth(rng, scene, Rc, tc)
        n_out = int(round(outlier_frac * P.shape[0]))
        idx = rng.choice(P.shape[0], size=n_out, replace=False)
        P[idx] = rng.uniform(P.min(axis=0), P.max(axis=0), size=(n_out, 3))
        clouds.append(P)
    Y, X = clouds[0], clouds[1]
    # x (camera 2) -> world: R2 x + t2 -> camera 1: R1^T (. - t1)
    R_gt = R1.T @ R2
    t_gt = R1.T @ (t2 - t1)
    return Pair(X=X.astype(np.float32), Y=Y.astype(np.float32), R_gt=R_gt, t_gt=t_gt,
                name="rgbd_20000x20000")


# Depth noise of depth_pair: standard deviation c0 + c1 z + c2 z^2 metres at
# depth z, over a sensor range of 0.4-6.5 m; its smallest value in that range
# is the one at 0.4 m.
DEPTH_ERROR = (1.0e-3, 0.0, 1.5e-3)
DEPTH_ERROR_MIN = 1.24e-3


def depth_pair(trial=0, M=20000, N=20000, outlier_frac=0.02, angle_deg=10.0, trans=0.05):
    """Two depth frames of one random room (as rgbd_pair) whose depth noise
    grows with the square of the depth (DEPTH_ERROR), the setting of the
    paper's confidence filtering (Sec. 3.3); M and N of the 20,000 pixels of
    each frame are kept at random, 2 % of them replaced by uniform samples in
    the cloud's box.  Each cloud is in its own camera frame (depth = z)."""
    rng = rng_for(4, trial)
    scene = _room_scene(rng)
    R2 = random_rotation(rng, math.radians(angle_deg))
    t2 = trans * random_unit(rng)
    clouds = []
    for (Rc, tc), n in (((np.eye(3), np.zeros(3)), M), ((R2, t2), N)):
        P = _render_depth(rng, scene, Rc, tc, noise=DEPTH_ERROR)
        P = P[rng.choice(P.shape[0], size=n, replace=False)]
        n_out = int(round(outlier_frac * n))
        idx = rng.choice(n, size=n_out, replace=False)
        P[idx] = rng.uniform(P.min(axis=0), P.max(axis=0), size=(n_out, 3))
        clouds.append(P)
    Y, X = clouds
    return Pair(X=X.astype(np.float32), Y=Y.astype(np.float32), R_gt=R2, t_gt=t2,
                name=f"depth_{M}x{N}")


# ---------------------------------------------------------------------------
# Workload 2: LiDAR stand-in (64-ring spinning scan of a street)
# ---------------------------------------------------------------------------

def _street_scene(rng):
    facades = []   # axis-aligned boxes (R=I) as (c, h)
    for side in (-1, 1):
        x = -70.0
        while x < 70.0:
            w = rng.uniform(6, 20)
            gap = rng.uniform(0, 4) if rng.uniform() < 0.5 else 0.0
            setback = rng.uniform(0, 4)
            height = rng.uniform(5, 20)
            y0 = side * (6.0 + setback)
            c = np.array([x + w / 2, y0 + side * 5.0, height / 2])
            facades.append((c, np.array([w / 2, 5.0, height / 2])))
            x += w + gap
        # back row so that rays through gaps still return
        facades.append((np.array([0.0, side * 30.0, 10.0]), np.array([80.0, 2.0, 10.0])))
    for xend in (-62.0, 62.0):
        facades.append((np.array([xend + np.sign(xend) * 2.0, 0.0, 10.0]), np.array([2.0, 40.0, 10.0])))
    cyl = []
    for _ in range(int(rng.integers(20, 41))):
        side = rng.choice([-1, 1])
        cyl.append((rng.uniform(-55, 55), side * rng.uniform(4.0, 5.8),
                    rng.uniform(0.1, 0.5), rng.uniform(2.0, 8.0)))
    return facades, cyl


def _lidar_scan(rng, scene, Rs, ts, keep):
    facades, cyl = scene
    el = np.radians(rng.uniform(-25.0, 3.0, size=64))
    az = np.arange(2048) * (2 * math.pi / 2048)
    E, A = np.meshgrid(el, az, indexing="ij")
    dl = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], axis=-1).reshape(-1, 3)
    dw = dl @ Rs.T
    o = np.broadcast_to(ts, dw.shape)
    with np.errstate(divide="ignore", invalid="ignore"):
        tg = np.where(dw[:, 2] < 0, -ts[2] / dw[:, 2], np.inf)
    t = tg
    I3 = np.eye(3)
    for (c, h) in facades:
        t = np.minimum(t, _hit_box(o, dw, I3, c, h))
    for (cx, cy, r, hgt) in cyl:
        t = np.minimum(t, _hit_cylinder(o, dw, cx, cy, r, hgt))
    ok = np.isfinite(t) & (t <= 80.0)
    t = t[ok] + rng.normal(scale=0.01, size=int(ok.sum()))
    P = dl[ok] * t[:, None]
    if P.shape[0] < keep:
        raise RuntimeError(f"scan returned only {P.shape[0]} points (< {keep})")
    sel = rng.choice(P.shape[0], size=keep, replace=False)
    return P[np.sort(sel)]


def lidar_pair(trial=0, M=100000, N=50000, dist=1.0, yaw_deg=10.0):
    """Target: M returns of a 64-ring, 2048-step scan (elevations in
    [-25, +3] deg, max range 80 m, range noise N(0, 0.01^2)) of a street with
    facades, ground and poles, sensor at 1.7 m.  Source: N returns of a second
    scan from a pose dist metres away with yaw_deg of yaw.  Points are in their
    own sensor frames."""
    rng = rng_for(2, trial)
    scene = _street_scene(rng)
    R1, t1 = np.eye(3), np.array([0.0, 0.0, 1.7])
    phi = rng.uniform(0, 2 * math.pi)
    R2 = rot_axis_angle([0, 0, 1], math.radians(yaw_deg))
    t2 = t1 + dist * np.array([math.cos(phi), math.sin(phi), 0.0])
    Y = _lidar_scan(rng, scene, R1, t1, M)
    X = _lidar_scan(rng, scene, R2, t2, N)
    R_gt = R1.T @ R2
    t_gt = R1.T @ (t2 - t1)
    return Pair(X=X.astype(np.float32), Y=Y.astype(np.float32), R_gt=R_gt, t_gt=t_gt,
                name=f"lidar_{M}x{N}")


# ---------------------------------------------------------------------------
# Small generic inputs for unit tests
# ---------------------------------------------------------------------------

def random_cloud(rng, n, scale=1.0):
    return (rng.normal(size=(n, 3)) * scale).astype(np.float32)


def random_unit_normals(rng, m):
    v = rng.normal(size=(m, 3))
    return (v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)


def plane_patch(rng, n, normal=(0.0, 0.0, 1.0), size=1.0, offset=0.0):
    """n points on a square patch of the plane through offset*normal."""
    nrm = np.asarray(normal, dtype=np.float64)
    nrm /= np.linalg.norm(nrm)
    a = np.cross(nrm, [1.0, 0.0, 0.0])
    if np.linalg.norm(a) < 1e-6:
        a = np.cross(nrm, [0.0, 1.0, 0.0])
    a /= np.linalg.norm(a)
    b = np.cross(nrm, a)
    uv = rng.uniform(-size / 2, size / 2, size=(n, 2))
    return uv[:, :1] * a + uv[:, 1:] * b + offset * nrm


# ---------------------------------------------------------------------------
# Batches of small pairs of uneven sizes (box / sphere / plane-patch scenes)
# ---------------------------------------------------------------------------

def _primitive_scene(rng, min_prims=1):
    """min_prims-3 primitives: (kind, parameters, area)."""
    prims = []
    for _ in range(int(rng.integers(min_prims, 4))):
        kind = int(rng.integers(0, 3))
        c = rng.uniform(-0.3, 0.3, size=3)
        if kind == 0:      # box: rotation, centre, half extents
            h = rng.uniform(0.1, 0.35, size=3)
            R = random_rotation(rng, rng.uniform(0, math.pi))
            area = 8.0 * (h[0] * h[1] + h[1] * h[2] + h[0] * h[2])
            prims.append(("box", (R, c, h), area))
        elif kind == 1:    # sphere
            r = rng.uniform(0.1, 0.35)
            prims.append(("sphere", (c, r), 4.0 * math.pi * r * r))
        else:              # square plane patch
            size = rng.uniform(0.3, 0.8)
            prims.append(("plane", (random_unit(rng), c, size), size * size))
    return prims


def _sample_scene(rng, prims, n):
    areas = np.array([a for _, _, a in prims])
    counts = rng.multinomial(n, areas / areas.sum())
    parts = []
    for (kind, par, _), k in zip(prims, counts):
        if k == 0:
            continue
        if kind == "box":
            R, c, h = par
            # faces drawn in proportion to their area
            fa = np.array([h[1] * h[2], h[1] * h[2], h[0] * h[2], h[0] * h[2],
                           h[0] * h[1], h[0] * h[1]])
            face = rng.choice(6, size=k, p=fa / fa.sum())
            ax = face // 2
            sign = np.where(face % 2 == 0, -1.0, 1.0)
            P = rng.uniform(-1.0, 1.0, size=(k, 3)) * h
            P[np.arange(k), ax] = sign * h[ax]
            parts.append(P @ R.T + c)
        elif kind == "sphere":
            c, r = par
            v = rng.normal(size=(k, 3))
            parts.append(r * v / np.linalg.norm(v, axis=1, keepdims=True) + c)
        else:
            nrm, c, size = par
            parts.append(plane_patch(rng, k, normal=nrm, size=size) + c)
    P = np.vstack(parts)
    return P[rng.permutation(len(P))]


def scene_pair(rng, M, N, max_angle_deg=60.0, trans=0.1, noise=0.005, max_outliers=0.1,
               name="scene"):
    """Target: M points on a random primitive scene.  Source: an independent
    N-point resample, rotated by U(0, max_angle) about a uniform axis,
    translated by U(-trans, trans)^3, noise N(0, noise^2) per coordinate, then
    a U(0, max_outliers) fraction replaced by uniform points in its box."""
    prims = _primitive_scene(rng)
    Y = _sample_scene(rng, prims, M)
    S = _sample_scene(rng, prims, N)
    Ra = random_rotation(rng, math.radians(rng.uniform(0.0, max_angle_deg)))
    ta = rng.uniform(-trans, trans, size=3)
    X = S @ Ra.T + ta + rng.normal(scale=noise, size=S.shape)
    nout = int(round(rng.uniform(0.0, max_outliers) * N))
    if nout:
        lo, hi = X.min(axis=0), X.max(axis=0)
        X[rng.choice(N, size=nout, replace=False)] = rng.uniform(lo, hi, size=(nout, 3))
    return Pair(X=X.astype(np.float32), Y=Y.astype(np.float32), R_gt=Ra.T.copy(),
                t_gt=-(Ra.T @ ta), name=name)


def uniform_rotation(rng):
    """A rotation drawn uniformly on SO(3): the unit quaternion of four
    independent standard normals."""
    w, x, y, z = (lambda q: q / np.linalg.norm(q))(rng.normal(size=4))
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def proposal_pair(rng, M, N, trans=0.1, noise=0.005, max_outliers=0.1, name="proposal"):
    """A scene pair for the learned initial-pose proposal: as scene_pair, but
    the scene has 2-3 primitives (one alone has symmetries that make its
    rotation ambiguous) and the source's rotation is uniform on SO(3)."""
    prims = _primitive_scene(rng, min_prims=2)
    Y = _sample_scene(rng, prims, M)
    S = _sample_scene(rng, prims, N)
    Ra = uniform_rotation(rng)
    ta = rng.uniform(-trans, trans, size=3)
    X = S @ Ra.T + ta + rng.normal(scale=noise, size=S.shape)
    nout = int(round(rng.uniform(0.0, max_outliers) * N))
    if nout:
        lo, hi = X.min(axis=0), X.max(axis=0)
        X[rng.choice(N, size=nout, replace=False)] = rng.uniform(lo, hi, size=(nout, 3))
    return Pair(X=X.astype(np.float32), Y=Y.astype(np.float32), R_gt=Ra.T.copy(),
                t_gt=-(Ra.T @ ta), name=name)


def proposal_pairs(n, split="eval", trial=0, nmin=1000, nmax=30000):
    """n proposal pairs with M and N independently log-uniform in [nmin,
    nmax]; the training and evaluation splits draw from different seeds."""
    rng = rng_for(5 if split == "eval" else 6, trial)
    lo, hi = math.log(nmin), math.log(nmax)
    out = []
    for i in range(n):
        M = int(round(math.exp(rng.uniform(lo, hi))))
        N = int(round(math.exp(rng.uniform(lo, hi))))
        out.append(proposal_pair(rng, M, N, name=f"proposal_{split}{trial}_{i}_{M}x{N}"))
    return out


def batch_pairs(n=256, trial=0, nmin=1000, nmax=30000):
    """n scene pairs with M and N independently log-uniform in [nmin, nmax]."""
    rng = rng_for(3, trial)
    lo, hi = math.log(nmin), math.log(nmax)
    out = []
    for i in range(n):
        M = int(round(math.exp(rng.uniform(lo, hi))))
        N = int(round(math.exp(rng.uniform(lo, hi))))
        out.append(scene_pair(rng, M, N, name=f"batch{trial}_{i}_{M}x{N}"))
    return out


WORKLOADS = {
    "range_scanner_2000x2000": range_scanner_pair,
    "rgbd_20000x20000": rgbd_pair,
    "lidar_100000x50000": lidar_pair,
}
