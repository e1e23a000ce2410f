"""Seeded synthetic scenes for dense deformable registration.

This module only manufactures inputs.  It holds none of the registration
method's arithmetic (no embedded-deformation blending, no skinning weights, no
association, no energies): it builds a tissue-like height-field surface, samples
a model point cloud with normals and a regular grid of graph nodes on it, moves
the surface by a known analytic deformation and a rigid scope pose, and
ray-casts a noisy depth map of the result through a pinhole camera.

Scale follows the paper's in-vivo setting (Sec. III and III-B): tissue 40-70 mm
from the scope, 0.2 mm point density, node grids of a few millimetres, and
deformations of 2-3 mm (Sec. III-D).  Every array is returned as float32, the
precision the GPU path stores its inputs in; the oracle promotes them exactly to
float64.  Units are millimetres.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class SceneSpec:
    name: str
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    patch: tuple            # (x0, x1, y0, y1) of the modelled tissue patch, mm
    pts_grid: tuple         # (nx, ny) model points (cell centres of the patch)
    jitter: float           # +- uniform jitter of model points in x and y, mm
    node_grid: tuple        # (mx, my) nodes
    node_spacing: float     # mm; nodes sit at cell centres of this grid
    deformation: str        # "smooth" (low-frequency field) or "breathing"
    bumps: tuple            # (min, max) number of Gaussian bumps on the surface
    rot_max_deg: float      # rigid pose bound
    trans_max: float        # rigid pose bound, mm
    noise_sigma: float      # depth noise, mm; stereo depth error scales as z^2 / (f b), so 1/fx here
    gn_iters: int
    pcg_iters: int
    seed: int


SPECS = {
    # 64x48 camera, ~3000 points, 48 nodes at 6 mm, smooth known field.
    "c1": SceneSpec("c1", 64, 48, 60.0, 60.0, 32.0, 24.0, (-24.0, 24.0, -18.0, 18.0),
                    (65, 49), 0.1, (8, 6), 6.0, "smooth", (0, 0), 5.0, 8.0, 0.2, 5, 20, 1),
    # 320x240, 60k points, 400 nodes at 5 mm, bumps + breathing.
    "c2": SceneSpec("c2", 320, 240, 128.0, 128.0, 160.0, 120.0, (-62.5, 62.5, -40.0, 40.0),
                    (300, 200), 0.05, (25, 16), 5.0, "breathing", (2, 4), 5.0, 8.0, 0.2 * 60 / 128, 10, 10, 2),
    # 640x480, 250k points at 0.2 mm, 1600 nodes at 2.5 mm, bumps + breathing.
    "c3": SceneSpec("c3", 640, 480, 256.0, 256.0, 320.0, 240.0, (-62.5, 62.5, -40.0, 40.0),
                    (625, 400), 0.02, (50, 32), 2.5, "breathing", (2, 4), 5.0, 8.0, 0.2 * 60 / 256, 10, 10, 3),
    # ragged sizes for edge-case tests: point and node counts that fill no tile evenly
    "ragged": SceneSpec("ragged", 64, 48, 60.0, 60.0, 32.0, 24.0, (-21.0, 21.0, -15.0, 15.0),
                        (37, 29), 0.1, (7, 5), 6.0, "smooth", (1, 2), 3.0, 3.0, 0.2, 4, 15, 7),
}


# ----------------------------------------------------------------------------------------
# surface


class Surface:
    """z = 60 + 3 sin(x/8) cos(y/10) + sum of Gaussian bumps (all mm)."""

    def __init__(self, bumps):
        # bumps: array (B, 4) of (x0, y0, amplitude, width)
        self.bumps = np.asarray(bumps, dtype=np.float64).reshape(-1, 4)

    def z(self, x, y):
        z = 60.0 + 3.0 * np.sin(x / 8.0) * np.cos(y / 10.0)
        for bx, by, a, w in self.bumps:
            z = z + a * np.exp(-((x - bx) ** 2 + (y - by) ** 2) / (2.0 * w * w))
        return z

    def grad(self, x, y):
        zx = (3.0 / 8.0) * np.cos(x / 8.0) * np.cos(y / 10.0)
        zy = -(3.0 / 10.0) * np.sin(x / 8.0) * np.sin(y / 10.0)
        for bx, by, a, w in self.bumps:
            e = a * np.exp(-((x - bx) ** 2 + (y - by) ** 2) / (2.0 * w * w))
            zx = zx - e * (x - bx) / (w * w)
            zy = zy - e * (y - by) / (w * w)
        return zx, zy

    def normal(self, x, y):
        """Unit normal facing the camera (negative z)."""
        zx, zy = self.grad(x, y)
        n = np.stack([zx, zy, -np.ones_like(zx)], axis=-1)
        return n / np.linalg.norm(n, axis=-1, keepdims=True)


# ----------------------------------------------------------------------------------------
# known deformations (analytic; the registration has to discover them)


class SmoothField:
    """X -> X + d(X), d a sum of two low-frequency sinusoids per component.

    Amplitudes <= 0.75 mm per sinusoid (<= 1.5 mm per component) and wavelengths
    of 180-360 mm keep the local rotation of the field below about 3 degrees.
    """

    def __init__(self, rng):
        self.k = np.zeros((3, 2, 3))
        self.a = rng.uniform(0.3, 0.75, size=(3, 2))
        self.ph = rng.uniform(0.0, 2.0 * np.pi, size=(3, 2))
        for c in range(3):
            for s in range(2):
                lam = rng.uniform(180.0, 360.0)
                th = rng.uniform(0.0, 2.0 * np.pi)
                self.k[c, s] = (2.0 * np.pi / lam) * np.array([np.cos(th), np.sin(th), 0.0])

    def __call__(self, X):
        X = np.asarray(X, dtype=np.float64)
        out = X.copy()
        for c in range(3):
            for s in range(2):
                out[..., c] += self.a[c, s] * np.sin(X @ self.k[c, s] + self.ph[c, s])
        return out


class BreathingField:
    """Displacement along the reference surface normal, a*sin(.)*sin(.) over the patch."""

    def __init__(self, rng, surface, patch):
        self.surface = surface
        self.patch = patch
        self.amp = rng.uniform(1.0, 3.0)

    def delta(self, x, y):
        x0, x1, y0, y1 = self.patch
        return self.amp * np.sin(np.pi * (x - x0) / (x1 - x0)) * np.sin(np.pi * (y - y0) / (y1 - y0))

    def __call__(self, X):
        X = np.asarray(X, dtype=np.float64)
        x, y = X[..., 0], X[..., 1]
        return X + self.delta(x, y)[..., None] * self.surface.normal(x, y)


class RigidField:
    """X -> Q X + c: a deformation an ED graph can represent exactly."""

    def __init__(self, Q, c):
        self.Q = np.asarray(Q, dtype=np.float64)
        self.c = np.asarray(c, dtype=np.float64)

    def __call__(self, X):
        return np.asarray(X, dtype=np.float64) @ self.Q.T + self.c


def _random_pose(rng, rot_max_deg, trans_max):
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    ang = math.radians(rng.uniform(0.0, rot_max_deg))
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    R = np.eye(3) + math.sin(ang) * K + (1.0 - math.cos(ang)) * (K @ K)
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    T = d * rng.uniform(0.0, trans_max)
    return R, T


def _jacobian_fd(f, X, h=1e-4):
    """3x3 Jacobian of a field f at points X (..., 3) by central differences."""
    X = np.asarray(X, dtype=np.float64)
    J = np.zeros(X.shape + (3,))
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        J[..., :, c] = (f(X + e) - f(X - e)) / (2.0 * h)
    return J


# ----------------------------------------------------------------------------------------
# depth rendering


def render_depth(spec, surface, field, R, T, rng, noise_sigma):
    """Ray-cast the posed, deformed surface into a depth map (0 = no return).

    For each pixel centre, a 2-D Newton iteration in float64 finds the canonical
    (x, y) whose deformed, posed surface point projects onto it; depth is that
    point's camera z.  A pixel stops iterating once it has converged (each
    pixel's iterates do not depend on the others, so only the unconverged ones
    are carried on).  Pixels that do not converge to 1e-9 px, or whose
    canonical point leaves the tissue patch, stay empty.  Gaussian noise is then
    added to valid pixels.
    """
    W, H = spec.width, spec.height
    fx, fy, cx, cy = spec.fx, spec.fy, spec.cx, spec.cy
    uu, vv = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    u = uu.ravel()
    v = vv.ravel()

    def cam_point(x, y):
        X = np.stack([x, y, surface.z(x, y)], axis=-1)
        Y = field(X)
        return Y @ R.T + T

    def residual(x, y, u, v):
        P = cam_point(x, y)
        return P[:, 0] / P[:, 2] * fx + cx - u, P[:, 1] / P[:, 2] * fy + cy - v, P[:, 2]

    # initial guess: intersect the pixel ray with the plane z = 60 in the canonical frame
    d_cam = np.stack([(u - cx) / fx, (v - cy) / fy, np.ones_like(u)], axis=-1)
    o = -R.T @ T
    d = d_cam @ R
    s = (60.0 - o[2]) / d[:, 2]
    x = o[0] + s * d[:, 0]
    y = o[1] + s * d[:, 1]
    h = 1e-6
    act = np.arange(u.size)          # pixels still iterating
    for _ in range(40):
        xa, ya, ua, va = x[act], y[act], u[act], v[act]
        fu, fv, _ = residual(xa, ya, ua, va)
        go = ~((np.abs(fu) < 1e-9) & (np.abs(fv) < 1e-9))
        act, xa, ya, ua, va, fu, fv = act[go], xa[go], ya[go], ua[go], va[go], fu[go], fv[go]
        if act.size == 0:
            break
        fu_x, fv_x, _ = residual(xa + h, ya, ua, va)
        fu_xm, fv_xm, _ = residual(xa - h, ya, ua, va)
        fu_y, fv_y, _ = residual(xa, ya + h, ua, va)
        fu_ym, fv_ym, _ = residual(xa, ya - h, ua, va)
        a = (fu_x - fu_xm) / (2 * h)
        b = (fu_y - fu_ym) / (2 * h)
        c = (fv_x - fv_xm) / (2 * h)
        e = (fv_y - fv_ym) / (2 * h)
        det = a * e - b * c
        det = np.where(np.abs(det) < 1e-30, 1e-30, det)
        x[act] = xa - (e * fu - b * fv) / det
        y[act] = ya - (-c * fu + a * fv) / det
    fu, fv, z = residual(x, y, u, v)
    ok = (np.abs(fu) < 1e-9) & (np.abs(fv) < 1e-9) & np.isfinite(z) & (z > 0)
    x0, x1, y0, y1 = spec.patch
    ok &= (x >= x0) & (x <= x1) & (y >= y0) & (y <= y1)
    depth = np.where(ok, z, 0.0)
    if noise_sigma > 0:
        noise = rng.normal(0.0, noise_sigma, size=depth.shape)
        depth = np.where(ok, depth + noise, 0.0)
    return depth.reshape(H, W)


# ----------------------------------------------------------------------------------------
# scene assembly


def batch_spec(b, base_seed=500):
    """Spec of problem b of the uneven batch: frame width from {320, ..., 640} (4:3,
    fx = 0.4 W, so every problem sees the same 150 x 112.5 mm field at 60 mm), a
    log-uniform point count in [20k, 300k] over the 125 x 80 mm patch and a
    log-uniform node count in [100, 2000] on a grid of the patch's aspect; the
    320x240 family otherwise (bumps, breathing, 10 x 10 iterations)."""
    rng = np.random.Generator(np.random.PCG64(base_seed + b))
    W = int(rng.choice([320, 384, 448, 512, 576, 640]))
    H = 3 * W // 4
    fx = 0.4 * W
    n_pts = math.exp(rng.uniform(math.log(20000.0), math.log(300000.0)))
    pitch = math.sqrt(10000.0 / n_pts)
    pnx, pny = max(2, int(round(125.0 / pitch))), max(2, int(round(80.0 / pitch)))
    m_nodes = math.exp(rng.uniform(math.log(100.0), math.log(2000.0)))
    s = math.sqrt(10000.0 / m_nodes)
    mx, my = max(2, int(round(125.0 / s))), max(2, int(round(80.0 / s)))
    return SceneSpec(f"batch{b}", W, H, fx, fx, W / 2.0, H / 2.0, (-62.5, 62.5, -40.0, 40.0), (pnx, pny),
                     min(0.05, 0.25 * pitch), (mx, my), s, "breathing", (2, 4), 5.0, 8.0, 0.2 * 60 / fx, 10, 10,
                     base_seed + b)


def make_scene(name, seed=None, noise_sigma=None, with_depth=True, deformation=None):
    """Build one synthetic registration problem.

    Returns a dict of float32/int arrays:
      camera   (width, height, fx, fy, cx, cy)
      points   (N, 3) canonical model points, normals (N, 3) unit, facing the camera
      nodes    (m, 3) node positions on the surface
      R, T     rigid pose, camera = R @ world + T
      depth    (H, W) depth map, 0 where empty
      gt_points (N, 3) float64: model points moved by the known deformation (world)
      gt_node_A, gt_node_t: the deformation's first-order expansion at each node
      sigma    Gaussian skinning width (= node spacing), gn_iters, pcg_iters
    """
    spec = name if isinstance(name, SceneSpec) else SPECS[name]
    name = spec.name
    seed = spec.seed if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    bmin, bmax = spec.bumps
    nb = int(rng.integers(bmin, bmax + 1)) if bmax > 0 else 0
    x0, x1, y0, y1 = spec.patch
    bumps = np.stack([rng.uniform(x0, x1, nb), rng.uniform(y0, y1, nb),
                      rng.uniform(1.0, 4.0, nb), rng.uniform(4.0, 10.0, nb)], axis=1) if nb else np.zeros((0, 4))
    surface = Surface(bumps)

    # model points: cell centres of the patch grid, jittered in x and y, lifted to z = S(x, y)
    nx, ny = spec.pts_grid
    px = x0 + (np.arange(nx) + 0.5) * (x1 - x0) / nx
    py = y0 + (np.arange(ny) + 0.5) * (y1 - y0) / ny
    gx, gy = np.meshgrid(px, py)
    gx = gx.ravel() + rng.uniform(-spec.jitter, spec.jitter, gx.size)
    gy = gy.ravel() + rng.uniform(-spec.jitter, spec.jitter, gy.size)
    pts = np.stack([gx, gy, surface.z(gx, gy)], axis=1)
    nrm = surface.normal(gx, gy)

    # nodes: cell centres of the node grid, lifted to the surface, row-major
    mx, my = spec.node_grid
    s = spec.node_spacing
    cxn = 0.5 * (x0 + x1) + (np.arange(mx) - 0.5 * (mx - 1)) * s
    cyn = 0.5 * (y0 + y1) + (np.arange(my) - 0.5 * (my - 1)) * s
    nX, nY = np.meshgrid(cxn, cyn)
    nodes = np.stack([nX.ravel(), nY.ravel(), surface.z(nX.ravel(), nY.ravel())], axis=1)

    kind = spec.deformation if deformation is None else deformation
    if kind == "rigid":
        Q, c = _random_pose(rng, 2.0, 1.0)
        field = RigidField(Q, c)
    elif kind == "smooth":
        field = SmoothField(rng)
    else:
        field = BreathingField(rng, surface, spec.patch)
    R, T = _random_pose(rng, spec.rot_max_deg, spec.trans_max)

    # everything the path consumes is float32; the truth is computed from those values
    pts32 = pts.astype(np.float32)
    nrm32 = nrm.astype(np.float32)
    nodes32 = nodes.astype(np.float32)
    R32 = R.astype(np.float32)
    T32 = T.astype(np.float32)
    sig = spec.noise_sigma if noise_sigma is None else noise_sigma
    depth = (render_depth(spec, surface, field, R32.astype(np.float64), T32.astype(np.float64), rng, sig)
             if with_depth else np.zeros((spec.height, spec.width)))
    gt_points = field(pts32.astype(np.float64))
    Jn = _jacobian_fd(field, nodes32.astype(np.float64))
    gt_t = field(nodes32.astype(np.float64)) - nodes32.astype(np.float64)
    return {
        "name": name,
        "camera": (spec.width, spec.height, spec.fx, spec.fy, spec.cx, spec.cy),
        "points": pts32,
        "normals": nrm32,
        "nodes": nodes32,
        "R": R32,
        "T": T32,
        "depth": depth.astype(np.float32),
        "gt_points": gt_points,
        "gt_node_A": Jn,
        "gt_node_t": gt_t,
        "sigma": float(s),
        "node_spacing": float(s),
        "gn_iters": spec.gn_iters,
        "pcg_iters": spec.pcg_iters,
        "seed": seed,
    }


def plane_scene(width=32, height=24, f=30.0, z0=50.0, n_side=12, node_side=3, spacing=8.0, k_shift=0.0):
    """A fronto-parallel plane at z = z0 seen head-on: normals (0, 0, -1) everywhere.

    Model points lie on the plane z0 + k_shift (so a common z translation of
    k_shift brings them onto the observed plane).  Used for closed-form checks.
    """
    cx, cy = width / 2.0, height / 2.0
    half = 0.5 * spacing * node_side
    xs = np.linspace(-half + 0.5, half - 0.5, n_side)
    X, Y = np.meshgrid(xs, xs)
    pts = np.stack([X.ravel(), Y.ravel(), np.full(X.size, z0 + k_shift)], axis=1).astype(np.float32)
    nrm = np.tile(np.array([0.0, 0.0, -1.0], dtype=np.float32), (pts.shape[0], 1))
    c = (np.arange(node_side) - 0.5 * (node_side - 1)) * spacing
    NX, NY = np.meshgrid(c, c)
    nodes = np.stack([NX.ravel(), NY.ravel(), np.full(NX.size, z0 + k_shift)], axis=1).astype(np.float32)
    depth = np.full((height, width), z0, dtype=np.float32)
    return {
        "name": "plane",
        "camera": (width, height, f, f, cx, cy),
        "points": pts, "normals": nrm, "nodes": nodes,
        "R": np.eye(3, dtype=np.float32), "T": np.zeros(3, dtype=np.float32),
        "depth": depth, "sigma": float(spacing), "node_spacing": float(spacing),
    }
