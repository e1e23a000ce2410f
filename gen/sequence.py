"""Seeded synthetic frame sequence: a scope sweeping over a breathing tissue sheet.

Manufactures inputs only (no registration arithmetic).  A 250 x 200 mm sheet,
z = 60 + 3 sin(x/8) cos(y/10) plus eight Gaussian bumps, breathes along its
normal with amplitude 3 mm and a period of 120 frames (respiration, Sec. III);
the camera (640x480, fx = fy = 256) looks down from about 60 mm above it on a
Lissajous sweep x = 55 sin(2 pi f / 300), y = 45 sin(4 pi f / 300) mm with a
wobble of at most 5 degrees, so new tissue enters the view frame by frame.
Each frame's depth is ray-cast to 1e-9 px through the deformed sheet with
Gaussian noise of 0.2 * 60 / fx mm.  The pose of every frame is given (the
paper's front end supplies it).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .scene import Surface, render_depth


@dataclasses.dataclass(frozen=True)
class _Cam:
    width: int = 640
    height: int = 480
    fx: float = 256.0
    fy: float = 256.0
    cx: float = 320.0
    cy: float = 240.0
    patch: tuple = (-125.0, 125.0, -100.0, 100.0)


class _SheetBreathing:
    """Displacement along the sheet normal: a(f) * b(x, y), a(f) = 3 sin(2 pi f / 120) mm."""

    def __init__(self, surface, patch, frame, period=120.0, amp=3.0):
        self.surface = surface
        self.patch = patch
        self.a = amp * math.sin(2.0 * math.pi * frame / period)

    def __call__(self, X):
        X = np.asarray(X, dtype=np.float64)
        x, y = X[..., 0], X[..., 1]
        x0, x1, y0, y1 = self.patch
        b = np.sin(np.pi * (x - x0) / (x1 - x0)) * np.sin(np.pi * (y - y0) / (y1 - y0))
        return X + (self.a * b)[..., None] * self.surface.normal(x, y)


def _rot(axis, deg):
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    ang = math.radians(deg)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1.0 - math.cos(ang)) * (K @ K)


class Sequence:
    """Frames of the sweep; frame(f) returns dict(camera, R, T, depth) (float32)."""

    def __init__(self, seed=5, n_frames=300, noise=True):
        self.rng = np.random.Generator(np.random.PCG64(seed))
        self.cam = _Cam()
        x0, x1, y0, y1 = self.cam.patch
        nb = 8
        bumps = np.stack([self.rng.uniform(x0, x1, nb), self.rng.uniform(y0, y1, nb),
                          self.rng.uniform(1.0, 4.0, nb), self.rng.uniform(4.0, 10.0, nb)], axis=1)
        self.surface = Surface(bumps)
        self.n_frames = n_frames
        self.noise = noise
        self.wobble_axes = self.rng.normal(size=(n_frames, 3))
        self.wobble_deg = self.rng.uniform(0.0, 5.0, n_frames)

    def pose(self, f):
        """camera = R world + T for a camera at (x_f, y_f, 0) looking along +z, wobbled."""
        c = np.array([55.0 * math.sin(2 * math.pi * f / 300.0), 45.0 * math.sin(4 * math.pi * f / 300.0), 0.0])
        R = _rot(self.wobble_axes[f % self.n_frames], self.wobble_deg[f % self.n_frames])
        T = -R @ c
        return R.astype(np.float32), T.astype(np.float32)

    def frame(self, f):
        R, T = self.pose(f)
        field = _SheetBreathing(self.surface, self.cam.patch, f)
        sig = 0.2 * 60.0 / self.cam.fx if self.noise else 0.0
        rng = np.random.Generator(np.random.PCG64(100003 * (f + 1)))
        depth = render_depth(self.cam, self.surface, field, R.astype(np.float64), T.astype(np.float64), rng, sig)
        c = self.cam
        return {"camera": (c.width, c.height, c.fx, c.fy, c.cx, c.cy), "R": R, "T": T,
                "depth": depth.astype(np.float32), "frame": f}
