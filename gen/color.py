"""Seeded synthetic colour inputs for the Eq.(13) colour fusion.

Manufactures inputs only: a smooth RGB image of the frame (values in [0, 1],
float32, H x W x 3) and random per-point colours.  No step of the method is
computed here.
"""
import numpy as np


def color_image(height, width, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    ph = rng.uniform(0.0, 2.0 * np.pi, size=3)
    fr = rng.uniform(0.03, 0.15, size=(3, 2))
    v, u = np.mgrid[0:height, 0:width].astype(np.float64)
    chans = [0.5 + 0.4 * np.sin(fr[c, 0] * u + fr[c, 1] * v + ph[c]) for c in range(3)]
    return np.stack(chans, axis=-1).astype(np.float32)


def point_colors(n, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, 1.0, size=(n, 3)).astype(np.float32)
