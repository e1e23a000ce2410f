"""Seeded synthetic key-point matches for the Eq.(9) correspondence term.

Manufactures inputs only: a key point is carried by one model point (drawn
without replacement), and its matched observation is that point's position
under the scene's known deformation (``gt_points``), mapped by the frame's
pose into the camera coordinates the depth map lives in, plus optional
isotropic Gaussian noise.  This stands in for the ORB/SURF feature matches of
the paper's front end (Sec. II-B), which are not reproduced.
"""
import numpy as np


def keypoints(sc, count, seed=0, noise=0.0):
    """(point index int32 (S,), target float32 (S, 3)) for a scene from ``make_scene``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = len(sc["points"])
    idx = np.sort(rng.choice(n, size=min(count, n), replace=False)).astype(np.int32)
    R = np.asarray(sc["R"], dtype=np.float64)
    T = np.asarray(sc["T"], dtype=np.float64)
    tgt = np.asarray(sc["gt_points"], dtype=np.float64)[idx] @ R.T + T
    if noise > 0:
        tgt = tgt + rng.normal(0.0, noise, tgt.shape)
    return idx, tgt.astype(np.float32)
