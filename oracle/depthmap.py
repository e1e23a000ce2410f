"""Per-frame depth preprocessing: vertex map and normal map of the depth image (Eq.(8)).

Eq.(8) needs, for a pixel u, the back-projected point Gamma and the depth
image's normal at u; the paper gives no formula for either.  Readings:
  V(u, v) = D(u, v) * ((u - cx) / fx, (v - cy) / fy, 1)      (pixel centre, no interpolation)
  N(u, v) = normalize(b x a), a = V(u+1, v) - V(u-1, v), b = V(u, v+1) - V(u, v-1)
N faces the camera (N_z < 0 for a fronto-parallel plane).  N is invalid on the
image border, where the pixel or any of its four neighbours has no depth, or
where b x a vanishes.
Test infrastructure only (see the package header).
"""
import numpy as np


def vertex_map(depth, camera):
    W, H, fx, fy, cx, cy = camera
    D = np.asarray(depth, dtype=np.float64)
    u, v = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    fx, fy, cx, cy = (float(np.float32(a)) for a in (fx, fy, cx, cy))
    return np.stack([D * ((u - cx) / fx), D * ((v - cy) / fy), D], axis=-1)


def normal_map(depth, camera):
    """Returns (N (H, W, 3), valid (H, W) bool); invalid normals are zero."""
    W, H = camera[0], camera[1]
    D = np.asarray(depth, dtype=np.float64)
    V = vertex_map(D, camera)
    N = np.zeros((H, W, 3))
    valid = np.zeros((H, W), dtype=bool)
    if W < 3 or H < 3:
        return N, valid
    a = V[1:-1, 2:] - V[1:-1, :-2]
    b = V[2:, 1:-1] - V[:-2, 1:-1]
    cr = np.stack([b[..., 1] * a[..., 2] - b[..., 2] * a[..., 1],
                   b[..., 2] * a[..., 0] - b[..., 0] * a[..., 2],
                   b[..., 0] * a[..., 1] - b[..., 1] * a[..., 0]], axis=-1)
    nn = np.sqrt((cr[..., 0] * cr[..., 0] + cr[..., 1] * cr[..., 1]) + cr[..., 2] * cr[..., 2])
    ok = ((D[1:-1, 1:-1] > 0) & (D[1:-1, 2:] > 0) & (D[1:-1, :-2] > 0)
          & (D[2:, 1:-1] > 0) & (D[:-2, 1:-1] > 0) & (nn > 0))
    inner = np.where(ok[..., None], cr / np.where(nn > 0, nn, 1.0)[..., None], 0.0)
    N[1:-1, 1:-1] = inner
    valid[1:-1, 1:-1] = ok
    return N, valid
