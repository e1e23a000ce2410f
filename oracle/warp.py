"""Embedded-deformation warp of points and normals (Eq.(1), Sec. II-D).

Test infrastructure only (see the package header).
"""
import numpy as np


def identity_params(m):
    """A_j = I, t_j = 0 for every node: the state each frame starts from."""
    x = np.zeros((m, 12))
    x[:, 0] = x[:, 4] = x[:, 8] = 1.0
    return x


def split(params):
    """params (m, 12) -> A (m, 3, 3) with A[:, :, c] = c-th column, t (m, 3)."""
    p = np.asarray(params, dtype=np.float64)
    A = np.stack([p[:, 0:3], p[:, 3:6], p[:, 6:9]], axis=2)
    return A, p[:, 9:12].copy()


def ed_warp(points, nodes, params, idx, w, R=None, T=None):
    """Eq.(1): v~ = R sum_j w_j [A_j (v - g_j) + g_j + t_j] + T over the k nodes of v.

    Reading: R, T are the one rigid scope pose of the frame (camera = R x + T),
    applied after blending; with R = None the result stays in world coordinates.
    """
    P = np.asarray(points, dtype=np.float64)
    G = np.asarray(nodes, dtype=np.float64)
    A, t = split(params)
    idx = np.asarray(idx)
    w = np.asarray(w, dtype=np.float64)
    out = np.zeros_like(P)
    for s in range(idx.shape[1]):
        j = idx[:, s]
        d = P - G[j]
        out += w[:, s:s + 1] * (np.einsum("nac,nc->na", A[j], d) + G[j] + t[j])
    if R is not None:
        out = out @ np.asarray(R, dtype=np.float64).T + np.asarray(T, dtype=np.float64)
    return out


def warp_normals(normals, params, idx, w, R=None):
    """Warped unit normals: normalize(R sum_j w_j A_j^{-T} n).

    The paper uses warped normals in its gates and fusion (Eq.(7), Alg. 1,
    Eq.(14)) without giving their formula.  Reading: the inverse transpose, the
    correct map of a normal under an affine transform.
    """
    Nn = np.asarray(normals, dtype=np.float64)
    A, _ = split(params)
    AinvT = np.linalg.inv(A).transpose(0, 2, 1)
    idx = np.asarray(idx)
    w = np.asarray(w, dtype=np.float64)
    out = np.zeros_like(Nn)
    for s in range(idx.shape[1]):
        j = idx[:, s]
        out += w[:, s:s + 1] * np.einsum("nac,nc->na", AinvT[j], Nn)
    if R is not None:
        out = out @ np.asarray(R, dtype=np.float64).T
    return out / np.linalg.norm(out, axis=1, keepdims=True)
