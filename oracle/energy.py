"""Energy terms of Eq.(3) that lie on the hot path: E_rot (Eqs.(4)-(5)), E_reg (Eq.(6)), E_data (Eq.(8)).

Reading of Eq.(3) with the paper's weights (Sec. III-B): E = w_rot E_rot +
w_reg E_reg + w_data E_data with w_rot = 1000, w_reg = 10000, w_data = 1; the
correspondence and pose terms are off this path (the pose is an input).
Test infrastructure only (see the package header).
"""
import numpy as np

from .warp import split


def rot_residuals(params):
    """Eq.(5): per node (c1.c2, c1.c3, c2.c3, c1.c1 - 1, c2.c2 - 1, c3.c3 - 1); Rot(A) is their square sum."""
    p = np.asarray(params, dtype=np.float64)
    c1, c2, c3 = p[:, 0:3], p[:, 3:6], p[:, 6:9]
    dot = lambda a, b: np.sum(a * b, axis=1)  # noqa: E731
    return np.stack([dot(c1, c2), dot(c1, c3), dot(c2, c3),
                     dot(c1, c1) - 1.0, dot(c2, c2) - 1.0, dot(c3, c3) - 1.0], axis=1)


def edges(nbrs):
    """Directed edges (j, l) for l in N(j); both directions appear (Eq.(6) sums over j and N(j))."""
    js = np.concatenate([np.full(len(n), j, dtype=np.int64) for j, n in enumerate(nbrs)]) if nbrs else np.zeros(0, np.int64)
    ls = np.concatenate([np.asarray(n, dtype=np.int64) for n in nbrs]) if nbrs else np.zeros(0, np.int64)
    return js, ls


def reg_residuals(params, nodes, nbrs):
    """Eq.(6) residual per directed edge: A_j (g_l - g_j) + g_j + t_j - (g_l + t_l), alpha_jl = 1."""
    A, t = split(params)
    G = np.asarray(nodes, dtype=np.float64)
    js, ls = edges(nbrs)
    e = G[ls] - G[js]
    return np.einsum("nac,nc->na", A[js], e) + G[js] + t[js] - G[ls] - t[ls], js, ls


def energies(params, nodes, nbrs, r_data):
    """Unweighted E_data, E_rot, E_reg (each a plain sum of squares)."""
    e_rot = float(np.sum(rot_residuals(params) ** 2))
    rr, _, _ = reg_residuals(params, nodes, nbrs)
    e_reg = float(np.sum(rr ** 2))
    e_data = float(np.sum(np.asarray(r_data, dtype=np.float64) ** 2))
    return e_data, e_rot, e_reg
