"""Sparse key-point correspondence term E_corr, Eq.(9) (Sec. II-E).

E_corr compares the new (warped) position of each matched key point with its
observed position.  Reading: like every term of the Eq.(3) objective it enters
the least-squares problem as a sum of squares, E_corr = sum_s |V~_s - V_s|^2,
with V~_s the Eq.(1) warp (pose included) of the key point's canonical model
point and V_s its matched 3-D position, both in the camera coordinates of
the frame (the pose R, T maps the warped model there, as for the data term).  A key point is
carried by one model point (index p_s), so it uses that point's k nodes and
skinning weights.  Weight w_corr = 10 (Sec. III-B lists w_corr twice, 10 and
1; the first is taken, the second read as a duplicate).

Per key point the residual has 3 rows (world axes a = 0, 1, 2).  Row a is a
data-term row whose normal is the unit axis e_a: d r_a / d x_j =
w_j kron((v - g_j, 1), R^T e_a), so J_s^T J_s sums to w_j w_l (d_j d_l^T) (x) I.
Test infrastructure only (see the package header).
"""
import numpy as np

from .system import data_jacobian_rows
from .warp import ed_warp


def corr_residuals(points, nodes, params, idx, w, R, T, kp_point, kp_target):
    """(S, 3) residuals V~_s - V_s of the key points (float64, camera coordinates)."""
    kp = np.asarray(kp_point, dtype=np.int64)
    if kp.size == 0:
        return np.zeros((0, 3))
    P = np.asarray(points, dtype=np.float64)[kp]
    vt = ed_warp(P, nodes, params, np.asarray(idx)[kp], np.asarray(w)[kp], R, T)
    return vt - np.asarray(kp_target, dtype=np.float64)


def corr_jacobian_rows(points, nodes, idx, w, R, kp_point):
    """(S, 3, k, 12): row a of key point s, node slot q (columns 3c + a' of node idx[p_s, q])."""
    kp = np.asarray(kp_point, dtype=np.int64)
    S = kp.size
    k = np.asarray(idx).shape[1]
    J = np.zeros((S, 3, k, 12))
    if S == 0:
        return J
    P = np.asarray(points, dtype=np.float64)[kp]
    for a in range(3):
        axis = np.zeros((S, 3))
        axis[:, a] = 1.0
        J[:, a] = data_jacobian_rows(P, nodes, np.asarray(idx)[kp], np.asarray(w)[kp], R, axis)
    return J


def corr_energy(res):
    """Unweighted E_corr = sum of squared residual components."""
    return float(np.sum(np.asarray(res, dtype=np.float64) ** 2))
