"""Gradients of the registration energy with correspondences and kNN sets held fixed.

The paper has no gradient; these are the derivatives of Eq.(3) restricted to
the hot-path terms, with the correspondence of every point and its k nodes
frozen (the skinning weights still move with the point for d/dv):
  dE/dx = 2 sum_terms w J^T r                       (= 2 g of the normal equations)
  dE/dv_i = 2 w_data r_i n'^T sum_j [w_ij A_j + (A_j d_ij + g_j + t_j) grad_v w_ij^T]
with n' = R^T N_p, d_ij = v_i - g_j and, for normalised Gaussian weights,
  grad_v w_ij = w_ij (-(v - g_j) + sum_l w_il (v - g_l)) / sigma^2.
Test infrastructure only (see the package header).
"""
import numpy as np

from .energy import reg_residuals, rot_residuals
from .system import data_jacobian_rows, reg_jacobian, rot_jacobian
from .warp import ed_warp, split


def data_residuals_fixed(points, nodes, params, idx, sigma, R, T, V, Np, valid):
    """Eq.(8) residuals with frozen correspondences (V, Np per point) and kNN sets;
    Gaussian weights are recomputed from the given points."""
    P = np.asarray(points, dtype=np.float64)
    G = np.asarray(nodes, dtype=np.float64)
    idx = np.asarray(idx)
    d = P[:, None, :] - G[idx]
    d2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    e = np.exp(-d2 / (2.0 * sigma * sigma))
    w = e / e.sum(axis=1, keepdims=True)
    vc = ed_warp(P, G, params, idx, w, R, T)
    diff = vc - V
    r = (Np[:, 0] * diff[:, 0] + Np[:, 1] * diff[:, 1]) + Np[:, 2] * diff[:, 2]
    return np.where(valid, r, 0.0)


def total_energy_fixed(params, points, nodes, nbrs, idx, sigma, R, T, V, Np, valid, weights):
    """w_rot E_rot + w_reg E_reg + w_data E_data at frozen correspondences (Gaussian weights)."""
    w_rot, w_reg, w_data = weights
    r = data_residuals_fixed(points, nodes, params, idx, sigma, R, T, V, Np, valid)
    rg, _, _ = reg_residuals(params, nodes, nbrs)
    return (w_data * float(np.sum(r * r)) + w_rot * float(np.sum(rot_residuals(params) ** 2))
            + w_reg * float(np.sum(rg * rg)))


def energy_grad_params(params, points, nodes, nbrs, idx, w, R, r, Np, valid, weights):
    """dE/dx (m, 12) assembled term by term from the Jacobians."""
    w_rot, w_reg, w_data = weights
    m = np.asarray(nodes).shape[0]
    idx = np.asarray(idx)
    out = np.zeros((m, 12))
    sel = np.nonzero(valid)[0]
    Jd = data_jacobian_rows(np.asarray(points)[sel], nodes, idx[sel], np.asarray(w)[sel], R, Np[sel])
    for s in range(idx.shape[1]):
        np.add.at(out, idx[sel, s], 2.0 * w_data * Jd[:, s, :] * r[sel, None])
    out += 2.0 * w_rot * np.einsum("mqe,mq->me", rot_jacobian(params), rot_residuals(params))
    js, ls, Jj, Jl = reg_jacobian(nodes, nbrs)
    rg, _, _ = reg_residuals(params, nodes, nbrs)
    np.add.at(out, js, 2.0 * w_reg * np.einsum("nqe,nq->ne", Jj, rg))
    np.add.at(out, ls, 2.0 * w_reg * np.einsum("nqe,nq->ne", Jl, rg))
    return out


def energy_grad_points(params, points, nodes, idx, sigma, R, r, Np, valid, w_data):
    """dE/dv (N, 3) for normalised Gaussian skinning weights."""
    P = np.asarray(points, dtype=np.float64)
    G = np.asarray(nodes, dtype=np.float64)
    idx = np.asarray(idx)
    A, t = split(params)
    d = P[:, None, :] - G[idx]                                  # (N, k, 3)
    d2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    e = np.exp(-d2 / (2.0 * sigma * sigma))
    w = e / e.sum(axis=1, keepdims=True)
    mean_d = np.einsum("nk,nkc->nc", w, d)
    gw = w[..., None] * (-d + mean_d[:, None, :]) / (sigma * sigma)   # (N, k, 3)
    Aj = A[idx]                                                 # (N, k, 3, 3)
    yj = np.einsum("nkac,nkc->nka", Aj, d) + G[idx] + t[idx]    # (N, k, 3)
    dv = np.einsum("nk,nkac->nac", w, Aj) + np.einsum("nka,nkc->nac", yj, gw)   # d warp / d v (world)
    nprime = np.asarray(Np, dtype=np.float64) @ np.asarray(R, dtype=np.float64)
    row = np.einsum("na,nac->nc", nprime, dv)
    return np.where(valid[:, None], 2.0 * w_data * np.asarray(r)[:, None] * row, 0.0)
