"""Projective association with the depth map and the visibility gates (Eqs.(7)-(8)).

Test infrastructure only (see the package header).
"""
import numpy as np


def project(vc, camera):
    """P of Eq.(8): pinhole projection to the nearest pixel.

    Reading: q = x / z, u_f = q * fx + cx, u = floor(u_f + 0.5) (likewise v); no
    interpolation.  Returns (u, v, u_f, v_f, inside) with inside = z > 0 and the
    pixel in the image.
    """
    W, H, fx, fy, cx, cy = camera
    fx, fy, cx, cy = (float(np.float32(a)) for a in (fx, fy, cx, cy))
    vc = np.asarray(vc, dtype=np.float64)
    z = vc[:, 2]
    pos = z > 0
    zs = np.where(pos, z, 1.0)
    uf = (vc[:, 0] / zs) * fx + cx
    vf = (vc[:, 1] / zs) * fy + cy
    uu = np.floor(uf + 0.5)
    vv = np.floor(vf + 0.5)
    inside = pos & (uu >= 0) & (uu < W) & (vv >= 0) & (vv < H)
    ui = np.where(inside, uu, 0).astype(np.int64)
    vi = np.where(inside, vv, 0).astype(np.int64)
    return ui, vi, uf, vf, inside


def associate(vc, nc, depth, camera, Nmap, Nvalid, eps_d, cos_eps_n):
    """Correspondences, gates and point-to-plane residuals for warped points in camera frame.

    Eq.(7) is garbled; readings: the gates apply to the warped point ("predicted
    visible points", Eq.(8)); distance gate |v~ - Gamma(P(v~))| < eps_d (Euclidean,
    strict); normal gate: the angle between the warped normal and the depth
    normal is below eps_n, i.e. n~ . N > cos(eps_n), strict.
    Residual (Eq.(8)): r = N(p)^T (v~ - Gamma(P(v~))), Gamma = lift of the pixel
    centre with its depth.

    Returns dict: corr (N,) int64 pixel index v*W+u or -1, r (N,), V (N, 3) the
    matched lifted pixel, Np (N, 3) its normal, plus the decision margins
    (distance of u_f, v_f from a rounding boundary, and slack of both gates)
    used to account for float32/float64 decision differences.
    """
    W, H, fx, fy, cx, cy = camera
    fx64, fy64, cx64, cy64 = (float(np.float32(a)) for a in (fx, fy, cx, cy))
    vc = np.asarray(vc, dtype=np.float64)
    nc = np.asarray(nc, dtype=np.float64)
    D = np.asarray(depth, dtype=np.float64)
    Nm = np.asarray(Nmap, dtype=np.float64)
    ui, vi, uf, vf, inside = project(vc, camera)
    d = D[vi, ui]
    nv = Nvalid[vi, ui]
    ok = inside & (d > 0) & nv
    V = np.stack([d * ((ui - cx64) / fx64), d * ((vi - cy64) / fy64), d], axis=1)
    Np = Nm[vi, ui]
    dx = vc[:, 0] - V[:, 0]
    dy = vc[:, 1] - V[:, 1]
    dz = vc[:, 2] - V[:, 2]
    dist = np.sqrt((dx * dx + dy * dy) + dz * dz)
    ndot = (nc[:, 0] * Np[:, 0] + nc[:, 1] * Np[:, 1]) + nc[:, 2] * Np[:, 2]
    ok &= (dist < eps_d) & (ndot > cos_eps_n)
    r = (Np[:, 0] * dx + Np[:, 1] * dy) + Np[:, 2] * dz
    corr = np.where(ok, vi * W + ui, -1)
    # margins: how close each decision was to flipping
    frac_u = np.abs((uf + 0.5) - np.round(uf + 0.5))
    frac_v = np.abs((vf + 0.5) - np.round(vf + 0.5))
    margin = np.minimum.reduce([frac_u, frac_v, np.abs(dist - eps_d), np.abs(ndot - cos_eps_n)])
    return {"corr": corr, "valid": ok, "r": np.where(ok, r, 0.0), "V": V, "Np": Np,
            "margin": margin, "dist": dist, "ndot": ndot}
