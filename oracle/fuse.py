"""Model update: deform the model, register it point-to-pixel and fuse the new depth (Sec. II-G).

Follows Alg. 2 steps 1-3 with Alg. 1 as the registration test and
Eqs.(12), (14), (15) as the update.  Readings where the paper is silent or
inconsistent:
  * Reg map (Alg. 2 step 2): each pixel keeps the projecting point nearest to
    the camera; equal depths go to the lower point index.
  * Alg. 1 gate: depth present, |z~ - D(p)| < tau and the angle between the
    warped normal and the depth normal below delta, i.e. n~ . N > cos(delta);
    tau = 10 mm, delta = 10 degrees (Sec. III-B).  Eq.(11)'s weight is read as
    this 0/1 gate (its stated growth with distance contradicts the text).
  * Eq.(12) averages depth along the ray; the fused point is taken as the
    weighted mean of positions, p <- (w p~ + Gamma_w(p)) / (w + 1) in world
    coordinates, whose camera-z component is Eq.(12) when p~ lies on the ray.
    Eq.(14) likewise for the normal, renormalised; Eq.(15) w <- min(w + 1, w_max)
    with w_max = 20 (Sec. III-B; the 10 in Sec. II-G conflicts).
  * Registered points are stamped with the frame index.  Every point moves to
    its warped position; every node moves by its own translation, g_j + t_j.
  * Eq.(13) (colour): a registered point's colour becomes the same weighted
    mean of its colour and the frame's colour at the matched pixel,
    c <- (w c + I(p)) / (w + 1), per channel, with the weight before the
    Eq.(15) update; colours are view-independent (no rotation).
Test infrastructure only (see the package header).
"""
import numpy as np

from .assoc import project
from .depthmap import vertex_map
from .warp import ed_warp, split, warp_normals


def zbuffer(vc, inside, ui, vi, W, H):
    """Winner point index per pixel (-1 = none): smallest camera z, then lowest index.

    Reading: depths are compared at float32 resolution (the precision the
    model is stored in); equal float32 depths go to the lower point index.
    """
    win = np.full(W * H, -1, dtype=np.int64)
    pts = np.nonzero(inside)[0]
    if len(pts) == 0:
        return win
    pix = vi[pts] * W + ui[pts]
    z32 = np.asarray(vc[pts, 2], dtype=np.float32)
    order = np.lexsort((pts, z32, pix))            # by pixel, then z, then index
    pix_s = pix[order]
    first = np.ones(len(order), dtype=bool)
    first[1:] = pix_s[1:] != pix_s[:-1]
    win[pix_s[first]] = pts[order[first]]
    return win


def fuse_warped(vw, nw, vc, nc, weight, stamp, depth, camera, R, T, Nmap, Nvalid, frame,
                tau=10.0, cos_delta=float(np.cos(np.deg2rad(10.0))), w_max=20.0, color=None, image=None):
    """Alg. 1-2 steps 2-3 and Eqs.(12)-(15) for an already warped model.

    vw, nw: warped points and unit normals in world coordinates; vc, nc: the same
    in the camera frame.  color (N, 3) and image (H, W, 3), if given, take part
    in Eq.(13).  Returns dict(points, normals, weight, stamp, registered (N,)
    bool, reg (H*W,) winner per pixel[, color]).
    """
    W, H = camera[0], camera[1]
    Rm = np.asarray(R, dtype=np.float64)
    Tv = np.asarray(T, dtype=np.float64)
    vw = np.asarray(vw, dtype=np.float64)
    nw = np.asarray(nw, dtype=np.float64)
    vc = np.asarray(vc, dtype=np.float64)
    nc = np.asarray(nc, dtype=np.float64)
    ui, vi, _, _, inside = project(vc, camera)
    win = zbuffer(vc, inside, ui, vi, W, H)
    n = vw.shape[0]
    is_winner = np.zeros(n, dtype=bool)
    is_winner[win[win >= 0]] = True
    D = np.asarray(depth, dtype=np.float64)
    d = D[vi, ui]
    Np = np.asarray(Nmap, dtype=np.float64)[vi, ui]
    ndot = (nc[:, 0] * Np[:, 0] + nc[:, 1] * Np[:, 1]) + nc[:, 2] * Np[:, 2]
    reg = is_winner & (d > 0) & Nvalid[vi, ui] & (np.abs(vc[:, 2] - d) < tau) & (ndot > cos_delta)
    Vm = vertex_map(D, camera)[vi, ui]
    gam_w = (Vm - Tv) @ Rm                                   # R^T (V - T)
    nobs_w = Np @ Rm                                         # R^T N
    om = np.asarray(weight, dtype=np.float64)
    p_new = np.where(reg[:, None], (om[:, None] * vw + gam_w) / (om[:, None] + 1.0), vw)
    nn = np.where(reg[:, None], (om[:, None] * nw + nobs_w) / (om[:, None] + 1.0), nw)
    nn = nn / np.linalg.norm(nn, axis=1, keepdims=True)
    om_new = np.where(reg, np.minimum(om + 1.0, w_max), om)
    st_new = np.where(reg, frame, np.asarray(stamp))
    out = {"points": p_new, "normals": nn, "weight": om_new, "stamp": st_new, "registered": reg, "reg": win}
    if color is not None:
        c = np.asarray(color, dtype=np.float64)
        Ip = np.asarray(image, dtype=np.float64)[vi, ui]
        out["color"] = np.where(reg[:, None], (om[:, None] * c + Ip) / (om[:, None] + 1.0), c)
    return out


def fuse(points, normals, weight, stamp, nodes, params, idx, w, depth, camera, R, T, Nmap, Nvalid,
         frame, tau=10.0, cos_delta=float(np.cos(np.deg2rad(10.0))), w_max=20.0, color=None, image=None):
    """Deform the model with the frame's final parameters, then fuse (see fuse_warped).

    Also returns the moved nodes g_j + t_j.
    """
    Rm = np.asarray(R, dtype=np.float64)
    Tv = np.asarray(T, dtype=np.float64)
    vw = ed_warp(points, nodes, params, idx, w)             # world
    nw = warp_normals(normals, params, idx, w)
    out = fuse_warped(vw, nw, vw @ Rm.T + Tv, nw @ Rm.T, weight, stamp, depth, camera, R, T, Nmap, Nvalid, frame,
                      tau, cos_delta, w_max, color, image)
    _, t = split(params)
    out["nodes"] = np.asarray(nodes, dtype=np.float64) + t
    return out
