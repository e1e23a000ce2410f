"""Joint rigid pose + ED registration: the global-pose terms of Eq.(3) (E_r, E_p
of Eq.(10)) and their 6 unknowns (Sec. II-E, II-F: "6 more variables").

Readings:
- Pose: camera = R world + T.  The scope position P of Eq.(10) is the camera
  centre C = -R^T T; the front end's pose (R0, T0) is both the prior and the
  start.
- E_r = |rho_r|^2 with rho_r = log(R R0^T), the rotation vector of the change
  of orientation (Euler-angle changes to first order); E_p = |C - C0|^2.  Like
  the other terms of Eq.(3) they enter as sums of squares, with w_r = 1e6,
  w_p = 1e3 (Sec. III-B).
- Perturbation xi = (dw, dt) of the pose: R <- exp([dw]x) R,
  T <- exp([dw]x) T + dt (a rigid motion applied in camera coordinates), so a
  warped point moves by d v~ = -[v~]x dw + dt.  Hence
    data row:      d r / d xi = (v~ x N, N)   (N the matched depth normal)
    key-point row: d r / d xi = [-[v~]x, I]
    E_r:           d rho_r / d dw = I: exact for the gradient, because the
                   inverse left Jacobian J of SO(3) satisfies J^T rho = rho;
                   the Gauss-Newton matrix takes I for J^T J
    E_p:           d C / d dt = -R^T, d C / d dw = 0 (first order).
- Joint normal equations [[H_ee, B], [B^T, H_pp]] (dx, dxi) = -(g_e, g_p),
  B = sum over terms of w J_e^T J_xi (12 per node x 6), solved by the
  textbook PCG of the fixed-damping form over the joint vector: lambda on the
  whole diagonal, block-Jacobi preconditioner extended by the damped 6x6 pose
  block.  Then x += dx and the pose takes the step xi.
Test infrastructure only (see the package header).
"""
import dataclasses

import numpy as np

from .depthmap import normal_map
from .gn import evaluate, linearize
from .graph import build_graph
from .pcg import block_jacobi, bsr_matvec
from .warp import identity_params


def skew(v):
    v = np.asarray(v, dtype=np.float64)
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def so3_exp(w):
    """Rotation matrix of the rotation vector w (Rodrigues)."""
    w = np.asarray(w, dtype=np.float64)
    th = float(np.linalg.norm(w))
    K = skew(w)
    if th < 1e-12:
        return np.eye(3) + K + 0.5 * K @ K
    return np.eye(3) + np.sin(th) / th * K + (1.0 - np.cos(th)) / (th * th) * K @ K


def so3_log(R):
    """Rotation vector of R (angle in [0, pi))."""
    R = np.asarray(R, dtype=np.float64)
    c = np.clip((np.trace(R) - 1.0) / 2.0, -1.0, 1.0)
    th = float(np.arccos(c))
    v = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    if th < 1e-8:
        return 0.5 * v
    return th / (2.0 * np.sin(th)) * v


def centre(R, T):
    return -np.asarray(R, dtype=np.float64).T @ np.asarray(T, dtype=np.float64)


def pose_residuals(R, T, R0, T0):
    """(rho_r, rho_p): log(R R0^T) and C - C0."""
    R = np.asarray(R, dtype=np.float64)
    return so3_log(R @ np.asarray(R0, dtype=np.float64).T), centre(R, T) - centre(R0, T0)


def pose_step(R, T, xi):
    """The pose after the step xi = (dw, dt)."""
    E = so3_exp(xi[:3])
    return E @ np.asarray(R, dtype=np.float64), E @ np.asarray(T, dtype=np.float64) + np.asarray(xi[3:])


def data_pose_rows(vc, Np):
    """(N, 6) pose columns of the data rows: (v~ x N, N)."""
    vc = np.asarray(vc, dtype=np.float64)
    Np = np.asarray(Np, dtype=np.float64)
    return np.concatenate([np.cross(vc, Np), Np], axis=1)


def corr_pose_rows(vk):
    """(S, 3, 6) pose columns of the key-point rows: [-[v~]x, I]."""
    vk = np.asarray(vk, dtype=np.float64)
    J = np.zeros((len(vk), 3, 6))
    for s, v in enumerate(vk):
        J[s, :, :3] = -skew(v)
        J[s, :, 3:] = np.eye(3)
    return J


def pose_border(pb, graph, x, R, asc, vc, kp_vc=None):
    """Pose parts of the joint system at a linearisation point: B (m, 12, 6), H_pp (6, 6) and g_p (6) of the
    data and key-point terms (the priors are added by joint_linearize)."""
    P = np.asarray(pb.points, dtype=np.float64)
    G = np.asarray(pb.nodes, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    m = len(G)
    idx, w = graph["idx"], graph["w"]
    k = idx.shape[1]
    B = np.zeros((m, 12, 6))
    Hpp = np.zeros((6, 6))
    gp = np.zeros(6)
    ok = np.asarray(asc["valid"])
    Jp = data_pose_rows(vc, asc["Np"])
    nprime = np.asarray(asc["Np"], dtype=np.float64) @ R      # rows (R^T N)^T
    r = np.asarray(asc["r"], dtype=np.float64)
    wd = pb.w_data
    iv = np.nonzero(ok)[0]
    Hpp += wd * Jp[iv].T @ Jp[iv]
    gp += wd * Jp[iv].T @ r[iv]
    for s in range(k):
        j = idx[iv, s]
        dh = np.concatenate([P[iv] - G[j], np.ones((len(iv), 1))], axis=1)
        Je = w[iv, s][:, None] * (dh[:, :, None] * nprime[iv][:, None, :]).reshape(len(iv), 12)   # index 3c + a
        np.add.at(B, j, wd * Je[:, :, None] * Jp[iv][:, None, :])
    if pb.kp_point is not None and len(pb.kp_point):
        r3 = asc["kp_r"]
        J3 = corr_pose_rows(kp_vc)
        for s, p in enumerate(np.asarray(pb.kp_point, dtype=np.int64)):
            if p < 0 or p >= len(P):
                continue
            Hpp += pb.w_corr * J3[s].T @ J3[s]
            gp += pb.w_corr * J3[s].T @ r3[s]
            for q in range(k):
                j = idx[p, q]
                dh = np.append(P[p] - G[j], 1.0)
                Je = np.zeros((3, 12))                          # d r3 / d x_j[3c + a] = w d_c R[:, a]
                for c in range(4):
                    Je[:, 3 * c:3 * c + 3] = w[p, q] * dh[c] * R
                B[j] += pb.w_corr * Je.T @ J3[s]
    return B, Hpp, gp


def joint_linearize(pb, graph, x, R, T, R0, T0, w_r, w_p, Nmap, Nvalid, corr_override=None):
    """Everything one joint step needs at (x, R, T)."""
    pbi = dataclasses.replace(pb, R=np.asarray(R), T=np.asarray(T))
    vc, nc, asc, blocks, g, e = linearize(pbi, graph, x, Nmap, Nvalid, corr_override)
    kp_vc = None
    if pb.kp_point is not None and len(pb.kp_point):
        kp_vc = asc["kp_r"] + np.asarray(pb.kp_target, dtype=np.float64)
    B, Hpp, gp = pose_border(pbi, graph, x, R, asc, vc, kp_vc)
    rho_r, rho_p = pose_residuals(R, T, R0, T0)
    Hpp[:3, :3] += w_r * np.eye(3)
    Hpp[3:, 3:] += w_p * np.asarray(R) @ np.asarray(R).T
    gp[:3] += w_r * rho_r
    gp[3:] += w_p * (-np.asarray(R) @ rho_p)
    e_pose = (float(rho_r @ rho_r), float(rho_p @ rho_p))
    return vc, asc, blocks, g, B, Hpp, gp, e, e_pose


def joint_pcg(row_ptr, col_idx, blocks, B, Hpp, g_e, g_p, lam, iters):
    """Textbook block-Jacobi PCG over the joint vector (12 m + 6) from 0, exactly `iters` iterations (early stop
    as the ED-only solve).  Returns (dx (12 m), dxi (6), info)."""
    m = len(row_ptr) - 1
    Me, _ = block_jacobi(row_ptr, col_idx, blocks, lam)
    Mp = np.linalg.inv(Hpp + lam * np.eye(6))
    Bf = B.reshape(m * 12, 6)

    def A(v):
        ve, vp = v[:12 * m], v[12 * m:]
        ye = bsr_matvec(row_ptr, col_idx, blocks, ve, lam) + Bf @ vp
        yp = Bf.T @ ve + (Hpp + lam * np.eye(6)) @ vp
        return np.concatenate([ye, yp])

    def M(v):
        ve = np.einsum("mef,mf->me", Me, v[:12 * m].reshape(m, 12)).reshape(-1)
        return np.concatenate([ve, Mp @ v[12 * m:]])

    x = np.zeros(12 * m + 6)
    r = -np.concatenate([np.asarray(g_e, dtype=np.float64).reshape(-1), g_p])
    z = M(r)
    p = z.copy()
    rz = float(r @ z)
    resid = [float(np.linalg.norm(r))]
    done = 0
    breakdown = False
    for _ in range(iters):
        if rz == 0.0:
            break
        q = A(p)
        pq = float(p @ q)
        if not pq > 0.0:
            breakdown = True
            break
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        z = M(r)
        rz_new = float(r @ z)
        resid.append(float(np.linalg.norm(r)))
        done += 1
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x[:12 * m], x[12 * m:], {"resid": resid, "iters": done, "breakdown": breakdown}


def joint_register(pb, graph=None, w_r=1e6, w_p=1e3, corr_sequence=None, x0=None):
    """pb.gn_iters joint steps from (x0 or identity, pb.R, pb.T), prior (pb.R, pb.T).
    Returns (x, R, T, report); report["iters"][it] has the energies at the step's point (e_r, e_p included)."""
    if graph is None:
        graph = build_graph(pb.points, pb.nodes, pb.k, pb.weight_kind, pb.sigma)
    m = np.asarray(pb.nodes).shape[0]
    x = identity_params(m) if x0 is None else np.array(x0, dtype=np.float64)
    R0 = np.asarray(pb.R, dtype=np.float64)
    T0 = np.asarray(pb.T, dtype=np.float64)
    R, T = R0.copy(), T0.copy()
    Nmap, Nvalid = normal_map(pb.depth, pb.camera)
    rep = {"iters": [], "graph": graph}
    for it in range(pb.gn_iters):
        co = None if corr_sequence is None else corr_sequence[it]
        vc, asc, blocks, g, B, Hpp, gp, e, ep = joint_linearize(pb, graph, x, R, T, R0, T0, w_r, w_p, Nmap, Nvalid,
                                                                co)
        dx, dxi, info = joint_pcg(graph["row_ptr"], graph["col_idx"], blocks, B, Hpp, g, gp, pb.lam, pb.pcg_iters)
        rep["iters"].append({"e_data": e[0], "e_rot": e[1], "e_reg": e[2], "e_corr": e[3], "e_r": ep[0],
                             "e_p": ep[1], "n_valid": int(asc["valid"].sum()), "resid": info["resid"],
                             "dxi": dxi})
        x = x + dx.reshape(m, 12)
        R, T = pose_step(R, T, dxi)
    pbf = dataclasses.replace(pb, R=R, T=T)
    _, _, asc, e = evaluate(pbf, graph, x, Nmap, Nvalid)
    rho_r, rho_p = pose_residuals(R, T, R0, T0)
    rep["final"] = {"e_data": e[0], "e_rot": e[1], "e_reg": e[2], "e_corr": e[3], "e_r": float(rho_r @ rho_r),
                    "e_p": float(rho_p @ rho_p), "n_valid": int(asc["valid"].sum()), "corr": asc["corr"]}
    return x, R, T, rep
