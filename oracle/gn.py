"""Per-frame Gauss-Newton registration of the ED graph to a depth map (Sec. II-E, II-F).

Reading of the optimiser (Sec. II-F says Levenberg-Marquardt, no detail): G
damped Gauss-Newton steps from A_j = I, t_j = 0 with the rigid pose fixed.
Each step re-warps the model, re-associates it with the depth map (holding the
correspondences fixed within the step), builds the normal equations and solves
them with exactly P block-Jacobi PCG iterations; x <- x + dx.  The kNN sets and
skinning weights are fixed for the frame because Eq.(2) depends on the
canonical point, not the warped one.
Test infrastructure only (see the package header).
"""
import dataclasses

import numpy as np

from .assoc import associate
from .corr import corr_energy, corr_residuals
from .depthmap import normal_map
from .energy import energies
from .graph import build_graph
from .pcg import block_jacobi, bsr_matvec, pcg
from .system import block_system
from .warp import ed_warp, identity_params, warp_normals


@dataclasses.dataclass
class Problem:
    points: np.ndarray
    normals: np.ndarray
    nodes: np.ndarray
    depth: np.ndarray
    camera: tuple
    R: np.ndarray
    T: np.ndarray
    k: int = 4
    weight_kind: str = "gauss"
    sigma: float = 1.0
    w_rot: float = 1000.0        # Sec. III-B
    w_reg: float = 10000.0       # Sec. III-B
    w_data: float = 1.0          # Sec. III-B
    eps_d: float = 15.0          # mm, Sec. III-B
    cos_eps_n: float = float(np.cos(np.deg2rad(10.0)))   # 10 degrees, Sec. III-B
    lam: float = 1e-3
    gn_iters: int = 10
    pcg_iters: int = 10
    kp_point: np.ndarray = None  # key points (Eq.(9)): carrying model point per key point
    kp_target: np.ndarray = None  # (S, 3) matched positions, camera coordinates of the frame
    w_corr: float = 10.0          # Sec. III-B

    @staticmethod
    def from_scene(sc, **kw):
        args = dict(points=sc["points"], normals=sc["normals"], nodes=sc["nodes"], depth=sc["depth"],
                    camera=sc["camera"], R=sc["R"], T=sc["T"], sigma=sc["sigma"],
                    gn_iters=sc.get("gn_iters", 10), pcg_iters=sc.get("pcg_iters", 10))
        args.update(kw)
        return Problem(**args)


def evaluate(pb, graph, x, Nmap, Nvalid, corr_override=None):
    """Warp and associate at parameters x; returns (vc, nc, assoc, (e_data, e_rot, e_reg, e_corr)).

    With key points, assoc["kp_r"] holds their Eq.(9) residuals."""
    vc = ed_warp(pb.points, pb.nodes, x, graph["idx"], graph["w"], pb.R, pb.T)
    nc = warp_normals(pb.normals, x, graph["idx"], graph["w"], pb.R)
    asc = associate(vc, nc, pb.depth, pb.camera, Nmap, Nvalid, pb.eps_d, pb.cos_eps_n)
    if corr_override is not None:
        asc = _adopt(asc, corr_override, vc, pb, Nmap)
    e_corr = 0.0
    if pb.kp_point is not None:
        asc = dict(asc)
        asc["kp_r"] = corr_residuals(pb.points, pb.nodes, x, graph["idx"], graph["w"], pb.R, pb.T,
                                     pb.kp_point, pb.kp_target)
        e_corr = corr_energy(asc["kp_r"])
    return vc, nc, asc, energies(x, pb.nodes, graph["nbrs"], asc["r"]) + (e_corr,)


def linearize(pb, graph, x, Nmap, Nvalid, corr_override=None, jac_round=None):
    """Warp, associate and assemble at parameters x; returns everything the step needs."""
    vc, nc, asc, e = evaluate(pb, graph, x, Nmap, Nvalid, corr_override)
    corr = None if pb.kp_point is None else {"point": pb.kp_point, "r": asc["kp_r"], "w_corr": pb.w_corr}
    blocks, g = block_system(pb.points, pb.nodes, x, graph["idx"], graph["w"], pb.R, asc, graph["nbrs"],
                             graph["row_ptr"], graph["col_idx"], (pb.w_rot, pb.w_reg, pb.w_data), jac_round, corr)
    return vc, nc, asc, blocks, g, e


def _adopt(asc, corr, vc, pb, Nmap):
    """Decision-sync: take a given correspondence set instead of this one's own decisions.

    Used only to separate rounding-boundary flips (float32 vs float64 warps) from
    kernel errors; residuals are still evaluated in float64 at this x.
    """
    W, H, fx, fy, cx, cy = pb.camera
    fx, fy, cx, cy = (float(np.float32(a)) for a in (fx, fy, cx, cy))
    corr = np.asarray(corr, dtype=np.int64)
    ok = corr >= 0
    pix = np.where(ok, corr, 0)
    vi, ui = pix // W, pix % W
    D = np.asarray(pb.depth, dtype=np.float64)
    d = D[vi, ui]
    V = np.stack([d * ((ui - cx) / fx), d * ((vi - cy) / fy), d], axis=1)
    Np = np.asarray(Nmap, dtype=np.float64)[vi, ui]
    diff = vc - V
    r = (Np[:, 0] * diff[:, 0] + Np[:, 1] * diff[:, 1]) + Np[:, 2] * diff[:, 2]
    out = dict(asc)
    out.update(corr=np.where(ok, corr, -1), valid=ok, r=np.where(ok, r, 0.0), V=V, Np=Np)
    return out


def gn_register(pb, graph=None, x0=None, corr_sequence=None, record=False, jac_round=None, refine_steps=0):
    """Run pb.gn_iters Gauss-Newton steps.  Returns (x, report).

    report["iters"][it] holds energies at the linearisation point of step it
    (unweighted e_data, e_rot, e_reg), the number of valid correspondences and
    the PCG residual norms; report["final"] the energies at the returned x.
    corr_sequence, if given, supplies the correspondence set of each step
    (decision-sync mode).

    jac_round / refine_steps emulate the low-precision form: the step is solved
    on H_lo (data-term Jacobian rows passed through jac_round before J^T J),
    then refined refine_steps times: rho = -g - (H + lambda I) dx with the
    unrounded H, dx += P iterations of PCG on H_lo for rho.
    """
    if graph is None:
        graph = build_graph(pb.points, pb.nodes, pb.k, pb.weight_kind, pb.sigma)
    m = np.asarray(pb.nodes).shape[0]
    x = identity_params(m) if x0 is None else np.array(x0, dtype=np.float64)
    Nmap, Nvalid = normal_map(pb.depth, pb.camera)
    rep = {"iters": [], "graph": graph}
    for it in range(pb.gn_iters):
        co = None if corr_sequence is None else corr_sequence[it]
        vc, nc, asc, blocks, g, e = linearize(pb, graph, x, Nmap, Nvalid, co, jac_round)
        Minv, spd = block_jacobi(graph["row_ptr"], graph["col_idx"], blocks, pb.lam)
        dx, info = pcg(graph["row_ptr"], graph["col_idx"], blocks, g, pb.lam, pb.pcg_iters, Minv)
        if jac_round is not None and refine_steps > 0:
            h32, _ = block_system(pb.points, pb.nodes, x, graph["idx"], graph["w"], pb.R, asc, graph["nbrs"],
                                  graph["row_ptr"], graph["col_idx"], (pb.w_rot, pb.w_reg, pb.w_data))
            for _ in range(refine_steps):
                rho = -np.asarray(g).reshape(-1) - bsr_matvec(graph["row_ptr"], graph["col_idx"], h32, dx, pb.lam)
                d2, _ = pcg(graph["row_ptr"], graph["col_idx"], blocks, -rho, pb.lam, pb.pcg_iters, Minv)
                dx = dx + d2
        entry = {"e_data": e[0], "e_rot": e[1], "e_reg": e[2], "e_corr": e[3],
                 "n_valid": int(asc["valid"].sum()),
                 "resid": info["resid"], "breakdown": info["breakdown"], "nonspd": int((~spd).sum())}
        if record:
            entry.update(corr=asc["corr"].copy(), margin=asc["margin"], blocks=blocks, g=g, dx=dx,
                         x=x.copy(), vc=vc, nc=nc)
        rep["iters"].append(entry)
        x = x + dx.reshape(m, 12)
    vc, nc, asc, e = evaluate(pb, graph, x, Nmap, Nvalid)
    rep["final"] = {"e_data": e[0], "e_rot": e[1], "e_reg": e[2], "e_corr": e[3],
                    "n_valid": int(asc["valid"].sum()),
                    "vc": vc, "corr": asc["corr"]}
    return x, rep
