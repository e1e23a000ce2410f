"""Adaptive Levenberg-Marquardt damping for the per-frame registration (Sec. II-F).

The paper names Levenberg-Marquardt and gives no schedule.  Reading (the
classical Levenberg/Marquardt strategy): each step solves the damped normal
equations (H + lambda I) dx = -g at the current parameters x; the step is
taken only if the objective of Eq.(3) at x + dx is lower than at x, and then
lambda shrinks by a factor `down`; otherwise x stays and lambda grows by a
factor `up`.  lambda is kept within [lambda_min, lambda_max].  The objective
compared is the weighted sum w_data E_data + w_rot E_rot + w_reg E_reg
(+ w_corr E_corr with key points), each energy evaluated with the
correspondences re-decided at the point evaluated (Eqs.(7)-(8)), exactly as
a Gauss-Newton step evaluates them at its linearisation point.
Test infrastructure only (see the package header).
"""
import dataclasses

import numpy as np

from .depthmap import normal_map
from .gn import evaluate, linearize
from .graph import build_graph
from .pcg import block_jacobi, pcg
from .warp import identity_params


@dataclasses.dataclass
class LMSchedule:
    lambda0: float = 1e-3      # the fixed damping of the Gauss-Newton form
    up: float = 10.0           # Marquardt's factor
    down: float = 0.1
    lambda_min: float = 1e-6
    lambda_max: float = 1e6


def lm_iterate(x0, linearize_fn, solve_fn, energy_fn, sched, iters, decisions=None):
    """The damping schedule, independent of the problem.

    linearize_fn(x) -> (E, state): the objective at x and what solve_fn needs;
    solve_fn(state, lam) -> dx; energy_fn(x) -> E.  decisions, if given, forces
    the accept (True) / reject (False) of each step (decision-sync mode).
    Returns (x, log) with one entry per step: E, E_trial, lambda, accepted."""
    x = x0
    lam = sched.lambda0
    log = []
    for it in range(iters):
        E, state = linearize_fn(x)
        dx = solve_fn(state, lam)
        xt = x + dx
        Et = energy_fn(xt)
        acc = bool(Et < E) if decisions is None else bool(decisions[it])
        log.append({"E": E, "E_trial": Et, "lambda": lam, "accepted": acc, "state": state, "dx": dx})
        if acc:
            x = xt
            lam = max(lam * sched.down, sched.lambda_min)
        else:
            lam = min(lam * sched.up, sched.lambda_max)
    return x, log


def objective(pb, e):
    """Weighted Eq.(3) objective from unweighted (e_data, e_rot, e_reg, e_corr)."""
    return pb.w_data * e[0] + pb.w_rot * e[1] + pb.w_reg * e[2] + pb.w_corr * e[3]


def lm_register(pb, sched=None, graph=None, x0=None, decisions=None, corr_sequence=None):
    """pb.gn_iters damped steps with the adaptive schedule.  Returns (x, report).

    report["iters"][it]: unweighted energies at the step's x (as gn_register),
    E and E_trial (weighted objective at x and x + dx), lambda used, accepted, dx.
    corr_sequence, if given, supplies the correspondence set at each step's x
    (decision-sync mode; the trial point always re-decides its own)."""
    sched = sched or LMSchedule()
    if graph is None:
        graph = build_graph(pb.points, pb.nodes, pb.k, pb.weight_kind, pb.sigma)
    m = np.asarray(pb.nodes).shape[0]
    x = identity_params(m) if x0 is None else np.array(x0, dtype=np.float64)
    Nmap, Nvalid = normal_map(pb.depth, pb.camera)
    rp, ci = graph["row_ptr"], graph["col_idx"]
    step = [0]

    def lin(xc):
        co = None if corr_sequence is None else corr_sequence[step[0]]
        step[0] += 1
        _, _, asc, blocks, g, e = linearize(pb, graph, xc.reshape(m, 12), Nmap, Nvalid, co)
        return objective(pb, e), (blocks, g, e, asc)

    def solve(state, lam):
        blocks, g = state[0], state[1]
        Minv, _ = block_jacobi(rp, ci, blocks, lam)
        dx, info = pcg(rp, ci, blocks, g, lam, pb.pcg_iters, Minv)
        return dx

    def energy(xc):
        return objective(pb, evaluate(pb, graph, xc.reshape(m, 12), Nmap, Nvalid)[3])

    xf, log = lm_iterate(x.reshape(-1), lin, solve, energy, sched, pb.gn_iters, decisions)
    rep = {"iters": [], "graph": graph}
    for ent in log:
        e, asc = ent["state"][2], ent["state"][3]
        rep["iters"].append({"e_data": e[0], "e_rot": e[1], "e_reg": e[2], "e_corr": e[3],
                             "n_valid": int(asc["valid"].sum()), "E": ent["E"], "E_trial": ent["E_trial"],
                             "lambda": ent["lambda"], "accepted": ent["accepted"], "dx": ent["dx"]})
    x = xf.reshape(m, 12)
    _, _, asc, e = evaluate(pb, graph, x, Nmap, Nvalid)
    rep["final"] = {"e_data": e[0], "e_rot": e[1], "e_reg": e[2], "e_corr": e[3], "E": objective(pb, e),
                    "n_valid": int(asc["valid"].sum()), "corr": asc["corr"]}
    return x, rep
