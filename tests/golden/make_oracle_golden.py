"""Writes the float64 oracle's registration result for a generated frame.

Calls only the input generators and oracle/: nothing here comes from the GPU
path.  Usage: python tests/golden/make_oracle_golden.py c3 [c3:bf16:2 c3:kp:500 ...]
A plain name runs the float64 oracle; name:prec:R runs its emulation of the
low-precision form (data-term Jacobian rows rounded to bf16 / fp16 before
J^T J, R refinement passes of each step against the unrounded system);
name:kp:S adds S generated key points (gen.keypoints, seed 7, 0.05 mm noise)
with the Eq.(9) term at w_corr = 10; name:lm runs the adaptive
Levenberg-Marquardt schedule (default factors) instead of the fixed damping;
name:joint registers the rigid pose with the ED graph (Eq.(10) terms,
w_r = 1e6, w_p = 1e3), storing the refined pose too; name:pcg:P runs the
plain oracle with P PCG iterations per step.  batch<b> is problem b of the
uneven batch (gen.batch_spec(b)).
Output: tests/golden/<name>[_<prec>_r<R> | _kp<S> | _lm | _joint | _pcg<P>]_oracle.npz with x
(m, 12) after the frame's iterations (independent decisions), the final
energies and the per-iteration data energies (and, for lm, the per-step
decisions and dampings).
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gen  # noqa: E402
import oracle  # noqa: E402

ROUND = {"bf16": oracle.round_bf16, "fp16": oracle.round_fp16}


def main(spec):
    parts = spec.split(":")
    name = parts[0]
    sc = gen.make_scene(gen.batch_spec(int(name[5:])) if name.startswith("batch") else name)
    pb = oracle.Problem.from_scene(sc)
    if len(parts) == 1:
        x, rep = oracle.gn_register(pb)
        out = f"{name}_oracle.npz"
    elif parts[1] == "joint":
        x, R, T, rep = oracle.joint_register(pb)
        out = f"{name}_joint_oracle.npz"
        extra_pose = dict(R=R, T=T, e_r_final=rep["final"]["e_r"], e_p_final=rep["final"]["e_p"])
    elif parts[1] == "lm":
        x, rep = oracle.lm_register(pb, oracle.LMSchedule())
        out = f"{name}_lm_oracle.npz"
    elif parts[1] == "pcg":
        P = int(parts[2])
        pb = oracle.Problem.from_scene(sc, pcg_iters=P)
        x, rep = oracle.gn_register(pb)
        out = f"{name}_pcg{P}_oracle.npz"
    elif parts[1] == "kp":
        S = int(parts[2])
        kp, tgt = gen.keypoints(sc, S, seed=7, noise=0.05)
        pb = oracle.Problem.from_scene(sc, kp_point=kp, kp_target=tgt, w_corr=10.0)
        x, rep = oracle.gn_register(pb)
        out = f"{name}_kp{S}_oracle.npz"
    else:
        prec, steps = parts[1], int(parts[2])
        rnd = ROUND[prec]
        x, rep = oracle.gn_register(pb, jac_round=lambda J: rnd(J.astype(np.float32)), refine_steps=steps)
        out = f"{name}_{prec}_r{steps}_oracle.npz"
    it = rep["iters"]
    extra = dict(extra_pose) if len(parts) > 1 and parts[1] == "joint" else {}
    if "accepted" in it[0]:
        extra.update(accepted=np.array([e["accepted"] for e in it]), lam=np.array([e["lambda"] for e in it]),
                     E=np.array([e["E"] for e in it]), E_trial=np.array([e["E_trial"] for e in it]))
    np.savez_compressed(os.path.join(HERE, out), x=x, e_data_final=rep["final"]["e_data"],
                        e_rot_final=rep["final"]["e_rot"], e_reg_final=rep["final"]["e_reg"],
                        n_valid_final=rep["final"]["n_valid"], e_corr_final=rep["final"]["e_corr"],
                        e_data=np.array([e["e_data"] for e in it]), n_valid=np.array([e["n_valid"] for e in it]),
                        **extra)
    print(out, "final e_data", rep["final"]["e_data"], "n_valid", rep["final"]["n_valid"])


if __name__ == "__main__":
    for sp in sys.argv[1:] or ["c3"]:
        main(sp)
