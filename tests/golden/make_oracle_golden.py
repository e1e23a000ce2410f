"""Writes the float64 oracle's registration result for a generated frame.

Calls only the scene generator and oracle/: nothing here comes from the GPU
path.  Usage: python tests/golden/make_oracle_golden.py c3
Output: tests/golden/<config>_oracle.npz with x (m, 12) after the frame's
Gauss-Newton iterations (independent decisions), the final data energy and the
per-iteration energies.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gen  # noqa: E402
import oracle  # noqa: E402


def main(name):
    sc = gen.make_scene(name)
    pb = oracle.Problem.from_scene(sc)
    x, rep = oracle.gn_register(pb)
    it = rep["iters"]
    np.savez_compressed(os.path.join(HERE, f"{name}_oracle.npz"), x=x, e_data_final=rep["final"]["e_data"],
                        e_rot_final=rep["final"]["e_rot"], e_reg_final=rep["final"]["e_reg"],
                        n_valid_final=rep["final"]["n_valid"],
                        e_data=np.array([e["e_data"] for e in it]), n_valid=np.array([e["n_valid"] for e in it]))
    print(name, "final e_data", rep["final"]["e_data"], "n_valid", rep["final"]["n_valid"])


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["c3"]:
        main(nm)
