"""The low-precision form: data-term normal matrix on the matrix cores from
bfloat16/float16 Jacobian rows with float32 accumulation, float32 matrix-free
refinement of each step, float64 PCG reductions.

H_lo is compared with the oracle's emulation (Jacobian rows rounded to the
type before forming J^T J), once with the full energy and once with the data
term alone (where the rounding is visible).  The registered parameters are
compared with the oracle's emulation of the same form (same rounding, same
number of refinement passes, stored by tests/golden/make_oracle_golden.py) at
the 1e-3 bar of the low-precision form.  The refined iterate is not the plain
float64 oracle's: each refinement pass adds another truncated PCG solve, so
the step goes further toward the exact Gauss-Newton step than the oracle's
ten PCG iterations do.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from gpu_util import Scene, random_params, rel_err
from oracle.gn import _adopt

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
PREC = {"bf16": (1, oracle.round_bf16), "fp16": (2, oracle.round_fp16)}


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("data_only", [False, True])
def test_low_precision_normal_matrix(lib, prec, data_only):
    s = Scene("c1")
    code, rnd = PREC[prec]
    s.params.precision = code
    if data_only:
        s.params.w_rot = 0.0
        s.params.w_reg = 0.0
    xg = random_params(s.m, 61, 0.003, 0.2)
    x = torch.tensor(xg, device="cuda")
    nmap = s.M.normal_map(s.depth, s.cam)
    blocks, g, corr, rep = s.M.build_normal_eq(s.pts, s.nodes, x, s.graph, nmap, s.cam, s.pose, s.params, s.ws)
    og = s.oracle_graph_from_gpu()
    Nm, ok = oracle.normal_map(s.sc["depth"], s.sc["camera"])
    pb = s.problem()
    vc = oracle.ed_warp(s.sc["points"], s.sc["nodes"], xg.astype(np.float64), og["idx"], og["w"], s.sc["R"], s.sc["T"])
    asc = _adopt({}, corr.cpu().numpy(), vc, pb, Nm.astype(np.float32))
    args = (s.sc["points"], s.sc["nodes"], xg.astype(np.float64), og["idx"], og["w"], s.sc["R"], asc, og["nbrs"],
            og["row_ptr"], og["col_idx"], (pb.w_rot, pb.w_reg, pb.w_data))
    h_lo, g_ref = oracle.block_system(*args, jac_round=lambda J: rnd(J.astype(np.float32)))
    h_32, _ = oracle.block_system(*args)
    nnzb = len(og["col_idx"])
    got = blocks.cpu().numpy()[:nnzb]
    assert rel_err(got, h_lo) < 1e-5
    assert rel_err(g.cpu().numpy(), g_ref) < 1e-5                 # the gradient stays float32
    if data_only:
        # the data term went through the low-precision type: the product is far
        # nearer the rounded emulation than the unrounded blocks
        d_lo = rel_err(h_lo, h_32)
        assert d_lo > 1e-5
        assert rel_err(got, h_lo) < 0.05 * d_lo


@pytest.mark.parametrize("prec,steps", [("bf16", 0), ("fp16", 0), ("bf16", 2), ("fp16", 2)])
def test_low_precision_registration_c3(lib, prec, steps):
    """640x480 / 250k points / 1600 nodes, independent decisions on both sides.

    Without refinement the form is the float64 oracle's algorithm with a
    rounded data-term matrix: it must meet the 1e-3 bar against the plain
    float64 oracle.  With refinement each step is solved further than ten PCG
    iterations reach, so it is held to the oracle's emulation of the refined
    form (same rounding, same passes) and its distance to the plain oracle is
    only reported.
    """
    s = Scene("c3")
    plain = np.load(os.path.join(HERE, "golden", "c3_oracle.npz"))
    emu_file = os.path.join(HERE, "golden", f"c3_{prec}_r{steps}_oracle.npz")
    assert os.path.exists(emu_file), f"missing same-form oracle run {emu_file} (tests/golden/make_oracle_golden.py)"
    gold = np.load(emu_file)
    xi = oracle.identity_params(s.m)
    s.params.precision = PREC[prec][0]
    s.params.refine_steps = steps
    x = s.M.identity_params(s.m)
    rep, _ = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, s.params, s.ws)
    r = s.M.read_report(rep)
    xg = x.cpu().numpy().astype(np.float64)
    xo = gold["x"]
    print(prec, steps, "vs same-form oracle", rel_err(xg, xo), rel_err(xg - xi, xo - xi),
          "vs plain float64 oracle", rel_err(xg, plain["x"]), "e_data", r[-1]["e_data"], float(gold["e_data_final"]))
    assert rel_err(xg, xo) < 1e-3
    assert rel_err(xg - xi, xo - xi) < 1e-2
    assert abs(r[-1]["e_data"] - float(gold["e_data_final"])) < 1e-3 * float(gold["e_data_final"])
    if steps == 0:
        assert rel_err(xg, plain["x"]) < 1e-3
    assert np.all(r["flags"] == 0)
