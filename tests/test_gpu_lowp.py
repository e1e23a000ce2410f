"""The low-precision form: data-term normal matrix on the matrix cores from
bfloat16/float16 Jacobian rows with float32 accumulation, float32 matrix-free
refinement of each step, float64 PCG reductions.

H_lo is compared with the oracle's emulation (Jacobian rows rounded to the
type before forming J^T J); the registered parameters with the plain float64
oracle at the 1e-3 bar, and the refinement must bring them closer.
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
def test_low_precision_normal_matrix(lib, prec):
    s = Scene("c1")
    code, rnd = PREC[prec]
    s.params.precision = code
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
    # the data term actually went through the low-precision type
    d_lo = rel_err(h_lo, h_32)
    assert d_lo > 1e-7


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_low_precision_registration_c3(lib, prec):
    s = Scene("c3")
    gold = np.load(os.path.join(HERE, "golden", "c3_oracle.npz"))
    xo = gold["x"]
    xi = oracle.identity_params(s.m)
    errs = {}
    for steps in (0, 2):
        s.params.precision = PREC[prec][0]
        s.params.refine_steps = steps
        x = s.M.identity_params(s.m)
        rep, _ = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, s.params, s.ws)
        r = s.M.read_report(rep)
        xg = x.cpu().numpy().astype(np.float64)
        errs[steps] = (rel_err(xg, xo), rel_err(xg - xi, xo - xi),
                       abs(r[-1]["e_data"] - float(gold["e_data_final"])) / float(gold["e_data_final"]))
    assert errs[2][0] < 1e-3 and errs[2][2] < 1e-3
    assert errs[2][1] <= errs[0][1]
