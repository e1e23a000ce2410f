"""The energy adjoint (dE/dx, dE/dv) through the C ABI and the autograd Function.

Correspondences are found once by the GPU and held fixed; the oracle adopts
them (float64 residuals at the same pixels) and evaluates the energy and its
gradient.  Central finite differences (h = 1e-4) of the float64 oracle energy
on 50 sampled parameters tie both to the mathematics.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import Scene, random_params, rel_err
from oracle.gn import _adopt

pytestmark = pytest.mark.gpu
W3 = (1000.0, 10000.0, 1.0)


def _setup(name, seed):
    s = Scene(name)
    xg = random_params(s.m, seed, 0.004, 0.3)
    x = torch.tensor(xg, device="cuda")
    nmap = s.M.normal_map(s.depth, s.cam)
    e, gp, gv, corr, rep = s.M.energy_vjp(s.pts, s.nodes, x, s.graph, nmap, s.cam, s.pose, s.params, s.ws)
    torch.cuda.synchronize()
    og = s.oracle_graph_from_gpu()
    Nm, ok = oracle.normal_map(s.sc["depth"], s.sc["camera"])
    pb = s.problem()
    vc = oracle.ed_warp(s.sc["points"], s.sc["nodes"], xg.astype(np.float64), og["idx"], og["w"], s.sc["R"], s.sc["T"])
    asc = _adopt({}, corr.cpu().numpy(), vc, pb, Nm.astype(np.float32))
    return s, xg, x, nmap, e, gp, gv, corr, og, asc


def _energy(s, xg, og, asc, pts=None):
    P = s.sc["points"] if pts is None else pts
    return oracle.total_energy_fixed(xg, P, s.sc["nodes"], og["nbrs"], og["idx"], s.sc["sigma"], s.sc["R"], s.sc["T"],
                                     asc["V"], asc["Np"], asc["valid"], W3)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_energy_and_gradients_match_oracle(lib, name):
    s, xg, x, nmap, e, gp, gv, corr, og, asc = _setup(name, 51)
    x64 = xg.astype(np.float64)
    assert float(e.cpu()[0]) == pytest.approx(_energy(s, x64, og, asc), rel=1e-5)
    ref = oracle.energy_grad_params(x64, s.sc["points"], s.sc["nodes"], og["nbrs"], og["idx"], og["w"], s.sc["R"],
                                    asc["r"], asc["Np"], asc["valid"], W3)
    assert rel_err(gp.cpu().numpy(), ref) < 1e-5
    refv = oracle.energy_grad_points(x64, s.sc["points"], s.sc["nodes"], og["idx"], s.sc["sigma"], s.sc["R"],
                                     asc["r"], asc["Np"], asc["valid"], 1.0)
    assert rel_err(gv.cpu().numpy().T, refv) < 1e-5


def test_c3_gradient_against_central_differences(lib):
    """640x480 / 250k points / 1600 nodes: 50 parameters (seed 33), h = 1e-4, float64 oracle energy."""
    s, xg, x, nmap, e, gp, gv, corr, og, asc = _setup("c3", 52)
    x64 = xg.astype(np.float64)
    rng = np.random.default_rng(33)
    flat = rng.choice(s.m * 12, 50, replace=False)
    idx = og["idx"]
    h = 1e-4
    fd = np.zeros(50)
    for q, f in enumerate(flat):
        j, c = divmod(int(f), 12)
        sel = np.nonzero(np.any(idx == j, axis=1))[0]          # only these points see node j
        sub = {k: asc[k][sel] for k in ("V", "Np", "valid")}

        def en(xx):
            rd = oracle.grad.data_residuals_fixed(s.sc["points"][sel], s.sc["nodes"], xx, idx[sel], s.sc["sigma"],
                                                  s.sc["R"], s.sc["T"], sub["V"], sub["Np"], sub["valid"])
            rg, _, _ = oracle.reg_residuals(xx, s.sc["nodes"], og["nbrs"])
            return W3[2] * np.sum(rd * rd) + W3[0] * np.sum(oracle.rot_residuals(xx) ** 2) + W3[1] * np.sum(rg * rg)
        xp = x64.copy(); xp[j, c] += h
        xm = x64.copy(); xm[j, c] -= h
        fd[q] = (en(xp) - en(xm)) / (2 * h)
    got = gp.cpu().numpy().reshape(-1)[flat]
    ref = oracle.energy_grad_params(x64, s.sc["points"], s.sc["nodes"], og["nbrs"], idx, og["w"], s.sc["R"],
                                    asc["r"], asc["Np"], asc["valid"], W3).reshape(-1)[flat]
    assert rel_err(ref, fd) < 1e-6                              # oracle gradient vs differences
    assert rel_err(got, fd) < 1e-5                              # GPU adjoint vs differences
    assert rel_err(gp.cpu().numpy(), oracle.energy_grad_params(
        x64, s.sc["points"], s.sc["nodes"], og["nbrs"], idx, og["w"], s.sc["R"], asc["r"], asc["Np"], asc["valid"],
        W3)) < 1e-5


def test_autograd_function(lib):
    s, xg, x, nmap, e, gp, gv, corr, og, asc = _setup("c1", 53)
    ctx = dict(points=s.pts, nodes=s.nodes, graph=s.graph, nmap=nmap, cam=s.cam, pose=s.pose, params=s.params,
               ws=s.ws)
    xr = x.clone().requires_grad_(True)
    pos = s.pts[:3].clone().requires_grad_(True)
    E = s.M.WarpEnergy.apply(xr, pos, ctx)
    (3.0 * E).backward()
    assert float(E.detach().cpu()) == pytest.approx(float(e.cpu()[0]), rel=1e-12)
    assert torch.allclose(xr.grad, 3.0 * gp, rtol=1e-6, atol=0)
    assert torch.allclose(pos.grad, 3.0 * gv, rtol=1e-6, atol=0)
