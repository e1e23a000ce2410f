"""Parity of the joint rigid pose + ED registration (Eq.(10)) with the oracle.

The GPU run records its correspondences; the oracle replays them
(decision-sync) from the same start and prior, so the comparison isolates the
joint system's arithmetic (pose columns, border, pose block, priors, joint
PCG, pose step) from float32-vs-float64 association flips.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import Scene, rel_err
from oracle.pose import joint_register

pytestmark = pytest.mark.gpu


def _run(s, params, w_r=1e6, w_p=1e3):
    x = s.M.identity_params(s.m)
    rep, pose, ch = s.M.joint_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, params, s.ws, w_r=w_r,
                                       w_p=w_p, corr_hist=True)
    torch.cuda.synchronize()
    P = pose.cpu().numpy().astype(np.float64)
    return x.cpu().numpy(), P[:9].reshape(3, 3), P[9:], s.M.read_report(rep), list(ch.cpu().numpy())


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_joint_registration_matches_oracle(lib, name):
    s = Scene(name)
    xg, Rg, Tg, r, cs = _run(s, s.params)
    pb = s.problem()
    og = s.oracle_graph_from_gpu()
    xo, Ro, To, orep = joint_register(pb, graph=og, corr_sequence=cs)
    R0, T0 = pb.R.astype(np.float64), pb.T.astype(np.float64)
    x0 = oracle.identity_params(s.m)
    dR = np.abs(Rg - Ro).max()
    dT = np.abs(Tg - To).max()
    print(name, "x rel", rel_err(xg, xo), "delta rel", rel_err(xg - x0, xo - x0), "|dR|", dR, "|dT|", dT,
          "pose moved", np.abs(Ro - R0).max(), np.abs(To - T0).max(), "e_pose", r["e_pose_r"][[1, -1]].tolist(),
          r["e_pose_p"][[1, -1]].tolist(), [orep["final"]["e_r"], orep["final"]["e_p"]])
    assert rel_err(xg, xo) < 1e-5
    assert rel_err(xg - x0, xo - x0) < 1e-4
    # the pose moves, and the GPU follows the oracle's move to float32 rounding
    assert np.abs(To - T0).max() > 1e-4
    assert dR <= 1e-3 * max(np.abs(Ro - R0).max(), 1e-6) + 2e-7
    assert dT <= 1e-3 * np.abs(To - T0).max() + 2e-5
    it = orep["iters"]
    for k in range(pb.gn_iters):
        assert r[k]["e_data"] == pytest.approx(it[k]["e_data"], rel=1e-5)
        assert r[k]["e_pose_r"] == pytest.approx(it[k]["e_r"], rel=2e-3, abs=1e-12)
        assert r[k]["e_pose_p"] == pytest.approx(it[k]["e_p"], rel=2e-3, abs=1e-9)
    assert r[0]["e_pose_r"] == 0.0 and r[0]["e_pose_p"] == 0.0
    assert r[-1]["e_pose_p"] == pytest.approx(orep["final"]["e_p"], rel=2e-3, abs=1e-9)
    assert np.all(r["flags"] == 0)


def test_stiff_priors_are_the_fixed_pose_registration(lib):
    """Priors far stiffer than the data keep the pose; the ED result is then the fixed-pose one (to the
    rounding of a different reduction order)."""
    s = Scene("c2")
    xg, Rg, Tg, r, _ = _run(s, s.params, w_r=1e15, w_p=1e15)
    x = s.M.identity_params(s.m)
    rp, _ = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, s.params, s.ws)
    torch.cuda.synchronize()
    R0 = np.asarray(s.sc["R"], np.float32).astype(np.float64)
    T0 = np.asarray(s.sc["T"], np.float32).astype(np.float64)
    assert np.abs(Rg - R0).max() <= 1e-6 and np.abs(Tg - T0).max() <= 1e-5
    assert rel_err(xg, x.cpu().numpy()) < 1e-5


def test_zero_steps_keep_the_pose(lib):
    """gn_iters = 0: the pose comes back as given, bit for bit, with zero pose energies."""
    s = Scene("c1")
    params = s.M.Params(sigma=s.params.sigma, gn_iters=0, pcg_iters=10)
    xg, Rg, Tg, r, _ = _run(s, params)
    R0 = np.asarray(s.sc["R"], np.float32).astype(np.float64)
    T0 = np.asarray(s.sc["T"], np.float32).astype(np.float64)
    assert np.array_equal(Rg, R0) and np.array_equal(Tg, T0)
    assert len(r) == 1 and r[0]["e_pose_r"] == 0.0 and r[0]["e_pose_p"] == 0.0
    assert np.array_equal(xg, s.M.identity_params(s.m).cpu().numpy())


def test_joint_with_keypoints_matches_oracle(lib):
    """All six terms of Eq.(3) together: the joint pose with 200 key points (their rows gain the pose columns
    [-[v~]x, I]; their part of the border and of the pose block)."""
    import gen
    s = Scene("c2")
    kp, tgt = gen.keypoints(s.sc, 200, seed=7, noise=0.05)
    keys = s.M.keypoints(torch.tensor(kp, device="cuda"), torch.tensor(tgt, device="cuda").contiguous(), 10.0)
    x = s.M.identity_params(s.m)
    rep, pose, ch = s.M.joint_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, s.params, s.ws,
                                       corr_hist=True, keys=keys)
    torch.cuda.synchronize()
    P = pose.cpu().numpy().astype(np.float64)
    Rg, Tg, xg, r = P[:9].reshape(3, 3), P[9:], x.cpu().numpy(), s.M.read_report(rep)
    cs = list(ch.cpu().numpy())
    pb = s.problem(kp_point=kp, kp_target=tgt, w_corr=10.0)
    xo, Ro, To, orep = joint_register(pb, graph=s.oracle_graph_from_gpu(), corr_sequence=cs)
    x0 = oracle.identity_params(s.m)
    T0 = pb.T.astype(np.float64)
    print("joint+kp x rel", rel_err(xg, xo), "delta rel", rel_err(xg - x0, xo - x0), "|dT|", np.abs(Tg - To).max(),
          "moved", np.abs(To - T0).max(), "e_corr", r["e_corr"][[0, -1]].tolist(), orep["final"]["e_corr"])
    assert rel_err(xg, xo) < 1e-5
    assert rel_err(xg - x0, xo - x0) < 1e-4
    assert np.abs(Rg - Ro).max() <= 1e-3 * np.abs(Ro - pb.R).max() + 2e-7
    assert np.abs(Tg - To).max() <= 1e-3 * np.abs(To - T0).max() + 2e-5
    for k in range(pb.gn_iters):
        assert r[k]["e_corr"] == pytest.approx(orep["iters"][k]["e_corr"], rel=1e-5)
        assert r[k]["e_data"] == pytest.approx(orep["iters"][k]["e_data"], rel=1e-5)
        assert r[k]["e_pose_p"] == pytest.approx(orep["iters"][k]["e_p"], rel=2e-3, abs=1e-9)
    assert np.all(r["flags"] == 0)
