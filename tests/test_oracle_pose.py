"""Pins of the oracle's joint rigid pose + ED registration (Eq.(10), Sec. II-F).

The pose columns of the data and key-point rows are checked against central
differences of residuals recomputed from a perturbed pose; the prior's
gradient against central differences of w_r E_r + w_p E_p; the border and
pose blocks against J^T W J of explicitly stacked rows; the joint PCG
against a dense Cholesky solve; and stiff priors against the fixed-pose
registration.
"""
import math

import numpy as np
import pytest

import gen
import oracle
from oracle.gn import linearize
from oracle.pose import (centre, corr_pose_rows, data_pose_rows, joint_linearize, joint_pcg, joint_register,
                         pose_border, pose_residuals, pose_step, so3_exp, so3_log)


def test_so3_closed_forms():
    th = 0.3
    Rz = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    np.testing.assert_allclose(so3_exp([0, 0, th]), Rz, atol=1e-15)
    w = np.array([0.2, -0.5, 0.4])
    np.testing.assert_allclose(so3_log(so3_exp(w)), w, atol=1e-13)
    np.testing.assert_allclose(so3_exp(w) @ so3_exp(w).T, np.eye(3), atol=1e-15)
    # camera centre: camera = R world + T maps C to the origin
    R, T = so3_exp(w), np.array([3.0, -1.0, 40.0])
    np.testing.assert_allclose(R @ centre(R, T) + T, 0.0, atol=1e-12)


@pytest.fixture(scope="module")
def c1():
    sc = gen.make_scene("c1")
    g = oracle.build_graph(sc["points"], sc["nodes"], 4, "gauss", sc["sigma"])
    return sc, g


def _params(m, seed):
    rng = np.random.default_rng(seed)
    x = oracle.identity_params(m)
    x[:, :9] += rng.normal(scale=0.02, size=(m, 9))
    x[:, 9:] = rng.normal(scale=0.3, size=(m, 3))
    return x


def _fd_pose_columns(f, R, T, h=1e-6):
    """Central differences of f(R, T) (any array) along the 6 pose directions."""
    cols = []
    for k in range(6):
        xi = np.zeros(6)
        xi[k] = h
        fp = f(*pose_step(R, T, xi))
        fm = f(*pose_step(R, T, -xi))
        cols.append((fp - fm) / (2 * h))
    return np.stack(cols, axis=-1)


def test_data_and_keypoint_pose_columns_match_differences(c1):
    sc, g = c1
    m = len(sc["nodes"])
    x = _params(m, 1)
    R, T = sc["R"].astype(np.float64), sc["T"].astype(np.float64)
    vc = oracle.ed_warp(sc["points"], sc["nodes"], x, g["idx"], g["w"], R, T)
    nc = oracle.warp_normals(sc["normals"], x, g["idx"], g["w"], R)
    Nmap, Nvalid = oracle.normal_map(sc["depth"], sc["camera"])
    asc = oracle.associate(vc, nc, sc["depth"], sc["camera"], Nmap, Nvalid, 15.0, math.cos(math.radians(10)))
    ok = asc["valid"]
    assert ok.sum() > 100
    V, Np = asc["V"][ok], asc["Np"][ok]

    def r_data(Ri, Ti):   # correspondences held fixed
        v = oracle.ed_warp(sc["points"], sc["nodes"], x, g["idx"], g["w"], Ri, Ti)[ok]
        return np.sum(Np * (v - V), axis=1)

    np.testing.assert_allclose(data_pose_rows(vc[ok], Np), _fd_pose_columns(r_data, R, T), rtol=1e-6, atol=1e-6)
    kp, tgt = gen.keypoints(sc, 25, seed=2, noise=0.1)

    def r_kp(Ri, Ti):
        return oracle.corr_residuals(sc["points"], sc["nodes"], x, g["idx"], g["w"], Ri, Ti, kp, tgt)

    vk = r_kp(R, T) + tgt.astype(np.float64)
    np.testing.assert_allclose(corr_pose_rows(vk), _fd_pose_columns(r_kp, R, T), rtol=1e-6, atol=1e-6)


def test_prior_gradient_matches_differences():
    """g_p of the priors is half the gradient of w_r E_r + w_p E_p along the pose step, also away from the
    prior (the identity Jacobian of E_r is exact for the gradient)."""
    R0, T0 = so3_exp([0.1, -0.2, 0.05]), np.array([1.0, 2.0, 50.0])
    R, T = pose_step(R0, T0, np.array([0.03, 0.02, -0.04, 0.5, -0.3, 0.8]))
    w_r, w_p = 1e6, 1e3

    def E(Ri, Ti):
        rr, rp = pose_residuals(Ri, Ti, R0, T0)
        return np.array(w_r * rr @ rr + w_p * rp @ rp)

    grad = 0.5 * _fd_pose_columns(E, R, T, h=1e-7)
    rho_r, rho_p = pose_residuals(R, T, R0, T0)
    want = np.concatenate([w_r * rho_r, -w_p * R @ rho_p])
    np.testing.assert_allclose(grad, want, rtol=1e-6, atol=1e-3)


def test_border_and_pose_block_are_jtwj_of_stacked_rows(c1):
    sc, g = c1
    m = len(sc["nodes"])
    kp, tgt = gen.keypoints(sc, 25, seed=4, noise=0.1)
    pb = oracle.Problem.from_scene(sc, kp_point=kp, kp_target=tgt, w_corr=10.0)
    x = _params(m, 2)
    R, T = pb.R.astype(np.float64), pb.T.astype(np.float64)
    Nmap, Nvalid = oracle.normal_map(pb.depth, pb.camera)
    vc, _, asc, _, _, _ = linearize(pb, g, x, Nmap, Nvalid)
    ok = asc["valid"]
    # explicit rows: data rows then the key points' 3 rows each, ED columns then pose columns
    Jd = oracle.data_jacobian_rows(pb.points, pb.nodes, g["idx"], g["w"], R, asc["Np"])
    Jk = oracle.corr_jacobian_rows(pb.points, pb.nodes, g["idx"], g["w"], R, kp)
    rows, res, wts = [], [], []
    for i in np.nonzero(ok)[0]:
        row = np.zeros(12 * m + 6)
        for s in range(4):
            j = g["idx"][i, s]
            row[12 * j:12 * j + 12] += Jd[i, s]
        row[12 * m:] = data_pose_rows(vc[i:i + 1], asc["Np"][i:i + 1])[0]
        rows.append(row)
        res.append(asc["r"][i])
        wts.append(pb.w_data)
    vk = asc["kp_r"] + tgt.astype(np.float64)
    J3 = corr_pose_rows(vk)
    for s, p in enumerate(kp):
        for a in range(3):
            row = np.zeros(12 * m + 6)
            for q in range(4):
                j = g["idx"][p, q]
                row[12 * j:12 * j + 12] += Jk[s, a, q]
            row[12 * m:] = J3[s, a]
            rows.append(row)
            res.append(asc["kp_r"][s, a])
            wts.append(pb.w_corr)
    J = np.array(rows)
    W = np.array(wts)
    H = J.T @ (W[:, None] * J)
    gv = J.T @ (W * np.array(res))
    B, Hpp, gp = pose_border(pb, g, x, R, asc, vc, vk)
    np.testing.assert_allclose(B.reshape(12 * m, 6), H[:12 * m, 12 * m:], rtol=1e-10, atol=1e-8)
    np.testing.assert_allclose(Hpp, H[12 * m:, 12 * m:], rtol=1e-10, atol=1e-8)
    np.testing.assert_allclose(gp, gv[12 * m:], rtol=1e-10, atol=1e-8)


def test_joint_pcg_reaches_the_dense_solution(c1):
    sc, g = c1
    m = len(sc["nodes"])
    pb = oracle.Problem.from_scene(sc)
    R0, T0 = pb.R.astype(np.float64), pb.T.astype(np.float64)
    R, T = pose_step(R0, T0, np.array([0.002, -0.001, 0.003, 0.2, 0.1, -0.3]))
    Nmap, Nvalid = oracle.normal_map(pb.depth, pb.camera)
    x = _params(m, 3)
    _, _, blocks, ge, B, Hpp, gp, _, _ = joint_linearize(pb, g, x, R, T, R0, T0, 1e6, 1e3, Nmap, Nvalid)
    He = oracle.dense_from_blocks(g["row_ptr"], g["col_idx"], blocks, m)
    Bf = B.reshape(12 * m, 6)
    H = np.block([[He, Bf], [Bf.T, Hpp]])
    gv = np.concatenate([np.asarray(ge).reshape(-1), gp])
    want = oracle.cholesky_solve(H, gv, pb.lam)
    dx, dxi, info = joint_pcg(g["row_ptr"], g["col_idx"], blocks, B, Hpp, ge, gp, pb.lam, 12 * m + 6)
    got = np.concatenate([dx, dxi])
    assert np.linalg.norm(got - want) <= 1e-6 * np.linalg.norm(want)


def test_stiff_priors_keep_the_pose_and_reduce_to_the_fixed_pose_registration(c1):
    sc, g = c1
    pb = oracle.Problem.from_scene(sc, gn_iters=3)
    xg, _ = oracle.gn_register(pb, graph=g)
    x, R, T, rep = joint_register(pb, graph=g, w_r=1e14, w_p=1e14)
    np.testing.assert_allclose(R, pb.R, atol=1e-9)
    np.testing.assert_allclose(T, pb.T, atol=1e-7)
    assert np.linalg.norm(x - xg) <= 1e-6 * np.linalg.norm(xg)


def test_joint_registration_lowers_the_objective(c1):
    """With the paper's weights the pose moves and the joint objective (pose terms included) ends below its
    start; the priors are zero at the start."""
    sc, g = c1
    pb = oracle.Problem.from_scene(sc, gn_iters=6)
    x, R, T, rep = joint_register(pb, graph=g)
    it = rep["iters"]

    def total(e):
        return pb.w_data * e["e_data"] + pb.w_rot * e["e_rot"] + pb.w_reg * e["e_reg"] + 1e6 * e["e_r"] + \
            1e3 * e["e_p"]

    assert total(rep["final"]) < total(it[0])
    assert it[0]["e_r"] == 0.0 and it[0]["e_p"] == 0.0
    assert rep["final"]["e_r"] > 0.0 and rep["final"]["e_p"] > 0.0
