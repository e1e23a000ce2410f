"""Full-size parity at the benchmark's configuration (640x480, 250,000 points, 1,600 nodes).

The oracle cannot redo the whole frame in seconds, so it checks sampled
outputs it can compute one at a time (kNN of sampled points, pattern rows and
normal-equation rows of sampled nodes), whole-image products it computes
quickly (normal map, correspondences on shared inputs, the PCG solve), and the
end-to-end parameters against the stored float64 oracle run of this frame
(tests/golden/make_oracle_golden.py).
"""
import os

import numpy as np
import pytest
import torch

import oracle
from gpu_util import Scene, check_energy, rel_err

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def c3(lib):
    return Scene("c3")


def _local_knn(s, j, radius):
    """Oracle kNN of every point within `radius` of node j; returns (point ids, idx rows)."""
    P = s.sc["points"].astype(np.float64)
    gj = s.sc["nodes"][j].astype(np.float64)
    cand = np.nonzero(np.sum((P - gj) ** 2, axis=1) < radius * radius)[0]
    idx, _ = oracle.knn(P[cand], s.sc["nodes"], 4)
    return cand, idx[:, :4]


def test_c3_normal_map_and_knn_samples(c3):
    s = c3
    got = s.M.normal_map(s.depth, s.cam).cpu().numpy()
    N, ok = oracle.normal_map(s.sc["depth"], s.sc["camera"])
    assert np.array_equal(got[..., :3].view(np.uint32), N.astype(np.float32).view(np.uint32))
    rng = np.random.default_rng(0)
    sel = np.sort(rng.choice(s.n, 4000, replace=False))
    idx, d2 = oracle.knn(s.sc["points"][sel], s.sc["nodes"], 4)
    assert np.array_equal(s.graph.knn_idx.cpu().numpy()[:, sel].T, idx[:, :4])
    w = oracle.skin_weights(d2, 4, "gauss", s.sc["sigma"])
    assert np.abs(s.graph.knn_w.cpu().numpy()[:, sel].T - w).max() <= 2e-7


def test_c3_pattern_and_rows_sampled(c3):
    s = c3
    g = s.graph
    info = g.info.cpu().numpy()
    assert info[3] == 0
    rp = g.row_ptr.cpu().numpy()
    ci = g.col_idx.cpu().numpy()
    lp = g.list_ptr.cpu().numpy()
    lst = g.list_pts.cpu().numpy()
    from gpu_util import random_params
    xg = random_params(s.m, 31, 0.003, 0.2)
    x = torch.tensor(xg, device="cuda")
    nmap = s.M.normal_map(s.depth, s.cam)
    blocks, gv, corr, _ = s.M.build_normal_eq(s.pts, s.nodes, x, g, nmap, s.cam, s.pose, s.params, s.ws)
    pos, nrm = s.M.warp(s.pts, s.nodes, x, g, s.pose)
    torch.cuda.synchronize()
    Nm, ok = oracle.normal_map(s.sc["depth"], s.sc["camera"])
    Nm32 = Nm.astype(np.float32)
    a = oracle.associate(pos.cpu().numpy().T, nrm.cpu().numpy().T, s.sc["depth"], s.sc["camera"], Nm32, ok,
                         s.params.eps_d, s.params.cos_eps_n)
    cg = corr.cpu().numpy()
    assert np.array_equal(cg, a["corr"])                       # decisions bit-exact on shared inputs
    rng = np.random.default_rng(1)
    rows = np.sort(rng.choice(s.m, 24, replace=False))
    radius = 3.0 * s.sc["node_spacing"]
    pts_all = []
    for j in rows:
        cand, idx = _local_knn(s, j, radius)
        mine = cand[np.any(idx == j, axis=1)]
        # list of node j: exactly these points, ordered by (sorted set, index)
        assert sorted(lst[lp[j]:lp[j + 1]]) == sorted(mine.tolist())
        nb = sorted(set(idx[np.any(idx == j, axis=1)].ravel().tolist()))
        assert list(ci[rp[j]:rp[j + 1]]) == nb                 # row j = {j} U N(j)
        pts_all.append(mine)
    sub = np.unique(np.concatenate(pts_all))
    # normal-equation rows from exactly those points (rows of the sampled nodes are then complete)
    og = s.oracle_graph_from_gpu()
    sub_idx = og["idx"][sub]
    sub_w = og["w"][sub]
    from oracle.gn import _adopt
    vc = oracle.ed_warp(s.sc["points"][sub], s.sc["nodes"], xg.astype(np.float64), sub_idx, sub_w,
                        s.sc["R"], s.sc["T"])
    pb = s.problem()
    asc = _adopt({}, cg[sub], vc, pb, Nm32)
    hb, hg = oracle.block_system(s.sc["points"][sub], s.sc["nodes"], xg.astype(np.float64), sub_idx, sub_w,
                                 s.sc["R"], asc, og["nbrs"], og["row_ptr"], og["col_idx"],
                                 (pb.w_rot, pb.w_reg, pb.w_data))
    gb = blocks.cpu().numpy()
    for j in rows:
        sl = slice(rp[j], rp[j + 1])
        assert rel_err(gb[sl], hb[sl]) < 1e-5, j
        assert rel_err(gv.cpu().numpy()[j], hg[j]) < 1e-5, j


def test_c3_pcg_full(c3):
    s = c3
    from gpu_util import random_params
    xg = random_params(s.m, 32, 0.003, 0.2)
    x = torch.tensor(xg, device="cuda")
    nmap = s.M.normal_map(s.depth, s.cam)
    blocks, gv, _, _ = s.M.build_normal_eq(s.pts, s.nodes, x, s.graph, nmap, s.cam, s.pose, s.params, s.ws)
    delta, rep = s.M.pcg_solve(s.graph, s.m, blocks, gv, s.params, s.ws)
    og = s.oracle_graph_from_gpu()
    nnzb = len(og["col_idx"])
    dx, info = oracle.pcg(og["row_ptr"], og["col_idx"], blocks.cpu().numpy()[:nnzb].astype(np.float64),
                          gv.cpu().numpy().astype(np.float64), float(np.float32(s.params.lam)), s.params.pcg_iters)
    assert rel_err(delta.cpu().numpy().reshape(-1), dx) < 1e-5
    assert s.M.read_report(rep)[0]["pcg_iters_done"] == info["iters"]


def test_c3_end_to_end_against_stored_oracle(c3):
    s = c3
    gold = np.load(os.path.join(HERE, "golden", "c3_oracle.npz"))
    x = s.M.identity_params(s.m)
    rep, _ = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, s.params, s.ws)
    r = s.M.read_report(rep)
    xg = x.cpu().numpy().astype(np.float64)
    xo = gold["x"]
    xi = oracle.identity_params(s.m)
    print("c3 x rel", rel_err(xg, xo), "delta rel", rel_err(xg - xi, xo - xi))
    assert rel_err(xg, xo) < 1e-5
    assert rel_err(xg - xi, xo - xi) < 1e-4
    check_energy(s, xi, r[0]["e_data"], xi, float(gold["e_data"][0]), label="c3 first step")
    check_energy(s, xg, r[-1]["e_data"], xo, float(gold["e_data_final"]), label="c3 final")
    assert np.all((r["flags"] & ~8) == 0)


def _against_stored(s, x, rep, name, pose_gpu=None):
    """Parameters and final data energy of a full-frame run against a stored oracle run of the same problem."""
    gold = np.load(os.path.join(HERE, "golden", f"c3_{name}_oracle.npz"))
    r = s.M.read_report(rep)
    xg = x.cpu().numpy().astype(np.float64)
    xo = gold["x"]
    xi = oracle.identity_params(s.m)
    print(name, "x rel", rel_err(xg, xo), "delta rel", rel_err(xg - xi, xo - xi), "e_data rel",
          abs(r[-1]["e_data"] - float(gold["e_data_final"])) / float(gold["e_data_final"]))
    assert rel_err(xg, xo) < 1e-5
    assert rel_err(xg - xi, xo - xi) < 1e-4
    pose_ref = (gold["R"], gold["T"]) if pose_gpu is not None else None
    check_energy(s, xg, r[-1]["e_data"], xo, float(gold["e_data_final"]), pose_gpu=pose_gpu, pose_ref=pose_ref,
                 label=f"c3 {name} final")
    assert np.all((r["flags"] & ~8) == 0)
    return gold, r


def test_c3_keypoints_against_stored_oracle(c3):
    """The frame with 500 key-point matches (Eq.(9), w_corr = 10), as the benchmark runs it."""
    import gen
    s = c3
    kp, tgt = gen.keypoints(s.sc, 500, seed=7, noise=0.05)
    keys = s.M.keypoints(torch.tensor(kp, device="cuda"), torch.tensor(tgt, device="cuda").contiguous(), 10.0)
    x = s.M.identity_params(s.m)
    rep, _ = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, s.params, s.ws, keys=keys)
    gold, r = _against_stored(s, x, rep, "kp500")
    assert r[-1]["e_corr"] == pytest.approx(float(gold["e_corr_final"]), rel=1e-4)


def test_c3_adaptive_lm_against_stored_oracle(c3):
    """The frame with the default adaptive schedule: the same accept / reject decisions and damping values as
    the stored oracle run (no decisions adopted from the GPU here)."""
    s = c3
    x = s.M.identity_params(s.m)
    rep, _ = s.M.lm_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, s.params, s.ws,
                             lm=s.M.LMParams())
    gold, r = _against_stored(s, x, rep, "lm")
    G = s.params.gn_iters
    assert [bool(v) for v in r["lm_accepted"][:G]] == [bool(v) for v in gold["accepted"]]
    np.testing.assert_allclose(r["lm_lambda"][:G], gold["lam"], rtol=1e-5)


def test_c3_joint_pose_against_stored_oracle(c3):
    """The frame with the pose as unknowns (Eq.(10), w_r = 1e6, w_p = 1e3); each side's final decisions are
    taken at its own refined pose."""
    s = c3
    x = s.M.identity_params(s.m)
    rep, pose, _ = s.M.joint_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, s.params, s.ws)
    P = pose.cpu().numpy().astype(np.float64)
    gold, r = _against_stored(s, x, rep, "joint", pose_gpu=(P[:9].reshape(3, 3), P[9:]))
    T0 = np.asarray(s.sc["T"], np.float32).astype(np.float64)
    moved = np.abs(gold["T"] - T0).max()
    assert moved > 0.1   # the pose moves (mm)
    assert np.abs(P[:9].reshape(3, 3) - gold["R"]).max() < 1e-5
    assert np.abs(P[9:] - gold["T"]).max() < 1e-3 * max(moved, 1.0)
