"""Edge cases of the HIP path against the oracle: empty model, empty depth,
ragged sizes, k = 1 and k = 8, a non-SPD diagonal block, capacity overflow."""
import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import Scene, random_params, rel_err

pytestmark = pytest.mark.gpu


def test_empty_model(lib):
    sc = gen.make_scene("c1")
    sc = dict(sc, points=np.zeros((0, 3), np.float32), normals=np.zeros((0, 3), np.float32))
    s = Scene(sc)
    g = s.graph
    info = g.info.cpu().numpy()
    assert info[0] == s.m and info[3] == 0                    # diagonal-only pattern
    assert np.array_equal(g.col_idx.cpu().numpy()[:s.m], np.arange(s.m))
    x = s.M.identity_params(s.m)
    rep, _ = s.M.gn_register(s.pts, s.nodes, x, g, s.depth, s.cam, s.pose, s.params, s.ws)
    r = s.M.read_report(rep)
    assert np.all(r["n_valid"] == 0) and np.all(r["pcg_iters_done"] == 0) and np.all(r["flags"] == 0)
    assert torch.equal(x, s.M.identity_params(s.m))


def test_empty_depth_regularisers_only(lib):
    sc = gen.make_scene("c1")
    sc = dict(sc, depth=np.zeros_like(sc["depth"]))
    s = Scene(sc)
    x0 = random_params(s.m, 21, scale_a=0.01, scale_t=0.2)
    x = torch.tensor(x0, device="cuda")
    rep, _ = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, s.params, s.ws)
    r = s.M.read_report(rep)
    assert np.all(r["n_valid"] == 0) and np.all(r["e_data"] == 0)
    xo, orep = oracle.gn_register(s.problem(), graph=s.oracle_graph_from_gpu(), x0=x0.astype(np.float64))
    print("delta rel", rel_err(x.cpu().numpy() - x0, xo - x0), "e_rot", r[-1]["e_rot"], orep["final"]["e_rot"],
          "e_reg", r[-1]["e_reg"], orep["final"]["e_reg"])
    assert rel_err(x.cpu().numpy() - x0, xo - x0) < 1e-4
    assert r[-1]["e_reg"] == pytest.approx(orep["final"]["e_reg"], rel=1e-4, abs=1e-8)
    assert r[-1]["e_rot"] == pytest.approx(orep["final"]["e_rot"], rel=1e-4, abs=1e-8)


def test_ragged_sizes_end_to_end(lib):
    s = Scene("ragged")
    assert s.n % 256 and s.m % 8 and s.m % 21
    ref = oracle.build_graph(s.sc["points"], s.sc["nodes"], 4, "gauss", s.sc["sigma"])
    assert np.array_equal(s.graph.knn_idx.cpu().numpy().T, ref["idx"])
    nnzb = int(s.graph.info.cpu().numpy()[0])
    assert np.array_equal(s.graph.col_idx.cpu().numpy()[:nnzb], ref["col_idx"])
    x = s.M.identity_params(s.m)
    xi = oracle.identity_params(s.m)
    rep, ch = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, s.params, s.ws, corr_hist=True)
    xo, orep = oracle.gn_register(s.problem(), graph=s.oracle_graph_from_gpu(), corr_sequence=list(ch.cpu().numpy()))
    print("x rel", rel_err(x.cpu().numpy(), xo), "delta rel", rel_err(x.cpu().numpy() - xi, xo - xi))
    assert rel_err(x.cpu().numpy(), xo) < 1e-5
    r = s.M.read_report(rep)
    assert r[-1]["e_data"] == pytest.approx(orep["final"]["e_data"], rel=1e-4)


def test_k1_block_diagonal_solved_in_one_iteration(lib):
    s = Scene("c1")
    s.params.k = 1
    s.params.pcg_iters = 1
    g = s.graph
    nnzb = int(g.info.cpu().numpy()[0])
    assert nnzb == s.m                                       # no node shares a point with another
    nmap = s.M.normal_map(s.depth, s.cam)
    x = torch.tensor(random_params(s.m, 22, 0.005, 0.2), device="cuda")
    blocks, gv, corr, _ = s.M.build_normal_eq(s.pts, s.nodes, x, g, nmap, s.cam, s.pose, s.params, s.ws)
    delta, rep = s.M.pcg_solve(g, s.m, blocks, gv, s.params, s.ws)
    hb = blocks.cpu().numpy()[:nnzb].astype(np.float64)
    lam = float(np.float32(s.params.lam))
    exact = np.concatenate([np.linalg.solve(hb[j] + lam * np.eye(12), -gv.cpu().numpy()[j].astype(np.float64))
                            for j in range(s.m)])
    assert rel_err(delta.cpu().numpy().reshape(-1), exact) < 1e-5
    assert s.M.read_report(rep)[0]["pcg_iters_done"] == 1


def test_k8_graph_and_normal_equations(lib):
    """k = 8: rows of up to 29 blocks.  The assembly splits a row's points over two waves with 18 statistic
    slots each and accumulates a longer row on one wave; this graph has rows of both kinds."""
    s = Scene("c1")
    s.params.k = 8
    s.params.sigma = 8.0
    g = s.graph
    ref = oracle.build_graph(s.sc["points"], s.sc["nodes"], 8, "gauss", 8.0)
    rl = np.diff(ref["row_ptr"])
    assert (rl > 18).any() and (rl <= 18).any()
    assert np.array_equal(g.knn_idx.cpu().numpy().T, ref["idx"])
    assert g.info.cpu().numpy()[3] == 0
    nnzb = int(g.info.cpu().numpy()[0])
    assert np.array_equal(g.col_idx.cpu().numpy()[:nnzb], ref["col_idx"])
    xg = random_params(s.m, 23, 0.005, 0.2)
    x = torch.tensor(xg, device="cuda")
    nmap = s.M.normal_map(s.depth, s.cam)
    blocks, gv, corr, _ = s.M.build_normal_eq(s.pts, s.nodes, x, g, nmap, s.cam, s.pose, s.params, s.ws)
    og = s.oracle_graph_from_gpu()
    Nm, ok = oracle.normal_map(s.sc["depth"], s.sc["camera"])
    from oracle.gn import evaluate
    pb = s.problem(k=8, sigma=8.0)
    _, _, asc, _ = evaluate(pb, og, xg.astype(np.float64), Nm.astype(np.float32), ok,
                            corr_override=corr.cpu().numpy())
    hb, hg = oracle.block_system(s.sc["points"], s.sc["nodes"], xg.astype(np.float64), og["idx"], og["w"],
                                 s.sc["R"], asc, og["nbrs"], og["row_ptr"], og["col_idx"],
                                 (pb.w_rot, pb.w_reg, pb.w_data))
    assert rel_err(blocks.cpu().numpy()[:nnzb], hb) < 1e-5
    assert rel_err(gv.cpu().numpy(), hg) < 1e-5


def test_non_spd_block_flagged(lib):
    sc = gen.make_scene("c1")
    far = np.array([[1000.0, 1000.0, 60.0]], np.float32)     # a node no point reaches
    sc = dict(sc, nodes=np.concatenate([sc["nodes"], far]))
    s = Scene(sc)
    s.params.k = 1
    s.params.lam = 0.0
    s.params.gn_iters = 1
    x = s.M.identity_params(s.m)
    rep, _ = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, s.params, s.ws)
    r = s.M.read_report(rep)
    assert r[0]["flags"] & 1                                  # MISSLAM_FLAG_NONSPD_BLOCK
    og = s.oracle_graph_from_gpu()
    pb = s.problem(k=1, lam=0.0, gn_iters=1)
    from oracle.gn import linearize
    Nm, ok = oracle.normal_map(s.sc["depth"], s.sc["camera"])
    _, _, _, blocks, _, _ = linearize(pb, og, oracle.identity_params(s.m), Nm.astype(np.float32), ok)
    _, spd = oracle.block_jacobi(og["row_ptr"], og["col_idx"], blocks, 0.0)
    assert not spd[-1]


def test_capacity_overflow_is_flagged_not_fatal(lib):
    s = Scene("c1")
    g = s.M.build_graph(s.pts, s.nodes, s.params, s.ws, bsr_cap=s.m + 5)
    info = g.info.cpu().numpy()
    assert info[3] & 16                                       # MISSLAM_FLAG_GRAPH_OVERFLOW
    x = s.M.identity_params(s.m)
    rep, _ = s.M.gn_register(s.pts, s.nodes, x, g, s.depth, s.cam, s.pose, s.params, s.ws)
    torch.cuda.synchronize()
    assert s.M.read_report(rep).shape[0] == s.params.gn_iters + 1


@pytest.mark.parametrize("k,step", [(4, 3), (8, 3), (4, 5)])
def test_long_node_lists(lib, k, step):
    """Coarse nodes over a dense model: every node list is longer than one LDS sort holds (MISSLAM_MAX_LIST),
    up to several pieces and an odd number of them; the lists must still be complete and in (sorted node set,
    point index) order, and the registration must follow the oracle."""
    sc = gen.make_scene("c2")
    nodes = sc["nodes"].reshape(16, 25, 3)[::step, ::step].reshape(-1, 3).copy()
    sc = dict(sc, nodes=nodes, sigma=5.0 * step, node_spacing=5.0 * step)
    s = Scene(sc)
    s.params.k = k
    g = s.graph
    info = g.info.cpu().numpy()
    assert info[3] == 0
    assert info[2] > 2 * 2048 if step == 5 else info[2] > 2048      # longest list
    ref = oracle.build_graph(sc["points"], sc["nodes"], k, "gauss", sc["sigma"])
    assert np.array_equal(g.knn_idx.cpu().numpy().T, ref["idx"])
    lp = g.list_ptr.cpu().numpy()
    lst = g.list_pts.cpu().numpy()
    keys = [tuple(sorted(r)) for r in ref["idx"]]
    for j in range(s.m):
        want = sorted(np.nonzero(np.any(ref["idx"] == j, axis=1))[0].tolist(), key=lambda p: (keys[p], p))
        assert lst[lp[j]:lp[j + 1]].tolist() == want, j
    x = s.M.identity_params(s.m)
    s.params.gn_iters = 3
    rep, ch = s.M.gn_register(s.pts, s.nodes, x, g, s.depth, s.cam, s.pose, s.params, s.ws, corr_hist=True)
    torch.cuda.synchronize()
    r = s.M.read_report(rep)
    assert np.all(r["flags"] == 0)
    xo, _ = oracle.gn_register(s.problem(), graph=s.oracle_graph_from_gpu(), corr_sequence=list(ch.cpu().numpy()))
    print("long lists k", k, "longest", info[2], "x rel", rel_err(x.cpu().numpy(), xo))
    assert rel_err(x.cpu().numpy(), xo) < 1e-5
