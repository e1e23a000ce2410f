"""Stage-wise and end-to-end parity of the HIP path (through the C ABI) with the float64 oracle.

Integer outputs (kNN sets, block pattern, node lists, correspondences) must be
bit-exact given the same inputs; float outputs are compared with the error
definitions of the oracle's readings (relative norms), at 1e-5 for float32
unless stated.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import Scene, random_params, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1(lib):
    return Scene("c1")


@pytest.fixture(scope="module")
def c2(lib):
    return Scene("c2")


def _f32_nmap(depth, cam):
    N, ok = oracle.normal_map(depth, cam)
    out = np.zeros(depth.shape + (4,), dtype=np.float32)
    out[..., :3] = N.astype(np.float32)
    out[..., 3] = depth
    return out, ok


# ---------------------------------------------------------------- a1: depth normal map
@pytest.mark.parametrize("name", ["c1", "c2"])
def test_normal_map_bit_exact(lib, name):
    s = Scene(name)
    got = s.M.normal_map(s.depth, s.cam).cpu().numpy()
    ref, ok = _f32_nmap(s.sc["depth"], s.sc["camera"])
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    assert np.array_equal(np.any(got[..., :3] != 0, axis=-1), ok)


# ---------------------------------------------------------------- a2: graph
@pytest.mark.parametrize("name", ["c1", "c2"])
def test_knn_and_pattern_bit_exact(lib, name):
    s = Scene(name)
    g = s.graph
    ref = oracle.build_graph(s.sc["points"], s.sc["nodes"], 4, "gauss", s.sc["sigma"])
    idx = g.knn_idx.cpu().numpy().T
    assert np.array_equal(idx, ref["idx"])
    w = g.knn_w.cpu().numpy().T
    assert np.abs(w - ref["w"]).max() <= 2e-7
    info = g.info.cpu().numpy()
    assert info[3] == 0
    nnzb = info[0]
    assert np.array_equal(g.row_ptr.cpu().numpy(), ref["row_ptr"])
    assert np.array_equal(g.col_idx.cpu().numpy()[:nnzb], ref["col_idx"])
    # node -> point lists: the points carrying the node, ordered by (sorted node set, index)
    lp = g.list_ptr.cpu().numpy()
    lst = g.list_pts.cpu().numpy()
    keys = [tuple(sorted(r)) for r in ref["idx"]]
    for j in range(0, s.m, max(1, s.m // 40)):
        want = sorted([p for p in range(s.n) if j in ref["idx"][p]], key=lambda p: (keys[p], p))
        assert list(lst[lp[j]:lp[j + 1]]) == want


def test_linear_weights(lib):
    s = Scene("c1")
    s.params.weight_kind = 1
    g = s.graph
    ref = oracle.build_graph(s.sc["points"], s.sc["nodes"], 4, "linear")
    assert np.array_equal(g.knn_idx.cpu().numpy().T, ref["idx"])
    assert np.abs(g.knn_w.cpu().numpy().T - ref["w"]).max() <= 2e-7


# ---------------------------------------------------------------- a3: warp
@pytest.mark.parametrize("name", ["c1", "c2"])
def test_warp_parity(lib, name):
    s = Scene(name)
    xg = random_params(s.m, 11)
    x = torch.tensor(xg, device="cuda")
    pos, nrm = s.M.warp(s.pts, s.nodes, x, s.graph, s.pose)
    og = s.oracle_graph_from_gpu()
    ref = oracle.ed_warp(s.sc["points"], s.sc["nodes"], xg, og["idx"], og["w"], s.sc["R"], s.sc["T"])
    got = pos.cpu().numpy().T
    err = np.linalg.norm(got - ref, axis=1).max() / np.linalg.norm(ref, axis=1).max()
    assert err < 1e-6
    refn = oracle.warp_normals(s.sc["normals"], xg, og["idx"], og["w"], s.sc["R"])
    assert np.abs(nrm.cpu().numpy().T - refn).max() < 1e-5
    # world-frame warp without a pose
    pw, _ = s.M.warp(s.pts, s.nodes, x, s.graph, None, normals=False)
    refw = oracle.ed_warp(s.sc["points"], s.sc["nodes"], xg, og["idx"], og["w"])
    assert np.linalg.norm(pw.cpu().numpy().T - refw, axis=1).max() / np.linalg.norm(refw, axis=1).max() < 1e-6


# ---------------------------------------------------------------- a4-a6: association and normal equations
@pytest.mark.parametrize("name", ["c1", "c2"])
def test_normal_equations_parity(lib, name):
    s = Scene(name)
    xg = random_params(s.m, 12, scale_a=0.005, scale_t=0.3)
    x = torch.tensor(xg, device="cuda")
    nmap = s.M.normal_map(s.depth, s.cam)
    blocks, g, corr, rep = s.M.build_normal_eq(s.pts, s.nodes, x, s.graph, nmap, s.cam, s.pose, s.params, s.ws)
    pos, nrm = s.M.warp(s.pts, s.nodes, x, s.graph, s.pose)
    torch.cuda.synchronize()
    og = s.oracle_graph_from_gpu()
    Nm, ok = oracle.normal_map(s.sc["depth"], s.sc["camera"])
    Nm32 = Nm.astype(np.float32)
    # association on the GPU's own float32 warp: decisions bit-exact
    a = oracle.associate(pos.cpu().numpy().T, nrm.cpu().numpy().T, s.sc["depth"], s.sc["camera"], Nm32, ok,
                         s.params.eps_d, s.params.cos_eps_n)
    cg = corr.cpu().numpy()
    assert np.array_equal(cg, a["corr"])
    assert a["valid"].sum() > 0.3 * s.n
    # normal equations at the same x and correspondences, float64
    pb = s.problem()
    from oracle.gn import evaluate
    vc, nc, asc, e = evaluate(pb, og, xg.astype(np.float64), Nm32, ok, corr_override=cg)
    hb, hg = oracle.block_system(s.sc["points"], s.sc["nodes"], xg.astype(np.float64), og["idx"], og["w"],
                                 s.sc["R"], asc, og["nbrs"], og["row_ptr"], og["col_idx"],
                                 (pb.w_rot, pb.w_reg, pb.w_data))
    nnzb = len(og["col_idx"])
    gb = blocks.cpu().numpy()[:nnzb].astype(np.float64)
    assert rel_err(gb, hb) < 1e-5
    # per-row check on data-dominated rows too
    assert rel_err(g.cpu().numpy(), hg) < 1e-5
    r = s.M.read_report(rep)[0]
    assert r["n_valid"] == a["valid"].sum()
    assert r["e_data"] == pytest.approx(e[0], rel=1e-5)
    assert r["e_rot"] == pytest.approx(e[1], rel=1e-5, abs=1e-9)
    assert r["e_reg"] == pytest.approx(e[2], rel=1e-5, abs=1e-9)


# ---------------------------------------------------------------- a7-a8: block-Jacobi PCG
@pytest.mark.parametrize("name", ["c1", "c2"])
def test_pcg_parity(lib, name):
    s = Scene(name)
    xg = random_params(s.m, 13, scale_a=0.005, scale_t=0.3)
    x = torch.tensor(xg, device="cuda")
    nmap = s.M.normal_map(s.depth, s.cam)
    blocks, g, corr, _ = s.M.build_normal_eq(s.pts, s.nodes, x, s.graph, nmap, s.cam, s.pose, s.params, s.ws)
    delta, rep = s.M.pcg_solve(s.graph, s.m, blocks, g, s.params, s.ws)
    torch.cuda.synchronize()
    og = s.oracle_graph_from_gpu()
    nnzb = len(og["col_idx"])
    hb = blocks.cpu().numpy()[:nnzb].astype(np.float64)
    hg = g.cpu().numpy().astype(np.float64)
    lam = float(np.float32(s.params.lam))
    dx, info = oracle.pcg(og["row_ptr"], og["col_idx"], hb, hg, lam, s.params.pcg_iters)
    r = s.M.read_report(rep)[0]
    assert r["pcg_iters_done"] == info["iters"]
    assert rel_err(delta.cpu().numpy().reshape(-1), dx) < 1e-4
    np.testing.assert_allclose(r["pcg_resid"][:info["iters"] + 1], info["resid"], rtol=1e-3)


# ---------------------------------------------------------------- end to end
def test_gn_register_c1(lib, c1):
    s = c1
    x = s.M.identity_params(s.m)
    rep, ch = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, s.params, s.ws, corr_hist=True)
    torch.cuda.synchronize()
    r = s.M.read_report(rep)
    pb = s.problem()
    og = s.oracle_graph_from_gpu()
    cs = list(ch.cpu().numpy())
    # the first step's decisions are taken at identical float32 inputs: bit-exact
    xo_indep, rep_indep = oracle.gn_register(pb, graph=og, record=True)
    assert np.array_equal(cs[0], rep_indep["iters"][0]["corr"])
    xo, orep = oracle.gn_register(pb, graph=og, corr_sequence=cs)
    xg = x.cpu().numpy().astype(np.float64)
    x0 = oracle.identity_params(s.m)
    print("c1 x rel", rel_err(xg, xo), "delta rel", rel_err(xg - x0, xo - x0))
    assert rel_err(xg, xo) < 1e-4
    assert rel_err(xg - x0, xo - x0) < 1e-3
    for it in range(pb.gn_iters):
        assert r[it]["e_data"] == pytest.approx(orep["iters"][it]["e_data"], rel=1e-4)
        assert r[it]["n_valid"] == orep["iters"][it]["n_valid"]
    assert r[-1]["e_data"] == pytest.approx(orep["final"]["e_data"], rel=1e-3)
    assert r[-1]["flags"] == 0


def test_deterministic(lib, c1):
    s = c1
    outs = []
    for _ in range(2):
        x = s.M.identity_params(s.m)
        rep, _ = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, s.params, s.ws)
        torch.cuda.synchronize()
        outs.append((x.cpu().numpy().copy(), s.M.read_report(rep).tobytes()))
    assert np.array_equal(outs[0][0].view(np.uint32), outs[1][0].view(np.uint32))
    assert outs[0][1] == outs[1][1]
