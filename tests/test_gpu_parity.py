"""Stage-wise and end-to-end parity of the HIP path (through the C ABI) with the float64 oracle.

Integer outputs (kNN sets, block pattern, node lists, correspondences) must be
bit-exact given the same inputs; float outputs are compared with the error
definitions of the oracle's readings (relative norms), at 1e-5 for float32
unless stated.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from gpu_util import Scene, check_energy, random_params, rel_err

HERE = os.path.dirname(os.path.abspath(__file__))

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


def test_knn_on_a_large_grid(lib):
    """20,000 nodes filling a cube: the node grid has about 57^3 cells, far more than the 4096 that the grid
    kernel sorts in LDS, so its device-memory path builds it.  The kNN sets of sampled points are checked
    against the brute-force oracle, bit for bit."""
    from paper_1803_02009_amd import misslam as M
    rng = np.random.default_rng(11)
    m, n = 20000, 30000
    nodes = rng.uniform(-100.0, 100.0, size=(m, 3)).astype(np.float32)
    pts = rng.uniform(-100.0, 100.0, size=(n, 3)).astype(np.float32)
    nrm = np.tile(np.array([0.0, 0.0, 1.0], np.float32), (n, 1))
    dev = "cuda"
    P = torch.tensor(np.concatenate([pts.T, nrm.T]), device=dev).contiguous()
    G = torch.tensor(np.ascontiguousarray(nodes.T), device=dev).contiguous()
    params = M.Params(sigma=5.0)
    g = M.build_graph(P, G, params, M.Workspace())
    torch.cuda.synchronize()
    # the grid's cell count as the kernel sizes it: well above the LDS path's 4096
    ext = nodes.astype(np.float64).max(0) - nodes.astype(np.float64).min(0)
    e = np.sort(ext)[::-1]
    h = 2.0 * np.sqrt(e[0] * e[1] / m)
    cells = np.prod(np.floor(ext / h) + 1.0)
    while cells > (1 << 18):
        h *= 1.25
        cells = np.prod(np.floor(ext / h) + 1.0)
    assert cells > 4096 * 10
    sample = np.arange(0, n, 60)
    ref_idx, _ = oracle.knn(pts[sample], nodes, params.k)
    idx = g.knn_idx.cpu().numpy().T[sample]
    assert np.array_equal(idx, ref_idx[:, :params.k])


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


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_data_only_normal_equations_per_block(lib, name):
    """The data term alone (w_rot = w_reg = 0): every block of J^T J and every node's slice of J^T r on its own.

    With the regularisers on, their 1e4-scale entries dominate any norm over the whole system, so a small error
    in the data-only entries would hide; here each 12x12 block is compared relative to its own size, and the
    diagonal blocks' damping (lambda) is the only other term."""
    s = Scene(name)
    s.params.w_rot = 0.0
    s.params.w_reg = 0.0
    xg = random_params(s.m, 14, scale_a=0.005, scale_t=0.3)
    x = torch.tensor(xg, device="cuda")
    nmap = s.M.normal_map(s.depth, s.cam)
    blocks, g, corr, rep = s.M.build_normal_eq(s.pts, s.nodes, x, s.graph, nmap, s.cam, s.pose, s.params, s.ws)
    torch.cuda.synchronize()
    og = s.oracle_graph_from_gpu()
    Nm, ok = oracle.normal_map(s.sc["depth"], s.sc["camera"])
    pb = s.problem(w_rot=0.0, w_reg=0.0)
    from oracle.gn import evaluate
    _, _, asc, e = evaluate(pb, og, xg.astype(np.float64), Nm.astype(np.float32), ok, corr_override=corr.cpu().numpy())
    hb, hg = oracle.block_system(s.sc["points"], s.sc["nodes"], xg.astype(np.float64), og["idx"], og["w"],
                                 s.sc["R"], asc, og["nbrs"], og["row_ptr"], og["col_idx"], (0.0, 0.0, pb.w_data))
    nnzb = len(og["col_idx"])
    gb = blocks.cpu().numpy()[:nnzb].astype(np.float64).reshape(nnzb, 144)
    hb = hb.reshape(nnzb, 144)
    norms = np.linalg.norm(hb, axis=1)
    live = norms > 0
    assert live.sum() > 0.5 * nnzb
    err = np.linalg.norm(gb - hb, axis=1)
    worst = float((err[live] / norms[live]).max())
    print(name, "data-only blocks: worst per-block rel err", worst, "over", int(live.sum()), "blocks")
    assert worst < 1e-5
    if np.any(err[~live] != 0.0):   # blocks the oracle leaves at zero
        bad = np.nonzero(~live & (err != 0.0))[0]
        rows = np.searchsorted(og["row_ptr"], bad, side="right") - 1
        print("blocks zero in the oracle but not on the GPU:", [(int(r), int(og["col_idx"][b]),
              float(np.abs(gb[b]).max())) for r, b in zip(rows[:8], bad[:8])], "of", len(bad))
    assert np.all(err[~live] <= 1e-5 * np.median(norms[live]))
    # J^T r per node: its terms carry residuals of both signs, so it is compared against the rounding its
    # float32 residuals carry: r comes from the float32 warp of ~60 mm positions, a few ulps of 60 mm (about
    # 1e-5 mm), times sum_i w_ij |(v_i - g_j, 1)| over the node's valid points (|n'| = 1).
    gg = g.cpu().numpy().astype(np.float64).reshape(s.m, 12)
    hgn = hg.reshape(s.m, 12)
    val = asc["valid"]
    d = np.linalg.norm(np.concatenate([s.sc["points"][:, None, :].astype(np.float64) - s.sc["nodes"][og["idx"]],
                                       np.ones(og["idx"].shape + (1,))], axis=2), axis=2)
    scale = np.bincount(og["idx"][val].ravel(), weights=(og["w"][val] * d[val]).ravel(), minlength=s.m)
    gerr = np.linalg.norm(gg - hgn, axis=1)
    print(name, "data-only J^T r: worst error / (1e-5 |g_j| + 1e-5 mm x scale_j)",
          float((gerr / (1e-5 * np.linalg.norm(hgn, axis=1) + 1e-5 * scale + 1e-30)).max()))
    assert np.all(gerr <= 1e-5 * np.linalg.norm(hgn, axis=1) + 1e-5 * scale)
    r = s.M.read_report(rep)[0]
    assert r["e_data"] == pytest.approx(e[0], rel=1e-5)
    # the report's rotation and regularisation energies are unweighted: still those of x
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
    assert rel_err(delta.cpu().numpy().reshape(-1), dx) < 1e-5
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
    assert rel_err(xg, xo) < 1e-5
    assert rel_err(xg - x0, xo - x0) < 1e-4
    for it in range(pb.gn_iters):
        assert r[it]["e_data"] == pytest.approx(orep["iters"][it]["e_data"], rel=1e-5)
        assert r[it]["n_valid"] == orep["iters"][it]["n_valid"]
    # the final evaluation's decisions are each side's own (not synced)
    check_energy(s, xg, r[-1]["e_data"], xo, orep["final"]["e_data"], label="c1 final")
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


def test_gn_register_c2_against_stored_oracle(lib, c2):
    """The plain float32 form at 320x240 (60,000 points, 400 nodes, 10 x 10) against the float64 oracle run
    of the same seed (tests/golden/c2_oracle.npz), each side taking its own correspondence decisions."""
    s = c2
    gold = np.load(os.path.join(HERE, "golden", "c2_oracle.npz"))
    x = s.M.identity_params(s.m)
    rep, _ = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, s.params, s.ws)
    torch.cuda.synchronize()
    r = s.M.read_report(rep)
    xg = x.cpu().numpy().astype(np.float64)
    xo = gold["x"]
    xi = oracle.identity_params(s.m)
    print("c2 independent: x rel", rel_err(xg, xo), "delta rel", rel_err(xg - xi, xo - xi))
    assert rel_err(xg, xo) < 1e-5
    assert rel_err(xg - xi, xo - xi) < 1e-4
    check_energy(s, xi, r[0]["e_data"], xi, float(gold["e_data"][0]), label="c2 first step")
    check_energy(s, xg, r[-1]["e_data"], xo, float(gold["e_data_final"]), label="c2 final")
    assert np.all(r["flags"] == 0)
