"""Fusion and growth of 640x480 sweep frames against the oracle (Alg. 1-3, Eqs.(12), (14), (15)).

Frame 0 of the sweep lifts the first model on the GPU and in the oracle: counts, stamps and weights bit for
bit, positions and nodes to float32 rounding.  Frame 1 registers the GPU's model on the GPU; the GPU's own
float32 warps of the registered parameters feed the oracle's fusion, whose z-buffer winners and registration
decisions must match bit for bit; the GPU's fused model then feeds both growths, compared as for frame 0.
The 640x480 frame holds 307200 pixels and a model of about 290k points, so every kernel runs at the size of
the sequence.
"""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

SPACING = 2.5


def _compare_growth(counts, P, W, S, G, X, m_before, ref, label):
    counts = counts.cpu().numpy()
    n_out, m_out = int(counts[0]), int(counts[1])
    print(label, "counts", counts.tolist(), "oracle lifted", ref["lifted"], "culled", ref["culled"], "merged",
          ref["merged"], "new nodes", ref["new_nodes"])
    assert counts[2] == ref["lifted"] and counts[3] == ref["culled"] and counts[4] == ref["merged"]
    assert counts[5] == ref["new_nodes"] and counts[6] == 0
    assert n_out == len(ref["points"]) and m_out == len(ref["nodes"])
    Pn, Wn, Sn, Gn, Xn = (t.cpu().numpy() for t in (P, W, S, G, X))
    np.testing.assert_array_equal(Sn[:n_out], ref["stamp"])
    np.testing.assert_array_equal(Wn[:n_out], ref["weight"])
    dp = np.abs(Pn[:3, :n_out].T - ref["points"]).max()
    dn = np.abs(Pn[3:, :n_out].T - ref["normals"]).max()
    print(label, "max |dp|", dp, "max |dn|", dn)
    assert dp <= 1e-5 and dn <= 1e-6
    np.testing.assert_allclose(Gn[:, :m_out].T, ref["nodes"], rtol=0, atol=1e-5)
    ident = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], np.float32)
    assert np.all(Xn[m_before:m_out] == ident)
    return n_out, m_out


def test_sweep_640x480_lift_register_fuse_grow(lib):
    from gen.sequence import Sequence
    from paper_1803_02009_amd import misslam as M
    seq = Sequence()
    d0, d1 = seq.frame(0), seq.frame(1)
    assert d0["depth"].shape == (480, 640)
    cap_n, cap_m = 1_000_000, 8000
    P = torch.zeros((6, cap_n), device="cuda")
    W = torch.zeros(cap_n, device="cuda")
    S = torch.zeros(cap_n, dtype=torch.int32, device="cuda")
    G = torch.zeros((3, cap_m), device="cuda")
    X = torch.zeros((cap_m, 12), device="cuda")
    ws, wsg = M.Workspace(), M.Workspace()
    cam = M.camera(*d0["camera"])

    # frame 0: lift the whole frame into an empty model
    dep0 = torch.tensor(d0["depth"], device="cuda")
    nm0 = M.normal_map(dep0, cam)
    none = torch.full((cam.height, cam.width), -1, dtype=torch.int32, device="cuda")
    counts = M.grow(P, W, S, 0, G, X, 0, none, torch.zeros(1, dtype=torch.int32, device="cuda"), nm0, cam,
                    M.pose(d0["R"], d0["T"]), M.grow_params(0, SPACING), wsg)
    torch.cuda.synchronize()
    Nm0, ok0 = oracle.normal_map(d0["depth"], d0["camera"])
    assert np.array_equal(nm0.cpu().numpy()[..., :3].view(np.uint32), Nm0.astype(np.float32).view(np.uint32))
    e3 = np.zeros((0, 3))
    ref0 = oracle.grow(e3, e3, np.zeros(0), np.zeros(0, np.int64), np.zeros(0, bool), none.cpu().numpy().reshape(-1),
                       d0["depth"], d0["camera"], d0["R"], d0["T"], Nm0.astype(np.float32), ok0, 0, e3, SPACING)
    n, m = _compare_growth(counts, P, W, S, G, X, 0, ref0, "frame 0")
    assert n > 0.9 * cam.width * cam.height and m > 1000

    # frame 1: register the model, then fuse
    params = M.Params(sigma=SPACING, gn_iters=10, pcg_iters=10)
    g = M.build_graph(P[:, :n], G[:, :m], params, ws)
    dep1 = torch.tensor(d1["depth"], device="cuda")
    pose1 = M.pose(d1["R"], d1["T"])
    x = X[:m]
    rep, _ = M.gn_register(P[:, :n], G[:, :m], x, g, dep1, cam, pose1, params, ws)
    r = M.read_report(rep)
    assert np.all(r["flags"] == 0) and r[-1]["e_data"] < r[0]["e_data"]
    vw, nw = M.warp(P[:, :n], G[:, :m], x, g, None)
    vc, nc = M.warp(P[:, :n], G[:, :m], x, g, pose1)
    w0, st0 = W[:n].cpu().numpy().copy(), S[:n].cpu().numpy().copy()
    nodes0, x0 = G[:, :m].cpu().numpy().copy(), x.cpu().numpy().copy()
    nm1 = M.normal_map(dep1, cam)
    reg, regd = M.fuse(P[:, :n], W[:n], S[:n], G[:, :m], x, g, nm1, cam, pose1, M.fuse_params(1), ws, outputs=True)
    torch.cuda.synchronize()
    Nm1, ok1 = oracle.normal_map(d1["depth"], d1["camera"])
    out = oracle.fuse_warped(vw.cpu().numpy().T, nw.cpu().numpy().T, vc.cpu().numpy().T, nc.cpu().numpy().T, w0, st0,
                             d1["depth"], d1["camera"], d1["R"], d1["T"], Nm1.astype(np.float32), ok1, 1)
    assert np.array_equal(reg.cpu().numpy().reshape(-1), out["reg"])
    regg = regd.cpu().numpy().astype(bool)
    assert np.array_equal(regg, out["registered"])
    print("frame 1: n", n, "m", m, "registered", int(regg.sum()), "e_data", r["e_data"][[0, -1]].tolist())
    assert regg.sum() > 0.2 * n
    Pf = P[:, :n].cpu().numpy()
    assert np.abs(Pf[:3].T - out["points"]).max() <= 2e-5 * np.abs(out["points"]).max()
    assert np.abs(Pf[3:].T - out["normals"]).max() < 1e-6
    assert np.array_equal(W[:n].cpu().numpy(), out["weight"].astype(np.float32))
    assert np.array_equal(S[:n].cpu().numpy(), out["stamp"])
    assert np.array_equal(G[:, :m].cpu().numpy(), (nodes0.T + x0[:, 9:12]).T.astype(np.float32))

    # frame 1 growth on the GPU's fused model, in both
    fused = (P[:, :n].cpu().numpy(), W[:n].cpu().numpy(), S[:n].cpu().numpy(), G[:, :m].cpu().numpy())
    counts = M.grow(P, W, S, n, G, X, m, reg, regd, nm1, cam, pose1, M.grow_params(1, SPACING), wsg)
    torch.cuda.synchronize()
    pf, wf, sf, nd = fused
    ref1 = oracle.grow(pf[:3].T, pf[3:].T, wf, sf, regg, reg.cpu().numpy().reshape(-1), d1["depth"], d1["camera"],
                       d1["R"], d1["T"], Nm1.astype(np.float32), ok1, 1, nd.T, SPACING)
    n1, m1 = _compare_growth(counts, P, W, S, G, X, m, ref1, "frame 1")
    assert ref1["lifted"] > 1000 and n1 > n
