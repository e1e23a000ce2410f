"""Parity of the fusion step (Alg. 1-2, Eqs.(12), (14), (15)) with the oracle.

The oracle receives the GPU's own float32 world and camera warps, so the
z-buffer winners and the registration decisions are compared bit for bit;
fused positions and normals to float32 rounding.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import Scene, random_params

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_fuse_stagewise(lib, name):
    s = Scene(name)
    rng = np.random.default_rng(5)
    xg = random_params(s.m, 41, 0.003, 0.3)
    x = torch.tensor(xg, device="cuda")
    vw, nw = s.M.warp(s.pts, s.nodes, x, s.graph, None)
    vc, nc = s.M.warp(s.pts, s.nodes, x, s.graph, s.pose)
    w0 = rng.integers(1, 21, s.n).astype(np.float32)
    st0 = rng.integers(0, 5, s.n).astype(np.int32)
    nmap = s.M.normal_map(s.depth, s.cam)
    pts2 = s.pts.clone()
    nodes2 = s.nodes.clone()
    x2 = x.clone()
    w = torch.tensor(w0, device="cuda")
    st = torch.tensor(st0, device="cuda")
    reg, regd = s.M.fuse(pts2, w, st, nodes2, x2, s.graph, nmap, s.cam, s.pose, s.M.fuse_params(7), s.ws,
                         outputs=True)
    torch.cuda.synchronize()
    Nm, ok = oracle.normal_map(s.sc["depth"], s.sc["camera"])
    out = oracle.fuse_warped(vw.cpu().numpy().T, nw.cpu().numpy().T, vc.cpu().numpy().T, nc.cpu().numpy().T,
                             w0, st0, s.sc["depth"], s.sc["camera"], s.sc["R"], s.sc["T"], Nm.astype(np.float32), ok,
                             7)
    assert np.array_equal(reg.cpu().numpy().reshape(-1), out["reg"])
    regg = regd.cpu().numpy().astype(bool)
    assert np.array_equal(regg, out["registered"])
    assert regg.sum() > 0.2 * s.n
    P = pts2.cpu().numpy()
    assert np.abs(P[:3].T - out["points"]).max() <= 2e-5 * np.abs(out["points"]).max()
    assert np.abs(P[3:].T - out["normals"]).max() < 1e-6
    assert np.array_equal(w.cpu().numpy(), out["weight"].astype(np.float32))
    assert np.array_equal(st.cpu().numpy(), out["stamp"])
    # nodes follow their own translation; parameters restart at identity
    assert np.array_equal(nodes2.cpu().numpy(), (s.nodes.cpu().numpy().T + xg[:, 9:12]).T.astype(np.float32))
    assert torch.equal(x2, s.M.identity_params(s.m))


def test_fuse_after_registration_end_to_end(lib):
    """Register then fuse: the fused model lies closer to the observed surface than the unfused one."""
    s = Scene("c2")
    x = s.M.identity_params(s.m)
    s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, s.params, s.ws)
    vw, _ = s.M.warp(s.pts, s.nodes, x, s.graph, None)
    pts2 = s.pts.clone()
    w = torch.full((s.n,), 3.0, device="cuda")
    st = torch.zeros(s.n, dtype=torch.int32, device="cuda")
    nmap = s.M.normal_map(s.depth, s.cam)
    reg, regd = s.M.fuse(pts2, w, st, s.nodes.clone(), x.clone(), s.graph, nmap, s.cam, s.pose,
                         s.M.fuse_params(1), s.ws, outputs=True)
    regg = regd.cpu().numpy().astype(bool)
    gt = s.sc["gt_points"]
    before = np.linalg.norm(vw.cpu().numpy().T[regg] - gt[regg], axis=1)
    after = np.linalg.norm(pts2.cpu().numpy()[:3].T[regg] - gt[regg], axis=1)
    assert regg.sum() > 0.3 * s.n
    # fusion moves registered points a quarter of the way (w = 3) toward the noisy observation
    assert np.all(w.cpu().numpy()[regg] == 4.0) and np.all(st.cpu().numpy()[regg] == 1)
    assert np.isfinite(after).all() and after.mean() < before.mean() + 0.05


def test_fuse_color_matches_oracle(lib):
    """Eq.(13): registered points' colours are the weighted mean of theirs and the frame's colour at the pixel;
    positions, normals, weights and stamps are those of the colourless fusion, bit for bit."""
    import gen
    s = Scene("c2")
    rng = np.random.default_rng(9)
    xg = random_params(s.m, 43, 0.003, 0.3)
    x = torch.tensor(xg, device="cuda")
    vw, nw = s.M.warp(s.pts, s.nodes, x, s.graph, None)
    vc, nc = s.M.warp(s.pts, s.nodes, x, s.graph, s.pose)
    w0 = rng.integers(1, 21, s.n).astype(np.float32)
    st0 = rng.integers(0, 5, s.n).astype(np.int32)
    img = gen.color_image(s.cam.height, s.cam.width, seed=3)
    col0 = gen.point_colors(s.n, seed=4)
    nmap = s.M.normal_map(s.depth, s.cam)
    runs = []
    for with_color in (False, True):
        pts2, nodes2, x2 = s.pts.clone(), s.nodes.clone(), x.clone()
        w = torch.tensor(w0, device="cuda")
        st = torch.tensor(st0, device="cuda")
        col = torch.tensor(np.ascontiguousarray(col0.T), device="cuda")
        kw = dict(image=torch.tensor(img, device="cuda"), color=col) if with_color else {}
        reg, regd = s.M.fuse(pts2, w, st, nodes2, x2, s.graph, nmap, s.cam, s.pose, s.M.fuse_params(7), s.ws,
                             outputs=True, **kw)
        torch.cuda.synchronize()
        runs.append((pts2.cpu().numpy(), w.cpu().numpy(), st.cpu().numpy(), regd.cpu().numpy(), col.cpu().numpy()))
    for a, b in zip(runs[0][:4], runs[1][:4]):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    Nm, ok = oracle.normal_map(s.sc["depth"], s.sc["camera"])
    out = oracle.fuse_warped(vw.cpu().numpy().T, nw.cpu().numpy().T, vc.cpu().numpy().T, nc.cpu().numpy().T,
                             w0, st0, s.sc["depth"], s.sc["camera"], s.sc["R"], s.sc["T"], Nm.astype(np.float32), ok,
                             7, color=col0, image=img)
    regg = runs[1][3].astype(bool)
    assert np.array_equal(regg, out["registered"]) and regg.sum() > 0.2 * s.n
    C = runs[1][4].T
    assert np.abs(C[regg] - out["color"][regg]).max() <= 1e-6
    assert np.array_equal(C[~regg], col0[~regg])
    assert np.abs(C[regg] - col0[regg]).max() > 0.01
