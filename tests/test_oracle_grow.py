"""Pins of the growth / maintenance oracle (Alg. 2 steps 3-5, Alg. 3) on hand-built cases."""
import numpy as np
import pytest

import oracle

CAM = (4, 3, 10.0, 10.0, 1.5, 1.0)
I3 = np.eye(3, dtype=np.float32)
Z3 = np.zeros(3, dtype=np.float32)


def _frame(depth=50.0):
    D = np.full((3, 4), depth, dtype=np.float32)
    N = np.zeros((3, 4, 3), dtype=np.float32)
    N[..., 2] = -1.0
    return D, N, np.ones((3, 4), dtype=bool)


def _model(n):
    p = np.zeros((n, 3), np.float32)
    nrm = np.tile(np.array([0, 0, -1], np.float32), (n, 1))
    return p, nrm


def test_lift_unregistered_pixels_on_their_rays():
    D, N, ok = _frame()
    D[0, 0] = 0.0                                   # empty pixel: never lifted
    ok[2, 3] = False                                # no normal: never lifted
    p, nrm = _model(2)
    p[:] = [[100, 100, 100], [200, 200, 200]]       # far from each other and from the frame
    reg = np.full(12, -1)
    reg[5] = 0                                      # pixel (u=1, v=1): winner 0, registered
    reg[6] = 1                                      # pixel (u=2, v=1): winner 1, failed the gate
    out = oracle.grow(p, nrm, np.array([5.0, 5.0], np.float32), np.array([7, 7]), np.array([True, False]), reg, D,
                      CAM, I3, Z3, N, ok, 7, np.zeros((0, 3), np.float32), 100.0, voxel=0.22)
    assert out["lifted"] == 12 - 3                  # all but the empty, the normal-less and the registered pixel
    lifted = out["points"][2:]
    # pixel (u=2, v=1) is lifted: D ((u - cx)/fx, (v - cy)/fy, 1) = 50 (0.05, 0, 1)
    pix = [v * 4 + u for v in range(3) for u in range(4) if (v * 4 + u) not in (0, 11, 5)]
    k = pix.index(6)
    np.testing.assert_allclose(lifted[k], [2.5, 0.0, 50.0], rtol=0, atol=1e-6)
    assert np.all(out["weight"][2:] == 1.0) and np.all(out["stamp"][2:] == 7)
    np.testing.assert_allclose(out["normals"][2:], np.tile([0, 0, -1], (9, 1)))


def test_lift_applies_the_inverse_pose():
    D, N, ok = _frame()
    ang = np.deg2rad(30.0)
    R = np.array([[np.cos(ang), 0, np.sin(ang)], [0, 1, 0], [-np.sin(ang), 0, np.cos(ang)]], np.float32)
    T = np.array([1.0, -2.0, 3.0], np.float32)
    out = oracle.grow(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32), np.zeros(0, np.float32),
                      np.zeros(0, int), np.zeros(0, bool), np.full(12, -1), D, CAM, R, T, N, ok, 1,
                      np.zeros((0, 3), np.float32), 100.0, voxel=1e-3)
    V = np.array([50 * (2 - 1.5) / 10, 50 * (1 - 1.0) / 10, 50.0])
    world = np.linalg.solve(R.astype(np.float64), V - T)       # camera = R world + T
    np.testing.assert_allclose(out["points"][6], world, atol=1e-5)
    np.testing.assert_allclose(out["normals"][6], np.linalg.solve(R.astype(np.float64), [0, 0, -1.0]), atol=1e-6)


def test_removal_rule():
    D, N, ok = _frame(0.0)                          # empty frame: nothing lifted
    p, nrm = _model(5)
    p[:] = np.arange(15, dtype=np.float32).reshape(5, 3) * 10.0
    w = np.array([1.5, 2.0, 1.0, 1.0, 0.5], np.float32)
    st = np.array([9, 9, 10, 20, 20])                # frame 20: ages 11, 11, 10, 0, 0
    out = oracle.grow(p, nrm, w, st, np.array([0, 0, 0, 1, 0], bool), np.full(12, -1), D, CAM, I3, Z3, N, ok, 20,
                      np.zeros((0, 3), np.float32), 1000.0, voxel=0.22)
    assert out["culled"] == 1                       # age 11 and weight 1.5 < 2; the rest survive
    np.testing.assert_array_equal(out["points"], p[1:])


def test_voxel_merge_only_in_touched_voxels():
    D, N, ok = _frame(0.0)
    p, nrm = _model(6)
    p[:] = [[0.05, 0.05, 50.01], [0.15, 0.10, 50.02],   # one voxel of 0.22 mm, one point stamped this frame
            [1.05, 0.05, 50.05], [1.10, 0.12, 50.10],   # another voxel, nobody stamped this frame
            [3.00, 3.00, 50.00],                        # alone and stamped
            [0.20, 0.01, 50.03]]                        # joins the first voxel
    nrm[1] = [0.6, 0, -0.8]
    w = np.array([3, 4, 5, 6, 7, 2], np.float32)
    st = np.array([5, 9, 5, 5, 9, 4])
    out = oracle.grow(p, nrm, w, st, np.zeros(6, bool), np.full(12, -1), D, CAM, I3, Z3, N, ok, 9,
                      np.zeros((0, 3), np.float32), 1000.0, voxel=0.22)
    assert out["merged"] == 2 and len(out["points"]) == 4
    m = (p[[0, 1, 5]].astype(np.float64)).mean(axis=0)
    np.testing.assert_allclose(out["points"][0], m, atol=1e-6)
    nm = (nrm[[0, 1, 5]].astype(np.float64)).sum(axis=0)
    np.testing.assert_allclose(out["normals"][0], nm / np.linalg.norm(nm), atol=1e-6)
    assert out["weight"][0] == 4 and out["stamp"][0] == 9
    np.testing.assert_array_equal(out["points"][1:], p[[2, 3, 4]])


def test_colour_follows_lift_merge_and_removal():
    """Survivors keep their colour, lifted points take the pixel's colour, a merged voxel the mean of its
    members', removed points' colours leave with them (Eq.(13) carried through Alg. 2-3)."""
    D, N, ok = _frame()
    ok[:] = False
    ok[1, 2] = True                                 # only pixel (u=2, v=1) can be lifted
    p, nrm = _model(5)
    p[:] = [[0.05, 0.05, 50.01], [0.15, 0.10, 50.02],   # one touched voxel (point 1 stamped this frame)
            [3.0, 3.0, 50.0],                           # alone, kept
            [9.0, 9.0, 50.0],                           # old and light: removed
            [0.20, 0.01, 50.03]]                        # joins the first voxel
    w = np.array([3, 4, 5, 1, 2], np.float32)
    st = np.array([5, 9, 8, -5, 7])
    col = np.array([[0.1, 0.2, 0.3], [0.5, 0.6, 0.7], [0.9, 0.8, 0.7], [0.0, 0.0, 1.0], [0.3, 0.1, 0.2]],
                   np.float32)
    img = np.zeros((3, 4, 3), np.float32)
    img[1, 2] = [0.25, 0.5, 0.75]
    out = oracle.grow(p, nrm, w, st, np.zeros(5, bool), np.full(12, -1), D, CAM, I3, Z3, N, ok, 9,
                      np.zeros((0, 3), np.float32), 1000.0, voxel=0.22, color=col, image=img)
    assert out["culled"] == 1 and out["lifted"] == 1 and out["merged"] == 2
    c = out["color"]
    assert len(c) == len(out["points"]) == 3
    np.testing.assert_allclose(c[0], col[[0, 1, 4]].astype(np.float64).mean(axis=0), atol=1e-7)
    np.testing.assert_array_equal(c[1], col[2])
    np.testing.assert_array_equal(c[2], img[1, 2])


def test_stability_flag():
    """S_i (Sec. II-G, Alg. 3): stable once registered in enough frames (weight >= tau_weight) and from then
    on; removal takes only unstable points older than tau_time; a merged voxel is stable when a member is;
    lifted points start unstable at tau_weight 2 (their weight is 1) and stable at tau_weight 1."""
    D, N, ok = _frame(0.0)                          # empty frame: nothing lifted
    p, nrm = _model(6)
    p[:] = [[0, 0, 50], [10, 0, 50], [20, 0, 50], [30, 0, 50], [40.05, 0.05, 50.01], [40.10, 0.10, 50.02]]
    w = np.array([1.0, 1.0, 3.0, 1.0, 1.0, 5.0], np.float32)
    st = np.array([5, 5, 5, 20, 20, 3])            # frame 20: ages 15, 15, 15, 0, 0, 17
    S0 = np.array([0, 1, 0, 0, 0, 0], bool)
    args = (np.zeros(6, bool), np.full(12, -1), D, CAM, I3, Z3, N, ok, 20, np.zeros((0, 3), np.float32), 1000.0)
    out = oracle.grow(p, nrm, w, st, *args, voxel=0.22, stable=S0)
    # 0: unstable and old: removed.  1: flagged stable: kept, light and old as it is.  2: weight 3 >= 2: stable,
    # kept.  3: unstable but seen this frame: kept, unstable.  4 and 5 share a voxel that 4 touches this frame:
    # merged into 4, stable because 5 (weight 5) is.
    assert out["culled"] == 1 and out["merged"] == 1
    np.testing.assert_array_equal(out["points"][:3], p[[1, 2, 3]])
    np.testing.assert_array_equal(out["stable"], [True, True, False, True])
    # without the flag plane the weight alone decides, which removes point 1 as well
    out_w = oracle.grow(p, nrm, w, st, *args, voxel=0.22)
    assert out_w["culled"] == 2 and "stable" not in out_w
    # with S_i = (weight >= tau_weight) on entry the two agree
    out_s = oracle.grow(p, nrm, w, st, *args, voxel=0.22, stable=w >= 2.0)
    np.testing.assert_array_equal(out_s["points"], out_w["points"])
    D2, N2, ok2 = _frame()
    for tw, want in ((2.0, False), (1.0, True)):
        o2 = oracle.grow(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32), np.zeros(0, np.float32),
                         np.zeros(0, int), np.zeros(0, bool), np.full(12, -1), D2, CAM, I3, Z3, N2, ok2, 1,
                         np.zeros((0, 3), np.float32), 1000.0, voxel=1e-3, tau_weight=tw, stable=np.zeros(0, bool))
        assert o2["lifted"] == 12 and np.all(o2["stable"] == want)


def test_node_regeneration():
    D, N, ok = _frame(0.0)
    p, nrm = _model(4)
    p[:] = [[1.0, 1.0, 50.0], [3.0, 1.0, 50.0],     # a node voxel (s = 5) far from every node
            [21.0, 1.0, 50.0], [22.0, 2.0, 50.0]]   # a voxel whose centroid is within s of node 0
    nodes = np.array([[20.0, 0.0, 50.0]], np.float32)
    out = oracle.grow(p, nrm, np.full(4, 5.0, np.float32), np.full(4, 3), np.zeros(4, bool), np.full(12, -1), D,
                      CAM, I3, Z3, N, ok, 3, nodes, 5.0, voxel=0.22)
    assert out["new_nodes"] == 1
    np.testing.assert_allclose(out["nodes"][0], nodes[0])
    np.testing.assert_allclose(out["nodes"][1], [2.0, 1.0, 50.0], atol=1e-6)


@pytest.mark.parametrize("seed", [0, 1])
def test_merge_and_regeneration_against_brute_force(seed):
    """Random clouds: every output point is the mean of the touched voxel it leads, each untouched point
    survives unchanged, and every new node is at least s from every old node."""
    rng = np.random.default_rng(seed)
    D, N, ok = _frame(0.0)
    n = 400
    p = (rng.uniform(0, 3, (n, 3)) + [0, 0, 50]).astype(np.float32)
    nrm = np.tile(np.array([0, 0, -1], np.float32), (n, 1))
    st = rng.choice([3, 8], n)
    w = np.full(n, 5.0, np.float32)
    nodes = (rng.uniform(0, 3, (3, 3)) + [0, 0, 50]).astype(np.float32)
    out = oracle.grow(p, nrm, w, st, np.zeros(n, bool), np.full(12, -1), D, CAM, I3, Z3, N, ok, 8, nodes, 1.0,
                      voxel=0.4)
    keys = np.floor(p.astype(np.float64) / np.float64(np.float32(0.4))).astype(np.int64)
    expect = []
    for i in range(n):
        same = np.nonzero(np.all(keys == keys[i], axis=1))[0]
        touched = np.any(st[same] == 8)
        if touched and len(same) > 1:
            if same[0] == i:
                expect.append(p[same].astype(np.float64).mean(axis=0))
        else:
            expect.append(p[i].astype(np.float64))
    np.testing.assert_allclose(out["points"], np.array(expect), atol=2e-6)
    new = out["nodes"][3:].astype(np.float64)
    d2 = ((new[:, None, :] - nodes[None, :, :].astype(np.float64)) ** 2).sum(-1)
    assert np.all(d2 >= 1.0 - 1e-9)
    # every node voxel (edge 1) of the final cloud whose centroid is >= 1 from the old nodes gets one
    fin = out["points"].astype(np.float64)
    nk = np.floor(fin).astype(np.int64)
    cents = [fin[np.all(nk == k, axis=1)].mean(axis=0) for k in np.unique(nk, axis=0)]
    far = [c for c in cents if (((c - nodes.astype(np.float64)) ** 2).sum(-1)).min() >= 1.0]
    assert len(far) == out["new_nodes"]
