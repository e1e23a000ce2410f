"""Pins of the float64 oracle against facts the paper and the mathematics fix.

None of these compares the oracle with itself: each checks a closed form, an
invariant, a brute-force enumeration, a library routine for a special case, a
finite difference, or recovery of a deformation the generator knows
independently.
"""
import itertools
import math

import numpy as np
import pytest

import gen
import oracle
from oracle.energy import reg_residuals
from oracle.fuse import zbuffer


def rot(axis, deg):
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    t = math.radians(deg)
    return np.eye(3) + math.sin(t) * K + (1 - math.cos(t)) * K @ K


def params_from(A, t):
    m = A.shape[0]
    x = np.zeros((m, 12))
    for c in range(3):
        x[:, 3 * c:3 * c + 3] = A[:, :, c]
    x[:, 9:12] = t
    return x


@pytest.fixture(scope="module")
def c1():
    return gen.make_scene("c1")


@pytest.fixture(scope="module")
def c1_graph(c1):
    return oracle.build_graph(c1["points"], c1["nodes"], 4, "gauss", c1["sigma"])


# ---------------------------------------------------------------- P10: kNN by brute force
def test_knn_brute_force_with_ties():
    rng = np.random.default_rng(0)
    nodes = rng.integers(-3, 4, size=(12, 3)).astype(np.float64)   # integer grid: many exact ties
    pts = rng.integers(-3, 4, size=(40, 3)).astype(np.float64) + 0.5 * rng.integers(0, 2, size=(40, 3))
    idx, d2 = oracle.knn(pts, nodes, 4)
    for i, p in enumerate(pts):
        cand = sorted((float(np.sum((p - g) ** 2)), j) for j, g in enumerate(nodes))
        assert [j for _, j in cand[:5]] == list(idx[i])
        assert np.allclose([d for d, _ in cand[:5]], d2[i])


# ---------------------------------------------------------------- Eq.(2) weights
def test_linear_weights_eq2_hand_values():
    # distances 1, 2, 3, 4 to the k=4 nodes and 5 to the fifth: w = 1 - d/5, then normalised
    d2 = np.array([[1.0, 4.0, 9.0, 16.0, 25.0]])
    w = oracle.skin_weights(d2, 4, "linear")
    raw = np.array([0.8, 0.6, 0.4, 0.2])
    assert np.allclose(w[0], raw / raw.sum(), rtol=0, atol=1e-15)
    # all weights zero (fifth node as far as the fourth) falls back to 1/k
    w0 = oracle.skin_weights(np.array([[4.0, 4.0, 4.0, 4.0, 4.0]]), 4, "linear")
    assert np.allclose(w0, 0.25)


def test_gauss_weights_normalised_and_monotone(c1_graph):
    w = c1_graph["w"]
    assert np.allclose(w.sum(axis=1), 1.0, atol=1e-14)
    assert np.all(np.diff(w, axis=1) <= 1e-15)       # nearer nodes weigh more


@pytest.mark.parametrize("sigma", [1.0, 2.5, 6.0])
def test_gauss_weights_hand_values(sigma):
    """Squared distances 0, sigma^2, 4 sigma^2 and 9 sigma^2 give raw weights 1, e^-1/2, e^-2, e^-9/2 (the
    Gaussian of standard deviation sigma).  The decimals are the tabulated values of those exponentials, so a
    weight of exp(-d^2 / sigma^2) (0.3679 at d = sigma) or one without the square fails."""
    e_half, e_2, e_9half = 0.6065306597126334, 0.1353352832366127, 0.011108996538242306
    raw = np.array([1.0, e_half, e_2, e_9half])
    d2 = np.array([[0.0, 1.0, 4.0, 9.0, 16.0]]) * sigma * sigma
    w = oracle.skin_weights(d2, 4, "gauss", sigma)
    assert np.allclose(w[0], raw / 1.7529749395, rtol=0, atol=1e-10)
    assert w[0, 1] / w[0, 0] == pytest.approx(e_half, rel=1e-14)
    # the fifth node's distance plays no part in the Gaussian kind
    w5 = oracle.skin_weights(np.array([[0.0, 1.0, 4.0, 9.0, 1e6]]) * sigma * sigma, 4, "gauss", sigma)
    assert np.array_equal(w, w5)


# ---------------------------------------------------------------- node graph
def test_node_graph_is_symmetric_coinfluence(c1_graph):
    nb = c1_graph["nbrs"]
    m = len(nb)
    idx = c1_graph["idx"]
    pairs = set()
    for row in idx:
        for a, b in itertools.permutations(row, 2):
            pairs.add((int(a), int(b)))
    got = {(j, int(l)) for j in range(m) for l in nb[j]}
    assert got == pairs
    rp, ci = c1_graph["row_ptr"], c1_graph["col_idx"]
    for j in range(m):
        cols = ci[rp[j]:rp[j + 1]]
        assert list(cols) == sorted(set(nb[j]) | {j})


# ---------------------------------------------------------------- P1 rigid reproduction
def test_rigid_field_reproduced_exactly(c1, c1_graph):
    Q = rot([0.3, -0.5, 0.8], 7.0)
    c = np.array([1.5, -0.7, 2.0])
    G = c1["nodes"].astype(np.float64)
    A = np.repeat(Q[None], len(G), axis=0)
    t = G @ Q.T + c - G                                  # (Q - I) g + c
    x = params_from(A, t)
    R = c1["R"].astype(np.float64)
    T = c1["T"].astype(np.float64)
    v = oracle.ed_warp(c1["points"], G, x, c1_graph["idx"], c1_graph["w"], R, T)
    expect = (c1["points"].astype(np.float64) @ Q.T + c) @ R.T + T
    assert np.abs(v - expect).max() < 1e-12
    nrm = oracle.warp_normals(c1["normals"], x, c1_graph["idx"], c1_graph["w"], R)
    en = c1["normals"].astype(np.float64) @ (R @ Q).T
    assert np.abs(nrm - en / np.linalg.norm(en, axis=1, keepdims=True)).max() < 1e-12
    rr, _, _ = reg_residuals(x, G, c1_graph["nbrs"])
    assert np.abs(rr).max() < 1e-12
    assert np.abs(oracle.rot_residuals(x)).max() < 1e-14


@pytest.mark.parametrize("kind", ["stretch", "shear"])
def test_warped_normal_is_normal_to_the_warped_surface(c1, c1_graph, kind):
    """With one non-orthogonal affine map shared by every node the warp of Eq.(1) is that affine map, so the
    warped surface is known by geometry: a tangent step v + h t (t orthogonal to n) lands on the warped
    surface, and the warped normal must be orthogonal to every warped tangent step (and point to the same
    side as the mapped normal).  The warped tangents come from ed_warp itself, not from a retyped formula;
    mapping normals by A (instead of its inverse transpose) tilts them by several degrees here and fails."""
    if kind == "stretch":
        A = np.diag([2.0, 1.0, 0.7])
    else:
        A = np.array([[1.0, 0.6, 0.0], [0.0, 1.0, 0.3], [0.2, 0.0, 1.0]])
    G = c1["nodes"].astype(np.float64)
    c = np.array([0.4, -1.1, 0.8])
    x = params_from(np.repeat(A[None], len(G), axis=0), G @ A.T + c - G)
    P = c1["points"].astype(np.float64)[::7]
    Nn = c1["normals"].astype(np.float64)[::7]
    idx, w = c1_graph["idx"][::7], c1_graph["w"][::7]
    nrm = oracle.warp_normals(Nn, x, idx, w)
    base = oracle.ed_warp(P, G, x, idx, w)
    # two tangent directions per point, orthogonal to its normal
    ref = np.where(np.abs(Nn[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    t1 = np.cross(Nn, ref)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(Nn, t1)
    h = 0.01
    for t in (t1, t2):
        step = oracle.ed_warp(P + h * t, G, x, idx, w) - base
        cosang = np.sum(nrm * step, axis=1) / np.linalg.norm(step, axis=1)
        assert np.abs(cosang).max() < 1e-11
    assert np.all(np.sum(nrm * (Nn @ A.T), axis=1) > 0)
    assert np.allclose(np.linalg.norm(nrm, axis=1), 1.0, atol=1e-14)
    # the mapping by A itself is measurably off the surface normal (the pin discriminates)
    bad = Nn @ A.T
    bad /= np.linalg.norm(bad, axis=1, keepdims=True)
    step = oracle.ed_warp(P + h * t1, G, x, idx, w) - base
    assert np.abs(np.sum(bad * step, axis=1) / np.linalg.norm(step, axis=1)).max() > 0.05


# ---------------------------------------------------------------- P2 identity
def test_identity_params(c1, c1_graph):
    G = c1["nodes"]
    x = oracle.identity_params(len(G))
    R = c1["R"].astype(np.float64)
    T = c1["T"].astype(np.float64)
    v = oracle.ed_warp(c1["points"], G, x, c1_graph["idx"], c1_graph["w"], R, T)
    assert np.abs(v - (c1["points"].astype(np.float64) @ R.T + T)).max() < 1e-12
    e = oracle.energies(x, G, c1_graph["nbrs"], np.zeros(1))
    assert e[1] == 0.0 and e[2] == 0.0


# ---------------------------------------------------------------- P3 closed forms
@pytest.mark.parametrize("s", [0.5, 1.0, 1.3])
def test_rot_closed_form(s):
    x = params_from(np.array([s * np.eye(3)]), np.zeros((1, 3)))
    assert np.sum(oracle.rot_residuals(x) ** 2) == pytest.approx(3 * (s * s - 1) ** 2, abs=1e-15)


def test_rot_hand_example():
    # columns c1 = (1, 1, 0), c2 = (0, 1, 0), c3 = (0, 0, 2): dots 1, 0, 0; norms^2 - 1 = 1, 0, 3
    A = np.array([[1.0, 0, 0], [1.0, 1.0, 0], [0, 0, 2.0]])
    x = params_from(A[None], np.zeros((1, 3)))
    assert np.allclose(oracle.rot_residuals(x)[0], [1, 0, 0, 1, 0, 3])


def test_reg_two_nodes_closed_form():
    G = np.array([[0.0, 0, 0], [4.0, 1.0, -2.0]])
    delta = np.array([0.3, -0.2, 0.7])
    x = oracle.identity_params(2)
    x[0, 9:12] = delta
    nb = [np.array([1]), np.array([0])]
    rr, _, _ = reg_residuals(x, G, nb)
    assert np.sum(rr ** 2) == pytest.approx(2 * np.sum(delta ** 2), rel=1e-14)


# ---------------------------------------------------------------- depth normals
def test_normal_map_planes():
    cam = (32, 24, 30.0, 30.0, 16.0, 12.0)
    N, ok = oracle.normal_map(np.full((24, 32), 50.0), cam)
    assert ok[1:-1, 1:-1].all() and not ok[0].any() and not ok[:, -1].any()
    assert np.abs(N[ok] - [0, 0, -1]).max() < 1e-14
    # tilted plane z = 50 + 0.2 x: depth along each pixel ray
    u, v = np.meshgrid(np.arange(32.0), np.arange(24.0))
    qx = (u - 16) / 30.0
    D = 50.0 / (1 - 0.2 * qx)
    N, ok = oracle.normal_map(D, cam)
    n = np.array([0.2, 0.0, -1.0]) / math.sqrt(1.04)
    assert np.abs(N[ok] - n).max() < 1e-12
    D2 = D.copy()
    D2[10, 10] = 0
    _, ok2 = oracle.normal_map(D2, cam)
    assert not ok2[10, 10] and not ok2[10, 11] and not ok2[11, 10] and not ok2[9, 10] and not ok2[10, 9]


# ---------------------------------------------------------------- association
def test_projection_and_gates_by_hand():
    cam = (8, 6, 10.0, 10.0, 4.0, 3.0)
    D = np.full((6, 8), 20.0)
    N, ok = oracle.normal_map(D, cam)
    # point on the ray of pixel (5, 2) at z = 20.5: residual = -0.5 (normal (0,0,-1))
    u, v = 5, 2
    z = 20.5
    p = np.array([[(u - 4) / 10 * z, (v - 3) / 10 * z, z]])
    n = np.array([[0.0, 0.0, -1.0]])
    a = oracle.associate(p, n, D, cam, N, ok, 15.0, math.cos(math.radians(10)))
    assert a["corr"][0] == v * 8 + u
    assert a["r"][0] == pytest.approx(-0.5, abs=1e-12)
    # normal 11 degrees off fails the angle gate; 9 degrees passes
    for deg, want in [(11.0, False), (9.0, True)]:
        nn = np.array([[math.sin(math.radians(deg)), 0.0, -math.cos(math.radians(deg))]])
        assert oracle.associate(p, nn, D, cam, N, ok, 15.0, math.cos(math.radians(10)))["valid"][0] == want
    # 16 mm away along the ray fails the distance gate; behind the camera and off-image are invalid
    far = p * (36.0 / 20.5)
    assert not oracle.associate(far, n, D, cam, N, ok, 15.0, 0.9)["valid"][0]
    assert not oracle.associate(-p, n, D, cam, N, ok, 15.0, 0.9)["valid"][0]
    off = np.array([[100.0, 0.0, 20.0]])
    assert not oracle.associate(off, n, D, cam, N, ok, 15.0, 0.9)["valid"][0]
    # border pixels have no normal: invalid
    pb_ = np.array([[(0 - 4) / 10 * 20, 0.0, 20.0]])
    assert not oracle.associate(pb_, n, D, cam, N, ok, 15.0, 0.9)["valid"][0]


def test_rounding_to_nearest_pixel():
    cam = (8, 6, 10.0, 10.0, 4.0, 3.0)
    ui, vi, uf, vf, inside = oracle.assoc.project(np.array([[0.049 * 20, 0.051 * 20, 20.0],
                                                           [-0.449 * 20, 0.0, 20.0]]), cam)
    assert list(ui) == [4, 0] and list(vi) == [4, 3]      # 4.49 -> 4, 3.51 -> 4, -0.49 -> 0
    assert inside.all()


# ---------------------------------------------------------------- P5/P11 Jacobians and gradient
def _fixed_setup(c1, c1_graph, seed=5):
    rng = np.random.default_rng(seed)
    G = c1["nodes"].astype(np.float64)
    m = len(G)
    x = oracle.identity_params(m) + rng.normal(scale=0.02, size=(m, 12))
    x[:, 9:12] = rng.normal(scale=0.3, size=(m, 3))
    R = c1["R"].astype(np.float64)
    T = c1["T"].astype(np.float64)
    vc = oracle.ed_warp(c1["points"], G, x, c1_graph["idx"], c1_graph["w"], R, T)
    nc = oracle.warp_normals(c1["normals"], x, c1_graph["idx"], c1_graph["w"], R)
    Nm, ok = oracle.normal_map(c1["depth"], c1["camera"])
    a = oracle.associate(vc, nc, c1["depth"], c1["camera"], Nm, ok, 15.0, math.cos(math.radians(10)))
    return x, R, T, a


def test_gradient_params_matches_central_fd(c1, c1_graph):
    x, R, T, a = _fixed_setup(c1, c1_graph)
    G = c1["nodes"]
    wts = (1000.0, 10000.0, 1.0)
    args = (c1["points"], G, c1_graph["nbrs"], c1_graph["idx"], c1["sigma"], R, T, a["V"], a["Np"], a["valid"], wts)
    grad = oracle.energy_grad_params(x, c1["points"], G, c1_graph["nbrs"], c1_graph["idx"], c1_graph["w"], R,
                                     a["r"], a["Np"], a["valid"], wts)
    rng = np.random.default_rng(7)
    h = 1e-5
    for flat in rng.choice(x.size, 40, replace=False):
        j, e = divmod(int(flat), 12)
        xp = x.copy(); xp[j, e] += h
        xm = x.copy(); xm[j, e] -= h
        fd = (oracle.total_energy_fixed(xp, *args) - oracle.total_energy_fixed(xm, *args)) / (2 * h)
        assert fd == pytest.approx(grad[j, e], rel=1e-5, abs=1e-4)


def test_normal_equations_gradient_is_half_energy_gradient(c1, c1_graph):
    x, R, T, a = _fixed_setup(c1, c1_graph, seed=6)
    G = c1["nodes"]
    wts = (1000.0, 10000.0, 1.0)
    _, g = oracle.block_system(c1["points"], G, x, c1_graph["idx"], c1_graph["w"], R, a, c1_graph["nbrs"],
                               c1_graph["row_ptr"], c1_graph["col_idx"], wts)
    args = (c1["points"], G, c1_graph["nbrs"], c1_graph["idx"], c1["sigma"], R, T, a["V"], a["Np"], a["valid"], wts)
    h = 1e-5
    for j, e in [(0, 0), (5, 9), (17, 4), (30, 11), (47, 7)]:
        xp = x.copy(); xp[j, e] += h
        xm = x.copy(); xm[j, e] -= h
        fd = (oracle.total_energy_fixed(xp, *args) - oracle.total_energy_fixed(xm, *args)) / (2 * h)
        assert 2 * g[j, e] == pytest.approx(fd, rel=1e-5, abs=1e-4)


def test_data_jacobian_rows_match_fd(c1, c1_graph):
    x, R, T, a = _fixed_setup(c1, c1_graph, seed=8)
    G = c1["nodes"]
    idx = c1_graph["idx"]
    sel = np.nonzero(a["valid"])[0][:25]
    J = oracle.data_jacobian_rows(c1["points"][sel], G, idx[sel], c1_graph["w"][sel], R, a["Np"][sel])
    h = 1e-6
    for q, i in enumerate(sel[:6]):
        for s in range(4):
            j = idx[i, s]
            for e in range(12):
                xp = x.copy(); xp[j, e] += h
                xm = x.copy(); xm[j, e] -= h
                rp = a["Np"][i] @ (oracle.ed_warp(c1["points"][i:i + 1], G, xp, idx[i:i + 1], c1_graph["w"][i:i + 1], R, T)[0] - a["V"][i])
                rm = a["Np"][i] @ (oracle.ed_warp(c1["points"][i:i + 1], G, xm, idx[i:i + 1], c1_graph["w"][i:i + 1], R, T)[0] - a["V"][i])
                assert (rp - rm) / (2 * h) == pytest.approx(J[q, s, e], abs=1e-7)


def test_gradient_points_matches_central_fd(c1, c1_graph):
    x, R, T, a = _fixed_setup(c1, c1_graph, seed=9)
    G = c1["nodes"]
    idx = c1_graph["idx"]
    wts = (0.0, 0.0, 1.0)     # E_rot and E_reg do not depend on the points; leaving them out keeps FD clean
    gp = oracle.energy_grad_points(x, c1["points"], G, idx, c1["sigma"], R, a["r"], a["Np"], a["valid"], 1.0)
    P = c1["points"].astype(np.float64)
    sel = np.nonzero(a["valid"])[0][::97][:20]
    h = 1e-5
    for i in sel:
        for c in range(3):
            Pp = P.copy(); Pp[i, c] += h
            Pm = P.copy(); Pm[i, c] -= h
            ep = oracle.total_energy_fixed(x, Pp, G, c1_graph["nbrs"], idx, c1["sigma"], R, T, a["V"], a["Np"], a["valid"], wts)
            em = oracle.total_energy_fixed(x, Pm, G, c1_graph["nbrs"], idx, c1["sigma"], R, T, a["V"], a["Np"], a["valid"], wts)
            assert (ep - em) / (2 * h) == pytest.approx(gp[i, c], rel=1e-5, abs=1e-6)


# ---------------------------------------------------------------- P6 assembly
def test_bsr_assembly_equals_dense_jtwj(c1, c1_graph):
    x, R, T, a = _fixed_setup(c1, c1_graph, seed=10)
    G = c1["nodes"]
    wts = (1000.0, 10000.0, 1.0)
    J, wd, r, H, g = oracle.dense_system(c1["points"], G, x, c1_graph["idx"], c1_graph["w"], R, a,
                                         c1_graph["nbrs"], wts)
    blocks, gb = oracle.block_system(c1["points"], G, x, c1_graph["idx"], c1_graph["w"], R, a, c1_graph["nbrs"],
                                     c1_graph["row_ptr"], c1_graph["col_idx"], wts)
    Hb = oracle.dense_from_blocks(c1_graph["row_ptr"], c1_graph["col_idx"], blocks, len(G))
    assert np.abs(Hb - H).max() <= 1e-9 * np.abs(H).max()
    assert np.abs(gb.reshape(-1) - g).max() <= 1e-9 * np.abs(g).max()
    # no mass outside the pattern
    assert np.allclose(H, H.T, atol=1e-9 * np.abs(H).max())


# ---------------------------------------------------------------- P7 PCG
def test_pcg_matches_cholesky(c1, c1_graph):
    x, R, T, a = _fixed_setup(c1, c1_graph, seed=11)
    G = c1["nodes"]
    wts = (1.0, 1.0, 1.0)             # moderate conditioning so full-length CG converges in float64
    blocks, g = oracle.block_system(c1["points"], G, x, c1_graph["idx"], c1_graph["w"], R, a, c1_graph["nbrs"],
                                    c1_graph["row_ptr"], c1_graph["col_idx"], wts)
    H = oracle.dense_from_blocks(c1_graph["row_ptr"], c1_graph["col_idx"], blocks, len(G))
    ref = oracle.cholesky_solve(H, g, 1e-3)
    dx, info = oracle.pcg(c1_graph["row_ptr"], c1_graph["col_idx"], blocks, g, 1e-3, 12 * len(G))
    assert np.linalg.norm(dx - ref) <= 1e-10 * np.linalg.norm(ref)
    assert not info["breakdown"]


def test_pcg_block_diagonal_exact_in_one_step():
    rng = np.random.default_rng(3)
    m = 5
    blocks = []
    for _ in range(m):
        B = rng.normal(size=(12, 12))
        blocks.append(B @ B.T + 12 * np.eye(12))
    blocks = np.array(blocks)
    row_ptr = np.arange(m + 1)
    col_idx = np.arange(m)
    g = rng.normal(size=12 * m)
    dx, info = oracle.pcg(row_ptr, col_idx, blocks, g, 0.5, 1)
    ref = np.concatenate([np.linalg.solve(blocks[j] + 0.5 * np.eye(12), -g[12 * j:12 * j + 12]) for j in range(m)])
    assert np.abs(dx - ref).max() < 1e-12


def test_pcg_zero_rhs_returns_zero():
    blocks = np.array([np.eye(12)])
    dx, info = oracle.pcg(np.array([0, 1]), np.array([0]), blocks, np.zeros(12), 1e-3, 10)
    assert np.all(dx == 0) and info["iters"] == 0


# ---------------------------------------------------------------- P4 plane target
def test_plane_translation_recovered_in_one_step():
    sc = gen.plane_scene(k_shift=0.8)
    pb = oracle.Problem.from_scene(sc, lam=1e-12, gn_iters=1, pcg_iters=400)
    x, rep = oracle.gn_register(pb)
    assert rep["iters"][0]["n_valid"] == len(sc["points"])
    shift = float(np.float32(50.8)) - 50.0      # the model plane sits at float32(z0 + 0.8)
    assert np.abs(x[:, 9:12] - [0.0, 0.0, -shift]).max() < 1e-9
    assert np.abs(x[:, :9] - oracle.identity_params(9)[:, :9]).max() < 1e-8
    assert rep["final"]["e_data"] < 1e-14


# ---------------------------------------------------------------- P8 recovery of a known field
def test_gn_recovers_known_rigid_field():
    """Noise-free depth of a rigidly moved surface (2 deg, 1 mm): the minimum of Eq.(3)
    is the rigid field itself, up to the pixel discretisation of the point-to-plane
    residual (curvature x footprint^2 / 2 ~ 6 um at 1 mm pixels on this surface)."""
    sc = gen.make_scene("c1", noise_sigma=0.0, deformation="rigid")
    pb = oracle.Problem.from_scene(sc, gn_iters=6, pcg_iters=600)
    x, rep = oracle.gn_register(pb)
    g = rep["graph"]
    vw = oracle.ed_warp(pb.points, pb.nodes, x, g["idx"], g["w"])
    err = np.linalg.norm(vw - sc["gt_points"], axis=1)
    vis = rep["final"]["corr"] >= 0
    assert vis.sum() > 0.8 * len(err)
    assert err[vis].max() < 0.01
    assert err.max() < 0.01


def test_gn_tracks_smooth_field_to_noise_level(c1):
    """Noisy C1: the data residual falls to the depth-noise level (sigma = 0.2 mm)."""
    pb = oracle.Problem.from_scene(c1)
    x, rep = oracle.gn_register(pb)
    n = rep["final"]["n_valid"]
    assert math.sqrt(rep["final"]["e_data"] / n) < 0.25
    assert rep["final"]["e_data"] < 0.7 * rep["iters"][0]["e_data"]


# ---------------------------------------------------------------- P9 fusion
def test_fusion_weighted_average_on_ray():
    cam = (16, 12, 20.0, 20.0, 8.0, 6.0)
    D = np.full((12, 16), 61.0)
    Nm, ok = oracle.normal_map(D, cam)
    u, v = 9, 7
    p = np.array([[(u - 8) / 20 * 60.0, (v - 6) / 20 * 60.0, 60.0]])
    n = np.array([[0.0, 0.0, -1.0]])
    G = p.copy()
    x = oracle.identity_params(1)
    idx = np.zeros((1, 1), dtype=np.int64)
    w = np.ones((1, 1))
    out = oracle.fuse(p, n, np.array([3.0]), np.array([0]), G, x, idx, w, D, cam, np.eye(3), np.zeros(3), Nm, ok,
                      frame=7)
    assert out["registered"][0]
    assert out["points"][0, 2] == pytest.approx(60.25, abs=1e-12)
    # stays on the ray
    assert out["points"][0, 0] / out["points"][0, 2] == pytest.approx((u - 8) / 20, abs=1e-12)
    assert out["weight"][0] == 4.0 and out["stamp"][0] == 7
    out2 = oracle.fuse(p, n, np.array([20.0]), np.array([0]), G, x, idx, w, D, cam, np.eye(3), np.zeros(3), Nm, ok,
                       frame=8)
    assert out2["weight"][0] == 20.0                    # w_max cap
    # 11 mm away: not registered (tau = 10 mm)
    D3 = np.full((12, 16), 71.5)
    Nm3, ok3 = oracle.normal_map(D3, cam)
    out3 = oracle.fuse(p, n, np.array([3.0]), np.array([0]), G, x, idx, w, D3, cam, np.eye(3), np.zeros(3), Nm3,
                       ok3, frame=9)
    assert not out3["registered"][0] and out3["weight"][0] == 3.0 and out3["points"][0, 2] == 60.0


def test_color_fusion_telescopes_to_the_observation():
    """Eq.(13) on one point seen n times with the same colour I from weight w0 (below the cap): the recursion
    c <- (w c + I)/(w + 1), w <- w + 1 telescopes to c_n = I + (c_0 - I) w0 / (w0 + n); an unregistered point
    keeps its colour, and a constant colour is a fixed point."""
    cam = (16, 12, 20.0, 20.0, 8.0, 6.0)
    D = np.full((12, 16), 61.0)
    Nm, ok = oracle.normal_map(D, cam)
    u, v = 9, 7
    p = np.array([[(u - 8) / 20 * 60.0, (v - 6) / 20 * 60.0, 60.0]])
    nrm = np.array([[0.0, 0.0, -1.0]])
    x = oracle.identity_params(1)
    idx = np.zeros((1, 1), dtype=np.int64)
    wk = np.ones((1, 1))
    I = np.zeros((12, 16, 3))
    I[v, u] = [0.9, 0.2, 0.5]
    c0 = np.array([[0.1, 0.7, 0.5]])
    w0 = 2.0
    c, w, pts = c0.copy(), np.array([w0]), p.copy()
    for it in range(5):
        out = oracle.fuse(pts, nrm, w, np.array([0]), pts.copy(), x, idx, wk, D, cam, np.eye(3), np.zeros(3), Nm,
                          ok, frame=it, color=c, image=I)
        assert out["registered"][0]
        c, w, pts = out["color"], out["weight"], out["points"]
    want = I[v, u] + (c0[0] - I[v, u]) * w0 / (w0 + 5)
    np.testing.assert_allclose(c[0], want, rtol=0, atol=1e-14)
    assert c[0, 2] == 0.5
    D3 = np.full((12, 16), 71.5)
    Nm3, ok3 = oracle.normal_map(D3, cam)
    out3 = oracle.fuse(p, nrm, np.array([3.0]), np.array([0]), p.copy(), x, idx, wk, D3, cam, np.eye(3), np.zeros(3),
                       Nm3, ok3, frame=9, color=c0, image=I)
    assert not out3["registered"][0] and np.array_equal(out3["color"], c0)


def test_zbuffer_nearest_then_lowest_index():
    vc = np.array([[0, 0, 5.0], [0, 0, 4.0], [0, 0, 4.0], [0, 0, 9.0]])
    ui = np.array([1, 1, 1, 2])
    vi = np.array([0, 0, 0, 0])
    win = zbuffer(vc, np.ones(4, bool), ui, vi, 3, 1)
    assert list(win) == [-1, 1, 3]


# ---------------------------------------------------------------- bf16 / fp16 rounding
def test_low_precision_rounding():
    one = 1.0
    ulp = 2.0 ** -7
    assert oracle.round_bf16(one + ulp / 2)[()] == one                 # tie to even (down)
    assert oracle.round_bf16(one + 3 * ulp / 2)[()] == one + 2 * ulp  # tie to even (up)
    assert oracle.round_bf16(one + ulp * 0.51)[()] == one + ulp
    assert oracle.round_fp16(one + 2.0 ** -11)[()] == one
    assert oracle.round_fp16(65519.0)[()] == 65504.0
