"""Pins of the oracle's key-point correspondence term (Eq.(9)).

Checked against central differences of the residual, the closed form a pure
translation gives, the structure orthonormality of R forces on J^T J, the
explicit dense rows, and recovery of a known translation by the whole
Gauss-Newton loop.
"""
import math

import numpy as np
import pytest

import gen
import oracle
from oracle.corr import corr_energy, corr_jacobian_rows, corr_residuals


def rot(axis, deg):
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    t = math.radians(deg)
    return np.eye(3) + math.sin(t) * K + (1 - math.cos(t)) * K @ K


@pytest.fixture(scope="module")
def c1():
    sc = gen.make_scene("c1")
    g = oracle.build_graph(sc["points"], sc["nodes"], 4, "gauss", sc["sigma"])
    return sc, g


def _random_params(m, seed):
    rng = np.random.default_rng(seed)
    x = oracle.identity_params(m)
    x[:, :9] += rng.normal(scale=0.05, size=(m, 9))
    x[:, 9:] = rng.normal(scale=0.7, size=(m, 3))
    return x


def test_jacobian_matches_central_differences(c1):
    sc, g = c1
    m = len(sc["nodes"])
    x = _random_params(m, 3)
    R, T = rot([1, 2, 3], 12.0), np.array([3.0, -2.0, 5.0])
    kp, tgt = gen.keypoints(sc, 25, seed=1, noise=0.3)
    J = corr_jacobian_rows(sc["points"], sc["nodes"], g["idx"], g["w"], R, kp)
    h = 1e-6
    for s in (0, 7, 19):
        for q in range(4):
            j = g["idx"][kp[s], q]
            for e in (0, 4, 8, 9, 11):
                xp, xm = x.copy(), x.copy()
                xp[j, e] += h
                xm[j, e] -= h
                fd = (corr_residuals(sc["points"], sc["nodes"], xp, g["idx"], g["w"], R, T, kp[s:s + 1], tgt[s:s + 1])
                      - corr_residuals(sc["points"], sc["nodes"], xm, g["idx"], g["w"], R, T, kp[s:s + 1],
                                       tgt[s:s + 1]))[0] / (2 * h)
                np.testing.assert_allclose(J[s, :, q, e], fd, rtol=0, atol=1e-7)


def test_translation_closed_form(c1):
    sc, g = c1
    m = len(sc["nodes"])
    d = np.array([0.4, -1.1, 2.5])
    x = oracle.identity_params(m)
    x[:, 9:12] = d                       # every node translated: the warp is v + d (weights sum to 1)
    kp = np.arange(0, len(sc["points"]), 97)
    P = sc["points"].astype(np.float64)
    r = corr_residuals(sc["points"], sc["nodes"], x, g["idx"], g["w"], np.eye(3), np.zeros(3), kp, P[kp] + d)
    assert np.abs(r).max() < 1e-12
    r2 = corr_residuals(sc["points"], sc["nodes"], x, g["idx"], g["w"], np.eye(3), np.zeros(3), kp, P[kp])
    np.testing.assert_allclose(r2, np.broadcast_to(d, r2.shape), atol=1e-12)
    assert corr_energy(r2) == pytest.approx(len(kp) * float(d @ d), rel=1e-12)


def test_gauss_newton_block_is_kron_with_identity(c1):
    """R orthonormal: sum over the 3 rows of J_j^T J_l = w_j w_l (d_j d_l^T) (x) I3."""
    sc, g = c1
    R = rot([0.3, -1, 0.5], 33.0)
    kp = np.array([5, 120, 777])
    J = corr_jacobian_rows(sc["points"], sc["nodes"], g["idx"], g["w"], R, kp)
    P = sc["points"].astype(np.float64)
    G = sc["nodes"].astype(np.float64)
    for s, p in enumerate(kp):
        for a in range(4):
            for b in range(4):
                ja, jb = g["idx"][p, a], g["idx"][p, b]
                da = np.append(P[p] - G[ja], 1.0)
                db = np.append(P[p] - G[jb], 1.0)
                blk = sum(np.outer(J[s, r, a], J[s, r, b]) for r in range(3))
                want = g["w"][p, a] * g["w"][p, b] * np.kron(np.outer(da, db), np.eye(3))
                np.testing.assert_allclose(blk, want, rtol=0, atol=1e-10)


def test_block_system_matches_explicit_rows(c1):
    sc, g = c1
    m = len(sc["nodes"])
    x = _random_params(m, 5)
    R, T = rot([2, 1, 0], 7.0), np.array([1.0, 0.5, -2.0])
    kp, tgt = gen.keypoints(sc, 40, seed=2, noise=0.5)
    rc = corr_residuals(sc["points"], sc["nodes"], x, g["idx"], g["w"], R, T, kp, tgt)
    corr = {"point": kp, "r": rc, "w_corr": 10.0}
    asc = {"valid": np.zeros(len(sc["points"]), bool), "r": np.zeros(len(sc["points"])),
           "Np": np.zeros((len(sc["points"]), 3))}
    w = (0.0, 0.0, 0.0)
    _, _, _, H, gd = oracle.dense_system(sc["points"], sc["nodes"], x, g["idx"], g["w"], R, asc, g["nbrs"], w,
                                         corr)
    blocks, gb = oracle.block_system(sc["points"], sc["nodes"], x, g["idx"], g["w"], R, asc, g["nbrs"],
                                     g["row_ptr"], g["col_idx"], w, None, corr)
    Hb = oracle.dense_from_blocks(g["row_ptr"], g["col_idx"], blocks, m)
    np.testing.assert_allclose(Hb, H, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(gb.reshape(-1), gd, rtol=1e-12, atol=1e-9)
    assert np.abs(H).max() > 1.0


def test_gauss_newton_recovers_translation_from_key_points():
    """Only key points constrain the data (w_data = 0): targets are the model points shifted by d, so the
    optimum is every node translated by d with A = I (all terms zero); GN must reach it."""
    sc = gen.make_scene("c1")
    d = np.array([0.6, -0.4, 1.2])
    kp = np.arange(0, len(sc["points"]), 11).astype(np.int32)
    R, T = sc["R"].astype(np.float64), sc["T"].astype(np.float64)
    # targets in camera coordinates: the translated canonical point under the pose
    tgt = ((sc["points"][kp].astype(np.float64) + d) @ R.T + T).astype(np.float32)
    pb = oracle.Problem.from_scene(sc, w_data=0.0, kp_point=kp, kp_target=tgt, gn_iters=6, pcg_iters=60)
    x, rep = oracle.gn_register(pb)
    e0, e1 = rep["iters"][0]["e_corr"], rep["final"]["e_corr"]
    assert e0 > 1.0 and e1 < 1e-6 * e0
    np.testing.assert_allclose(x[:, 9:12], np.broadcast_to(d, (len(x), 3)), atol=1e-3)
    np.testing.assert_allclose(x[:, :9], oracle.identity_params(len(x))[:, :9], atol=1e-3)
