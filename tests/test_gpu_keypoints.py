"""Parity of the key-point correspondence term (Eq.(9)) on the GPU with the oracle.

The GPU run records its correspondences; the oracle replays them
(decision-sync) with the same key points, so the comparison isolates the
term's arithmetic from float32-vs-float64 association flips.
"""
import dataclasses

import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import Scene, rel_err

pytestmark = pytest.mark.gpu


def _keys(s, count, seed, noise=0.05, w_corr=10.0, extra=None):
    kp, tgt = gen.keypoints(s.sc, count, seed=seed, noise=noise)
    if extra is not None:
        kp = np.concatenate([kp, np.asarray(extra, np.int32)])
        tgt = np.concatenate([tgt, np.zeros((len(extra), 3), np.float32)])
    point = torch.tensor(kp, device="cuda")
    target = torch.tensor(tgt, device="cuda").contiguous()
    return kp, tgt, point, target, s.M.keypoints(point, target, w_corr)


def _run(s, keys=None, params=None):
    x = s.M.identity_params(s.m)
    rep, ch = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, params or s.params, s.ws,
                              corr_hist=True, keys=keys)
    torch.cuda.synchronize()
    return x.cpu().numpy(), s.M.read_report(rep), list(ch.cpu().numpy())


@pytest.mark.parametrize("name,count", [("c1", 40), ("c2", 200)])
def test_keypoint_registration_matches_oracle(lib, name, count):
    s = Scene(name)
    kp, tgt, point, target, keys = _keys(s, count, seed=7)
    xg, r, cs = _run(s, keys)
    pb = s.problem(kp_point=kp, kp_target=tgt, w_corr=10.0)
    og = s.oracle_graph_from_gpu()
    xo, orep = oracle.gn_register(pb, graph=og, corr_sequence=cs)
    x0 = oracle.identity_params(s.m)
    print(name, "x rel", rel_err(xg, xo), "delta rel", rel_err(xg - x0, xo - x0),
          "e_corr", r["e_corr"][[0, -1]].tolist(), [orep["iters"][0]["e_corr"], orep["final"]["e_corr"]])
    assert rel_err(xg, xo) < 1e-5
    assert rel_err(xg - x0, xo - x0) < 1e-4
    # each key-point residual is a difference of ~60 mm float32 positions: a few ulps of 60 mm through the
    # warp, about 1e-5 mm per coordinate, so |dE_corr| <= 2 sqrt(3 S E_corr) 1e-5 + 3 S 1e-10 (S key points)
    for it in range(pb.gn_iters):
        e_it = orep["iters"][it]["e_corr"]
        bound = 2.0 * np.sqrt(3 * count * e_it) * 1e-5 + 3 * count * 1e-10
        assert abs(r[it]["e_corr"] - e_it) <= bound
        assert r[it]["e_data"] == pytest.approx(orep["iters"][it]["e_data"], rel=1e-5)
    assert r[-1]["e_corr"] == pytest.approx(orep["final"]["e_corr"], rel=1e-3)
    assert np.all(r["flags"] == 0)
    # the term pulls the key points toward their matches
    assert r[-1]["e_corr"] < 0.5 * r[0]["e_corr"]


def test_no_keypoints_is_the_plain_registration(lib):
    s = Scene("c1")
    xa, ra, _ = _run(s)
    empty_p = torch.zeros(0, dtype=torch.int32, device="cuda")
    empty_t = torch.zeros((0, 3), dtype=torch.float32, device="cuda")
    xb, rb, _ = _run(s, s.M.keypoints(empty_p, empty_t))
    assert np.array_equal(xa.view(np.uint32), xb.view(np.uint32))
    assert ra.tobytes() == rb.tobytes()


def test_out_of_range_points_are_skipped(lib):
    s = Scene("c1")
    _, _, _, _, keys = _keys(s, 30, seed=3)
    xa, ra, _ = _run(s, keys)
    _, _, _, _, keys2 = _keys(s, 30, seed=3, extra=[-1, s.n, s.n + 7])
    xb, rb, _ = _run(s, keys2)
    assert np.array_equal(xa.view(np.uint32), xb.view(np.uint32))
    assert ra.tobytes() == rb.tobytes()


def test_zero_weight_reports_but_does_not_pull(lib):
    s = Scene("c2")
    _, _, _, _, keys0 = _keys(s, 200, seed=7, w_corr=0.0)
    x0, r0, _ = _run(s)
    xz, rz, _ = _run(s, keys0)
    assert np.array_equal(x0.view(np.uint32), xz.view(np.uint32))   # the term adds exact zeros
    assert rz[0]["e_corr"] > 0
    _, _, _, _, keys = _keys(s, 200, seed=7)
    xk, rk, _ = _run(s, keys)
    assert rk[-1]["e_corr"] < rz[-1]["e_corr"]
