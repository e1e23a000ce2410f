"""Parity of the adaptive Levenberg-Marquardt registration (Sec. II-F) with the oracle.

The GPU run records its correspondences at every step's x and its accept /
reject decisions; the oracle replays both (decision-sync), so the comparison
isolates the arithmetic from float32-vs-float64 association flips and from
near-ties between the two objectives.  Where the oracle's own objectives are
clearly apart, its decision must be the GPU's.
"""
import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import Scene, rel_err
from oracle.lm import LMSchedule, lm_register

pytestmark = pytest.mark.gpu


def _run_lm(s, params, lm, keys=None):
    x = s.M.identity_params(s.m)
    rep, ch = s.M.lm_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, params, s.ws, lm=lm, keys=keys,
                              corr_hist=True)
    torch.cuda.synchronize()
    return x.cpu().numpy(), s.M.read_report(rep), list(ch.cpu().numpy())


def _sched(lm):
    return LMSchedule(lambda0=float(np.float32(lm.lambda0)), up=float(np.float32(lm.up)),
                      down=float(np.float32(lm.down)), lambda_min=float(np.float32(lm.lambda_min)),
                      lambda_max=float(np.float32(lm.lambda_max)))


def _check(s, params, lm, r, xg, cs, pb_kw=None, keys=None):
    G = params.gn_iters
    acc = [bool(v) for v in r["lm_accepted"][:G]]
    pb = s.problem(gn_iters=G, pcg_iters=params.pcg_iters, w_rot=params.w_rot, w_reg=params.w_reg,
                   **(pb_kw or {}))
    og = s.oracle_graph_from_gpu()
    xo, orep = lm_register(pb, _sched(lm), graph=og, decisions=acc, corr_sequence=cs)
    x0 = oracle.identity_params(s.m)
    it = orep["iters"]
    print("decisions", "".join("A" if a else "r" for a in acc), "x rel", rel_err(xg, xo), "delta rel",
          rel_err(xg - x0, xo - x0), "E", [float(v) for v in r["lm_e"][:G]], "lambda",
          [float(v) for v in r["lm_lambda"][:G]])
    assert rel_err(xg, xo) < 1e-5
    assert rel_err(xg - x0, xo - x0) < 1e-4
    for k in range(G):
        assert r[k]["lm_e"] == pytest.approx(it[k]["E"], rel=1e-5)
        assert r[k]["lm_lambda"] == pytest.approx(it[k]["lambda"], rel=1e-5)
        # the GPU's own bookkeeping: the decision follows its objectives; the next step starts at the trial
        # point when the step was taken and at the same x (the same objective, bit for bit) when not
        assert acc[k] == (r[k]["lm_e_trial"] < r[k]["lm_e"])
        if k + 1 < G:
            assert r[k + 1]["lm_e"] == (r[k]["lm_e_trial"] if acc[k] else r[k]["lm_e"])
        # where the oracle's own objectives are clearly apart it decides the same way
        gap = abs(it[k]["E_trial"] - it[k]["E"]) / abs(it[k]["E"])
        if gap > 1e-3:
            assert acc[k] == (it[k]["E_trial"] < it[k]["E"])
    assert np.all(r["flags"][:G] == 0)
    return acc


def test_lm_matches_oracle(lib):
    s = Scene("c2")
    lm = s.M.LMParams()
    xg, r, cs = _run_lm(s, s.params, lm)
    acc = _check(s, s.params, lm, r, xg, cs)
    assert all(acc)   # a well-posed frame: every damped step lowers the objective


def test_lm_rejects_steps_on_an_oscillating_problem(lib):
    """Data term alone with 50 PCG iterations: undamped steps raise the objective now and then; the
    adaptive schedule rejects them and ends below the fixed-damping run."""
    s = Scene("c1")
    params = s.M.Params(sigma=s.params.sigma, gn_iters=6, pcg_iters=50, w_rot=0.0, w_reg=1.0)
    lm = s.M.LMParams()
    xg, r, cs = _run_lm(s, params, lm)
    acc = _check(s, params, lm, r, xg, cs)
    assert any(acc) and not all(acc)
    x = s.M.identity_params(s.m)
    rp, _ = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, params, s.ws)
    rg = s.M.read_report(rp)
    E_fixed = rg[-1]["e_data"] + params.w_reg * rg[-1]["e_reg"]
    E_lm = r[-1]["e_data"] + params.w_reg * r[-1]["e_reg"]
    assert E_lm < E_fixed


def test_unit_schedule_is_the_fixed_damping_registration(lib):
    """up = down = 1 keeps lambda at the fixed damping; when every step is taken the result is that of
    misslam_gn_register bit for bit (the same kernels, the same update x + dx in float32)."""
    s = Scene("c1")
    lm = s.M.LMParams(lambda0=s.params.lam, up=1.0, down=1.0, lambda_min=s.params.lam, lambda_max=s.params.lam)
    xl, rl, _ = _run_lm(s, s.params, lm)
    assert np.all(rl["lm_accepted"][:s.params.gn_iters] == 1)
    x = s.M.identity_params(s.m)
    rp, _ = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, s.params, s.ws)
    rg = s.M.read_report(rp)
    assert np.array_equal(xl.view(np.uint32), x.cpu().numpy().view(np.uint32))
    for f in ("e_data", "e_rot", "e_reg", "n_valid", "pcg_resid"):
        assert np.array_equal(rl[f], rg[f]), f


def test_lm_with_keypoints_matches_oracle(lib):
    s = Scene("c2")
    kp, tgt = gen.keypoints(s.sc, 200, seed=7, noise=0.05)
    keys = s.M.keypoints(torch.tensor(kp, device="cuda"), torch.tensor(tgt, device="cuda").contiguous(), 10.0)
    lm = s.M.LMParams()
    xg, r, cs = _run_lm(s, s.params, lm, keys=keys)
    _check(s, s.params, lm, r, xg, cs, pb_kw=dict(kp_point=kp, kp_target=tgt, w_corr=10.0))
    assert r[-1]["e_corr"] < 0.5 * r[0]["e_corr"]


def test_every_step_rejected_leaves_x_and_raises_lambda(lib):
    """A start whose undamped steps overshoot by orders of magnitude (columns of A at 0.1, rotation weight
    1e5, 60 PCG iterations): every step is rejected, x stays bitwise the start, the objective is the same at
    every step and lambda grows tenfold per step."""
    s = Scene("c1")
    params = s.M.Params(sigma=s.params.sigma, gn_iters=6, pcg_iters=60, w_rot=1e5, w_reg=1.0)
    x = s.M.identity_params(s.m)
    x[:, :9] *= 0.1
    x0 = x.clone()
    rep, _ = s.M.lm_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, params, s.ws, lm=s.M.LMParams())
    torch.cuda.synchronize()
    r = s.M.read_report(rep)
    G = params.gn_iters
    assert np.all(r["lm_accepted"][:G] == 0)
    assert torch.equal(x, x0)
    assert np.all(r["lm_e"][:G] == r["lm_e"][0]) and np.all(r["lm_e_trial"][:G] > 100 * r["lm_e"][:G])
    lam = np.float32(1e-3)
    for k in range(G):
        assert r[k]["lm_lambda"] == lam
        lam = np.float32(min(lam * np.float32(10.0), np.float32(1e6)))
    assert r[-1]["e_data"] == r[0]["e_data"] and r[-1]["e_rot"] == pytest.approx(r[0]["e_rot"], rel=1e-6)


def test_zero_steps(lib):
    """gn_iters = 0: only the final entry, x untouched."""
    s = Scene("c1")
    params = s.M.Params(sigma=s.params.sigma, gn_iters=0, pcg_iters=10)
    x = s.M.identity_params(s.m)
    rep, _ = s.M.lm_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, params, s.ws, lm=s.M.LMParams())
    torch.cuda.synchronize()
    r = s.M.read_report(rep)
    assert len(r) == 1 and torch.equal(x, s.M.identity_params(s.m)) and r[0]["e_data"] > 0
