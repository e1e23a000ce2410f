"""Pins of the oracle's adaptive Levenberg-Marquardt schedule (Sec. II-F).

The schedule is pinned on a one-residual textbook problem worked by hand,
on its reduction to the fixed-damping Gauss-Newton loop, on the large-damping
limit (a scaled gradient step, which fixes where lambda enters), and on the
bookkeeping a rejected or taken step must leave on a registration problem
where undamped steps oscillate.
"""
import math

import numpy as np
import pytest

import gen
import oracle
from oracle.gn import linearize
from oracle.lm import LMSchedule, lm_iterate, lm_register, objective


def test_atan_worked_by_hand():
    """r(x) = atan x from x = 2: the Gauss-Newton step overshoots (|x| grows), so the first two damped steps
    are rejected; lambda = 0.1 gives x = 2 - J r / (J^2 + 0.1) with J = 1/5, r = atan 2, which is taken."""
    def lin(x):
        r, J = math.atan(x), 1.0 / (1.0 + x * x)
        return r * r, (r, J)

    def solve(state, lam):
        r, J = state
        return -J * r / (J * J + lam)

    x, log = lm_iterate(2.0, lin, solve, lambda x: math.atan(x) ** 2, LMSchedule(), 6)
    assert [e["accepted"] for e in log] == [False, False, True, True, True, True]
    assert [e["lambda"] for e in log] == pytest.approx([1e-3, 1e-2, 1e-1, 1e-2, 1e-3, 1e-4], rel=1e-12)
    x3 = 2.0 - 0.2 * math.atan(2.0) / (0.04 + 0.1)
    assert log[3]["state"][0] == pytest.approx(math.atan(x3), rel=1e-12)
    assert log[2]["E_trial"] == pytest.approx(math.atan(x3) ** 2, rel=1e-12)
    assert abs(x) < 1e-6


@pytest.fixture(scope="module")
def c1():
    sc = gen.make_scene("c1")
    return sc, oracle.build_graph(sc["points"], sc["nodes"], 4, "gauss", sc["sigma"])


def test_fixed_schedule_taking_every_step_is_gauss_newton(c1):
    sc, g = c1
    pb = oracle.Problem.from_scene(sc, gn_iters=4, pcg_iters=10)
    xg, _ = oracle.gn_register(pb, graph=g)
    xl, rep = lm_register(pb, LMSchedule(lambda0=pb.lam, up=1.0, down=1.0), graph=g, decisions=[True] * 4)
    assert np.array_equal(xg, xl)
    assert all(e["lambda"] == pb.lam for e in rep["iters"])


def test_large_damping_is_a_scaled_gradient_step(c1):
    """(H + lambda I) dx = -g with lambda >> |H| gives dx = -g / lambda up to a relative |H| / lambda (|H| is
    about 1e7 here, so 1e-8 at lambda = 1e15)."""
    sc, g = c1
    lam = 1e15
    pb = oracle.Problem.from_scene(sc, gn_iters=1, pcg_iters=10)
    m = len(sc["nodes"])
    _, rep = lm_register(pb, LMSchedule(lambda0=lam, lambda_max=lam), graph=g, decisions=[True])
    Nmap, Nvalid = oracle.normal_map(pb.depth, pb.camera)
    _, _, _, _, grad, _ = linearize(pb, g, oracle.identity_params(m), Nmap, Nvalid)
    grad = np.asarray(grad).reshape(-1)
    np.testing.assert_allclose(rep["iters"][0]["dx"] * lam, -grad, rtol=0, atol=1e-6 * np.abs(grad).max())


def test_rejected_and_taken_steps_on_an_oscillating_problem(c1):
    """Data term alone (w_rot = 0, w_reg = 1) with 50 PCG iterations: the undamped steps make the objective
    go up and down; the damped loop never lets it rise and ends below the fixed-damping loop."""
    sc, g = c1
    kw = dict(gn_iters=6, pcg_iters=50, w_rot=0.0, w_reg=1.0)
    pb = oracle.Problem.from_scene(sc, **kw)
    sched = LMSchedule()
    x, rep = lm_register(pb, sched, graph=g)
    it = rep["iters"]
    acc = [e["accepted"] for e in it]
    assert not all(acc) and any(acc)
    for k in range(len(it) - 1):
        a, b = it[k], it[k + 1]
        assert a["accepted"] == (a["E_trial"] < a["E"])
        # the next step starts where this one left x: at the trial point if taken, else at the same x
        assert b["E"] == (a["E_trial"] if a["accepted"] else a["E"])
        want = max(a["lambda"] * sched.down, sched.lambda_min) if a["accepted"] else \
            min(a["lambda"] * sched.up, sched.lambda_max)
        assert b["lambda"] == pytest.approx(want, rel=1e-15)
    assert all(b["E"] <= a["E"] for a, b in zip(it, it[1:]))
    assert rep["final"]["E"] == min(it[-1]["E"], it[-1]["E_trial"])
    xg, rg = oracle.gn_register(oracle.Problem.from_scene(sc, **kw), graph=g)
    f = rg["final"]
    assert rep["final"]["E"] < objective(pb, (f["e_data"], f["e_rot"], f["e_reg"], f["e_corr"]))
