"""Device-side failure handling of the registration, forced from the host.

- Solve timeouts: a spin limit of one poll per wait makes the one-launch solves give up their waits (every
  kernel still exits normally).  A step whose solve timed out is discarded as a whole: the parameters (and the
  pose) keep every bit, in the fixed, joint, adaptive-damping, low-precision and batched forms.
- Non-finite values: a NaN parameter makes every step's update non-finite; each step is discarded.
- Non-finite depth (NaN, +inf) is no measurement: the normal map, decisions and result follow the oracle.
- FRAME_REJECT is set exactly when the mean |r| exceeds the threshold, and changes nothing else.
- A graph overflow found at setup reaches every report entry of the registration.
"""
import dataclasses

import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import Scene, rel_err

pytestmark = pytest.mark.gpu
TIMEOUT = 0x20
NONFINITE = 0x4
FRAME_REJECT = 0x8
GRAPH_OVERFLOW = 0x10


def _bits(a):
    return np.asarray(a, np.float32).view(np.uint32)


def _spin(s, **kw):
    return dataclasses.replace(s.params, sync_spin_limit=1, **kw)


@pytest.fixture(scope="module")
def c2(lib):
    s = Scene("c2")
    _ = s.graph
    return s


@pytest.mark.parametrize("form", [0, 1])   # textbook, pipelined
def test_timeout_discards_the_whole_step(c2, form):
    s = c2
    one = dataclasses.replace(s.params, gn_iters=1, solve_form=form)
    x_ok = s.M.identity_params(s.m)
    s.M.gn_register(s.pts, s.nodes, x_ok, s.graph, s.depth, s.cam, s.pose, one, s.ws)
    timed_out = 0
    for _ in range(3):
        x = s.M.identity_params(s.m)
        rep, _ = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose,
                                 _spin(s, gn_iters=1, solve_form=form), s.ws)
        torch.cuda.synchronize()
        f = int(s.M.read_report(rep)[0]["flags"])
        want = s.M.identity_params(s.m) if f & TIMEOUT else x_ok
        assert np.array_equal(_bits(x.cpu()), _bits(want.cpu())), f
        timed_out += bool(f & TIMEOUT)
    print("fixed form: steps timed out", timed_out, "of 3")
    assert timed_out > 0


def test_timeout_discards_joint_step_and_pose(c2):
    s = c2
    timed_out = 0
    P0 = np.concatenate([np.asarray(s.sc["R"], np.float32).reshape(9), np.asarray(s.sc["T"], np.float32)])
    for _ in range(3):
        x = s.M.identity_params(s.m)
        rep, pose, _ = s.M.joint_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose,
                                          _spin(s, gn_iters=1), s.ws)
        torch.cuda.synchronize()
        f = int(s.M.read_report(rep)[0]["flags"])
        if f & TIMEOUT:
            timed_out += 1
            assert np.array_equal(_bits(x.cpu()), _bits(s.M.identity_params(s.m).cpu()))
            assert np.array_equal(_bits(pose.cpu()), _bits(P0))
    print("joint form: steps timed out", timed_out, "of 3")
    assert timed_out > 0


def test_timeout_rejects_the_lm_step(c2):
    s = c2
    G = 3
    x = s.M.identity_params(s.m)
    rep, _ = s.M.lm_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, _spin(s, gn_iters=G), s.ws,
                             lm=s.M.LMParams())
    torch.cuda.synchronize()
    r = s.M.read_report(rep)
    flags = [int(v) for v in r["flags"][:G]]
    print("adaptive damping: step flags", flags, "accepted", list(r["lm_accepted"][:G]))
    assert any(f & TIMEOUT for f in flags)
    for k in range(G):
        if flags[k] & TIMEOUT:
            assert r[k]["lm_accepted"] == 0
    if all(f & TIMEOUT for f in flags):
        assert np.array_equal(_bits(x.cpu()), _bits(s.M.identity_params(s.m).cpu()))


@pytest.mark.parametrize("refine", [0, 2])
def test_timeout_discards_low_precision_step(c2, refine):
    s = c2
    timed_out = 0
    for _ in range(3):
        x = s.M.identity_params(s.m)
        p = _spin(s, gn_iters=1, precision=1, refine_steps=refine)
        rep, _ = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, p, s.ws)
        torch.cuda.synchronize()
        f = int(s.M.read_report(rep)[0]["flags"])
        if f & TIMEOUT:
            timed_out += 1
            assert np.array_equal(_bits(x.cpu()), _bits(s.M.identity_params(s.m).cpu()))
    print("bf16 form, refine", refine, ": steps timed out", timed_out, "of 3")
    assert timed_out > 0


def test_timeout_discards_batched_steps(lib):
    probs = [Scene(gen.make_scene(gen.batch_spec(b))) for b in (4, 15)]
    M = probs[0].M
    items = [dict(points=s.pts, nodes=s.nodes, x=M.identity_params(s.m), graph=s.graph, depth=s.depth, cam=s.cam,
                  pose=s.pose) for s in probs]
    p = dataclasses.replace(probs[0].params, gn_iters=1, sync_spin_limit=1)
    bt = M.Batch(items, p, rows_per_wg=16)
    reps = bt.register()
    torch.cuda.synchronize()
    seen = 0
    for it, rep in zip(items, reps):
        f = int(M.read_report(rep)[0]["flags"])
        if f & TIMEOUT:
            seen += 1
            assert np.array_equal(_bits(it["x"].cpu()), _bits(M.identity_params(it["x"].shape[0]).cpu()))
    bt.close()
    print("batch: problems timed out", seen, "of", len(items))
    assert seen > 0


@pytest.mark.parametrize("precision", [0, 1])
def test_nonfinite_parameter_discards_every_step(lib, precision):
    s = Scene("c1")
    p = dataclasses.replace(s.params, gn_iters=2, precision=precision)
    x0 = s.M.identity_params(s.m)
    x0[5, 9] = float("nan")
    x = x0.clone()
    rep, _ = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, p, s.ws)
    torch.cuda.synchronize()
    r = s.M.read_report(rep)
    assert all(int(f) & NONFINITE for f in r["flags"][:2])
    assert np.array_equal(_bits(x.cpu()), _bits(x0.cpu()))


def test_nonfinite_depth_is_no_measurement(lib):
    sc = gen.make_scene("c1")
    d = sc["depth"].copy()
    rng = np.random.default_rng(5)
    holes = rng.random(d.shape) < 0.03
    d[holes] = np.nan
    d[20, 10:40] = np.inf
    sc = dict(sc, depth=d)
    s = Scene(sc)
    got = s.M.normal_map(s.depth, s.cam).cpu().numpy()
    N, ok = oracle.normal_map(d, sc["camera"])
    assert np.array_equal(got[..., :3].view(np.uint32), N.astype(np.float32).view(np.uint32))
    assert np.array_equal(np.any(got[..., :3] != 0, axis=-1), ok)
    assert not ok[holes].any()
    x = s.M.identity_params(s.m)
    rep, ch = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, s.params, s.ws, corr_hist=True)
    torch.cuda.synchronize()
    r = s.M.read_report(rep)
    assert np.all(r["flags"] == 0)
    cs = list(ch.cpu().numpy())
    pix = np.concatenate([c[c >= 0] for c in cs])
    assert np.isfinite(d.reshape(-1)[pix]).all()              # no correspondence lands on a hole
    xo, _ = oracle.gn_register(s.problem(), graph=s.oracle_graph_from_gpu(), corr_sequence=cs)
    print("holed depth: x rel", rel_err(x.cpu().numpy(), xo))
    assert rel_err(x.cpu().numpy(), xo) < 1e-5


def test_frame_reject_threshold(c2):
    s = c2
    one = dataclasses.replace(s.params, gn_iters=1)
    x = s.M.identity_params(s.m)
    rep, ch = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, one, s.ws, corr_hist=True)
    torch.cuda.synchronize()
    x_plain = x.cpu().numpy()
    assert int(s.M.read_report(rep)[0]["flags"]) == 0
    from oracle.gn import _adopt
    og = s.oracle_graph_from_gpu()
    pb = s.problem()
    Nm, _ = oracle.normal_map(s.sc["depth"], s.sc["camera"])
    vc = oracle.ed_warp(pb.points, pb.nodes, oracle.identity_params(s.m), og["idx"], og["w"], pb.R, pb.T)
    a = _adopt({}, ch.cpu().numpy()[0], vc, pb, Nm.astype(np.float32))
    mean_abs = float(np.abs(a["r"][a["valid"]]).mean())
    for scale, want in ((0.99, FRAME_REJECT), (1.01, 0)):
        x = s.M.identity_params(s.m)
        p = dataclasses.replace(one, reject_threshold=scale * mean_abs)
        rep, _ = s.M.gn_register(s.pts, s.nodes, x, s.graph, s.depth, s.cam, s.pose, p, s.ws)
        torch.cuda.synchronize()
        assert int(s.M.read_report(rep)[0]["flags"]) == want, scale
        assert np.array_equal(_bits(x.cpu()), _bits(x_plain))   # a flag only: the step is taken
    print("mean |r| at identity", mean_abs)


def test_graph_overflow_reaches_every_report(lib):
    s = Scene("c1")
    g = s.graph
    x_ok = s.M.identity_params(s.m)
    s.M.gn_register(s.pts, s.nodes, x_ok, g, s.depth, s.cam, s.pose, s.params, s.ws)
    g.info[3] = GRAPH_OVERFLOW   # as graph setup leaves it after cutting a row or a list
    x = s.M.identity_params(s.m)
    rep, _ = s.M.gn_register(s.pts, s.nodes, x, g, s.depth, s.cam, s.pose, s.params, s.ws)
    torch.cuda.synchronize()
    r = s.M.read_report(rep)
    assert all(int(f) == GRAPH_OVERFLOW for f in r["flags"])
    assert np.array_equal(_bits(x.cpu()), _bits(x_ok.cpu()))
