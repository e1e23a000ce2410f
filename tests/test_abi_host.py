"""Host-side checks of the C ABI: exported symbols, struct layout, argument validation.

These run without a GPU: every call below returns on the host before any
HIP call (argument checks precede all launches).
"""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_1803_02009_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "misslam.h")


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(misslam_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def test_struct_layout_matches_header():
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "misslam.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(misslam_camera), sizeof(misslam_pose),
         sizeof(misslam_points), sizeof(misslam_nodes), sizeof(misslam_graph), sizeof(misslam_params),
         sizeof(misslam_report), sizeof(misslam_fuse_params), sizeof(misslam_problem), sizeof(misslam_keypoints),
         sizeof(misslam_lm_params), sizeof(misslam_pose_weights));
  printf("%zu %zu %zu %zu %zu %zu %zu\n", offsetof(misslam_params, eps_d), offsetof(misslam_params, lambda),
         offsetof(misslam_report, n_valid), offsetof(misslam_graph, info), offsetof(misslam_params, solve_launch),
         offsetof(misslam_report, lm_e), offsetof(misslam_report, lm_accepted));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split("\n")
    sizes = [int(v) for v in out[0].split()]
    want = [ctypes.sizeof(t) for t in (_lib.Camera, _lib.Pose, _lib.Points, _lib.Nodes, _lib.Graph, _lib.Params,
                                       _lib.Report, _lib.FuseParams, _lib.Problem, _lib.Keypoints, _lib.LMParams,
                                       _lib.PoseWeights)]
    assert sizes == want
    offs = [int(v) for v in out[1].split()]
    assert offs == [_lib.Params.eps_d.offset, _lib.Params.lambda_.offset, _lib.Report.n_valid.offset,
                    _lib.Graph.info.offset, _lib.Params.solve_launch.offset, _lib.Report.lm_e.offset,
                    _lib.Report.lm_accepted.offset]


def test_header_constants_match_binding():
    text = open(HEADER).read()
    defs = {k: int(v, 0) for k, v in re.findall(r"#define\s+MISSLAM_([A-Z_0-9]+)\s+(-?(?:0x[0-9a-fA-F]+|\d+))", text)}
    want = {"FLAG_SYNC_TIMEOUT": _lib.FLAG_SYNC_TIMEOUT, "PREC_FP32": _lib.PREC_FP32, "PREC_BF16": _lib.PREC_BF16,
            "PREC_FP16": _lib.PREC_FP16, "LAUNCH_PLAIN": _lib.LAUNCH_PLAIN,
            "LAUNCH_COOPERATIVE": _lib.LAUNCH_COOPERATIVE, "LAUNCH_KERNELS": _lib.LAUNCH_KERNELS,
            "SOLVE_PIPELINED": _lib.SOLVE_PIPELINED, "SOLVE_TEXTBOOK": _lib.SOLVE_TEXTBOOK, "MAX_K": _lib.MAX_K, "MAX_PCG": _lib.MAX_PCG,
            "MAX_ROW": _lib.MAX_ROW, "MAX_LIST": _lib.MAX_LIST, "SOLVE_ROWS": _lib.SOLVE_ROWS,
            "MAX_KEYPOINTS": _lib.MAX_KEYPOINTS, "NOALLOC_SCRATCH_BYTES": _lib.NOALLOC_SCRATCH_BYTES}
    for k, v in want.items():
        assert defs[k] == v, k


def test_default_params_are_the_papers(lib):
    p = _lib.Params()
    lib.misslam_default_params(ctypes.byref(p))
    assert (p.k, p.w_rot, p.w_reg, p.w_data, p.eps_d) == (4, 1000.0, 10000.0, 1.0, 15.0)
    assert abs(p.cos_eps_n - 0.984807753012208) < 1e-15
    assert (p.gn_iters, p.pcg_iters, p.precision) == (10, 10, _lib.PREC_FP32)
    assert p.solve_launch == _lib.LAUNCH_PLAIN


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.misslam_status_string(code)
    assert lib.misslam_status_string(-99) == b"unknown status"


def test_workspace_query(lib):
    p = _lib.Params()
    lib.misslam_default_params(ctypes.byref(p))
    small = lib.misslam_workspace_bytes(1000, 10, 64, 48, ctypes.byref(p))
    big = lib.misslam_workspace_bytes(250000, 1600, 640, 480, ctypes.byref(p))
    assert 0 < small < big
    assert lib.misslam_workspace_bytes(-1, 10, 64, 48, ctypes.byref(p)) == 0
    assert lib.misslam_workspace_bytes(10, 0, 64, 48, ctypes.byref(p)) == 0
    bad = _lib.Params()
    lib.misslam_default_params(ctypes.byref(bad))
    bad.k = 9
    assert lib.misslam_workspace_bytes(10, 10, 64, 48, ctypes.byref(bad)) == 0
    bad.k = 4
    bad.pcg_iters = _lib.MAX_PCG + 1
    assert lib.misslam_workspace_bytes(10, 10, 64, 48, ctypes.byref(bad)) == 0
    bad.pcg_iters = 10
    bad.solve_launch = _lib.LAUNCH_KERNELS
    assert lib.misslam_workspace_bytes(10, 10, 64, 48, ctypes.byref(bad)) > 0
    bad.solve_launch = 3
    assert lib.misslam_workspace_bytes(10, 10, 64, 48, ctypes.byref(bad)) == 0


FAKE = 0x1000   # never dereferenced: every call below fails validation first


def _structs(n=100, m=10, k=4):
    pts = _lib.Points(n, n, *([FAKE] * 6), 0, 0)
    nds = _lib.Nodes(m, m, FAKE, FAKE, FAKE, FAKE)
    gr = _lib.Graph(k, m * _lib.MAX_ROW, *([FAKE] * 8))
    p = _lib.Params()
    _lib.load().misslam_default_params(ctypes.byref(p))
    cam = _lib.Camera(64, 48, 60.0, 60.0, 32.0, 24.0)
    pose = _lib.Pose()
    return pts, nds, gr, p, cam, pose


def test_validation_errors(lib):
    pts, nds, gr, p, cam, pose = _structs()
    B = ctypes.byref
    # null pointers
    assert lib.misslam_build_graph(None, B(nds), B(p), B(gr), FAKE, 1 << 30, None) == _lib.EINVAL
    assert lib.misslam_warp(B(pts), B(nds), B(gr), None, None, None, None) == _lib.EINVAL
    assert lib.misslam_normal_map(None, B(cam), FAKE, None) == _lib.EINVAL
    # k mismatch between graph and params
    gr5 = _lib.Graph(5, gr.bsr_cap, *([FAKE] * 8))
    assert lib.misslam_build_graph(B(pts), B(nds), B(p), B(gr5), FAKE, 1 << 30, None) == _lib.ESHAPE
    # fewer nodes than k
    nds3 = _lib.Nodes(3, 3, FAKE, FAKE, FAKE, FAKE)
    assert lib.misslam_build_graph(B(pts), B(nds3), B(p), B(gr), FAKE, 1 << 30, None) == _lib.ESHAPE
    # workspace too small
    assert lib.misslam_build_graph(B(pts), B(nds), B(p), B(gr), FAKE, 16, None) == _lib.EWORKSPACE
    assert lib.misslam_gn_register(B(pts), B(nds), B(gr), FAKE, B(cam), B(pose), B(p), FAKE, None, FAKE, 16,
                                   None) == _lib.EWORKSPACE
    # key points: required, count >= 0, arrays when count > 0, finite non-negative weight; float32 form only
    kpr = lib.misslam_gn_register_keypoints
    assert kpr(B(pts), B(nds), B(gr), FAKE, B(cam), B(pose), B(p), None, FAKE, None, FAKE, 1 << 40,
               None) == _lib.EINVAL
    for bad in (_lib.Keypoints(-1, 10.0, FAKE, FAKE), _lib.Keypoints(3, 10.0, None, FAKE),
                _lib.Keypoints(3, 10.0, FAKE, None), _lib.Keypoints(3, float("nan"), FAKE, FAKE),
                _lib.Keypoints(3, -1.0, FAKE, FAKE)):
        assert kpr(B(pts), B(nds), B(gr), FAKE, B(cam), B(pose), B(p), B(bad), FAKE, None, FAKE, 1 << 40,
                   None) == _lib.EINVAL
    plp = _lib.Params()
    lib.misslam_default_params(B(plp))
    plp.precision = _lib.PREC_BF16
    ok_keys = _lib.Keypoints(3, 10.0, FAKE, FAKE)
    assert kpr(B(pts), B(nds), B(gr), FAKE, B(cam), B(pose), B(plp), B(ok_keys), FAKE, None, FAKE, 1 << 40,
               None) == _lib.EUNSUPPORTED
    # adaptive damping: a schedule is required and must be ordered, finite, up >= 1, 0 < down <= 1;
    # float32 form only
    lmr = lib.misslam_lm_register
    good = _lib.LMParams()
    lib.misslam_default_lm_params(B(good))
    assert (good.lambda0, good.up, good.down, good.lambda_min, good.lambda_max) == pytest.approx(
        (1e-3, 10.0, 0.1, 1e-6, 1e6), rel=1e-6)
    assert lmr(B(pts), B(nds), B(gr), FAKE, B(cam), B(pose), B(p), None, None, FAKE, None, FAKE, 1 << 40,
               None) == _lib.EINVAL
    for bad in (_lib.LMParams(1e-3, 0.5, 0.1, 1e-6, 1e6), _lib.LMParams(1e-3, 10.0, 0.0, 1e-6, 1e6),
                _lib.LMParams(1e-3, 10.0, 1.5, 1e-6, 1e6), _lib.LMParams(1e-7, 10.0, 0.1, 1e-6, 1e6),
                _lib.LMParams(10.0, 10.0, 0.1, 1e-6, 1.0), _lib.LMParams(1e-3, 10.0, 0.1, -1.0, 1e6),
                _lib.LMParams(float("nan"), 10.0, 0.1, 1e-6, 1e6), _lib.LMParams(1e-3, float("inf"), 0.1, 1e-6, 1e6)):
        assert lmr(B(pts), B(nds), B(gr), FAKE, B(cam), B(pose), B(p), None, B(bad), FAKE, None, FAKE, 1 << 40,
                   None) == _lib.EINVAL
    assert lmr(B(pts), B(nds), B(gr), FAKE, B(cam), B(pose), B(plp), None, B(good), FAKE, None, FAKE, 1 << 40,
               None) == _lib.EUNSUPPORTED
    # joint pose: weights and an output pose are required, weights finite and >= 0; float32 form only
    jr = lib.misslam_joint_register
    pw = _lib.PoseWeights(1e6, 1e3)
    assert jr(B(pts), B(nds), B(gr), FAKE, B(cam), B(pose), None, None, B(p), FAKE, FAKE, None, FAKE, 1 << 40,
              None) == _lib.EINVAL
    assert jr(B(pts), B(nds), B(gr), FAKE, B(cam), B(pose), B(pw), None, B(p), None, FAKE, None, FAKE, 1 << 40,
              None) == _lib.EINVAL
    for bad in (_lib.PoseWeights(-1.0, 1e3), _lib.PoseWeights(1e6, float("nan")), _lib.PoseWeights(float("inf"), 1.0)):
        assert jr(B(pts), B(nds), B(gr), FAKE, B(cam), B(pose), B(bad), None, B(p), FAKE, FAKE, None, FAKE, 1 << 40,
                  None) == _lib.EINVAL
    assert jr(B(pts), B(nds), B(gr), FAKE, B(cam), B(pose), B(pw), None, B(plp), FAKE, FAKE, None, FAKE, 1 << 40,
              None) == _lib.EUNSUPPORTED
    assert jr(B(pts), B(nds), B(gr), FAKE, B(cam), B(pose), B(pw), B(_lib.Keypoints(-1, 10.0, FAKE, FAKE)), B(p),
              FAKE, FAKE, None, FAKE, 1 << 40, None) == _lib.EINVAL
    # colour fusion needs the image and the colours
    fp = _lib.FuseParams(10.0, 0.98, 20.0, 1)
    fc = lib.misslam_fuse_color
    assert fc(B(pts), B(nds), B(gr), FAKE, B(cam), B(pose), B(fp), None, FAKE, 1 << 20, None, None, FAKE, 1 << 40,
              None) == _lib.EINVAL
    assert fc(B(pts), B(nds), B(gr), FAKE, B(cam), B(pose), B(fp), FAKE, None, 1 << 20, None, None, FAKE, 1 << 40,
              None) == _lib.EINVAL
    assert fc(B(pts), B(nds), B(gr), FAKE, B(cam), B(pose), B(fp), FAKE, FAKE, 1, None, None, FAKE, 1 << 40,
              None) == _lib.EINVAL
    gpar = _lib.GrowParams()
    gc = lib.misslam_grow_color
    assert gc(B(pts), B(nds), FAKE, FAKE, FAKE, B(cam), B(pose), B(gpar), FAKE, FAKE, 1, FAKE, FAKE, 1 << 40,
              None) == _lib.EINVAL
    # n above capacity, bad camera, bad k
    over = _lib.Points(200, 100, *([FAKE] * 6), 0, 0)
    assert lib.misslam_warp(B(over), B(nds), B(gr), None, FAKE, None, None) == _lib.EINVAL
    badcam = _lib.Camera(0, 48, 60.0, 60.0, 32.0, 24.0)
    assert lib.misslam_normal_map(FAKE, B(badcam), FAKE, None) == _lib.EINVAL
    p2 = _lib.Params()
    lib.misslam_default_params(ctypes.byref(p2))
    p2.k = 0
    assert lib.misslam_build_graph(B(pts), B(nds), B(p2), B(gr), FAKE, 1 << 30, None) == _lib.EINVAL
    p2.k = 4
    p2.lambda_ = -1.0
    assert lib.misslam_pcg_solve(B(gr), 10, FAKE, FAKE, B(p2), FAKE, FAKE, FAKE, 1 << 30, None) == _lib.EINVAL


def test_noalloc_registration_checks_on_host(lib):
    """The allocation-free registration checks every size before any HIP call: a frame whose scratch exceeds
    the fixed array is refused (ECAPACITY), as are the low-precision forms and missing arguments."""
    B = ctypes.byref
    nr = lib.misslam_gn_register_noalloc
    pts, nds, gr, p, cam, pose = _structs()
    assert nr(B(pts), B(nds), B(gr), FAKE, B(cam), B(pose), B(p), None, None, None) == _lib.EINVAL
    assert nr(B(pts), B(nds), B(gr), None, B(cam), B(pose), B(p), FAKE, None, None) == _lib.EINVAL
    plp = _lib.Params()
    lib.misslam_default_params(B(plp))
    plp.precision = _lib.PREC_FP16
    assert nr(B(pts), B(nds), B(gr), FAKE, B(cam), B(pose), B(plp), FAKE, None, None) == _lib.EUNSUPPORTED
    # the benchmark frame's scratch is below the array, twice its points is not; the workspace query of the
    # same frame (every form's buffers) is larger than the array
    big_cam = _lib.Camera(640, 480, 256.0, 256.0, 320.0, 240.0)
    p.sigma = 2.5
    full = lib.misslam_workspace_bytes(250000, 1600, 640, 480, B(p))
    assert full > _lib.NOALLOC_SCRATCH_BYTES
    over_pts, over_nds, over_gr, _, _, _ = _structs(n=600000, m=1600)
    assert nr(B(over_pts), B(over_nds), B(over_gr), FAKE, B(big_cam), B(pose), B(p), FAKE, None,
              None) == _lib.ECAPACITY
    huge_cam = _lib.Camera(4096, 4096, 1600.0, 1600.0, 2048.0, 2048.0)
    assert nr(B(pts), B(nds), B(gr), FAKE, B(huge_cam), B(pose), B(p), FAKE, None, None) == _lib.ECAPACITY


def test_profiler_api_on_host(lib):
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    assert lib.misslam_profile_get(b"nope", ctypes.byref(ms), ctypes.byref(cnt)) == _lib.EINVAL
    lib.misslam_profile_reset()
    assert lib.misslam_profile_get(b"assemble", ctypes.byref(ms), ctypes.byref(cnt)) == _lib.OK
    assert cnt.value == 0 and ms.value == 0.0
    prev = lib.misslam_profile_enable(1)
    assert lib.misslam_profile_enable(prev) == 1
