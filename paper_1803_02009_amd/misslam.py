"""Tensor-level Python binding of libmisslam: same names as the C entry points.

PyTorch provides device memory and the current HIP stream; every step of the
method runs in the library's gfx950 kernels.  Layouts:
  points  (6, N) float32 cuda: rows px, py, pz, nx, ny, nz (canonical frame)
  nodes   (3, m) float32 cuda: rows gx, gy, gz
  x       (m, 12) float32 cuda: node parameters (c1, c2, c3, t)
  depth   (H, W) float32 cuda
"""
import atexit
import ctypes
import dataclasses
import json
import math
import os
import sys
import weakref

import numpy as np
import torch

from . import _lib
from ._lib import check, load


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, dtype, name):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")


@dataclasses.dataclass
class Params:
    """Solver settings (paper defaults, Sec. III-B)."""
    k: int = 4
    weight_kind: int = _lib.WEIGHT_GAUSS
    sigma: float = 1.0
    w_rot: float = 1000.0
    w_reg: float = 10000.0
    w_data: float = 1.0
    eps_d: float = 15.0
    cos_eps_n: float = math.cos(math.radians(10.0))
    lam: float = 1e-3
    gn_iters: int = 10
    pcg_iters: int = 10
    precision: int = _lib.PREC_FP32
    refine_steps: int = 0
    reject_threshold: float = 0.0
    solve_launch: int = _lib.LAUNCH_PLAIN
    sync_spin_limit: int = 0
    solve_form: int = _lib.SOLVE_TEXTBOOK
    asm_waves: int = 0

    def c(self):
        return _lib.Params(self.k, self.weight_kind, self.sigma, self.w_rot, self.w_reg, self.w_data, self.eps_d,
                           self.cos_eps_n, self.lam, self.gn_iters, self.pcg_iters, self.precision,
                           self.refine_steps, self.reject_threshold, self.solve_launch,
                           self.sync_spin_limit, self.solve_form, self.asm_waves)


def camera(width, height, fx, fy, cx, cy):
    return _lib.Camera(int(width), int(height), float(fx), float(fy), float(cx), float(cy))


def pose(R, T):
    R = np.asarray(R, dtype=np.float32).reshape(9)
    T = np.asarray(T, dtype=np.float32).reshape(3)
    return _lib.Pose((ctypes.c_float * 9)(*R.tolist()), (ctypes.c_float * 3)(*T.tolist()))


def _need_rows(t, dtype, name):
    """A (rows, cols) tensor whose rows are contiguous planes (a column slice of a larger buffer is fine)."""
    if not (t.is_cuda and t.dtype == dtype and t.dim() == 2 and (t.shape[1] <= 1 or t.stride(1) == 1)):
        raise ValueError(f"{name} must be a (rows, n) {dtype} CUDA tensor with contiguous rows")


def points_struct(points, w=None, stamp=None, capacity=None, stable=None):
    _need_rows(points, torch.float32, "points")
    n = points.shape[1]
    base = points.data_ptr()
    cap = n if capacity is None else capacity
    row = points.stride(0) * 4
    if stable is not None:
        _need(stable, torch.uint8, "stable")
    return _lib.Points(n, cap, base, base + row, base + 2 * row, base + 3 * row, base + 4 * row, base + 5 * row,
                       w.data_ptr() if w is not None else 0, stamp.data_ptr() if stamp is not None else 0,
                       stable.data_ptr() if stable is not None else 0)


def nodes_struct(nodes, x):
    _need_rows(nodes, torch.float32, "nodes")
    _need(x, torch.float32, "x")
    m = nodes.shape[1]
    base = nodes.data_ptr()
    row = nodes.stride(0) * 4
    return _lib.Nodes(m, m, base, base + row, base + 2 * row, x.data_ptr())


def identity_params(m, device="cuda"):
    x = torch.zeros((m, 12), dtype=torch.float32, device=device)
    x[:, 0] = 1.0
    x[:, 4] = 1.0
    x[:, 8] = 1.0
    return x


class Workspace:
    """Caller-owned scratch for the library (grown on demand, never shrunk)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes):
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        return self.buf


def workspace_bytes(n, m, width, height, params):
    return int(load().misslam_workspace_bytes(n, m, width, height, ctypes.byref(params.c())))


class Graph:
    """Per-frame graph tensors (see misslam_graph in include/misslam.h)."""

    def __init__(self, k, n, m, bsr_cap=None, device="cuda"):
        self.k, self.n, self.m = k, n, m
        self.bsr_cap = int(bsr_cap if bsr_cap is not None else m * _lib.MAX_ROW)
        i32 = dict(dtype=torch.int32, device=device)
        self.knn_idx = torch.empty((k, max(n, 1)), **i32)
        self.knn_w = torch.empty((k, max(n, 1)), dtype=torch.float32, device=device)
        self.row_ptr = torch.empty(m + 1, **i32)
        self.col_idx = torch.empty(self.bsr_cap, **i32)
        self.list_ptr = torch.empty(m + 1, **i32)
        self.list_pts = torch.empty(max(k * n, 1), **i32)
        self.list_key = torch.empty(max(2 * k * n, 2), **i32)
        self.info = torch.zeros(8, **i32)

    def c(self):
        return _lib.Graph(self.k, self.bsr_cap, self.knn_idx.data_ptr(), self.knn_w.data_ptr(),
                          self.row_ptr.data_ptr(), self.col_idx.data_ptr(), self.list_ptr.data_ptr(),
                          self.list_pts.data_ptr(), self.list_key.data_ptr(), self.info.data_ptr())


REPORT_DTYPE = np.dtype([("e_data", "<f8"), ("e_rot", "<f8"), ("e_reg", "<f8"),
                         ("pcg_resid", "<f8", (_lib.MAX_PCG + 1,)), ("n_valid", "<i4"), ("flags", "<i4"),
                         ("pcg_iters_done", "<i4"), ("reserved", "<i4"), ("e_corr", "<f8"), ("lm_e", "<f8"),
                         ("lm_e_trial", "<f8"), ("lm_lambda", "<f4"), ("lm_accepted", "<i4"), ("e_pose_r", "<f8"),
                         ("e_pose_p", "<f8")])
assert REPORT_DTYPE.itemsize == ctypes.sizeof(_lib.Report)


def new_report(count):
    return torch.zeros(count * REPORT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")


def read_report(rep):
    """Device report buffer -> numpy structured array (synchronises)."""
    return np.frombuffer(rep.cpu().numpy().tobytes(), dtype=REPORT_DTYPE)


# ------------------------------------------------------------------------------ entry points

def normal_map(depth, cam):
    _need(depth, torch.float32, "depth")
    out = torch.empty((cam.height, cam.width, 4), dtype=torch.float32, device=depth.device)
    check("misslam_normal_map", load().misslam_normal_map(_ptr(depth), ctypes.byref(cam), _ptr(out), _stream()))
    return out


def build_graph(points, nodes, params, ws, bsr_cap=None):
    n, m = points.shape[1], nodes.shape[1]
    g = Graph(params.k, n, m, bsr_cap)
    x = identity_params(m)
    pc = params.c()
    nb = workspace_bytes(n, m, 1, 1, params)
    buf = ws.get(nb)
    check("misslam_build_graph", load().misslam_build_graph(
        ctypes.byref(points_struct(points)), ctypes.byref(nodes_struct(nodes, x)), ctypes.byref(pc),
        ctypes.byref(g.c()), _ptr(buf), ctypes.c_size_t(buf.numel()), _stream()))
    return g


def warp(points, nodes, x, graph, pose_=None, normals=True):
    n = points.shape[1]
    pos = torch.empty((3, n), dtype=torch.float32, device=points.device)
    nrm = torch.empty((3, n), dtype=torch.float32, device=points.device) if normals else None
    pz = ctypes.byref(pose_) if pose_ is not None else None
    check("misslam_warp", load().misslam_warp(
        ctypes.byref(points_struct(points)), ctypes.byref(nodes_struct(nodes, x)), ctypes.byref(graph.c()), pz,
        _ptr(pos), _ptr(nrm), _stream()))
    return pos, nrm


def build_normal_eq(points, nodes, x, graph, nmap, cam, pose_, params, ws):
    n, m = points.shape[1], nodes.shape[1]
    blocks = torch.zeros((graph.bsr_cap, 12, 12), dtype=torch.float32, device=points.device)
    g = torch.empty((m, 12), dtype=torch.float32, device=points.device)
    corr = torch.empty(max(n, 1), dtype=torch.int32, device=points.device)
    rep = new_report(1)
    buf = ws.get(workspace_bytes(n, m, cam.width, cam.height, params))
    check("misslam_build_normal_eq", load().misslam_build_normal_eq(
        ctypes.byref(points_struct(points)), ctypes.byref(nodes_struct(nodes, x)), ctypes.byref(graph.c()),
        _ptr(nmap), ctypes.byref(cam), ctypes.byref(pose_), ctypes.byref(params.c()), _ptr(blocks), _ptr(g),
        _ptr(corr), _ptr(rep), _ptr(buf), ctypes.c_size_t(buf.numel()), _stream()))
    return blocks, g, corr[:n], rep


def pcg_solve(graph, m, blocks, g, params, ws):
    delta = torch.empty((m, 12), dtype=torch.float32, device=blocks.device)
    rep = new_report(1)
    buf = ws.get(workspace_bytes(0, m, 1, 1, params))
    check("misslam_pcg_solve", load().misslam_pcg_solve(
        ctypes.byref(graph.c()), m, _ptr(blocks), _ptr(g), ctypes.byref(params.c()), _ptr(delta), _ptr(rep),
        _ptr(buf), ctypes.c_size_t(buf.numel()), _stream()))
    return delta, rep


class Keypoints:
    """Key-point matches of Eq.(9): point (S,) int32 carrying model points, target (S, 3) float32 positions in the
    frame's camera coordinates.  Holds the device tensors, so they live as long as this object."""

    def __init__(self, point, target, w_corr=10.0):
        _need(point, torch.int32, "point")
        _need(target, torch.float32, "target")
        if target.dim() != 2 or target.shape[1] != 3 or target.shape[0] != point.shape[0]:
            raise ValueError("target must be (S, 3) matching point (S,)")
        self.point, self.target, self.w_corr = point, target, float(w_corr)

    def c(self):
        return _lib.Keypoints(int(self.point.shape[0]), self.w_corr, _ptr(self.point), _ptr(self.target))


def keypoints(point, target, w_corr=10.0):
    return Keypoints(point, target, w_corr)


def gn_register(points, nodes, x, graph, depth, cam, pose_, params, ws, corr_hist=False, keys=None):
    """Runs params.gn_iters Gauss-Newton steps, updating x in place; returns (report, corr_hist or None).

    keys (from keypoints()) adds the Eq.(9) key-point term."""
    n, m = points.shape[1], nodes.shape[1]
    rep = new_report(params.gn_iters + 1)
    ch = torch.empty((params.gn_iters, n), dtype=torch.int32, device=points.device) if corr_hist else None
    buf = ws.get(workspace_bytes(n, m, cam.width, cam.height, params))
    common = (ctypes.byref(points_struct(points)), ctypes.byref(nodes_struct(nodes, x)), ctypes.byref(graph.c()),
              _ptr(depth), ctypes.byref(cam), ctypes.byref(pose_), ctypes.byref(params.c()))
    tail = (_ptr(rep), _ptr(ch), _ptr(buf), ctypes.c_size_t(buf.numel()), _stream())
    if keys is None:
        check("misslam_gn_register", load().misslam_gn_register(*common, *tail))
    else:
        kc = keys.c()
        check("misslam_gn_register_keypoints", load().misslam_gn_register_keypoints(*common, ctypes.byref(kc), *tail))
    return rep, ch


def gn_register_noalloc(points, nodes, x, graph, depth, cam, pose_, params, corr_hist=False):
    """misslam_gn_register_noalloc: the float32 registration with the library's own per-device scratch array
    instead of a workspace (nothing is allocated by the call).  Returns (report, corr_hist or None); the report
    and the history are the caller's outputs, allocated here by torch."""
    n = points.shape[1]
    rep = new_report(params.gn_iters + 1)
    ch = torch.empty((params.gn_iters, n), dtype=torch.int32, device=points.device) if corr_hist else None
    check("misslam_gn_register_noalloc",
          load().misslam_gn_register_noalloc(ctypes.byref(points_struct(points)), ctypes.byref(nodes_struct(nodes, x)),
                                             ctypes.byref(graph.c()), _ptr(depth), ctypes.byref(cam),
                                             ctypes.byref(pose_), ctypes.byref(params.c()), _ptr(rep), _ptr(ch),
                                             _stream()))
    return rep, ch


@dataclasses.dataclass
class LMParams:
    """Adaptive damping schedule (Sec. II-F): classical Levenberg-Marquardt factors."""
    lambda0: float = 1e-3
    up: float = 10.0
    down: float = 0.1
    lambda_min: float = 1e-6
    lambda_max: float = 1e6

    def c(self):
        return _lib.LMParams(self.lambda0, self.up, self.down, self.lambda_min, self.lambda_max)


def lm_register(points, nodes, x, graph, depth, cam, pose_, params, ws, lm=None, keys=None, corr_hist=False):
    """Registration with adaptive Levenberg-Marquardt damping, updating x in place; returns (report, corr_hist
    or None).  The report's lm_* fields hold each step's objective at x and at x + dx, its damping and whether
    the step was taken."""
    n, m = points.shape[1], nodes.shape[1]
    rep = new_report(params.gn_iters + 1)
    ch = torch.empty((params.gn_iters, n), dtype=torch.int32, device=points.device) if corr_hist else None
    buf = ws.get(workspace_bytes(n, m, cam.width, cam.height, params))
    kc = keys.c() if keys is not None else None
    lc = (lm or LMParams()).c()
    check("misslam_lm_register", load().misslam_lm_register(
        ctypes.byref(points_struct(points)), ctypes.byref(nodes_struct(nodes, x)), ctypes.byref(graph.c()),
        _ptr(depth), ctypes.byref(cam), ctypes.byref(pose_), ctypes.byref(params.c()),
        ctypes.byref(kc) if kc is not None else None, ctypes.byref(lc), _ptr(rep), _ptr(ch), _ptr(buf),
        ctypes.c_size_t(buf.numel()), _stream()))
    return rep, ch


def joint_register(points, nodes, x, graph, depth, cam, pose_, params, ws, w_r=1e6, w_p=1e3, corr_hist=False,
                   keys=None):
    """Joint registration of the rigid pose and the ED graph (Eq.(10) pose terms, weights of Sec. III-B),
    with the Eq.(9) key points when keys is given; updates x in place.  Returns (report, pose (12,) float32
    device tensor: R row-major then T, corr_hist or None)."""
    n, m = points.shape[1], nodes.shape[1]
    rep = new_report(params.gn_iters + 1)
    ch = torch.empty((params.gn_iters, n), dtype=torch.int32, device=points.device) if corr_hist else None
    pose_out = torch.empty(12, dtype=torch.float32, device=points.device)
    buf = ws.get(workspace_bytes(n, m, cam.width, cam.height, params))
    pw = _lib.PoseWeights(float(w_r), float(w_p))
    kc = keys.c() if keys is not None else None
    check("misslam_joint_register", load().misslam_joint_register(
        ctypes.byref(points_struct(points)), ctypes.byref(nodes_struct(nodes, x)), ctypes.byref(graph.c()),
        _ptr(depth), ctypes.byref(cam), ctypes.byref(pose_), ctypes.byref(pw),
        ctypes.byref(kc) if kc is not None else None, ctypes.byref(params.c()),
        _ptr(pose_out), _ptr(rep), _ptr(ch), _ptr(buf), ctypes.c_size_t(buf.numel()), _stream()))
    return rep, pose_out, ch


def fuse_params(frame, tau=10.0, cos_delta=math.cos(math.radians(10.0)), w_max=20.0):
    """Alg. 1 thresholds and the Eq.(15) cap (Sec. III-B: 10 mm, 10 degrees, 20)."""
    return _lib.FuseParams(float(tau), float(cos_delta), float(w_max), int(frame))


def fuse(points, w, stamp, nodes, x, graph, nmap, cam, pose_, fp, ws, outputs=False, image=None, color=None):
    """Deforms and fuses in place: points (6, N), w (N), stamp (N int32), nodes (3, m) and x (reset to identity).
    With image (H, W, 3) and color (3, >= N) float32 (contiguous rows), the point colours are fused too
    (Eq.(13)), in place.

    Returns (reg_map (H, W) int32, registered (N,) int32) when outputs=True.
    """
    n, m = points.shape[1], nodes.shape[1]
    _need(w, torch.float32, "w")
    _need(stamp, torch.int32, "stamp")
    reg = torch.empty((cam.height, cam.width), dtype=torch.int32, device=points.device) if outputs else None
    regd = torch.empty(max(n, 1), dtype=torch.int32, device=points.device) if outputs else None
    buf = ws.get(workspace_bytes(n, m, cam.width, cam.height, Params()))
    if image is None and color is None:
        check("misslam_fuse", load().misslam_fuse(
            ctypes.byref(points_struct(points, w, stamp)), ctypes.byref(nodes_struct(nodes, x)),
            ctypes.byref(graph.c()), _ptr(nmap), ctypes.byref(cam), ctypes.byref(pose_), ctypes.byref(fp), _ptr(reg),
            _ptr(regd), _ptr(buf), ctypes.c_size_t(buf.numel()), _stream()))
    else:
        stride = _color_stride(image, color, cam, n)
        check("misslam_fuse_color", load().misslam_fuse_color(
            ctypes.byref(points_struct(points, w, stamp)), ctypes.byref(nodes_struct(nodes, x)),
            ctypes.byref(graph.c()), _ptr(nmap), ctypes.byref(cam), ctypes.byref(pose_), ctypes.byref(fp),
            _ptr(image), _ptr(color), ctypes.c_int64(stride), _ptr(reg), _ptr(regd), _ptr(buf),
            ctypes.c_size_t(buf.numel()), _stream()))
    return (reg, regd[:n]) if outputs else None


def grow_params(frame, node_spacing, voxel=0.22, tau_weight=2.0, tau_time=10):
    """Alg. 2 steps 3-5 / Alg. 3 settings (Sec. III-B: 0.22 mm box, 10 frames; the weight bound is a reading)."""
    return _lib.GrowParams(float(voxel), float(node_spacing), float(tau_weight), int(tau_time), int(frame))


def _color_stride(image, color, cam, n):
    _need(image, torch.float32, "image")
    if tuple(image.shape) != (cam.height, cam.width, 3):
        raise ValueError("image must be (H, W, 3)")
    _need_rows(color, torch.float32, "color")
    if color.shape[0] != 3 or color.shape[1] < n:
        raise ValueError("color must be (3, >= N)")
    return color.stride(0)


def grow(points, w, stamp, n, nodes, x, m, reg_map, registered, nmap, cam, pose_, gp, ws, image=None, color=None,
         stable=None):
    """Growth and maintenance after fuse (misslam_grow).

    points (6, capacity), w, stamp (capacity), nodes (3, node_capacity), x (node_capacity, 12): the model with
    n points and m nodes in use; rewritten in place.  With image (H, W, 3) and color (3, capacity) the point
    colours follow (misslam_grow_color); with stable (capacity,) uint8 the stability flags S_i.  Returns the
    device counts tensor (7,) int64: new n, new m, lifted, removed, merged away, new nodes, overflow.
    """
    counts = torch.zeros(7, dtype=torch.int64, device=points.device)
    cap = points.shape[1]
    pstruct = points_struct(points, w, stamp, capacity=cap, stable=stable)
    pstruct.n = int(n)
    nstruct = nodes_struct(nodes, x)
    nstruct.m = int(m)
    nstruct.capacity = nodes.shape[1]
    buf = ws.get(load().misslam_grow_workspace_bytes(int(n), cam.width, cam.height))
    if image is None and color is None:
        check("misslam_grow", load().misslam_grow(
            ctypes.byref(pstruct), ctypes.byref(nstruct), _ptr(reg_map), _ptr(registered), _ptr(nmap),
            ctypes.byref(cam), ctypes.byref(pose_), ctypes.byref(gp), _ptr(counts), _ptr(buf),
            ctypes.c_size_t(buf.numel()), _stream()))
    else:
        stride = _color_stride(image, color, cam, cap)
        check("misslam_grow_color", load().misslam_grow_color(
            ctypes.byref(pstruct), ctypes.byref(nstruct), _ptr(reg_map), _ptr(registered), _ptr(nmap),
            ctypes.byref(cam), ctypes.byref(pose_), ctypes.byref(gp), _ptr(image), _ptr(color), ctypes.c_int64(stride),
            _ptr(counts), _ptr(buf), ctypes.c_size_t(buf.numel()), _stream()))
    return counts


def energy_vjp(points, nodes, x, graph, nmap, cam, pose_, params, ws, corr=None, grad_e=None, want_params=True,
               want_points=True):
    """Energy (and gradients) at x.  corr=None: associate now; else hold the given correspondences.

    Returns (energy (1,) float64, grad_params (m, 12) or None, grad_points (3, N) or None, corr, report).
    """
    n, m = points.shape[1], nodes.shape[1]
    dev = points.device
    e = torch.empty(1, dtype=torch.float64, device=dev)
    gp = torch.empty((m, 12), dtype=torch.float32, device=dev) if want_params else None
    gv = torch.empty((3, n), dtype=torch.float32, device=dev) if want_points else None
    co = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if corr is None else None
    rep = new_report(1)
    buf = ws.get(workspace_bytes(n, m, cam.width, cam.height, params))
    check("misslam_energy_vjp", load().misslam_energy_vjp(
        ctypes.byref(points_struct(points)), ctypes.byref(nodes_struct(nodes, x)), ctypes.byref(graph.c()),
        _ptr(nmap), ctypes.byref(cam), ctypes.byref(pose_), ctypes.byref(params.c()), _ptr(corr), _ptr(co),
        _ptr(grad_e), _ptr(gp), _ptr(gv), _ptr(e), _ptr(rep), _ptr(buf), ctypes.c_size_t(buf.numel()), _stream()))
    return e, gp, gv, (corr if corr is not None else co[:n]), rep


class WarpEnergy(torch.autograd.Function):
    """E(x, v) of Eq.(3) (data + rotation + regularisation) as a differentiable function.

    Forward finds the correspondences; backward holds them (and the kNN sets)
    fixed and runs the library's adjoint kernels for dE/dx and dE/dv.
    Usage: WarpEnergy.apply(x, positions, context) with context = dict(points,
    nodes, graph, nmap, cam, pose, params, ws); positions (3, N) are the
    canonical coordinates (rows 0-2 of points).
    """

    @staticmethod
    def forward(ctx, x, positions, context):
        pts = context["points"]
        if positions.data_ptr() != pts.data_ptr():
            pts = torch.cat([positions.detach(), pts[3:]], 0).contiguous()
        e, _, _, corr, _ = energy_vjp(pts, context["nodes"], x.detach().contiguous(), context["graph"],
                                      context["nmap"], context["cam"], context["pose"], context["params"],
                                      context["ws"], want_params=False, want_points=False)
        ctx.context = context
        ctx.save_for_backward(x.detach().contiguous(), pts, corr)
        return e[0]

    @staticmethod
    def backward(ctx, grad_out):
        x, pts, corr = ctx.saved_tensors
        c = ctx.context
        ge = grad_out.detach().reshape(1).to(torch.float32).contiguous()
        _, gp, gv, _, _ = energy_vjp(pts, c["nodes"], x, c["graph"], c["nmap"], c["cam"], c["pose"], c["params"],
                                     c["ws"], corr=corr, grad_e=ge, want_params=ctx.needs_input_grad[0],
                                     want_points=ctx.needs_input_grad[1])
        return gp, gv, None


# Batches still open when the interpreter exits are closed by an exit hook, while the HIP runtime is still
# up; a batch collected during interpreter shutdown makes no library call.
_open_batches = weakref.WeakSet()


@atexit.register
def _close_open_batches():
    for b in list(_open_batches):
        b.close()


def tile_cache_path():
    """The JSON file of tuned batch tiles: $MISSLAM_TILE_CACHE, else ~/.cache/misslam/tiles.json."""
    return os.environ.get("MISSLAM_TILE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "misslam",
                                                                 "tiles.json")


def _bucket(v):
    return 1 << max(0, math.ceil(math.log2(max(int(v), 1))))


def tile_key(problems, params):
    """Cache key of a batch: point and node totals rounded up to powers of two, the largest frame, the
    precision, and the settings the tiles depend on (k, PCG iterations, recurrence, problem count)."""
    n = sum(int(pr["points"].shape[1]) for pr in problems)
    m = sum(int(pr["nodes"].shape[1]) for pr in problems)
    w, h = max((pr["cam"].width * pr["cam"].height, pr["cam"].width, pr["cam"].height) for pr in problems)[1:]
    return (f"N{_bucket(n)}-m{_bucket(m)}-{w}x{h}-prec{params.precision}-k{params.k}-pcg{params.pcg_iters}"
            f"-form{params.solve_form}-count{len(problems)}")


def _read_tile_cache(path):
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _write_tile_cache(path, key, entry):
    d = _read_tile_cache(path)
    d[key] = entry
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


class Batch:
    """Uneven problems registered together (misslam_batch_*): one launch per
    phase over every problem, the frame captured once into a hipGraph.

    problems: list of dicts with keys points (6, N), nodes (3, m), x (m, 12),
    graph (Graph), depth (H, W), cam, pose.  Tensors must stay alive and keep
    their addresses while the batch is used.  rows_per_wg: solve tile (1..21)
    or 0 to choose the tiles (solve rows per workgroup and, with
    params.asm_waves 0, assembly waves per node row).  Chosen tiles come from
    the tile cache (tile_cache_path()) when it holds this batch's key, else the
    first register() times the candidates and stores its choice there;
    tile_cache=False skips the cache.  tile_source says which: "given",
    "cache" or "tuned".
    """

    def __init__(self, problems, params, rows_per_wg=0, tile_cache=True):
        self.keep = []
        _open_batches.add(self)
        self.tile_source = "given" if rows_per_wg else "tuned"
        self._store_key = None
        if rows_per_wg == 0 and params.asm_waves == 0 and tile_cache:
            key = tile_key(problems, params)
            hit = _read_tile_cache(tile_cache_path()).get(key)
            if (isinstance(hit, dict) and hit.get("rows_per_wg") in range(1, 22)
                    and hit.get("asm_waves") in (1, 2)):
                rows_per_wg = int(hit["rows_per_wg"])
                params = dataclasses.replace(params, asm_waves=int(hit["asm_waves"]))
                self.tile_source = "cache"
            else:
                self._store_key = key
        self.params = params
        self.reports = []
        arr = (_lib.Problem * len(problems))()
        for i, pr in enumerate(problems):
            rep = new_report(params.gn_iters + 1)
            self.reports.append(rep)
            _need(pr["depth"], torch.float32, "depth")
            self.keep.append((pr, rep))
            arr[i] = _lib.Problem(points_struct(pr["points"]), nodes_struct(pr["nodes"], pr["x"]), pr["graph"].c(),
                                  pr["depth"].data_ptr(), pr["cam"], pr["pose"], rep.data_ptr())
        self._arr = arr
        h = ctypes.c_void_p()
        check("misslam_batch_create", load().misslam_batch_create(arr, len(problems), ctypes.byref(params.c()),
                                                                  int(rows_per_wg), ctypes.byref(h)))
        self.h = h
        nb = load().misslam_batch_workspace_bytes(h)
        self.ws = torch.empty(max(int(nb), 1), dtype=torch.uint8, device="cuda")

    def register(self):
        check("misslam_batch_register", load().misslam_batch_register(self.h, _ptr(self.ws),
                                                                      ctypes.c_size_t(self.ws.numel()), _stream()))
        if self._store_key is not None:   # the first call chose the tiles: keep them for the next process
            try:
                _write_tile_cache(tile_cache_path(), self._store_key,
                                  {"rows_per_wg": self.tile, "asm_waves": self.asm_waves})
            except OSError:
                pass
            self._store_key = None
        return self.reports

    @property
    def tile(self):
        return int(load().misslam_batch_tile(self.h))

    @property
    def asm_waves(self):
        return int(load().misslam_batch_asm_waves(self.h))

    def close(self):
        if getattr(self, "h", None):
            load().misslam_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        if sys.is_finalizing():   # the exit hook has closed it, or the runtime may be gone
            return
        try:
            self.close()
        except Exception:  # pragma: no cover
            pass
