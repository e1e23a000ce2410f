#!/usr/bin/env python3
"""Throughput of MIS-SLAM's per-frame deformable registration on one MI355X.

One step = one frame of the hot path on the 640x480 / 250,000-point /
1,600-node synthetic tissue problem: graph setup (kNN, skinning weights, node
graph, lists), depth normal map, 10 Gauss-Newton iterations of 10 PCG
iterations each, and the fusion of the frame into the deformed model.  Inputs
are resident in HBM before timing starts; each step first restores the model
(points, normals, weights, stamps, node positions: about 9 MB of device
copies) because fusion updates it in place.

Prints one JSON line.  value = Gauss-Newton iterations per second over whole
frames; ms_per_step = ms per frame.  A second, profiled region (HIP events
around each phase, on the library's stream) gives the per-phase breakdown and
the roofline of the dominant kernel.  The low-precision form (bf16 data-term
normal matrix on the matrix cores, two float32 refinement passes) is timed on
the same frame and reported beside it with its error against the oracle's
emulation of that form.  The CPU baseline is the float64 oracle on a bounded
sample of the same frame.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP32_VALU_PEAK = 157.3       # TFLOP/s vendor figure
MFMA_BF16_PEAK = 2500.0      # TFLOP/s, dense bf16 matrix cores, vendor figure

# source files each timed kernel is compiled from (its counter figures are void once any of them changes)
KERNEL_SOURCES = {
    "point_pass": ["k_step.hip"],
    "assemble": ["k_step.hip"],
    "pcg": ["k_pcg.hip"],
}
COUNTERS_MD = os.path.join(ROOT, "profiles", "c3_hbm_counters.md")


def kernel_source_hash(phase):
    """Short sha256 of the sources a phase's kernel is built from (its own file and the shared headers)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1803_02009_amd", "csrc")
    for f in KERNEL_SOURCES[phase] + ["common.h", "frame.h"]:
        h.update(open(os.path.join(csrc, f), "rb").read())
    h.update(open(os.path.join(ROOT, "include", "misslam.h"), "rb").read())
    return h.hexdigest()[:16]


def counter_traffic(phase):
    """HBM bytes per launch of a phase's kernel from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE, each scaled by its reading for a plain copy of known size), or None when the summary
    has no row for it or was taken on other sources."""
    if not os.path.exists(COUNTERS_MD):
        return None
    for line in open(COUNTERS_MD):
        cells = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
        if len(cells) == 7 and cells[0] == phase:
            try:
                return int(cells[5]) if cells[6] == kernel_source_hash(phase) else None
            except ValueError:
                return None
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--seq-frames", type=int, default=8,
                    help="frames of the sweeping sequence (0: skip; 300 is the whole sweep)")
    ap.add_argument("--no-cold", action="store_true", help="skip the frame timed after a 512 MiB cache flush")
    ap.add_argument("--no-lowp", action="store_true")
    ap.add_argument("--no-keypoints", action="store_true")
    ap.add_argument("--no-lm", action="store_true")
    ap.add_argument("--no-joint", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run 5 device-to-device copies of this many MiB (counter calibration) and exit")
    return ap.parse_args()


def algorithmic_bytes(phase, n, m, nnzb, k, width, height, pcg_iters, n_valid):
    """Bytes one launch of a phase must move at minimum (float32 / int32 streams)."""
    if phase == "point_pass":
        # read v, n (24 B), k idx + k w (8k B), the matched pixel (16 B, valid points);
        # write r, n', corr (20 B); node table reads are cache-resident
        return n * (24 + 8 * k + 20) + n_valid * 16
    if phase == "assemble":
        # per point: k idx + k w, v, n', r, corr; per list entry 4 B; out: blocks, g
        return n * (8 * k + 12 + 12 + 4 + 4) + k * n * 4 + nnzb * 576 + m * 48 + m * 48
    if phase == "pcg":
        # per iteration: the whole BSR once (576 B/block) + ~8 vector passes of 12 m floats + M (576 B/node)
        return pcg_iters * (nnzb * 576 + m * 576 + 8 * 12 * m * 4) + m * 576
    if phase == "bjacobi":
        return m * 576 * 2
    if phase == "normal_map":
        return width * height * (4 + 16)
    return 0


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the per-frame registration does not shard across GPUs).", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_mib > 0:   # a plain copy of known size, to scale the HBM byte counters
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_dispatch": src.numel() * 4}))
        return

    import gen
    from paper_1803_02009_amd import _lib
    from paper_1803_02009_amd import misslam as M

    # the sweep's frames are generated on the host first, in worker processes forked before any GPU use
    seq_frames = generate_sequence(args.seq_frames + 1) if args.seq_frames > 0 else None
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    lib = _lib.load()
    sc = gen.make_scene(args.config)
    dev = "cuda"
    pts = torch.tensor(np.concatenate([sc["points"].T, sc["normals"].T]), device=dev).contiguous()
    nodes = torch.tensor(np.ascontiguousarray(sc["nodes"].T), device=dev).contiguous()
    depth = torch.tensor(sc["depth"], device=dev).contiguous()
    cam = M.camera(*sc["camera"])
    pose = M.pose(sc["R"], sc["T"])
    params = M.Params(sigma=sc["sigma"], gn_iters=sc["gn_iters"], pcg_iters=sc["pcg_iters"])
    ws = M.Workspace()
    n, m = pts.shape[1], nodes.shape[1]
    G = params.gn_iters
    x = M.identity_params(m)
    x0 = x.clone()
    state = {}

    pts0, nodes0 = pts.clone(), nodes.clone()
    w = torch.zeros(n, dtype=torch.float32, device=dev)
    stamp = torch.zeros(n, dtype=torch.int32, device=dev)
    w0, stamp0 = w.clone(), stamp.clone()
    fp = M.fuse_params(frame=1)

    def frame(p=params, keys=None, lm=None, joint=False):
        pts.copy_(pts0)
        nodes.copy_(nodes0)
        w.copy_(w0)
        stamp.copy_(stamp0)
        x.copy_(x0)
        g = M.build_graph(pts, nodes, p, ws)
        if joint:
            rep, pz, _ = M.joint_register(pts, nodes, x, g, depth, cam, pose, p, ws)
            state["pose"] = pz
        elif lm is None:
            rep, _ = M.gn_register(pts, nodes, x, g, depth, cam, pose, p, ws, keys=keys)
        else:
            rep, _ = M.lm_register(pts, nodes, x, g, depth, cam, pose, p, ws, lm=lm, keys=keys)
        state["graph"], state["rep"], state["x"] = g, rep, x.clone()
        nmap = M.normal_map(depth, cam)
        M.fuse(pts, w, stamp, nodes, x, g, nmap, cam, pose, fp, ws)

    def timed(p, steps, keys=None, lm=None, joint=False):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            frame(p, keys, lm, joint)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    for _ in range(max(1, args.warmup)):
        frame()
    elapsed = timed(params, args.steps)
    ms_frame = 1000.0 * elapsed / args.steps
    gn_per_s = G * args.steps / elapsed

    # profiled region: per-phase HIP events on the library's stream
    lib.misslam_profile_reset()
    lib.misslam_profile_enable(1)
    for _ in range(args.steps):
        frame()
    torch.cuda.synchronize()
    lib.misslam_profile_enable(0)
    import ctypes
    phases = {}
    for ph in ["normal_map", "build_graph", "list_pack", "point_pass", "assemble", "energy", "bjacobi", "pcg", "fuse",
               "refine"]:
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        _lib.check("misslam_profile_get", lib.misslam_profile_get(ph.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
        phases[ph] = {"total_ms": ms.value, "launches": cnt.value,
                      "avg_us": 1000.0 * ms.value / cnt.value if cnt.value else 0.0}
    rep = M.read_report(state["rep"])
    info = state["graph"].info.cpu().numpy()
    nnzb = int(info[0])
    n_valid = int(np.mean([r["n_valid"] for r in rep[:G]]))
    per_iter = ["point_pass", "assemble", "energy", "bjacobi", "pcg"]
    gn_iter_ms = sum(phases[p]["total_ms"] for p in per_iter) / (args.steps * G)
    # roofline of each per-iteration kernel; the dominant one (most time per frame) is `roofline`
    lines = {}
    for ph in ["point_pass", "assemble", "pcg"]:
        if not phases[ph]["launches"]:
            continue
        abytes = algorithmic_bytes(ph, n, m, nnzb, params.k, cam.width, cam.height, params.pcg_iters, n_valid)
        achieved = abytes / (phases[ph]["avg_us"] * 1e-6) / 1e9
        lines[ph] = {"kernel": ph, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counter_traffic(ph),
                     "algorithmic_bytes_per_launch": int(abytes), "avg_launch_us": round(phases[ph]["avg_us"], 2),
                     "ms_per_frame": round(phases[ph]["total_ms"] / args.steps, 4)}
    dominant = max(lines, key=lambda p: lines[p]["ms_per_frame"])
    roofline = lines[dominant]

    # accuracy against the stored float64 oracle result of the same frame
    acc = accuracy(state, rep, os.path.join(ROOT, "tests", "golden", f"{args.config}_oracle.npz"))
    hbm = copy_bandwidth(torch)
    mfma = mfma_peak(torch, lib)
    cold = None if args.no_cold else cold_frames(torch, frame, args.steps)

    # the low-precision form on the same frame: without refinement (the float64
    # oracle's algorithm on a rounded data term) and with two refinement passes
    lowp = None if args.no_lowp else lowp_bench(M, _lib, sc, frame, timed, state, G, args)
    kpb = None if args.no_keypoints else keypoint_bench(M, sc, frame, timed, state, params, G, args, torch)
    lmb = None if args.no_lm else lm_bench(M, frame, timed, state, params, G, args)
    jb = None if args.no_joint else joint_bench(M, sc, frame, timed, state, params, G, args)

    out = {
        "metric": "GN iters/s + ms/frame at 640x480, 1600 ED nodes, rel err vs FP64 oracle",
        "value": round(gn_per_s, 2),
        "unit": "GN iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_frame, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {cam.width}x{cam.height} depth, {n} points, {m} nodes, k={params.k}, "
                               f"{G} GN x {params.pcg_iters} PCG per frame; step = graph setup + registration + fusion",
                   "nnzb": nnzb, "n_valid_mean": n_valid},
        "ms_per_frame": round(ms_frame, 4),
        "gn_iter_ms_profiled": round(gn_iter_ms, 4),
        "phases": {k: {"avg_us": round(v["avg_us"], 2), "launches": v["launches"]} for k, v in phases.items()},
        "accuracy": acc,
        "report_final": {"e_data": float(rep[-1]["e_data"]), "e_rot": float(rep[-1]["e_rot"]),
                         "e_reg": float(rep[-1]["e_reg"]), "n_valid": int(rep[-1]["n_valid"]),
                         "flags": int(rep[-1]["flags"])},
        "roofline": roofline,
        "roofline_other": [v for k, v in lines.items() if k != dominant],
        "hbm_copy": hbm,
        "mfma_bf16_probe": mfma,
    }
    if cold is not None:
        out["cold_cache"] = cold
    if lowp is not None:
        out["low_precision"] = lowp
    if kpb is not None:
        out["keypoints"] = kpb
    if lmb is not None:
        out["adaptive_lm"] = lmb
    if jb is not None:
        out["joint_pose"] = jb
    if not args.no_batch:
        out["batch"] = batch_bench(M, _lib, args)
    if seq_frames is not None:
        out["sequence"] = sequence_bench(M, seq_frames)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, params)
    print(json.dumps(out))


def copy_bandwidth(torch, mib=256, reps=10):
    """Achievable HBM bandwidth: a device-to-device copy of mib MiB (read + write bytes over the event time)."""
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * src.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return {"copy_mib": mib, "achieved_gbs": round(gbs, 1), "of_peak": round(gbs / HBM_PEAK_GBS, 4)}


def mfma_peak(torch, lib, iters=20000):
    """Achievable dense bf16 matrix-core rate: four workgroups of four waves per CU, each wave running eight
    independent chains of 16x16x32 multiply-adds (misslam_probe_mfma_bf16), timed with events."""
    import ctypes
    blocks = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    sink = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    flops = ctypes.c_int64()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for _ in range(2):
        lib.misslam_probe_mfma_bf16(iters // 10, blocks, ctypes.c_void_p(sink.data_ptr()), ctypes.byref(flops), stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    st = lib.misslam_probe_mfma_bf16(iters, blocks, ctypes.c_void_p(sink.data_ptr()), ctypes.byref(flops), stream)
    e1.record()
    torch.cuda.synchronize()
    if st != 0:
        return None
    tflops = flops.value / (e0.elapsed_time(e1) * 1e-3) / 1e12
    return {"achieved_tflops": round(tflops, 1), "of_peak": round(tflops / MFMA_BF16_PEAK, 4),
            "peak_tflops": MFMA_BF16_PEAK, "workgroups": blocks}


def cold_frames(torch, frame, steps, flush_mib=512):
    """The frame with cold caches: before each frame a 512 MiB buffer is written, which evicts the 256 MB
    last-level cache and the L2s; the frame alone is timed with events on the same stream."""
    buf = torch.empty(flush_mib << 18, dtype=torch.float32, device="cuda")
    times = []
    for k in range(steps):
        buf.fill_(float(k))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        frame()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    del buf
    return {"flush_mib": flush_mib, "ms_per_frame": round(float(np.mean(times)), 4),
            "ms_per_frame_min": round(float(np.min(times)), 4)}


_SEQ = None


def _sequence_frame(f):
    global _SEQ
    if _SEQ is None:
        from gen.sequence import Sequence
        _SEQ = Sequence()
    return _SEQ.frame(f)


def generate_sequence(frames):
    """Frames 0..frames-1 of the sweep, generated in parallel worker processes (fork, before any GPU use)."""
    import multiprocessing as mp
    workers = max(1, min(16, len(os.sched_getaffinity(0)), frames))
    t0 = time.perf_counter()
    if workers == 1:
        data = [_sequence_frame(f) for f in range(frames)]
    else:
        with mp.get_context("fork").Pool(workers) as pool:
            data = pool.map(_sequence_frame, range(frames), chunksize=1)
    print(f"sequence: {frames} frames generated in {time.perf_counter() - t0:.1f} s on {workers} processes",
          file=sys.stderr, flush=True)
    return data


def batch_bench(M, _lib, args, count=16):
    """16 uneven problems (frames 320x240 to 640x480, 21k-264k points, 104-1716 nodes):
    16 single registration calls against one batched call replayed from its hipGraph."""
    import torch

    import gen
    probs = []
    for b in range(count):
        sc = gen.make_scene(gen.batch_spec(b))
        pts = torch.tensor(np.concatenate([sc["points"].T, sc["normals"].T]), device="cuda").contiguous()
        nodes = torch.tensor(np.ascontiguousarray(sc["nodes"].T), device="cuda").contiguous()
        depth = torch.tensor(sc["depth"], device="cuda").contiguous()
        params = M.Params(sigma=sc["sigma"], gn_iters=sc["gn_iters"], pcg_iters=sc["pcg_iters"])
        ws = M.Workspace()
        g = M.build_graph(pts, nodes, params, ws)
        probs.append(dict(points=pts, nodes=nodes, x=M.identity_params(nodes.shape[1]), graph=g, depth=depth,
                          cam=M.camera(*sc["camera"]), pose=M.pose(sc["R"], sc["T"]), params=params, ws=ws))
    torch.cuda.synchronize()
    n_tot = sum(p["points"].shape[1] for p in probs)
    m_tot = sum(p["nodes"].shape[1] for p in probs)
    G = probs[0]["params"].gn_iters

    def singles():
        for p in probs:
            p["x"].copy_(M.identity_params(p["x"].shape[0]))
            M.gn_register(p["points"], p["nodes"], p["x"], p["graph"], p["depth"], p["cam"], p["pose"], p["params"],
                          p["ws"])

    bt = M.Batch(probs, probs[0]["params"], rows_per_wg=0)

    def batched():
        for p in probs:
            p["x"].copy_(M.identity_params(p["x"].shape[0]))
        bt.register()

    res = {}
    for name, fn in (("single_calls", singles), ("batched_graph", batched)):
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        res[name] = {"ms_per_batch_frame": round(1000 * dt, 4), "gn_iters_per_s": round(count * G / dt, 1)}
    out = {"workload": f"{count} uneven problems, {n_tot} points and {m_tot} nodes in all, {G} GN x "
                       f"{probs[0]['params'].pcg_iters} PCG each; a step registers every problem once",
           "solve_tile_rows": bt.tile, "asm_waves_per_row": bt.asm_waves, "tile_source": bt.tile_source, **res,
           "speedup": round(res["single_calls"]["ms_per_batch_frame"] / res["batched_graph"]["ms_per_batch_frame"], 3)}
    bt.close()
    return out


def lowp_bench(M, _lib, sc, frame, timed, state, G, args):
    """The low-precision forms on the same frame: bf16 and fp16 data terms without refinement (the float64
    oracle's algorithm on a rounded data term) and with two refinement passes, each against the plain and the
    same-form oracle runs.  Beside them, the float32 form with the PCG work of two refinement passes (three
    10-iteration solves per step: 30 PCG iterations), against the oracle run with 30 PCG iterations."""
    lowp = {"form": "bf16 / fp16 data-term J^T J on the matrix cores (fp32 accumulation); refine_steps fp32 "
                    "matrix-free refinement passes per GN step"}
    plain = os.path.join(ROOT, "tests", "golden", f"{args.config}_oracle.npz")
    for prec, code in (("bf16", _lib.PREC_BF16), ("fp16", _lib.PREC_FP16)):
        for steps in (0, 2):
            lp = M.Params(sigma=sc["sigma"], gn_iters=sc["gn_iters"], pcg_iters=sc["pcg_iters"],
                          precision=code, refine_steps=steps)
            for _ in range(max(1, args.warmup)):
                frame(lp)
            lp_elapsed = timed(lp, args.steps)
            lp_rep = M.read_report(state["rep"])
            entry = {"refine_steps": steps, "ms_per_frame": round(1000.0 * lp_elapsed / args.steps, 4),
                     "gn_iters_per_s": round(G * args.steps / lp_elapsed, 2),
                     "accuracy_vs_fp64_oracle": accuracy(state, lp_rep, plain),
                     "accuracy_vs_same_form_oracle": accuracy(
                         state, lp_rep, os.path.join(ROOT, "tests", "golden", f"{args.config}_{prec}_r{steps}_oracle.npz")),
                     "e_data_final": float(lp_rep[-1]["e_data"])}
            lowp[f"{prec}_r{steps}"] = entry
    p30 = M.Params(sigma=sc["sigma"], gn_iters=sc["gn_iters"], pcg_iters=3 * sc["pcg_iters"])
    for _ in range(max(1, args.warmup)):
        frame(p30)
    el = timed(p30, args.steps)
    rep30 = M.read_report(state["rep"])
    lowp["fp32_pcg30"] = {"pcg_iters": p30.pcg_iters, "ms_per_frame": round(1000.0 * el / args.steps, 4),
                          "gn_iters_per_s": round(G * args.steps / el, 2),
                          "accuracy_vs_same_work_oracle": accuracy(
                              state, rep30, os.path.join(ROOT, "tests", "golden", f"{args.config}_pcg30_oracle.npz")),
                          "e_data_final": float(rep30[-1]["e_data"])}
    for prec in ("bf16", "fp16"):
        lowp[f"{prec}_r2_vs_fp32_same_pcg_work"] = round(
            lowp["fp32_pcg30"]["ms_per_frame"] / lowp[f"{prec}_r2"]["ms_per_frame"], 3)
    return lowp


def keypoint_bench(M, sc, frame, timed, state, params, G, args, torch):
    """The Eq.(9) key-point term added to the same frame: 500 generated matches (gen.keypoints, seed 7,
    0.05 mm noise, w_corr = 10), against the stored float64 oracle run of the same problem."""
    import gen
    kp, tgt = gen.keypoints(sc, 500, seed=7, noise=0.05)
    keys = M.keypoints(torch.tensor(kp, device="cuda"), torch.tensor(tgt, device="cuda").contiguous(), 10.0)
    for _ in range(max(1, args.warmup)):
        frame(params, keys)
    el = timed(params, args.steps, keys)
    rep = M.read_report(state["rep"])
    gold = os.path.join(ROOT, "tests", "golden", f"{args.config}_kp500_oracle.npz")
    acc = accuracy(state, rep, gold)
    if os.path.exists(gold):
        z = np.load(gold)
        acc["rel_err_e_corr_final"] = float(abs(rep[-1]["e_corr"] - z["e_corr_final"]) / z["e_corr_final"])
    return {"workload": "the same frame with 500 key-point matches (Eq.(9), w_corr = 10)",
            "ms_per_frame": round(1000.0 * el / args.steps, 4), "gn_iters_per_s": round(G * args.steps / el, 2),
            "e_corr": [float(rep[0]["e_corr"]), float(rep[-1]["e_corr"])], "accuracy_vs_fp64_oracle": acc}


def sequence_bench(M, data):
    """The sweeping, breathing 250 x 200 mm sheet at 640x480: frame 0 lifts the first model and its nodes;
    every later frame runs graph setup, registration (10 x 10), fusion and growth/maintenance.  Frames are
    generated on the host before timing; only the GPU frame loop is timed, frame by frame (a host read of the
    new model size closes every frame, as a caller sizing the next frame's buffers must)."""
    import torch

    frames = len(data) - 1
    cap_n, cap_m = 2_000_000, 12_000
    P = torch.zeros((6, cap_n), device="cuda")
    W = torch.zeros(cap_n, device="cuda")
    S = torch.zeros(cap_n, dtype=torch.int32, device="cuda")
    G = torch.zeros((3, cap_m), device="cuda")
    X = torch.zeros((cap_m, 12), device="cuda")
    params = M.Params(sigma=2.5, gn_iters=10, pcg_iters=10)
    ws, ws_g = M.Workspace(), M.Workspace()
    frames_in = []
    for d in data:
        frames_in.append(dict(depth=torch.tensor(d["depth"], device="cuda"), cam=M.camera(*d["camera"]),
                              pose=M.pose(d["R"], d["T"])))
    torch.cuda.synchronize()
    # frame 0: the first model is the lifted frame
    f0 = frames_in[0]
    nmap = M.normal_map(f0["depth"], f0["cam"])
    none = torch.full((f0["cam"].height, f0["cam"].width), -1, dtype=torch.int32, device="cuda")
    c = M.grow(P, W, S, 0, G, X, 0, none, torch.zeros(1, dtype=torch.int32, device="cuda"), nmap, f0["cam"],
               f0["pose"], M.grow_params(0, 2.5), ws_g).cpu().numpy()
    n, m = int(c[0]), int(c[1])
    sizes = [(n, m)]
    torch.cuda.synchronize()
    flags = overflow = 0
    first_flag = {}      # flag bit -> first frame whose report carries it
    first_overflow = None
    per_frame = []
    t0 = time.perf_counter()
    for f in range(1, frames + 1):
        tf = time.perf_counter()
        fi = frames_in[f]
        g = M.build_graph(P[:, :n], G[:, :m], params, ws)
        rep, _ = M.gn_register(P[:, :n], G[:, :m], X[:m], g, fi["depth"], fi["cam"], fi["pose"], params, ws)
        nmap = M.normal_map(fi["depth"], fi["cam"])
        reg, regd = M.fuse(P[:, :n], W[:n], S[:n], G[:, :m], X[:m], g, nmap, fi["cam"], fi["pose"],
                           M.fuse_params(f), ws, outputs=True)
        c = M.grow(P, W, S, n, G, X, m, reg, regd, nmap, fi["cam"], fi["pose"], M.grow_params(f, 2.5),
                   ws_g).cpu().numpy()
        ff = int(np.bitwise_or.reduce(M.read_report(rep)["flags"]))
        flags |= ff
        for bit in range(8):
            if ff & (1 << bit) and (1 << bit) not in first_flag:
                first_flag[1 << bit] = f
        if c[6] and first_overflow is None:
            first_overflow = f
        overflow |= int(c[6])
        n, m = int(c[0]), int(c[1])
        sizes.append((n, m))
        per_frame.append(1000.0 * (time.perf_counter() - tf))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / frames
    out = {"workload": f"sweep over a breathing 250x200 mm sheet, 640x480, frames 1..{frames} after the lifted "
                       f"frame 0; graph + 10x10 registration + fusion + growth per frame",
           "frames": frames, "ms_per_frame": round(1000 * dt, 3), "report_flags": flags,
           "first_frame_of_flag": {str(k): v for k, v in sorted(first_flag.items())},
           "capacity_overflow": overflow, "first_capacity_overflow_frame": first_overflow,
           "final_points_nodes": sizes[-1]}
    if frames <= 20:
        out["points_nodes_per_frame"] = sizes
    else:   # ms per frame against model size, in bins of 25 frames
        out["by_model_size"] = [{"frames": [f0_ + 1, min(f0_ + 25, frames)],
                                 "points_nodes_at_end": sizes[min(f0_ + 25, frames)],
                                 "ms_per_frame": round(float(np.mean(per_frame[f0_:f0_ + 25])), 3)}
                                for f0_ in range(0, frames, 25)]
    return out


def lm_bench(M, frame, timed, state, params, G, args):
    """The same frame with adaptive Levenberg-Marquardt damping (default schedule): each step also evaluates
    the objective at its trial point.  Against the stored float64 oracle run of the same schedule."""
    lm = M.LMParams()
    for _ in range(max(1, args.warmup)):
        frame(params, None, lm)
    el = timed(params, args.steps, None, lm)
    rep = M.read_report(state["rep"])
    gold = os.path.join(ROOT, "tests", "golden", f"{args.config}_lm_oracle.npz")
    acc = accuracy(state, rep, gold)
    dec = "".join("A" if a else "r" for a in rep["lm_accepted"][:G])
    out = {"workload": "the same frame, adaptive damping (lambda0 1e-3, x0.1 on a taken step, x10 on a rejected "
                       "one, within [1e-6, 1e6])",
           "ms_per_frame": round(1000.0 * el / args.steps, 4), "gn_iters_per_s": round(G * args.steps / el, 2),
           "decisions": dec, "lambda": [float(v) for v in rep["lm_lambda"][:G]],
           "accuracy_vs_fp64_oracle": acc}
    if os.path.exists(gold):
        z = np.load(gold)
        out["oracle_decisions"] = "".join("A" if a else "r" for a in z["accepted"])
    return out


def joint_bench(M, sc, frame, timed, state, params, G, args):
    """The same frame registering the rigid pose with the ED graph (Eq.(10) terms, w_r = 1e6, w_p = 1e3), the
    generated pose as start and prior; against the stored float64 oracle run of the same problem."""
    for _ in range(max(1, args.warmup)):
        frame(params, None, None, True)
    el = timed(params, args.steps, None, None, True)
    rep = M.read_report(state["rep"])
    gold = os.path.join(ROOT, "tests", "golden", f"{args.config}_joint_oracle.npz")
    acc = accuracy(state, rep, gold)
    P = state["pose"].cpu().numpy().astype(np.float64)
    R0 = np.asarray(sc["R"], np.float32).astype(np.float64)
    T0 = np.asarray(sc["T"], np.float32).astype(np.float64)
    out = {"workload": "the same frame, pose + ED unknowns (Eq.(10) priors at the generated pose)",
           "ms_per_frame": round(1000.0 * el / args.steps, 4), "gn_iters_per_s": round(G * args.steps / el, 2),
           "pose_moved": {"max_abs_dR": float(np.abs(P[:9].reshape(3, 3) - R0).max()),
                          "max_abs_dT_mm": float(np.abs(P[9:] - T0).max())},
           "e_data": [float(rep[0]["e_data"]), float(rep[-1]["e_data"])], "accuracy_vs_fp64_oracle": acc}
    if os.path.exists(gold):
        z = np.load(gold)
        acc["max_abs_err_R"] = float(np.abs(P[:9].reshape(3, 3) - z["R"]).max())
        acc["max_abs_err_T_mm"] = float(np.abs(P[9:] - z["T"]).max())
    return out


def accuracy(state, rep, gold):
    """Relative errors of the frame's parameters and final data energy against a stored oracle run."""
    if not os.path.exists(gold):
        return {}
    xg = state["x"].cpu().numpy().astype(np.float64)
    z = np.load(gold)
    xo = z["x"]
    xi = np.zeros_like(xo)
    xi[:, [0, 4, 8]] = 1.0
    return {"rel_err_params": float(np.linalg.norm(xg - xo) / np.linalg.norm(xo)),
            "rel_err_params_delta": float(np.linalg.norm((xg - xi) - (xo - xi)) / np.linalg.norm(xo - xi)),
            "rel_err_e_data_final": float(abs(rep[-1]["e_data"] - z["e_data_final"]) / z["e_data_final"])}


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(sc, params, reps=3):
    """Float64 oracle on the same frame: its graph setup once, then one GN iteration (10 PCG) timed reps times
    with BLAS limited to one thread and reps times with BLAS on every core the process may use; medians.
    NumPy's elementwise work runs on one thread either way."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    import oracle
    from oracle.gn import linearize
    from oracle.pcg import block_jacobi, pcg

    pb = oracle.Problem.from_scene(sc, gn_iters=1)
    t0 = time.perf_counter()
    graph = oracle.build_graph(pb.points, pb.nodes, pb.k, pb.weight_kind, pb.sigma)
    t1 = time.perf_counter()
    Nmap, Nvalid = oracle.normal_map(pb.depth, pb.camera)
    x = oracle.identity_params(len(pb.nodes))

    def gn_iteration():
        ta = time.perf_counter()
        _, _, _, blocks, g, _ = linearize(pb, graph, x, Nmap, Nvalid)
        Minv, _ = block_jacobi(graph["row_ptr"], graph["col_idx"], blocks, pb.lam)
        pcg(graph["row_ptr"], graph["col_idx"], blocks, g, pb.lam, params.pcg_iters, Minv)
        return time.perf_counter() - ta

    def timed(limit):
        ctx = threadpool_limits(limit) if threadpool_limits else None
        try:
            return float(np.median([gn_iteration() for _ in range(reps)]))
        finally:
            if ctx is not None:
                ctx.__exit__(None, None, None)

    cores = len(os.sched_getaffinity(0))
    one = timed(1)
    allc = timed(cores)
    return {"value": round(1.0 / allc, 4), "unit": "GN iters/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"one GN iteration ({params.pcg_iters} PCG) of the same frame after the oracle's graph setup "
                      f"({t1 - t0:.1f} s), median of {reps}, float64 numpy/scipy, BLAS on the {cores} cores the "
                      f"process may use; one_thread: the same with BLAS on 1 thread",
            "gn_iter_s": round(allc, 3), "graph_setup_s": round(t1 - t0, 2),
            "one_thread": {"value": round(1.0 / one, 4), "gn_iter_s": round(one, 3), "cores": 1}}


if __name__ == "__main__":
    main()
