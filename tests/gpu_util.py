"""Helpers shared by the GPU tests: upload a generated scene and run oracle stages on GPU outputs."""
import math

import numpy as np
import torch

import gen


class Scene:
    def __init__(self, name, **kw):
        from paper_1803_02009_amd import misslam as M
        self.M = M
        self.sc = sc = gen.make_scene(name, **kw) if isinstance(name, str) else name
        self.dev = "cuda"
        self.pts = torch.tensor(np.concatenate([sc["points"].T, sc["normals"].T]), device=self.dev).contiguous()
        self.nodes = torch.tensor(np.ascontiguousarray(sc["nodes"].T), device=self.dev).contiguous()
        self.depth = torch.tensor(sc["depth"], device=self.dev).contiguous()
        self.cam = M.camera(*sc["camera"])
        self.pose = M.pose(sc["R"], sc["T"])
        self.params = M.Params(sigma=sc["sigma"], gn_iters=sc.get("gn_iters", 10), pcg_iters=sc.get("pcg_iters", 10))
        self.ws = M.Workspace()
        self.n = self.pts.shape[1]
        self.m = self.nodes.shape[1]
        self._graph = None

    @property
    def graph(self):
        if self._graph is None:
            self._graph = self.M.build_graph(self.pts, self.nodes, self.params, self.ws)
            torch.cuda.synchronize()
        return self._graph

    def problem(self, **kw):
        import oracle
        p = self.params
        args = dict(k=p.k, sigma=p.sigma, w_rot=p.w_rot, w_reg=p.w_reg, w_data=p.w_data, eps_d=p.eps_d,
                    cos_eps_n=p.cos_eps_n, lam=float(np.float32(p.lam)), gn_iters=p.gn_iters, pcg_iters=p.pcg_iters)
        args.update(kw)
        return oracle.Problem.from_scene(self.sc, **args)

    def oracle_graph_from_gpu(self):
        """Oracle graph dict built on the GPU's kNN sets and weights (for stage-wise checks)."""
        import oracle
        g = self.graph
        idx = g.knn_idx.cpu().numpy().T.astype(np.int64)
        w = g.knn_w.cpu().numpy().T.astype(np.float64)
        nbrs = oracle.node_graph(idx, self.m, self.params.k)
        rp, ci = oracle.bsr_pattern(nbrs)
        return {"idx": idx, "w": w, "nbrs": nbrs, "row_ptr": rp, "col_idx": ci}


def random_params(m, seed, scale_a=0.02, scale_t=0.5):
    rng = np.random.default_rng(seed)
    x = np.zeros((m, 12))
    x[:, 0] = x[:, 4] = x[:, 8] = 1.0
    x[:, :9] += rng.normal(scale=scale_a, size=(m, 9))
    x[:, 9:] = rng.normal(scale=scale_t, size=(m, 3))
    return x.astype(np.float32)


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


COS10 = math.cos(math.radians(10.0))


def check_energy(s, x_gpu, e_gpu, x_ref=None, e_ref=None, tol=1e-5, pose_gpu=None, pose_ref=None, label=""):
    """The data energy a registration reports for its state, against float64.

    (1) e_gpu, reported for parameters x_gpu, equals the float64 energy of that state: the oracle's residuals at
        x_gpu over the GPU's own correspondences (those of one point pass at x_gpu, which is what the report
        evaluates), within tol.
    (2) The GPU's float32 decisions at x_gpu differ from the oracle's float64 decisions at the same x_gpu only
        for points within rounding of a pixel boundary or a gate threshold: at most 1e-3 of the valid points.
    When the oracle's own run is given (x_ref, its energy e_ref), the gap between the two runs' energies is
    printed with its two parts: the flipped decisions' share and the share of the parameter difference (points
    whose decisions agree).  That gap follows from the parameters, which the callers gate on their own.
    pose_gpu / pose_ref: (R, T) of each side when the pose was refined too (default: the scene's pose).
    Returns the number of flipped decisions at x_gpu."""
    import dataclasses

    import oracle
    from oracle.gn import _adopt, evaluate
    og = s.oracle_graph_from_gpu()
    pb = s.problem()
    Nm, ok = oracle.normal_map(s.sc["depth"], s.sc["camera"])
    Nm32 = Nm.astype(np.float32)

    def posed(pose):
        return pb if pose is None else dataclasses.replace(pb, R=np.asarray(pose[0], np.float64),
                                                           T=np.asarray(pose[1], np.float64))
    pbg = posed(pose_gpu)
    xg64 = np.asarray(x_gpu, np.float64)
    x = torch.tensor(np.asarray(x_gpu, np.float32), device="cuda")
    nmap = s.M.normal_map(s.depth, s.cam)
    pg = s.pose if pose_gpu is None else s.M.pose(np.asarray(pose_gpu[0], np.float32),
                                                  np.asarray(pose_gpu[1], np.float32))
    _, _, corr, _ = s.M.build_normal_eq(s.pts, s.nodes, x, s.graph, nmap, s.cam, pg, s.params, s.ws)
    cg = corr.cpu().numpy()
    vc = oracle.ed_warp(pb.points, pb.nodes, xg64, og["idx"], og["w"], pbg.R, pbg.T)
    asc_g = _adopt({}, cg, vc, pb, Nm32)
    e64 = float(np.sum(asc_g["r"] ** 2)) * pb.w_data
    _, _, asc_64, _ = evaluate(pbg, og, xg64, Nm32, ok)
    flips = int(np.sum(cg != asc_64["corr"]))
    nvalid = int(asc_64["valid"].sum())
    msg = (f"{label} E_data {e_gpu:.6f} vs float64 of the same state {e64:.6f} ({abs(e_gpu - e64) / e64:.2e} rel);"
           f" {flips} of {nvalid} decisions flip against float64 at the same x")
    if x_ref is not None:
        _, _, asc_r, _ = evaluate(posed(pose_ref), og, np.asarray(x_ref, np.float64), Nm32, ok)
        same = cg == asc_r["corr"]
        d = asc_g["r"] ** 2 - asc_r["r"] ** 2
        msg += (f"; gap to the oracle run {(e_gpu - e_ref) / e_ref:+.2e} rel = flips {np.sum(d[~same]) / e_ref:+.2e}"
                f" ({int((~same).sum())} points) + parameters {np.sum(d[same]) / e_ref:+.2e}"
                f" + arithmetic {(e_gpu - e64) / e_ref:+.2e}")
    print(msg)
    assert abs(e_gpu - e64) <= tol * e64, msg
    assert flips <= 1e-3 * max(nvalid, 1), msg
    return flips
