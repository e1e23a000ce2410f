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
