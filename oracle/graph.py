"""Point-to-node neighbourhoods, skinning weights and the node graph (Sec. II-D, II-E).

Test infrastructure only (see the package header).
"""
import numpy as np


def sq_dist(points, nodes):
    """Squared Euclidean distances, formed as ((dx*dx + dy*dy) + dz*dz) in float64.

    The order of the sum is fixed so that the nearest-node decision is
    reproducible bit for bit by any implementation that keeps the same order.
    """
    P = np.asarray(points, dtype=np.float64)
    G = np.asarray(nodes, dtype=np.float64)
    dx = P[:, None, 0] - G[None, :, 0]
    dy = P[:, None, 1] - G[None, :, 1]
    dz = P[:, None, 2] - G[None, :, 2]
    return (dx * dx + dy * dy) + dz * dz


def knn(points, nodes, k, chunk=8192):
    """The k+1 nearest nodes of every point, ordered by (squared distance, node index).

    Sec. II-D: each point is moved by its k nearest ED nodes, and Eq.(2) needs the
    distance to the (k+1)-th.  Reading: Euclidean distance in the canonical frame,
    ties broken towards the lower node index.  Returns (idx (N, k+1) int64,
    d2 (N, k+1) float64); when there are only k nodes the last column is -1 / inf.
    """
    P = np.asarray(points, dtype=np.float64)
    G = np.asarray(nodes, dtype=np.float64)
    n, m = P.shape[0], G.shape[0]
    kk = min(k + 1, m)
    idx = np.full((n, k + 1), -1, dtype=np.int64)
    d2o = np.full((n, k + 1), np.inf)
    for s in range(0, n, chunk):
        d2 = sq_dist(P[s:s + chunk], G)
        order = np.argsort(d2, axis=1, kind="stable")[:, :kk]   # stable: ties keep index order
        idx[s:s + chunk, :kk] = order
        d2o[s:s + chunk, :kk] = np.take_along_axis(d2, order, axis=1)
    return idx, d2o


def skin_weights(d2, k, kind="gauss", sigma=1.0):
    """Normalised skinning weights over the k nearest nodes (Eq.(2)).

    Reading: the weights are normalised to sum to one over the k nodes, which is
    what lets identical node transforms reproduce a rigid motion.
      kind="gauss":  w_j proportional to exp(-|v - g_j|^2 / (2 sigma^2))
      kind="linear": Eq.(2), w_j proportional to max(0, 1 - |v - g_j| / d_max) with
                     d_max the distance to the (k+1)-th node; all-zero rows get 1/k.
    """
    d2 = np.asarray(d2, dtype=np.float64)
    if kind == "gauss":
        w = np.exp(-d2[:, :k] / (2.0 * sigma * sigma))
    elif kind == "linear":
        d = np.sqrt(d2[:, :k])
        dmax = np.sqrt(d2[:, k])
        w = np.maximum(0.0, 1.0 - d / dmax[:, None])
        w = np.where(np.isfinite(w), w, 0.0)
    else:
        raise ValueError(kind)
    s = w.sum(axis=1, keepdims=True)
    uniform = np.full_like(w, 1.0 / k)
    return np.where(s > 0, w / np.where(s > 0, s, 1.0), uniform)


def node_graph(idx, m, k):
    """N(j) of Eq.(6): l is a neighbour of j iff some point has both j and l among its k nodes.

    Reading (the embedded-deformation construction the paper follows for its
    regularisers): co-influence of two nodes on a common point.  The relation is
    symmetric and excludes j itself.  Returns a list of sorted int arrays.
    """
    idx = np.asarray(idx)[:, :k]
    adj = np.zeros((m, m), dtype=bool)
    for a in range(k):
        for b in range(k):
            if a != b:
                adj[idx[:, a], idx[:, b]] = True
    np.fill_diagonal(adj, False)
    return [np.nonzero(adj[j])[0] for j in range(m)]


def bsr_pattern(nbrs):
    """Block pattern of the normal equations: row j holds {j} and N(j), columns ascending."""
    m = len(nbrs)
    cols = [np.unique(np.concatenate([[j], nbrs[j]])).astype(np.int64) for j in range(m)]
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum([len(c) for c in cols])
    col_idx = np.concatenate(cols) if m else np.zeros(0, dtype=np.int64)
    return row_ptr, col_idx


def build_graph(points, nodes, k, kind="gauss", sigma=1.0):
    idx, d2 = knn(points, nodes, k)
    w = skin_weights(d2, k, kind, sigma)
    nbrs = node_graph(idx, len(nodes), k)
    row_ptr, col_idx = bsr_pattern(nbrs)
    return {"idx": idx[:, :k], "idx_all": idx, "d2": d2, "w": w, "nbrs": nbrs,
            "row_ptr": row_ptr, "col_idx": col_idx}
