"""Gauss-Newton linearisation of Eq.(3) and the normal equations H dx = -g (Sec. II-F).

The paper solves Eq.(3) by Levenberg-Marquardt without stating the linear
algebra.  Reading: Gauss-Newton normal equations H = sum_terms w J^T J,
g = sum_terms w J^T r, with 12x12 blocks per node pair.

Jacobians (x_j = (c1, c2, c3, t_j), x[3c + a] = A_j[a, c]):
  data, point i, node j (Eq.(8) with correspondences held fixed):
      d r_i / d x_j = w_ij * kron((v_i - g_j, 1), R^T N_p)       (length 12, index 3c + a)
  rot, node j (Eq.(5)): rows of d(c_a . c_b)/d(c_1, c_2, c_3)
  reg, directed edge (j, l), e = g_l - g_j (Eq.(6)):
      d r / d x_j = [e_1 I, e_2 I, e_3 I, I],  d r / d x_l = [0, 0, 0, -I]
Test infrastructure only (see the package header).
"""
import numpy as np

from .energy import edges, reg_residuals, rot_residuals


def data_jacobian_rows(points, nodes, idx, w, R, Np):
    """Per-point, per-node data Jacobian rows: (N, k, 12)."""
    P = np.asarray(points, dtype=np.float64)
    G = np.asarray(nodes, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    nprime = np.asarray(Np, dtype=np.float64) @ R           # rows: (R^T N)^T
    idx = np.asarray(idx)
    n, k = idx.shape
    J = np.zeros((n, k, 12))
    for s in range(k):
        d = P - G[idx[:, s]]
        dh = np.concatenate([d, np.ones((n, 1))], axis=1)  # (v - g_j, 1)
        J[:, s, :] = w[:, s:s + 1] * (dh[:, :, None] * nprime[:, None, :]).reshape(n, 12)
    return J


def rot_jacobian(params):
    """(m, 6, 12) Jacobian of the Eq.(5) residuals; the t columns are zero."""
    p = np.asarray(params, dtype=np.float64)
    m = p.shape[0]
    c = [p[:, 0:3], p[:, 3:6], p[:, 6:9]]
    J = np.zeros((m, 6, 12))
    pairs = [(0, 1), (0, 2), (1, 2)]
    for row, (a, b) in enumerate(pairs):
        J[:, row, 3 * a:3 * a + 3] = c[b]
        J[:, row, 3 * b:3 * b + 3] = c[a]
    for a in range(3):
        J[:, 3 + a, 3 * a:3 * a + 3] = 2.0 * c[a]
    return J


def reg_jacobian(nodes, nbrs):
    """Per directed edge: (js, ls, Jj (E, 3, 12), Jl (E, 3, 12))."""
    G = np.asarray(nodes, dtype=np.float64)
    js, ls = edges(nbrs)
    e = G[ls] - G[js]
    E = len(js)
    Jj = np.zeros((E, 3, 12))
    Jl = np.zeros((E, 3, 12))
    I = np.eye(3)
    for c in range(3):
        Jj[:, :, 3 * c:3 * c + 3] = e[:, c, None, None] * I
    Jj[:, :, 9:12] = I
    Jl[:, :, 9:12] = -I
    return js, ls, Jj, Jl


def dense_system(points, nodes, params, idx, w, R, assoc, nbrs, weights, corr=None):
    """Explicit dense Jacobian and normal equations (small problems only).

    Rows: one per valid data point, 6 per node (rot), 3 per directed edge (reg),
    3 per key point when corr = {"point", "r" (S, 3), "w_corr"} is given (Eq.(9));
    columns 12 m.  Returns (J, wdiag, r, H, g) with H = J^T diag(w) J and
    g = J^T diag(w) r.
    """
    w_rot, w_reg, w_data = weights
    m = np.asarray(nodes).shape[0]
    valid = assoc["valid"]
    Jd = data_jacobian_rows(points, nodes, idx, w, R, assoc["Np"])
    rows, wts, res = [], [], []
    idx = np.asarray(idx)
    for i in np.nonzero(valid)[0]:
        row = np.zeros(12 * m)
        for s in range(idx.shape[1]):
            j = idx[i, s]
            row[12 * j:12 * j + 12] += Jd[i, s]
        rows.append(row)
        wts.append(w_data)
        res.append(assoc["r"][i])
    Jr = rot_jacobian(params)
    rr = rot_residuals(params)
    for j in range(m):
        for q in range(6):
            row = np.zeros(12 * m)
            row[12 * j:12 * j + 12] = Jr[j, q]
            rows.append(row)
            wts.append(w_rot)
            res.append(rr[j, q])
    js, ls, Jj, Jl = reg_jacobian(nodes, nbrs)
    rg, _, _ = reg_residuals(params, nodes, nbrs)
    for e in range(len(js)):
        for a in range(3):
            row = np.zeros(12 * m)
            row[12 * js[e]:12 * js[e] + 12] += Jj[e, a]
            row[12 * ls[e]:12 * ls[e] + 12] += Jl[e, a]
            rows.append(row)
            wts.append(w_reg)
            res.append(rg[e, a])
    if corr is not None and len(corr["point"]):
        from .corr import corr_jacobian_rows
        Jc = corr_jacobian_rows(points, nodes, idx, w, R, corr["point"])
        for s, p in enumerate(np.asarray(corr["point"])):
            for a in range(3):
                row = np.zeros(12 * m)
                for q in range(idx.shape[1]):
                    j = idx[p, q]
                    row[12 * j:12 * j + 12] += Jc[s, a, q]
                rows.append(row)
                wts.append(corr["w_corr"])
                res.append(corr["r"][s, a])
    J = np.array(rows) if rows else np.zeros((0, 12 * m))
    wd = np.array(wts)
    r = np.array(res)
    H = J.T @ (wd[:, None] * J)
    g = J.T @ (wd * r)
    return J, wd, r, H, g


def block_system(points, nodes, params, idx, w, R, assoc, nbrs, row_ptr, col_idx, weights, jac_round=None,
                 corr=None):
    """The same normal equations accumulated block by block into the BSR pattern.

    Every term's contribution J_a^T J_b is added to block (a, b); the sums use
    np.bincount over block ids, one entry of the 12x12 block at a time.
    jac_round, if given, maps the data-term Jacobian rows before they enter
    the blocks (not the gradient): the rounding a low-precision matrix-core
    product applies to its inputs.  corr = {"point", "r" (S, 3), "w_corr"}
    adds the key-point term of Eq.(9).
    Returns (blocks (nnzb, 12, 12), g (m, 12)).
    """
    w_rot, w_reg, w_data = weights
    G = np.asarray(nodes, dtype=np.float64)
    m = G.shape[0]
    nnzb = len(col_idx)
    # block id lookup (row, col) -> position
    lookup = {}
    for j in range(m):
        for p in range(row_ptr[j], row_ptr[j + 1]):
            lookup[(j, int(col_idx[p]))] = p
    key = np.full((m, m), -1, dtype=np.int64) if m <= 20000 else None
    for (a, b), p in lookup.items():
        key[a, b] = p

    blocks = np.zeros((nnzb, 12, 12))
    gvec = np.zeros((m, 12))

    # data term
    valid = assoc["valid"]
    vi = np.nonzero(valid)[0]
    idx = np.asarray(idx)
    k = idx.shape[1]
    r = assoc["r"]
    chunk = 20000
    for s0 in range(0, len(vi), chunk):
        sel = vi[s0:s0 + chunk]
        Jd = data_jacobian_rows(np.asarray(points)[sel], G, idx[sel], np.asarray(w)[sel], R, assoc["Np"][sel])
        for a in range(k):
            ja = idx[sel, a]
            gvec += w_data * np.stack([np.bincount(ja, weights=Jd[:, a, e] * r[sel], minlength=m)
                                       for e in range(12)], axis=1)
            for b in range(k):
                jb = idx[sel, b]
                bid = key[ja, jb]
                Jl = Jd if jac_round is None else jac_round(Jd)
                outer = Jl[:, a, :, None] * Jl[:, b, None, :]
                for e in range(12):
                    for f in range(12):
                        blocks[:, e, f] += w_data * np.bincount(bid, weights=outer[:, e, f], minlength=nnzb)

    # rot term
    Jr = rot_jacobian(params)
    rr = rot_residuals(params)
    diag = key[np.arange(m), np.arange(m)]
    blocks[diag] += w_rot * np.einsum("mqe,mqf->mef", Jr, Jr)
    gvec += w_rot * np.einsum("mqe,mq->me", Jr, rr)

    # reg term
    js, ls, Jj, Jl = reg_jacobian(G, nbrs)
    rg, _, _ = reg_residuals(params, G, nbrs)
    for (ia, Ja), (ib, Jb) in [((js, Jj), (js, Jj)), ((js, Jj), (ls, Jl)),
                               ((ls, Jl), (js, Jj)), ((ls, Jl), (ls, Jl))]:
        contrib = w_reg * np.einsum("nqe,nqf->nef", Ja, Jb)
        np.add.at(blocks, key[ia, ib], contrib)
    np.add.at(gvec, js, w_reg * np.einsum("nqe,nq->ne", Jj, rg))
    np.add.at(gvec, ls, w_reg * np.einsum("nqe,nq->ne", Jl, rg))

    # key-point term
    if corr is not None and len(corr["point"]):
        from .corr import corr_jacobian_rows
        kp = np.asarray(corr["point"], dtype=np.int64)
        Jc = corr_jacobian_rows(points, G, idx, w, R, kp)        # (S, 3, k, 12)
        rc = np.asarray(corr["r"], dtype=np.float64)             # (S, 3)
        wc = corr["w_corr"]
        for a in range(k):
            ja = idx[kp, a]
            np.add.at(gvec, ja, wc * np.einsum("sre,sr->se", Jc[:, :, a, :], rc))
            for b in range(k):
                jb = idx[kp, b]
                np.add.at(blocks, key[ja, jb], wc * np.einsum("sre,srf->sef", Jc[:, :, a, :], Jc[:, :, b, :]))
    return blocks, gvec


def dense_from_blocks(row_ptr, col_idx, blocks, m):
    H = np.zeros((12 * m, 12 * m))
    for j in range(m):
        for p in range(row_ptr[j], row_ptr[j + 1]):
            l = int(col_idx[p])
            H[12 * j:12 * j + 12, 12 * l:12 * l + 12] = blocks[p]
    return H
