"""Model growth and maintenance after fusion (Alg. 2 steps 3-5, Alg. 3).

Readings where the paper is silent or loose:
  * Group 2 (Alg. 2 step 3): every pixel with depth and a valid depth normal
    whose Reg winner is absent or failed the Alg. 1 test is lifted into the
    world, p = R^T (V(u) - T), n = R^T N(u), with weight 1 (the unit
    observation weight of Eq.(15)) and the frame's stamp.  Lifted points follow
    the surviving points, in pixel order.
  * Removal (Alg. 2 step 4, Alg. 3): a point is deleted when its age
    frame - stamp exceeds tau_time (10, Sec. III-B) and its weight is below
    tau_weight (2; the paper gives no value).  Points registered this frame
    were stamped by the fusion, so the rule reaches only the others.
  * Down-sampling (Alg. 3, "fixed box" of 0.22 mm, Sec. III-B): voxels of edge
    `voxel` with the origin at 0; key floor(coordinate / voxel) in float64.  A
    voxel is touched when one of its points carries this frame's stamp.  The
    points of a touched voxel with two or more members merge into the member
    of lowest index: mean position, renormalised mean normal (float64 sums in
    ascending index order), largest weight, largest stamp.
  * Node regeneration (Alg. 2 step 5; silent): voxels of the node spacing s
    with the origin at 0; every such voxel holding points gives the centroid
    of its points (float64, ascending index), and a node is added there when
    no node of the frame lies within s of it (d^2 >= s^2).  New nodes follow
    the old ones in ascending (kz, ky, kx) order of their voxel.  kNN sets,
    N(j) and the pattern are rebuilt by the next frame's graph setup, and the
    parameters restart at identity.
  * Colour (Eq.(13)), when the model carries it: survivors keep theirs, a
    lifted point takes the frame's colour at its pixel, a merged voxel the
    mean of its members' colours (float64, ascending index).
  * Stability S_i (Sec. II-G: unstable points, seen in few frames and not
    recently, are dropped; Alg. 3): a point becomes stable once it has been
    registered in enough frames, its weight (one per registration, Eq.(15))
    having reached tau_weight, and stays stable from then on, as in the
    point fusion of Keller et al. 2013 that the section follows.  Removal
    deletes an unstable point whose age exceeds tau_time; a lifted point
    starts stable only if its weight 1 reaches tau_weight; a merged voxel is
    stable when one of its members is.  With S_i = (weight >= tau_weight) on
    entry the removal is the weight rule above.
Test infrastructure only (see the package header).
"""
import numpy as np


def _vertex(depth, camera):
    W, H, fx, fy, cx, cy = camera
    fx, fy, cx, cy = (float(np.float32(a)) for a in (fx, fy, cx, cy))
    D = np.asarray(depth, dtype=np.float64)
    v, u = np.mgrid[0:H, 0:W]
    return np.stack([D * ((u - cx) / fx), D * ((v - cy) / fy), D], axis=-1)


def voxel_keys(p, edge):
    """Integer voxel coordinates (N, 3) of float32 points, floor(x / edge) in float64."""
    return np.floor(np.asarray(p, dtype=np.float64) / float(edge)).astype(np.int64)


def _groups(keys):
    """Members of each distinct key, ascending index, groups in (kz, ky, kx) order."""
    order = np.lexsort((np.arange(len(keys)), keys[:, 0], keys[:, 1], keys[:, 2]))
    ks = keys[order]
    start = np.ones(len(order), dtype=bool)
    start[1:] = np.any(ks[1:] != ks[:-1], axis=1)
    bounds = np.append(np.nonzero(start)[0], len(order))
    return [order[bounds[g]:bounds[g + 1]] for g in range(len(bounds) - 1)]


def grow(points, normals, weight, stamp, registered, reg, depth, camera, R, T, Nmap, Nvalid, frame, nodes,
         node_spacing, voxel=0.22, tau_time=10, tau_weight=2.0, color=None, image=None, stable=None):
    """Alg. 2 steps 3-5 and Alg. 3 on a fused model.  Returns dict(points, normals,
    weight, stamp (float32/int arrays of the new model), nodes (old + new),
    lifted, culled, merged (counts)[, color][, stable]).  stable: the points'
    S_i flags (bool) when the model carries them."""
    P = np.asarray(points, dtype=np.float64)
    Nn = np.asarray(normals, dtype=np.float64)
    w = np.asarray(weight, dtype=np.float64)
    st = np.asarray(stamp, dtype=np.int64)
    regd = np.asarray(registered, dtype=bool)
    W, H = camera[0], camera[1]
    Rm = np.asarray(R, dtype=np.float64)
    Tv = np.asarray(T, dtype=np.float64)

    # stability, then removal (Alg. 3)
    S = w >= tau_weight
    if stable is not None:
        S = S | np.asarray(stable, dtype=bool)
    keep = ~((frame - st > tau_time) & ~S)
    # Group 2: unregistered pixels with depth and a normal
    win = np.asarray(reg, dtype=np.int64).reshape(-1)
    reg_pix = np.zeros(W * H, dtype=bool)
    has = win >= 0
    reg_pix[has] = regd[win[has]]
    D = np.asarray(depth, dtype=np.float64).reshape(-1)
    lift = (D > 0) & np.asarray(Nvalid, dtype=bool).reshape(-1) & ~reg_pix
    V = _vertex(depth, camera).reshape(-1, 3)[lift]
    Nm = np.asarray(Nmap, dtype=np.float64).reshape(-1, 3)[lift]
    dv = V - Tv
    # R^T (V - T) and R^T N, each component summed as ((r0 x0 + r1 x1) + r2 x2)
    lp = np.stack([(Rm[0, a] * dv[:, 0] + Rm[1, a] * dv[:, 1]) + Rm[2, a] * dv[:, 2] for a in range(3)],
                  axis=1).astype(np.float32)
    ln = np.stack([(Rm[0, a] * Nm[:, 0] + Rm[1, a] * Nm[:, 1]) + Rm[2, a] * Nm[:, 2] for a in range(3)],
                  axis=1).astype(np.float32)

    pts = np.concatenate([P[keep].astype(np.float32), lp])
    nrm = np.concatenate([Nn[keep].astype(np.float32), ln])
    wt = np.concatenate([w[keep], np.ones(len(lp))]).astype(np.float32)
    stp = np.concatenate([st[keep], np.full(len(lp), frame, dtype=np.int64)])
    stab = np.concatenate([S[keep], np.full(len(lp), 1.0 >= tau_weight)])
    col = None
    if color is not None:
        col = np.concatenate([np.asarray(color, dtype=np.float32)[keep],
                              np.asarray(image, dtype=np.float32).reshape(-1, 3)[lift]])

    # down-sampling of touched voxels (Alg. 3)
    alive = np.ones(len(pts), dtype=bool)
    merged = 0
    if len(pts):
        for members in _groups(voxel_keys(pts, np.float32(voxel))):
            if len(members) < 2 or not np.any(stp[members] == frame):
                continue
            lead = members[0]
            pm = pts[members].astype(np.float64)
            nm = nrm[members].astype(np.float64)
            ps = np.zeros(3)
            ns = np.zeros(3)
            for q in range(len(members)):          # ascending index order
                ps = ps + pm[q]
                ns = ns + nm[q]
            pts[lead] = (ps / len(members)).astype(np.float32)
            nmean = ns / len(members)
            nrm[lead] = (nmean / np.sqrt((nmean[0] * nmean[0] + nmean[1] * nmean[1]) + nmean[2] * nmean[2])).astype(
                np.float32)
            wt[lead] = wt[members].max()
            stp[lead] = stp[members].max()
            stab[lead] = stab[members].any()
            if col is not None:
                cm = col[members].astype(np.float64)
                cs = np.zeros(3)
                for q in range(len(members)):
                    cs = cs + cm[q]
                col[lead] = (cs / len(members)).astype(np.float32)
            alive[members[1:]] = False
            merged += len(members) - 1
    pts, nrm, wt, stp, stab = pts[alive], nrm[alive], wt[alive], stp[alive], stab[alive]
    if col is not None:
        col = col[alive]

    # node regeneration (Alg. 2 step 5)
    G = np.asarray(nodes, dtype=np.float32)
    s = float(np.float32(node_spacing))
    new_nodes = []
    if len(pts):
        G64 = G.astype(np.float64)
        for members in _groups(voxel_keys(pts, np.float32(node_spacing))):
            pm = pts[members].astype(np.float64)
            c = np.zeros(3)
            for q in range(len(members)):
                c = c + pm[q]
            c = c / len(members)
            if len(G64):
                d = c[None, :] - G64
                d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
                if np.min(d2) < s * s:
                    continue
            new_nodes.append(c.astype(np.float32))
    nodes_out = np.concatenate([G, np.array(new_nodes, dtype=np.float32).reshape(-1, 3)])
    out = {"points": pts, "normals": nrm, "weight": wt, "stamp": stp, "nodes": nodes_out,
           "lifted": int(lift.sum()), "culled": int((~keep).sum()), "merged": merged, "new_nodes": len(new_nodes)}
    if col is not None:
        out["color"] = col
    if stable is not None:
        out["stable"] = stab
    return out
