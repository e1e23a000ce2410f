"""Block-Jacobi preconditioned conjugate gradients for (H + lambda I) dx = -g.

The paper's optimiser is Levenberg-Marquardt (Sec. II-F) with no linear-algebra
detail.  Reading: fixed damping lambda added to the diagonal, block-Jacobi
preconditioner M = blockdiag(H_jj + lambda I)^-1, and the textbook
preconditioned CG recurrence run for exactly P iterations from dx = 0; it stops
early only when r^T z = 0 (exact solution) or p^T A p <= 0 (breakdown, flagged).
Test infrastructure only (see the package header).
"""
import numpy as np
import scipy.linalg


def block_jacobi(row_ptr, col_idx, blocks, lam):
    """Inverses of the damped diagonal blocks, (m, 12, 12)."""
    m = len(row_ptr) - 1
    out = np.zeros((m, 12, 12))
    spd = np.ones(m, dtype=bool)
    for j in range(m):
        for p in range(row_ptr[j], row_ptr[j + 1]):
            if col_idx[p] == j:
                Hjj = blocks[p] + lam * np.eye(12)
                try:
                    c = scipy.linalg.cho_factor(Hjj)
                    out[j] = scipy.linalg.cho_solve(c, np.eye(12))
                except np.linalg.LinAlgError:
                    spd[j] = False
                    out[j] = np.eye(12)
    return out, spd


def bsr_matvec(row_ptr, col_idx, blocks, x, lam):
    m = len(row_ptr) - 1
    X = x.reshape(m, 12)
    rows = np.repeat(np.arange(m), np.diff(row_ptr))
    contrib = np.einsum("pef,pf->pe", blocks, X[col_idx])
    y = np.zeros((m, 12))
    np.add.at(y, rows, contrib)
    return (y + lam * X).reshape(-1)


def pcg(row_ptr, col_idx, blocks, g, lam, iters, Minv=None):
    """Returns (dx, info) with info = {resid: [|r_0|, ..., |r_P|], breakdown, iters}."""
    m = len(row_ptr) - 1
    if Minv is None:
        Minv, _ = block_jacobi(row_ptr, col_idx, blocks, lam)
    apply_M = lambda v: np.einsum("mef,mf->me", Minv, v.reshape(m, 12)).reshape(-1)  # noqa: E731
    A = lambda v: bsr_matvec(row_ptr, col_idx, blocks, v, lam)  # noqa: E731
    x = np.zeros(12 * m)
    r = -np.asarray(g, dtype=np.float64).reshape(-1)
    z = apply_M(r)
    p = z.copy()
    rz = float(r @ z)
    resid = [float(np.linalg.norm(r))]
    breakdown = False
    done = 0
    for _ in range(iters):
        if rz == 0.0:
            break
        q = A(p)
        pq = float(p @ q)
        if not pq > 0.0:
            breakdown = True
            break
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        z = apply_M(r)
        rz_new = float(r @ z)
        resid.append(float(np.linalg.norm(r)))
        done += 1
        beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
    return x, {"resid": resid, "breakdown": breakdown, "iters": done}


def cholesky_solve(H, g, lam):
    """Direct solution of (H + lambda I) dx = -g by dense Cholesky (reference for PCG)."""
    n = H.shape[0]
    c = scipy.linalg.cho_factor(H + lam * np.eye(n))
    return scipy.linalg.cho_solve(c, -np.asarray(g, dtype=np.float64).reshape(-1))
