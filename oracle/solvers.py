"""Linear solves on the fine and coarse level (oracle; test infrastructure only).

The paper solves with GCR-type Krylov methods (section "Comparison of the
cost": SAP-preconditioned GCR on the fine grid, GCR on the coarse grid) and
does not state a tolerance.  Solutions are unique, so the oracle uses plain
restarted GCR (or a dense LU solve on small systems); only the solution is
compared, never iteration counts.
"""
from __future__ import annotations

import numpy as np


def gcr(apply, b, tol=1e-12, m=16, max_iter=20000):
    """Restarted GCR(m) for A x = b, batched over the leading axis of b.

    `apply` maps an array shaped like b to A times it.  Returns (x, iters,
    relative residuals)."""
    b = np.asarray(b)
    n = b.shape[0]
    flat = lambda a: a.reshape(n, -1)
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.linalg.norm(flat(b), axis=1)
    bn[bn == 0] = 1.0
    it = 0
    while it < max_iter:
        P, AP = [], []
        for _ in range(m):
            res = np.linalg.norm(flat(r), axis=1) / bn
            if np.all(res <= tol) or it >= max_iter:
                return x, it, res
            p = r.copy()
            ap = apply(p)
            for q, aq in zip(P, AP):
                beta = np.einsum("nk,nk->n", flat(aq).conj(), flat(ap))
                ap = ap - beta.reshape((n,) + (1,) * (b.ndim - 1)) * aq
                p = p - beta.reshape((n,) + (1,) * (b.ndim - 1)) * q
            nrm = np.linalg.norm(flat(ap), axis=1)
            ap = ap / nrm.reshape((n,) + (1,) * (b.ndim - 1))
            p = p / nrm.reshape((n,) + (1,) * (b.ndim - 1))
            alpha = np.einsum("nk,nk->n", flat(ap).conj(), flat(r))
            sh = (n,) + (1,) * (b.ndim - 1)
            x = x + alpha.reshape(sh) * p
            r = r - alpha.reshape(sh) * ap
            P.append(p)
            AP.append(ap)
            it += 1
        # restart with the true residual
        r = b - apply(x)
    res = np.linalg.norm(flat(r), axis=1) / bn
    return x, it, res


def dense_solve(A, b):
    """x = A^{-1} b for b[n][dim] via LU."""
    return np.linalg.solve(A, np.asarray(b).T).T
