"""Block decomposition, chirally split block basis, restrictor and prolongator
(oracle; test infrastructure only).

Follows the paper's section "Local coherence and block decomposition"
(eq:block_decomp, eq:block_def, eq:block_grid, eq:block_field) and section
"Multigrid decompositions" (eq:mg_basis, eq:res_mg, eq:pro_mg), with the
chirality-preserving extension eq:chirality:B of the appendix "Chirality on the
coarse subspaces".

Readings:
* block B_y = {x : 0 <= x_mu - y_mu b_mu < b_mu} (the lower bound is lost in
  the printed eq:block_def);
* coarse index i = alpha*Nv + c, alpha = 0 (gamma5 = +1, spins 0,1) and
  alpha = 1 (gamma5 = -1, spins 2,3);
* orthonormalisation: classical Gram-Schmidt with one re-orthogonalisation,
  in the order c = 0..Nv-1, positive real diagonal (the QR factor is then
  unique); a vector whose residual norm falls below 1e-10 of its norm raises
  RankError.
"""
from __future__ import annotations

import numpy as np


class RankError(ValueError):
    pass


class Blocking:
    def __init__(self, L, b):
        self.L = tuple(int(x) for x in L)
        self.b = tuple(int(x) for x in b)
        for mu in range(4):
            if self.L[mu] % self.b[mu]:
                raise ValueError("block size must divide the lattice size")
        self.L1 = tuple(self.L[mu] // self.b[mu] for mu in range(4))
        self.V1 = int(np.prod(self.L1))
        self.Vb = int(np.prod(self.b))

    def to_blocks(self, f):
        """[n][L0..L3][...] -> [n][V1][b0][b1][b2][b3][...]"""
        n = f.shape[0]
        rest = f.shape[5:]
        shp = [n]
        for mu in range(4):
            shp += [self.L1[mu], self.b[mu]]
        g = f.reshape(*shp, *rest)
        nr = len(rest)
        perm = [0, 1, 3, 5, 7, 2, 4, 6, 8] + [9 + i for i in range(nr)]
        g = g.transpose(perm)
        return g.reshape(n, self.V1, *self.b, *rest)

    def from_blocks(self, g):
        n = g.shape[0]
        rest = g.shape[6:]
        g = g.reshape(n, *self.L1, *self.b, *rest)
        nr = len(rest)
        perm = [0, 1, 5, 2, 6, 3, 7, 4, 8] + [9 + i for i in range(nr)]
        g = g.transpose(perm)
        return g.reshape(n, *self.L, *rest)

    def block_of(self, x):
        y = [x[mu] // self.b[mu] for mu in range(4)]
        return ((y[0] * self.L1[1] + y[1]) * self.L1[2] + y[2]) * self.L1[3] + y[3]

    def coarse_neighbour(self, y, mu, sign):
        c = np.unravel_index(y, self.L1)
        c = list(int(v) for v in c)
        c[mu] = (c[mu] + sign) % self.L1[mu]
        return int(np.ravel_multi_index(c, self.L1))

    def neighbour_table(self):
        """[V1][9]: direction 0 = self, 1+2mu = +mu, 2+2mu = -mu."""
        t = np.empty((self.V1, 9), dtype=np.int64)
        for y in range(self.V1):
            t[y, 0] = y
            for mu in range(4):
                t[y, 1 + 2 * mu] = self.coarse_neighbour(y, mu, +1)
                t[y, 2 + 2 * mu] = self.coarse_neighbour(y, mu, -1)
        return t


def gram_schmidt(W, tol=1e-10):
    """Orthonormalise W[..., c, k] over c (classical GS, twice), batched.

    Returns Q with Q[..., c, :] orthonormal and
    span(Q[..., :c+1, :]) = span(W[..., :c+1, :])."""
    W = np.array(W, dtype=np.complex128, copy=True)
    Q = np.zeros_like(W)
    nv = W.shape[-2]
    for c in range(nv):
        w = W[..., c, :]
        n0 = np.linalg.norm(w, axis=-1)
        for _ in range(2):
            if c:
                coef = np.einsum("...dk,...k->...d", Q[..., :c, :].conj(), w)
                w = w - np.einsum("...d,...dk->...k", coef, Q[..., :c, :])
        nrm = np.linalg.norm(w, axis=-1)
        if np.any(nrm <= tol * n0) or np.any(n0 == 0):
            raise RankError("block basis is rank deficient at vector %d" % c)
        Q[..., c, :] = w / nrm[..., None]
    return Q


class BlockBasis:
    """phi^{B_y}_{alpha c}: Nv vectors per block and chirality (eq:mg_basis)."""

    def __init__(self, blocking: Blocking, testvecs_lat):
        """testvecs_lat: [Nv][L0..L3][4][3] (the global fields phi_c)."""
        self.bl = blocking
        self.Nv = testvecs_lat.shape[0]
        self.nc = 2 * self.Nv
        vb = blocking.to_blocks(testvecs_lat)          # [Nv][V1][b..][4][3]
        vb = np.moveaxis(vb, 0, 1)                       # [V1][Nv][b..][4][3]
        phi = np.empty((blocking.V1, 2, self.Nv, *blocking.b, 2, 3), dtype=np.complex128)
        for a in range(2):
            # P_alpha theta_{B_y} phi_c: keep the two spins of chirality alpha
            w = vb[..., 2 * a:2 * a + 2, :]
            wf = w.reshape(blocking.V1, self.Nv, -1)
            q = gram_schmidt(wf)
            phi[:, a] = q.reshape(blocking.V1, self.Nv, *blocking.b, 2, 3)
        self.phi = phi

    def restrict(self, psi_lat):
        """eq:res_mg: [n][L..][4][3] -> [n][V1][2*Nv]"""
        pb = self.bl.to_blocks(psi_lat)                  # [n][V1][b..][4][3]
        n = pb.shape[0]
        out = np.empty((n, self.bl.V1, 2, self.Nv), dtype=np.complex128)
        for a in range(2):
            part = pb[..., 2 * a:2 * a + 2, :].reshape(n, self.bl.V1, -1)
            ph = self.phi[:, a].reshape(self.bl.V1, self.Nv, -1)
            out[:, :, a, :] = np.einsum("yck,nyk->nyc", ph.conj(), part)
        return out.reshape(n, self.bl.V1, self.nc)

    def prolong(self, coarse):
        """eq:pro_mg: [n][V1][2*Nv] -> [n][L..][4][3]"""
        n = coarse.shape[0]
        c = coarse.reshape(n, self.bl.V1, 2, self.Nv)
        pb = np.zeros((n, self.bl.V1, *self.bl.b, 4, 3), dtype=np.complex128)
        for a in range(2):
            ph = self.phi[:, a].reshape(self.bl.V1, self.Nv, -1)
            v = np.einsum("nyc,yck->nyk", c[:, :, a, :], ph)
            pb[..., 2 * a:2 * a + 2, :] = v.reshape(n, self.bl.V1, *self.bl.b, 2, 3)
        return self.bl.from_blocks(pb)

    def deficit(self, psi_lat):
        """eq:cdeficit: |(1 - P) psi| / |psi| per field, P = T R the projector on
        the block subspace ([n][L..][4][3] -> [n])."""
        d = psi_lat - self.prolong(self.restrict(psi_lat))
        n = psi_lat.shape[0]
        num = np.linalg.norm(d.reshape(n, -1), axis=1)
        den = np.linalg.norm(psi_lat.reshape(n, -1), axis=1)
        return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)

    def basis_canonical(self):
        """The basis as canonical fine fields, [V1][2*Nv][V][4][3] (tiny lattices)."""
        V1, nc = self.bl.V1, self.nc
        eye = np.zeros((V1 * nc, V1, nc), dtype=np.complex128)
        eye.reshape(V1 * nc, V1 * nc)[np.arange(V1 * nc), np.arange(V1 * nc)] = 1
        f = self.prolong(eye)
        return f.reshape(V1, nc, -1, 4, 3)


def coarse_gamma5(Nv):
    """(gamma5)_1 = diag(1_{Nv}, -1_{Nv}) per coarse site (appendix on chirality)."""
    return np.concatenate([np.ones(Nv), -np.ones(Nv)])
