"""Galerkin coarse operator and coarse-level objects (oracle; test
infrastructure only).

* D_1 = R M T, Q_1 = R Q T = (gamma5)_1 D_1 (section "Variance reduction using
  deflation"; appendix "Chirality on the coarse subspaces" shows the two agree
  when the basis preserves chirality).
* Nearest-neighbour stencil structure of the coarse operator (fig:A): per
  coarse site one self block and one block for each of the 2d = 8 neighbours,
  each (2 Nv) x (2 Nv).
* Coarse gamma matrices (gamma5 gamma_k)_1 with an open time index
  (eq:coarse:gamma, used with an unsummed x0 in eq:G_LL:exact).
* Top level from coarse modes W (a non-recursive level, allowed by the remark
  after eq:mglma:decomp): W = chirally split, orthonormalised coarse vectors,
  D_2 = W^+ D_1 W, Q_2 = W^+ Q_1 W = (gamma5)_2 D_2.

Stencil reading: entry D1[y][dir] collects the fine hops leaving block y
through its +mu (dir = 1+2mu) or -mu (dir = 2+2mu) face; dir = 0 collects the
clover/diagonal term and the hops that stay inside the block.  The apply sums
all nine entries, so lattices with a coarse extent of 1 or 2 (where neighbours
coincide) need no special case.
"""
from __future__ import annotations

import numpy as np

from .dirac import WilsonClover, gammas, spin_mul
from .subspace import BlockBasis, gram_schmidt, coarse_gamma5


def _face_mask(bl, mu, which):
    """Lattice mask of sites whose local block coordinate along mu is
    b_mu - 1 (which='hi') or 0 (which='lo')."""
    L = bl.L
    x = np.arange(L[mu]) % bl.b[mu]
    m1 = (x == (bl.b[mu] - 1)) if which == "hi" else (x == 0)
    shape = [1, 1, 1, 1]
    shape[mu] = L[mu]
    return m1.reshape(shape)


def galerkin(D: WilsonClover, B: BlockBasis, chunk=8):
    """D1[V1][9][nc][nc] with D1 = R M T entry by entry (stencil form)."""
    bl = B.bl
    nc, V1 = B.nc, bl.V1
    D1 = np.zeros((V1, 9, nc, nc), dtype=np.complex128)
    kappa = D.kappa
    for j0 in range(0, nc, chunk):
        j1 = min(nc, j0 + chunk)
        e = np.zeros((j1 - j0, V1, nc), dtype=np.complex128)
        for j in range(j0, j1):
            e[j - j0, :, j] = 1.0
        Phi = B.prolong(e)                          # Phi_j = sum_y phi_{y,j}
        self_part = D.clover_apply(Phi)
        for mu in range(4):
            hi = _face_mask(bl, mu, "hi")[None, ..., None, None]
            lo = _face_mask(bl, mu, "lo")[None, ..., None, None]
            fw = -kappa * D.hop(Phi, mu, +1)
            bw = -kappa * D.hop(Phi, mu, -1)
            self_part = self_part + np.where(hi, 0, fw) + np.where(lo, 0, bw)
            D1[:, 1 + 2 * mu, :, j0:j1] = np.moveaxis(B.restrict(np.where(hi, fw, 0)), 0, -1)
            D1[:, 2 + 2 * mu, :, j0:j1] = np.moveaxis(B.restrict(np.where(lo, bw, 0)), 0, -1)
        D1[:, 0, :, j0:j1] = np.moveaxis(B.restrict(self_part), 0, -1)
    return D1


def coarse_apply(D1, nbr, v):
    """out[n][y] = sum_dir D1[y][dir] v[n][nbr[y][dir]]  (fig:A stencil)."""
    out = np.zeros_like(v)
    for d in range(9):
        out += np.einsum("yij,nyj->nyi", D1[:, d], v[:, nbr[:, d]])
    return out


def coarse_dense(D1, nbr):
    """Dense (V1*nc) x (V1*nc) matrix of the coarse stencil."""
    V1, _, nc, _ = D1.shape
    A = np.zeros((V1 * nc, V1 * nc), dtype=np.complex128)
    for y in range(V1):
        for d in range(9):
            z = nbr[y, d]
            A[y * nc:(y + 1) * nc, z * nc:(z + 1) * nc] += D1[y, d]
    return A


def coarse_gammas(B: BlockBasis):
    """Gamma1[V1][b0][3][nc][nc]: (gamma5 gamma_k)_1 restricted to the fine time
    slice y0*b0 + t of block y (eq:coarse:gamma with an open time index)."""
    bl = B.bl
    g, g5 = gammas()
    Nv, nc = B.Nv, B.nc
    # full 4-spin form of every basis vector on its block
    full = np.zeros((bl.V1, nc, *bl.b, 4, 3), dtype=np.complex128)
    for a in range(2):
        full[:, a * Nv:(a + 1) * Nv, ..., 2 * a:2 * a + 2, :] = B.phi[:, a]
    out = np.zeros((bl.V1, bl.b[0], 3, nc, nc), dtype=np.complex128)
    for k in range(1, 4):
        G = g5 @ g[k]
        gf = spin_mul(G, full)
        # sum over the spatial block sites, spin and colour, time kept open
        out[:, :, k - 1] = np.einsum("yitxzwsc,yjtxzwsc->ytij", full.conj(), gf)
    return out


class TopLevel:
    """Exact top level spanned by chirally split coarse modes."""

    def __init__(self, modes, D1, nbr, Nv):
        """modes: [Nlm][V1][nc] coarse vectors (any full-rank set)."""
        Nlm, V1, nc = modes.shape
        self.Nlm, self.r = Nlm, 2 * Nlm
        g5c = coarse_gamma5(Nv)
        cols = []
        for a in range(2):
            keep = (g5c > 0) if a == 0 else (g5c < 0)
            part = modes * keep[None, None, :]
            q = gram_schmidt(part.reshape(Nlm, -1))
            cols.append(q)
        # W[V1*nc][r], column index alpha*Nlm + m
        self.W = np.concatenate(cols, axis=0).T.copy()
        AW = coarse_apply(D1, nbr, self.W.T.reshape(self.r, V1, nc)).reshape(self.r, -1).T
        self.D2 = self.W.conj().T @ AW
        self.g5 = np.concatenate([np.ones(Nlm), -np.ones(Nlm)])
        self.Q2 = self.g5[:, None] * self.D2

    def gammas(self, Gamma1, bl):
        """Gamma2[L0][3][r][r] = W^+ (gamma5 gamma_k)_1(x0) W."""
        V1, b0, _, nc, _ = Gamma1.shape
        Wy = self.W.reshape(V1, nc, self.r)
        out = np.zeros((bl.L[0], 3, self.r, self.r), dtype=np.complex128)
        y0 = np.unravel_index(np.arange(V1), bl.L1)[0]
        for t in range(b0):
            m = np.einsum("yia,ykij,yjb->ykab", Wy.conj(), Gamma1[:, t], Wy)
            for y in range(V1):
                out[y0[y] * b0 + t] += m[y]
        return out


def low_modes(D1, nbr, Nv, nev):
    """The nev eigenpairs of Q_1 = (gamma5)_1 D_1 with the smallest |lambda|
    (sec. "Low-mode averaging for the current correlator": the low modes are
    eigenvectors of the Hermitian operator with the smallest-magnitude
    eigenvalues).  Dense: Q_1 assembled column by column, numpy's Hermitian
    eigensolver, eigenvalues ordered by |lambda| (ties keep numpy's order).
    Returns (lam[nev], vecs[nev][V1][nc]).  For small coarse lattices."""
    V1, nc = D1.shape[0], D1.shape[2]
    A = coarse_dense(D1, nbr)
    g5c = np.tile(coarse_gamma5(Nv), V1)
    Q = g5c[:, None] * A
    Q = 0.5 * (Q + Q.conj().T)
    w, v = np.linalg.eigh(Q)
    idx = np.argsort(np.abs(w), kind="stable")[:nev]
    return w[idx], v[:, idx].T.reshape(nev, V1, nc)


def parity_sites(L1):
    """Even and odd coarse sites, each in increasing order of the block index
    y (C order over L1, last direction fastest); parity = sum of the block
    coordinates mod 2.  Returns (even, odd) index arrays."""
    y = np.arange(int(np.prod(L1)))
    par = np.sum(np.stack(np.unravel_index(y, tuple(L1))), axis=0) % 2
    return y[par == 0], y[par == 1]


def _site_rows(sites, nc):
    return (sites[:, None] * nc + np.arange(nc)[None, :]).reshape(-1)


def eo_split(D1, nbr, L1):
    """The four parity blocks (A_ee, A_eo, A_oe, A_oo) of the dense coarse
    operator, rows and columns in the order of parity_sites (even-odd
    preconditioning of the coarse operator, sec. "Comparison of the cost")."""
    nc = D1.shape[2]
    A = coarse_dense(D1, nbr)
    e, o = parity_sites(L1)
    re, ro = _site_rows(e, nc), _site_rows(o, nc)
    return A[np.ix_(re, re)], A[np.ix_(re, ro)], A[np.ix_(ro, re)], A[np.ix_(ro, ro)]


def schur_even(D1, nbr, L1):
    """S = 1 - A_ee^{-1} A_eo A_oo^{-1} A_oe on the even sites (dense; the
    Schur complement of A_oo, multiplied from the left by A_ee^{-1})."""
    Aee, Aeo, Aoe, Aoo = eo_split(D1, nbr, L1)
    return np.eye(Aee.shape[0]) - np.linalg.solve(Aee, Aeo @ np.linalg.solve(Aoo, Aoe))


def solve_eo(D1, nbr, L1, b):
    """x = D_1^{-1} b through the reduced system: S x_e = A_ee^{-1} (b_e -
    A_eo A_oo^{-1} b_o), then x_o = A_oo^{-1} (b_o - A_oe x_e).
    b: [V1][nc]; returns [V1][nc]."""
    V1, nc = b.shape
    Aee, Aeo, Aoe, Aoo = eo_split(D1, nbr, L1)
    e, o = parity_sites(L1)
    be, bo = b[e].reshape(-1), b[o].reshape(-1)
    S = schur_even(D1, nbr, L1)
    rhs = np.linalg.solve(Aee, be - Aeo @ np.linalg.solve(Aoo, bo))
    xe = np.linalg.solve(S, rhs)
    xo = np.linalg.solve(Aoo, bo - Aoe @ xe)
    x = np.zeros_like(b)
    x[e] = xe.reshape(-1, nc)
    x[o] = xo.reshape(-1, nc)
    return x


# ---- nested hierarchy: inner levels (sec. "Multigrid low-mode averaging") ----

def level2_of(L1, r):
    """For every level-1 site y (C order over L1) the index z of the level-2
    block that contains it (eq:block_nested_decomp: blocks of r_mu level-1
    sites per direction, z in C order over L1 / r)."""
    L2 = tuple(L1[mu] // r[mu] for mu in range(4))
    yc = np.stack(np.unravel_index(np.arange(int(np.prod(L1))), tuple(L1)))
    zc = yc // np.asarray(r)[:, None]
    return np.ravel_multi_index(tuple(zc), L2)


def inner_restrictor(L1, r, nc):
    """Dense R_l (V2 nc x V1 nc) of an inner level: (R psi)_a(z) =
    sqrt(V2/V1) sum_{y in z} psi_a(y), component by component.  The
    prolongator T_l is its (real) transpose."""
    V1 = int(np.prod(L1))
    V2 = V1 // int(np.prod(r))
    z = level2_of(L1, r)
    R = np.zeros((V2 * nc, V1 * nc))
    w = np.sqrt(V2 / V1)
    for y in range(V1):
        for a in range(nc):
            R[z[y] * nc + a, y * nc + a] = w
    return R


def level2_dense(D1, nbr, L1, r):
    """D_2 = R_1 D_1 T_1 (the recursion Q_{l+1} = R_l Q_l T_l; R_1 acts
    component-wise, so it commutes with the coarse gamma5), dense."""
    nc = D1.shape[2]
    R = inner_restrictor(L1, r, nc)
    return R @ coarse_dense(D1, nbr) @ R.T


def eo_constant_vectors(L1, nc):
    """Y: (Vh nc) x nc, column a = component a equal to 1/sqrt(Vh) on every
    even site (the subspace a one-block coarser level spans, restricted to the
    even sites), the deflation subspace of the even-odd coarse GCR."""
    Vh = int(np.prod(L1)) // 2
    Y = np.zeros((Vh * nc, nc))
    for a in range(nc):
        Y[a::nc, a] = 1.0 / np.sqrt(Vh)
    return Y


def solve_eo_deflated(S, Y, bh):
    """S x = bh through the deflated system: x0 = Y E^-1 Y^+ bh (E = Y^+ S Y),
    z from P_L S z = P_L bh (least squares: P_L S is singular on range Y),
    x = x0 + P_R z with P_L = 1 - S Y E^-1 Y^+, P_R = 1 - Y E^-1 Y^+ S."""
    E = Y.conj().T @ S @ Y
    Ei = np.linalg.inv(E)
    PL = np.eye(S.shape[0]) - S @ Y @ Ei @ Y.conj().T
    PR = np.eye(S.shape[0]) - Y @ Ei @ Y.conj().T @ S
    x0 = Y @ (Ei @ (Y.conj().T @ bh))
    z = np.linalg.lstsq(PL @ S, PL @ bh, rcond=None)[0]
    return x0 + PR @ z


# ---------------------------------------------------------------------------
# coarsening without chiral split (appendix on the spectra of coarse and fine
# operators: the coarse spin degree of freedom trivial)
# ---------------------------------------------------------------------------
def nonchiral_basis(bl, testvecs_lat):
    """Per block y the Nv fields theta_{B_y} v_c over all four spins,
    Gram-Schmidt in order c: [V1][Nv][b0..b3][4][3]."""
    Nv = testvecs_lat.shape[0]
    vb = np.moveaxis(bl.to_blocks(testvecs_lat), 0, 1)         # [V1][Nv][b..][4][3]
    q = gram_schmidt(vb.reshape(bl.V1, Nv, -1))
    return q.reshape(bl.V1, Nv, *bl.b, 4, 3)


def nonchiral_dense(Qd, bl, testvecs_lat):
    """Q_nc = T_nc^+ Q T_nc (dense, (V1 Nv) x (V1 Nv)) for the dense Hermitian
    fine operator Qd (canonical order) and the block basis without chiral
    split; coarse index y * Nv + c.  Tiny lattices only."""
    Nv = testvecs_lat.shape[0]
    phi = nonchiral_basis(bl, testvecs_lat)
    cols = np.zeros((bl.V1 * Nv, bl.V1, *bl.b, 4, 3), dtype=np.complex128)
    for y in range(bl.V1):
        for c in range(Nv):
            cols[y * Nv + c, y] = phi[y, c]
    T = bl.from_blocks(cols).reshape(bl.V1 * Nv, -1).T             # [12 V][V1 Nv]
    return T.conj().T @ Qd @ T
