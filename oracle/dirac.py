"""Fine-grid Wilson-clover operator, FP64 (oracle; test infrastructure only).

The paper fixes the fermion discretisation only by name: N_f = 2
non-perturbatively O(a)-improved Wilson fermions with hopping parameter kappa
and clover coefficient c_sw (tab:ensembles and section "Numerical study").
It works with the Hermitian operator Q = gamma5 D (section "Variance reduction
using deflation").  The readings taken here:

* kappa-normalised operator  M = 2 kappa D
      (M psi)(x) = (1 + A(x)) psi(x)
                   - kappa sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
                                    + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]
  with the clover term  A(x) = i kappa c_sw sum_{mu<nu} sigma_{mu nu} F_{mu nu}(x),
  sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu],
  F_{mu nu} = traceless part of (Q_{mu nu} - Q_{mu nu}^+)/8, Q_{mu nu} the sum of
  the four counter-clockwise plaquette leaves at x;
* chiral Euclidean gamma basis, gamma5 = gamma0 gamma1 gamma2 gamma3 = diag(1,1,-1,-1);
* fermion boundary phases bc[mu] on hops that wrap around the lattice
  (default antiperiodic in time, periodic in space); links are periodic.
"""
from __future__ import annotations

import numpy as np

DEFAULT_BC = (-1.0, 1.0, 1.0, 1.0)


# ---------------------------------------------------------------------------
# Dirac algebra
# ---------------------------------------------------------------------------
def gammas():
    """Return (gamma[0..3], gamma5) as 4x4 complex arrays (chiral basis)."""
    s1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    s2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    s3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
    one = np.eye(2, dtype=np.complex128)
    z = np.zeros((2, 2), dtype=np.complex128)
    g = [np.block([[z, -one], [-one, z]])]
    for s in (s1, s2, s3):
        g.append(np.block([[z, -1j * s], [1j * s, z]]))
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    return g, g5


def sigma(mu, nu):
    g, _ = gammas()
    return 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])


# ---------------------------------------------------------------------------
# Layout helpers (canonical flat arrays <-> lattice-shaped arrays)
# ---------------------------------------------------------------------------
def gauge_to_lattice(U, L):
    """canonical [V][4][3][3] -> [4][L0][L1][L2][L3][3][3]"""
    return np.moveaxis(np.asarray(U).reshape(*L, 4, 3, 3), 4, 0)


def fields_to_lattice(psi, L):
    """canonical [n][V][4][3] -> [n][L0][L1][L2][L3][4][3]"""
    psi = np.asarray(psi)
    return psi.reshape(psi.shape[0], *L, 4, 3)


def fields_to_canonical(psi):
    return psi.reshape(psi.shape[0], -1, 4, 3)


def shift(f, mu, sign, lat0, phase=1.0):
    """g(x) = f(x + sign*mu) with `phase` applied to values that wrapped.

    `lat0` is the axis of f holding x0."""
    ax = lat0 + mu
    g = np.roll(f, -sign, axis=ax)
    if phase != 1.0:
        L = f.shape[ax]
        idx = [slice(None)] * f.ndim
        idx[ax] = L - 1 if sign > 0 else 0
        g[tuple(idx)] *= phase
    return g


def spin_mul(G, psi):
    """Apply a 4x4 spin matrix to psi[..., spin, colour]."""
    return np.einsum("st,...tc->...sc", G, psi)


def colour_mul(U, psi):
    """(U psi)[..., s, a] = sum_b U[..., a, b] psi[..., s, b]"""
    return np.einsum("...ab,...sb->...sa", U, psi)


def colour_mul_dag(U, psi):
    """(U^+ psi)[..., s, a] = sum_b conj(U[..., b, a]) psi[..., s, b]"""
    return np.einsum("...ba,...sb->...sa", U.conj(), psi)


# ---------------------------------------------------------------------------
# Clover term
# ---------------------------------------------------------------------------
def _dag(A):
    return np.swapaxes(A, -1, -2).conj()


def clover_leaves(Ul, mu, nu):
    """Sum of the four counter-clockwise plaquette leaves Q_{mu nu}(x).

    Ul: [4][L0..L3][3][3]."""
    def sh(A, d, s):
        return shift(A, d, s, 0)
    Um, Un = Ul[mu], Ul[nu]
    # x -> x+mu -> x+mu+nu -> x+nu -> x
    q = Um @ sh(Un, mu, +1) @ _dag(sh(Um, nu, +1)) @ _dag(Un)
    # x -> x+nu -> x+nu-mu -> x-mu -> x
    q = q + Un @ _dag(sh(sh(Um, nu, +1), mu, -1)) @ _dag(sh(Un, mu, -1)) @ sh(Um, mu, -1)
    # x -> x-mu -> x-mu-nu -> x-nu -> x
    q = q + (_dag(sh(Um, mu, -1)) @ _dag(sh(sh(Un, mu, -1), nu, -1))
             @ sh(sh(Um, mu, -1), nu, -1) @ sh(Un, nu, -1))
    # x -> x-nu -> x-nu+mu -> x+mu -> x
    q = q + _dag(sh(Un, nu, -1)) @ sh(Um, nu, -1) @ sh(sh(Un, nu, -1), mu, +1) @ _dag(Um)
    return q


def field_strength(Ul, mu, nu):
    """F_{mu nu}(x): traceless part of (Q_{mu nu} - Q_{mu nu}^+)/8 (anti-Hermitian)."""
    q = clover_leaves(Ul, mu, nu)
    F = (q - _dag(q)) / 8.0
    tr = np.trace(F, axis1=-2, axis2=-1) / 3.0
    return F - tr[..., None, None] * np.eye(3)


def clover(U, L, kappa, csw):
    """1 + A(x) as a 12x12 matrix per site (index 3*spin + colour).

    Returns [L0][L1][L2][L3][12][12]."""
    Ul = gauge_to_lattice(U, L)
    A = np.zeros((*L, 12, 12), dtype=np.complex128)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            F = field_strength(Ul, mu, nu)
            A += np.einsum("st,...ab->...satb", sigma(mu, nu), F).reshape(*L, 12, 12)
    A *= 1j * kappa * csw
    A += np.eye(12)
    return A


# ---------------------------------------------------------------------------
# Operator application
# ---------------------------------------------------------------------------
class WilsonClover:
    """M and Q = gamma5 M on one gauge field (kappa-normalised)."""

    def __init__(self, U, L, kappa, csw, bc=DEFAULT_BC):
        self.L = tuple(int(l) for l in L)
        self.kappa = float(kappa)
        self.csw = float(csw)
        self.bc = tuple(float(b) for b in bc)
        self.Ul = gauge_to_lattice(U, self.L)
        self.Cl = clover(U, self.L, kappa, csw)
        g, g5 = gammas()
        self.g, self.g5 = g, g5
        one = np.eye(4)
        self.pm = [one - g[mu] for mu in range(4)]  # forward projector (1 - gamma_mu)
        self.pp = [one + g[mu] for mu in range(4)]  # backward projector (1 + gamma_mu)
        # U_mu(x - mu), needed by the backward hop
        self.Ub = [shift(self.Ul[mu], mu, -1, 0) for mu in range(4)]

    @property
    def V(self):
        return int(np.prod(self.L))

    def hop(self, psi, mu, sign):
        """One directional hop term (without the -kappa), psi: [n][L..][4][3].

        sign=+1: (1 - gamma_mu) U_mu(x) psi(x+mu)
        sign=-1: (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu)
        """
        ps = shift(psi, mu, sign, 1, self.bc[mu])
        if sign > 0:
            return spin_mul(self.pm[mu], colour_mul(self.Ul[mu], ps))
        return spin_mul(self.pp[mu], colour_mul_dag(self.Ub[mu], ps))

    def clover_apply(self, psi):
        n = psi.shape[0]
        v = psi.reshape(n, *self.L, 12)
        return np.einsum("...ij,n...j->n...i", self.Cl, v).reshape(psi.shape)

    def M(self, psi):
        out = self.clover_apply(psi)
        for mu in range(4):
            out -= self.kappa * (self.hop(psi, mu, +1) + self.hop(psi, mu, -1))
        return out

    def Q(self, psi):
        return spin_mul(self.g5, self.M(psi))

    # canonical-layout conveniences --------------------------------------
    def M_canon(self, psi):
        return fields_to_canonical(self.M(fields_to_lattice(psi, self.L)))

    def dense(self):
        """Dense 12V x 12V matrix of M (small lattices only)."""
        n = 12 * self.V
        out = np.empty((n, n), dtype=np.complex128)
        chunk = 384
        for j0 in range(0, n, chunk):
            j1 = min(n, j0 + chunk)
            e = np.zeros((j1 - j0, n), dtype=np.complex128)
            e[np.arange(j1 - j0), np.arange(j0, j1)] = 1.0
            out[:, j0:j1] = self.M_canon(e.reshape(j1 - j0, self.V, 4, 3)).reshape(j1 - j0, n).T
        return out


def gamma5_field(psi):
    _, g5 = gammas()
    return spin_mul(g5, psi)


def low_modes(D, nev):
    """The nev eigenpairs of Q = gamma5 M with the smallest |lambda| (sec.
    "Low-mode averaging for the current correlator": the low modes are
    eigenvectors of the Hermitian operator with the smallest-magnitude
    eigenvalues).  Dense Q = gamma5 M (the dense M above, gamma5 acting on
    the spin index), numpy's Hermitian eigensolver, ordered by |lambda|.
    Returns (lam[nev], vecs[nev][V][4][3] canonical).  Tiny lattices only."""
    n = 12 * D.V
    Mdense = D.dense()
    g5 = np.tile(np.repeat(np.array([1.0, 1.0, -1.0, -1.0]), 3), D.V)
    Q = g5[:, None] * Mdense
    Q = 0.5 * (Q + Q.conj().T)
    w, v = np.linalg.eigh(Q)
    idx = np.argsort(np.abs(w), kind="stable")[:nev]
    return w[idx], v[:, idx].T.reshape(nev, D.V, 4, 3)
