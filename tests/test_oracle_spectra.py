"""Pins of the oracle's coarse operator without chiral split (appendix on the
spectra of coarse and fine operators): Hermiticity, the low-mode-averaging
limit (one block, exact eigenvectors as test vectors: the coarse operator
is the diagonal of their eigenvalues), and containment of the non-chiral
block basis in the span of the chirally split one."""
import numpy as np

from oracle import dirac, subspace, coarse
from paper_2412_06347_amd import synth


def _Q(D, L):
    V = int(np.prod(L))
    g5 = np.kron(np.eye(V), np.kron(np.diag([1, 1, -1, -1]), np.eye(3)))
    return g5 @ D.dense()


def test_nonchiral_hermitian_and_contained():
    L, b, Nv = (4, 2, 2, 4), (2, 2, 2, 2), 5
    U = synth.gauge_field(L, 0.3, 41)
    D = dirac.WilsonClover(U, L, 0.124, 1.0)
    bl = subspace.Blocking(L, b)
    tv = dirac.fields_to_lattice(synth.gaussian_fields(Nv, L, 42), L)
    Q = _Q(D, L)
    A = coarse.nonchiral_dense(Q, bl, tv)
    assert A.shape == (bl.V1 * Nv, bl.V1 * Nv)
    assert np.abs(A - A.conj().T).max() < 1e-13 * np.abs(A).max()
    # every non-chiral basis field lies in the chiral block basis' span, and
    # they are orthonormal per block
    phi = coarse.nonchiral_basis(bl, tv)
    B = subspace.BlockBasis(bl, tv)
    Tc = B.basis_canonical().reshape(bl.V1 * B.nc, -1).T
    P = Tc @ Tc.conj().T
    cols = np.zeros((bl.V1 * Nv, bl.V1, *b, 4, 3), dtype=complex)
    for y in range(bl.V1):
        for c in range(Nv):
            cols[y * Nv + c, y] = phi[y, c]
    Tn = bl.from_blocks(cols).reshape(bl.V1 * Nv, -1).T
    assert np.abs(P @ Tn - Tn).max() < 1e-12
    assert np.abs(Tn.conj().T @ Tn - np.eye(bl.V1 * Nv)).max() < 1e-12


def test_nonchiral_lma_limit_is_diagonal():
    """One block (the whole lattice) and the Nv lowest exact eigenvectors of Q
    as test vectors: Q_nc = diag(lambda_c)."""
    L, Nv = (4, 2, 2, 2), 6
    U = synth.gauge_field(L, 0.3, 43)
    D = dirac.WilsonClover(U, L, 0.124, 1.0)
    Q = _Q(D, L)
    lam, vec = np.linalg.eigh(0.5 * (Q + Q.conj().T))
    order = np.argsort(np.abs(lam))[:Nv]
    tv = dirac.fields_to_lattice(vec[:, order].T.reshape(Nv, -1, 4, 3), L)
    bl = subspace.Blocking(L, L)
    A = coarse.nonchiral_dense(Q, bl, tv)
    # Gram-Schmidt of orthonormal vectors keeps them up to a phase: diag(lambda)
    assert np.abs(A - np.diag(lam[order])).max() < 1e-12
