"""Pins of the oracle's block basis, restrictor/prolongator, Galerkin coarse
operator and top level: partition of the lattice, QR uniqueness against
numpy's Householder QR, RT = 1, the chirality relations of the appendix,
the Galerkin identity against a dense R M T, (gamma5)_1 D_1 Hermitian,
exact eigenvalue reproduction and gauge invariance of D_1, and the low modes
of Q_1 against the singular values of D_1."""
import numpy as np
import pytest

from oracle import dirac, subspace, coarse
from paper_2412_06347_amd import synth


def _setup(L, b, Nv, seed=1, kappa=0.124, csw=1.0):
    U = synth.gauge_field(L, 0.3, seed)
    D = dirac.WilsonClover(U, L, kappa, csw)
    bl = subspace.Blocking(L, b)
    tv = dirac.fields_to_lattice(synth.gaussian_fields(Nv, L, seed + 100), L)
    B = subspace.BlockBasis(bl, tv)
    return U, D, bl, tv, B


def test_block_partition():
    L, b = (4, 6, 2, 4), (2, 3, 2, 1)
    bl = subspace.Blocking(L, b)
    assert bl.V1 == 2 * 2 * 1 * 4
    f = np.arange(np.prod(L)).reshape(1, *L).astype(float)
    blocks = bl.to_blocks(f[..., None])[..., 0]
    assert sorted(blocks.ravel()) == list(range(np.prod(L)))    # each site once
    assert np.array_equal(bl.from_blocks(blocks[..., None])[..., 0], f)
    for y in range(bl.V1):
        for s in blocks[0, y].ravel():
            x = np.unravel_index(int(s), L)
            assert bl.block_of(x) == y


def test_gram_schmidt_matches_qr():
    rng = np.random.default_rng(1)
    W = rng.standard_normal((5, 7, 40)) + 1j * rng.standard_normal((5, 7, 40))
    Q = subspace.gram_schmidt(W)
    for i in range(5):
        q, r = np.linalg.qr(W[i].T)
        ph = np.diag(r) / np.abs(np.diag(r))
        q = q * ph[None, :]           # positive real diagonal of R
        assert np.abs(Q[i].T - q).max() < 1e-12
    with pytest.raises(subspace.RankError):
        W2 = W.copy()
        W2[:, 3] = W2[:, 1] * (2 - 1j)
        subspace.gram_schmidt(W2)


def test_restrict_prolong_identities():
    L, b, Nv = (4, 4, 2, 2), (2, 2, 2, 2), 3
    U, D, bl, tv, B = _setup(L, b, Nv)
    T = B.basis_canonical().reshape(bl.V1 * B.nc, -1).T          # 12V x (V1 nc)
    assert np.abs(T.conj().T @ T - np.eye(T.shape[1])).max() < 1e-13   # RT = 1
    P = T @ T.conj().T
    assert np.abs(P @ P - P).max() < 1e-13
    G5 = np.kron(np.eye(bl.L[0] * bl.L[1] * bl.L[2] * bl.L[3]), np.kron(np.diag([1, 1, -1, -1]), np.eye(3)))
    assert np.abs(P @ G5 - G5 @ P).max() < 1e-13                 # [P, gamma5] = 0
    g5c = np.tile(subspace.coarse_gamma5(Nv), bl.V1)
    R = T.conj().T
    assert np.abs(R @ G5 - g5c[:, None] * R).max() < 1e-13       # R gamma5 = (gamma5)_1 R
    # restrict/prolong of the class agree with the dense matrices
    psi = dirac.fields_to_lattice(synth.gaussian_fields(2, L, 7), L)
    rc = B.restrict(psi).reshape(2, -1)
    assert np.abs(rc - (R @ psi.reshape(2, -1).T).T).max() < 1e-12
    c = synth.gaussian_coarse(2, bl.V1, B.nc, 8)
    assert np.abs(B.prolong(c).reshape(2, -1) - (T @ c.reshape(2, -1).T).T).max() < 1e-12


@pytest.mark.parametrize("L,b", [((4, 4, 6, 2), (2, 2, 2, 2)),    # coarse extents 2,2,3,1
                                 ((6, 2, 2, 4), (2, 1, 2, 4)),     # b=1 and b=L directions
                                 ((6, 6, 3, 3), (2, 2, 1, 1))])    # coarse extents 3
def test_galerkin_identity(L, b):
    Nv = 2
    U, D, bl, tv, B = _setup(L, b, Nv)
    D1 = coarse.galerkin(D, B)
    nbr = bl.neighbour_table()
    A = coarse.coarse_dense(D1, nbr)
    T = B.basis_canonical().reshape(bl.V1 * B.nc, -1).T
    brute = T.conj().T @ D.dense() @ T
    assert np.abs(A - brute).max() < 1e-13 * np.abs(brute).max()
    g5c = np.tile(subspace.coarse_gamma5(Nv), bl.V1)
    Q1 = g5c[:, None] * A
    assert np.abs(Q1 - Q1.conj().T).max() < 1e-13
    # coarse apply == R M T psi
    c = synth.gaussian_coarse(2, bl.V1, B.nc, 3)
    lhs = coarse.coarse_apply(D1, nbr, c).reshape(2, -1)
    rhs = B.restrict(D.M(B.prolong(c))).reshape(2, -1)
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()


def test_exact_eigenvalue_reproduction():
    """Test vectors = exact eigenvectors of Q => Q_1 has exactly those eigenvalues
    (appendix on the spectra of coarse and fine operators)."""
    L, b, Nv = (4, 2, 2, 4), (2, 2, 2, 2), 4
    U = synth.gauge_field(L, 0.3, 5)
    D = dirac.WilsonClover(U, L, 0.124, 1.0)
    G5 = np.kron(np.eye(int(np.prod(L))), np.kron(np.diag([1, 1, -1, -1]), np.eye(3)))
    Q = G5 @ D.dense()
    w, v = np.linalg.eigh(Q)
    idx = np.argsort(np.abs(w))[:Nv]
    tv = v[:, idx].T.reshape(Nv, *L, 4, 3)
    bl = subspace.Blocking(L, b)
    B = subspace.BlockBasis(bl, tv)
    D1 = coarse.galerkin(D, B)
    A = coarse.coarse_dense(D1, bl.neighbour_table())
    g5c = np.tile(subspace.coarse_gamma5(Nv), bl.V1)
    w1 = np.linalg.eigvalsh(g5c[:, None] * A)
    for lam in w[idx]:
        assert np.min(np.abs(w1 - lam)) < 1e-12


def test_galerkin_gauge_invariant():
    L, b, Nv = (4, 2, 4, 2), (2, 2, 2, 2), 2
    U, D, bl, tv, B = _setup(L, b, Nv, seed=4)
    D1 = coarse.galerkin(D, B)
    Om = synth.gauge_transform(L, seed=2).reshape(*L, 3, 3)
    Ul = dirac.gauge_to_lattice(U, L)
    Ut = np.stack([Om @ Ul[mu] @ np.swapaxes(dirac.shift(Om, mu, +1, 0), -1, -2).conj()
                   for mu in range(4)])
    Dt = dirac.WilsonClover(np.moveaxis(Ut, 0, 4).reshape(-1, 4, 3, 3), L, D.kappa, D.csw)
    Bt = subspace.BlockBasis(bl, dirac.colour_mul(Om, tv))
    D1t = coarse.galerkin(Dt, Bt)
    assert np.abs(D1t - D1).max() < 1e-12


def test_top_level():
    L, b, Nv, Nlm = (4, 2, 4, 2), (2, 2, 2, 2), 3, 2
    U, D, bl, tv, B = _setup(L, b, Nv)
    D1 = coarse.galerkin(D, B)
    nbr = bl.neighbour_table()
    modes = synth.gaussian_coarse(Nlm, bl.V1, B.nc, 5)
    top = coarse.TopLevel(modes, D1, nbr, Nv)
    W = top.W
    assert np.abs(W.conj().T @ W - np.eye(2 * Nlm)).max() < 1e-13
    g5c = np.tile(subspace.coarse_gamma5(Nv), bl.V1)
    assert np.abs(g5c[:, None] * W - W * top.g5[None, :]).max() < 1e-14   # definite chirality
    A = coarse.coarse_dense(D1, nbr)
    assert np.abs(top.D2 - W.conj().T @ A @ W).max() < 1e-12
    assert np.abs(top.Q2 - top.Q2.conj().T).max() < 1e-12


def test_low_modes():
    """The oracle's low modes of Q_1 = (gamma5)_1 D_1: since (gamma5)_1 is a
    unitary diagonal sign matrix, |lambda| of Q_1 are the singular values of
    D_1 (an independent factorisation that never uses gamma5); the pairs come
    ordered by |lambda|, orthonormal, and satisfy Q_1 v = lambda v with the
    stencil apply (not the dense matrix the eigensolver saw)."""
    L, b, Nv = (4, 2, 4, 2), (2, 2, 2, 2), 3
    U, D, bl, tv, B = _setup(L, b, Nv, seed=6)
    D1 = coarse.galerkin(D, B)
    nbr = bl.neighbour_table()
    nev = 7
    lam, vec = coarse.low_modes(D1, nbr, Nv, nev)
    sv = np.sort(np.linalg.svd(coarse.coarse_dense(D1, nbr), compute_uv=False))
    assert np.abs(np.sort(np.abs(lam)) - sv[:nev]).max() < 1e-12
    assert np.all(np.diff(np.abs(lam)) >= -1e-14)
    V = vec.reshape(nev, -1)
    assert np.abs(V.conj() @ V.T - np.eye(nev)).max() < 1e-12
    g5 = subspace.coarse_gamma5(Nv)[None, None, :]
    Qv = g5 * coarse.coarse_apply(D1, nbr, vec)
    assert np.abs(Qv - lam[:, None, None] * vec).max() < 1e-12


def test_fine_low_modes():
    """The oracle's low modes of Q = gamma5 M: |lambda| equal the singular
    values of M (gamma5 unitary), ordered, orthonormal, Q psi = lambda psi with
    the stencil M (not the dense matrix the eigensolver saw); on unit links the
    smallest |lambda| is the free-field closed form min_p |1 - 2 kappa sum cos p
    +- 2 i kappa |sin p|| (antiperiodic time)."""
    L = (4, 2, 2, 4)
    U = synth.gauge_field(L, 0.3, 8)
    D = dirac.WilsonClover(U, L, 0.124, 1.0)
    nev = 6
    lam, vec = dirac.low_modes(D, nev)
    sv = np.sort(np.linalg.svd(D.dense(), compute_uv=False))
    assert np.abs(np.sort(np.abs(lam)) - sv[:nev]).max() < 1e-12
    assert np.all(np.diff(np.abs(lam)) >= -1e-14)
    V = vec.reshape(nev, -1)
    assert np.abs(V.conj() @ V.T - np.eye(nev)).max() < 1e-12
    Qv = dirac.fields_to_canonical(dirac.gamma5_field(D.M(dirac.fields_to_lattice(vec, L))))
    assert np.abs(Qv - lam[:, None, None, None] * vec).max() < 1e-12
    # free field: |lambda| of Q = |eigenvalues of M| = |1 - 2k sum_mu cos p_mu +- 2ik |sin p||
    Uf = np.tile(np.eye(3, dtype=np.complex128), (int(np.prod(L)), 4, 1, 1))
    kap = 0.11
    Df = dirac.WilsonClover(Uf, L, kap, 1.0)
    lamf, _ = dirac.low_modes(Df, 1)
    ps = [2 * np.pi * (np.arange(L[0]) + 0.5) / L[0]] + [2 * np.pi * np.arange(l) / l for l in L[1:]]
    P = np.meshgrid(*ps, indexing="ij")
    re = 1 - 2 * kap * sum(np.cos(p) for p in P)
    im = 2 * kap * np.sqrt(sum(np.sin(p) ** 2 for p in P))
    assert abs(abs(lamf[0]) - np.sqrt(re ** 2 + im ** 2).min()) < 1e-12


def test_deficit():
    """eq:cdeficit: 0 for the test vectors (each lies in the span of its block
    projections), 1 for a field orthogonal to the block subspace, and
    |P psi|^2 + |(1 - P) psi|^2 = |psi|^2 (P an orthogonal projector)."""
    L, b, Nv = (4, 2, 4, 2), (2, 2, 2, 2), 3
    U, D, bl, tv, B = _setup(L, b, Nv, seed=9)
    assert np.abs(B.deficit(tv)).max() < 1e-13
    psi = dirac.fields_to_lattice(synth.gaussian_fields(2, L, 44), L)
    ort = psi - B.prolong(B.restrict(psi))
    assert np.abs(B.deficit(ort) - 1.0).max() < 1e-13
    eps = B.deficit(psi)
    pn = np.linalg.norm(B.prolong(B.restrict(psi)).reshape(2, -1), axis=1)
    n = np.linalg.norm(psi.reshape(2, -1), axis=1)
    assert np.abs((pn / n) ** 2 + eps ** 2 - 1.0).max() < 1e-13


def test_even_odd_split():
    """The oracle's even-odd reduction of D_1 (coarse solves with the even-odd
    preconditioned coarse operator, sec. "Comparison of the cost"), pinned by
    * the parity lists against coordinates taken from fine sites through
      Blocking.block_of (an independent route to the block index),
    * the stencil (fig:A): with every coarse extent even, the same-parity
      blocks of the dense D_1 are block diagonal (one nc x nc block per site),
    * the Schur determinant identity det D_1 = det A_ee det A_oo det S,
    * the reduced solve plus reconstruction against a dense solve of D_1."""
    L, b, Nv = (4, 4, 8, 4), (2, 2, 2, 2), 3
    U, D, bl, tv, B = _setup(L, b, Nv, seed=12)
    D1 = coarse.galerkin(D, B)
    nbr = bl.neighbour_table()
    L1 = bl.L1
    nc = 2 * Nv
    e, o = coarse.parity_sites(L1)
    assert len(e) == len(o) == bl.V1 // 2
    assert np.all(np.diff(e) > 0) and np.all(np.diff(o) > 0)
    for y, par in [(int(s), 0) for s in e] + [(int(s), 1) for s in o]:
        yc = None
        for x0 in range(L[0]):
            for x1 in range(L[1]):
                for x2 in range(L[2]):
                    for x3 in range(L[3]):
                        if bl.block_of((x0, x1, x2, x3)) == y and yc is None:
                            yc = (x0 // b[0], x1 // b[1], x2 // b[2], x3 // b[3])
        assert sum(yc) % 2 == par
    Aee, Aeo, Aoe, Aoo = coarse.eo_split(D1, nbr, L1)
    Vh = bl.V1 // 2
    for M in (Aee, Aoo):
        blk = M.reshape(Vh, nc, Vh, nc)
        off = blk * (1 - np.eye(Vh))[:, None, :, None]
        assert np.abs(off).max() == 0.0
    A = coarse.coarse_dense(D1, nbr)
    # the split covers A exactly
    assert abs(np.linalg.norm(A) ** 2 - sum(np.linalg.norm(M) ** 2 for M in (Aee, Aeo, Aoe, Aoo))) < 1e-9
    S = coarse.schur_even(D1, nbr, L1)
    s_a, l_a = np.linalg.slogdet(A)
    parts = [np.linalg.slogdet(M) for M in (Aee, Aoo, S)]
    assert abs(l_a - sum(p[1] for p in parts)) < 1e-9
    assert abs(s_a - np.prod([p[0] for p in parts])) < 1e-9
    rhs = synth.gaussian_coarse(1, bl.V1, nc, 3)[0]
    x = coarse.solve_eo(D1, nbr, L1, rhs)
    ref = np.linalg.solve(A, rhs.reshape(-1)).reshape(bl.V1, nc)
    assert np.abs(x - ref).max() < 1e-11 * np.abs(ref).max()
    # the reduced system is better conditioned than D_1 on this operator
    assert np.linalg.cond(S) < np.linalg.cond(A)
    # deflation with the constant even-site vectors: Y orthonormal, the
    # projector identity S P_R = P_L S, and the deflated solve reproduces S^-1 b
    Y = coarse.eo_constant_vectors(L1, nc)
    assert np.abs(Y.T @ Y - np.eye(nc)).max() < 1e-14
    E = Y.T @ S @ Y
    Ei = np.linalg.inv(E)
    PL = np.eye(S.shape[0]) - S @ Y @ Ei @ Y.T
    PR = np.eye(S.shape[0]) - Y @ Ei @ Y.T @ S
    assert np.abs(S @ PR - PL @ S).max() < 1e-12
    bh = rhs[e].reshape(-1)
    xd = coarse.solve_eo_deflated(S, Y, bh)
    assert np.abs(xd - np.linalg.solve(S, bh)).max() < 1e-10 * np.abs(xd).max()


def test_inner_level():
    """Inner-level R_1, T_1 and D_2 = R_1 D_1 T_1 (nested hierarchy), pinned by
    * the level-2 block index of every level-1 site against Blocking.block_of
      on the fine lattice with the level-2 block size (an independent route),
    * R_1 T_1 = 1 and T_1 R_1 a projector,
    * the nearest-neighbour structure: D_2 couples a level-2 block only to
      itself and its eight neighbours on the level-2 grid,
    * the limit of one level-2 block (the coarsest lattice of fig:nesting):
      D_2 equals the top level spanned by the constant coarse vectors, one per
      coarse component, built by the TopLevel route (chiral split, Gram-Schmidt,
      stencil apply)."""
    L, b, Nv = (8, 4, 4, 8), (2, 2, 2, 2), 2
    U, D, bl, tv, B = _setup(L, b, Nv, seed=21)
    D1 = coarse.galerkin(D, B)
    nbr = bl.neighbour_table()
    nc = 2 * Nv
    r = (2, 1, 2, 2)
    b2 = tuple(b[mu] * r[mu] for mu in range(4))
    bl2 = subspace.Blocking(L, b2)
    z = coarse.level2_of(bl.L1, r)
    for y in range(bl.V1):
        yc = np.unravel_index(y, bl.L1)
        x = tuple(int(yc[mu]) * b[mu] for mu in range(4))
        assert z[y] == bl2.block_of(x)
    R = coarse.inner_restrictor(bl.L1, r, nc)
    assert np.abs(R @ R.T - np.eye(R.shape[0])).max() < 1e-14
    P = R.T @ R
    assert np.abs(P @ P - P).max() < 1e-14
    D2 = coarse.level2_dense(D1, nbr, bl.L1, r)
    nbr2 = bl2.neighbour_table()
    V2 = bl2.V1
    for zz in range(V2):
        for zp in range(V2):
            if zp not in nbr2[zz]:
                assert np.abs(D2[zz * nc:(zz + 1) * nc, zp * nc:(zp + 1) * nc]).max() == 0.0
    # one level-2 block: the top level from the constant coarse vectors
    rall = bl.L1
    D2one = coarse.level2_dense(D1, nbr, bl.L1, rall)
    modes = np.zeros((Nv, bl.V1, nc), dtype=np.complex128)
    for c in range(Nv):
        modes[c, :, c] = 1.0
        modes[c, :, Nv + c] = 1.0
    top = coarse.TopLevel(modes, D1, nbr, Nv)
    assert np.abs(D2one - top.D2).max() < 1e-12
