"""Pins of the oracle's contractions and estimators: brute-force correlators
from dense propagators, the telescoping sum sum_ij C_ij = C, exact dilution of
the stochastic estimator, the exact top-level formula against the brute-force
S_2 S_2 term, the coarse-gamma route against prolonged fields, and the
free-field point correlator against a momentum-space closed form."""
import numpy as np
import pytest

from oracle import dirac, subspace, coarse, solvers, estimators as est
from paper_2412_06347_amd import synth


@pytest.fixture(scope="module")
def small():
    L, b, Nv, Nlm = (4, 2, 2, 4), (2, 2, 2, 2), 3, 2
    U = synth.gauge_field(L, 0.3, 21)
    D = dirac.WilsonClover(U, L, 0.124, 1.0)
    bl = subspace.Blocking(L, b)
    tv = dirac.fields_to_lattice(synth.gaussian_fields(Nv, L, 22), L)
    B = subspace.BlockBasis(bl, tv)
    D1 = coarse.galerkin(D, B)
    nbr = bl.neighbour_table()
    A1 = coarse.coarse_dense(D1, nbr)
    top = coarse.TopLevel(synth.gaussian_coarse(Nlm, bl.V1, B.nc, 23), D1, nbr, Nv)
    Md = D.dense()
    S = np.linalg.inv(Md)
    T = B.basis_canonical().reshape(bl.V1 * B.nc, -1).T
    Sge1 = T @ np.linalg.inv(A1) @ T.conj().T
    S2 = T @ top.W @ np.linalg.inv(top.D2) @ top.W.conj().T @ T.conj().T
    pieces = [S - Sge1, Sge1 - S2, S2]
    return dict(L=L, D=D, bl=bl, B=B, D1=D1, top=top, S=S, pieces=pieces, T=T)


def _col(S, L, y, a):
    V = int(np.prod(L))
    s = np.ravel_multi_index(y, L)
    return S[:, s * 12 + a].reshape(*L, 4, 3)


def test_gamma5_hermiticity_of_pieces(small):
    L = small["L"]
    V = int(np.prod(L))
    G5 = np.kron(np.eye(V), np.kron(np.diag([1, 1, -1, -1]), np.eye(3)))
    for P in [small["S"]] + small["pieces"]:
        assert np.abs(G5 @ P.conj().T @ G5 - P).max() < 1e-11 * np.abs(P).max()


def test_point_correlator_vs_brute_force(small):
    """Average of point-source correlators over all spatial source positions
    equals eq:tmr evaluated with the dense propagator."""
    L, S = small["L"], small["S"]
    C = est.exact_correlator(S, S, L)
    L3 = L[1] * L[2] * L[3]
    for y0 in range(L[0]):
        acc = np.zeros(L[0], dtype=complex)
        for ys in np.ndindex(L[1], L[2], L[3]):
            y = (y0,) + ys
            cols = np.stack([_col(S, L, y, a) for a in range(12)])
            acc += est.point_correlator(cols, cols, y0)
        acc /= L3
        expect = np.array([C[(y0 + t) % L[0], y0] for t in range(L[0])])
        assert np.abs(acc - expect).max() < 1e-12 * np.abs(expect).max()


def test_telescoping_sum(small):
    """sum_ij C_ij = C (eq:C_ij) and sum_k C_Lk = C (eq:cdecomp)."""
    L, S, P = small["L"], small["S"], small["pieces"]
    C = est.exact_correlator(S, S, L)
    Cij = [[est.exact_correlator(P[i], P[j], L) for j in range(3)] for i in range(3)]
    tot = sum(Cij[i][j] for i in range(3) for j in range(3))
    assert np.abs(tot - C).max() < 1e-12 * np.abs(C).max()
    CL = est.level_sums(Cij)
    assert np.abs(sum(CL) - C).max() < 1e-12 * np.abs(C).max()
    # each level against the assignment of fig:C written out term by term
    tol = 1e-12 * np.abs(C).max()
    assert np.abs(CL[0] - (Cij[0][0] + Cij[0][1] + Cij[1][0] + Cij[0][2] + Cij[2][0])).max() < tol
    assert np.abs(CL[1] - (Cij[1][1] + Cij[1][2] + Cij[2][1])).max() < tol
    assert np.abs(CL[2] - Cij[2][2]).max() < tol
    # C is real up to rounding for the isovector vector current
    assert np.abs(C.imag).max() < 1e-10 * np.abs(C).max()


def test_exact_dilution(small):
    """Replacing the noise by every unit vector of the slice turns the
    stochastic estimator eq:C_stoch2 into the exact C_ij(t_n + t, t_n)."""
    L, P = small["L"], small["pieces"]
    tn = 1
    L3 = L[1] * L[2] * L[3]
    for (i, j) in [(0, 0), (0, 1), (2, 1)]:
        Cx = est.exact_correlator(P[i], P[j], L)
        acc = np.zeros(L[0], dtype=complex)
        for xs in range(L3):
            for c in range(3):
                xi = np.zeros((L3, 3), dtype=complex)
                xi[xs, c] = 1.0
                eta = est.spin_diluted_sources(L, xi, tn).reshape(4, -1)
                Si = (P[i] @ eta.T).T.reshape(4, *L, 4, 3)
                Sj = (P[j] @ eta.T).T.reshape(4, *L, 4, 3)
                acc += est.stochastic_pair(Si, Sj, tn, L)
        expect = np.array([Cx[(tn + t) % L[0], tn] for t in range(L[0])])
        assert np.abs(acc - expect).max() < 1e-12 * np.abs(expect).max()


def test_noise_values():
    xi = synth.z4_noise(50, (4, 4, 4, 4), 3)
    assert np.allclose(np.abs(xi.real), 1 / np.sqrt(2))
    assert np.allclose(np.abs(xi.imag), 1 / np.sqrt(2))
    assert abs(xi.mean()) < 0.05


def test_exact_top_vs_brute_force(small):
    """eq:G_LL:exact equals the time-averaged brute-force C_22."""
    L, bl, B, top, P = small["L"], small["bl"], small["B"], small["top"], small["pieces"]
    G1 = coarse.coarse_gammas(B)
    G2 = top.gammas(G1, bl)
    got = est.exact_top(top.Q2, G2, L)
    expect = est.timeavg(est.exact_correlator(P[2], P[2], L))
    assert np.abs(got - expect).max() < 1e-12 * np.abs(expect).max()


def test_coarse_gamma_route(small):
    """c_b^+ (gamma5 gamma_k)_1(x0) c_a equals the slice bilinear of the
    prolonged fields (eq:coarse:gamma with an open time index)."""
    L, bl, B = small["L"], small["bl"], small["B"]
    G1 = coarse.coarse_gammas(B)
    g, g5 = dirac.gammas()
    ca = synth.gaussian_coarse(1, bl.V1, B.nc, 31)
    cb = synth.gaussian_coarse(1, bl.V1, B.nc, 32)
    fa, fb = B.prolong(ca), B.prolong(cb)
    y0 = np.unravel_index(np.arange(bl.V1), bl.L1)[0]
    for k in range(1, 4):
        fine = est.slice_bilinear(fb, g5 @ g[k], fa)[0]
        crs = np.zeros(L[0], dtype=complex)
        for y in range(bl.V1):
            for t in range(bl.b[0]):
                crs[y0[y] * bl.b[0] + t] += cb[0, y].conj() @ G1[y, t, k - 1] @ ca[0, y]
        assert np.abs(fine - crs).max() < 1e-12 * np.abs(fine).max()


def test_gcr_matches_dense(small):
    D = small["D"]
    L = small["L"]
    b = dirac.fields_to_lattice(synth.gaussian_fields(2, L, 40), L)
    x, it, res = solvers.gcr(D.M, b, tol=1e-12)
    assert np.all(res <= 1e-12)
    xd = (small["S"] @ b.reshape(2, -1).T).T
    assert np.abs(x.reshape(2, -1) - xd).max() < 1e-10 * np.abs(xd).max()


def test_free_field_point_correlator_closed_form():
    """Free field: S(x,0) = (1/V) sum_p e^{ipx} M(p)^{-1}; the point correlator
    from solver-built columns equals the momentum-space closed form."""
    L = (8, 4, 4, 2)
    kappa = 0.115
    V = int(np.prod(L))
    U = np.zeros((V, 4, 3, 3), dtype=complex)
    U[:] = np.eye(3)
    D = dirac.WilsonClover(U, L, kappa, 1.0)
    src = est.point_sources(L, (0, 0, 0, 0))
    x, _, res = solvers.gcr(D.M, src, tol=1e-13)
    got = est.point_correlator(x, x, 0)
    # closed form
    g, g5 = dirac.gammas()
    n = np.stack(np.meshgrid(*[np.arange(l) for l in L], indexing="ij"), -1)
    p = 2 * np.pi * n / np.array(L)
    p[..., 0] += np.pi / L[0]
    Mp = (1 - 2 * kappa * np.cos(p).sum(-1))[..., None, None] * np.eye(4)
    for mu in range(4):
        Mp = Mp + 2j * kappa * np.sin(p[..., mu])[..., None, None] * g[mu]
    Sp = np.linalg.inv(Mp)
    # S(x,0) = (1/V) sum_p e^{ipx} S(p); the antiperiodic shift is a phase e^{i pi x0/L0}
    Sx = np.fft.ifftn(Sp, axes=(0, 1, 2, 3))
    Sx = Sx * np.exp(1j * np.pi * np.arange(L[0]) / L[0])[:, None, None, None, None, None]
    expect = np.zeros(L[0], dtype=complex)
    for k in range(1, 4):
        Gs, Gk = g[k] @ g5, g5 @ g[k]
        # -1/3 sum_x tr_spin[S Gs S^+ Gk] * 3 colours
        m = np.einsum("...ab,bc,...dc,de->...ae", Sx, Gs, Sx.conj(), Gk)
        expect += -np.trace(m, axis1=-2, axis2=-1).sum(axis=(1, 2, 3))
    assert np.abs(got - expect).max() < 1e-10 * np.abs(expect).max()


def test_level_sums_by_bilinearity(small):
    """Each level sum equals a difference of correlators of cumulative pieces
    S_{>=k} = sum_{i>=k} S_i, computed from the dense propagators alone:
    C_Lk = C(S_{>=k}, S_{>=k}) - C(S_{>=k+1}, S_{>=k+1}).  A level sum that
    took i < k instead of i > k, or dropped a cross term, fails here."""
    L, P = small["L"], small["pieces"]
    Cij = [[est.exact_correlator(P[i], P[j], L) for j in range(3)] for i in range(3)]
    CL = est.level_sums(Cij)
    cum = [P[0] + P[1] + P[2], P[1] + P[2], P[2]]
    Ccum = [est.exact_correlator(Sk, Sk, L) for Sk in cum] + [0.0]
    scale = np.abs(Ccum[0]).max()
    for k in range(3):
        assert np.abs(CL[k] - (Ccum[k] - Ccum[k + 1])).max() < 1e-12 * scale
    # the levels are not all equal to the diagonal terms (the cross terms matter)
    assert np.abs(CL[0] - Cij[0][0]).max() > 1e-6 * scale


def test_level_estimates_point_average(small):
    """Point sources at every site, averaged level by level, give the
    time-averaged level sums of the brute-force C_ij (eq:timetrans)."""
    L, P = small["L"], small["pieces"]
    Cij = [[est.exact_correlator(P[i], P[j], L) for j in range(3)] for i in range(3)]
    expect = np.array([est.timeavg(c) for c in est.level_sums(Cij)])
    pieces, t_src = [], []
    for y in np.ndindex(*L):
        pieces.append([np.stack([_col(Pk, L, y, a) for a in range(12)]) for Pk in P])
        t_src.append(y[0])
    got = est.level_estimates(est.point_correlator, pieces, t_src)
    assert np.abs(got - expect).max() < 1e-12 * np.abs(expect).max()


def test_level_estimates_exact_dilution(small):
    """Unit-vector noise on one slice: N times the source mean of the
    stochastic level estimates equals the brute-force level sums at that
    source time (eq:C_stoch with exact dilution)."""
    L, P = small["L"], small["pieces"]
    tn = 2
    L3 = L[1] * L[2] * L[3]
    Cij = [[est.exact_correlator(P[i], P[j], L) for j in range(3)] for i in range(3)]
    CL = est.level_sums(Cij)
    expect = np.array([[c[(tn + t) % L[0], tn] for t in range(L[0])] for c in CL])
    pieces = []
    for xs in range(L3):
        for c in range(3):
            xi = np.zeros((L3, 3), dtype=complex)
            xi[xs, c] = 1.0
            eta = est.spin_diluted_sources(L, xi, tn).reshape(4, -1)
            pieces.append([(Pk @ eta.T).T.reshape(4, *L, 4, 3) for Pk in P])
    got = est.level_estimates(lambda a, b, t: est.stochastic_pair(a, b, t, L), pieces, [tn] * len(pieces))
    assert np.abs(len(pieces) * got - expect).max() < 1e-12 * np.abs(expect).max()
