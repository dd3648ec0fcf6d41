"""Sources, propagator pieces and correlator contractions (oracle; test
infrastructure only).

Definitions followed (lattice units a = 1):

* isovector vector correlator eq:tmr
      C(x0,y0) = -1/(3 L^3) sum_k sum_{x,y} tr{ S(x,y) gamma_k S(y,x) gamma_k };
* level decomposition eq:C_ij, C = sum_ij C_ij, level sums C_Lk;
* time-translation average eq:timetrans  G(t) = (1/L0) sum_{y0} C(t+y0, y0);
* exact coarsest-level term eq:G_LL:exact;
* stochastic time-diluted wall sources with noise uniform on
  {+-1 +- i}/sqrt(2), spin-diagonal (4 inversions per source), and the
  estimator eq:C_stoch / eq:C_stoch2 (section "Stochastic estimator on
  level k").

Readings:
* the propagator is S = M^{-1} with the kappa-normalised M (so S differs from
  D^{-1} by the factor 2 kappa, and correlators by (2 kappa)^2);
* a point source at y stands in for the sum over the spatial source position:
  C_pt(x0,y0) = -1/3 sum_k sum_x tr{S(x,y) gamma_k S(y,x) gamma_k}, using
  S(y,x) = gamma5 S(x,y)^+ gamma5 (every S_l built from a chirality-preserving
  basis has this property);
* the level pieces are S_0 = S - T D1^{-1} R, S_1 = T D1^{-1} R - T W D2^{-1} W^+ R,
  S_2 = T W D2^{-1} W^+ R (eq:mglma:decomp with the identities of the
  chirality appendix, T Q_l^{-1} R gamma5 = T D_l^{-1} R).
"""
from __future__ import annotations

import numpy as np

from .dirac import gammas, spin_mul


# ---------------------------------------------------------------------------
# sources
# ---------------------------------------------------------------------------
def point_sources(L, y):
    """The 12 unit sources e_{y,(s,c)} as lattice fields [12][L..][4][3]."""
    e = np.zeros((12, *L, 4, 3), dtype=np.complex128)
    for a in range(12):
        e[(a,) + tuple(y) + (a // 3, a % 3)] = 1.0
    return e


def spin_diluted_sources(L, xi, t):
    """eta^{(s)}(x) = delta_{x0,t} e_s (x) xi(x): [4][L..][4][3].

    xi: [L1*L2*L3][3] colour noise on the slice."""
    eta = np.zeros((4, *L, 4, 3), dtype=np.complex128)
    xs = xi.reshape(L[1], L[2], L[3], 3)
    for s in range(4):
        eta[s, t, :, :, :, s, :] = xs
    return eta


# ---------------------------------------------------------------------------
# basic bilinears
# ---------------------------------------------------------------------------
def slice_bilinear(a, G, b):
    """f[..., x0] = sum_xvec a(x)^+ G b(x) for lattice fields [..., L..., 4, 3]."""
    gb = spin_mul(G, b)
    return np.einsum("...tijksc,...tijksc->...t", a.conj(), gb)


def point_correlator(Si, Sj, y0):
    """C_ij(y0+t, y0), t = 0..L0-1, for point-source columns Si, Sj [12][L..][4][3]
    (columns a = 3*spin + colour of S_i(., y) and S_j(., y))."""
    g, g5 = gammas()
    L0 = Si.shape[1]
    C = np.zeros(L0, dtype=np.complex128)
    for k in range(1, 4):
        src = g[k] @ g5            # acts on the source spin index
        snk = g5 @ g[k]            # acts on the sink spin index
        f = np.stack([slice_bilinear(Sj[b][None], snk, Si)[:, :] for b in range(12)])
        # f[b, a, x0] = psi^j_b(x)^+ (g5 g_k) psi^i_a(x) summed over the slice
        for a in range(12):
            for b in range(12):
                if a % 3 != b % 3:
                    continue
                w = src[a // 3, b // 3]
                if w != 0:
                    C += w * f[b, a]
    C *= -1.0 / 3.0
    return np.roll(C, -y0)


def stochastic_pair(Si, Sj, tn, L):
    """One-source estimator term G^n_ij(t_n + t, t_n), t = 0..L0-1 (eq:C_stoch2).

    Si[s], Sj[s]: S_i eta^{(s)}, S_j eta^{(s)} for the four spin-diluted
    sources [4][L..][4][3]."""
    g, g5 = gammas()
    L3 = L[1] * L[2] * L[3]
    out = np.zeros(L[0], dtype=np.complex128)
    for k in range(1, 4):
        Gk = g5 @ g[k]
        Gin = g5 @ g[k].conj().T            # gamma5 gamma_k^+ acting on the source
        for s in range(4):
            for sp in range(4):
                c = Gin[sp, s]
                if c == 0:
                    continue
                out += np.conj(c) * slice_bilinear(Sj[sp], Gk, Si[s])
    out *= -1.0 / (3.0 * L3)
    return np.roll(out, -int(tn))


def timeavg(C):
    """eq:timetrans for a full C[x0][y0]: G(t) = (1/L0) sum_y0 C(t+y0, y0)."""
    L0 = C.shape[0]
    return np.array([sum(C[(t + y) % L0, y] for y in range(L0)) for t in range(L0)]) / L0


# ---------------------------------------------------------------------------
# exact (brute-force) correlators from dense propagators (tiny lattices)
# ---------------------------------------------------------------------------
def exact_correlator(Si, Sj, L):
    """C_ij(x0,y0) of eq:C_ij from dense propagators S[V*12][V*12]."""
    g, _ = gammas()
    V = int(np.prod(L))
    L3 = V // L[0]
    Ai = Si.reshape(V, 12, V, 12)
    Aj = Sj.reshape(V, 12, V, 12)
    t_of = np.arange(V) // L3
    C = np.zeros((L[0], L[0]), dtype=np.complex128)
    for k in range(1, 4):
        G = np.kron(g[k], np.eye(3))
        Ti = np.einsum("xayb,bc->xayc", Ai, G)
        Tj = np.einsum("xayb,bc->xayc", Aj, G)
        # tr{S_i(x,y) g_k S_j(y,x) g_k}
        m = np.einsum("xayc,ycxa->xy", Ti, Tj)
        for x0 in range(L[0]):
            for y0 in range(L[0]):
                C[x0, y0] += m[np.ix_(t_of == x0, t_of == y0)].sum()
    return -C / (3.0 * L3)


# ---------------------------------------------------------------------------
# exact top-level term
# ---------------------------------------------------------------------------
def exact_top(Q2, Gamma2, L):
    """eq:G_LL:exact: G(t) = -1/(3 L0 L^3) sum_k sum_y0 tr{G_k(y0+t) Q2^-1 G_k(y0) Q2^-1}.

    Gamma2[L0][3][r][r] = (gamma5 gamma_k)_2(x0)."""
    L0 = L[0]
    L3 = L[1] * L[2] * L[3]
    Qi = np.linalg.inv(Q2)
    A = np.einsum("tkab,bc->tkac", Gamma2, Qi)     # G_k(x0) Q2^-1
    G = np.zeros(L0, dtype=np.complex128)
    for t in range(L0):
        for y0 in range(L0):
            x0 = (y0 + t) % L0
            G[t] += np.einsum("kab,kba->", A[x0], A[y0])
    return -G / (3.0 * L0 * L3)


# ---------------------------------------------------------------------------
# level assembly
# ---------------------------------------------------------------------------
def level_sums(Cij):
    """C_Lk = C_kk + sum_{i>k} (C_ik + C_ki) for a dict or array Cij[i][j]."""
    n = len(Cij)
    return [Cij[k][k] + sum(Cij[i][k] + Cij[k][i] for i in range(k + 1, n)) for k in range(n)]


def level_estimates(pair, pieces, t_src):
    """Level terms averaged over sources (eq:C_stoch for stochastic sources;
    for point sources at time y0 = t_src[n] the average over the source times
    is eq:timetrans).

    pair(Si, Sj, t) returns the one-source two-point function of the pieces
    Si, Sj in the frame t = 0..L0-1 relative to the source time (stochastic_pair
    or point_correlator).  pieces[n][i] holds S_i applied to the columns of
    source n (the level pieces S_0, S_1, ... of eq:mglma:decomp).  For each
    source the C_ij are formed, reduced to the level sums C_Lk (level_sums),
    and the result is the mean over the sources, one row per level."""
    nsrc = len(pieces)
    out = None
    for n in range(nsrc):
        P = pieces[n]
        Cij = [[pair(P[i], P[j], int(t_src[n])) for j in range(len(P))] for i in range(len(P))]
        CL = np.array(level_sums(Cij))
        out = CL if out is None else out + CL
    return out / nsrc
