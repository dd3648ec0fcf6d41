"""GPU parity of the spectral diagnostics (appendices on the spectra of
coarse and fine operators and on the condition numbers of coarse-grid
operators): the coarse operator without chiral split against the oracle's
T_nc^+ Q T_nc, and the low eigenvalues and the largest |lambda| of every
level's Hermitian operator (fine Q, chiral Q_1, level-2 Q_2, non-chiral
Q_nc) against the oracle's dense eigendecompositions; with the basis built
from the lowest exact modes of Q, the chiral Q_1 reproduces their
eigenvalues (fig:spectra)."""
import numpy as np
import pytest

from oracle import coarse, subspace
from paper_2412_06347_amd import synth
from tests.gpu_util import to_dev, from_dev
from tests.gpu_setup import Pair

pytestmark = pytest.mark.gpu

OP_FINE, OP_COARSE, OP_LEVEL2, OP_NONCHIRAL = 0, 1, 2, 3


@pytest.fixture(scope="module")
def pair():
    P = Pair((4, 4, 4, 4), (2, 2, 2, 2), 6, kappa=0.124)
    V = int(np.prod(P.L))
    g5 = np.kron(np.eye(V), np.kron(np.diag([1, 1, -1, -1]), np.eye(3)))
    P.Qd = g5 @ P.D.dense()
    return P


def _low(A, k):
    lam = np.linalg.eigvalsh(0.5 * (A + A.conj().T))
    return lam[np.argsort(np.abs(lam))[:k]], np.abs(lam).max()


def test_nonchiral_operator_parity(pair):
    P = pair
    tvd = P.fine_dev(P.tv)
    P.ctx.build_nonchiral(tvd)
    import torch
    Nv = P.Nv
    out = torch.empty((P.bl.V1, 9, Nv, Nv, 2), dtype=torch.float64, device="cuda")
    P.ctx.export_nonchiral_op(out)
    got = coarse.coarse_dense(from_dev(out), P.nbr)
    ref = coarse.nonchiral_dense(P.Qd, P.bl, P.lat(P.tv))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("non-chiral coarse operator vs oracle: %.2e" % err)
    assert err < 1e-12


@pytest.mark.parametrize("op", [OP_FINE, OP_COARSE, OP_LEVEL2, OP_NONCHIRAL])
def test_level_spectra_parity(pair, op):
    P = pair
    ctx = P.ctx
    nev, ng = 4, 6
    if op == OP_FINE:
        ref, amax = _low(P.Qd, nev)
        init = P.fine_dev(synth.gaussian_fields(nev + ng, P.L, 71))
    elif op == OP_COARSE:
        A = coarse.coarse_dense(P.D1, P.nbr)
        g5 = np.tile(subspace.coarse_gamma5(P.Nv), P.bl.V1)
        ref, amax = _low(g5[:, None] * A, nev)
        init = to_dev(synth.gaussian_coarse(nev + ng, P.bl.V1, 2 * P.Nv, 72))
    elif op == OP_LEVEL2:
        ctx.build_level2((4, 4, 2, 2))
        r = (2, 2, 1, 1)
        A2 = coarse.level2_dense(P.D1, P.nbr, P.bl.L1, r)
        V2 = ctx.V2
        g5 = np.tile(subspace.coarse_gamma5(P.Nv), V2)
        ref, amax = _low(g5[:, None] * A2, nev)
        init = to_dev(synth.gaussian_coarse(nev + ng, V2, 2 * P.Nv, 73))
    else:
        ctx.build_nonchiral(P.fine_dev(P.tv))
        ref, amax = _low(coarse.nonchiral_dense(P.Qd, P.bl, P.lat(P.tv)), nev)
        init = to_dev(synth.gaussian_coarse(nev + ng, P.bl.V1, P.Nv, 74))
    rc, lam, vec, st = ctx.level_eigs(op, init, nev, tol=1e-12)
    print("op %d: lambda %s vs %s, |lambda|_max %.4f vs %.4f" % (op, lam, ref, st["lambda_max_abs"], amax))
    assert np.abs(lam - ref).max() < 1e-10 * np.abs(ref).max()
    assert abs(st["lambda_max_abs"] - amax) < 0.02 * amax


def test_exact_modes_reproduced_by_chiral_coarse_operator(pair):
    """The block basis from the Nv lowest exact modes of Q (device
    eigensolver): the Nv lowest eigenvalues of the chiral Q_1 equal those of
    Q (fig:spectra), which the non-chiral operator does not guarantee."""
    P = pair
    ctx = P.ctx
    Nv = P.Nv
    rc, lam, modes, st = ctx.level_eigs(OP_FINE, P.fine_dev(synth.gaussian_fields(2 * Nv + 4, P.L, 75)), 2 * Nv,
                                        tol=1e-12)
    ctx.build_subspace(modes[:Nv].contiguous())
    rc, lam1, _, _ = ctx.level_eigs(OP_COARSE, to_dev(synth.gaussian_coarse(Nv + 6, P.bl.V1, 2 * Nv, 76)), Nv,
                                    tol=1e-12)
    print("Q lowest", lam[:Nv], "Q_1 lowest", lam1)
    assert np.abs(np.sort(lam1) - np.sort(lam[:Nv])).max() < 1e-10
    ctx.build_nonchiral(modes[:Nv].contiguous())
    rc, lamn, _, _ = ctx.level_eigs(OP_NONCHIRAL, to_dev(synth.gaussian_coarse(Nv + 6, P.bl.V1, Nv, 77)), Nv,
                                    tol=1e-12, raise_on_error=False)
    print("non-chiral lowest", lamn)
    # restore the fixture's subspace for other tests
    ctx.build_subspace(P.fine_dev(P.tv))
