"""Pins of the oracle's SAP smoother: the block operator equals the dense
restriction of M to the block's sites (with the wrap-around couplings of a
block that spans a whole extent), the minimal-residual block solve converges
to the dense block solution, a cycle with exact block solves leaves a zero
residual on the blocks visited last, and SAP cycles converge to M^{-1} r."""
import numpy as np

from oracle import dirac, subspace, sap
from paper_2412_06347_amd import synth

L, B = (4, 2, 2, 4), (2, 2, 2, 2)      # block grid (2, 1, 1, 2): extents one and two


def _setup(seed=3):
    U = synth.gauge_field(L, 0.3, seed)
    D = dirac.WilsonClover(U, L, 0.124, 1.0)
    bl = subspace.Blocking(L, B)
    return D, bl


def _idx(mask):
    sites = np.flatnonzero(mask.ravel())
    return (sites[:, None] * 12 + np.arange(12)[None, :]).ravel()


def test_block_operator_is_dense_restriction():
    D, bl = _setup()
    Md = D.dense()
    rng = np.random.default_rng(5)
    for y in range(bl.V1):
        mask = sap.block_mask(bl, y)
        idx = _idx(mask)
        assert len(idx) == 12 * bl.Vb
        s = np.zeros((*L, 4, 3), dtype=np.complex128)
        v = rng.standard_normal(len(idx)) + 1j * rng.standard_normal(len(idx))
        s.reshape(-1)[idx] = v
        got = sap.block_apply(D, mask, s).reshape(-1)
        assert np.abs(got[idx] - Md[np.ix_(idx, idx)] @ v).max() < 1e-12
        assert np.abs(np.delete(got, idx)).max() == 0.0


def test_mr_block_solve_converges_to_dense():
    D, bl = _setup()
    Md = D.dense()
    rho = dirac.fields_to_lattice(synth.gaussian_fields(1, L, 41), L)[0]
    for y in (0, bl.V1 - 1):
        mask = sap.block_mask(bl, y)
        idx = _idx(mask)
        d = sap.mr_block(D, mask, rho, 400).reshape(-1)
        ref = np.linalg.solve(Md[np.ix_(idx, idx)], rho.reshape(-1)[idx])
        assert np.linalg.norm(d[idx] - ref) / np.linalg.norm(ref) < 1e-10
        assert np.abs(np.delete(d, idx)).max() == 0.0


def test_cycle_residual_vanishes_on_last_colour():
    D, bl = _setup()
    r = dirac.fields_to_lattice(synth.gaussian_fields(1, L, 42), L)[0]
    z = sap.sap_cycle(D, bl, r, np.zeros_like(r), 400)
    res = r - D.M(z[None])[0]
    on1 = np.zeros(L, dtype=bool)
    for y in range(bl.V1):
        if sap.block_colour(bl, y) == 1:
            on1 |= sap.block_mask(bl, y)
    assert on1.sum() * 2 == np.prod(L)
    rel = lambda a: np.linalg.norm(a) / np.linalg.norm(r)
    assert rel(res[on1]) < 1e-10
    assert rel(res[~on1]) > 1e-3


def test_sap_iteration_converges():
    D, bl = _setup()
    r = dirac.fields_to_lattice(synth.gaussian_fields(1, L, 43), L)[0]
    x = np.linalg.solve(D.dense(), r.reshape(-1)).reshape(r.shape)
    z = np.zeros_like(r)
    errs = []
    for _ in range(12):
        z = sap.sap_cycle(D, bl, r, z, 4)
        errs.append(np.linalg.norm(z - x) / np.linalg.norm(x))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-2 * errs[0]
