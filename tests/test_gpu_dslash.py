"""GPU parity of the clover term and the Wilson-clover apply against the
oracle (FP64 to 1e-12 relative; FP32 / FP16 errors bounded and reported)."""
import numpy as np
import pytest

from oracle import dirac
from paper_2412_06347_amd import synth
from tests.gpu_util import to_dev, from_dev, relerr

pytestmark = pytest.mark.gpu

CASES = [
    # L, block, kappa, csw, eps
    ((4, 4, 4, 4), (2, 2, 2, 2), 0.120, 1.0, 0.3),      # the 4^4 workload
    ((6, 4, 6, 2), (3, 2, 3, 1), 0.124, 1.3, 0.3),      # odd blocks, extent-2 direction
    ((8, 2, 4, 6), (8, 1, 2, 3), 0.125, 1.0, 0.25),     # block = L in time, b = 1
]


def _ctx(L, b, kappa, csw, eps, seed=1):
    import torch
    from paper_2412_06347_amd import mglma
    U = synth.gauge_field(L, eps, seed)
    ctx = mglma.Context(L, b, kappa, csw)
    ctx.load_gauge(to_dev(U))
    torch.cuda.synchronize()
    return ctx, U


@pytest.mark.parametrize("case", CASES)
def test_clover_parity(case):
    import torch
    L, b, kappa, csw, eps = case
    ctx, U = _ctx(*case)
    out = torch.empty((ctx.V, 2, 6, 6, 2), dtype=torch.float64, device="cuda")
    ctx.export_clover(out)
    got = from_dev(out)
    Cl = dirac.clover(U, L, kappa, csw).reshape(-1, 12, 12)
    ref = np.stack([Cl[:, :6, :6], Cl[:, 6:, 6:]], axis=1)
    assert np.abs(got - ref).max() < 1e-13


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("gamma5", [0, 1])
def test_apply_parity(case, gamma5):
    import torch
    from paper_2412_06347_amd import mglma
    L, b, kappa, csw, eps = case
    ctx, U = _ctx(*case)
    D = dirac.WilsonClover(U, L, kappa, csw)
    nrhs = 3
    psi = synth.gaussian_fields(nrhs, L, seed=7)
    ref = D.M(dirac.fields_to_lattice(psi, L))
    if gamma5:
        ref = dirac.gamma5_field(ref)
    ref = dirac.fields_to_canonical(ref)
    for prec, tol in [(mglma.F64, 1e-12), (mglma.F32, 2e-6), (mglma.F16, 2e-3)]:
        x = ctx.fine(nrhs, prec)
        y = ctx.fine(nrhs, prec)
        ctx.import_fields(to_dev(psi), x, prec)
        ctx.apply_D(x, y, prec, gamma5)
        out = torch.empty((nrhs, ctx.V, 4, 3, 2), dtype=torch.float64, device="cuda")
        ctx.export_fields(y, out, prec)
        got = from_dev(out)
        err = relerr(got, ref)
        print("L=%s prec=%d gamma5=%d rel err %.3e" % (L, prec, gamma5, err))
        assert err < tol


@pytest.mark.parametrize("nrhs", [2, 4, 7])
def test_apply_f16_batches(nrhs):
    """FP16 batches go through the packed kernel in groups of three right-hand
    sides; ragged last groups (4 = 3 + 1, 7 = 3 + 3 + 1) and a lattice whose
    volume is not a multiple of the 256-site tile (6 x 4 x 6 x 2 = 288)."""
    import torch
    from paper_2412_06347_amd import mglma
    case = CASES[1]
    L = case[0]
    ctx, U = _ctx(*case)
    D = dirac.WilsonClover(U, L, case[2], case[3])
    psi = synth.gaussian_fields(nrhs, L, seed=70 + nrhs)
    for gamma5 in (0, 1):
        ref = D.M(dirac.fields_to_lattice(psi, L))
        if gamma5:
            ref = dirac.gamma5_field(ref)
        ref = dirac.fields_to_canonical(ref)
        x = ctx.fine(nrhs, mglma.F16)
        y = ctx.fine(nrhs, mglma.F16)
        ctx.import_fields(to_dev(psi), x, mglma.F16)
        ctx.apply_D(x, y, mglma.F16, gamma5)
        out = torch.empty((nrhs, ctx.V, 4, 3, 2), dtype=torch.float64, device="cuda")
        ctx.export_fields(y, out, mglma.F16)
        got = from_dev(out)
        for r in range(nrhs):
            err = relerr(got[r], ref[r])
            print("nrhs=%d rhs=%d gamma5=%d rel err %.3e" % (nrhs, r, gamma5, err))
            assert err < 2e-3


def test_import_export_roundtrip():
    import torch
    from paper_2412_06347_amd import mglma
    ctx, U = _ctx(*CASES[1])
    psi = synth.gaussian_fields(2, CASES[1][0], seed=3)
    x = ctx.fine(2, mglma.F64)
    ctx.import_fields(to_dev(psi), x)
    out = torch.empty((2, ctx.V, 4, 3, 2), dtype=torch.float64, device="cuda")
    ctx.export_fields(x, out)
    assert np.array_equal(from_dev(out), psi)


@pytest.mark.parametrize("L,b", [((32, 16, 16, 16), (4, 4, 4, 4))])
def test_apply_parity_full_size(L, b):
    """The 16^3 x 32 workload at full size, FP64, in the launch configuration
    the benchmark times."""
    import torch
    from paper_2412_06347_amd import mglma
    ctx, U = _ctx(L, b, 0.124, 1.0, 0.3, seed=2)
    D = dirac.WilsonClover(U, L, 0.124, 1.0)
    psi = synth.gaussian_fields(1, L, seed=9)
    ref = dirac.fields_to_canonical(D.M(dirac.fields_to_lattice(psi, L)))
    x = ctx.fine(1, mglma.F64)
    y = ctx.fine(1, mglma.F64)
    ctx.import_fields(to_dev(psi), x)
    ctx.apply_D(x, y)
    out = torch.empty((1, ctx.V, 4, 3, 2), dtype=torch.float64, device="cuda")
    ctx.export_fields(y, out)
    assert relerr(from_dev(out), ref) < 1e-12
