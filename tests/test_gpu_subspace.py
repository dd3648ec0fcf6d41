"""GPU parity of the block basis, R/T, the Galerkin operator and the coarse
apply against the oracle (FP64 to 1e-12 relative; FP32 and BF16 bounded)."""
import numpy as np
import pytest

from paper_2412_06347_amd import synth
from tests.gpu_util import to_dev, from_dev, relerr
from tests.gpu_setup import Pair

pytestmark = pytest.mark.gpu

CASES = [
    ((4, 4, 4, 4), (2, 2, 2, 2), 8),        # the 4^4 workload: 2^4 blocks, 8 test vectors
    ((6, 4, 6, 2), (3, 2, 3, 1), 3),        # odd blocks, coarse extents 2/3, nc = 6
    ((8, 8, 4, 4), (4, 4, 4, 4), 8),        # 4^4 blocks, coarse extent 1 in space
    ((4, 4, 4, 8), (2, 2, 2, 4), 20),       # nc = 40: partial 16-row / 16-column matrix-core tiles
    ((4, 4, 4, 4), (2, 2, 2, 2), 40),       # nc = 80: the VALU Galerkin kernel (n_c > 64)
]


@pytest.fixture(scope="module", params=CASES, ids=["4^4", "odd", "b4", "nc40", "nc80"])
def pair(request):
    L, b, Nv = request.param
    return Pair(L, b, Nv)


def test_basis_parity(pair):
    import torch
    bl, Nv = pair.bl, pair.Nv
    out = torch.empty((bl.V1, 2 * Nv, bl.Vb, 4, 3, 2), dtype=torch.float64, device="cuda")
    pair.ctx.export_basis(out)
    got = from_dev(out)
    E = np.zeros((bl.V1, 2, Nv, bl.Vb, 4, 3), dtype=complex)
    for a in range(2):
        E[:, a, :, :, 2 * a:2 * a + 2, :] = pair.B.phi[:, a].reshape(bl.V1, Nv, bl.Vb, 2, 3)
    E = E.reshape(bl.V1, 2 * Nv, bl.Vb, 4, 3)
    assert np.abs(got - E).max() < 1e-12


def test_coarse_operator_parity(pair):
    import torch
    bl, nc = pair.bl, 2 * pair.Nv
    out = torch.empty((bl.V1, 9, nc, nc, 2), dtype=torch.float64, device="cuda")
    pair.ctx.export_coarse_op(out)
    got = from_dev(out)
    assert relerr(got, pair.D1) < 1e-12


def test_coarse_gammas_parity(pair):
    import torch
    from oracle import coarse
    bl, Nv = pair.bl, pair.Nv
    out = torch.empty((bl.V1, bl.b[0], 3, Nv, Nv, 2), dtype=torch.float64, device="cuda")
    pair.ctx.export_coarse_gammas(out)
    ref = coarse.coarse_gammas(pair.B)[:, :, :, :Nv, Nv:]
    assert relerr(from_dev(out), ref) < 1e-12


# prec 2: FP32 fields with the FP16 copy of the basis (bound: the FP16
# rounding of the basis, 2^-11 relative per entry)
@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 2e-6), (2, 1e-3)])
def test_restrict_prolong_parity(pair, prec, tol):
    import torch
    from paper_2412_06347_amd import mglma
    n = 19    # more than one 16-wide tile of right-hand sides
    fp = 1 if prec == 2 else prec
    psi = synth.gaussian_fields(n, pair.L, 77)
    ref_c = pair.B.restrict(pair.lat(psi))
    x = pair.fine_dev(psi, fp)
    cdt = torch.float64 if prec == 0 else torch.float32
    c = torch.empty((n, pair.bl.V1, 2 * pair.Nv, 2), dtype=cdt, device="cuda")
    pair.ctx.restrict(x, c, prec)
    e_r = relerr(from_dev(c), ref_c)
    assert e_r < tol
    cv = synth.gaussian_coarse(n, pair.bl.V1, 2 * pair.Nv, 78)
    ref_f = pair.canon(pair.B.prolong(cv))
    ct = to_dev(cv).to(cdt)
    y = pair.ctx.fine(n, fp)
    pair.ctx.prolong(ct, y, prec)
    e_p = relerr(pair.fine_host(y, fp), ref_f)
    print("prec %d: restrict %.2e prolong %.2e" % (prec, e_r, e_p))
    assert e_p < tol


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 2e-6), (3, 2e-2)])
@pytest.mark.parametrize("gamma5", [0, 1])
def test_coarse_apply_parity(pair, prec, tol, gamma5):
    import torch
    from oracle import coarse, subspace
    n = 19    # more than one 16-wide tile of right-hand sides
    v = synth.gaussian_coarse(n, pair.bl.V1, 2 * pair.Nv, 91)
    ref = coarse.coarse_apply(pair.D1, pair.nbr, v)
    if gamma5:
        ref = ref * subspace.coarse_gamma5(pair.Nv)[None, None, :]
    cdt = torch.float64 if prec == 0 else torch.float32
    x = to_dev(v).to(cdt)
    y = torch.empty_like(x)
    pair.ctx.coarse_apply(x, y, prec, gamma5)
    err = relerr(from_dev(y), ref)
    print("coarse apply prec=%d gamma5=%d rel err %.3e" % (prec, gamma5, err))
    assert err < tol


def test_rank_deficient_basis_is_an_error():
    import torch
    from paper_2412_06347_amd import mglma
    L, b = (4, 4, 4, 4), (2, 2, 2, 2)
    U = synth.gauge_field(L, 0.3, 1)
    ctx = mglma.Context(L, b, 0.12, 1.0)
    ctx.load_gauge(to_dev(U))
    tv = synth.gaussian_fields(3, L, 5)
    tv[2] = (1 - 2j) * tv[0]
    x = ctx.fine(3)
    ctx.import_fields(to_dev(tv), x)
    with pytest.raises(mglma.MglmaError) as e:
        ctx.build_subspace(x)
    assert e.value.code == -5
