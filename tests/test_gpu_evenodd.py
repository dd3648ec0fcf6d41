"""GPU parity of the even-odd reduced coarse operator (the paper's coarse
solves use the even-odd preconditioned coarse operator, sec. "Comparison of
the cost") against the oracle's dense Schur complement, and the coarse and
fine solves that run on it.

S = 1 - D_ee^{-1} D_eo D_oo^{-1} D_oe is applied by the library with the hop
blocks D_yy^{-1} D_y,dir in bfloat16 (FP32 accumulation).  Two references:
the exact S of the oracle (bound: the bfloat16 rounding of operator and
vector, a few 1e-3), and the same product with the oracle's blocks rounded to
bfloat16 the way the library stores them (FP64 -> FP32 -> bfloat16, round to
nearest even) and the inputs of each hop rounded likewise, which leaves only
FP32 accumulation order (bound 1e-4, norm-wise)."""
import numpy as np
import pytest

from oracle import coarse
from paper_2412_06347_amd import synth
from tests.gpu_util import to_dev, from_dev, relerr
from tests.gpu_setup import Pair

pytestmark = pytest.mark.gpu

CASES = [
    # L, block, Nv
    ((4, 4, 4, 4), (2, 2, 2, 2), 8),      # L1 = 2^4, nc = 16 (whole tiles)
    ((4, 4, 4, 8), (2, 2, 2, 4), 20),     # nc = 40 (ragged tile)
    ((8, 4, 4, 4), (2, 2, 2, 2), 3),      # L1 = (4, 2, 2, 2), nc = 6
]


@pytest.fixture(scope="module", params=CASES, ids=["nc16", "nc40", "L1_4222"])
def pair(request):
    L, b, Nv = request.param
    return Pair(L, b, Nv)


def _bf16(a):
    """FP64 -> FP32 -> bfloat16 (round to nearest even), back as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _cbf(z):
    return _bf16(z.real) + 1j * _bf16(z.imag)


def _emulated_schur(pair, x):
    """x: [n][Vh][nc] even-site vectors (FP32 values).  The library's S x with
    its bfloat16 roundings, every product in FP64."""
    D1, nbr, L1 = pair.D1, pair.nbr, pair.bl.L1
    e, o = coarse.parity_sites(L1)
    pos = np.empty(pair.bl.V1, dtype=np.int64)
    pos[e] = np.arange(len(e))
    pos[o] = np.arange(len(o))
    H = np.stack([[np.linalg.solve(D1[y, 0], D1[y, 1 + d]) for d in range(8)] for y in range(pair.bl.V1)])
    Hb = _cbf(H)

    def hop(sites, xin):
        xb = _cbf(xin)
        out = np.zeros((xin.shape[0], len(sites), xin.shape[2]), dtype=np.complex128)
        for k, y in enumerate(sites):
            for d in range(8):
                out[:, k] += xb[:, pos[nbr[y, 1 + d]]] @ Hb[y, d].T
        return out

    t = hop(o, x)
    t = t.real.astype(np.float32) + 1j * t.imag.astype(np.float32)
    return x - hop(e, t)


def test_schur_apply_parity(pair):
    import torch
    assert pair.ctx.has_eo
    V1, nc = pair.bl.V1, 2 * pair.Nv
    Vh = V1 // 2
    for nrhs in (1, 5, 17):
        x = synth.gaussian_coarse(nrhs, Vh, nc, 40 + nrhs)
        x = x.real.astype(np.float32) + 1j * x.imag.astype(np.float32)
        xd = to_dev(x).float()
        yd = torch.empty_like(xd)
        pair.ctx.coarse_schur_apply(xd, yd)
        torch.cuda.synchronize()
        y = from_dev(yd)
        S = coarse.schur_even(pair.D1, pair.nbr, pair.bl.L1)
        ref = (x.reshape(nrhs, -1) @ S.T).reshape(x.shape)
        emu = _emulated_schur(pair, x)
        e_exact, e_emu = relerr(y, ref), relerr(y, emu)
        print("nrhs %d: vs exact S %.2e, vs emulated bfloat16 %.2e" % (nrhs, e_exact, e_emu))
        assert e_emu < 1e-4
        assert e_exact < 2e-2
        # every right-hand side on its own (no mixing of the batch)
        for r in range(nrhs):
            assert relerr(y[r], emu[r]) < 1e-4


def test_schur_arguments(pair):
    import torch
    from paper_2412_06347_amd import mglma
    Vh, nc = pair.bl.V1 // 2, 2 * pair.Nv
    x = torch.zeros((2, Vh, nc, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(mglma.MglmaError) as ex:       # in place
        pair.ctx.coarse_schur_apply(x, x)
    assert ex.value.code == -1


def test_coarse_solve_even_odd(pair):
    """Coarse solves to 1e-11 through the reduced system and through D_1
    agree with the dense solution; the reduced system needs no more
    defect-correction rounds."""
    import torch
    from paper_2412_06347_amd import mglma
    A = coarse.coarse_dense(pair.D1, pair.nbr)
    v = synth.gaussian_coarse(3, pair.bl.V1, 2 * pair.Nv, 18)
    ref = np.linalg.solve(A, v.reshape(3, -1).T).T.reshape(v.shape)
    rounds = {}
    for eo in (1, 0):
        x = torch.empty((3, pair.bl.V1, 2 * pair.Nv, 2), dtype=torch.float64, device="cuda")
        p = mglma.default_params(tol=1e-11, coarse=mglma.BF16, coarse_iters=12, coarse_eo=eo)
        st = pair.ctx.coarse_solve(to_dev(v), x, p)
        assert relerr(from_dev(x), ref) < 1e-9
        assert max(s["true_rel_res"] for s in st) <= 1e-11
        rounds[eo] = st[0]["outer"]
    print("defect-correction rounds: even-odd %d, full %d" % (rounds[1], rounds[0]))
    assert rounds[1] <= rounds[0]


def test_coarse_solve_deflated(pair):
    """The even-odd coarse GCR deflated with the constant even-site vectors
    (coarse_eo = 2) solves to 1e-11, matches the dense solution and needs no
    more defect-correction rounds than the undeflated reduced system."""
    import torch
    from paper_2412_06347_amd import mglma
    A = coarse.coarse_dense(pair.D1, pair.nbr)
    v = synth.gaussian_coarse(3, pair.bl.V1, 2 * pair.Nv, 19)
    ref = np.linalg.solve(A, v.reshape(3, -1).T).T.reshape(v.shape)
    rounds = {}
    for eo in (2, 1):
        x = torch.empty((3, pair.bl.V1, 2 * pair.Nv, 2), dtype=torch.float64, device="cuda")
        p = mglma.default_params(tol=1e-11, coarse=mglma.BF16, coarse_iters=8, coarse_eo=eo)
        st = pair.ctx.coarse_solve(to_dev(v), x, p)
        assert relerr(from_dev(x), ref) < 1e-9
        assert max(s["true_rel_res"] for s in st) <= 1e-11
        rounds[eo] = st[0]["outer"]
    print("defect-correction rounds: deflated %d, even-odd %d" % (rounds[2], rounds[1]))
    assert rounds[2] <= rounds[1]
    # and as the coarse solve of the preconditioner
    b = synth.gaussian_fields(2, pair.L, 24)
    xd = pair.ctx.fine(2)
    p = mglma.default_params(tol=1e-10, inner=mglma.F32, coarse=mglma.BF16, coarse_iters=4, coarse_eo=2)
    pair.ctx.solve(pair.fine_dev(b), xd, p)
    x = pair.fine_host(xd)
    r = pair.canon(pair.D.M(pair.lat(x))) - b
    assert (np.linalg.norm(r.reshape(2, -1), axis=1) / np.linalg.norm(b.reshape(2, -1), axis=1)).max() <= 1e-10


def test_fine_solve_even_odd(pair):
    """The MG-preconditioned fine solve with the even-odd coarse GCR reaches
    1e-10 in the oracle's FP64 residual, in no more inner iterations than
    with the coarse GCR on D_1 at the same number of coarse steps."""
    import torch
    from paper_2412_06347_amd import mglma
    b = synth.gaussian_fields(2, pair.L, 23)
    inner = {}
    for eo in (1, 0):
        xd = pair.ctx.fine(2)
        p = mglma.default_params(tol=1e-10, inner=mglma.F32, coarse=mglma.BF16, coarse_iters=8, coarse_eo=eo)
        rc, st = pair.ctx.solve(pair.fine_dev(b), xd, p)
        x = pair.fine_host(xd)
        r = pair.canon(pair.D.M(pair.lat(x))) - b
        res = np.linalg.norm(r.reshape(2, -1), axis=1) / np.linalg.norm(b.reshape(2, -1), axis=1)
        assert res.max() <= 1e-10
        inner[eo] = sum(s["inner"] for s in st)
    print("inner iterations: even-odd %d, full %d" % (inner[1], inner[0]))
    assert inner[1] <= inner[0]


def test_odd_coarse_extent_falls_back():
    """A coarse extent of 3: no even-odd form (query 8 = 0, the Schur apply
    reports SHAPE) and solves asking for it run the GCR on D_1."""
    import torch
    from paper_2412_06347_amd import mglma
    pair = Pair((6, 4, 4, 4), (2, 2, 2, 2), 3)
    assert not pair.ctx.has_eo
    Vh, nc = 24, 6
    x = torch.zeros((1, Vh, nc, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(mglma.MglmaError) as ex:
        pair.ctx.coarse_schur_apply(x, torch.empty_like(x))
    assert ex.value.code == -2
    A = coarse.coarse_dense(pair.D1, pair.nbr)
    v = synth.gaussian_coarse(1, pair.bl.V1, nc, 5)
    ref = np.linalg.solve(A, v.reshape(1, -1).T).T.reshape(v.shape)
    xc = torch.empty((1, pair.bl.V1, nc, 2), dtype=torch.float64, device="cuda")
    pair.ctx.coarse_solve(to_dev(v), xc, mglma.default_params(tol=1e-11, coarse=mglma.BF16, coarse_eo=1))
    assert relerr(from_dev(xc), ref) < 1e-9
