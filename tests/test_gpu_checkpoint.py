"""Checkpoint of the subspace and top level through the C ABI: a context that
loads the file reproduces the saving context's basis, D_1, coarse gammas and
solves bit for bit, its top level to rounding; mismatched or truncated files
are refused."""
import os
import numpy as np
import pytest

from paper_2412_06347_amd import synth
from tests.gpu_util import to_dev, from_dev, relerr
from tests.gpu_setup import Pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pair():
    return Pair((8, 4, 4, 8), (4, 2, 2, 4), 6, kappa=0.124, Nlm=2)


def _ctx(pair, kappa=None):
    import torch
    from paper_2412_06347_amd import mglma
    ctx = mglma.Context(pair.L, pair.b, pair.kappa if kappa is None else kappa, 1.0)
    ctx.load_gauge(to_dev(pair.U))
    torch.cuda.synchronize()
    return ctx


def _exports(ctx, pair):
    import torch
    V1, nc, Nv = pair.bl.V1, 2 * pair.Nv, pair.Nv
    op = torch.empty((V1, 9, nc, nc, 2), dtype=torch.float64, device="cuda")
    ctx.export_coarse_op(op)
    gam = torch.empty((V1, pair.bl.b[0], 3, Nv, Nv, 2), dtype=torch.float64, device="cuda")
    ctx.export_coarse_gammas(gam)
    return op.cpu().numpy(), gam.cpu().numpy()


def test_save_load_roundtrip(pair, tmp_path):
    from paper_2412_06347_amd import mglma
    path = tmp_path / "subspace.ckpt"
    pair.ctx.save(path)
    ctx2 = _ctx(pair)
    ctx2.load(path)
    assert ctx2.nc == pair.ctx.nc and ctx2.query(5) == pair.ctx.query(5)
    a_op, a_gam = _exports(pair.ctx, pair)
    b_op, b_gam = _exports(ctx2, pair)
    assert np.array_equal(a_op, b_op) and np.array_equal(a_gam, b_gam)
    assert relerr(ctx2.contract_top(), pair.ctx.contract_top()) < 1e-12
    b = synth.gaussian_fields(2, pair.L, 91)
    p = mglma.default_params(tol=1e-10, inner=mglma.F32, coarse=mglma.BF16)
    xs = []
    for ctx in (pair.ctx, ctx2):
        bd = ctx.fine(2)
        ctx.import_fields(to_dev(b), bd)
        xd = ctx.fine(2)
        ctx.solve(bd, xd, p)
        xs.append(xd.cpu().numpy())
    assert np.array_equal(xs[0], xs[1])


def test_load_errors(pair, tmp_path):
    from paper_2412_06347_amd import mglma
    path = tmp_path / "s.ckpt"
    pair.ctx.save(path)
    other = _ctx(pair, kappa=0.121)              # different kappa
    with pytest.raises(mglma.MglmaError) as e:
        other.load(path)
    assert e.value.code == -2
    short = tmp_path / "short.ckpt"
    short.write_bytes(path.read_bytes()[:200000])
    ctx = _ctx(pair)
    with pytest.raises(mglma.MglmaError) as e:
        ctx.load(short)
    assert e.value.code == -2
    with pytest.raises(mglma.MglmaError) as e:
        ctx.load(tmp_path / "missing.ckpt")
    assert e.value.code == -1
    fresh = _ctx(pair)
    with pytest.raises(mglma.MglmaError) as e:   # nothing to save
        fresh.save(tmp_path / "none.ckpt")
    assert e.value.code == -7
