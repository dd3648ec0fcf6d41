"""Edge cases at the C ABI: empty batches are no-ops that leave the outputs
untouched, solves reject them, and batch sizes above the documented maxima
are rejected before any launch."""
import ctypes as C
import numpy as np
import pytest

from tests.gpu_setup import Pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pair():
    p = Pair((4, 4, 4, 8), (2, 2, 2, 2), 3)
    p.ctx.build_level2((4, 4, 4, 4))
    return p


def _p(t):
    return C.c_void_p(t.data_ptr())


def test_empty_batches_are_noops(pair):
    import torch
    from paper_2412_06347_amd import mglma
    L = mglma.lib()
    ctx = pair.ctx
    h = ctx._ctx
    fin = torch.full((1, 12, ctx.V, 2), 7.0, dtype=torch.float64, device="cuda")
    fout = torch.full_like(fin, 3.0)
    cin = torch.full((1, ctx.V1, ctx.nc, 2), 5.0, dtype=torch.float64, device="cuda")
    cout = torch.full_like(cin, 2.0)
    c2 = torch.full((1, ctx.V2, ctx.nc, 2), 4.0, dtype=torch.float64, device="cuda")
    calls = [
        ("apply_D", lambda: L.mglma_apply_D(h, 0, 0, _p(fin), _p(fout), 0)),
        ("restrict", lambda: L.mglma_restrict(h, 0, _p(fin), _p(cout), 0)),
        ("prolong", lambda: L.mglma_prolong(h, 0, _p(cin), _p(fout), 0)),
        ("coarse_apply", lambda: L.mglma_coarse_apply(h, 0, 0, _p(cin), _p(cout), 0)),
        ("level2_restrict", lambda: L.mglma_level2_restrict(h, 0, _p(cin), _p(c2), 0)),
        ("level2_prolong", lambda: L.mglma_level2_prolong(h, 0, _p(c2), _p(cout), 0)),
        ("level2_apply", lambda: L.mglma_level2_apply(h, 0, 0, _p(c2), _p(cout), 0)),
    ]
    for name, f in calls:
        assert f() == 0, name
    torch.cuda.synchronize()
    assert float(fout.min()) == 3.0 and float(fout.max()) == 3.0
    assert float(cout.min()) == 2.0 and float(cout.max()) == 2.0
    assert float(c2.min()) == 4.0 and float(c2.max()) == 4.0


def test_solves_reject_empty_and_oversized(pair):
    import torch
    from paper_2412_06347_amd import mglma
    L = mglma.lib()
    h = pair.ctx._ctx
    x = torch.zeros((1, 12, pair.ctx.V, 2), dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    p = mglma.default_params()
    assert L.mglma_solve(h, C.byref(p), _p(x), _p(y), 0, None) == -1
    assert L.mglma_coarse_solve(h, C.byref(p), _p(x), _p(y), 0, None) == -1
    assert L.mglma_level2_solve(h, C.byref(p), _p(x), _p(y), 0, None) == -1
    # above the documented batch maxima: refused before any launch
    assert L.mglma_apply_D(h, 0, 0, _p(x), _p(y), 65536) == -1
    assert L.mglma_solve(h, C.byref(p), _p(x), _p(y), 4097, None) == -1
    assert L.mglma_coarse_schur_apply(h, _p(x), _p(y), 0) == -1
