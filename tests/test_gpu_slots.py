"""Resident right-hand-side slots (mglma_slots_*): right-hand sides that join
a running solve between outer cycles and leave as they converge follow the
arithmetic of mglma_solve alone."""
import numpy as np
import pytest

from paper_2412_06347_amd import synth
from tests.gpu_util import to_dev, relerr

pytestmark = pytest.mark.gpu

WL = dict(L=(8, 8, 8, 8), block=(4, 4, 4, 4), eps=0.3, kappa=0.124, csw=1.0, Nv=6, seed=11)


@pytest.fixture(scope="module")
def ens():
    import torch
    from paper_2412_06347_amd import mglma
    L = WL["L"]
    ctx = mglma.Context(L, WL["block"], WL["kappa"], WL["csw"])
    ctx.load_gauge(to_dev(synth.gauge_field(L, WL["eps"], WL["seed"])))
    tv = ctx.fine(WL["Nv"])
    ctx.import_fields(to_dev(synth.gaussian_fields(WL["Nv"], L, 1011)), tv)
    ctx.build_subspace(tv)
    src = ctx.fine(16)
    ctx.import_fields(to_dev(synth.gaussian_fields(16, L, 1012)), src)
    # the serving settings: SAP smoothing, FGCR(6), one restart cycle per outer cycle
    p = mglma.default_params(tol=1e-10, max_outer=30, max_inner=6, gcr_m=6, inner_tol=1e-5, nu_post=2, sap_mr=4,
                             coarse_iters=4, smoother=mglma.F16, inner=mglma.F32, coarse=mglma.BF16, use_mg=1,
                             smoother_alg=mglma.SMOOTH_SAP, coarse_eo=1)
    torch.cuda.synchronize()
    return ctx, src, p


def alone(ctx, src, p, k):
    x = ctx.fine(1)
    rc, st = ctx.solve(src[k:k + 1].contiguous(), x, p)
    return x, st[0]


def test_slots_equal_solve(ens):
    import torch
    from paper_2412_06347_amd import mglma
    ctx, src, p = ens
    pool = mglma.Slots(ctx, 8)
    ids = pool.load(src[:5].contiguous())
    steps = 0
    while True:
        st = pool.step(p)
        steps += 1
        if all(st[i] != 1 for i in ids):
            break
        assert steps < p.max_outer
    x = ctx.fine(5)
    stats = pool.take(ids, x)
    assert all(s["status"] == 0 and s["true_rel_res"] <= 1e-10 for s in stats)
    for k in range(5):
        xa, sa = alone(ctx, src, p, k)
        d = float((x[k] - xa[0]).abs().max())
        print("rhs %d: outer %d vs %d, max |x_slots - x_alone| = %.2e" % (k, stats[k]["outer"], sa["outer"], d))
        assert stats[k]["outer"] == sa["outer"]
        assert d <= 1e-13 * float(xa.abs().max())
    pool.close()


def test_slots_join_and_leave(ens):
    """Four right-hand sides start; after one outer cycle four more join;
    finished ones are taken while others still run and new ones load into the
    freed slots.  Every result equals its solve alone."""
    import torch
    from paper_2412_06347_amd import mglma
    ctx, src, p = ens
    pool = mglma.Slots(ctx, 8)
    slot_of = {}
    pending = list(range(16))
    started_while_running = 0
    ids = pool.load(src[0:4].contiguous())
    slot_of.update({int(i): k for i, k in zip(ids, range(0, 4))})
    pending = pending[4:]
    st = pool.step(p)
    results = {}
    for _ in range(200):
        running = [i for i, k in slot_of.items() if st[i] == 1]
        free = pool.nslots - len(slot_of)
        if pending and free > 0:
            n = min(free, 3, len(pending))
            if running:
                started_while_running += n
            ks = pending[:n]
            pending = pending[n:]
            ids = pool.load(src[ks[0]:ks[0] + n].contiguous())
            slot_of.update({int(i): k for i, k in zip(ids, ks)})
        st = pool.step(p)
        done = [i for i in slot_of if st[i] not in (0, 1)]
        if done:
            x = ctx.fine(len(done))
            stt = pool.take(done, x)
            for j, i in enumerate(done):
                assert stt[j]["status"] == 0
                results[slot_of.pop(i)] = x[j].clone()
        if not pending and not slot_of:
            break
    assert len(results) == 16 and started_while_running > 0
    for k in range(16):
        xa, _ = alone(ctx, src, p, k)
        assert float((results[k] - xa[0]).abs().max()) <= 1e-13 * float(xa.abs().max()), k
    pool.close()


def test_slots_errors(ens):
    from paper_2412_06347_amd import mglma
    ctx, src, p = ens
    pool = mglma.Slots(ctx, 2)
    with pytest.raises(mglma.MglmaError):
        pool.load(src[:3].contiguous())           # more than the free slots
    ids = pool.load(src[:1].contiguous())
    with pytest.raises(mglma.MglmaError):
        pool.take(ids, ctx.fine(1))               # still running
    z = ctx.fine(1)
    z.zero_()
    idz = pool.load(z)                            # a zero source is finished at once
    x = ctx.fine(1)
    st = pool.take(idz, x)
    assert st[0]["status"] == 0 and float(x.abs().max()) == 0.0
    pool.close()
