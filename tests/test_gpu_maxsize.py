"""The largest configuration's lattice on one GPU: 48^3 x 96 (V = 10,616,832
sites), 4^4 blocks.  The oracle cannot build the clover term of a lattice
this size in test time, so the gauge field is the seeded 48 x 24^3 field of
the benchmark tiled twice in every direction, with periodic fermion phases
in every direction (antiperiodic time would make a field tiled twice in
time periodic, not antiperiodic, over the large extent).  The operator then
commutes with translations by one tile and maps tiled fields to tiled
fields, which makes every full-size result checkable on one tile with the
oracle:

* the FP64 apply of a tiled field against the oracle's apply on one tile;
* the block basis of N_v = 32 tiled Gaussian test vectors (the stated
  N_v of this configuration, n_c = 64) on sampled blocks against the
  oracle's Gram-Schmidt, and (gamma5 gamma_k)_1 of those blocks against the
  oracle's coarse gammas;
* the mixed-precision MG solve (the benchmark's solver settings) of tiled
  right-hand sides: every tile of the solution equal, and one tile solving
  the small system to 1e-10 under the oracle's operator (the residual of a
  tiled field is the tiled residual);
* the stochastic estimator of this configuration for one time-diluted,
  spin-diluted source: N_lm = 64 top modes (r = 128), the four solves, the
  coarse pieces, the level terms with the exact top row, consistency of the
  level rows with the source's full correlator, and the Galerkin identity
  D_1 v = R M T v in FP64.
"""
import numpy as np
import pytest

from oracle import dirac
from paper_2412_06347_amd import synth
from tests.gpu_util import to_dev, from_dev, relerr

pytestmark = pytest.mark.gpu

LS = (48, 24, 24, 24)
LB = (96, 48, 48, 48)
B = (4, 4, 4, 4)
EPS, KAPPA, CSW, SEED = 0.25, 0.125, 1.0, 3
NV = 32
NLM = 64
BC = (1.0, 1.0, 1.0, 1.0)


def _tile(f, L):
    """[n][V_small][...] canonical fields -> the same fields tiled 2x in every direction."""
    n, rest = f.shape[0], f.shape[2:]
    g = f.reshape(n, *L, *rest)
    g = np.tile(g, (1, 2, 2, 2, 2) + (1,) * len(rest))
    return g.reshape(n, -1, *rest)


def _tiles(f):
    """[n][V_big][4][3] -> [16][n][V_small][4][3], the 16 tiles in order."""
    n = f.shape[0]
    g = f.reshape(n, 2, LS[0], 2, LS[1], 2, LS[2], 2, LS[3], 4, 3)
    g = g.transpose(1, 3, 5, 7, 0, 2, 4, 6, 8, 9, 10)
    return g.reshape(16, n, -1, 4, 3)


@pytest.fixture(scope="module")
def big():
    import torch
    from paper_2412_06347_amd import mglma
    Us = synth.gauge_field(LS, EPS, SEED)
    D = dirac.WilsonClover(Us, LS, KAPPA, CSW, bc=BC)
    ctx = mglma.Context(LB, B, KAPPA, CSW, bc=BC)
    Ud = to_dev(_tile(Us[None], LS)[0])
    ctx.load_gauge(Ud)
    del Ud
    torch.cuda.synchronize()
    return ctx, D


def _export(ctx, dev):
    import torch
    out = torch.empty((dev.shape[0], ctx.V, 4, 3, 2), dtype=torch.float64, device="cuda")
    ctx.export_fields(dev, out)
    h = from_dev(out)
    del out
    return h


def test_maxsize_apply(big):
    ctx, D = big
    assert ctx.V == int(np.prod(LB))
    ps = synth.gaussian_fields(2, LS, 301)
    x = ctx.fine(2)
    ctx.import_fields(to_dev(_tile(ps, LS)), x)
    y = ctx.fine(2)
    ctx.apply_D(x, y)
    got = _tiles(_export(ctx, y))
    del x, y
    ref = dirac.fields_to_canonical(D.M(dirac.fields_to_lattice(ps, LS)))
    e = max(relerr(got[k], ref) for k in range(16))
    print("48^3x96 FP64 apply, largest tile error vs oracle: %.2e" % e)
    assert e < 1e-12


def test_maxsize_mg_solve(big):
    import torch
    import bench
    from paper_2412_06347_amd import mglma
    ctx, D = big
    tvs = synth.gaussian_fields(NV, LS, 400)
    tv = ctx.fine(NV)
    for c in range(NV):
        ctx.import_fields(to_dev(_tile(tvs[c:c + 1], LS)), tv[c:c + 1])
    ctx.build_subspace(tv)
    del tv
    torch.cuda.empty_cache()
    assert ctx.V1 == int(np.prod(LB)) // 256 and ctx.nc == 2 * NV
    # sampled blocks: basis and coarse gammas against the oracle (block y of
    # the large lattice holds the test vectors of block y mod tile)
    import types
    from oracle import coarse as ocoarse, subspace as osub
    L1b = [LB[m] // B[m] for m in range(4)]
    ys = np.random.default_rng(303).choice(ctx.V1, 8, replace=False)
    yc = np.array(np.unravel_index(ys, L1b)).T
    tl = tvs.reshape(NV, *LS, 4, 3)
    tb = np.stack([tl[:, (y[0] * B[0]) % LS[0]:(y[0] * B[0]) % LS[0] + B[0],
                      (y[1] * B[1]) % LS[1]:(y[1] * B[1]) % LS[1] + B[1],
                      (y[2] * B[2]) % LS[2]:(y[2] * B[2]) % LS[2] + B[2],
                      (y[3] * B[3]) % LS[3]:(y[3] * B[3]) % LS[3] + B[3]] for y in yc])
    del tl
    Vb = int(np.prod(B))
    phi = np.empty((len(ys), 2, NV, *B, 2, 3), dtype=np.complex128)
    ref_b = []
    for a in range(2):
        q = osub.gram_schmidt(tb[..., 2 * a:2 * a + 2, :].reshape(len(ys), NV, -1))
        phi[:, a] = q.reshape(len(ys), NV, *B, 2, 3)
        ref_b.append(q.reshape(len(ys), NV, Vb, 2, 3))
    # the exported basis would take 130 GB at this size: probe it instead.
    # The restriction of the oracle's basis vector j of block y, placed on
    # block y, is e_j on y exactly when the library's block basis equals the
    # oracle's (both orthonormal).  Eight basis indices per pass, all sampled
    # blocks in the same fields (the blocks are disjoint).
    lo = np.array(np.unravel_index(np.arange(Vb), B)).T                 # local coordinates
    sites = np.stack([np.ravel_multi_index(((y * np.array(B))[:, None] + lo.T), LB) for y in yc])
    sites_d = torch.as_tensor(sites.reshape(-1), device="cuda")
    ys_d = torch.as_tensor(ys, device="cuda")
    err_b = 0.0
    for j0 in range(0, 2 * NV, 8):
        canon = torch.zeros((8, ctx.V, 4, 3, 2), dtype=torch.float64, device="cuda")
        for q in range(8):
            a, c = divmod(j0 + q, NV)
            vals = np.zeros((len(ys), Vb, 4, 3), dtype=np.complex128)
            vals[:, :, 2 * a:2 * a + 2, :] = ref_b[a][:, c]
            canon[q, sites_d] = to_dev(vals.reshape(-1, 4, 3))
        f = ctx.fine(8)
        ctx.import_fields(canon, f)
        del canon
        rc_ = ctx.coarse(8)
        ctx.restrict(f, rc_)
        del f
        got = from_dev(rc_[:, ys_d])                                      # [8][ns][nc]
        want = np.zeros_like(got)
        for q in range(8):
            want[q, :, j0 + q] = 1.0
        err_b = max(err_b, float(np.abs(got - want).max()))
    print("48^3x96, Nv = 32: sampled block bases vs oracle (probe) %.2e" % err_b)
    assert err_b < 1e-12
    sub = types.SimpleNamespace(bl=types.SimpleNamespace(V1=len(ys), b=B), phi=phi, Nv=NV, nc=2 * NV)
    G1o = ocoarse.coarse_gammas(sub)[..., :NV, NV:]
    gd = torch.empty((ctx.V1, B[0], 3, NV, NV, 2), dtype=torch.float64, device="cuda")
    ctx.export_coarse_gammas(gd)
    G1h = from_dev(gd[torch.as_tensor(ys, device="cuda")])
    del gd
    e_g = np.abs(G1h - G1o).max() / np.abs(G1o).max()
    print("48^3x96, Nv = 32: sampled basis and coarse gammas vs oracle, gammas %.2e" % e_g)
    assert e_g < 1e-12
    # the probe's fields stay in torch's cache unless handed back; the
    # library allocates its solver workspaces with hipMalloc
    torch.cuda.empty_cache()
    bs = synth.gaussian_fields(2, LS, 302)
    b = ctx.fine(2)
    ctx.import_fields(to_dev(_tile(bs, LS)), b)
    x = ctx.fine(2)
    rc, st = ctx.solve(b, x, bench.mixed_params(mglma, max_inner=400))
    print("48^3x96 MG solve: %d iterations, true rel res %s" % (st[0]["inner"], [s["true_rel_res"] for s in st]))
    assert rc == 0 and max(s["true_rel_res"] for s in st) <= 1e-10
    tiles = _tiles(_export(ctx, x))
    del b, x
    spread = max(relerr(tiles[k], tiles[0]) for k in range(1, 16))
    print("largest difference between tiles of the solution: %.2e" % spread)
    assert spread < 1e-12
    r = bs - dirac.fields_to_canonical(D.M(dirac.fields_to_lattice(tiles[0], LS)))
    res = (np.linalg.norm(r.reshape(2, -1), axis=1) / np.linalg.norm(bs.reshape(2, -1), axis=1)).max()
    print("one tile under the oracle's operator: relative residual %.2e" % res)
    assert res <= 1.05e-10


def test_maxsize_stochastic_levels(big):
    """One time-diluted source of the stochastic estimator at this size, with
    the stated top level (N_lm = 64 seeded coarse modes, r = 128)."""
    import time
    import torch
    import bench
    from paper_2412_06347_amd import mglma
    ctx, D = big
    assert ctx.nc == 2 * NV            # the subspace of the previous test
    # this lattice fills most of the device: hand back torch's cached blocks
    # and the previous solve's workspaces before the top level and the solves
    torch.cuda.empty_cache()
    ctx.release_workspace()
    t0 = time.time()
    modes = to_dev(synth.gaussian_coarse(NLM, ctx.V1, ctx.nc, 304))
    ctx.set_top_modes(modes)
    del modes
    torch.cuda.synchronize()
    t_top = time.time() - t0
    assert ctx.r == 2 * NLM
    L3 = LB[1] * LB[2] * LB[3]
    xi = to_dev(synth.z4_noise(1, LB, 305))
    tn = synth.time_slices(1, LB[0], 306)
    eta = ctx.fine(4)
    ctx.noise_sources(xi, tn, eta)
    x = ctx.fine(4)
    free, total = torch.cuda.mem_get_info()
    print("48^3x96 before the solves: %.1f of %.1f GB free, library resident %.1f GB"
          % (free / 1e9, total / 1e9, ctx.resident_bytes() / 1e9), flush=True)
    t0 = time.time()
    rc, st = ctx.solve(eta, x, bench.mixed_params(mglma, max_inner=400))
    torch.cuda.synchronize()
    t_solve = time.time() - t0
    assert rc == 0 and max(s["true_rel_res"] for s in st) <= 1e-10
    cg, ct = ctx.coarse(4), ctx.coarse(4)
    cp = mglma.default_params(tol=1e-10, coarse=mglma.BF16, coarse_iters=12, max_outer=40, coarse_eo=1)
    ctx.coarse_pieces(eta, cg, ct, cp)
    t0 = time.time()
    lv = ctx.contract_levels(mglma.SRC_STOCH, tn, fine=x, coarse=[cg, ct], exact_top=True)
    t_con = time.time() - t0
    print("48^3x96 one source: top level %.2f s, 4 solves %.2f s (%d iterations, res %.2e), levels %.3f s" %
          (t_top, t_solve, st[0]["inner"], max(s["true_rel_res"] for s in st), t_con))
    assert lv.shape == (4, LB[0]) and np.all(np.isfinite(lv))
    full = ctx.contract_pair(mglma.SRC_STOCH, tn, x, x)
    assert relerr(lv[0] + lv[1] + lv[2], full) < 1e-12
    assert relerr(lv[3], ctx.contract_top()) < 1e-14
    # the coarse piece solves D_1 g = R eta (FP64 stencil apply) and the
    # Galerkin identity D_1 v = R M T v holds at this size
    re_ = ctx.coarse(4)
    ctx.restrict(eta, re_)
    dg = ctx.coarse(4)
    ctx.coarse_apply(cg, dg)
    assert relerr(from_dev(dg), from_dev(re_)) <= 1.05e-10
    v = to_dev(synth.gaussian_coarse(1, ctx.V1, ctx.nc, 307))
    y1 = torch.empty_like(v)
    ctx.coarse_apply(v, y1)
    f = ctx.fine(1)
    ctx.prolong(v, f)
    g2 = ctx.fine(1)
    ctx.apply_D(f, g2)
    y2 = torch.empty_like(v)
    ctx.restrict(g2, y2)
    assert relerr(from_dev(y1), from_dev(y2)) < 1e-12
