#!/usr/bin/env python3
"""Benchmark of the MG low-mode-averaging hot path on one MI355X.

One step = one pass of the whole hot path over one synthetic gauge field:
clover build, block basis (Gram-Schmidt), Galerkin coarse operator, coarse
gammas, exact top level, 12 point sources, the 12 mixed-precision MG solves
to a true FP64 relative residual of 1e-10, the coarse-level pieces
D_1^{-1} R eta and W D_2^{-1} W^+ R eta, and the contractions (fine point
correlator, coarse-route correlators, exact top term, level sums).

Prints ONE JSON line (rank 0).  Only N = 1 GPU is supported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

WORKLOADS = {
    # 24^3 x 48, eps = 0.25, kappa = 0.125, c_sw = 1, 12 point-source RHS batched,
    # 4^4 blocks, Nv = 24 test vectors, Nlm = 16 top modes
    "24c48": dict(L=(48, 24, 24, 24), block=(4, 4, 4, 4), eps=0.25, kappa=0.125, csw=1.0, Nv=24, Nlm=16,
                  seed=3),
    # 16^3 x 32, eps = 0.3, kappa = 0.124
    "16c32": dict(L=(32, 16, 16, 16), block=(4, 4, 4, 4), eps=0.3, kappa=0.124, csw=1.0, Nv=24, Nlm=16, seed=2),
    # 48^3 x 96, eps = 0.25, kappa = 0.125, 4^4 blocks, Nv = 32, Nlm = 64, 48 time-diluted
    # spin-diluted sources (192 right-hand sides); run by --c4
    "48c96": dict(L=(96, 48, 48, 48), block=(4, 4, 4, 4), eps=0.25, kappa=0.125, csw=1.0, Nv=32, Nlm=64, seed=4,
                  nsrc=48),
    # 32^3 x 64, eps = 0.25, kappa = 0.125, the third volume of the wider serving mix
    "32c64": dict(L=(64, 32, 32, 32), block=(4, 4, 4, 4), eps=0.25, kappa=0.125, csw=1.0, Nv=24, Nlm=16, seed=6),
    # 4^4, eps = 0.3, kappa = 0.120, 2^4 blocks
    "4c4": dict(L=(4, 4, 4, 4), block=(2, 2, 2, 2), eps=0.3, kappa=0.120, csw=1.0, Nv=8, Nlm=4, seed=1),
}

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def mixed_params(mglma, **kw):
    p = dict(tol=1e-10, max_outer=10, max_inner=120, gcr_m=6, inner_tol=1e-5, nu_post=2, sap_mr=4,
             coarse_iters=4, smoother=mglma.F16, inner=mglma.F32, coarse=mglma.BF16, use_mg=1,
             smoother_alg=mglma.SMOOTH_SAP, coarse_eo=1)
    p.update(kw)
    return mglma.default_params(**p)


def fp64_params(mglma, **kw):
    p = dict(tol=1e-10, max_outer=3, max_inner=400, gcr_m=8, inner_tol=1e-11, nu_post=6, coarse_iters=16,
             smoother=mglma.F64, inner=mglma.F64, coarse=mglma.F64, use_mg=1)
    p.update(kw)
    return mglma.default_params(**p)


class Pipeline:
    """Resident inputs and the step of the hot path."""

    def __init__(self, wl, log_setup=True):
        import torch
        from paper_2412_06347_amd import mglma, synth
        self.torch, self.mglma, self.synth = torch, mglma, synth
        self.wl = wl
        L = wl["L"]
        t0 = time.time()
        U = synth.gauge_field(L, wl["eps"], wl["seed"])
        self.U = torch.from_numpy(U.view(np.float64)).cuda()
        del U
        self.ctx = mglma.Context(L, wl["block"], wl["kappa"], wl["csw"])
        ctx = self.ctx
        ctx.load_gauge(self.U)
        # test vectors: Gaussian fields improved by three rounds of approximate
        # inverse iteration (40 unpreconditioned FP32 GCR steps each) -- an
        # input to the hot path, prepared outside the timed region
        tv = synth.gaussian_fields(wl["Nv"], L, wl["seed"] + 1000)
        x = ctx.fine(wl["Nv"])
        ctx.import_fields(torch.from_numpy(tv.view(np.float64)).cuda(), x)
        del tv
        y = ctx.fine(wl["Nv"])
        p = mglma.default_params(use_mg=0, inner=mglma.F32, max_outer=1, max_inner=40, gcr_m=16, tol=1e-30,
                                 inner_tol=1e-30)
        for _ in range(3):
            ctx.solve(x, y, p, raise_on_error=False)
            nrm = torch.linalg.vector_norm(y.reshape(wl["Nv"], -1), dim=1)
            x = (y / nrm[:, None, None, None]).contiguous()
        self.tv = x
        del y
        # top modes: the Nlm lowest eigenvectors of Q_1 from the device eigensolver
        # (residual <= 1e-12), started from a seeded Gaussian block of 2 Nlm vectors
        ctx.build_subspace(self.tv)
        nc, V1 = ctx.nc, ctx.V1
        init = torch.from_numpy(synth.gaussian_coarse(2 * wl["Nlm"], V1, nc, 4242).view(np.float64)).cuda()
        rc, lam, m, st = ctx.coarse_eigs(init, wl["Nlm"], tol=1e-12)
        self.eig = dict(nev=wl["Nlm"], nblk=2 * wl["Nlm"], seconds=round(st["seconds"], 3), iters=st["iters"],
                        applies=st["applies"], max_res=st["max_res"],
                        lambda_min_abs=float(np.abs(lam).min()), lambda_max_abs=float(np.abs(lam).max()))
        self.modes = m.contiguous()
        self.src = ctx.fine(12)
        self.x = ctx.fine(12)
        self.cg = ctx.coarse(12)
        self.ct = ctx.coarse(12)
        torch.cuda.synchronize()
        if log_setup:
            log("setup %.1f s (V=%d, V1=%d, nc=%d, resident %.2f GB)" % (time.time() - t0, ctx.V, V1, nc,
                                                                         ctx.resident_bytes() / 1e9))

    def step(self, params):
        ctx, mglma = self.ctx, self.mglma
        ctx.load_gauge(self.U)                         # clover term
        ctx.build_subspace(self.tv)                    # basis, Galerkin D_1, coarse gammas
        ctx.set_top_modes(self.modes)                  # W, D_2, (gamma5 gamma_k)_2
        ctx.point_sources((0, 0, 0, 0), self.src)      # 12 point sources
        rc, stats = ctx.solve(self.src, self.x, params)
        cp = mglma.default_params(tol=1e-10, coarse=mglma.BF16, coarse_iters=12, max_outer=40, coarse_eo=1)
        ctx.coarse_pieces(self.src, self.cg, self.ct, cp)
        # level terms in the library: G(S) - G(S_>=1), G(S_>=1) - G(S_2), the
        # point estimate G(S_2) and eq:G_LL:exact
        lv = ctx.contract_levels(mglma.SRC_POINT, [0], fine=self.x, coarse=[self.cg, self.ct], exact_top=True)
        levels = dict(L0=lv[0], L1=lv[1], L2pt=lv[2], L2exact=lv[3])
        return stats, levels


def dslash_alg_bytes(V, nrhs, b):
    """Algorithmic HBM bytes of one Wilson-clover apply on nrhs right-hand
    sides with b-byte reals: per site the four links (4 x 18 reals) and the
    clover term (2 x 36 reals) once, and per right-hand side one spinor read
    and one written (2 x 24 reals)."""
    return V * (144 + 48 * nrhs) * b


def measured_traffic(workload):
    """HBM bytes per launch of the FP16 12-RHS apply from the committed
    hardware-counter summary, or None when the kernel source has changed
    since the counters were taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "dslash_traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    csrc = os.path.join(here, "paper_2412_06347_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read() for f in ("dslash.hip", "wilson.h", "wilson_h.h"))
    if hashlib.sha256(src).hexdigest() != rec.get("dslash_source_sha256"):
        return None
    return rec.get("f16_12rhs_hbm_bytes_per_launch")


# MI355X published dense FP32 vector peak (it counts packed FP32 issue)
FP32_PEAK_TFLOPS = 157.3
# the FP32 rate without packed FP32 instructions, which the library is built
# without: 256 CUs x 64 FP32 FMA lanes x 2 flop x 2.4 GHz
FP32_NONPACKED_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12

# flops per site and right-hand side: one Wilson-clover apply 1824 (clover
# 504, each of the 8 hops 165), the minimal-residual vector work of one SAP
# block step 336 (<t,s>, <t,t>, d += omega s, s -= omega t), the residual
# subtraction 24
HOP_FLOPS, CLOVER_FLOPS, MR_VEC_FLOPS, RESID_FLOPS = 165, 504, 336, 24


def sap_alg_flops(V, block, L, nrhs, nmr):
    """Algorithmic flops of one SAP half-sweep launch (the blocks of one
    colour: V/2 sites): per site and right-hand side the residual
    r - M z (a full apply) and nmr block steps (the block operator keeps the
    hops that stay inside the block: 2 (b_mu - 1) / b_mu per direction on
    average, 2 when the block spans the extent)."""
    hops = sum(2.0 if L[mu] == block[mu] else 2.0 * (block[mu] - 1) / block[mu] for mu in range(4))
    per_site = (8 * HOP_FLOPS + CLOVER_FLOPS + RESID_FLOPS
                + nmr * (hops * HOP_FLOPS + CLOVER_FLOPS + MR_VEC_FLOPS))
    return V / 2 * nrhs * per_site


def measured_sap_traffic(workload):
    """HBM bytes per SAP half-sweep launch (FP16 links, 12 RHS) from the
    committed hardware-counter summary, or None when the kernel source has
    changed since the counters were taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "sap_traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    csrc = os.path.join(here, "paper_2412_06347_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read() for f in ("sap.hip", "wilson.h", "wilson_h.h"))
    if hashlib.sha256(src).hexdigest() != rec.get("sap_source_sha256"):
        return None
    return rec.get("hbm_bytes_per_launch")


def kernel_time(torch, fn, reps, stream):
    """Average duration of fn() in ms, timed with HIP events on `stream`."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def plain_gcr_iterations(P, mglma):
    """Iterations the restarted GCR(16) without preconditioner needs for the
    first point-source system to reach 1e-10, run in FP64 on the GPU (an
    algorithmic count, used to scale the host timing of the oracle)."""
    x = P.ctx.fine(1)
    p = mglma.default_params(tol=1e-10, max_outer=1, max_inner=5000, gcr_m=16, inner_tol=1e-10, use_mg=0,
                             inner=mglma.F64, smoother=mglma.F64, coarse=mglma.F64)
    rc, st = P.ctx.solve(P.src[:1].contiguous(), x, p, raise_on_error=False)
    return int(st[0]["inner"]), float(st[0]["true_rel_res"])


def cpu_baseline(wl, n_iter_needed, budget_s=20.0):
    """The oracle (numpy FP64) on a bounded sample of the same workload: its
    restarted GCR(16) on one point-source system of the same lattice, timed
    per iteration (median of the repetitions) with one thread and with every
    host thread allowed; solves/s = 1 / (time per iteration x the iterations
    that GCR(16) needs for this system to reach 1e-10).  Also, as a complete
    (not extrapolated) figure: the median of five full oracle solves to
    1e-10 of the 4^4 workload."""
    from threadpoolctl import threadpool_limits
    from oracle import dirac, estimators, solvers
    from paper_2412_06347_amd import synth
    L = wl["L"]
    U = synth.gauge_field(L, wl["eps"], wl["seed"])
    D = dirac.WilsonClover(U, L, wl["kappa"], wl["csw"])
    b = estimators.point_sources(L, (0, 0, 0, 0))[:1]
    ncpu = os.cpu_count() or 1

    def per_iter(threads, budget):
        with threadpool_limits(threads):
            t0 = time.time()
            D.M(b)
            t_apply = time.time() - t0
            n_it = max(5, int(budget / (1.2 * t_apply)))
            # one GCR(16) run of n_it iterations (one operator apply each); the
            # per-iteration times are the differences of the apply start times
            stamps = []

            def timed_apply(v):
                stamps.append(time.time())
                return D.M(v)

            t0 = time.time()
            x, it, res = solvers.gcr(timed_apply, b, tol=1e-10, m=16, max_iter=n_it)
            t = time.time() - t0
            stamps.append(t0 + t)
        dt = np.diff(stamps) if len(stamps) > 1 else np.array([t / max(it, 1)])
        return float(np.median(dt)), it, float(res[0]), t

    t1, it1, res1, tt1 = per_iter(1, budget_s / 2)
    tn, itn, resn, ttn = per_iter(ncpu, budget_s / 2)
    best, cores = (tn, ncpu) if tn < t1 else (t1, 1)
    # complete oracle solves of the 4^4 workload (W1), median of five
    w1 = WORKLOADS["4c4"]
    U1 = synth.gauge_field(w1["L"], w1["eps"], w1["seed"])
    D1 = dirac.WilsonClover(U1, w1["L"], w1["kappa"], w1["csw"])
    b1 = estimators.point_sources(w1["L"], (0, 0, 0, 0))[:1]
    with threadpool_limits(1):
        ts, its = [], []
        for _ in range(6):
            t0 = time.time()
            x1, k1, r1 = solvers.gcr(D1.M, b1, tol=1e-10, m=16, max_iter=5000)
            ts.append(time.time() - t0)
            its.append(k1)
    cpu = open("/proc/cpuinfo").read().split("model name")[1].split(":")[1].split("\n")[0].strip()
    return dict(value=float(1.0 / (best * n_iter_needed)), unit="solves/s", cores=cores, kind="oracle",
                sample="numpy FP64 oracle (%s, %d host threads): its restarted GCR(16) on one point-source system "
                       "of the %s lattice, median time per iteration %.2f s with 1 thread (%d iterations, %.1f s) "
                       "and %.2f s with %d threads allowed (%d iterations, %.1f s); one solve to 1e-10 = %d "
                       "iterations of the same GCR(16) (count from an FP64 run of it to convergence)"
                       % (cpu, ncpu, "x".join(map(str, L)), t1, it1, tt1, tn, ncpu, itn, ttn, n_iter_needed),
                per_iteration_s={"1": t1, str(ncpu): tn},
                w1_full_solve={"workload": "4^4, kappa=0.120, point source, GCR(16) to 1e-10, 1 thread",
                               "median_s": float(np.median(ts[1:])), "runs": len(ts) - 1,
                               "iterations": int(np.median(its)), "solves_per_s": float(1.0 / np.median(ts[1:]))})


def local_coherence(wl, degree=64):
    """fig:lc on a synthetic ensemble: the 2 Nv lowest modes of Q to a residual
    of 1e-12 from the device eigensolver, the block basis built from the Nv
    lowest (sec. "Local coherence and block decomposition"), and 1 - eps_c for
    every computed mode c."""
    import torch
    from paper_2412_06347_amd import mglma, synth
    L, Nv = wl["L"], wl["Nv"]
    U = torch.from_numpy(synth.gauge_field(L, wl["eps"], wl["seed"]).view(np.float64)).cuda()
    ctx = mglma.Context(L, wl["block"], wl["kappa"], wl["csw"])
    ctx.load_gauge(U)
    nev, nblk = 2 * Nv, min(64, 2 * Nv + 16)
    init = ctx.fine(nblk)
    for k0 in range(0, nblk, 8):      # seeded start block, a few fields at a time (host memory)
        k1 = min(nblk, k0 + 8)
        ctx.import_fields(torch.from_numpy(synth.gaussian_fields(k1 - k0, L, 9000 + k0).view(np.float64)).cuda(),
                          init[k0:k1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, lam, modes, st = ctx.fine_eigs(init, nev, tol=1e-12, degree=degree, max_iter=300, raise_on_error=False)
    torch.cuda.synchronize()
    t_eig = time.perf_counter() - t0
    del init
    ctx.build_subspace(modes[:Nv].contiguous())
    eps = ctx.deficit(modes)
    print(json.dumps({
        "diagnostic": "local coherence (fig:lc) on synthetic fields",
        "workload": "%dx%d^3, eps=%g, kappa=%g, c_sw=%g, %d^4 blocks, Nv=%d" %
                    (L[0], L[1], wl["eps"], wl["kappa"], wl["csw"], wl["block"][0], Nv),
        "eigensolver": {"rc": rc, "nev": nev, "nblk": nblk, "degree": degree, "seconds": round(t_eig, 2),
                        "iters": st["iters"], "vector_applies": st["applies"], "max_res": st["max_res"],
                        "spectrum_bound": st["spectrum_bound"]},
        "lambda": [round(float(x), 8) for x in lam],
        "one_minus_eps": [round(float(1 - e), 6) for e in eps],
    }), flush=True)


def hierarchy(wl, reps=3):
    """The paper's four-level estimator structure (tab:blocks: level-1 blocks,
    level-2 blocks of twice their size, one level-3 block spanned by the
    constant coarse vectors, evaluated exactly) on the bench workload: time of
    the level-2 operator build and of the level-2 propagator pieces for the 12
    point sources, the cost of a solve on each level against the fine solve
    (measured and modelled ratio Phi, level 1 also with the K-cycle), the
    four level contributions of the point correlator, and
    the stochastic estimator with per-level source counts (fine solves only for
    L0) timed level by level."""
    import torch
    from paper_2412_06347_amd import mglma, synth as synth_mod
    P = Pipeline(wl, log_setup=False)
    ctx = P.ctx
    P.step(mixed_params(mglma))
    Nv, nc, V1 = ctx.query(3), ctx.nc, ctx.V1
    b2 = [2 * b for b in wl["block"]]

    def timed_out(f):
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = f()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, out

    def timed(f):
        return timed_out(f)[0]

    t_build = timed(lambda: ctx.build_level2(b2))
    # cost of a solve on each level (App. "Performance model": Phi(Lk) = cost of
    # the fine solve / cost of the level-k solve; the model takes equal
    # iteration counts, Phi = 12 V / (nc V_k)): the 12 point sources batched,
    # each level solved to 1e-10 (level k: its restriction of the sources)
    V = int(np.prod(wl["L"]))
    xf, Re, x1 = ctx.fine(12), ctx.coarse(12), ctx.coarse(12)
    R2, x2 = ctx.level2_field(12), ctx.level2_field(12)
    ctx.restrict(P.src, Re)
    ctx.level2_restrict(Re, R2)
    t_fine, (_, st_f) = timed_out(lambda: ctx.solve(P.src, xf, mixed_params(mglma)))
    capped = dict(tol=1e-10, coarse=mglma.BF16, max_outer=40, max_inner=1)
    lv_solvers = {
        "L1 GCR on the even-odd reduced D_1 (12 steps per FP64 round)":
            (1, mglma.default_params(coarse_iters=12, coarse_eo=1, **capped)),
        "L1 K-cycle (4 flexible steps per round; each: 4 GCR steps on D_2, 4 MR steps on D_1)":
            (1, mglma.default_params(coarse_iters=4, coarse_eo=0, kcycle=4, kcycle_nu=4, **capped)),
        "L2 GCR on D_2 (8 steps per FP64 round)": (2, mglma.default_params(coarse_iters=8, **capped)),
    }
    cost = {"L0 MG solve (bench settings)": dict(ms=round(1e3 * t_fine, 2), iterations=st_f[0]["inner"])}
    for name, (lev, prm) in lv_solvers.items():
        if lev == 1:
            t, st = timed_out(lambda: ctx.coarse_solve(Re, x1, prm))
        else:
            t, st = timed_out(lambda: ctx.level2_solve(R2, x2, prm))
        Vk = V1 if lev == 1 else ctx.V2
        cost[name] = dict(ms=round(1e3 * t, 2), rounds=st[0]["outer"], level_applies=st[0].get("coarse"),
                          max_rel_res=max(q["true_rel_res"] for q in st), Phi=round(t_fine / t, 1),
                          Phi_model=round(12 * V / (nc * Vk), 1))
    modes = np.zeros((Nv, V1, nc), dtype=np.complex128)
    for c in range(Nv):
        modes[c, :, c] = 1.0
        modes[c, :, Nv + c] = 1.0
    ctx.set_top_modes(torch.from_numpy(modes.view(np.float64).reshape(Nv, V1, nc, 2)).cuda())
    cp = mglma.default_params(tol=1e-10, coarse=mglma.BF16, coarse_iters=12, max_outer=40, coarse_eo=1)
    cg1, ct, cg2 = ctx.coarse(12), ctx.coarse(12), ctx.coarse(12)
    t_p1 = timed(lambda: ctx.coarse_pieces(P.src, cg1, ct, cp))
    t_p2 = timed(lambda: ctx.level2_pieces(P.src, cg2, cp))
    rows = ctx.contract_levels(mglma.SRC_POINT, [0], fine=P.x, coarse=[cg1, cg2, ct], exact_top=True)
    G3 = rows[4]
    L0 = wl["L"][0]
    lv = dict(L0=rows[0], L1=rows[1], L2=rows[2], L3_point=rows[3])
    # stochastic estimator with per-level source counts (sec. "Stochastic estimator
    # on level k": few sources for the level that needs fine solves, more for the
    # coarse levels; spin-diluted time-slice noise, 4 right-hand sides per source)
    Lat = wl["L"]
    V3 = Lat[1] * Lat[2] * Lat[3]
    nsrc = {"L0": 2, "L1": 8, "L2": 32}

    def noise(n, seed):
        xi = np.ascontiguousarray(synth_mod.z4_noise(n, Lat, seed))
        t = synth_mod.time_slices(n, Lat[0], seed + 1)
        eta = ctx.fine(4 * n)
        ctx.noise_sources(torch.from_numpy(xi.view(np.float64).reshape(n, V3, 3, 2)).cuda(), t, eta)
        return eta, t

    stoch, tlev = {}, {}
    for lvname, seed in (("L0", 7100), ("L1", 7200), ("L2", 7300)):
        n = nsrc[lvname]
        eta, t = noise(n, seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g1, tp, g2 = ctx.coarse(4 * n), ctx.coarse(4 * n), ctx.coarse(4 * n)
        # the level's estimator from its own sources: row 0 of the level
        # assembly over the two cumulative pieces that bound it
        if lvname == "L0":
            x = ctx.fine(4 * n)
            ctx.solve(eta, x, mixed_params(mglma))
            ctx.coarse_pieces(eta, g1, None, cp)
            G = ctx.contract_levels(mglma.SRC_STOCH, t, fine=x, coarse=[g1])[0]
        elif lvname == "L1":
            ctx.coarse_pieces(eta, g1, None, cp)
            ctx.level2_pieces(eta, g2, cp)
            G = ctx.contract_levels(mglma.SRC_STOCH, t, coarse=[g1, g2])[0]
        else:
            ctx.coarse_pieces(eta, g1, tp, cp)
            ctx.level2_pieces(eta, g2, cp)
            G = ctx.contract_levels(mglma.SRC_STOCH, t, coarse=[g2, tp])[0]
        torch.cuda.synchronize()
        tlev[lvname] = time.perf_counter() - t0
        stoch[lvname] = G
    print(json.dumps({
        "diagnostic": "four-level hierarchy (nested blocks, eq:mglma:decomp) on the bench workload",
        "levels": {"1": "%s blocks, V1=%d, nc=%d" % ("x".join(map(str, wl["block"])), V1, nc),
                   "2": "%s blocks, V2=%d" % ("x".join(map(str, b2)), ctx.V2),
                   "3": "one block: the %d constant coarse vectors, exact (eq:G_LL:exact)" % nc},
        "build_level2_ms": round(1e3 * t_build, 2),
        "cost_per_level_12rhs": cost,
        "level1_pieces_ms_12rhs": round(1e3 * t_p1, 2),
        "level2_pieces_ms_12rhs": round(1e3 * t_p2, 2),
        "point_correlator_t": list(range(0, L0, max(1, L0 // 8))),
        "C_levels_real": {k: [float(v[t].real) for t in range(0, L0, max(1, L0 // 8))] for k, v in lv.items()},
        "G_L3_exact_real": [float(G3[t].real) for t in range(0, L0, max(1, L0 // 8))],
        "stochastic": {"sources_per_level": nsrc,
                       "seconds_per_level": {k: round(v, 3) for k, v in tlev.items()},
                       "G_levels_real": {k: [float(v[t].real) for t in range(0, L0, max(1, L0 // 8))]
                                         for k, v in stoch.items()},
                       "G_total_real": [float((sum(stoch.values()) + G3)[t].real)
                                        for t in range(0, L0, max(1, L0 // 8))]},
    }), flush=True)


def config4(wl, gb_per_rhs=23.0):
    """The largest configuration as stated: 48^3 x 96 (seeded synthetic field,
    eps = 0.25, kappa = 0.125), 4^4 blocks, Nv = 32 test vectors (nc = 64),
    Nlm = 64 coarse low modes (r = 128), 48 time-diluted Z4 sources x 4
    spins = 192 right-hand sides solved as multi-RHS batches sized by the
    free HBM, and the translation-averaged low-mode contraction eq:G_LL:exact.
    Test vectors: Gaussian fields drawn on the device (seeded torch
    generator), improved by three rounds of 40 plain FP32 GCR(8) steps in
    batches of four.  Prints one JSON line with the times and sizes."""
    import torch
    from paper_2412_06347_amd import mglma, synth as synth_mod
    L, Nv, Nlm, nsrc = wl["L"], wl["Nv"], wl["Nlm"], wl["nsrc"]
    out = {"diagnostic": "48^3x96 configuration (N_v = %d, N_lm = %d, %d sources x 4 spins)" % (Nv, Nlm, nsrc)}
    t0 = time.time()
    def prog(done, tot):
        if done == tot or (done >> 20) % 8 == 0:
            log("c4: gauge field %d / %d links (%.0f s)" % (done, tot, time.time() - t0))
    U = synth_mod.gauge_field(L, wl["eps"], wl["seed"], progress=prog)
    out["gauge_host_s"] = round(time.time() - t0, 1)
    ctx = mglma.Context(L, wl["block"], wl["kappa"], wl["csw"])
    Ud = torch.from_numpy(U.view(np.float64)).cuda()
    del U
    ctx.load_gauge(Ud)
    del Ud
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log("c4: gauge loaded (%.1f s), resident %.1f GB" % (time.time() - t0, ctx.resident_bytes() / 1e9))
    # test vectors
    t1 = time.time()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(wl["seed"] + 1000)
    tv = ctx.fine(Nv)
    tv.normal_(generator=gen)
    p = mglma.default_params(use_mg=0, inner=mglma.F32, max_outer=1, max_inner=40, gcr_m=8, tol=1e-30,
                             inner_tol=1e-30)
    y = ctx.fine(4)
    for _ in range(3):
        for k0 in range(0, Nv, 4):
            ctx.solve(tv[k0:k0 + 4], y, p, raise_on_error=False)
            nrm = torch.linalg.vector_norm(y.reshape(4, -1), dim=1)
            tv[k0:k0 + 4] = y / nrm[:, None, None, None]
    del y
    torch.cuda.synchronize()
    ctx.release_workspace()          # the GCR workspace of the batches of four
    torch.cuda.empty_cache()
    out["testvec_s"] = round(time.time() - t1, 1)
    t1 = time.time()
    ctx.build_subspace(tv)
    torch.cuda.synchronize()
    out["build_subspace_s"] = round(time.time() - t1, 2)
    del tv
    torch.cuda.empty_cache()
    out["resident_GB_after_subspace"] = round(ctx.resident_bytes() / 1e9, 1)
    log("c4: subspace built (%.1f s), resident %.1f GB" % (time.time() - t1, ctx.resident_bytes() / 1e9))
    # top level: Nlm low modes of Q_1 from the device eigensolver
    t1 = time.time()
    # in pieces of 20 iterations, each continuing from the previous piece's
    # whole block (a progress line per piece), at most 40 iterations: the
    # synthetic field's low modes come in near-degenerate momentum shells and
    # N_lm = 64 cuts through one of them, whose members the filter does not
    # separate (a 128-vector block leaves the same 16 pairs unconverged after
    # 120 iterations)
    nblk = Nlm + 32
    init = torch.from_numpy(synth_mod.gaussian_coarse(nblk, ctx.V1, ctx.nc, 4242).view(np.float64)).cuda()
    its = 0
    for piece in range(2):
        rc, lam, blk, st = ctx.coarse_eigs(init, Nlm, tol=1e-12, max_iter=20, raise_on_error=False,
                                           out_block=True)
        its += st["iters"]
        log("c4: eigensolver %d iterations, %d of %d pairs converged, largest residual %.2e (%.0f s)"
            % (its, st["nconv"], Nlm, st["max_res"], time.time() - t1))
        del init
        init = blk
        if rc == 0:
            break
    modes = blk[:Nlm].clone()
    del init, blk
    torch.cuda.synchronize()
    out["eigs"] = dict(rc=rc, seconds=round(time.time() - t1, 1), iters=its, nconv=st["nconv"],
                       max_res=st["max_res"], block=nblk,
                       ritz_values=[round(float(v), 6) for v in lam])
    t1 = time.time()
    ctx.set_top_modes(modes.contiguous())
    torch.cuda.synchronize()
    out["set_top_modes_s"] = round(time.time() - t1, 3)
    del modes
    t1 = time.time()
    G_exact = ctx.contract_top()
    out["contract_top_ms"] = round(1e3 * (time.time() - t1), 2)
    ctx.release_workspace()
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    nb = int(max(1, min(3, (0.8 * free / 1e9) // (4 * gb_per_rhs))))     # sources per batch
    out["free_GB_before_solves"] = round(free / 1e9, 1)
    out["rhs_per_batch"] = 4 * nb
    log("c4: top level set; %.1f GB free, %d right-hand sides per batch" % (free / 1e9, 4 * nb))
    # stochastic sources, multi-RHS MG solves, coarse pieces, level assembly
    V3 = L[1] * L[2] * L[3]
    xi = np.ascontiguousarray(synth_mod.z4_noise(nsrc, L, 7400))
    tn = synth_mod.time_slices(nsrc, L[0], 7401)
    params = mixed_params(mglma, max_inner=200)
    cp = mglma.default_params(tol=1e-10, coarse=mglma.BF16, coarse_iters=12, max_outer=40, coarse_eo=1)
    acc = torch.zeros((3, L[0], 2), dtype=torch.float64, device="cuda")
    eta, x = ctx.fine(4 * nb), ctx.fine(4 * nb)
    cg, ct = ctx.coarse(4 * nb), ctx.coarse(4 * nb)
    res, iters, t_solve, t_pieces, t_con = [], [], 0.0, 0.0, 0.0
    torch.cuda.synchronize()
    t1 = time.time()
    for n0 in range(0, nsrc, nb):
        k = min(nb, nsrc - n0)
        ta = time.time()
        ctx.noise_sources(torch.from_numpy(xi[n0:n0 + k].view(np.float64).reshape(k, V3, 3, 2)).cuda(),
                          tn[n0:n0 + k], eta[:4 * k])
        rcs, st = ctx.solve(eta[:4 * k], x[:4 * k], params, raise_on_error=False)
        torch.cuda.synchronize()
        tb = time.time()
        ctx.coarse_pieces(eta[:4 * k], cg[:4 * k], ct[:4 * k], cp)
        torch.cuda.synchronize()
        tc = time.time()
        ctx.contract_levels_acc(mglma.SRC_STOCH, tn[n0:n0 + k], acc, 1.0 / nsrc, n0 > 0, fine=x[:4 * k],
                                coarse=[cg[:4 * k], ct[:4 * k]])
        torch.cuda.synchronize()
        td = time.time()
        t_solve += tb - ta
        t_pieces += tc - tb
        t_con += td - tc
        res += [q["true_rel_res"] for q in st]
        iters += [q["inner"] for q in st]
        if n0 == 0:
            log("c4: first batch: solve %.2f s, pieces %.2f s, contraction %.3f s, res %.2e" %
                (tb - ta, tc - tb, td - tc, max(res)))
    total = time.time() - t1
    lv = acc.cpu().numpy()
    lv = lv[..., 0] + 1j * lv[..., 1]
    ts = list(range(0, L[0], L[0] // 8))
    out.update({"solves": 4 * nsrc, "seconds_total": round(total, 2), "solves_per_s": 4 * nsrc / total,
                "fine_solve_s": round(t_solve, 2), "coarse_pieces_s": round(t_pieces, 2),
                "contraction_s": round(t_con, 3), "max_true_rel_res": max(res),
                "inner_iterations_max": max(iters),
                "G_L0_real": [float(lv[0][t].real) for t in ts], "G_L1_real": [float(lv[1][t].real) for t in ts],
                "G_L2_exact_real": [float(G_exact[t].real) for t in ts], "t": ts})
    print(json.dumps(out), flush=True)


def spectra_and_conditioning(wl, Nv=16, seed=5100):
    """Appendices on the spectra of coarse and fine operators and on the
    condition numbers of coarse-grid operators, on a synthetic ensemble: the
    2 Nv lowest modes of Q (device eigensolver, residual <= 1e-12), the block
    basis (4^4 blocks) from the Nv lowest, the lowest eigenvalues of the
    chirally split Q_1 and of the coarse operator without chiral split; then
    for the operators of the hierarchy (fine Q; Q_1 on 4^4 blocks; Q_2 on
    8^4 blocks; the low-mode-averaging operator diag(lambda_1..lambda_Nv))
    their dimension, condition number |lambda|_max / |lambda|_min and the
    iteration count of unpreconditioned FP64 GCR(16) on a random right-hand
    side to 1e-10."""
    import torch
    from paper_2412_06347_amd import mglma, synth as synth_mod
    L = wl["L"]
    U = torch.from_numpy(synth_mod.gauge_field(L, wl["eps"], wl["seed"]).view(np.float64)).cuda()
    ctx = mglma.Context(L, wl["block"], wl["kappa"], wl["csw"])
    ctx.load_gauge(U)
    nev = 2 * Nv
    nblk = nev + 16
    init = ctx.fine(nblk)
    for k0 in range(0, nblk, 8):
        k1 = min(nblk, k0 + 8)
        ctx.import_fields(torch.from_numpy(synth_mod.gaussian_fields(k1 - k0, L, seed + k0).view(np.float64)).cuda(),
                          init[k0:k1])
    t0 = time.perf_counter()
    rc, lam_f, modes, st_f = ctx.level_eigs(mglma.OP_FINE, init, nev, tol=1e-12, degree=64, max_iter=300,
                                            raise_on_error=False)
    t_f = time.perf_counter() - t0
    del init
    tv = modes[:Nv].contiguous()
    ctx.build_subspace(tv)
    V1, nc = ctx.V1, ctx.nc

    def coarse_low(op, n_per_site, nsites, k, sd):
        init = torch.from_numpy(synth_mod.gaussian_coarse(k + 16, nsites, n_per_site, sd).view(np.float64)).cuda()
        return ctx.level_eigs(op, init, k, tol=1e-12, max_iter=300, raise_on_error=False)

    rc1, lam_1, _, st_1 = coarse_low(mglma.OP_COARSE, nc, V1, nev, seed + 1)
    ctx.build_nonchiral(tv)
    rcn, lam_n, _, st_n = coarse_low(mglma.OP_NONCHIRAL, Nv, V1, nev, seed + 2)
    ctx.build_level2([2 * b for b in wl["block"]])
    V2 = ctx.V2
    rc2, lam_2, _, st_2 = coarse_low(mglma.OP_LEVEL2, nc, V2, 8, seed + 3)
    # iteration counts of unpreconditioned FP64 GCR(16), random right-hand side, to 1e-10
    g = torch.Generator(device="cuda")
    g.manual_seed(seed + 4)
    b = ctx.fine(1)
    b.normal_(generator=g)
    x = ctx.fine(1)
    pf = mglma.default_params(tol=1e-10, max_outer=1, max_inner=20000, gcr_m=16, inner_tol=1e-10, use_mg=0,
                              inner=mglma.F64, smoother=mglma.F64, coarse=mglma.F64)
    rcf, sf = ctx.solve(b, x, pf, raise_on_error=False)
    pc = mglma.default_params(tol=1e-10, max_outer=2000, coarse_iters=16, coarse=mglma.F64, coarse_eo=0)
    bc = ctx.coarse(1)
    bc.normal_(generator=g)
    xc = ctx.coarse(1)
    s1 = ctx.coarse_solve(bc, xc, pc)
    b2 = ctx.level2_field(1)
    b2.normal_(generator=g)
    x2 = ctx.level2_field(1)
    s2 = ctx.level2_solve(b2, x2, pc)
    lma = np.abs(lam_f[:Nv])
    ops = {
        "LMA diag(lambda_1..lambda_%d) (one block)" % Nv: dict(dim=Nv, cond=float(lma.max() / lma.min()),
                                                               gcr16_iterations=None),
        "Q_2 (8^4 blocks, chiral)": dict(dim=V2 * nc, cond=st_2["lambda_max_abs"] / float(np.abs(lam_2).min()),
                                         gcr16_iterations=s2[0]["coarse"], res=s2[0]["true_rel_res"]),
        "Q_1 (4^4 blocks, chiral)": dict(dim=V1 * nc, cond=st_1["lambda_max_abs"] / float(np.abs(lam_1).min()),
                                         gcr16_iterations=s1[0]["coarse"], res=s1[0]["true_rel_res"]),
        "Q (fine)": dict(dim=12 * ctx.V, cond=st_f["lambda_max_abs"] / float(np.abs(lam_f).min()),
                         gcr16_iterations=sf[0]["inner"], res=sf[0]["true_rel_res"]),
    }
    rnd = lambda a: [round(float(v), 8) for v in a]
    print(json.dumps({
        "diagnostic": "spectra and condition numbers of the operators of the hierarchy (synthetic fields)",
        "workload": "%dx%d^3, eps=%g, kappa=%g, c_sw=%g; basis from the %d lowest modes of Q" %
                    (L[0], L[1], wl["eps"], wl["kappa"], wl["csw"], Nv),
        "fine_eigs": {"rc": rc, "seconds": round(t_f, 1), "iters": st_f["iters"], "max_res": st_f["max_res"]},
        "lowest_abs_lambda": {"Q": rnd(np.abs(lam_f)), "Q_1 chiral": rnd(np.abs(lam_1)),
                              "Q_nc (no chiral split)": rnd(np.abs(lam_n))},
        "chiral_reproduces_lowest_%d" % Nv: float(np.abs(np.sort(np.abs(lam_1))[:Nv] -
                                                         np.sort(np.abs(lam_f))[:Nv]).max()),
        "nonchiral_below_Q_min": int(np.sum(np.abs(lam_n) < np.abs(lam_f).min() * (1 - 1e-9))),
        "operators": ops,
    }), flush=True)


def setup_recipes(wl, reps=2):
    """Test-vector preparation recipes on the bench workload (the basis should
    span approximations of the low modes of Q, sec. "Local coherence and block
    decomposition"): setup time and the 12 point-source MG solve that follows
    (iterations, time), for Gaussian vectors as they are, the bench's recipe
    (inverse iteration with unpreconditioned GCR) and the adaptive setup
    (inverse iteration with the multigrid solver of the current subspace,
    mglma_adaptive_setup)."""
    import torch
    from paper_2412_06347_amd import mglma, synth as synth_mod
    L, Nv = wl["L"], wl["Nv"]
    U = torch.from_numpy(synth_mod.gauge_field(L, wl["eps"], wl["seed"]).view(np.float64)).cuda()
    ctx = mglma.Context(L, wl["block"], wl["kappa"], wl["csw"])
    ctx.load_gauge(U)
    src, x = ctx.fine(12), ctx.fine(12)
    ctx.point_sources((0, 0, 0, 0), src)
    plain = mglma.default_params(use_mg=0, inner=mglma.F32, max_outer=1, max_inner=40, gcr_m=16)

    def fresh():
        tv = ctx.fine(Nv)
        ctx.import_fields(torch.from_numpy(synth_mod.gaussian_fields(Nv, L, wl["seed"] + 1000).view(np.float64))
                          .cuda(), tv)
        torch.cuda.synchronize()
        return tv

    def gaussian(tv):
        ctx.build_subspace(tv)

    def bench_recipe(tv):
        # three rounds of 40 unpreconditioned FP32 GCR steps on M y = v, normalised
        ctx.adaptive_setup(tv, plain, rounds=3, iters=40)

    def adaptive(mg_rounds, mg_iters):
        # one plain round of 20 steps, then multigrid rounds
        def f(tv):
            ctx.adaptive_setup(tv, plain, rounds=1, iters=20)
            ctx.adaptive_setup(tv, mixed_params(mglma), rounds=mg_rounds, iters=mg_iters)
        return f

    out = {}
    for name, f in (("gaussian", gaussian), ("inverse iteration, 3 x 40 plain GCR steps", bench_recipe),
                    ("adaptive: 1 x 20 plain GCR steps, then 2 x 4 MG iterations", adaptive(2, 4)),
                    ("adaptive: 1 x 20 plain GCR steps, then 3 x 6 MG iterations", adaptive(3, 6))):
        ts, tsol = [], []
        for _ in range(reps):
            tv = fresh()
            t0 = time.perf_counter()
            f(tv)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            rc, st = ctx.solve(src, x, mixed_params(mglma, max_inner=400), raise_on_error=False)
            torch.cuda.synchronize()
            tsol.append(time.perf_counter() - t0)
        out[name] = dict(setup_s=round(min(ts), 3), solve_ms=round(1e3 * min(tsol), 1), status=rc,
                         iterations=max(q["inner"] for q in st), max_rel_res=max(q["true_rel_res"] for q in st))
    print(json.dumps({"diagnostic": "test-vector setup recipes on the bench workload, then the 12-RHS MG solve",
                      "workload": "%dx%d^3, %d^4 blocks, Nv=%d" % (L[0], L[1], wl["block"][0], Nv),
                      "recipes": out}), flush=True)


def serving(reqs_n=60, seed=7, iso_n=24, max_src=8, emit=True, mix=("16c32", "24c48")):
    """Serving mix (a reduced version of the serving workload: resident
    ensembles, by default 16^3 x 32 and 24^3 x 48): requests of 1-max_src
    stochastic time-slice sources (x 4 spin-diluted right-hand sides) on a
    uniformly drawn ensemble.  The isolated service rate from requests run
    one at a time, then a Poisson stream at 0.8 of it; solves/s and p50/p99
    latency (arrival to the returned correlator levels)."""
    import torch
    from paper_2412_06347_amd.serve import Server, poisson_arrivals
    free, _ = torch.cuda.mem_get_info()
    ens = {name: WORKLOADS[name] for name in mix}
    vols = " and ".join("%d^3x%d" % (ens[n]["L"][1], ens[n]["L"][0]) for n in mix)
    g = np.random.default_rng(seed)

    def draw(n):
        return [(list(ens)[int(g.integers(len(ens)))], int(g.integers(1, max_src + 1))) for _ in range(n)]

    def run(srv, items, arrivals):
        reqs = []
        t0 = time.perf_counter()
        for k, ((name, n_src), t) in enumerate(zip(items, arrivals)):
            while time.perf_counter() - t0 < t:
                time.sleep(0.0005)
            reqs.append(srv.submit(name, n_src, 1000 + k))
            if emit and (k + 1) % 10 == 0:
                log("serving: %d/%d requests arrived, %d done (%.0f s)"
                    % (k + 1, len(items), sum(r.done.is_set() for r in reqs), time.perf_counter() - t0))
        for k, r in enumerate(reqs):
            r.wait(600)
            if emit:
                log("serving: request %d/%d done (%s, %d sources, %.2f s)"
                    % (k + 1, len(reqs), r.ensemble, r.n_src, r.t_done - r.t_arrival))
        return reqs

    srv = Server(hbm_budget=0.8 * free, max_batch_rhs=48)
    t0 = time.perf_counter()
    for name, wl in ens.items():
        srv.add_ensemble(name, wl)
        log("serving: ensemble %s resident, %d slots (%.0f s)" % (name, srv.slots[name], time.perf_counter() - t0))
    setup = time.perf_counter() - t0
    srv.start()
    # isolated service rate: requests one at a time (each submitted when the
    # previous one has returned); the Poisson stream then runs at 0.8 of it
    iso = draw(iso_n)
    t_iso = []
    for k, (name, n_src) in enumerate(iso):
        r = srv.submit(name, n_src, 500 + k)
        r.wait(600)
        t_iso.append(r.t_done - r.t_arrival)
        if emit:
            log("serving: isolated request %d/%d (%s, %d sources, %.2f s)" % (k + 1, len(iso), name, n_src, t_iso[-1]))
    cap = dict(n=len(iso), solves=4 * sum(n for _, n in iso), seconds=float(np.sum(t_iso)),
               mean_service_s=float(np.mean(t_iso)))
    cap["solves_per_s"] = cap["solves"] / cap["seconds"]
    srv.completed.clear()
    srv.batches.clear()
    mean_rhs = 4 * np.mean([n for _, n in iso])
    rate = 0.8 / cap["mean_service_s"]
    stream = draw(reqs_n)
    reqs = run(srv, stream, poisson_arrivals(reqs_n, rate, seed + 1))
    srv.stop()
    st = srv.stats()
    res = max(r.result["max_true_rel_res"] for r in reqs)
    for eng in srv.engines.values():
        eng.pool.close()
        eng.ctx.close()
    out = {"workload": "requests of 1-%d spin-diluted time-slice sources on resident %s "
                       "ensembles, mixed-precision MG to 1e-10, right-hand sides join and leave between outer "
                       "cycles" % (max_src, vols),
           "isolated_solves_per_s": cap["solves_per_s"], "isolated_mean_service_s": cap["mean_service_s"],
           "poisson_requests": st["n"], "requests_per_s": rate,
           "offered_solves_per_s": rate * mean_rhs, "solves_per_s": st["solves_per_s"],
           "p50_s": st["p50_s"], "p99_s": st["p99_s"], "max_true_rel_res": res}
    if not emit:
        return out
    print(json.dumps({"diagnostic": "serving mix: resident %s ensembles, requests of 1-%d sources, continuous "
                                    "batching (right-hand sides join and leave between outer cycles)"
                                    % (vols, max_src),
                      "setup_s": round(setup, 1), "slots": srv.slots,
                      "isolated": cap,
                      "poisson": {"requests_per_s": rate, "offered_solves_per_s": rate * mean_rhs,
                                  **{k: st[k] for k in ("n", "solves", "solves_per_s", "p50_s", "p99_s", "cycles")}},
                      "max_true_rel_res": res}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="24c48", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison step")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-serve", action="store_true", help="skip the bounded serving leg")
    ap.add_argument("--calib-copy", action="store_true", help="only run a plain 1 GiB device copy (counter scale)")
    ap.add_argument("--dslash-only", action="store_true",
                    help="only run the Wilson-clover apply of the workload (for hardware-counter runs)")
    ap.add_argument("--lc", action="store_true",
                    help="local-coherence diagnostic instead of the bench: the 2 Nv lowest exact modes of Q "
                         "(device eigensolver), the block basis from the Nv lowest, the deficits of all "
                         "(default workload 16c32)")
    ap.add_argument("--hier", action="store_true",
                    help="four-level hierarchy diagnostic instead of the bench: level-2 build and pieces timed, "
                         "level contributions of the point correlator")
    ap.add_argument("--sap-only", action="store_true",
                    help="only run SAP smoother cycles of the workload (for hardware-counter runs)")
    ap.add_argument("--serve", action="store_true",
                    help="serving diagnostic instead of the bench: two resident ensembles, requests of 1-48 "
                         "sources, the isolated service rate, then a Poisson stream of 500 requests at 0.8 of it; "
                         "solves/s and p50/p99 latency")
    ap.add_argument("--serve-wide", action="store_true",
                    help="the same with three resident ensembles (16^3x32, 24^3x48, 32^3x64) and requests of "
                         "1-48 sources")
    ap.add_argument("--cond", action="store_true",
                    help="spectra and condition numbers of the hierarchy's operators instead of the bench "
                         "(default workload 16c32)")
    ap.add_argument("--c4", action="store_true",
                    help="the 48^3x96 configuration (Nv = 32, Nlm = 64, 48 sources x 4 spins) instead of the bench")
    ap.add_argument("--setup", action="store_true",
                    help="test-vector setup diagnostic instead of the bench: Gaussian vectors, inverse iteration "
                         "with plain GCR, adaptive setup with the multigrid solver; setup time and the MG solve")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one MI355X only: the hot path runs on a single GPU "
              "(multi-GPU sharding is not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.calib_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes_read": a.numel() * 8, "copies": 3}))
        return
    from paper_2412_06347_amd import mglma, synth
    if args.lc:
        local_coherence(WORKLOADS["16c32" if args.workload == "24c48" else args.workload])
        return
    wl = WORKLOADS[args.workload]
    if args.hier:
        hierarchy(wl)
        return
    if args.setup:
        setup_recipes(wl)
        return
    if args.c4:
        config4(WORKLOADS["48c96"])
        return
    if args.cond:
        spectra_and_conditioning(WORKLOADS["16c32" if args.workload == "24c48" else args.workload])
        return
    if args.serve:
        serving(reqs_n=500, iso_n=24, max_src=48)
        return
    if args.serve_wide:
        serving(reqs_n=40, iso_n=12, max_src=48, mix=("16c32", "24c48", "32c64"))
        return
    if args.sap_only:
        # the SAP smoother of the step (FP16 links, 12 RHS, the bench's block
        # steps), 5 cycles = 10 half-sweep launches, for hardware-counter runs
        L = wl["L"]
        U = torch.from_numpy(synth.gauge_field(L, wl["eps"], wl["seed"]).view(np.float64)).cuda()
        ctx = mglma.Context(L, wl["block"], wl["kappa"], wl["csw"])
        ctx.load_gauge(U)
        r, z = ctx.fine(12, mglma.F32), ctx.fine(12, mglma.F32)
        r.copy_(torch.randn(r.shape, device="cuda"))
        z.zero_()
        nmr = mixed_params(mglma).sap_mr
        ctx.sap_smooth(r, z, 5, nmr, mglma.F16)
        torch.cuda.synchronize()
        print(json.dumps({"sap_only": True, "V": ctx.V, "launches": "10 SAP half-sweeps, 12 rhs, %d block steps" % nmr}))
        return
    if args.dslash_only:
        L = wl["L"]
        U = torch.from_numpy(synth.gauge_field(L, wl["eps"], wl["seed"]).view(np.float64)).cuda()
        ctx = mglma.Context(L, wl["block"], wl["kappa"], wl["csw"])
        ctx.load_gauge(U)
        for prec, nr in [(mglma.F16, 12), (mglma.F32, 12), (mglma.F64, 1), (mglma.F32, 1), (mglma.F16, 1)]:
            x, y = ctx.fine(nr, prec), ctx.fine(nr, prec)
            x.copy_(torch.randn(x.shape, device="cuda").to(x.dtype))
            for _ in range(5):
                ctx.apply_D(x, y, prec)
        torch.cuda.synchronize()
        print(json.dumps({"dslash_only": True, "V": ctx.V,
                          "launches": "5 x (f16 12rhs, f32 12rhs, f64 1rhs, f32 1rhs, f16 1rhs)"}))
        return
    P = Pipeline(wl)
    stream = torch.cuda.current_stream()
    params = mixed_params(mglma)
    for _ in range(args.warmup):
        P.step(params)
    torch.cuda.synchronize()
    lat = []
    stats = levels = None
    # the dominant kernel's launches are timed with HIP events on the
    # library's stream over the timed steps
    P.ctx.sap_timing(True)
    t_all0 = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        stats, levels = P.step(params)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    t_all = time.perf_counter() - t_all0
    sap_ms_total, sap_launches = P.ctx.sap_elapsed()
    P.ctx.sap_timing(False)
    nsolve = 12 * args.steps
    value = nsolve / t_all
    res = max(s["true_rel_res"] for s in stats)
    log("mixed: %.3f s/step, max true rel res %.2e, outer %s inner %s" % (
        t_all / args.steps, res, [s["outer"] for s in stats][:1], [s["inner"] for s in stats][:1]))
    out = {}
    # FP64 comparison (same pipeline, every precision FP64)
    fp64 = None
    if not args.no_fp64:
        t0 = time.perf_counter()
        st64, lv64 = P.step(fp64_params(mglma))
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        fp64 = dict(solves_per_s=12 / t64, s_per_step=t64, max_true_rel_res=max(s["true_rel_res"] for s in st64),
                    corr_L0_rel_diff_vs_mixed=float(np.linalg.norm(lv64["L0"] - levels["L0"]) /
                                                    np.linalg.norm(lv64["L0"])))
        log("fp64: %.3f s/step" % t64)
    # Wilson-clover applies (the metric's Dslash GB/s) and the dominant kernel
    # of the step, the SAP half-sweep of the smoother on the 12-RHS batch.
    # HIP events on the library's stream.
    ctx = P.ctx
    V = ctx.V
    nr = 12
    sr, sz = ctx.fine(nr, mglma.F32), ctx.fine(nr, mglma.F32)
    sr.copy_(torch.randn(sr.shape, device="cuda"))
    sz.zero_()
    nmr = params.sap_mr
    # in the timed steps (above), and for reference 20 launches back to back
    # inside one library call
    ms_sap = sap_ms_total / max(sap_launches, 1)
    ms_sap_b2b = kernel_time(torch, lambda: ctx.sap_smooth(sr, sz, 10, nmr, mglma.F16), 3, stream) / 20
    sap_flops = sap_alg_flops(V, wl["block"], wl["L"], nr, nmr)
    ach_sap = sap_flops / (ms_sap * 1e-3) / 1e12
    del sr, sz

    def apply_ms(prec, nrhs):
        x = ctx.fine(nrhs, prec)
        y = ctx.fine(nrhs, prec)
        x.copy_(torch.randn(x.shape, device="cuda").to(x.dtype))
        return kernel_time(torch, lambda: ctx.apply_D(x, y, prec), 20, stream)

    n_plain_it = plain_gcr_iterations(P, mglma) if not args.no_cpu else None
    ms16 = apply_ms(mglma.F16, nr)
    ms32 = apply_ms(mglma.F32, nr)
    ms64_1 = apply_ms(mglma.F64, 1)
    ms32_1 = apply_ms(mglma.F32, 1)
    ms16_1 = apply_ms(mglma.F16, 1)
    dslash_gbs = {
        "f16_12rhs": dslash_alg_bytes(V, nr, 2) / (ms16 * 1e-3) / 1e9,
        "f32_12rhs": dslash_alg_bytes(V, nr, 4) / (ms32 * 1e-3) / 1e9,
        "f64_1rhs": dslash_alg_bytes(V, 1, 8) / (ms64_1 * 1e-3) / 1e9,
        "f32_1rhs": dslash_alg_bytes(V, 1, 4) / (ms32_1 * 1e-3) / 1e9,
        "f16_1rhs": dslash_alg_bytes(V, 1, 2) / (ms16_1 * 1e-3) / 1e9,
    }
    traffic16 = measured_traffic(args.workload)
    traffic_sap = measured_sap_traffic(args.workload)
    # bounded serving leg (continuous batching): the step's context is freed
    # first; two resident ensembles, 12 requests one at a time for the
    # isolated service rate and a Poisson stream of 40 requests at 0.8 of it
    eig_info = P.eig
    serve = None
    if not args.no_serve:
        P.ctx.close()
        del P
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        serve = serving(reqs_n=40, iso_n=12, max_src=8, emit=False)
    cpu = None
    if not args.no_cpu:
        n_plain, res_plain = n_plain_it
        log("plain FP64 GCR(16): %d iterations to %.2e" % (n_plain, res_plain))
        cpu = cpu_baseline(wl, n_plain, args.cpu_budget)
    L = wl["L"]
    line = {
        "metric": "MG solves/s to rel. residual 1e-10 (mixed vs FP64); Dslash HBM GB/s; p50/p99 latency",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_all / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 Krylov + SAP smoother (f32, f16 links) + bf16 coarse, f64 outer",
        "data": "synthetic",
        "config": {"workload": "%dx%d^3 Wilson-clover, eps=%g, kappa=%g, c_sw=%g, %d^4 blocks, Nv=%d, Nlm=%d, "
                               "12 point-source RHS batched, mixed-precision MG-GCR to 1e-10" %
                               (L[0], L[1], wl["eps"], wl["kappa"], wl["csw"], wl["block"][0], wl["Nv"], wl["Nlm"]),
                   "lattice": list(L), "block": list(wl["block"]), "nrhs": 12},
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "unit": "s per 12-RHS step"},
        "serving": serve,
        "max_true_rel_res": res,
        "fp64_path": fp64,
        "speedup_mixed_vs_fp64": (value / fp64["solves_per_s"]) if fp64 else None,
        "dslash_GBs": dslash_gbs,
        "roofline": {"bound": "alu", "kernel": "k_sap_half<__half2, 3> (SAP half-sweep, 12 RHS, %d block steps)" % nmr,
                     "achieved": ach_sap, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach_sap / FP32_PEAK_TFLOPS, "traffic": traffic_sap, "avg_ms": ms_sap,
                     "peak_kind": "MI355X published FP32 vector peak",
                     "peak_nonpacked": FP32_NONPACKED_TFLOPS, "frac_nonpacked": ach_sap / FP32_NONPACKED_TFLOPS,
                     "peak_nonpacked_kind": "FP32 FMA without packed FP32 instructions (the library's build): "
                                            "256 CUs x 64 lanes x 2 flop x 2.4 GHz",
                     "launches_timed": sap_launches, "avg_ms_back_to_back": ms_sap_b2b,
                     "alg_flops_per_launch": sap_flops},
        # the Wilson-clover multi-RHS apply, HBM-bound (Dslash HBM GB/s of the metric)
        "roofline_dslash": {"bound": "hbm", "kernel": "k_dslash_h<3> (FP16 storage, FP32 sums, 12 RHS)",
                            "achieved": dslash_gbs["f16_12rhs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": dslash_gbs["f16_12rhs"] / HBM_PEAK_GBS, "traffic": traffic16,
                            "avg_ms": ms16, "alg_bytes_per_launch": dslash_alg_bytes(V, nr, 2)},
        "cpu_baseline": cpu,
        "top_modes_setup": eig_info,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
