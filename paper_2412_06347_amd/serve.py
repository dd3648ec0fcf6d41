"""Request loop serving multigrid low-mode-averaging estimates on one GPU.

Each *ensemble* (one lattice volume with its gauge field) keeps its context
resident: links, clover term, block basis, Galerkin operator, coarse gammas
and top level stay in HBM for its lifetime.  A request asks for the
translation-averaged correlator from `n_src` stochastic time-diluted,
spin-diluted wall sources (4 right-hand sides each, section "Stochastic
estimator on level k") and receives the level terms G_L0, G_L1 (stochastic,
eq:C_stoch with the level sums) and G_L2 (exact, eq:G_LL:exact).

Batching: every ensemble has a worker thread with its own HIP stream.  While
a batch of that ensemble is on the GPU, newly arriving requests wait in its
queue; when the batch retires, the worker admits as many queued requests as
fit the ensemble's right-hand-side slots and HBM share into the next
multi-right-hand-side batch.  Workers of different ensembles run
concurrently, so their kernels overlap on the device.  Every right-hand side
follows the same arithmetic alone or in a batch (per-rhs Krylov scalars,
fixed-order reductions, frozen once converged), so a request's result does
not depend on what it was batched with.

Admission: ensembles are admitted while their resident bytes plus the
workspace of their largest batch fit the HBM budget; a batch is formed only
from requests whose right-hand sides fit the ensemble's slot count.
"""
from __future__ import annotations

import collections
import dataclasses
import queue
import threading
import time
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    ensemble: str
    n_src: int
    seed: int
    t_arrival: float
    t_start: float = 0.0
    t_done: float = 0.0
    result: Optional[dict] = None
    error: Optional[BaseException] = None
    done: threading.Event = dataclasses.field(default_factory=threading.Event)

    @property
    def nrhs(self):
        return 4 * self.n_src

    def wait(self, timeout=None):
        if not self.done.wait(timeout):
            raise TimeoutError("request %d not finished" % self.rid)
        if self.error is not None:
            raise self.error
        return self.result


class AdmissionError(RuntimeError):
    pass


def workspace_bytes_per_rhs(V, gcr_m=8, nu_post=6):
    """Device bytes the solve needs per right-hand side: 2*gcr_m + 8 FP32 and
    8 FP64 fine fields (Krylov directions, residuals, smoother, outputs) and
    the nu_post + 1 FP16 Krylov basis vectors of the CA-GCR smoother."""
    return V * 12 * ((2 * gcr_m + 8) * 8 + 8 * 16 + (nu_post + 1) * 4)


class Engine:
    """GPU side of one ensemble (all compute through the C ABI)."""

    def __init__(self, name, wl, params=None, coarse_params=None):
        import torch
        from paper_2412_06347_amd import mglma, synth
        self.torch, self.mglma, self.synth = torch, mglma, synth
        self.name, self.wl = name, wl
        self.stream = torch.cuda.Stream()
        L = tuple(wl["L"])
        self.L = L
        with torch.cuda.stream(self.stream):
            U = synth.gauge_field(L, wl["eps"], wl["seed"])
            self.U = torch.from_numpy(U.view(np.float64)).cuda()
            del U
            ctx = mglma.Context(L, wl["block"], wl["kappa"], wl["csw"], stream=self.stream)
            self.ctx = ctx
            ctx.load_gauge(self.U)
            Nv, Nlm = wl["Nv"], wl["Nlm"]
            tv = synth.gaussian_fields(Nv, L, wl["seed"] + 1000)
            x = ctx.fine(Nv)
            ctx.import_fields(torch.from_numpy(tv.view(np.float64)).cuda(), x)
            y = ctx.fine(Nv)
            p = mglma.default_params(use_mg=0, inner=mglma.F32, max_outer=1, max_inner=40, gcr_m=16, tol=1e-30,
                                     inner_tol=1e-30)
            for _ in range(3):
                ctx.solve(x, y, p, raise_on_error=False)
                nrm = torch.linalg.vector_norm(y.reshape(Nv, -1), dim=1)
                x = (y / nrm[:, None, None, None]).contiguous()
            del y
            ctx.build_subspace(x)
            del x
            # top level: the Nlm lowest eigenvectors of Q_1 (device eigensolver)
            init = torch.from_numpy(synth.gaussian_coarse(2 * Nlm, ctx.V1, ctx.nc, wl["seed"] + 4242).view(np.float64))
            rc, lam, m, st = ctx.coarse_eigs(init.cuda(), Nlm, tol=1e-12)
            ctx.set_top_modes(m.contiguous())
            self.G_top = ctx.contract_top()
        self.stream.synchronize()
        # SAP smoothing (FGCR(6), 2 cycles of 4 block steps) where the block
        # grid allows it (every extent even or one), CA-GCR(6) otherwise
        grid = [L[mu] // wl["block"][mu] for mu in range(4)]
        if all(e == 1 or e % 2 == 0 for e in grid) and int(np.prod(wl["block"])) <= 256:
            smooth = dict(gcr_m=6, nu_post=2, sap_mr=4, smoother_alg=mglma.SMOOTH_SAP)
        else:
            smooth = dict(gcr_m=4, nu_post=6, smoother_alg=mglma.SMOOTH_CAGCR)
        self.params = params or mglma.default_params(tol=1e-10, max_outer=10, max_inner=120, inner_tol=1e-5,
                                                     coarse_iters=4, smoother=mglma.F16, inner=mglma.F32,
                                                     coarse=mglma.BF16, coarse_eo=1, **smooth)
        self.coarse_params = coarse_params or mglma.default_params(tol=1e-10, coarse=mglma.BF16, coarse_iters=12,
                                                                   max_outer=40, coarse_eo=1)
        self.resident = ctx.resident_bytes() + self.U.numel() * 8

    @property
    def V(self):
        return self.ctx.V

    def run(self, reqs: List[Request]) -> List[dict]:
        torch, mglma, synth = self.torch, self.mglma, self.synth
        ctx, L = self.ctx, self.L
        nsrc = sum(r.n_src for r in reqs)
        with torch.cuda.stream(self.stream):
            xi = np.concatenate([synth.z4_noise(r.n_src, L, r.seed) for r in reqs])
            tn = np.concatenate([synth.time_slices(r.n_src, L[0], r.seed) for r in reqs])
            xid = torch.from_numpy(np.ascontiguousarray(xi).view(np.float64)).cuda()
            eta = ctx.fine(4 * nsrc)
            ctx.noise_sources(xid, tn, eta)
            x = ctx.fine(4 * nsrc)
            rc, stats = ctx.solve(eta, x, self.params)
            cg, ct = ctx.coarse(4 * nsrc), ctx.coarse(4 * nsrc)
            ctx.coarse_pieces(eta, cg, ct, self.coarse_params)
            out, k = [], 0
            for r in reqs:
                # level terms and source mean in the library (eq:C_stoch)
                s = slice(4 * k, 4 * (k + r.n_src))
                lv = ctx.contract_levels(mglma.SRC_STOCH, tn[k:k + r.n_src], fine=x[s], coarse=[cg[s], ct[s]])
                L0, L1 = lv[0], lv[1]
                st = stats[4 * k: 4 * (k + r.n_src)]
                out.append(dict(L0=L0, L1=L1, L2=self.G_top.copy(), G=L0 + L1 + self.G_top,
                                max_true_rel_res=max(q["true_rel_res"] for q in st),
                                inner=max(q["inner"] for q in st)))
                k += r.n_src
        self.stream.synchronize()
        return out


class Server:
    """Continuous-batching request loop over several resident ensembles.

    engine_factory(name, wl) builds the GPU side of an ensemble; tests of the
    host logic pass a stand-in."""

    def __init__(self, hbm_budget: float, max_batch_rhs: int = 48,
                 engine_factory: Callable = Engine, bytes_per_rhs: Callable = workspace_bytes_per_rhs):
        self.budget = float(hbm_budget)
        self.max_batch_rhs = int(max_batch_rhs)
        self.factory = engine_factory
        self.bytes_per_rhs = bytes_per_rhs
        self.engines: Dict[str, object] = {}
        self.slots: Dict[str, int] = {}
        self.queues: Dict[str, collections.deque] = {}
        self.cv = threading.Condition()
        self.used = 0.0
        self.threads: List[threading.Thread] = []
        self.running = False
        self.completed: List[Request] = []
        self.batches: List[List[int]] = []
        self._rid = 0
        self.t_start = None

    # -- ensembles ---------------------------------------------------------
    def add_ensemble(self, name, wl, max_rhs=None):
        eng = self.factory(name, wl)
        slots = self.max_batch_rhs if max_rhs is None else int(max_rhs)
        per = self.bytes_per_rhs(eng.V)
        # shrink the slot count until resident + workspace fits the budget
        while slots > 0 and self.used + eng.resident + slots * per > self.budget:
            slots -= 4
        if slots <= 0:
            raise AdmissionError("ensemble %s does not fit the HBM budget (%.2f GB resident, %.2f GB per rhs, "
                                 "%.2f GB left)" % (name, eng.resident / 1e9, per / 1e9, (self.budget - self.used) / 1e9))
        with self.cv:
            self.engines[name] = eng
            self.slots[name] = slots
            self.queues[name] = collections.deque()
            self.used += eng.resident + slots * per
            if self.running:
                self._spawn(name)
        return slots

    # -- requests ------------------------------------------------------------
    def submit(self, ensemble, n_src, seed) -> Request:
        with self.cv:
            if ensemble not in self.engines:
                raise KeyError(ensemble)
            if 4 * n_src > self.slots[ensemble]:
                raise AdmissionError("request needs %d right-hand sides, ensemble %s has %d slots"
                                     % (4 * n_src, ensemble, self.slots[ensemble]))
            self._rid += 1
            r = Request(self._rid, ensemble, int(n_src), int(seed), time.perf_counter())
            self.queues[ensemble].append(r)
            self.cv.notify_all()
            return r

    def _take_batch(self, name):
        q = self.queues[name]
        batch, rhs = [], 0
        while q and rhs + q[0].nrhs <= self.slots[name]:
            r = q.popleft()
            batch.append(r)
            rhs += r.nrhs
        return batch

    def _worker(self, name):
        eng = self.engines[name]
        while True:
            with self.cv:
                while self.running and not self.queues[name]:
                    self.cv.wait(0.05)
                if not self.running and not self.queues[name]:
                    return
                batch = self._take_batch(name)
            if not batch:
                continue
            t0 = time.perf_counter()
            for r in batch:
                r.t_start = t0
            try:
                results = eng.run(batch)
                err = None
            except BaseException as e:  # a failing batch fails its requests, not the server
                results, err = [None] * len(batch), e
            t1 = time.perf_counter()
            with self.cv:
                self.batches.append([r.rid for r in batch])
                for r, res in zip(batch, results):
                    r.result, r.error, r.t_done = res, err, t1
                    self.completed.append(r)
                    r.done.set()

    def _spawn(self, name):
        th = threading.Thread(target=self._worker, args=(name,), daemon=True)
        th.start()
        self.threads.append(th)

    def start(self):
        with self.cv:
            self.running = True
            self.t_start = time.perf_counter()
            for name in self.engines:
                self._spawn(name)

    def stop(self):
        with self.cv:
            self.running = False
            self.cv.notify_all()
        for th in self.threads:
            th.join()
        self.threads = []

    # -- statistics ---------------------------------------------------------
    def stats(self):
        done = [r for r in self.completed if r.error is None]
        if not done:
            return dict(n=0)
        lat = np.array([r.t_done - r.t_arrival for r in done])
        t0 = min(r.t_arrival for r in done)
        t1 = max(r.t_done for r in done)
        solves = sum(r.nrhs for r in done)
        return dict(n=len(done), solves=solves, wall_s=t1 - t0, solves_per_s=solves / max(t1 - t0, 1e-9),
                    p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                    batches=len(self.batches))


def poisson_arrivals(n, rate, seed):
    """Arrival times of a Poisson stream (rate per second), seeded."""
    g = np.random.default_rng(seed)
    return np.cumsum(g.exponential(1.0 / rate, size=n))
