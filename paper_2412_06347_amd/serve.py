"""Request loop serving multigrid low-mode-averaging estimates on one GPU.

Each *ensemble* (one lattice volume with its gauge field) keeps its context
resident: links, clover term, block basis, Galerkin operator, coarse gammas
and top level stay in HBM for its lifetime.  A request asks for the
translation-averaged correlator from `n_src` stochastic time-diluted,
spin-diluted wall sources (4 right-hand sides each, section "Stochastic
estimator on level k") and receives the level terms G_L0, G_L1 (stochastic,
eq:C_stoch with the level sums) and G_L2 (exact, eq:G_LL:exact).

Continuous batching: every ensemble has a worker thread with its own HIP
stream and a pool of resident right-hand-side slots in the library
(mglma_slots_*).  The worker loops over outer cycles of the multigrid solve:
before each cycle it admits queued requests whose right-hand sides fit the
free slots (their sources and coarse pieces are formed and loaded into the
pool), runs one cycle for every running right-hand side (at most one FGCR
restart cycle), and completes each request whose right-hand sides have all
converged (solutions taken from the pool, level terms contracted in the
library), which frees its slots for the queue.  A request that arrives while
others are on the GPU therefore starts at the next cycle, not after the
running ones finish.  Workers of different ensembles run concurrently, so
their kernels overlap on the device.  Every right-hand side follows the
arithmetic of a solve alone (per-rhs Krylov scalars, fixed-order reductions,
frozen once converged), so a request's result does not depend on what ran
beside it.

Admission: ensembles are admitted while their resident bytes plus the
workspace of their slot pool fit the HBM budget; the request at the head of
an ensemble's queue joins with as many of its sources as fit the free slots
(4 right-hand sides per source) and keeps the head until all have joined, so
a request larger than the pool is solved in parts whose level terms are
added to its source mean in the library (mglma_contract_levels_acc).
"""
from __future__ import annotations

import collections
import dataclasses
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
    joined_running: int = 0          # requests already running when this one was admitted
    next_src: int = 0                # sources admitted so far (a request may join in parts)
    done_src: int = 0                # sources whose solves have finished
    work: Optional[dict] = None      # the engine's per-request state while running
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


def workspace_bytes_per_rhs(V, gcr_m=6):
    """Device bytes per right-hand side slot: b, x and the FP64 residual held
    by the slot (3 FP64 fine fields), the FGCR directions and preconditioned
    vectors with the inner residual, correction and smoother vectors (2 gcr_m
    + 4 FP32 fields), the FP64 apply of the outer cycle, and the source and
    its coarse pieces while a request is admitted (3 FP64 fields)."""
    return V * 12 * (3 * 16 + (2 * gcr_m + 4) * 8 + 16 + 3 * 16)


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
            # test vectors: Gaussian fields improved by three rounds of 40
            # unpreconditioned FP32 GCR steps, in batches that fit the device
            x = ctx.fine(Nv)
            for k0 in range(0, Nv, 8):
                k1 = min(Nv, k0 + 8)
                tv = synth.gaussian_fields(k1 - k0, L, wl["seed"] + 1000 + k0)
                ctx.import_fields(torch.from_numpy(tv.view(np.float64)).cuda(), x[k0:k1])
                del tv
            nb = int(wl.get("tv_batch", Nv))
            y = ctx.fine(nb)
            p = mglma.default_params(use_mg=0, inner=mglma.F32, max_outer=1, max_inner=40, gcr_m=16 if nb == Nv else 8,
                                     tol=1e-30, inner_tol=1e-30)
            for _ in range(3):
                for k0 in range(0, Nv, nb):
                    k1 = min(Nv, k0 + nb)
                    ctx.solve(x[k0:k1], y[:k1 - k0], p, raise_on_error=False)
                    nrm = torch.linalg.vector_norm(y[:k1 - k0].reshape(k1 - k0, -1), dim=1)
                    x[k0:k1] = y[:k1 - k0] / nrm[:, None, None, None]
            del y
            ctx.release_workspace()
            ctx.build_subspace(x)
            del x
            # top level: the Nlm lowest eigenvectors of Q_1 (device eigensolver)
            init = torch.from_numpy(synth.gaussian_coarse(min(2 * Nlm, Nlm + 32), ctx.V1, ctx.nc,
                                                          wl["seed"] + 4242).view(np.float64))
            rc, lam, m, st = ctx.coarse_eigs(init.cuda(), Nlm, tol=1e-12, max_iter=int(wl.get("eig_iter", 100)),
                                             raise_on_error=False)
            ctx.set_top_modes(m.contiguous())
            del m, init
            self.G_top = ctx.contract_top()
            # the setup's workspaces (batched GCR, eigensolver) are not needed
            # by the requests: give them back before the ensemble is admitted
            ctx.release_workspace()
        self.stream.synchronize()
        # SAP smoothing (FGCR(6), 2 cycles of 4 block steps) where the block
        # grid allows it (every extent even or one), CA-GCR(6) otherwise
        grid = [L[mu] // wl["block"][mu] for mu in range(4)]
        if all(e == 1 or e % 2 == 0 for e in grid) and int(np.prod(wl["block"])) <= 256:
            smooth = dict(gcr_m=6, nu_post=2, sap_mr=4, smoother_alg=mglma.SMOOTH_SAP)
        else:
            smooth = dict(gcr_m=4, nu_post=6, smoother_alg=mglma.SMOOTH_CAGCR)
        # an outer cycle is one FGCR restart cycle (max_inner = gcr_m): the
        # granularity at which right-hand sides join and leave the pool
        self.params = params or mglma.default_params(tol=1e-10, max_outer=60, max_inner=smooth["gcr_m"],
                                                     inner_tol=1e-5, coarse_iters=4, smoother=mglma.F16,
                                                     inner=mglma.F32, coarse=mglma.BF16, coarse_eo=1, **smooth)
        self.pool = None
        self.coarse_params = coarse_params or mglma.default_params(tol=1e-10, coarse=mglma.BF16, coarse_iters=12,
                                                                   max_outer=40, coarse_eo=1)
        self.resident = ctx.resident_bytes() + self.U.numel() * 8

    @property
    def V(self):
        return self.ctx.V

    # -- continuous batching through the library's slot pool -----------------
    def open_pool(self, nslots):
        self.pool = self.mglma.Slots(self.ctx, nslots)

    def _noise(self, r):
        """The request's seeded sources (all of them, drawn once)."""
        if r.work is None:
            L = self.L
            r.work = dict(xi=np.ascontiguousarray(self.synth.z4_noise(r.n_src, L, r.seed)),
                          tn=self.synth.time_slices(r.n_src, L[0], r.seed), acc=None, stats=[])
        return r.work

    def _pieces(self, xi, tn):
        torch, ctx = self.torch, self.ctx
        xid = torch.from_numpy(np.ascontiguousarray(xi).view(np.float64)).cuda()
        eta = ctx.fine(4 * len(tn))
        ctx.noise_sources(xid, tn, eta)
        cg, ct = ctx.coarse(4 * len(tn)), ctx.coarse(4 * len(tn))
        ctx.coarse_pieces(eta, cg, ct, self.coarse_params)
        return eta, cg, ct

    def admit(self, parts):
        """parts: (request, first source, end source) admitted together; their
        sources and coarse pieces are formed and the right-hand sides join the
        pool."""
        with self.torch.cuda.stream(self.stream):
            xi = np.concatenate([self._noise(r)["xi"][a:b] for r, a, b in parts])
            tn = np.concatenate([r.work["tn"][a:b] for r, a, b in parts])
            eta, cg, ct = self._pieces(xi, tn)
            ids = self.pool.load(eta)
        out, k = [], 0
        for r, a, b in parts:
            n = 4 * (b - a)
            out.append(dict(req=r, a=a, b=b, ids=ids[k:k + n], tn=tn[k // 4:k // 4 + b - a], cg=cg[k:k + n],
                            ct=ct[k:k + n]))
            k += n
        return out

    def step(self):
        """One outer cycle of every running right-hand side; slot states."""
        with self.torch.cuda.stream(self.stream):
            return self.pool.step(self.params)

    def done(self, part, status):
        return all(status[i] != 1 for i in part["ids"])

    def finish(self, part):
        """Take a part's solutions from the pool and add its level terms to the
        request's source mean (in the library); returns the request's result
        once every source is done, else None."""
        r = part["req"]
        w = r.work
        with self.torch.cuda.stream(self.stream):
            x = self.ctx.fine(len(part["ids"]))
            st = self.pool.take(part["ids"], x)
            bad = [q["status"] for q in st if q["status"] != 0]
            if bad:
                raise RuntimeError("request %d: solve failed (status %d)" % (r.rid, bad[0]))
            if w["acc"] is None:
                w["acc"] = self.torch.empty((3, self.L[0], 2), dtype=self.torch.float64, device="cuda")
            self.ctx.contract_levels_acc(self.mglma.SRC_STOCH, part["tn"], w["acc"], 1.0 / r.n_src,
                                         r.done_src > 0, fine=x, coarse=[part["cg"], part["ct"]])
            w["stats"] += st
            r.done_src += part["b"] - part["a"]
            if r.done_src < r.n_src:
                return None
            lv = w["acc"].cpu().numpy()
        lv = lv[..., 0] + 1j * lv[..., 1]
        res = self._result(lv, w["stats"])
        r.work = None
        return res

    def _result(self, lv, st):
        return dict(L0=lv[0], L1=lv[1], L2=self.G_top.copy(), G=lv[0] + lv[1] + self.G_top,
                    max_true_rel_res=max(q["true_rel_res"] for q in st), inner=max(q["inner"] for q in st))

    def run(self, reqs: List[Request]) -> List[dict]:
        """The requests solved on their own (mglma_solve with the same
        settings, all sources of a request at once), for comparisons with the
        results of the request loop."""
        out = []
        with self.torch.cuda.stream(self.stream):
            for r in reqs:
                xi = self.synth.z4_noise(r.n_src, self.L, r.seed)
                tn = self.synth.time_slices(r.n_src, self.L[0], r.seed)
                eta, cg, ct = self._pieces(xi, tn)
                x = self.ctx.fine(4 * r.n_src)
                rc, st = self.ctx.solve(eta, x, self.params)
                lv = self.ctx.contract_levels(self.mglma.SRC_STOCH, tn, fine=x, coarse=[cg, ct])
                out.append(self._result(lv, st))
        self.stream.synchronize()
        return out


class Server:
    """Continuous-batching request loop over several resident ensembles.

    engine_factory(name, wl) builds the GPU side of an ensemble (open_pool,
    admit, step, done, finish); tests of the host logic pass a stand-in.
    `batches` records, per outer cycle of an ensemble, the requests that
    shared it."""

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
        eng.open_pool(slots)
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
            if n_src < 1 or self.slots[ensemble] < 4:
                raise AdmissionError("request of %d sources on ensemble %s with %d slots"
                                     % (n_src, ensemble, self.slots[ensemble]))
            self._rid += 1
            r = Request(self._rid, ensemble, int(n_src), int(seed), time.perf_counter())
            self.queues[ensemble].append(r)
            self.cv.notify_all()
            return r

    def _admit_from_queue(self, name, free):
        """Parts (request, first source, end source) that fit `free` slots, in
        arrival order; a request larger than the free slots joins in parts
        and keeps the head of the queue until all its sources are in."""
        q = self.queues[name]
        parts = []
        while q and free >= 4:
            r = q[0]
            k = min(r.n_src - r.next_src, free // 4)
            parts.append((r, r.next_src, r.next_src + k))
            r.next_src += k
            free -= 4 * k
            if r.next_src == r.n_src:
                q.popleft()
        return parts

    def _complete(self, reqs, results, err):
        t1 = time.perf_counter()
        with self.cv:
            for r, res in zip(reqs, results):
                if r.done.is_set():
                    continue
                r.result, r.error, r.t_done = res, err, t1
                self.completed.append(r)
                r.done.set()

    def _worker(self, name):
        eng = self.engines[name]
        running = []            # parts on the GPU
        failed = set()
        while True:
            with self.cv:
                while self.running and not self.queues[name] and not running:
                    self.cv.wait(0.05)
                if not self.running and not self.queues[name] and not running:
                    return
                free = self.slots[name] - sum(4 * (b - a) for (_, a, b) in (p["key"] for p in running))
                admitted = self._admit_from_queue(name, free)
            if admitted:
                t0 = time.perf_counter()
                n_run = len({id(p["req"]) for p in running})
                for r, a, b in admitted:
                    if a == 0:
                        r.t_start = t0
                        r.joined_running = n_run
                try:
                    for p, key in zip(eng.admit(admitted), admitted):
                        p["key"] = key
                        running.append(p)
                except BaseException as e:   # a failing admission fails its requests, not the server
                    bad = [r for r, _, _ in admitted]
                    failed |= {r.rid for r in bad}
                    self._complete(bad, [None] * len(bad), e)
            if not running:
                continue
            try:
                status = eng.step()
            except BaseException as e:
                reqs = list({id(p["req"]): p["req"] for p in running}.values())
                failed |= {r.rid for r in reqs}
                self._complete(reqs, [None] * len(reqs), e)
                running = []
                continue
            with self.cv:
                self.batches.append(sorted({p["req"].rid for p in running}))
            still = []
            for p in running:
                r = p["req"]
                if not eng.done(p, status):
                    still.append(p)
                    continue
                try:
                    res = eng.finish(p)
                    if res is not None and r.rid not in failed:
                        self._complete([r], [res], None)
                except BaseException as e:
                    failed.add(r.rid)
                    self._complete([r], [None], e)
            running = still

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
                    cycles=len(self.batches))


def poisson_arrivals(n, rate, seed):
    """Arrival times of a Poisson stream (rate per second), seeded."""
    g = np.random.default_rng(seed)
    return np.cumsum(g.exponential(1.0 / rate, size=n))
