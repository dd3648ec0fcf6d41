"""Thin ctypes binding of libmglma.so (argument marshalling only).

Every computation runs in the HIP library; this module only passes device
pointers (``torch.Tensor.data_ptr()``), sizes and the current HIP stream.  It
raises if the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmglma.so")

F64, F32, F16, BF16 = 0, 1, 2, 3
SRC_POINT, SRC_STOCH = 0, 1
OP_FINE, OP_COARSE, OP_LEVEL2, OP_NONCHIRAL = 0, 1, 2, 3
SMOOTH_MR, SMOOTH_CAGCR, SMOOTH_SAP = 0, 1, 2

SYMBOLS = [
    "mglma_create", "mglma_destroy", "mglma_set_stream", "mglma_strerror", "mglma_query",
    "mglma_resident_bytes", "mglma_fine_bytes", "mglma_coarse_bytes",
    "mglma_load_gauge", "mglma_export_clover", "mglma_import_fields", "mglma_export_fields",
    "mglma_apply_D", "mglma_build_subspace", "mglma_export_basis", "mglma_export_coarse_op",
    "mglma_export_coarse_gammas",
    "mglma_restrict", "mglma_prolong", "mglma_coarse_apply", "mglma_set_top_modes",
    "mglma_solve", "mglma_coarse_solve", "mglma_coarse_pieces",
    "mglma_point_sources", "mglma_noise_sources",
    "mglma_contract_point", "mglma_contract_point_coarse", "mglma_contract_stoch",
    "mglma_contract_stoch_coarse", "mglma_contract_top", "mglma_coarse_eigs", "mglma_fine_eigs",
    "mglma_deficit", "mglma_coarse_schur_apply",
    "mglma_build_level2", "mglma_export_level2_op", "mglma_level2_restrict", "mglma_level2_prolong",
    "mglma_level2_apply", "mglma_level2_solve", "mglma_level2_pieces", "mglma_save", "mglma_load",
    "mglma_adaptive_setup", "mglma_sap_smooth", "mglma_sap_timing", "mglma_sap_elapsed",
    "mglma_contract_pair", "mglma_contract_levels", "mglma_contract_levels_noalloc",
    "mglma_contract_levels_acc", "mglma_release_workspace", "mglma_level_eigs", "mglma_build_nonchiral",
    "mglma_export_nonchiral_op", "mglma_slots_create", "mglma_slots_destroy", "mglma_slots_load", "mglma_slots_step", "mglma_slots_take",
]


class Lattice(C.Structure):
    _fields_ = [("L", C.c_int * 4), ("block", C.c_int * 4), ("kappa", C.c_double),
                ("csw", C.c_double), ("bc", C.c_double * 4)]


class SolveParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_outer", C.c_int), ("max_inner", C.c_int),
                ("gcr_m", C.c_int), ("inner_tol", C.c_double), ("nu_post", C.c_int),
                ("coarse_iters", C.c_int), ("smoother", C.c_int), ("inner", C.c_int),
                ("coarse", C.c_int), ("use_mg", C.c_int), ("smoother_alg", C.c_int),
                ("coarse_eo", C.c_int), ("kcycle", C.c_int), ("kcycle_nu", C.c_int),
                ("sap_mr", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("outer", C.c_int), ("inner", C.c_int), ("coarse", C.c_int),
                ("true_rel_res", C.c_double), ("seconds", C.c_double), ("status", C.c_int)]


class EigParams(C.Structure):
    _fields_ = [("nev", C.c_int), ("nguard", C.c_int), ("degree", C.c_int), ("max_iter", C.c_int),
                ("tol", C.c_double), ("out_block", C.c_int)]


class EigStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("applies", C.c_int), ("nconv", C.c_int), ("max_res", C.c_double),
                ("spectrum_bound", C.c_double), ("seconds", C.c_double), ("lambda_max_abs", C.c_double)]


class MglmaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("mglma error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmglma.so not built (run __graft_entry__.build() or "
                              "python -m paper_2412_06347_amd.build)")
        L = C.CDLL(LIB_PATH)
        L.mglma_strerror.restype = C.c_char_p
        L.mglma_query.restype = C.c_long
        L.mglma_resident_bytes.restype = C.c_size_t
        L.mglma_fine_bytes.restype = C.c_size_t
        L.mglma_coarse_bytes.restype = C.c_size_t
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise MglmaError(rc, lib().mglma_strerror(rc).decode())
    return rc


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def default_params(**kw):
    p = SolveParams(tol=1e-10, max_outer=12, max_inner=200, gcr_m=16, inner_tol=1e-5,
                    nu_post=4, coarse_iters=16, smoother=F32, inner=F32, coarse=F32, use_mg=1,
                    smoother_alg=SMOOTH_MR, coarse_eo=1, kcycle=0, kcycle_nu=2, sap_mr=4)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class Context:
    """One lattice + its resident gauge field, subspace and top level."""

    def __init__(self, L, block, kappa, csw, bc=(-1.0, 1.0, 1.0, 1.0), stream=None):
        import torch
        self.L = tuple(int(x) for x in L)
        self.block = tuple(int(x) for x in block)
        lat = Lattice((C.c_int * 4)(*self.L), (C.c_int * 4)(*self.block), float(kappa),
                      float(csw), (C.c_double * 4)(*bc))
        self._ctx = C.c_void_p()
        _check(lib().mglma_create(C.byref(self._ctx), C.byref(lat), C.c_void_p(0)))
        self.set_stream(stream if stream is not None else torch.cuda.current_stream())

    def set_stream(self, stream):
        self.stream = stream
        _check(lib().mglma_set_stream(self._ctx, C.c_void_p(stream.cuda_stream)))

    def close(self):
        if self._ctx:
            lib().mglma_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- sizes ----------------------------------------------------------
    def query(self, what):
        return int(lib().mglma_query(self._ctx, what))

    @property
    def V(self):
        return self.query(0)

    @property
    def V1(self):
        return self.query(1)

    @property
    def nc(self):
        return self.query(4)

    @property
    def r(self):
        return self.query(6)

    def resident_bytes(self):
        return int(lib().mglma_resident_bytes(self._ctx))

    def release_workspace(self):
        """Free the workspaces kept between calls and the reuse list."""
        _check(lib().mglma_release_workspace(self._ctx))

    # ---- allocation helpers (device memory from torch) ------------------
    def fine(self, nrhs, prec=F64, device="cuda"):
        import torch
        per = {F64: torch.float64, F32: torch.float32, F16: torch.float16}[prec]
        return torch.empty((nrhs, 12, self.V, 2), dtype=per, device=device)

    def coarse(self, nrhs, device="cuda"):
        import torch
        return torch.empty((nrhs, self.V1, self.nc, 2), dtype=torch.float64, device=device)

    def coarse32(self, nrhs, device="cuda"):
        import torch
        return torch.empty((nrhs, self.V1, self.nc, 2), dtype=torch.float32, device=device)

    # ---- fine level -------------------------------------------------------
    def load_gauge(self, U):
        _check(lib().mglma_load_gauge(self._ctx, _ptr(U)))

    def export_clover(self, out):
        _check(lib().mglma_export_clover(self._ctx, _ptr(out)))

    def import_fields(self, canon, dev, prec=F64):
        _check(lib().mglma_import_fields(self._ctx, prec, _ptr(canon), _ptr(dev), canon.shape[0]))

    def export_fields(self, dev, canon, prec=F64):
        _check(lib().mglma_export_fields(self._ctx, prec, _ptr(dev), _ptr(canon), dev.shape[0]))

    def apply_D(self, x, y, prec=F64, gamma5=0):
        _check(lib().mglma_apply_D(self._ctx, prec, gamma5, _ptr(x), _ptr(y), x.shape[0]))

    # ---- subspace ---------------------------------------------------------
    def build_subspace(self, testvecs):
        _check(lib().mglma_build_subspace(self._ctx, testvecs.shape[0], _ptr(testvecs)))

    def adaptive_setup(self, testvecs, params=None, rounds=1, iters=8):
        """Refine the test vectors in place (inverse iteration with the current
        solver) and rebuild the subspace from them after every round."""
        _check(lib().mglma_adaptive_setup(self._ctx, C.byref(params or default_params()), _ptr(testvecs),
                                          testvecs.shape[0], int(rounds), int(iters)))

    def sap_smooth(self, r, z, ncycle=1, nmr=4, prec=F16):
        """ncycle SAP cycles on M z = r (FP32 device fields, z in place)."""
        _check(lib().mglma_sap_smooth(self._ctx, prec, int(ncycle), int(nmr), _ptr(r), _ptr(z), r.shape[0]))

    def sap_timing(self, enable=True):
        """Start (or stop) recording the launch durations of the SAP half-sweeps."""
        _check(lib().mglma_sap_timing(self._ctx, int(bool(enable))))

    def sap_elapsed(self):
        """(summed ms, launches) of the SAP half-sweeps recorded since the last call."""
        ms, n = C.c_double(0.0), C.c_int(0)
        _check(lib().mglma_sap_elapsed(self._ctx, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def export_basis(self, out):
        _check(lib().mglma_export_basis(self._ctx, _ptr(out)))

    def export_coarse_op(self, out):
        _check(lib().mglma_export_coarse_op(self._ctx, _ptr(out)))

    def export_coarse_gammas(self, out):
        _check(lib().mglma_export_coarse_gammas(self._ctx, _ptr(out)))

    def restrict(self, fine, coarse, prec=F64):
        _check(lib().mglma_restrict(self._ctx, prec, _ptr(fine), _ptr(coarse), fine.shape[0]))

    def prolong(self, coarse, fine, prec=F64):
        _check(lib().mglma_prolong(self._ctx, prec, _ptr(coarse), _ptr(fine), coarse.shape[0]))

    def coarse_apply(self, x, y, prec=F64, gamma5=0):
        _check(lib().mglma_coarse_apply(self._ctx, prec, gamma5, _ptr(x), _ptr(y), x.shape[0]))

    @property
    def V2(self):
        return self.query(9)

    # ---- checkpoint ----------------------------------------------------------
    def save(self, path):
        _check(lib().mglma_save(self._ctx, str(path).encode()))

    def load(self, path):
        _check(lib().mglma_load(self._ctx, str(path).encode()))

    # ---- level 2 of the nested hierarchy -------------------------------------
    def build_level2(self, b2):
        _check(lib().mglma_build_level2(self._ctx, (C.c_int * 4)(*[int(v) for v in b2])))

    def export_level2_op(self, out):
        _check(lib().mglma_export_level2_op(self._ctx, _ptr(out)))

    def level2_restrict(self, x1, y2, prec=F64):
        _check(lib().mglma_level2_restrict(self._ctx, prec, _ptr(x1), _ptr(y2), x1.shape[0]))

    def level2_prolong(self, x2, y1, prec=F64):
        _check(lib().mglma_level2_prolong(self._ctx, prec, _ptr(x2), _ptr(y1), x2.shape[0]))

    def level2_apply(self, x, y, prec=F64, gamma5=0):
        _check(lib().mglma_level2_apply(self._ctx, prec, gamma5, _ptr(x), _ptr(y), x.shape[0]))

    def level2_solve(self, b, x, params=None):
        n = b.shape[0]
        st = (SolveStats * max(n, 1))()
        _check(lib().mglma_level2_solve(self._ctx, C.byref(params or default_params()), _ptr(b), _ptr(x), n, st))
        return [dict(outer=s.outer, inner=s.inner, coarse=s.coarse, true_rel_res=s.true_rel_res) for s in st[:n]]

    def level2_pieces(self, eta, ge2, params=None):
        _check(lib().mglma_level2_pieces(self._ctx, C.byref(params or default_params()), _ptr(eta), _ptr(ge2),
                                         eta.shape[0]))

    def level2_field(self, nrhs, prec=F64, device="cuda"):
        import torch
        per = {F64: torch.float64, F32: torch.float32}[prec]
        return torch.empty((nrhs, self.V2, self.nc, 2), dtype=per, device=device)

    @property
    def has_eo(self):
        return self.query(8) == 1

    def coarse_schur_apply(self, x, y):
        """y = (1 - D_ee^-1 D_eo D_oo^-1 D_oe) x on even-site FP32 vectors [n][V1/2][nc][2]."""
        _check(lib().mglma_coarse_schur_apply(self._ctx, _ptr(x), _ptr(y), x.shape[0]))

    def set_top_modes(self, modes):
        _check(lib().mglma_set_top_modes(self._ctx, modes.shape[0], _ptr(modes)))

    # ---- solves -------------------------------------------------------------
    def solve(self, b, x, params=None, raise_on_error=True):
        n = b.shape[0]
        st = (SolveStats * max(n, 1))()
        rc = lib().mglma_solve(self._ctx, C.byref(params or default_params()), _ptr(b), _ptr(x), n, st)
        if raise_on_error:
            _check(rc)
        return rc, [dict(outer=s.outer, inner=s.inner, coarse=s.coarse, true_rel_res=s.true_rel_res,
                         seconds=s.seconds, status=s.status) for s in st[:n]]

    def coarse_solve(self, b, x, params=None):
        n = b.shape[0]
        st = (SolveStats * max(n, 1))()
        _check(lib().mglma_coarse_solve(self._ctx, C.byref(params or default_params()), _ptr(b), _ptr(x), n, st))
        return [dict(outer=s.outer, inner=s.inner, coarse=s.coarse, true_rel_res=s.true_rel_res) for s in st[:n]]

    def coarse_pieces(self, eta, ge1, top=None, params=None):
        _check(lib().mglma_coarse_pieces(self._ctx, C.byref(params or default_params()), _ptr(eta),
                                         _ptr(ge1), _ptr(top), eta.shape[0]))

    def coarse_eigs(self, init, nev, tol=1e-12, degree=0, max_iter=0, raise_on_error=True, out_block=False):
        """Low modes of Q_1: init is the [nblk][V1][nc] complex128 start block
        (nguard = nblk - nev).  Returns (rc, eigenvalues, eigenvectors, stats);
        with out_block the whole final block (nblk pairs), from which a later
        call continues."""
        return self._eigs(lib().mglma_coarse_eigs, (self.V1, self.nc, 2), init, nev, tol, degree, max_iter,
                          raise_on_error, out_block)

    def fine_eigs(self, init, nev, tol=1e-12, degree=0, max_iter=0, raise_on_error=True):
        """Low modes of Q = gamma5 M: init is [nblk][12][V][2] float64 (device
        layout).  Returns (rc, eigenvalues, eigenvectors, stats)."""
        return self._eigs(lib().mglma_fine_eigs, (12, self.V, 2), init, nev, tol, degree, max_iter,
                          raise_on_error)

    def _eigs(self, fn, shape, init, nev, tol, degree, max_iter, raise_on_error, out_block=False):
        import torch
        nb = init.shape[0]
        par = EigParams(nev=nev, nguard=nb - nev, degree=degree, max_iter=max_iter, tol=tol,
                        out_block=1 if out_block else 0)
        nout = nb if out_block else nev
        ev = np.zeros(max(nout, 1), dtype=np.float64)
        vec = torch.empty((max(nout, 1),) + shape, dtype=torch.float64, device=init.device)
        st = EigStats()
        rc = fn(self._ctx, C.byref(par), _ptr(init), ev.ctypes.data_as(C.c_void_p), _ptr(vec), C.byref(st))
        if raise_on_error:
            _check(rc)
        return rc, ev[:nout], vec[:nout], dict(iters=st.iters, applies=st.applies, nconv=st.nconv,
                                             max_res=st.max_res, spectrum_bound=st.spectrum_bound,
                                             lambda_max_abs=st.lambda_max_abs,
                                             seconds=st.seconds)

    def level_eigs(self, op, init, nev, tol=1e-12, degree=0, max_iter=0, raise_on_error=True):
        """Low modes of the Hermitian operator of a level (OP_FINE, OP_COARSE,
        OP_LEVEL2, OP_NONCHIRAL); init [nblk][...] in that level's layout."""
        shape = tuple(init.shape[1:])
        fn = lambda *a: lib().mglma_level_eigs(a[0], int(op), *a[1:])
        return self._eigs(fn, shape, init, nev, tol, degree, max_iter, raise_on_error)

    def build_nonchiral(self, testvecs):
        _check(lib().mglma_build_nonchiral(self._ctx, _ptr(testvecs)))

    def export_nonchiral_op(self, out):
        _check(lib().mglma_export_nonchiral_op(self._ctx, _ptr(out)))

    def deficit(self, fine):
        """Local-coherence deficits |(1 - P) psi| / |psi| of nrhs fine fields."""
        n = fine.shape[0]
        eps = np.zeros(max(n, 1), dtype=np.float64)
        _check(lib().mglma_deficit(self._ctx, n, _ptr(fine), eps.ctypes.data_as(C.c_void_p)))
        return eps[:n]

    # ---- sources and contractions --------------------------------------------
    def point_sources(self, y, out):
        _check(lib().mglma_point_sources(self._ctx, (C.c_int * 4)(*y), _ptr(out)))

    def noise_sources(self, xi, t, out):
        t = np.ascontiguousarray(t, dtype=np.int32)
        _check(lib().mglma_noise_sources(self._ctx, xi.shape[0], _ptr(xi),
                                         t.ctypes.data_as(C.POINTER(C.c_int)), _ptr(out)))

    def _corr(self, fn, a, b, t0):
        out = np.zeros((self.L[0], 2), dtype=np.float64)
        _check(fn(self._ctx, _ptr(a), _ptr(b), int(t0), out.ctypes.data_as(C.c_void_p)))
        return out[:, 0] + 1j * out[:, 1]

    def contract_point(self, psi_i, psi_j, y0):
        return self._corr(lib().mglma_contract_point, psi_i, psi_j, y0)

    def contract_point_coarse(self, ci, cj, y0):
        return self._corr(lib().mglma_contract_point_coarse, ci, cj, y0)

    def contract_stoch(self, psi_i, psi_j, tn):
        return self._corr(lib().mglma_contract_stoch, psi_i, psi_j, tn)

    def contract_stoch_coarse(self, ci, cj, tn):
        return self._corr(lib().mglma_contract_stoch_coarse, ci, cj, tn)

    def contract_top(self):
        out = np.zeros((self.L[0], 2), dtype=np.float64)
        _check(lib().mglma_contract_top(self._ctx, out.ctypes.data_as(C.c_void_p)))
        return out[:, 0] + 1j * out[:, 1]

    def contract_pair(self, kind, t_src, psi_i, psi_j, coarse=False):
        """Source-averaged two-point function of two pieces (eq:C_stoch2 /
        eq:tmr columns of nsrc = len(t_src) sources)."""
        t = np.ascontiguousarray(t_src, dtype=np.int32)
        out = np.zeros((self.L[0], 2), dtype=np.float64)
        _check(lib().mglma_contract_pair(self._ctx, int(kind), len(t), t.ctypes.data_as(C.POINTER(C.c_int)),
                                         int(bool(coarse)), _ptr(psi_i), _ptr(psi_j),
                                         out.ctypes.data_as(C.c_void_p)))
        return out[:, 0] + 1j * out[:, 1]

    def contract_levels(self, kind, t_src, fine=None, coarse=(), exact_top=False):
        """Level terms from cumulative pieces [fine] + coarse, averaged over the
        sources; rows as documented for mglma_contract_levels."""
        t = np.ascontiguousarray(t_src, dtype=np.int32)
        nco = len(coarse)
        arr = (C.c_void_p * max(nco, 1))(*[c.data_ptr() for c in coarse])
        nrow = (1 if fine is not None else 0) + nco + (1 if exact_top else 0)
        out = np.zeros((max(nrow, 1), self.L[0], 2), dtype=np.float64)
        _check(lib().mglma_contract_levels(self._ctx, int(kind), len(t), t.ctypes.data_as(C.POINTER(C.c_int)),
                                           _ptr(fine), nco, arr, int(bool(exact_top)),
                                           out.ctypes.data_as(C.c_void_p)))
        return out[:nrow, :, 0] + 1j * out[:nrow, :, 1]

    def contract_levels_acc(self, kind, t_src, out, weight, accumulate, fine=None, coarse=()):
        """out (device, [m][L0][2] float64) (+)= weight * the level rows of
        these sources (asynchronous)."""
        t = np.ascontiguousarray(t_src, dtype=np.int32)
        nco = len(coarse)
        arr = (C.c_void_p * max(nco, 1))(*[c.data_ptr() for c in coarse])
        _check(lib().mglma_contract_levels_acc(self._ctx, int(kind), len(t), t.ctypes.data_as(C.POINTER(C.c_int)),
                                               _ptr(fine), nco, arr, C.c_double(weight), int(bool(accumulate)),
                                               _ptr(out)))

    def contract_levels_noalloc(self, kind, t_src, fine=None, coarse=()):
        """contract_levels without the exact top row, through the entry point
        that allocates nothing (fixed device workspace)."""
        t = np.ascontiguousarray(t_src, dtype=np.int32)
        nco = len(coarse)
        arr = (C.c_void_p * max(nco, 1))(*[c.data_ptr() for c in coarse])
        nrow = (1 if fine is not None else 0) + nco
        out = np.zeros((max(nrow, 1), self.L[0], 2), dtype=np.float64)
        _check(lib().mglma_contract_levels_noalloc(self._ctx, int(kind), len(t), t.ctypes.data_as(C.POINTER(C.c_int)),
                                                   _ptr(fine), nco, arr, out.ctypes.data_as(C.c_void_p)))
        return out[:nrow, :, 0] + 1j * out[:nrow, :, 1]


class Slots:
    """Resident right-hand-side slots of one context (continuous batching):
    load() sources into free slots, step() one outer cycle of every running
    slot, take() finished solutions."""

    def __init__(self, ctx, nslots):
        self.ctx, self.nslots = ctx, int(nslots)
        self._h = C.c_void_p()
        _check(lib().mglma_slots_create(ctx._ctx, self.nslots, C.byref(self._h)))
        self.status = np.zeros(self.nslots, dtype=np.int32)

    def close(self):
        if self._h:
            lib().mglma_slots_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, b):
        ids = np.zeros(b.shape[0], dtype=np.int32)
        _check(lib().mglma_slots_load(self._h, b.shape[0], _ptr(b), ids.ctypes.data_as(C.POINTER(C.c_int))))
        return ids

    def step(self, params):
        """One outer cycle; returns the state of every slot id (0 free,
        1 running, 2 converged, < 0 failed)."""
        _check(lib().mglma_slots_step(self._h, C.byref(params),
                                      self.status.ctypes.data_as(C.POINTER(C.c_int))))
        return self.status.copy()

    def take(self, ids, x):
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        n = len(ids)
        st = (SolveStats * max(n, 1))()
        _check(lib().mglma_slots_take(self._h, n, ids.ctypes.data_as(C.POINTER(C.c_int)), _ptr(x), st))
        return [dict(outer=s.outer, inner=s.inner, true_rel_res=s.true_rel_res, status=s.status) for s in st[:n]]
