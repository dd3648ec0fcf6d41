"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module holds input recipes only (random numbers and the synthetic gauge
ensemble); it contains none of the multigrid low-mode-averaging arithmetic.
All arrays are numpy complex128 in the canonical layout:

* site index ``s = ((x0*L1 + x1)*L2 + x2)*L3 + x3`` (time is direction 0);
* spinor fields ``[n][s][spin 4][colour 3]``;
* gauge field ``[s][mu][a][b]`` with ``U_mu(x)`` the link from x to x+mu;
* coarse fields ``[n][y][2*Nv]`` with ``y`` the block index ordered like ``s``.

The gauge recipe is the synthetic stand-in for the paper's CLS/openQCD
ensembles (section "Numerical study"): links ``U = exp(i*eps*H)`` with ``H``
a traceless Hermitian Gaussian matrix ``sum_a h_a lambda_a / 2``,
``h_a ~ N(0, 1)``, independently per link.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "generator", "gauge_field", "gaussian_fields", "z4_noise", "time_slices",
    "gauge_transform", "volume",
]


def volume(L):
    return int(L[0]) * int(L[1]) * int(L[2]) * int(L[3])


def generator(seed: int, stream: int = 0) -> np.random.Generator:
    """Counter-based Philox generator keyed by (seed, stream)."""
    return np.random.Generator(np.random.Philox(key=[int(seed) & 0xFFFFFFFFFFFFFFFF,
                                                     int(stream) & 0xFFFFFFFFFFFFFFFF]))


def _gell_mann():
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def _exp_i_hermitian(H, eps, chunk=1 << 20):
    """exp(i*eps*H) for a batch of Hermitian 3x3 matrices via eigh."""
    out = np.empty_like(H)
    n = H.shape[0]
    for i0 in range(0, n, chunk):
        h = H[i0:i0 + chunk]
        w, v = np.linalg.eigh(h)
        ph = np.exp(1j * eps * w)
        out[i0:i0 + chunk] = np.einsum("nab,nb,ncb->nac", v, ph, v.conj())
    return out


def gauge_field(L, eps: float, seed: int, progress=None) -> np.ndarray:
    """Random SU(3) links, canonical ``[V][4][3][3]`` complex128.  progress,
    if given, is called with (links done, links) after each chunk."""
    V = volume(L)
    g = generator(seed, 1)
    lam = _gell_mann() / 2
    U = np.empty((V * 4, 3, 3), dtype=np.complex128)
    chunk = 1 << 20
    for i0 in range(0, V * 4, chunk):
        n = min(chunk, V * 4 - i0)
        h = g.standard_normal((n, 8))
        H = np.tensordot(h, lam, axes=(1, 0))
        U[i0:i0 + n] = _exp_i_hermitian(H, eps)
        if progress is not None:
            progress(i0 + n, V * 4)
    return U.reshape(V, 4, 3, 3)


def gaussian_fields(n: int, L, seed: int, stream: int = 2) -> np.ndarray:
    """n spinor fields with independent N(0,1) real and imaginary parts."""
    V = volume(L)
    g = generator(seed, stream)
    re = g.standard_normal((n, V, 4, 3))
    im = g.standard_normal((n, V, 4, 3))
    return re + 1j * im


def gaussian_coarse(n: int, V1: int, nc: int, seed: int, stream: int = 3) -> np.ndarray:
    g = generator(seed, stream)
    return g.standard_normal((n, V1, nc)) + 1j * g.standard_normal((n, V1, nc))


def z4_noise(n: int, L, seed: int, stream: int = 4) -> np.ndarray:
    """Colour noise on one time slice per source: values uniform on
    {1+i, 1-i, -1+i, -1-i}/sqrt(2) (section "Stochastic estimator on level k").
    Shape ``[n][L1*L2*L3][3]``."""
    V3 = int(L[1]) * int(L[2]) * int(L[3])
    g = generator(seed, stream)
    b = g.integers(0, 4, size=(n, V3, 3))
    re = np.where(b & 1, -1.0, 1.0)
    im = np.where(b & 2, -1.0, 1.0)
    return (re + 1j * im) / np.sqrt(2.0)


def z2_noise(n: int, L, seed: int, stream: int = 5) -> np.ndarray:
    """Real {+1,-1} colour noise, shape ``[n][L1*L2*L3][3]``."""
    V3 = int(L[1]) * int(L[2]) * int(L[3])
    g = generator(seed, stream)
    return np.where(g.integers(0, 2, size=(n, V3, 3)) == 1, -1.0, 1.0).astype(np.complex128)


def time_slices(n: int, L0: int, seed: int, stream: int = 6) -> np.ndarray:
    """Source time slices t_n drawn uniformly (with replacement)."""
    return generator(seed, stream).integers(0, int(L0), size=n).astype(np.int32)


def gauge_transform(L, seed: int, stream: int = 7) -> np.ndarray:
    """Random SU(3) matrix per site, ``[V][3][3]`` (for covariance checks)."""
    V = volume(L)
    g = generator(seed, stream)
    lam = _gell_mann() / 2
    H = np.tensordot(g.standard_normal((V, 8)), lam, axes=(1, 0))
    return _exp_i_hermitian(H, 2.0)
