"""Schwarz alternating procedure (SAP) smoother (oracle; test infrastructure
only: imported by tests/, never by the library).

The paper's fine solver is GCR preconditioned by SAP (section "Comparison of
the cost", citing Luscher 2003).  The procedure, written out:

* the lattice is divided into the blocks of eq:block_def, coloured like a
  chessboard: the colour of block y is the parity of y_0 + y_1 + y_2 + y_3;
* a cycle on M z = r visits colour 0, then colour 1; for a colour, the
  residual rho = r - M z is formed once, then every block B of that colour
  adds to z on its sites an approximate solution of M_BB d = rho_B, where
  M_BB = P_B M P_B is the restriction of M to the block's sites (all
  couplings between two sites of the block, including a hop that wraps
  around the lattice when the block spans a whole extent);
* the block solve is nmr minimal-residual steps from d = 0: s = rho_B, then
  t = M_BB s, omega = <t, s> / <t, t>, d += omega s, s -= omega t.

Blocks of one colour do not couple when every block-grid extent is even (or
one), so their order within the colour does not matter.
"""
from __future__ import annotations

import numpy as np


def block_colour(bl, y):
    """Chessboard colour of block y (eq:block_def block index)."""
    c = np.unravel_index(y, bl.L1)
    return int(sum(int(v) for v in c) % 2)


def block_mask(bl, y):
    """Boolean lattice mask [L0][L1][L2][L3] of the sites of block y."""
    c = [int(v) for v in np.unravel_index(y, bl.L1)]
    m = np.zeros(bl.L, dtype=bool)
    sl = tuple(slice(c[mu] * bl.b[mu], (c[mu] + 1) * bl.b[mu]) for mu in range(4))
    m[sl] = True
    return m


def block_apply(D, mask, s):
    """M_BB s for a field s [L..][4][3] that lives on the block's sites."""
    f = np.where(mask[..., None, None], s, 0.0)[None]
    out = D.M(f)[0]
    return np.where(mask[..., None, None], out, 0.0)


def mr_block(D, mask, rho, nmr):
    """nmr minimal-residual steps on M_BB d = rho_B from d = 0."""
    d = np.zeros_like(rho)
    s = np.where(mask[..., None, None], rho, 0.0)
    for _ in range(nmr):
        t = block_apply(D, mask, s)
        tt = np.vdot(t, t).real
        if tt == 0.0:
            break
        omega = np.vdot(t, s) / tt
        d = d + omega * s
        s = s - omega * t
    return d


def sap_cycle(D, bl, r, z, nmr):
    """One SAP cycle on M z = r for one field r, z [L..][4][3]; returns the new z."""
    z = z.copy()
    for colour in (0, 1):
        rho = r - D.M(z[None])[0]
        for y in range(bl.V1):
            if block_colour(bl, y) != colour:
                continue
            z = z + mr_block(D, block_mask(bl, y), rho, nmr)
    return z
