"""Plain FP64 CPU oracle for multigrid low-mode averaging (arXiv:2412.06347).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (``paper_2412_06347_amd/csrc``); the only common module is the seeded
input generator ``paper_2412_06347_amd.synth``, which holds no method
arithmetic.

Everything is numpy complex128, written for readability: lattice fields are
kept as ``[..., L0, L1, L2, L3, spin 4, colour 3]`` arrays so that a hop is an
``np.roll``.  Each function cites the passage of the paper it follows.

Modules
-------
dirac       gamma matrices, clover term, Wilson-clover M and Q = gamma5 M
subspace    block decomposition, chirally split basis, R and T
coarse      Galerkin coarse operator, coarse apply, coarse gamma5
solvers     GCR / dense solves on the fine and coarse level
estimators  sources, propagator pieces S_l, contractions, level assembly
cost        the paper's inversion-cost formula

Functions whose result is not pinned by an independent check are marked
"parity unpinned" in their docstring.
"""
