"""Inversion-cost bookkeeping of the paper (oracle; test infrastructure only).

cost = 4 * sum_k N_eta(Lk) / Phi(Lk)   (section "Comparison of the cost"),
with the modelled ratio Phi(Lk) = 12 V / (N_s N_c V_k) for blocked levels
k > 0 (eq:model:ratio), Phi(L0) = 1, and levels evaluated exactly costing 0.
"""
from __future__ import annotations


def model_ratio(L, block, Ns=2, Nc=50):
    V = L[0] * L[1] * L[2] * L[3]
    Vk = V // (block[0] * block[1] * block[2] * block[3])
    return 12.0 * V / (Ns * Nc * Vk)


def cost(n_eta, ratios):
    """n_eta[k] sources on level k (None = exact), ratios[k] = Phi(Lk)."""
    return 4.0 * sum(n / r for n, r in zip(n_eta, ratios) if n is not None)
