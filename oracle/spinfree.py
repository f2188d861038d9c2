"""Spatial -> spin-orbital expansion of spin-free integrals (oracle only).

Spin-orbital index: alpha orbital p -> p, beta orbital p -> n + p.
h_so[p s, q t] = h[p, q] d(s, t);  (p s q s' | r t s t') = (pq|rs) d(s, s') d(t, t').
"""
import numpy as np


def expand(h, g):
    n = h.shape[0]
    M = 2 * n
    hs = np.zeros((M, M), dtype=np.result_type(h, np.float64))
    gs = np.zeros((M, M, M, M), dtype=np.result_type(g, np.float64))
    for s in range(2):
        hs[s * n:(s + 1) * n, s * n:(s + 1) * n] = h
        for t in range(2):
            gs[s * n:(s + 1) * n, s * n:(s + 1) * n, t * n:(t + 1) * n, t * n:(t + 1) * n] = g
    return hs, gs
