"""Dense projected Hamiltonian of a small space and its exact spectrum (oracle only).

H is assembled row by row from the Slater-Condon couplings of oracle.csc;
eigenpairs come from numpy.linalg.eigh (LAPACK).  Intended for spaces up to
about 1.3e4 determinants.
"""
from __future__ import annotations

import numpy as np

from . import csc


def hamiltonian(dets, h, g, e_core=0.0, real=False):
    n = len(dets)
    H = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        cols, vals = csc.h_row(dets, h, g, i, e_core)
        H[i, cols] += vals
    if real:
        return H.real.copy()
    return H


def lowest(H, k=1):
    w, V = np.linalg.eigh(H)
    return w[:k], V[:, :k]
