"""Eigenvalue error bounds of the Eigenvalue Bound Analysis subsection (oracle only).

gap theorem:           |dE| <= ||r||^2 / gamma_0
rigorous gap bound:    gamma_0 >= (E1~ - ||r1||) - E0~ =: gamma_0^-
"""


def gap_bound(resid_norm: float, gap: float) -> float:
    if gap <= 0:
        raise ValueError("gap must be positive")
    return resid_norm * resid_norm / gap


def gap_lower_bound(e0: float, e1: float, r1: float) -> float:
    return (e1 - r1) - e0
