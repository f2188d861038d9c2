"""Plain Davidson eigensolver (oracle; test infrastructure only).

Follows the solver description of the Results section: Rayleigh-Ritz on the
expansion space, residual r = H C - E C appended (after preconditioning) as a
new expansion vector, convergence on ||r||.  Preconditioners:
  * traditional Davidson (Eq. davidsonPreconditioner):
        t_i = r_i / (lambda - H_ii), 0 where |lambda - H_ii| is small;
  * compression-compatible (Eq. sparsePreconditioner):
        s_i = r_i / (lambda - H_ii) if |lambda - H_ii| >= 1e-12 else 0,
        t_i = s_i if |s_i| >= eps ||s|| else 0.
With eps = 0 the second reduces to the first with a 1e-12 guard.

Readings where the paper gives no detail: the initial guess is the unit
vectors at the k smallest diagonal entries (ties to the lower index); new
directions are orthogonalised twice by classical Gram-Schmidt and dropped if
their norm falls below 1e-10 (linear dependence); on reaching m_max the space
is restarted from the current Ritz vectors.
"""
from __future__ import annotations

import numpy as np


def precondition(r, lam, diag, eps=0.0, guard=1e-12):
    den = lam - diag
    s = np.where(np.abs(den) >= guard, r / np.where(np.abs(den) >= guard, den, 1.0), 0.0)
    if eps > 0.0:
        ns = np.linalg.norm(s)
        s = np.where(np.abs(s) >= eps * ns, s, 0.0)
    return s


def davidson(matvec, diag, k=1, tol=1e-8, max_iter=200, m_max=None, eps=0.0, dtype=np.complex128,
             guess=None, history=None):
    n = len(diag)
    k = min(k, n)
    m_max = m_max or max(8 * k, 16)
    m_max = min(m_max, n)
    if guess is None:
        order = np.argsort(diag, kind="stable")[:k]
        V = np.zeros((n, k), dtype=dtype)
        V[order, np.arange(k)] = 1.0
    else:
        V = np.array(guess, dtype=dtype).reshape(n, -1)
        V, _ = np.linalg.qr(V)
    W = np.column_stack([matvec(V[:, i]) for i in range(V.shape[1])])
    theta_old = None
    for it in range(1, max_iter + 1):
        G = V.conj().T @ W
        G = 0.5 * (G + G.conj().T)
        theta, Y = np.linalg.eigh(G)
        theta, Y = theta[:k], Y[:, :k]
        X = V @ Y
        R = W @ Y - X * theta
        rn = np.linalg.norm(R, axis=0)
        if history is not None:
            history.append(dict(iter=it, energies=theta.copy(), resid=rn.copy(),
                                dE=None if theta_old is None else theta - theta_old))
        theta_old = theta.copy()
        if np.all(rn <= tol):
            return theta, X, rn, it
        new = []
        for i in range(k):
            if rn[i] <= tol:
                continue
            t = precondition(R[:, i], theta[i], diag, eps)
            basis = np.column_stack([V] + new) if new else V
            for _ in range(2):
                t = t - basis @ (basis.conj().T @ t)
            nt = np.linalg.norm(t)
            if nt < 1e-10:
                continue
            new.append(t / nt)
        if not new:
            return theta, X, rn, it
        if V.shape[1] + len(new) > m_max:
            Wx = W @ Y
            V, W = X.copy(), Wx
            # re-orthonormalise the restart block against itself
            Q, Rr = np.linalg.qr(V)
            V = Q
            W = np.linalg.solve(Rr.T, W.T).T if Rr.shape[0] == Rr.shape[1] else W
            for j in range(len(new)):
                t = new[j]
                for _ in range(2):
                    t = t - V @ (V.conj().T @ t)
                new[j] = t / np.linalg.norm(t)
        Wn = np.column_stack([matvec(t) for t in new])
        V = np.column_stack([V] + new)
        W = np.column_stack([W, Wn])
    return theta, X, rn, max_iter
