"""Restarted, right-preconditioned GMRES and flexible GMRES (paper Sec. 7).

The paper solves the interface system (I - S) g = b with GMRES to a relative
residual of 1e-6 and does not state the variant.  Reading used here: right
preconditioning, x0 = 0, restart length m (50 by default), modified
Gram-Schmidt Arnoldi, complex Givens rotations, stop when the Givens residual
estimate is <= tol ||b||, then confirm with the explicit residual and keep
iterating if the confirmation fails.  FGMRES keeps Z_j = P^{-1} v_j.

Pins (tests/test_oracle_krylov.py): agreement with a dense direct solve on tiny
systems, the exact-termination property (n steps for an n x n system), and the
iteration count of scipy's own GMRES on the same preconditioned operator.
"""
from __future__ import annotations

import numpy as np


def givens(a, b):
    """Complex rotation (c real, s complex) with [c s; -conj(s) c] [a; b] = [r; 0]."""
    if b == 0:
        return 1.0, 0.0 + 0.0j
    if a == 0:
        return 0.0, np.conj(b) / abs(b)
    r = np.hypot(abs(a), abs(b))
    c = abs(a) / r
    s = (a / abs(a)) * np.conj(b) / r
    return c, s


class GmresResult:
    def __init__(self, x, iters, relres, history, converged):
        self.x, self.iters, self.relres, self.history, self.converged = x, iters, relres, history, converged


def gmres(apply_A, b, apply_M=None, tol=1e-6, restart=50, maxit=1000, flexible=False):
    """Solve A x = b with right preconditioning x = M^{-1} y (M^{-1} = apply_M).

    Returns GmresResult(x, iterations, final true relative residual, history of the
    Givens estimates relative to ||b||, converged flag)."""
    b = np.asarray(b, dtype=np.complex128)
    ident = lambda v: v.copy()  # noqa: E731
    M = apply_M or ident
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    hist = [1.0]
    if nb == 0:
        return GmresResult(x, 0, 0.0, [0.0], True)
    it = 0
    r = b.copy()
    beta = nb
    while it < maxit:
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart)
        sn = np.zeros(restart, dtype=np.complex128)
        e1 = np.zeros(restart + 1, dtype=np.complex128)
        e1[0] = beta
        j_done = 0
        for j in range(restart):
            z = M(V[j])
            if flexible:
                Z.append(z)
            w = apply_A(z)
            for i in range(j + 1):  # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            for i in range(j):  # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            e1[j + 1] = -np.conj(sn[j]) * e1[j]
            e1[j] = cs[j] * e1[j]
            it += 1
            j_done = j + 1
            est = abs(e1[j + 1]) / nb
            hist.append(est)
            breakdown = abs(H[j, j]) == 0 or np.linalg.norm(w) == 0
            if est <= tol or breakdown or it >= maxit:
                break
            V.append(w / np.linalg.norm(w))
        # solve the upper-triangular least-squares system and update x
        y = np.zeros(j_done, dtype=np.complex128)
        for i in range(j_done - 1, -1, -1):
            y[i] = (e1[i] - H[i, i + 1:j_done] @ y[i + 1:j_done]) / H[i, i]
        if flexible:
            dx = sum(y[i] * Z[i] for i in range(j_done))
        else:
            dx = M(sum(y[i] * V[i] for i in range(j_done)))
        x = x + dx
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        if beta <= tol * nb:
            return GmresResult(x, it, beta / nb, hist, True)
        if it >= maxit:
            break
    return GmresResult(x, it, beta / nb, hist, False)
