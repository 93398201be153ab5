"""Adjoint-state gradient of a data misfit with respect to m = 1/c^2.

Misfit L(m) = 1/2 sum_s ||P u_s - d_s||^2 with A(m) u_s = f_s and P the receiver
sampling.  A depends on m only through its diagonal (-k^2 m_p, and the outer
absorbing faces through alpha_b = k sqrt(m_p)), so

    dL/dm_p = sum_s -Re( conj(lambda_{s,p}) dA_pp/dm_p u_{s,p} ),
    A^H lambda_s = P^T (P u_s - d_s).

A is complex symmetric (A = A^T), hence A^H = conj(A) and the adjoint field is
lambda_s = conj(mu_s) with A mu_s = conj(P^T r_s): the adjoint solve reuses the
forward operator, factors and preconditioner.

Pins (tests/test_oracle_gradient.py): central finite differences of L on seeded
directions, and the dot-product identity <A u, v> = <u, A^T v>.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .fd import Grid


def misfit_and_gradient(grid: Grid, f, rec_idx, d, solve=None):
    """Return (L, dL/dm [ny, nx]) with forward and adjoint solves by ``solve(rhs)``
    (default: global sparse LU).  f: [nsrc, ny, nx]; d: [nsrc, nrec]."""
    A = grid.matrix()
    if solve is None:
        lu = spla.splu(A.tocsc())
        solve = lambda rhs: lu.solve(rhs.ravel()).reshape(rhs.shape)  # noqa: E731
    dA = grid.dA_dm_diag().ravel()
    n = grid.size
    L = 0.0
    grad = np.zeros(n)
    for s in range(f.shape[0]):
        u = solve(f[s]).ravel()
        r = u[rec_idx] - d[s]
        L += 0.5 * float(np.vdot(r, r).real)
        adj = np.zeros(n, dtype=np.complex128)
        np.add.at(adj, rec_idx, r)
        mu = solve(np.conj(adj).reshape(grid.ny, grid.nx)).ravel()
        lam = np.conj(mu)
        grad += -np.real(np.conj(lam) * dA * u)
    return L, grad.reshape(grid.ny, grid.nx)


def misfit(grid: Grid, f, rec_idx, d):
    """L(m) by global direct solves."""
    lu = spla.splu(grid.matrix().tocsc())
    L = 0.0
    for s in range(f.shape[0]):
        u = lu.solve(f[s].ravel())
        r = u[rec_idx] - d[s]
        L += 0.5 * float(np.vdot(r, r).real)
    return L
