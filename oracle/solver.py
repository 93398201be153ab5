"""End-to-end oracle solves: direct, and the domain-decomposition method (Secs. 3-7).

``dd_solve``: lifting b (Sec. 4, eq. (3)), GMRES on (I - S) g = b (eq. (5)) with the
chosen sweeping preconditioner (Secs. 5-6), and reconstruction of the field from
the converged interface data (u_i = A_i^{-1}(f_i + B_i g), Sec. 4).
"""
from __future__ import annotations

import numpy as np

from . import sweep
from .dd import Decomposition
from .fd import Grid, direct_solve
from .krylov import gmres


class DDResult:
    def __init__(self, u, g, gm):
        self.u, self.g, self.gmres = u, g, gm
        self.iters = gm.iters
        self.relres = gm.relres
        self.history = gm.history


def dd_solve(dd: Decomposition, f, precond="bj", tol=1e-6, restart=50, maxit=2000, flexible=False,
             width=None, combine="restricted", compose="product"):
    """Solve A u = f through the interface problem.  f: [ny, nx] complex."""
    f = np.asarray(f, dtype=np.complex128)
    b = dd.lifting(f)
    if precond == "none":
        M = None
    elif precond == "sgs":
        M = lambda r: sweep.apply_sgs(dd, r)  # noqa: E731
    else:
        M = lambda r: sweep.apply_bj(dd, r, width=width, combine=combine, compose=compose)  # noqa: E731
    res = gmres(dd.apply_operator, b, M, tol=tol, restart=restart, maxit=maxit, flexible=flexible)
    u = dd.reconstruct(f, res.x)
    return DDResult(u, res.x, res)


def direct(grid: Grid, f):
    """u = A^{-1} f on the global grid (sparse LU)."""
    f = np.asarray(f, dtype=np.complex128)
    flat = f.reshape(-1, grid.size) if f.ndim == 3 else f.ravel()
    return direct_solve(grid.matrix(), flat).reshape(f.shape)


def volume_residual(grid: Grid, u, f):
    """||f - A u|| / ||f|| on the global grid (the residual of eq. (1) discretised, Sec. 3),
    per right-hand side: u and f are [ny, nx] (returns a float) or [nrhs, ny, nx] (returns an
    array of nrhs floats).

    Pins (tests/test_oracle_fd.py): zero to round-off for the direct solution; a known value
    for a single perturbed entry of f; A u against a node-by-node evaluation of the 5-point
    stencil with the absorbing ghost values."""
    A = grid.matrix()
    u = np.asarray(u, dtype=np.complex128)
    f = np.asarray(f, dtype=np.complex128)
    if u.ndim == 2:
        r = f.ravel() - A @ u.ravel()
        return float(np.linalg.norm(r) / np.linalg.norm(f.ravel()))
    U = u.reshape(u.shape[0], -1).T
    F = f.reshape(f.shape[0], -1).T
    R = F - A @ U
    return np.linalg.norm(R, axis=0) / np.linalg.norm(F, axis=0)
