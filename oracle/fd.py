"""Global 5-point finite-difference Helmholtz operator (paper Sec. 3, eq. (1)).

Problem: (-Lap - kappa^2) u = f in the unit square, kappa^2 = k^2 m with
m = 1/c^2, and the first-order absorbing condition (d_n - T) u = 0 on the outer
boundary with T = i alpha (impedance operator, Sec. 3; time dependence
e^{-i omega t}, so outgoing waves satisfy d_n u - i kappa u = 0).

The paper discretises with P7 finite elements and does not give a discrete
Robin form; this oracle uses the face template below (a reading recorded in the
design notes).  A face joins a node p of the grid (or of a subdomain) to an
outside node q.  The Robin condition (d_n - i alpha) u = g is imposed at the
face midpoint with second-order differences,

    (u_q - u_p)/h - i alpha (u_p + u_q)/2 = g,

so the outside value is the ghost u_q = (g + beta+ u_p) / beta-, with
beta+- = 1/h +- i alpha/2.  Substituting the ghost into the 5-point row of p
adds -rho/h^2 to the diagonal (rho = beta+/beta-) and g/(beta- h^2) to the right
hand side.  On the outer boundary g = 0 and alpha = k sqrt(m_p).

Pins (tests/test_oracle_fd.py): second-order convergence to smooth manufactured
solutions with Robin data (checks the stencil, the ghost elimination and the
sign of i alpha), symmetry A = A^T, and outgoing phase for a point source.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def robin_coeffs(alpha, h):
    """Face coefficients of the Robin template for impedance alpha (array or scalar).

    Returns (beta_minus, beta_plus, rho, sigma, inj):
      ghost      u_q = (g + beta_plus u_p) / beta_minus
      diagonal   -rho / h^2 added to the row of p
      injection  g * inj added to the right-hand side, inj = 1 / (beta_minus h^2)
      outgoing   data seen from the other side of the face:
                 (u_p - u_q)/h - i alpha (u_p + u_q)/2 = -rho g - sigma u_p,
                 sigma = 2 i alpha / (h beta_minus)
    """
    alpha = np.asarray(alpha, dtype=np.complex128)
    bm = 1.0 / h - 0.5j * alpha
    bp = 1.0 / h + 0.5j * alpha
    rho = bp / bm
    sigma = 2j * alpha / (h * bm)
    inj = 1.0 / (bm * h * h)
    return bm, bp, rho, sigma, inj


class Grid:
    """Interior grid nx x ny, h = 1/(nx+1), nodes (ix+1) h, (iy+1) h; flat index iy*nx + ix."""

    def __init__(self, nx, ny, h, k, m):
        self.nx, self.ny, self.h, self.k = nx, ny, float(h), float(k)
        self.m = np.asarray(m, dtype=np.float64)
        assert self.m.shape == (ny, nx)

    @property
    def size(self):
        return self.nx * self.ny

    def outer_alpha(self):
        """alpha_b = k sqrt(m_p) at outer faces (local wavenumber; a design reading)."""
        return self.k * np.sqrt(self.m)

    def outer_face_count(self):
        """Number of outer-boundary faces of every node (0..2 on a grid with nx, ny >= 2)."""
        c = np.zeros((self.ny, self.nx), dtype=np.int64)
        c[:, 0] += 1
        c[:, -1] += 1
        c[0, :] += 1
        c[-1, :] += 1
        return c

    def matrix(self):
        """Sparse global operator A (CSR, complex128), Sec. 3 eq. (1) with the face template."""
        nx, ny, h, k = self.nx, self.ny, self.h, self.k
        n = nx * ny
        _, _, rho_b, _, _ = robin_coeffs(self.outer_alpha(), h)
        diag = (4.0 / h**2 - k * k * self.m).astype(np.complex128)
        diag = diag - self.outer_face_count() * rho_b / h**2
        rows, cols, vals = [np.arange(n)], [np.arange(n)], [diag.ravel()]
        idx = np.arange(n).reshape(ny, nx)
        off = -1.0 / h**2
        # x neighbours
        a, b = idx[:, :-1].ravel(), idx[:, 1:].ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [np.full(a.size, off, np.complex128)] * 2
        # y neighbours
        a, b = idx[:-1, :].ravel(), idx[1:, :].ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [np.full(a.size, off, np.complex128)] * 2
        A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
        return A

    def outer_rhs(self, g_west=None, g_east=None, g_south=None, g_north=None):
        """Right-hand-side contribution g * inj of nonzero outer Robin data (manufactured tests).

        Each g_* is an array along its face (length ny for west/east, nx for south/north)."""
        h = self.h
        _, _, _, _, inj = robin_coeffs(self.outer_alpha(), h)
        r = np.zeros((self.ny, self.nx), dtype=np.complex128)
        if g_west is not None:
            r[:, 0] += g_west * inj[:, 0]
        if g_east is not None:
            r[:, -1] += g_east * inj[:, -1]
        if g_south is not None:
            r[0, :] += g_south * inj[0, :]
        if g_north is not None:
            r[-1, :] += g_north * inj[-1, :]
        return r

    def dA_dm_diag(self):
        """Derivative of the diagonal of A with respect to m_p (A depends on m only there).

        d/dm_p [-k^2 m_p - sum_outer rho_b/h^2] with rho = beta+/beta-, alpha_b = k sqrt(m_p):
        d rho/d alpha = (i/h)/beta-^2 and d alpha/d m = k / (2 sqrt(m))."""
        h, k = self.h, self.k
        alpha = self.outer_alpha()
        bm, _, _, _, _ = robin_coeffs(alpha, h)
        drho = (1j / h) / bm**2 * (k / (2.0 * np.sqrt(self.m)))
        return (-k * k - self.outer_face_count() * drho / h**2).astype(np.complex128)


def direct_solve(A, f):
    """u = A^{-1} f by sparse LU (SuperLU); f may be [n] or [nrhs, n]."""
    lu = spla.splu(A.tocsc())
    f = np.asarray(f, dtype=np.complex128)
    if f.ndim == 1:
        return lu.solve(f)
    return np.stack([lu.solve(fi) for fi in f])
