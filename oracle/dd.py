"""Non-overlapping checkerboard decomposition and the interface problem (paper Secs. 3-4).

Subdomain i = (i1, i2) (1-based, i1 = column in x, i2 = row in y) owns the nodes
ix in [(i1-1) snx, i1 snx), iy in [(i2-1) sny, i2 sny), numbered locally
ly * snx + lx.  Its local problem (Sec. 3, eq. (2)) is the 5-point operator on
its own nodes with the Robin face template (see ``oracle.fd``) on every face:
outer faces carry the absorbing condition (data 0, alpha = k sqrt(m_p)) and
interface faces carry the transmission data g received from the neighbour, with
alpha_f = k sqrt((m_p + m_q)/2), the same value seen from both sides.

The data that i sends to a neighbour j through face (p in i, q in j) is the
Robin data j's own condition would see, (-d_{n_ij} - T) u_i, which with the face
template is  out_q = -rho g_p - sigma u_p  (g_p the data i received on the same
face).  Summed over the faces of i this is the local scattering operator of
Sec. 4, including the reflection term k = j.

Higher-order transmission (transmission=2; the paper's own condition is a higher-order
absorbing one, a Pade approximation with a rotated branch cut and auxiliary interface
fields): on interface faces the condition gains a tangential second-derivative term,

    d_n u - i alpha a u - (i b / alpha) d_tt u = g,

the form of a second-order expansion of the one-way operator d_n - i alpha sqrt(1 +
d_tt / alpha^2) (Taylor: a = 1, b = 1/2).  With the face template it reads

    (u_q - u_p)/h - i alpha a (u_p + u_q)/2 - beta-_e (C u_p)_e = g_e,

beta+- built from alpha a, where C is the symmetric tangential operator along the face
with edge weights s_{e,e+1} = (kappa_e + kappa_{e+1}) / (2 h^2), kappa = (i b / alpha) /
beta- (with constant alpha this is (i b / alpha) times the second difference), and
homogeneous Neumann closure at the face ends.  The Taylor coefficients make S expand
the grid-scale tangential modes on this 5-point grid (GMRES then stalls); the default
(a, b) = (1 + 0.2 i, 0.15 exp(-i pi/4)) damps them (Re of the impedance negative for
evanescent modes, as the rotated branch cut does) and was chosen by a sweep of block-
Jacobi GMRES iterations at 10 and 15 points per wavelength.  The ghost becomes u_q = (g + beta+ u_p)/beta- +
(C u_p)_e, so the row of p gains -(C u_p)_e / h^2: the local matrix stays banded and
complex symmetric.  The data sent across the face keep the first-order form with
matrices along the face: out = -R g - Sigma u_line with M = B+ + B- C, R = M B-^{-1},
Sigma = M B-^{-1} M - B- (R = diag(rho), Sigma = diag(sigma) when C = 0).  The outer
faces keep the first-order absorbing condition, so the global problem, and with it the
solution, do not depend on the transmission order; only the convergence does.

Pade transmission (transmission=3, the paper's own condition, Sec. 7): on interface faces the
impedance alpha of the face template becomes the dense symmetric matrix X of oracle.habc (the
rotated Pade approximation of the one-way operator with N_pade auxiliary fields eliminated), so
the ghost values are u_q = Q (g + beta+ u_p) with Q = (I/h - (i/2) X)^{-1}: the face nodes' rows
gain the dense block -rho / h^2, the incoming data enter as (Q / h^2) g, and the data sent across
are -rho g - sigma u_p, all n x n matrices along the face (oracle.habc.face_maps).  The local
matrix stays complex symmetric; it is no longer banded along the vertical faces.

Pins (tests/test_oracle_dd.py): the reconstructed u equals the global direct
solve to round-off on every decomposition (1 x 1 included); the traces of the
global solution satisfy (I - S) g = b exactly; the dense S has the group
structure of Sec. 5; GMRES agrees with a dense solve of (I - S) g = b; for the
second-order transmission the same identities and A = A^T (tests/test_oracle_habc.py
for the Pade transmission).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import habc
from .fd import Grid, robin_coeffs
from .layout import Layout, neighbours, norm1, subdomains

# face identifiers: west (lx = 0), east (lx = snx-1), south (ly = 0), north (ly = sny-1)
FACES = ("W", "E", "S", "N")

# (a, b) of the second-order transmission condition d_n u - i alpha a u - (i b / alpha) d_tt u = g
SECOND_ORDER = (1.0 + 0.2j, 0.15 * np.exp(-0.25j * np.pi))


class Subdomain:
    def __init__(self, dd, i):
        self.i = i
        g = dd.grid
        snx, sny = dd.snx, dd.sny
        self.x0 = (i[0] - 1) * snx
        self.y0 = (i[1] - 1) * sny
        self.snx, self.sny = snx, sny
        i1, i2 = i
        nb = {"W": (i1 - 1, i2), "E": (i1 + 1, i2), "S": (i1, i2 - 1), "N": (i1, i2 + 1)}
        self.nbr = {}
        for f, j in nb.items():
            if 1 <= j[0] <= dd.n1 and 1 <= j[1] <= dd.n2:
                self.nbr[f] = j
        lx = np.arange(snx)
        ly = np.arange(sny)
        # local indices of the edge nodes of each face, ordered along the interface
        self.edge = {
            "W": ly * snx + 0,
            "E": ly * snx + (snx - 1),
            "S": 0 * snx + lx,
            "N": (sny - 1) * snx + lx,
        }
        m_loc = g.m[self.y0:self.y0 + sny, self.x0:self.x0 + snx]
        self.m_loc = m_loc
        # face alpha for every face node: outer -> k sqrt(m_p); interface -> k sqrt(mean)
        self.alpha = {}
        for f in FACES:
            mp = m_loc.ravel()[self.edge[f]]
            if f in self.nbr:
                if f == "W":
                    mq = g.m[self.y0:self.y0 + sny, self.x0 - 1]
                elif f == "E":
                    mq = g.m[self.y0:self.y0 + sny, self.x0 + snx]
                elif f == "S":
                    mq = g.m[self.y0 - 1, self.x0:self.x0 + snx]
                else:
                    mq = g.m[self.y0 + sny, self.x0:self.x0 + snx]
                self.alpha[f] = g.k * np.sqrt(0.5 * (mp + mq))
            else:
                self.alpha[f] = g.k * np.sqrt(mp)
        # second-order transmission: zeroth-order impedance alpha a on interface faces
        a0, b0 = (dd.tcoef if dd.transmission == 2 else (1.0, 0.0))
        # Pade transmission: the dense face maps of every interface face
        self.pade = {}
        if dd.transmission == 3:
            npade, phi = dd.tcoef
            for f in self.nbr:
                self.pade[f] = habc.face_maps(np.real(self.alpha[f]), g.h, npade, phi)
        self.coef = {f: robin_coeffs(self.alpha[f] * (a0 if f in self.nbr else 1.0), g.h) for f in FACES}
        # tangential operator C of every interface face (zero for first-order transmission)
        self.tang = {}
        for f in self.nbr:
            bm = self.coef[f][0]
            n_e = bm.size
            C = np.zeros((n_e, n_e), dtype=np.complex128)
            if dd.transmission == 2 and n_e > 1:
                kappa = (1j * b0 / self.alpha[f]) / bm
                s_e = (kappa[:-1] + kappa[1:]) / (2.0 * g.h * g.h)
                e = np.arange(n_e - 1)
                C[e, e + 1] = s_e
                C[e + 1, e] = s_e
                C[e, e] -= s_e
                C[e + 1, e + 1] -= s_e
            self.tang[f] = C
        self.A = self._matrix(g)
        self._lu = None

    def _matrix(self, g):
        """Local operator A_i: 5-point stencil + the Robin closure on all four faces."""
        snx, sny, h, k = self.snx, self.sny, g.h, g.k
        n = snx * sny
        diag = (4.0 / h**2 - k * k * self.m_loc.ravel()).astype(np.complex128)
        for f in FACES:
            if f in self.pade:
                continue
            rho = self.coef[f][2]
            np.add.at(diag, self.edge[f], -rho / h**2)
        idx = np.arange(n).reshape(sny, snx)
        rows, cols, vals = [np.arange(n)], [np.arange(n)], [diag]
        # Pade transmission: the dense block -rho / h^2 on the nodes of each interface face
        for f, P in self.pade.items():
            e = self.edge[f]
            rows.append(np.repeat(e, e.size))
            cols.append(np.tile(e, e.size))
            vals.append((-P["rho"] / h**2).ravel())
        off = -1.0 / h**2
        for a, b in ((idx[:, :-1].ravel(), idx[:, 1:].ravel()), (idx[:-1, :].ravel(), idx[1:, :].ravel())):
            rows += [a, b]
            cols += [b, a]
            vals += [np.full(a.size, off, np.complex128)] * 2
        # second-order transmission: the row of each interface edge node gains -(C u_line)_e / h^2
        for f, C in self.tang.items():
            if not C.any():
                continue
            e = self.edge[f]
            r, c = np.nonzero(C)
            rows.append(e[r])
            cols.append(e[c])
            vals.append(-C[r, c] / h**2)
        return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))

    @property
    def lu(self):
        if self._lu is None:
            self._lu = spla.splu(self.A)
        return self._lu

    def restrict(self, u_global):
        """Owned part of a global [ny, nx] field, flattened in local order."""
        return u_global[self.y0:self.y0 + self.sny, self.x0:self.x0 + self.snx].ravel()


class Decomposition:
    """The n1 x n2 checkerboard of a grid (Sec. 2) with its interface layout."""

    def __init__(self, grid: Grid, n1: int, n2: int, transmission: int = 1, tcoef=None):
        if grid.nx % n1 or grid.ny % n2:
            raise ValueError("grid size must be divisible by the decomposition")
        if transmission not in (1, 2, 3):
            raise ValueError("transmission must be 1 (Robin), 2 (second order) or 3 (Pade)")
        self.grid, self.n1, self.n2 = grid, n1, n2
        self.transmission = transmission
        # (a, b) of the second-order condition d_n u - i alpha a u - (i b / alpha) d_tt u = g;
        # (N_pade, phi) of the Pade condition
        if tcoef is None:
            tcoef = habc.PADE_DEFAULT if transmission == 3 else SECOND_ORDER
        self.tcoef = tcoef
        self.snx, self.sny = grid.nx // n1, grid.ny // n2
        self.layout = Layout(n1, n2, self.snx, self.sny)
        self.nif = self.layout.nif
        self.sub = {i: Subdomain(self, i) for i in subdomains(n1, n2)}
        # Where independent local problems are solved: None = one after the other in this process;
        # otherwise a callable (kind, keys, data) -> [result per key] that runs the same methods
        # (scatter_subdomain, lift_subdomain, reconstruct_subdomain) elsewhere, e.g. in processes
        # that each own a row of subdomains as the paper's MPI ranks do (Sec. 7).  The arithmetic
        # is the same either way.
        self.mapper = None

    def _map(self, kind, keys, data):
        if self.mapper is not None:
            return self.mapper(kind, keys, data)
        fn = {"scatter": self.scatter_subdomain, "lift": self.lift_subdomain,
              "reconstruct": self.reconstruct_subdomain}[kind]
        return [fn(i, *data) for i in keys]

    # -- local solves and traces (Sec. 4) ---------------------------------
    def local_rhs(self, i, g, f_loc=None):
        """f_i + B_i g: source plus injected incoming Robin data of every interface face."""
        s = self.sub[i]
        r = np.zeros(s.snx * s.sny, dtype=np.complex128) if f_loc is None else np.array(f_loc, dtype=np.complex128)
        if g is not None:
            for f, j in s.nbr.items():
                if f in s.pade:
                    r[s.edge[f]] += s.pade[f]["inj"] @ g[self.layout.block(i, j)]
                else:
                    inj = s.coef[f][4]
                    r[s.edge[f]] += inj * g[self.layout.block(i, j)]
        return r

    def local_solve(self, i, g, f_loc=None):
        """u_i = A_i^{-1} (f_i + B_i g)  (Sec. 3 eq. (2); with g = 0 the lifting, eq. (3))."""
        return self.sub[i].lu.solve(self.local_rhs(i, g, f_loc))

    def face_maps(self, i, f):
        """R and Sigma of face f of subdomain i (out = -R g - Sigma u_line along the face)."""
        s = self.sub[i]
        if f in s.pade:
            return s.pade[f]["rho"], s.pade[f]["sigma"]
        bm, bp = s.coef[f][0], s.coef[f][1]
        M = np.diag(bp) + bm[:, None] * s.tang[f]
        R = M / bm[None, :]
        Sig = R @ M - np.diag(bm)
        return R, Sig

    def outgoing(self, i, u_loc, g):
        """Data sent by i to every neighbour j: {j: (-d_{n_ij} - T) u_i on Gamma_ij} (Sec. 4).

        out = -rho g_p - sigma u_p, where g_p is the data i received on that face (0 if g is None);
        with the second-order transmission, out = -R g - Sigma u_line along the face."""
        s = self.sub[i]
        out = {}
        for f, j in s.nbr.items():
            gin = np.zeros(s.edge[f].size, np.complex128) if g is None else g[self.layout.block(i, j)]
            if f in s.pade:
                P = s.pade[f]
                out[j] = -P["rho"] @ gin - P["sigma"] @ u_loc[s.edge[f]]
            elif not s.tang[f].any():
                _, _, rho, sigma, _ = s.coef[f]
                out[j] = -rho * gin - sigma * u_loc[s.edge[f]]
            else:
                R, Sig = self.face_maps(i, f)
                out[j] = -R @ gin - Sig @ u_loc[s.edge[f]]
        return out

    def scatter_subdomain(self, i, g):
        """The local scattering operators of i applied to its incoming data (f = 0):
        {j: sum_k S_{m(j,i), m(i,k)} g_{m(i,k)}} over all k in D_i (Sec. 4)."""
        return self.outgoing(i, self.local_solve(i, g), g)

    def scatter_many(self, keys, g):
        """scatter_subdomain for every subdomain in keys (independent local problems)."""
        return self._map("scatter", list(keys), (g,))

    def lift_subdomain(self, i, f):
        """Outgoing traces of the lifting w_i of the source f ([ny, nx]) of subdomain i (eq. (3))."""
        w = self.local_solve(i, None, self.sub[i].restrict(f))
        return self.outgoing(i, w, None)

    def reconstruct_subdomain(self, i, f, g):
        """u_i = A_i^{-1}(f_i + B_i g) of subdomain i, in local order."""
        return self.local_solve(i, g, self.sub[i].restrict(f))

    # -- global interface operators ----------------------------------------
    def apply_S(self, g):
        """S g: every block m(j,i) receives the scattered data of its sender i (Sec. 4)."""
        out = np.zeros(self.nif, dtype=np.complex128)
        keys = list(self.sub)
        for i, sc in zip(keys, self.scatter_many(keys, g)):
            for j, v in sc.items():
                out[self.layout.block(j, i)] = v
        return out

    def apply_operator(self, g):
        """(I - S) g, Sec. 4 eq. (5)."""
        return g - self.apply_S(g)

    def lifting(self, f):
        """b_{m(j,i)} = (-d_{n_ij} - T) w_i with w_i the lifting of the source (Sec. 4, eq. (3))."""
        b = np.zeros(self.nif, dtype=np.complex128)
        keys = list(self.sub)
        for i, out in zip(keys, self._map("lift", keys, (f,))):
            for j, v in out.items():
                b[self.layout.block(j, i)] = v
        return b

    def reconstruct(self, f, g):
        """u_i = A_i^{-1}(f_i + B_i g) on every subdomain, assembled into a global [ny, nx] field."""
        u = np.zeros((self.grid.ny, self.grid.nx), dtype=np.complex128)
        keys = list(self.sub)
        for i, ui in zip(keys, self._map("reconstruct", keys, (f, g))):
            s = self.sub[i]
            u[s.y0:s.y0 + s.sny, s.x0:s.x0 + s.snx] = ui.reshape(s.sny, s.snx)
        return u

    def traces_of(self, u):
        """Incoming data g*_{m(i,j)} of a global field u: the Robin data that makes i's ghost
        value equal u at j's node, g = (u_q - u_p)/h - i alpha (u_p + u_q)/2 (minus
        beta- C u_p along the face for the second-order transmission)."""
        h = self.grid.h
        g = np.zeros(self.nif, dtype=np.complex128)
        for i, s in self.sub.items():
            uloc = s.restrict(u)
            for f, j in s.nbr.items():
                t = self.sub[j]
                fq = {"W": "E", "E": "W", "S": "N", "N": "S"}[f]
                up = uloc[s.edge[f]]
                uq = t.restrict(u)[t.edge[fq]]
                if f in s.pade:  # (u_q - u_p)/h - (i/2) X (u_p + u_q) = bm u_q - bp u_p with matrices
                    g[self.layout.block(i, j)] = s.pade[f]["bm"] @ uq - s.pade[f]["bp"] @ up
                    continue
                bm, bp = s.coef[f][0], s.coef[f][1]  # (u_q - u_p)/h - i alpha a (u_p + u_q)/2 = bm u_q - bp u_p
                g[self.layout.block(i, j)] = bm * uq - bp * up - bm * (s.tang[f] @ up)
        return g

    def dense_S(self):
        """S assembled column by column from unit vectors (tiny problems only)."""
        n = self.nif
        S = np.zeros((n, n), dtype=np.complex128)
        e = np.zeros(n, dtype=np.complex128)
        for c in range(n):
            e[:] = 0
            e[c] = 1
            S[:, c] = self.apply_S(e)
        return S

    def subdomains_on(self, a):
        return [i for i in self.sub if norm1(i) == a]

    def neighbours(self, i):
        return neighbours(i, self.n1, self.n2)
