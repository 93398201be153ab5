"""Pins of the oracle's discretisation (Sec. 3, eq. (1)) against the mathematics.

* second-order convergence to smooth manufactured solutions with Robin data on the
  outer faces (catches a wrong stencil term, a wrong ghost elimination, a wrong
  sign or factor of i alpha, or a misplaced m);
* complex symmetry A = A^T (the basis of the adjoint shortcut);
* the e^{-i omega t} convention: a point source radiates outgoing waves that match
  the free-space Green's function (i/4) H0^(1)(k r) and not the incoming one.
"""
import numpy as np
import pytest
from scipy.special import hankel1, hankel2

from oracle.fd import Grid, direct_solve


def _manufactured(n, k, variable_m):
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1) * h
    y = (np.arange(n) + 1) * h
    X, Y = np.meshgrid(x, y)

    def mfun(X, Y):
        return 1.0 + 0.2 * np.sin(X + 2 * Y) if variable_m else np.ones_like(X)

    # u* = exp(i (a x + b y)) (1 + 0.3 x y^2): smooth, complex, not a plane wave
    a, b = 3.0, -2.0

    def u(X, Y):
        return np.exp(1j * (a * X + b * Y)) * (1 + 0.3 * X * Y**2)

    def ux(X, Y):
        e = np.exp(1j * (a * X + b * Y))
        return e * (1j * a * (1 + 0.3 * X * Y**2) + 0.3 * Y**2)

    def uy(X, Y):
        e = np.exp(1j * (a * X + b * Y))
        return e * (1j * b * (1 + 0.3 * X * Y**2) + 0.6 * X * Y)

    def lap(X, Y):
        e = np.exp(1j * (a * X + b * Y))
        p = 1 + 0.3 * X * Y**2
        uxx = e * (-(a * a) * p + 2j * a * 0.3 * Y**2)
        uyy = e * (-(b * b) * p + 2j * b * 0.6 * X * Y + 0.6 * X)
        return uxx + uyy

    m = mfun(X, Y)
    g = Grid(n, n, h, k, m)
    f = -lap(X, Y) - k * k * m * u(X, Y)
    alpha = k * np.sqrt(m)
    # Robin data (d_n - i alpha) u* at the face midpoints, alpha of the boundary node
    xm_w, xm_e, ym_s, ym_n = h / 2, 1 - h / 2, h / 2, 1 - h / 2
    gw = -ux(xm_w, y) - 1j * alpha[:, 0] * u(xm_w, y)
    ge = ux(xm_e, y) - 1j * alpha[:, -1] * u(xm_e, y)
    gs = -uy(x, ym_s) - 1j * alpha[0, :] * u(x, ym_s)
    gn = uy(x, ym_n) - 1j * alpha[-1, :] * u(x, ym_n)
    rhs = f + g.outer_rhs(gw, ge, gs, gn)
    uh = direct_solve(g.matrix(), rhs.ravel()).reshape(n, n)
    return np.max(np.abs(uh - u(X, Y)))


@pytest.mark.parametrize("variable_m", [False, True])
def test_manufactured_second_order(variable_m):
    errs = [_manufactured(n, 6.0, variable_m) for n in (15, 31, 63)]
    rates = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.5 < r < 4.6 for r in rates), (errs, rates)
    assert errs[-1] < 2e-3


def test_symmetric():
    rng = np.random.default_rng(0)
    n = 12
    g = Grid(n, n, 1 / (n + 1), 20.0, 1 + 0.2 * rng.random((n, n)))
    A = g.matrix()
    assert abs(A - A.T).max() == 0
    # not Hermitian: the absorbing faces make it non-self-adjoint
    assert abs(A - A.conj().T).max() > 0


def test_outgoing_green_function():
    """Homogeneous medium, narrow Gaussian source at the centre: the field along a ray
    follows the outgoing (i/4) H0^(1)(k r), not the incoming (i/4) H0^(2)(k r)."""
    n = 159
    h = 1.0 / (n + 1)
    k = 2 * np.pi * 6
    g = Grid(n, n, h, k, np.ones((n, n)))
    x = (np.arange(n) + 1) * h
    X, Y = np.meshgrid(x, x)
    s = 1.5 * h
    f = np.exp(-((X - 0.5) ** 2 + (Y - 0.5) ** 2) / (2 * s * s)) / (2 * np.pi * s * s)
    u = direct_solve(g.matrix(), f.ravel().astype(np.complex128)).reshape(n, n)
    iy = n // 2
    r = np.abs(x - 0.5)
    sel = (r > 0.1) & (r < 0.3)
    ray = u[iy, sel]
    out = 0.25j * hankel1(0, k * r[sel])
    inc = 0.25j * hankel2(0, k * r[sel])

    def corr(a, b):
        return abs(np.vdot(a, b)) / (np.linalg.norm(a) * np.linalg.norm(b))

    assert corr(ray, out) > 0.97
    assert corr(ray, inc) < 0.5
    # the phase advances outward at about k per unit length
    ph = np.unwrap(np.angle(u[iy, n // 2 + 10:n // 2 + 45]))
    slope = np.polyfit(x[n // 2 + 10:n // 2 + 45], ph, 1)[0]
    assert abs(slope / k - 1) < 0.05


def test_dA_dm_matches_finite_difference():
    """The analytic derivative of the diagonal w.r.t. m (used by the gradient) against
    a central difference of the assembled matrix."""
    rng = np.random.default_rng(1)
    n = 9
    m = 1 + 0.2 * rng.random((n, n))
    g = Grid(n, n, 1 / (n + 1), 30.0, m)
    eps = 1e-6
    gp = Grid(n, n, g.h, g.k, m + eps)
    gm = Grid(n, n, g.h, g.k, m - eps)
    fd = (gp.matrix().diagonal() - gm.matrix().diagonal()) / (2 * eps)
    an = g.dA_dm_diag().ravel()
    assert np.max(np.abs(fd - an) / np.abs(an)) < 1e-7


def _stencil_by_node(nx, ny, h, k, m, u):
    """A u evaluated node by node from the definition (Sec. 3, eq. (1) with the face template):
    (4 u_p - sum of the in-grid neighbours)/h^2 - k^2 m_p u_p, where an outer face contributes the
    ghost value u_q = (beta+/beta-) u_p of the absorbing condition (data 0, alpha = k sqrt(m_p))."""
    out = np.zeros((ny, nx), dtype=np.complex128)
    for iy in range(ny):
        for ix in range(nx):
            up = u[iy, ix]
            alpha = k * np.sqrt(m[iy, ix])
            ghost = (1.0 / h + 0.5j * alpha) / (1.0 / h - 0.5j * alpha) * up
            s = 0.0j
            for jy, jx in ((iy, ix - 1), (iy, ix + 1), (iy - 1, ix), (iy + 1, ix)):
                s += u[jy, jx] if (0 <= jx < nx and 0 <= jy < ny) else ghost
            out[iy, ix] = (4.0 * up - s) / h**2 - k * k * m[iy, ix] * up
    return out


def test_volume_residual_pins():
    """oracle.solver.volume_residual: A u against the node-by-node stencil; exactly zero residual
    for f = A u and |delta| / ||f'|| after one entry of f is perturbed by delta; round-off for the
    direct solution; one value per right-hand side for a batch."""
    from oracle.solver import direct, volume_residual

    rng = np.random.default_rng(11)
    nx, ny = 9, 7
    h = 1.0 / (nx + 1)
    m = 1.0 + 0.2 * rng.random((ny, nx))
    g = Grid(nx, ny, h, 25.0, m)
    u = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    Au = _stencil_by_node(nx, ny, h, 25.0, m, u)
    assert np.max(np.abs((g.matrix() @ u.ravel()).reshape(ny, nx) - Au)) <= 1e-12 * np.max(np.abs(Au))
    assert volume_residual(g, u, Au) <= 1e-15
    delta = 0.37 - 0.21j
    fp = Au.copy()
    fp[3, 4] += delta
    assert abs(volume_residual(g, u, fp) - abs(delta) / np.linalg.norm(fp)) <= 1e-14
    f = rng.standard_normal((2, ny, nx)) + 0j
    ud = direct(g, f)
    r = volume_residual(g, ud, f)
    assert r.shape == (2,) and np.all(r < 1e-13)
    r2 = volume_residual(g, np.stack([u, u]), np.stack([Au, fp]))
    assert r2[0] <= 1e-15 and abs(r2[1] - abs(delta) / np.linalg.norm(fp)) <= 1e-14
