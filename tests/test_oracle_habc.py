"""Pins of the oracle's Pade transmission condition (oracle.habc and transmission=3 of
oracle.dd): the paper's experiments use a Pade-type high-order absorbing condition with
N_pade = 8 and phi = pi/3 on every interface (Sec. 7).

* the rational function against the square root it approximates, propagating and evanescent
  (the decaying branch), with the error falling as N grows, and the unrotated expansion failing
  on evanescent modes (why the branch cut is rotated);
* the matrix function R(D) (partial fractions with inverses) against the spectral definition
  V R(Lambda) V^T of the symmetric tangential operator, and D 1 = 0 (Neumann ends);
* the face template's algebra: ghost values satisfy the condition, the data sent across equal
  -rho g - sigma u_p;
* N = 0 without rotation is the Robin condition exactly;
* the traces of the global solution satisfy the interface system exactly and reconstruct the
  global solution; the local matrices stay complex symmetric;
* qualitatively, fewer block-Jacobi GMRES iterations than the Robin condition on a homogeneous
  medium (the paper's reason for the condition).
"""
import numpy as np
import pytest

import workload as W
from cases import CASES, rel
from oracle import habc, solver
from oracle.dd import Decomposition
from oracle.fd import Grid


def _sqrt_outgoing(z):
    """sqrt(1 + z) on the branch of outgoing / decaying waves: >= 0 for z >= -1, i sqrt(-1 - z) below."""
    z = np.asarray(z, dtype=np.float64)
    return np.where(z >= -1.0, np.sqrt(np.maximum(1.0 + z, 0.0)), 1j * np.sqrt(np.maximum(-1.0 - z, 0.0)))


def test_pade_rational_approximates_the_square_root():
    zp = np.linspace(-0.95, 0.0, 60)   # propagating modes
    ze = np.linspace(-5.0, -1.05, 60)  # evanescent modes
    errs = []
    for n in (2, 4, 8, 16):
        ep = np.max(np.abs(habc.pade_sqrt(zp, n, np.pi / 3) - _sqrt_outgoing(zp)))
        ee = np.max(np.abs(habc.pade_sqrt(ze, n, np.pi / 3) - _sqrt_outgoing(ze)))
        errs.append((ep, ee))
    for (p0, e0), (p1, e1) in zip(errs, errs[1:]):
        assert p1 < p0 and e1 < e0
    ep8, ee8 = errs[2]
    assert ep8 < 1e-3 and ee8 < 2e-2
    # C0 is the value at z = 0, i.e. approximately sqrt(1) = 1
    assert abs(habc.pade_coefficients(8, np.pi / 3)[0] - 1.0) < 1e-8
    # without the rotation the expansion is real on the real axis and misses evanescent modes
    assert np.max(np.abs(habc.pade_sqrt(ze, 8, 0.0) - _sqrt_outgoing(ze))) > 1.0


def test_face_operator_is_the_matrix_function_of_the_tangential_operator():
    rng = np.random.default_rng(4)
    n, h = 12, 1.0 / 65
    kappa = 40.0 * (1.0 + 0.2 * rng.random(n))
    D = habc.tangential_operator(kappa, h)
    assert np.allclose(D, D.T)
    assert np.allclose(D @ np.ones(n), 0.0)
    lam, V = np.linalg.eigh(D)
    assert lam.max() < 1e-9  # negative semidefinite: d_tau (kappa^-2 d_tau)
    for npade, phi in ((8, np.pi / 3), (3, np.pi / 4)):
        R = habc.face_operator(D, npade, phi)
        spectral = (V * habc.pade_sqrt(lam, npade, phi)[None, :]) @ V.T
        assert rel(R, spectral) < 1e-12
        assert rel(R, R.T) < 1e-13
        X = habc.face_impedance(kappa, h, npade, phi)
        assert rel(X, np.sqrt(kappa)[:, None] * spectral * np.sqrt(kappa)[None, :]) < 1e-12
    # D is the second difference d_tau (kappa^-2 d_tau): on a smooth profile along a face of constant
    # kappa it reproduces -(pi / L)^2 / kappa^2 times the profile (second order in h)
    m, hh, kc = 64, 1.0 / 257, 30.0
    t = (np.arange(m) + 0.5) * hh
    v = np.cos(np.pi * t / (m * hh))
    Dv = habc.tangential_operator(np.full(m, kc), hh) @ v
    want = -(np.pi / (m * hh)) ** 2 / kc**2 * v
    assert np.max(np.abs(Dv - want)[1:-1]) < 1e-3 * np.max(np.abs(want))
    # constant kappa: X = kappa R(D)
    D1 = habc.tangential_operator(np.full(n, 40.0), h)
    assert rel(habc.face_impedance(np.full(n, 40.0), h, 8, np.pi / 3), 40.0 * habc.face_operator(D1, 8, np.pi / 3)) < 1e-13


def test_face_template_algebra():
    rng = np.random.default_rng(5)
    n, h = 10, 1.0 / 41
    kappa = 25.0 * (1.0 + 0.1 * rng.random(n))
    P = habc.face_maps(kappa, h, 8, np.pi / 3)
    X = P["X"]
    g = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    up = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    uq = P["Q"] @ (g + P["bp"] @ up)  # ghost values of the side that owns up
    assert rel((uq - up) / h - 0.5j * X @ (up + uq), g) < 1e-12
    # what the other side's condition sees (its own node is the ghost q, its ghost is p)
    seen = (up - uq) / h - 0.5j * X @ (uq + up)
    assert rel(seen, -P["rho"] @ g - P["sigma"] @ up) < 1e-12
    eye = np.eye(n)
    assert rel(P["rho"], 2.0 / h * P["Q"] - eye) < 1e-12
    assert rel(P["sigma"], 4.0 / h * (P["Q"] / h - eye)) < 1e-10
    for k in ("rho", "sigma", "inj"):
        assert rel(P[k], P[k].T) < 1e-12


def test_pade_without_terms_or_rotation_is_the_robin_condition():
    wl = CASES["rect"].wl
    g = Grid(wl.nx, wl.ny, wl.h, wl.k, W.slowness2(wl))
    d1 = Decomposition(g, wl.n1, wl.n2, transmission=1)
    d3 = Decomposition(g, wl.n1, wl.n2, transmission=3, tcoef=(0, 0.0))
    for i in d1.sub:
        assert rel(d3.sub[i].A.toarray(), d1.sub[i].A.toarray()) < 1e-14
    f = W.sources(wl)[0]
    assert rel(d3.lifting(f), d1.lifting(f)) < 1e-13
    gv = W.random_interface_vector(d1.nif, seed=9)
    assert rel(d3.apply_operator(gv), d1.apply_operator(gv)) < 1e-13


@pytest.mark.parametrize("name", ["small", "rect", "ragged", "strip", "one"])
def test_pade_interface_identities(name):
    wl = CASES[name].wl
    g = Grid(wl.nx, wl.ny, wl.h, wl.k, W.slowness2(wl))
    dd = Decomposition(g, wl.n1, wl.n2, transmission=3)
    f = W.sources(wl)[0]
    ud = solver.direct(g, f)
    gs = dd.traces_of(ud)
    b = dd.lifting(f)
    assert np.linalg.norm(dd.apply_operator(gs) - b) <= 1e-11 * np.linalg.norm(b)
    assert rel(dd.reconstruct(f, gs), ud) < 1e-11
    for s in dd.sub.values():
        A = s.A.toarray()
        assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()


def test_pade_needs_fewer_iterations_than_robin():
    """Homogeneous medium, 5 x 5 subdomains of 32^2, 10 points per wavelength: block-Jacobi
    GMRES to 1e-6 (a qualitative check of the condition's purpose; measured 15 against 24)."""
    wl = W.Workload("homog160", 160, 160, 5, 5, 10.0, "homogeneous", 0, ((0.5, 0.5),))
    g = Grid(wl.nx, wl.ny, wl.h, wl.k, W.slowness2(wl))
    f = W.sources(wl)[0]
    it = {}
    for tr in (1, 3):
        it[tr] = solver.dd_solve(Decomposition(g, wl.n1, wl.n2, transmission=tr), f, precond="bj", tol=1e-6).iters
    assert it[3] < it[1]
