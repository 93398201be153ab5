"""Pins of the oracle's adjoint gradient against central finite differences and the
dot-product identity of the (complex symmetric) operator."""
import numpy as np

import workload as W
from oracle import gradient, solver
from oracle.dd import Decomposition
from oracle.fd import Grid


def _problem(n=16, nsrc=2, seed=7):
    h = 1.0 / (n + 1)
    k = 2 * np.pi / (10 * h)
    rng = np.random.default_rng(seed)
    from scipy.ndimage import gaussian_filter

    z = gaussian_filter(rng.standard_normal((n, n)), 2.0)
    m_true = np.clip(1 + 0.1 * z / z.std(), 0.8, 1.2)
    m0 = gaussian_filter(m_true, 3.0, mode="nearest")
    f = np.stack([W.gaussian_source(n, n, h, (s + 0.5) / nsrc, 0.15) for s in range(nsrc)])
    rec = ((n - 3) * n + np.arange(n)).astype(np.int64)
    d = np.stack([solver.direct(Grid(n, n, h, k, m_true), f[s]).ravel()[rec] for s in range(nsrc)])
    return h, k, m_true, m0, f, rec, d


def test_gradient_central_differences():
    h, k, m_true, m0, f, rec, d = _problem()
    n = m0.shape[0]
    L0, grad = gradient.misfit_and_gradient(Grid(n, n, h, k, m0), f, rec, d)
    eps = 1e-6
    for j in range(6):
        dm = np.random.default_rng(100 + j).standard_normal(m0.shape)
        dm /= np.abs(dm).max()
        Lp = gradient.misfit(Grid(n, n, h, k, m0 + eps * dm), f, rec, d)
        Lm = gradient.misfit(Grid(n, n, h, k, m0 - eps * dm), f, rec, d)
        fd = (Lp - Lm) / (2 * eps)
        an = float(np.sum(grad * dm))
        assert abs(fd - an) <= 1e-5 * abs(an), (fd, an)


def test_gradient_through_dd_solves():
    """The same gradient with every solve done by the domain-decomposition method."""
    h, k, m_true, m0, f, rec, d = _problem(n=16, nsrc=1)
    n = m0.shape[0]
    g = Grid(n, n, h, k, m0)
    dd = Decomposition(g, 2, 2)
    solve = lambda rhs: solver.dd_solve(dd, rhs, tol=1e-13).u  # noqa: E731
    L1, g1 = gradient.misfit_and_gradient(g, f, rec, d, solve=solve)
    L0, g0 = gradient.misfit_and_gradient(g, f, rec, d)
    assert abs(L1 - L0) <= 1e-10 * L0
    assert np.linalg.norm(g1 - g0) <= 1e-9 * np.linalg.norm(g0)


def test_dot_product_identity():
    h, k, m_true, m0, f, rec, d = _problem()
    n = m0.shape[0]
    A = Grid(n, n, h, k, m0).matrix()
    rng = np.random.default_rng(9)
    u = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    v = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    lhs = np.vdot(v, A @ u)
    rhs = np.vdot(A.conj().T @ v, u)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # complex symmetry: A^H v = conj(A conj(v))
    assert np.allclose(A.conj().T @ v, np.conj(A @ np.conj(v)), rtol=1e-14, atol=0)


def test_stored_finite_differences_reproduce():
    """tests/golden/grad_512_fd.json (written by tests/golden/make_grad_fd.py from the oracle) holds
    the oracle's misfit at m0 +- eps dm_j for the 512^2 gradient workload; the loss at m0 and
    direction 0 are recomputed here."""
    import importlib.util
    import json
    import os

    here = os.path.dirname(os.path.abspath(__file__))
    gold = json.load(open(os.path.join(here, "golden", "grad_512_fd.json")))
    spec = importlib.util.spec_from_file_location("make_grad_fd", os.path.join(here, "golden", "make_grad_fd.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    import workload as W
    from oracle import gradient, solver
    from oracle.fd import Grid

    wl, m_true, m0, f, rec = mod.problem()
    assert gold["eps"] == mod.EPS and len(gold["directions"]) == mod.NDIR
    u = solver.direct(Grid(wl.nx, wl.ny, wl.h, wl.k, m_true), f)
    d = np.ascontiguousarray(u.reshape(f.shape[0], -1)[:, rec])
    L0 = gradient.misfit(Grid(wl.nx, wl.ny, wl.h, wl.k, m0), f, rec, d)
    assert abs(L0 - gold["loss_m0"]) <= 1e-11 * L0
    dm = W.gradient_direction(m0.shape, 0)
    Lp = gradient.misfit(Grid(wl.nx, wl.ny, wl.h, wl.k, m0 + mod.EPS * dm), f, rec, d)
    e0 = gold["directions"][0]
    assert abs(Lp - e0["loss_plus"]) <= 1e-11 * Lp
    for e in gold["directions"]:
        assert abs(e["fd"] - (e["loss_plus"] - e["loss_minus"]) / (2 * gold["eps"])) <= 1e-12 * abs(e["fd"])
