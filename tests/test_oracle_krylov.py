"""Pins of the oracle's GMRES (Sec. 7) against dense solves and scipy's GMRES."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import sweep
from oracle.dd import Decomposition
from oracle.fd import Grid
from oracle.krylov import givens, gmres


def test_givens():
    rng = np.random.default_rng(0)
    for _ in range(50):
        a, b = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        c, s = givens(a, b)
        G = np.array([[c, s], [-np.conj(s), c]])
        v = G @ np.array([a, b])
        assert abs(v[1]) < 1e-15 * abs(v[0])
        assert np.allclose(G.conj().T @ G, np.eye(2), atol=1e-15)


@pytest.mark.parametrize("flexible", [False, True])
def test_gmres_dense(flexible):
    rng = np.random.default_rng(1)
    n = 40
    A = np.eye(n) + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    Mi = np.linalg.inv(np.diag(np.diag(A)))
    res = gmres(lambda v: A @ v, b, lambda v: Mi @ v, tol=1e-12, restart=n, flexible=flexible)
    x = np.linalg.solve(A, b)
    assert res.converged
    assert np.linalg.norm(res.x - x) <= 1e-10 * np.linalg.norm(x)
    # exact termination: at most n steps without restarts
    assert res.iters <= n


def test_gmres_restart_converges():
    rng = np.random.default_rng(2)
    n = 60
    A = np.eye(n) + 0.5 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 0j
    res = gmres(lambda v: A @ v, b, None, tol=1e-10, restart=5, maxit=2000)
    assert res.converged
    assert np.linalg.norm(A @ res.x - b) <= 1e-10 * np.linalg.norm(b)


def test_iterations_match_scipy_gmres():
    """Same preconditioned operator (I - S) P^{-1}: our GMRES(50) iteration count equals
    scipy's to within one."""
    n = 24
    h = 1.0 / (n + 1)
    rng = np.random.default_rng(3)
    g = Grid(n, n, h, 2 * np.pi / (10 * h), 1 + 0.2 * rng.random((n, n)))
    dd = Decomposition(g, 3, 3)
    b = rng.standard_normal(dd.nif) + 1j * rng.standard_normal(dd.nif)
    M = lambda v: sweep.apply_bj(dd, v)  # noqa: E731
    res = gmres(dd.apply_operator, b, M, tol=1e-8, restart=50)
    AM = spla.LinearOperator((dd.nif, dd.nif), matvec=lambda v: dd.apply_operator(M(v)), dtype=np.complex128)
    count = []
    y, info = spla.gmres(AM, b, rtol=1e-8, atol=0, restart=50, maxiter=100,
                         callback=lambda pr: count.append(pr), callback_type="pr_norm")
    assert info == 0
    assert abs(len(count) - res.iters) <= 1
    x = M(y)
    assert np.linalg.norm(x - res.x) <= 1e-6 * np.linalg.norm(x)


def test_zero_rhs():
    res = gmres(lambda v: 2 * v, np.zeros(5, dtype=complex))
    assert res.iters == 0 and np.all(res.x == 0)
