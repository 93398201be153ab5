"""Pins of the oracle's sweeping preconditioners (Secs. 5-6) against dense linear algebra.

* Proposition 1: the product of the elementary factors equals S_L (and S_U), and
  each factor is inverted by flipping its sign;
* the sweep implementation of S_U^{-1} S_L^{-1} equals dense triangular solves
  (scipy.linalg.solve_triangular);
* block Jacobi equals the dense restricted block formula of Sec. 6, and the
  literal additive formula for the "additive" reading;
* one partial sweep (p = 1) is SGS, for every composition.
"""
import numpy as np
import pytest

from oracle import layout, sweep
from oracle.dd import Decomposition
from oracle.fd import Grid


def _dd(nx, ny, n1, n2, seed=4):
    h = 1.0 / (nx + 1)
    k = 2 * np.pi / (8 * h)
    rng = np.random.default_rng(seed)
    m = 1 + 0.3 * rng.random((ny, nx))
    return Decomposition(Grid(nx, ny, h, k, m), n1, n2)


def _vec(n, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


@pytest.mark.parametrize("n1,n2", [(2, 2), (3, 3), (3, 4), (4, 2)])
def test_proposition_1(n1, n2):
    dd = _dd(3 * n1, 2 * n2, n1, n2)
    lay = dd.layout
    S = dd.dense_S()
    SL, SU = sweep.dense_SL_SU(lay, S)
    n = lay.nif
    prod_L = np.eye(n, dtype=complex)
    prod_U = np.eye(n, dtype=complex)
    for a in range(3, lay.n_g + 2):
        E = np.zeros((n, n), dtype=complex)
        E[lay.group_slice(a), lay.group_slice(a - 1)] = S[lay.group_slice(a), lay.group_slice(a - 1)]
        prod_L = prod_L @ (np.eye(n) - E)
        # (I + E)(I - E) = I because E^2 = 0
        assert np.abs((np.eye(n) + E) @ (np.eye(n) - E) - np.eye(n)).max() < 1e-15 * max(1, np.abs(E).max() ** 2)
        F = np.zeros((n, n), dtype=complex)
        F[lay.group_slice(a - 1), lay.group_slice(a)] = S[lay.group_slice(a - 1), lay.group_slice(a)]
        prod_U = (np.eye(n) - F) @ prod_U
    assert np.abs(prod_L - SL).max() < 1e-14
    assert np.abs(prod_U - SU).max() < 1e-14
    # S_L + S_U - I recovers I - S (the diagonal blocks of S vanish)
    assert np.abs(SL + SU - np.eye(n) - (np.eye(n) - S)).max() < 1e-14


@pytest.mark.parametrize("n1,n2", [(2, 2), (3, 3), (4, 3), (2, 5)])
def test_sgs_sweep_is_dense_triangular_solve(n1, n2):
    dd = _dd(3 * n1, 2 * n2, n1, n2)
    S = dd.dense_S()
    r = _vec(dd.nif, 1)
    st = sweep.SweepStats()
    z = sweep.apply_sgs(dd, r, stats=st)
    zd = sweep.dense_sgs(dd.layout, S, r)
    assert np.linalg.norm(z - zd) <= 1e-12 * np.linalg.norm(zd)
    assert st.steps == 2 * (dd.layout.n_g - 1)
    assert st.local_solves == 2 * (n1 * n2 - 1)


@pytest.mark.parametrize("n1,n2,width", [(3, 3, None), (4, 4, None), (3, 5, None), (5, 3, None), (4, 4, 2), (3, 3, 1)])
@pytest.mark.parametrize("combine", ["restricted", "additive"])
def test_bj_is_dense_block_formula(n1, n2, width, combine):
    dd = _dd(2 * n1, 2 * n2, n1, n2)
    S = dd.dense_S()
    r = _vec(dd.nif, 2)
    st = sweep.SweepStats()
    z = sweep.apply_bj(dd, r, width=width, combine=combine, stats=st)
    zd = sweep.dense_bj(dd.layout, S, r, width=width, combine=combine)
    assert np.linalg.norm(z - zd) <= 1e-12 * np.linalg.norm(zd)
    assert st.steps == sweep.step_counts(n1, n2, width)[1]


@pytest.mark.parametrize("n1,n2", [(2, 2), (2, 3), (3, 2)])
@pytest.mark.parametrize("compose", ["product", "residual"])
def test_one_partial_sweep_is_sgs(n1, n2, compose):
    """p = 1 (width >= N_g - 1): block Jacobi coincides with SGS."""
    dd = _dd(2 * n1, 2 * n2, n1, n2)
    n_g = dd.layout.n_g
    assert layout.num_partial_sweeps(n1, n2, n_g - 1) == 1
    r = _vec(dd.nif, 3)
    z_sgs = sweep.apply_sgs(dd, r)
    z_bj = sweep.apply_bj(dd, r, width=n_g - 1, compose=compose)
    if compose == "product":
        assert np.array_equal(z_bj, z_sgs)
    else:
        assert np.linalg.norm(z_bj - z_sgs) <= 1e-12 * np.linalg.norm(z_sgs)


def test_bj_differs_from_sgs_with_two_partial_sweeps():
    dd = _dd(8, 8, 4, 4)
    r = _vec(dd.nif, 4)
    assert layout.num_partial_sweeps(4, 4) == 2
    z_sgs = sweep.apply_sgs(dd, r)
    z_bj = sweep.apply_bj(dd, r)
    assert np.linalg.norm(z_bj - z_sgs) > 1e-3 * np.linalg.norm(z_sgs)
