"""Pins of the second-order transmission condition in the oracle (NEXT row: higher-order transmission).

The condition d_n u - i alpha a u - (i b / alpha) d_tt u = g on interface faces changes the local
matrices and the data sent across faces, never the global problem (the outer faces keep the
first-order absorbing condition). Hence the same identities as for the first-order condition must
hold exactly: the traces g* of the global solution solve (I - S) g = b, and the reconstruction from
g* is the global solution; a wrong R or Sigma band, a sign of the tangential term or a face-end
closure that differs between the two sides of a face breaks them. Further: the local matrices stay
complex symmetric (the symmetric edge weights), the condition reduces to the first-order one for
(a, b) = (1, 0), and a face of one entry has no tangential term.
"""
import numpy as np
import pytest

import workload as W
from oracle import solver
from oracle.dd import SECOND_ORDER, Decomposition
from oracle.fd import Grid


def _grid(nx, ny, seed=3, ppw=8.0):
    h = 1.0 / (nx + 1)
    k = 2 * np.pi / (ppw * h)
    rng = np.random.default_rng(seed)
    from scipy.ndimage import gaussian_filter

    z = gaussian_filter(rng.standard_normal((ny, nx)), 2.0)
    m = 1.0 / np.clip(1 + 0.1 * z / z.std(), 0.8, 1.2) ** 2
    f = W.gaussian_source(nx, ny, h, 0.37, 0.61 * (ny + 1) * h)
    f = f + 0.3j * W.gaussian_source(nx, ny, h, 0.8, 0.2 * (ny + 1) * h)
    return Grid(nx, ny, h, k, m), f


CASES = [(12, 12, 1, 1), (12, 12, 2, 2), (12, 12, 3, 2), (12, 18, 2, 3), (16, 16, 4, 4), (15, 10, 5, 2), (8, 8, 8, 1),
         (9, 9, 9, 9)]


@pytest.mark.parametrize("tcoef", [None, (1.0, 0.5), (0.8 + 0.1j, 0.3 * np.exp(-1j))])
@pytest.mark.parametrize("nx,ny,n1,n2", CASES)
def test_second_order_traces_solve_interface_system(nx, ny, n1, n2, tcoef):
    g, f = _grid(nx, ny)
    dd = Decomposition(g, n1, n2, transmission=2, tcoef=tcoef)
    u = solver.direct(g, f)
    gs = dd.traces_of(u)
    b = dd.lifting(f)
    if dd.nif:
        assert np.linalg.norm(dd.apply_operator(gs) - b) <= 1e-12 * np.linalg.norm(b)
    assert np.linalg.norm(dd.reconstruct(f, gs) - u) <= 1e-12 * np.linalg.norm(u)
    for s in dd.sub.values():
        assert abs(s.A - s.A.T).max() == 0.0


def test_second_order_with_zero_tangential_term_is_first_order():
    g, f = _grid(12, 12)
    d1 = Decomposition(g, 3, 2)
    d2 = Decomposition(g, 3, 2, transmission=2, tcoef=(1.0, 0.0))
    assert np.array_equal(d1.dense_S(), d2.dense_S())
    assert np.array_equal(d1.lifting(f), d2.lifting(f))


def test_second_order_changes_the_interface_operator_only_along_faces():
    """S differs from the first-order S, and a one-entry face carries no tangential term."""
    g, f = _grid(12, 12)
    d1 = Decomposition(g, 3, 2)
    d2 = Decomposition(g, 3, 2, transmission=2)
    assert np.abs(d1.dense_S() - d2.dense_S()).max() > 1e-3
    g9, _ = _grid(9, 9)
    d9 = Decomposition(g9, 9, 9, transmission=2)  # 1 x 1 subdomains: faces of one entry
    assert all(not C.any() for s in d9.sub.values() for C in s.tang.values())


def test_second_order_face_maps_against_the_ghost_relation():
    """R and Sigma from the closed form against the two-sided ghost construction: the data j
    sends is i's condition evaluated on j's ghost line u~ = B-^{-1}(g + B+ u) + C u."""
    g, _ = _grid(12, 12)
    dd = Decomposition(g, 2, 2, transmission=2)
    i = (1, 1)
    s = dd.sub[i]
    f = "E"
    bm, bp = s.coef[f][0], s.coef[f][1]
    C = s.tang[f]
    rng = np.random.default_rng(0)
    u = rng.standard_normal(bm.size) + 1j * rng.standard_normal(bm.size)
    gin = rng.standard_normal(bm.size) + 1j * rng.standard_normal(bm.size)
    ghost = (gin + bp * u) / bm + C @ u
    direct = bm * u - bp * ghost - bm * (C @ ghost)
    R, Sig = dd.face_maps(i, f)
    assert np.allclose(-R @ gin - Sig @ u, direct, rtol=1e-13, atol=0)


def test_second_order_gmres_converges_in_fewer_iterations():
    """Property (not a pin of a value): on the bench physics at 128^2, 4 x 4 the block-Jacobi
    preconditioned GMRES needs fewer iterations with the default second-order condition."""
    wl = W.Workload("t", 128, 128, 4, 4, 10.0, "random_smooth", 3, ((0.37, 0.61),))
    m = W.slowness2(wl)
    g = Grid(wl.nx, wl.ny, wl.h, wl.k, m)
    f = W.sources(wl)[0]
    it = {}
    for order in (1, 2):
        dd = Decomposition(g, 4, 4, transmission=order)
        r = solver.dd_solve(dd, f, precond="bj", tol=1e-6, maxit=300)
        assert r.relres <= 1e-6
        it[order] = r.iters
    assert it[2] < 0.8 * it[1], it
    assert SECOND_ORDER[1] != 0
