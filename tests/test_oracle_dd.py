"""Pins of the oracle's interface problem (Secs. 3-4) against the global direct solve.

The discrete face template is consistent: the global solution restricted to each
subdomain solves every local problem when the transmission data are its own
traces.  Hence (I - S) g* = b holds exactly for the traces g* of the global
solution, and the field reconstructed from the solution of (I - S) g = b is the
global solution, on any checkerboard (1 x 1 included).  A wrong sign or factor
in rho / sigma / the injection, a transposed block of the m layout or a missing
reflection term breaks these identities.
"""
import numpy as np
import pytest

import workload as W
from oracle.dd import Decomposition
from oracle.fd import Grid
from oracle import solver


def _setup(nx, ny, n1, n2, seed=3, ppw=8.0):
    h = 1.0 / (nx + 1)
    k = 2 * np.pi / (ppw * h)
    rng = np.random.default_rng(seed)
    from scipy.ndimage import gaussian_filter

    z = gaussian_filter(rng.standard_normal((ny, nx)), 2.0)
    m = 1.0 / np.clip(1 + 0.1 * z / z.std(), 0.8, 1.2) ** 2
    g = Grid(nx, ny, h, k, m)
    f = W.gaussian_source(nx, ny, h, 0.37, 0.61 * (ny + 1) * h)
    f = f + 0.3j * W.gaussian_source(nx, ny, h, 0.8, 0.2 * (ny + 1) * h)
    return g, Decomposition(g, n1, n2), f


CASES = [(12, 12, 1, 1), (12, 12, 2, 2), (12, 12, 3, 2), (12, 18, 2, 3), (16, 16, 4, 4), (15, 10, 5, 2), (8, 8, 8, 1)]


@pytest.mark.parametrize("nx,ny,n1,n2", CASES)
def test_traces_of_global_solution_solve_interface_system(nx, ny, n1, n2):
    g, dd, f = _setup(nx, ny, n1, n2)
    u = solver.direct(g, f)
    gs = dd.traces_of(u)
    b = dd.lifting(f)
    if dd.nif == 0:
        return
    res = dd.apply_operator(gs) - b
    assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(b)
    # and the reconstruction from g* is the global solution
    ur = dd.reconstruct(f, gs)
    assert np.linalg.norm(ur - u) <= 1e-12 * np.linalg.norm(u)


@pytest.mark.parametrize("nx,ny,n1,n2", CASES)
def test_dense_interface_solve_reproduces_direct(nx, ny, n1, n2):
    g, dd, f = _setup(nx, ny, n1, n2)
    u = solver.direct(g, f)
    b = dd.lifting(f)
    if dd.nif:
        S = dd.dense_S()
        gg = np.linalg.solve(np.eye(dd.nif) - S, b)
    else:
        gg = b
    ur = dd.reconstruct(f, gg)
    assert np.linalg.norm(ur - u) <= 1e-11 * np.linalg.norm(u)


def test_S_group_structure():
    """Sec. 5: S_{a,b} = 0 unless |a - b| = 1 (neighbours differ by one in |i|_1)."""
    g, dd, _ = _setup(12, 12, 3, 4)
    S = dd.dense_S()
    lay = dd.layout
    for a in range(2, lay.n_g + 2):
        for c in range(2, lay.n_g + 2):
            blk = S[lay.group_slice(a), lay.group_slice(c)]
            if abs(a - c) == 1:
                assert np.abs(blk).max() > 0
            else:
                assert np.abs(blk).max() == 0


def test_local_solve_is_dense_solve():
    """A_i from the sparse assembly against a dense solve of the same local problem,
    and the scattering of unit data against the explicit formula -rho g - sigma u."""
    g, dd, _ = _setup(12, 12, 2, 2)
    i = (1, 2)
    s = dd.sub[i]
    rng = np.random.default_rng(5)
    gv = rng.standard_normal(dd.nif) + 1j * rng.standard_normal(dd.nif)
    rhs = dd.local_rhs(i, gv)
    u1 = dd.local_solve(i, gv)
    u2 = np.linalg.solve(s.A.toarray(), rhs)
    assert np.allclose(u1, u2, rtol=1e-12, atol=0)


def test_one_by_one_is_direct():
    """1 x 1 decomposition: no interfaces, the lifting alone is the direct solve."""
    g, dd, f = _setup(10, 10, 1, 1)
    assert dd.nif == 0
    r = solver.dd_solve(dd, f, precond="bj")
    u = solver.direct(g, f)
    assert r.iters == 0
    assert np.linalg.norm(r.u - u) <= 1e-13 * np.linalg.norm(u)
