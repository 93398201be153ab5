"""Shared parity cases: the same seeded problem for the oracle (CPU) and the HIP path."""
from __future__ import annotations

import dataclasses
import sys

import numpy as np

import workload as W


@dataclasses.dataclass(frozen=True)
class Case:
    name: str
    wl: W.Workload


def _wl(name, nx, ny, n1, n2, medium="random_smooth", seed=3, ppw=10.0, src=((0.37, 0.61),)):
    return W.Workload(name, nx, ny, n1, n2, ppw, medium, seed, src)


CASES = {
    # the 64^2, 2 x 2 homogeneous problem (10 points per wavelength, source at the centre)
    "small": Case("small", W.SMALL),
    # the 1024^2 / 8 x 8 random-medium problem at 256^2 (32^2 subdomains): same physics, several tiles
    "grf256": Case("grf256", W.scaled(W.FP64_1024, 256)),
    # ragged solve blocks (10 x 10 subdomains: 100 rows = 3 full blocks of 32 + 4)
    "ragged": Case("ragged", _wl("ragged", 40, 30, 4, 3)),
    # rectangular subdomains and grid (16 x 12)
    "rect": Case("rect", _wl("rect", 48, 24, 3, 2, seed=5)),
    # a single subdomain: no interfaces
    "one": Case("one", _wl("one", 16, 16, 1, 1)),
    # about 3 points per wavelength: the local matrices need row interchanges
    "pivot": Case("pivot", _wl("pivot", 40, 40, 2, 2, ppw=3.2)),
    # a long strip of subdomains (5 x 10, paper's Table 1 layout) with 8 x 8 subdomains
    "strip": Case("strip", _wl("strip", 40, 80, 5, 10, seed=7, ppw=8.0, src=((0.5, 0.3),))),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_problem(wl: W.Workload):
    from oracle.dd import Decomposition
    from oracle.fd import Grid

    m = W.slowness2(wl)
    g = Grid(wl.nx, wl.ny, wl.h, wl.k, m)
    dd = Decomposition(g, wl.n1, wl.n2) if True else None
    return m, g, dd


def gpu_context(hbj, wl: W.Workload, m, **kw):
    import torch

    mt = torch.as_tensor(m, dtype=torch.float64, device="cuda")
    return hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=mt, **kw)


def sub_index(wl, i):
    """Library subdomain index of multi-index i = (i1, i2)."""
    return (i[1] - 1) * wl.n1 + (i[0] - 1)


def residual_rounding_bound(grid, u, f):
    """Bound on the difference between two evaluations of ||f - A u|| / ||f|| that sum in
    different orders: each entry of f - A u carries a rounding error of at most about
    gamma (|f_p| + sum_q |A_pq| |u_q|) with gamma = 8 eps for the five stencil terms and the
    subtraction (Higham, Accuracy and Stability of Numerical Algorithms, Sec. 3.1), so the two
    relative residuals differ by at most 2 gamma || |f| + |A| |u| || / ||f||.  A residual near
    round-off (a converged solve) can differ by much more than its own relative precision."""
    A = abs(grid.matrix())
    u = np.asarray(u).ravel()
    f = np.asarray(f).ravel()
    gamma = 8 * np.finfo(np.float64).eps
    return 2 * gamma * np.linalg.norm(np.abs(f) + A @ np.abs(u)) / np.linalg.norm(f)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    d = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (d if d > 0 else 1.0)
