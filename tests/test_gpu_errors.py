"""Failure paths of the C ABI, each forced from the host with valid inputs.

Bad media, calls out of order, an exactly singular local matrix (2 x 2 grid, k = 0: a
pure Neumann Laplacian whose last band-LU pivot is exactly zero, as LAPACK's zgbtrf also
reports), GMRES stopped by maxit, and duplicated receivers.
"""
import numpy as np
import pytest

import workload as W
from cases import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _c(nx, ny, val=1.0):
    return torch.full((ny, nx), val, dtype=torch.float64, device="cuda")


def test_bad_medium_rejected(hbj):
    for bad in (float("nan"), -1.0, 0.0, float("inf")):
        c = _c(16, 16)
        c[3, 5] = bad
        say(f"[errors] medium value {bad}")
        with pytest.raises(hbj.HbjError) as ei:
            hbj.setup(16, 16, 10.0, 2, 2, c=c)
        assert ei.value.code == hbj.EINVAL


def test_bad_slowness_rejected(hbj):
    ctx = hbj.setup(16, 16, 10.0, 2, 2, c=_c(16, 16))
    m = _c(16, 16)
    m[0, 0] = float("nan")
    with pytest.raises(hbj.HbjError) as ei:
        ctx.set_slowness2(m)
    assert ei.value.code == hbj.EINVAL
    ctx.close()


def test_out_of_order(hbj):
    ctx = hbj.setup(16, 16, 10.0, 2, 2, c=_c(16, 16))
    f = torch.zeros((16, 16), dtype=torch.complex128, device="cuda")
    say("[errors] solve before factor")
    with pytest.raises(hbj.HbjError) as ei:
        ctx.solve(f)
    assert ei.value.code == hbj.ESTATE
    ctx.factor()
    ctx.set_slowness2(_c(16, 16, 1.1))  # a new medium invalidates the factors
    with pytest.raises(hbj.HbjError) as ei:
        ctx.apply_operator(torch.zeros(ctx.nif, dtype=torch.complex128, device="cuda"))
    assert ei.value.code == hbj.ESTATE
    ctx.close()


def test_zero_pivot_reported(hbj):
    ctx = hbj.setup(2, 2, 0.0, 1, 1, c=_c(2, 2))
    say("[errors] singular local matrix")
    with pytest.raises(hbj.HbjError) as ei:
        ctx.factor()
    assert ei.value.code == hbj.ZERO_PIVOT
    assert "subdomain 0 row 3" in str(ei.value)
    ctx.close()


def test_not_converged_fills_stats(hbj):
    wl = W.SMALL
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=torch.as_tensor(W.slowness2(wl), device="cuda"))
    ctx.factor()
    f = torch.as_tensor(W.sources(wl)[0], device="cuda")
    say("[errors] maxit=2")
    u, st = ctx.solve(f, tol=1e-12, maxit=2, check=False)
    assert st.code == hbj.NOT_CONVERGED
    assert st.iters == 2 and st.converged == 0 and st.relres > 1e-12
    assert torch.isfinite(torch.view_as_real(u)).all()
    with pytest.raises(hbj.HbjError) as ei:
        ctx.solve(f, tol=1e-12, maxit=2)
    assert ei.value.code == hbj.NOT_CONVERGED
    ctx.close()


def test_duplicate_receivers_rejected(hbj):
    wl = W.SMALL
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=torch.as_tensor(W.slowness2(wl), device="cuda"))
    ctx.factor()
    f = torch.as_tensor(W.sources(wl), device="cuda")
    rec = torch.tensor([5, 7, 5], dtype=torch.int32, device="cuda")
    d = torch.zeros((1, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(hbj.HbjError) as ei:
        ctx.gradient(f, rec, d)
    assert ei.value.code == hbj.EINVAL
    ctx.close()
