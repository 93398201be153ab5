"""The allocation-free volume residual (hbj_volume_residual_noalloc) against hbj_volume_residual,
through the C ABI: two calls in a row, the second on a smaller grid with fewer right-hand sides,
so the second call reads the shared per-device scratch after a larger call left it dirty.

Both entry points run the same partial-sum kernel; the allocation-free one sums the partials
and takes the ratio on the device, the other on the host, so the results agree to rounding of
the final division and square root (both correctly rounded in IEEE arithmetic).
"""
import numpy as np
import pytest

import workload as W
from cases import CASES, gpu_context, oracle_problem, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _fields(wl, nrhs, seed):
    rng = np.random.default_rng(seed)
    shape = (nrhs, wl.ny, wl.nx)
    u = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    f = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return f, u


def test_noalloc_volume_residual_matches_the_allocating_entry_point(hbj):
    # first call: 256^2 grid, 5 right-hand sides (one with a zero source, one a solved field)
    wl = CASES["grf256"].wl
    m, g, dd = oracle_problem(wl)
    ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE)
    ctx.factor()
    f, u = _fields(wl, 5, seed=31)
    f[1] = 0.0
    f[4] = W.sources(wl)[0]
    ft = torch.as_tensor(f, device="cuda")
    ut = torch.as_tensor(u, device="cuda")
    ut[4] = ctx.solve(ft[4], tol=1e-10)[0]
    say("[no-alloc residual] 256^2 grid, 5 right-hand sides")
    out = torch.full((5,), -1.0, dtype=torch.float64, device="cuda")
    ctx.volume_residual_noalloc(ft, ut, out)
    want = ctx.volume_residual(ft, ut)
    got = out.cpu().numpy()
    say(f"  no-alloc {list(got)}\n  allocating {want}")
    np.testing.assert_allclose(got, want, rtol=4 * np.finfo(np.float64).eps, atol=0)
    assert got[4] < 1e-8  # the solved field

    # the limit is checked on the host before anything is enqueued
    big = torch.zeros((hbj.VR_NOALLOC_MAX_RHS + 1, 1), dtype=torch.complex128, device="cuda")
    sentinel = torch.full((hbj.VR_NOALLOC_MAX_RHS + 1,), -7.0, dtype=torch.float64, device="cuda")
    code = hbj._lib.hbj_volume_residual_noalloc(ctx._h, hbj._P(big.data_ptr()), hbj._P(big.data_ptr()),
                                                hbj.VR_NOALLOC_MAX_RHS + 1, hbj._P(sentinel.data_ptr()))
    assert code == hbj.EINVAL
    assert bool((sentinel == -7.0).all())
    ctx.close()

    # second call: a smaller grid (48 x 24, 3 x 2 subdomains) and fewer right-hand sides
    wl2 = CASES["rect"].wl
    m2, g2, dd2 = oracle_problem(wl2)
    ctx2 = gpu_context(hbj, wl2, m2)
    f2, u2 = _fields(wl2, 2, seed=32)
    ft2 = torch.as_tensor(f2, device="cuda")
    ut2 = torch.as_tensor(u2, device="cuda")
    say("[no-alloc residual] 48 x 24 grid, 2 right-hand sides")
    out2 = torch.full((2,), -1.0, dtype=torch.float64, device="cuda")
    ctx2.volume_residual_noalloc(ft2, ut2, out2)
    want2 = ctx2.volume_residual(ft2, ut2)
    got2 = out2.cpu().numpy()
    say(f"  no-alloc {list(got2)}\n  allocating {want2}")
    np.testing.assert_allclose(got2, want2, rtol=4 * np.finfo(np.float64).eps, atol=0)
    ctx2.close()
