"""The volume residual ||f - A u|| / ||f|| of the global problem (Sec. 3, eq. (1)) and the
GMRES / flexible GMRES choice of hbj_solve, through the C ABI.

The library's residual kernel is compared with the oracle's volume_residual (pinned on the CPU
against a node-by-node stencil) for random fields, where the residual is of order one, and for
fields from solves, where it measures the solution quality.
"""
import numpy as np
import pytest

import workload as W
from cases import CASES, gpu_context, oracle_problem, rel, residual_rounding_bound, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name", ["small", "rect", "ragged", "grf256"])
def test_volume_residual_matches_oracle(hbj, name):
    from oracle import solver

    wl = CASES[name].wl
    m, g, dd = oracle_problem(wl)
    say(f"[volume residual] case={name}")
    ctx = gpu_context(hbj, wl, m)  # the residual needs the medium only (no factorisation)
    rng = np.random.default_rng(21)
    shape = (3, wl.ny, wl.nx)
    u = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    f = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    f[2] = 0.0  # a zero source: the residual is then ||A u|| itself
    got = ctx.volume_residual(torch.as_tensor(f, device="cuda"), torch.as_tensor(u, device="cuda"))
    want = solver.volume_residual(g, u[:2], f[:2])
    au = np.linalg.norm(g.matrix() @ u[2].ravel())
    say(f"  gpu {got} oracle {list(want)} |A u| {au:.6e}")
    assert max(abs(got[k] - want[k]) / want[k] for k in range(2)) < 1e-12
    assert abs(got[2] - au) / au < 1e-12
    # the exact field of f has a residual at round-off
    ud = solver.direct(g, f[0])
    r = ctx.volume_residual(torch.as_tensor(f[:1], device="cuda"), torch.as_tensor(ud[None], device="cuda"))[0]
    assert r < 1e-12 and solver.volume_residual(g, ud, f[0]) < 1e-12
    ctx.close()


def test_volume_residual_of_solves_and_bad_arguments(hbj):
    from oracle import solver

    wl = CASES["grf256"].wl
    m, g, dd = oracle_problem(wl)
    ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE)
    ctx.factor()
    f = W.sources(wl)[0]
    ft = torch.as_tensor(f, device="cuda")
    say("[volume residual of solves]")
    prev = None
    for tol in (1e-6, 1e-9, 1e-12):
        u, st = ctx.solve(ft, tol=tol)
        r = ctx.volume_residual(ft, u)[0]
        ro = solver.volume_residual(g, _np(u), f)
        say(f"  tol {tol:g}: iters {st.iters}, volume residual gpu {r:.3e} oracle {ro:.3e}")
        assert abs(r - ro) <= residual_rounding_bound(g, _np(u), f)
        if prev is not None:
            assert r < prev
        prev = r
    assert prev < 1e-9
    with pytest.raises(ValueError):
        ctx.volume_residual(ft[None], u)
    ctx.close()


@pytest.mark.parametrize("name,kw,restart", [
    ("grf256", dict(precond=2), 50),
    ("grf256", dict(precond=2), 7),
    ("grf256", dict(precond=2, precision=1), 50),
    ("ragged", dict(precond=2, operator_form=0), 50),
])
def test_gmres_and_flexible_gmres_agree(hbj, name, kw, restart):
    """flexible=0 (only the Krylov basis kept, one more preconditioner application per cycle) and
    flexible=1 (preconditioned directions kept) give the same iterates up to rounding."""
    from oracle import solver

    wl = CASES[name].wl
    m, g, dd = oracle_problem(wl)
    kw = dict(kw)
    kw.setdefault("operator_form", hbj.OP_DENSE)
    ctx = gpu_context(hbj, wl, m, **kw)
    ctx.factor()
    f = W.sources(wl)[0]
    ft = torch.as_tensor(f, device="cuda")
    ud = solver.direct(g, f)
    res = {}
    for flex in (False, True):
        for orth in (hbj.ORTH_CGS2, hbj.ORTH_DCGS2):
            ctx.set_orthogonalization(orth)
            say(f"[gmres] case={name} {kw} restart={restart} flexible={flex} orth={orth}")
            u, st = ctx.solve(ft, tol=1e-12, restart=restart, maxit=3000, flexible=flex)
            assert st.relres <= 1e-12
            res[(flex, orth)] = (_np(u), st.iters)
    its = [v[1] for v in res.values()]
    say(f"  iterations {its}")
    assert max(its) - min(its) <= 1
    for u, _ in res.values():
        assert rel(u, ud) < 1e-8
    opts = hbj.SolveOpts(1e-6, 50, 100, 2)
    code = hbj._lib.hbj_solve(ctx._h, hbj._P(ft.data_ptr()), hbj._P(torch.empty_like(ft).data_ptr()), 1,
                              hbj.ctypes.byref(opts), None)
    assert code == hbj.EINVAL
    ctx.close()
