"""GMRES iterations replayed as HIP graphs against the same iterations launched one by one.

The graph of Arnoldi step j holds the very launches of the eager path (same kernels, same
arguments), so every replay must reproduce the eager solution bit for bit. Each test replays the
graphs several times, with eager work of the program and synchronisations between the replays, and
checks every replay against the eager result.
"""
import numpy as np
import pytest

import workload as W
from cases import CASES, gpu_context, oracle_problem, rel, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name,kw,restart,orth", [
    ("grf256", dict(precond=2), 50, 1),
    ("grf256", dict(precond=2), 7, 1),            # several restart cycles reuse the captured steps
    ("grf256", dict(precond=2), 7, 0),            # classical Gram-Schmidt twice
    ("grf256", dict(precond=2, precision=1), 50, 1),  # mixed: complex64 preconditioner, FGMRES
    ("grf256", dict(precond=2, bj_combine=1, bj_compose=1), 50, 1),
    ("strip", dict(precond=1), 50, 1),
])
def test_graph_replays_match_eager(hbj, name, kw, restart, orth):
    from oracle import solver

    wl = CASES[name].wl
    m, g, dd = oracle_problem(wl)
    ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE, **kw)
    ctx.factor()
    ctx.set_orthogonalization(orth)
    f = torch.as_tensor(W.sources(wl)[0], device="cuda")
    say(f"[graphs] case={name} {kw} restart={restart}: eager")
    ctx.set_graphs(False)
    u0, s0 = ctx.solve(f, tol=1e-12, restart=restart, maxit=3000)
    u0 = _np(u0)
    assert rel(u0, solver.direct(g, _np(f))) < 1e-8
    ctx.set_graphs(True)
    r = torch.as_tensor(W.random_interface_vector(ctx.nif, seed=31), device="cuda")
    for rep in range(3):
        say(f"  replay {rep}")
        u, st = ctx.solve(f, tol=1e-12, restart=restart, maxit=3000)
        torch.cuda.synchronize()
        assert st.iters == s0.iters
        assert np.array_equal(_np(u), u0)
        # eager work of the program between replays
        z = ctx.apply_preconditioner(r)
        _ = (z * 2).sum().item()
    ctx.close()


def test_graphs_with_two_rhs_and_refactor(hbj):
    """Two right-hand sides in lockstep; a new medium and factorisation drop the captured graphs."""
    wl = CASES["grf256"].wl
    m, g, dd = oracle_problem(wl)
    ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE, precond=2)
    ctx.factor()
    f = torch.as_tensor(np.stack([W.sources(wl)[0], W.gaussian_source(wl.nx, wl.ny, wl.h, 0.3, 0.7)]), device="cuda")
    say("[graphs] nrhs=2 eager / replay")
    ctx.set_graphs(False)
    u0, _ = ctx.solve(f, tol=1e-10)
    u0 = _np(u0)
    ctx.set_graphs(True)
    for _ in range(2):
        u, _ = ctx.solve(f, tol=1e-10)
        assert np.array_equal(_np(u), u0)
    say("[graphs] new medium")
    m2 = np.asarray(m) * 1.05
    ctx.set_slowness2(torch.as_tensor(m2, device="cuda"))
    ctx.factor()
    u1, _ = ctx.solve(f, tol=1e-10)
    ctx.set_graphs(False)
    u1e, _ = ctx.solve(f, tol=1e-10)
    assert np.array_equal(_np(u1), _np(u1e))
    assert rel(_np(u1), u0) > 1e-3  # the new medium really changed the solution
    ctx.close()
