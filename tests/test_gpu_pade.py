"""The Pade transmission condition (the paper's condition, Sec. 7: N_pade = 8, phi = pi/3) in the
dense operator form, through the C ABI, against the oracle's transmission=3 decomposition
(oracle.habc; pinned in tests/test_oracle_habc.py).

The library factors the Robin-closed local matrices and corrects the dense operators by a
Woodbury identity on the edge nodes; the operator, lifting, reconstruction and preconditioner are
compared vector for vector with the oracle, which builds the dense face blocks into its local
matrices directly, and the solution with the global direct solve.
"""
import numpy as np
import pytest

import workload as W
from cases import CASES, gpu_context, rel, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _np(t):
    return t.detach().cpu().numpy()


def _pade_problem(wl):
    from oracle.dd import Decomposition
    from oracle.fd import Grid

    m = W.slowness2(wl)
    g = Grid(wl.nx, wl.ny, wl.h, wl.k, m)
    return m, g, Decomposition(g, wl.n1, wl.n2, transmission=3)


@pytest.mark.parametrize("name", ["small", "rect", "ragged", "grf256", "strip"])
def test_pade_operators_match_oracle(hbj, name):
    from oracle import sweep

    wl = CASES[name].wl
    m, g, dd = _pade_problem(wl)
    say(f"[pade] case={name}")
    ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE, transmission=3)
    ctx.factor()
    gv = W.random_interface_vector(ctx.nif, seed=61)
    f = W.sources(wl)[0]
    e_op = rel(_np(ctx.apply_operator(torch.as_tensor(gv, device="cuda"))), dd.apply_operator(gv))
    e_lift = rel(_np(ctx.lifting(torch.as_tensor(f, device="cuda"))), dd.lifting(f))
    u = _np(ctx.reconstruct(torch.as_tensor(f[None], device="cuda"), torch.as_tensor(gv[None], device="cuda")))[0]
    e_rec = rel(u, dd.reconstruct(f, gv))
    e_pc = rel(_np(ctx.apply_preconditioner(torch.as_tensor(gv, device="cuda"))), sweep.apply_bj(dd, gv))
    say(f"  operator {e_op:.1e} lifting {e_lift:.1e} reconstruction {e_rec:.1e} preconditioner {e_pc:.1e}")
    assert e_op < 1e-12
    assert e_lift < 1e-12
    assert e_rec < 1e-12
    assert e_pc < 1e-11
    ctx.close()


@pytest.mark.parametrize("name", ["small", "grf256", "strip"])
def test_pade_solve_matches_direct_solution(hbj, name):
    from oracle import solver

    wl = CASES[name].wl
    m, g, dd = _pade_problem(wl)
    f = W.sources(wl)[0]
    ft = torch.as_tensor(f, device="cuda")
    ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE, transmission=3)
    ctx.factor()
    u, st = ctx.solve(ft, tol=1e-12, maxit=3000)
    ud = solver.direct(g, f)
    e = rel(_np(u), ud)
    _, st6 = ctx.solve(ft, tol=1e-6)
    ref = solver.dd_solve(dd, f, precond="bj", tol=1e-6)
    say(f"[pade solve] case={name}: tol 1e-12 iters {st.iters} error {e:.1e}; tol 1e-6 iters GPU {st6.iters} "
        f"oracle {ref.iters}")
    assert st.relres <= 1e-12
    assert e < 1e-8
    assert abs(st6.iters - ref.iters) <= 1
    ctx.close()


def test_pade_many_right_hand_sides_and_mixed(hbj):
    """5 right-hand sides (matrix-product operators and reconstruction), and complex64 operators in
    the preconditioner (mixed form)."""
    from oracle import solver

    wl = CASES["grf256"].wl
    m, g, dd = _pade_problem(wl)
    ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE, transmission=3)
    ctx.factor()
    G = W.random_interface_vector(ctx.nif, seed=62, nrhs=5)
    w = _np(ctx.apply_operator(torch.as_tensor(G, device="cuda")))
    for k in range(5):
        assert rel(w[k], dd.apply_operator(G[k])) < 1e-12
    rng = np.random.default_rng(63)
    F = rng.standard_normal((5, wl.ny, wl.nx)) + 1j * rng.standard_normal((5, wl.ny, wl.nx))
    F[3] = 0.0
    b = _np(ctx.lifting(torch.as_tensor(F, device="cuda")))
    u = _np(ctx.reconstruct(torch.as_tensor(F, device="cuda"), torch.as_tensor(G, device="cuda")))
    for k in range(5):
        assert rel(b[k], dd.lifting(F[k])) < 1e-12 or (k == 3 and np.abs(b[k]).max() == 0.0)
        assert rel(u[k], dd.reconstruct(F[k], G[k])) < 1e-12
    ctx.close()
    f = W.sources(wl)[0]
    ft = torch.as_tensor(f, device="cuda")
    mctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE, transmission=3, precision=hbj.MIXED)
    mctx.factor()
    um, sm = mctx.solve(ft, tol=1e-10)
    e = rel(_np(um), solver.direct(g, f))
    say(f"[pade mixed] iters {sm.iters} relres {sm.relres:.1e} error vs direct {e:.1e}")
    assert sm.relres <= 1e-10 and e < 1e-7
    mctx.close()


def test_pade_needs_the_dense_form(hbj):
    wl = CASES["small"].wl
    m = W.slowness2(wl)
    with pytest.raises(RuntimeError):
        gpu_context(hbj, wl, m, operator_form=hbj.OP_BANDED, transmission=3)
    ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE, transmission=3)
    ctx.factor()
    with pytest.raises(RuntimeError):
        ctx.local_solve([0], torch.zeros((1, ctx.n_loc), dtype=torch.complex128, device="cuda"))
    ctx.close()
