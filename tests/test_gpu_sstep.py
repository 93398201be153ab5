"""s-step Arnoldi cycles (hbj_set_orthogonalization(ORTH_SSTEP)), through the C ABI.

A block of s steps builds the Newton basis y_{i+1} = (I - S) P^{-1} y_i - y_i and makes it
orthonormal in one inner-product pass and one update pass; in exact arithmetic the iterates are
those of single Arnoldi steps.  So the s-step solves must reach the direct solution, take the
iterations of the delayed-reorthogonalisation form (within one), and give the same field to the
solve's tolerance, for every block size, with restarts shorter and longer than a block, one and
many right-hand sides in lockstep (the matrix-product path), complex64 preconditioners, banded
operators, a right-hand side that is zero beside others (its basis vectors are zero: the block
factorisation reports it and leaves it out) and an iteration limit inside a block.  Cases outside
the s-step form (non-flexible GMRES, restarts above 63) fall back to the delayed form bit for bit.
"""
import numpy as np
import pytest

import workload as W
from cases import CASES, gpu_context, oracle_problem, rel, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _np(t):
    return t.detach().cpu().numpy()


def _sources(wl, nrhs):
    srcs = [W.sources(wl)[0]] + [W.gaussian_source(wl.nx, wl.ny, wl.h, x, 0.3) for x in np.linspace(0.2, 0.8, nrhs - 1)]
    return np.stack(srcs) if nrhs > 1 else srcs[0]


def _solve_both(hbj, ctx, ft, block, **kw):
    out = {}
    for mode in (hbj.ORTH_DCGS2, hbj.ORTH_SSTEP):
        ctx.set_orthogonalization(mode)
        ctx.set_sstep_block(block)
        u, st = ctx.solve(ft, **kw)
        torch.cuda.synchronize()
        out[mode] = (_np(u), st)
    ctx.set_orthogonalization(hbj.ORTH_DCGS2)
    return out[hbj.ORTH_DCGS2], out[hbj.ORTH_SSTEP]


@pytest.mark.parametrize("name,kw,restart,nrhs,block", [
    ("grf256", dict(precond=2), 50, 1, 8),
    ("grf256", dict(precond=2), 50, 1, 3),
    ("grf256", dict(precond=2), 7, 1, 8),  # restart shorter than a block
    ("grf256", dict(precond=2), 11, 1, 4),  # blocks of 4, 4, 3
    ("grf256", dict(precond=2, precision=1), 50, 1, 8),  # complex64 preconditioner
    ("grf256", dict(precond=2), 50, 3, 8),
    ("grf256", dict(precond=2), 50, 20, 8),  # matrix-product operators
    ("grf256", dict(precond=2, precision=1), 13, 5, 6),
    ("strip", dict(precond=1), 50, 1, 8),
    ("ragged", dict(precond=2, operator_form=0), 50, 1, 5),  # banded operators
    ("rect", dict(precond=2), 63, 2, 1),  # block of one step, the longest restart of the form
])
def test_sstep_matches_direct_and_dcgs(hbj, name, kw, restart, nrhs, block):
    from oracle import solver

    wl = CASES[name].wl
    m, g, dd = oracle_problem(wl)
    kw = dict(kw)
    kw.setdefault("operator_form", hbj.OP_DENSE)
    ctx = gpu_context(hbj, wl, m, **kw)
    ctx.factor()
    f = _sources(wl, nrhs)
    ft = torch.as_tensor(f, device="cuda")
    say(f"[sstep] case={name} {kw} restart={restart} nrhs={nrhs} block={block}")
    (ud, sd), (us, ss) = _solve_both(hbj, ctx, ft, block, tol=1e-12, restart=restart, maxit=4000)
    ctx.close()
    say(f"  iterations DCGS2 {sd.iters} s-step {ss.iters}, relres {sd.relres:.1e} / {ss.relres:.1e}")
    assert ss.converged == nrhs and ss.relres <= 1e-12
    assert abs(ss.iters - sd.iters) <= 1
    ud = ud.reshape(nrhs, wl.ny, wl.nx)
    us = us.reshape(nrhs, wl.ny, wl.nx)
    srcs = f.reshape(nrhs, wl.ny, wl.nx)
    for k in range(nrhs):
        ref = solver.direct(g, srcs[k])
        e = rel(us[k], ref)
        say(f"  rhs {k}: s-step vs direct {e:.1e}, vs DCGS2 {rel(us[k], ud[k]):.1e}")
        assert e < 1e-8
        assert rel(us[k], ud[k]) < 1e-9


def test_sstep_every_block_size_same_iterations(hbj):
    """Block sizes 1..8 at tol 1e-6: the iteration count of GMRES does not depend on s."""
    wl = CASES["grf256"].wl
    m, g, dd = oracle_problem(wl)
    ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE, precond=2)
    ctx.factor()
    ft = torch.as_tensor(_sources(wl, 1), device="cuda")
    ctx.set_orthogonalization(hbj.ORTH_DCGS2)
    u0, s0 = ctx.solve(ft, tol=1e-6)
    u0 = _np(u0)
    ctx.set_orthogonalization(hbj.ORTH_SSTEP)
    for block in range(1, 9):
        ctx.set_sstep_block(block)
        say(f"[sstep block] {block}")
        u, st = ctx.solve(ft, tol=1e-6)
        say(f"  iterations {st.iters} (DCGS2 {s0.iters}), history length {len(st.history)}")
        assert st.iters == s0.iters
        assert rel(_np(u), u0) < 1e-7
        assert np.allclose(st.history, s0.history, rtol=1e-5, atol=1e-12)
    ctx.close()


def test_sstep_zero_column_and_iteration_limit(hbj):
    """A zero right-hand side beside nonzero ones stays zero; maxit stops inside a block."""
    wl = CASES["grf256"].wl
    m, g, dd = oracle_problem(wl)
    ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE, precond=2)
    ctx.factor()
    f = _sources(wl, 5)
    f[2] = 0.0
    ft = torch.as_tensor(f, device="cuda")
    ctx.set_orthogonalization(hbj.ORTH_SSTEP)
    say("[sstep] zero column among 5")
    u, st = ctx.solve(ft, tol=1e-10)
    u = _np(u)
    assert st.converged == 5
    assert np.all(u[2] == 0)
    from oracle import solver
    for k in (0, 1, 3, 4):
        assert rel(u[k].reshape(wl.ny, wl.nx), solver.direct(g, f[k])) < 1e-7
    for maxit in (1, 3, 10):
        say(f"[sstep] maxit={maxit}")
        u, st = ctx.solve(ft[0], tol=1e-14, maxit=maxit, restart=50, check=False)
        assert st.code == hbj.NOT_CONVERGED and st.iters == maxit
        assert torch.isfinite(torch.view_as_real(u)).all()
    ctx.close()


@pytest.mark.parametrize("flexible,restart", [(False, 50), (True, 80)])
def test_sstep_falls_back_to_dcgs(hbj, flexible, restart):
    """Non-flexible GMRES and restarts above 63 run the delayed-reorthogonalisation form."""
    wl = CASES["ragged"].wl
    m, g, dd = oracle_problem(wl)
    ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE, precond=2)
    ctx.factor()
    ft = torch.as_tensor(_sources(wl, 1), device="cuda")
    say(f"[sstep fallback] flexible={flexible} restart={restart}")
    (ud, sd), (us, ss) = _solve_both(hbj, ctx, ft, 8, tol=1e-10, restart=restart, maxit=4000, flexible=flexible)
    ctx.close()
    assert ss.iters == sd.iters
    assert list(ss.history) == list(sd.history)
    assert np.array_equal(us, ud)


def test_sstep_bad_values(hbj):
    wl = W.SMALL
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=torch.as_tensor(W.slowness2(wl), device="cuda"))
    for bad in (0, 9, -1):
        with pytest.raises(hbj.HbjError) as ei:
            ctx.set_sstep_block(bad)
        assert ei.value.code == hbj.EINVAL
    with pytest.raises(hbj.HbjError) as ei:
        ctx.set_orthogonalization(4)
    assert ei.value.code == hbj.EINVAL
    ctx.close()


def test_auto_picks_sstep_for_large_blocks(hbj):
    """The default (ORTH_AUTO) runs s-step cycles once the Krylov vectors of all right-hand sides
    hold 2^20 entries (80 sources on the 512^2 grid of 8 x 8 subdomains: 80 x 14336), bit for bit
    as ORTH_SSTEP, and the delayed form below that (8 sources), bit for bit as ORTH_DCGS2."""
    wl = W.scaled(W.FP64_1024, 512)
    m = W.slowness2(wl)
    ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE, precond=2)
    ctx.factor()
    xs = np.linspace(0.1, 0.9, 80)
    f = np.stack([W.gaussian_source(wl.nx, wl.ny, wl.h, x, 0.1) for x in xs])
    assert ctx.nif * 80 >= 1 << 20 and ctx.nif * 8 < 1 << 20
    for nrhs, explicit in ((80, hbj.ORTH_SSTEP), (8, hbj.ORTH_DCGS2)):
        ft = torch.as_tensor(f[:nrhs], device="cuda")
        runs = []
        for mode in (hbj.ORTH_AUTO, explicit):
            ctx.set_orthogonalization(mode)
            say(f"[auto] nrhs={nrhs} mode={mode}")
            u, st = ctx.solve(ft, tol=1e-8)
            torch.cuda.synchronize()
            runs.append((_np(u), st.iters, list(st.history)))
        assert runs[0][1] == runs[1][1] and runs[0][2] == runs[1][2]
        assert np.array_equal(runs[0][0], runs[1][0])
    ctx.close()
