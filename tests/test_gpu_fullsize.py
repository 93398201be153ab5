"""Parity at the benchmark's full sizes, in the launch configuration bench.py times.

1024^2, 8 x 8 (FP64 and mixed):
* the oracle's domain decomposition runs at full size on the CPU (64 local SuperLU
  factorisations of 128^2 subdomains), so the operator, the lifting, the reconstruction, the
  block-Jacobi preconditioner and the refined complex64 banded operator are compared vector for
  vector;
* the FP64 solve at tol 1e-12 is compared element by element with the oracle's global direct
  solution u = A^{-1} f (SuperLU on the 1024^2 grid), the plain definition of the result, and its
  iteration count at the benchmark's tol 1e-6 with the oracle's own DD-GMRES;
* the solves to tol 1e-8 are checked through a property that holds at any size: the Robin traces
  g* of the GPU field satisfy the oracle's interface system (I - S) g* = b;
* the mixed-precision fields agree with the FP64 one.

2048^2, 16 x 16, 64 sources: the operator on sampled subdomains; sampled columns against
single-right-hand-side solves of the same precision and against tight FP64 solves; the oracle's
interface residual of the sampled columns' traces; every column's volume residual from the oracle.
"""
import numpy as np
import pytest

import workload as W
from cases import rel, residual_rounding_bound, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def full(hbj):
    from oracle.dd import Decomposition
    from oracle.fd import Grid

    wl = W.FP64_1024
    say(f"[fullsize] {wl.name}: oracle decomposition {wl.nx}^2, {wl.n1}x{wl.n2}")
    m = W.slowness2(wl)
    dd = Decomposition(Grid(wl.nx, wl.ny, wl.h, wl.k, m), wl.n1, wl.n2)
    mt = torch.as_tensor(m, device="cuda")
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=mt, precond=hbj.PC_BJ, operator_form=hbj.OP_DENSE)
    ctx.factor()
    torch.cuda.synchronize()
    yield wl, m, dd, ctx
    ctx.close()


def test_fullsize_operator_lifting_reconstruction(full):
    wl, m, dd, ctx = full
    gv = W.random_interface_vector(ctx.nif, seed=41)
    f = W.sources(wl)[0]
    say("[fullsize] operator")
    w = _np(ctx.apply_operator(torch.as_tensor(gv, device="cuda")))
    assert rel(w, dd.apply_operator(gv)) < 1e-12
    say("[fullsize] lifting")
    b = _np(ctx.lifting(torch.as_tensor(f, device="cuda")))
    assert rel(b, dd.lifting(f)) < 1e-12
    say("[fullsize] reconstruction")
    u = _np(ctx.reconstruct(torch.as_tensor(f[None], device="cuda"), torch.as_tensor(gv[None], device="cuda")))[0]
    assert rel(u, dd.reconstruct(f, gv)) < 1e-12


def test_fullsize_preconditioner(full):
    from oracle import sweep

    wl, m, dd, ctx = full
    r = W.random_interface_vector(ctx.nif, seed=42)
    say("[fullsize] block-Jacobi preconditioner (16 sweep steps)")
    z = _np(ctx.apply_preconditioner(torch.as_tensor(r, device="cuda")))
    assert rel(z, sweep.apply_bj(dd, r)) < 1e-11


def test_fullsize_split_banded_solves(full, hbj):
    """The banded form with every local solve split over 16 runs of column blocks (the launch shape
    for the sweep steps' batches of a few solves): operator and block-Jacobi preconditioner at
    1024^2 against the oracle."""
    from oracle import sweep

    wl, m, dd, _ = full
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=torch.as_tensor(m, device="cuda"), precond=hbj.PC_BJ,
                    operator_form=hbj.OP_BANDED)
    ctx.factor()
    ctx.set_solve_tuning(hbj.SOLVE_SHAPE_SPLIT)
    ctx.set_solve_partitions(16)
    gv = W.random_interface_vector(ctx.nif, seed=41)
    say("[fullsize] split banded solves: operator")
    w = _np(ctx.apply_operator(torch.as_tensor(gv, device="cuda")))
    assert rel(w, dd.apply_operator(gv)) < 1e-12
    r = W.random_interface_vector(ctx.nif, seed=42)
    say("[fullsize] split banded solves: block-Jacobi preconditioner")
    z = _np(ctx.apply_preconditioner(torch.as_tensor(r, device="cuda")))
    ctx.close()
    assert rel(z, sweep.apply_bj(dd, r)) < 1e-11


@pytest.fixture(scope="module")
def direct_full(full):
    """The oracle's global direct solution u = A^{-1} f of the 1024^2 workload (SuperLU)."""
    from oracle import solver

    wl, m, dd, ctx = full
    say(f"[fullsize] oracle global direct solve (SuperLU, {wl.nx}^2)")
    return solver.direct(dd.grid, W.sources(wl)[0])


@pytest.mark.timeout(900)
def test_fullsize_solve_matches_direct_solution(full, direct_full, hbj):
    """FP64 solve at tol 1e-12 against the oracle's global direct solution (relative error 1e-8);
    the iteration count at tol 1e-6 against the oracle's DD-GMRES (within one); the volume
    residual of the GPU field from the oracle and from the library."""
    from oracle import solver

    wl, m, dd, ctx = full
    f = W.sources(wl)[0]
    ft = torch.as_tensor(f, device="cuda")
    say("[fullsize] FP64 solve, tol 1e-12")
    u, st = ctx.solve(ft, tol=1e-12, maxit=2000)
    assert st.relres <= 1e-12
    say(f"  iters {st.iters}, relres {st.relres:.2e}")
    ud = direct_full
    e = rel(_np(u), ud)
    vr_o = solver.volume_residual(dd.grid, _np(u), f)
    vr_g = ctx.volume_residual(ft, u)[0]
    bound = residual_rounding_bound(dd.grid, _np(u), f)
    say(f"  error vs direct solution {e:.2e}; volume residual oracle {vr_o:.2e} library {vr_g:.2e} "
        f"(rounding bound of their difference {bound:.1e})")
    assert e < 1e-8
    # both sum f - A u in their own order; at a converged field the residual is near round-off
    assert abs(vr_g - vr_o) <= bound
    say("[fullsize] FP64 solve, tol 1e-6, against the oracle's DD-GMRES")
    _, st6 = ctx.solve(ft, tol=1e-6)
    ref = solver.dd_solve(dd, f, precond="bj", tol=1e-6)
    say(f"  iters GPU {st6.iters} oracle {ref.iters}; oracle relres {ref.relres:.2e}")
    assert abs(st6.iters - ref.iters) <= 1


def test_fullsize_solve_fp64_and_mixed(full, hbj):
    """FP64 GMRES to 1e-8; the traces of the GPU field solve the oracle's interface system.
    Mixed precision (complex64 factors and preconditioner) to 1e-6 and 1e-8: error against the
    FP64 field."""
    wl, m, dd, ctx = full
    f = W.sources(wl)[0]
    ft = torch.as_tensor(f, device="cuda")
    say("[fullsize] FP64 solve, tol 1e-8")
    u, st = ctx.solve(ft, tol=1e-8)
    assert st.relres <= 1e-8
    u = _np(u)
    gs = dd.traces_of(u)
    b = dd.lifting(f)
    res = np.linalg.norm(dd.apply_operator(gs) - b) / np.linalg.norm(b)
    say(f"  iters {st.iters}, relres {st.relres:.2e}, oracle interface residual of the traces {res:.2e}")
    # GMRES stops at a true interface residual <= 1e-8; the oracle's recomputation agrees to rounding
    assert res < 5e-8
    mctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=torch.as_tensor(m, device="cuda"), precision=hbj.MIXED,
                     precond=hbj.PC_BJ, operator_form=hbj.OP_DENSE)
    mctx.factor()
    for tol, bound in ((1e-6, 1e-5), (1e-8, 1e-7)):
        um, sm = mctx.solve(ft, tol=tol)
        e = rel(_np(um), u)
        say(f"  mixed tol {tol:g}: iters {sm.iters} (FP64 {st.iters}), relres {sm.relres:.2e}, error vs FP64 {e:.2e}")
        assert sm.relres <= tol
        assert e < bound
    mctx.close()


def test_fullsize_mixed_banded_operator(full, hbj):
    """The banded operator with complex64 factors and FP64 refinement of every local solve, at
    full size, against the oracle's FP64 operator."""
    wl, m, dd, _ = full
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=torch.as_tensor(m, device="cuda"), precision=hbj.MIXED,
                    precond=hbj.PC_BJ, operator_form=hbj.OP_BANDED)
    ctx.factor()
    gv = W.random_interface_vector(ctx.nif, seed=45)
    say("[fullsize] mixed banded operator (refined local solves)")
    w = _np(ctx.apply_operator(torch.as_tensor(gv, device="cuda")))
    e = rel(w, dd.apply_operator(gv))
    say(f"  error vs oracle {e:.2e}")
    assert e < 1e-11
    ctx.close()


@pytest.mark.timeout(900)
def test_fullsize_multi_source_sampled(hbj):
    """2048^2, 16 x 16, 64 sources (complex64 factors, MFMA operators, lockstep FGMRES): the
    operator on sampled subdomains against the oracle; every column's convergence and volume
    residual (oracle); sampled columns against single-right-hand-side solves (same precision, and
    FP64 to tol 1e-10) and through the oracle's interface residual of their traces."""
    from oracle import solver
    from oracle.dd import Decomposition
    from oracle.fd import Grid

    wl = W.MULTI_2048
    say(f"[fullsize] {wl.name}")
    m = W.slowness2(wl)
    dd = Decomposition(Grid(wl.nx, wl.ny, wl.h, wl.k, m), wl.n1, wl.n2)
    mt = torch.as_tensor(m, device="cuda")
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=mt, precision=hbj.MIXED, precond=hbj.PC_BJ,
                    operator_form=hbj.OP_DENSE)
    ctx.factor()
    nr = 4  # the matrix-product path
    gv = W.random_interface_vector(ctx.nif, seed=43, nrhs=nr)
    w = _np(ctx.apply_operator(torch.as_tensor(gv, device="cuda")))
    for s in (0, 17, 255):  # a corner, an interior and the opposite corner subdomain
        key = list(dd.sub)[s]
        for k in range(nr):
            out = dd.scatter_subdomain(key, gv[k])
            for j, v in out.items():
                blk = dd.layout.block(j, key)
                assert rel(w[k][blk], gv[k][blk] - v) < 1e-12
    say("[fullsize] 64-source solve")
    fs = W.sources(wl)
    f = torch.as_tensor(fs, device="cuda")
    u, st = ctx.solve(f, tol=1e-6)
    say(f"  iters {st.iters}, relres {st.relres:.2e}, converged {st.converged}/64")
    assert st.converged == 64 and st.relres <= 1e-6
    # every column's volume residual, by the oracle (8 columns at a time) and by the library
    vr_g = ctx.volume_residual(f, u)
    vr_o = []
    for k0 in range(0, 64, 8):
        vr_o += list(solver.volume_residual(dd.grid, _np(u[k0:k0 + 8]), fs[k0:k0 + 8]))
    say(f"  volume residual: max {max(vr_o):.2e} (oracle), library agrees to "
        f"{max(abs(a - b) / b for a, b in zip(vr_g, vr_o)):.1e}")
    assert max(abs(a - b) / b for a, b in zip(vr_g, vr_o)) < 1e-6
    assert max(vr_o) < 1e-3
    cols = (0, 21, 42, 63)
    worst_same, worst_fp64 = 0.0, 0.0
    ctx64 = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=mt, precision=hbj.FP64, precond=hbj.PC_BJ,
                      operator_form=hbj.OP_DENSE)
    ctx64.factor()
    for k in cols:
        say(f"  column {k}: single-right-hand-side solves")
        u1, s1 = ctx.solve(f[k], tol=1e-6)
        u2, s2 = ctx64.solve(f[k], tol=1e-10)
        e1 = float(torch.linalg.vector_norm(u[k] - u1) / torch.linalg.vector_norm(u1))
        e2 = float(torch.linalg.vector_norm(u[k] - u2) / torch.linalg.vector_norm(u2))
        gs = dd.traces_of(_np(u[k]))
        b = dd.lifting(fs[k])
        res = np.linalg.norm(dd.apply_operator(gs) - b) / np.linalg.norm(b)
        say(f"    vs mixed single solve {e1:.2e} (iters {s1.iters}); vs FP64 tol 1e-10 {e2:.2e}; "
            f"oracle interface residual of its traces {res:.2e}")
        worst_same, worst_fp64 = max(worst_same, e1), max(worst_fp64, e2)
        assert res < 5e-6
    ctx64.close()
    ctx.close()
    assert worst_same < 1e-6
    assert worst_fp64 < 1e-4


@pytest.fixture(scope="module")
def full2(hbj):
    from oracle.dd import Decomposition
    from oracle.fd import Grid

    wl = W.FP64_1024
    say(f"[fullsize order 2] {wl.name}: oracle decomposition with the second-order transmission")
    m = W.slowness2(wl)
    dd = Decomposition(Grid(wl.nx, wl.ny, wl.h, wl.k, m), wl.n1, wl.n2, transmission=2)
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=torch.as_tensor(m, device="cuda"), precond=hbj.PC_BJ,
                    operator_form=hbj.OP_DENSE, transmission=2)
    ctx.factor()
    torch.cuda.synchronize()
    yield wl, m, dd, ctx
    ctx.close()


def test_fullsize_second_order(full2):
    """Second-order transmission at 1024^2, 8 x 8: operator, lifting and reconstruction against the
    oracle vector for vector; the FP64 solve to 1e-8 through the traces-residual property."""
    wl, m, dd, ctx = full2
    gv = W.random_interface_vector(ctx.nif, seed=44)
    f = W.sources(wl)[0]
    say("[fullsize order 2] operator, lifting, reconstruction")
    assert rel(_np(ctx.apply_operator(torch.as_tensor(gv, device="cuda"))), dd.apply_operator(gv)) < 1e-12
    assert rel(_np(ctx.lifting(torch.as_tensor(f, device="cuda"))), dd.lifting(f)) < 1e-12
    u = _np(ctx.reconstruct(torch.as_tensor(f[None], device="cuda"), torch.as_tensor(gv[None], device="cuda")))[0]
    assert rel(u, dd.reconstruct(f, gv)) < 1e-12
    say("[fullsize order 2] FP64 solve, tol 1e-8")
    u, st = ctx.solve(torch.as_tensor(f, device="cuda"), tol=1e-8)
    assert st.relres <= 1e-8
    gs = dd.traces_of(_np(u))
    b = dd.lifting(f)
    res = np.linalg.norm(dd.apply_operator(gs) - b) / np.linalg.norm(b)
    say(f"  iters {st.iters}, relres {st.relres:.2e}, oracle interface residual of the traces {res:.2e}")
    assert res < 5e-8


@pytest.mark.timeout(900)
def test_fullsize_pade(full, direct_full, hbj):
    """The Pade transmission at 1024^2, 8 x 8 in the bench's configuration: the operator on sampled
    subdomains against the oracle's transmission=3 decomposition, and the solve at tol 1e-12
    against the global direct solution; iterations at tol 1e-6 beside the Robin condition's."""
    from oracle.dd import Decomposition

    wl, m, dd, _ = full
    say("[fullsize pade] oracle decomposition with the Pade transmission")
    ddp = Decomposition(dd.grid, wl.n1, wl.n2, transmission=3)
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=torch.as_tensor(m, device="cuda"), precond=hbj.PC_BJ,
                    operator_form=hbj.OP_DENSE, transmission=3)
    ctx.factor()
    gv = W.random_interface_vector(ctx.nif, seed=46)
    w = _np(ctx.apply_operator(torch.as_tensor(gv, device="cuda")))
    for s in (0, 27, 63):  # a corner, an interior and the opposite corner subdomain
        key = list(ddp.sub)[s]
        for j, v in ddp.scatter_subdomain(key, gv).items():
            blk = ddp.layout.block(j, key)
            assert rel(w[blk], gv[blk] - v) < 1e-12
    ft = torch.as_tensor(W.sources(wl)[0], device="cuda")
    u, st = ctx.solve(ft, tol=1e-12, maxit=3000)
    e = rel(_np(u), direct_full)
    _, st6 = ctx.solve(ft, tol=1e-6)
    say(f"  tol 1e-12: iters {st.iters}, error vs direct {e:.1e}; tol 1e-6: iters {st6.iters}")
    assert st.relres <= 1e-12 and e < 1e-8
    ctx.close()
