"""Parity at the benchmark's full sizes, in the launch configuration bench.py times.

The oracle's domain decomposition runs at full size on the CPU (64 local SuperLU factorisations
of 128^2 subdomains), so the operator, the lifting, the reconstruction and the preconditioner of
the 1024^2 workload are compared vector for vector. The solutions are checked through properties
that hold at any size: the Robin traces g* of the GPU field must satisfy the oracle's interface
system (I - S) g* = b, and the mixed-precision field must agree with the FP64 one. The 2048^2
multi-source workload is checked on sampled subdomains of the operator and through its
residuals.
"""
import numpy as np
import pytest

import workload as W
from cases import rel, say

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
    assert res < 1e-6
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


def test_fullsize_multi_source_sampled(hbj):
    """2048^2, 16 x 16, 64 sources (complex64 factors, MFMA operators, lockstep FGMRES): the
    operator on sampled subdomains against the oracle, and every column's residual."""
    from oracle.dd import Decomposition
    from oracle.fd import Grid

    wl = W.MULTI_2048
    say(f"[fullsize] {wl.name}")
    m = W.slowness2(wl)
    dd = Decomposition(Grid(wl.nx, wl.ny, wl.h, wl.k, m), wl.n1, wl.n2)
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=torch.as_tensor(m, device="cuda"), precision=hbj.MIXED,
                    precond=hbj.PC_BJ, operator_form=hbj.OP_DENSE)
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
    f = torch.as_tensor(W.sources(wl), device="cuda")
    u, st = ctx.solve(f, tol=1e-6)
    say(f"  iters {st.iters}, relres {st.relres:.2e}, converged {st.converged}/64")
    assert st.converged == 64 and st.relres <= 1e-6
    ctx.close()


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
    assert res < 1e-6
