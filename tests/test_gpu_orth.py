"""The two Gram-Schmidt variants of the Arnoldi steps, against the direct solution and each other.

Classical Gram-Schmidt applied twice and Gram-Schmidt with delayed reorthogonalisation build the
same Krylov space with a basis that is orthonormal to working precision, so both reach the direct
solution and take the same number of iterations up to rounding (within one). The cases cover
restarts (the delayed form closes every cycle with a coefficient-only step), flexible GMRES (mixed
precision), several right-hand sides in lockstep (few and many: the matrix-product path), banded
operators and the symmetric Gauss-Seidel preconditioner.
"""
import numpy as np
import pytest

import workload as W
from cases import CASES, gpu_context, oracle_problem, rel, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name,kw,restart,nrhs", [
    ("grf256", dict(precond=2), 50, 1),
    ("grf256", dict(precond=2), 7, 1),
    ("grf256", dict(precond=2), 3, 1),
    ("grf256", dict(precond=2, precision=1), 50, 1),  # flexible GMRES
    ("grf256", dict(precond=2), 50, 3),
    ("grf256", dict(precond=2, precision=1), 11, 5),  # matrix-product operators, restarts
    ("strip", dict(precond=1), 50, 1),
    ("ragged", dict(precond=2, operator_form=0), 50, 1),  # banded operators
])
def test_orthogonalizations_agree(hbj, name, kw, restart, nrhs):
    from oracle import solver

    wl = CASES[name].wl
    m, g, dd = oracle_problem(wl)
    kw = dict(kw)
    kw.setdefault("operator_form", hbj.OP_DENSE)
    ctx = gpu_context(hbj, wl, m, **kw)
    ctx.factor()
    srcs = [W.sources(wl)[0]] + [W.gaussian_source(wl.nx, wl.ny, wl.h, x, 0.3)
                                 for x in np.linspace(0.2, 0.8, nrhs - 1)]
    f = np.stack(srcs) if nrhs > 1 else srcs[0]
    ft = torch.as_tensor(f, device="cuda")
    out = {}
    for mode in (hbj.ORTH_CGS2, hbj.ORTH_DCGS2):
        ctx.set_orthogonalization(mode)
        say(f"[orth] case={name} {kw} restart={restart} nrhs={nrhs} mode={mode}")
        u, st = ctx.solve(ft, tol=1e-12, restart=restart, maxit=3000)
        assert st.relres <= 1e-12
        assert st.converged == nrhs
        out[mode] = (_np(u).reshape(nrhs, wl.ny, wl.nx), st)
    (u2, s2), (ud, sd) = out[hbj.ORTH_CGS2], out[hbj.ORTH_DCGS2]
    say(f"  iters CGS2 {s2.iters} DCGS2 {sd.iters}")
    assert abs(s2.iters - sd.iters) <= 1
    for k in range(nrhs):
        ref = solver.direct(g, srcs[k])
        assert rel(ud[k], ref) < 1e-8
        assert rel(u2[k], ref) < 1e-8
    ctx.close()


def test_orthogonalization_iteration_limit_and_bad_mode(hbj):
    """maxit stops the delayed form after exactly that many columns; unknown modes are refused."""
    wl = W.SMALL
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=torch.as_tensor(W.slowness2(wl), device="cuda"))
    ctx.factor()
    f = torch.as_tensor(W.sources(wl)[0], device="cuda")
    for mode in (hbj.ORTH_CGS2, hbj.ORTH_DCGS2):
        ctx.set_orthogonalization(mode)
        for maxit in (1, 2, 3):
            say(f"[orth] mode={mode} maxit={maxit}")
            u, st = ctx.solve(f, tol=1e-14, maxit=maxit, restart=2, check=False)
            assert st.code == hbj.NOT_CONVERGED and st.iters == maxit
            assert torch.isfinite(torch.view_as_real(u)).all()
    with pytest.raises(hbj.HbjError) as ei:
        ctx.set_orthogonalization(7)
    assert ei.value.code == hbj.EINVAL
    ctx.close()
