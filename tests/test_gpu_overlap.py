"""The operator applied beside the backward pass (hbj_set_operator_overlap), through the C ABI.

Inside GMRES the operator rows of the subdomains whose data the backward pass has already finalised run
on a second stream while the remaining backward steps run. Every row is computed by the same kernel from
the same data as without the overlap, so the solves must agree bit for bit (iterates, residual history,
field); a missing wait would let a row read data the pass has not written yet and change them. Cases:
block Jacobi and SGS, FP64 and complex64 preconditioner, one and two right-hand sides, aligned, ragged,
rectangular and strip decompositions; two solves in a row reuse the events.
"""
import numpy as np
import pytest

import workload as W
from cases import CASES, gpu_context, oracle_problem, rel, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _sources(wl, n):
    xs = np.linspace(0.3, 0.7, n)
    return np.stack([W.gaussian_source(wl.nx, wl.ny, wl.h, x, 0.4 * (wl.ny + 1) * wl.h) for x in xs])


@pytest.mark.parametrize("name,precision,precond,nrhs", [
    ("grf256", 0, 2, 1), ("grf256", 1, 2, 1), ("grf256", 0, 1, 1), ("grf256", 0, 2, 2),
    ("strip", 0, 2, 1), ("ragged", 0, 2, 1), ("rect", 0, 1, 2), ("small", 0, 2, 1)])
def test_overlap_is_bit_identical(hbj, name, precision, precond, nrhs):
    from oracle import solver

    wl = CASES[name].wl
    m, g, dd = oracle_problem(wl)
    f = _sources(wl, nrhs)
    ft = torch.as_tensor(f if nrhs > 1 else f[0], device="cuda")
    out = {}
    for on in (0, 1):
        ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE, precision=precision, precond=precond)
        ctx.set_operator_overlap(on)
        ctx.factor()
        runs = []
        for rep in range(2):
            say(f"[overlap={on}] case={name} precision={precision} precond={precond} nrhs={nrhs} rep={rep}")
            u, st = ctx.solve(ft, tol=1e-10, maxit=2000, hist_len=512)
            torch.cuda.synchronize()
            runs.append((u.cpu().numpy(), st.iters, list(st.history)))
        ctx.close()
        out[on] = runs
    for rep in range(2):
        u0, it0, h0 = out[0][rep]
        u1, it1, h1 = out[1][rep]
        say(f"  rep {rep}: iterations {it0} / {it1}, max |du| {np.max(np.abs(u0 - u1)):.1e}")
        assert it0 == it1
        assert h0 == h1
        assert np.array_equal(u0, u1)
    # and the field is the solution
    u = out[1][0][0].reshape(nrhs, -1)
    for k in range(nrhs):
        e = rel(u[k], np.asarray(solver.direct(g, f[k])).ravel())
        say(f"  rhs {k}: error vs direct {e:.1e}")
        assert e < 1e-8 if precision == 0 else e < 1e-7


def test_overlap_bad_value(hbj):
    wl = W.SMALL
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=torch.as_tensor(W.slowness2(wl), device="cuda"))
    with pytest.raises(hbj.HbjError) as ei:
        hbj._check(hbj._lib.hbj_set_operator_overlap(ctx._h, 2))
    assert ei.value.code == hbj.EINVAL
    ctx.close()
