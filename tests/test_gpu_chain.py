"""Chained sweep steps on the many-right-hand-side path (hbj_set_step_chaining), through the C ABI.

Each sweep step writes its outputs also into the gathered tile of the next step, and the other
positions of every step's tile are gathered at the start of the pass.  Every tile entry is the same
value, rounded the same way, as a gather launch before the step would read, so preconditioner
applications and solves must agree bit for bit with chaining on and off, for FP64 and complex64
preconditioner operators, several right-hand-side counts (one and two 64-column tiles), every
variant of the step kernel that reads gathered tiles (and one that does not: chaining then stays
off), ragged and rectangular decompositions and block-Jacobi widths; and the preconditioner must
match the oracle.
"""
import numpy as np
import pytest

import workload as W
from cases import CASES, gpu_context, oracle_problem, rel, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name,kw,nr", [
    ("grf256", {}, 20), ("grf256", dict(precision=1), 20), ("ragged", {}, 5), ("ragged", dict(precision=1), 70),
    ("rect", {}, 20), ("grf256", dict(bj_width=3), 20), ("strip", {}, 8)])
@pytest.mark.parametrize("variant", [None, 7, 12, 18, 4])
def test_chained_steps_bit_identical(hbj, name, kw, nr, variant):
    from oracle import sweep

    wl = CASES[name].wl
    m, g, dd = oracle_problem(wl)
    ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE, precond=2, **kw)
    ctx.factor()
    if variant is not None:
        ctx.set_tuning([variant] * 4)
    gv = W.random_interface_vector(ctx.nif, seed=17, nrhs=nr)
    gt = torch.as_tensor(gv, device="cuda")
    out = {}
    for on in (1, 0, 1):
        ctx.set_step_chaining(on)
        say(f"[chain={on}] case={name} {kw} nrhs={nr} variant={variant}")
        out.setdefault(on, []).append(_np(ctx.apply_preconditioner(gt)))
    assert np.array_equal(out[1][0], out[0][0])
    assert np.array_equal(out[1][1], out[0][0])
    tol = 1e-11 if not kw.get("precision") else 1e-5
    for k in (0, nr - 1):
        ref = sweep.apply_bj(dd, gv[k], width=kw.get("bj_width"))
        assert rel(out[1][0][k], ref) < tol
    ctx.close()


def test_chained_solves_bit_identical(hbj):
    wl = CASES["grf256"].wl
    m, g, dd = oracle_problem(wl)
    xs = np.linspace(0.2, 0.8, 12)
    f = np.stack([W.gaussian_source(wl.nx, wl.ny, wl.h, x, 0.3) for x in xs])
    ft = torch.as_tensor(f, device="cuda")
    res = {}
    for precision in (0, 1):
        ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE, precond=2, precision=precision)
        ctx.factor()
        for on in (0, 1):
            ctx.set_step_chaining(on)
            say(f"[chain solve] precision={precision} chaining={on}")
            u, st = ctx.solve(ft, tol=1e-10)
            torch.cuda.synchronize()
            res[(precision, on)] = (_np(u), st.iters, list(st.history))
        ctx.close()
        a, b = res[(precision, 0)], res[(precision, 1)]
        assert a[1] == b[1] and a[2] == b[2]
        assert np.array_equal(a[0], b[0])


def test_chaining_bad_value(hbj):
    wl = W.SMALL
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=torch.as_tensor(W.slowness2(wl), device="cuda"))
    with pytest.raises(hbj.HbjError) as ei:
        hbj._check(hbj._lib.hbj_set_step_chaining(ctx._h, 2))
    assert ei.value.code == hbj.EINVAL
    ctx.close()
