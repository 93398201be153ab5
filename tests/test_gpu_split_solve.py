"""Local solves split over runs of column blocks (launch shape 4), through the C ABI.

Each banded local solve of a batch can run on np workgroups: every run of column blocks but the
last is solved from a zero incoming window state, a chain over the runs' transfer matrices (formed
once per factorisation) recovers the true incoming states, and every run but the first is solved
again from its true state.  The substitution is linear in its incoming state, so the split solves
must give the sequential solves' results up to rounding, for every run count (two runs, runs of
one block, counts above the number of blocks, ragged last runs), with and without row
interchanges, for complex128 and complex64 factors, for the operator, the lifting, the
reconstruction and the block-Jacobi preconditioner, after a change of the medium (new transfer
matrices), and inside GMRES to the direct solution.  Every result is also compared with the oracle.
"""
import numpy as np
import pytest

import workload as W
from cases import CASES, gpu_context, oracle_problem, rel, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NRHS = 3


def _np(t):
    return t.detach().cpu().numpy()


def _sources(wl, n):
    xs = np.linspace(0.2, 0.8, n)
    return np.stack([W.gaussian_source(wl.nx, wl.ny, wl.h, x, 0.5 * (wl.ny + 1) * wl.h) for x in xs])


def _run(ctx, gt, ft):
    return (_np(ctx.apply_operator(gt)), _np(ctx.lifting(ft)), _np(ctx.reconstruct(ft, gt)),
            _np(ctx.apply_preconditioner(gt)))


def _nblk(wl):
    return -(-(wl.nx // wl.n1) * (wl.ny // wl.n2) // 16)


@pytest.mark.parametrize("name,precision", [("ragged", 0), ("pivot", 0), ("grf256", 0), ("rect", 0), ("strip", 0),
                                            ("grf256", 1), ("pivot", 1)])
def test_split_matches_sequential_and_oracle(hbj, name, precision):
    from oracle import sweep

    wl = CASES[name].wl
    m, g, dd = oracle_problem(wl)
    ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_BANDED, precision=precision, precond=hbj.PC_BJ)
    ctx.factor()
    gv = W.random_interface_vector(ctx.nif, seed=51, nrhs=NRHS)
    f = _sources(wl, NRHS)
    gt, ft = torch.as_tensor(gv, device="cuda"), torch.as_tensor(f, device="cuda")
    ctx.set_solve_tuning(0)
    say(f"[split] case={name} precision={precision}: sequential solves")
    ref = _run(ctx, gt, ft)
    ctx.set_solve_tuning(hbj.SOLVE_SHAPE_SPLIT)
    nblk = _nblk(wl)
    # complex64 factors: the split solves round differently at complex64 precision (the operator is
    # refined to FP64 in both shapes)
    tol = 1e-11 if precision == 0 else (1e-11, 1e-5, 1e-5, 1e-5)
    for npr in sorted({2, 3, 5, 16, nblk, nblk + 7}):
        ctx.set_solve_partitions(npr)
        say(f"[split] case={name} precision={precision} runs={npr} (blocks {nblk})")
        out = _run(ctx, gt, ft)
        for i, what in enumerate(("operator", "lifting", "reconstruction", "preconditioner")):
            e = rel(out[i], ref[i])
            say(f"  {what}: split vs sequential {e:.1e}")
            assert e < (tol if np.isscalar(tol) else tol[i])
    ctx.set_solve_partitions(0)
    out = _run(ctx, gt, ft)
    ctx.close()
    oref = ([dd.apply_operator(gv[k]) for k in range(NRHS)], [dd.lifting(f[k]) for k in range(NRHS)],
            [dd.reconstruct(f[k], gv[k]) for k in range(NRHS)])
    otol = (1e-10 if name == "pivot" else 1e-12) if precision == 0 else (1e-10, 1e-4, 1e-4)
    for i, what in enumerate(("operator", "lifting", "reconstruction")):
        t = otol if np.isscalar(otol) else otol[i]
        e = max(rel(out[i][k], oref[i][k]) for k in range(NRHS))
        say(f"  {what}: split (default runs) vs oracle {e:.1e}")
        assert e < t
    if precision == 0:
        e = max(rel(out[3][k], sweep.apply_bj(dd, gv[k])) for k in range(NRHS))
        say(f"  preconditioner: split vs oracle {e:.1e}")
        assert e < (1e-9 if name == "pivot" else 1e-11)


def test_split_zero_sources_and_medium_change(hbj):
    """Entries with no source and no incoming data (a point source) and a new medium: the transfer
    matrices follow the new factorisation."""
    wl = CASES["grf256"].wl
    m, g, dd = oracle_problem(wl)
    ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_BANDED)
    ctx.factor()
    f = np.zeros((2, wl.ny, wl.nx), complex)
    f[0, 40, 50] = 1.0
    f[1, 200, 17] = 1.0 - 0.5j
    ft = torch.as_tensor(f, device="cuda")
    for shape in (0, hbj.SOLVE_SHAPE_SPLIT):
        ctx.set_solve_tuning(shape)
        say(f"[split] point sources, shape {shape}")
        b = _np(ctx.lifting(ft))
        for k in range(2):
            assert rel(b[k], dd.lifting(f[k])) < 1e-12
    from oracle.dd import Decomposition
    from oracle.fd import Grid

    m2 = m * (1.0 + 0.05 * np.sin(np.arange(m.size).reshape(m.shape) * 0.01))
    dd2 = Decomposition(Grid(wl.nx, wl.ny, wl.h, wl.k, m2), wl.n1, wl.n2)
    ctx.set_slowness2(torch.as_tensor(m2, device="cuda"))
    ctx.factor()
    gv = W.random_interface_vector(ctx.nif, seed=52)
    say("[split] new medium, split solves")
    w = _np(ctx.apply_operator(torch.as_tensor(gv, device="cuda")))
    ctx.close()
    assert rel(w, dd2.apply_operator(gv)) < 1e-12


@pytest.mark.parametrize("name,runs", [("grf256", 5), ("pivot", 3), ("ragged", 16)])
def test_split_banded_solve_matches_direct(hbj, name, runs):
    from oracle import solver

    wl = CASES[name].wl
    m, g, dd = oracle_problem(wl)
    f = W.sources(wl)[0]
    ft = torch.as_tensor(f, device="cuda")
    res = {}
    for shape in (0, hbj.SOLVE_SHAPE_SPLIT):
        ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_BANDED, precond=hbj.PC_BJ)
        ctx.factor()
        ctx.set_solve_tuning(shape)
        ctx.set_solve_partitions(runs)
        say(f"[split solve] case={name} shape={shape} runs={runs}")
        u, st = ctx.solve(ft, tol=1e-12, maxit=2000)
        ctx.close()
        res[shape] = (_np(u), st)
    (u0, s0), (u1, s1) = res[0], res[hbj.SOLVE_SHAPE_SPLIT]
    ref = solver.direct(g, f)
    say(f"  iterations {s0.iters} / {s1.iters}, vs direct {rel(u1, ref):.1e}")
    assert s1.converged == 1 and abs(s1.iters - s0.iters) <= 1
    assert rel(u1, ref) < 1e-8
    assert rel(u1, u0) < 1e-9


def test_split_tuner_and_bad_values(hbj):
    """The autotuner times the split shape beside the others (five candidates per class)."""
    wl = CASES["grf256"].wl
    m, g, dd = oracle_problem(wl)
    hbj.set_tune_cache_path("")
    try:
        ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_BANDED)
        ctx.factor()
        gv = W.random_interface_vector(ctx.nif, seed=53)
        say("[split] tuner")
        w = _np(ctx.apply_operator(torch.as_tensor(gv, device="cuda")))
        t = ctx.solve_tuning()
        for bad in (1, -1, 4097):
            with pytest.raises(hbj.HbjError) as ei:
                ctx.set_solve_partitions(bad)
            assert ei.value.code == hbj.EINVAL
        ctx.close()
    finally:
        hbj.set_tune_cache_path(None)
    assert t
    for key, ch in t.items():
        say(f"  {key}: shape {ch['shape']}, us {ch['us']}")
        assert len(ch["us"]) == len(hbj.SOLVE_SHAPES) and 0 <= ch["shape"] < len(hbj.SOLVE_SHAPES)
        assert ch["us"][hbj.SOLVE_SHAPE_SPLIT] > 0
    assert rel(w, dd.apply_operator(gv)) < 1e-12


def test_backward_window_follows_the_interchanges(hbj):
    """Without row interchanges the backward solves carry only U's ku superdiagonals; a new medium
    whose factorisation interchanges rows (about 3 points per wavelength) brings back the full band.
    The operator against the oracle on one context through both factorisations, for the one-solve
    kernels, the split solves and the MFMA tiles."""
    from oracle.dd import Decomposition
    from oracle.fd import Grid

    wl = CASES["pivot"].wl
    m_piv = W.slowness2(wl)
    m_smooth = m_piv * (3.2 / 10.0) ** 2  # the same medium at 10 points per wavelength
    ctx = gpu_context(hbj, wl, m_smooth, operator_form=hbj.OP_BANDED)
    gv = W.random_interface_vector(ctx.nif, seed=54, nrhs=20)
    gt = torch.as_tensor(gv, device="cuda")
    for label, m in (("no interchanges", m_smooth), ("interchanges", m_piv), ("no interchanges again", m_smooth)):
        ctx.set_slowness2(torch.as_tensor(m, device="cuda"))
        ctx.factor()
        dd = Decomposition(Grid(wl.nx, wl.ny, wl.h, wl.k, m), wl.n1, wl.n2)
        ref = [dd.apply_operator(gv[k]) for k in range(20)]
        ctx.set_solve_tuning(-1)  # the tuner's class keys record whether rows were interchanged
        ctx.apply_operator(gt[0])
        kl = wl.nx // wl.n1  # = ku
        flag = f"|wb{16 + 2 * kl}|p1|" if label == "interchanges" else f"|wb{16 + kl}|p0|"
        assert any(flag in key for key in ctx.solve_tuning()), (label, list(ctx.solve_tuning()))
        for shape in (0, hbj.SOLVE_SHAPE_MFMA, hbj.SOLVE_SHAPE_SPLIT):
            ctx.set_solve_tuning(shape)
            for cols in (1, 20):  # one right-hand side (split solves) and 20 (MFMA tiles)
                say(f"[backward window] {label}, shape {shape}, {cols} right-hand sides")
                w = _np(ctx.apply_operator(gt[0] if cols == 1 else gt))
                w = w.reshape(cols, -1)
                e = max(rel(w[k], ref[k]) for k in range(cols))
                say(f"  vs oracle {e:.1e}")
                assert e < 1e-10
    ctx.close()
