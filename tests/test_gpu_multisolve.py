"""Banded local solves of many right-hand sides per subdomain on MFMA, through the C ABI.

Batches that average 8 or more right-hand sides per subdomain run 16 of them per workgroup on the
matrix cores (hbj_set_multi_solve): the banded operator, preconditioner, lifting and reconstruction
with many sources, and the formation of the dense operators at factor time (one right-hand side
per interface position). Each result is compared with the oracle and with the kernels that run one
workgroup per solve. Cases: 32^2 subdomains (aligned windows), ragged 10 x 10 (padded windows),
rectangular 16 x 12, the pivoting case (row interchanges inside column blocks), the 5 x 10 strip of
8 x 8 subdomains; 20 right-hand sides, so that every subdomain has one full tile and one partial.
"""
import numpy as np
import pytest

import workload as W
from cases import CASES, gpu_context, oracle_problem, rel, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NRHS = 20


def _np(t):
    return t.detach().cpu().numpy()


def _sources(wl, n):
    xs = np.linspace(0.15, 0.85, n)
    ys = (0.3, 0.5, 0.7)
    return np.stack([W.gaussian_source(wl.nx, wl.ny, wl.h, x, ys[k % 3] * (wl.ny + 1) * wl.h)
                     for k, x in enumerate(xs)])


@pytest.fixture(scope="module")
def banded(hbj):
    cache = {}

    def get(name, precision=0):
        key = (name, precision)
        if key not in cache:
            wl = CASES[name].wl
            m, g, dd = oracle_problem(wl)
            say(f"[setup banded] case={name} precision={precision}")
            ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_BANDED, precision=precision)
            ctx.factor()
            torch.cuda.synchronize()
            cache[key] = (wl, m, g, dd, ctx)
        return cache[key]

    yield get
    for v in cache.values():
        v[4].close()


# Bound on the relative error against the oracle of the banded solves of a case (both launch shapes).
# 1e-12 everywhere except the pivoting case: about 3 points per wavelength, so its local matrices are
# the worst conditioned and the rounding of the elimination grows accordingly.
CASE_TOL = {"pivot": 1e-10}


def _tol(name):
    return CASE_TOL.get(name, 1e-12)


def _both_modes(hbj, ctx, fn):
    """fn() with every batch on the MFMA tiles, then with one workgroup per solve (depths as tuned)."""
    out = {}
    for mode in (hbj.MSOLVE_MFMA, hbj.MSOLVE_CHAINS):
        ctx.set_multi_solve(mode)
        ctx.set_solve_tuning(hbj.SOLVE_SHAPE_MFMA if mode == hbj.MSOLVE_MFMA else -1)
        out[mode] = fn()
    ctx.set_multi_solve(hbj.MSOLVE_MFMA)
    ctx.set_solve_tuning(-1)
    return out[hbj.MSOLVE_MFMA], out[hbj.MSOLVE_CHAINS]


@pytest.mark.parametrize("name", ["small", "ragged", "rect", "pivot", "grf256", "strip"])
def test_many_rhs_operator_lifting_reconstruction(hbj, banded, name):
    wl, m, g, dd, ctx = banded(name)
    gv = W.random_interface_vector(ctx.nif, seed=31, nrhs=NRHS)
    f = _sources(wl, NRHS)
    gt, ft = torch.as_tensor(gv, device="cuda"), torch.as_tensor(f, device="cuda")

    def run():
        say(f"[banded {NRHS} RHS] case={name}")
        w = _np(ctx.apply_operator(gt))
        b = _np(ctx.lifting(ft))
        u = _np(ctx.reconstruct(ft, gt))
        return w, b, u

    mm, chains = _both_modes(hbj, ctx, run)
    ref = ([dd.apply_operator(gv[k]) for k in range(NRHS)], [dd.lifting(f[k]) for k in range(NRHS)],
           [dd.reconstruct(f[k], gv[k]) for k in range(NRHS)])
    for what, a, c, r in zip(("operator", "lifting", "reconstruction"), mm, chains, ref):
        ea = max(rel(a[k], r[k]) for k in range(NRHS))
        ec = max(rel(c[k], r[k]) for k in range(NRHS))
        say(f"  {what}: MFMA {ea:.1e}, one workgroup per solve {ec:.1e} vs oracle; between them {rel(a, c):.1e}")
        assert ea < _tol(name)
        assert ec < _tol(name)
        assert rel(a, c) < _tol(name)


@pytest.mark.parametrize("name", ["ragged", "pivot", "grf256", "strip"])
def test_many_rhs_preconditioner(hbj, banded, name):
    from oracle import sweep

    wl, m, g, dd, ctx = banded(name)
    r = W.random_interface_vector(ctx.nif, seed=32, nrhs=NRHS)
    rt = torch.as_tensor(r, device="cuda")
    say(f"[banded preconditioner {NRHS} RHS] case={name}")
    z, zc = _both_modes(hbj, ctx, lambda: _np(ctx.apply_preconditioner(rt)))
    e = max(rel(z[k], sweep.apply_bj(dd, r[k])) for k in range(NRHS))
    say(f"  vs oracle {e:.1e}")
    assert e < 1e-11
    assert rel(z, zc) < 1e-13


@pytest.mark.parametrize("name", ["grf256", "pivot"])
def test_many_rhs_mixed_precision(hbj, banded, name):
    """complex64 factors: the f32 MFMA solves; the operator is refined to FP64."""
    from oracle import sweep

    wl, m, g, dd, ctx = banded(name, precision=hbj.MIXED)
    gv = W.random_interface_vector(ctx.nif, seed=33, nrhs=NRHS)
    gt = torch.as_tensor(gv, device="cuda")
    say(f"[banded mixed {NRHS} RHS] case={name}")
    (w, z), (wc, zc) = _both_modes(hbj, ctx, lambda: (_np(ctx.apply_operator(gt)), _np(ctx.apply_preconditioner(gt))))
    ew = max(rel(w[k], dd.apply_operator(gv[k])) for k in range(NRHS))
    ez = max(rel(z[k], sweep.apply_bj(dd, gv[k])) for k in range(NRHS))
    say(f"  refined operator {ew:.1e}; complex64 preconditioner {ez:.1e}; vs chains {rel(z, zc):.1e}")
    assert ew < 1e-10
    assert ez < 1e-3
    assert rel(z, zc) < 1e-5


def test_many_rhs_solve(hbj, banded):
    from oracle import solver

    wl, m, g, dd, ctx = banded("grf256")
    f = _sources(wl, 16)
    say("[banded solve 16 RHS]")
    u, st = ctx.solve(torch.as_tensor(f, device="cuda"), tol=1e-12, maxit=3000)
    assert st.converged == 16 and st.relres <= 1e-12
    u = _np(u)
    e = max(rel(u[k], solver.direct(g, f[k])) for k in range(16))
    say(f"  iters {st.iters}, max error vs direct {e:.1e}")
    assert e < 1e-8


@pytest.mark.parametrize("name,transmission", [("grf256", 1), ("ragged", 1), ("pivot", 1), ("rect", 1),
                                               ("grf256", 2)])
def test_dense_operators_formed_on_mfma(hbj, name, transmission):
    """hbj_factor forms T_s and W_s from one solve per interface position: 16 per workgroup."""
    from oracle.dd import Decomposition

    wl = CASES[name].wl
    m, g, dd = oracle_problem(wl)
    if transmission == 2:
        dd = Decomposition(g, wl.n1, wl.n2, transmission=2)
    gv = W.random_interface_vector(dd.nif, seed=34)
    f = _sources(wl, 1)[0]
    res = {}
    for mode in (hbj.MSOLVE_MFMA, hbj.MSOLVE_CHAINS):
        ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE, transmission=transmission)
        ctx.set_multi_solve(mode)
        if mode == hbj.MSOLVE_MFMA:
            ctx.set_solve_tuning(hbj.SOLVE_SHAPE_MFMA)
        say(f"[dense operators] case={name} transmission={transmission} mode={mode}")
        ctx.factor()
        gt, ft = torch.as_tensor(gv, device="cuda"), torch.as_tensor(f, device="cuda")
        res[mode] = (_np(ctx.apply_operator(gt)), _np(ctx.lifting(ft)), _np(ctx.reconstruct(ft, gt)))
        ctx.close()
    ref = (dd.apply_operator(gv), dd.lifting(f), dd.reconstruct(f, gv))
    for what, a, c, r in zip(("operator", "lifting", "reconstruction"), res[hbj.MSOLVE_MFMA],
                             res[hbj.MSOLVE_CHAINS], ref):
        ea, ec = rel(a, r), rel(c, r)
        say(f"  {what}: MFMA {ea:.1e}, one workgroup per solve {ec:.1e} vs oracle; between them {rel(a, c):.1e}")
        assert ea < _tol(name)
        assert ec < _tol(name)
        assert rel(a, c) < _tol(name)


def test_multi_solve_bad_mode(hbj):
    wl = W.SMALL
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=torch.as_tensor(W.slowness2(wl), device="cuda"))
    with pytest.raises(hbj.HbjError) as ei:
        ctx.set_multi_solve(2)
    assert ei.value.code == hbj.EINVAL
    ctx.close()
