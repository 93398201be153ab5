"""Dataflow sweeps (one launch per preconditioner application) against the oracle and against
the stepped launches, through the C ABI.

The two execution forms compute the same sums in different orders: they agree to 1e-13
relative; each agrees with the oracle to the tolerances of the other parity tests (1e-12 for
one operator application, 1e-11 for a preconditioner application).
"""
import numpy as np
import pytest

import workload as W
from cases import CASES, gpu_context, oracle_problem, rel, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def pair(hbj):
    """(dataflow context, stepped context) of one case, factored once per module."""
    cache = {}

    def get(name, **kw):
        key = (name, tuple(sorted(kw.items())))
        if key not in cache:
            wl = CASES[name].wl
            say(f"[setup] case={name} {kw}")
            m, g, dd = oracle_problem(wl)
            a = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE, sweep_exec=hbj.SWEEP_DATAFLOW, **kw)
            b = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE, sweep_exec=hbj.SWEEP_STEPPED, **kw)
            a.factor()
            b.factor()
            torch.cuda.synchronize()
            cache[key] = (wl, g, dd, a, b)
        return cache[key]

    yield get
    for v in cache.values():
        v[3].close()
        v[4].close()


CASES_PC = [
    ("small", dict(precond=2), dict(kind="bj")),
    ("grf256", dict(precond=2), dict(kind="bj")),
    ("grf256", dict(precond=1), dict(kind="sgs")),
    ("grf256", dict(precond=2, bj_width=3), dict(kind="bj", width=3)),
    ("grf256", dict(precond=2, bj_combine=1), dict(kind="bj", combine="additive")),
    ("grf256", dict(precond=2, bj_compose=1), dict(kind="bj", compose="residual")),
    ("strip", dict(precond=2, bj_width=2), dict(kind="bj", width=2)),
    ("ragged", dict(precond=2), dict(kind="bj")),
    ("rect", dict(precond=1), dict(kind="sgs")),
    ("pivot", dict(precond=2), dict(kind="bj")),
]


@pytest.mark.parametrize("name,kw,okw", CASES_PC)
def test_dataflow_preconditioner(pair, name, kw, okw):
    from oracle import sweep

    wl, g, dd, a, b = pair(name, **kw)
    r = W.random_interface_vector(a.nif, seed=11)
    rt = torch.as_tensor(r, device="cuda")
    say(f"[dataflow precond] case={name} {kw}")
    za = _np(a.apply_preconditioner(rt))
    zb = _np(b.apply_preconditioner(rt))
    assert rel(za, zb) < 1e-13
    assert rel(za, sweep.apply_preconditioner(dd, r, **okw)) < 1e-11


@pytest.mark.parametrize("name", ["small", "grf256", "ragged", "rect", "strip"])
def test_dataflow_operator(pair, name):
    wl, g, dd, a, b = pair(name, precond=2)
    gv = W.random_interface_vector(a.nif, seed=12)
    gt = torch.as_tensor(gv, device="cuda")
    say(f"[dataflow operator] case={name}")
    wa = _np(a.apply_operator(gt))
    wb = _np(b.apply_operator(gt))
    assert rel(wa, wb) < 1e-13
    assert rel(wa, dd.apply_operator(gv)) < 1e-12


@pytest.mark.parametrize("nrhs", [2, 3])
def test_dataflow_few_rhs(pair, nrhs):
    """Right-hand sides below the matrix-product threshold run as separate task columns."""
    from oracle import sweep

    wl, g, dd, a, b = pair("grf256", precond=2)
    gv = W.random_interface_vector(a.nif, seed=13, nrhs=nrhs)
    gt = torch.as_tensor(gv, device="cuda")
    say(f"[dataflow nrhs={nrhs}]")
    z = _np(a.apply_preconditioner(gt))
    w = _np(a.apply_operator(gt))
    for k in range(nrhs):
        assert rel(z[k], sweep.apply_bj(dd, gv[k])) < 1e-11
        assert rel(w[k], dd.apply_operator(gv[k])) < 1e-12


@pytest.mark.parametrize("name,kw", [("grf256", {}), ("strip", {}), ("grf256", dict(precond=1)),
                                     ("grf256", dict(precision=1)), ("grf256", dict(bj_combine=1))])
def test_dataflow_solve(pair, name, kw):
    """GMRES with the fused preconditioner + operator launch: same iterations as the stepped
    form, solution within 1e-8 of the direct solve."""
    from oracle import solver

    kw = dict(dict(precond=2), **kw)
    wl, g, dd, a, b = pair(name, **kw)
    f = torch.as_tensor(W.sources(wl)[0], device="cuda")
    say(f"[dataflow solve] case={name} {kw}")
    ua, sa = a.solve(f, tol=1e-12, maxit=3000)
    ub, sb = b.solve(f, tol=1e-12, maxit=3000)
    say(f"  iters dataflow {sa.iters} stepped {sb.iters}")
    assert abs(sa.iters - sb.iters) <= 1
    assert rel(_np(ua), solver.direct(g, _np(f))) < 1e-8


def test_dataflow_repeated_launches_reuse_counters(pair):
    """Counter regions alternate between launches: many launches in a row stay exact."""
    wl, g, dd, a, b = pair("small", precond=2)
    r = torch.as_tensor(W.random_interface_vector(a.nif, seed=14), device="cuda")
    z0 = _np(a.apply_preconditioner(r))
    for _ in range(7):
        z = _np(a.apply_preconditioner(r))
        assert np.array_equal(z, z0)


def test_dataflow_wait_limit_reports_error_and_recovers(pair, hbj):
    """A task whose waits can never complete (forced from the host) makes the launch report
    HBJ_EWAIT once its bounded wait gives up; every wave exits and the next call is exact."""
    wl, g, dd, a, b = pair("small", precond=2)
    r = torch.as_tensor(W.random_interface_vector(a.nif, seed=15), device="cuda")
    z0 = _np(a.apply_preconditioner(r))
    say("[dataflow wait limit] stalled task")
    # 2 x 2: tasks 0-7 are the first forward step of (1,1); task 10 is a second-step task of
    # (1,2), which waits on the forward tasks of (1,1)
    a.set_sweep_wait(max_polls=2000, stall_task=10)
    with pytest.raises(hbj.HbjError) as ei:
        a.apply_preconditioner(r)
    assert ei.value.code == hbj.EWAIT
    a.set_sweep_wait()
    z = _np(a.apply_preconditioner(r))
    assert np.array_equal(z, z0)
