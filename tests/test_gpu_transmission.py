"""Second-order transmission condition: the HIP path against the oracle, through the C ABI.

The condition changes the local matrices (tangential couplings along interface faces), the data
sent across faces (R and Sigma bands along each face) and, with them, the dense operators, the
lifting and the reconstruction. Each is compared with the oracle's decomposition built with the
same condition, at the tolerances of the first-order tests; the solve is checked against the
global direct solution (the condition does not change the global problem). Cases: aligned
(32^2 subdomains), ragged (10 x 10), rectangular (16 x 12) and the 5 x 10 strip (8 x 8), in the dense and
the banded operator forms.
"""
import numpy as np
import pytest

import workload as W
from cases import CASES, gpu_context, rel, say, sub_index

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def ctx2(hbj):
    from oracle.dd import Decomposition
    from oracle.fd import Grid

    cache = {}

    def get(name, **kw):
        key = (name, tuple(sorted(kw.items())))
        if key not in cache:
            wl = CASES[name].wl
            say(f"[setup order 2] case={name} {kw}")
            m = W.slowness2(wl)
            g = Grid(wl.nx, wl.ny, wl.h, wl.k, m)
            dd = Decomposition(g, wl.n1, wl.n2, transmission=2)
            kw2 = dict(kw)
            kw2.setdefault("operator_form", hbj.OP_DENSE)
            ctx = gpu_context(hbj, wl, m, transmission=2, **kw2)
            ctx.factor()
            torch.cuda.synchronize()
            cache[key] = (wl, m, g, dd, ctx)
        return cache[key]

    yield get
    for v in cache.values():
        v[4].close()


@pytest.mark.parametrize("name", ["grf256", "ragged", "rect", "strip"])
def test_second_order_local_solve(ctx2, name):
    wl, m, g, dd, ctx = ctx2(name)
    subs = list(dd.sub)
    rng = np.random.default_rng(5)
    rhs = rng.standard_normal((len(subs), ctx.n_loc)) + 1j * rng.standard_normal((len(subs), ctx.n_loc))
    say(f"[order 2 local_solve] case={name}")
    x = _np(ctx.local_solve([sub_index(wl, i) for i in subs], torch.as_tensor(rhs, device="cuda")))
    for k, i in enumerate(subs):
        assert rel(x[k], dd.sub[i].lu.solve(rhs[k])) < 1e-12


@pytest.mark.parametrize("name", ["grf256", "ragged", "rect", "strip"])
def test_second_order_operator_lifting_reconstruction(ctx2, name):
    wl, m, g, dd, ctx = ctx2(name)
    f = W.sources(wl)[0]
    gv = W.random_interface_vector(ctx.nif, seed=21)
    say(f"[order 2 operator / lifting / reconstruction] case={name}")
    w = _np(ctx.apply_operator(torch.as_tensor(gv, device="cuda")))
    assert rel(w, dd.apply_operator(gv)) < 1e-12
    b = _np(ctx.lifting(torch.as_tensor(f, device="cuda")))
    assert rel(b, dd.lifting(f)) < 1e-12
    u = _np(ctx.reconstruct(torch.as_tensor(f[None], device="cuda"), torch.as_tensor(gv[None], device="cuda")))[0]
    assert rel(u, dd.reconstruct(f, gv)) < 1e-12


def test_second_order_many_rhs(ctx2):
    """The matrix-product operators and the many-RHS reconstruction (5 columns)."""
    wl, m, g, dd, ctx = ctx2("grf256")
    gv = W.random_interface_vector(ctx.nif, seed=22, nrhs=5)
    f = np.stack([W.gaussian_source(wl.nx, wl.ny, wl.h, x, 0.4) for x in np.linspace(0.2, 0.8, 5)])
    say("[order 2 operator, 5 RHS]")
    w = _np(ctx.apply_operator(torch.as_tensor(gv, device="cuda")))
    b = _np(ctx.lifting(torch.as_tensor(f, device="cuda")))
    u = _np(ctx.reconstruct(torch.as_tensor(f, device="cuda"), torch.as_tensor(gv, device="cuda")))
    for k in range(5):
        assert rel(w[k], dd.apply_operator(gv[k])) < 1e-12
        assert rel(b[k], dd.lifting(f[k])) < 1e-12
        assert rel(u[k], dd.reconstruct(f[k], gv[k])) < 1e-12


@pytest.mark.parametrize("name", ["grf256", "strip", "rect"])
def test_second_order_preconditioner(ctx2, name):
    from oracle import sweep

    wl, m, g, dd, ctx = ctx2(name, precond=2)
    r = W.random_interface_vector(ctx.nif, seed=23)
    say(f"[order 2 preconditioner] case={name}")
    z = _np(ctx.apply_preconditioner(torch.as_tensor(r, device="cuda")))
    assert rel(z, sweep.apply_bj(dd, r)) < 1e-11


@pytest.mark.parametrize("name,kw", [("grf256", dict(precond=2)), ("ragged", dict(precond=2)),
                                     ("grf256", dict(precond=2, precision=1)), ("strip", dict(precond=1))])
def test_second_order_solve(ctx2, hbj, name, kw):
    from oracle import solver

    wl, m, g, dd, ctx = ctx2(name, **kw)
    f = W.sources(wl)[0]
    say(f"[order 2 solve] case={name} {kw}")
    u, st = ctx.solve(torch.as_tensor(f, device="cuda"), tol=1e-12, maxit=3000)
    assert st.relres <= 1e-12
    assert rel(_np(u), solver.direct(g, f)) < 1e-8
    if kw.get("precision", 0) == 0:
        kind = {1: "sgs", 2: "bj"}[kw["precond"]]
        ro = solver.dd_solve(dd, f, precond=kind, tol=1e-12, maxit=3000)
        say(f"  iters GPU {st.iters} oracle {ro.iters}")
        assert abs(ro.iters - st.iters) <= 1


def test_second_order_needs_fewer_iterations(ctx2, hbj):
    """On the bench physics at 256^2 (8 x 8 of 32^2), to 1e-6: fewer block-Jacobi GMRES iterations
    than the first-order condition, same field."""
    wl, m, g, dd, ctx = ctx2("grf256", precond=2)
    f = torch.as_tensor(W.sources(wl)[0], device="cuda")
    c1 = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE, precond=2)
    c1.factor()
    u1, s1 = c1.solve(f, tol=1e-10)
    u2, s2 = ctx.solve(f, tol=1e-10)
    say(f"[order 2 vs 1] iterations {s2.iters} vs {s1.iters}")
    assert s2.iters < s1.iters
    assert rel(_np(u2), _np(u1)) < 1e-7
    c1.close()


@pytest.mark.parametrize("name,precision", [("grf256", 0), ("ragged", 0), ("strip", 0), ("grf256", 1)])
def test_second_order_banded_form(ctx2, hbj, name, precision):
    """Banded local solves: the traces follow the solves in a second kernel (whole-face fields);
    mixed precision refines the complex64 solves before the traces are taken."""
    from oracle import solver, sweep

    wl, m, g, dd, ctx = ctx2(name, operator_form=hbj.OP_BANDED, precision=precision)
    gv = W.random_interface_vector(ctx.nif, seed=24)
    f = W.sources(wl)[0]
    say(f"[order 2 banded] case={name} precision={precision}")
    assert rel(_np(ctx.apply_operator(torch.as_tensor(gv, device="cuda"))), dd.apply_operator(gv)) < 1e-11
    assert rel(_np(ctx.lifting(torch.as_tensor(f, device="cuda"))), dd.lifting(f)) < 1e-12
    if precision == 0:
        z = _np(ctx.apply_preconditioner(torch.as_tensor(gv, device="cuda")))
        assert rel(z, sweep.apply_bj(dd, gv)) < 1e-11
    u, st = ctx.solve(torch.as_tensor(f, device="cuda"), tol=1e-12, maxit=3000)
    assert st.relres <= 1e-12
    assert rel(_np(u), solver.direct(g, f)) < 1e-8
