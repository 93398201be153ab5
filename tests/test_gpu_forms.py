"""GPU tests of the mixed-precision form and the adjoint gradient against the oracle.

Mixed precision: complex64 factors for the preconditioner; the operator's local
solves are refined with an FP64 residual, so the operator agrees with the FP64 one
to near double precision, and FGMRES reaches FP64 residuals.  The errors against
the FP64 oracle are printed for every result.

Gradient: dL/dm from forward + adjoint GPU solves against the oracle's direct-solve
gradient and against central finite differences of the misfit.
"""
import numpy as np
import pytest

import workload as W
from cases import CASES, gpu_context, oracle_problem, rel, say, sub_index

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def mixed(hbj):
    wl = CASES["grf256"].wl
    m, g, dd = oracle_problem(wl)
    say("[setup] mixed grf256")
    ctx = gpu_context(hbj, wl, m, precision=hbj.MIXED)
    ctx.factor()
    ref = gpu_context(hbj, wl, m, precision=hbj.FP64)
    ref.factor()
    yield wl, m, g, dd, ctx, ref
    ctx.close()
    ref.close()


def test_mixed_local_solve_error(hbj, mixed):
    wl, m, g, dd, ctx, ref = mixed
    subs = list(dd.sub)[:8]
    rng = np.random.default_rng(3)
    rhs = rng.standard_normal((len(subs), ctx.n_loc)) + 1j * rng.standard_normal((len(subs), ctx.n_loc))
    say("[mixed local_solve]")
    x = _np(ctx.local_solve([sub_index(wl, i) for i in subs], torch.as_tensor(rhs, device="cuda"),
                            precision=hbj.MIXED))
    errs = [rel(x[k], dd.sub[i].lu.solve(rhs[k])) for k, i in enumerate(subs)]
    say(f"  complex64 local solve error vs FP64 oracle: max {max(errs):.2e}")
    assert max(errs) < 1e-4


def test_mixed_operator_is_refined_to_fp64(mixed):
    wl, m, g, dd, ctx, ref = mixed
    gv = W.random_interface_vector(ctx.nif, seed=4)
    say("[mixed operator]")
    w = _np(ctx.apply_operator(torch.as_tensor(gv, device="cuda")))
    e = rel(w, dd.apply_operator(gv))
    say(f"  refined operator error vs oracle: {e:.2e}")
    assert e < 1e-10


def test_mixed_preconditioner_error(mixed):
    from oracle import sweep

    wl, m, g, dd, ctx, ref = mixed
    r = W.random_interface_vector(ctx.nif, seed=5)
    say("[mixed preconditioner]")
    z = _np(ctx.apply_preconditioner(torch.as_tensor(r, device="cuda")))
    e = rel(z, sweep.apply_bj(dd, r))
    say(f"  complex64 preconditioner error vs oracle: {e:.2e}")
    assert e < 1e-3


@pytest.mark.parametrize("tol", [1e-6, 1e-8])
def test_mixed_solve_reaches_fp64_residual(mixed, tol):
    from oracle import solver

    wl, m, g, dd, ctx, ref = mixed
    f = W.sources(wl)[0]
    say(f"[mixed solve] tol={tol}")
    u, st = ctx.solve(torch.as_tensor(f, device="cuda"), tol=tol, maxit=500)
    u64, st64 = ref.solve(torch.as_tensor(f, device="cuda"), tol=tol, maxit=500)
    ud = solver.direct(g, f)
    e, e64 = rel(_np(u), ud), rel(_np(u64), ud)
    say(f"  mixed: iters {st.iters} relres {st.relres:.2e} err vs oracle {e:.2e}; "
        f"fp64: iters {st64.iters} err {e64:.2e}")
    say(f"  refined local solves: at most {st.local_ir_max} complex64 solves, "
        f"largest final relative local residual {st.local_ir_resid:.2e}")
    assert st.relres <= tol
    assert abs(st.iters - st64.iters) <= 3
    # the banded operator's refinement reaches FP64-level local residuals in a few solves
    assert 2 <= st.local_ir_max <= 8
    assert 0 < st.local_ir_resid <= 1e-12
    assert st64.local_ir_max == 0 and st64.local_ir_resid == 0
    # the same solution quality as the FP64 solver at the same tolerance
    assert e < 10 * max(e64, tol)


# ---------------------------------------------------------------------------
# adjoint gradient
# ---------------------------------------------------------------------------

def _gradient_problem(nx, n1, nsrc, seed=2):
    base = W.GRAD_512
    wl = W.scaled(base, nx, n1=n1, n2=n1, sources=W.sources_along_line(nsrc, 0.05))
    m_true = W.slowness2(W.scaled(base, nx, medium="grf_m"))
    m0 = W.smoothed_model(m_true, 20.0 * nx / 512)
    f = W.sources(wl)
    rec = W.receiver_row(wl)
    return wl, m_true, m0, f, rec


def _data(wl, m_true, f, rec):
    from oracle.fd import Grid
    from oracle import solver

    g = Grid(wl.nx, wl.ny, wl.h, wl.k, m_true)
    u = solver.direct(g, f)
    return np.ascontiguousarray(u.reshape(f.shape[0], -1)[:, rec])


@pytest.mark.parametrize("nx,n1,nsrc,transmission", [(64, 4, 3, 1), (512, 8, 16, 1), (128, 4, 3, 2)])
def test_gradient_matches_oracle_direct(hbj, nx, n1, nsrc, transmission):
    from oracle import gradient
    from oracle.fd import Grid

    wl, m_true, m0, f, rec = _gradient_problem(nx, n1, nsrc)
    d = _data(wl, m_true, f, rec)
    say(f"[gradient] nx={nx} {n1}x{n1} sources={nsrc} transmission={transmission}")
    # the interface condition changes the iteration, not the global problem nor its adjoint
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=torch.as_tensor(m0, device="cuda"),
                    transmission=transmission)
    ctx.factor()
    loss, grad = ctx.gradient(torch.as_tensor(f, device="cuda"), torch.as_tensor(rec, device="cuda"),
                              torch.as_tensor(d, device="cuda"), tol=1e-12)
    grad = _np(grad)
    ctx.close()
    L0, g0 = gradient.misfit_and_gradient(Grid(wl.nx, wl.ny, wl.h, wl.k, m0), f, rec.astype(np.int64), d)
    e = rel(grad, g0)
    say(f"  loss {loss:.6e} vs oracle {L0:.6e}; gradient error vs direct-solve gradient {e:.2e}")
    assert abs(loss - L0) <= 1e-8 * abs(L0)
    assert e < 1e-8


def test_gradient_central_differences_oracle_loss(hbj):
    """Directional derivatives <grad, dm> against central differences of the oracle's direct misfit."""
    from oracle import gradient
    from oracle.fd import Grid

    wl, m_true, m0, f, rec = _gradient_problem(64, 4, 3)
    d = _data(wl, m_true, f, rec)
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=torch.as_tensor(m0, device="cuda"))
    ctx.factor()
    say("[gradient fd] nx=64")
    loss, grad = ctx.gradient(torch.as_tensor(f, device="cuda"), torch.as_tensor(rec, device="cuda"),
                              torch.as_tensor(d, device="cuda"), tol=1e-12)
    grad = _np(grad)
    ctx.close()
    eps = 1e-6
    worst = 0.0
    for j in range(20):
        dm = W.gradient_direction(m0.shape, j)
        Lp = gradient.misfit(Grid(wl.nx, wl.ny, wl.h, wl.k, m0 + eps * dm), f, rec, d)
        Lm = gradient.misfit(Grid(wl.nx, wl.ny, wl.h, wl.k, m0 - eps * dm), f, rec, d)
        fd = (Lp - Lm) / (2 * eps)
        an = float(np.sum(grad * dm))
        worst = max(worst, abs(fd - an) / abs(an))
    say(f"  worst relative FD error over 20 directions: {worst:.2e}")
    assert worst < 1e-5


@pytest.mark.timeout(600)
def test_gradient_full_size_central_differences_oracle_loss(hbj):
    """512^2, 8 x 8 of 64^2, 16 sources: the adjoint gradient from GPU solves at tol 1e-12 against
    central differences (eps = 1e-6) of the oracle's direct-solve misfit on the 20 seeded
    directions, as stored by tests/golden/make_grad_fd.py."""
    import json
    import os

    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "grad_512_fd.json")))
    wl, m_true, m0, f, rec = _gradient_problem(512, 8, 16)
    assert gold["workload"] == wl.name.split("@")[0] and len(gold["directions"]) == 20
    d = _data(wl, m_true, f, rec)
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=torch.as_tensor(m0, device="cuda"))
    ctx.factor()
    say("[gradient fd] nx=512 16 sources, 20 directions against the oracle's misfit")
    loss, grad = ctx.gradient(torch.as_tensor(f, device="cuda"), torch.as_tensor(rec, device="cuda"),
                              torch.as_tensor(d, device="cuda"), tol=1e-12)
    grad = _np(grad)
    ctx.close()
    say(f"  loss {loss:.10e} (oracle at m0 {gold['loss_m0']:.10e})")
    assert abs(loss - gold["loss_m0"]) <= 1e-8 * gold["loss_m0"]
    worst = 0.0
    for ent in gold["directions"]:
        dm = W.gradient_direction(m0.shape, ent["j"])
        an = float(np.sum(grad * dm))
        err = abs(ent["fd"] - an) / abs(an)
        worst = max(worst, err)
        say(f"  direction {ent['j']}: fd {ent['fd']:.10e} adjoint {an:.10e} rel {err:.1e}")
    assert worst < 1e-5


def test_autograd_function(hbj):
    from paper_2209_10886_amd.autograd import misfit

    wl, m_true, m0, f, rec = _gradient_problem(64, 4, 2)
    d = _data(wl, m_true, f, rec)
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=torch.as_tensor(m0, device="cuda"))
    m = torch.as_tensor(m0, device="cuda").requires_grad_(True)
    say("[autograd]")
    L = misfit(m, ctx, torch.as_tensor(f, device="cuda"), torch.as_tensor(rec, device="cuda"),
               torch.as_tensor(d, device="cuda"), 1e-12)
    (2.0 * L).backward()
    loss, grad = ctx.gradient(torch.as_tensor(f, device="cuda"), torch.as_tensor(rec, device="cuda"),
                              torch.as_tensor(d, device="cuda"), tol=1e-12)
    ctx.close()
    assert abs(L.item() - loss) <= 1e-12 * abs(loss)
    assert torch.allclose(m.grad, 2.0 * grad, rtol=1e-9, atol=0)
