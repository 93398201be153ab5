"""HIP path against the oracle, element by element, through the C ABI.

Tolerances (complex128): band factors 1e-13 relative to the largest entry of the
column; one local solve 1e-12; the interface operators 1e-11 (a composition of up
to 2 N_g local solves); solutions at tol 1e-12 within 1e-8 of the oracle's.
"""
import numpy as np
import pytest

import workload as W
from cases import CASES, gpu_context, oracle_problem, rel, say, sub_index

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _to_np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def ctxs(hbj):
    cache = {}

    def get(name, **kw):
        key = (name, tuple(sorted(kw.items())))
        if key not in cache:
            wl = CASES[name].wl
            say(f"[setup] case={name} {kw} nx={wl.nx} ny={wl.ny} n1={wl.n1} n2={wl.n2}")
            m, g, dd = oracle_problem(wl)
            ctx = gpu_context(hbj, wl, m, **kw)
            ctx.factor()
            torch.cuda.synchronize()
            cache[key] = (wl, m, g, dd, ctx)
        return cache[key]

    yield get
    for v in cache.values():
        v[4].close()


@pytest.mark.parametrize("name", ["small", "ragged", "rect", "pivot"])
def test_band_lu_matches_lapack(ctxs, name):
    from scipy.linalg import lapack

    wl, m, g, dd, ctx = ctxs(name)
    for i in [(1, 1), (wl.n1, wl.n2)]:
        s = sub_index(wl, i)
        say(f"[band_lu] case={name} sub={s}")
        A = dd.sub[i].A.toarray()
        n, kl = A.shape[0], ctx.kl
        ldab = 2 * kl + kl + 1
        ab = np.zeros((ldab, n), dtype=np.complex128)
        for j in range(n):
            for r in range(max(0, j - kl), min(n, j + kl + 1)):
                ab[2 * kl + r - j, j] = A[r, j]
        lu, piv, info = lapack.zgbtrf(ab, kl, kl)
        assert info == 0
        gab, gip = ctx.band_factors(s)
        gab = _to_np(gab).T
        gip = _to_np(gip)
        assert np.array_equal(gip, piv), "pivot sequence differs from LAPACK"
        scale = np.abs(lu).max(axis=0, keepdims=True)
        err = np.abs(gab - lu) / scale
        assert err.max() < 1e-13, err.max()


@pytest.mark.parametrize("name", ["small", "ragged", "rect", "grf256", "pivot"])
def test_local_solve(ctxs, name):
    wl, m, g, dd, ctx = ctxs(name)
    subs = list(dd.sub)
    rng = np.random.default_rng(11)
    rhs = rng.standard_normal((len(subs), ctx.n_loc)) + 1j * rng.standard_normal((len(subs), ctx.n_loc))
    say(f"[local_solve] case={name} batch={len(subs)}")
    x = _to_np(ctx.local_solve([sub_index(wl, i) for i in subs], torch.as_tensor(rhs, device="cuda")))
    for k, i in enumerate(subs):
        ref = dd.sub[i].lu.solve(rhs[k])
        assert rel(x[k], ref) < 1e-12, (i, rel(x[k], ref))


@pytest.mark.parametrize("name", ["small", "ragged", "rect", "grf256", "strip", "pivot"])
def test_lifting_and_operator(ctxs, name):
    wl, m, g, dd, ctx = ctxs(name)
    f = W.sources(wl)[0]
    say(f"[lifting] case={name}")
    b = _to_np(ctx.lifting(torch.as_tensor(f, device="cuda")))
    assert rel(b, dd.lifting(f)) < 1e-12
    gv = W.random_interface_vector(ctx.nif, seed=1)
    say(f"[operator] case={name}")
    w = _to_np(ctx.apply_operator(torch.as_tensor(gv, device="cuda")))
    assert rel(w, dd.apply_operator(gv)) < 1e-12


@pytest.mark.parametrize("name,kw,okw", [
    ("small", dict(precond=1), dict(kind="sgs")),
    ("small", dict(precond=2), dict(kind="bj")),
    ("grf256", dict(precond=1), dict(kind="sgs")),
    ("grf256", dict(precond=2), dict(kind="bj")),
    ("grf256", dict(precond=2, bj_width=3), dict(kind="bj", width=3)),
    ("grf256", dict(precond=2, bj_combine=1), dict(kind="bj", combine="additive")),
    ("grf256", dict(precond=2, bj_compose=1), dict(kind="bj", compose="residual")),
    ("strip", dict(precond=2), dict(kind="bj")),
    ("strip", dict(precond=2, bj_width=1), dict(kind="bj", width=1)),
    ("rect", dict(precond=2), dict(kind="bj")),
])
def test_preconditioner(ctxs, name, kw, okw):
    from oracle import sweep

    wl, m, g, dd, ctx = ctxs(name, **kw)
    r = W.random_interface_vector(ctx.nif, seed=2)
    say(f"[precond] case={name} {kw}")
    z = _to_np(ctx.apply_preconditioner(torch.as_tensor(r, device="cuda")))
    zo = sweep.apply_preconditioner(dd, r, **okw)
    assert rel(z, zo) < 1e-11, rel(z, zo)
    expect = sweep.step_counts(wl.n1, wl.n2, okw.get("width"))[0 if okw["kind"] == "sgs" else 1]
    assert ctx.steps_per_preconditioner() == expect


def test_operator_multi_rhs(ctxs):
    wl, m, g, dd, ctx = ctxs("grf256")
    gv = W.random_interface_vector(ctx.nif, seed=3, nrhs=3)
    say("[operator nrhs=3] case=grf256")
    w = _to_np(ctx.apply_operator(torch.as_tensor(gv, device="cuda")))
    z = _to_np(ctx.apply_preconditioner(torch.as_tensor(gv, device="cuda")))
    from oracle import sweep

    for k in range(3):
        assert rel(w[k], dd.apply_operator(gv[k])) < 1e-12
        assert rel(z[k], sweep.apply_bj(dd, gv[k])) < 1e-11


@pytest.mark.parametrize("name,precond", [("small", 2), ("grf256", 2), ("grf256", 1), ("ragged", 2), ("one", 2),
                                          ("strip", 2), ("rect", 0), ("pivot", 2)])
def test_solve_matches_direct(ctxs, name, precond):
    from oracle import solver

    wl, m, g, dd, ctx = ctxs(name, precond=precond)
    f = W.sources(wl)[0]
    say(f"[solve] case={name} precond={precond}")
    u, st = ctx.solve(torch.as_tensor(f, device="cuda"), tol=1e-12, maxit=3000)
    u = _to_np(u)
    ud = solver.direct(g, f)
    assert rel(u, ud) < 1e-8, rel(u, ud)
    assert st.relres <= 1e-12
    # the oracle's own DD-GMRES takes the same number of iterations (within one)
    kind = {0: "none", 1: "sgs", 2: "bj"}[precond]
    if dd.nif and wl.nx * wl.ny <= 256 * 256:
        ro = solver.dd_solve(dd, f, precond=kind, tol=1e-12, maxit=3000)
        assert abs(ro.iters - st.iters) <= 1, (ro.iters, st.iters)


def test_solve_multi_rhs_columns_independent(ctxs):
    from oracle import solver

    wl, m, g, dd, ctx = ctxs("grf256")
    f = np.stack([W.gaussian_source(wl.nx, wl.ny, wl.h, x, 0.2) for x in (0.2, 0.5, 0.8)])
    say("[solve nrhs=3] case=grf256")
    u, st = ctx.solve(torch.as_tensor(f, device="cuda"), tol=1e-12, maxit=3000)
    u = _to_np(u)
    for k in range(3):
        assert rel(u[k], solver.direct(g, f[k])) < 1e-8


def test_zero_rhs(ctxs):
    wl, m, g, dd, ctx = ctxs("small")
    f = torch.zeros((wl.ny, wl.nx), dtype=torch.complex128, device="cuda")
    say("[zero rhs]")
    u, st = ctx.solve(f)
    assert st.iters == 0 and torch.count_nonzero(u).item() == 0


# ---------------------------------------------------------------------------
# dense scattering operators (formed at factor time) must reproduce the same operators
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["small", "ragged", "rect", "grf256", "strip", "pivot"])
def test_dense_operator(ctxs, name):
    wl, m, g, dd, ctx = ctxs(name, operator_form=1)
    gv = W.random_interface_vector(ctx.nif, seed=1)
    say(f"[dense operator] case={name}")
    w = _to_np(ctx.apply_operator(torch.as_tensor(gv, device="cuda")))
    assert rel(w, dd.apply_operator(gv)) < 1e-12


@pytest.mark.parametrize("name", ["small", "ragged", "rect", "grf256", "strip", "pivot"])
def test_dense_lifting(ctxs, name):
    """Dense lifting operators (rows of A_s^{-1} at the edge nodes, from the unit-datum
    solves): the lifting data of a Gaussian source, of a random field (every subdomain has a
    source), and of an all-zero right-hand side."""
    wl, m, g, dd, ctx = ctxs(name, operator_form=1)
    rng = np.random.default_rng(21)
    f0 = W.sources(wl)[0]
    f1 = (rng.standard_normal((wl.ny, wl.nx)) + 1j * rng.standard_normal((wl.ny, wl.nx))).astype(np.complex128)
    f = np.stack([f0, f1, np.zeros_like(f0)])
    say(f"[dense lifting] case={name}")
    b = _to_np(ctx.lifting(torch.as_tensor(f, device="cuda")))
    assert rel(b[0], dd.lifting(f0)) < 1e-12
    assert rel(b[1], dd.lifting(f1)) < 1e-12
    assert np.count_nonzero(b[2]) == 0


@pytest.mark.parametrize("name", ["small", "ragged", "rect", "grf256", "pivot"])
@pytest.mark.parametrize("form", [0, 1])
def test_reconstruct(ctxs, name, form):
    """u = A_s^{-1}(f_s + B_s g) on every subdomain, banded (one local solve each) or dense
    (source part by local solves, transmission part through the lifting matrices); a Gaussian
    source, a random source and a zero source, each with random interface data."""
    wl, m, g, dd, ctx = ctxs(name, operator_form=form)
    rng = np.random.default_rng(23)
    f0 = W.sources(wl)[0]
    f1 = (rng.standard_normal((wl.ny, wl.nx)) + 1j * rng.standard_normal((wl.ny, wl.nx))).astype(np.complex128)
    f = np.stack([f0, f1, np.zeros_like(f0)])
    gv = W.random_interface_vector(ctx.nif, seed=24, nrhs=3)
    say(f"[reconstruct] case={name} form={form}")
    u = _to_np(ctx.reconstruct(torch.as_tensor(f, device="cuda"), torch.as_tensor(gv, device="cuda")))
    for k in range(3):
        assert rel(u[k], dd.reconstruct(f[k], gv[k])) < 1e-12
    if form == 1:
        # five columns: the transmission part as MFMA products (one read of W_s for all columns)
        f5 = np.concatenate([f, f[:2] * (1 + 1j)])
        g5 = W.random_interface_vector(ctx.nif, seed=25, nrhs=5)
        u5 = _to_np(ctx.reconstruct(torch.as_tensor(f5, device="cuda"), torch.as_tensor(g5, device="cuda")))
        for k in range(5):
            assert rel(u5[k], dd.reconstruct(f5[k], g5[k])) < 1e-12


@pytest.mark.parametrize("name,kw,okw", [
    ("small", dict(precond=2), dict(kind="bj")),
    ("grf256", dict(precond=1), dict(kind="sgs")),
    ("grf256", dict(precond=2), dict(kind="bj")),
    ("grf256", dict(precond=2, bj_combine=1, bj_compose=1), dict(kind="bj", combine="additive", compose="residual")),
    ("strip", dict(precond=2, bj_width=2), dict(kind="bj", width=2)),
    ("rect", dict(precond=2), dict(kind="bj")),
])
def test_dense_preconditioner(ctxs, name, kw, okw):
    from oracle import sweep

    wl, m, g, dd, ctx = ctxs(name, operator_form=1, **kw)
    r = W.random_interface_vector(ctx.nif, seed=2)
    say(f"[dense precond] case={name} {kw}")
    z = _to_np(ctx.apply_preconditioner(torch.as_tensor(r, device="cuda")))
    assert rel(z, sweep.apply_preconditioner(dd, r, **okw)) < 1e-11


@pytest.mark.parametrize("name,kw", [("small", {}), ("grf256", {}), ("strip", {}), ("pivot", {}),
                                     ("grf256", dict(precision=1))])
def test_dense_solve(ctxs, name, kw):
    from oracle import solver

    wl, m, g, dd, ctx = ctxs(name, operator_form=1, **kw)
    f = W.sources(wl)[0]
    say(f"[dense solve] case={name} {kw}")
    u, st = ctx.solve(torch.as_tensor(f, device="cuda"), tol=1e-12, maxit=3000)
    ud = solver.direct(g, f)
    e = rel(_to_np(u), ud)
    say(f"  iters {st.iters} relres {st.relres:.2e} err vs direct {e:.2e}")
    assert e < 1e-8
    assert st.relres <= 1e-12


# ---------------------------------------------------------------------------
# many right-hand sides: the dense operators run as MFMA products (>= 4 columns)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,kw", [("grf256", {}), ("rect", {}), ("ragged", {}), ("grf256", dict(precision=1))])
def test_dense_operators_many_rhs(ctxs, name, kw):
    from oracle import sweep

    wl, m, g, dd, ctx = ctxs(name, operator_form=1, **kw)
    nr = 5
    gv = W.random_interface_vector(ctx.nif, seed=7, nrhs=nr)
    say(f"[dense many-rhs] case={name} {kw} nrhs={nr}")
    w = _to_np(ctx.apply_operator(torch.as_tensor(gv, device="cuda")))
    z = _to_np(ctx.apply_preconditioner(torch.as_tensor(gv, device="cuda")))
    tol_pc = 1e-11 if not kw else 1e-5  # complex64 operators inside the mixed preconditioner
    for k in range(nr):
        assert rel(w[k], dd.apply_operator(gv[k])) < 1e-12
        assert rel(z[k], sweep.apply_bj(dd, gv[k])) < tol_pc
    # the autotuner timed every variant on the first launch of each kind and kept one, or read the
    # choice of an earlier context with the same geometry from the tuning cache (nothing timed)
    tun = ctx.tuning()
    used = ("c64" if kw else "c128") + " steps"
    assert tun[used]["k_steps_per_batch"] in (2, 4, 8)
    us = list(tun[used]["us"].values())
    assert all(v > 0 for v in us) or all(v == 0 for v in us)


@pytest.mark.parametrize("variant,nr", [(v, 20) for v in range(22)] + [(1, 70), (4, 70), (10, 70), (13, 70), (15, 70),
                                                                       (16, 70), (17, 70), (19, 70), (20, 70)])
@pytest.mark.parametrize("kw", [{}, dict(precision=1)])
def test_operator_kernel_variants(hbj, ctxs, kw, variant, nr):
    """Every variant of the many-RHS operator kernel (tile depth 2/4/8 or a ring of 4/8 k-steps,
    incoming data gathered into tiles or read from the interface vector, one or two wavefront
    groups, XCD-ordered tiles), forced, against the oracle; 70 columns span two 64-column tiles."""
    from oracle import sweep

    wl, m, g, dd, ctx = ctxs("ragged", operator_form=1, **kw)
    gv = W.random_interface_vector(ctx.nif, seed=11, nrhs=nr)
    say(f"[operator kernel variant] {variant} nrhs={nr} {kw}")
    ctx.set_tuning([variant] * 4)
    try:
        w = _to_np(ctx.apply_operator(torch.as_tensor(gv, device="cuda")))
        z = _to_np(ctx.apply_preconditioner(torch.as_tensor(gv, device="cuda")))
        tun = ctx.tuning()
    finally:
        ctx.set_tuning([-1] * 4)
    tol_pc = 1e-11 if not kw else 1e-5
    for k in range(nr):
        assert rel(w[k], dd.apply_operator(gv[k])) < 1e-12
        assert rel(z[k], sweep.apply_bj(dd, gv[k])) < tol_pc
    used = ("c64" if kw else "c128") + " steps"
    want = hbj.mm_variant_fields(variant)
    for key in ("k_steps_per_batch", "incoming", "wave_groups", "k_waves", "ring", "xcd_order"):
        assert tun[used][key] == want[key]


def test_set_tuning_rejects_bad_variants(hbj, ctxs):
    wl, m, g, dd, ctx = ctxs("ragged", operator_form=1)
    with pytest.raises(hbj.HbjError):
        ctx.set_tuning([0, 0, 22, 0])
    with pytest.raises(hbj.HbjError):
        ctx.set_tuning([-2, 0, 0, 0])


def test_dense_solve_many_rhs(ctxs):
    from oracle import solver

    wl, m, g, dd, ctx = ctxs("grf256", operator_form=1)
    f = np.stack([W.gaussian_source(wl.nx, wl.ny, wl.h, x, 0.3) for x in np.linspace(0.1, 0.9, 6)])
    say("[dense solve nrhs=6]")
    u, st = ctx.solve(torch.as_tensor(f, device="cuda"), tol=1e-12, maxit=3000)
    u = _to_np(u)
    for k in range(6):
        assert rel(u[k], solver.direct(g, f[k])) < 1e-8
