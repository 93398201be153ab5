"""Autotuned launch shapes of the banded local solves and of the dense operator kernel, through the C ABI.

A batch of banded solves runs in one of five shapes: one workgroup per solve at three register prefetch
depths (the same arithmetic in the same order: results bit for bit equal), 16 right-hand sides per
workgroup on MFMA, or each solve split over runs of column blocks (both equal up to rounding). The autotuner times the candidates on the first batch of each
class, keeps the fastest and records it in the tuning cache file; a later context reads the decision back
instead of timing. Every shape is compared with the oracle. The variant of the many-right-hand-side
operator kernel goes to the same cache.
"""
import json
import os

import numpy as np
import pytest

import workload as W
from cases import CASES, gpu_context, oracle_problem, rel, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NRHS = 20


def _np(t):
    return t.detach().cpu().numpy()


def _run(ctx, gt, ft):
    return _np(ctx.apply_operator(gt)), _np(ctx.lifting(ft)), _np(ctx.reconstruct(ft, gt))


def _sources(wl, n):
    xs = np.linspace(0.2, 0.8, n)
    return np.stack([W.gaussian_source(wl.nx, wl.ny, wl.h, x, 0.5 * (wl.ny + 1) * wl.h) for x in xs])


@pytest.mark.parametrize("name,precision", [("ragged", 0), ("pivot", 0), ("grf256", 0), ("grf256", 1)])
def test_every_shape_matches(hbj, name, precision):
    wl = CASES[name].wl
    m, g, dd = oracle_problem(wl)
    ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_BANDED, precision=precision)
    ctx.factor()
    gv = W.random_interface_vector(ctx.nif, seed=41, nrhs=NRHS)
    f = _sources(wl, NRHS)
    gt, ft = torch.as_tensor(gv, device="cuda"), torch.as_tensor(f, device="cuda")
    out = {}
    for shape in range(len(hbj.SOLVE_SHAPES)):
        say(f"[solve shape {shape}] case={name} precision={precision}")
        ctx.set_solve_tuning(shape)
        out[shape] = _run(ctx, gt, ft)
    ctx.set_solve_tuning(-1)
    say(f"[solve shape auto] case={name} precision={precision}")
    auto = _run(ctx, gt, ft)
    tuned = ctx.solve_tuning()
    say(f"  tuned classes: {json.dumps(tuned)}")
    ctx.close()
    assert tuned, "the autotuner made no decision"
    for key, ch in tuned.items():
        assert 0 <= ch["shape"] < len(hbj.SOLVE_SHAPES)
    # one workgroup per solve: the prefetch depth changes nothing
    for shape in (1, 2):
        for a, b in zip(out[0], out[shape]):
            assert np.array_equal(a, b)
    ref = ([dd.apply_operator(gv[k]) for k in range(NRHS)], [dd.lifting(f[k]) for k in range(NRHS)],
           [dd.reconstruct(f[k], gv[k]) for k in range(NRHS)])
    # complex64 factors: the operator is refined to FP64 (1e-10); lifting and reconstruction are not
    tol = (1e-10 if name == "pivot" else 1e-12) if precision == 0 else (1e-10, 1e-4, 1e-4)
    for i, what in enumerate(("operator", "lifting", "reconstruction")):
        t = tol if np.isscalar(tol) else tol[i]
        for shape in (0, 3, 4):
            e = max(rel(out[shape][i][k], ref[i][k]) for k in range(NRHS))
            say(f"  {what}: shape {shape} vs oracle {e:.1e}")
            assert e < t
        # the tuned run equals the shape it picked for this batch class (or another within rounding)
        assert rel(auto[i], out[0][i]) < t


def test_decisions_go_to_the_cache_file_and_are_reused(hbj, tmp_path):
    wl = CASES["ragged"].wl
    m, g, dd = oracle_problem(wl)
    path = tmp_path / "tune.json"
    hbj.set_tune_cache_path(str(path))
    try:
        gv = torch.as_tensor(W.random_interface_vector(dd.nif, seed=42, nrhs=NRHS), device="cuda")
        say("[tuning cache] first context times")
        a = gpu_context(hbj, wl, m, operator_form=hbj.OP_BANDED)
        a.factor()
        wa = _np(a.apply_operator(gv))
        ta = a.solve_tuning()
        a.close()
        assert ta and all(max(ch["us"]) > 0 for ch in ta.values())
        entries = json.loads(path.read_text())["entries"]
        for key, ch in ta.items():
            assert entries[key]["variant"] == ch["shape"]
        say("[tuning cache] second context reads the file")
        hbj.set_tune_cache_path(str(path))  # as a fresh process would: read the file again
        b = gpu_context(hbj, wl, m, operator_form=hbj.OP_BANDED)
        b.factor()
        wb = _np(b.apply_operator(gv))
        tb = b.solve_tuning()
        b.close()
        assert {k: v["shape"] for k, v in tb.items()} == {k: v["shape"] for k, v in ta.items()}
        assert all(max(ch["us"]) == 0 for ch in tb.values())  # nothing timed
        assert np.array_equal(wa, wb)
    finally:
        hbj.set_tune_cache_path(None)


def test_no_timing_without_tuning(hbj, monkeypatch):
    """HBJ_TUNE=0: the batches take MFMA tiles where they average 8 or more right-hand sides per tile."""
    wl = CASES["rect"].wl
    m, g, dd = oracle_problem(wl)
    monkeypatch.setenv("HBJ_TUNE", "0")
    hbj.set_tune_cache_path("")
    try:
        ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_BANDED)
        ctx.factor()
        gv = W.random_interface_vector(ctx.nif, seed=43, nrhs=NRHS)
        say("[no tuning] rect")
        w = _np(ctx.apply_operator(torch.as_tensor(gv, device="cuda")))
        t = ctx.solve_tuning()
        ctx.close()
    finally:
        hbj.set_tune_cache_path(None)
    assert t
    for key, ch in t.items():
        assert max(ch["us"]) == 0
        per = int(key.split("|r")[1].split("|")[0])
        assert ch["shape"] == (3 if "|mm|" in key and per >= 8 else 0)
    e = max(rel(w[k], dd.apply_operator(gv[k])) for k in range(NRHS))
    assert e < 1e-12


def test_bad_shape(hbj):
    wl = W.SMALL
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=torch.as_tensor(W.slowness2(wl), device="cuda"))
    for bad in (-2, len(hbj.SOLVE_SHAPES)):
        with pytest.raises(hbj.HbjError) as ei:
            ctx.set_solve_tuning(bad)
        assert ei.value.code == hbj.EINVAL
    ctx.close()


def _dense_run(hbj, wl, m, gv, precision):
    ctx = gpu_context(hbj, wl, m, operator_form=hbj.OP_DENSE, precision=precision)
    ctx.factor()
    w = _np(ctx.apply_operator(gv))
    z = _np(ctx.apply_preconditioner(gv))
    t = ctx.tuning()
    ctx.close()
    return w, z, t


@pytest.mark.parametrize("precision", [0, 1])
def test_operator_kernel_choice_is_cached(hbj, tmp_path, precision):
    """A first context times the variants of the dense operator kernel and stores its choices; a second
    context reads them back (no timing) and gives the same results bit for bit."""
    wl = CASES["ragged"].wl
    m, g, dd = oracle_problem(wl)
    path = tmp_path / "tune.json"
    used = [("c64" if precision else "c128") + " steps", "c128 operator"]
    hbj.set_tune_cache_path(str(path))
    try:
        gv = torch.as_tensor(W.random_interface_vector(dd.nif, seed=44, nrhs=NRHS), device="cuda")
        say(f"[operator kernel cache] first context times, precision={precision}")
        wa, za, ta = _dense_run(hbj, wl, m, gv, precision)
        for k in used:
            assert ta[k]["us"] is not None and all(v > 0 for v in ta[k]["us"].values())
        entries = json.loads(path.read_text())["entries"]
        mm = {k: v for k, v in entries.items() if k.startswith("mm|")}
        assert len(mm) == 2
        for key, e in mm.items():
            assert 0 <= e["variant"] < hbj.MM_VARIANTS
            assert len(e["us"]) == hbj.MM_VARIANTS
        say("[operator kernel cache] second context reads the file")
        hbj.set_tune_cache_path(str(path))
        wb, zb, tb = _dense_run(hbj, wl, m, gv, precision)
        for k in used:
            assert {q: tb[k][q] for q in ("incoming", "k_steps_per_batch", "ring", "wave_groups", "k_waves")} == \
                {q: ta[k][q] for q in ("incoming", "k_steps_per_batch", "ring", "wave_groups", "k_waves")}
            assert all(v == 0 for v in tb[k]["us"].values())
        assert np.array_equal(wa, wb)
        assert np.array_equal(za, zb)
        e = max(rel(wa[k], dd.apply_operator(_np(gv)[k])) for k in range(NRHS))
        assert e < 1e-12
    finally:
        hbj.set_tune_cache_path(None)


def test_operator_kernel_untimed_default(hbj, monkeypatch):
    """HBJ_TUNE=0 and no cache: the operator kernel takes variant 15 for sweep steps, 7 for the operator."""
    wl = CASES["ragged"].wl
    m, g, dd = oracle_problem(wl)
    monkeypatch.setenv("HBJ_TUNE", "0")
    hbj.set_tune_cache_path("")
    try:
        gv = W.random_interface_vector(dd.nif, seed=45, nrhs=NRHS)
        say("[operator kernel untimed] ragged")
        w, z, t = _dense_run(hbj, wl, m, torch.as_tensor(gv, device="cuda"), 0)
    finally:
        hbj.set_tune_cache_path(None)
    assert t["c128 steps"] == dict(hbj.mm_variant_fields(15), us=t["c128 steps"]["us"])
    assert t["c128 operator"] == dict(hbj.mm_variant_fields(7), us=t["c128 operator"]["us"])
    for k in ("c128 steps", "c128 operator"):
        assert all(v == 0 for v in t[k]["us"].values())
    assert max(rel(w[k], dd.apply_operator(gv[k])) for k in range(NRHS)) < 1e-12
