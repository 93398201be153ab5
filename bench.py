"""Benchmark: Helmholtz solves/s of the block-Jacobi sweeping preconditioner in GMRES.

Workload (default): 1024 x 1024 interior grid (h = 1/1025), 8 x 8 checkerboard of
128 x 128 subdomains, 10 points per wavelength (k = 2 pi / (10 h)), smooth seeded
random medium c in [0.8, 1.2], one Gaussian source at (0.5, 0.1); GMRES(50) to
relative residual 1e-6 with the block-Jacobi preconditioner, complex128.

A step is one solve(): lifting, GMRES on (I - S) g = b and reconstruction, with
every input already resident in HBM.  Setup and the factorisation are done once
before the timed region (reported separately).

Prints one JSON line.  Besides the contract fields it carries
  roofline      the dominant kernel's algorithmic bytes per launch over its mean
                launch time (HIP events on the solver stream, profiled solve after
                the timed region), against 8 TB/s; for many right-hand sides, where
                the operators are matrix-core products, their flops per launch
                against the FP32 / FP64 matrix peak;
  cpu_baseline  the CPU oracle (numpy/scipy, one core) timed on a bounded sample:
                lifting + a few GMRES iterations + reconstruction, scaled to one
                full solve with the GPU's iteration count;
  mixed         the same problem with complex64 factors (FGMRES, refined operator).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="fp64_1024_8x8_grf")
    p.add_argument("--tol", type=float, default=1e-6)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison")
    p.add_argument("--no-banded", action="store_true", help="skip the banded-operator comparison")
    p.add_argument("--graphs", action="store_true", help="replay the GMRES iterations as HIP graphs")
    p.add_argument("--no-many-rhs", action="store_true",
                   help="skip the banded solves of many right-hand sides per subdomain (MFMA against one "
                        "workgroup per solve)")
    p.add_argument("--no-tight", action="store_true",
                   help="skip the run of the same solve to relative residual 1e-8")
    p.add_argument("--no-second-order", action="store_true",
                   help="skip the run with the second-order transmission condition")
    p.add_argument("--transmission", type=int, default=1, choices=(1, 2),
                   help="transmission condition of the main run (1: Robin, as the workloads specify; 2: second order)")
    p.add_argument("--cpu-seconds", type=float, default=20.0, help="target CPU time of the oracle sample")
    return p.parse_args()


def traffic_from_profiles(kernel_symbol, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary (FETCH_SIZE and
    WRITE_SIZE, scaled by a copy of known size), if it was taken on this workload from the
    current source of the kernel; None otherwise."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        ent = json.load(open(path)).get(f"{workload}/{kernel_symbol}")
        if not ent:
            return None
        src = os.path.join(ROOT, "paper_2209_10886_amd", "csrc", ent["source"])
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        if ent.get("source_sha") != sha:
            return None
        return ent["bytes_per_launch"]
    except Exception:
        return None


def cpu_baseline(wl, m, f, iters_gpu, target_s):
    """Time the oracle on a bounded sample and scale to one solve (single core)."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import numpy as np

    from oracle import sweep
    from oracle.dd import Decomposition
    from oracle.fd import Grid

    t0 = time.perf_counter()
    dd = Decomposition(Grid(wl.nx, wl.ny, wl.h, wl.k, m), wl.n1, wl.n2)
    for s in dd.sub.values():
        _ = s.lu  # sparse LU of every subdomain (setup, not timed)
    t_factor = time.perf_counter() - t0
    t1 = time.perf_counter()
    b = dd.lifting(f)
    u = dd.reconstruct(f, b)  # same cost as the reconstruction of a solve
    t_lr = time.perf_counter() - t1
    # GMRES iterations: one preconditioner application + one operator application each
    v = b / np.linalg.norm(b)
    n_it = 0
    t2 = time.perf_counter()
    while True:
        z = sweep.apply_bj(dd, v)
        w = dd.apply_operator(z)
        v = w / np.linalg.norm(w)
        n_it += 1
        el = time.perf_counter() - t2
        if el * (n_it + 1) / n_it > target_s or n_it >= 50:
            break
    t_it = (time.perf_counter() - t2) / n_it
    per_solve = t_lr + iters_gpu * t_it
    del u
    return {
        "value": 1.0 / per_solve,
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{wl.nx}^2 grid, {wl.n1}x{wl.n2} subdomains: lifting + reconstruction ({t_lr:.2f} s) and "
                   f"{n_it} preconditioned GMRES iterations ({t_it:.2f} s each, scipy SuperLU local solves); "
                   f"scaled to {iters_gpu} iterations; subdomain factorisation ({t_factor:.1f} s) excluded as on the GPU"),
    }


def run_form(hbj, wl, mt, ft, u, precision, operator_form, steps, warmup, tol, profile_names, graphs=False,
             transmission=1):
    """Setup + factor (untimed), warmup solves, timed solves, one profiled solve."""
    import torch

    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=mt, precision=precision, precond=hbj.PC_BJ,
                    operator_form=operator_form, transmission=transmission, device=mt.device)
    ctx.set_graphs(graphs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.factor()
    torch.cuda.synchronize()
    t_factor = time.perf_counter() - t0
    st = None
    for _ in range(warmup):
        _, st = ctx.solve(ft, tol=tol, out=u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, st = ctx.solve(ft, tol=tol, out=u)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.reset_kernel_stats()
    ctx.set_profiling(True)
    ctx.solve(ft, tol=tol, out=u)
    ctx.set_profiling(False)
    stats = {name: ctx.kernel_stats(kc) for kc, name in profile_names.items()}
    tuning = {k: v for k, v in ctx.tuning().items() if v["k_steps_per_batch"] is not None}
    ctx.close()
    return {"seconds": dt, "steps": steps, "factor_s": t_factor, "stats": st, "kernels": stats, "tuning": tuning}


def merge_kernels(kernels):
    """Classes that time the same kernel symbol are merged (its launches, time and bytes)."""
    out = {}
    for name, ks in kernels.items():
        sym = name.split(" (")[0]
        m = out.setdefault(sym, {"launches": 0, "ms": 0.0, "bytes": 0.0, "flops": 0.0, "classes": []})
        for k in ("launches", "ms", "bytes", "flops"):
            m[k] += ks[k]
        m["classes"].append(name)
    return out


# dense matrix-core peaks of MI355X (TFLOP/s) for the contractions of the many-right-hand-side form
MFMA_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}


def roofline_of(kernels, workload, mfma=None):
    """Roofline of the kernel with the most time. mfma maps kernel symbols that are dense
    contractions (the operator products for many right-hand sides) to their precision: those are
    priced in TFLOP/s against the matrix-core peak, every other kernel in GB/s against HBM."""
    mfma = mfma or {}
    merged = merge_kernels(kernels)
    name, ks = max(merged.items(), key=lambda kv: kv[1]["ms"])
    avg_ms = ks["ms"] / ks["launches"]
    bpl = ks["bytes"] / ks["launches"]
    fpl = ks["flops"] / ks["launches"]
    detail = {c: {"launches": kernels[c]["launches"], "avg_launch_ms": kernels[c]["ms"] / max(1, kernels[c]["launches"]),
                  "bytes_per_launch": kernels[c]["bytes"] / max(1, kernels[c]["launches"]),
                  "GB/s": kernels[c]["bytes"] / max(1e-12, kernels[c]["ms"] * 1e-3) / 1e9,
                  "TFLOP/s": kernels[c]["flops"] / max(1e-12, kernels[c]["ms"] * 1e-3) / 1e12}
              for c in ks["classes"]}
    share = ks["ms"] / max(1e-12, sum(k["ms"] for k in kernels.values()))
    if name in mfma:
        peak = MFMA_PEAK_TFLOPS[mfma[name]]
        achieved = fpl / (avg_ms * 1e-3) / 1e12
        return {"bound": "mfma", "kernel": name, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": None, "flops_per_launch": fpl, "bytes_per_launch": bpl,
                "avg_launch_ms": avg_ms, "launches": ks["launches"], "share_of_kernel_time": share,
                "launch_kinds": detail}
    achieved = bpl / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_from_profiles(name, workload),
            "bytes_per_launch": bpl, "avg_launch_ms": avg_ms, "launches": ks["launches"],
            "share_of_kernel_time": share, "launch_kinds": detail}


def factor_seconds(hbj, wl, mt, precision, transmission, multi_solve):
    """Wall time of hbj_factor (band LU, repack, and the dense operators) with the given kind of
    multi-right-hand-side solves."""
    import torch

    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=mt, precision=precision, precond=hbj.PC_BJ,
                    operator_form=hbj.OP_DENSE, transmission=transmission, device=mt.device)
    ctx.set_multi_solve(multi_solve)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.factor()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    return dt


def many_rhs_solves(hbj, wl, mt, nrhs, precision, names, reps=3):
    """The banded operator (one local solve per subdomain and right-hand side) on nrhs columns:
    16 right-hand sides per workgroup on MFMA against one workgroup per solve."""
    import torch

    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=mt, precision=precision, precond=hbj.PC_BJ,
                    operator_form=hbj.OP_BANDED, device=mt.device)
    ctx.factor()
    gen = torch.Generator(device=mt.device).manual_seed(5)
    g = torch.randn(nrhs, ctx.nif, dtype=torch.complex128, device=mt.device, generator=gen)
    out = {}
    peak = MFMA_PEAK_TFLOPS["f64" if precision == hbj.FP64 else "f32"]
    for mode, key in ((hbj.MSOLVE_MFMA, "mfma"), (hbj.MSOLVE_CHAINS, "one_solve_per_workgroup")):
        ctx.set_multi_solve(mode)
        w = ctx.apply_operator(g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.apply_operator(g, out=w)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        ctx.reset_kernel_stats()
        ctx.set_profiling(True)
        ctx.apply_operator(g, out=w)
        ctx.set_profiling(False)
        ks = [ctx.kernel_stats(k) for k in (hbj.K_FWD, hbj.K_BWD)]
        ms = sum(k["ms"] for k in ks)
        fl = sum(k["flops"] for k in ks)
        by = sum(k["bytes"] for k in ks)
        tf = fl / (ms * 1e-3) / 1e12
        out[key] = {"ms_per_apply": dt * 1e3, "local_solves_per_s": ctx.ndom * nrhs / dt,
                    "solve_kernels_ms": ms, "TFLOP/s": tf, "frac_of_mfma_peak": tf / peak,
                    "factor_GB/s": by / (ms * 1e-3) / 1e9}
    ctx.close()
    out["right_hand_sides"] = nrhs
    out["peak_TFLOP/s"] = peak
    return out


def solve_gbs(kernels, names):
    b = sum(kernels[n]["bytes"] for n in names)
    t = sum(kernels[n]["ms"] for n in names)
    return b / (t * 1e-3) / 1e9 if t > 0 else None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU form of the sweep is a "
              "design, not a measured configuration", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2209_10886_amd as hbj
    import workload as W

    wl = W.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    log(f"[bench] workload {wl.name}: generating medium and sources")
    m = W.slowness2(wl)
    f_all = W.sources(wl)
    nsrc = f_all.shape[0]
    f = f_all[0] if nsrc == 1 else f_all
    mt = torch.as_tensor(m, device=dev)
    ft = torch.as_tensor(f, device=dev)
    u = torch.empty_like(ft)
    # the multi-source and mixed workloads store the factors in complex64
    headline_prec = hbj.MIXED if wl.name.startswith(("mixed", "multi")) else hbj.FP64
    if nsrc > 1:
        args.no_banded = True
        args.no_cpu = args.no_cpu or nsrc > 1
        args.no_mixed = True
    names64 = {hbj.K_FWD: "k_fwd<double,16,4,5>", hbj.K_BWD: "k_bwd<double,16,2,3>",
               hbj.K_SCATTER: "k_scatter_apply<double2,16> (sweep steps)",
               hbj.K_OPERATOR: "k_scatter_apply<double2,16> (operator)",
               hbj.K_SWEEP: "k_sweep_df<double2,16>", hbj.K_LIFT: "k_lift_partial+k_recon_dense",
               hbj.K_KRYLOV: "krylov (Gram-Schmidt kernels of one iteration)"}
    names32 = {hbj.K_FWD: "k_fwd<float,16,4,8>", hbj.K_BWD: "k_bwd<float,16,2,4>",
               hbj.K_SCATTER: "k_scatter_apply<float2,16> (sweep steps)",
               hbj.K_OPERATOR: "k_scatter_apply<double2,16> (operator)",
               hbj.K_SWEEP: "k_sweep_df", hbj.K_LIFT: "k_lift_partial+k_recon_dense",
               hbj.K_KRYLOV: "krylov (Gram-Schmidt kernels of one iteration)"}
    mfma = {}
    if nsrc >= 4:
        # from 4 right-hand sides on the operators run as matrix-core products (k_scatter_mm)
        for nm_ in (names64, names32):
            nm_[hbj.K_SCATTER] = ("k_scatter_mm<float2,float> (sweep steps)" if nm_ is names32
                                  else "k_scatter_mm<double2,double> (sweep steps)")
            nm_[hbj.K_OPERATOR] = "k_scatter_mm<double2,double> (operator)"
            nm_[hbj.K_LIFT] = "k_lift_partial+k_recon_mm"
        mfma = {"k_scatter_mm<float2,float>": "f32", "k_scatter_mm<double2,double>": "f64"}

    log(f"[bench] {'FP64' if headline_prec == hbj.FP64 else 'mixed'}, dense scattering operators (headline), "
        f"{nsrc} right-hand side(s)")
    main_run = run_form(hbj, wl, mt, ft, u, headline_prec, hbj.OP_DENSE, args.steps, args.warmup, args.tol,
                        names64 if headline_prec == hbj.FP64 else names32, graphs=args.graphs,
                        transmission=args.transmission)
    u_main = u.clone()
    st = main_run["stats"]
    ms_per_step = main_run["seconds"] / max(args.steps, 1) * 1e3
    log(f"[bench] {ms_per_step:.2f} ms/solve, iters {st.iters}, relres {st.relres:.2e}, "
        f"factor {main_run['factor_s']:.2f} s")
    roof = roofline_of(main_run["kernels"], wl.name, mfma)
    log(f"[bench] dominant {roof['kernel']}: {roof['avg_launch_ms']:.4f} ms avg, {roof['achieved']:.1f} {roof['unit']}")

    result = {
        "metric": "Helmholtz solves/s at rel-res 1e-6; subdomain-solve HBM GB/s (FP64 vs mixed)",
        "value": args.steps * nsrc / main_run["seconds"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if headline_prec == hbj.FP64 else "c64 factors, c128 Krylov",
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": [wl.nx, wl.ny], "decomposition": [wl.n1, wl.n2],
                   "subdomain": [wl.sub_nx, wl.sub_ny], "points_per_wavelength": wl.ppw, "k": wl.k,
                   "medium": wl.medium, "sources": nsrc, "tol": args.tol,
                   "krylov": "GMRES(50), right-preconditioned, delayed reorthogonalisation", "preconditioner": "block Jacobi, width N1",
                   "operator_form": "dense local scattering operators (formed at factor time)",
                   "transmission": "Robin (first order)" if args.transmission == 1 else
                   "second order on interface faces"},
        "iters": st.iters,
        "relres": st.relres,
        "steps_per_pc": st.steps_per_pc,
        "factor_s": main_run["factor_s"],
        "subdomain_solve_gbs": solve_gbs(main_run["kernels"], [names64[hbj.K_FWD], names64[hbj.K_BWD]])
        if headline_prec == hbj.FP64 else None,
        "roofline": roof,
    }
    if main_run["tuning"]:
        result["autotuned_operator_tiles"] = main_run["tuning"]
    # the dense operators come from one banded solve per interface position (16 per workgroup on
    # MFMA by default); the same factorisation with one workgroup per solve, for comparison
    result["factor_s_one_solve_per_workgroup"] = factor_seconds(hbj, wl, mt, headline_prec, args.transmission,
                                                                hbj.MSOLVE_CHAINS)
    log(f"[bench] factor {main_run['factor_s']:.2f} s; with one workgroup per solve "
        f"{result['factor_s_one_solve_per_workgroup']:.2f} s")

    if not args.no_tight and nsrc == 1 and args.tol > 1e-8:
        # the FP64 workload is also specified to relative residual 1e-8: the same solve to that tolerance
        log("[bench] same solve to relative residual 1e-8")
        tr = run_form(hbj, wl, mt, ft, u, headline_prec, hbj.OP_DENSE, args.steps, 1, 1e-8,
                      names64 if headline_prec == hbj.FP64 else names32, graphs=args.graphs,
                      transmission=args.transmission)
        result["tol_1e-8"] = {"solves_per_s": args.steps / tr["seconds"], "iters": tr["stats"].iters,
                              "relres": tr["stats"].relres,
                              "ms_per_solve": tr["seconds"] / max(args.steps, 1) * 1e3}
        log(f"[bench] to 1e-8: {result['tol_1e-8']['ms_per_solve']:.2f} ms/solve, iters {tr['stats'].iters}")

    if not args.no_banded:
        log("[bench] FP64, banded local solves inside GMRES")
        br = run_form(hbj, wl, mt, ft, u, hbj.FP64, hbj.OP_BANDED, 1, 0, args.tol, names64)
        result["banded_fp64"] = {
            "solves_per_s": 1.0 / br["seconds"], "iters": br["stats"].iters, "relres": br["stats"].relres,
            "subdomain_solve_gbs": solve_gbs(br["kernels"], [names64[hbj.K_FWD], names64[hbj.K_BWD]]),
            "roofline": roofline_of(br["kernels"], wl.name + "/banded")}

    if not args.no_mixed:
        log("[bench] mixed precision (complex64 factors and preconditioner operators)")
        mr = run_form(hbj, wl, mt, ft, u, hbj.MIXED, hbj.OP_DENSE, args.steps, 1, args.tol, names32,
                      graphs=args.graphs)
        result["mixed"] = {"solves_per_s": args.steps / mr["seconds"], "iters": mr["stats"].iters,
                           "relres": mr["stats"].relres, "factor_s": mr["factor_s"],
                           "roofline": roofline_of(mr["kernels"], wl.name + "/mixed")}
        if not args.no_banded:
            mb = run_form(hbj, wl, mt, ft, u, hbj.MIXED, hbj.OP_BANDED, 1, 0, args.tol, names32)
            result["banded_mixed"] = {
                "solves_per_s": 1.0 / mb["seconds"], "iters": mb["stats"].iters,
                "subdomain_solve_gbs": solve_gbs(mb["kernels"], [names32[hbj.K_FWD], names32[hbj.K_BWD]])}

    if not args.no_second_order and nsrc == 1 and args.transmission == 1:
        # the workload fixes the Robin transmission condition; the second-order one (interface faces
        # only, same field) is measured beside it
        log("[bench] second-order transmission condition (dense form, same precision)")
        u1 = u_main
        sr = run_form(hbj, wl, mt, ft, u, headline_prec, hbj.OP_DENSE, args.steps, 1, args.tol,
                      names64 if headline_prec == hbj.FP64 else names32, graphs=args.graphs, transmission=2)
        diff = float((torch.linalg.vector_norm(u - u1) / torch.linalg.vector_norm(u1)).item())
        result["second_order_transmission"] = {
            "solves_per_s": args.steps / sr["seconds"], "iters": sr["stats"].iters, "relres": sr["stats"].relres,
            "factor_s": sr["factor_s"], "rel_diff_vs_robin_field": diff}
        log(f"[bench] second order: {sr['seconds'] / args.steps * 1e3:.2f} ms/solve, iters {sr['stats'].iters}, "
            f"field differs from the Robin run by {diff:.1e}")

    if not args.no_many_rhs and nsrc == 1:
        for prec, key, nm in ((hbj.FP64, "banded_64rhs_fp64", names64), (hbj.MIXED, "banded_64rhs_mixed", names32)):
            log(f"[bench] banded operator on 64 right-hand sides ({key}): MFMA against one workgroup per solve")
            result[key] = many_rhs_solves(hbj, wl, mt, 64, prec, nm)
            r = result[key]
            log(f"[bench]   MFMA {r['mfma']['ms_per_apply']:.1f} ms ({r['mfma']['TFLOP/s']:.1f} TFLOP/s), "
                f"one per workgroup {r['one_solve_per_workgroup']['ms_per_apply']:.1f} ms")

    if not args.no_cpu:
        log("[bench] CPU oracle sample")
        result["cpu_baseline"] = cpu_baseline(wl, m, f, st.iters, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
