"""Benchmark: Helmholtz solves/s of the block-Jacobi sweeping preconditioner in GMRES.

Workload of the headline (default): 1024 x 1024 interior grid (h = 1/1025), 8 x 8 checkerboard
of 128 x 128 subdomains, 10 points per wavelength (k = 2 pi / (10 h)), smooth seeded random
medium c in [0.8, 1.2], one Gaussian source at (0.5, 0.1); GMRES(50) to relative residual 1e-6
with the block-Jacobi preconditioner, complex128.

A step is one solve(): lifting, GMRES on (I - S) g = b and reconstruction, with every input
already resident in HBM.  Setup and the factorisation are done once before the timed region
(reported separately).

Prints one JSON line.  Besides the contract fields it carries
  roofline      the dominant kernel's algorithmic bytes per launch over its mean launch time
                (HIP events on the solver stream, from a profiled solve right after the timed
                region), against 8 TB/s; traffic = HBM bytes per launch from the committed
                rocprofv3 counter summary (profiles/traffic.json), when it was taken from the
                current source of the kernel;
  cpu_baseline  the CPU oracle (numpy/scipy, one process) timed on a bounded sample: lifting +
                a few GMRES iterations + reconstruction, scaled to one full solve with the GPU's
                iteration count; cpu_baseline_row_owners: the same oracle with one process per
                row of subdomains (the paper's rank layout, Sec. 7);
  legs          the other workloads, each on the GPU: the FP64 solve to 1e-8, the banded local
                solves (subdomain-solve GB/s, FP64 and complex64), mixed precision (complex64
                factors, FGMRES) to 1e-6 and 1e-8 with the error against the FP64 field, the
                second-order transmission, banded solves of 64 right-hand sides, the 2048^2
                64-source block solve (MFMA), and the 512^2 adjoint gradient.
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
# dense matrix-core peaks of MI355X (TFLOP/s) for the contractions of the many-right-hand-side form
MFMA_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="fp64_1024_8x8_grf")
    p.add_argument("--tol", type=float, default=1e-6)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
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
    p.add_argument("--no-multi", action="store_true", help="skip the 2048^2 64-source leg")
    p.add_argument("--orth", choices=("cgs2", "dcgs2", "sstep", "auto"), default=None,
                   help="Gram-Schmidt form of the Arnoldi steps for every context (default: the library's)")
    p.add_argument("--sstep-block", type=int, default=None, help="steps per block of the s-step form (1-8)")
    p.add_argument("--no-gradient", action="store_true", help="skip the 512^2 adjoint-gradient leg")
    p.add_argument("--transmission", type=int, default=1, choices=(1, 2, 3),
                   help="transmission condition of the main run (1: Robin, as the workloads specify; 2: second order; "
                        "3: the paper's Pade condition)")
    p.add_argument("--no-pade", action="store_true", help="skip the run with the paper's Pade transmission")
    p.add_argument("--overlap", action="store_true",
                   help="apply the operator beside the backward pass (hbj_set_operator_overlap; off by default)")
    p.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of each oracle sample")
    p.add_argument("--only", choices=("banded", "multi", "gradient"),
                   help="run one leg alone and print its figures (for profiling runs; no headline line)")
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


# ---------------------------------------------------------------------------
# CPU oracle baselines (run before the GPU is touched: the row-owner processes are forked)
# ---------------------------------------------------------------------------

def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def usable_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _owner_main(conn, grid_args, n1, n2):
    """Row-owner process: keeps the factors of the subdomains it is sent (one row of the
    checkerboard) and runs the oracle's per-subdomain methods on request, on one core."""
    from threadpoolctl import threadpool_limits

    from oracle.dd import Decomposition
    from oracle.fd import Grid

    # after the oracle's imports: numpy and scipy each load their own BLAS, and a limit set
    # before scipy is loaded leaves scipy's thread pool at the machine's width (eight such
    # processes would then oversubscribe every core)
    threadpool_limits(1)
    dd = Decomposition(Grid(*grid_args), n1, n2)
    while True:
        msg = conn.recv()
        if msg is None:
            break
        kind, keys, data = msg
        conn.send(dd._map(kind, keys, data))


class RowOwners:
    """One process per row of subdomains (row i2 -> process (i2 - 1) mod nproc), as the paper
    assigns rows to MPI ranks (Sec. 7); a mapper for oracle.dd.Decomposition.  The processes are
    started fresh (spawn: no BLAS thread pool inherited from this process) and every reply is
    awaited for at most `timeout` seconds."""

    def __init__(self, grid_args, n1, n2, nproc, timeout=120.0):
        import multiprocessing as mp

        ctx = mp.get_context("spawn")
        self.nproc, self.timeout = nproc, timeout
        self.conns, self.procs = [], []
        for _ in range(nproc):
            a, b = ctx.Pipe()
            p = ctx.Process(target=_owner_main, args=(b, grid_args, n1, n2), daemon=True)
            p.start()
            self.conns.append(a)
            self.procs.append(p)

    def __call__(self, kind, keys, data):
        by = {}
        for idx, i in enumerate(keys):
            by.setdefault((i[1] - 1) % self.nproc, []).append((idx, i))
        for o, lst in by.items():
            self.conns[o].send((kind, [i for _, i in lst], data))
        out = [None] * len(keys)
        for o, lst in by.items():
            if not self.conns[o].poll(self.timeout):
                raise TimeoutError(f"row-owner process {o} gave no reply within {self.timeout:.0f} s")
            for (idx, _), r in zip(lst, self.conns[o].recv()):
                out[idx] = r
        return out

    def close(self):
        for c in self.conns:
            try:
                c.send(None)
            except (BrokenPipeError, OSError):
                pass
        for p in self.procs:
            p.join(timeout=10)
            if p.is_alive():
                p.terminate()
                p.join(timeout=5)


def time_oracle(dd, f, target_s):
    """Lifting + reconstruction once, then preconditioned GMRES iterations (one block-Jacobi
    application and one operator application each) until about target_s seconds."""
    import numpy as np

    from oracle import sweep

    t1 = time.perf_counter()
    b = dd.lifting(f)
    u = dd.reconstruct(f, b)  # same cost as the reconstruction of a solve
    t_lr = time.perf_counter() - t1
    log(f"[bench]   oracle lifting + reconstruction {t_lr:.2f} s")
    v = b / np.linalg.norm(b)
    n_it = 0
    t2 = time.perf_counter()
    while True:
        z = sweep.apply_bj(dd, v)
        w = dd.apply_operator(z)
        v = w / np.linalg.norm(w)
        n_it += 1
        el = time.perf_counter() - t2
        log(f"[bench]   oracle iteration {n_it}: {el / n_it:.2f} s each")
        if el * (n_it + 1) / n_it > target_s or n_it >= 50:
            break
    del u
    return t_lr, (time.perf_counter() - t2) / n_it, n_it


def cpu_baselines(wl, m, f, target_s):
    """Per-iteration and lifting+reconstruction costs of the oracle: one process on one core, and
    one process per row of subdomains.  Returns the raw timings; the solves/s figures use the GPU's
    iteration count once it is known.  The row-owner variant is dropped (with a note) if its
    processes fail or stall."""
    from threadpoolctl import threadpool_limits

    from oracle.dd import Decomposition
    from oracle.fd import Grid

    grid_args = (wl.nx, wl.ny, wl.h, wl.k, m)
    out = {}
    with threadpool_limits(1):
        t0 = time.perf_counter()
        dd = Decomposition(Grid(*grid_args), wl.n1, wl.n2)
        for s in dd.sub.values():
            _ = s.lu  # sparse LU of every subdomain (setup, not timed)
        t_factor = time.perf_counter() - t0
        log(f"[bench] CPU oracle, one process: factorisation {t_factor:.1f} s")
        t_lr, t_it, n_it = time_oracle(dd, f, target_s)
        out["single"] = {"t_lr": t_lr, "t_it": t_it, "n_it": n_it, "t_factor": t_factor, "cores": 1}
        del dd
    nproc = min(wl.n2, usable_cores())
    if nproc > 1:
        log(f"[bench] CPU oracle, {nproc} row-owner processes")
        pool = None
        try:
            pool = RowOwners(grid_args, wl.n1, wl.n2, nproc)
            dd = Decomposition(Grid(*grid_args), wl.n1, wl.n2)
            dd.mapper = pool
            t0 = time.perf_counter()
            dd.lifting(f)  # factors every subdomain in its owner (setup, not timed)
            t_factor = time.perf_counter() - t0
            log(f"[bench]   row owners: factorisation and first lifting {t_factor:.1f} s")
            t_lr, t_it, n_it = time_oracle(dd, f, target_s)
            out["rows"] = {"t_lr": t_lr, "t_it": t_it, "n_it": n_it, "t_factor": t_factor, "cores": nproc}
        except Exception as exc:  # a failed baseline must not take the GPU measurement with it
            log(f"[bench]   row-owner baseline dropped: {exc!r}")
            out["rows_error"] = repr(exc)
        finally:
            if pool is not None:
                pool.close()
    return out


def cpu_entry(wl, timing, iters_gpu, kind_note):
    per_solve = timing["t_lr"] + iters_gpu * timing["t_it"]
    return {
        "value": 1.0 / per_solve,
        "unit": "solves/s",
        "cores": timing["cores"],
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "host_cpu_count": os.cpu_count(),
        "host_usable_cores": usable_cores(),
        "sample": (f"{wl.nx}^2 grid, {wl.n1}x{wl.n2} subdomains, {kind_note}: lifting + reconstruction "
                   f"({timing['t_lr']:.2f} s) and {timing['n_it']} preconditioned GMRES iterations "
                   f"({timing['t_it']:.3f} s each, scipy SuperLU local solves); scaled to {iters_gpu} iterations; "
                   f"subdomain factorisation ({timing['t_factor']:.1f} s) excluded as on the GPU"),
    }


# ---------------------------------------------------------------------------
# GPU legs
# ---------------------------------------------------------------------------

OVERLAP = False  # hbj_set_operator_overlap for every context of the run (--overlap sets it)
ORTH = None  # hbj_set_orthogonalization for every context of the run (--orth; None: the library's default)
SSTEP_BLOCK = None  # hbj_set_sstep_block (--sstep-block)


def run_form(hbj, wl, mt, ft, u, precision, operator_form, steps, warmup, tol, profile_names, graphs=False,
             transmission=1, keep=False):
    """Setup + factor (untimed), warmup solves, timed solves, one profiled solve."""
    import torch

    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=mt, precision=precision, precond=hbj.PC_BJ,
                    operator_form=operator_form, transmission=transmission, device=mt.device)
    ctx.set_graphs(graphs)
    ctx.set_operator_overlap(OVERLAP)
    if ORTH is not None:
        ctx.set_orthogonalization(ORTH)
    if SSTEP_BLOCK is not None:
        ctx.set_sstep_block(SSTEP_BLOCK)
    torch.cuda.synchronize()
    # the first factorisation also runs the autotuner of the banded solve batches when the tuning
    # cache has no entry for them yet; the second one is the steady-state figure
    t0 = time.perf_counter()
    ctx.factor()
    torch.cuda.synchronize()
    t_factor_first = time.perf_counter() - t0
    t0 = time.perf_counter()
    ctx.factor()
    torch.cuda.synchronize()
    t_factor = time.perf_counter() - t0
    st = None
    if warmup == 0:
        ctx.solve(ft, tol=tol, maxit=2, out=u, check=False)  # untimed: the autotuner sees every batch class
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
    res = {"seconds": dt, "steps": steps, "factor_s": t_factor, "factor_first_s": t_factor_first, "stats": st,
           "kernels": stats, "tuning": tuning, "solve_tuning": ctx.solve_tuning()}
    if keep:
        res["ctx"] = ctx
    else:
        ctx.close()
    return res


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


def roofline_of(kernels, workload, mfma=None):
    """Roofline of the kernel with the most time. mfma maps kernel symbols that are dense
    contractions (the operator products for many right-hand sides) to their precision: those are
    priced in TFLOP/s against the matrix-core peak, every other kernel in GB/s against HBM."""
    mfma = mfma or {}
    merged = merge_kernels({k: v for k, v in kernels.items() if v["launches"] > 0})
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
    traffic = traffic_from_profiles(name, workload)
    return {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_source": ("profiles/traffic.json: rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE of this kernel on "
                               "this workload, scaled by a copy of known size; taken from the current kernel source")
            if traffic is not None else None,
            "bytes_per_launch": bpl, "avg_launch_ms": avg_ms, "launches": ks["launches"],
            "share_of_kernel_time": share, "launch_kinds": detail}


def factor_seconds(hbj, wl, mt, precision, transmission, multi_solve):
    """Wall time of hbj_factor (band LU, repack, and the dense operators) with the given kind of
    multi-right-hand-side solves."""
    import torch

    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=mt, precision=precision, precond=hbj.PC_BJ,
                    operator_form=hbj.OP_DENSE, transmission=transmission, device=mt.device)
    ctx.set_multi_solve(multi_solve)
    ctx.factor()  # the autotuner's first look at these batches (untimed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.factor()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    return dt


def many_rhs_solves(hbj, wl, mt, nrhs, precision, reps=3):
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
        # every batch on MFMA tiles, or one workgroup per solve at the autotuned prefetch depth
        ctx.set_solve_tuning(hbj.SOLVE_SHAPE_MFMA if mode == hbj.MSOLVE_MFMA else -1)
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


def relerr(a, b):
    import torch

    return float((torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item())


def kernel_names(hbj, many):
    # the banded substitutions run in the autotuned launch shape (the legs report the choices under
    # "solve_tuning"): one workgroup per solve at prefetch depth D, or split over runs of column
    # blocks (two passes and the transfer chain; the class's bytes are still those of one sequential
    # substitution per solve)
    names64 = {hbj.K_FWD: "forward substitution (k_fwd<double,16,4,D> or k_fwd_part+k_part_chain)",
               hbj.K_BWD: "backward substitution (k_bwd<double,16,2,D> or k_bwd_part+k_part_chain)",
               hbj.K_SCATTER: "k_scatter_apply<double2> (sweep steps)",
               hbj.K_OPERATOR: "k_scatter_apply<double2> (operator)",
               hbj.K_SWEEP: "k_sweep_df<double2,16>", hbj.K_LIFT: "k_lift_partial+k_recon_dense",
               hbj.K_KRYLOV: "krylov (Gram-Schmidt kernels of one iteration)"}
    names32 = {hbj.K_FWD: "forward substitution (k_fwd<float,16,4,D> or k_fwd_part+k_part_chain)",
               hbj.K_BWD: "backward substitution (k_bwd<float,16,2,D> or k_bwd_part+k_part_chain)",
               hbj.K_SCATTER: "k_scatter_apply<float2> (sweep steps)",
               hbj.K_OPERATOR: "k_scatter_apply<double2> (operator)",
               hbj.K_SWEEP: "k_sweep_df", hbj.K_LIFT: "k_lift_partial+k_recon_dense",
               hbj.K_KRYLOV: "krylov (Gram-Schmidt kernels of one iteration)"}
    mfma = {}
    if many:
        # from 4 right-hand sides on the operators run as matrix-core products (k_scatter_mm)
        names32[hbj.K_SCATTER] = "k_scatter_mm<float2,float> (sweep steps)"
        names64[hbj.K_SCATTER] = "k_scatter_mm<double2,double> (sweep steps)"
        for nm_ in (names64, names32):
            nm_[hbj.K_OPERATOR] = "k_scatter_mm<double2,double> (operator)"
            nm_[hbj.K_LIFT] = "k_lift_partial+k_recon_mm"
        mfma = {"k_scatter_mm<float2,float>": "f32", "k_scatter_mm<double2,double>": "f64"}
    return names64, names32, mfma


def multi_source_leg(hbj, steps=2, warmup=1):
    """2048^2, 16 x 16 of 128^2, 64 sources: complex64 factors, MFMA operator products, lockstep
    FGMRES to 1e-6 (one block solve of 64 right-hand sides per step)."""
    import torch

    import workload as W

    wl = W.MULTI_2048
    dev = torch.device("cuda:0")
    log(f"[bench] {wl.name}: 64-source block solve")
    mt = torch.as_tensor(W.slowness2(wl), device=dev)
    ft = torch.as_tensor(W.sources(wl), device=dev)
    u = torch.empty_like(ft)
    names64, names32, mfma = kernel_names(hbj, True)
    r = run_form(hbj, wl, mt, ft, u, hbj.MIXED, hbj.OP_DENSE, steps, warmup, 1e-6, names32, keep=True)
    ctx = r.pop("ctx")
    vr = ctx.volume_residual(ft, u)
    ctx.close()
    st = r["stats"]
    kr = r["kernels"][names32[hbj.K_KRYLOV]]
    mm = r["kernels"][names32[hbj.K_SCATTER]]
    out = {
        "workload": wl.name, "sources": 64, "tol": 1e-6,
        "solves_per_s": steps * 64 / r["seconds"], "ms_per_block_solve": r["seconds"] / steps * 1e3,
        "iters": st.iters, "converged": st.converged, "relres": st.relres, "factor_s": r["factor_s"],
        "volume_residual_max": max(vr),
        "roofline": roofline_of(r["kernels"], wl.name, mfma),
        "step_products_f32": {"avg_launch_ms": mm["ms"] / max(1, mm["launches"]),
                              "TFLOP/s": mm["flops"] / max(1e-12, mm["ms"] * 1e-3) / 1e12,
                              "frac_of_f32_mfma_peak": mm["flops"] / max(1e-12, mm["ms"] * 1e-3) / 1e12
                              / MFMA_PEAK_TFLOPS["f32"]},
        "orthogonalization": ({None: "default: s-step cycles (blocks of 8 steps) at this size", 0: "cgs2", 1: "dcgs2",
                               2: "s-step", 3: "auto"}[ORTH] + (f", blocks of {SSTEP_BLOCK}" if SSTEP_BLOCK else "")),
        "gram_schmidt": {"ms_per_iteration": kr["ms"] / max(1, st.iters),
                         "GB/s": kr["bytes"] / max(1e-12, kr["ms"] * 1e-3) / 1e9,
                         "frac_of_hbm_peak": kr["bytes"] / max(1e-12, kr["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "autotuned_operator_tiles": r["tuning"],
    }
    log(f"[bench]   {out['ms_per_block_solve']:.1f} ms per block solve ({out['solves_per_s']:.1f} solves/s), "
        f"iters {st.iters}, step products {out['step_products_f32']['TFLOP/s']:.1f} TFLOP/s, "
        f"Gram-Schmidt {out['gram_schmidt']['GB/s']:.0f} GB/s")
    # the same block solve with the paper's Pade transmission condition (the workload leaves the
    # transmission condition open; the field is the same)
    log(f"[bench] {wl.name}: 64-source block solve with the Pade transmission")
    u0 = u.clone()
    pr = run_form(hbj, wl, mt, ft, u, hbj.MIXED, hbj.OP_DENSE, steps, warmup, 1e-6, names32, transmission=3)
    out["pade_transmission"] = {
        "solves_per_s": steps * 64 / pr["seconds"], "ms_per_block_solve": pr["seconds"] / steps * 1e3,
        "iters": pr["stats"].iters, "converged": pr["stats"].converged, "relres": pr["stats"].relres,
        "factor_s": pr["factor_s"], "rel_diff_vs_robin_field": relerr(u, u0)}
    log(f"[bench]   Pade: {out['pade_transmission']['ms_per_block_solve']:.1f} ms per block solve, "
        f"iters {pr['stats'].iters}, factor {pr['factor_s']:.2f} s")
    del u0
    del ft, u, mt
    torch.cuda.empty_cache()
    return out


def gradient_leg(hbj, reps=2):
    """512^2, 8 x 8 of 64^2, 16 sources: loss and dL/dm by forward + adjoint solves at tol 1e-12.
    The synthetic data d = P u(m_true) come from a GPU solve at tol 1e-12 with the true model."""
    import torch

    import workload as W

    wl = W.GRAD_512
    dev = torch.device("cuda:0")
    log(f"[bench] {wl.name}: adjoint gradient, 16 sources")
    m_true = W.slowness2(wl)
    m0 = W.smoothed_model(m_true, 20.0)
    ft = torch.as_tensor(W.sources(wl), device=dev)
    rec = torch.as_tensor(W.receiver_row(wl), device=dev)
    ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=torch.as_tensor(m_true, device=dev), precond=hbj.PC_BJ,
                    operator_form=hbj.OP_DENSE, device=dev)
    ctx.factor()
    ut, _ = ctx.solve(ft, tol=1e-12, maxit=3000)
    d = ut.reshape(16, -1)[:, rec.long()].contiguous()
    ctx.set_slowness2(torch.as_tensor(m0, device=dev))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.factor()
    torch.cuda.synchronize()
    t_factor = time.perf_counter() - t0
    loss, grad = ctx.gradient(ft, rec, d, tol=1e-12, maxit=3000)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        loss, grad = ctx.gradient(ft, rec, d, tol=1e-12, maxit=3000)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    ctx.close()
    out = {"workload": wl.name, "sources": 16, "receivers": int(rec.numel()), "tol": 1e-12,
           "gradient_s": dt, "solves_per_s": 32 / dt, "factor_s": t_factor, "loss": loss,
           "grad_norm": float(torch.linalg.vector_norm(grad).item())}
    log(f"[bench]   gradient {dt * 1e3:.1f} ms (32 solves at tol 1e-12), loss {loss:.6e}")
    return out


def banded_legs(hbj, wl, mt, ft, u, tol, names64, names32, u_ref, mixed=True):
    """GMRES with a banded local solve per application of every operator (in the autotuned launch
    shape: one workgroup per subdomain solve, or each solve split over runs of column blocks): FP64,
    and complex64 factors with FP64-refined operator solves."""
    out = {}
    log("[bench] FP64, banded local solves inside GMRES")
    br = run_form(hbj, wl, mt, ft, u, hbj.FP64, hbj.OP_BANDED, 1, 0, tol, names64)
    out["banded_fp64"] = {
        "solves_per_s": 1.0 / br["seconds"], "iters": br["stats"].iters, "relres": br["stats"].relres,
        "subdomain_solve_gbs": solve_gbs(br["kernels"], [names64[hbj.K_FWD], names64[hbj.K_BWD]]),
        "roofline": roofline_of(br["kernels"], wl.name + "/banded"), "solve_tuning": br["solve_tuning"]}
    out["banded_fp64"]["subdomain_solve_frac_of_hbm_peak"] = out["banded_fp64"]["subdomain_solve_gbs"] / HBM_PEAK_GBS
    log(f"[bench]   {br['seconds'] * 1e3:.1f} ms per solve, subdomain solves "
        f"{out['banded_fp64']['subdomain_solve_gbs']:.0f} GB/s")
    if mixed:
        mb = run_form(hbj, wl, mt, ft, u, hbj.MIXED, hbj.OP_BANDED, 1, 0, tol, names32)
        out["banded_mixed"] = {
            "solves_per_s": 1.0 / mb["seconds"], "iters": mb["stats"].iters,
            "local_ir_max": mb["stats"].local_ir_max, "local_ir_resid": mb["stats"].local_ir_resid,
            "subdomain_solve_gbs": solve_gbs(mb["kernels"], [names32[hbj.K_FWD], names32[hbj.K_BWD]]),
            "solve_tuning": mb["solve_tuning"]}
        out["banded_mixed"]["subdomain_solve_frac_of_hbm_peak"] = \
            out["banded_mixed"]["subdomain_solve_gbs"] / HBM_PEAK_GBS
        if u_ref is not None:
            out["banded_mixed"]["err_vs_fp64_field"] = relerr(u, u_ref)
        log(f"[bench]   mixed: {mb['seconds'] * 1e3:.1f} ms per solve, subdomain solves "
            f"{out['banded_mixed']['subdomain_solve_gbs']:.0f} GB/s")
    return out


def only_leg(args):
    """One leg alone (profiling runs): its figures as one JSON line."""
    import torch

    import paper_2209_10886_amd as hbj
    import workload as W

    if args.only == "multi":
        print(json.dumps({"leg": "multi_source_2048", **multi_source_leg(hbj)}), flush=True)
        return
    if args.only == "gradient":
        print(json.dumps({"leg": "gradient_512", **gradient_leg(hbj)}), flush=True)
        return
    wl = W.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    mt = torch.as_tensor(W.slowness2(wl), device=dev)
    ft = torch.as_tensor(W.sources(wl)[0], device=dev)
    u = torch.empty_like(ft)
    names64, names32, _ = kernel_names(hbj, False)
    out = banded_legs(hbj, wl, mt, ft, u, args.tol, names64, names32, None, mixed=not args.no_mixed)
    print(json.dumps({"leg": "banded", "workload": wl.name, **out}), flush=True)


def main():
    global OVERLAP, ORTH, SSTEP_BLOCK
    args = parse()
    OVERLAP = args.overlap
    ORTH = {"cgs2": 0, "dcgs2": 1, "sstep": 2, "auto": 3, None: None}[args.orth]  # the library's ORTH_* values
    SSTEP_BLOCK = args.sstep_block
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU form of the sweep is a "
              "design, not a measured configuration", file=sys.stderr)
        sys.exit(2)
    if args.only:
        only_leg(args)
        return
    import workload as W

    wl = W.WORKLOADS[args.workload]
    log(f"[bench] workload {wl.name}: generating medium and sources")
    m = W.slowness2(wl)
    f_all = W.sources(wl)
    nsrc = f_all.shape[0]
    f = f_all[0] if nsrc == 1 else f_all
    cpu = None
    if not args.no_cpu and nsrc == 1:
        cpu = cpu_baselines(wl, m, f, args.cpu_seconds)

    import torch

    import paper_2209_10886_amd as hbj

    dev = torch.device("cuda:0")
    mt = torch.as_tensor(m, device=dev)
    ft = torch.as_tensor(f, device=dev)
    u = torch.empty_like(ft)
    # the multi-source and mixed workloads store the factors in complex64
    headline_prec = hbj.MIXED if wl.name.startswith(("mixed", "multi")) else hbj.FP64
    if nsrc > 1:
        args.no_banded = args.no_mixed = args.no_multi = True
    names64, names32, mfma = kernel_names(hbj, nsrc >= 4)
    names_main = names64 if headline_prec == hbj.FP64 else names32

    log(f"[bench] {'FP64' if headline_prec == hbj.FP64 else 'mixed'}, dense scattering operators (headline), "
        f"{nsrc} right-hand side(s)")
    main_run = run_form(hbj, wl, mt, ft, u, headline_prec, hbj.OP_DENSE, args.steps, args.warmup, args.tol,
                        names_main, graphs=args.graphs, transmission=args.transmission, keep=True)
    ctx_main = main_run.pop("ctx")
    u_main = u.clone()
    st = main_run["stats"]
    ms_per_step = main_run["seconds"] / max(args.steps, 1) * 1e3
    log(f"[bench] {ms_per_step:.2f} ms/solve, iters {st.iters}, relres {st.relres:.2e}, "
        f"factor {main_run['factor_s']:.2f} s")
    roof = roofline_of(main_run["kernels"], wl.name, mfma)
    log(f"[bench] dominant {roof['kernel']}: {roof['avg_launch_ms']:.4f} ms avg, {roof['achieved']:.1f} {roof['unit']}")
    # accuracy of the timed solve: volume residual of the field, and its error against the same
    # solver run to tol 1e-12 (which the parity tests hold within 1e-8 of the direct solution)
    vres = ctx_main.volume_residual(ft, u_main)
    u_ref = None
    if nsrc == 1:
        u_ref, st_ref = ctx_main.solve(ft, tol=1e-12, maxit=3000)
    ctx_main.close()

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
                   "krylov": "FGMRES(50), right-preconditioned, delayed reorthogonalisation",
                   "preconditioner": "block Jacobi, width N1",
                   "operator_form": "dense local scattering operators (formed at factor time)",
                   "operator_overlap": OVERLAP,
                   "transmission": {1: "Robin (first order)", 2: "second order on interface faces",
                                    3: "Pade (8 auxiliary fields, rotation pi/3) on interface faces"}[args.transmission]},
        "iters": st.iters,
        "relres": st.relres,
        "volume_residual": max(vres),
        "steps_per_pc": st.steps_per_pc,
        "factor_s": main_run["factor_s"],
        "roofline": roof,
    }
    if u_ref is not None:
        result["err_vs_tol1e-12_field"] = relerr(u_main, u_ref)
        result["reference_solve_tol1e-12"] = {"iters": st_ref.iters, "relres": st_ref.relres}
    if main_run["tuning"]:
        result["autotuned_operator_tiles"] = main_run["tuning"]
    # launch shapes of the banded solve batches (at factor time: the unit-datum solves that form the
    # dense operators), chosen by the autotuner or read from its cache file
    result["solve_tuning"] = main_run["solve_tuning"]
    result["factor_first_s"] = main_run["factor_first_s"]
    # the dense operators come from one banded solve per interface position (16 per workgroup on
    # MFMA by default); the same factorisation with one workgroup per solve, for comparison
    result["factor_s_one_solve_per_workgroup"] = factor_seconds(hbj, wl, mt, headline_prec, args.transmission,
                                                                hbj.MSOLVE_CHAINS)
    log(f"[bench] factor {main_run['factor_s']:.2f} s; with one workgroup per solve "
        f"{result['factor_s_one_solve_per_workgroup']:.2f} s")

    if not args.no_tight and nsrc == 1 and args.tol > 1e-8:
        # the FP64 workload is also specified to relative residual 1e-8: the same solve to that tolerance
        log("[bench] same solve to relative residual 1e-8")
        tr = run_form(hbj, wl, mt, ft, u, headline_prec, hbj.OP_DENSE, args.steps, 1, 1e-8, names_main,
                      graphs=args.graphs, transmission=args.transmission)
        result["tol_1e-8"] = {"solves_per_s": args.steps / tr["seconds"], "iters": tr["stats"].iters,
                              "relres": tr["stats"].relres,
                              "ms_per_solve": tr["seconds"] / max(args.steps, 1) * 1e3}
        if u_ref is not None:
            result["tol_1e-8"]["err_vs_tol1e-12_field"] = relerr(u, u_ref)
        log(f"[bench] to 1e-8: {result['tol_1e-8']['ms_per_solve']:.2f} ms/solve, iters {tr['stats'].iters}")

    if not args.no_banded:
        result.update(banded_legs(hbj, wl, mt, ft, u, args.tol, names64, names32, u_ref,
                                  mixed=not args.no_mixed))

    if not args.no_mixed:
        log("[bench] mixed precision (complex64 factors and preconditioner operators)")
        mixed = {}
        for tol in (args.tol, 1e-8):
            mr = run_form(hbj, wl, mt, ft, u, hbj.MIXED, hbj.OP_DENSE, args.steps, 1, tol, names32,
                          graphs=args.graphs)
            leg = {"solves_per_s": args.steps / mr["seconds"], "iters": mr["stats"].iters,
                   "relres": mr["stats"].relres, "factor_s": mr["factor_s"]}
            if u_ref is not None:
                leg["err_vs_fp64_field"] = relerr(u, u_ref)
            if tol == args.tol:
                leg["roofline"] = roofline_of(mr["kernels"], wl.name + "/mixed")
            mixed[f"tol_{tol:g}"] = leg
            log(f"[bench] mixed to {tol:g}: {mr['seconds'] / args.steps * 1e3:.2f} ms/solve, iters "
                f"{mr['stats'].iters}, error vs FP64 field {leg.get('err_vs_fp64_field', float('nan')):.2e}")
        result["mixed"] = mixed

    if not args.no_second_order and nsrc == 1 and args.transmission == 1:
        # the workload fixes the Robin transmission condition; the second-order one (interface faces
        # only, same field) is measured beside it
        log("[bench] second-order transmission condition (dense form, same precision)")
        sr = run_form(hbj, wl, mt, ft, u, headline_prec, hbj.OP_DENSE, args.steps, 1, args.tol, names_main,
                      graphs=args.graphs, transmission=2)
        diff = relerr(u, u_main)
        result["second_order_transmission"] = {
            "solves_per_s": args.steps / sr["seconds"], "iters": sr["stats"].iters, "relres": sr["stats"].relres,
            "factor_s": sr["factor_s"], "rel_diff_vs_robin_field": diff}
        log(f"[bench] second order: {sr['seconds'] / args.steps * 1e3:.2f} ms/solve, iters {sr['stats'].iters}, "
            f"field differs from the Robin run by {diff:.1e}")

    if not args.no_pade and nsrc == 1 and args.transmission == 1:
        # the paper's own transmission condition (Sec. 7), same field
        log("[bench] Pade transmission condition (dense form, same precision)")
        pr = run_form(hbj, wl, mt, ft, u, headline_prec, hbj.OP_DENSE, args.steps, 1, args.tol, names_main,
                      graphs=args.graphs, transmission=3)
        diff = relerr(u, u_main)
        result["pade_transmission"] = {
            "solves_per_s": args.steps / pr["seconds"], "iters": pr["stats"].iters, "relres": pr["stats"].relres,
            "factor_s": pr["factor_s"], "rel_diff_vs_robin_field": diff, "n_pade": 8, "phi": "pi/3"}
        log(f"[bench] Pade: {pr['seconds'] / args.steps * 1e3:.2f} ms/solve, iters {pr['stats'].iters}, "
            f"factor {pr['factor_s']:.2f} s, field differs from the Robin run by {diff:.1e}")

    if not args.no_many_rhs and nsrc == 1:
        for prec, key in ((hbj.FP64, "banded_64rhs_fp64"), (hbj.MIXED, "banded_64rhs_mixed")):
            log(f"[bench] banded operator on 64 right-hand sides ({key}): MFMA against one workgroup per solve")
            result[key] = many_rhs_solves(hbj, wl, mt, 64, prec)
            r = result[key]
            log(f"[bench]   MFMA {r['mfma']['ms_per_apply']:.1f} ms ({r['mfma']['TFLOP/s']:.1f} TFLOP/s), "
                f"one per workgroup {r['one_solve_per_workgroup']['ms_per_apply']:.1f} ms")

    del mt, ft, u, u_main, u_ref
    torch.cuda.empty_cache()
    if not args.no_multi:
        result["multi_source_2048"] = multi_source_leg(hbj)
    if not args.no_gradient and nsrc == 1:
        result["gradient_512"] = gradient_leg(hbj)

    if cpu is not None:
        result["cpu_baseline"] = cpu_entry(wl, cpu["single"], st.iters, "one process")
        if "rows" in cpu:
            result["cpu_baseline_row_owners"] = cpu_entry(
                wl, cpu["rows"], st.iters, f"{cpu['rows']['cores']} row-owner processes (the paper's rank layout)")
        elif "rows_error" in cpu:
            result["cpu_baseline_row_owners"] = {"value": None, "error": cpu["rows_error"]}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
