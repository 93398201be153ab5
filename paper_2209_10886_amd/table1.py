"""SGS full sweeps versus block-Jacobi partial sweeps on long checkerboards.

The paper's comparison (Sec. 7, Table 1): iterations ("ni"), sequential steps per
preconditioner application ("ns") and GMRES time ("t") for the full sweeping
preconditioner (SP) and the block-Jacobi sweeping preconditioner (BSP) on N1 x N2 =
5 x 5, 5 x 10, 5 x 15, 5 x 20 checkerboards, GMRES to relative residual 1e-6.

Here every subdomain is 128 x 128 grid points, the medium is the seeded smooth random
field used by the 1024^2 workload, 10 points per wavelength, one Gaussian source at
(0.5, 0.1 of the height).  Times are MI355X wall times of hbj_solve (lifting + GMRES +
reconstruction) with the dense scattering operators, after one warmup solve.

    python -m paper_2209_10886_amd.table1 [--sub 128] [--out profiles/table1_sp_vs_bsp.md]
    python -m paper_2209_10886_amd.table1 --ablation fp64_1024_8x8_grf --out profiles/ablation_readings_1024_8x8.md
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time


def run(sub=128, layouts=((5, 5), (5, 10), (5, 15), (5, 20)), tol=1e-6, ppw=10.0, reps=2):
    import torch

    import paper_2209_10886_amd as hbj
    import workload as W

    rows = []
    for n1, n2 in layouts:
        nx, ny = n1 * sub, n2 * sub
        wl = W.Workload(f"strip_{n1}x{n2}", nx, ny, n1, n2, ppw, "random_smooth", 0, ((0.5, 0.1 * (ny + 1) / (nx + 1)),))
        m = torch.as_tensor(W.slowness2(wl), device="cuda")
        f = torch.as_tensor(W.sources(wl)[0], device="cuda")
        for name, pc in (("SP", hbj.PC_SGS), ("BSP", hbj.PC_BJ)):
            ctx = hbj.setup(nx, ny, wl.k, n1, n2, m=m, precond=pc, operator_form=hbj.OP_DENSE)
            ctx.factor()
            u, st = ctx.solve(f, tol=tol, maxit=2000)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                u, st = ctx.solve(f, tol=tol, maxit=2000, out=u)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            rows.append({"layout": f"{n1}x{n2}", "grid": [nx, ny], "preconditioner": name, "ni": st.iters,
                         "ns": st.steps_per_pc, "t_ms": dt * 1e3, "relres": st.relres})
            print(json.dumps(rows[-1]), flush=True)
            ctx.close()
    return rows


def ablation(wl_name="fp64_1024_8x8_grf", tol=1e-6, reps=3):
    """Readings of Sec. 6 that the paper leaves open, on one workload: interval width (number of
    partial sweeps), the combination at shared groups, the composition of the two passes."""
    import torch

    import paper_2209_10886_amd as hbj
    import workload as W

    wl = W.WORKLOADS[wl_name]
    m = torch.as_tensor(W.slowness2(wl), device="cuda")
    f = torch.as_tensor(W.sources(wl)[0], device="cuda")
    ng = wl.n1 + wl.n2 - 1
    variants = [("SGS (one interval)", dict(precond=hbj.PC_SGS))]
    for w in sorted({1, 2, 4, wl.n1, ng - 2}):
        if 1 <= w < ng - 1:
            variants.append((f"BJ width {w}", dict(precond=hbj.PC_BJ, bj_width=w)))
    variants += [(f"BJ width {wl.n1}, additive", dict(precond=hbj.PC_BJ, bj_combine=hbj.BJ_ADDITIVE)),
                 (f"BJ width {wl.n1}, residual", dict(precond=hbj.PC_BJ, bj_compose=hbj.BJ_RESIDUAL)),
                 (f"BJ width {wl.n1}, additive + residual",
                  dict(precond=hbj.PC_BJ, bj_combine=hbj.BJ_ADDITIVE, bj_compose=hbj.BJ_RESIDUAL)),
                 ("none", dict(precond=hbj.PC_NONE))]
    rows = []
    for name, kw in variants:
        ctx = hbj.setup(wl.nx, wl.ny, wl.k, wl.n1, wl.n2, m=m, operator_form=hbj.OP_DENSE, **kw)
        ctx.factor()
        u, st = ctx.solve(f, tol=tol, maxit=3000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            u, st = ctx.solve(f, tol=tol, maxit=3000, out=u)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        rows.append({"variant": name, "ni": st.iters, "ns": st.steps_per_pc, "t_ms": dt * 1e3,
                     "relres": st.relres, "converged": st.converged})
        print(json.dumps(rows[-1]), flush=True)
        ctx.close()
    return wl, rows


def ablation_markdown(wl, rows, tol=1e-6):
    out = [f"# Readings of Sec. 6: interval width, shared-group combination, composition ({wl.name})", "",
           f"{wl.nx}^2 grid, {wl.n1} x {wl.n2} subdomains, one Gaussian source, GMRES(50) to relative residual "
           f"{tol:g}, dense scattering operators, MI355X wall time per solve. ns = sequential sweep steps per "
           "preconditioner application.", "",
           "| variant | ni | ns | ni x ns | t (ms) |", "|---|---|---|---|---|"]
    for r in rows:
        conv = "" if r["converged"] else " (not converged)"
        out.append(f"| {r['variant']} | {r['ni']}{conv} | {r['ns']} | {r['ni'] * r['ns']} | {r['t_ms']:.2f} |")
    return "\n".join(out) + "\n"


def markdown(rows, sub):
    out = ["# SP versus BSP on long checkerboards (the layout of Table 1)", "",
           f"Subdomains of {sub}^2 grid points, 10 points per wavelength, seeded smooth random medium, one Gaussian",
           "source; GMRES(50) to relative residual 1e-6; dense scattering operators; MI355X wall time per solve.",
           "ns is the number of sequential sweep steps per preconditioner application (paper: SP 16/26/36/46,",
           "BSP 10). Iteration counts differ from the paper's (first-order Robin transmission on finite",
           "differences instead of the Pade high-order condition on P7 elements).", "",
           "| N1 x N2 | SP ni | SP ns | SP t (ms) | BSP ni | BSP ns | BSP t (ms) |", "|---|---|---|---|---|---|---|"]
    by = {}
    for r in rows:
        by.setdefault(r["layout"], {})[r["preconditioner"]] = r
    ratios = []
    for lay, d in by.items():
        sp, bsp = d["SP"], d["BSP"]
        out.append(f"| {lay} | {sp['ni']} | {sp['ns']} | {sp['t_ms']:.2f} | {bsp['ni']} | {bsp['ns']} | "
                   f"{bsp['t_ms']:.2f} |")
        ratios.append(sp["t_ms"] / bsp["t_ms"])
    out += ["", "Command (MI355X, repository root): `python -u -m paper_2209_10886_amd.table1 --out "
            "profiles/table1_sp_vs_bsp.md`.", "",
            "SP/BSP time ratios: " + ", ".join(f"{x:.2f}" for x in ratios) + " for the layouts above. The paper's MPI "
            "timings on one multi-core CPU give 1.28, 1.48, 1.77, 2.08. On the GPU one sweep step is a single launch of "
            "a few microseconds, so the step count weighs less than when a step means MPI exchanges between row ranks. "
            "The growth with N2 is the same: SP needs 2(N1 + N2 - 2) steps, BSP 2 N1."]
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sub", type=int, default=128)
    ap.add_argument("--out", default=None)
    ap.add_argument("--ablation", default=None, help="workload name: sweep the readings of Sec. 6 instead")
    a = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    if a.ablation:
        wl, rows = ablation(a.ablation)
        md = ablation_markdown(wl, rows)
    else:
        rows = run(a.sub)
        md = markdown(rows, a.sub)
    print(md)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(md)


if __name__ == "__main__":
    main()
