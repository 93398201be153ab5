"""Write grad_512_fd.json: central differences of the oracle's direct-solve misfit for the
adjoint-gradient workload (512^2 grid, 8 x 8 subdomains of 64^2, 10 points per wavelength, 16
sources along y = 0.05, receivers on the row y = 0.95).

Every number comes from ``oracle/``: the data d = P u(m_true) and the losses
L(m0 +- eps dm_j) = 1/2 sum_s ||P u_s - d_s||^2 with global sparse LU solves, for the 20 seeded
directions dm_j of ``workload.gradient_direction`` and eps = 1e-6.  The GPU test compares
<dL/dm, dm_j> from the adjoint solves with (L+ - L-) / (2 eps).

Usage (about 5 minutes on one core):  python tests/golden/make_grad_fd.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workload as W  # noqa: E402
from oracle import gradient, solver  # noqa: E402
from oracle.fd import Grid  # noqa: E402

EPS = 1e-6
NDIR = 20


def problem():
    wl = W.GRAD_512
    m_true = W.slowness2(wl)
    m0 = W.smoothed_model(m_true, 20.0)
    f = W.sources(wl)
    rec = W.receiver_row(wl)
    return wl, m_true, m0, f, rec


def main():
    wl, m_true, m0, f, rec = problem()
    t0 = time.perf_counter()
    u = solver.direct(Grid(wl.nx, wl.ny, wl.h, wl.k, m_true), f)
    d = np.ascontiguousarray(u.reshape(f.shape[0], -1)[:, rec])
    L0 = gradient.misfit(Grid(wl.nx, wl.ny, wl.h, wl.k, m0), f, rec, d)
    out = {"workload": wl.name, "eps": EPS, "loss_m0": L0, "directions": []}
    for j in range(NDIR):
        dm = W.gradient_direction(m0.shape, j)
        Lp = gradient.misfit(Grid(wl.nx, wl.ny, wl.h, wl.k, m0 + EPS * dm), f, rec, d)
        Lm = gradient.misfit(Grid(wl.nx, wl.ny, wl.h, wl.k, m0 - EPS * dm), f, rec, d)
        out["directions"].append({"j": j, "loss_plus": Lp, "loss_minus": Lm, "fd": (Lp - Lm) / (2 * EPS)})
        print(f"direction {j}: fd {(Lp - Lm) / (2 * EPS):.12e} ({time.perf_counter() - t0:.0f} s)", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grad_512_fd.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(f"wrote {path}")


if __name__ == "__main__":
    main()
