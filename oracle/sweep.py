"""Sweeping preconditioners on the interface system (paper Secs. 5-6).

Groups.  V_a selects the interface blocks whose receiver lies on anti-diagonal
a = |i|_1, a = 2 .. N_g + 1 (Sec. 5).  Neighbours differ by one in |i|_1, so S
only couples groups a and a +- 1 and S_L = I - sum_a V_a S_{a,a-1} V_{a-1}^T is
the block lower triangle of I - S (Proposition 1); S_U is the mirror image.

SGS (Sec. 5, eq. (7)).  P^{-1} = S_U^{-1} S_L^{-1}.  S_L^{-1} r is a forward
sweep: for a = 3 .. N_g + 1, every subdomain of anti-diagonal a - 1 solves its
local problem with its current incoming data and adds its outgoing traces into
the blocks of its neighbours on anti-diagonal a.  S_U^{-1} is the backward sweep
a = N_g + 1 .. 3 into anti-diagonal a - 1.  One step per value of a: 2 (N_g - 1)
sequential steps.

Block Jacobi (Sec. 6).  The anti-diagonals are cut into p closed intervals
[s_b, e_b] of width w = N_1; each interval is swept on its own (a partial
sweep) and all partial sweeps advance in lockstep, so a pass takes w steps.
Readings of what the paper leaves open (recorded in the design notes):
  * the block inverse is of W_b^T S_L W_b = I_b - L_b, a partial forward sweep
    over the interval (the paper writes I_b + S_{L,b});
  * consecutive closed intervals share one group; by default ("restricted")
    that group's output comes from the upstream interval only and the
    downstream interval takes it as input (from the pass input, not from the
    interval that updates it); "additive" adds both contributions literally;
  * forward and backward passes compose as a product B_U^{-1} B_L^{-1} like
    SGS ("product"); "residual" uses the additive-projection update with the
    residual recomputed between the two halves.
With p = 1 every variant reduces to SGS exactly.

Pins (tests/test_oracle_sweep.py): Proposition 1 on the assembled S, equality
of the sweeps with dense triangular solves and with the dense restricted block
formula, p = 1 against SGS, and the step counts of Table 1.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .layout import bj_backward_blocks, bj_forward_blocks


class SweepStats:
    def __init__(self):
        self.steps = 0
        self.local_solves = 0


def _sweep_step(dd, src, dst, antidiags, direction, stats):
    """One lockstep step: solve every subdomain on the anti-diagonals ``antidiags`` (one per
    interval) with incoming data from ``src`` and add its outgoing traces into ``dst`` toward
    anti-diagonal a + direction.  The subdomains of a step read only their own groups, which no
    subdomain of the same step writes, so they are independent local problems."""
    lay = dd.layout
    keys = [i for a in antidiags for i in dd.subdomains_on(a)]
    for i, out in zip(keys, dd.scatter_many(keys, src)):
        stats.local_solves += 1
        for j, v in out.items():
            if j[0] + j[1] == i[0] + i[1] + direction:
                dst[lay.block(j, i)] += v


def forward_pass(dd, r, blocks, combine="restricted", stats=None):
    """Forward partial sweeps over the closed intervals ``blocks`` in lockstep.

    Each interval [s, e] computes y_s = r_s and y_a = r_a + S_{a,a-1} y_{a-1} for
    a = s+1 .. e.  Returns (y, number of lockstep steps)."""
    stats = stats or SweepStats()
    lay = dd.layout
    y = r.copy()
    # additive reading: every interval contributes its own copy of the shared group
    extra = np.zeros_like(r)
    nsteps = max(e - s for s, e in blocks)
    for t in range(1, nsteps + 1):
        src = r if t == 1 else y
        _sweep_step(dd, src, y, [s + t - 1 for (s, e) in blocks if s + t <= e], +1, stats)
        stats.steps += 1
    if combine == "additive":
        for b, (s, e) in enumerate(blocks):
            if b > 0:
                extra[lay.group_slice(s)] += r[lay.group_slice(s)]
        y = y + extra
    return y, nsteps


def backward_pass(dd, r, blocks, combine="restricted", stats=None):
    """Backward partial sweeps: interval [s, e] computes z_e = r_e and
    z_{a-1} = r_{a-1} + S_{a-1,a} z_a for a = e .. s+1."""
    stats = stats or SweepStats()
    lay = dd.layout
    z = r.copy()
    extra = np.zeros_like(r)
    nsteps = max(e - s for s, e in blocks)
    for t in range(1, nsteps + 1):
        src = r if t == 1 else z
        _sweep_step(dd, src, z, [e - t + 1 for (s, e) in blocks if e - t >= s], -1, stats)
        stats.steps += 1
    if combine == "additive":
        for b, (s, e) in enumerate(blocks):
            if b > 0:
                extra[lay.group_slice(e)] += r[lay.group_slice(e)]
        z = z + extra
    return z, nsteps


def sgs_blocks(dd):
    n_g = dd.layout.n_g
    return [(2, n_g + 1)]


def apply_sgs(dd, r, stats=None):
    """P_SGS^{-1} r = S_U^{-1} S_L^{-1} r (Sec. 5, eq. (7)): one full forward, one full backward sweep."""
    y, _ = forward_pass(dd, r, sgs_blocks(dd), stats=stats)
    z, _ = backward_pass(dd, y, sgs_blocks(dd), stats=stats)
    return z


def apply_bj(dd, r, width=None, combine="restricted", compose="product", stats=None):
    """Block-Jacobi sweeping preconditioner (Sec. 6) applied to r."""
    fb = bj_forward_blocks(dd.n1, dd.n2, width)
    bb = bj_backward_blocks(dd.n1, dd.n2, width)
    y, _ = forward_pass(dd, r, fb, combine, stats)
    if compose == "product":
        z, _ = backward_pass(dd, y, bb, combine, stats)
        return z
    if compose == "residual":
        # x^{k+1/2} = B_L^{-1} r;  r^{k+1/2} = r - (I - S) x^{k+1/2};  x^{k+1} = x^{k+1/2} + B_U^{-1} r^{k+1/2}
        r_half = r - dd.apply_operator(y)
        z, _ = backward_pass(dd, r_half, bb, combine, stats)
        return y + z
    raise ValueError(compose)


def apply_preconditioner(dd, r, kind="bj", **kw):
    if kind == "none":
        return r.copy()
    if kind == "sgs":
        return apply_sgs(dd, r, stats=kw.get("stats"))
    if kind == "bj":
        return apply_bj(dd, r, **kw)
    raise ValueError(kind)


def step_counts(n1, n2, width=None):
    """(SGS steps, BJ steps) per preconditioner application: 2 (N_g - 1) and 2 min(w, N_g - 1)."""
    n_g = n1 + n2 - 1
    fb = bj_forward_blocks(n1, n2, width)
    bb = bj_backward_blocks(n1, n2, width)
    bj = max(e - s for s, e in fb) + max(e - s for s, e in bb)
    return 2 * (n_g - 1), bj


# ---------------------------------------------------------------------------
# Dense forms of the same operators, for pinning the sweeps (tiny problems)
# ---------------------------------------------------------------------------

def selector(lay, groups):
    """Columns of the identity for the positions of the given groups (V_a or W_b)."""
    pos = np.concatenate([np.arange(lay.nif)[lay.group_slice(a)] for a in groups])
    return pos


def dense_SL_SU(lay, S):
    """S_L = I - sum V_a S_{a,a-1} V_{a-1}^T and S_U = I - sum V_{a-1} S_{a-1,a} V_a^T (Prop. 1)."""
    n = lay.nif
    SL = np.eye(n, dtype=np.complex128)
    SU = np.eye(n, dtype=np.complex128)
    for a in range(3, lay.n_g + 2):
        ra, rb = lay.group_slice(a), lay.group_slice(a - 1)
        SL[ra, rb] -= S[ra, rb]
        SU[rb, ra] -= S[rb, ra]
    return SL, SU


def dense_sgs(lay, S, r):
    """S_U^{-1} S_L^{-1} r by dense triangular solves (textbook routine)."""
    SL, SU = dense_SL_SU(lay, S)
    y = sla.solve_triangular(SL, r, lower=True, unit_diagonal=True)
    return sla.solve_triangular(SU, y, lower=False, unit_diagonal=True)


def dense_block_inverse(lay, M, r, blocks, upstream_owned, combine="restricted"):
    """sum_b W~_b (W_b^T M W_b)^{-1} W_b^T r for the closed intervals ``blocks``.

    Restricted: W~_b keeps only the groups owned by interval b; a group shared by
    two intervals is owned by ``upstream_owned(b, group)``.  Additive: W~_b = W_b."""
    out = np.zeros(lay.nif, dtype=np.complex128)
    for b, (s, e) in enumerate(blocks):
        pos = selector(lay, range(s, e + 1))
        xb = np.linalg.solve(M[np.ix_(pos, pos)], r[pos])
        if combine == "additive":
            out[pos] += xb
            continue
        keep = np.zeros(lay.nif, dtype=bool)
        for a in range(s, e + 1):
            if upstream_owned(b, a):
                keep[lay.group_slice(a)] = True
        mask = keep[pos]
        out[pos[mask]] += xb[mask]
    return out


def dense_bj(lay, S, r, width=None, combine="restricted"):
    """Block-Jacobi (product composition) from the dense S_L, S_U and the interval selectors."""
    SL, SU = dense_SL_SU(lay, S)
    fb = bj_forward_blocks(lay.n1, lay.n2, width)
    bb = bj_backward_blocks(lay.n1, lay.n2, width)

    def own_f(b, a):  # forward: shared lower group s_b (b > 0) belongs to interval b-1
        return not (b > 0 and a == fb[b][0])

    def own_b(b, a):  # backward: shared upper group e_b (b > 0) belongs to interval b-1
        return not (b > 0 and a == bb[b][1])

    y = dense_block_inverse(lay, SL, r, fb, own_f, combine)
    return dense_block_inverse(lay, SU, y, bb, own_b, combine)
