"""Host replay of the partitioned single-right-hand-side band solves (no GPU).

csrc/k_trisolve.hip can split the column blocks of one subdomain's forward (backward) substitution
into np runs of bpp blocks that run on separate workgroups: a first pass solves every run but the
last (in processing order) from a zero incoming window state, a chain applies the runs' transfer
matrices Phi (the response of the outgoing state to each unit incoming state, formed once per
factorisation) to recover the true incoming states, and a second pass solves every run but the
first from its true state.  The substitution is linear in its incoming state and its right-hand
side, so the result equals the sequential substitution's up to rounding.

This test replays the kernels' recurrences in numpy, with the same window layout (16-row blocks,
kl (kv) state rows, row interchanges inside the forward window) and the same index clamps, on
random block matrices and permutations, for every partition count from 2 to the number of blocks
and ragged last runs, and checks the partitioned results against the sequential ones.  It also
checks that every index the kernels form stays inside its buffer.  The fragments replayed here are
looked up in the kernel source.
"""
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2209_10886_amd", "csrc", "k_trisolve.hip")
RT = os.path.join(ROOT, "paper_2209_10886_amd", "csrc", "runtime.hip")
NB = 16


def layout(nblk, np_req):
    """Partition count and blocks per run as the host computes them (every run nonempty)."""
    npart = max(2, min(np_req, nblk))
    bpp = (nblk + npart - 1) // npart
    npart = (nblk + bpp - 1) // bpp
    return npart, bpp


def problem(rng, nblk, kl, kv, swaps=0.5):
    wf, wb = NB + kl, NB + kv
    cplx = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    Mf = cplx(nblk, wf, NB) * 0.3
    Mb = cplx(nblk, wb, NB) * 0.3
    ident = rng.random(nblk) >= swaps
    P = np.tile(np.arange(wf), (nblk, 1))
    for b in range(nblk):
        if not ident[b]:
            for t in range(NB):  # interchanges of a block row with a row below it in the window
                k = rng.integers(t, wf)
                P[b, [t, k]] = P[b, [k, t]]
    return Mf, Mb, P, ident


# ---------------------------------------------------------------- sequential (k_fwd / k_bwd)
def fwd_seq(Mf, P, ident, rhs, kl):
    nblk, wf = Mf.shape[0], NB + kl
    ylen = nblk * NB
    win = np.array([rhs[q] if q < ylen else 0 for q in range(wf)], dtype=complex)
    y = np.zeros(ylen, complex)
    for b in range(nblk):
        if not ident[b]:
            win = win[P[b]]
        acc = Mf[b] @ win[:NB]
        y[b * NB:(b + 1) * NB] = acc[:NB]
        new = np.zeros(wf, complex)
        new[:kl] = acc[NB:] + win[NB:]
        for t in range(NB):
            row = (b + 1) * NB + kl + t
            new[kl + t] = rhs[row] if row < ylen else 0
        win = new
    return y


def bwd_seq(Mb, y, kv):
    nblk, wb = Mb.shape[0], NB + kv
    ylen = nblk * NB
    j0 = (nblk - 1) * NB
    win = np.array([y[j0 - kv + q] if j0 - kv + q >= 0 else 0 for q in range(wb)], dtype=complex)
    x = np.zeros(ylen, complex)
    for b in range(nblk - 1, -1, -1):
        acc = Mb[b] @ win[kv:]
        x[b * NB:(b + 1) * NB] = acc[kv:]
        new = np.zeros(wb, complex)
        new[NB:] = acc[:kv] + win[:kv]
        for t in range(NB):
            row = (b - 1) * NB - kv + t
            new[t] = y[row] if row >= 0 else 0
        win = new
    return x


# ---------------------------------------------------------------- partitioned
def fwd_run(Mf, P, ident, rhs, kl, b0, b1, state, outs, y):
    """One forward run over blocks [b0, b1) from window state `state` (None: from the right-hand
    side, the first run); returns the outgoing state.  Fresh rows always come from rhs."""
    ylen, wf = len(rhs), NB + kl
    win = np.zeros(wf, complex)
    for q in range(wf):
        row = b0 * NB + q
        win[q] = rhs[row] if row < ylen else 0
    if state is not None:
        win[:kl] = state
    for b in range(b0, b1):
        for d in range(3):  # the prefetch clamps of the kernel (depth 3): in range
            assert b0 <= min(b + d, b1 - 1) < b1
            assert 0 <= min((b + d + 1) * NB + kl + NB - 1, ylen - 1) < ylen
        if not ident[b]:
            win = win[P[b]]
        acc = Mf[b] @ win[:NB]
        if outs:
            y[b * NB:(b + 1) * NB] = acc[:NB]
        new = np.zeros(wf, complex)
        new[:kl] = acc[NB:] + win[NB:]
        for t in range(NB):
            row = (b + 1) * NB + kl + t
            new[kl + t] = rhs[row] if row < ylen else 0
        win = new
    return win[:kl].copy()


def bwd_run(Mb, y, kv, b0, b1, state, outs, x):
    ylen, wb = len(y), NB + kv
    win = np.zeros(wb, complex)
    for q in range(wb):
        row = (b1 - 1) * NB - kv + q
        win[q] = y[row] if row >= 0 else 0
    if state is not None:
        win[NB:] = state
    for b in range(b1 - 1, b0 - 1, -1):
        for d in range(3):
            assert b0 <= max(b - d, b0) < b1
            assert 0 <= max((b - d - 1) * NB - kv, 0) < ylen
        acc = Mb[b] @ win[kv:]
        if outs:
            x[b * NB:(b + 1) * NB] = acc[kv:]
        new = np.zeros(wb, complex)
        new[NB:] = acc[:kv] + win[:kv]
        for t in range(NB):
            row = (b - 1) * NB - kv + t
            new[t] = y[row] if row >= 0 else 0
        win = new
    return win[NB:].copy()


def phi_fwd(Mf, P, ident, kl, b0, b1):
    """Transfer matrix of a forward run: column j = outgoing state for unit incoming state j and
    zero right-hand side (the formation kernel's recurrence)."""
    wf = NB + kl
    phi = np.zeros((kl, kl), complex)
    for j in range(kl):
        win = np.zeros(wf, complex)
        win[j] = 1
        for b in range(b0, b1):
            if not ident[b]:
                win = win[P[b]]
            acc = Mf[b] @ win[:NB]
            new = np.zeros(wf, complex)
            new[:kl] = acc[NB:] + win[NB:]
            win = new
        phi[:, j] = win[:kl]
    return phi


def phi_bwd(Mb, kv, b0, b1):
    wb = NB + kv
    phi = np.zeros((kv, kv), complex)
    for j in range(kv):
        win = np.zeros(wb, complex)
        win[NB + j] = 1
        for b in range(b1 - 1, b0 - 1, -1):
            acc = Mb[b] @ win[kv:]
            new = np.zeros(wb, complex)
            new[NB:] = acc[:kv] + win[:kv]
            win = new
        phi[:, j] = win[NB:]
    return phi


def fwd_part(Mf, P, ident, rhs, kl, npart, bpp):
    nblk = Mf.shape[0]
    rng_of = lambda o: (o * bpp, min(o * bpp + bpp, nblk))
    y = np.zeros(len(rhs), complex)
    sig, tt = {}, {}
    for o in range(npart - 1):  # first pass: run 0 exact (outputs), the others from zero state
        b0, b1 = rng_of(o)
        assert b0 < b1
        if o == 0:
            tt[1] = fwd_run(Mf, P, ident, rhs, kl, b0, b1, None, True, y)
        else:
            sig[o] = fwd_run(Mf, P, ident, rhs, kl, b0, b1, np.zeros(kl), False, y)
    for o in range(1, npart - 1):  # the chain
        tt[o + 1] = sig[o] + phi_fwd(Mf, P, ident, kl, *rng_of(o)) @ tt[o]
    for o in range(1, npart):  # second pass
        b0, b1 = rng_of(o)
        assert b0 < b1
        fwd_run(Mf, P, ident, rhs, kl, b0, b1, tt[o], True, y)
    return y


def bwd_part(Mb, y, kv, npart, bpp):
    nblk = Mb.shape[0]
    rng_of = lambda o: ((npart - 1 - o) * bpp, min((npart - 1 - o) * bpp + bpp, nblk))  # run o from the top
    x = np.zeros(len(y), complex)
    sig, tt = {}, {}
    for o in range(npart - 1):
        b0, b1 = rng_of(o)
        assert b0 < b1
        if o == 0:
            tt[1] = bwd_run(Mb, y, kv, b0, b1, None, True, x)
        else:
            sig[o] = bwd_run(Mb, y, kv, b0, b1, np.zeros(kv), False, x)
    for o in range(1, npart - 1):
        tt[o + 1] = sig[o] + phi_bwd(Mb, kv, *rng_of(o)) @ tt[o]
    for o in range(1, npart):
        b0, b1 = rng_of(o)
        assert b0 < b1
        bwd_run(Mb, y, kv, b0, b1, tt[o], True, x)
    return x


def test_layout_covers_every_block_once():
    for nblk in range(1, 80):
        for req in range(2, 40):
            npart, bpp = layout(nblk, req)
            if nblk < 2:
                continue
            blocks = [b for o in range(npart) for b in range(o * bpp, min(o * bpp + bpp, nblk))]
            assert blocks == list(range(nblk)), (nblk, req)
            assert 2 <= npart <= min(req, nblk) or (npart == 2 and nblk >= 2)
            assert all(o * bpp < min(o * bpp + bpp, nblk) for o in range(npart))


def test_first_pass_writes_every_right_hand_side_row_it_reads():
    """Pass 1 of the forward solve writes the right-hand sides: run o the rows [b0 nb, b1 nb + kl +
    nb) before it reads them (the rows of its window and the rows entering it), the last run its own
    rows; together every row, so that pass 2 finds them all."""
    for nblk in (2, 3, 7, 64, 1024):
        for kl in (8, 32, 128):
            ylen = nblk * NB
            for req in (2, 3, 5, 16, 64):
                npart, bpp = layout(nblk, req)
                covered = set()
                for o in range(npart):
                    b0, b1 = o * bpp, min(o * bpp + bpp, nblk)
                    hi = ylen if o == npart - 1 else min(b1 * NB + kl + NB, ylen)
                    mine = set(range(b0 * NB, hi))
                    covered |= mine
                    if o == npart - 1:
                        continue
                    reads = {r for r in range(b0 * NB, b0 * NB + kl + NB) if r < ylen}  # initial window
                    for b in range(b0, b1):
                        reads |= {r for r in range((b + 1) * NB + kl, (b + 2) * NB + kl) if r < ylen}
                    assert reads <= mine, (nblk, kl, req, o)
                assert covered == set(range(ylen))


def test_partitioned_forward_and_backward_match_sequential():
    rng = np.random.default_rng(7)
    for nblk, kl, ku in ((9, 32, 32), (7, 16, 16), (12, 48, 24), (5, 8, 8)):
        kv = kl + ku
        Mf, Mb, P, ident = problem(rng, nblk, kl, kv)
        ylen = nblk * NB
        rhs = rng.standard_normal(ylen) + 1j * rng.standard_normal(ylen)
        rhs[ylen - 5:] = 0  # padding rows past the subdomain
        y = fwd_seq(Mf, P, ident, rhs, kl)
        x = bwd_seq(Mb, y, kv)
        for req in range(2, nblk + 2):
            npart, bpp = layout(nblk, req)
            yp = fwd_part(Mf, P, ident, rhs, kl, npart, bpp)
            assert np.allclose(yp, y, rtol=1e-11, atol=1e-11 * np.abs(y).max()), (nblk, kl, req)
            xp = bwd_part(Mb, y, kv, npart, bpp)
            assert np.allclose(xp, x, rtol=1e-11, atol=1e-11 * np.abs(x).max()), (nblk, kv, req)


def test_state_and_transfer_buffers_in_bounds():
    """sig / tt: [entry][np][ns] with ns >= kv; Phi: [subdomain][np - 2][S][S] (column-major)."""
    for nent in (1, 8, 64):
        for npart in (2, 3, 8, 16):
            for kl, kv in ((128, 256), (32, 64)):
                ns = kv
                size = nent * npart * ns
                for slot in (0, nent - 1):
                    for o in range(npart):
                        for S in (kl, kv):
                            assert (slot * npart + o) * ns + S - 1 < size
                nsub = 4
                for S in (kl, kv):
                    psize = nsub * max(npart - 2, 0) * S * S
                    for s in range(nsub):
                        for o in range(1, npart - 1):
                            base = (s * (npart - 2) + (o - 1)) * S * S
                            assert 0 <= base and base + (S - 1) * S + S - 1 < psize


def test_kernel_source_matches_the_replay():
    src = open(SRC).read()
    rt = open(RT).read()
    for frag in ("const int b0 = o * pl.bpp, b1 = min(b0 + pl.bpp, nblk);",
                 "const int o = phase == 1 ? (int)blockIdx.y : (int)blockIdx.y + 1;",
                 "const int p = pl.np - 1 - o;",
                 "if (q < kl && o > 0) v = phase == 3 ? tin[q] : czero<C>();",
                 "if (q >= NB && o > 0) v = phase == 3 ? tin[q - NB] : czero<C>();",
                 "const int row = (b1 - 1) * NB - kv + q;",
                 "min(b + D, b1 - 1)", "max(b - D, b0)",
                 "C* dst = o == 0 ? tt + ((size_t)slot * pl.np + 1) * pl.ns : sig + ((size_t)slot * pl.np + o) * pl.ns;",
                 "((size_t)e.s * (pl.np - 2) + (o - 1)) * S * S",
                 "const int o = 1 + t / W, w = t - (o - 1) * W;", "const int slot = blockIdx.x % nent;",
                 "kChainRows = 16", "const int ntasks = (pl.np - 2) * W;",
                 "if (o >= 1 && o + 1 <= pl.np - 1) {  // the chain's output state o + 1 starts unset",
                 "const C* src = tt + ((size_t)slot * pl.np + o) * pl.ns;",
                 "st_coh(tt + ((size_t)slot * pl.np + o + 1) * pl.ns + i, v);",
                 "const int hi = o == pl.np - 1 ? ylen : min(b1 * NB + kl + NB, ylen);",
                 "return nent;",
                 "std::max(1, std::min(std::min((pl.np - 2) * W, 2 * W), kChainGridMax / std::max(nent, 1)))"):
        assert frag in src, frag
    for frag in ("int bpp = (nblk + np - 1) / np;", "np = (nblk + bpp - 1) / bpp;"):
        assert frag in rt, frag


def test_chain_tickets_wait_only_for_smaller_tickets():
    """The chain's tasks: the workgroups of entry blockIdx % nent claim ticket t of the entry's
    counter -> (step o, row slice w) in step order; a task of step o reads the state o, written by
    the W tasks of step o - 1 of its entry, which must all hold smaller tickets of the same counter
    (the launch then completes whatever the number of resident workgroups); the states o >= 2 that
    the tasks wait for are exactly those the first pass marks unset (runs 1 .. np - 2 mark state
    o + 1); every entry has a workgroup, and every task's rows and counter stay in their buffers."""
    rows_per_task, grid_max = 16, 1024
    for nent in (1, 7, 8, 64, 200):
        for npart in (3, 4, 16):
            for S in (10, 16, 128, 256, 560):
                W = (S + rows_per_task - 1) // rows_per_task
                ntasks = (npart - 2) * W
                nctr = nent
                marked = {o + 1 for o in range(1, npart - 1)}
                assert marked == set(range(2, npart))  # every state a task waits for, and no other
                per = max(1, min(min(ntasks, 2 * W), grid_max // max(nent, 1)))
                grid = nent * per
                assert {b % nent for b in range(grid)} == set(range(nent))
                for slot in (0, nent - 1):
                    assert slot < nctr  # the entry's ticket counter
                    ticket = {}
                    for t in range(ntasks):
                        o, w = 1 + t // W, t % W
                        assert 1 <= o <= npart - 2 and 0 <= w < W
                        ticket[(o, w)] = t
                        assert slot < nctr  # its ticket counter
                        assert (o == 1) or (o in marked)
                        assert w * rows_per_task < S
                    for (o, w), t in ticket.items():
                        if o >= 2:
                            assert all(ticket[(o - 1, ww)] < t for ww in range(W))
