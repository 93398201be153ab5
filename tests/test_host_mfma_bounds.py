"""Host check of the B-operand addressing of the many-right-hand-side MFMA kernels (no GPU).

k_scatter_mm and k_recon_mm (csrc/k_scatter_mm.hip) give every lane a right-hand-side column
rb0 + 16 (tb0 + t) + i of a 64-column tile.  When fewer than 64 right-hand sides are in flight,
that column can lie past the padded width rpad = 16 ceil(nrhs / 16); the kernels clamp it (to
nrhs - 1, or rpad - 1 for the reconstruction's gathered tiles) and drop the products of those
columns.  This test replays the kernels' index arithmetic over every lane of the launch grid for
1..130 right-hand sides and checks that every B load stays inside its buffer, and that the same
arithmetic without the clamp would not.
"""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2209_10886_amd", "csrc", "k_scatter_mm.hip")
TB = 4  # 16-column blocks per 64-column tile


def _scatter_max_index(nrhs, nsub, L, nif, face_rows, direct, ns, clamp=True):
    """Largest B element index of k_scatter_mm over the grid (nsub, ceil(nrhs/64)) and all lanes.
    face_rows: (in_off, c0, c1) of every present face of the subdomain."""
    rpad = (nrhs + 15) // 16 * 16
    tw = TB // ns
    worst = -1
    for z in range((nrhs + 16 * TB - 1) // (16 * TB)):
        rb0 = z * 16 * TB
        for grp in range(ns):
            tb0 = grp * tw
            for t in range(tw):
                for i in range(16):
                    r = rb0 + 16 * (tb0 + t) + i
                    if clamp:
                        r = min(r, nrhs - 1)
                    for j in range(nsub):
                        for (in_off, c0, c1) in face_rows:
                            for cc in (c0, c1 - 1):  # the addresses are monotone in cc
                                if direct:
                                    idx = r * nif + (in_off - c0) + cc
                                else:
                                    idx = j * L * rpad + r + cc * rpad
                                worst = max(worst, idx)
    size = nrhs * nif if direct else nsub * L * rpad
    return worst, size


def _recon_max_index(nrhs, ndom, L, clamp=True):
    rpad = (nrhs + 15) // 16 * 16
    worst = -1
    for z in range((nrhs + 16 * TB - 1) // (16 * TB)):
        rb0 = z * 16 * TB
        for t in range(TB):
            for i in range(16):
                jr = rb0 + 16 * t + i
                if clamp:
                    jr = min(jr, rpad - 1)
                s = ndom - 1
                idx = s * L * rpad + (L - 1) * rpad + jr
                worst = max(worst, idx)
    return worst, ndom * L * rpad


def test_kernel_source_has_the_clamps():
    src = open(SRC).read()
    assert re.search(r"min\(rb0 \+ 16 \* \(tb0 \+ t\) \+ i, nrhs - 1\)", src)
    assert re.search(r"min\(rb0 \+ 16 \* t \+ i, rpad - 1\)", src)


def test_b_operand_loads_stay_in_bounds():
    # a 16 x 12 subdomain with all four faces present, interface vector of 10 such blocks
    snx, sny = 16, 12
    L = 2 * snx + 2 * sny
    faces = [(0, 0, sny), (sny, sny, 2 * sny), (2 * sny, 2 * sny, 2 * sny + snx), (2 * sny + snx, 2 * sny + snx, L)]
    nif = 10 * L
    overflow_seen = False
    for nrhs in range(1, 131):
        for direct in (False, True):
            for ns in (1, 2):
                worst, size = _scatter_max_index(nrhs, 3, L, nif, faces, direct, ns)
                assert worst < size, (nrhs, direct, ns, worst, size)
                w0, _ = _scatter_max_index(nrhs, 3, L, nif, faces, direct, ns, clamp=False)
                overflow_seen |= w0 >= size
        worst, size = _recon_max_index(nrhs, 5, L)
        assert worst < size, (nrhs, worst, size)
    # without the clamps the same grid reads past the buffers (the fault the clamps fixed)
    assert overflow_seen
    assert _recon_max_index(20, 5, L, clamp=False)[0] >= _recon_max_index(20, 5, L)[1]


KW = 4  # wavefronts splitting the k range of a tile


def _ring_lane_loads(snx, sny, in_off, direct, rpad, ring):
    """Replay of the register-ring k-loop of k_scatter_mm (RING > 0) for one tile: for every
    wavefront w, k-step m (including the prefetches past the end) and lane row k, the column the
    lane reads, whether it enters the products, and its B offset relative to jr."""
    L = 2 * snx + 2 * sny
    b1, b2, b3 = sny, 2 * sny, 2 * sny + snx
    present = [o >= 0 for o in in_off]
    pm = sum(1 << f for f in range(4) if present[f])
    fo = ([in_off[0], in_off[1] - b1, in_off[2] - b2, in_off[3] - b3] if direct else [0, 0, 0, 0])
    cs = 1 if direct else rpad
    nst = (L + 4 * KW - 1) // (4 * KW)
    nsp = (nst + ring - 1) // ring * ring
    out = []
    for w in range(KW):
        for m in range(nsp + ring):
            for k in range(4):
                col = 4 * (KW * m + w) + k
                c1, c2, c3 = col >= b1, col >= b2, col >= b3
                f = int(c1) + int(c2) + int(c3)
                ok = col < L and bool((pm >> f) & 1)
                fof = fo[0] + int(c1) * (fo[1] - fo[0]) + int(c2) * (fo[2] - fo[1]) + int(c3) * (fo[3] - fo[2])
                cc = col if ok else 0
                off = fof + cc * cs if ok else 0
                out.append((w, m, k, col, f, ok, cc, off))
    return out, L


def test_ring_kloop_covers_every_column_once_and_stays_in_bounds():
    for snx, sny in ((16, 12), (10, 10), (128, 128), (8, 24)):
        L = 2 * snx + 2 * sny
        nif = 10 * L
        for absent in ((), (0,), (2, 3), (1,), (0, 1, 2)):
            # interface offsets of the present faces somewhere inside a vector of nif positions
            in_off = [-1 if f in absent else 3 * L + f * max(snx, sny) for f in range(4)]
            face_lo = [0, sny, 2 * sny, 2 * sny + snx]
            face_hi = [sny, 2 * sny, 2 * sny + snx, L]
            for direct in (False, True):
                for ring in (4, 8):
                    rpad = 64
                    loads, _ = _ring_lane_loads(snx, sny, in_off, direct, rpad, ring)
                    seen = {}
                    for (w, m, k, col, f, ok, cc, off) in loads:
                        assert 0 <= cc < L  # the A load
                        if direct:
                            assert 0 <= off < nif  # B relative to the right-hand side's row r * nif
                        else:
                            assert 0 <= off < L * rpad  # B relative to subdomain j's tile
                        if ok:
                            assert face_lo[f] <= col < face_hi[f] and in_off[f] >= 0
                            if direct:
                                assert off == in_off[f] + (col - face_lo[f])
                            else:
                                assert off == col * rpad
                            seen[col] = seen.get(col, 0) + 1
                    want = {c for f in range(4) if in_off[f] >= 0 for c in range(face_lo[f], face_hi[f])}
                    assert set(seen) == want
                    assert all(v == 1 for v in seen.values())


def test_kernel_source_has_the_ring_arithmetic():
    src = open(SRC).read()
    assert "const int col = 4 * (KWT * m + w) + k;" in src
    assert "const int fo = fo0 + (int)c1 * (fo1 - fo0) + (int)c2 * (fo2 - fo1) + (int)c3 * (fo3 - fo2);" in src
    assert "const int off = ok ? fo + cc * ics : 0;" in src
