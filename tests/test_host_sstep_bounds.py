"""Host check of the index arithmetic of the block Gram-Schmidt kernels (no GPU).

csrc/k_sstep.hip sizes the inner-product launch from the problem (positions per workgroup, chunks, the parts
of a batch's k-steps) and indexes a swizzled LDS tile, the partial sums and the coefficient records.  This
test replays that arithmetic in Python over every workgroup, wavefront and lane for a range of vector
lengths, right-hand-side counts and block shapes, and checks that every load and store stays inside its
buffer, that the positions of a column are each summed exactly once, that the k-steps of a batch are each
taken by one wavefront per tile, and that the swizzle is a permutation of each tile row.  The formulas
replayed here are also looked up in the kernel source, so that the two cannot drift apart unnoticed.
"""
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2209_10886_amd", "csrc", "k_sstep.hip")
HDR = os.path.join(ROOT, "paper_2209_10886_amd", "csrc", "hbj_internal.h")

KSB, MAXB = 8, 64
COEF_LD = 129 + MAXB * KSB


def target_wgs(nt):
    return 512 if nt >= 4 else 768 if nt == 3 else 1024


def kparts(nt):
    return 1 if nt == 3 else 4 // nt


def positions_per_wg(n, ncol, wgs):
    cp = (n * ncol + wgs - 1) // wgs
    return max(64, (cp + 63) // 64 * 64)


def chunks(n, ncol, wgs):
    cp = positions_per_wg(n, ncol, wgs)
    return (n + cp - 1) // cp


def partial_elems(n, ncol):
    return ncol * chunks(n, ncol, target_wgs(1)) * kparts(1) * MAXB * KSB


def at(row, c):
    return row * 64 + (c ^ (row & 15))


def replay_dots(n, ncol, k1, sb, slots):
    """Every address of k_bgs_dots for one block; returns the number of times each position is summed."""
    nvt = k1 + sb
    nt = (nvt + 15) // 16
    assert nt <= 4
    wgs, kp_n = target_wgs(nt), kparts(nt)
    cp, nchunk = positions_per_wg(n, ncol, wgs), chunks(n, ncol, wgs)
    pe = partial_elems(n, ncol)
    assert ncol * nchunk * kp_n * nvt * KSB <= pe
    rows, nl = 16 * nt, 4 * nt
    ks = 16 // kp_n
    summed = [0] * n
    for wv in range(4):
        for j in range(nl):
            assert min(wv + 4 * j, nvt - 1) < slots  # basis slot loaded
            for lane in range(64):
                assert 0 <= at(wv + 4 * j, lane) < rows * 64  # tile store
    for chunk in range(nchunk):
        p0, p1 = min(chunk * cp, n), min(chunk * cp + cp, n)
        for p in range(p0, p1, 64):
            assert 0 <= p and min(p + 63, n - 1) < n  # pos = min(p + lane, n - 1)
            for q in range(p, min(p + 64, p1)):  # the lanes with p + lane < p1
                summed[q] += 1
        # k-steps of a batch: per tile, every one by exactly one wavefront
        for t in range(nt):
            taken = []
            for wv in range(4):
                mt = wv if nt == 3 else wv % nt
                kp = 0 if nt == 3 else wv // nt
                if mt != t:
                    continue
                taken += [kp * ks + qq for qq in range(ks)]
            assert sorted(taken) == list(range(16))
        for wv in range(4):
            mt = wv if nt == 3 else wv % nt
            kp = 0 if nt == 3 else wv // nt
            if mt >= nt:
                continue
            for lane in range(64):
                r16, kk = lane & 15, lane >> 4
                arow = 16 * mt + r16
                brow = k1 + ((r16 & 7) if (r16 & 7) < sb else 0)
                assert arow < rows and brow < nvt <= rows
                for qq in range(ks):
                    c = 4 * (kp * ks + qq) + kk
                    assert 0 <= at(arow, c) < rows * 64 and 0 <= at(brow, c) < rows * 64
                for r in range(4):  # partial stores
                    i = 16 * mt + kk + 4 * r
                    if r16 < 8 and i < nvt:
                        for col in (0, ncol - 1):
                            idx = (((col * nchunk + chunk) * kp_n + kp) * nvt) * KSB + i * KSB + r16
                            assert 0 <= idx < pe
    # the reduction reads nchunk * kp partial sets per column
    nset = nchunk * kp_n
    assert (ncol - 1) * nset * nvt * KSB + (nset - 1) * nvt * KSB + nvt * KSB - 1 < pe
    return summed


def test_swizzle_is_a_permutation_of_each_row():
    for row in range(64):
        assert sorted(at(row, c) - row * 64 for c in range(64)) == list(range(64))
    # 16 rows at one position: distinct 16-byte slots modulo 16 (no two lanes in one bank group)
    for c in range(64):
        assert len({at(row, c) % 16 for row in range(16)}) == 16


def test_every_position_summed_once_and_loads_in_bounds():
    cases = []
    for n in (1, 15, 63, 64, 65, 1000, 7168, 28672):
        for ncol in (1, 4, 5, 64):
            for m in (5, 50, 63):
                for k1, sb in ((1, 1), (1, min(8, m)), (m // 2 + 1, min(8, m - m // 2)), (m + 1 - min(8, m), min(8, m))):
                    if k1 >= 1 and sb >= 1 and k1 + sb <= m + 1:
                        cases.append((n, ncol, k1, sb, m + 1))
    cases.append((122880, 64, 49, 2, 51))  # the 2048^2, 16 x 16 workload's last block of a cycle
    cases.append((122880, 64, 41, 8, 51))
    for n, ncol, k1, sb, slots in cases:
        summed = replay_dots(n, ncol, k1, sb, slots)
        assert summed == [1] * n, (n, ncol, k1, sb)


def test_update_and_coefficient_records_in_bounds():
    for n in (1, 511, 512, 513, 28672):
        gx = (n + 512 - 1) // 512
        covered = set()
        for bx in range(gx):
            for u in range(2):
                for tid in range(256):
                    q = (bx * 2 + u) * 256 + tid
                    pos = q if q < n else n - 1
                    assert 0 <= pos < n
                    if q < n:
                        covered.add(q)
        assert covered == set(range(n))
    # record: R (64), R^{-1} (64), pivot index, C (k1 x 8); C row k1 - 1 <= 62 with k1 + sb <= 64
    for k1 in range(1, MAXB):
        assert 129 + (k1 - 1) * KSB + KSB - 1 < COEF_LD
        assert 129 + k1 * KSB <= COEF_LD


def test_kernel_source_matches_the_replay():
    src = open(SRC).read()
    hdr = open(HDR).read()
    for frag in ("row * 64 + (c ^ (row & 15))", "nt >= 4 ? 512 : nt == 3 ? 768 : 1024", "nt == 3 ? 1 : 4 / nt",
                 "std::max<long>(64, (cp + 63) / 64 * 64)", "(NT == 3) ? 1 : 4 / NT", "(NT == 3) ? wv : wv % NT",
                 "(NT == 3) ? 0 : wv / NT", "min(wv + 4 * j, nvt - 1)", "const int pos = min(p + lane, n - 1);",
                 "const bool in = p + lane < p1;", "(((size_t)col * nchunk + chunk) * KP + kp) * nvt * kSB",
                 "const int c = 4 * (kp * KS + qq) + kk;", "k1 + (lok ? l : 0)"):
        assert frag in src, frag
    for frag in ("kSstepMax = 8", "kSstepMaxBasis = 64", "kSstepCoefLd = 129 + kSstepMaxBasis * kSstepMax"):
        assert frag in hdr, frag
