"""Pins of the oracle's index layer against the paper's printed values (Sec. 2, Sec. 7, Table 1)."""
import os

import pytest

from oracle import layout, sweep

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLD, name)) as fh:
        return [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]


def test_m_map_worked_example():
    """Sec. 2: m((1,1),(1,2)) = 1, m((1,1),(2,1)) = 2, m((1,2),(1,1)) = 3 (any grid >= 2 x 2)."""
    for n1, n2 in [(2, 2), (3, 3), (5, 5), (5, 10), (8, 8)]:
        mm = layout.m_map(n1, n2)
        for i1, i2, j1, j2, m in _rows("m_map_worked_example.txt"):
            assert mm[((int(i1), int(i2)), (int(j1), int(j2)))] == int(m)


@pytest.mark.parametrize("n1,n2", [(1, 2), (2, 1), (2, 2), (3, 4), (5, 5), (8, 8), (5, 20)])
def test_counts_and_pairs(n1, n2):
    """Sec. 2: N_e = 2 N1 N2 - N1 - N2 interfaces, 2 N_e ordered pairs, N_g = N1 + N2 - 1."""
    n_dom, n_e, n_g = layout.counts(n1, n2)
    assert n_dom == n1 * n2
    ps = layout.pairs(n1, n2)
    assert len(ps) == 2 * n_e
    # every interface appears once in each direction
    assert len({frozenset(p) for p in ps}) == n_e
    assert n_g == n1 + n2 - 1
    # the number of anti-diagonals of the checkerboard is N_g
    assert len({i1 + i2 for i1 in range(1, n1 + 1) for i2 in range(1, n2 + 1)}) == n_g


def test_pair_order_brute_force():
    """The m map is monotone for the pair order of Definition 2 (brute force over all pairs of pairs)."""
    n1, n2 = 4, 3
    mm = layout.m_map(n1, n2)

    def less(i, j):  # Definition 1, written independently of order_key
        return (i[0] + i[1] < j[0] + j[1]) or (i[0] + i[1] == j[0] + j[1] and i[0] < j[0])

    def pless(p, q):  # Definition 2
        return less(p[0], q[0]) or (p[0] == q[0] and less(p[1], q[1]))

    items = list(mm.items())
    for p, mp in items:
        for q, mq in items:
            if p != q:
                assert (mp < mq) == pless(p, q)


@pytest.mark.parametrize("n1,n2", [(2, 2), (3, 2), (4, 4), (5, 10)])
def test_groups_contiguous(n1, n2):
    """V_a selects blocks whose receiver has |i|_1 = a; in m order they are contiguous and increasing in a."""
    lay = layout.Layout(n1, n2, 3, 2)
    g = lay.group_of_position()
    assert list(g) == sorted(g)
    for a in range(2, lay.n_g + 2):
        sl = lay.group_slice(a)
        assert (g[sl] == a).all() and (g == a).sum() == sl.stop - sl.start


def test_table1_step_counts():
    """Table 1, column ns: SP 16/26/36/46 and BSP 10 for 5 x {5, 10, 15, 20}."""
    for n1, n2, sp_ns, bsp_ns in _rows("table1_steps.txt"):
        sgs, bj = sweep.step_counts(int(n1), int(n2))
        assert sgs == int(sp_ns)
        assert bj == int(bsp_ns)


def test_text_step_counts():
    """Sec. 7 text: 8 forward steps of the full sweep on 5 x 5, 5 forward BJ steps; 5 x 10 has two cuts."""
    vals = {(q, int(a), int(b)): int(v) for q, a, b, v in _rows("sweep_steps_text.txt")}
    n_g = 5 + 5 - 1
    assert n_g - 1 == vals[("full_forward_steps", 5, 5)]
    assert sweep.step_counts(5, 5)[0] == vals[("full_total_steps", 5, 5)]
    fb = layout.bj_forward_blocks(5, 5)
    assert max(e - s for s, e in fb) == vals[("bj_forward_steps", 5, 5)]
    assert layout.num_partial_sweeps(5, 10) == vals[("bj_partial_sweeps", 5, 10)]


def test_bj_intervals_cover_and_share():
    """Closed intervals of Sec. 6 cover [2, N_g + 1]; consecutive ones share exactly one group."""
    for n1, n2 in [(2, 2), (3, 5), (5, 5), (5, 20), (8, 8), (16, 16)]:
        _, _, n_g = layout.counts(n1, n2)
        for blocks in (layout.bj_forward_blocks(n1, n2), sorted(layout.bj_backward_blocks(n1, n2))):
            assert blocks[0][0] == 2 and blocks[-1][1] == n_g + 1
            for (s0, e0), (s1, e1) in zip(blocks, blocks[1:]):
                assert e0 == s1
            assert all(e - s <= n1 for s, e in blocks)
        # width N_g - 1 reduces to a single interval: the full SGS sweep
        assert layout.bj_forward_blocks(n1, n2, n_g - 1) == [(2, n_g + 1)]
