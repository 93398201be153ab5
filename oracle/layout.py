"""Multi-indices, orders and the interface layout map m (paper Sec. 2).

Subdomains are multi-indices i = (i1, i2), 1-based: i1 is the column (x) and i2
the row (y) of an n1 x n2 checkerboard.  Interface unknowns are indexed by
ordered pairs (i, j) with j a neighbour of i; the block of index m(i, j) holds
the data that subdomain i RECEIVES from j (Sec. 4: g_{m(j,i)} is the data seen
by j on its interface with i).

Parity pins: the worked values of m printed in Sec. 2 and the counts N_e, N_g
of Sec. 2 (tests/test_oracle_layout.py).
"""
from __future__ import annotations

import math


def norm1(i):
    """Discrete l1 norm |i|_1 = |i1| + |i2| (Sec. 2)."""
    return abs(i[0]) + abs(i[1])


def order_key(i):
    """Sort key of the lexicographic order on multi-indices (Sec. 2, Definition 1):
    i < j iff |i|_1 < |j|_1, or |i|_1 = |j|_1 and i1 < j1."""
    return (norm1(i), i[0])


def pair_key(p):
    """Sort key of the order on pairs (Sec. 2, Definition 2):
    (i, j) < (k, l) iff i < k, or i = k and j < l."""
    return (order_key(p[0]), order_key(p[1]))


def subdomains(n1, n2):
    """All multi-indices of an n1-column, n2-row checkerboard, in lexicographic order."""
    return sorted(((i1, i2) for i1 in range(1, n1 + 1) for i2 in range(1, n2 + 1)), key=order_key)


def neighbours(i, n1, n2):
    """D_i: subdomains sharing an interface with i (Sec. 3, eq. (2))."""
    i1, i2 = i
    out = []
    for j in ((i1 - 1, i2), (i1 + 1, i2), (i1, i2 - 1), (i1, i2 + 1)):
        if 1 <= j[0] <= n1 and 1 <= j[1] <= n2:
            out.append(j)
    return sorted(out, key=order_key)


def pairs(n1, n2):
    """Every ordered pair (i, j), j in D_i, sorted by the pair order (Definition 2)."""
    ps = [(i, j) for i in subdomains(n1, n2) for j in neighbours(i, n1, n2)]
    return sorted(ps, key=pair_key)


def m_map(n1, n2):
    """The monotone map m from ordered pairs to 1, 2, ... (Sec. 2)."""
    return {p: k + 1 for k, p in enumerate(pairs(n1, n2))}


def counts(n1, n2):
    """(N_dom, N_e, N_g) of Sec. 2: subdomains, interior interfaces, diagonal groups."""
    n_dom = n1 * n2
    n_e = 2 * n1 * n2 - n1 - n2
    n_g = n1 + n2 - 1
    return n_dom, n_e, n_g


def antidiagonal(a, n1, n2):
    """Subdomains with |i|_1 = a, in lexicographic order (increasing i1)."""
    return [i for i in subdomains(n1, n2) if norm1(i) == a]


class Layout:
    """Interface-vector layout of an n1 x n2 checkerboard of sub_nx x sub_ny subdomains.

    Block m(i, j) occupies ``offset[(i, j)] : offset[(i, j)] + size[(i, j)]`` of the
    global interface vector; blocks follow the m order.  A block on a vertical
    interface (i and j in the same row) has sub_ny entries ordered by increasing
    y; a block on a horizontal interface has sub_nx entries ordered by increasing x.
    """

    def __init__(self, n1, n2, sub_nx, sub_ny):
        self.n1, self.n2 = n1, n2
        self.sub_nx, self.sub_ny = sub_nx, sub_ny
        self.pairs = pairs(n1, n2)
        self.m = {p: k + 1 for k, p in enumerate(self.pairs)}
        self.size = {}
        self.offset = {}
        off = 0
        for (i, j) in self.pairs:
            sz = sub_ny if i[1] == j[1] else sub_nx
            self.size[(i, j)] = sz
            self.offset[(i, j)] = off
            off += sz
        self.nif = off
        self.n_dom, self.n_e, self.n_g = counts(n1, n2)

    def block(self, i, j):
        o = self.offset[(i, j)]
        return slice(o, o + self.size[(i, j)])

    def group_slice(self, a):
        """Positions of V_a: blocks whose receiver lies on anti-diagonal a (Sec. 5).
        The pair order makes every group one contiguous range."""
        idx = [k for k, (i, _) in enumerate(self.pairs) if norm1(i) == a]
        if not idx:
            return slice(0, 0)
        first, last = self.pairs[idx[0]], self.pairs[idx[-1]]
        return slice(self.offset[first], self.offset[last] + self.size[last])

    def group_of_position(self):
        """Anti-diagonal index of the receiver of every interface position (int array)."""
        import numpy as np

        g = np.empty(self.nif, dtype=np.int64)
        for (i, j) in self.pairs:
            g[self.block(i, j)] = norm1(i)
        return g


def bj_forward_blocks(n1, n2, width=None):
    """Closed anti-diagonal intervals [s_b, e_b] of the forward block-Jacobi selectors
    W_{L,b} (Sec. 6): s_b = 2 + (b-1) w, e_b = min(2 + b w, N_g + 1), w = N_1 by default."""
    _, _, n_g = counts(n1, n2)
    w = n1 if width is None else width
    p = math.ceil((n_g - 1) / w)
    return [(2 + (b - 1) * w, min(2 + b * w, n_g + 1)) for b in range(1, p + 1)]


def bj_backward_blocks(n1, n2, width=None):
    """Closed intervals of the backward selectors W_{U,b} (Sec. 6):
    [max(2, (1 + N_g) - b w), (1 + N_g) - (b-1) w]."""
    _, _, n_g = counts(n1, n2)
    w = n1 if width is None else width
    p = math.ceil((n_g - 1) / w)
    return [(max(2, (1 + n_g) - b * w), (1 + n_g) - (b - 1) * w) for b in range(1, p + 1)]


def num_partial_sweeps(n1, n2, width=None):
    """p = ceil((N_g - 1) / w): fewest closed width-w intervals covering [2, N_g + 1]."""
    _, _, n_g = counts(n1, n2)
    w = n1 if width is None else width
    return math.ceil((n_g - 1) / w)
