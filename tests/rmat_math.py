"""Closed forms and brute-force references used to pin the oracle.

Everything here is written from the definitions in the paper (Sec. 1, the
R-MAT process; Sec. 2, the path table and the sampling loop), independently
of the oracle's C code, and is used only by the tests.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np

LETTER_BITS = {0: (0, 0), 1: (0, 1), 2: (1, 0), 3: (1, 1)}  # a, b, c, d -> (row, col)


def cell_probabilities(q, k: int) -> np.ndarray:
    """Closed form of Sec. 1: P(edge = (r, c)) = prod_t q[2 r_t + c_t] over the
    k bit positions.  Returns a (2^k, 2^k) array indexed [row, col]."""
    P = np.ones((1, 1))
    Q = np.array([[q[0], q[1]], [q[2], q[3]]], dtype=np.float64)
    for _ in range(k):
        P = np.kron(P, Q)
    return P


def naive_rmat(q, k: int, m: int, rng: np.random.Generator):
    """The per-bit recursive process of Sec. 1: k quadrant choices per edge,
    each fixing one row bit and one column bit, most significant first."""
    cum = np.cumsum(np.asarray(q, dtype=np.float64))
    row = np.zeros(m, np.uint64)
    col = np.zeros(m, np.uint64)
    for _ in range(k):
        u = rng.random(m)
        letter = np.searchsorted(cum, u, side="right").clip(0, 3)
        row = (row << np.uint64(1)) | (letter >> 1).astype(np.uint64)
        col = (col << np.uint64(1)) | (letter & 1).astype(np.uint64)
    return row, col


def letters_of(code: int, depth: int):
    """Root-most letter first."""
    return [(code >> (2 * (depth - 1 - i))) & 3 for i in range(depth)]


def exact_product(q_frac, letters) -> Fraction:
    p = Fraction(1)
    for x in letters:
        p *= q_frac[x]
    return p


def edge_law_from_table(length, row, col, weights, n_items: int, k: int) -> np.ndarray:
    """Exact law of the first k letters of a stream of iid items drawn with
    probability weights[j] (Sec. 2 sampling loop, leftovers discarded).
    Brute force over item sequences; only for tiny k.  Returns (2^k, 2^k)."""
    out = np.zeros((1 << k, 1 << k))
    items = [(int(length[j]), int(row[j]), int(col[j]), float(weights[j])) for j in range(n_items)
             if weights[j] > 0]

    def rec(filled, r, c, prob):
        for (L, rb, cb, w) in items:
            take = min(L, k - filled)
            nr = (r << take) | (rb >> (L - take))
            nc = (c << take) | (cb >> (L - take))
            if filled + take >= k:
                out[nr, nc] += prob * w
            else:
                rec(filled + take, nr, nc, prob * w)

    rec(0, 0, 0, 1.0)
    return out


def samples_per_edge_law(length, weights, n_items: int, k: int, nmax: int = 64) -> np.ndarray:
    """Exact law of N = number of samples until at least k letters are known,
    for iid item lengths.  DP over the filled count."""
    lw = {}
    for j in range(n_items):
        if weights[j] > 0:
            lw[int(length[j])] = lw.get(int(length[j]), 0.0) + float(weights[j])
    state = np.zeros(k)
    state[0] = 1.0
    law = np.zeros(nmax + 1)
    for n in range(1, nmax + 1):
        nxt = np.zeros(k)
        for f in range(k):
            if state[f] == 0.0:
                continue
            for L, w in lw.items():
                if f + L >= k:
                    law[n] += state[f] * w
                else:
                    nxt[f + L] += state[f] * w
        state = nxt
    return law


def full_trees(t: int, cap: int):
    """All sets of t expanded nodes (ancestor-closed, containing the root) of
    the 4-ary quadrant tree with nodes at depth < cap expandable.  Nodes are
    (depth, code)."""
    def grow(expanded, frontier_start):
        if len(expanded) == t:
            yield frozenset(expanded)
            return
        # candidate children of expanded nodes not yet expanded, in a canonical
        # order, to enumerate each set once: only add nodes greater than the
        # last added one
        cands = set()
        for (D, code) in expanded:
            if D + 1 < cap:
                for x in range(4):
                    cands.add((D + 1, code * 4 + x))
        cands -= set(expanded)
        for c in sorted(cands):
            if c > frontier_start:
                yield from grow(expanded + [c], c)

    yield from grow([(0, 0)], (0, 0))


def leaves_of(expanded):
    out = []
    for (D, code) in expanded:
        for x in range(4):
            ch = (D + 1, code * 4 + x)
            if ch not in expanded:
                out.append(ch)
    return out


def entropy_bits(q) -> float:
    return -sum(x * np.log2(x) for x in q if x > 0)


def all_nodes(cap: int):
    for D in range(cap):
        for code in range(4 ** D):
            yield (D, code)


def count_letters(code: int, depth: int):
    n = [0, 0, 0, 0]
    for x in letters_of(code, depth):
        n[x] += 1
    return n


def combos(n: int, r: int):
    return itertools.combinations(range(n), r)
