"""Pins of the oracle's K x K stochastic Kronecker tables (Sec. 3, reading
R21) against what the mathematics fixes: K = 2 is R-MAT itself (the pinned
R-MAT oracle, bit for bit); path probabilities are exact products of the
initiator's entries; a variable table is a complete K^2-ary prefix code; its
expanded set is the first t nodes of the tie order (brute force); the sampled
edges follow the Kronecker cell law prod P[i_l][j_l]."""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle

P3 = [0.3, 0.1, 0.05, 0.1, 0.2, 0.05, 0.05, 0.05, 0.1]
# dyadic: every product is exact in binary floating point
P3_DYADIC = [8 / 32, 4 / 32, 2 / 32, 4 / 32, 6 / 32, 1 / 32, 2 / 32, 1 / 32, 4 / 32]
P4_DYADIC = [x / 64 for x in (8, 4, 4, 2, 4, 8, 2, 4, 4, 2, 6, 2, 2, 4, 2, 6)]


def _chi2_p(obs, exp):
    keep = exp >= 5
    o = np.concatenate([obs[keep], [obs[~keep].sum()]]) if (~keep).any() else obs[keep]
    e = np.concatenate([exp[keep], [exp[~keep].sum()]]) if (~keep).any() else exp[keep]
    return float(stats.chi2.sf(((o - e) ** 2 / e).sum(), len(e) - 1))


@pytest.mark.parametrize("q,k,bound,mode", [((0.57, 0.19, 0.19, 0.05), 26, 4096, oracle.VARIABLE),
                                            ((0.57, 0.19, 0.19, 0.05), 16, 256, oracle.FIXED),
                                            ((0.45, 0.22, 0.22, 0.11), 34, 20_000, oracle.VARIABLE),
                                            ((0.25, 0.25, 0.25, 0.25), 12, 5000, oracle.VARIABLE),
                                            ((0.9, 0.025, 0.025, 0.05), 64, 8192, oracle.VARIABLE),
                                            ((0.6, 0.0, 0.3, 0.1), 10, 64, oracle.FIXED)])
def test_k2_is_rmat(q, k, bound, mode):
    a = oracle.build_table(*q, k, bound, mode)
    b = oracle.kron_build_table(list(q), 2, k, bound, mode)
    for f in ("length", "code", "row", "col", "thr", "alias", "w"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert np.array_equal(a.p.view(np.uint64), b.p.view(np.uint64))
    e0 = 2 ** 32 - 500 if k > 32 else 3
    sa, da = oracle.generate(a, 9, e0, 3000)
    sb, db = oracle.generate(b, 9, e0, 3000)
    assert np.array_equal(sa, sb) and np.array_equal(da, db)


@pytest.mark.parametrize("P,K,bound", [(P3_DYADIC, 3, 700), (P4_DYADIC, 4, 3000)])
def test_probabilities_are_exact_products_and_a_complete_code(P, K, bound):
    t = oracle.kron_build_table(P, K, 12, bound, oracle.VARIABLE)
    L = K * K
    fr = [Fraction(x) for x in P]
    total = Fraction(0)
    kraft = 0
    for j in range(t.n_items):
        code, depth = int(t.code[j]), int(t.length[j])
        digits = [(code // L ** pos) % L for pos in range(depth)][::-1]   # root-most first
        exact = Fraction(1)
        for x in digits:
            exact *= fr[x]
        assert Fraction(float(t.p[j])) == exact
        total += exact
        kraft += L ** (t.cap - depth)
        # row / column values: the digits' row and column parts, root-most most significant
        r = c = 0
        for x in digits:
            r, c = r * K + x // K, c * K + x % K
        assert (int(t.row[j]), int(t.col[j])) == (r, c)
    assert total == 1 and kraft == L ** t.cap
    assert t.n_items == 1 + (L - 1) * ((t.n_items - 1) // (L - 1))


def test_expanded_set_is_the_first_t_nodes_of_the_order():
    """Brute force for K = 3: sort every node of depth <= 3 by (p desc,
    depth asc, code asc), expand the first t, compare the leaves."""
    K, L = 3, 9
    for bound in (10, 30, 60, 100):
        t = oracle.kron_build_table(P3, K, 12, bound, oracle.VARIABLE)
        n_exp = (t.n_items - 1) // (L - 1)
        nodes = []
        for depth in range(0, 4):
            for digits in itertools.product(range(L), repeat=depth):
                counts = [0] * L
                for x in digits:
                    counts[x] += 1
                p = 1.0
                for x in range(L):
                    for _ in range(counts[x]):
                        p = p * P3[x]
                code = 0
                for x in digits:
                    code = code * L + x
                nodes.append((-p, depth, code))
        nodes.sort()
        expanded = set((d, c) for _, d, c in nodes[:n_exp])
        # the enumeration is deep enough: expanded nodes have depth <= 2 and every
        # depth-3 node is less probable than the last expanded one
        assert max(d for d, _ in expanded) <= 2
        assert max(-np_ for np_, d, _ in nodes if d == 3) < -nodes[n_exp - 1][0]
        leaves = set()
        for d, c in expanded:
            for x in range(L):
                if (d + 1, c * L + x) not in expanded:
                    leaves.add((d + 1, c * L + x))
        got = set(zip(t.length.astype(int)[:t.n_items], t.code.astype(int)[:t.n_items]))
        assert got == leaves


@pytest.mark.parametrize("P,K", [(P3, 3), (P4_DYADIC, 4)])
def test_edges_follow_the_kronecker_law(P, K):
    k, m = 2, 1 << 16
    t = oracle.kron_build_table(P, K, k, 200, oracle.VARIABLE)
    s, d = oracle.generate(t, 4, 0, m)
    n = K ** k
    assert s.max() < n and d.max() < n
    obs = np.bincount(s.astype(np.int64) * n + d, minlength=n * n).astype(float)
    exp = np.zeros(n * n)
    for r in range(n):
        for c in range(n):
            pr = 1.0
            for lvl in range(k):
                i, j = (r // K ** (k - 1 - lvl)) % K, (c // K ** (k - 1 - lvl)) % K
                pr *= P[i * K + j]
            exp[r * n + c] = pr * m
    assert _chi2_p(obs, exp) > 1e-4


def test_ids_stay_below_K_to_the_k():
    t = oracle.kron_build_table(P3, 3, 40, 4000, oracle.VARIABLE)    # 3^40 < 2^64
    s, d = oracle.generate(t, 1, 2 ** 40, 20_000)
    assert int(s.max()) < 3 ** 40 and int(d.max()) < 3 ** 40
    assert int(s.max()) > 3 ** 39   # the leading digit is used
    t5 = oracle.kron_build_table([1 / 25] * 25, 5, 13, 1000, oracle.FIXED)
    s5, d5 = oracle.generate(t5, 2, 0, 50_000)
    assert int(max(s5.max(), d5.max())) < 5 ** 13


def test_invalid_initiators():
    for P, K, k, bound, mode in [([1.0], 1, 5, 100, 1), ([1 / 289] * 289, 17, 5, 1000, 1),
                                 ([0.2] * 9, 3, 5, 100, 1), (P3, 3, 41, 100, 1),
                                 (P3, 3, 5, 9, oracle.VARIABLE), (P3, 3, 5, 8, oracle.FIXED),
                                 ([0.5, -0.1, 0.3, 0.3], 2, 5, 100, 1)]:
        with pytest.raises(oracle.OracleError):
            oracle.kron_build_table(P, K, k, bound, mode)
    t = oracle.kron_build_table(P3, 3, 10, 100, oracle.VARIABLE)
    with pytest.raises(oracle.OracleError):
        oracle.generate(t, 1, 0, 10, flags=oracle.SCRAMBLE)
