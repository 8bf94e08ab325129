"""Pins of the oracle's partitioned generator (Sec. 3, reading R20) against
what probability fixes: the binomial law of every split (exact pmf from
scipy), the multinomial law of a node's four-way split (enumerated), the
R-MAT law of the whole partitioned graph (closed-form cell probabilities),
and the communication-free property (any row range reproduces the counts of
the full computation)."""
from __future__ import annotations

import itertools
import math

import numpy as np
import pytest
from scipy import stats

import oracle

G500 = (0.57, 0.19, 0.19, 0.05)


def _chi2_p(observed: np.ndarray, expected: np.ndarray) -> float:
    """Pearson chi-squared p-value after merging cells with expectation < 5."""
    order = np.argsort(expected)
    obs, exp = observed[order].astype(float), expected[order].astype(float)
    mo, me, acc_o, acc_e = [], [], 0.0, 0.0
    for o, e in zip(obs, exp):
        acc_o += o
        acc_e += e
        if acc_e >= 5:
            mo.append(acc_o)
            me.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0 and me:
        mo[-1] += acc_o
        me[-1] += acc_e
    mo, me = np.array(mo), np.array(me)
    chi2 = float(((mo - me) ** 2 / me).sum())
    return float(stats.chi2.sf(chi2, len(me) - 1))


@pytest.mark.parametrize("n,p", [
    (20, 0.3),            # inversion
    (200, 0.1),           # inversion (n p = 20)
    (100, 0.5),           # BTPE, symmetric
    (1000, 0.05),         # BTPE (n p = 50)
    (10 ** 6, 0.3),       # BTPE, large n
    (10 ** 9, 1e-8),      # inversion with large n
    (2 ** 40, 0.19),      # BTPE, huge n
    (500, 0.8),           # p > 1/2 drawn as n - Bin(n, 1 - p)
])
def test_binomial_draws_follow_the_binomial_law(n, p):
    draws = np.array([oracle.binomial(7, i, i // 3, 3, n, p) for i in range(6000)], dtype=np.int64)
    mean, sd = n * p, math.sqrt(n * p * (1 - p))
    lo, hi = int(max(0, math.floor(mean - 8 * sd))), int(min(n, math.ceil(mean + 8 * sd)))
    assert draws.min() >= lo and draws.max() <= hi
    ks = np.arange(lo, hi + 1)
    if len(ks) > 5000:   # huge n: compare on 60 equiprobable quantile bins of the exact law
        edges = stats.binom.ppf(np.linspace(0, 1, 61)[1:-1], n, p)
        obs = np.bincount(np.searchsorted(edges, draws, side="right"), minlength=60)
        cdf = np.concatenate([[0.0], stats.binom.cdf(edges, n, p), [1.0]])
        exp = np.diff(cdf) * len(draws)
    else:
        obs = np.bincount(draws - lo, minlength=len(ks))
        exp = stats.binom.pmf(ks, n, p) * len(draws)
    assert _chi2_p(obs, exp) > 1e-4
    assert abs(draws.mean() - mean) < 5 * sd / math.sqrt(len(draws)) + 1e-9


def test_binomial_degenerate_probabilities():
    assert oracle.binomial(1, 0, 0, 0, 12345, 0.0) == 0
    assert oracle.binomial(1, 0, 0, 0, 12345, 1.0) == 12345
    assert oracle.binomial(1, 0, 0, 0, 0, 0.4) == 0


def test_one_split_is_multinomial():
    """A single level (2 x 2 tiles) splits m edges Multinomial(m; a, b, c, d)."""
    m, runs = 8, 4000
    t = oracle.build_table(*G500, 10, 256, oracle.VARIABLE)
    seen = {}
    for s in range(runs):
        c = tuple(int(x) for x in oracle.partition_counts(t, 1000 + s, m, 1).ravel())
        seen[c] = seen.get(c, 0) + 1
    cells = [c for c in itertools.product(range(m + 1), repeat=4) if sum(c) == m]
    pmf = np.array([stats.multinomial.pmf(c, m, G500) for c in cells])
    obs = np.array([seen.get(c, 0) for c in cells])
    assert sum(seen.values()) == runs and set(seen) <= set(cells)
    assert _chi2_p(obs, pmf * runs) > 1e-4


def test_partitioned_graph_has_the_rmat_law():
    """k = 3 with 2 x 2 tiles: the cell frequencies of the whole partitioned
    graph match prod_levels q(row bit, col bit) (Sec. 1)."""
    k, tb, m = 3, 1, 1 << 16
    q = (0.45, 0.22, 0.22, 0.11)
    t = oracle.build_table(*q, k, 64, oracle.VARIABLE)
    counts, s, d = oracle.generate_partition(t, 5, m, tb)
    assert int(counts.sum()) == m == len(s)
    obs = np.bincount(s.astype(np.int64) * 8 + d, minlength=64)
    exp = np.zeros(64)
    for r in range(8):
        for c in range(8):
            pr = 1.0
            for lvl in range(k):
                rb, cb = (r >> (k - 1 - lvl)) & 1, (c >> (k - 1 - lvl)) & 1
                pr *= q[2 * rb + cb]
            exp[r * 8 + c] = pr * m
    assert _chi2_p(obs, exp) > 1e-4


@pytest.mark.parametrize("k,tb,m", [(12, 3, 100_000), (20, 6, 10 ** 7), (34, 5, 2 ** 40), (40, 15, 123_456)])
def test_counts_sum_and_row_partitions_agree(k, tb, m):
    """The counts sum to m; any range of tile rows, computed alone, equals
    that slice of the full computation (no communication needed)."""
    t = oracle.build_table(*G500, k, 1000, oracle.VARIABLE)
    full = oracle.partition_counts(t, 9, m, tb)
    assert int(full.sum()) == m
    rows = 1 << tb
    for r0, r1 in ((0, 1), (rows // 3, rows // 2 + 1), (rows - 1, rows)):
        part = oracle.partition_counts(t, 9, m, tb, r0, r1)
        assert np.array_equal(part, full[r0:r1])


def test_tile_edges_carry_their_tile():
    k, tb = 14, 3
    t = oracle.build_table(*G500, k, 512, oracle.VARIABLE)
    counts, s, d = oracle.generate_partition(t, 2, 50_000, tb, 2, 5)
    kk = k - tb
    rows = np.repeat(np.repeat(np.arange(2, 5), 1 << tb), counts.ravel().astype(np.int64))
    cols = np.repeat(np.tile(np.arange(1 << tb), 3), counts.ravel().astype(np.int64))
    assert np.array_equal(s >> kk, rows) and np.array_equal(d >> kk, cols)


def test_partition_rejects_bad_arguments():
    t = oracle.build_table(*G500, 10, 256, oracle.VARIABLE)
    for args in ((0, 0, 1), (10, 0, 1), (3, 4, 4), (3, 0, 9)):
        with pytest.raises(oracle.OracleError):
            oracle.partition_counts(t, 1, 100, *args)
    with pytest.raises(oracle.OracleError):
        oracle.partition_counts(t, 1, 2 ** 53 + 1, 3)
