"""Pins of the oracle's out-degree counters and degree distribution (the
workload's out-degree histogram read literally, one counter per node):
the uniform initiator's degrees follow Binomial(m, 2^-k), a node's
out-degree follows Binomial(m, prod over its id bits of a+b or c+d) (the
row marginal, which tells the source from the destination when b != c),
counts add up to m over nodes and over degree bins, clipping fills the last
bin, and edge ranges add."""
from __future__ import annotations

import numpy as np
import pytest
from scipy import stats

import oracle


def _chi2_pvalue(observed: np.ndarray, expected: np.ndarray, min_expected: float = 5.0) -> float:
    """Chi-squared test with adjacent bins pooled until each expects >= min_expected."""
    obs, exp = [], []
    o_acc = e_acc = 0.0
    for o, e in zip(observed, expected):
        o_acc += o
        e_acc += e
        if e_acc >= min_expected:
            obs.append(o_acc)
            exp.append(e_acc)
            o_acc = e_acc = 0.0
    if e_acc > 0:
        obs[-1] += o_acc
        exp[-1] += e_acc
    obs, exp = np.array(obs), np.array(exp)
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    return float(stats.chi2.sf(chi2, len(obs) - 1))


def test_uniform_initiator_degrees_are_binomial():
    k, m = 14, 1 << 18
    t = oracle.build_table(0.25, 0.25, 0.25, 0.25, k, 256, oracle.VARIABLE)
    deg = oracle.out_degrees(t, 5, 0, m)
    dist = oracle.degree_distribution(deg, int(deg.max()) + 1)
    d = np.arange(dist.size)
    expected = (1 << k) * stats.binom.pmf(d, m, 2.0 ** -k)
    expected[-1] += (1 << k) * stats.binom.sf(d[-1], m, 2.0 ** -k)
    assert _chi2_pvalue(dist.astype(float), expected) > 1e-3


def test_node_degree_follows_the_row_marginal():
    # b != c: the source (row) marginal a+b = 0.8 differs from the column one a+c = 0.6
    q, k, m = (0.5, 0.3, 0.1, 0.1), 6, 1 << 20
    t = oracle.build_table(*q, k, 1024, oracle.VARIABLE)
    deg = oracle.out_degrees(t, 11, 0, m).astype(float)
    v = np.arange(1 << k)
    ones = np.array([bin(x).count("1") for x in v])
    p = (q[0] + q[1]) ** (k - ones) * (q[2] + q[3]) ** ones
    z = (deg - m * p) / np.sqrt(m * p * (1 - p))
    assert np.abs(z).max() < 5.0
    # the column marginal does not fit: the counters are indexed by source
    pc = (q[0] + q[2]) ** (k - ones) * (q[1] + q[3]) ** ones
    zc = (deg - m * pc) / np.sqrt(m * pc * (1 - pc))
    assert np.abs(zc).max() > 20.0


@pytest.mark.parametrize("q,k,bound,mode", [((0.57, 0.19, 0.19, 0.05), 16, 4096, oracle.VARIABLE),
                                            ((0.45, 0.22, 0.22, 0.11), 12, 256, oracle.FIXED)])
def test_counts_add_up_and_clip(q, k, bound, mode):
    m = 300_001
    t = oracle.build_table(*q, k, bound, mode)
    deg = oracle.out_degrees(t, 3, 77, m, slice_edges=1 << 16)
    assert deg.size == 1 << k and int(deg.sum()) == m
    top = int(deg.max())
    dist = oracle.degree_distribution(deg, top)
    assert int(dist.sum()) == 1 << k
    assert int((np.arange(top + 1, dtype=np.uint64) * dist).sum()) == m
    clip = oracle.degree_distribution(deg, 8)
    assert np.array_equal(clip[:8], dist[:8]) and int(clip[8]) == int(dist[8:].sum())
    # brute force on the first edges: direct count of sources
    src, _ = oracle.generate(t, 3, 77, 5000)
    brute = np.zeros(1 << k, np.uint64)
    for s in src:
        brute[int(s)] += 1
    assert np.array_equal(oracle.out_degrees(t, 3, 77, 5000), brute)


def test_edge_ranges_add():
    t = oracle.build_table(0.57, 0.19, 0.19, 0.05, 18, 1024, oracle.VARIABLE)
    whole = oracle.out_degrees(t, 9, 2 ** 40 - 1000, 200_000)
    parts = oracle.out_degrees(t, 9, 2 ** 40 - 1000, 70_001) + oracle.out_degrees(t, 9, 2 ** 40 - 1000 + 70_001, 129_999)
    assert np.array_equal(whole, parts)
