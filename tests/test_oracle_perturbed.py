"""Pins of the oracle's perturbed tables (Sec. 3, reading R22): with no
perturbation they are the base table and the plain stream; every parameter
set is a normalised perturbation within the stated band; edge e is exactly
the plain edge of table e mod P; the whole stream follows the mixture of
the tables' closed-form R-MAT laws."""
from __future__ import annotations

import numpy as np
import pytest
from scipy import stats

import oracle

G500 = (0.57, 0.19, 0.19, 0.05)


def test_no_perturbation_is_the_base_table_and_stream():
    base = oracle.build_table(*G500, 20, 4096, oracle.VARIABLE)
    tabs = oracle.build_perturbed_tables(*G500, 20, 4096, oracle.VARIABLE, 4, 0.0, 99)
    for t in tabs:
        for f in ("length", "code", "row", "col", "thr", "alias", "w"):
            assert np.array_equal(getattr(t, f), getattr(base, f))
    s, d = oracle.generate_set(tabs, 5, 1000, 4000)
    bs, bd = oracle.generate(base, 5, 1000, 4000)
    assert np.array_equal(s, bs) and np.array_equal(d, bd)


@pytest.mark.parametrize("q", [G500, (0.45, 0.22, 0.22, 0.11), (0.6, 0.0, 0.3, 0.1)])
@pytest.mark.parametrize("eps", [0.05, 0.3, 0.9])
def test_parameters_are_normalised_perturbations(q, eps):
    P = oracle.perturbed_params(*q, 16, eps, 7)
    assert np.allclose(P.sum(axis=1), 1.0, rtol=0, atol=1e-15)
    qq = np.array(q)
    for row in P:
        nz = qq > 0
        assert np.all(row[~nz] == 0)
        ratio = row[nz] / qq[nz]
        assert np.all(ratio >= (1 - eps) / (1 + eps) - 1e-12) and np.all(ratio <= (1 + eps) / (1 - eps) + 1e-12)
    assert len({tuple(r) for r in P}) == 16          # distinct tables
    assert not np.array_equal(P, oracle.perturbed_params(*q, 16, eps, 8))


def test_edge_e_comes_from_table_e_mod_P():
    tabs = oracle.build_perturbed_tables(*G500, 24, 1000, oracle.VARIABLE, 8, 0.2, 3)
    e0, m = 2 ** 32 - 77, 4000
    s, d = oracle.generate_set(tabs, 11, e0, m)
    for i, t in enumerate(tabs):
        ts, td = oracle.generate(t, 11, e0, m)
        sel = (np.arange(e0, e0 + m, dtype=np.uint64) % 8) == i
        assert np.array_equal(s[sel], ts[sel]) and np.array_equal(d[sel], td[sel])


def test_stream_follows_the_mixture_law():
    k, m, n_t = 2, 1 << 16, 4
    P = oracle.perturbed_params(*G500, n_t, 0.5, 21)
    tabs = [oracle.build_table(*q, k, 64, oracle.VARIABLE) for q in P]
    s, d = oracle.generate_set(tabs, 2, 0, m)
    obs = np.bincount(s.astype(np.int64) * 4 + d, minlength=16).astype(float)
    exp = np.zeros(16)
    for q in P:
        for r in range(4):
            for c in range(4):
                pr = 1.0
                for lvl in range(k):
                    rb, cb = (r >> (k - 1 - lvl)) & 1, (c >> (k - 1 - lvl)) & 1
                    pr *= q[2 * rb + cb]
                exp[r * 4 + c] += pr * m / n_t
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    assert stats.chi2.sf(chi2, 15) > 1e-4


def test_bad_perturbation_arguments():
    for n, eps in ((3, 0.1), (128, 0.1), (0, 0.1), (4, -0.1), (4, 1.0), (4, float("nan"))):
        with pytest.raises(oracle.OracleError):
            oracle.perturbed_params(*G500, n, eps, 1)
