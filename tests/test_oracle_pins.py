"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (tests/golden/, each with its citation), closed forms of the R-MAT
process, exact rational arithmetic, brute force over tiny instances, and a
third-party Philox4x32-10 implementation.
"""
from __future__ import annotations

import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle
import rmat_math as rm

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")

G500 = (0.57, 0.19, 0.19, 0.05)
SKEW = (0.9, 0.025, 0.025, 0.05)
CFG3 = (0.45, 0.22, 0.22, 0.11)
DYADIC = (9 / 16, 3 / 16, 3 / 16, 1 / 16)  # sums to exactly 1 in binary


def _dirichlet(seed):
    q = np.random.default_rng(seed).dirichlet([4, 2, 2, 1])
    q[3] = 1.0 - q[0] - q[1] - q[2]
    return tuple(float(x) for x in q)


def _golden_rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


# ---------------------------------------------------------------------------
# Philox4x32-10 against rocRAND's engine (third-party black box, host side)
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    out = tmp_path_factory.mktemp("rocrand") / "philox_ref"
    subprocess.check_call([hipcc, "-O1", "-I/opt/rocm/include", "--offload-arch=gfx950",
                           os.path.join(HERE, "philox_rocrand_ref.cpp"), "-o", str(out)],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return str(out)


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(2024)
    cases = [(0, 0, 0), (1, 0, 0), (7, 1, 0), (7, 123456789, 1), (2**64 - 1, 2**64 - 1, 5),
             (0x0123456789ABCDEF, 2**32 + 5, 3)]
    for _ in range(300):
        cases.append((int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2)),
                      int(rng.integers(0, 2**63)), int(rng.integers(0, 16))))
    inp = "".join(f"{s} {e} {j}\n" for s, e, j in cases)
    res = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True)
    lines = res.stdout.strip().splitlines()
    assert len(lines) == len(cases)
    for (s, e, j), ln in zip(cases, lines):
        ref = [int(h, 16) for h in ln.split()]
        got = oracle.philox4x32_10([e & 0xFFFFFFFF, e >> 32, j, 0], [s & 0xFFFFFFFF, s >> 32])
        assert list(got) == ref, (s, e, j)


# ---------------------------------------------------------------------------
# Table construction
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("row", _golden_rows("fig1_table_sizes.txt"))
def test_fig1_table_sizes(row):
    bound, var_size, fixed_size = int(row[0]), int(row[1]), row[2]
    if bound > 2**22:
        pytest.skip("largest Fig. 1 bounds are covered by test_fig1_table_sizes_large")
    t = oracle.build_table(*G500, 30, bound, oracle.VARIABLE)
    assert t.n_items == var_size
    if fixed_size != "-":
        tf = oracle.build_table(*G500, 30, bound, oracle.FIXED)
        assert tf.n_items == int(fixed_size)


@pytest.mark.slow
def test_fig1_table_sizes_large():
    for row in _golden_rows("fig1_table_sizes.txt"):
        bound, var_size = int(row[0]), int(row[1])
        if bound > 2**22:
            t = oracle.build_table(*G500, 30, bound, oracle.VARIABLE)
            assert t.n_items == var_size
            assert int(t.w.sum()) == 2**32 and np.all(np.abs(t.w[: t.n_items] - t.p[: t.n_items] * 2.0**32) < 1)
            del t


@pytest.mark.parametrize("row", _golden_rows("skewed_bits_per_sample.txt"))
def test_skewed_bits_per_sample(row):
    a, b, c, d = map(float, row[:4])
    k, mode, bound = int(row[4]), row[5], int(row[6])
    printed, decimals = float(row[7]), int(row[8])
    t = oracle.build_table(a, b, c, d, k, bound, oracle.VARIABLE if mode == "variable" else oracle.FIXED)
    # the paper's figure, printed to `decimals` places
    assert abs(t.expected_len - printed) <= 0.5 * 10.0 ** (-decimals) + 1e-12


def test_entropy_identity_and_speedup():
    """Sec. 2: a sample of the variable table yields >= log2(1/pmax) bits; each
    letter carries H bits.  For a complete prefix code of iid letters the leaf
    entropy equals E[L] * H exactly (Wald), which fixes that leaf probabilities
    are products of their letters.  The golden file pins H and 2/H."""
    (a, b, c, d, H, ratio), = [tuple(map(float, r)) for r in _golden_rows("graph500_entropy.txt")]
    q = (a, b, c, d)
    Hq = rm.entropy_bits(q)
    assert round(Hq, 2) == H and round(2 / Hq, 2) == ratio
    for bound in (4096, 65536, 1 << 20):
        t = oracle.build_table(*q, 40, bound, oracle.VARIABLE)
        p = t.p[: t.n_items]
        L = t.length[: t.n_items].astype(np.float64)
        leaf_entropy = float(-(p * np.log2(p)).sum())
        assert abs(leaf_entropy - Hq * float((p * L).sum())) < 1e-9
        assert leaf_entropy >= np.log2(1.0 / p.max()) - 1e-12
    # fixed length l = 10 (2^20 entries) gives exactly 10 letters; the variable
    # table of the same bound beats it by a factor close to 2/H
    tf = oracle.build_table(*q, 40, 1 << 20, oracle.FIXED)
    assert tf.expected_len == 10.0
    gain = t.expected_len / tf.expected_len
    assert 1.15 < gain <= 2 / Hq + 0.02


@pytest.mark.parametrize("q", [G500, SKEW, CFG3, DYADIC, _dirichlet(1), _dirichlet(2)])
@pytest.mark.parametrize("bound,mode", [(256, oracle.FIXED), (4096, oracle.VARIABLE), (300, oracle.VARIABLE),
                                        (65536, oracle.VARIABLE)])
def test_leaves_form_complete_prefix_code(q, bound, mode):
    t = oracle.build_table(*q, 30, bound, mode)
    n = t.n_items
    D = t.length[:n].astype(np.int64)
    # Kraft equality of a complete 4-ary prefix code
    assert int(np.sum(4 ** (15 - D))) == 4 ** 15
    # tree order: left-aligned codes strictly increasing
    lac = t.code[:n].astype(np.int64) << (2 * (15 - D))
    assert np.all(np.diff(lac) > 0)
    # padding
    assert np.all(t.length[n:] == 0) and np.all(t.w[n:] == 0)
    # row/col bits are the letters' bits (Sec. 1: a upper-left, b upper-right, ...)
    for j in range(0, n, max(1, n // 200)):
        lets = rm.letters_of(int(t.code[j]), int(D[j]))
        r = c = 0
        for x in lets:
            r = (r << 1) | rm.LETTER_BITS[x][0]
            c = (c << 1) | rm.LETTER_BITS[x][1]
        assert (int(t.row[j]), int(t.col[j])) == (r, c)


@pytest.mark.parametrize("q", [G500, SKEW, DYADIC, _dirichlet(3)])
def test_leaf_probability_is_product_of_letters(q):
    """Sec. 2: a path's probability is the product of its letters.  Checked in
    exact rational arithmetic; each float product may round once per letter."""
    t = oracle.build_table(*q, 30, 4096, oracle.VARIABLE)
    qf = [Fraction(x) for x in q]
    total = Fraction(0)
    for j in range(t.n_items):
        exact = rm.exact_product(qf, rm.letters_of(int(t.code[j]), int(t.length[j])))
        total += exact
        got = Fraction(float(t.p[j]))
        assert abs(got - exact) <= exact * Fraction(int(t.length[j]) + 1, 2**53)
    s = sum(qf)
    if s == 1:
        assert total == 1  # complete prefix code of a distribution summing to 1
    else:
        assert abs(float(total) - 1.0) < 1e-12


@pytest.mark.parametrize("k,bound", [(3, 12), (4, 20), (5, 30), (3, 40), (4, 70)])
@pytest.mark.parametrize("q", [G500, SKEW, (0.25, 0.25, 0.25, 0.25), _dirichlet(5), (0.6, 0.0, 0.3, 0.1)])
def test_expansion_is_first_t_nodes_in_order(k, bound, q):
    """The priority queue of Sec. 2 with readings R2-R4 equals: sort every
    expandable node (depth < min(15, k)) by (probability desc, depth asc, code
    asc) and expand the first t = ceil((bound - 4) / 3) of them."""
    cap = min(15, k)
    t = oracle.build_table(*q, k, bound, oracle.VARIABLE)
    nodes = []
    for (D, code) in rm.all_nodes(cap):
        p = oracle.canonical_product(q, rm.count_letters(code, D))
        nodes.append((-p, D, code))
    nodes.sort()
    n_expand = min(-(-(bound - 4) // 3), len(nodes))
    expanded = {(D, code) for (_, D, code) in nodes[:n_expand]}
    want = sorted(rm.leaves_of(expanded), key=lambda v: v[1] << (2 * (15 - v[0])))
    got = [(int(t.length[j]), int(t.code[j])) for j in range(t.n_items)]
    assert got == want


@pytest.mark.parametrize("n_exp", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("q", [G500, SKEW, _dirichlet(7), _dirichlet(8)])
def test_table_maximises_minimum_probability(n_exp, q):
    """Sec. 2 claims the queue produces the entry set that maximises the
    minimum entry probability.  Brute force over every 4-ary tree with the
    same number of expansions."""
    k = 8
    t = oracle.build_table(*q, k, 1 + 3 * n_exp + 3, oracle.VARIABLE)
    assert t.n_items == 1 + 3 * n_exp
    qf = [Fraction(x) for x in q]
    ours = min(rm.exact_product(qf, rm.letters_of(int(t.code[j]), int(t.length[j]))) for j in range(t.n_items))
    best = Fraction(0)
    for tree in set(rm.full_trees(n_exp, min(15, k))):
        mn = min(rm.exact_product(qf, rm.letters_of(code, D)) for (D, code) in rm.leaves_of(tree))
        best = max(best, mn)
    assert ours == best


def test_tie_break_reading():
    """Reading R3 on a fully tied alphabet: bound 8 expands the root and then
    the lowest-code child, a."""
    t = oracle.build_table(0.25, 0.25, 0.25, 0.25, 10, 8, oracle.VARIABLE)
    got = [(int(t.length[j]), int(t.code[j])) for j in range(t.n_items)]
    assert got == [(2, 0), (2, 1), (2, 2), (2, 3), (1, 1), (1, 2), (1, 3)]


def test_depth_cap_is_min_15_k():
    t = oracle.build_table(*SKEW, 40, 1 << 16, oracle.VARIABLE)
    assert t.length[: t.n_items].max() == 15
    t = oracle.build_table(*SKEW, 9, 1 << 16, oracle.VARIABLE)
    assert t.length[: t.n_items].max() == 9
    # every expandable node expanded: 4^k leaves
    t = oracle.build_table(*G500, 3, 1 << 16, oracle.VARIABLE)
    assert t.n_items == 64 and np.all(t.length[:64] == 3)


# ---------------------------------------------------------------------------
# Quantisation and alias table
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("q", [G500, SKEW, CFG3, DYADIC, _dirichlet(11), (1.0, 0.0, 0.0, 0.0), (0.5, 0.5, 0.0, 0.0)])
@pytest.mark.parametrize("bound,mode", [(4, oracle.FIXED), (256, oracle.FIXED), (5, oracle.VARIABLE),
                                        (4096, oracle.VARIABLE), (65536, oracle.VARIABLE), (1000, oracle.VARIABLE)])
def test_alias_table_conserves_mass(q, bound, mode):
    t = oracle.build_table(*q, 34, bound, mode)
    C = t.capacity
    nb = t.n_buckets
    assert nb == 1 << t.bucket_bits and nb >= t.n_items > nb // 2
    assert C << t.bucket_bits == 2**32
    w = t.w
    assert int(w.sum()) == 2**32 and np.all(w >= 0)
    # weights are the probabilities scaled to 2^32, rounded up or down (never
    # off by a unit or more), and an item with a larger fractional part is
    # never rounded down while one with a smaller part is rounded up
    x = t.p[: t.n_items] * 2.0**32
    wi = w[: t.n_items]
    assert np.all(np.abs(wi - x) < 1.0)
    frac = x - np.floor(x)
    up = wi > np.floor(x)
    if up.any() and (~up).any():
        assert frac[up].min() >= frac[~up].max()
    thr = t.thr.astype(np.int64)
    al = t.alias.astype(np.int64)
    selfb = al == np.arange(nb)
    assert np.all(thr[~selfb] < C) and np.all(thr[selfb] == C)
    # mass conservation: item j's share of all 2^32 words equals w_j
    mass = np.where(selfb, C, thr).astype(np.int64)
    np.add.at(mass, al[~selfb], C - thr[~selfb])
    assert np.array_equal(mass, w)


def test_alias_sampling_law_is_exact():
    """The sampled law is w / 2^32: enumerate every 32-bit word with the
    bucket/threshold rule for a small table."""
    t = oracle.build_table(*_dirichlet(21), 8, 20, oracle.VARIABLE)
    x = np.arange(0, 2**32, 4099, dtype=np.uint64)  # a lattice of words ...
    b = t.bucket_bits
    bucket = ((x >> np.uint64(4)) & np.uint64(t.n_buckets - 1)).astype(np.int64)
    f = (((x >> np.uint64(b + 4)) << np.uint64(4)) | (x & np.uint64(15))).astype(np.int64)
    item = np.where(f < t.thr[bucket], bucket, t.alias[bucket])
    freq = np.bincount(item, minlength=t.n_buckets) / len(x)
    # ... whose frequencies match w / 2^32 up to the lattice's resolution
    assert np.allclose(freq, t.w / 2.0**32, atol=2 * t.n_buckets * 4099 / 2**32)


# ---------------------------------------------------------------------------
# Sampling
# ---------------------------------------------------------------------------
def _strings_edge(t, seed, e):
    """Sec. 2 sampling loop written with bit strings: append sampled paths,
    output the first k characters (leftovers discarded per edge)."""
    k = t.k
    rs, cs = "", ""
    s = 0
    words = None
    while len(rs) < k:
        if s % 4 == 0:
            words = oracle.philox4x32_10([e & 0xFFFFFFFF, e >> 32, s // 4, 0], [seed & 0xFFFFFFFF, seed >> 32])
        x = int(words[s % 4])
        s += 1
        # bucket: the b bits above the lowest four; f: the other bits, in order
        bucket = (x >> 4) % t.n_buckets
        f = (x >> (t.bucket_bits + 4)) * 16 + x % 16
        item = bucket if f < int(t.thr[bucket]) else int(t.alias[bucket])
        for letter in rm.letters_of(int(t.code[item]), int(t.length[item])):
            rs += str(rm.LETTER_BITS[letter][0])
            cs += str(rm.LETTER_BITS[letter][1])
    return int(rs[:k], 2), int(cs[:k], 2), s


@pytest.mark.parametrize("q,k,bound,mode", [(G500, 16, 256, oracle.FIXED), (G500, 26, 4096, oracle.VARIABLE),
                                            (CFG3, 34, 65536, oracle.VARIABLE), (SKEW, 64, 8192, oracle.VARIABLE),
                                            (_dirichlet(4), 5, 64, oracle.FIXED), (G500, 1, 5, oracle.VARIABLE)])
def test_sampler_matches_string_definition(q, k, bound, mode):
    t = oracle.build_table(*q, k, bound, mode)
    seed = 0xDEADBEEF12345
    e0 = 2**32 - 20
    src, dst, ns = oracle.generate(t, seed, e0, 40, samples=True)
    for i in range(40):
        r, c, s = _strings_edge(t, seed, e0 + i)
        assert (int(src[i]), int(dst[i]), int(ns[i])) == (r, c, s)


@pytest.mark.parametrize("k", [2, 4, 6])
@pytest.mark.parametrize("q,bound,mode", [(G500, 4096, oracle.VARIABLE), (G500, 16, oracle.FIXED),
                                          (SKEW, 1000, oracle.VARIABLE), (_dirichlet(31), 300, oracle.VARIABLE),
                                          (_dirichlet(32), 64, oracle.FIXED)])
def test_chi_squared_against_closed_form(k, q, bound, mode):
    """Edge law vs Sec. 1's closed form P(r, c) = prod_t q(r_t, c_t)."""
    try:
        t = oracle.build_table(*q, k, bound, mode)
    except oracle.OracleError:
        assert mode == oracle.FIXED  # l > k is rejected
        return
    m = 1 << 21
    src, dst = oracle.generate(t, 99 + k, 12345, m, threads=8)
    cells = src.astype(np.int64) * (1 << k) + dst
    obs = np.bincount(cells, minlength=1 << (2 * k))
    exp = rm.cell_probabilities(q, k).ravel() * m
    keep = exp > 5
    chi2 = float(((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()) + float(obs[~keep].sum() - exp[~keep].sum())
    pval = stats.chi2.sf(chi2, int(keep.sum()) - 1)
    assert pval > 1e-5, (chi2, keep.sum())


def test_two_sample_against_naive_process():
    q = _dirichlet(41)
    k = 5
    t = oracle.build_table(*q, k, 200, oracle.VARIABLE)
    m = 1 << 20
    s1, d1 = oracle.generate(t, 5, 0, m, threads=8)
    s2, d2 = rm.naive_rmat(q, k, m, np.random.default_rng(5))
    c1 = np.bincount(s1.astype(np.int64) * 32 + d1, minlength=1024)
    c2 = np.bincount(s2.astype(np.int64) * 32 + d2.astype(np.int64), minlength=1024)
    keep = (c1 + c2) > 10
    table = np.vstack([c1[keep], c2[keep]])
    chi2, pval, _, _ = stats.chi2_contingency(table)
    assert pval > 1e-5


@pytest.mark.parametrize("q,k,bound,mode", [(G500, 3, 20, oracle.VARIABLE), (_dirichlet(51), 4, 16, oracle.VARIABLE),
                                            (SKEW, 4, 40, oracle.VARIABLE), (_dirichlet(52), 3, 64, oracle.FIXED)])
def test_exact_law_of_table_within_quantisation_bound(q, k, bound, mode):
    """Law of the first k letters of an iid item stream drawn from the
    quantised table equals the R-MAT law up to the quantisation error."""
    t = oracle.build_table(*q, k, bound, mode)
    law = rm.edge_law_from_table(t.length, t.row, t.col, t.w / 2.0**32, t.n_items, k)
    exact = rm.cell_probabilities(q, k)
    tv = 0.5 * np.abs(law - exact).sum()
    qerr = 0.5 * np.abs(t.w[: t.n_items] / 2.0**32 - t.p[: t.n_items]).sum()
    assert abs(law.sum() - 1.0) < 1e-12
    assert tv <= k * qerr + 1e-12


@pytest.mark.parametrize("q,k,bound,mode", [(G500, 26, 4096, oracle.VARIABLE), (CFG3, 34, 65536, oracle.VARIABLE),
                                            (G500, 16, 256, oracle.FIXED)])
def test_samples_per_edge_law(q, k, bound, mode):
    """Mean and distribution of samples per edge vs the exact renewal law."""
    t = oracle.build_table(*q, k, bound, mode)
    law = rm.samples_per_edge_law(t.length, t.w / 2.0**32, t.n_items, k)
    m = 1 << 21
    _, _, ns = oracle.generate(t, 3, 0, m, threads=8, samples=True)
    n = np.arange(len(law))
    mean = float((law * n).sum())
    sd = float(np.sqrt((law * n * n).sum() - mean**2))
    assert abs(ns.mean() - mean) < 5 * sd / np.sqrt(m) + 1e-12
    obs = np.bincount(ns, minlength=len(law))[: len(law)]
    for v in np.nonzero(law * m > 100)[0]:
        assert abs(obs[v] - law[v] * m) < 6 * np.sqrt(law[v] * m)


def test_generate_chunk_invariance():
    t = oracle.build_table(*CFG3, 34, 4096, oracle.VARIABLE)
    s, d = oracle.generate(t, 11, 1000, 50000, threads=3)
    parts = [(1000, 17), (1017, 20000), (21017, 29983)]
    cat_s = np.concatenate([oracle.generate(t, 11, b, n)[0] for b, n in parts])
    cat_d = np.concatenate([oracle.generate(t, 11, b, n)[1] for b, n in parts])
    assert np.array_equal(s, cat_s) and np.array_equal(d, cat_d)


def test_ids_below_2_to_k_and_widths():
    for k in (1, 7, 31, 32, 33, 64):
        t = oracle.build_table(*G500, k, 4096, oracle.VARIABLE)
        src, dst = oracle.generate(t, 1, 0, 4000)
        if k < 64:
            assert int(src.max()) < 2**k and int(dst.max()) < 2**k
        assert src.dtype == (np.uint32 if k <= 32 else np.uint64)


def test_reduce_matches_generate():
    t = oracle.build_table(*CFG3, 20, 4096, oracle.VARIABLE)
    src, dst = oracle.generate(t, 3, 777, 100000, threads=4)
    hist, x = oracle.generate_reduce(t, 3, 777, 100000, hist_bits=8, threads=3)
    assert np.array_equal(hist, np.bincount(src >> 12, minlength=256).astype(np.uint64))
    acc = 0
    for i in range(0, 100000):
        acc ^= oracle.edge_mix(777 + i, int(src[i]), int(dst[i]))
    assert acc == x
    # the source-prefix histogram follows the closed form m (a+b)^#0 (c+d)^#1
    p0 = CFG3[0] + CFG3[1]
    bits = np.array([bin(v).count("1") for v in range(256)])
    exp = 100000 * p0 ** (8 - bits) * (1 - p0) ** bits
    keep = exp > 5
    chi2 = float(((hist[keep] - exp[keep]) ** 2 / exp[keep]).sum())
    assert stats.chi2.sf(chi2, int(keep.sum()) - 1) > 1e-5


@pytest.mark.parametrize("args", [
    (0.5, 0.5, 0.1, -0.1, 10, 100, oracle.VARIABLE),   # negative letter
    (0.5, 0.2, 0.2, 0.2, 10, 100, oracle.VARIABLE),    # sum != 1
    (0.25, 0.25, 0.25, 0.25, 0, 100, oracle.VARIABLE),  # k < 1
    (0.25, 0.25, 0.25, 0.25, 65, 100, oracle.VARIABLE),  # k > 64
    (0.25, 0.25, 0.25, 0.25, 10, 4, oracle.VARIABLE),  # bound < 5
    (0.25, 0.25, 0.25, 0.25, 10, 3, oracle.FIXED),     # l < 1
    (0.25, 0.25, 0.25, 0.25, 2, 256, oracle.FIXED),    # l = 4 > k
    (0.25, 0.25, 0.25, 0.25, 20, 2**24 + 1, oracle.VARIABLE),
    (0.25, 0.25, 0.25, 0.25, 20, 100, 2),
    (float("nan"), 0.5, 0.25, 0.25, 10, 100, oracle.VARIABLE),
])
def test_invalid_inputs_rejected(args):
    with pytest.raises(oracle.OracleError) as ei:
        oracle.build_table(*args)
    assert ei.value.name == "EINVAL"


# ---------------------------------------------------------------------------
# Sec. 3 generalizations: undirected mirror and id scramble (reading R19)

@pytest.mark.parametrize("k", [1, 2, 3, 4, 7, 10, 16])
@pytest.mark.parametrize("key", [0, 1, 0x0123456789ABCDEF, 2**64 - 1])
def test_scramble_is_a_permutation(k, key):
    """The scramble relabels ids: a bijection of [0, 2^k) for every key."""
    img = sorted(oracle.scramble(k, key, x) for x in range(1 << k))
    assert img == list(range(1 << k))


def test_scramble_depends_on_key_and_k():
    a = [oracle.scramble(16, 1, x) for x in range(256)]
    b = [oracle.scramble(16, 2, x) for x in range(256)]
    assert a != b and a != list(range(256))
    # ids stay below 2^k for k up to 64
    for k in (31, 32, 33, 63, 64):
        for x in (0, 1, (1 << k) - 1, (1 << (k - 1)) + 12345):
            assert 0 <= oracle.scramble(k, 99, x) < (1 << k)


@pytest.mark.parametrize("k,bound,e0,m", [(12, 256, 0, 5000), (26, 4096, 2**32 - 100, 3000), (64, 2000, 2**64 - 500, 500),
                                          (33, 1000, 7, 2000)])
def test_undirected_mirrors_the_lower_triangle(k, bound, e0, m):
    """Sec. 3: an undirected graph mirrors edges of the lower-left triangle
    (row > column) to the upper right: (min, max) of the directed edge."""
    t = oracle.build_table(0.57, 0.19, 0.19, 0.05, k, bound, oracle.VARIABLE)
    s, d = oracle.generate(t, 3, e0, m)
    us, ud = oracle.generate(t, 3, e0, m, flags=oracle.UNDIRECTED)
    assert np.array_equal(us, np.minimum(s, d)) and np.array_equal(ud, np.maximum(s, d))
    assert np.all(us <= ud)


def test_scramble_relabels_every_id_by_the_same_map():
    """The scramble is one map applied to sources and destinations alike, after
    the mirror; the degree sequence of the graph is unchanged."""
    k, key = 12, 0xC0FFEE
    t = oracle.build_table(0.45, 0.22, 0.22, 0.11, k, 1000, oracle.VARIABLE)
    s, d = oracle.generate(t, 8, 0, 1 << 15)
    pi = np.array([oracle.scramble(k, key, x) for x in range(1 << k)], dtype=np.uint32)
    ss, sd = oracle.generate(t, 8, 0, 1 << 15, flags=oracle.SCRAMBLE, scramble_key=key)
    assert np.array_equal(ss, pi[s]) and np.array_equal(sd, pi[d])
    bs, bd = oracle.generate(t, 8, 0, 1 << 15, flags=oracle.SCRAMBLE | oracle.UNDIRECTED, scramble_key=key)
    assert np.array_equal(bs, pi[np.minimum(s, d)]) and np.array_equal(bd, pi[np.maximum(s, d)])
    deg = np.sort(np.bincount(s, minlength=1 << k))
    sdeg = np.sort(np.bincount(ss, minlength=1 << k))
    assert np.array_equal(deg, sdeg)


def test_epilogue_rejects_unknown_flags():
    t = oracle.build_table(0.57, 0.19, 0.19, 0.05, 10, 256, oracle.VARIABLE)
    with pytest.raises(oracle.OracleError):
        oracle.generate(t, 1, 0, 10, flags=4)
