"""Pins for the sparse-sign embedding (Section 2.1, eq. sparse_sign_sketch) and its generator."""
import itertools
import os

import numpy as np
import pytest
from scipy import stats

from oracle import philox, sketch

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        yield v[:6], v[6:]


@pytest.mark.parametrize("inp,out", list(_kat()))
def test_philox_known_answers(inp, out):
    got = [int(x) for x in philox.philox4x32_10(*inp)]
    assert got == out


@pytest.mark.parametrize("inp,out", list(_kat()))
def test_seven_round_form_is_the_prefix_of_the_published_generator(inp, out):
    """The sketch's seven-round Philox is the first seven rounds of the published ten-round form:
    rounds 7, 8 and 9 (keys advanced 7, 8, 9 times) carry its output to the known answers.  A
    wrong key schedule, round count or round function in either part misses them."""
    seven = philox.philox4x32_7(*inp)
    got = [int(x) for x in philox.philox4x32_rounds(*seven, inp[4], inp[5], 3, first=7)]
    assert got == out
    # and it is not the ten-round output itself
    assert [int(x) for x in seven] != out


def test_sketch_signs_are_the_low_bits_of_the_row_draws():
    """Signs: bit 0 of each row draw; balanced and uncorrelated with the row they go with."""
    rows, signs = sketch.rows_and_signs(0, 200000, 80, 8, seed=5)
    neg = signs < 0
    assert abs(neg.mean() - 0.5) < 4 * 0.5 / np.sqrt(neg.size)
    # sign frequency per row index: chi-square test of independence of row and sign
    table = np.zeros((80, 2))
    np.add.at(table, (rows.ravel(), neg.ravel().astype(int)), 1)
    _, pval, _, _ = stats.chi2_contingency(table)
    assert pval > 1e-4


def test_philox_vectorised_matches_scalar():
    c = np.arange(17, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15 & 0xFFFFFFFF)
    vec = philox.philox4x32_10(c, c + np.uint64(1), c * np.uint64(3), c ^ np.uint64(5), 11, 12)
    for i in range(17):
        one = philox.philox4x32_10(int(c[i]), int(c[i]) + 1, int(c[i]) * 3, int(c[i]) ^ 5, 11, 12)
        assert [int(v[i]) for v in vec] == [int(o) for o in one]


@pytest.mark.parametrize("d,zeta", [(80, 8), (200, 8), (5, 5), (64, 1), (96, 32)])
def test_columns_distinct_rows_unit_norm(d, zeta):
    rows, signs = sketch.rows_and_signs(1000, 4000, d, zeta, seed=1)
    assert rows.min() >= 0 and rows.max() < d
    srt = np.sort(rows, axis=1)
    assert np.all(np.diff(srt, axis=1) > 0)            # zeta distinct rows per column
    assert set(np.unique(signs)) <= {-1.0, 1.0}
    S = sketch.sketch_matrix(4000, d, zeta, seed=1)
    norms = np.sqrt(np.asarray(S.multiply(S).sum(axis=0))).ravel()
    assert np.max(np.abs(norms - 1.0)) <= 4 * np.finfo(float).eps


def test_rows_uniform_and_signs_balanced():
    d, zeta, cnt = 80, 8, 40000
    rows, signs = sketch.rows_and_signs(0, cnt, d, zeta, seed=7)
    counts = np.bincount(rows.ravel(), minlength=d)
    assert stats.chisquare(counts).pvalue > 1e-4
    assert abs(signs.mean()) < 4.0 / np.sqrt(signs.size)


def test_floyd_subsets_uniform():
    """Every zeta-subset of a small row set is equally likely (Floyd's algorithm)."""
    d, zeta, cnt = 6, 3, 60000
    rows, _ = sketch.rows_and_signs(0, cnt, d, zeta, seed=3)
    subsets = list(itertools.combinations(range(d), zeta))
    index = {s: i for i, s in enumerate(subsets)}
    counts = np.bincount([index[tuple(sorted(r))] for r in rows], minlength=len(subsets))
    assert stats.chisquare(counts).pvalue > 1e-4


def test_norm_preserved_in_expectation():
    """E ||S x||^2 = ||x||^2 for the Rademacher sparse sign matrix."""
    n, d, zeta = 3000, 80, 8
    x = np.random.default_rng(0).standard_normal(n)
    vals = [np.linalg.norm(sketch.sketch_matrix(n, d, zeta, seed=s) @ x) ** 2 for s in range(60)]
    ratio = np.mean(vals) / np.dot(x, x)
    assert abs(ratio - 1.0) < 0.05


def test_distortion_decreases_with_d():
    """Observed distortion of a random 20-dim subspace falls as d grows (trend of the paper's tables)."""
    n, m = 4000, 20
    Qx, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((n, m)))
    eps = []
    for d in (40, 80, 320, 1280):
        s = np.linalg.svd(sketch.sketch_matrix(n, d, 8, seed=2) @ Qx, compute_uv=False)
        eps.append(max(s.max() ** 2 - 1, 1 - s.min() ** 2))
    assert all(a > b for a, b in zip(eps, eps[1:]))
    assert eps[-1] < 0.5
