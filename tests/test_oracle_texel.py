"""Pins of the oracle's texel parametrisation (Section 3.1, Fig. texels,
eq. projected-pixels, eq. idtexel).  CPU only."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "texel_counts.txt")


def test_worked_example_fig_texels():
    # Section 3.1, Fig. texels: s = 6 gives (s^2+s)/2 = 21 texels.
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert rows
    for scheme, s, n in rows:
        assert oracle.texel_count(int(s), int(scheme)) == int(n)


def _cells(s):
    """All cells (a, b) of the triangle domain u, v >= 0, u + v < 1."""
    return [(a, b) for a in range(s) for b in range(s - a)]


def _interior_points(s, a, b, upper):
    """float32 points strictly inside cell (a, b); the lower-left triangle of a
    full cell, or its upper-right half when ``upper``."""
    if not upper:
        fr = [(0.1, 0.1), (0.3, 0.2), (0.6, 0.25), (0.2, 0.7)]
    else:
        fr = [(0.9, 0.9), (0.7, 0.8), (0.45, 0.65), (0.95, 0.3)]
    return [(np.float32((a + fu) / s), np.float32((b + fv) / s)) for fu, fv in fr]


def _exact_class(s, u, v):
    """Cell of a float32 point by exact rational arithmetic."""
    su = Fraction(float(u)) * s
    sv = Fraction(float(v)) * s
    a, b = math.floor(su), math.floor(sv)
    upper = (su - a) + (sv - b) >= 1
    return a, b, upper


@pytest.mark.parametrize("scheme", [oracle.SQUARE, oracle.SPLIT])
def test_texel_ids_are_a_bijection_consistent_with_cells(scheme):
    """For s <= 64 every cell (and, in SPLIT, every half cell) gets one id,
    distinct cells get distinct ids, and the ids fill [0, |X_t|)."""
    for s in range(1, 65):
        n = oracle.texel_count(s, scheme)
        seen = {}
        for a, b in _cells(s):
            halves = [False]
            if scheme == oracle.SPLIT and a + b <= s - 2:
                halves.append(True)
            for upper in halves:
                ids = set()
                for u, v in _interior_points(s, a, b, upper):
                    ca, cb, cu = _exact_class(s, u, v)
                    assert (ca, cb) == (a, b)
                    if scheme == oracle.SPLIT and a + b <= s - 2:
                        assert cu == upper
                    ids.add(oracle.texel_id(s, scheme, u, v))
                assert len(ids) == 1, (s, a, b, upper, ids)
                seen[(a, b, upper)] = ids.pop()
        vals = sorted(seen.values())
        assert vals == list(range(n)), (s, scheme)


def test_counts_closed_forms():
    # SQUARE is the paper's (s^2 + s)/2 (Section 3.1); SPLIT halves every full
    # square cell, adding s(s-1)/2 more: s^2.
    for s in range(1, 200):
        assert oracle.texel_count(s, oracle.SQUARE) == (s * s + s) // 2
        assert oracle.texel_count(s, oracle.SPLIT) == s * s
    assert oracle.texel_count(0, oracle.SQUARE) == -1


def test_printed_formula_is_not_injective():
    """Reading of eq. idtexel: (a^2 + a)/2 + b collides on the stated domain
    (e.g. s = 2: cells (0,1) and (1,0) both give 1), so the oracle uses the
    row index r = s - 1 - a instead of a."""
    s = 2
    printed = {(a, b): (a * a + a) // 2 + b for a, b in _cells(s)}
    assert len(set(printed.values())) < len(printed)
    ids = {(a, b): oracle.texel_id(s, oracle.SQUARE, np.float32((a + .25) / s), np.float32((b + .25) / s))
           for a, b in _cells(s)}
    assert len(set(ids.values())) == len(ids)
    # the row layout of the reading: row r = s-1-a holds b = 0..r at r(r+1)/2 + b
    for (a, b), i in ids.items():
        r = s - 1 - a
        assert i == r * (r + 1) // 2 + b


def test_random_points_match_exact_cells():
    """Random points: the id depends only on the exact cell (FP32 rounding of
    s*u can only matter within an ulp of a cell boundary; such points are
    skipped)."""
    rng = np.random.default_rng(5)
    for scheme in (oracle.SQUARE, oracle.SPLIT):
        for s in (1, 2, 3, 4, 7, 16):
            ref = {}
            for _ in range(3000):
                u, v = rng.random(2)
                if u + v >= 1:
                    u, v = 1 - u, 1 - v
                u, v = np.float32(u), np.float32(v)
                su, sv = Fraction(float(u)) * s, Fraction(float(v)) * s
                fu, fv = su - math.floor(su), sv - math.floor(sv)
                if min(fu, 1 - fu, fv, 1 - fv, abs(fu + fv - 1)) < Fraction(1, 10 ** 5):
                    continue
                key = _exact_class(s, u, v)
                if scheme == oracle.SQUARE or key[0] + key[1] > s - 2:
                    key = key[:2]
                i = oracle.texel_id(s, scheme, u, v)
                assert 0 <= i < oracle.texel_count(s, scheme)
                if key in ref:
                    assert ref[key] == i
                ref[key] = i
            assert len(set(ref.values())) == len(ref)


def test_out_of_triangle_points_are_clamped():
    for scheme in (oracle.SQUARE, oracle.SPLIT):
        for s in (1, 3, 5):
            n = oracle.texel_count(s, scheme)
            for u, v in [(-0.5, 0.2), (0.2, -1.0), (0.8, 0.8), (2.0, 2.0), (float("nan"), 0.1),
                         (0.1, float("nan")), (float("inf"), 0.0), (-float("inf"), float("inf"))]:
                i = oracle.texel_id(s, scheme, u, v)
                assert 0 <= i < n
            # u < 0 clamps to the column a = 0; u + v > 1 to the diagonal cell
            assert oracle.texel_id(s, scheme, -0.5, 0.0) == oracle.texel_id(s, scheme, 0.0, 0.0)
            assert oracle.texel_id(s, scheme, 0.99, 0.99) == oracle.texel_id(s, scheme, 0.99, 0.0)


def test_texel_resolution_closed_forms():
    """s = max(1, ceil(gamma sqrt(a))) (Section 3.1): gamma = 0 never
    subdivides, empty triangles keep one texel, perfect squares are exact."""
    a = np.array([0, 1, 4, 16, 17, 100, 101, 10**6], np.int32)
    assert np.array_equal(oracle.texel_resolution(a, 0.0), np.ones(8, np.int32))
    assert np.array_equal(oracle.texel_resolution(a, 1.0), [1, 1, 2, 4, 5, 10, 11, 1000])
    assert np.array_equal(oracle.texel_resolution(a, 0.5), [1, 1, 1, 2, 3, 5, 6, 500])
    assert oracle.texel_resolution(np.array([10**9], np.int32), 1000.0)[0] == 4096


def test_triangle_max_pixels_by_hand():
    tri = np.full((3, 4, 5), -1, np.int32)
    tri[0, :2, :2] = 0          # 4 pixels of triangle 0 in frame 0
    tri[1, :, :] = 1            # 20 pixels of triangle 1 in frame 1
    tri[2, 0, 0] = 0            # 1 pixel of 0, 3 of 2 in frame 2
    tri[2, 1, :3] = 2
    assert list(oracle.triangle_max_pixels(tri, 4)) == [4, 20, 3, 0]
