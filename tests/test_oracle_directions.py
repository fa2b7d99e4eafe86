"""Pins of the oracle's line enumeration (Sec. 3.2, Farey series and the set A^{d-1}).

Every expected value here comes from the paper (Fig. 1, the A^1 count), from a
closed form (Moebius inversion over the box) or from an independent brute-force
scan written in this file; none comes from the oracle itself.
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def brute_lines(d, order):
    """Independent scan: primitive vectors of the box, first nonzero > 0, sorted."""
    out = []
    for e in itertools.product(range(-order, order + 1), repeat=d):
        g = 0
        for x in e:
            g = math.gcd(g, abs(x))
        if g != 1:
            continue
        first = next(x for x in e if x != 0)
        if first < 0:
            continue
        out.append(e)
    out.sort(key=lambda e: (max(abs(x) for x in e), sum(x * x for x in e), e))
    return np.array(out, dtype=np.int32)


def mobius(k):
    res, m, p = 1, k, 2
    while p * p <= m:
        if m % p == 0:
            m //= p
            if m % p == 0:
                return 0
            res = -res
        p += 1
    if m > 1:
        res = -res
    return res


def lines_closed_form(d, order):
    """#lines = (1/2) #primitive vectors of [-order, order]^d \\ {0}
    = (1/2) sum_k mu(k) ((2 floor(order/k) + 1)^d - 1)   (Moebius inversion)."""
    total = sum(mobius(k) * ((2 * (order // k) + 1) ** d - 1) for k in range(1, order + 1))
    assert total % 2 == 0
    return total // 2


def farey1(order):
    """F^1 of Sec. 3.2: 0 <= p <= q <= order, q >= 1, gcd(p, q) = 1."""
    return [(p, q) for q in range(1, order + 1) for p in range(0, q + 1) if math.gcd(p, q) == 1]


def farey2(order):
    """F^2 of Sec. 3.2: 0 <= p <= q <= r <= order, r >= 1, gcd(p, q, r) = 1."""
    return [(p, q, r) for r in range(1, order + 1) for q in range(0, r + 1)
            for p in range(0, q + 1) if math.gcd(math.gcd(p, q), r) == 1]


@pytest.mark.parametrize("d,order", [(2, o) for o in range(1, 9)] + [(3, o) for o in range(1, 5)])
def test_lines_equal_brute_force(d, order):
    got = oracle.lines(d, order)
    ref = brute_lines(d, order)
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("d,order", [(2, o) for o in range(1, 33)] + [(3, o) for o in range(1, 9)])
def test_line_count_closed_form(d, order):
    assert len(oracle.lines(d, order)) == lines_closed_form(d, order)


@pytest.mark.parametrize("order", range(1, 33))
def test_2d_count_matches_paper_formula(order):
    # Sec. 3.2: A^1 = 4 (|F^1| - 1)
    assert len(oracle.lines(2, order)) == 4 * (len(farey1(order)) - 1)


def test_3d_paper_formula_erratum():
    # Sec. 3.2 prints A^2 = 24(|F^2| - |F^1|) - 2 A^1; a direct count gives fewer
    # lines, by exactly A^1 - 1 for every order checked.  The enumeration follows
    # the definition (lines through 0 of the box), not the printed count.
    for order in range(1, 8):
        a1 = 4 * (len(farey1(order)) - 1)
        printed = 24 * (len(farey2(order)) - len(farey1(order))) - 2 * a1
        true = len(oracle.lines(3, order))
        assert true == lines_closed_form(3, order)
        assert printed - true == a1 - 1


def test_fig1_order3():
    g = json.load(open(os.path.join(GOLD, "fig1_farey_order3.json")))
    assert sorted(map(tuple, g["farey_points_first_octant"])) == sorted(farey1(3))
    ls = oracle.lines(2, 3)
    assert len(ls) == g["num_lines"]
    slopes = set()
    for a, b in ls:
        slopes.add("inf" if a == 0 else str(Fraction(int(b), int(a))))
    assert slopes == set(g["slopes_as_fractions"])


def test_first_lines_prefix_and_perp_closure():
    # the first P lines are a prefix of every larger listing
    big = oracle.lines(2, 6)
    for P in (8, 16, 24, 32):
        fl = oracle.first_lines(2, P)
        assert np.array_equal(fl, big[:P])
        s = {tuple(x) for x in fl}
        for a, b in fl:
            perp = (-b, a) if (-b > 0 or (-b == 0 and a > 0)) else (b, -a)
            assert perp in s, (P, (a, b))
    big3 = oracle.lines(3, 3)
    assert np.array_equal(oracle.first_lines(3, 16), big3[:16])
    assert tuple(big3[0]) == (0, 0, 1) and tuple(big3[2]) == (1, 0, 0)


def test_default_ntilde_sec4():
    g = json.load(open(os.path.join(GOLD, "ntilde_sec4.json")))
    for n, nt in zip(g["points_per_axis"], g["ntilde"]):
        assert oracle.default_ntilde(n) == nt


def test_default_weights_formula():
    # a(k) = h^(2d-1) |k| / gcd(k) evaluated at several k on each line
    for d, h in ((2, 0.25), (3, 0.5)):
        dirs = oracle.first_lines(d, 16)
        w = oracle.default_weights(d, h, dirs)
        for e, wp in zip(dirs, w):
            for m in (1, 2, 3):
                k = m * e
                g = 0
                for x in k:
                    g = math.gcd(g, abs(int(x)))
                a = h ** (2 * d - 1) * math.sqrt(float(np.sum(k.astype(float) ** 2))) / g
                assert abs(a - wp) <= 1e-15 * a
