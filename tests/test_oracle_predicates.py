"""Pins for the oracle's exact predicates (not GPU).

Orientation and in-circle signs are checked against exact rational / big
integer evaluation of their defining determinants on random inputs, on
inputs at the top of the grid range (|coord| ~ 2^52), and on adversarial
near-degenerate inputs (points one grid unit off a circle or a line).  The
tie-break of cocircular points is checked against the determinant with an
explicit, concrete tiny perturbation of the lifted coordinate.
"""
import random
from fractions import Fraction

import pytest

import brute_delaunay as bd


def _rand_pts(rng, k, lo, hi):
    return [(rng.randrange(lo, hi), rng.randrange(lo, hi)) for _ in range(k)]


def _incircle_fraction(a, b, c, d):
    # circumcentre of a, b, c as exact fractions, compare squared distances
    (ax, ay), (bx, by), (cx, cy) = a, b, c
    D = 2 * (ax * (by - cy) + bx * (cy - ay) + cx * (ay - by))
    ux = Fraction((ax * ax + ay * ay) * (by - cy) + (bx * bx + by * by) * (cy - ay) + (cx * cx + cy * cy) * (ay - by), D)
    uy = Fraction((ax * ax + ay * ay) * (cx - bx) + (bx * bx + by * by) * (ax - cx) + (cx * cx + cy * cy) * (bx - ax), D)
    r2 = (ux - ax) ** 2 + (uy - ay) ** 2
    d2 = (ux - d[0]) ** 2 + (uy - d[1]) ** 2
    inside = (d2 < r2) - (d2 > r2)
    return inside if D > 0 else -inside


@pytest.mark.parametrize("scale_bits", [10, 30, 50, 52])
def test_orient_random(orc, scale_bits):
    rng = random.Random(1000 + scale_bits)
    for _ in range(400):
        a, b, c = _rand_pts(rng, 3, -(1 << scale_bits), 1 << scale_bits)
        assert orc.orient(a, b, c) == bd.orient(a, b, c)


@pytest.mark.parametrize("scale_bits", [10, 30, 50, 52])
def test_incircle_random_vs_fraction(orc, scale_bits):
    rng = random.Random(2000 + scale_bits)
    n = 0
    while n < 300:
        a, b, c, d = _rand_pts(rng, 4, 0, 1 << scale_bits)
        if bd.orient(a, b, c) == 0:
            continue
        n += 1
        assert orc.incircle(a, b, c, d) == _incircle_fraction(a, b, c, d)


def _cocircular(rng, lo_bits=40, hi_bits=50):
    """Four distinct integer points exactly on one circle (Pythagorean triples
    scaled to a common hypotenuse), first three counter-clockwise."""
    trip = [(3, 4, 5), (5, 12, 13), (8, 15, 17), (7, 24, 25), (0, 1, 1)]
    while True:
        cx, cy = rng.randrange(1 << lo_bits, 1 << hi_bits), rng.randrange(1 << lo_bits, 1 << hi_bits)
        R = 5 * 13 * 17 * 25 * rng.randrange(1, 1 << 16)
        pts = []
        for (p, q, h) in rng.sample(trip, 4):
            f = R // h
            sx, sy = rng.choice([1, -1]), rng.choice([1, -1])
            if rng.random() < 0.5:
                p, q = q, p
            pts.append((cx + sx * p * f, cy + sy * q * f))
        if len(set(pts)) < 4:
            continue
        a, b, c, d = pts
        if bd.orient(a, b, c) < 0:
            a, b = b, a
        if bd.orient(a, b, c) == 0:
            continue
        return a, b, c, d


def test_incircle_near_cocircular(orc):
    """Points exactly on a circle at grid scale, and one grid unit off it."""
    rng = random.Random(7)
    for _ in range(200):
        a, b, c, d = _cocircular(rng)
        assert bd.incircle_plain([a, b, c, d]) == 0
        assert orc.incircle(a, b, c, d) == 0
        for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1), (1, 1)):
            d2 = (d[0] + dx, d[1] + dy)
            want = bd.incircle_plain([a, b, c, d2])
            assert want == _incircle_fraction(a, b, c, d2)
            assert orc.incircle(a, b, c, d2) == want


def test_orient_near_collinear(orc):
    rng = random.Random(11)
    for _ in range(300):
        a = (rng.randrange(0, 1 << 52), rng.randrange(0, 1 << 52))
        dx, dy = rng.randrange(1, 1 << 20), rng.randrange(1, 1 << 20)
        t = rng.randrange(1, 1 << 10)
        b = (a[0] + dx, a[1] + dy)
        c = (a[0] + t * dx + rng.choice([-1, 0, 1]), a[1] + t * dy)
        assert orc.orient(a, b, c) == bd.orient(a, b, c)


def test_incircle_sos_matches_explicit_perturbation(orc):
    """Every cocircular 4-tuple of a square-lattice patch, every rank order."""
    import itertools
    rng = random.Random(5)
    base = [(0, 0), (4, 0), (4, 4), (0, 4), (2, 2 + 0), (6, 2), (2, 6)]
    circle = [(0, 0), (4, 0), (4, 4), (0, 4)]
    # all orderings of the four cocircular corners and random distinct ranks
    checked = 0
    for perm in itertools.permutations(circle):
        a, b, c, d = perm
        if bd.orient(a, b, c) <= 0:
            continue
        for _ in range(4):
            ranks = rng.sample(range(100), 4)
            want = bd.incircle_perturbed([a, b, c, d], ranks)
            assert want != 0
            assert orc.incircle_sos(a, b, c, d, ranks) == want
            checked += 1
    assert checked > 20
    # non-degenerate inputs are unaffected by the perturbation
    for _ in range(200):
        a, b, c, d = [base[k] for k in rng.sample(range(len(base)), 4)]
        if bd.orient(a, b, c) == 0 or bd.incircle_plain([a, b, c, d]) == 0:
            continue
        assert orc.incircle_sos(a, b, c, d, rng.sample(range(100), 4)) == bd.incircle_plain([a, b, c, d])


def test_incircle_sos_large_circle(orc):
    """Exactly cocircular points at grid scale, random ranks."""
    rng = random.Random(9)
    for _ in range(100):
        a, b, c, d = _cocircular(rng)
        ranks = rng.sample(range(1 << 20), 4)
        assert orc.incircle_sos(a, b, c, d, ranks) == bd.incircle_perturbed([a, b, c, d], ranks)
