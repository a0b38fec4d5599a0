"""Brute-force periodic Delaunay neighbours, exact, for tiny inputs.

Independent of the oracle: plain Python integers, no floating point in any
decision.  A triangle (i, a, b) of the periodic point set is Delaunay when no
point lies strictly inside its circumcircle (empty-circumcircle property,
Sec. II.C.3 of the paper).  Ties (four or more cocircular points) are broken
by perturbing the lifted coordinate w = x^2 + y^2 of each point by eps^e with
a concrete tiny eps = 2^-B, the point of highest tag getting the largest
perturbation (e = 1), the next e = 2, ...; the determinant is evaluated
exactly with the perturbation scaled to integers.
"""
from __future__ import annotations

import math

PERT_BITS = 400


def orient(a, b, c):
    d = (a[0] - c[0]) * (b[1] - c[1]) - (a[1] - c[1]) * (b[0] - c[0])
    return (d > 0) - (d < 0)


def incircle_perturbed(pts, tags):
    """Sign of det[[x, y, w + eps^e, 1]] for four integer points, w = x^2 + y^2,
    eps = 2^-PERT_BITS, e = 1 for the highest tag, 2 for the next, ..."""
    order = sorted(range(4), key=lambda k: -tags[k])
    expo = [0] * 4
    for rank, k in enumerate(order):
        expo[k] = rank + 1
    B = PERT_BITS
    rows = []
    for k, (x, y) in enumerate(pts):
        w = (x * x + y * y) << (4 * B)
        w += 1 << ((4 - expo[k]) * B)
        rows.append((x, y, w, 1))
    return _sign(_det4(rows))


def incircle_plain(pts):
    """Unperturbed sign, computed as the 3x3 determinant after translating the
    fourth point to the origin (equal to the 4x4 lifted determinant)."""
    (ax, ay), (bx, by), (cx, cy), (dx, dy) = pts
    ax, ay, bx, by, cx, cy = ax - dx, ay - dy, bx - dx, by - dy, cx - dx, cy - dy
    return _sign(_det3([(ax, ay, ax * ax + ay * ay), (bx, by, bx * bx + by * by), (cx, cy, cx * cx + cy * cy)]))


def _sign(v):
    return (v > 0) - (v < 0)


def _det3(m):
    return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
            - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
            + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))


def _det4(m):
    tot = 0
    for j in range(4):
        minor = [[m[r][c] for c in range(4) if c != j] for r in range(1, 4)]
        tot += (-1) ** j * m[0][j] * _det3(minor)
    return tot


def periodic_neighbours(X, Y, LX, LY):
    """Exact Delaunay neighbours on the torus of integer points.

    X, Y: integer coordinates in [0, LX) x [0, LY).  Returns a list of sets of
    tags and the number of triangles.  Assumes every Delaunay circumradius is
    below min(LX, LY)/4 (checked)."""
    n = len(X)
    pts = []
    for sy in (-1, 0, 1):
        for sx in (-1, 0, 1):
            for t in range(n):
                pts.append((X[t] + sx * LX, Y[t] + sy * LY, t))
    half = min(LX, LY) // 2
    nbrs = [set() for _ in range(n)]
    tri_count = 0
    for i in range(n):
        pi = (X[i], Y[i])
        cand = [p for p in pts if p[2] != i and (p[0] - pi[0]) ** 2 + (p[1] - pi[1]) ** 2 < half * half]
        for ia in range(len(cand)):
            a = cand[ia]
            for ib in range(len(cand)):
                if ib == ia:
                    continue
                b = cand[ib]
                if a[2] == b[2]:
                    continue
                if orient(pi, a[:2], b[:2]) <= 0:
                    continue
                empty = True
                for p in cand:
                    if p is a or p is b:
                        continue
                    s = incircle_plain([pi, a[:2], b[:2], p[:2]])
                    if s == 0:
                        s = incircle_perturbed([pi, a[:2], b[:2], p[:2]], [i, a[2], b[2], p[2]])
                    if s > 0:
                        empty = False
                        break
                if empty:
                    # circumradius check (exact): |u|^2 < (L/4)^2 with u the centre rel. to i
                    bx, by = a[0] - pi[0], a[1] - pi[1]
                    cx, cy = b[0] - pi[0], b[1] - pi[1]
                    den = 2 * (bx * cy - by * cx)
                    b2, c2 = bx * bx + by * by, cx * cx + cy * cy
                    ux, uy = cy * b2 - by * c2, bx * c2 - cx * b2
                    assert 16 * (ux * ux + uy * uy) < min(LX, LY) ** 2 * den * den, \
                        "circumradius precondition violated"
                    nbrs[i].add(a[2])
                    nbrs[i].add(b[2])
                    tri_count += 1
    return nbrs, tri_count // 3


def ccw_ring(i, nb, X, Y, LX, LY):
    """Order the neighbour tags of i counter-clockwise (min-image directions),
    starting at the smallest tag."""
    def ang(t):
        dx = X[t] - X[i]
        dy = Y[t] - Y[i]
        if 2 * dx > LX:
            dx -= LX
        elif 2 * dx < -LX:
            dx += LX
        if 2 * dy > LY:
            dy -= LY
        elif 2 * dy < -LY:
            dy += LY
        return math.atan2(dy, dx)
    r = sorted(nb, key=ang)
    k = r.index(min(r))
    return r[k:] + r[:k]
