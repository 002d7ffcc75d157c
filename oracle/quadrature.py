"""Quadrature on flat and geodesic (sphere) triangles.

The paper computes its spherical integrals with "higher-order integration rules" on a
sphere mesh whose refined vertices are projected to the sphere (Sec. 6, opening
paragraph) but does not name the rule.  Reading used here: a geodesic triangle K is the
radial projection of the flat triangle spanned by its three unit vertices a, b, c; for
a flat point x the surface element is dS = h |x|^-3 dA with h the distance of the flat
plane from the origin, so

    int_K f(s) ds = int_flat f(x / |x|) h / |x|^3 dA,   A_flat * h = |det(a,b,c)| / 2.

The flat triangle is cut uniformly into 4^r sub-triangles and Radon's 7-point
degree-5 rule is applied on each (Radon 1948; Stroud's T2:5-1).
"""
from __future__ import annotations

import numpy as np


def radon7():
    """Barycentric points [7,3] and weights [7] (summing to 1) of Radon's rule."""
    r15 = np.sqrt(15.0)
    a = (6.0 - r15) / 21.0
    b = (6.0 + r15) / 21.0
    wa = (155.0 - r15) / 1200.0
    wb = (155.0 + r15) / 1200.0
    pts = np.array([
        [1 / 3, 1 / 3, 1 / 3],
        [a, a, 1 - 2 * a], [a, 1 - 2 * a, a], [1 - 2 * a, a, a],
        [b, b, 1 - 2 * b], [b, 1 - 2 * b, b], [1 - 2 * b, b, b],
    ])
    w = np.array([9.0 / 40.0, wa, wa, wa, wb, wb, wb])
    return pts, w


def composite_barycentric(r: int):
    """Radon's rule on the 4^r congruent sub-triangles of a triangle.

    Returns barycentric points [7*4^r, 3] and weights [7*4^r] relative to the area of
    the whole triangle (they sum to 1).
    """
    n = 2 ** r
    subs = []
    for j in range(n):
        for i in range(n - j):
            # "upward" sub-triangle with corners (i,j), (i+1,j), (i,j+1) in (l1,l2)/n
            subs.append(((i, j), (i + 1, j), (i, j + 1)))
            if i + j <= n - 2:
                # "downward" sub-triangle (i+1,j), (i+1,j+1), (i,j+1)
                subs.append(((i + 1, j), (i + 1, j + 1), (i, j + 1)))
    assert len(subs) == n * n
    rp, rw = radon7()
    pts, wts = [], []
    for corners in subs:
        c = np.array([[1.0 - (p + q) / n, p / n, q / n] for p, q in corners])  # [3 corners, 3 bary]
        pts.append(rp @ c)
        wts.append(rw / (n * n))
    return np.concatenate(pts), np.concatenate(wts)


def flat_triangle_rule(p0, p1, p2, r: int):
    """Points [Q,d] and weights [Q] of the composite rule on a flat triangle."""
    bary, w = composite_barycentric(r)
    P = np.stack([p0, p1, p2]).astype(np.float64)
    e1, e2 = P[1] - P[0], P[2] - P[0]
    if len(p0) == 2:
        area = 0.5 * abs(e1[0] * e2[1] - e1[1] * e2[0])
    else:
        area = 0.5 * np.linalg.norm(np.cross(e1, e2))
    return bary @ P, w * area


def sphere_triangle_rule(a, b, c, r: int):
    """Points s_p [Q,3] (unit vectors) and weights w_p [Q] on the geodesic triangle abc."""
    bary, w = composite_barycentric(r)
    V = np.stack([a, b, c]).astype(np.float64)
    x = bary @ V
    nx = np.linalg.norm(x, axis=1)
    det = abs(np.linalg.det(V))
    return x / nx[:, None], w * det / (2.0 * nx ** 3)


def spherical_excess(a, b, c):
    """Closed-form area of the geodesic triangle abc (Van Oosterom-Strackee)."""
    num = abs(np.dot(a, np.cross(b, c)))
    den = 1.0 + np.dot(a, b) + np.dot(b, c) + np.dot(c, a)
    return 2.0 * np.arctan2(num, den)
