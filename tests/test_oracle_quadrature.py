"""Pins of the oracle's quadrature against closed forms.

* Radon's 7-point rule, composite over 4^r sub-triangles, integrates every monomial
  u^i v^j with i + j <= 5 exactly on the reference triangle: int u^i v^j = i! j! / (i+j+2)!.
* On a geodesic triangle the weights sum to its area, whose closed form is the spherical
  excess (Van Oosterom-Strackee); the error falls as the rule is refined.
* Over the whole octahedral sphere mesh: sum of areas -> 4 pi, int s s^T -> (4 pi / 3) I.
"""
import math

import numpy as np
import pytest

from oracle.quadrature import (composite_barycentric, flat_triangle_rule, radon7,
                               sphere_triangle_rule, spherical_excess)
from paper_2102_09038_amd.inputs import octahedral_sphere


def test_radon_weights_sum_to_one():
    _, w = radon7()
    assert abs(w.sum() - 1.0) < 1e-15


@pytest.mark.parametrize("r", [0, 1, 2])
def test_composite_rule_degree5_exact(r):
    p, w = flat_triangle_rule(np.array([0.0, 0.0]), np.array([1.0, 0.0]), np.array([0.0, 1.0]), r)
    for i in range(6):
        for j in range(6 - i):
            exact = math.factorial(i) * math.factorial(j) / math.factorial(i + j + 2)
            got = np.sum(w * p[:, 0] ** i * p[:, 1] ** j)
            assert abs(got - exact) < 1e-15, (i, j, got, exact)


def test_composite_rule_not_exact_degree6():
    # a rule exact to degree 5 only: u^6 must show an error at r = 0 (guards a silent
    # replacement by some other rule)
    p, w = flat_triangle_rule(np.array([0.0, 0.0]), np.array([1.0, 0.0]), np.array([0.0, 1.0]), 0)
    exact = math.factorial(6) * 1 / math.factorial(8)
    assert abs(np.sum(w * p[:, 0] ** 6) - exact) > 1e-6


def test_composite_points_are_inside_and_weights_positive():
    bary, w = composite_barycentric(3)
    assert len(w) == 7 * 64
    assert np.all(bary > 0) and np.allclose(bary.sum(1), 1.0)
    assert np.all(w > 0) and abs(w.sum() - 1) < 1e-14


def test_sphere_triangle_area_converges_to_excess():
    svert, stri = octahedral_sphere(1)
    a, b, c = svert[stri[3]]
    exact = spherical_excess(a, b, c)
    errs = []
    for r in range(0, 4):
        s, w = sphere_triangle_rule(a, b, c, r)
        assert np.allclose(np.linalg.norm(s, axis=1), 1.0)
        errs.append(abs(w.sum() - exact))
    assert errs[-1] < 5e-9 * exact
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))


@pytest.mark.parametrize("level", [0, 2])
def test_whole_sphere_moments(level):
    svert, stri = octahedral_sphere(level)
    area = 0.0
    second = np.zeros((3, 3))
    for t in stri:
        s, w = sphere_triangle_rule(*svert[t], 3)
        area += w.sum()
        second += np.einsum("p,pi,pj->ij", w, s, s)
    assert abs(area - 4 * math.pi) < 1e-6
    assert np.allclose(second, 4 * math.pi / 3 * np.eye(3), atol=1e-6)
