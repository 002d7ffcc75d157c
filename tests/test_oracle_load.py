"""Pins of the oracle's even load vector l+ (Sec. 2: the source enters the even equation as
the functional l+(w) = (q, w); Sec. 4 discretises it with the P1 x even-P0 basis
phi_i mu_k, so l+[i, k] = int_R q phi_i * int_S mu_k, and int_S mu_k = 2|K_k| = m_k).

The source is isotropic and given by its nodal values (a linear q is then represented
exactly).  Checked against what the mathematics fixes, independently of the oracle's
consistent-mass product:
* q = 1: 1^T l+ = 4 pi |R| (the sphere's area times the domain's volume);
* q = x_1: 1^T l+ = 4 pi int_R x_1 = 2 pi on the unit square and cube;
* l+[:, k] / m_k is one vector for every k (the source does not depend on the direction);
* every entry: l+[i, k] = 2 |K_k| int_R x_1 phi_i, with |K_k| the closed-form spherical
  excess and the spatial integral by a quadrature rule exact for quadratics on each cell
  (edge midpoints on triangles; the symmetric 4-point rule on tetrahedra), on media with
  a heterogeneous sigma_t, so that a weighted mass in place of the plain one, or |K_k| in
  place of 2 |K_k|, fails.
The sphere areas enter through the composite quadrature of the oracle's m_k, so the sums
carry its area defect (below 1e-6 at r_q = 2 on these meshes).
"""
import math

import numpy as np
import pytest

from oracle.discretize import discretize, upper_pairs
from oracle.quadrature import spherical_excess
from paper_2102_09038_amd.inputs import blockwise_sigma_t, grid2d, grid3d, octahedral_sphere


def _mesh(dim):
    if dim == 2:
        v, c, blk = grid2d(6)
    else:
        v, c, blk = grid3d(3)
    return v, c.astype(np.int64), blk


def _load(dim, q_of_x, level=1):
    v, c, blk = _mesh(dim)
    st = blockwise_sigma_t(blk, 2, seed=3)
    sv, stri = octahedral_sphere(level)
    D = discretize(v, c, st, 0.5 * st, 0.5, sv, stri, q_of_x(v), r_q=2, with_scattering=False)
    return v, c, sv, stri, D


def _closed_form_m(sv, stri):
    up, _ = upper_pairs(sv, stri)
    return np.array([2.0 * spherical_excess(*sv[stri[t]]) for t in up])


def _x1_phi_integrals(v, c):
    """int_R x_1 phi_i for every vertex i, by a rule exact for quadratics on each cell."""
    d = v.shape[1]
    if d == 2:
        bary = np.array([[0.5, 0.5, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5]])
        w = np.full(3, 1.0 / 3.0)
    else:
        a, b = 0.5854101966249685, 0.1381966011250105
        bary = np.array([[a, b, b, b], [b, a, b, b], [b, b, a, b], [b, b, b, a]])
        w = np.full(4, 0.25)
    out = np.zeros(len(v))
    for cell in c:
        X = v[cell]
        vol = abs(np.linalg.det((X[1:] - X[0]).T)) / math.factorial(d)
        for bp, wp in zip(bary, w):
            x1 = bp @ X[:, 0]
            out[cell] += vol * wp * x1 * bp
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_load_totals(dim):
    _, _, sv, stri, D = _load(dim, lambda x: np.ones(len(x)))
    assert abs(D.q.sum() - 4.0 * math.pi) < 1e-6 * 4.0 * math.pi
    _, _, sv, stri, D = _load(dim, lambda x: x[:, 0].copy())
    assert abs(D.q.sum() - 2.0 * math.pi) < 1e-6 * 2.0 * math.pi


@pytest.mark.parametrize("dim", [2, 3])
def test_load_isotropic(dim):
    _, _, _, _, D = _load(dim, lambda x: np.sin(3 * x[:, 0]) + x[:, 1] ** 2, level=2)
    shape = D.q / D.m[None, :]
    assert np.abs(shape - shape[:, :1]).max() <= 1e-14 * np.abs(shape).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_load_entries(dim):
    v, c, sv, stri, D = _load(dim, lambda x: x[:, 0].copy())
    ref = np.outer(_x1_phi_integrals(v, c), _closed_form_m(sv, stri))
    err = np.abs(D.q - ref).max() / np.abs(ref).max()
    assert err < 1e-6, err
