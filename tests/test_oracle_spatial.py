"""Pins of the oracle's spatial P1/P0 matrices (Sec. 4) against exact integrals.

* 1^T Mt+ 1 = sum_j sigma_t,j |T_j|; the unweighted mass integrates x exactly.
* (D_n)_{j,i} = |T_j| d_n phi_i: D_n 1 = 0 and D_n x_m = delta_nm |T_j| (linear
  functions are reproduced exactly by P1).
* boundary facets: measures add up to the perimeter / surface, normals are outward
  unit axis vectors on the unit square / cube, and each boundary block's facet mass
  integrates 1 over the boundary.
"""
import numpy as np
import pytest

from oracle.discretize import (boundary_facets, derivative_matrices, facet_mass_local,
                               p1_geometry, p1_mass)
from paper_2102_09038_amd.inputs import grid2d, grid3d


@pytest.fixture(params=[2, 3])
def mesh(request):
    if request.param == 2:
        v, c, _ = grid2d(5)
    else:
        v, c, _ = grid3d(3)
    return v, c.astype(np.int64)


def test_volumes(mesh):
    v, c = mesh
    vol, grads = p1_geometry(v, c)
    assert abs(vol.sum() - 1.0) < 1e-13 and np.all(vol > 0)
    assert np.allclose(grads.sum(1), 0.0, atol=1e-12)


def test_mass(mesh):
    v, c = mesh
    rng = np.random.default_rng(0)
    w = rng.uniform(1, 3, len(c))
    vol, _ = p1_geometry(v, c)
    M = p1_mass(v, c, w)
    assert abs(M.sum() - np.sum(w * vol)) < 1e-12
    M1 = p1_mass(v, c, np.ones(len(c)))
    d = v.shape[1]
    for n in range(d):
        assert abs(np.ones(len(v)) @ (M1 @ v[:, n]) - 0.5) < 1e-13
        # int x_n^2 = 1/3 is reproduced exactly since x_n is in P1
        assert abs(v[:, n] @ (M1 @ v[:, n]) - 1.0 / 3.0) < 1e-13
    assert np.allclose((M - M.T).toarray(), 0)


def test_derivatives(mesh):
    v, c = mesh
    vol, _ = p1_geometry(v, c)
    D = derivative_matrices(v, c)
    d = v.shape[1]
    for n in range(d):
        assert np.allclose(D[n] @ np.ones(len(v)), 0, atol=1e-14)
        for m in range(d):
            ref = vol if n == m else np.zeros_like(vol)
            assert np.allclose(D[n] @ v[:, m], ref, atol=1e-14)


def test_boundary(mesh):
    v, c = mesh
    d = v.shape[1]
    f, nu, meas = boundary_facets(v, c)
    assert abs(meas.sum() - 2 * d) < 1e-12
    assert np.allclose(np.linalg.norm(nu, axis=1), 1)
    centres = v[f].mean(1)
    # outward: the normal points from the domain centre towards the facet
    assert np.all(np.sum(nu * (centres - 0.5), axis=1) > 0)
    assert np.allclose(np.abs(nu).max(1), 1.0)
    loc = facet_mass_local(d)
    assert abs(loc.sum() - 1.0) < 1e-15
