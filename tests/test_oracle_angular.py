"""Pins of the oracle's angular assembly (Sec. 4 matrices, Sec. 1 HG kernel).

* HG normalisation 2 pi int_{-1}^{1} k(t) dt = 1 (Sec. 1), by adaptive quadrature.
* S+ 1 = M_S+ 1 and S- v_n = g M_S- v_n for v_n = coefficients of s_n: the constants
  and the linear functions s_n lie in the discrete spaces and are eigenfunctions of the
  scattering operator with eigenvalues 1 and g (Sec. 2.3); both hold up to the
  quadrature error, which must fall as the angular rule is refined.
* Spectrum of (S+-, M_S+-): eigenvalues in [0, 1] / [0, g] (Sec. 5.1), clusters at g^l
  with multiplicity 2l+1 (spherical harmonics, Sec. 2.3).
* g = 0: k = 1/(4 pi) so S+ = m m^T / (4 pi) and S- = 0 exactly (Sec. 1 and Table 1's
  g = 0 column, where the PCG needs one iteration).
* Symmetry and positive semi-definiteness of S+-.
* sum_k 2 T_k = int_S s s^T = (4 pi / 3) I; sum_k omega_k(nu) = int_S |s.nu| = 2 pi.
"""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.linalg as sla

from oracle.discretize import (angular_moments, angular_quadrature, hg_pm, omega,
                               scattering_matrices, upper_pairs)
from paper_2102_09038_amd.inputs import octahedral_sphere


@pytest.mark.parametrize("g", [0.0, 0.3, 0.9, 0.99])
def test_hg_normalisation(g):
    f = lambda t: hg_pm(2 - 2 * t, 2 + 2 * t, g)[0]
    val, _ = si.quad(f, -1, 1, points=[1.0], limit=400, epsabs=1e-13, epsrel=1e-13)
    assert abs(2 * math.pi * val - 1.0) < 1e-9


def test_hg_symmetric_pair():
    # k(-t) evaluated through |s + s'|^2 equals k evaluated at -t directly
    t = np.linspace(-1, 1, 11)
    kp, km = hg_pm(2 - 2 * t, 2 + 2 * t, 0.6)
    kp2, _ = hg_pm(2 + 2 * t, 2 - 2 * t, 0.6)
    assert np.allclose(km, kp2, rtol=1e-14)


@pytest.fixture(scope="module")
def mesh1():
    return octahedral_sphere(1)


def _assemble(mesh, g, rq):
    q = angular_quadrature(*mesh, rq)
    Sp, Sm = scattering_matrices(q, g)
    m, T = angular_moments(q)
    MSm = np.zeros_like(Sm)
    for k in range(len(m)):
        MSm[3 * k:3 * k + 3, 3 * k:3 * k + 3] = 2 * T[k]
    return q, Sp, Sm, m, T, MSm


def test_upper_pairs_and_antipodes(mesh1):
    svert, stri = mesh1
    up, partner = upper_pairs(svert, stri)
    assert len(up) == len(stri) // 2
    for t, p in zip(up, partner):
        assert np.allclose(svert[stri[t]].mean(0), -svert[stri[p]].mean(0))
    bad = stri.copy()
    bad[-1] = bad[0]
    with pytest.raises(ValueError):
        upper_pairs(svert, bad)


@pytest.mark.parametrize("g", [0.5, 0.8])
def test_row_sums_and_odd_eigvec_converge(mesh1, g):
    e_even, e_odd = [], []
    for rq in (1, 2, 3):
        q, Sp, Sm, m, T, MSm = _assemble(mesh1, g, rq)
        e_even.append(np.abs(Sp.sum(1) - m).max() / m.max())
        errs = []
        for n in range(3):
            v = np.zeros(Sm.shape[0]); v[n::3] = 1.0
            errs.append(np.abs(Sm @ v - g * (MSm @ v)).max() / np.abs(MSm @ v).max())
        e_odd.append(max(errs))
    assert e_even[-1] < 1e-4 and e_odd[-1] < 1e-4
    assert e_even[2] < e_even[0] and e_odd[2] < e_odd[0]


@pytest.mark.parametrize("g", [0.5, 0.7])
def test_spectrum_bounds_and_clusters(g):
    mesh = octahedral_sphere(2)
    q, Sp, Sm, m, T, MSm = _assemble(mesh, g, 2)
    assert np.allclose(Sp, Sp.T, rtol=0, atol=1e-14 * np.abs(Sp).max())
    assert np.allclose(Sm, Sm.T, rtol=0, atol=1e-14 * np.abs(Sm).max())
    lp = sla.eigh(Sp, np.diag(m), eigvals_only=True)[::-1]
    lm = sla.eigh(Sm, MSm, eigvals_only=True)[::-1]
    assert lp.min() > -1e-12 and lp.max() < 1 + 1e-6
    assert lm.min() > -1e-12 and lm.max() < g + 1e-6
    # even: l = 0 (1), l = 2 (5), l = 4 (9); odd: l = 1 (3), l = 3 (7), l = 5 (11)
    assert abs(lp[0] - 1.0) < 1e-6
    assert np.allclose(lp[1:6], g ** 2, rtol=0.1)
    assert np.allclose(lm[0:3], g, rtol=1e-5)
    assert np.allclose(lm[3:10], g ** 3, rtol=0.1)
    assert np.allclose(lm[10:21], g ** 5, rtol=0.25)
    # the clusters are separated from the next degree
    assert lp[5] > 1.5 * lp[6] and lm[20] > 1.5 * lm[21]


def test_isotropic_case_exact(mesh1):
    q, Sp, Sm, m, T, MSm = _assemble(mesh1, 0.0, 1)
    assert np.abs(Sm).max() == 0.0
    assert np.allclose(Sp, np.outer(m, m) / (4 * math.pi), rtol=1e-13, atol=0)


def test_moments_and_omega(mesh1):
    q = angular_quadrature(*mesh1, 3)
    m, T = angular_moments(q)
    assert abs(m.sum() - 4 * math.pi) < 1e-7
    assert np.allclose(2 * T.sum(0), 4 * math.pi / 3 * np.eye(3), atol=1e-7)
    nus = np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0], [0.6, 0.8, 0]])
    om = omega(q, nus)
    assert np.allclose(om.sum(1), 2 * math.pi, atol=1e-6)
    assert np.all(om >= 0)


def test_scattering_psd(mesh1):
    q, Sp, Sm, m, T, MSm = _assemble(mesh1, 0.7, 1)
    assert np.linalg.eigvalsh(Sp).min() > -1e-12
    assert np.linalg.eigvalsh(Sm).min() > -1e-12
