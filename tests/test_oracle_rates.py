"""Pins of the oracle's dense convergence rates (Sec. 6.2): rho <= eta <= c (Lemma in Sec. 5.3),
the eigenvalues of the iteration matrix are real and in [0, 1), the paper's symmetric form of
eta^2 agrees with lambda_max(T^T A T, A), and a pure absorber gives T = 0."""
import numpy as np
import pytest

from oracle.discretize import discretize_instance
from oracle.operators import Operators
from oracle.rates import rates_dense
from paper_2102_09038_amd.inputs import tiny_instance


@pytest.mark.parametrize("g,l,n_even", [(0.0, 1, 0), (0.7, 2, 2), (0.9, 3, 0)])
def test_rate_bounds_and_forms(g, l, n_even):
    inst = tiny_instance(n=3, sphere_level=1, g=g, ratio=0.95, n_even=n_even)
    D = discretize_instance(inst)
    ops = Operators(D, n_even=n_even, n_odd=inst.n_odd)
    rho, eta, eta_sym, ev = rates_dense(ops, l)
    assert np.abs(ev.imag).max() <= 1e-10
    assert ev.real.min() >= -1e-10 and ev.real.max() < 1
    assert rho <= eta + 1e-12 <= D.c + 1e-9
    assert abs(eta - eta_sym) <= 1e-8
    assert rho > 0.05


def test_pure_absorber_rates_vanish():
    inst = tiny_instance(n=3, sphere_level=1, g=0.7, ratio=0.0, n_even=0)
    D = discretize_instance(inst)
    rho, eta, _, _ = rates_dense(Operators(D, n_even=0, n_odd=inst.n_odd), 1)
    assert rho <= 1e-10 and eta <= 1e-10
