"""Pins of the oracle's derived outputs (scalar flux and particle balance, Sec. 2).

For the constant intensity u = 1 every term has a closed form, exact up to the sphere
quadrature defect (which shrinks with the sphere level):
* scalar flux: the sphere's area, 4 pi, at every vertex;
* leakage: the integral over the boundary of the integral of |s . nu| over the sphere,
  2 pi times the boundary measure;
* absorption: 4 pi times the integral of sigma_t - sigma_s over the domain.
At the converged solution the balance closes: source = absorption + leakage, because the
transport term vanishes on constants (A 1 = 0), to the solver's residual.
"""
import numpy as np
import pytest

from oracle.discretize import discretize_instance
from oracle.operators import Operators
from oracle.solver import richardson
from paper_2102_09038_amd.inputs import tiny_instance


@pytest.mark.parametrize("kw,perimeter", [
    (dict(n=4, sphere_level=1, g=0.5, ratio=0.9), 4.0),
    (dict(n=3, sphere_level=2, g=0.7, ratio=0.95), 4.0),
    (dict(n=2, sphere_level=1, g=0.6, ratio=0.9, dim=3), 6.0),
])
def test_constant_intensity_closed_forms(kw, perimeter):
    inst = tiny_instance(**kw)
    D = discretize_instance(inst)
    ops = Operators(D)
    phi, b = ops.derived(np.ones((D.nRp, D.nS)))
    assert np.allclose(phi, 4 * np.pi, rtol=1e-6, atol=0)
    assert abs(b["leakage"] - 2 * np.pi * perimeter) <= 1e-6 * 2 * np.pi * perimeter
    sigma_a = float(np.sum((D.Mt - D.Ms) @ np.ones(D.nRp)))     # integral of sigma_t - sigma_s
    assert abs(b["absorption"] - 4 * np.pi * sigma_a) <= 1e-6 * 4 * np.pi * sigma_a


def test_balance_closes_at_the_solution():
    inst = tiny_instance(n=4, sphere_level=1, g=0.8, ratio=0.95)
    D = discretize_instance(inst)
    ops = Operators(D, n_even=inst.n_even, n_odd=inst.n_odd)
    u, info = richardson(ops, l=inst.l, tol=1e-13)
    phi, b = ops.derived(u)
    assert abs(b["imbalance"]) <= 1e-11 * b["source"]
    assert b["absorption"] > 0 and b["leakage"] > 0
    # off the solution the imbalance is minus the sum of the residual's entries
    v = np.random.default_rng(70).standard_normal(u.shape)
    _, bv = ops.derived(v)
    r = ops.EmK(v) - D.q
    assert abs(bv["imbalance"] + float(np.sum(r))) <= 1e-10 * (abs(bv["absorption"]) + abs(bv["leakage"]) + bv["source"])
