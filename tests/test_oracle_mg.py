"""Pins of the oracle's multigrid for the E_0 blocks (oracle/mg.py), each against something
other than the code itself:

* the prolongation reproduces every linear function exactly (the coarse P1 space lies in the
  fine one on nested Freudenthal lattices);
* the Galerkin operator P^T E_0 P equals the E_0 block the oracle assembles directly on the
  mesh with twice the cell size (same media, block-aligned), in 2D and 3D and for several
  directions: nested spaces make the Galerkin product the coarse discretisation;
* the Chebyshev recurrence multiplies each eigencomponent of a diagonal problem by the
  closed form T_nu((theta - lam) / delta) / T_nu(theta / delta);
* Gershgorin's bound is an upper bound of the spectrum of D^{-1} A;
* the V-cycle is symmetric and positive definite;
* CG with the V-cycle reaches the sparse-LU solution, with iteration counts that barely grow
  when the mesh is refined (against Jacobi CG, whose counts grow with the refinement);
* the smoother-precision roundings: BF16 rounding at exact halfway points goes to the even
  neighbour, stays within half a unit in the last place, is odd-symmetric; the cycle on the
  rounded levels is still symmetric positive definite and its CG still reaches the LU solution.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import mg
from oracle.discretize import discretize_instance
from oracle.operators import Operators
from paper_2102_09038_amd import inputs


def test_level_sizes():
    assert mg.level_sizes(33) == [33, 17, 9, 5, 3]
    assert mg.level_sizes(25) == [25, 13, 7, 4]
    assert mg.level_sizes(4) == [4]
    assert mg.level_sizes(5) == [5, 3]


@pytest.mark.parametrize("d", [2, 3])
def test_lattice_detection(d):
    vert = (inputs.grid2d(6) if d == 2 else inputs.grid3d(4))[0]
    m = 7 if d == 2 else 5
    assert mg.lattice_size(vert, d) == m
    assert mg.lattice_size(3.0 * vert + 1.0, d) == m
    perm = np.arange(len(vert))
    perm[[1, 2]] = perm[[2, 1]]
    assert mg.lattice_size(vert[perm], d) is None


@pytest.mark.parametrize("d,m", [(2, 9), (3, 5), (3, 9)])
def test_prolongation_reproduces_linear_functions(d, m):
    mc = (m + 1) // 2
    P = mg.prolongation(m, d)
    rng = np.random.default_rng(3)
    fine = np.stack(np.meshgrid(*[np.arange(m)] * d, indexing="ij")[::-1], axis=-1).reshape(-1, d)
    coarse = 2.0 * np.stack(np.meshgrid(*[np.arange(mc)] * d, indexing="ij")[::-1], axis=-1).reshape(-1, d)
    for _ in range(3):
        a, b = rng.standard_normal(), rng.standard_normal(d)
        np.testing.assert_allclose(P @ (a + coarse @ b), a + fine @ b, rtol=0, atol=1e-13)
    np.testing.assert_allclose(np.asarray(P.sum(axis=1)).ravel(), 1.0)


@pytest.mark.parametrize("d,n,ks", [(2, 8, [0, 3, 7]), (3, 4, [0, 2, 5])])
def test_galerkin_is_coarse_discretisation(d, n, ks):
    blk = 4 if d == 2 else 2
    fine = inputs.make_instance("f", d, n, 1, 0.6, 0.9, block=blk, seed=5, n_even=0, n_odd=3, l=2)
    coarse = inputs.make_instance("c", d, n // 2, 1, 0.6, 0.9, block=blk // 2, seed=5, n_even=0, n_odd=3, l=2)
    assert len(np.unique(fine.sigma_t)) > 1
    Of = Operators(discretize_instance(fine, with_scattering=False), n_even=0, n_odd=3)
    Oc = Operators(discretize_instance(coarse, with_scattering=False), n_even=0, n_odd=3)
    P = mg.prolongation(n + 1, d)
    for k in ks:
        Ag = (P.T @ Of.E0_block(k) @ P).toarray()
        Ac = Oc.E0_block(k).toarray()
        np.testing.assert_allclose(Ag, Ac, rtol=0, atol=1e-12 * np.abs(Ac).max())


def test_chebyshev_closed_form():
    lam = np.linspace(0.05, 1.0, 40)
    A = sp.diags(lam)
    e0 = np.random.default_rng(1).standard_normal(lam.size)
    b = A @ e0                                       # exact solution e0; start from 0
    for lo, nu in [(0.15, 2), (0.15, 3), (0.3, 5), (0.02, 8)]:
        x = mg.chebyshev(A, np.ones_like(lam), 1.0, lo, nu, b)
        theta, delta = 0.5 * (1.0 + lo), 0.5 * (1.0 - lo)
        t = (theta - lam) / delta
        Tn = np.where(np.abs(t) <= 1, np.cos(nu * np.arccos(np.clip(t, -1, 1))),
                      np.cosh(nu * np.arccosh(np.maximum(np.abs(t), 1))) * np.sign(t) ** nu)
        factor = Tn / np.cosh(nu * np.arccosh(theta / delta))
        np.testing.assert_allclose(e0 - x, factor * e0, rtol=1e-11, atol=1e-13)


def e0_blocks(d, n, ks, seed=7):
    inst = inputs.make_instance("m", d, n, 1, 0.8, 0.9, block=max(1, n // 4), seed=seed, n_even=0, n_odd=3, l=2)
    ops = Operators(discretize_instance(inst, with_scattering=False), n_even=0, n_odd=3)
    return [sp.csr_matrix(ops.E0_block(k)) for k in ks]


def test_gershgorin_bounds_spectrum():
    A = e0_blocks(3, 4, [3])[0]
    levels = mg.hierarchy(A, 5, 3)
    for L in levels:
        Dh = sp.diags(np.sqrt(L["dinv"]))
        ev = np.linalg.eigvalsh((Dh @ L["A"] @ Dh).toarray())
        assert ev.max() <= L["lam"] * (1 + 1e-12)
        assert ev.min() > 0


@pytest.mark.parametrize("d,n", [(2, 16), (3, 4)])
def test_vcycle_symmetric_positive(d, n):
    A = e0_blocks(d, n, [1])[0]
    levels = mg.hierarchy(A, n + 1, d)
    assert len(levels) >= 2
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal(A.shape[0]), rng.standard_normal(A.shape[0])
    Bx, By = mg.vcycle(levels, x), mg.vcycle(levels, y)
    assert abs(Bx @ y - x @ By) <= 1e-12 * np.linalg.norm(Bx) * np.linalg.norm(y)
    assert x @ Bx > 0 and y @ By > 0


def cg_jacobi_iters(A, b, tol):
    it = [0]
    spla.cg(A, b, rtol=tol, maxiter=10000, M=sp.diags(1.0 / A.diagonal()), callback=lambda _: it.__setitem__(0, it[0] + 1))
    return it[0]


def test_mg_cg_solves_and_scales():
    rng = np.random.default_rng(4)
    res = {}
    for n in (4, 8):
        A = e0_blocks(3, n, [0])[0]
        b = rng.standard_normal(A.shape[0])
        x, its = mg.mg_cg(A, b, n + 1, 3, tol=1e-13)
        xr = spla.spsolve(sp.csc_matrix(A), b)
        assert np.linalg.norm(x - xr) <= 1e-10 * np.linalg.norm(xr)
        res[n] = (its, cg_jacobi_iters(A, b, 1e-8), mg.mg_cg(A, b, n + 1, 3, tol=1e-8)[1])
    print(res)
    (_, j4, m4), (_, j8, m8) = res[4], res[8]
    assert m8 < j8 / 3
    assert m8 - m4 <= 4 and j8 > j4 + 10


def test_bf16_rounding():
    one = 1.0
    assert mg.round_bf16(np.array([one + 2.0 ** -8]))[0] == 1.0                  # tie: to even (1.0)
    assert mg.round_bf16(np.array([one + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6   # tie: to even
    assert mg.round_bf16(np.array([one + 2.0 ** -8 + 2.0 ** -20]))[0] == 1.0 + 2.0 ** -7
    x = np.random.default_rng(5).standard_normal(10000) * 10.0 ** np.random.default_rng(6).uniform(-5, 5, 10000)
    r = mg.round_bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-12))
    np.testing.assert_array_equal(mg.round_bf16(-x), -r)
    assert np.all(mg.round_bf16(r) == r)                                          # idempotent
    np.testing.assert_array_equal(mg.round_f32(x), x.astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("smoother", ["f32", "bf16"])
def test_rounded_smoother_cycle(smoother):
    A = e0_blocks(3, 4, [2])[0]
    levels = mg.hierarchy(A, 5, 3, smoother)
    rng = np.random.default_rng(8)
    x, y = rng.standard_normal(A.shape[0]), rng.standard_normal(A.shape[0])
    Bx, By = mg.vcycle(levels, x), mg.vcycle(levels, y)
    assert abs(Bx @ y - x @ By) <= 1e-12 * np.linalg.norm(Bx) * np.linalg.norm(y)
    assert x @ Bx > 0 and y @ By > 0
    exact = mg.hierarchy(A, 5, 3)
    for L, E in zip(levels, exact):
        d = (L["A"] - E["A"]).toarray()
        assert np.abs(d).max() <= (2.0 ** -8 if smoother == "bf16" else 2.0 ** -24) * np.abs(E["A"].toarray()).max()
    b = rng.standard_normal(A.shape[0])
    xs, its = mg.mg_cg(A, b, 5, 3, tol=1e-13, levels=levels)
    xr = spla.spsolve(sp.csc_matrix(A), b)
    assert np.linalg.norm(xs - xr) <= 1e-10 * np.linalg.norm(xr)
