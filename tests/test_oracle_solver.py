"""Pins of the oracle's operators and Richardson iteration (Secs. 3-5).

* The Richardson iterate equals the even block of a direct sparse LU of the full
  mixed system (Sec. 4) on tiny 2D and 3D meshes.
* Fixed point: the exact solution is left unchanged by one step (reading of the
  correction right-hand side, Sec. 5.4 vs Alg. 3).
* Conservation: with the test function 1 (A 1 = 0), 1^T (M+ + R - K+) u = 1^T q.
* Pure absorber sigma_s = 0: E_0 = E, K+ = 0, and one step with l = 1 is exact.
* g = 0: the odd preconditioner of the Sec. 5.1 lemma is exact (K- = 0) and
  P_1^l = E_0^{-1} = E^{-1} for every l (Sec. 6.2).
* The lemma's formula inverts M- - K-_N, K-_N = (M W_N Lambda_N W_N^T M) (x) Ms-.
* Spectral equivalences (1 - cg) E_0 <= E <= E_0 (Sec. 5.3) and
  (1 - c lambda_{d+1}) (M- - K-_N) <= M- - K- <= M- - K-_N (Sec. 2.6 / 5.1).
* Contraction: the iteration matrix (I - P_G)(I - P_1 (E - K)) factorises as stated
  in Sec. 5, P_G is idempotent, and its (E-K)-norm eta is <= c (Lemma in Sec. 5.3).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.discretize import discretize_instance
from oracle.mixed import solve_mixed
from oracle.operators import Operators
from oracle.solver import richardson, richardson_step
from paper_2102_09038_amd.inputs import tiny_instance


def build(**kw):
    inst = tiny_instance(**kw)
    D = discretize_instance(inst)
    return inst, D, Operators(D, n_even=inst.n_even, n_odd=inst.n_odd)


def dense(op, n_rows, n_cols):
    cols = []
    for j in range(n_rows * n_cols):
        e = np.zeros(n_rows * n_cols); e[j] = 1.0
        cols.append(op(e.reshape(n_rows, n_cols, order="F")).reshape(-1, order="F"))
    return np.array(cols).T


@pytest.mark.parametrize("kw", [
    dict(n=4, sphere_level=1, g=0.5, ratio=0.9),
    dict(n=3, sphere_level=1, g=0.8, ratio=0.95, n_even=0, l=3),
    dict(n=2, sphere_level=0, g=0.6, ratio=0.9, dim=3, n_even=2, n_odd=1),
])
def test_richardson_matches_mixed_lu(kw):
    inst, D, ops = build(**kw)
    u, info = richardson(ops, l=inst.l, tol=1e-13, max_iter=200)
    up, _ = solve_mixed(D)
    assert info["rel_resid"] <= 1e-13
    assert np.linalg.norm(u - up) <= 1e-11 * np.linalg.norm(up)
    # energy decreases monotonically (Sec. 3)
    hist = info["stop_quantity"]
    assert all(hist[i + 1] < hist[i] for i in range(len(hist) - 1))


def test_fixed_point_and_conservation():
    inst, D, ops = build(n=4, sphere_level=1, g=0.5, ratio=0.9)
    up, _ = solve_mixed(D)
    u1 = richardson_step(ops, up, inst.l)
    assert np.linalg.norm(u1 - up) <= 1e-12 * np.linalg.norm(up)
    lhs = np.sum(ops.M_even(up) + ops.R(up) - ops.K_even(up))
    assert abs(lhs - np.sum(D.q)) <= 1e-12 * abs(np.sum(D.q))
    assert np.abs(ops.A(np.ones((D.nRp, D.nS)))).max() < 1e-14


def test_pure_absorber():
    inst, D, ops = build(n=4, sphere_level=1, g=0.5, ratio=0.0)
    U = np.random.default_rng(1).standard_normal((D.nRp, D.nS))
    assert np.allclose(ops.E0_apply(U), ops.E(U), rtol=1e-13, atol=1e-13 * np.abs(ops.E(U)).max())
    assert np.abs(ops.K_even(U)).max() == 0.0
    u1 = richardson_step(ops, np.zeros_like(D.q), 1)
    up, _ = solve_mixed(D)
    assert np.linalg.norm(u1 - up) <= 1e-12 * np.linalg.norm(up)


def test_isotropic_preconditioners_exact():
    inst, D, ops = build(n=3, sphere_level=1, g=0.0, ratio=0.9)
    rng = np.random.default_rng(2)
    B = rng.standard_normal((D.nRm, 3 * D.nS))
    assert np.allclose(ops.odd_precond(B), ops.odd_solve(B), rtol=1e-12, atol=1e-12)
    R = rng.standard_normal((D.nRp, D.nS))
    E0r = ops.E0_solve(R)
    for l in (1, 3):
        assert np.allclose(ops.P1(R, l), E0r, rtol=1e-11, atol=1e-11 * np.abs(E0r).max())
    assert np.allclose(ops.E(E0r), R, atol=1e-10 * np.abs(R).max())


def test_odd_preconditioner_inverts_truncated_operator():
    inst, D, ops = build(n=3, sphere_level=1, g=0.7, ratio=0.9, n_odd=1)
    lam, W = ops.odd_eig()
    dN = 3
    SN = ops.MSm @ W[:, :dN] @ np.diag(lam[:dN]) @ W[:, :dN].T @ ops.MSm
    B = np.random.default_rng(3).standard_normal((D.nRm, 3 * D.nS))
    X = ops.odd_precond(B, dN=dN)
    back = ops.M_odd(X) - D.ms[:, None] * (X @ SN)
    assert np.allclose(back, B, rtol=1e-10, atol=1e-10 * np.abs(B).max())
    assert np.allclose(W.T @ ops.MSm @ W, np.eye(W.shape[0]), atol=1e-10)


def test_spectral_equivalences():
    inst, D, ops = build(n=3, sphere_level=1, g=0.7, ratio=0.9)
    n = D.nRp * D.nS
    E = dense(ops.E, D.nRp, D.nS)
    E0 = dense(ops.E0_apply, D.nRp, D.nS)
    assert np.allclose(E, E.T, atol=1e-12 * np.abs(E).max())
    ev = sla.eigh(E, E0, eigvals_only=True)
    cg = D.c * D.g
    lam, W = ops.odd_eig()
    # E <= E_0 needs the odd spectrum bounded by g; the discrete top eigenvalue exceeds
    # g by the quadrature defect, which enters the constant exactly:
    # (M- - K-)^{-1} <= (1 - c lam_max)^{-1} M-^{-1}.
    upper = max(1.0, (1 - cg) / (1 - D.c * lam[0]))
    assert 0 < lam[0] - D.g < 1e-5
    assert ev.min() >= 1 - cg - 1e-10 and ev.max() <= upper + 1e-10
    assert ev.max() > 1 - 1e-6   # the bound is attained up to the defect
    # odd operator vs its truncation, on the angular factor (block per cell)
    dN = 6
    SN = ops.MSm @ W[:, :dN] @ np.diag(lam[:dN]) @ W[:, :dN].T @ ops.MSm
    c = D.c
    ev2 = sla.eigh(ops.MSm - c * D.Sm, ops.MSm - c * SN, eigvals_only=True)
    assert ev2.min() >= 1 - c * lam[dN] - 1e-10 and ev2.max() <= 1 + 1e-10


@pytest.mark.parametrize("g,l", [(0.5, 1), (0.5, 3), (0.9, 2)])
def test_contraction_and_factorisation(g, l):
    inst, D, ops = build(n=3, sphere_level=1, g=g, ratio=0.95, n_even=2)
    nR, nS = D.nRp, D.nS
    EmK = dense(ops.EmK, nR, nS)
    P1 = dense(lambda X: ops.P1(X, l), nR, nS)
    P2P1 = dense(lambda X: ops.P2P1(X, l), nR, nS)
    Wang, _ = ops.even_eig()
    Wfull = np.kron(Wang, np.eye(nR))
    PG = Wfull @ np.linalg.solve(Wfull.T @ EmK @ Wfull, Wfull.T @ EmK)
    I = np.eye(nR * nS)
    it = I - P2P1 @ EmK
    assert np.allclose(it, (I - PG) @ (I - P1 @ EmK), atol=1e-9)
    assert np.allclose(PG @ PG, PG, atol=1e-9)
    # eta = ||it||_{E-K} = sqrt(lambda_max(it^T EmK it, EmK))
    eta = np.sqrt(sla.eigh(it.T @ EmK @ it, EmK, eigvals_only=True).max())
    assert eta <= D.c + 1e-9
    assert np.allclose(P1, P1.T, atol=1e-9 * np.abs(P1).max())


# ---------------------------------------------------------------- non-stationary inner iteration
@pytest.mark.parametrize("l", [1, 2, 3, 5])
def test_inner_pcg_is_the_krylov_projection(l):
    """l steps of E_0-preconditioned CG from 0 reach the E-orthogonal projection of E^{-1} r
    onto span{(E_0^{-1} E)^j E_0^{-1} r, j < l}, which P1_krylov forms from an explicit basis
    and a small dense solve (no recurrence in common with P1_pcg)."""
    inst, D, ops = build(n=4, sphere_level=1, g=0.8, ratio=0.95)
    r = np.random.default_rng(50 + l).standard_normal((D.nRp, D.nS))
    z = ops.P1_pcg(r, l)
    zk = ops.P1_krylov(r, l)
    assert np.linalg.norm(z - zk) <= 1e-10 * np.linalg.norm(zk)
    # Galerkin: the residual r - E z is l2-orthogonal to the Krylov space
    basis = [ops.E0_solve(r)]
    for _ in range(l - 1):
        basis.append(ops.E0_solve(ops.E(basis[-1])))
    res = r - ops.E(z)
    for b in basis:
        assert abs(np.sum(b * res)) <= 1e-10 * np.linalg.norm(b) * np.linalg.norm(r)


def test_inner_pcg_beats_richardson_in_energy_and_terminates():
    """Its E-norm error is never above that of P_1^l r (the Richardson iterate lies in the same
    Krylov space), and with l at the system's dimension it is E^{-1} r."""
    inst, D, ops = build(n=2, sphere_level=0, g=0.9, ratio=0.99)
    n = D.nRp * D.nS
    E = dense(ops.E, D.nRp, D.nS)
    r = np.random.default_rng(60).standard_normal((D.nRp, D.nS))
    x = np.linalg.solve(E, r.reshape(-1, order="F")).reshape(r.shape, order="F")

    def enorm(v):
        f = v.reshape(-1, order="F")
        return float(np.sqrt(f @ E @ f))
    for l in (1, 2, 3, 4, 6):
        e_pcg = enorm(x - ops.P1_pcg(r, l))
        e_rich = enorm(x - ops.P1(r, l))
        assert e_pcg <= e_rich * (1 + 1e-12)
    assert np.linalg.norm(ops.P1_pcg(r, n) - x) <= 1e-10 * np.linalg.norm(x)
    assert np.array_equal(ops.P1_pcg(np.zeros_like(r), 3), np.zeros_like(r))


@pytest.mark.parametrize("kw", [
    dict(n=4, sphere_level=1, g=0.5, ratio=0.9),
    dict(n=3, sphere_level=1, g=0.9, ratio=0.99, n_even=0, l=2),
])
def test_richardson_with_inner_pcg_matches_mixed_lu(kw):
    """The outer iteration keeps its fixed point with the nonlinear inner iteration: it reaches
    the even block of the direct solve of the mixed system."""
    inst, D, ops = build(**kw)
    u, info = richardson(ops, l=inst.l, tol=1e-13, max_iter=200, inner="pcg")
    up, _ = solve_mixed(D)
    assert info["rel_resid"] <= 1e-13
    assert np.linalg.norm(u - up) <= 1e-11 * np.linalg.norm(up)
    u_r, info_r = richardson(ops, l=inst.l, tol=1e-13, max_iter=200)
    assert info["iters"] <= info_r["iters"]
