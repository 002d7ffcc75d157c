"""Convergence rates of the Richardson iteration (paper Sec. 6.2) by dense linear algebra on
tiny meshes.  Test infrastructure only.

The iteration matrix of Alg. 3 is T = I - P_2 P_1 (E - K+) = (I - P_G)(I - P_1 (E - K+)).
* rho = spectral radius of T.
* eta = its norm in the (E - K+) energy norm: eta^2 = lambda_max(T^T A T, A), A = E - K+.
  Sec. 6.2 rewrites it, since P_G is an A-orthogonal projection and P_1 is A-symmetric, as
  the largest eigenvalue of (I - P_1 A)(I - P_G)(I - P_1 A) = (I - P_1 A) T; both forms are
  returned so that tests can check they agree.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .operators import Operators


def _dense(op, nR, nS):
    n = nR * nS
    cols = []
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        cols.append(op(e.reshape(nR, nS, order="F")).reshape(-1, order="F"))
    return np.array(cols).T


def rates_dense(ops: Operators, l: int, inner: str = "richardson"):
    """(rho, eta, eta from the paper's symmetric form, eigenvalues of T)."""
    D = ops.D
    nR, nS = D.nRp, D.nS
    A = _dense(ops.EmK, nR, nS)
    P2P1 = _dense(lambda X: ops.P2P1(X, l, inner=inner), nR, nS)
    P1 = _dense(lambda X: ops.P1(X, l) if inner == "richardson" else ops.P1_pcg(X, l), nR, nS)
    I = np.eye(nR * nS)
    T = I - P2P1 @ A
    ev = np.linalg.eigvals(T)
    rho = float(np.max(np.abs(ev)))
    eta = float(np.sqrt(max(sla.eigh(T.T @ A @ T, A, eigvals_only=True).max(), 0.0)))
    B = (I - P1 @ A) @ T
    eta_sym = float(np.sqrt(max(np.max(np.linalg.eigvals(B).real), 0.0)))
    return rho, eta, eta_sym, ev
