"""Direct sparse LU of the full mixed system (paper Sec. 4):

    [ R + M+ - K+    -A^T    ] [u+]   [l+]
    [ A           M- - K-    ] [u-] = [l-]

with K+ = S+ (x) Ms+, K- = S- (x) Ms-, M+ = M_S+ (x) Mt+, M- = M_S- (x) Mt-,
A = sum_n A_n (x) D_n, R = blkdiag(R_k), assembled as explicit sparse Kronecker
products.  Its even block is the unique solution of the even-parity system, so it
checks the whole Schur-complement / Richardson machinery on tiny meshes.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretize import Discretization


def mixed_matrix(D: Discretization):
    Kp = sp.kron(sp.csr_matrix(D.Sp), D.Ms)
    Km = sp.kron(sp.csr_matrix(D.Sm), sp.diags(D.ms))
    Mp = sp.kron(sp.diags(D.m), D.Mt)
    Mm = sp.kron(sp.csr_matrix(D.MSm()), sp.diags(D.mt))
    A = sum(sp.kron(sp.csr_matrix(D.Aang(n)), D.D[n]) for n in range(D.d))
    R = sp.block_diag([D.Rk(k) for k in range(D.nS)])
    return sp.bmat([[R + Mp - Kp, -A.T], [A, Mm - Km]], format="csc")


def solve_mixed(D: Discretization):
    """Returns (U+ [nRp, nS], U- [nRm, 3nS]) from a direct solve (l- = 0: isotropic q)."""
    n_even = D.nRp * D.nS
    rhs = np.concatenate([D.q.reshape(-1, order="F"), np.zeros(D.nRm * 3 * D.nS)])
    x = spla.spsolve(mixed_matrix(D), rhs)
    return (x[:n_even].reshape(D.nRp, D.nS, order="F"),
            x[n_even:].reshape(D.nRm, 3 * D.nS, order="F"))
