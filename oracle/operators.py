"""Operators of the even-parity system and its preconditioners (paper Secs. 4-5).

All even-space vectors are matrices U [n_R+, n_S+] and odd-space vectors V [n_R-, n_S-]
(odd column 3k + m), vec = column stacking; Kronecker products act through the
identity of Sec. 5.1:
(B (x) C) vec X = vec(C X B^T).

Exact inner solves (independent of the HIP path's PCG / CG):
* (M- - K-)^{-1}: M- - K- = M_S- (x) Mt- - S- (x) Ms- is block diagonal over cells
  because Mt-, Ms- are diagonal (Sec. 4), so row j of Z solves
  Z[j,:] (sigma_t,j |T_j|) (M_S- - Delta_j S-) = B[j,:],  Delta_j = sigma_s,j / sigma_t,j,
  by a dense Cholesky per distinct Delta.
* E_0^{-1}: sparse LU per direction block (the paper's own choice, Sec. 6.4).
* E_c^{-1}: sparse LU of the assembled coarse matrix.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretize import Discretization


class Operators:
    def __init__(self, D: Discretization, n_even: int = 0, n_odd: int = 5):
        self.D = D
        self.n_even = n_even
        self.n_odd = n_odd
        self.MSm = D.MSm()
        self.Aang = [D.Aang(n) for n in range(D.d)]
        self.Rks = [D.Rk(k) for k in range(D.nS)]
        self._odd_fact = {}
        self._E0 = None
        self._Ec = None
        self._W = None

    # ------------------------------------------------------------------ Kronecker operators
    def K_even(self, U):
        """K+ u = (S+ (x) Ms+) u  ->  Ms+ U S+ (S+ symmetric), Sec. 4."""
        return self.D.Ms @ U @ self.D.Sp

    def K_odd(self, V):
        """K- v = (S- (x) Ms-) v  ->  Ms- V S-."""
        return self.D.ms[:, None] * (V @ self.D.Sm)

    def M_even(self, U):
        """M+ u = (M_S+ (x) Mt+) u  ->  Mt+ U M_S+."""
        return (self.D.Mt @ U) * self.D.m[None, :]

    def M_odd(self, V):
        """M- v = (M_S- (x) Mt-) v  ->  Mt- V M_S-."""
        return self.D.mt[:, None] * (V @ self.MSm)

    def A(self, U):
        """A u = sum_n (A_n (x) D_n) u  ->  sum_n D_n U A_n^T  [nRm, 3nS]."""
        return sum(self.D.D[n] @ U @ self.Aang[n].T for n in range(self.D.d))

    def At(self, V):
        """A^T v  ->  sum_n D_n^T V A_n  [nRp, nS]."""
        return sum(self.D.D[n].T @ V @ self.Aang[n] for n in range(self.D.d))

    def R(self, U):
        """R u = blkdiag(R_1..R_nS) u  ->  column k is R_k U[:,k]."""
        return np.stack([self.Rks[k] @ U[:, k] for k in range(self.D.nS)], axis=1)

    # ------------------------------------------------------------------ odd solve
    def _odd_chol(self, delta):
        key = float(delta)
        if key not in self._odd_fact:
            self._odd_fact[key] = sla.cho_factor(self.MSm - key * self.D.Sm, lower=True)
        return self._odd_fact[key]

    def odd_solve(self, B):
        """Z = (M- - K-)^{-1} B exactly, per cell (block-diagonal structure)."""
        delta = self.D.sigma_s / self.D.sigma_t
        Z = np.empty_like(B)
        for dv in np.unique(delta):
            rows = np.nonzero(delta == dv)[0]
            Z[rows] = sla.cho_solve(self._odd_chol(dv), B[rows].T).T / self.D.mt[rows, None]
        return Z

    def odd_apply(self, V):
        """(M- - K-) V."""
        return self.M_odd(V) - self.K_odd(V)

    # ------------------------------------------------------------------ E and E - K+
    def E(self, U):
        """E u = A^T (M- - K-)^{-1} A u + M+ u + R u (Schur complement, Sec. 4); Alg. 1 with an
        exact inner solve."""
        return self.At(self.odd_solve(self.A(U))) + self.M_even(U) + self.R(U)

    def EmK(self, U):
        return self.E(U) - self.K_even(U)

    # ------------------------------------------------------------------ E_0 (Sec. 5.3)
    def E0_block(self, k):
        """E_0 block k = (1-cg)^{-1} sum_{n,m<=d} 2 T_k(n,m) D_n^T Mt-^{-1} D_m + m_k Mt+ + R_k.

        Derived from E_0 = (1-cg)^{-1} A^T M-^{-1} A + R + M+ (Sec. 5.3) with
        A_n^T (M_S-)^{-1} A_m = diag_k(2 T_k(n, m)).
        """
        D = self.D
        cg = D.c * D.g
        inv_mt = sp.diags(1.0 / D.mt)
        out = D.m[k] * D.Mt + self.Rks[k]
        for n in range(D.d):
            for mm in range(D.d):
                out = out + (2.0 * D.T[k, n, mm] / (1.0 - cg)) * (D.D[n].T @ inv_mt @ D.D[mm])
        return sp.csc_matrix(out)

    def E0_apply(self, U):
        return np.stack([self.E0_block(k) @ U[:, k] for k in range(self.D.nS)], axis=1)

    def E0_solve(self, B):
        if self._E0 is None:
            self._E0 = [spla.splu(self.E0_block(k)) for k in range(self.D.nS)]
        return np.stack([self._E0[k].solve(B[:, k]) for k in range(self.D.nS)], axis=1)

    def P1(self, r, l):
        """P_1^l r (Sec. 5.3): z_0 = 0, z_{i+1} = z_i - E_0^{-1}(E z_i - r), i < l.

        Alg. 2 is printed with a loop over k = 0..l (l+1 steps) while the defining recursion and the
        complexity count ("l-1 applications of E and l applications of E_0^{-1}") give
        l steps; l steps are taken.
        """
        z = self.E0_solve(r)
        for _ in range(l - 1):
            z = z - self.E0_solve(self.E(z) - r)
        return z

    def P1_pcg(self, r, l):
        """l steps of the conjugate gradient method on E z = r preconditioned by E_0, from
        z_0 = 0: the non-stationary inner iteration Sec. 5.3 names as the better choice.
        Inner products are those of the vectorised matrices (sum of elementwise products)."""
        z = np.zeros_like(r)
        res = r.copy()
        y = self.E0_solve(res)
        p = y.copy()
        gamma = float(np.sum(res * y))
        for i in range(l):
            q = self.E(p)
            pq = float(np.sum(p * q))
            alpha = gamma / pq if pq != 0.0 else 0.0
            z = z + alpha * p
            if i + 1 == l:
                break
            res = res - alpha * q
            y = self.E0_solve(res)
            gamma_new = float(np.sum(res * y))
            beta = gamma_new / gamma if gamma != 0.0 else 0.0
            p = y + beta * p
            gamma = gamma_new
        return z

    def P1_krylov(self, r, l):
        """The result P1_pcg must reach in exact arithmetic, from its definition rather than the
        recurrence: the E-orthogonal projection of E^{-1} r onto the Krylov space
        span{(E_0^{-1} E)^j E_0^{-1} r : j < l}, i.e. z = V (V^T E V)^{-1} V^T r for a basis V.
        The basis is orthonormalised (Gram-Schmidt, twice) for a stable small solve."""
        shape = r.shape
        v = self.E0_solve(r)
        basis = []
        for j in range(l):
            w = v.reshape(-1).copy()
            for _ in range(2):
                for b in basis:
                    w -= np.dot(b, w) * b
            nw = np.linalg.norm(w)
            if nw == 0.0:
                break
            basis.append(w / nw)
            v = self.E0_solve(self.E(basis[-1].reshape(shape)))
        V = np.stack(basis, axis=1)
        EV = np.stack([self.E(V[:, j].reshape(shape)).reshape(-1) for j in range(V.shape[1])], axis=1)
        c = np.linalg.solve(V.T @ EV, V.T @ r.reshape(-1))
        return (V @ c).reshape(shape)

    # ------------------------------------------------------------------ derived outputs
    def derived(self, U):
        """Scalar flux phi = U m (the integral of the intensity over the sphere: the odd part
        integrates to zero and the even basis function of direction k has integral m_k), and
        the balance terms from testing the even equation with the constant 1: source 1^T q,
        absorption 1^T (M+ - K+) U, leakage 1^T R U (the outflow through the vacuum boundary)."""
        D = self.D
        source = float(np.sum(D.q))
        absorption = float(np.sum(self.M_even(U) - self.K_even(U)))
        leakage = float(np.sum(self.R(U)))
        return U @ D.m, {"source": source, "absorption": absorption, "leakage": leakage,
                         "imbalance": source - absorption - leakage}

    # ------------------------------------------------------------------ subspace correction
    def even_eig(self):
        """W_N+ [nS, d_N] (M_S+-orthonormal) and Lambda_N+ for the d_N = (N+1)(N+2)/2
        largest generalized eigenvalues of S+ w = lambda M_S+ w (Sec. 5.4)."""
        if self._W is None:
            dN = (self.n_even + 1) * (self.n_even + 2) // 2
            lam, W = sla.eigh(self.D.Sp, np.diag(self.D.m))
            self._W = (W[:, ::-1][:, :dN].copy(), lam[::-1][:dN].copy())
        return self._W

    def odd_eig(self):
        """Full generalized eigendecomposition of (S-, M_S-), eigenvalues non-increasing."""
        lam, W = sla.eigh(self.D.Sm, self.MSm)
        return lam[::-1].copy(), W[:, ::-1].copy()

    def Ec_matrix(self):
        """E_c = W^T (E - K+) W with W = W_N+ (x) I (correction equation, Sec. 5.4), assembled exactly.

        Blocks (a, b) over the d_N angular modes, each a sparse [nRp, nRp] matrix:
          W^T K+ W = Lambda (x) Ms+,  W^T M+ W = I (x) Mt+,
          W^T R W  = sum_k W(k,a) W(k,b) R_k,
          W^T A^T (M- - K-)^{-1} A W = sum_{n,m} D_n^T diag(G_nm(Delta_j)[a,b] / mt_j) D_m,
          G_nm(Delta) = (A_n W)^T (M_S- - Delta S-)^{-1} (A_m W).
        The paper leaves the transport block "to the reader"; this is its exact value,
        using that (M- - K-) is block diagonal over cells.
        """
        D = self.D
        W, lam = self.even_eig()
        dN = W.shape[1]
        delta = D.sigma_s / D.sigma_t
        AW = [self.Aang[n] @ W for n in range(D.d)]
        G = {}
        for dv in np.unique(delta):
            cf = self._odd_chol(dv)
            G[float(dv)] = [[AW[n].T @ sla.cho_solve(cf, AW[mm]) for mm in range(D.d)]
                            for n in range(D.d)]
        blocks = [[None] * dN for _ in range(dN)]
        for a in range(dN):
            for b in range(dN):
                blk = sp.csr_matrix((D.nRp, D.nRp))
                if a == b:
                    blk = blk + D.Mt - lam[a] * D.Ms
                for k in range(D.nS):
                    wk = W[k, a] * W[k, b]
                    if wk != 0.0:
                        blk = blk + wk * self.Rks[k]
                for n in range(D.d):
                    for mm in range(D.d):
                        coef = np.array([G[float(dv)][n][mm][a, b] for dv in delta]) / D.mt
                        blk = blk + D.D[n].T @ sp.diags(coef) @ D.D[mm]
                blocks[a][b] = blk
        return sp.csc_matrix(sp.bmat(blocks))

    def Ec_solve(self, Qc):
        """Solve E_c vec(Uc) = vec(Qc) for Qc [nRp, d_N]."""
        if self._Ec is None:
            self._Ec = spla.splu(self.Ec_matrix())
        v = self._Ec.solve(Qc.reshape(-1, order="F"))
        return v.reshape(Qc.shape, order="F")

    def P2P1(self, r, l, inner="richardson"):
        """P_2 P_1 r = s + W E_c^{-1} W^T (r - (E - K+) s), s = P_1^l r (product preconditioner,
        Sec. 5); inner="pcg" takes s from P1_pcg instead."""
        s = self.P1(r, l) if inner == "richardson" else self.P1_pcg(r, l)
        W, _ = self.even_eig()
        qc = (self.EmK(s) - r) @ W
        uc = self.Ec_solve(qc)
        return s - uc @ W.T

    # ------------------------------------------------------------------ the PCG preconditioner
    def odd_precond(self, B, dN=None):
        """(M- - K-_N)^{-1} B by the explicit formula of the lemma in Sec. 5.1:
        x = (W_N (x) I)(I (x) Mt- - Lambda_N (x) Ms-)^{-1} (W_N^T (x) I) b
            + (((M_S-)^{-1} - W_N W_N^T) (x) Mt-^{-1}) b."""
        lam, W = self.odd_eig()
        if dN is None:
            dN = (self.n_odd + 1) * (self.n_odd + 2) // 2
        WN, lN = W[:, :dN], lam[:dN]
        C = B @ WN
        C = C / (self.D.mt[:, None] - lN[None, :] * self.D.ms[:, None])
        return C @ WN.T + (np.linalg.solve(self.MSm, B.T).T - (B @ WN) @ WN.T) / self.D.mt[:, None]
