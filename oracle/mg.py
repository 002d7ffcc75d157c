"""Geometric multigrid for the E_0 blocks on lattice meshes, and CG preconditioned by it.

TEST INFRASTRUCTURE ONLY (see the package docstring): plain SciPy sparse algebra, one
direction block at a time.

Sec. 5.5 names multigrid as the solver of the E_0 blocks (each an anisotropic
diffusion-reaction problem on the P1 space).  The construction is this oracle's reading of
that remark:

* Meshes: the Freudenthal (Kuhn) triangulation of a box with n cells per axis, vertex
  (i, j[, k]) numbered i + m (j + m k), m = n + 1, every cell edge joining lattice points
  whose difference has entries in {0, 1}.  Halving n gives the triangulation with cells
  twice as large in the same orientation; each coarse cell is a union of fine cells, so the
  coarse P1 space lies inside the fine one.
* Prolongation P (the P1 interpolant): fine vertex 2I takes coarse vertex I; a fine vertex
  with odd coordinates on a set S of axes is the midpoint of the coarse edge from
  floor(f / 2) to ceil(f / 2) and takes half of each end.
* Coarse operators: Galerkin, A_{l+1} = P^T A_l P.  Levels are added while the cell count per
  axis is even and at least 4.
* Smoother: the Chebyshev iteration on D^{-1} A (D = diag A) over the interval
  [lo * lam, lam], lam = max_i sum_j |a_ij| / a_ii (Gershgorin's bound on the spectrum of
  D^{-1} A); the three-term recurrence of Saad, Iterative Methods for Sparse Linear Systems
  (2nd ed.), Alg. 12.1, from a given start.
* V-cycle z = B r: nu Chebyshev steps from 0, residual, restriction by P^T, the next level's
  cycle, correction by P, nu Chebyshev steps; on the coarsest level nu_c steps from 0.
  Pre- and post-smoothing use the same polynomial, so B is symmetric.
* CG preconditioned by one V-cycle per iteration, from x = 0, stopping when
  r.r <= tol^2 b.b (the stopping rule of the all-direction CG).
* Smoother precision: the cycle may work on every level's matrix rounded entry by entry to
  FP32 or to BF16 (round to nearest even, BF16 by way of FP32), its Jacobi scaling and
  Gershgorin bound taken from the rounded matrix; the CG's own products keep the exact E_0.
  The rounded matrices are symmetric, so the cycle stays a fixed symmetric operator.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

# smoother settings of the reading above
NU = 4            # Chebyshev steps before and after the coarse correction
LO = 0.02         # lower end of the smoothing interval, as a fraction of lam
NU_COARSE = 8     # Chebyshev steps on the coarsest level
LO_COARSE = 0.02


def lattice_size(vert: np.ndarray, d: int) -> int | None:
    """m (vertices per axis) when vert is the lattice of a box, numbered i + m (j + m k)."""
    nv = vert.shape[0]
    m = int(round(nv ** (1.0 / d)))
    if m ** d != nv or m < 2:
        return None
    lo, hi = vert[:, :d].min(axis=0), vert[:, :d].max(axis=0)
    idx = np.arange(nv)
    for a in range(d):
        coord = (idx // m ** a) % m
        if not np.allclose(vert[:, a], lo[a] + (hi[a] - lo[a]) * coord / (m - 1), rtol=0, atol=1e-12):
            return None
    return m


def prolongation(m: int, d: int) -> sp.csr_matrix:
    """P1 interpolation from the lattice with (m + 1) / 2 vertices per axis to the one with m."""
    assert m % 2 == 1
    mc = (m + 1) // 2
    rows, cols, vals = [], [], []
    for f, c in enumerate(itertools.product(range(m), repeat=d)):
        c = c[::-1]                                   # (i, j[, k]) with i fastest
        lo = [x // 2 for x in c]
        hi = [(x + 1) // 2 for x in c]
        il = sum(lo[a] * mc ** a for a in range(d))
        ih = sum(hi[a] * mc ** a for a in range(d))
        if il == ih:
            rows.append(f); cols.append(il); vals.append(1.0)
        else:
            rows += [f, f]; cols += [il, ih]; vals += [0.5, 0.5]
    return sp.csr_matrix((vals, (rows, cols)), shape=(m ** d, mc ** d))


def level_sizes(m: int) -> list[int]:
    """Vertices per axis of every level, finest first."""
    out = [m]
    while (out[-1] - 1) % 2 == 0 and out[-1] - 1 >= 4:
        out.append((out[-1] - 1) // 2 + 1)
    return out


def round_f32(v: np.ndarray) -> np.ndarray:
    """Each value rounded to the nearest FP32 number (ties to even), as FP64."""
    return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(v: np.ndarray) -> np.ndarray:
    """Each value rounded to FP32, then to the nearest BF16 number (ties to even), as FP64."""
    u = np.asarray(v, dtype=np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def hierarchy(A: sp.spmatrix, m: int, d: int, smoother: str | None = None) -> list[dict]:
    """Levels finest first: operator, prolongation to the finer level, Jacobi scaling and the
    Gershgorin bound lam of D^{-1} A.  smoother "f32" or "bf16": every level's operator (the
    Galerkin products taken exactly, then rounded) in that precision."""
    rnd = {None: None, "f32": round_f32, "bf16": round_bf16}[smoother]
    sizes = level_sizes(m)
    levels = []
    Al = sp.csr_matrix(A)
    for li, ml in enumerate(sizes):
        As = Al
        if rnd is not None:
            As = Al.copy()
            As.data = rnd(As.data)
        dg = As.diagonal()
        lam = float(np.max(np.asarray(abs(As).sum(axis=1)).ravel() / dg))
        lev = {"A": As, "m": ml, "dinv": 1.0 / dg, "lam": lam}
        levels.append(lev)
        if li + 1 < len(sizes):
            P = prolongation(ml, d)
            lev["P"] = P
            Al = sp.csr_matrix(P.T @ Al @ P)
    return levels


def chebyshev(A, dinv, lam, lo, nu, b, x=None):
    """nu steps of the Chebyshev iteration for A x = b, Jacobi-scaled, on [lo lam, lam]."""
    lmax, lmin = lam, lo * lam
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    sigma = theta / delta
    x = np.zeros_like(b) if x is None else x.copy()
    r = b - A @ x
    dk = dinv * r / theta
    rho = 1.0 / sigma
    for j in range(nu):
        x = x + dk
        if j + 1 == nu:
            break
        r = r - A @ dk
        rho_new = 1.0 / (2.0 * sigma - rho)
        dk = rho_new * rho * dk + (2.0 * rho_new / delta) * (dinv * r)
        rho = rho_new
    return x


def vcycle(levels, r, l=0, nu=NU, lo=LO, nu_c=NU_COARSE, lo_c=LO_COARSE):
    """z = B r on level l (the V-cycle of the module docstring)."""
    L = levels[l]
    if l == len(levels) - 1:
        return chebyshev(L["A"], L["dinv"], L["lam"], lo_c, nu_c, r)
    x = chebyshev(L["A"], L["dinv"], L["lam"], lo, nu, r)
    res = r - L["A"] @ x
    e = vcycle(levels, L["P"].T @ res, l + 1, nu, lo, nu_c, lo_c)
    x = x + L["P"] @ e
    return chebyshev(L["A"], L["dinv"], L["lam"], lo, nu, r, x)


def mg_cg(A, b, m, d, tol, maxit=1000, levels=None, smoother=None):
    """CG on A x = b preconditioned by one V-cycle per iteration (Saad, Alg. 9.1), x_0 = 0.
    Returns (x, iterations)."""
    levels = hierarchy(A, m, d, smoother) if levels is None else levels
    x = np.zeros_like(b)
    bb = float(b @ b)
    if bb == 0.0:
        return x, 0
    r = b.copy()
    z = vcycle(levels, r)
    p = z.copy()
    rz = float(r @ z)
    for it in range(maxit):
        q = A @ p
        pq = float(p @ q)
        a = rz / pq if pq != 0.0 else 0.0
        x = x + a * p
        r = r - a * q
        if float(r @ r) <= tol * tol * bb:
            return x, it + 1
        z = vcycle(levels, r)
        rzn = float(r @ z)
        beta = rzn / rz if rz != 0.0 else 0.0
        p = z + beta * p
        rz = rzn
    return x, maxit
