"""Galerkin matrices of the mixed even/odd discretisation (paper Sec. 4).

Spaces (Sec. 4): X_h^+ = continuous P1 on the spatial mesh (basis phi_i), X_h^- = P0
(cell indicators chi_j); S_h^+ = even piecewise constants on the sphere mesh (mu_k =
indicator of K_k and its antipode -K_k, one per antipodal pair), S_h^- = odd piecewise
linears.  Reading of the odd space (the paper only says "P1", n_S^- = 3 n_S^+): the
functions psi_(k,m) = s_m mu_k, m = 1..3, i.e. the restrictions of linear functions
of s to each antipodal pair; they are odd because s is odd and mu_k even.

Matrices (the definitions listed after the mixed system in Sec. 4, with the Kronecker layout U[i,k], spatial index fastest):

  S+_{kk'}          = int_S (S mu_k) mu_k'         = 2 int_{K_k} int_{K_k'} [k(s.s') + k(-s.s')]
  S-_{(k,n),(k',m)} = int_S (S psi_kn) psi_k'm    = 2 int_{K_k} int_{K_k'} s_n s'_m [k(s.s') - k(-s.s')]
  (M_S+)_{kk}       = 2 |K_k|,   (M_S-) block k  = 2 T_k,   T_k = int_{K_k} s s^T
  (A_n)_{(k,m),k}   = int_S s_n psi_(k,m) mu_k    = 2 T_k(n, m)
  omega_k(nu)       = int_S |s.nu| mu_k^2          = 2 int_{K_k} |s.nu|
  (Mt+)_{ii'} = int sigma_t phi_i phi_i',  (Mt-)_{jj} = sigma_t,j |T_j|   (likewise sigma_s)
  (D_n)_{j,i} = int d(phi_i)/dr_n chi_j = |T_j| d_n phi_i|_{T_j}
  (R_k)_{ii'} = int_{dR} omega_k(nu) phi_i phi_i'

k is the Henyey-Greenstein phase function (Sec. 1), evaluated through
|s - s'|^2 = 2 - 2 s.s' (the identity used in the asymptotic-smoothness proof of Sec. 5.2):
1 - 2 g t + g^2 = (1-g)^2 + g |s - s'|^2 and 1 + 2 g t + g^2 = (1-g)^2 + g |s + s'|^2.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import scipy.sparse as sp

from .quadrature import sphere_triangle_rule


# --------------------------------------------------------------------------- sphere
def upper_pairs(svert: np.ndarray, stri: np.ndarray):
    """Indices of the triangles whose centroid lies in the upper half-sphere (z > 0,
    ties broken on y then x; Sec. 4 picks triangles with midpoints in a half-sphere), in the order
    of ``stri``, and each one's antipodal partner.  Raises ValueError when the mesh is
    not antipodally symmetric."""
    cen = svert[stri].mean(axis=1)
    key = np.where(cen[:, 2] != 0, cen[:, 2], np.where(cen[:, 1] != 0, cen[:, 1], cen[:, 0]))
    up = np.nonzero(key > 0)[0]
    lookup = {}
    for t, tri in enumerate(stri):
        lookup[frozenset(tuple(np.round(svert[v], 10) + 0.0) for v in tri)] = t
    partner = []
    for t in up:
        kk = frozenset(tuple(np.round(-svert[v], 10) + 0.0) for v in stri[t])
        if kk not in lookup:
            raise ValueError(f"sphere triangle {t} has no antipodal partner")
        partner.append(lookup[kk])
    if 2 * len(up) != len(stri):
        raise ValueError("sphere mesh is not split evenly into antipodal pairs")
    return up, np.array(partner)


def hg_pm(d2, e2, g):
    """k(s.s') and k(-s.s') from d2 = |s-s'|^2, e2 = |s+s'|^2 (HG phase function, Sec. 1)."""
    c = (1.0 - g * g) / (4.0 * math.pi)
    a = (1.0 - g) ** 2 + g * d2
    b = (1.0 - g) ** 2 + g * e2
    return c / (a * np.sqrt(a)), c / (b * np.sqrt(b))


@dataclasses.dataclass
class AngularQuadrature:
    pts: np.ndarray   # [nS, Q, 3] unit vectors on each upper triangle
    wts: np.ndarray   # [nS, Q]


def angular_quadrature(svert, stri, r_q: int) -> AngularQuadrature:
    up, _ = upper_pairs(svert, stri)
    P, W = [], []
    for t in up:
        a, b, c = svert[stri[t]]
        p, w = sphere_triangle_rule(a, b, c, r_q)
        P.append(p)
        W.append(w)
    return AngularQuadrature(np.array(P), np.array(W))


def scattering_rows(q: AngularQuadrature, g: float, rows, max_pairs: int = 1 << 23):
    """Rows ``rows`` (pair indices k) of S+ [len(rows), nS] and of S- as
    [len(rows), 3, nS, 3] (entry [r, n, k', m] = S-_{(k_r,n),(k',m)}).

    The double sum over the points p of K_k and q of every K_k' is taken over slices of p
    holding at most ``max_pairs`` point pairs, so that the temporaries stay bounded at high
    quadrature levels; every entry is the same double sum, added slice by slice."""
    P, W = q.pts, q.wts
    nS, Q = P.shape[0], P.shape[1]
    Sp = np.zeros((len(rows), nS))
    Sm = np.zeros((len(rows), 3, nS, 3))
    step = max(1, max_pairs // (nS * Q))
    for r, k in enumerate(rows):
        for p0 in range(0, Q, step):
            Pk, Wk = P[k, p0:p0 + step], W[k, p0:p0 + step]
            diff = Pk[:, None, None, :] - P[None, :, :, :]         # [p, nS, Q', 3]
            summ = Pk[:, None, None, :] + P[None, :, :, :]
            d2 = np.einsum("ijkl,ijkl->ijk", diff, diff)
            e2 = np.einsum("ijkl,ijkl->ijk", summ, summ)
            kp, km = hg_pm(d2, e2, g)
            ww = Wk[:, None, None] * W[None, :, :]                 # [p, nS, Q']
            Sp[r] += 2.0 * np.einsum("pkq->k", ww * (kp + km))
            F = ww * (kp - km)
            Sm[r] += 2.0 * np.einsum("pn,pkq,kqm->nkm", Pk, F, P)
    return Sp, Sm


def scattering_matrices(q: AngularQuadrature, g: float):
    """Dense S+ [nS, nS] and S- [3nS, 3nS] (odd index 3k + m, pair-major)."""
    nS = q.pts.shape[0]
    Sp, Sm4 = scattering_rows(q, g, range(nS))
    return Sp, Sm4.reshape(3 * nS, 3 * nS)


def angular_moments(q: AngularQuadrature):
    """m_k = 2|K_k| [nS] and T_k = int_{K_k} s s^T [nS, 3, 3]."""
    m = 2.0 * q.wts.sum(axis=1)
    T = np.einsum("kp,kpi,kpj->kij", q.wts, q.pts, q.pts)
    return m, T


def omega(q: AngularQuadrature, normals: np.ndarray):
    """omega_k(nu_F) = 2 int_{K_k} |s . nu_F|  ->  [n_facet, nS]."""
    nu = np.zeros((normals.shape[0], 3))
    nu[:, : normals.shape[1]] = normals
    return 2.0 * np.einsum("kp,fkp->fk", q.wts, np.abs(np.einsum("kpi,fi->fkp", q.pts, nu)))


# --------------------------------------------------------------------------- spatial
def p1_geometry(vert: np.ndarray, cell: np.ndarray):
    """Per cell: volume [nc] and gradients of the barycentric coordinates [nc, d+1, d]."""
    d = vert.shape[1]
    X = vert[cell]                                   # [nc, d+1, d]
    J = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))  # columns = edges
    vol = np.abs(np.linalg.det(J)) / math.factorial(d)
    Jinv = np.linalg.inv(J)                          # row i = grad of lambda_{i+1}
    grads = np.concatenate([-Jinv.sum(axis=1, keepdims=True), Jinv], axis=1)
    return vol, grads


def p1_mass(vert, cell, weight):
    """int w phi_i phi_i' for piecewise-constant w: local |T| (1 + delta) / ((d+1)(d+2))."""
    d = vert.shape[1]
    vol, _ = p1_geometry(vert, cell)
    nv = len(vert)
    loc = (np.ones((d + 1, d + 1)) + np.eye(d + 1)) / ((d + 1) * (d + 2))
    rows, cols, vals = [], [], []
    for a in range(d + 1):
        for b in range(d + 1):
            rows.append(cell[:, a]); cols.append(cell[:, b])
            vals.append(weight * vol * loc[a, b])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(nv, nv))


def derivative_matrices(vert, cell):
    """D_n [n_cell, n_vert], (D_n)_{j,i} = |T_j| d_n phi_i on T_j, n = 1..d."""
    d = vert.shape[1]
    vol, grads = p1_geometry(vert, cell)
    out = []
    for n in range(d):
        rows = np.repeat(np.arange(len(cell)), d + 1)
        out.append(sp.csr_matrix(((vol[:, None] * grads[:, :, n]).ravel(), (rows, cell.ravel())),
                                 shape=(len(cell), len(vert))))
    return out


def boundary_facets(vert, cell):
    """Facets owned by exactly one cell, with their outward unit normal and measure.

    The outward normal is -grad(lambda_o)/|grad(lambda_o)| for the vertex o opposite the
    facet; the facet measure is d |T| |grad(lambda_o)|.
    """
    d = vert.shape[1]
    vol, grads = p1_geometry(vert, cell)
    owner = {}
    for c, tri in enumerate(cell):
        for o in range(d + 1):
            f = tuple(sorted(int(v) for i, v in enumerate(tri) if i != o))
            owner.setdefault(f, []).append((c, o))
    facets, normals, meas = [], [], []
    for f, own in owner.items():
        if len(own) == 1:
            c, o = own[0]
            gr = grads[c, o]
            gn = np.linalg.norm(gr)
            facets.append(f)
            normals.append(-gr / gn)
            meas.append(d * vol[c] * gn)
    order = np.lexsort(np.array(facets).T[::-1])
    return (np.array(facets, dtype=np.int64)[order], np.array(normals)[order],
            np.array(meas)[order])


def facet_mass_local(d):
    """P1 mass on a (d-1)-simplex with d vertices, divided by its measure."""
    return (np.ones((d, d)) + np.eye(d)) / (d * (d + 1))


# --------------------------------------------------------------------------- bundle
@dataclasses.dataclass
class Discretization:
    d: int
    nRp: int
    nRm: int
    nS: int                      # n_S^+ (number of antipodal pairs)
    g: float
    c: float                     # max sigma_s / sigma_t
    sigma_t: np.ndarray
    sigma_s: np.ndarray
    Mt: sp.csr_matrix            # P1 mass weighted by sigma_t
    Ms: sp.csr_matrix            # P1 mass weighted by sigma_s
    M1: sp.csr_matrix            # unweighted P1 mass
    mt: np.ndarray               # diag of P0 mass weighted by sigma_t  (= sigma_t |T|)
    ms: np.ndarray               # likewise sigma_s
    D: list                      # [d] sparse [nRm, nRp]
    facets: np.ndarray           # [nF, d] vertex indices
    fnormal: np.ndarray          # [nF, d]
    fmeas: np.ndarray            # [nF]
    Omega: np.ndarray            # [nF, nS]
    m: np.ndarray                # [nS] diag of M_S+
    T: np.ndarray                # [nS, 3, 3]
    Sp: Optional[np.ndarray]     # [nS, nS]
    Sm: Optional[np.ndarray]     # [3nS, 3nS]
    quad: AngularQuadrature
    q: np.ndarray                # [nRp, nS] even load vector l+ (matrix form)

    @property
    def nSm(self):
        return 3 * self.nS

    def MSm(self):
        """M_S^- as a dense block-diagonal matrix [3nS, 3nS]."""
        out = np.zeros((self.nSm, self.nSm))
        for k in range(self.nS):
            out[3 * k:3 * k + 3, 3 * k:3 * k + 3] = 2.0 * self.T[k]
        return out

    def Aang(self, n):
        """A_n [3nS, nS] dense: (A_n)_{(k,m),k} = 2 T_k(n,m)."""
        out = np.zeros((self.nSm, self.nS))
        for k in range(self.nS):
            out[3 * k:3 * k + 3, k] = 2.0 * self.T[k][n, :]
        return out

    def Rk(self, k):
        """Boundary block R_k = sum_F omega_k(nu_F) B_F (sparse [nRp, nRp])."""
        d = self.d
        loc = facet_mass_local(d)
        rows, cols, vals = [], [], []
        for a in range(d):
            for b in range(d):
                rows.append(self.facets[:, a]); cols.append(self.facets[:, b])
                vals.append(self.Omega[:, k] * self.fmeas * loc[a, b])
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.nRp, self.nRp))


def discretize(vert, cell, sigma_t, sigma_s, g, svert, stri, q_nodal, r_q=2,
               with_scattering=True) -> Discretization:
    """Assemble every matrix of the mixed system of Sec. 4 for one instance."""
    vert = np.asarray(vert, float)
    cell = np.asarray(cell, np.int64)
    d = vert.shape[1]
    sigma_t = np.asarray(sigma_t, float)
    sigma_s = np.asarray(sigma_s, float)
    vol, _ = p1_geometry(vert, cell)
    Mt = p1_mass(vert, cell, sigma_t)
    Ms = p1_mass(vert, cell, sigma_s)
    M1 = p1_mass(vert, cell, np.ones(len(cell)))
    D = derivative_matrices(vert, cell)
    facets, fnormal, fmeas = boundary_facets(vert, cell)
    quad = angular_quadrature(np.asarray(svert, float), np.asarray(stri), r_q)
    m, T = angular_moments(quad)
    Om = omega(quad, fnormal)
    Sp = Sm = None
    if with_scattering:
        Sp, Sm = scattering_matrices(quad, g)
    q = np.outer(M1 @ np.asarray(q_nodal, float), m)
    return Discretization(d=d, nRp=len(vert), nRm=len(cell), nS=quad.pts.shape[0], g=float(g),
                          c=float(np.max(sigma_s / sigma_t)), sigma_t=sigma_t, sigma_s=sigma_s,
                          Mt=Mt, Ms=Ms, M1=M1, mt=sigma_t * vol, ms=sigma_s * vol, D=D,
                          facets=facets, fnormal=fnormal, fmeas=fmeas, Omega=Om, m=m, T=T,
                          Sp=Sp, Sm=Sm, quad=quad, q=q)


def discretize_instance(inst, with_scattering=True) -> Discretization:
    return discretize(inst.vert, inst.cell, inst.sigma_t, inst.sigma_s, inst.g, inst.svert,
                      inst.stri, inst.q_nodal, inst.quad_level, with_scattering)
