"""Convergence rates of the Richardson iteration on the device (paper Sec. 6.2).

The iteration matrix of Alg. 3 is T = I - P_2 P_1 A with A = E - K+.  Its spectral radius rho
and its A-norm eta (eta^2 = largest eigenvalue of (I - P_1 A)(I - P_G)(I - P_1 A) =
(I - P_1 A) T, an A-self-adjoint operator when P_1 is the fixed SPD P_1^l) are estimated by
Krylov methods whose every operator application is a librte call:
* rho: Arnoldi on T (Euclidean inner product, twice-orthogonalised basis); the eigenvalues
  of T are real and in [0, 1) because it is similar to the A-self-adjoint
  (I - P_G)(I - P_1 A)(I - P_G).
* eta: Lanczos on (I - P_1 A) T in the A inner product, with full reorthogonalisation.
Each stops when its estimate changes by less than tol (relative) over 5 steps, or after m
steps.  The small projected eigenproblems are solved on the host.
"""
from __future__ import annotations

import numpy as np

from . import rte


def iteration_rates(h, opts, m: int = 60, tol: float = 1e-5, seed: int = 0, want=("rho", "eta")):
    import torch
    d = h.dims
    shape = (d.nSp, d.nRp)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    Kv = torch.empty(shape, dtype=torch.float64, device="cuda")

    def A(v):
        y = torch.empty_like(v)
        h.apply_E(v, y, opts)
        h.apply_scatter(1, v, Kv)
        return y - Kv

    def prec(which, v):
        y = torch.empty_like(v)
        h.precond(which, v, y, opts)
        return y

    def T(v):
        return v - prec(1, A(v))

    out = {}
    if "rho" in want:
        V = [torch.randn(shape, dtype=torch.float64, device="cuda", generator=gen)]
        V[0] /= torch.linalg.norm(V[0])
        H = np.zeros((m + 1, m))
        hist = []
        for j in range(m):
            w = T(V[j])
            for _ in range(2):
                for i in range(j + 1):
                    c = float(torch.sum(V[i] * w))
                    H[i, j] += c
                    w -= c * V[i]
            H[j + 1, j] = float(torch.linalg.norm(w))
            hist.append(float(np.max(np.abs(np.linalg.eigvals(H[:j + 1, :j + 1])))))
            if H[j + 1, j] <= 1e-14 * abs(H[0, 0]) or (j >= 5 and abs(hist[-1] - hist[-6]) <= tol * hist[-1]):
                break
            V.append(w / H[j + 1, j])
        out["rho"] = hist[-1]
        out["rho_steps"] = len(hist)
    if "eta" in want:
        v = torch.randn(shape, dtype=torch.float64, device="cuda", generator=gen)
        Av = A(v)
        nv = float(torch.sum(v * Av)) ** 0.5
        V, AV = [v / nv], [Av / nv]
        Hs = np.zeros((m, m))
        hist = []
        for j in range(m):
            Tv = T(V[j])
            w = Tv - prec(0, A(Tv))                   # (I - P_1 A) T v_j
            for _ in range(2):
                for i in range(j + 1):
                    c = float(torch.sum(w * AV[i]))  # <w, v_i>_A
                    Hs[i, j] += c
                    w -= c * V[i]
            Aw = A(w)
            beta = max(float(torch.sum(w * Aw)), 0.0) ** 0.5
            S = 0.5 * (Hs[:j + 1, :j + 1] + Hs[:j + 1, :j + 1].T)
            hist.append(max(float(np.linalg.eigvalsh(S).max()), 0.0) ** 0.5)
            if j + 1 == m or beta <= 1e-14 or (j >= 5 and abs(hist[-1] - hist[-6]) <= tol * hist[-1]):
                break
            Hs[j + 1, j] = beta
            V.append(w / beta)
            AV.append(Aw / beta)
        out["eta"] = hist[-1]
        out["eta_steps"] = len(hist)
    return out
