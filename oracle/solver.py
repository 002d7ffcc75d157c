"""Outer preconditioned Richardson iteration (paper Sec. 5, discrete Richardson iteration
with the product preconditioner P_2 P_1; Alg. 3).

    r_n      = (E - K+) u_n - q
    s        = P_1^l r_n
    u_{n+.5} = u_n - s
    q_c      = W^T ((E - K+) s - r_n)
    E_c u_c  = q_c
    u_{n+1}  = u_{n+.5} + W u_c

Reading: Alg. 3 prints the correction right-hand side with an extra "- q" term; with it
the exact solution would not be a fixed point (u_n = u gives r = 0, s = 0 but
q_c = -W^T q), whereas the correction equation of Sec. 5.4 gives W^T((E-K)P_1 - I) r_n.
The term is dropped.

Stopping: primary rule ||r_n||_2 <= tol ||q||_2; the paper's own quantity
||u_n - u_{n-1}||_{E-K} (Sec. 6.4) is reported alongside; it equals
sqrt(delta^T (r_n - r_{n-1})) with delta = u_n - u_{n-1}.
"""
from __future__ import annotations

import math

import numpy as np

from .operators import Operators


def richardson(ops: Operators, l: int = 4, tol: float = 1e-8, max_iter: int = 200, u0=None,
               callback=None, inner: str = "richardson"):
    """Run Alg. 3 from u0 (default 0). Returns (u, info dict).  inner="pcg" applies P_1 as
    l steps of E_0-preconditioned CG (Sec. 5.3's non-stationary alternative)."""
    D = ops.D
    q = D.q
    u = np.zeros_like(q) if u0 is None else np.array(u0, dtype=float)
    W, _ = ops.even_eig()
    qn = float(np.linalg.norm(q))
    hist, stopq = [], []
    r_prev = None
    step_prev = None
    e1 = None
    it = 0
    while True:
        r = ops.EmK(u) - q
        rel = float(np.linalg.norm(r)) / qn
        hist.append(rel)
        if step_prev is not None:
            en = math.sqrt(max(float(np.sum(step_prev * (r - r_prev))), 0.0))
            if e1 is None:
                e1 = en
            stopq.append(en / e1 if e1 > 0 else 0.0)
        if callback is not None:
            callback(it, u, r)
        if rel <= tol or it >= max_iter:
            break
        s = ops.P1(r, l) if inner == "richardson" else ops.P1_pcg(r, l)
        uc = ops.Ec_solve((ops.EmK(s) - r) @ W)
        step = -s + uc @ W.T
        u = u + step
        r_prev, step_prev = r, step
        it += 1
    return u, {"iters": it, "rel_resid": hist[-1], "history": hist, "stop_quantity": stopq}


def richardson_step(ops: Operators, u, l: int):
    """One step u -> u - P_2 P_1 ((E - K+) u - q)."""
    r = ops.EmK(u) - ops.D.q
    return u - ops.P2P1(r, l)
