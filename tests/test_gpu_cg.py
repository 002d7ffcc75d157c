"""E_0^{-1} by the sliced-ELL CG (every direction block in the same launches, Jacobi
preconditioning, per-direction early exit; Sec. 5.3) against the oracle's sparse LU of each
block, and the solves that use it.

* FP64 vectors at cg_tol 1e-13: 1e-10 relative, on a 2D and a 3D mesh with blockwise media,
  including a zero right-hand side in one direction (that direction takes no iteration and
  returns 0) and bitwise repeatability (all sums in a fixed order).
* FP32 vectors and values (precision MIXED): the solve stops at a relative residual of 1e-6,
  so the error is bounded by the block's condition number times that; 1e-4 is asserted on
  these small blocks.
* End to end: an FP64 solve with the CG E_0 against the oracle's iterate (1e-10), and a mixed
  solve within 1e-6 of it.
* The served form's 3D request (32^3 cubes in Kuhn tetrahedra, 512 sphere triangles, g = 0.8):
  sampled directions of E_0^{-1} against the oracle's LU, and a mixed-precision solve to a
  relative residual of 1e-6 whose residual is recomputed in FP64 with the exact odd inverse.
"""
import time

import numpy as np
import pytest

from oracle.discretize import discretize_instance
from oracle.operators import Operators
from oracle.solver import richardson
from paper_2102_09038_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def to_dev(U):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(U, dtype=np.float64).T)).cuda()


def from_dev(t):
    return t.cpu().numpy().T


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


CASES = {
    "2d-24x24-s128": lambda: inputs.make_instance("cg-2d-24", 2, 24, 2, 0.8, 0.95, block=8, seed=31, n_even=0, n_odd=5,
                                                  l=3, quad_level=2),
    "3d-6x6x6-s32": lambda: inputs.make_instance("cg-3d-6", 3, 6, 1, 0.8, 0.9, block=2, seed=32, n_even=0, n_odd=3,
                                                 l=3, quad_level=2),
}


@pytest.fixture(scope="module", params=list(CASES))
def cgcase(request):
    from paper_2102_09038_amd import rte
    inst = CASES[request.param]()
    print(f"[cg {request.param}] nR+={len(inst.vert)} nS+={len(inst.stri) // 2}", flush=True)
    D = discretize_instance(inst)
    ops = Operators(D, n_even=inst.n_even, n_odd=inst.n_odd)
    h = rte.Handle.from_instance(inst, e0_solver=rte.RTE_E0_CG, mixed=1)
    yield request.param, inst, D, ops, h
    h.close()


def test_cg_fp64(cgcase):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h = cgcase
    B = np.random.default_rng(51).standard_normal((D.nRp, D.nS))
    B[:, 1] = 0.0
    o = rte.default_solve_opts(e0_solver=rte.RTE_E0_CG, cg_tol=1e-13, cg_max_iter=20000)
    X = torch.empty_like(to_dev(B))
    h.apply_E0inv(to_dev(B), X, o)
    ref = ops.E0_solve(B)
    err = rel(from_dev(X), ref)
    print(f"[{name}] CG FP64 {err:.2e}")
    assert err < 1e-10
    assert torch.count_nonzero(X[1]) == 0
    X2 = torch.empty_like(X)
    h.apply_E0inv(to_dev(B), X2, o)
    assert torch.equal(X, X2)


def test_cg_fp32(cgcase):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h = cgcase
    B = np.random.default_rng(52).standard_normal((D.nRp, D.nS))
    o = rte.default_solve_opts(e0_solver=rte.RTE_E0_CG, precision=rte.RTE_MIXED, cg_max_iter=20000)
    X = torch.empty_like(to_dev(B))
    h.apply_E0inv(to_dev(B), X, o)
    err = rel(from_dev(X), ops.E0_solve(B))
    print(f"[{name}] CG FP32 {err:.2e}")
    assert err < 1e-4


def test_cg_solves(cgcase):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h = cgcase
    odd = rte.RTE_ODD_CONDENSED
    o = rte.default_solve_opts(l=inst.l, tol=1e-12, max_iter=400, odd_solver=odd, e0_solver=rte.RTE_E0_CG,
                               cg_tol=1e-13, cg_max_iter=20000)
    uref, rinfo = richardson(ops, l=inst.l, tol=1e-12, max_iter=400)
    U = torch.empty((D.nS, D.nRp), dtype=torch.float64, device="cuda")
    st, info = h.solve(U, opts=o)
    err = rel(from_dev(U), uref)
    print(f"[{name}] FP64 solve with CG E_0: {info.iters} iters (oracle {rinfo['iters']}), {err:.2e}, "
          f"CG iterations {info.cg_iters_total} (max {info.cg_iters_max})")
    assert info.rel_resid <= 1e-12 and err < 1e-10 and abs(info.iters - rinfo["iters"]) <= 1
    om = rte.default_solve_opts(l=inst.l, tol=1e-10, max_iter=400, odd_solver=odd, e0_solver=rte.RTE_E0_CG,
                                precision=rte.RTE_MIXED, cg_max_iter=20000)
    Um = torch.empty_like(U)
    st, mi = h.solve(Um, opts=om)
    em = rel(from_dev(Um), uref)
    print(f"[{name}] mixed solve with FP32 CG E_0: {mi.iters} iters, {em:.2e}")
    assert mi.rel_resid <= 1e-10 and em < 1e-6


def test_cg_3d_request_full_size():
    """The served form's large 3D request at full size."""
    import scipy.sparse.linalg as spla
    from paper_2102_09038_amd import rte
    inst = inputs.make_instance("req-3d-32-s512", 3, 32, 3, 0.8, 0.9, seed=1001, n_even=0, n_odd=5, l=4, tol=1e-6)
    print(f"[3d] {inst.name}: nR+ {len(inst.vert)}, r_q {inst.quad_level}", flush=True)
    t0 = time.perf_counter()
    h = rte.Handle.from_instance(inst, e0_solver=rte.RTE_E0_CG, mixed=2, odd_eig=0, coarse_solver=rte.RTE_COARSE_QUICK)
    print(f"[3d] assembled in {time.perf_counter() - t0:.1f} s", flush=True)
    D = discretize_instance(inst, with_scattering=False)
    ops = Operators(D, n_even=0, n_odd=5)
    B = np.random.default_rng(53).standard_normal((D.nRp, D.nS))
    X = torch.empty_like(to_dev(B))
    h.apply_E0inv(to_dev(B), X, rte.default_solve_opts(e0_solver=rte.RTE_E0_CG, cg_tol=1e-12, cg_max_iter=20000))
    Xg = from_dev(X)
    for k in (0, 100, D.nS - 1):
        ref = spla.splu(ops.E0_block(k)).solve(B[:, k])
        e = rel(Xg[:, k], ref)
        print(f"[3d] E_0^-1 direction {k}: {e:.2e}", flush=True)
        assert e < 1e-9
    o = rte.default_solve_opts(l=4, tol=1e-6, max_iter=400, odd_solver=rte.RTE_ODD_CONDENSED, e0_solver=rte.RTE_E0_CG,
                               precision=rte.RTE_MIXED, cg_max_iter=20000, profile=1)
    U = torch.empty((D.nS, D.nRp), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, info = h.solve(U, opts=o)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"[3d] mixed solve: {info.iters} iters in {dt:.2f} s (E_0^-1 {info.t_e0inv:.2f} s over {info.n_e0inv} "
          f"applications), CG iterations max {info.cg_iters_max}", flush=True)
    assert info.rel_resid <= 1e-6
    # the residual recomputed in FP64 (the condensed FP64 E and the FP64 scatter GEMM)
    EU = torch.empty_like(U)
    h.apply_E(U, EU, rte.default_solve_opts(odd_solver=rte.RTE_ODD_CONDENSED))
    KU = torch.empty_like(U)
    h.apply_scatter(1, U, KU)
    q = torch.from_numpy(np.ascontiguousarray(h.get_array(rte.ARRAY_Q, (D.nRp, D.nS)).T)).cuda()
    r = float(torch.linalg.norm(EU - KU - q) / torch.linalg.norm(q))
    print(f"[3d] recomputed relative residual {r:.2e}")
    assert r <= 1.01e-6
    h.close()


def test_apply_E0(cgcase):
    """The CG's SpMV kernel (rte_apply_E0) against the oracle's E_0 blocks."""
    name, inst, D, ops, h = cgcase
    X = np.random.default_rng(54).standard_normal((D.nRp, D.nS))
    Y = torch.empty_like(to_dev(X))
    h.apply_E0(to_dev(X), Y)
    err = rel(from_dev(Y), ops.E0_apply(X))
    print(f"[{name}] E_0 X {err:.2e}")
    assert err < 1e-13
