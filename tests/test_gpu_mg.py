"""E_0^{-1} by CG preconditioned by the geometric multigrid V-cycle (RTE_E0_MG) against the
oracle (oracle/mg.py for the cycle, sparse LU for the blocks, the Richardson iterate for the
solve).

* One V-cycle (rte_apply_mg, FP64 vectors, the level matrices in the FP32 smoother precision)
  against the oracle's cycle on the same FP32-rounded levels on every direction, 1e-10 relative:
  2D and 3D lattices with several levels, a lattice whose coarsest level has an odd cell count,
  and one with a single level (the cycle is then eight Chebyshev steps); row counts that leave
  ragged tiles.
* E_0^{-1} in FP64 at cg_tol 1e-13 against the LU (1e-10), with a zero right-hand side in one
  direction and bitwise repeatability; FP32 (mixed) to 1e-4.  The largest per-direction
  iteration count at tol 1e-8 against the oracle's multigrid CG (within one).
* End to end: FP64 solve with the multigrid E_0 against the oracle's iterate (1e-10).
* The served form's 3D request (32^3 cubes, 512 sphere triangles): sampled directions of
  E_0^{-1} against the LU, and a mixed solve to 1e-6 whose residual is recomputed in FP64.
* A mesh that is not a lattice is refused at assembly.
* The host footprint estimate against the bytes an admitted multigrid slot holds, including the
  served 3D configuration.
"""
import time

import numpy as np
import pytest

from oracle import mg
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
    # m = 17: levels 17, 9, 5, 3
    "2d-16-s32": lambda: inputs.make_instance("mg-2d-16", 2, 16, 1, 0.8, 0.95, block=4, seed=61, n_even=0, n_odd=3,
                                              l=3, quad_level=2),
    # m = 13: levels 13, 7, 4 (the coarsest with 3 cells per axis)
    "2d-12-s128": lambda: inputs.make_instance("mg-2d-12", 2, 12, 2, 0.6, 0.9, block=3, seed=62, n_even=0, n_odd=3,
                                               l=3, quad_level=2),
    # m = 9: levels 9, 5, 3
    "3d-8-s32": lambda: inputs.make_instance("mg-3d-8", 3, 8, 1, 0.8, 0.9, block=2, seed=63, n_even=0, n_odd=3,
                                             l=3, quad_level=2),
    # m = 6: one level
    "3d-5-s32": lambda: inputs.make_instance("mg-3d-5", 3, 5, 1, 0.5, 0.9, block=5, seed=64, n_even=0, n_odd=3,
                                             l=3, quad_level=2),
}


@pytest.fixture(scope="module", params=list(CASES))
def mgcase(request):
    from paper_2102_09038_amd import rte
    inst = CASES[request.param]()
    d = inst.dim
    m = mg.lattice_size(inst.vert, d)
    print(f"[mg {request.param}] nR+={len(inst.vert)} nS+={len(inst.stri) // 2} levels {mg.level_sizes(m)}",
          flush=True)
    D = discretize_instance(inst)
    ops = Operators(D, n_even=inst.n_even, n_odd=inst.n_odd)
    h = rte.Handle.from_instance(inst, e0_solver=rte.RTE_E0_MG, mixed=1)
    yield request.param, inst, D, ops, h, m
    h.close()


def test_vcycle_matches_oracle(mgcase):
    name, inst, D, ops, h, m = mgcase
    X = np.random.default_rng(71).standard_normal((D.nRp, D.nS))
    Y = torch.empty_like(to_dev(X))
    h.apply_mg(to_dev(X), Y)
    Yg = from_dev(Y)
    worst = 0.0
    for k in range(D.nS):
        levels = mg.hierarchy(ops.E0_block(k), m, inst.dim, smoother="f32")
        worst = max(worst, rel(Yg[:, k], mg.vcycle(levels, X[:, k])))
    print(f"[{name}] V-cycle worst direction {worst:.2e}")
    assert worst < 1e-10
    Y2 = torch.empty_like(Y)
    h.apply_mg(to_dev(X), Y2)
    assert torch.equal(Y, Y2)


def test_mg_e0inv_fp64(mgcase):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h, m = mgcase
    B = np.random.default_rng(72).standard_normal((D.nRp, D.nS))
    B[:, 1] = 0.0
    o = rte.default_solve_opts(e0_solver=rte.RTE_E0_MG, cg_tol=1e-13, cg_max_iter=2000)
    X = torch.empty_like(to_dev(B))
    h.apply_E0inv(to_dev(B), X, o)
    err = rel(from_dev(X), ops.E0_solve(B))
    print(f"[{name}] multigrid CG FP64 {err:.2e}")
    assert err < 1e-10
    assert torch.count_nonzero(X[1]) == 0
    X2 = torch.empty_like(X)
    h.apply_E0inv(to_dev(B), X2, o)
    assert torch.equal(X, X2)


def test_mg_e0inv_fp32(mgcase):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h, m = mgcase
    B = np.random.default_rng(73).standard_normal((D.nRp, D.nS))
    o = rte.default_solve_opts(e0_solver=rte.RTE_E0_MG, precision=rte.RTE_MIXED, cg_max_iter=2000)
    X = torch.empty_like(to_dev(B))
    h.apply_E0inv(to_dev(B), X, o)
    err = rel(from_dev(X), ops.E0_solve(B))
    print(f"[{name}] multigrid CG FP32 {err:.2e}")
    assert err < 1e-4


def test_mg_iteration_counts(mgcase):
    """The largest per-direction iteration count of E_0^{-1} at tol 1e-8 against the oracle's
    multigrid CG on the same right-hand sides (equal, up to one iteration where a residual
    sits at the threshold)."""
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h, m = mgcase
    B = np.random.default_rng(74).standard_normal((D.nRp, D.nS))
    o = rte.default_solve_opts(e0_solver=rte.RTE_E0_MG, cg_tol=1e-8, cg_max_iter=2000)
    X = torch.empty_like(to_dev(B))
    h.apply_E0inv(to_dev(B), X, o)
    iters = h.last_cg_iters()
    ref = [mg.mg_cg(ops.E0_block(k), B[:, k], m, inst.dim, tol=1e-8, smoother="f32")[1] for k in range(D.nS)]
    print(f"[{name}] iterations device {max(iters)} (oracle {max(ref)}), per direction {iters}")
    assert all(abs(a - b) <= 1 for a, b in zip(iters, ref))


def test_mg_solve_end_to_end(mgcase):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h, m = mgcase
    o = rte.default_solve_opts(l=inst.l, tol=1e-12, max_iter=400, odd_solver=rte.RTE_ODD_CONDENSED,
                               e0_solver=rte.RTE_E0_MG, cg_tol=1e-13, cg_max_iter=2000)
    uref, rinfo = richardson(ops, l=inst.l, tol=1e-12, max_iter=400)
    U = torch.empty((D.nS, D.nRp), dtype=torch.float64, device="cuda")
    st, info = h.solve(U, opts=o)
    err = rel(from_dev(U), uref)
    print(f"[{name}] FP64 solve with the multigrid E_0: {info.iters} iters (oracle {rinfo['iters']}), {err:.2e}, "
          f"CG iterations {info.cg_iters_total} (max {info.cg_iters_max})")
    assert info.rel_resid <= 1e-12 and err < 1e-10 and abs(info.iters - rinfo["iters"]) <= 1


def test_not_a_lattice_is_refused():
    from paper_2102_09038_amd import rte
    inst = inputs.make_instance("mg-bad", 2, 6, 1, 0.5, 0.9, block=3, seed=65, n_even=0, n_odd=3, l=2, quad_level=2)
    perm = np.arange(len(inst.vert))
    perm[[3, 4]] = perm[[4, 3]]
    inv = np.argsort(perm)
    inst.vert = inst.vert[perm]
    inst.cell = inv[inst.cell].astype(np.int32)
    inst.q_nodal = inst.q_nodal[perm]
    with pytest.raises(rte.RteError) as e:
        rte.Handle.from_instance(inst, e0_solver=rte.RTE_E0_MG)
    assert e.value.status == rte.RTE_E_ARG
    h = rte.Handle.from_instance(inst, e0_solver=rte.RTE_E0_CG)     # the Jacobi CG takes any mesh
    h.close()


def test_mg_3d_request_full_size():
    """The served form's large 3D request at full size with the multigrid E_0."""
    import scipy.sparse.linalg as spla
    from paper_2102_09038_amd import rte
    inst = inputs.make_instance("req-3d-32-s512", 3, 32, 3, 0.8, 0.9, seed=1001, n_even=0, n_odd=5, l=4, tol=1e-6)
    print(f"[3d mg] {inst.name}: nR+ {len(inst.vert)}, r_q {inst.quad_level}", flush=True)
    t0 = time.perf_counter()
    h = rte.Handle.from_instance(inst, e0_solver=rte.RTE_E0_MG, mixed=2, odd_eig=0,
                                 coarse_solver=rte.RTE_COARSE_QUICK)
    print(f"[3d mg] assembled in {time.perf_counter() - t0:.1f} s", flush=True)
    D = discretize_instance(inst, with_scattering=False)
    ops = Operators(D, n_even=0, n_odd=5)
    B = np.random.default_rng(75).standard_normal((D.nRp, D.nS))
    X = torch.empty_like(to_dev(B))
    o64 = rte.default_solve_opts(e0_solver=rte.RTE_E0_MG, cg_tol=1e-12, cg_max_iter=2000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.apply_E0inv(to_dev(B), X, o64)
    torch.cuda.synchronize()
    print(f"[3d mg] FP64 E_0^-1 to 1e-12 in {1e3 * (time.perf_counter() - t0):.1f} ms "
          f"(max iterations {max(h.last_cg_iters())})", flush=True)
    Xg = from_dev(X)
    for k in (0, 100, D.nS - 1):
        ref = spla.splu(ops.E0_block(k)).solve(B[:, k])
        e = rel(Xg[:, k], ref)
        print(f"[3d mg] E_0^-1 direction {k}: {e:.2e}", flush=True)
        assert e < 1e-9
    o = rte.default_solve_opts(l=4, tol=1e-6, max_iter=400, odd_solver=rte.RTE_ODD_CONDENSED, e0_solver=rte.RTE_E0_MG,
                               precision=rte.RTE_MIXED, cg_max_iter=2000, profile=1)
    U = torch.empty((D.nS, D.nRp), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, info = h.solve(U, opts=o)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"[3d mg] mixed solve: {info.iters} iters in {dt:.2f} s (E_0^-1 {info.t_e0inv:.2f} s over {info.n_e0inv} "
          f"applications), CG iterations max {info.cg_iters_max}", flush=True)
    assert info.rel_resid <= 1e-6
    EU = torch.empty_like(U)
    h.apply_E(U, EU, rte.default_solve_opts(odd_solver=rte.RTE_ODD_CONDENSED))
    KU = torch.empty_like(U)
    h.apply_scatter(1, U, KU)
    q = torch.from_numpy(np.ascontiguousarray(h.get_array(rte.ARRAY_Q, (D.nRp, D.nS)).T)).cuda()
    r = float(torch.linalg.norm(EU - KU - q) / torch.linalg.norm(q))
    print(f"[3d mg] recomputed relative residual {r:.2e}")
    assert r <= 1.01e-6
    h.close()


@pytest.mark.parametrize("case", ["2d-16", "3d-8", "3d-16-served"])
def test_mg_estimated_footprint_matches_admitted_slot(case):
    """rte_estimate_footprint (host only, before assembly) against the bytes a multigrid slot
    holds once admitted (handle and workspace), including the served 3D configuration (FP32
    only, no odd eigendecomposition, the quick coarse set-up: block-tridiagonal Cholesky)."""
    from paper_2102_09038_amd import rte
    if case == "2d-16":
        inst, kw = CASES["2d-16-s32"](), dict(mixed=1)
    elif case == "3d-8":
        inst, kw = CASES["3d-8-s32"](), dict(mixed=1)
    else:
        inst = inputs.make_instance("mg-3d-16", 3, 16, 2, 0.8, 0.9, block=8, seed=66, n_even=0, n_odd=5, l=4,
                                    tol=1e-6)
        kw = dict(mixed=2, odd_eig=0, coarse_solver=rte.RTE_COARSE_QUICK)
    est, peak = rte.estimate_footprint(inst, e0_solver=rte.RTE_E0_MG, **kw)
    h = rte.Handle.from_instance(inst, e0_solver=rte.RTE_E0_MG, **kw)
    o = rte.default_solve_opts(l=4, tol=1e-6, max_iter=200, precision=rte.RTE_MIXED, e0_solver=rte.RTE_E0_MG,
                               odd_solver=rte.RTE_ODD_CONDENSED)
    b = rte.Batch(max_slots=1)
    U = torch.empty((h.dims.nSp, h.dims.nRp), dtype=torch.float64, device="cuda")
    b.admit(h, U, o)
    actual = b.usage()[2]
    print(f"[{case}] estimated {est} bytes (peak {peak}), slot holds {actual}")
    assert 0.8 * actual <= est <= 1.5 * actual + (1 << 20)
    assert b.step(1000) == 0
    (s, st, info), = b.poll()
    assert st == rte.RTE_OK and info.rel_resid <= 1e-6
    b.close()
    h.close()
