"""GPU parity: every librte entry point against the FP64 oracle on the same seeded inputs.

Bar (FP64): relative l2 (or max-abs relative to the array's max) <= 1e-10 for operators
and converged iterates; assembled matrices <= 1e-12 (they differ only by summation
order and the kernel's rsqrt vs the oracle's division).
Sizes: tiny 2D/3D meshes (ragged GEMM tiles: 25 x 16 and 32 x 48 operands) and the
16x16 / 128-triangle instance (several 128-wide tiles plus a ragged tail).
"""
import numpy as np
import pytest

from oracle.discretize import discretize_instance
from oracle.operators import Operators
from oracle.solver import richardson
from paper_2102_09038_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def to_dev(U):
    """(n_rows, n_cols) numpy matrix -> its column-major storage as a cuda tensor."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(U, dtype=np.float64).T)).cuda()


def from_dev(t):
    return t.cpu().numpy().T


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def make(inst, **kw):
    from paper_2102_09038_amd import rte
    D = discretize_instance(inst)
    ops = Operators(D, n_even=inst.n_even, n_odd=inst.n_odd)
    h = rte.Handle.from_instance(inst, **kw)
    return D, ops, h


def varied_ratio(inst, seed=5):
    rng = np.random.default_rng(seed)
    inst.sigma_s = inst.sigma_t * rng.uniform(0.5, 0.95, size=len(inst.sigma_t))
    return inst


CASES = {
    "tiny2d": lambda: inputs.tiny_instance(n=4, sphere_level=1, g=0.5, ratio=0.9, n_even=2, n_odd=3, l=2),
    "tiny2d-hetero": lambda: varied_ratio(inputs.tiny_instance(n=5, sphere_level=1, g=0.7, ratio=0.9,
                                                               n_even=0, n_odd=3, l=3)),
    "tiny3d": lambda: inputs.tiny_instance(n=2, sphere_level=1, g=0.6, ratio=0.9, dim=3, n_even=2, n_odd=1),
    "small": inputs.config_small,
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    inst = CASES[request.param]()
    print(f"[case {request.param}] nR+={len(inst.vert)} nS+={len(inst.stri)//2}", flush=True)
    from paper_2102_09038_amd import rte
    D, ops, h = make(inst, e0_solver=rte.RTE_E0_BANDED, mixed=1)
    yield request.param, inst, D, ops, h
    h.close()


def test_assembly(case):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h = case
    nS = D.nS
    assert h.dims.nRp == D.nRp and h.dims.nRm == D.nRm and h.dims.nSp == nS
    Sp = h.get_array(rte.ARRAY_SP, (nS, nS))
    Sm = h.get_array(rte.ARRAY_SM, (3 * nS, 3 * nS))
    assert relmax(Sp, D.Sp) < 1e-12
    assert relmax(Sm, D.Sm) < 1e-12
    assert relmax(h.get_array(rte.ARRAY_M, (nS,)), D.m) < 1e-13
    T = h.get_array(rte.ARRAY_T, (9 * nS,)).reshape(nS, 3, 3)
    assert relmax(T, D.T) < 1e-13
    q = h.get_array(rte.ARRAY_Q, (D.nRp, nS))
    assert relmax(q, D.q) < 1e-13


def test_eigenbases(case):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h = case
    W, lam = ops.even_eig()
    dN = W.shape[1]
    lg = h.get_array(rte.ARRAY_LAMP, (dN,))
    assert np.allclose(lg, lam, rtol=0, atol=1e-10)
    Wg = h.get_array(rte.ARRAY_WP, (D.nS, dN))
    # the spanned subspace is unique (eigenvectors are not, inside clusters)
    assert relmax(Wg @ Wg.T, W @ W.T) < 1e-8
    lm, _ = ops.odd_eig()
    assert np.allclose(h.get_array(rte.ARRAY_LAMM, (3 * D.nS,)), lm, rtol=0, atol=1e-10)


def test_scatter(case):
    name, inst, D, ops, h = case
    rng = np.random.default_rng(11)
    U = rng.standard_normal((D.nRp, D.nS))
    Y = torch.empty_like(to_dev(U))
    h.apply_scatter(1, to_dev(U), Y)
    assert rel(from_dev(Y), ops.K_even(U)) < 1e-12
    V = rng.standard_normal((D.nRm, 3 * D.nS))
    Yv = torch.empty_like(to_dev(V))
    h.apply_scatter(-1, to_dev(V), Yv)
    assert rel(from_dev(Yv), ops.K_odd(V)) < 1e-12


def test_scatter_fp32(case):
    """FP32 MFMA scatter GEMMs (the preconditioner's K+ in mixed precision) against the
    oracle's FP64 products: inputs rounded to FP32 and FP32 sums of n_S terms stay within
    about sqrt(n_S) 2^-24 relative; 2e-5 is asserted.  Both output dtypes are checked."""
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h = case
    rng = np.random.default_rng(12)
    for parity, X, ref in ((1, rng.standard_normal((D.nRp, D.nS)), None),
                           (-1, rng.standard_normal((D.nRm, 3 * D.nS)), None)):
        ref = ops.K_even(X) if parity == 1 else ops.K_odd(X)
        Xf = to_dev(X).float().contiguous()
        Y64 = torch.empty(Xf.shape, dtype=torch.float64, device="cuda")
        Y32 = torch.empty(Xf.shape, dtype=torch.float32, device="cuda")
        h.apply_scatter(parity, Xf, Y64, dtype_in=rte.RTE_DT_F32, dtype_out=rte.RTE_DT_F64)
        h.apply_scatter(parity, Xf, Y32, dtype_in=rte.RTE_DT_F32, dtype_out=rte.RTE_DT_F32)
        e64 = rel(from_dev(Y64), ref)
        e32 = rel(from_dev(Y32.double()), ref)
        print(f"[{name}] K{'+' if parity == 1 else '-'} FP32 MFMA: {e64:.2e} (FP32 out {e32:.2e})")
        assert e64 < 2e-5 and e32 < 2e-5
    with pytest.raises(rte.RteError):
        h.apply_scatter(1, Xf, Y64, dtype_in=rte.RTE_DT_BF16, dtype_out=rte.RTE_DT_F32)


ODD = {"pcg": 0, "exact": 1, "condensed": 2}


@pytest.mark.parametrize("odd", list(ODD))
def test_apply_E(case, odd):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h = case
    o = rte.default_solve_opts(pcg_tol_resid=1e-14, pcg_max_iter=500, odd_solver=ODD[odd])
    U = np.random.default_rng(12).standard_normal((D.nRp, D.nS))
    Y = torch.empty_like(to_dev(U))
    uniform = np.ptp(D.sigma_s / D.sigma_t) <= 1e-13 * np.max(D.sigma_s / D.sigma_t)
    if odd == "condensed" and not uniform:
        with pytest.raises(rte.RteError) as e:
            h.apply_E(to_dev(U), Y, o)
        assert e.value.status == rte.RTE_E_ARG
        return
    h.apply_E(to_dev(U), Y, o)
    assert rel(from_dev(Y), ops.E(U)) < 1e-10


def test_apply_E_many_tiles():
    """Condensed E U where the FP64 transport GEMM takes the direct-to-LDS kernel over many
    whole tiles (48 x 48 squares, 128 sphere triangles: 128 x 4608 x 128, 36 tiles, so the
    work-group to XCD map also takes its leftover branch), against the oracle."""
    from paper_2102_09038_amd import rte
    inst = inputs.make_instance("tiles-48x48-s128", 2, 48, 2, 0.5, 0.95, seed=9, n_even=0, n_odd=5, l=4,
                                quad_level=2)
    D, ops, h = make(inst)
    o = rte.default_solve_opts(odd_solver=rte.RTE_ODD_CONDENSED)
    U = np.random.default_rng(19).standard_normal((D.nRp, D.nS))
    Y = torch.empty_like(to_dev(U))
    h.apply_E(to_dev(U), Y, o)
    err = rel(from_dev(Y), ops.E(U))
    print(f"[tiles] E U rel err {err:.2e}")
    assert err < 1e-10
    h.close()


@pytest.mark.parametrize("e0", ["cg", "banded"])
def test_apply_E0inv(case, e0):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h = case
    o = rte.default_solve_opts(cg_tol=1e-14, cg_max_iter=50000,
                               e0_solver=rte.RTE_E0_CG if e0 == "cg" else rte.RTE_E0_BANDED)
    B = np.random.default_rng(13).standard_normal((D.nRp, D.nS))
    X = torch.empty_like(to_dev(B))
    h.apply_E0inv(to_dev(B), X, o)
    assert rel(from_dev(X), ops.E0_solve(B)) < 1e-10


@pytest.mark.parametrize("which", [0, 1])
def test_precond(case, which):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h = case
    o = rte.default_solve_opts(l=inst.l, cg_tol=1e-14, cg_max_iter=50000, pcg_tol_resid=1e-14,
                               pcg_tol_inner=1e-14, pcg_max_iter=500)
    r = np.random.default_rng(14).standard_normal((D.nRp, D.nS))
    S = torch.empty_like(to_dev(r))
    h.precond(which, to_dev(r), S, o)
    ref = ops.P1(r, inst.l) if which == 0 else ops.P2P1(r, inst.l)
    assert rel(from_dev(S), ref) < 1e-10


@pytest.mark.parametrize("path", ["pcg-cg", "exact-banded", "condensed-banded"])
def test_solve(case, path):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h = case
    o = rte.default_solve_opts(l=inst.l, tol=1e-12, cg_tol=1e-13, cg_max_iter=50000, pcg_tol_resid=1e-14,
                               pcg_tol_inner=1e-12, pcg_max_iter=500)
    if path != "pcg-cg":
        o.odd_solver = ODD[path.split("-")[0]]
        o.e0_solver = rte.RTE_E0_BANDED
    if path.startswith("condensed") and np.ptp(D.sigma_s / D.sigma_t) > 0:
        pytest.skip("condensed form needs a uniform sigma_s/sigma_t")
    U = torch.empty((D.nS, D.nRp), dtype=torch.float64, device="cuda")
    st, info = h.solve(U, opts=o)
    uref, rinfo = richardson(ops, l=inst.l, tol=1e-12, max_iter=200)
    print(f"[{name} {path}] gpu iters {info.iters} rel_resid {info.rel_resid:.2e}  oracle iters {rinfo['iters']}")
    assert info.rel_resid <= 1e-12
    assert rel(from_dev(U), uref) < 1e-10
    assert abs(info.iters - rinfo["iters"]) <= 1


def test_deterministic(case):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h = case
    o = rte.default_solve_opts(pcg_tol_resid=1e-12)
    U = to_dev(np.random.default_rng(15).standard_normal((D.nRp, D.nS)))
    Y1 = torch.empty_like(U)
    Y2 = torch.empty_like(U)
    h.apply_E(U, Y1, o)
    h.apply_E(U, Y2, o)
    assert torch.equal(Y1, Y2)


# ----------------------------------------------------------------------------- inner PCG
@pytest.mark.parametrize("which", [0, 1])
def test_inner_pcg_precond(case, which):
    """P_1 as l steps of E_0-preconditioned CG (and P_2 after it) against the oracle's CG."""
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h = case
    o = rte.default_solve_opts(l=inst.l + 1, cg_tol=1e-14, cg_max_iter=50000, pcg_tol_resid=1e-14,
                               pcg_tol_inner=1e-14, pcg_max_iter=500, inner=rte.RTE_INNER_PCG)
    r = np.random.default_rng(16).standard_normal((D.nRp, D.nS))
    S = torch.empty_like(to_dev(r))
    h.precond(which, to_dev(r), S, o)
    ref = ops.P1_pcg(r, inst.l + 1) if which == 0 else ops.P2P1(r, inst.l + 1, inner="pcg")
    err = rel(from_dev(S), ref)
    print(f"[{name}] inner PCG precond {which}: {err:.2e}")
    assert err < 1e-10
    Z = torch.empty_like(S)
    h.precond(which, torch.zeros_like(S), Z, o)
    assert torch.count_nonzero(Z) == 0          # r = 0: every step size is 0, nothing non-finite


def test_inner_pcg_solve(case):
    """The outer iteration with the inner PCG, on the production path (banded E_0, exact or
    condensed odd solve), reaches the oracle's iterate with the same inner method."""
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h = case
    odd = rte.RTE_ODD_CONDENSED if np.ptp(D.sigma_s / D.sigma_t) == 0 else rte.RTE_ODD_EXACT
    o = rte.default_solve_opts(l=inst.l, tol=1e-12, odd_solver=odd, e0_solver=rte.RTE_E0_BANDED,
                               inner=rte.RTE_INNER_PCG)
    U = torch.empty((D.nS, D.nRp), dtype=torch.float64, device="cuda")
    st, info = h.solve(U, opts=o)
    uref, rinfo = richardson(ops, l=inst.l, tol=1e-12, max_iter=200, inner="pcg")
    print(f"[{name}] inner PCG: gpu iters {info.iters} rel_resid {info.rel_resid:.2e}  oracle iters {rinfo['iters']}")
    assert info.rel_resid <= 1e-12
    assert rel(from_dev(U), uref) < 1e-10
    assert abs(info.iters - rinfo["iters"]) <= 1


def test_derived_outputs(case):
    """Scalar flux and balance terms of a random U against the oracle's plain definitions, and
    the closed balance at a converged solution."""
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h = case
    V = np.random.default_rng(17).standard_normal((D.nRp, D.nS))
    phi = torch.empty(D.nRp, dtype=torch.float64, device="cuda")
    b = h.derived_outputs(to_dev(V), phi)
    phi_ref, b_ref = ops.derived(V)
    assert rel(phi.cpu().numpy(), phi_ref) < 1e-13
    scale = abs(b_ref["absorption"]) + abs(b_ref["leakage"]) + abs(b_ref["source"])
    for key in ("source", "absorption", "leakage", "imbalance"):
        assert abs(b[key] - b_ref[key]) <= 1e-12 * scale, key
    odd = rte.RTE_ODD_CONDENSED if np.ptp(D.sigma_s / D.sigma_t) == 0 else rte.RTE_ODD_EXACT
    U = torch.empty((D.nS, D.nRp), dtype=torch.float64, device="cuda")
    h.solve(U, opts=rte.default_solve_opts(l=inst.l, tol=1e-12, odd_solver=odd, e0_solver=rte.RTE_E0_BANDED))
    bs = h.derived_outputs(U)
    print(f"[{name}] source {bs['source']:.6e} absorption {bs['absorption']:.6e} leakage {bs['leakage']:.6e} "
          f"imbalance {bs['imbalance']:.1e}")
    assert abs(bs["imbalance"]) <= 1e-10 * bs["source"]
    assert h.derived_outputs(U, phi) == bs      # repeatable (fixed-order sums)


@pytest.mark.parametrize("name,coarse", [("tiny2d", "band"), ("tiny2d", "block"), ("small", "block"),
                                        ("tiny2d-hetero", "quick")])
def test_coarse_solvers(name, coarse):
    """The correction's coarse system solved by the band solve (factored on the device) or by
    the block-tridiagonal Cholesky instead of the explicit inverse: P_2 P_1 r and the converged
    iterate against the oracle (sparse LU of E_c).  The small instance has 4335 coarse unknowns
    in blocks of one half-bandwidth, the last one ragged."""
    from paper_2102_09038_amd import rte
    inst = CASES[name]()
    how = {"band": rte.RTE_COARSE_BAND, "block": rte.RTE_COARSE_BLOCK, "quick": rte.RTE_COARSE_QUICK}[coarse]
    print(f"[{name}] coarse solver {coarse}", flush=True)
    D, ops, h = make(inst, e0_solver=rte.RTE_E0_BANDED, coarse_solver=how)
    o = rte.default_solve_opts(l=inst.l, tol=1e-12, odd_solver=rte.RTE_ODD_EXACT, e0_solver=rte.RTE_E0_BANDED)
    r = np.random.default_rng(18).standard_normal((D.nRp, D.nS))
    S = torch.empty_like(to_dev(r))
    h.precond(1, to_dev(r), S, o)
    err = rel(from_dev(S), ops.P2P1(r, inst.l))
    U = torch.empty((D.nS, D.nRp), dtype=torch.float64, device="cuda")
    st, info = h.solve(U, opts=o)
    uref, rinfo = richardson(ops, l=inst.l, tol=1e-12, max_iter=200)
    eu = rel(from_dev(U), uref)
    print(f"[{name} {coarse}] P2P1 {err:.2e}; solve {info.iters} iters (oracle {rinfo['iters']}), {eu:.2e}")
    assert err < 1e-10 and eu < 1e-10
    if coarse == "block":
        # the batch captures the block solve's kernels as well
        b = rte.Batch(max_slots=2)
        Ub = torch.full_like(U, float("nan"))
        b.admit(h, Ub, o)
        assert b.step(1000) == 0
        torch.cuda.synchronize()
        (_, st, binfo), = b.poll()
        assert st == rte.RTE_OK and binfo.iters == info.iters
        assert rel(from_dev(Ub), uref) < 1e-10
        b.close()
    h.close()


# ----------------------------------------------------------------------------- mixed precision
# Bars: one application of the reduced-precision operators carries BF16 / FP32 rounding
# (BF16 keeps 8 significant bits: relative error ~ 2^-9 per product, averaged over the
# GEMM's accumulation), so single applications are checked loosely; the converged
# solution of the Richardson iteration, whose residual is FP64, must match the FP64
# oracle to 1e-6.

def _uniform(D):
    return np.ptp(D.sigma_s / D.sigma_t) <= 1e-13 * np.max(D.sigma_s / D.sigma_t)


def test_mixed_apply_E(case):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h = case
    if not _uniform(D):
        pytest.skip("mixed transport needs the condensed form (uniform ratio)")
    o = rte.default_solve_opts(odd_solver=rte.RTE_ODD_CONDENSED, precision=rte.RTE_MIXED)
    U = np.random.default_rng(21).standard_normal((D.nRp, D.nS))
    Y = torch.empty_like(to_dev(U))
    h.apply_E(to_dev(U), Y, o)
    err = rel(from_dev(Y), ops.E(U))
    print(f"[{name}] mixed E rel err {err:.2e}")
    assert 1e-12 < err < 2e-2


def test_mixed_E0inv(case):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h = case
    o = rte.default_solve_opts(e0_solver=rte.RTE_E0_BANDED, precision=rte.RTE_MIXED)
    B = np.random.default_rng(22).standard_normal((D.nRp, D.nS))
    X = torch.empty_like(to_dev(B))
    h.apply_E0inv(to_dev(B), X, o)
    err = rel(from_dev(X), ops.E0_solve(B))
    print(f"[{name}] FP32-factor E0^-1 rel err {err:.2e}")
    assert err < 1e-4


def test_mixed_solve(case):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h = case
    if not _uniform(D):
        pytest.skip("mixed transport needs the condensed form (uniform ratio)")
    o = rte.default_solve_opts(l=inst.l, tol=1e-10, odd_solver=rte.RTE_ODD_CONDENSED, e0_solver=rte.RTE_E0_BANDED,
                               precision=rte.RTE_MIXED, max_iter=400)
    U = torch.empty((D.nS, D.nRp), dtype=torch.float64, device="cuda")
    st, info = h.solve(U, opts=o)
    uref, rinfo = richardson(ops, l=inst.l, tol=1e-12, max_iter=200)
    err = rel(from_dev(U), uref)
    print(f"[{name}] mixed solve iters {info.iters} (fp64 oracle {rinfo['iters']}) rel err {err:.2e}")
    assert info.rel_resid <= 1e-10
    assert err < 1e-6
    o.inner = rte.RTE_INNER_PCG
    st, info = h.solve(U, opts=o)
    err = rel(from_dev(U), uref)
    print(f"[{name}] mixed solve with inner PCG: iters {info.iters}, rel err {err:.2e}")
    assert info.rel_resid <= 1e-10
    assert err < 1e-6


def test_mixed_solve_fine_sphere_low_scattering():
    """Regression: on a 2048-triangle sphere mesh with weak anisotropy and a moderate ratio
    the mixed-precision preconditioner must keep converging like the FP64 one.  The
    transport operator's diagonal blocks (odd moments of small sphere triangles) are nearly
    singular; with the operator rounded to 8-bit BF16 the iteration diverged on such
    problems, with its BF16 hi/lo pair it follows the FP64 iteration."""
    from paper_2102_09038_amd import rte
    inst = inputs.make_instance("fine-sphere", 2, 12, 4, 0.55, 0.73, seed=1006, n_even=0, n_odd=5, l=4, tol=1e-8)
    h = rte.Handle.from_instance(inst, e0_solver=rte.RTE_E0_BANDED, mixed=1)
    U64 = torch.empty((h.dims.nSp, h.dims.nRp), dtype=torch.float64, device="cuda")
    Um = torch.empty_like(U64)
    its = {}
    for name, prec, U in (("fp64", rte.RTE_FP64, U64), ("mixed", rte.RTE_MIXED, Um)):
        o = rte.default_solve_opts(l=4, tol=1e-8, max_iter=200, precision=prec, odd_solver=rte.RTE_ODD_CONDENSED,
                                   e0_solver=rte.RTE_E0_BANDED)
        st, info = h.solve(U, opts=o)
        its[name] = info.iters
    err = float(torch.linalg.norm(Um - U64) / torch.linalg.norm(U64))
    print(f"fine sphere: fp64 {its['fp64']} iters, mixed {its['mixed']} iters, rel diff {err:.2e}")
    assert its["mixed"] <= its["fp64"] + 1
    assert err < 1e-6
    h.close()


# ----------------------------------------------------------------------------- degenerate cases
DEGENERATE = {
    # sigma_s = 0: E_0 = E, the even problem decouples per direction and P_1 is exact
    "pure-absorber": lambda: inputs.tiny_instance(n=5, sphere_level=1, g=0.6, ratio=0.0, n_even=0, n_odd=3, l=3),
    # g = 0: isotropic scattering (S- = 0)
    "isotropic": lambda: inputs.tiny_instance(n=4, sphere_level=1, g=0.0, ratio=0.9, n_even=2, n_odd=3, l=3),
    # one square: 4 vertices, 2 cells, every kernel with a single ragged tile
    "one-square": lambda: inputs.tiny_instance(n=1, sphere_level=1, g=0.5, ratio=0.8, n_even=0, n_odd=3, l=2),
}


@pytest.mark.parametrize("name", list(DEGENERATE))
def test_degenerate_solves(name):
    from paper_2102_09038_amd import rte
    inst = DEGENERATE[name]()
    D, ops, h = make(inst, e0_solver=rte.RTE_E0_BANDED, mixed=1)
    uref, rinfo = richardson(ops, l=inst.l, tol=1e-12, max_iter=200)
    for odd in (rte.RTE_ODD_EXACT, rte.RTE_ODD_CONDENSED):
        o = rte.default_solve_opts(l=inst.l, tol=1e-12, max_iter=200, odd_solver=odd, e0_solver=rte.RTE_E0_BANDED,
                                   pcg_tol_resid=1e-14)
        U = torch.empty((D.nS, D.nRp), dtype=torch.float64, device="cuda")
        st, info = h.solve(U, opts=o)
        err = rel(from_dev(U), uref)
        print(f"[{name} odd={odd}] {info.iters} iters (oracle {rinfo['iters']}), rel err {err:.2e}")
        assert err < 1e-10
        if name == "pure-absorber":
            assert info.iters <= 1
    h.close()


def test_odd_part_matches_mixed_direct_solve(case):
    """u- returned by rte_solve against the odd block of the oracle's direct solve of the full
    mixed system (eq. mixed_discrete)."""
    from oracle.mixed import solve_mixed
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h = case
    if D.nRp * D.nS + D.nRm * 3 * D.nS > 30_000:
        pytest.skip("direct solve of the mixed system too large for this case")
    up_ref, um_ref = solve_mixed(D)
    o = rte.default_solve_opts(l=inst.l, tol=1e-12, max_iter=300, odd_solver=rte.RTE_ODD_EXACT,
                               e0_solver=rte.RTE_E0_BANDED)
    U = torch.empty((D.nS, D.nRp), dtype=torch.float64, device="cuda")
    Um = torch.full((3 * D.nS, D.nRm), float("nan"), dtype=torch.float64, device="cuda")
    h.solve(U, opts=o, U_odd=Um)
    eu = rel(from_dev(U), up_ref)
    em = rel(from_dev(Um), um_ref)
    print(f"[{name}] even {eu:.2e} odd {em:.2e}")
    assert eu < 1e-10 and em < 1e-10


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d", "small"])
def test_without_odd_eigendecomposition(name):
    """Assembly with odd_eig = 0 (uniform ratio): H = (M_S- - delta S-)^{-1} from a dense
    Cholesky inverse instead of the eigenbasis.  The condensed and exact ApplyE and the whole
    solve match the oracle (1e-10) and the default handle (1e-12); the coarse matrix's
    transport term, assembled through H, gives the same P_2 P_1; the PCG odd solve is refused."""
    from paper_2102_09038_amd import rte
    inst = CASES[name]()
    D, ops, h0 = make(inst, e0_solver=rte.RTE_E0_BANDED, mixed=1)
    h = rte.Handle.from_instance(inst, e0_solver=rte.RTE_E0_BANDED, mixed=1, odd_eig=0)
    rng = np.random.default_rng(21)
    U = rng.standard_normal((D.nRp, D.nS))
    ref = ops.E(U)
    for odd in ("exact", "condensed"):
        o = rte.default_solve_opts(odd_solver=ODD[odd])
        Y = torch.empty_like(to_dev(U))
        Y0 = torch.empty_like(Y)
        h.apply_E(to_dev(U), Y, o)
        h0.apply_E(to_dev(U), Y0, o)
        assert rel(from_dev(Y), ref) < 1e-10
        assert rel(from_dev(Y), from_dev(Y0)) < 1e-12
    o = rte.default_solve_opts(l=inst.l, odd_solver=rte.RTE_ODD_CONDENSED, e0_solver=rte.RTE_E0_BANDED)
    P = torch.empty_like(to_dev(U))
    P0 = torch.empty_like(P)
    h.precond(1, to_dev(U), P, o)
    h0.precond(1, to_dev(U), P0, o)
    assert rel(from_dev(P), from_dev(P0)) < 1e-11
    with pytest.raises(rte.RteError):
        h.apply_E(to_dev(U), P, rte.default_solve_opts(odd_solver=rte.RTE_ODD_PCG))
    o = rte.default_solve_opts(l=inst.l, tol=1e-12, max_iter=300, odd_solver=rte.RTE_ODD_CONDENSED,
                               e0_solver=rte.RTE_E0_BANDED)
    Us = torch.empty_like(to_dev(U))
    st, info = h.solve(Us, opts=o)
    uref, _ = richardson(ops, l=inst.l, tol=1e-12, max_iter=300)
    err = rel(from_dev(Us), uref)
    print(f"[{name}] odd_eig=0: solve {info.iters} iters, rel err vs oracle {err:.2e}")
    assert err < 1e-10
    assert h.footprint() < h0.footprint()
    h.close()
    h0.close()
