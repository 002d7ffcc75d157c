"""GPU parity on heterogeneous media and at the quadrature levels the product runs.

* Blockwise sigma_t (U[1,10] per 8 x 8 block of squares, as in the realistic workload) on a
  32 x 32 grid with 128 sphere triangles, g = 0.9: the assembled arrays (1e-12), E in its
  three forms, E_0^{-1} by CG and banded, P_1^l and P_2 P_1^l (which carries E_c, Sec. 5.4),
  and the converged iterate of every solve path (1e-10) against the oracle.  Three variants:
  a uniform ratio sigma_s / sigma_t = 0.99 with the correction space N+ = 0 (d = 1) and
  N+ = 2 (d = 6), and a ratio drawn per cell in [0.5, 0.95] (the exact and PCG odd solves;
  the condensed form refuses it).
* S+ and S- at quadrature levels 3, 4 and 5 (g = 0.8 and 0.95) against oracle values stored
  by tests/golden/make_scattering_golden.py (the oracle needs minutes per row there), 1e-12.
"""
import os

import numpy as np
import pytest

from oracle.discretize import discretize_instance
from oracle.operators import Operators
from oracle.solver import richardson
from paper_2102_09038_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def to_dev(U):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(U, dtype=np.float64).T)).cuda()


def from_dev(t):
    return t.cpu().numpy().T


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def blockwise(n_even=0, per_cell=False):
    inst = inputs.make_instance(f"blockwise-32x32-s128-g0.9-n{n_even}{'-percell' if per_cell else ''}", 2, 32, 2,
                                0.9, 0.99, block=8, seed=21, n_even=n_even, n_odd=5, l=4, quad_level=2)
    if per_cell:
        rng = np.random.default_rng(23)
        inst.sigma_s = inst.sigma_t * rng.uniform(0.5, 0.95, size=len(inst.sigma_t))
    return inst


MEDIA = {"uniform": lambda: blockwise(0), "uniform-d6": lambda: blockwise(2), "percell": lambda: blockwise(0, True)}


@pytest.fixture(scope="module", params=list(MEDIA))
def media(request):
    from paper_2102_09038_amd import rte
    inst = MEDIA[request.param]()
    assert np.ptp(inst.sigma_t) > 1.0               # the medium really is heterogeneous
    print(f"[media {request.param}] sigma_t in [{inst.sigma_t.min():.2f}, {inst.sigma_t.max():.2f}]", flush=True)
    D = discretize_instance(inst)
    ops = Operators(D, n_even=inst.n_even, n_odd=inst.n_odd)
    h = rte.Handle.from_instance(inst, e0_solver=rte.RTE_E0_BANDED)
    cache = {}
    yield request.param, inst, D, ops, h, cache
    h.close()


def oracle_solution(media_case):
    name, inst, D, ops, h, cache = media_case
    if "u" not in cache:
        cache["u"] = richardson(ops, l=inst.l, tol=1e-12, max_iter=400)
    return cache["u"]


def uniform_ratio(D):
    """The library's test: sigma_s / sigma_t varies by at most 1e-13 relative."""
    r = D.sigma_s / D.sigma_t
    return np.ptp(r) <= 1e-13 * np.max(r)


def test_media_assembly(media):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h, _ = media
    nS = D.nS
    assert relmax(h.get_array(rte.ARRAY_SP, (nS, nS)), D.Sp) < 1e-12
    assert relmax(h.get_array(rte.ARRAY_SM, (3 * nS, 3 * nS)), D.Sm) < 1e-12
    assert relmax(h.get_array(rte.ARRAY_Q, (D.nRp, nS)), D.q) < 1e-13


@pytest.mark.parametrize("odd", ["pcg", "exact", "condensed"])
def test_media_apply_E(media, odd):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h, _ = media
    o = rte.default_solve_opts(pcg_tol_resid=1e-14, pcg_max_iter=500,
                               odd_solver={"pcg": 0, "exact": 1, "condensed": 2}[odd])
    U = np.random.default_rng(41).standard_normal((D.nRp, D.nS))
    Y = torch.empty_like(to_dev(U))
    if odd == "condensed" and not uniform_ratio(D):
        with pytest.raises(rte.RteError) as e:
            h.apply_E(to_dev(U), Y, o)
        assert e.value.status == rte.RTE_E_ARG
        return
    h.apply_E(to_dev(U), Y, o)
    err = rel(from_dev(Y), ops.E(U))
    print(f"[{name}] E ({odd}) {err:.2e}")
    assert err < 1e-10


@pytest.mark.parametrize("e0", ["cg", "banded"])
def test_media_E0inv(media, e0):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h, _ = media
    o = rte.default_solve_opts(cg_tol=1e-14, cg_max_iter=50000,
                               e0_solver=rte.RTE_E0_CG if e0 == "cg" else rte.RTE_E0_BANDED)
    B = np.random.default_rng(42).standard_normal((D.nRp, D.nS))
    X = torch.empty_like(to_dev(B))
    h.apply_E0inv(to_dev(B), X, o)
    err = rel(from_dev(X), ops.E0_solve(B))
    print(f"[{name}] E_0^-1 ({e0}) {err:.2e}")
    assert err < 1e-10


@pytest.mark.parametrize("which", [0, 1])
def test_media_precond(media, which):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h, _ = media
    odd = rte.RTE_ODD_CONDENSED if uniform_ratio(D) else rte.RTE_ODD_EXACT
    o = rte.default_solve_opts(l=inst.l, odd_solver=odd, e0_solver=rte.RTE_E0_BANDED)
    r = np.random.default_rng(43).standard_normal((D.nRp, D.nS))
    S = torch.empty_like(to_dev(r))
    h.precond(which, to_dev(r), S, o)
    ref = ops.P1(r, inst.l) if which == 0 else ops.P2P1(r, inst.l)
    err = rel(from_dev(S), ref)
    print(f"[{name}] {'P2 P1' if which else 'P1'} {err:.2e}")
    assert err < 1e-10


@pytest.mark.parametrize("path", ["pcg-cg", "exact-banded", "condensed-banded"])
def test_media_solve(media, path):
    from paper_2102_09038_amd import rte
    name, inst, D, ops, h, _ = media
    if path.startswith("condensed") and not uniform_ratio(D):
        pytest.skip("the condensed form needs a uniform sigma_s / sigma_t (refusal tested above)")
    o = rte.default_solve_opts(l=inst.l, tol=1e-12, max_iter=400, cg_tol=1e-13, cg_max_iter=50000,
                               pcg_tol_resid=1e-14, pcg_tol_inner=1e-12, pcg_max_iter=500)
    if path != "pcg-cg":
        o.odd_solver = rte.RTE_ODD_EXACT if path.startswith("exact") else rte.RTE_ODD_CONDENSED
        o.e0_solver = rte.RTE_E0_BANDED
    uref, rinfo = oracle_solution(media)
    U = torch.empty((D.nS, D.nRp), dtype=torch.float64, device="cuda")
    st, info = h.solve(U, opts=o)
    err = rel(from_dev(U), uref)
    print(f"[{name} {path}] gpu iters {info.iters} rel_resid {info.rel_resid:.2e}  oracle iters {rinfo['iters']}  "
          f"err {err:.2e}")
    assert info.rel_resid <= 1e-12
    assert err < 1e-10
    assert abs(info.iters - rinfo["iters"]) <= 1


# ----------------------------------------------------------------------------- quadrature levels
SCAT = ["scattering_l2_g0.8_rq3", "scattering_l1_g0.95_rq4", "scattering_l2_g0.95_rq5"]


@pytest.mark.parametrize("name", SCAT)
def test_scattering_quadrature_levels(name):
    from paper_2102_09038_amd import rte
    z = np.load(os.path.join(GOLDEN, name + ".npz"))
    level, g, rq, rows = int(z["level"]), float(z["g"]), int(z["r_q"]), list(z["rows"])
    inst = inputs.make_instance(f"sphere-l{level}-rq{rq}", 2, 2, level, g, 0.9, sigma_t=1.0, quad_level=rq,
                                n_even=0, n_odd=1, l=1)
    print(f"[{name}] sphere level {level}, g {g}, r_q {rq}, {len(rows)} rows", flush=True)
    h = rte.Handle.from_instance(inst, odd_eig=0)
    nS = h.dims.nSp
    Sp = h.get_array(rte.ARRAY_SP, (nS, nS))
    Sm = h.get_array(rte.ARRAY_SM, (3 * nS, 3 * nS))
    h.close()
    sm_rows = [3 * k + n for k in rows for n in range(3)]
    e1 = relmax(Sp[rows], z["Sp"])
    e2 = relmax(Sm[sm_rows], z["Sm"])
    print(f"[{name}] S+ {e1:.2e}  S- {e2:.2e}")
    assert e1 < 1e-12 and e2 < 1e-12
