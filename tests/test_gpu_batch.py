"""GPU tests of the lockstep batch (rte_batch_*): every slot must compute exactly what
rte_solve computes with the same handle and options, whether it runs alone, in a mix of
instances of different sizes, or is admitted while others are already iterating; the
budget and the slot requirements are enforced before anything is admitted.

The grouped E_0 solve runs the same per-system code as the single-instance launch and every
other step is the same kernel sequence per slot, so the comparison is exact (bitwise); the
FP64 result is also checked against the oracle (1e-10, the FP64 parity bar).
"""
import numpy as np
import pytest

from oracle.discretize import discretize_instance
from oracle.operators import Operators
from oracle.solver import richardson
from paper_2102_09038_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def instances():
    """Problems of different sizes, band widths and dimensions (each with a uniform ratio,
    which the condensed form needs)."""
    return [
        inputs.tiny_instance(n=4, sphere_level=1, g=0.5, ratio=0.9, n_even=2, n_odd=3, l=4),
        inputs.tiny_instance(n=6, sphere_level=1, g=0.7, ratio=0.95, n_even=0, n_odd=3, l=4),
        inputs.tiny_instance(n=2, sphere_level=1, g=0.6, ratio=0.9, dim=3, n_even=0, n_odd=1, l=4),
        inputs.config_small(),
    ]


@pytest.fixture(scope="module")
def handles():
    from paper_2102_09038_amd import rte
    insts = instances()
    hs = [rte.Handle.from_instance(i, e0_solver=rte.RTE_E0_BANDED, mixed=1) for i in insts]
    yield insts, hs
    for h in hs:
        h.close()


def opts_for(precision, tol=1e-10):
    from paper_2102_09038_amd import rte
    return rte.default_solve_opts(l=4, tol=tol, max_iter=300, precision=precision, e0_solver=rte.RTE_E0_BANDED,
                                  odd_solver=rte.RTE_ODD_CONDENSED, pcg_tol_resid=1e-13, pcg_tol_inner=1e-10)


def alone(h, o):
    U = torch.empty((h.dims.nSp, h.dims.nRp), dtype=torch.float64, device="cuda")
    st, info = h.solve(U, opts=o)
    torch.cuda.synchronize()
    return U, info


def test_batch_with_band_coarse_solve_equals_single_solves():
    """Handles assembled with the quick coarse set-up (E_c by the device band factorisation and
    the band solve, as the server assembles): captured and replayed, bitwise the solo solves."""
    from paper_2102_09038_amd import rte
    insts = [i for i in instances() if i.n_even == 0]
    hs = [rte.Handle.from_instance(i, e0_solver=rte.RTE_E0_BANDED, mixed=1, coarse_solver=rte.RTE_COARSE_QUICK)
          for i in insts]
    o = opts_for(rte.RTE_MIXED)
    ref = [alone(h, o) for h in hs]
    b = rte.Batch(max_slots=8, use_graphs=True)
    outs = [torch.full((h.dims.nSp, h.dims.nRp), np.nan, dtype=torch.float64, device="cuda") for h in hs]
    slots = [b.admit(h, U, o) for h, U in zip(hs, outs)]
    assert b.step(1000) == 0
    torch.cuda.synchronize()
    done = {s: (st, info) for s, st, info in b.poll()}
    for k, (s, U) in enumerate(zip(slots, outs)):
        st, info = done[s]
        assert st == rte.RTE_OK and info.iters == ref[k][1].iters
        assert torch.equal(U, ref[k][0])
    b.close()
    for h in hs:
        h.close()


@pytest.mark.parametrize("graphs", [True, False])
def test_batch_with_block_coarse_solve_equals_single_solves(graphs):
    """Handles whose coarse system takes the block-tridiagonal Cholesky (forced here on small
    instances): the batch runs their block solves slot by slot, inside the captured graphs or
    eagerly, and matches the solo solves bit for bit."""
    from paper_2102_09038_amd import rte
    insts = instances()[:3]
    hs = [rte.Handle.from_instance(i, e0_solver=rte.RTE_E0_BANDED, mixed=1, coarse_solver=rte.RTE_COARSE_BLOCK)
          for i in insts]
    o = opts_for(rte.RTE_FP64)
    ref = [alone(h, o) for h in hs]
    b = rte.Batch(max_slots=8, use_graphs=graphs)
    outs = [torch.full((h.dims.nSp, h.dims.nRp), np.nan, dtype=torch.float64, device="cuda") for h in hs]
    slots = [b.admit(h, U, o) for h, U in zip(hs, outs)]
    assert b.step(1000) == 0
    torch.cuda.synchronize()
    done = {s: (st, info) for s, st, info in b.poll()}
    for k, (s, U) in enumerate(zip(slots, outs)):
        st, info = done[s]
        assert st == rte.RTE_OK and info.iters == ref[k][1].iters
        assert torch.equal(U, ref[k][0])
    b.close()
    for h in hs:
        h.close()


@pytest.mark.parametrize("graphs", [True, False])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_equals_single_solves(handles, prec, graphs):
    """Graph mode replays the captured iteration many times, with host synchronisations and
    eager work (admission, polling) in between; every replay feeds the next, and the final
    results must equal the eager solo solves bit for bit."""
    from paper_2102_09038_amd import rte
    insts, hs = handles
    o = opts_for(rte.RTE_FP64 if prec == "fp64" else rte.RTE_MIXED)
    ref = [alone(h, o) for h in hs]
    b = rte.Batch(max_slots=8, use_graphs=graphs)
    outs = [torch.full((h.dims.nSp, h.dims.nRp), np.nan, dtype=torch.float64, device="cuda") for h in hs]
    slots = [b.admit(h, U, o) for h, U in zip(hs, outs)]
    left = b.step(1000)
    torch.cuda.synchronize()
    assert left == 0
    done = {s: (st, info) for s, st, info in b.poll()}
    assert sorted(done) == sorted(slots)
    for k, (s, U) in enumerate(zip(slots, outs)):
        st, info = done[s]
        Ur, ir = ref[k]
        print(f"[{prec} graphs={graphs} slot {s}] iters {info.iters} (alone {ir.iters}) rel_resid {info.rel_resid:.2e}")
        assert st == rte.RTE_OK
        assert info.iters == ir.iters
        assert info.rel_resid == ir.rel_resid
        assert torch.equal(U, Ur)
    assert b.usage() == (0, 0, 0)
    b.close()


def test_batch_fp64_matches_oracle(handles):
    from paper_2102_09038_amd import rte
    insts, hs = handles
    inst, h = insts[0], hs[0]
    b = rte.Batch(max_slots=2)
    U = torch.empty((h.dims.nSp, h.dims.nRp), dtype=torch.float64, device="cuda")
    b.admit(h, U, opts_for(rte.RTE_FP64, tol=1e-12))
    b.step(1000)
    (s, st, info), = b.poll()
    assert st == rte.RTE_OK and info.rel_resid <= 1e-12
    D = discretize_instance(inst)
    uref, _ = richardson(Operators(D, n_even=inst.n_even, n_odd=inst.n_odd), l=inst.l, tol=1e-12, max_iter=200)
    Ug = U.cpu().numpy().T
    assert np.linalg.norm(Ug - uref) / np.linalg.norm(uref) < 1e-10
    b.close()


def test_admission_while_running(handles):
    """Continuous batching: a slot admitted after others have iterated, and a slot admitted
    into the place of one that finished, still compute their solo results."""
    from paper_2102_09038_amd import rte
    insts, hs = handles
    o = opts_for(rte.RTE_MIXED)
    ref = [alone(h, o) for h in hs]
    b = rte.Batch(max_slots=2)
    outs = [torch.empty((h.dims.nSp, h.dims.nRp), dtype=torch.float64, device="cuda") for h in hs]
    pending = list(range(len(hs)))
    owner = {}
    results = {}
    steps = 0
    while pending or owner:
        while pending and b.usage()[0] + b.usage()[1] < 2:
            k = pending.pop(0)
            owner[b.admit(hs[k], outs[k], o)] = k
        b.step(3)
        steps += 1
        for s, st, info in b.poll():
            results[owner.pop(s)] = (st, info)
        assert steps < 1000
    torch.cuda.synchronize()
    for k in range(len(hs)):
        st, info = results[k]
        assert st == rte.RTE_OK
        assert info.iters == ref[k][1].iters
        assert torch.equal(outs[k], ref[k][0])
    b.close()


def test_budget_and_requirements(handles):
    from paper_2102_09038_amd import rte
    insts, hs = handles
    U = torch.empty((hs[3].dims.nSp, hs[3].dims.nRp), dtype=torch.float64, device="cuda")
    small = rte.Batch(max_slots=4, hbm_budget=1 << 20)
    with pytest.raises(rte.RteError) as e:
        small.admit(hs[3], U, opts_for(rte.RTE_MIXED))
    assert e.value.status == rte.RTE_E_NOMEM
    assert small.usage() == (0, 0, 0)
    small.close()
    b = rte.Batch(max_slots=1)
    b.admit(hs[3], U, opts_for(rte.RTE_MIXED))
    U1 = torch.empty((hs[0].dims.nSp, hs[0].dims.nRp), dtype=torch.float64, device="cuda")
    with pytest.raises(rte.RteError) as e:        # no free slot
        b.admit(hs[0], U1, opts_for(rte.RTE_MIXED))
    assert e.value.status == rte.RTE_E_ARG
    b.close()
    b = rte.Batch(max_slots=4)
    b.admit(hs[3], U, opts_for(rte.RTE_MIXED))
    with pytest.raises(rte.RteError) as e:        # one precision per batch
        b.admit(hs[0], U1, opts_for(rte.RTE_FP64))
    assert e.value.status == rte.RTE_E_ARG
    with pytest.raises(rte.RteError) as e:        # a handle holds one slot at a time
        b.admit(hs[3], U1, opts_for(rte.RTE_MIXED))
    assert e.value.status == rte.RTE_E_ARG
    bad = opts_for(rte.RTE_MIXED)
    bad.odd_solver = rte.RTE_ODD_PCG
    with pytest.raises(rte.RteError) as e:        # the PCG odd solve is not batched
        b.admit(hs[0], U1, bad)
    assert e.value.status == rte.RTE_E_ARG
    bad = opts_for(rte.RTE_MIXED)
    bad.inner = rte.RTE_INNER_PCG
    with pytest.raises(rte.RteError) as e:        # nor the inner PCG of P_1
        b.admit(hs[0], U1, bad)
    assert e.value.status == rte.RTE_E_ARG
    b.close()


def test_estimated_footprint_matches_admitted_slot(handles):
    """rte_estimate_footprint (host only, before assembly) against the bytes a slot holds."""
    from paper_2102_09038_amd import rte
    insts, hs = handles
    for inst, h in zip(insts, hs):
        est, _ = rte.estimate_footprint(inst, e0_solver=rte.RTE_E0_BANDED, mixed=1)
        b = rte.Batch(max_slots=1)
        U = torch.empty((h.dims.nSp, h.dims.nRp), dtype=torch.float64, device="cuda")
        b.admit(h, U, opts_for(rte.RTE_MIXED))
        actual = b.usage()[2]
        print(f"{inst.name}: estimated {est} bytes, slot holds {actual}")
        assert 0.8 * actual <= est <= 1.5 * actual + (1 << 20)
        b.step(1000)
        b.poll()
        b.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_cg_slots_in_lockstep_equal_single_solves(prec):
    """Slots whose E_0 is solved by CG (Jacobi- or multigrid-preconditioned) advance together on
    the batch's stream lanes (more slots than lanes, so lanes are shared), beside a banded slot;
    one CG slot stops at a small iteration cap, so the slots leave the lockstep at different
    check points.  Every slot must equal its solo solve bit for bit."""
    from paper_2102_09038_amd import rte
    insts = [
        inputs.tiny_instance(n=4, sphere_level=1, g=0.5, ratio=0.9, n_even=0, n_odd=3, l=4),
        inputs.tiny_instance(n=6, sphere_level=1, g=0.7, ratio=0.95, n_even=0, n_odd=3, l=4),
        inputs.tiny_instance(n=2, sphere_level=1, g=0.6, ratio=0.9, dim=3, n_even=0, n_odd=1, l=4),
        inputs.make_instance("cg-2d-24", 2, 24, 2, 0.8, 0.95, block=8, seed=31, n_even=0, n_odd=5, l=4),
        inputs.make_instance("cg-3d-6", 3, 6, 1, 0.8, 0.9, block=2, seed=32, n_even=0, n_odd=3, l=4),
        inputs.tiny_instance(n=8, sphere_level=1, g=0.4, ratio=0.9, n_even=0, n_odd=3, l=4, seed=9),
    ]
    e0 = [rte.RTE_E0_CG, rte.RTE_E0_MG, rte.RTE_E0_CG, rte.RTE_E0_MG, rte.RTE_E0_CG, rte.RTE_E0_BANDED]
    hs = [rte.Handle.from_instance(i, e0_solver=e, mixed=1) for i, e in zip(insts, e0)]
    precision = rte.RTE_FP64 if prec == "fp64" else rte.RTE_MIXED
    opts = []
    for k, e in enumerate(e0):
        o = rte.default_solve_opts(l=4, tol=1e-10, max_iter=300, precision=precision, e0_solver=e,
                                   odd_solver=rte.RTE_ODD_CONDENSED, cg_tol=1e-13,
                                   cg_max_iter=7 if k == 2 else 20000)
        opts.append(o)
    ref = []
    for h, o in zip(hs, opts):
        U = torch.empty((h.dims.nSp, h.dims.nRp), dtype=torch.float64, device="cuda")
        st, info = h.solve(U, opts=o, raise_on_notconv=False)
        torch.cuda.synchronize()
        ref.append((st, U, info))
    b = rte.Batch(max_slots=8)
    outs = [torch.full((h.dims.nSp, h.dims.nRp), np.nan, dtype=torch.float64, device="cuda") for h in hs]
    slots = [b.admit(h, U, o) for h, U, o in zip(hs, outs, opts)]
    assert b.step(1000) == 0
    torch.cuda.synchronize()
    done = {s: (st, info) for s, st, info in b.poll()}
    assert sorted(done) == sorted(slots)
    for k, (s, U) in enumerate(zip(slots, outs)):
        st, info = done[s]
        st0, U0, i0 = ref[k]
        print(f"[cg lockstep {prec} slot {k}] status {st} iters {info.iters} (alone {i0.iters}) "
              f"rel_resid {info.rel_resid:.2e}", flush=True)
        assert st == st0
        assert info.iters == i0.iters
        assert np.float64(info.rel_resid).tobytes() == np.float64(i0.rel_resid).tobytes()
        assert torch.equal(U.view(torch.int64), U0.view(torch.int64))
    b.close()
    for h in hs:
        h.close()
