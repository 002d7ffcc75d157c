"""Checkpoint / resume and the stagnation status of the outer iteration (Alg. 3).

* The iteration is stationary: u_{n+1} depends on u_n alone (Alg. 2's P_1^l and the subspace
  correction are fixed maps of the residual), so a solve stopped after 3 steps
  (RTE_E_NOTCONV, iterate returned) and resumed from U0 = that iterate reaches the result of
  the uninterrupted run bit for bit, with the remaining iteration count; in FP64 and mixed
  precision, as a single solve and as a batch slot.
* The stagnation test: with stall_ratio 0.01 (any real contraction is slower than that) and
  stall_iters 2 the solve stops with RTE_E_STALL at iteration 3 and returns the same iterate as
  a run capped at 3 iterations; with the test off the same solve converges.
"""
import numpy as np
import pytest

from paper_2102_09038_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    from paper_2102_09038_amd import rte
    inst = inputs.make_instance("resume-16x16-s128-g0.8", 2, 16, 2, 0.8, 0.95, block=4, seed=61, n_even=0, n_odd=5,
                                l=4, quad_level=2)
    h = rte.Handle.from_instance(inst, e0_solver=rte.RTE_E0_BANDED, mixed=1, odd_eig=0)
    yield h
    h.close()


def _opts(rte, precision, **kw):
    o = dict(l=4, tol=1e-10, max_iter=500, odd_solver=rte.RTE_ODD_CONDENSED, e0_solver=rte.RTE_E0_BANDED,
             precision=precision)
    o.update(kw)
    return rte.default_solve_opts(**o)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_resume_is_bitwise(handle, precision):
    from paper_2102_09038_amd import rte
    p = rte.RTE_FP64 if precision == "fp64" else rte.RTE_MIXED
    d = handle.dims
    full = torch.empty((d.nSp, d.nRp), dtype=torch.float64, device="cuda")
    st, info = handle.solve(full, opts=_opts(rte, p))
    assert st == rte.RTE_OK and info.iters > 3
    part = torch.empty_like(full)
    st3, i3 = handle.solve(part, opts=_opts(rte, p, max_iter=3), raise_on_notconv=False)
    assert st3 == rte.RTE_E_NOTCONV and i3.iters == 3
    res = torch.empty_like(full)
    st, ir = handle.solve(res, U0=part, opts=_opts(rte, p))
    print(f"[{precision}] {info.iters} iterations uninterrupted, 3 + {ir.iters} resumed")
    assert st == rte.RTE_OK and ir.iters == info.iters - 3
    assert torch.equal(res, full)
    # the same resumption as a batch slot
    b = rte.Batch(max_slots=2)
    Ub = torch.full_like(full, float("nan"))
    b.admit(handle, Ub, _opts(rte, p), U0=part)
    assert b.step(1000) == 0
    torch.cuda.synchronize()
    (_, stb, ib), = b.poll()
    b.close()
    assert stb == rte.RTE_OK and ib.iters == info.iters - 3
    assert torch.equal(Ub, full)


def test_stall_status(handle):
    from paper_2102_09038_amd import rte
    d = handle.dims
    U = torch.empty((d.nSp, d.nRp), dtype=torch.float64, device="cuda")
    st, info = handle.solve(U, opts=_opts(rte, rte.RTE_FP64, stall_ratio=0.01, stall_iters=2), raise_on_notconv=False)
    assert st == rte.RTE_E_STALL and info.iters == 3
    U3 = torch.empty_like(U)
    handle.solve(U3, opts=_opts(rte, rte.RTE_FP64, max_iter=3), raise_on_notconv=False)
    assert torch.equal(U, U3)
    with pytest.raises(rte.RteError) as e:
        handle.solve(U, opts=_opts(rte, rte.RTE_FP64, stall_ratio=0.01, stall_iters=2))
    assert e.value.status == rte.RTE_E_STALL
    # the batch reports it per slot
    b = rte.Batch(max_slots=2)
    Ub = torch.empty_like(U)
    b.admit(handle, Ub, _opts(rte, rte.RTE_FP64, stall_ratio=0.01, stall_iters=2))
    assert b.step(1000) == 0
    torch.cuda.synchronize()
    (_, stb, ib), = b.poll()
    b.close()
    assert stb == rte.RTE_E_STALL and ib.iters == 3 and torch.equal(Ub, U3)
    with pytest.raises(rte.RteError) as e:
        handle.solve(U, opts=_opts(rte, rte.RTE_FP64, stall_ratio=0.0, stall_iters=2))
    assert e.value.status == rte.RTE_E_ARG
