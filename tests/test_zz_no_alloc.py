"""rte_apply_scatter_noalloc (no device allocation: its intermediates live in a fixed 64 MiB
scratch array per device) against rte_apply_scatter on the same inputs, through the C ABI.

Bar: FP64 arithmetic 1e-10 relative (the two entry points may split the GEMM differently),
FP32 MFMA arithmetic 1e-6.  Two calls in a row share the array, the second on a smaller
problem; both parities and every dtype pair are checked.  A problem whose intermediates
exceed the array is refused with RTE_E_ARG before any device work, and the largest that fits
is computed correctly.
"""
import numpy as np
import pytest

from paper_2102_09038_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _compare(h, parity, dtin, dtout, seed):
    from paper_2102_09038_amd import rte
    d = h.dims
    n, m = (d.nRp, d.nSp) if parity == 1 else (d.nRm, d.nSm)
    X = torch.from_numpy(np.random.default_rng(seed).standard_normal((m, n))).cuda()
    if dtin == rte.RTE_DT_F32:
        X = X.float().contiguous()
    tout = torch.float64 if dtout == rte.RTE_DT_F64 else torch.float32
    ref = torch.empty((m, n), dtype=tout, device="cuda")
    h.apply_scatter(parity, X, ref, dtype_in=dtin, dtype_out=dtout)
    got = torch.full((m, n), float("nan"), dtype=tout, device="cuda")
    h.apply_scatter_noalloc(parity, X, got, dtype_in=dtin, dtype_out=dtout)
    torch.cuda.synchronize()
    err = float(torch.linalg.norm((got - ref).double()) / torch.linalg.norm(ref.double()))
    bar = 1e-10 if dtin == rte.RTE_DT_F64 and dtout == rte.RTE_DT_F64 else 1e-6
    print(f"  parity {parity:+d} in {dtin} out {dtout}: {err:.2e}", flush=True)
    assert err < bar


def test_noalloc_matches_scatter_two_calls():
    from paper_2102_09038_amd import rte
    pairs = [(rte.RTE_DT_F64, rte.RTE_DT_F64), (rte.RTE_DT_F64, rte.RTE_DT_F32), (rte.RTE_DT_F32, rte.RTE_DT_F64),
             (rte.RTE_DT_F32, rte.RTE_DT_F32)]
    # the larger problem first, then a smaller one on the same scratch array
    for inst in (inputs.config_small(), inputs.tiny_instance(n=4, sphere_level=1)):
        print(f"[no-alloc] {inst.name}", flush=True)
        h = rte.Handle.from_instance(inst, mixed=1, odd_eig=0)
        for i, (dtin, dtout) in enumerate(pairs):
            for parity in (1, -1):
                _compare(h, parity, dtin, dtout, seed=100 + 2 * i + (parity > 0))
        h.close()


def test_noalloc_size_limit():
    """64 x 64 squares, 2048 sphere triangles: the product X S+ takes 4225 * 1024 * 8 =
    34.6 MB, which fits; with an FP32 result the FP64 copy doubles it to 69.2 MB, beyond the
    67.1 MB array, and the call is refused with the output untouched."""
    from paper_2102_09038_amd import rte
    inst = inputs.make_instance("noalloc-64x64-s2048", 2, 64, 4, 0.5, 0.9, sigma_t=1.0, quad_level=2, n_even=0,
                                n_odd=1, l=1)
    print(f"[no-alloc] {inst.name}", flush=True)
    h = rte.Handle.from_instance(inst, odd_eig=0)
    _compare(h, 1, rte.RTE_DT_F64, rte.RTE_DT_F64, seed=7)
    d = h.dims
    X = torch.zeros((d.nSp, d.nRp), dtype=torch.float64, device="cuda")
    Y = torch.full((d.nSp, d.nRp), 3.0, dtype=torch.float32, device="cuda")
    with pytest.raises(rte.RteError) as e:
        h.apply_scatter_noalloc(1, X, Y, dtype_out=rte.RTE_DT_F32)
    assert e.value.status == rte.RTE_E_ARG and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((Y == 3.0).all())
    h.close()
