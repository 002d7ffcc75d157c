#!/usr/bin/env python3
"""Benchmark of the preconditioned Richardson solver on one MI355X.

One step = one complete solve (Alg. 3 of the paper) of the realistic instance
(128 x 128 "/" grid on [0,1]^2, 2048 sphere triangles, HG g = 0.9, sigma_t ~ U[1,10]
per 8x8 block with seed 1, sigma_s = 0.99 sigma_t, Gaussian-bump source, l = 4,
N+ = 0, N- = 5) from u = 0 to a relative residual of 1e-6, with inputs already resident
in HBM (assembly happens once, outside the timed region).

Prints ONE JSON line.  ``roofline`` is the dominant kernel (by time in the timed
steps), measured live with HIP events recorded by librte on the solve's stream;
``gemm`` is the scattering / odd-inverse GEMM against the FP64 MFMA peak;
``cpu_baseline`` times the oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_MFMA_PEAK_TFLOPS = 78.6    # MI355X dense FP64 matrix
BF16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix
FP32_MFMA_PEAK_TFLOPS = 157.3   # MI355X dense FP32 matrix


def cores_used():
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    return min(n, int(env)) if env and env.isdigit() else n


def cpu_baseline(inst, iters, l, seed=0):
    """Time the oracle on a bounded sample of the same solve and extrapolate to solves/s.

    Sampled (and scaled by the sampling factor): the HG scattering rows of 4 of the
    n_S+ direction pairs (oracle double quadrature, x n_S+/4 for the full S+ and S-), the
    sparse LU factorisation and one solve of 4 of the E_0 blocks (x n_S+/4), and the exact
    odd solve (dense Cholesky of an n_S- x n_S- SPD matrix, applied to 1/16 of the cells,
    x 16).  Timed in full: the spatial assembly, the angular quadrature and moments, and
    A, A^T, M+, R and the even scattering product on a full even vector.  Per outer
    iteration Alg. 3 costs l E_0 solves, l+1 applications of E and 2 of K+.
    """
    import numpy as np
    import scipy.linalg as sla
    import scipy.sparse.linalg as spla

    from oracle.discretize import discretize_instance, scattering_rows
    from oracle.operators import Operators

    rng = np.random.default_rng(seed)
    t = time.perf_counter
    t0 = t()
    D = discretize_instance(inst, with_scattering=False)
    ops = Operators(D, n_even=inst.n_even, n_odd=inst.n_odd)
    t_spatial = t() - t0
    nS = D.nS
    P = 4
    rows = np.linspace(0, nS - 1, P).astype(int)
    t0 = t()
    scattering_rows(D.quad, inst.g, rows)
    t_S = (t() - t0) * nS / P
    t0 = t()
    lus = [spla.splu(ops.E0_block(int(k))) for k in rows]
    t_e0f = (t() - t0) * nS / P
    b = rng.standard_normal(D.nRp)
    t0 = t()
    for lu in lus:
        lu.solve(b)
    t_e0s = (t() - t0) * nS / P
    MSm = ops.MSm
    t0 = t()
    cf = sla.cho_factor(MSm, lower=True)
    t_chol = t() - t0
    frac = 16
    B = rng.standard_normal((D.nRm // frac, 3 * nS))
    t0 = t()
    sla.cho_solve(cf, B.T)
    t_odd = (t() - t0) * frac
    U = rng.standard_normal((D.nRp, nS))
    Sfake = rng.standard_normal((nS, nS))
    t0 = t()
    V = ops.A(U)
    ops.At(V)
    ops.M_even(U)
    ops.R(U)
    t_glue = t() - t0
    t0 = t()
    D.Ms @ (U @ Sfake)
    t_k = t() - t0
    t_E = t_odd + t_glue
    t_iter = l * t_e0s + (l + 1) * t_E + 2 * t_k
    t_setup = t_spatial + t_S + t_e0f + t_chol
    t_solve = t_setup + iters * t_iter
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": cores_used(), "kind": "oracle",
            "sample": (f"oracle on the same instance: S rows of {P}/{nS} direction pairs, E_0 LU of {P}/{nS} "
                       f"blocks, odd Cholesky solve on 1/{frac} of the cells, full spatial/glue operators; "
                       f"extrapolated to assembly + {iters} outer iterations (the GPU's count)"),
            "est_seconds_per_solve": t_solve, "est_setup_s": t_setup, "est_iter_s": t_iter}


def ell_entries(inst):
    """Entries per direction of the CG's sliced-ELL storage of the P1 pattern: every slice of 64
    rows holds 64 entries per slot, as many slots as its longest row."""
    import numpy as np
    import scipy.sparse as sp
    c = np.asarray(inst.cell)
    nv, n = c.shape[1], len(inst.vert)
    rows = np.repeat(c, nv, axis=1).ravel()
    cols = np.tile(c, (1, nv)).ravel()
    A = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
    A.sum_duplicates()
    rl = np.diff(A.indptr)
    rl = np.concatenate([rl, np.zeros((-n) % 64, dtype=rl.dtype)])
    return int(rl.reshape(-1, 64).max(axis=1).sum() * 64)


COPY_BYTES = 4 << 30
ROOT = os.path.dirname(os.path.abspath(__file__))


def measured_traffic(key):
    """HBM bytes per launch of a kernel from the committed counter summary, or None when
    no summary holds the key or the kernel's source changed since the counters were taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.md"))):
        for line in open(path):
            f = line.split()
            if len(f) == 5 and f[0] == "traffic:" and f[1] == key:
                src = os.path.join(ROOT, f[2])
                if not os.path.exists(src):
                    return None
                if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != f[3]:
                    return None
                return float(f[4])
    return None


def kernel_passes(h, inst, torch, rte):
    """The launches the HBM counter passes read, in this order: the condensed ApplyE in FP64
    (transport GEMM, A^T kernel) and in mixed precision (BF16 GEMM, FP32 A^T kernel), each
    twice; E_0^{-1} with FP64 and with FP32 band factors, twice each; the scatter GEMM U S+
    in FP64 and in FP32 MFMA, twice each; a plain device copy of COPY_BYTES, twice."""
    d = h.dims
    gen = torch.Generator(device="cuda").manual_seed(0)
    X = torch.randn((d.nSp, d.nRp), dtype=torch.float64, device="cuda", generator=gen)
    Y = torch.empty_like(X)
    for prec in (rte.RTE_FP64, rte.RTE_MIXED):
        e_opts = rte.default_solve_opts(odd_solver=rte.RTE_ODD_CONDENSED, precision=prec)
        for _ in range(2):
            h.apply_E(X, Y, e_opts)
    for prec in (rte.RTE_FP64, rte.RTE_MIXED):
        o = rte.default_solve_opts(e0_solver=rte.RTE_E0_BANDED, precision=prec)
        for _ in range(2):
            h.apply_E0inv(X, Y, o)
    for _ in range(2):
        h.apply_E0(X, Y)
    Xf = X.float()
    for _ in range(2):
        h.apply_scatter(1, X, Y)
    for _ in range(2):
        h.apply_scatter(1, Xf, Y, dtype_in=rte.RTE_DT_F32, dtype_out=rte.RTE_DT_F64)
    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"kernel_passes": ["apply_E condensed fp64 x2", "apply_E condensed mixed x2",
                                        "E0inv banded fp64 x2", "E0inv banded fp32 x2", "E0 SpMV fp64 x2",
                                        "K+ fp64 x2", "K+ fp32 x2",
                                        f"device copy {COPY_BYTES} bytes x2"]}))


def batched_form(torch, rte, inputs, count, tol, log, with_server=True, graph_modes=(False,)):
    """The batched form: count seeded instances of uneven size (N ~ U{32..128}, 128/512/2048
    sphere triangles, g ~ U[0,0.95], ratio ~ U[0.5,0.999]).
    - Baseline: the plain FP64 GPU solve, one instance at a time (assembled, solved and
      released in turn; solve and assembly timed separately).
    - Lockstep: every instance that fits the device-memory budget assembled beforehand in
      mixed-only form, all admitted at once and stepped to completion in mixed precision; its
      rate is compared with the FP64 rate over the same instances (like for like).
    - Server (with_server): all instances arrive at once; the continuous-batching loop
      assembles them on worker threads within the budget and steps them (end to end).
    All stop at the same FP64 relative residual tol.  Every result's error is taken against a
    tight FP64 reference solve of its instance (relative residual 1e-11), for the FP64 and the
    mixed results alike, and against the FP64 result at tol."""
    import numpy as np

    from paper_2102_09038_amd import serve

    insts = inputs.instance_distribution(count=count, seed=3, tol=tol)
    base = dict(l=4, max_iter=2000, odd_solver=rte.RTE_ODD_CONDENSED, e0_solver=rte.RTE_E0_BANDED)
    o64 = rte.default_solve_opts(precision=rte.RTE_FP64, tol=tol, **base)
    otight = rte.default_solve_opts(precision=rte.RTE_FP64, tol=1e-11, **base)
    omx = rte.default_solve_opts(precision=rte.RTE_MIXED, tol=tol, **base)
    # ---- baseline: plain FP64, one instance at a time; then an untimed tight reference solve
    ref, tight, t64, it64, asm64, res64 = [], [], [], [], [], []
    for i, inst in enumerate(insts):
        ta = time.perf_counter()
        h = rte.Handle.from_instance(inst, e0_solver=rte.RTE_E0_BANDED, mixed=0, odd_eig=0,
                                     coarse_solver=rte.RTE_COARSE_QUICK)
        asm64.append(time.perf_counter() - ta)
        U = torch.empty((h.dims.nSp, h.dims.nRp), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, info = h.solve(U, opts=o64, raise_on_notconv=False)
        torch.cuda.synchronize()
        t64.append(time.perf_counter() - t0)
        it64.append(info.iters)
        res64.append(info.rel_resid)
        ref.append(U.cpu())
        h.solve(U, opts=otight, raise_on_notconv=False)
        tight.append(U.cpu())
        h.close()
        del U
        log(f"[fp64 {i + 1}/{len(insts)}] {inst.name}: {info.iters} iters, {1e3 * t64[-1]:.0f} ms, "
            f"assembly {asm64[-1]:.2f} s")

    def err(U, i, against):
        R = against[i]
        return float(torch.linalg.norm(U - R) / torch.linalg.norm(R))

    err64_tight = [err(ref[i], i, tight) for i in range(len(insts))]
    budget = int(240e9)
    # ---- lockstep stepping of pre-assembled instances (mixed-only form), in order while their
    #      handles fit the budget together
    hs, sub, held = [], [], 0
    for i, inst in enumerate(insts):
        b_est, p_est = rte.estimate_footprint(inst, e0_solver=rte.RTE_E0_BANDED, mixed=2, odd_eig=0,
                                              coarse_solver=rte.RTE_COARSE_QUICK)
        if held + max(b_est, p_est) > budget:
            continue
        hs.append(rte.Handle.from_instance(inst, e0_solver=rte.RTE_E0_BANDED, mixed=2, odd_eig=0,
                                           coarse_solver=rte.RTE_COARSE_QUICK))
        sub.append(i)
        held += b_est
    t64_sub = sum(t64[i] for i in sub)
    lockstep = {}
    for graphs in graph_modes:
        b = rte.Batch(max_slots=len(hs), use_graphs=graphs)
        Us = [torch.empty((h.dims.nSp, h.dims.nRp), dtype=torch.float64, device="cuda") for h in hs]
        for h, U in zip(hs, Us):
            b.admit(h, U, omx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        left = b.step(100000)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res = b.poll()
        assert left == 0 and len(res) == len(hs)
        by_slot = {slot: info for slot, _, info in res}
        e_tight = [err(Us[j].cpu(), i, tight) for j, i in enumerate(sub)]
        e_64 = [err(Us[j].cpu(), i, ref) for j, i in enumerate(sub)]
        lockstep["graphs" if graphs else "direct"] = {
            "instances": len(hs), "solves_per_s": len(hs) / dt, "step_s": dt,
            "fp64_same_instances_solves_per_s": len(hs) / t64_sub,
            "speedup_vs_fp64_same_instances": t64_sub / dt,
            "lockstep_iters": max(i.iters for i in by_slot.values()),
            "max_rel_resid": max(i.rel_resid for i in by_slot.values()),
            "rel_err_vs_tight_reference": {"max": max(e_tight), "median": float(np.median(e_tight))},
            "rel_err_vs_fp64_result": {"max": max(e_64), "median": float(np.median(e_64))}}
        log(f"[lockstep graphs={graphs}] {len(hs)} solves in {dt:.2f} s (FP64 one at a time: {t64_sub:.2f} s)")
        b.close()
        del Us
    for h in hs:
        h.close()
    out = {
        "workload": f"batched form: {len(insts)} seeded instances (N 32..128, 128/512/2048 sphere triangles, "
                    f"g 0..0.95, ratio 0.5..0.999), rel. residual {tol:g}",
        "fp64_one_at_a_time": {"solves_per_s": len(insts) / sum(t64), "solve_s": sum(t64),
                               "assembly_s": sum(asm64),
                               "end_to_end_solves_per_s": len(insts) / (sum(t64) + sum(asm64)),
                               "iters_total": int(sum(it64)), "max_rel_resid": max(res64),
                               "rel_err_vs_tight_reference": {"max": max(err64_tight),
                                                              "median": float(np.median(err64_tight))}},
        "mixed_lockstep_preassembled": lockstep,
    }
    if with_server:
        reqs = [serve.Request(rid=i, inst=inst, arrival=0.0) for i, inst in enumerate(insts)]
        srv = serve.Server(budget, omx, max_slots=len(insts), workers=4, keep_results=True)
        t0 = time.perf_counter()
        done = srv.run(reqs)
        wall = time.perf_counter() - t0
        srv.close()
        e_tight = [err(r.U.cpu(), r.rid, tight) for r in done]
        e_64 = [err(r.U.cpu(), r.rid, ref) for r in done]
        log(f"[server] {len(done)} solved in {wall:.1f} s ({srv.t_step:.1f} s stepping), "
            f"peak {srv.peak_live} live slots")
        out["mixed_server"] = {
            "solves_per_s_stepping": len(insts) / srv.t_step, "step_s": srv.t_step, "wall_s": wall,
            "end_to_end_solves_per_s": len(insts) / wall,
            "speedup_end_to_end_vs_fp64": (sum(t64) + sum(asm64)) / wall,
            "speedup_stepping_vs_fp64_solves": sum(t64) / srv.t_step,
            "iters_total": int(sum(r.iters for r in done)),
            "all_converged": all(r.status == rte.RTE_OK for r in done),
            "max_rel_resid": max(r.rel_resid for r in done),
            "rel_err_vs_tight_reference": {"max": max(e_tight), "median": float(np.median(e_tight)),
                                           "per_instance": [round(e, 12) for e in e_tight]},
            "rel_err_vs_fp64_result": {"max": max(e_64), "median": float(np.median(e_64))},
            "peak_live_slots": srv.peak_live, "hbm_budget": budget, "assembly_workers": 4}
    return out


def batch_bench(args, torch, rte, inputs):
    def log(msg):
        print(msg, file=sys.stderr, flush=True)
    print(json.dumps(batched_form(torch, rte, inputs, args.count, args.tol, log, with_server=True,
                                  graph_modes=(True, False))))


def serving_runs(torch, rte, inputs, rates, requests, tol, warm=8, log=None, errors=True, fraction_3d=0.0):
    """The served form: Poisson arrivals (seed 4) of requests drawn like the batched form,
    served by the continuous-batching loop (mixed precision, assembly on worker threads,
    admission by predicted footprint) and, as the baseline, by plain FP64 solves one at a
    time in arrival order.  Latency = completion - arrival; the first warm-up requests of
    each run are not counted.  rates: list of requests/s or 'half' (half the capacity the
    batched loop reached at the highest numeric rate).  errors: every measured batched result
    is compared, after the run, with a tight FP64 solve (relative residual 1e-11) of its
    request.  fraction_3d: that share of the requests are the 3D ones (32^3 Kuhn tetrahedra, 512
    sphere triangles, g = 0.8), solved with the CG E_0 (cg_tol 1e-8 in FP64, 1e-6 in FP32; the
    tight reference 1e-12) in both forms."""
    import numpy as np

    from paper_2102_09038_amd import serve

    log = log or (lambda msg: None)
    n = requests + warm
    insts = inputs.instance_distribution(count=n, seed=4, tol=tol, large_3d_fraction=fraction_3d)
    base = dict(l=4, tol=tol, max_iter=2000, odd_solver=rte.RTE_ODD_CONDENSED, e0_solver=rte.RTE_E0_BANDED)
    omx = rte.default_solve_opts(precision=rte.RTE_MIXED, **base)
    o64 = rte.default_solve_opts(precision=rte.RTE_FP64, **base)
    rng = np.random.Generator(np.random.PCG64(4))
    unit = np.cumsum(rng.exponential(1.0, size=n))          # arrivals at rate 1, scaled per run
    unit -= unit[0]

    def stats(reqs, t_wall):
        m = [r for r in reqs if r.rid >= warm]
        lat = [r.latency for r in m]
        first = min(r.arrival for r in m)
        last = max(r.done_at for r in m)
        return {"p50_s": serve.percentile(lat, 50), "p99_s": serve.percentile(lat, 99),
                "mean_s": float(np.mean(lat)), "solves_per_s": len(m) / (last - first),
                "all_converged": all(r.status == rte.RTE_OK for r in m),
                "n_failed": sum(r.status not in (rte.RTE_OK, rte.RTE_E_NOTCONV) for r in m), "wall_s": t_wall}

    otight = rte.default_solve_opts(precision=rte.RTE_FP64, **dict(base, tol=1e-11))

    def with_e0(o, inst, cg_tol):
        """o with the E_0 solver the server uses for inst (CG for 3D meshes)."""
        e0 = serve.Server.e0_solver_for(inst)
        if e0 == rte.RTE_E0_BANDED:
            return o, e0
        oc = rte.rte_solve_opts.from_buffer_copy(o)
        oc.e0_solver, oc.cg_tol, oc.cg_max_iter = e0, cg_tol, 20000
        return oc, e0

    def errors_vs_tight(done_mixed, done_fp64):
        """Each measured result of both forms against a tight FP64 solve of its request (untimed,
        after the runs)."""
        by_rid = {r.rid: r for r in done_fp64}
        em, ef, names = [], [], []
        tick = progress("tight reference")
        for r in sorted(done_mixed, key=lambda r: r.rid):
            tick()
            if r.rid < warm or r.U is None:
                continue
            ot, e0 = with_e0(otight, r.inst, 1e-12)
            h = rte.Handle.from_instance(r.inst, e0_solver=e0, mixed=0, odd_eig=0,
                                         coarse_solver=rte.RTE_COARSE_QUICK)
            R = torch.empty_like(r.U)
            h.solve(R, opts=ot, raise_on_notconv=False)
            nr = torch.linalg.norm(R)
            em.append(float(torch.linalg.norm(r.U - R) / nr))
            names.append((r.rid, r.inst.name, r.iters, float(r.rel_resid)))
            f = by_rid.get(r.rid)
            if f is not None and f.U is not None:
                ef.append(float(torch.linalg.norm(f.U - R) / nr))
                f.U = None
            h.close()
            r.U = None

        def summ(v, worst=None):
            if not v:
                return None
            out = {"max": max(v), "median": float(np.median(v)), "per_request": [round(e, 12) for e in v]}
            if worst:
                rid, name, iters, res = worst[int(np.argmax(v))]
                out["worst"] = {"request": rid, "instance": name, "iters": iters, "rel_resid": res}
            return out
        return summ(em, names), summ(ef)

    def progress(what):
        """a callback that logs every 16th completed request (long runs print as they go)"""
        count = [0]

        def tick(*_):
            count[0] += 1
            if count[0] % 16 == 0 or count[0] == n:
                log(f"[serve]   {what}: {count[0]}/{n}")
        return tick

    def run_batched(rate):
        reqs = [serve.Request(rid=i, inst=insts[i], arrival=float(unit[i] / rate)) for i in range(n)]
        srv = serve.Server(int(240e9), omx, max_slots=n, workers=4, keep_results=errors,
                           on_done=progress("batched done"))
        t0 = time.perf_counter()
        done = srv.run(reqs)
        srv.close()
        st = stats(done, time.perf_counter() - t0)
        st["peak_live_slots"] = srv.peak_live
        return st, done

    def run_fp64_serial(rate):
        reqs = [serve.Request(rid=i, inst=insts[i], arrival=float(unit[i] / rate)) for i in range(n)]
        t0 = time.perf_counter()
        tick = progress("fp64 done")
        for r in reqs:
            wait = r.arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            o, e0 = with_e0(o64, r.inst, 1e-8)
            h = rte.Handle.from_instance(r.inst, e0_solver=e0, mixed=0, odd_eig=0,
                                         coarse_solver=rte.RTE_COARSE_QUICK)
            U = torch.empty((h.dims.nSp, h.dims.nRp), dtype=torch.float64, device="cuda")
            st, info = h.solve(U, opts=o, raise_on_notconv=False)
            torch.cuda.synchronize()
            r.status, r.iters = st, info.iters
            r.done_at = time.perf_counter() - t0
            if errors and r.rid >= warm:
                r.U = U
            h.close()
            tick()
        return stats(reqs, time.perf_counter() - t0), reqs

    numeric = [float(x) for x in rates if x != "half"]
    n3 = sum(1 for i in insts[warm:] if i.dim == 3)
    out = {"workload": f"served form: Poisson arrivals (seed 4), {requests} measured requests per rate after "
                       f"{warm} warm-up, drawn like the batched form"
                       + (f" plus {n3} 3D requests (32^3, 512 sphere triangles, g = 0.8)" if n3 else " (2D)")
                       + f", rel. residual {tol:g}",
           "rates": {}}
    for x in rates:
        rate = float(x) if x != "half" else 0.5 * out["rates"][str(x_max(numeric))]["batched"]["solves_per_s"]
        log(f"[serve] rate {rate:.2f}/s: batched")
        b, done_b = run_batched(rate)
        log(f"[serve] rate {rate:.2f}/s: fp64 one at a time")
        f, done_f = run_fp64_serial(rate)
        if errors:
            b["rel_err_vs_tight_reference"], f["rel_err_vs_tight_reference"] = errors_vs_tight(done_b, done_f)
        key = str(x) if x != "half" else f"half capacity ({rate:.2f}/s)"
        out["rates"][key] = {"rate": rate, "batched": b, "fp64_one_at_a_time": f}
        log(f"[serve] rate {rate:.2f}/s: batched p50 {b['p50_s']:.2f} s p99 {b['p99_s']:.2f} s "
            f"{b['solves_per_s']:.2f}/s | fp64 p50 {f['p50_s']:.2f} s p99 {f['p99_s']:.2f} s {f['solves_per_s']:.2f}/s")
    return out


def e0inv_3d(torch, rte, inputs, log):
    """E_0^{-1} of the served form's 3D request (32^3 cubes in Kuhn tetrahedra, 512 sphere
    triangles, g = 0.8) by the Jacobi CG and by the multigrid-preconditioned CG, FP32 to 1e-6
    and FP64 to 1e-10, and its mixed solve to 1e-6 with the multigrid E_0."""
    import numpy as np
    inst = inputs.make_instance("req-3d-32-s512", 3, 32, 3, 0.8, 0.9, seed=1001, n_even=0, n_odd=5, l=4, tol=1e-6)
    t0 = time.perf_counter()
    h = rte.Handle.from_instance(inst, e0_solver=rte.RTE_E0_MG, mixed=1, odd_eig=0,
                                 coarse_solver=rte.RTE_COARSE_QUICK)
    out = {"workload": "served 3D request: 32^3 cubes (Kuhn tetrahedra), 512 sphere triangles, g 0.8",
           "n_R+": len(inst.vert), "n_S+": h.dims.nSp, "assembly_s": time.perf_counter() - t0}
    B = torch.from_numpy(np.random.default_rng(91).standard_normal((h.dims.nSp, h.dims.nRp))).cuda()
    X = torch.empty_like(B)
    for e0, name in ((rte.RTE_E0_CG, "jacobi_cg"), (rte.RTE_E0_MG, "multigrid_cg")):
        res = {}
        for prec, pname, tol in ((rte.RTE_MIXED, "fp32", 1e-6), (rte.RTE_FP64, "fp64", 1e-10)):
            o = rte.default_solve_opts(e0_solver=e0, precision=prec, cg_tol=tol, cg_max_iter=20000)
            h.apply_E0inv(B, X, o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h.apply_E0inv(B, X, o)
            torch.cuda.synchronize()
            res[pname] = {"ms": 1e3 * (time.perf_counter() - t0), "cg_tol": tol,
                          "max_iters": max(h.last_cg_iters())}
            log(f"[3d E_0^-1] {name} {pname}: {res[pname]['ms']:.1f} ms, {res[pname]['max_iters']} iterations")
        out[name] = res
    # the CG's SpMV on this request (rte_apply_E0, FP64, all 256 directions), timed like the 2D
    # one: HIP events on its stream; the explicit values, the column pattern, X and Y once
    len_ell = ell_entries(inst)
    nb = h.dims.nSp * len_ell * 8 + len_ell * 4 + 2 * h.dims.nRp * h.dims.nSp * 8
    stream = torch.cuda.current_stream()
    h.apply_E0(B, X, stream=stream.cuda_stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_spmv = 20
    ev0.record(stream)
    for _ in range(n_spmv):
        h.apply_E0(B, X, stream=stream.cuda_stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / n_spmv
    gbs = nb / (ms * 1e-3) / 1e9
    out["spmv"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                   "kernel": "cg_spmv_kernel<double> (E_0 X, sliced ELL, all directions)", "avg_launch_ms": ms,
                   "launches": n_spmv, "bytes_per_launch": nb, "ell_entries_per_direction": len_ell}
    log(f"[3d spmv] {ms:.4f} ms, {gbs:.0f} GB/s = {gbs / HBM_PEAK_GBS:.3f} of {HBM_PEAK_GBS:.0f} GB/s")
    o = rte.default_solve_opts(l=4, tol=1e-6, max_iter=400, odd_solver=rte.RTE_ODD_CONDENSED, e0_solver=rte.RTE_E0_MG,
                               precision=rte.RTE_MIXED, cg_max_iter=2000)
    U = torch.empty_like(B)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, info = h.solve(U, opts=o)
    torch.cuda.synchronize()
    out["mixed_solve_multigrid"] = {"s": time.perf_counter() - t0, "iters": info.iters, "rel_resid": info.rel_resid}
    log(f"[3d solve] multigrid E_0, mixed: {info.iters} iterations in {out['mixed_solve_multigrid']['s']:.2f} s")
    h.close()
    return out


def x_max(v):
    m = max(v)
    return int(m) if float(m).is_integer() else m


def serve_bench(args, torch, rte, inputs):
    def log(msg):
        print(msg, file=sys.stderr, flush=True)
    rates = [x for x in args.rates.split(",") if x]
    print(json.dumps(serving_runs(torch, rte, inputs, rates, args.requests, args.tol, log=log,
                                  fraction_3d=args.fraction_3d)))


def rates_study(args, torch, rte, inputs):
    """Convergence rates rho and eta of the iteration matrix (Sec. 6.2) on the lattice
    stand-in (56 x 56 squares on (0,7)^2, c = 10/10.01): g = 0 over angular grids of
    16..1024 even directions (N+ = 0, P_1 = E^{-1}), and g in {0.1, 0.5, 0.9} over
    d_N in {1, 6, 15} and l = 1..4 at 64 even directions."""
    from paper_2102_09038_amd.rates import iteration_rates

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    def one(inst, ls):
        t0 = time.perf_counter()
        h = rte.Handle.from_instance(inst, e0_solver=rte.RTE_E0_BANDED)
        res = {}
        for l in ls:
            o = rte.default_solve_opts(l=l, odd_solver=rte.RTE_ODD_EXACT, e0_solver=rte.RTE_E0_BANDED)
            r = iteration_rates(h, o, m=80, tol=1e-5)
            res[l] = {"rho": r["rho"], "eta": r["eta"], "steps": [r["rho_steps"], r["eta_steps"]]}
            log(f"[rates] {inst.name} N+={inst.n_even} l={l}: rho {r['rho']:.3f} eta {r['eta']:.3f} "
                f"({time.perf_counter() - t0:.1f} s)")
        h.close()
        return res

    out = {"study": "convergence rates rho, eta of (I - P_G)(I - P_1^l (E - K+))",
           "workload": "lattice stand-in 56x56 on (0,7)^2, sigma_s/sigma_a 10/0.01 and 0/1, c = 0.999",
           "isotropic": {}, "anisotropic": {}}
    for lev in ((1, 2, 3, 4) if args.rates_isotropic else ()):
        inst = inputs.lattice_standin(sphere_level=lev, g=0.0, n_even=0)
        out["isotropic"][4 ** (lev + 1)] = one(inst, [1])[1]
    for g in [float(x) for x in args.rates_g.split(",") if x]:
        for n_even in (0, 2, 4):
            # d_N = 15 makes a coarse system of 48735 unknowns: block-tridiagonal Cholesky
            inst = inputs.lattice_standin(sphere_level=2, g=g, n_even=n_even)
            d_n = (n_even + 1) * (n_even + 2) // 2
            out["anisotropic"][f"g={g} d_N={d_n}"] = one(inst, [1, 2, 3, 4])
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the short served-form run")
    ap.add_argument("--no-batched", action="store_true", help="skip the short batched-form run")
    ap.add_argument("--only", choices=["kernels", "batch", "serve", "rates", "e0inv3d"], default=None,
                    help="'kernels': assemble the realistic instance, run the dominant kernels twice each "
                         "and a plain 4 GiB device copy (the reference for HBM counter passes), then exit; "
                         "'batch': the batched form (seeded instances of uneven size, mixed precision, "
                         "lockstep batch) against the same instances solved one at a time in FP64; "
                         "'rates': the convergence-rate study on the lattice stand-in; "
                         "'e0inv3d': E_0^{-1} of the served 3D request by the Jacobi and the multigrid CG, "
                         "and its mixed solve")
    ap.add_argument("--count", type=int, default=64, help="instances of the batched form")
    ap.add_argument("--rates", default="50,200,1000,half",
                    help="served form: Poisson arrival rates in requests/s ('half' = half the capacity "
                         "measured at the highest listed rate)")
    ap.add_argument("--requests", type=int, default=64, help="served form: measured requests per rate")
    ap.add_argument("--rates-isotropic", type=int, default=1, help="rates study: include the g = 0 table (0/1)")
    ap.add_argument("--rates-g", default="0.1,0.5,0.9", help="rates study: anisotropy factors g of the d_N x l tables")
    ap.add_argument("--fraction-3d", type=float, default=0.0,
                    help="served form: share of 3D requests (32^3 Kuhn tetrahedra, 512 sphere triangles)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver has no multi-GPU path "
              "(instances would shard by direction and by cells; nothing here uses a second GPU).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2102_09038_amd import inputs, rte

    if args.only == "batch":
        batch_bench(args, torch, rte, inputs)
        return
    if args.only == "serve":
        serve_bench(args, torch, rte, inputs)
        return
    if args.only == "rates":
        rates_study(args, torch, rte, inputs)
        return
    if args.only == "e0inv3d":
        print(json.dumps(e0inv_3d(torch, rte, inputs, lambda m: print(m, file=sys.stderr, flush=True))))
        return
    inst = inputs.config_realistic()
    ta = time.perf_counter()
    # the condensed odd solve only: no odd eigendecomposition at assembly
    h = rte.Handle.from_instance(inst, e0_solver=rte.RTE_E0_BANDED, mixed=1, odd_eig=0)
    t_assemble = time.perf_counter() - ta
    d = h.dims
    # band layout of the E_0 factors (every shape that holds the band) and the tile map of each
    # GEMM shape, timed on the device, the fastest kept (setup, outside the timed solves)
    ta = time.perf_counter()
    tune = h.autotune()
    t_tune = time.perf_counter() - ta
    gemm_tune = tune.pop("gemm")
    print(f"[autotune] {t_tune:.2f} s: " + "; ".join(
        f"{k} default {v['default']} chosen {v['chosen']} timed " +
        ", ".join(f"{hp}:{ms:.3f}ms" for hp, ms in v["timed"]) for k, v in tune.items()) + "; gemm " + ", ".join(
        f"{g['kind']} {g['m']}x{g['n']}x{g['k']} map {g['map']}" +
        ("" if g["from_cache"] else " (" + "/".join(f"{ms:.3f}" for ms in g["ms"]) + " ms)") for g in gemm_tune),
        file=sys.stderr, flush=True)
    if args.only == "kernels":
        kernel_passes(h, inst, torch, rte)
        return
    e0_bw, _, _ = h.band()
    opts = rte.default_solve_opts(l=inst.l, tol=args.tol, max_iter=1000, odd_solver=rte.RTE_ODD_CONDENSED,
                                  e0_solver=rte.RTE_E0_BANDED, pcg_tol_inner=1e-6, profile=1)
    U = torch.empty((d.nSp, d.nRp), dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        h.solve(U, opts=opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        st, info = h.solve(U, opts=opts)
        infos.append(info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = args.steps / dt
    print(f"[fp64] {args.steps} solves in {dt:.2f} s", file=sys.stderr, flush=True)

    t_e0 = sum(i.t_e0inv for i in infos)
    n_e0 = sum(i.n_e0inv for i in infos)
    t_gm = sum(i.t_gemm for i in infos)
    n_gm = sum(i.n_gemm for i in infos)
    fl_gm = sum(i.gemm_flops for i in infos)
    t_sc = sum(i.t_scatter for i in infos)
    n_sc = sum(i.n_scatter for i in infos)
    fl_sc = sum(i.scatter_flops for i in infos)
    # algorithmic bytes of one E_0^{-1} launch: the band factor streamed twice (forward and
    # backward sweep) plus the right-hand side read and the solution written once
    n, bw = d.nRp, e0_bw
    factor_entries = n * (bw + 1) - bw * (bw + 1) // 2
    e0_bytes = d.nSp * (2 * factor_entries * 8 + 2 * n * 8)
    e0_gbs = e0_bytes / (t_e0 / n_e0) / 1e9 if n_e0 else 0.0
    gemm_tf = fl_gm / t_gm / 1e12 if t_gm else 0.0
    scatter_tf = fl_sc / t_sc / 1e12 if t_sc else 0.0
    e0_roof = {"bound": "hbm", "achieved": e0_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": e0_gbs / HBM_PEAK_GBS, "traffic": measured_traffic("band_solve_f64"),
               "kernel": "band_solve_kernel<double> (E_0^-1, all directions)",
               "avg_launch_ms": 1e3 * t_e0 / max(n_e0, 1), "launches": n_e0,
               "bytes_per_launch": e0_bytes, "time_share": t_e0 / dt}
    gemm_roof = {"bound": "mfma", "achieved": gemm_tf, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                 "frac": gemm_tf / FP64_MFMA_PEAK_TFLOPS, "traffic": measured_traffic("gemm_f64_transport"),
                 "kernel": "gemm_f64_dtl_kernel (condensed transport term of E; direct-to-LDS tiles)",
                 "avg_launch_ms": 1e3 * t_gm / max(n_gm, 1), "launches": n_gm,
                 "flops_per_launch": fl_gm / max(n_gm, 1), "time_share": t_gm / dt}
    dominant, other = (e0_roof, gemm_roof) if t_e0 >= t_gm else (gemm_roof, e0_roof)

    out = {
        "metric": "solves/sec to 1e-6 rel. residual (mixed vs FP64); scatter GEMM TFLOP/s; p99 latency",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": inst.name, "n_R+": d.nRp, "n_R-": d.nRm, "n_S+": d.nSp, "n_S-": d.nSm,
                   "tol": args.tol, "l": inst.l, "N+": inst.n_even, "N-": inst.n_odd,
                   "odd_solver": "condensed", "e0_solver": "banded", "e0_band": e0_bw, "precision": "fp64"},
        "iters": [i.iters for i in infos], "rel_resid": [i.rel_resid for i in infos],
        "t_assemble_s": t_assemble,
        "band_layout": {k: {"default": v["default"], "chosen": v["chosen"],
                            "timed_ms": {f"{hp[0]}x{hp[1]}": ms for hp, ms in v["timed"]}}
                        for k, v in tune.items()},
        "gemm_tile_map": [{"kind": g["kind"], "mnk": [g["m"], g["n"], g["k"]], "map": g["map"],
                           "timed_ms": g["ms"] if not g["from_cache"] else None} for g in gemm_tune],
        "t_autotune_s": t_tune,
        "roofline": dominant, "roofline_other": other,
        "scatter_gemm": {"bound": "mfma", "achieved": scatter_tf, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": scatter_tf / FP64_MFMA_PEAK_TFLOPS, "kernel": "gemm_mfma_kernel<double> (U S+, eq. tpmv; last round split over K)",
                         "avg_launch_ms": 1e3 * t_sc / max(n_sc, 1), "launches": n_sc,
                         "flops_per_launch": fl_sc / max(n_sc, 1), "traffic": measured_traffic("gemm_f64_scatter")},
    }
    # particle balance of the FP64 solution (source = absorption + leakage up to the residual)
    out["balance"] = h.derived_outputs(U)
    # ---- the SpMV of the CG E_0 solve (Sec. 5.3), rte_apply_E0 on all 1024 directions, timed
    #      with HIP events on the stream it is launched on; algorithmic bytes per launch: the
    #      explicit values of every block, the shared column pattern, X read and Y written once
    len_ell = ell_entries(inst)
    spmv_bytes = d.nSp * len_ell * 8 + len_ell * 4 + 2 * d.nRp * d.nSp * 8
    stream = torch.cuda.current_stream()
    Xs = torch.randn((d.nSp, d.nRp), dtype=torch.float64, device="cuda")
    Ys = torch.empty_like(Xs)
    h.apply_E0(Xs, Ys, stream=stream.cuda_stream)        # builds the explicit values once
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_spmv = 20
    ev0.record(stream)
    for _ in range(n_spmv):
        h.apply_E0(Xs, Ys, stream=stream.cuda_stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    spmv_ms = ev0.elapsed_time(ev1) / n_spmv
    spmv_gbs = spmv_bytes / (spmv_ms * 1e-3) / 1e9
    out["spmv"] = {"bound": "hbm", "achieved": spmv_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": spmv_gbs / HBM_PEAK_GBS, "traffic": measured_traffic("cg_spmv_f64"),
                   "kernel": "cg_spmv_kernel<double> (E_0 X, sliced ELL, all directions)",
                   "avg_launch_ms": spmv_ms, "launches": n_spmv, "bytes_per_launch": spmv_bytes,
                   "ell_entries_per_direction": len_ell}
    # E_0^{-1} by the CG path on the same workload (context for the banded solve above)
    cg_out = {}
    for name, prec, tol in (("fp64", rte.RTE_FP64, 1e-10), ("fp32", rte.RTE_MIXED, 1e-6)):
        oc = rte.default_solve_opts(e0_solver=rte.RTE_E0_CG, precision=prec, cg_tol=tol, cg_max_iter=20000,
                                    profile=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.apply_E0inv(Xs, Ys, oc)
        torch.cuda.synchronize()
        cg_out[name] = {"ms": 1e3 * (time.perf_counter() - t0), "cg_tol": tol}
    out["e0inv_cg"] = cg_out
    del Xs, Ys
    # ---- the mixed-precision form of the same solve: BF16/FP32 preconditioner (condensed
    #      transport GEMM in BF16 with FP32 accumulation, FP32 E_0 band factors), FP64
    #      outer residual, dots and coarse solve
    U64 = U.clone()
    mopts = rte.default_solve_opts(l=inst.l, tol=args.tol, max_iter=1000, odd_solver=rte.RTE_ODD_CONDENSED,
                                   e0_solver=rte.RTE_E0_BANDED, precision=rte.RTE_MIXED, profile=1)
    Um = torch.empty_like(U)
    for _ in range(args.warmup):
        h.solve(Um, opts=mopts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    minfos = []
    for _ in range(args.steps):
        st, info = h.solve(Um, opts=mopts)
        minfos.append(info)
    torch.cuda.synchronize()
    mdt = time.perf_counter() - t0
    print(f"[mixed] {args.steps} solves in {mdt:.2f} s", file=sys.stderr, flush=True)
    tb = sum(i.t_gemm_bf16 for i in minfos)
    fb = sum(i.gemm_bf16_flops for i in minfos)
    nb = sum(i.n_gemm_bf16 for i in minfos)
    bf16_tf = fb / tb / 1e12 if tb else 0.0
    t_e0m = sum(i.t_e0inv for i in minfos)
    n_e0m = sum(i.n_e0inv for i in minfos)
    e0m_bytes = d.nSp * (2 * factor_entries * 4 + 2 * n * 8)
    ts32 = sum(i.t_scatter_f32 for i in minfos)
    fs32 = sum(i.scatter_f32_flops for i in minfos)
    ns32 = sum(i.n_scatter_f32 for i in minfos)
    s32_tf = fs32 / ts32 / 1e12 if ts32 else 0.0
    e0m_gbs = e0m_bytes / (t_e0m / max(n_e0m, 1)) / 1e9 if n_e0m else 0.0
    out["mixed"] = {
        "value": args.steps / mdt, "unit": "solves/s", "ms_per_step": 1e3 * mdt / args.steps,
        "speedup_vs_fp64": (args.steps / mdt) / value, "iters": [i.iters for i in minfos],
        "rel_resid": [i.rel_resid for i in minfos],
        "rel_err_vs_fp64_solution": float(torch.linalg.norm(Um - U64) / torch.linalg.norm(U64)),
        "dtype": "bf16 transport GEMM (fp32 acc), fp32 MFMA scatter GEMM in the preconditioner, fp32 E_0 factors, "
                 "fp64 residual/dots/coarse",
        "scatter_gemm_fp32": {"bound": "mfma", "achieved": s32_tf, "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                              "frac": s32_tf / FP32_MFMA_PEAK_TFLOPS, "kernel": "gemm_mfma_kernel<float> (U S+)",
                              "avg_launch_ms": 1e3 * ts32 / max(ns32, 1), "launches": ns32,
                              "flops_per_launch": fs32 / max(ns32, 1), "traffic": measured_traffic("gemm_f32_scatter")},
        # the method's contraction, 2 n_R- (d n_S+)^2 per launch (the operator's diagonal blocks
        # are zero in the BF16 copy and applied by the A^T kernel; K is the full d n_S+)
        "gemm_bf16": {"bound": "mfma", "achieved": bf16_tf, "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": bf16_tf / BF16_MFMA_PEAK_TFLOPS, "avg_launch_ms": 1e3 * tb / max(nb, 1),
                      "launches": nb, "flops_per_launch": fb / max(nb, 1),
                      "traffic": measured_traffic("gemm_bf16_transport")},
        "e0inv_fp32": {"bound": "hbm", "achieved": e0m_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": e0m_gbs / HBM_PEAK_GBS, "avg_launch_ms": 1e3 * t_e0m / max(n_e0m, 1),
                       "bytes_per_launch": e0m_bytes, "traffic": measured_traffic("band_solve_f32")},
    }
    # the side measurements below (other correction space, other inner iteration) repeat each
    # solve a fixed few times, whatever --steps says, so the whole line stays within minutes
    side_steps, side_warmup = min(args.steps, 4), min(args.warmup, 1)
    # ---- the same workload with the larger correction space N+ = 4 (d_N = 15, 249615 coarse
    #      unknowns solved by the block-tridiagonal Cholesky)
    h4 = rte.Handle.from_instance(inputs.config_realistic(n_even=4), e0_solver=rte.RTE_E0_BANDED, mixed=1, odd_eig=0)
    out["n_even_4"] = {}
    for name, base_opts in (("fp64", opts), ("mixed", mopts)):
        o4 = rte.default_solve_opts(l=base_opts.l, tol=base_opts.tol, max_iter=base_opts.max_iter,
                                    odd_solver=base_opts.odd_solver, e0_solver=base_opts.e0_solver,
                                    precision=base_opts.precision)
        U4 = torch.empty_like(U)
        for _ in range(side_warmup):
            h4.solve(U4, opts=o4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        i4 = [h4.solve(U4, opts=o4)[1] for _ in range(side_steps)]
        torch.cuda.synchronize()
        dt4 = time.perf_counter() - t0
        print(f"[n_even 4 {name}] {side_steps} solves in {dt4:.2f} s", file=sys.stderr, flush=True)
        out["n_even_4"][name] = {"value": side_steps / dt4, "unit": "solves/s", "ms_per_step": 1e3 * dt4 / side_steps,
                                 "steps": side_steps, "warmup": side_warmup,
                                 "iters": [i.iters for i in i4], "rel_resid": [i.rel_resid for i in i4],
                                 "rel_diff_vs_fp64_solution": float(torch.linalg.norm(U4 - U64) / torch.linalg.norm(U64))}
    h4.close()
    # ---- P_1 as l steps of E_0-preconditioned CG (the non-stationary inner iteration of
    #      Sec. 5.3) instead of P_1^l, in both precisions; same workload and residual
    out["inner_pcg"] = {}
    for name, base_opts, base_value in (("fp64", opts, value), ("mixed", mopts, out["mixed"]["value"])):
        po = rte.default_solve_opts(l=base_opts.l, tol=base_opts.tol, max_iter=base_opts.max_iter,
                                    odd_solver=base_opts.odd_solver, e0_solver=base_opts.e0_solver,
                                    precision=base_opts.precision, inner=rte.RTE_INNER_PCG)
        Up = torch.empty_like(U)
        for _ in range(side_warmup):
            h.solve(Up, opts=po)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pinfos = [h.solve(Up, opts=po)[1] for _ in range(side_steps)]
        torch.cuda.synchronize()
        pdt = time.perf_counter() - t0
        print(f"[inner pcg {name}] {side_steps} solves in {pdt:.2f} s", file=sys.stderr, flush=True)
        out["inner_pcg"][name] = {
            "value": side_steps / pdt, "unit": "solves/s", "ms_per_step": 1e3 * pdt / side_steps,
            "steps": side_steps, "warmup": side_warmup,
            "speedup_vs_richardson_inner": (side_steps / pdt) / base_value,
            "iters": [i.iters for i in pinfos], "rel_resid": [i.rel_resid for i in pinfos],
            "rel_diff_vs_fp64_solution": float(torch.linalg.norm(Up - U64) / torch.linalg.norm(U64))}
    h.close()
    def log(msg):
        print(msg, file=sys.stderr, flush=True)
    # the 3D request's E_0^{-1}: Jacobi against multigrid-preconditioned CG
    out["e0inv_3d_request"] = e0inv_3d(torch, rte, inputs, log)
    if not args.no_batched:
        # the batched form on 16 instances of its distribution (the full 64 are bench.py --only batch)
        out["batched"] = batched_form(torch, rte, inputs, 16, args.tol, log, with_server=False)
    if not args.no_serving:
        # the served form at one arrival rate, reduced to 64 requests (the full study is
        # bench.py --only serve)
        sv = serving_runs(torch, rte, inputs, ["50"], 64, args.tol, warm=4)
        r = sv["rates"]["50"]
        out["serving"] = {"workload": sv["workload"], "rate_per_s": 50,
                          "p50_latency_s": r["batched"]["p50_s"], "p99_latency_s": r["batched"]["p99_s"],
                          "solves_per_s": r["batched"]["solves_per_s"],
                          "fp64_one_at_a_time": {"p50_latency_s": r["fp64_one_at_a_time"]["p50_s"],
                                                 "p99_latency_s": r["fp64_one_at_a_time"]["p99_s"],
                                                 "solves_per_s": r["fp64_one_at_a_time"]["solves_per_s"]},
                          "all_converged": r["batched"]["all_converged"],
                          "rel_err_vs_tight_reference": {k: v for k, v in
                                                         r["batched"]["rel_err_vs_tight_reference"].items()
                                                         if k != "per_request"},
                          "fp64_rel_err_vs_tight_reference": {k: v for k, v in
                                                              r["fp64_one_at_a_time"]["rel_err_vs_tight_reference"].items()
                                                              if k != "per_request"}}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, infos[-1].iters, inst.l)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
