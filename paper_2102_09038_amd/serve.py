"""Continuous-batching request loop over librte's lockstep batch (rte_batch_*).

Requests (problem instances with an arrival time) are assembled on worker threads, each on
its own HIP stream, as soon as they have arrived and their predicted peak device footprint
(rte_estimate_footprint) fits into what the budget leaves.  Assembled requests are admitted
into the running batch between its steps; the batch advances every admitted solve by one
outer iteration per step; finished solves are polled, their handles freed, and their
latency (completion - arrival) recorded.  A request's result is the result rte_solve
computes for it alone: the batch runs the same arithmetic per slot.

The loop runs in real time: a request is not touched before its arrival time.

Requests on 2D meshes solve E_0 by band factors; requests on 3D meshes, whose bands are too
wide to factor, by the all-direction CG.  The two kinds step in two lockstep batches, one
after the other in the same loop, so that the grouped band solves of the 2D slots never wait
for a CG.
"""
from __future__ import annotations

import dataclasses
import queue
import threading
import time
from typing import Callable, List, Optional

import numpy as np

from . import rte


@dataclasses.dataclass
class Request:
    rid: int
    inst: object                     # an inputs.Instance
    arrival: float                   # seconds after the start of the run
    # filled in by the server
    assembled_at: float = float("nan")
    admitted_at: float = float("nan")
    done_at: float = float("nan")
    status: int = -1
    iters: int = 0
    rel_resid: float = float("nan")
    error: str = ""                  # the library's message when the request failed
    U: object = None                 # the solution (torch tensor on the device), if kept

    @property
    def latency(self) -> float:
        return self.done_at - self.arrival


def _is_lattice(vert) -> bool:
    """vert are the points of an m^d lattice of a box, numbered i + m (j + m k) (the meshes the
    multigrid E_0 solve accepts; the library checks the cells itself)."""
    nv, d = vert.shape
    m = int(round(nv ** (1.0 / d)))
    if m < 2 or m ** d != nv:
        return False
    lo, hi = vert.min(axis=0), vert.max(axis=0)
    idx = np.arange(nv)
    for a in range(d):
        c = (idx // m ** a) % m
        if not np.allclose(vert[:, a], lo[a] + (hi[a] - lo[a]) * c / (m - 1), rtol=0, atol=1e-12):
            return False
    return True


class Server:
    """One lockstep batch plus assembly workers.

    budget: device bytes the requests' handles (operators + solver workspace) may hold
    together, counted from admission of a request's assembly to the release of its slot.
    """

    def __init__(self, budget: int, solve_opts, max_slots: int = 256, workers: int = 4, mixed_assembly: int = 2,
                 keep_results: bool = False, on_done: Optional[Callable[[Request], None]] = None,
                 odd_eig: int = 0, use_graphs: bool = False, coarse_solver: int = rte.RTE_COARSE_QUICK):
        import torch
        # graph mode beside assembly workers: served runs once reported assembly inputs that
        # were not positive definite; the inputs that failed came from a vendor factorisation
        # whose result varied with concurrent device work, which assembly no longer uses for
        # the served configuration (odd_eig = 0, quick coarse set-up)
        self.torch = torch
        self.budget = int(budget)
        self.opts = solve_opts
        # the same options with the CG E_0 solves (multigrid-preconditioned on lattice meshes,
        # Jacobi otherwise), for the requests that use them
        self.opts_cg = rte.rte_solve_opts.from_buffer_copy(solve_opts)
        self.opts_cg.e0_solver = rte.RTE_E0_CG
        self.opts_mg = rte.rte_solve_opts.from_buffer_copy(solve_opts)
        self.opts_mg.e0_solver = rte.RTE_E0_MG
        self.batch = rte.Batch(max_slots=max_slots, hbm_budget=0, use_graphs=use_graphs)
        self.batch_cg = rte.Batch(max_slots=max_slots, hbm_budget=0, use_graphs=False)
        self.workers = workers
        self.mixed_assembly = mixed_assembly
        # the batch runs the condensed odd solve only: no odd eigendecomposition at assembly
        # (uniform sigma_s / sigma_t; ignored otherwise)
        self.odd_eig = odd_eig
        # short set-up first: the coarse system by the device band factorisation where it
        # applies (assembly bounds the served rate)
        self.coarse_solver = coarse_solver
        self.keep = keep_results
        self.on_done = on_done
        self.reserved = 0                          # bytes promised to requests being assembled or in slots
        self.stream = torch.cuda.Stream()
        self.slot_of = {}                          # (batch, slot) -> (request, handle, reserved bytes, U)
        self.t_step = 0.0                          # seconds inside batch steps
        self.peak_live = 0
        self.peak_reserved = 0                     # the most bytes promised at any time (<= budget)

    # ---------------------------------------------------------------------------- helpers
    @staticmethod
    def e0_solver_for(inst) -> int:
        """Band factors for 2D meshes; for 3D ones (bands too wide) the all-direction CG,
        preconditioned by the multigrid V-cycle when the mesh is a lattice."""
        if inst.dim == 2:
            return rte.RTE_E0_BANDED
        return rte.RTE_E0_MG if _is_lattice(inst.vert) else rte.RTE_E0_CG

    def _estimate(self, req):
        if not hasattr(req, "_est"):
            b, p = rte.estimate_footprint(req.inst, e0_solver=self.e0_solver_for(req.inst), mixed=self.mixed_assembly,
                                          odd_eig=self.odd_eig, coarse_solver=self.coarse_solver)
            req._est = (b, max(b, p))
        return req._est

    def _assemble(self, req: Request, stream):
        h = rte.Handle.from_instance(req.inst, stream=stream.cuda_stream, e0_solver=self.e0_solver_for(req.inst),
                                     mixed=self.mixed_assembly, odd_eig=self.odd_eig,
                                     coarse_solver=self.coarse_solver)
        return h

    # ---------------------------------------------------------------------------- main loop
    def run(self, requests: List[Request], step_iters: int = 1) -> List[Request]:
        torch = self.torch
        pending = sorted(requests, key=lambda r: r.arrival)
        ready: "queue.Queue" = queue.Queue()
        todo: "queue.Queue" = queue.Queue()
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0

        def worker():
            stream = torch.cuda.Stream()
            while True:
                item = todo.get()
                if item is None:
                    return
                req, est = item
                try:
                    h = self._assemble(req, stream)
                    req.assembled_at = now()
                    ready.put((req, h, est))
                except BaseException as e:            # reported by the main loop
                    e.args = (f"request {req.rid} ({getattr(req.inst, 'name', '?')}): {e}",)
                    ready.put((req, e, est))

        threads = [threading.Thread(target=worker, daemon=True) for _ in range(self.workers)]
        for t in threads:
            t.start()
        waiting = []                                  # arrived, not yet handed to a worker
        in_flight = 0                                 # handed to a worker, not yet admitted
        finished: List[Request] = []
        try:
            while len(finished) < len(requests):
                t = now()
                while pending and pending[0].arrival <= t:
                    waiting.append(pending.pop(0))
                # hand arrived requests to the workers while their predicted peak fits
                while waiting:
                    req = waiting[0]
                    b, peak = self._estimate(req)
                    if peak > self.budget:
                        raise RuntimeError(f"request {req.rid} needs {peak} bytes, more than the whole budget")
                    if self.reserved + peak > self.budget:
                        break
                    waiting.pop(0)
                    self.reserved += peak
                    self.peak_reserved = max(self.peak_reserved, self.reserved)
                    todo.put((req, (b, peak)))
                    in_flight += 1
                # admit what the workers have assembled
                while True:
                    try:
                        req, h, (b, peak) = ready.get_nowait()
                    except queue.Empty:
                        break
                    in_flight -= 1
                    if isinstance(h, rte.RteError):
                        # the request fails alone (its status is the library's); the loop goes on
                        self.reserved -= peak
                        req.done_at = now()
                        req.status, req.error = h.status, str(h)
                        finished.append(req)
                        if self.on_done:
                            self.on_done(req)
                        continue
                    if isinstance(h, BaseException):
                        raise h
                    self.reserved -= peak - b          # the assembly peak is over
                    U = torch.empty((h.dims.nSp, h.dims.nRp), dtype=torch.float64, device="cuda")
                    e0 = self.e0_solver_for(req.inst)
                    cg = e0 != rte.RTE_E0_BANDED
                    which = self.batch_cg if cg else self.batch
                    o = self.opts if not cg else self.opts_mg if e0 == rte.RTE_E0_MG else self.opts_cg
                    slot = which.admit(h, U, o, stream=self.stream.cuda_stream)
                    req.admitted_at = now()
                    self.slot_of[(int(cg), slot)] = (req, h, b, U)
                if self.slot_of:
                    self.peak_live = max(self.peak_live, len(self.slot_of))
                    ts = time.perf_counter()
                    polled = []
                    for cg, which in ((0, self.batch), (1, self.batch_cg)):
                        if any(key[0] == cg for key in self.slot_of):
                            which.step(step_iters, stream=self.stream.cuda_stream)
                            polled += [((cg, slot), st, info) for slot, st, info in which.poll()]
                    self.t_step += time.perf_counter() - ts
                    for key, st, info in polled:
                        req, h, b, U = self.slot_of.pop(key)
                        req.done_at = now()
                        req.status, req.iters, req.rel_resid = st, info.iters, info.rel_resid
                        if self.keep:
                            req.U = U
                        h.close()
                        self.reserved -= b
                        finished.append(req)
                        if self.on_done:
                            self.on_done(req)
                else:
                    # nothing to step: wait for an arrival or an assembly
                    if pending and not waiting and in_flight == 0:
                        time.sleep(max(0.0, min(0.01, pending[0].arrival - now())))
                    else:
                        try:
                            item = ready.get(timeout=0.01)
                            ready.put(item)
                        except queue.Empty:
                            pass
        finally:
            for _ in threads:
                todo.put(None)
            for t in threads:
                t.join(timeout=60)
            torch.cuda.synchronize()
        return finished

    def close(self):
        self.batch.close()
        self.batch_cg.close()


def percentile(values, q):
    v = sorted(values)
    if not v:
        return float("nan")
    k = (len(v) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(v) - 1)
    return v[lo] + (v[hi] - v[lo]) * (k - lo)
