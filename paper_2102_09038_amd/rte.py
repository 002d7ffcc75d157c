"""ctypes binding of librte (include/rte.h): the same entry points, argument marshalling only.

Device operands are torch tensors on ``cuda`` (their ``data_ptr()`` is passed through);
the stream is torch's current stream unless given.  Every computation happens in
librte's HIP kernels; there is no CPU fallback: importing this module without a built
``librte.so`` raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librte.so")

RTE_OK, RTE_E_ARG, RTE_E_PHYS, RTE_E_MESH, RTE_E_NOMEM, RTE_E_HIP, RTE_E_NOTCONV, RTE_E_NONFINITE, RTE_E_STALL = range(9)
RTE_FP64, RTE_MIXED = 0, 1
RTE_DT_F64, RTE_DT_F32, RTE_DT_BF16 = 0, 1, 2
RTE_ODD_PCG, RTE_ODD_EXACT, RTE_ODD_CONDENSED = 0, 1, 2
RTE_E0_CG, RTE_E0_BANDED, RTE_E0_MG = 0, 1, 2
RTE_INNER_RICHARDSON, RTE_INNER_PCG = 0, 1
RTE_COARSE_AUTO, RTE_COARSE_INVERSE, RTE_COARSE_BAND, RTE_COARSE_BLOCK, RTE_COARSE_QUICK = 0, 1, 2, 3, 4
ARRAY_SP, ARRAY_SM, ARRAY_M, ARRAY_T, ARRAY_Q, ARRAY_LAMP, ARRAY_WP, ARRAY_LAMM, ARRAY_CG_ITERS = range(9)
STATUS_NAMES = ["OK", "E_ARG", "E_PHYS", "E_MESH", "E_NOMEM", "E_HIP", "E_NOTCONV", "E_NONFINITE"]


class rte_problem_desc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_vert", C.c_int32), ("vert", C.POINTER(C.c_double)),
                ("n_cell", C.c_int32), ("cell", C.POINTER(C.c_int32)),
                ("sigma_t", C.POINTER(C.c_double)), ("sigma_s", C.POINTER(C.c_double)),
                ("g", C.c_double), ("n_svert", C.c_int32), ("svert", C.POINTER(C.c_double)),
                ("n_stri", C.c_int32), ("stri", C.POINTER(C.c_int32)),
                ("q_nodal", C.POINTER(C.c_double)), ("g_inflow", C.POINTER(C.c_double))]


class rte_assemble_opts(C.Structure):
    _fields_ = [("quad_level", C.c_int32), ("n_even", C.c_int32), ("n_odd", C.c_int32),
                ("e0_solver", C.c_int32), ("mixed", C.c_int32), ("odd_eig", C.c_int32),
                ("coarse_solver", C.c_int32)]


class rte_solve_opts(C.Structure):
    _fields_ = [("l", C.c_int32), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("precision", C.c_int32), ("odd_solver", C.c_int32), ("e0_solver", C.c_int32),
                ("pcg_tol_resid", C.c_double), ("pcg_tol_inner", C.c_double),
                ("pcg_max_iter", C.c_int32), ("cg_tol", C.c_double), ("cg_max_iter", C.c_int32),
                ("profile", C.c_int32), ("inner", C.c_int32), ("stall_ratio", C.c_double),
                ("stall_iters", C.c_int32)]


RTE_TUNE_FORCE = 1
# the (ring depth H, phase count P) shapes the band solve kernel is built for
BAND_SHAPES = [(9, 1), (17, 1), (33, 1), (9, 2), (17, 2), (33, 2), (17, 3), (33, 3), (33, 4)]


class rte_tune_report(C.Structure):
    _fields_ = [("n_cand", C.c_int32 * 2), ("H", (C.c_int32 * 9) * 2), ("P", (C.c_int32 * 9) * 2),
                ("ms", (C.c_double * 9) * 2), ("chosen_H", C.c_int32 * 2), ("chosen_P", C.c_int32 * 2),
                ("default_H", C.c_int32 * 2), ("default_P", C.c_int32 * 2), ("from_cache", C.c_int32 * 2),
                ("n_gemm", C.c_int32), ("gemm_kind", C.c_int32 * 4), ("gemm_m", C.c_int32 * 4),
                ("gemm_n", C.c_int32 * 4), ("gemm_k", C.c_int32 * 4), ("gemm_ms", (C.c_double * 4) * 4),
                ("gemm_map", C.c_int32 * 4), ("gemm_from_cache", C.c_int32 * 4)]


class rte_solve_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("rel_resid", C.c_double), ("stop_quantity", C.c_double),
                ("pcg_iters_total", C.c_int64), ("cg_iters_total", C.c_int64),
                ("cg_iters_max", C.c_int32), ("t_solve", C.c_double), ("t_e0inv", C.c_double),
                ("n_e0inv", C.c_int64), ("t_gemm", C.c_double), ("n_gemm", C.c_int64),
                ("gemm_flops", C.c_double), ("t_gemm_bf16", C.c_double), ("n_gemm_bf16", C.c_int64),
                ("gemm_bf16_flops", C.c_double), ("t_scatter", C.c_double), ("n_scatter", C.c_int64),
                ("scatter_flops", C.c_double), ("t_scatter_f32", C.c_double), ("n_scatter_f32", C.c_int64),
                ("scatter_f32_flops", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = {
    "rte_default_assemble_opts": (None, [C.POINTER(rte_assemble_opts)]),
    "rte_default_solve_opts": (None, [C.POINTER(rte_solve_opts)]),
    "rte_assemble": (C.c_int, [C.POINTER(rte_problem_desc), C.POINTER(rte_assemble_opts), C.c_void_p,
                               C.POINTER(C.c_void_p)]),
    "rte_query_dims": (C.c_int, [C.c_void_p] + [C.POINTER(C.c_int32)] * 4),
    "rte_footprint": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "rte_query_band": (C.c_int, [C.c_void_p] + [C.POINTER(C.c_int32)] * 3),
    "rte_apply_scatter": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                                    C.c_void_p]),
    "rte_apply_scatter_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                                            C.c_void_p]),
    "rte_apply_E": (C.c_int, [C.c_void_p, C.POINTER(rte_solve_opts), C.c_void_p, C.c_void_p, C.c_void_p]),
    "rte_apply_E0": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "rte_apply_E0inv": (C.c_int, [C.c_void_p, C.POINTER(rte_solve_opts), C.c_void_p, C.c_void_p, C.c_void_p]),
    "rte_apply_mg": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "rte_precond": (C.c_int, [C.c_void_p, C.POINTER(rte_solve_opts), C.c_int32, C.c_void_p, C.c_void_p,
                              C.c_void_p]),
    "rte_solve": (C.c_int, [C.c_void_p, C.POINTER(rte_solve_opts), C.c_void_p, C.c_void_p, C.c_void_p,
                            C.POINTER(rte_solve_info), C.c_void_p]),
    "rte_get_array": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t]),
    "rte_destroy": (C.c_int, [C.c_void_p]),
    "rte_estimate_footprint": (C.c_int, [C.POINTER(rte_problem_desc), C.POINTER(rte_assemble_opts),
                                         C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "rte_batch_create": (C.c_int, [C.c_int32, C.c_size_t, C.POINTER(C.c_void_p)]),
    "rte_batch_admit": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(rte_solve_opts), C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.POINTER(C.c_int32)]),
    "rte_batch_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_int32)]),
    "rte_batch_poll": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(rte_solve_info),
                                 C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "rte_batch_set_graphs": (C.c_int, [C.c_void_p, C.c_int32]),
    "rte_batch_usage": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_size_t)]),
    "rte_batch_destroy": (C.c_int, [C.c_void_p]),
    "rte_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "rte_set_band_layout": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p]),
    "rte_derived_outputs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "rte_last_error": (C.c_char_p, []),
}


def load_library(path: str = _LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"librte.so not built at {path}; run paper_2102_09038_amd.build.build()")
    lib = C.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = load_library()


class RteError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 8 else status}: {msg}")
        self.status = status


def _check(st):
    if st != RTE_OK:
        raise RteError(st, lib.rte_last_error().decode())
    return st


def _dptr(a):
    return C.cast(a.ctypes.data, C.POINTER(C.c_double))


def _iptr(a):
    return C.cast(a.ctypes.data, C.POINTER(C.c_int32))


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_assemble_opts(**kw) -> rte_assemble_opts:
    o = rte_assemble_opts()
    lib.rte_default_assemble_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def default_solve_opts(**kw) -> rte_solve_opts:
    o = rte_solve_opts()
    lib.rte_default_solve_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


@dataclass
class Dims:
    nRp: int
    nRm: int
    nSp: int
    nSm: int


def _make_desc(vert, cell, sigma_t, sigma_s, g, svert, stri, q_nodal):
    keep = [np.ascontiguousarray(vert, np.float64), np.ascontiguousarray(cell, np.int32),
            np.ascontiguousarray(sigma_t, np.float64), np.ascontiguousarray(sigma_s, np.float64),
            np.ascontiguousarray(svert, np.float64), np.ascontiguousarray(stri, np.int32),
            np.ascontiguousarray(q_nodal, np.float64)]
    v, c, st, ss, sv, stt, q = keep
    d = rte_problem_desc()
    d.dim = v.shape[1]
    d.n_vert = v.shape[0]
    d.vert = _dptr(v)
    d.n_cell = c.shape[0]
    d.cell = _iptr(c)
    d.sigma_t = _dptr(st)
    d.sigma_s = _dptr(ss)
    d.g = float(g)
    d.n_svert = sv.shape[0]
    d.svert = _dptr(sv)
    d.n_stri = stt.shape[0]
    d.stri = _iptr(stt)
    d.q_nodal = _dptr(q)
    d.g_inflow = None
    return keep, d


def estimate_footprint(inst, **opt_kw):
    """(bytes, peak_bytes) a handle of this instance will hold once assembled with these
    options (rte_estimate_footprint; host work only, no GPU needed)."""
    kw = dict(quad_level=inst.quad_level, n_even=inst.n_even, n_odd=inst.n_odd)
    kw.update(opt_kw)
    keep, d = _make_desc(inst.vert, inst.cell, inst.sigma_t, inst.sigma_s, inst.g, inst.svert, inst.stri,
                         inst.q_nodal)
    o = default_assemble_opts(**kw)
    b, p = C.c_size_t(0), C.c_size_t(0)
    _check(lib.rte_estimate_footprint(C.byref(d), C.byref(o), C.byref(b), C.byref(p)))
    return b.value, p.value


class Handle:
    """Owns an rte_handle; thin wrapper over the C entry points."""

    def __init__(self, vert, cell, sigma_t, sigma_s, g, svert, stri, q_nodal, opts=None, stream=None,
                 **opt_kw):
        self._keep, d = _make_desc(vert, cell, sigma_t, sigma_s, g, svert, stri, q_nodal)
        self.desc = d
        self.opts = opts if opts is not None else default_assemble_opts(**opt_kw)
        h = C.c_void_p()
        _check(lib.rte_assemble(C.byref(d), C.byref(self.opts), _stream(stream), C.byref(h)))
        self.h = h
        a = [C.c_int32() for _ in range(4)]
        _check(lib.rte_query_dims(h, *[C.byref(x) for x in a]))
        self.dims = Dims(*[x.value for x in a])

    @classmethod
    def from_instance(cls, inst, stream=None, **opt_kw):
        kw = dict(quad_level=inst.quad_level, n_even=inst.n_even, n_odd=inst.n_odd)
        kw.update(opt_kw)
        return cls(inst.vert, inst.cell, inst.sigma_t, inst.sigma_s, inst.g, inst.svert, inst.stri,
                   inst.q_nodal, stream=stream, **kw)

    def close(self):
        if getattr(self, "h", None):
            lib.rte_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def footprint(self) -> int:
        b = C.c_size_t()
        _check(lib.rte_footprint(self.h, C.byref(b)))
        return b.value

    def autotune(self, force=False, stream=None) -> dict:
        """Time the E_0 band solve in every factor layout that holds the band, and each GEMM
        shape of the handle in its four tile maps, and keep the fastest (rte_autotune).
        Returns, per precision of banded factors present, the shapes timed with their
        milliseconds per E_0^{-1}, the default and the chosen shape; under "gemm" a list of
        {kind, m, n, k, ms (per map), map, from_cache}."""
        r = rte_tune_report()
        _check(lib.rte_autotune(self.h, RTE_TUNE_FORCE if force else 0, _stream(stream), C.byref(r)))
        out = {}
        for i, name in ((0, "fp64"), (1, "fp32")):
            if r.chosen_H[i] == 0:
                continue
            out[name] = {"timed": [((r.H[i][c], r.P[i][c]), r.ms[i][c]) for c in range(r.n_cand[i])],
                         "default": (r.default_H[i], r.default_P[i]), "chosen": (r.chosen_H[i], r.chosen_P[i]),
                         "from_cache": bool(r.from_cache[i])}
        kinds = {1: "fp64", 2: "fp32", 4: "bf16"}
        out["gemm"] = [{"kind": kinds.get(r.gemm_kind[i], r.gemm_kind[i]), "m": r.gemm_m[i], "n": r.gemm_n[i],
                        "k": r.gemm_k[i], "ms": list(r.gemm_ms[i]), "map": r.gemm_map[i],
                        "from_cache": bool(r.gemm_from_cache[i])} for i in range(r.n_gemm)]
        return out

    def set_band_layout(self, precision, H, P, stream=None):
        """Lay the E_0 factors of one precision out in the band solve shape (H, P)."""
        _check(lib.rte_set_band_layout(self.h, int(precision), int(H), int(P), _stream(stream)))

    def band(self):
        """(E_0 band width, coarse unknowns, coarse band width)."""
        a = [C.c_int32() for _ in range(3)]
        _check(lib.rte_query_band(self.h, *[C.byref(x) for x in a]))
        return tuple(x.value for x in a)

    def get_array(self, which: int, shape) -> np.ndarray:
        out = np.empty(shape, dtype=np.float64, order="F")
        _check(lib.rte_get_array(self.h, which, out.ctypes.data, out.nbytes))
        return out

    def last_cg_iters(self) -> list:
        """Iterations every direction took in the last E_0^{-1} by CG."""
        out = np.empty(self.dims.nSp, dtype=np.int32)
        _check(lib.rte_get_array(self.h, ARRAY_CG_ITERS, out.ctypes.data, out.nbytes))
        return out.tolist()

    # --- operators on torch device tensors (column-major matrices are passed as the
    #     transposed-contiguous storage: a (n_rows, n_cols) Fortran matrix == a torch tensor
    #     of shape (n_cols, n_rows) contiguous)
    def apply_scatter(self, parity, X, Y, dtype_in=RTE_DT_F64, dtype_out=RTE_DT_F64, stream=None):
        _check(lib.rte_apply_scatter(self.h, parity, dtype_in, C.c_void_p(X.data_ptr()), dtype_out,
                                     C.c_void_p(Y.data_ptr()), _stream(stream)))

    def apply_scatter_noalloc(self, parity, X, Y, dtype_in=RTE_DT_F64, dtype_out=RTE_DT_F64, stream=None):
        _check(lib.rte_apply_scatter_noalloc(self.h, parity, dtype_in, C.c_void_p(X.data_ptr()), dtype_out,
                                             C.c_void_p(Y.data_ptr()), _stream(stream)))

    def apply_E(self, X, Y, opts=None, stream=None):
        o = opts or default_solve_opts()
        _check(lib.rte_apply_E(self.h, C.byref(o), C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()),
                               _stream(stream)))

    def apply_E0(self, X, Y, stream=None):
        _check(lib.rte_apply_E0(self.h, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()), _stream(stream)))

    def apply_mg(self, X, Y, stream=None):
        _check(lib.rte_apply_mg(self.h, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()), _stream(stream)))

    def apply_E0inv(self, X, Y, opts=None, stream=None):
        o = opts or default_solve_opts()
        _check(lib.rte_apply_E0inv(self.h, C.byref(o), C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()),
                                   _stream(stream)))

    def precond(self, which, r, s, opts=None, stream=None):
        o = opts or default_solve_opts()
        _check(lib.rte_precond(self.h, C.byref(o), which, C.c_void_p(r.data_ptr()), C.c_void_p(s.data_ptr()),
                               _stream(stream)))

    def solve(self, U, U0=None, opts=None, stream=None, raise_on_notconv=True, U_odd=None):
        o = opts or default_solve_opts()
        info = rte_solve_info()
        st = lib.rte_solve(self.h, C.byref(o), C.c_void_p(U0.data_ptr() if U0 is not None else 0),
                           C.c_void_p(U.data_ptr()), C.c_void_p(U_odd.data_ptr() if U_odd is not None else 0),
                           C.byref(info), _stream(stream))
        # the iteration cap and the stagnation test return the last iterate: raised only when asked
        if st != RTE_OK and (raise_on_notconv or st not in (RTE_E_NOTCONV, RTE_E_STALL)):
            _check(st)
        return st, info


    def derived_outputs(self, U, phi=None, stream=None) -> dict:
        """Scalar flux into phi (device, n_R+; optional) and the particle balance of U."""
        bal = np.zeros(4)
        _check(lib.rte_derived_outputs(self.h, C.c_void_p(U.data_ptr()),
                                       C.c_void_p(phi.data_ptr() if phi is not None else 0),
                                       C.c_void_p(bal.ctypes.data), _stream(stream)))
        return {"source": bal[0], "absorption": bal[1], "leakage": bal[2], "imbalance": bal[3]}


class Batch:
    """Lockstep batch of solves (rte_batch_*): admit handles with their output arrays, step
    all live slots together, poll finished ones.  Handles and arrays must outlive their slot."""

    def __init__(self, max_slots=64, hbm_budget=0, use_graphs=False):
        self.b = C.c_void_p()
        _check(lib.rte_batch_create(int(max_slots), int(hbm_budget), C.byref(self.b)))
        self._keep = {}
        _check(lib.rte_batch_set_graphs(self.b, 1 if use_graphs else 0))

    def close(self):
        if self.b:
            lib.rte_batch_destroy(self.b)
            self.b = C.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def admit(self, handle, U, opts=None, U0=None, stream=None) -> int:
        o = opts or default_solve_opts()
        slot = C.c_int32(-1)
        _check(lib.rte_batch_admit(self.b, handle.h, C.byref(o), C.c_void_p(U0.data_ptr() if U0 is not None else 0),
                                   C.c_void_p(U.data_ptr()), _stream(stream), C.byref(slot)))
        self._keep[slot.value] = (handle, U, U0)
        return slot.value

    def step(self, outer_iters=1, stream=None) -> int:
        n = C.c_int32(0)
        _check(lib.rte_batch_step(self.b, int(outer_iters), _stream(stream), C.byref(n)))
        return n.value

    def poll(self, max_out=None):
        m = max_out if max_out is not None else 4096
        slots = (C.c_int32 * m)()
        infos = (rte_solve_info * m)()
        stats = (C.c_int32 * m)()
        n = C.c_int32(0)
        _check(lib.rte_batch_poll(self.b, m, slots, infos, stats, C.byref(n)))
        out = []
        for i in range(n.value):
            self._keep.pop(slots[i], None)
            out.append((slots[i], stats[i], infos[i]))
        return out

    def usage(self):
        nl, nd, ub = C.c_int32(0), C.c_int32(0), C.c_size_t(0)
        _check(lib.rte_batch_usage(self.b, C.byref(nl), C.byref(nd), C.byref(ub)))
        return nl.value, nd.value, ub.value
