// extern "C" entry points of librte (declared in include/rte.h).  Every call converts
// internal exceptions into an rte_status and records the message for rte_last_error().
#include <new>

#include "ops.h"
#include "rte_internal.h"
#include "solver_detail.h"

namespace {
thread_local std::string g_last_error;

template <typename F>
rte_status guarded(F&& f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const rte::Error& e) {
        g_last_error = e.what();
        return e.status;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return RTE_E_NOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return RTE_E_ARG;
    }
}

hipStream_t as_stream(void* p) { return reinterpret_cast<hipStream_t>(p); }

void check_opts(const rte_solve_opts* o) {
    if (!o) rte::fail(RTE_E_ARG, "null solve options");
    if (o->l < 1 || o->l > 64) rte::fail(RTE_E_ARG, "l must lie in 1..64");
    if (!(o->tol > 0) || o->max_iter < 0) rte::fail(RTE_E_ARG, "tol must be > 0 and max_iter >= 0");
    if (o->precision != RTE_FP64 && o->precision != RTE_MIXED) rte::fail(RTE_E_ARG, "unknown precision");
    if (o->odd_solver != RTE_ODD_PCG && o->odd_solver != RTE_ODD_EXACT && o->odd_solver != RTE_ODD_CONDENSED)
        rte::fail(RTE_E_ARG, "unknown odd solver");
    if (o->e0_solver != RTE_E0_CG && o->e0_solver != RTE_E0_BANDED && o->e0_solver != RTE_E0_MG)
        rte::fail(RTE_E_ARG, "unknown E_0 solver");
    if (o->inner != RTE_INNER_RICHARDSON && o->inner != RTE_INNER_PCG) rte::fail(RTE_E_ARG, "unknown inner iteration");
    if (!(o->pcg_tol_resid > 0) || !(o->pcg_tol_inner > 0) || !(o->cg_tol > 0) || o->pcg_max_iter < 1 ||
        o->cg_max_iter < 1)
        rte::fail(RTE_E_ARG, "inner tolerances must be > 0 and iteration caps >= 1");
    if (o->stall_iters < 0 || (o->stall_iters > 0 && !(o->stall_ratio > 0)))
        rte::fail(RTE_E_ARG, "stall_iters must be >= 0 and stall_ratio > 0 when it is on");
}

rte::Handle* as_handle(rte_handle* h) {
    if (!h) rte::fail(RTE_E_ARG, "null handle");
    return reinterpret_cast<rte::Handle*>(h);
}
}  // namespace

extern "C" {

void rte_default_assemble_opts(rte_assemble_opts* o) {
    if (!o) return;
    o->quad_level = 2;
    o->n_even = 0;
    o->n_odd = 5;
    o->e0_solver = RTE_E0_CG;
    o->mixed = 0;
    o->odd_eig = 1;
    o->coarse_solver = RTE_COARSE_AUTO;
}

void rte_default_solve_opts(rte_solve_opts* o) {
    if (!o) return;
    o->l = 4;
    o->tol = 1e-8;
    o->max_iter = 200;
    o->precision = RTE_FP64;
    o->odd_solver = RTE_ODD_PCG;
    o->e0_solver = RTE_E0_CG;
    o->pcg_tol_resid = 1e-12;
    o->pcg_tol_inner = 1e-10;
    o->pcg_max_iter = 200;
    o->cg_tol = 1e-10;
    o->cg_max_iter = 20000;
    o->profile = 0;
    o->inner = RTE_INNER_RICHARDSON;
    o->stall_ratio = 1.0;
    o->stall_iters = 0;
}

rte_status rte_assemble(const rte_problem_desc* desc, const rte_assemble_opts* opts, void* hip_stream,
                        rte_handle** out) {
    return guarded([&] {
        if (!out) rte::fail(RTE_E_ARG, "null output handle pointer");
        *out = nullptr;
        rte::Handle* h = rte::assemble(desc, opts, as_stream(hip_stream));
        // set-up of this device for rte_apply_scatter_noalloc (the address of its scratch
        // array), after validation and assembly so that invalid input still fails first
        try {
            rte::noalloc_setup();
        } catch (...) {
            delete h;
            throw;
        }
        *out = reinterpret_cast<rte_handle*>(h);
        return RTE_OK;
    });
}

rte_status rte_query_dims(const rte_handle* hh, int32_t* nRp, int32_t* nRm, int32_t* nSp, int32_t* nSm) {
    return guarded([&] {
        const rte::Handle* h = as_handle(const_cast<rte_handle*>(hh));
        if (nRp) *nRp = h->nRp;
        if (nRm) *nRm = h->nRm;
        if (nSp) *nSp = h->nS;
        if (nSm) *nSm = h->nSm;
        return RTE_OK;
    });
}

rte_status rte_query_band(const rte_handle* hh, int32_t* e0_bw, int32_t* coarse_n, int32_t* coarse_bw) {
    return guarded([&] {
        const rte::Handle* h = as_handle(const_cast<rte_handle*>(hh));
        if (e0_bw) *e0_bw = h->have_e0_banded ? h->sbw : 0;
        if (coarse_n) *coarse_n = h->nc;
        if (coarse_bw) *coarse_bw = h->cbw;
        return RTE_OK;
    });
}

rte_status rte_footprint(const rte_handle* hh, size_t* bytes) {
    return guarded([&] {
        const rte::Handle* h = as_handle(const_cast<rte_handle*>(hh));
        if (!bytes) rte::fail(RTE_E_ARG, "null output");
        *bytes = h->footprint();
        return RTE_OK;
    });
}

rte_status rte_apply_scatter(rte_handle* hh, int32_t parity, int32_t dtype_in, const void* X, int32_t dtype_out,
                             void* Y, void* hip_stream) {
    return guarded([&] {
        rte::Handle* h = as_handle(hh);
        if (!X || !Y) rte::fail(RTE_E_ARG, "null operand");
        if (parity != 1 && parity != -1) rte::fail(RTE_E_ARG, "parity must be +1 or -1");
        rte::apply_scatter(h, parity, dtype_in, X, dtype_out, Y, as_stream(hip_stream));
        return RTE_OK;
    });
}

rte_status rte_apply_scatter_noalloc(rte_handle* hh, int32_t parity, int32_t dtype_in, const void* X,
                                     int32_t dtype_out, void* Y, void* hip_stream) {
    return guarded([&] {
        rte::Handle* h = as_handle(hh);
        if (!X || !Y) rte::fail(RTE_E_ARG, "null operand");
        if (parity != 1 && parity != -1) rte::fail(RTE_E_ARG, "parity must be +1 or -1");
        rte::apply_scatter_noalloc(h, parity, dtype_in, X, dtype_out, Y, as_stream(hip_stream));
        return RTE_OK;
    });
}

rte_status rte_apply_E(rte_handle* hh, const rte_solve_opts* o, const double* X, double* Y, void* hip_stream) {
    return guarded([&] {
        rte::Handle* h = as_handle(hh);
        check_opts(o);
        if (!X || !Y) rte::fail(RTE_E_ARG, "null operand");
        rte::apply_E(h, o, X, Y, as_stream(hip_stream), nullptr);
        return RTE_OK;
    });
}

rte_status rte_apply_E0(rte_handle* hh, const double* X, double* Y, void* hip_stream) {
    return guarded([&] {
        rte::Handle* h = as_handle(hh);
        if (!X || !Y) rte::fail(RTE_E_ARG, "null operand");
        rte::apply_E0(h, X, Y, as_stream(hip_stream));
        return RTE_OK;
    });
}

rte_status rte_apply_mg(rte_handle* hh, const double* X, double* Y, void* hip_stream) {
    return guarded([&] {
        rte::Handle* h = as_handle(hh);
        if (!X || !Y) rte::fail(RTE_E_ARG, "null operand");
        rte::apply_mg(h, X, Y, as_stream(hip_stream));
        return RTE_OK;
    });
}

rte_status rte_apply_E0inv(rte_handle* hh, const rte_solve_opts* o, const double* X, double* Y,
                           void* hip_stream) {
    return guarded([&] {
        rte::Handle* h = as_handle(hh);
        check_opts(o);
        if (!X || !Y) rte::fail(RTE_E_ARG, "null operand");
        rte::apply_E0inv(h, o, X, Y, as_stream(hip_stream), nullptr, nullptr);
        return RTE_OK;
    });
}

rte_status rte_precond(rte_handle* hh, const rte_solve_opts* o, int32_t which, const double* r, double* s,
                       void* hip_stream) {
    return guarded([&] {
        rte::Handle* h = as_handle(hh);
        check_opts(o);
        if (!r || !s) rte::fail(RTE_E_ARG, "null operand");
        if (which != 0 && which != 1) rte::fail(RTE_E_ARG, "which must be 0 (P1) or 1 (P2 P1)");
        rte::precond(h, o, which, r, s, as_stream(hip_stream));
        return RTE_OK;
    });
}

rte_status rte_solve(rte_handle* hh, const rte_solve_opts* o, const double* U0, double* U_even, double* U_odd,
                     rte_solve_info* info, void* hip_stream) {
    return guarded([&] {
        rte::Handle* h = as_handle(hh);
        check_opts(o);
        if (!U_even) rte::fail(RTE_E_ARG, "null U_even");
        if (U_odd && !h->have_exact) rte::fail(RTE_E_ARG, "the odd part needs the exact odd inverse of the handle");
        const rte_status st = rte::solve(h, o, U0, U_even, U_odd, info, as_stream(hip_stream));
        if (st == RTE_E_NOTCONV) g_last_error = "iteration cap reached before the tolerance";
        if (st == RTE_E_NONFINITE) g_last_error = "residual is not finite";
        return st;
    });
}

rte_status rte_estimate_footprint(const rte_problem_desc* desc, const rte_assemble_opts* opts, size_t* bytes,
                                  size_t* peak_bytes) {
    return guarded([&] {
        if (!bytes) rte::fail(RTE_E_ARG, "null output");
        *bytes = rte::estimate_footprint(desc, opts, peak_bytes);
        return RTE_OK;
    });
}

rte_status rte_batch_create(int32_t max_slots, size_t hbm_budget, rte_batch** out) {
    return guarded([&] {
        if (!out) rte::fail(RTE_E_ARG, "null output");
        *out = nullptr;
        *out = reinterpret_cast<rte_batch*>(rte::batch_create(max_slots, hbm_budget));
        return RTE_OK;
    });
}

rte_status rte_batch_admit(rte_batch* b, rte_handle* hh, const rte_solve_opts* o, const double* U0, double* U,
                           void* hip_stream, int32_t* slot) {
    return guarded([&] {
        if (!b) rte::fail(RTE_E_ARG, "null batch");
        rte::Handle* h = as_handle(hh);
        check_opts(o);
        if (!U) rte::fail(RTE_E_ARG, "null U");
        const int id = rte::batch_admit(reinterpret_cast<rte::Batch*>(b), h, o, U0, U, as_stream(hip_stream));
        if (slot) *slot = id;
        return RTE_OK;
    });
}

rte_status rte_batch_step(rte_batch* b, int32_t outer_iters, void* hip_stream, int32_t* n_live) {
    return guarded([&] {
        if (!b) rte::fail(RTE_E_ARG, "null batch");
        if (outer_iters < 0) rte::fail(RTE_E_ARG, "outer_iters must be >= 0");
        const int nl = rte::batch_step(reinterpret_cast<rte::Batch*>(b), outer_iters, as_stream(hip_stream));
        if (n_live) *n_live = nl;
        return RTE_OK;
    });
}

rte_status rte_batch_poll(rte_batch* b, int32_t max_out, int32_t* slots, rte_solve_info* infos, int32_t* statuses,
                          int32_t* n_done) {
    return guarded([&] {
        if (!b) rte::fail(RTE_E_ARG, "null batch");
        if (max_out < 0) rte::fail(RTE_E_ARG, "max_out must be >= 0");
        const int n = rte::batch_poll(reinterpret_cast<rte::Batch*>(b), max_out, slots, infos, statuses);
        if (n_done) *n_done = n;
        return RTE_OK;
    });
}

rte_status rte_batch_set_graphs(rte_batch* b, int32_t use_graphs) {
    return guarded([&] {
        if (!b) rte::fail(RTE_E_ARG, "null batch");
        rte::batch_set_graphs(reinterpret_cast<rte::Batch*>(b), use_graphs != 0);
        return RTE_OK;
    });
}

rte_status rte_autotune(rte_handle* hh, int32_t flags, void* hip_stream, rte_tune_report* report) {
    return guarded([&] {
        if (!hh) rte::fail(RTE_E_ARG, "null handle");
        rte::autotune(reinterpret_cast<rte::Handle*>(hh), flags, static_cast<hipStream_t>(hip_stream), report);
        return RTE_OK;
    });
}

rte_status rte_set_band_layout(rte_handle* hh, int32_t precision, int32_t H, int32_t P, void* hip_stream) {
    return guarded([&] {
        if (!hh) rte::fail(RTE_E_ARG, "null handle");
        rte::set_band_layout(reinterpret_cast<rte::Handle*>(hh), precision, H, P, static_cast<hipStream_t>(hip_stream));
        return RTE_OK;
    });
}

rte_status rte_batch_usage(const rte_batch* b, int32_t* n_live, int32_t* n_done, size_t* used_bytes) {
    return guarded([&] {
        if (!b) rte::fail(RTE_E_ARG, "null batch");
        rte::batch_usage(reinterpret_cast<const rte::Batch*>(b), n_live, n_done, used_bytes);
        return RTE_OK;
    });
}

rte_status rte_batch_destroy(rte_batch* b) {
    return guarded([&] {
        rte::batch_destroy(reinterpret_cast<rte::Batch*>(b));
        return RTE_OK;
    });
}

rte_status rte_derived_outputs(rte_handle* hh, const double* U, double* phi, double* balance, void* hip_stream) {
    return guarded([&] {
        rte::Handle* h = as_handle(hh);
        if (!U) rte::fail(RTE_E_ARG, "null U_even");
        rte::derived_outputs(h, U, phi, balance, as_stream(hip_stream));
        return RTE_OK;
    });
}

rte_status rte_get_array(rte_handle* hh, int32_t which, void* host_dst, size_t host_bytes) {
    return guarded([&] {
        rte::Handle* h = as_handle(hh);
        if (!host_dst) rte::fail(RTE_E_ARG, "null destination");
        const void* src = nullptr;
        size_t bytes = 0;
        bool device = true;
        switch (which) {
            case 0: src = h->Sp.p; bytes = h->Sp.bytes(); break;
            case 1: src = h->Sm.p; bytes = h->Sm.bytes(); break;
            case 2: src = h->h_m.data(); bytes = h->h_m.size() * 8; device = false; break;
            case 3: src = h->h_T.data(); bytes = h->h_T.size() * 8; device = false; break;
            case 4: src = h->q.p; bytes = h->q.bytes(); break;
            case 5: src = h->h_lamp.data(); bytes = h->h_lamp.size() * 8; device = false; break;
            case 6: src = h->h_Wp.data(); bytes = h->h_Wp.size() * 8; device = false; break;
            case 7: src = h->h_lamm_full.data(); bytes = h->h_lamm_full.size() * 8; device = false; break;
            case 8:
                if (h->cg_iters.n < (size_t)h->nS) rte::fail(RTE_E_ARG, "no CG solve of E_0 has run");
                src = h->cg_iters.p;
                bytes = (size_t)h->nS * sizeof(int32_t);
                break;
            default: rte::fail(RTE_E_ARG, "unknown array id");
        }
        if (bytes != host_bytes) rte::fail(RTE_E_ARG, "host_bytes does not match the array size");
        if (device) {
            RTE_HIP(hipMemcpy(host_dst, src, bytes, hipMemcpyDeviceToHost));
        } else {
            std::memcpy(host_dst, src, bytes);
        }
        return RTE_OK;
    });
}

rte_status rte_destroy(rte_handle* hh) {
    return guarded([&] {
        (void)rte::take_free_error();
        delete reinterpret_cast<rte::Handle*>(hh);
        const hipError_t e = rte::take_free_error();
        if (e != hipSuccess)
            rte::fail(RTE_E_HIP, std::string("releasing the handle's device memory: hipFree failed: ") +
                                     hipGetErrorString(e));
        return RTE_OK;
    });
}

const char* rte_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace rte {
void apply_scatter(Handle* h, int parity, int dtin, const void* X, int dtout, void* Y, hipStream_t s) {
    if ((dtin != RTE_DT_F64 && dtin != RTE_DT_F32) || (dtout != RTE_DT_F64 && dtout != RTE_DT_F32))
        fail(RTE_E_ARG, "scatter operands are FP64 or FP32");
    const bool f32 = dtin == RTE_DT_F32;
    if (f32 && !(parity == 1 ? h->Sp_f.p : h->Sm_f.p))
        fail(RTE_E_ARG, "FP32 scatter operands need a handle assembled with mixed != 0");
    // the GEMM and the mass/diagonal epilogue run on FP64 intermediates in the handle's
    // workspace; an FP32 result is rounded at the end
    if (parity == 1) {
        const int n = h->nRp, m = h->nS;
        double* G = sv::ws(h, sv::W_EG);
        double* T = dtout == RTE_DT_F64 ? static_cast<double*>(Y) : sv::ws(h, sv::W_ET);
        // the odd workspace is scratch for the split last round of GEMM tiles, as in the solve
        double* scratch = sv::ws(h, sv::W_OZ);
        const size_t nscr = (size_t)h->nRm * h->nSm;
        if (f32)
            k::gemm_f32(n, m, m, 1.0f, static_cast<const float*>(X), n, h->Sp_f.p, m, 0.0f, G, n, s,
                        reinterpret_cast<float*>(scratch), 2 * nscr);
        else
            k::gemm_f64(n, m, m, 1.0, static_cast<const double*>(X), n, h->Sp.p, m, 0.0, G, n, s, scratch, nscr);
        k::spmm_pattern(h, h->Msv.p, G, T, s);
        if (dtout == RTE_DT_F32) k::cvt_f64_f32(T, static_cast<float*>(Y), (size_t)n * m, s);
    } else {
        const int n = h->nRm, m = h->nSm;
        double* T = dtout == RTE_DT_F64 ? static_cast<double*>(Y) : sv::ws(h, sv::W_OB);
        if (f32) k::gemm_f32(n, m, m, 1.0f, static_cast<const float*>(X), n, h->Sm_f.p, m, 0.0f, T, n, s);
        else k::gemm_f64(n, m, m, 1.0, static_cast<const double*>(X), n, h->Sm.p, m, 0.0, T, n, s);
        k::row_scale(h->ms.p, n, m, T, T, s);
        if (dtout == RTE_DT_F32) k::cvt_f64_f32(T, static_cast<float*>(Y), (size_t)n * m, s);
    }
}
}  // namespace rte
