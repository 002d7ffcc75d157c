// Lockstep preconditioned Richardson iteration over several problem instances (the batched
// and served forms of Alg. 3).  Every live slot takes one outer step per batch iteration:
// - the residuals of all slots are formed, and ONE host synchronisation reads every slot's
//   residual norm and step products;
// - in each of the l steps of P_1 (Alg. 2), the E_0^{-1} applications of all slots with banded
//   factors are one grouped band-solve launch per band shape, so that the direction systems of
//   small instances fill the GPU together; slots whose E_0 is solved by CG (3D meshes, whose
//   bands are too wide to factor) run their all-direction CG one after another;
// - the remaining per-slot work (ApplyE, the subspace correction) of the slots is spread over
//   a few lanes (streams of the batch, joined to the step's stream by events), so that the
//   kernels of small instances run side by side and fill the GPU together; each slot's own
//   launches keep their order on one lane, so its arithmetic is unchanged.
// Slots may be admitted while others are running and leave as soon as they converge, which
// is what a continuous-batching server needs.  The arithmetic of a slot is the arithmetic of
// rte_solve with the same options, so a slot's result does not depend on the other slots.
#include <chrono>
#include <cmath>

#include "solver_detail.h"

namespace rte {

using namespace sv;

struct BatchSlot {
    Handle* h = nullptr;
    double* U = nullptr;
    rte_solve_opts o{};
    rte_solve_info info{};
    rte_status status = RTE_OK;
    bool used = false, live = false, done = false;
    int iters = 0;
    bool have_step = false;
    double e1 = -1.0, en_prev = -1.0;
    int stall = 0;
    size_t bytes = 0;
    std::chrono::steady_clock::time_point t0;
};

struct Batch {
    int max_slots = 0;
    size_t budget = 0, used_bytes = 0;
    int precision = -1;                 // of the slots (the grouped solve's factor type)
    int l = 0;                          // P_1 steps of the slots (they advance together)
    std::vector<BatchSlot> slots;
    // the grouped E_0 band solves, one plan per pair of vectors it maps (0: W_ER -> W_ES, the
    // first step of P_1; 1: W_ET2 -> W_EZ, the later ones): slots whose band order is the given
    // vertex order are solved in place of those vectors, the others through W_BB / W_BX and the
    // permutation passes
    k::BandGroupPlan plan[2];
    // the coarse band solves (one system each) of the slots whose handle solves E_c by band
    // factors, one grouped launch
    k::BandGroupPlan cplan;
    bool plan_valid = false;
    // graph mode (off unless asked for): the two launch sequences of an iteration (residuals;
    // preconditioner and update) are captured once per set of live slots and replayed, on the
    // batch's own stream
    bool use_graphs = false;
    hipStream_t gs = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraphExec_t g_res = nullptr, g_prec = nullptr;
    bool graphs_valid = false;
    // the stream the last batch work went to: a step returns with its last phase still
    // running there, and that phase reads the job table and the graphs
    hipStream_t last = nullptr;
    // lanes for the per-slot work (default-priority non-blocking streams), with the events
    // that fork them from the step's stream and join them back
    static constexpr int kLanes = 4;
    hipStream_t lane[kLanes] = {};
    hipEvent_t ev_fork = nullptr, ev_join[kLanes] = {};
    void ensure_lanes() {
        if (lane[0]) return;
        for (int l = 0; l < kLanes; ++l) {
            RTE_HIP(hipStreamCreateWithFlags(&lane[l], hipStreamNonBlocking));
            RTE_HIP(hipEventCreateWithFlags(&ev_join[l], hipEventDisableTiming));
        }
        RTE_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
    }
    // wait for the batch's work in flight (before its job table or graphs are replaced or freed)
    void drain() {
        if (last) RTE_HIP(hipStreamSynchronize(last));
        if (gs && gs != last) RTE_HIP(hipStreamSynchronize(gs));
        for (int l = 0; l < kLanes; ++l)
            if (lane[l]) RTE_HIP(hipStreamSynchronize(lane[l]));
    }
    ~Batch() {
        if (last) (void)hipStreamSynchronize(last);
        if (gs) (void)hipStreamSynchronize(gs);
        for (int l = 0; l < kLanes; ++l)
            if (lane[l]) {
                (void)hipStreamSynchronize(lane[l]);
                (void)hipStreamDestroy(lane[l]);
                (void)hipEventDestroy(ev_join[l]);
            }
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (g_res) (void)hipGraphExecDestroy(g_res);
        if (g_prec) (void)hipGraphExecDestroy(g_prec);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (gs) (void)hipStreamDestroy(gs);
    }
};

namespace {

// the workspace a batch slot uses (condensed or exact odd solve, banded E_0)
const int kSlotWs[] = {W_OB, W_OZ, W_OG, W_EG, W_ET, W_ER, W_ES, W_ESTEP, W_EZ, W_ET2, W_BB, W_BX, W_CRHS, W_CSOL};

size_t ws_bytes(const Handle* h, int id) {
    const size_t odd = (size_t)h->nRm * h->nSm, even = (size_t)h->nRp * h->nS;
    size_t n;
    if (id <= W_OG) n = odd;
    else if (id <= W_BX) n = even;
    else n = (size_t)h->nc;
    return n * sizeof(double);
}

size_t slot_bytes(Handle* h, const rte_solve_opts* o) {
    size_t b = h->footprint();
    if (h->ws.size() < W_COUNT) h->ws.resize(W_COUNT);
    for (int id : kSlotWs)
        if (!h->ws[id].p) b += ws_bytes(h, id);
    if (o->e0_solver != RTE_E0_BANDED)
        for (int id : {W_CGR, W_CGP, W_CGQ})
            if (!h->ws[id].p) b += ws_bytes(h, id);
    return b;
}

// f(slot, stream) for every live slot: slot j of the live ones on lane j mod kLanes, the lanes
// ordered after the earlier work of s and s's later work after all of them (a single live
// slot runs on s itself)
template <typename F>
void for_slots(Batch* B, hipStream_t s, F&& f) {
    int nlive = 0;
    for (auto& sl : B->slots) nlive += sl.live ? 1 : 0;
    if (nlive <= 1) {
        for (auto& sl : B->slots)
            if (sl.live) f(sl, s);
        return;
    }
    const int used = std::min(nlive, Batch::kLanes);
    RTE_HIP(hipEventRecord(B->ev_fork, s));
    for (int l = 0; l < used; ++l) RTE_HIP(hipStreamWaitEvent(B->lane[l], B->ev_fork, 0));
    int j = 0;
    for (auto& sl : B->slots)
        if (sl.live) f(sl, B->lane[j++ % used]);
    for (int l = 0; l < used; ++l) {
        RTE_HIP(hipEventRecord(B->ev_join[l], B->lane[l]));
        RTE_HIP(hipStreamWaitEvent(s, B->ev_join[l], 0));
    }
}

void rebuild_plan(Batch* B, hipStream_t s) {
    B->drain();      // the previous plan's job table may still be read by a launch in flight
    const bool f32 = B->precision == RTE_MIXED;
    for (int pi = 0; pi < 2; ++pi) {
        std::vector<k::BandJob> jobs;
        for (auto& sl : B->slots) {
            if (!sl.live || sl.o.e0_solver != RTE_E0_BANDED) continue;
            Handle* h = sl.h;
            k::BandJob j{};
            j.BL = f32 ? static_cast<const void*>(h->L0f.p) : static_cast<const void*>(h->L0.p);
            j.BU = f32 ? static_cast<const void*>(h->L0Uf.p) : static_cast<const void*>(h->L0U.p);
            j.b = h->perm_identity ? ws(h, pi == 0 ? W_ER : W_ET2) : ws(h, W_BB);
            j.x = h->perm_identity ? ws(h, pi == 0 ? W_ES : W_EZ) : ws(h, W_BX);
            j.stride_sys = f32 ? h->e0_stride32 : h->e0_stride;
            j.G = f32 ? h->e0_g32 : h->e0_g64;
            j.stride_vec = (size_t)h->nRp;
            j.n = h->nRp;
            j.bw = h->sbw;
            j.nsys = h->nS;
            jobs.push_back(j);
        }
        k::band_group_plan(jobs, f32, B->plan[pi], s);
    }
    std::vector<k::BandJob> cjobs;
    for (auto& sl : B->slots) {
        if (!sl.live) continue;
        Handle* h = sl.h;
        if (h->Ecinv.p || h->cnb || !h->Lc.p) continue;
        k::BandJob j{};
        j.BL = h->Lc.p;
        j.BU = h->LcU.p;
        j.b = ws(h, W_CRHS);
        j.x = ws(h, W_CSOL);
        j.stride_sys = 0;
        j.G = 0;
        j.stride_vec = (size_t)h->nc;
        j.n = h->nc;
        j.bw = h->cbw;
        j.nsys = 1;
        cjobs.push_back(j);
    }
    B->cplan = k::BandGroupPlan{};
    if (!cjobs.empty()) k::band_group_plan(cjobs, false, B->cplan, s);
    B->plan_valid = true;
}

// X -> Y = E_0^{-1} X for every live slot (x_of / y_of give the slot's vectors, which plan pi
// of the grouped band solve maps)
template <typename XF, typename YF>
void grouped_e0inv(Batch* B, int pi, XF x_of, YF y_of, hipStream_t s) {
    const bool lowp = B->precision == RTE_MIXED;
    for_slots(B, s, [&](BatchSlot& sl, hipStream_t ls) {
        if (sl.o.e0_solver == RTE_E0_BANDED && !sl.h->perm_identity)
            k::permute_cols(sl.h->iperm.p, sl.h->nRp, sl.h->nS, x_of(sl), ws(sl.h, W_BB), true, ls);
    });
    // the CG slots: several run in lockstep on the lanes, beside the grouped band solve on s
    // (each solve reads its live count on the host; one host wait per check for all of them)
    std::vector<BatchSlot*> cg;
    for (auto& sl : B->slots)
        if (sl.live && sl.o.e0_solver != RTE_E0_BANDED) cg.push_back(&sl);
    const int used = std::min((int)cg.size(), Batch::kLanes);
    if (cg.size() >= 2) {
        RTE_HIP(hipEventRecord(B->ev_fork, s));
        for (int l = 0; l < used; ++l) RTE_HIP(hipStreamWaitEvent(B->lane[l], B->ev_fork, 0));
    }
    k::band_group_run(B->plan[pi], s);
    if (cg.size() == 1) {
        e0inv(cg[0]->h, &cg[0]->o, x_of(*cg[0]), y_of(*cg[0]), s, nullptr, nullptr, lowp);
    } else if (cg.size() >= 2) {
        std::vector<k::CgJob> jobs;
        std::vector<k::MgArgs> mgs(cg.size());
        jobs.reserve(cg.size());
        for (size_t j = 0; j < cg.size(); ++j)
            jobs.push_back(
                cg_job(cg[j]->h, &cg[j]->o, x_of(*cg[j]), y_of(*cg[j]), lowp, B->lane[j % used], &mgs[j]));
        k::cg_solve_many(jobs);
        for (int l = 0; l < used; ++l) {
            RTE_HIP(hipEventRecord(B->ev_join[l], B->lane[l]));
            RTE_HIP(hipStreamWaitEvent(s, B->ev_join[l], 0));
        }
    }
    for_slots(B, s, [&](BatchSlot& sl, hipStream_t ls) {
        if (sl.o.e0_solver == RTE_E0_BANDED && !sl.h->perm_identity)
            k::permute_cols(sl.h->iperm.p, sl.h->nRp, sl.h->nS, ws(sl.h, W_BX), y_of(sl), false, ls);
    });
}

// residuals r_n = (E - K+) u_n - q (FP64) of every live slot and the scalars of its
// stopping tests (r.r in S_DOT0, step.r_n in S_DOT1; the latter is unused before a slot's
// first step)
void enqueue_residuals(Batch* B, hipStream_t s) {
    for_slots(B, s, [&](BatchSlot& sl, hipStream_t ls) {
        Handle* h = sl.h;
        const size_t n = (size_t)h->nRp * h->nS;
        double* r = ws(h, W_ER);
        residual_like(h, &sl.o, sl.U, h->q.p, r, sl.o.pcg_tol_resid, ls, nullptr, false);
        k::dot(r, r, n, h->red.p, ls);
        k::reduce(h->red.p, h->scal.p, S_DOT0, ls);
        k::dot(ws(h, W_ESTEP), r, n, h->red.p, ls);
        k::reduce(h->red.p, h->scal.p, S_DOT1, ls);
    });
}

// P_1^l (Alg. 2) with grouped E_0 solves, the subspace correction (Sec. 5.4), step.r_n into
// S_DOT2 and the update u_{n+1} = u_n + step, for every live slot
void enqueue_precond_update(Batch* B, hipStream_t s) {
    const bool lowp = B->precision == RTE_MIXED;
    grouped_e0inv(B, 0, [](BatchSlot& sl) { return (const double*)ws(sl.h, W_ER); },
                  [](BatchSlot& sl) { return ws(sl.h, W_ES); }, s);
    for (int i = 1; i < B->l; ++i) {
        // the previous step's update z -= E_0^{-1}(...) (none before the first) and this
        // step's E z - r, per slot on its lane
        for_slots(B, s, [&](BatchSlot& sl, hipStream_t ls) {
            if (i > 1) k::axpby(-1.0, ws(sl.h, W_EZ), 1.0, ws(sl.h, W_ES), (size_t)sl.h->nRp * sl.h->nS, ls);
            apply_E_core(sl.h, &sl.o, ws(sl.h, W_ES), nullptr, ws(sl.h, W_ER), ws(sl.h, W_ET2), sl.o.pcg_tol_inner,
                         ls, nullptr, lowp);
        });
        grouped_e0inv(B, 1, [](BatchSlot& sl) { return (const double*)ws(sl.h, W_ET2); },
                      [](BatchSlot& sl) { return ws(sl.h, W_EZ); }, s);
    }
    // the last step's update, then the subspace correction: right-hand sides and the coarse
    // solves by explicit inverses or block factorisations per slot, band factors in one
    // grouped launch, then the steps and updates
    for_slots(B, s, [&](BatchSlot& sl, hipStream_t ls) {
        if (B->l > 1) k::axpby(-1.0, ws(sl.h, W_EZ), 1.0, ws(sl.h, W_ES), (size_t)sl.h->nRp * sl.h->nS, ls);
        correction_rhs(sl.h, &sl.o, ws(sl.h, W_ER), ws(sl.h, W_ES), ls, nullptr, lowp);
        if (sl.h->Ecinv.p || sl.h->cnb) coarse_solve(sl.h, ls);
    });
    if (!B->cplan.launches.empty()) k::band_group_run(B->cplan, s);
    for_slots(B, s, [&](BatchSlot& sl, hipStream_t ls) {
        Handle* h = sl.h;
        const size_t n = (size_t)h->nRp * h->nS;
        double* r = ws(h, W_ER);
        double* step = ws(h, W_ESTEP);
        correction_finish(h, ws(h, W_ES), step, ls);
        k::dot(step, r, n, h->red.p, ls);
        k::reduce(h->red.p, h->scal.p, S_DOT2, ls);
        k::axpby(1.0, step, 1.0, sl.U, n, ls);
    });
}

template <typename F>
hipGraphExec_t capture(hipStream_t s, F&& enqueue) {
    std::unique_lock<std::shared_mutex> lk(capture_mutex());
    RTE_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
        enqueue();
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(s, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    hipGraph_t g = nullptr;
    RTE_HIP(hipStreamEndCapture(s, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    RTE_HIP(e);
    return ex;
}

void recapture(Batch* B) {
    for (auto& sl : B->slots)
        if (sl.live && sl.o.e0_solver != RTE_E0_BANDED)
            fail(RTE_E_ARG, "graph mode needs banded E_0 slots (a CG solve reads its live count on the host)");
    B->drain();
    if (B->g_res) { RTE_HIP(hipGraphExecDestroy(B->g_res)); B->g_res = nullptr; }
    if (B->g_prec) { RTE_HIP(hipGraphExecDestroy(B->g_prec)); B->g_prec = nullptr; }
    B->g_res = capture(B->gs, [&] { enqueue_residuals(B, B->gs); });
    B->g_prec = capture(B->gs, [&] { enqueue_precond_update(B, B->gs); });
    B->graphs_valid = true;
}

void finish(BatchSlot& sl, rte_status st) {
    sl.status = st;
    sl.live = false;
    sl.done = true;
    sl.info.iters = sl.iters;
    sl.info.t_solve = std::chrono::duration<double>(std::chrono::steady_clock::now() - sl.t0).count();
}

}  // namespace

Batch* batch_create(int max_slots, size_t budget) {
    if (max_slots < 1 || max_slots > 4096) fail(RTE_E_ARG, "max_slots must lie in 1..4096");
    Batch* B = new Batch;
    B->max_slots = max_slots;
    B->budget = budget;
    B->slots.resize(max_slots);
    return B;
}

void batch_destroy(Batch* B) { delete B; }

int batch_admit(Batch* B, Handle* h, const rte_solve_opts* o, const double* U0, double* U, hipStream_t s) {
    if (o->e0_solver == RTE_E0_BANDED && !h->have_e0_banded)
        fail(RTE_E_ARG, "a banded E_0 slot needs a handle assembled with e0_solver = RTE_E0_BANDED");
    if (o->e0_solver != RTE_E0_BANDED && o->e0_solver != RTE_E0_CG && o->e0_solver != RTE_E0_MG)
        fail(RTE_E_ARG, "unknown E_0 solver");
    if (o->e0_solver == RTE_E0_MG && !h->mg_m)
        fail(RTE_E_ARG, "a multigrid E_0 slot needs a handle assembled with e0_solver = RTE_E0_MG");
    if (o->e0_solver != RTE_E0_BANDED && B->use_graphs) fail(RTE_E_ARG, "graph mode needs banded E_0 slots");
    if (o->odd_solver == RTE_ODD_PCG) fail(RTE_E_ARG, "batch slots use the exact or condensed odd solve");
    if (o->inner != RTE_INNER_RICHARDSON) fail(RTE_E_ARG, "batch slots use the Richardson inner iteration");
    if (o->precision == RTE_MIXED && !(h->have_mixed && (h->L0f.p || o->e0_solver != RTE_E0_BANDED)))
        fail(RTE_E_ARG, "a mixed-precision slot needs a handle assembled with mixed != 0");
    if (o->precision == RTE_FP64 && o->e0_solver == RTE_E0_BANDED && !h->L0.p)
        fail(RTE_E_ARG, "an FP64 slot needs the FP64 band factors");
    bool any = false;
    for (auto& sl : B->slots) any |= sl.used;
    if (any && o->precision != B->precision) fail(RTE_E_ARG, "all slots of a batch share one precision");
    if (any && o->l != B->l) fail(RTE_E_ARG, "all slots of a batch share one l");
    for (auto& sl : B->slots)
        if (sl.used && sl.h == h) fail(RTE_E_ARG, "a handle can hold one slot at a time");
    int id = -1;
    for (int i = 0; i < B->max_slots; ++i)
        if (!B->slots[i].used) { id = i; break; }
    if (id < 0) fail(RTE_E_ARG, "no free batch slot");
    const size_t bytes = slot_bytes(h, o);
    if (B->budget && B->used_bytes + bytes > B->budget) fail(RTE_E_NOMEM, "the batch's device-memory budget is full");
    for (int wid : kSlotWs) ws(h, wid);
    if (o->e0_solver != RTE_E0_BANDED) {
        // the CG's block values and vectors (and the multigrid's data) now, so that stepping
        // allocates nothing
        cg_prepare(h, o->precision == RTE_MIXED, s);
        if (o->e0_solver == RTE_E0_MG) mg_prepare(h, o->precision == RTE_MIXED, s);
        for (int wid : {W_CGR, W_CGP, W_CGQ}) ws(h, wid);
    }
    B->precision = o->precision;
    B->l = o->l;
    BatchSlot& sl = B->slots[id];
    sl = BatchSlot{};
    sl.h = h;
    sl.U = U;
    sl.o = *o;
    sl.o.profile = 0;
    sl.used = sl.live = true;
    sl.bytes = bytes;
    sl.t0 = std::chrono::steady_clock::now();
    B->used_bytes += bytes;
    const size_t n = (size_t)h->nRp * h->nS;
    if (U0) k::copy(U0, U, n, s);
    else k::fill(U, 0.0, n, s);
    B->plan_valid = false;
    B->graphs_valid = false;
    return id;
}

int batch_step(Batch* B, int outer_iters, hipStream_t caller) {
    hipStream_t s = caller;
    if (B->use_graphs) {
        // a captured sequence needs a stream other than the null stream: run on the batch's
        // own stream, ordered after the caller's earlier work and before its later work
        if (!B->gs) {
            RTE_HIP(hipStreamCreateWithFlags(&B->gs, hipStreamNonBlocking));
            RTE_HIP(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming));
            RTE_HIP(hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming));
        }
        s = B->gs;
        RTE_HIP(hipEventRecord(B->ev_in, caller));
        RTE_HIP(hipStreamWaitEvent(s, B->ev_in, 0));
    }
    B->ensure_lanes();
    int nlive = 0;
    for (int it = 0; it < outer_iters; ++it) {
        nlive = 0;
        for (auto& sl : B->slots) nlive += sl.live ? 1 : 0;
        if (nlive == 0) break;
        if (!B->plan_valid) {
            rebuild_plan(B, s);
            B->graphs_valid = false;
        }
        if (B->use_graphs && !B->graphs_valid) recapture(B);
        // ---- residuals and the scalars of the stopping tests; one synchronisation
        if (B->use_graphs) RTE_HIP(hipGraphLaunch(B->g_res, s));
        else enqueue_residuals(B, s);
        for (auto& sl : B->slots)
            if (sl.live)
                RTE_HIP(hipMemcpyAsync(sl.h->pinned, sl.h->scal.p, 10 * sizeof(double), hipMemcpyDeviceToHost, s));
        RTE_HIP(hipStreamSynchronize(s));
        bool changed = false;
        for (auto& sl : B->slots) {
            if (!sl.live) continue;
            const double* hp = sl.h->pinned;
            const double rr = hp[S_DOT0];
            if (!std::isfinite(rr)) { finish(sl, RTE_E_NONFINITE); changed = true; continue; }
            sl.info.rel_resid = std::sqrt(rr) / sl.h->qnorm;
            double en = -1.0;
            if (sl.have_step) {
                // ||u_n - u_{n-1}||^2_{E-K} = step^T (r_n - r_{n-1}); step^T r_{n-1} was left in
                // S_DOT2 by the previous iteration
                en = std::sqrt(std::max(hp[S_DOT1] - hp[S_DOT2], 0.0));
                if (sl.e1 < 0) sl.e1 = en;
                sl.info.stop_quantity = sl.e1 > 0 ? en / sl.e1 : 0.0;
            }
            if (sl.info.rel_resid <= sl.o.tol) { finish(sl, RTE_OK); changed = true; }
            else if (sl.iters >= sl.o.max_iter) { finish(sl, RTE_E_NOTCONV); changed = true; }
            else if (stall_step(&sl.o, en, sl.en_prev, sl.stall)) { finish(sl, RTE_E_STALL); changed = true; }
        }
        if (changed) {
            rebuild_plan(B, s);
            B->graphs_valid = false;
        }
        nlive = 0;
        for (auto& sl : B->slots) nlive += sl.live ? 1 : 0;
        if (nlive == 0) break;
        if (B->use_graphs && !B->graphs_valid) recapture(B);
        // ---- P_1^l, the subspace correction and the update
        if (B->use_graphs) RTE_HIP(hipGraphLaunch(B->g_prec, s));
        else enqueue_precond_update(B, s);
        for (auto& sl : B->slots)
            if (sl.live) {
                ++sl.iters;
                sl.have_step = true;
            }
    }
    if (B->use_graphs) {
        RTE_HIP(hipEventRecord(B->ev_out, s));
        RTE_HIP(hipStreamWaitEvent(caller, B->ev_out, 0));
    }
    B->last = s;
    return nlive;
}

void batch_set_graphs(Batch* B, bool on) {
    B->use_graphs = on;
    B->graphs_valid = false;
}

int batch_poll(Batch* B, int max_out, int32_t* slots, rte_solve_info* infos, int32_t* statuses) {
    int n = 0;
    for (int i = 0; i < B->max_slots && n < max_out; ++i) {
        BatchSlot& sl = B->slots[i];
        if (!sl.used || !sl.done) continue;
        if (slots) slots[n] = i;
        if (infos) infos[n] = sl.info;
        if (statuses) statuses[n] = sl.status;
        B->used_bytes -= sl.bytes;
        sl = BatchSlot{};
        ++n;
    }
    return n;
}

void batch_usage(const Batch* B, int32_t* n_live, int32_t* n_done, size_t* used_bytes) {
    int live = 0, done = 0;
    for (auto& sl : B->slots) {
        live += sl.live ? 1 : 0;
        done += (sl.used && sl.done) ? 1 : 0;
    }
    if (n_live) *n_live = live;
    if (n_done) *n_done = done;
    if (used_bytes) *used_bytes = B->used_bytes;
}

}  // namespace rte
