// Autotuning of the banded E_0 factor layout: the band solve's shape (ring depth H, phase
// count P) fixes how many 16-byte groups a factor row block holds, so each candidate shape
// is its own layout.  Every shape that holds the band is timed on the device with the
// handle's own factors, re-laid out, and the fastest stays in place.  Padding groups are
// zero and the solve sums every row's products in the same order in every shape, so the
// choice changes the speed only, never the result.
#include <map>
#include <mutex>
#include <tuple>

#include "solver_detail.h"

namespace rte {
namespace {

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, int> g_tune_cache;   // (n, bw, nsys, element bytes) -> G

void solve_launch(const double* BL, const double* BU, int n, int bw, int nsys, size_t stride, const double* b,
                  double* x, int G, hipStream_t s) {
    k::band_solve_blk(BL, BU, n, bw, nsys, stride, b, x, (size_t)n, nullptr, s, G);
}
void solve_launch(const float* BL, const float* BU, int n, int bw, int nsys, size_t stride, const double* b,
                  double* x, int G, hipStream_t s) {
    k::band_solve_blk_f32(BL, BU, n, bw, nsys, stride, b, x, (size_t)n, nullptr, s, G);
}

// average time of one E_0^{-1} launch (all directions) in milliseconds, on a right-hand
// side of ones
template <typename FT>
double time_solve(Handle* h, const FT* BL, const FT* BU, size_t stride, int G, hipStream_t s) {
    constexpr int kReps = 3;
    const int n = h->nRp, bw = h->sbw, nsys = h->nS;
    double* b = sv::ws(h, sv::W_BB);
    double* x = sv::ws(h, sv::W_BX);
    k::fill(b, 1.0, (size_t)n * nsys, s);
    solve_launch(BL, BU, n, bw, nsys, stride, b, x, G, s);      // warm-up
    hipEvent_t e0, e1;
    RTE_HIP(hipEventCreate(&e0));
    RTE_HIP(hipEventCreate(&e1));
    float ms = 0.f;
    try {
        RTE_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < kReps; ++r) solve_launch(BL, BU, n, bw, nsys, stride, b, x, G, s);
        RTE_HIP(hipEventRecord(e1, s));
        RTE_HIP(hipEventSynchronize(e1));
        RTE_HIP(hipEventElapsedTime(&ms, e0, e1));
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    RTE_HIP(hipEventDestroy(e0));
    RTE_HIP(hipEventDestroy(e1));
    return ms / kReps;
}

// L/U (stride, G) -> the layout of G2 groups, in place of the old buffers
template <typename FT>
void relayout_into(Handle* h, DBuf<FT>& L, DBuf<FT>& U, size_t& stride, int& G, int G2, int vec, hipStream_t s) {
    const int n = h->nRp, bw = h->sbw, nsys = h->nS;
    const size_t stride2 = k::band_blk_size_g(n, G2, vec);
    DBuf<FT> L2(stride2 * nsys), U2(stride2 * nsys);
    k::band_relayout(L.p, G, L2.p, G2, n, bw, nsys, stride, stride2, s);
    k::band_relayout(U.p, G, U2.p, G2, n, bw, nsys, stride, stride2, s);
    RTE_HIP(hipStreamSynchronize(s));
    L = std::move(L2);
    U = std::move(U2);
    stride = stride2;
    G = G2;
}

template <typename FT>
void tune(Handle* h, DBuf<FT>& L, DBuf<FT>& U, size_t& stride, int& G, bool force, hipStream_t s, int idx,
          rte_tune_report* rep) {
    constexpr int vec = 16 / (int)sizeof(FT);
    const int n = h->nRp, bw = h->sbw, nsys = h->nS;
    const auto key = std::make_tuple(n, bw, nsys, (int)sizeof(FT));
    const k::BandShape d = k::band_shape(bw, vec);
    rep->default_H[idx] = d.H;
    rep->default_P[idx] = d.P;
    int target = -1;
    if (!force) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) target = it->second;
    }
    if (target > 0) {
        rep->from_cache[idx] = 1;
    } else {
        // the current layout first, then every other shape that holds the band
        double best_ms = time_solve(h, L.p, U.p, stride, G, s);
        int best = G;
        int nc = 0;
        const k::BandShape cur = k::band_shape_of_groups(G);
        rep->H[idx][nc] = cur.H;
        rep->P[idx][nc] = cur.P;
        rep->ms[idx][nc++] = best_ms;
        for (int c = 0; c < k::kBandShapes; ++c) {
            const k::BandShape sh = k::band_shape_at(c);
            const int Gc = sh.H * sh.P;
            if (Gc == G || !k::band_layout_ok(bw, vec, Gc)) continue;
            const size_t stride_c = k::band_blk_size_g(n, Gc, vec);
            double t;
            {
                DBuf<FT> Lc(stride_c * nsys), Uc(stride_c * nsys);
                k::band_relayout(L.p, G, Lc.p, Gc, n, bw, nsys, stride, stride_c, s);
                k::band_relayout(U.p, G, Uc.p, Gc, n, bw, nsys, stride, stride_c, s);
                t = time_solve(h, Lc.p, Uc.p, stride_c, Gc, s);
            }
            rep->H[idx][nc] = sh.H;
            rep->P[idx][nc] = sh.P;
            rep->ms[idx][nc++] = t;
            if (t < 0.99 * best_ms) {     // a clear gain only
                best_ms = t;
                best = Gc;
            }
        }
        rep->n_cand[idx] = nc;
        if (best != G) {
            // confirm against the current layout in alternating rounds (single timings of
            // a few milliseconds vary by a few per cent)
            const size_t stride_b = k::band_blk_size_g(n, best, vec);
            DBuf<FT> Lb(stride_b * nsys), Ub(stride_b * nsys);
            k::band_relayout(L.p, G, Lb.p, best, n, bw, nsys, stride, stride_b, s);
            k::band_relayout(U.p, G, Ub.p, best, n, bw, nsys, stride, stride_b, s);
            double t_cur = 0.0, t_best = 0.0;
            for (int round = 0; round < 3; ++round) {
                t_cur += time_solve(h, L.p, U.p, stride, G, s);
                t_best += time_solve(h, Lb.p, Ub.p, stride_b, best, s);
            }
            if (t_best < 0.99 * t_cur) {
                L = std::move(Lb);
                U = std::move(Ub);
                stride = stride_b;
                G = best;
            } else {
                best = G;
            }
        }
        target = best;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = target;
    }
    if (target != G) relayout_into(h, L, U, stride, G, target, vec, s);
    const k::BandShape ch = k::band_shape_of_groups(G);
    rep->chosen_H[idx] = ch.H;
    rep->chosen_P[idx] = ch.P;
}

}  // namespace

void set_band_layout(Handle* h, int precision, int H, int P, hipStream_t s) {
    if (!h->have_e0_banded) fail(RTE_E_ARG, "the handle has no banded E_0 factors");
    const int G = H * P;
    if (H <= 0 || P <= 0 || k::band_shape_of_groups(G).H != H) fail(RTE_E_ARG, "not a band solve shape");
    if (precision == RTE_FP64) {
        if (!h->L0.p) fail(RTE_E_ARG, "the FP64 band factors are absent");
        if (!k::band_layout_ok(h->sbw, 2, G)) fail(RTE_E_ARG, "the shape cannot hold the band");
        if (G != h->e0_g64) relayout_into(h, h->L0, h->L0U, h->e0_stride, h->e0_g64, G, 2, s);
    } else if (precision == RTE_MIXED) {
        if (!h->L0f.p) fail(RTE_E_ARG, "the FP32 band factors are absent");
        if (!k::band_layout_ok(h->sbw, 4, G)) fail(RTE_E_ARG, "the shape cannot hold the band");
        if (G != h->e0_g32) relayout_into(h, h->L0f, h->L0Uf, h->e0_stride32, h->e0_g32, G, 4, s);
    } else {
        fail(RTE_E_ARG, "unknown precision");
    }
}

void autotune(Handle* h, int flags, hipStream_t s, rte_tune_report* rep) {
    if (!h->have_e0_banded) fail(RTE_E_ARG, "the handle has no banded E_0 factors to tune");
    rte_tune_report r{};
    const bool force = (flags & RTE_TUNE_FORCE) != 0;
    if (h->L0.p) tune(h, h->L0, h->L0U, h->e0_stride, h->e0_g64, force, s, 0, &r);
    if (h->L0f.p) tune(h, h->L0f, h->L0Uf, h->e0_stride32, h->e0_g32, force, s, 1, &r);
    if (rep) *rep = r;
}

}  // namespace rte
