// Autotuning of what changes the speed of a handle's kernels but not their results:
// - the banded E_0 factor layout: the band solve's shape (ring depth H, phase count P) fixes
//   how many 16-byte groups a factor row block holds, so each candidate shape is its own
//   layout.  Every shape that holds the band is timed on the device with the handle's own
//   factors, re-laid out, and the fastest stays in place.  Padding groups are zero and the
//   solve sums every row's products in the same order in every shape.
// - the tile map of each of the handle's GEMM shapes (the scatter GEMM U S+, the condensed
//   transport GEMM, in each precision present): the four combinations of the XCD swizzle of
//   the work-group ids and the traversal order of the tile grid, which reorder whole output
//   tiles only.
// The choices are kept per process and in a text file (RTE_TUNE_CACHE, else
// $HOME/.cache/rte/tune.txt; one choice per line, keyed by the device's architecture and
// compute-unit count), so that later processes take them without timing.
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <sys/stat.h>
#include <tuple>

#include "solver_detail.h"

namespace rte {
namespace {

typedef std::tuple<int, int, int, int> Key4;

struct TuneStore {
    std::mutex mu;
    bool loaded = false;
    std::string path, device;
    std::map<Key4, int> band;     // (n, bw, nsys, element bytes) -> groups per row block
    std::map<Key4, int> gemm;     // (kind, M, N, K) -> tile map
};

TuneStore& store() {
    static TuneStore t;
    return t;
}

// read the cache file once (call with the lock held); a missing or unreadable file is an
// empty cache
void load_locked(TuneStore& t) {
    if (t.loaded) return;
    t.loaded = true;
    int dev = 0;
    hipDeviceProp_t p{};
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
        t.device = std::string(p.gcnArchName) + ":" + std::to_string(p.multiProcessorCount);
    else
        t.device = "unknown";
    for (char& c : t.device)
        if (c == ' ') c = '_';
    if (const char* e = std::getenv("RTE_TUNE_CACHE")) {
        t.path = e;
    } else if (const char* home = std::getenv("HOME")) {
        const std::string dir = std::string(home) + "/.cache/rte";
        (void)mkdir((std::string(home) + "/.cache").c_str(), 0755);
        (void)mkdir(dir.c_str(), 0755);
        t.path = dir + "/tune.txt";
    }
    if (t.path.empty()) return;
    std::ifstream f(t.path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream in(line);
        std::string dv, what;
        int a = 0, b = 0, c = 0, d = 0, v = 0;
        if (!(in >> dv >> what >> a >> b >> c >> d >> v) || dv != t.device) continue;
        if (what == "band" && v > 0) t.band[Key4(a, b, c, d)] = v;
        else if (what == "gemm" && v >= 0 && v < 4) t.gemm[Key4(a, b, c, d)] = v;
    }
}

// record a choice in the file (call with the lock held); failures to write are ignored (the
// file only spares later processes the timing)
void append_locked(TuneStore& t, const char* what, const Key4& k, int v) {
    if (t.path.empty()) return;
    std::ofstream f(t.path, std::ios::app);
    if (!f) return;
    f << t.device << ' ' << what << ' ' << std::get<0>(k) << ' ' << std::get<1>(k) << ' ' << std::get<2>(k) << ' '
      << std::get<3>(k) << ' ' << v << '\n';
}

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
    TuneStore& ts = store();
    if (!force) {
        std::lock_guard<std::mutex> lk(ts.mu);
        load_locked(ts);
        auto it = ts.band.find(key);
        if (it != ts.band.end() && k::band_layout_ok(bw, vec, it->second)) target = it->second;
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
        std::lock_guard<std::mutex> lk(ts.mu);
        load_locked(ts);
        ts.band[key] = target;
        append_locked(ts, "band", key, target);
    }
    if (target != G) relayout_into(h, L, U, stride, G, target, vec, s);
    const k::BandShape ch = k::band_shape_of_groups(G);
    rep->chosen_H[idx] = ch.H;
    rep->chosen_P[idx] = ch.P;
}

// average milliseconds of run() over three launches after a warm-up
template <typename F>
double time_ms(F&& run, hipStream_t s) {
    run();
    hipEvent_t e0, e1;
    RTE_HIP(hipEventCreate(&e0));
    RTE_HIP(hipEventCreate(&e1));
    float ms = 0.f;
    try {
        RTE_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < 3; ++r) run();
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
    return ms / 3.0;
}

// time the four tile maps of one GEMM shape (run() launches it) and keep the fastest on a clear
// (1%) gain over map 0; from the cache unless forced
template <typename F>
void tune_gemm(int kind, int M, int N, int K, F&& run, bool force, hipStream_t s, rte_tune_report* rep) {
    const int i = rep->n_gemm;
    if (i >= 4) return;
    rep->n_gemm = i + 1;
    rep->gemm_kind[i] = kind;
    rep->gemm_m[i] = M;
    rep->gemm_n[i] = N;
    rep->gemm_k[i] = K;
    const Key4 key(kind, M, N, K);
    TuneStore& ts = store();
    {
        std::lock_guard<std::mutex> lk(ts.mu);
        load_locked(ts);
        auto it = ts.gemm.find(key);
        if (!force && it != ts.gemm.end()) {
            rep->gemm_map[i] = it->second;
            rep->gemm_from_cache[i] = 1;
            return;
        }
    }
    for (int m = 0; m < 4; ++m) {
        {
            std::lock_guard<std::mutex> lk(ts.mu);
            ts.gemm[key] = m;
        }
        rep->gemm_ms[i][m] = time_ms(run, s);
    }
    int best = 0;
    for (int m = 1; m < 4; ++m)
        if (rep->gemm_ms[i][m] < rep->gemm_ms[i][best]) best = m;
    if (rep->gemm_ms[i][best] >= 0.99 * rep->gemm_ms[i][0]) best = 0;
    std::lock_guard<std::mutex> lk(ts.mu);
    ts.gemm[key] = best;
    append_locked(ts, "gemm", key, best);
    rep->gemm_map[i] = best;
}

void tune_gemms(Handle* h, bool force, hipStream_t s, rte_tune_report* rep) {
    // operands from the handle's workspace (their values do not change the speed), with the
    // split-K scratch the solve gives the scatter GEMM
    double* X = sv::ws(h, sv::W_ET);
    double* Y = sv::ws(h, sv::W_EG);
    double* scratch = sv::ws(h, sv::W_OZ);
    const size_t nscratch = (size_t)h->nRm * h->nSm;
    const int nRp = h->nRp, nS = h->nS;
    k::fill(X, 1.0, (size_t)nRp * nS, s);
    tune_gemm(kGemmF64, nRp, nS, nS, [&] {
        k::gemm_f64(nRp, nS, nS, 1.0, X, nRp, h->Sp.p, nS, 0.0, Y, nRp, s, scratch, nscratch);
    }, force, s, rep);
    if (h->Sp_f.p)
        tune_gemm(kGemmF32, nRp, nS, nS, [&] {
            k::gemm_f32(nRp, nS, nS, 1.0f, X, nRp, h->Sp_f.p, nS, 0.0f, Y, nRp, s, reinterpret_cast<float*>(scratch),
                        2 * nscratch);
        }, force, s, rep);
    if (h->Gc.p) {
        const int dn = h->d * nS, nRm = h->nRm;
        double* B = sv::ws(h, sv::W_OB);
        double* Z = sv::ws(h, sv::W_OZ);
        k::fill(B, 1.0, (size_t)nRm * dn, s);
        tune_gemm(kGemmF64, dn, nRm, dn, [&] { k::gemm_f64(dn, nRm, dn, 1.0, h->Gc.p, dn, B, nRm, 0.0, Z, dn, s); },
                  force, s, rep);
        if (h->Gc_bf.p)
            tune_gemm(kGemmBF16, dn, nRm, dn, [&] {
                k::gemm_bf16(dn, nRm, dn, 1.0f, h->Gc_bf.p, dn, reinterpret_cast<const uint16_t*>(B), dn, 0.0f,
                             reinterpret_cast<float*>(Z), dn, s);
            }, force, s, rep);
    }
    RTE_HIP(hipStreamSynchronize(s));
}

}  // namespace

int gemm_map(int kind, int M, int N, int K) {
    TuneStore& ts = store();
    std::lock_guard<std::mutex> lk(ts.mu);
    if (ts.gemm.empty()) return 0;
    auto it = ts.gemm.find(Key4(kind, M, N, K));
    return it == ts.gemm.end() ? 0 : it->second;
}

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
    rte_tune_report r{};
    const bool force = (flags & RTE_TUNE_FORCE) != 0;
    if (h->L0.p) tune(h, h->L0, h->L0U, h->e0_stride, h->e0_g64, force, s, 0, &r);
    if (h->L0f.p) tune(h, h->L0f, h->L0Uf, h->e0_stride32, h->e0_g32, force, s, 1, &r);
    tune_gemms(h, force, s, &r);
    if (rep) *rep = r;
}

}  // namespace rte
