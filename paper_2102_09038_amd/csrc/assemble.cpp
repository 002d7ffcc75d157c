// rte_assemble: validation and assembly of every operator of the mixed even/odd
// discretisation (paper Sec. 4), the eigen-bases of the scattering matrices
// (Secs. 5.1, 5.4), the E_0 block data (Sec. 5.3) and the factored coarse matrix
// E_c = W^T (E - K+) W (Sec. 5.4).
//
// Host FP64 for the geometry (cheap, O(mesh size)); the O(n_S^2 Q^2) double quadrature
// of the HG kernel runs on the GPU (kernels_dense.hip); the symmetric eigensolves use
// rocSOLVER on the GPU.
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <deque>
#include <map>
#include <memory>
#include <numeric>
#include <thread>
#include <unordered_map>

#include "ops.h"
#include "rte_internal.h"
#include "solver_detail.h"

namespace rte {
namespace {

using Vec = std::vector<double>;

// ----------------------------------------------------------------------------- quadrature
// Radon's degree-5 7-point rule, composite over the 4^r congruent sub-triangles of each
// flat triangle, mapped radially onto the geodesic triangle with the surface element
// h / |x|^3 dA (h = distance of the flat plane from the origin).  The paper asks for
// "higher-order integration rules" on the projected sphere mesh (Sec. 6) without naming
// one; this is the rule both this library and its test oracle are defined by.
struct Rule {
    std::vector<std::array<double, 3>> bary;
    Vec w;
};

Rule composite_rule(int r) {
    const double r15 = std::sqrt(15.0);
    const double a = (6.0 - r15) / 21.0, b = (6.0 + r15) / 21.0;
    const double wa = (155.0 - r15) / 1200.0, wb = (155.0 + r15) / 1200.0;
    const double P[7][3] = {{1 / 3.0, 1 / 3.0, 1 / 3.0}, {a, a, 1 - 2 * a}, {a, 1 - 2 * a, a},
                            {1 - 2 * a, a, a},           {b, b, 1 - 2 * b}, {b, 1 - 2 * b, b},
                            {1 - 2 * b, b, b}};
    const double W[7] = {9.0 / 40.0, wa, wa, wa, wb, wb, wb};
    const int n = 1 << r;
    Rule R;
    auto add = [&](int p0, int q0, int p1, int q1, int p2, int q2) {
        const double c[3][3] = {{1.0 - (p0 + q0) / (double)n, p0 / (double)n, q0 / (double)n},
                                {1.0 - (p1 + q1) / (double)n, p1 / (double)n, q1 / (double)n},
                                {1.0 - (p2 + q2) / (double)n, p2 / (double)n, q2 / (double)n}};
        for (int i = 0; i < 7; ++i) {
            std::array<double, 3> x{};
            for (int v = 0; v < 3; ++v)
                for (int e = 0; e < 3; ++e) x[e] += P[i][v] * c[v][e];
            R.bary.push_back(x);
            R.w.push_back(W[i] / (double(n) * n));
        }
    };
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n - j; ++i) {
            add(i, j, i + 1, j, i, j + 1);
            if (i + j <= n - 2) add(i + 1, j, i + 1, j + 1, i, j + 1);
        }
    return R;
}

// ----------------------------------------------------------------------------- small dense
bool chol3(const double A[9], double L[9]) {
    std::fill(L, L + 9, 0.0);
    for (int j = 0; j < 3; ++j) {
        double s = A[3 * j + j];
        for (int k = 0; k < j; ++k) s -= L[3 * j + k] * L[3 * j + k];
        if (!(s > 0)) return false;
        L[3 * j + j] = std::sqrt(s);
        for (int i = j + 1; i < 3; ++i) {
            double t = A[3 * i + j];
            for (int k = 0; k < j; ++k) t -= L[3 * i + k] * L[3 * j + k];
            L[3 * i + j] = t / L[3 * j + j];
        }
    }
    return true;
}

void inv_lower3(const double L[9], double Li[9]) {
    std::fill(Li, Li + 9, 0.0);
    for (int j = 0; j < 3; ++j) {
        Li[3 * j + j] = 1.0 / L[3 * j + j];
        for (int i = j + 1; i < 3; ++i) {
            double s = 0;
            for (int k = j; k < i; ++k) s -= L[3 * i + k] * Li[3 * k + j];
            Li[3 * i + j] = s / L[3 * i + i];
        }
    }
}

bool inv3(const double A[9], double B[9]) {
    const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                       A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!(std::fabs(det) > 0)) return false;
    const double id = 1.0 / det;
    B[0] = (A[4] * A[8] - A[5] * A[7]) * id;
    B[1] = (A[2] * A[7] - A[1] * A[8]) * id;
    B[2] = (A[1] * A[5] - A[2] * A[4]) * id;
    B[3] = (A[5] * A[6] - A[3] * A[8]) * id;
    B[4] = (A[0] * A[8] - A[2] * A[6]) * id;
    B[5] = (A[2] * A[3] - A[0] * A[5]) * id;
    B[6] = (A[3] * A[7] - A[4] * A[6]) * id;
    B[7] = (A[1] * A[6] - A[0] * A[7]) * id;
    B[8] = (A[0] * A[4] - A[1] * A[3]) * id;
    return true;
}

// invert a d x d matrix (d <= 3), row-major; returns determinant
double invd(const double* J, double* Ji, int d) {
    if (d == 2) {
        const double det = J[0] * J[3] - J[1] * J[2];
        Ji[0] = J[3] / det; Ji[1] = -J[1] / det; Ji[2] = -J[2] / det; Ji[3] = J[0] / det;
        return det;
    }
    const double det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                       J[2] * (J[3] * J[7] - J[4] * J[6]);
    inv3(J, Ji);
    return det;
}

// f(k) for k in [0, n) over up to 16 host threads (contiguous ranges; f must touch disjoint
// data per k)
template <typename F>
void parallel_for(int n, F f) {
    const int nt = std::max(1, std::min<int>({16, (int)std::thread::hardware_concurrency(), n / 8}));
    if (nt == 1) {
        for (int k = 0; k < n; ++k) f(k);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            for (int k = (int)((long)n * t / nt); k < (int)((long)n * (t + 1) / nt); ++k) f(k);
        });
    for (auto& x : th) x.join();
}

// row-major lower band (band[r*(bw+1) + t], t = bw + c - r) -> blocked FP64 layout of
// kernels_band.hip (k::band_blk_index with 2 entries per group): rows of L (upper = false)
// or rows of L^T, at (r, t) = L(r+t, r) (upper = true)
Vec band_to_blocked(const Vec& band, int n, int bw, bool upper) {
    const size_t w1 = (size_t)bw + 1;
    Vec out(k::band_blk_size(n, bw, 2), 0.0);
    for (int r = 0; r < n; ++r)
        for (size_t t = 0; t < w1; ++t) {
            double v;
            if (!upper) v = band[(size_t)r * w1 + t];
            else v = (r + (int)t < n) ? band[(size_t)(r + t) * w1 + (w1 - 1 - t)] : 0.0;
            out[k::band_blk_index(r, (int)t, bw, 2)] = v;
        }
    return out;
}

// rocBLAS handle on the assembly stream; creation, destruction and every library call hold
// the capture lock shared
struct RocblasCtx {
    rocblas_handle h = nullptr;
    explicit RocblasCtx(hipStream_t s) {
        std::shared_lock<std::shared_mutex> lk(capture_mutex());
        if (rocblas_create_handle(&h) != rocblas_status_success) fail(RTE_E_HIP, "rocblas_create_handle failed");
        rocblas_set_stream(h, s);
    }
    ~RocblasCtx() {
        std::shared_lock<std::shared_mutex> lk(capture_mutex());
        if (h) rocblas_destroy_handle(h);
    }
};


// Inv = A^{-1} for the SPD matrix given by its lower band (row-major, band[r (bw+1) + bw + c - r]):
// dense Cholesky factorisation and inverse on the GPU, both triangles filled; what names the
// matrix in errors
void dense_spd_inverse(RocblasCtx& rb, hipStream_t s, const Vec& band, int n, int bw, DBuf<double>& Inv,
                       const char* what) {
    std::lock_guard<std::mutex> serial(solver_library_mutex());
    DBuf<double> dband;
    dband.upload(band, s);
    Inv.alloc((size_t)n * n);
    RTE_HIP(hipMemsetAsync(Inv.p, 0, (size_t)n * n * sizeof(double), s));
    k::band_to_dense(dband.p, n, bw, Inv.p, s);
    DBuf<int> info(1);
    int hinfo = 0;
    rocblas_status st;
    {
        std::shared_lock<std::shared_mutex> lk(capture_mutex());
        st = rocsolver_dpotrf(rb.h, rocblas_fill_lower, n, Inv.p, n, info.p);
    }
    if (st != rocblas_status_success) fail(RTE_E_HIP, "rocsolver_dpotrf failed");
    RTE_HIP(hipMemcpyAsync(&hinfo, info.p, sizeof(int), hipMemcpyDeviceToHost, s));
    RTE_HIP(hipStreamSynchronize(s));
    if (hinfo != 0) {
        // tell a matrix that arrived on the device intact from one that did not
        const Vec back = dband.download(s);
        size_t diff = 0;
        for (size_t e = 0; e < band.size(); ++e) diff += back[e] != band[e];
        fail(RTE_E_ARG, std::string(what) + " is not positive definite (Cholesky pivot " + std::to_string(hinfo) +
                            "; device copy of the input differs from the host matrix in " + std::to_string(diff) +
                            " of " + std::to_string(band.size()) + " entries)");
    }
    {
        std::shared_lock<std::shared_mutex> lk(capture_mutex());
        st = rocsolver_dpotri(rb.h, rocblas_fill_lower, n, Inv.p, n, info.p);
    }
    if (st != rocblas_status_success) fail(RTE_E_HIP, "rocsolver_dpotri failed");
    RTE_HIP(hipMemcpyAsync(&hinfo, info.p, sizeof(int), hipMemcpyDeviceToHost, s));
    RTE_HIP(hipStreamSynchronize(s));
    if (hinfo != 0) fail(RTE_E_HIP, std::string("rocsolver_dpotri failed on ") + what);
    k::symmetrize_lower(Inv.p, n, s);
    RTE_HIP(hipStreamSynchronize(s));
}

// eigenpairs of the symmetric n x n matrix A (col-major host); ascending eigenvalues
void syevd(RocblasCtx& rb, hipStream_t s, int n, Vec& A, Vec& lam) {
    std::lock_guard<std::mutex> serial(solver_library_mutex());
    DBuf<double> dA(A.size()), dD(n), dE(n);
    DBuf<int> info(1);
    RTE_HIP(hipMemcpyAsync(dA.p, A.data(), A.size() * 8, hipMemcpyHostToDevice, s));
    rocblas_status st;
    {
        std::shared_lock<std::shared_mutex> lk(capture_mutex());
        st = rocsolver_dsyevd(rb.h, rocblas_evect_original, rocblas_fill_lower, n, dA.p, n, dD.p, dE.p, info.p);
    }
    if (st != rocblas_status_success) fail(RTE_E_HIP, "rocsolver_dsyevd failed");
    int hinfo = 0;
    RTE_HIP(hipMemcpyAsync(&hinfo, info.p, sizeof(int), hipMemcpyDeviceToHost, s));
    lam.resize(n);
    RTE_HIP(hipMemcpyAsync(lam.data(), dD.p, n * 8, hipMemcpyDeviceToHost, s));
    RTE_HIP(hipMemcpyAsync(A.data(), dA.p, A.size() * 8, hipMemcpyDeviceToHost, s));
    RTE_HIP(hipStreamSynchronize(s));
    if (hinfo != 0) fail(RTE_E_HIP, "rocsolver_dsyevd did not converge");
}

// The dominant eigenpair of the symmetric n x n matrix A (col-major host) by power iteration on
// the device from v0, for a correction space of one mode (N+ = 0), where a full
// eigendecomposition is not needed.  The spectrum of the scaled S+ is the HG spectrum
// 1 > g^2 > ... (one per even degree, up to the quadrature defect) and v0 = M^{1/2} 1 is the
// discrete constant, already within the defect of the top eigenvector, so the iteration
// contracts by about g^2 per step from a small start.  Converged when the vector moves by at
// most 4e-16 (max norm) over 8 steps; false (the caller falls back to the full
// eigendecomposition) if that takes more than 4000 steps.
bool top_eigenpair(RocblasCtx& rb, hipStream_t s, int n, const Vec& A, const Vec& v0, Vec& v, double& lam) {
    DBuf<double> dA(A.size()), x(n), y(n);
    RTE_HIP(hipMemcpyAsync(dA.p, A.data(), A.size() * 8, hipMemcpyHostToDevice, s));
    RTE_HIP(hipMemcpyAsync(x.p, v0.data(), (size_t)n * 8, hipMemcpyHostToDevice, s));
    Vec prev(v0), cur(n);
    bool ok = false;
    {
        std::shared_lock<std::shared_mutex> lk(capture_mutex());
        const double one = 1.0, zero = 0.0;
        for (int it = 1; it <= 4000 && !ok; ++it) {
            if (rocblas_dgemv(rb.h, rocblas_operation_none, n, n, &one, dA.p, n, x.p, 1, &zero, y.p, 1) !=
                rocblas_status_success)
                fail(RTE_E_HIP, "rocblas_dgemv failed");
            double nrm = 0.0;
            if (rocblas_dnrm2(rb.h, n, y.p, 1, &nrm) != rocblas_status_success) fail(RTE_E_HIP, "rocblas_dnrm2 failed");
            if (!(nrm > 0.0) || !std::isfinite(nrm)) return false;
            const double inv = 1.0 / nrm;
            if (rocblas_dscal(rb.h, n, &inv, y.p, 1) != rocblas_status_success) fail(RTE_E_HIP, "rocblas_dscal failed");
            std::swap(x.p, y.p);
            if (it % 8 == 0) {
                RTE_HIP(hipMemcpyAsync(cur.data(), x.p, (size_t)n * 8, hipMemcpyDeviceToHost, s));
                RTE_HIP(hipStreamSynchronize(s));
                double d = 0.0;
                for (int i = 0; i < n; ++i) d = std::max(d, std::fabs(cur[i] - prev[i]));
                ok = d <= 4e-16;
                prev.swap(cur);
            }
        }
    }
    if (!ok) return false;
    v = prev;
    // Rayleigh quotient on the host, in a fixed order
    lam = 0.0;
    for (int j = 0; j < n; ++j) {
        double t = 0.0;
        for (int i = 0; i < n; ++i) t += A[i + (size_t)n * j] * v[i];
        lam += v[j] * t;
    }
    return true;
}

}  // namespace

Handle::~Handle() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (pinned) (void)hipHostFree(pinned);
    for (auto& r : prof) { evpool.push_back(r.a); evpool.push_back(r.b); }
    for (hipEvent_t e : evpool) (void)hipEventDestroy(e);
}

size_t Handle::footprint() const {
    size_t b = Sp.bytes() + Sm.bytes() + m.bytes() + T.bytes() + MSinv.bytes() + Wm.bytes() + lamm.bytes() +
               Wp.bytes() + Hodd.bytes() + Wfull.bytes() + WfullT.bytes() + lam_full.bytes() + cell.bytes() +
               Dc.bytes() + mt.bytes() + ms.bytes() + rowptr.bytes() + col.bytes() + Msv.bytes() + cls.bytes() +
               coefE0.bytes() + coefE.bytes() + diagE0.bytes() + vc_ptr.bytes() + vc_cell.bytes() + vc_loc.bytes() +
               q.bytes() + Lc.bytes() + LcU.bytes() + CLinv.bytes() + CLinvT.bytes() + CB.bytes() + CG.bytes() + cwork.bytes() + perm.bytes() + iperm.bytes() + L0.bytes() + L0U.bytes() + Ecinv.bytes() +
               Gc.bytes() + vcD.bytes() +
               MtMs.bytes() + bnd_row.bytes() + cg_iters.bytes() + ell_sptr.bytes() + ell_col.bytes() + ell_e.bytes() +
               ell_v64.bytes() + ell_dinv64.bytes() + ell_v32.bytes() + ell_dinv32.bytes() + cg_part.bytes() +
               cg_scal.bytes() + cg_state.bytes() +
               Sp_f.bytes() + Sm_f.bytes() + Gc_bf.bytes() + coefD.bytes() + L0f.bytes() + L0Uf.bytes() + red.bytes() +
               scal.bytes();
    for (auto& w : ws) b += w.bytes();
    for (auto& l : mgl) b += l.bytes();
    return b;
}

namespace {

// Phase timing of the assembly, printed to stderr when the environment sets RTE_TRACE
// (each phase is closed with a stream synchronisation so that GPU work is attributed to it).
struct PhaseTrace {
    bool on = std::getenv("RTE_TRACE") != nullptr;
    hipStream_t s;
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    explicit PhaseTrace(hipStream_t s_) : s(s_) {}
    void operator()(const char* name) {
        if (!on) return;
        (void)hipStreamSynchronize(s);
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[rte assemble] %-28s %9.3f s\n", name, std::chrono::duration<double>(now - t).count());
        t = now;
    }
};

// A boundary facet: its vertices (d of them, sorted), the cell it closes and that cell's
// vertex opposite it.
struct Facet {
    std::array<int, 3> v;
    int cell, opp;
};

// The state of one assembly, shared by its phases: the problem, the handle being filled and
// the host-side intermediates that later phases read.  assemble() runs the phases in order.
struct Asm {
    const rte_problem_desc* D;
    const rte_assemble_opts* o;
    hipStream_t s;
    Handle& h;
    PhaseTrace trace;
    std::unique_ptr<RocblasCtx> rb;            // from the eigen-bases on
    double cmax = 0;                           // max sigma_s / sigma_t
    int d = 0, nv = 0, nRp = 0, nRm = 0;       // dimension, vertices per cell, P1 / P0 unknowns
    int nS = 0, nSm = 0, Q = 0;                // directions, odd unknowns per cell, points per direction
    std::vector<int> upper;                    // sphere triangle of each upper-half direction
    Vec pts, wts;                              // quadrature points (unit vectors) and weights
    Vec MSinv, LkInv;                          // inverses of the blocks 2 T_k and of their Cholesky factors
    Vec vol, Dc, mt, ms;                       // cell volumes, |K| grad(lambda), sigma_t |K|, sigma_s |K|
    std::vector<int> rp, ci, diagpos;          // P1 pattern (CSR, sorted rows) and its diagonal entries
    int nnz = 0;
    std::vector<Facet> facets;                 // boundary facets
    std::vector<std::array<double, 3>> ncls_dir;   // distinct boundary normals (up to sign)
    std::vector<int> fcls;                     // normal class of each facet
    Vec fmeas;                                 // facet measures
    int nb = 0, nstiff = 0;                    // boundary normal classes, stiffness classes
    std::vector<std::pair<int, int>> nm;       // (n, m) of each stiffness class, n <= m
    Vec cls, Msv, M1v;                         // class values on the pattern; sigma_s and unit mass matrices
    Vec omega, coefE0, coefE, diagE0;          // omega_k(nu_c); per-direction class coefficients; diag E_0
    std::vector<int> vcp, vcc, vcl;            // vertex -> incident (cell, local vertex index)
    Vec qv;                                    // the source l+ (nRp x nS)
    bool odd_eig = false;                      // the odd eigenbasis is computed
    Vec Wfull;                                 // host full odd eigenbasis (odd_eig only)
    Vec Hh;                                    // host H = (M_S- - delta S-)^{-1} (uniform delta only)

    Asm(const rte_problem_desc* D_, const rte_assemble_opts* o_, hipStream_t s_, Handle& h_)
        : D(D_), o(o_), s(s_), h(h_), trace(s_) {}

    // position of the entry (i, jv) in the pattern
    int find(int i, int jv) const {
        const int* b = ci.data() + rp[i];
        const int* e = ci.data() + rp[i + 1];
        return (int)(std::lower_bound(b, e, jv) - ci.data());
    }

    void init();
    void sphere();
    void quadrature();
    void geometry();
    void pattern();
    void boundary();
    void classes();
    void incidence_and_source();
    void upload();
    void scattering();
    void odd_basis();
    void condensed_from_H();
    Vec whitened_odd_scatter() const;
    void odd_eigenbasis();
    void odd_inverse();
    void even_basis();
    void coarse();
    void e0_data();
    void mg_hierarchy();
    void reduced_precision();
};

// validation (host.cpp) and the handle's sizes
void Asm::init() {
    cmax = validate_problem(D, o);
    d = D->dim;
    nv = d + 1;
    nRp = D->n_vert;
    nRm = D->n_cell;
    h.stream = s;
    h.d = d; h.nRp = nRp; h.nRm = nRm; h.g = D->g; h.c = cmax;
    h.n_even = o->n_even; h.n_odd = o->n_odd;
    h.dNp = (o->n_even + 1) * (o->n_even + 2) / 2;
    h.dNm = (o->n_odd + 1) * (o->n_odd + 2) / 2;
}

// sphere: the upper half of the directions, paired with their antipodes (host.cpp)
void Asm::sphere() {
    upper = pair_sphere(D);
    nS = (int)upper.size();
    h.nS = nS;
    h.nSm = nSm = 3 * nS;
    if (h.dNm > h.nSm || h.dNp > nS) fail(RTE_E_ARG, "eigen-basis larger than the angular space");
}

// angular quadrature: points and weights of every direction, the moments m_k and T_k, and the
// inverses of the 3x3 blocks 2 T_k of M_S- and of their Cholesky factors
void Asm::quadrature() {
    const Rule R = composite_rule(o->quad_level);
    Q = (int)R.w.size();
    pts.assign((size_t)nS * Q * 3, 0.0);
    wts.assign((size_t)nS * Q, 0.0);
    h.h_m.assign(nS, 0.0);
    h.h_T.assign((size_t)nS * 9, 0.0);
    for (int k = 0; k < nS; ++k) {
        const int* t = D->stri + 3 * upper[k];
        const double* a = D->svert + 3 * t[0];
        const double* b = D->svert + 3 * t[1];
        const double* c = D->svert + 3 * t[2];
        const double det = std::fabs(a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
                                     a[2] * (b[0] * c[1] - b[1] * c[0]));
        if (!(det > 0)) fail(RTE_E_MESH, "degenerate sphere triangle");
        for (int p = 0; p < Q; ++p) {
            double x[3];
            for (int e = 0; e < 3; ++e) x[e] = R.bary[p][0] * a[e] + R.bary[p][1] * b[e] + R.bary[p][2] * c[e];
            const double nx = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
            const double w = R.w[p] * det / (2.0 * nx * nx * nx);
            const size_t o3 = ((size_t)k * Q + p) * 3;
            for (int e = 0; e < 3; ++e) pts[o3 + e] = x[e] / nx;
            wts[(size_t)k * Q + p] = w;
            h.h_m[k] += 2.0 * w;
            for (int e = 0; e < 3; ++e)
                for (int f = 0; f < 3; ++f) h.h_T[9 * k + 3 * e + f] += w * pts[o3 + e] * pts[o3 + f];
        }
    }
    // inverse of the 3x3 blocks 2 T_k of M_S-
    MSinv.assign((size_t)nS * 9, 0.0);
    LkInv.assign((size_t)nS * 9, 0.0);
    for (int k = 0; k < nS; ++k) {
        double B[9], L[9];
        for (int e = 0; e < 9; ++e) B[e] = 2.0 * h.h_T[9 * k + e];
        if (!inv3(B, &MSinv[9 * k]) || !chol3(B, L)) fail(RTE_E_MESH, "singular odd mass block");
        inv_lower3(L, &LkInv[9 * k]);
    }
}

// spatial geometry: cell volumes, scaled barycentric gradients, the sigma_t and sigma_s cell
// masses, and whether sigma_s / sigma_t is uniform
void Asm::geometry() {
    vol.assign(nRm, 0.0);
    Dc.assign((size_t)nRm * nv * d, 0.0);
    for (int j = 0; j < nRm; ++j) {
        const int* cj = D->cell + nv * j;
        double J[9], Ji[9];
        for (int r = 0; r < d; ++r)          // J[r][e] = x_{e+1,r} - x_{0,r}  (columns = edges)
            for (int e = 0; e < d; ++e) J[r * d + e] = D->vert[d * cj[e + 1] + r] - D->vert[d * cj[0] + r];
        const double det = invd(J, Ji, d);
        const double v = std::fabs(det) / (d == 2 ? 2.0 : 6.0);
        if (!(v > 0) || !std::isfinite(det)) fail(RTE_E_MESH, "degenerate spatial cell " + std::to_string(j));
        vol[j] = v;
        // grad lambda_{e+1} = row e of J^{-1}; grad lambda_0 = -sum
        for (int n = 0; n < d; ++n) {
            double s0 = 0;
            for (int e = 0; e < d; ++e) {
                const double gv = Ji[e * d + n];
                Dc[((size_t)j * nv + e + 1) * d + n] = v * gv;
                s0 += gv;
            }
            Dc[((size_t)j * nv) * d + n] = -v * s0;
        }
    }
    mt.assign(nRm, 0.0);
    ms.assign(nRm, 0.0);
    for (int j = 0; j < nRm; ++j) { mt[j] = D->sigma_t[j] * vol[j]; ms[j] = D->sigma_s[j] * vol[j]; }
    // the ratio sigma_s / sigma_t counts as uniform when every cell's ratio agrees to a few
    // ulps (sigma_s = 0.99 sigma_t rounds differently cell by cell); the single inverse then
    // uses the mean ratio, a relative perturbation of the odd operator below 1e-13
    h.uniform_delta = true;
    {
        double lo = 1e300, hi = -1e300, sum = 0;
        for (int j = 0; j < nRm; ++j) {
            const double r = D->sigma_s[j] / D->sigma_t[j];
            lo = std::min(lo, r); hi = std::max(hi, r); sum += r;
        }
        h.delta0 = sum / nRm;
        if (hi - lo > 1e-13 * std::max(hi, 1e-300)) h.uniform_delta = false;
    }
}

// the P1 pattern (host.cpp) and its diagonal entries
void Asm::pattern() {
    p1_pattern(D, rp, ci);
    nnz = rp[nRp];
    h.nnz = nnz;
    diagpos.assign(nRp, 0);
    for (int i = 0; i < nRp; ++i) diagpos[i] = find(i, i);
}

// boundary facets, their measures and their normal classes
void Asm::boundary() {
    std::map<std::array<int, 3>, std::pair<int, int>> owner;   // sorted verts -> (count, cell*8+opp)
    for (int j = 0; j < nRm; ++j)
        for (int o_ = 0; o_ < nv; ++o_) {
            std::array<int, 3> f{-1, -1, -1};
            int c = 0;
            for (int a = 0; a < nv; ++a)
                if (a != o_) f[c++] = D->cell[nv * j + a];
            std::sort(f.begin(), f.begin() + d);
            auto it = owner.find(f);
            if (it == owner.end()) owner[f] = {1, j * 8 + o_};
            else it->second.first++;
        }
    for (auto& kv : owner)
        if (kv.second.first == 1) facets.push_back({kv.first, kv.second.second / 8, kv.second.second % 8});
    // normals, measures, normal classes (normals equal up to sign share omega)
    fcls.assign(facets.size(), 0);
    fmeas.assign(facets.size(), 0.0);
    for (size_t f = 0; f < facets.size(); ++f) {
        const int j = facets[f].cell, op = facets[f].opp;
        double g3[3] = {0, 0, 0}, gn = 0;
        for (int n = 0; n < d; ++n) { g3[n] = Dc[((size_t)j * nv + op) * d + n] / vol[j]; gn += g3[n] * g3[n]; }
        gn = std::sqrt(gn);
        std::array<double, 3> nu{-g3[0] / gn, -g3[1] / gn, -g3[2] / gn};
        fmeas[f] = d * vol[j] * gn;
        // canonical sign: first component with |x| > 1e-12 positive
        for (int e = 0; e < 3; ++e)
            if (std::fabs(nu[e]) > 1e-12) {
                if (nu[e] < 0) for (auto& x : nu) x = -x;
                break;
            }
        int cid = -1;
        for (size_t c = 0; c < ncls_dir.size(); ++c)
            if (std::fabs(ncls_dir[c][0] - nu[0]) < 1e-12 && std::fabs(ncls_dir[c][1] - nu[1]) < 1e-12 &&
                std::fabs(ncls_dir[c][2] - nu[2]) < 1e-12) { cid = (int)c; break; }
        if (cid < 0) { cid = (int)ncls_dir.size(); ncls_dir.push_back(nu); }
        fcls[f] = cid;
    }
    nb = (int)ncls_dir.size();
    nstiff = d * (d + 1) / 2;
    h.ncls_stiff = nstiff;
    h.nbcls = nb;
    h.ncls = nstiff + 1 + nb;
    if (h.ncls > kMaxClasses)
        fail(RTE_E_ARG, "boundary has too many distinct facet normals (" + std::to_string(nb) +
                            "); at most " + std::to_string(kMaxClasses - nstiff - 1) + " are supported");
}

// value classes of the pattern, omega_k of each boundary normal class, and the per-direction
// class coefficients of E_0 and of M+ + R with the diagonal of every E_0 block
void Asm::classes() {
    // stiffness classes (n <= m): sum_j D_n(j,a) D_m(j,b) / mt_j (+ the (m,n) term when n < m)
    const int ncls = h.ncls;
    cls.assign((size_t)ncls * nnz, 0.0);
    Msv.assign(nnz, 0.0);
    M1v.assign(nnz, 0.0);
    for (int n = 0; n < d; ++n) nm.push_back({n, n});
    for (int n = 0; n < d; ++n)
        for (int m = n + 1; m < d; ++m) nm.push_back({n, m});
    const double mloc_d = 1.0 / ((d + 1) * (d + 2));
    for (int j = 0; j < nRm; ++j) {
        const int* cj = D->cell + nv * j;
        for (int a = 0; a < nv; ++a)
            for (int b = 0; b < nv; ++b) {
                const int e = find(cj[a], cj[b]);
                const double* Da = &Dc[((size_t)j * nv + a) * d];
                const double* Db = &Dc[((size_t)j * nv + b) * d];
                for (int c = 0; c < nstiff; ++c) {
                    const int n = nm[c].first, m = nm[c].second;
                    double v = Da[n] * Db[m];
                    if (n != m) v += Da[m] * Db[n];
                    cls[(size_t)c * nnz + e] += v / mt[j];
                }
                const double loc = (a == b ? 2.0 : 1.0) * mloc_d * vol[j];
                cls[(size_t)nstiff * nnz + e] += D->sigma_t[j] * loc;
                Msv[e] += D->sigma_s[j] * loc;
                M1v[e] += loc;
            }
    }
    const double floc = 1.0 / (d * (d + 1));
    for (size_t f = 0; f < facets.size(); ++f) {
        const int c = nstiff + 1 + fcls[f];
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) {
                const int e = find(facets[f].v[a], facets[f].v[b]);
                cls[(size_t)c * nnz + e] += (a == b ? 2.0 : 1.0) * floc * fmeas[f];
            }
    }
    // omega_k(nu_c) = 2 sum_p w_p |s_p . nu_c|
    omega.assign((size_t)nb * nS, 0.0);
    for (int c = 0; c < nb; ++c)
        for (int k = 0; k < nS; ++k) {
            double acc = 0;
            for (int p = 0; p < Q; ++p) {
                const double* sp = &pts[((size_t)k * Q + p) * 3];
                acc += wts[(size_t)k * Q + p] *
                       std::fabs(sp[0] * ncls_dir[c][0] + sp[1] * ncls_dir[c][1] + sp[2] * ncls_dir[c][2]);
            }
            omega[(size_t)c * nS + k] = 2.0 * acc;
        }
    // per-direction coefficients: E_0 block k and (M+ + R) block k
    const double alpha = 2.0 / (1.0 - cmax * D->g);
    coefE0.assign((size_t)nS * ncls, 0.0);
    coefE.assign((size_t)nS * ncls, 0.0);
    diagE0.assign((size_t)nRp * nS, 0.0);
    for (int k = 0; k < nS; ++k) {
        for (int c = 0; c < nstiff; ++c)
            coefE0[(size_t)k * ncls + c] = alpha * h.h_T[9 * k + 3 * nm[c].first + nm[c].second];
        coefE0[(size_t)k * ncls + nstiff] = coefE[(size_t)k * ncls + nstiff] = h.h_m[k];
        for (int c = 0; c < nb; ++c)
            coefE0[(size_t)k * ncls + nstiff + 1 + c] = coefE[(size_t)k * ncls + nstiff + 1 + c] =
                omega[(size_t)c * nS + k];
    }
    {   // the diagonal of every E_0 block (Jacobi), directions split over host threads
        Vec cd((size_t)ncls * nRp);
        for (int c = 0; c < ncls; ++c)
            for (int i = 0; i < nRp; ++i) cd[(size_t)c * nRp + i] = cls[(size_t)c * nnz + diagpos[i]];
        parallel_for(nS, [&](int k) {
            for (int i = 0; i < nRp; ++i) {
                double v = 0;
                for (int c = 0; c < ncls; ++c) v += coefE0[(size_t)k * ncls + c] * cd[(size_t)c * nRp + i];
                diagE0[i + (size_t)nRp * k] = v;
            }
        });
    }
}

// vertex -> incident cells, and the source l+ with its norm
void Asm::incidence_and_source() {
    vcp.assign(nRp + 1, 0);
    vcc.assign((size_t)nRm * nv, 0);
    vcl.assign((size_t)nRm * nv, 0);
    for (int j = 0; j < nRm; ++j)
        for (int a = 0; a < nv; ++a) vcp[D->cell[nv * j + a] + 1]++;
    for (int i = 0; i < nRp; ++i) vcp[i + 1] += vcp[i];
    {
        std::vector<int> fillp(vcp.begin(), vcp.end() - 1);
        for (int j = 0; j < nRm; ++j)
            for (int a = 0; a < nv; ++a) {
                const int v = D->cell[nv * j + a];
                vcc[fillp[v]] = j;
                vcl[fillp[v]++] = a;
            }
    }
    // source l+[:,k] = m_k (M1 q_nodal)
    Vec Mq(nRp, 0.0);
    for (int i = 0; i < nRp; ++i)
        for (int e = rp[i]; e < rp[i + 1]; ++e) Mq[i] += M1v[e] * D->q_nodal[ci[e]];
    qv.assign((size_t)nRp * nS, 0.0);
    Vec qk2(nS);
    parallel_for(nS, [&](int k) {
        double a = 0;
        for (int i = 0; i < nRp; ++i) {
            const double v = h.h_m[k] * Mq[i];
            qv[i + (size_t)nRp * k] = v;
            a += v * v;
        }
        qk2[k] = a;
    });
    double qn2 = 0;
    for (int k = 0; k < nS; ++k) qn2 += qk2[k];   // fixed order
    h.qnorm = std::sqrt(qn2);
}

// uploads of the mesh, pattern and class data, and the sliced-ELL layout of the E_0 blocks
void Asm::upload() {
    h.m.upload(h.h_m, s);
    h.T.upload(h.h_T, s);
    h.MSinv.upload(MSinv, s);
    h.cell.upload(std::vector<int>(D->cell, D->cell + (size_t)nRm * nv), s);
    h.Dc.upload(Dc, s);
    h.mt.upload(mt, s);
    h.ms.upload(ms, s);
    h.rowptr.upload(rp, s);
    h.col.upload(ci, s);
    {
        std::vector<int> sptr, ecol, epos;
        h.ell_len = sliced_ell(nRp, rp, ci, &sptr, &ecol, &epos);
        h.ell_nslice = (nRp + 63) / 64;
        for (int sl = 0; sl < h.ell_nslice; ++sl) h.ell_wmax = std::max(h.ell_wmax, sptr[sl + 1] - sptr[sl]);
        h.ell_sptr.upload(sptr, s);
        h.ell_col.upload(ecol, s);
        h.ell_e.upload(epos, s);
    }
    h.Msv.upload(Msv, s);
    h.cls.upload(cls, s);
    h.coefE0.upload(coefE0, s);
    h.coefE.upload(coefE, s);
    h.diagE0.upload(diagE0, s);
    h.vc_ptr.upload(vcp, s);
    h.vc_cell.upload(vcc, s);
    h.vc_loc.upload(vcl, s);
    {   // per-incidence gradient coefficients, interleaved mass values, boundary-row flags
        Vec vd(vcc.size() * (size_t)d);
        for (size_t e = 0; e < vcc.size(); ++e)
            for (int n = 0; n < d; ++n) vd[e * d + n] = Dc[((size_t)vcc[e] * nv + vcl[e]) * d + n];
        h.vcD.upload(vd, s);
        Vec mm(2 * (size_t)nnz);
        for (int e = 0; e < nnz; ++e) {
            mm[2 * (size_t)e] = cls[(size_t)nstiff * nnz + e];
            mm[2 * (size_t)e + 1] = Msv[e];
        }
        h.MtMs.upload(mm, s);
        std::vector<int> br(nRp, 0);
        for (int i = 0; i < nRp; ++i)
            for (int e = rp[i]; e < rp[i + 1]; ++e)
                for (int c = 0; c < nb; ++c)
                    if (cls[(size_t)(nstiff + 1 + c) * nnz + e] != 0.0) br[i] = 1;
        h.bnd_row.upload(br, s);
    }
    h.q.upload(qv, s);
}

// scattering matrices S+ and S- (quadrature of the HG kernel on the GPU)
void Asm::scattering() {
    {
        DBuf<double> dp, dw;
        dp.upload(pts, s);
        dw.upload(wts, s);
        h.Sp.alloc((size_t)nS * nS);
        h.Sm.alloc((size_t)h.nSm * h.nSm);
        k::hg_scatter(dp.p, dw.p, nS, Q, D->g, h.Sp.p, h.Sm.p, s);
        RTE_HIP(hipStreamSynchronize(s));
    }
    h.h_Sp = h.Sp.download(s);
    h.h_Sm = h.Sm.download(s);
}

// eigen-bases (rocSOLVER), odd part
void Asm::odd_basis() {
    // The odd eigendecomposition of (S-, M_S-) serves the PCG preconditioner (its top pairs),
    // the exact odd inverse for a per-cell ratio (all pairs) and the transport term of E_c.
    // With a uniform ratio delta and opts->odd_eig == 0 it is skipped: the exact and condensed
    // forms only need H = (M_S- - delta S-)^{-1}, which a dense Cholesky inverse on the GPU gives
    // directly, and the E_c term is (A_n W+)^T H (A_m W+).
    odd_eig = o->odd_eig != 0 || !h.uniform_delta;
    h.have_odd_eig = odd_eig;
    if (odd_eig) odd_eigenbasis();
    else odd_inverse();
}

// condensed transport matrix G from H: block (n, n') = A_n^T H A_n', i.e.
// G[(n,k),(n',k')] = sum_{m,m'} 2 T_k(n,m) H[3k+m, 3k'+m'] 2 T_k'(n',m'), and its diagonal
// blocks as stiffness-class coefficients
void Asm::condensed_from_H() {
    const int dn = d * nS;
    Vec G((size_t)dn * dn);
    // the columns of direction k2 per task (host threads; every entry is computed alone)
    parallel_for(nS, [&](int k2) {
        for (int k1 = 0; k1 < nS; ++k1) {
            double Hb[9];
            for (int m = 0; m < 3; ++m)
                for (int m2 = 0; m2 < 3; ++m2) Hb[3 * m + m2] = Hh[(3 * k1 + m) + (size_t)nSm * (3 * k2 + m2)];
            for (int n = 0; n < d; ++n)
                for (int n2 = 0; n2 < d; ++n2) {
                    double v = 0;
                    for (int m = 0; m < 3; ++m)
                        for (int m2 = 0; m2 < 3; ++m2)
                            v += 2.0 * h.h_T[9 * k1 + 3 * n + m] * Hb[3 * m + m2] * 2.0 * h.h_T[9 * k2 + 3 * n2 + m2];
                    G[(n * nS + k1) + (size_t)dn * (n2 * nS + k2)] = v;
                }
        }
    });
    h.Gc.upload(G, s);
    // its diagonal d x d blocks G_kk(n, m) as coefficients of the stiffness classes (n <= m;
    // the class of n < m holds both orders): the mixed-precision path applies them exactly
    Vec cd((size_t)nS * nstiff);
    for (int k2 = 0; k2 < nS; ++k2)
        for (int c = 0; c < nstiff; ++c)
            cd[(size_t)k2 * nstiff + c] = G[(nm[c].first * nS + k2) + (size_t)dn * (nm[c].second * nS + k2)];
    h.coefD.upload(cd, s);
}

// C = L^-1 S- L^-T (S- symmetrised) for M_S- = L L^T blockwise (L = blockdiag of the Cholesky
// factors of 2 T_k): the odd scattering matrix in coordinates where M_S- is the identity
Vec Asm::whitened_odd_scatter() const {
    Vec A((size_t)nSm * nSm);
    // rows 3 kb .. 3 kb + 2 per task (host threads; every entry is computed alone)
    parallel_for(nS, [&](int kb) {
        for (int kc = 0; kc < nS; ++kc) {
            const double* Li = &LkInv[9 * kb];
            const double* Lj = &LkInv[9 * kc];
            double blk[9], tmp[9];
            for (int n = 0; n < 3; ++n)
                for (int m = 0; m < 3; ++m) {
                    const double a1 = h.h_Sm[(3 * kb + n) + (size_t)nSm * (3 * kc + m)];
                    const double a2 = h.h_Sm[(3 * kc + m) + (size_t)nSm * (3 * kb + n)];
                    blk[3 * n + m] = 0.5 * (a1 + a2);
                }
            for (int n = 0; n < 3; ++n)          // tmp = Li * blk
                for (int m = 0; m < 3; ++m) {
                    double v = 0;
                    for (int e = 0; e < 3; ++e) v += Li[3 * n + e] * blk[3 * e + m];
                    tmp[3 * n + m] = v;
                }
            for (int n = 0; n < 3; ++n)          // A = tmp * Lj^T
                for (int m = 0; m < 3; ++m) {
                    double v = 0;
                    for (int e = 0; e < 3; ++e) v += tmp[3 * n + e] * Lj[3 * m + e];
                    A[(3 * kb + n) + (size_t)nSm * (3 * kc + m)] = v;
                }
        }
    });
    return A;
}

// odd: S- W = M_S- W Lambda; with M_S- = L L^T blockwise: (L^-1 S- L^-T) V = V Lambda, W = L^-T V
void Asm::odd_eigenbasis() {
    Vec A = whitened_odd_scatter();
    Vec lam;
    syevd(*rb, s, nSm, A, lam);
    // W = L^-T V, reorder to non-increasing eigenvalues
    Wfull.assign((size_t)nSm * nSm, 0.0);
    h.h_lamm_full.resize(nSm);
    for (int c = 0; c < nSm; ++c) {
        const int src = nSm - 1 - c;
        h.h_lamm_full[c] = lam[src];
        for (int kb = 0; kb < nS; ++kb) {
            const double* Li = &LkInv[9 * kb];
            for (int n = 0; n < 3; ++n) {
                double v = 0;     // (L^-T)(n, e) = Li(e, n)
                for (int e = 0; e < 3; ++e) v += Li[3 * e + n] * A[(3 * kb + e) + (size_t)nSm * src];
                Wfull[(3 * kb + n) + (size_t)nSm * c] = v;
            }
        }
    }
    Vec Wm((size_t)nSm * h.dNm), lm(h.dNm);
    for (int c = 0; c < h.dNm; ++c) {
        lm[c] = h.h_lamm_full[c];
        std::copy(Wfull.begin() + (size_t)nSm * c, Wfull.begin() + (size_t)nSm * (c + 1), Wm.begin() + (size_t)nSm * c);
    }
    h.Wm.upload(Wm, s);
    h.lamm.upload(lm, s);
    // exact odd inverse: full basis (row-major K x N views for the GEMM) and, when the
    // ratio sigma_s / sigma_t is uniform, H = (M_S- - delta S-)^{-1} = W diag(1/(1-delta lam)) W^T
    {
        Vec WT((size_t)nSm * nSm), Wrm((size_t)nSm * nSm);
        for (int r = 0; r < nSm; ++r)
            for (int c = 0; c < nSm; ++c) {
                Wrm[(size_t)r * nSm + c] = Wfull[r + (size_t)nSm * c];   // B(k=r, n=c) = W[r, c]
                WT[(size_t)c * nSm + r] = Wfull[r + (size_t)nSm * c];    // B(k=c, n=r) = W[r, c]
            }
        h.Wfull.upload(Wrm, s);
        h.WfullT.upload(WT, s);
        h.lam_full.upload(h.h_lamm_full, s);
        if (h.uniform_delta) {
            Vec Wsc(Wfull);
            for (int c = 0; c < nSm; ++c) {
                const double f = 1.0 / (1.0 - h.delta0 * h.h_lamm_full[c]);
                for (int r = 0; r < nSm; ++r) Wsc[r + (size_t)nSm * c] *= f;
            }
            // H = Wsc W^T : as GEMM with A = Wsc (col-major), B = W^T (row-major K x N: B(k=c, n=r) = W[r,c])
            DBuf<double> dWsc;
            dWsc.upload(Wsc, s);
            h.Hodd.alloc((size_t)nSm * nSm);
            k::gemm_f64(nSm, nSm, nSm, 1.0, dWsc.p, nSm, h.WfullT.p, nSm, 0.0, h.Hodd.p, nSm, s);
            RTE_HIP(hipStreamSynchronize(s));
            Hh = h.Hodd.download(s);
            condensed_from_H();
        }
        h.have_exact = true;
    }
}

// H = (M_S- - delta S-)^{-1} = L^-T (I - R)^{-1} L^-1 with R = delta C, C the whitened odd
// scattering matrix.  The spectrum of C lies in [-1, 1] (the odd Legendre moments of the
// normalised kernel), so that of R lies inside (-1, 1) for delta < 1, and
//   (I - R)^{-1} = (I + R)(I + R^2)(I + R^4) ...
// converges doubly exponentially: X <- X + X Z, Z <- Z^2 from X = I + R, Z = R, until the next
// factor is below the FP64 resolution of X.  Every product is this library's FP64 MFMA GEMM,
// whose summation order is fixed, so H (and the condensed operator built from it) is bitwise
// the same in every assembly of an instance, whatever else runs on the device; a dense
// factorisation by a vendor library is not guaranteed to be (one varied in its last bits when
// assemblies overlapped other work on the device).
void Asm::odd_inverse() {
    const size_t n = (size_t)nSm, nn = n * n;
    const Vec C = whitened_odd_scatter();
    Vec X0(nn), Z0(nn), LiRM(nn, 0.0);
    for (size_t e = 0; e < nn; ++e) {
        Z0[e] = h.delta0 * C[e];
        X0[e] = Z0[e];
    }
    for (size_t i = 0; i < n; ++i) X0[i + n * i] += 1.0;
    // L^-1 by rows: LiRM[r n + c] = (L^-1)(r, c), block diagonal
    for (int k = 0; k < nS; ++k)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) LiRM[(size_t)(3 * k + a) * n + 3 * k + b] = LkInv[9 * k + 3 * a + b];
    DBuf<double> X, Xn, Z, Zn, Li, red(k::kRedBlocks), scal(1);
    X.upload(X0, s);
    Z.upload(Z0, s);
    Li.upload(LiRM, s);
    Xn.alloc(nn);
    Zn.alloc(nn);
    // ||Z||_F of the current factor, read on the host
    auto norm2 = [&](const double* v) {
        k::dot(v, v, nn, red.p, s);
        k::reduce(red.p, scal.p, 0, s);
        double r = 0.0;
        RTE_HIP(hipMemcpyAsync(&r, scal.p, sizeof(double), hipMemcpyDeviceToHost, s));
        RTE_HIP(hipStreamSynchronize(s));
        return r;
    };
    // X and every power of R are polynomials in the symmetric C, hence symmetric: as the
    // row-major right operand of the GEMM they need no transpose
    double zprev = norm2(Z.p);
    bool converged = false;
    for (int it = 0; it < 64 && !converged; ++it) {
        k::gemm_f64((int)n, (int)n, (int)n, 1.0, Z.p, (int)n, Z.p, (int)n, 0.0, Zn.p, (int)n, s);
        std::swap(Z.p, Zn.p);
        const double z = norm2(Z.p);
        if (!std::isfinite(z) || (it >= 4 && z >= zprev))
            fail(RTE_E_ARG, "M_S- - delta S- is not positive definite (the inverse's product does not converge)");
        zprev = z;
        k::copy(X.p, Xn.p, nn, s);
        k::gemm_f64((int)n, (int)n, (int)n, 1.0, X.p, (int)n, Z.p, (int)n, 1.0, Xn.p, (int)n, s);
        std::swap(X.p, Xn.p);
        converged = std::sqrt(z) <= 1e-18;
    }
    if (!converged) fail(RTE_E_ARG, "M_S- - delta S- is not positive definite (the inverse's product does not converge)");
    // H = L^-T X L^-1: T = L^-T X (A = L^-T column-major is L^-1 by rows), H = T L^-1
    k::gemm_f64((int)n, (int)n, (int)n, 1.0, Li.p, (int)n, X.p, (int)n, 0.0, Zn.p, (int)n, s);
    h.Hodd.alloc(nn);
    k::gemm_f64((int)n, (int)n, (int)n, 1.0, Zn.p, (int)n, Li.p, (int)n, 0.0, h.Hodd.p, (int)n, s);
    k::symmetrize_lower(h.Hodd.p, (int)n, s);
    RTE_HIP(hipStreamSynchronize(s));
    Hh = h.Hodd.download(s);
    condensed_from_H();
    h.have_exact = true;
}

// eigen-bases, even part: the top dN+ eigenpairs of (S+, M+) (Sec. 5.4)
void Asm::even_basis() {
    // ---- coarse needs P_n = W_full^T (A_n W+) later; keep Wfull on the host until then
    h.h_Sm.clear();
    h.h_Sm.shrink_to_fit();
    // even
    Vec Ap((size_t)nS * nS);
    Vec isq(nS);
    for (int k = 0; k < nS; ++k) isq[k] = 1.0 / std::sqrt(h.h_m[k]);
    for (int a = 0; a < nS; ++a)
        for (int b = 0; b < nS; ++b)
            Ap[a + (size_t)nS * b] =
                0.5 * (h.h_Sp[a + (size_t)nS * b] + h.h_Sp[b + (size_t)nS * a]) * isq[a] * isq[b];
    h.h_lamp.resize(h.dNp);
    h.h_Wp.resize((size_t)nS * h.dNp);
    bool done = false;
    if (h.dNp == 1) {
        Vec v0(nS), v;
        double msum = 0.0;
        for (int k = 0; k < nS; ++k) { v0[k] = std::sqrt(h.h_m[k]); msum += h.h_m[k]; }
        for (int k = 0; k < nS; ++k) v0[k] /= std::sqrt(msum);
        double lam = 0.0;
        if (top_eigenpair(*rb, s, nS, Ap, v0, v, lam)) {
            h.h_lamp[0] = lam;
            for (int k = 0; k < nS; ++k) h.h_Wp[k] = v[k] * isq[k];
            done = true;
        }
    }
    if (!done) {
        Vec lp;
        syevd(*rb, s, nS, Ap, lp);
        for (int c = 0; c < h.dNp; ++c) {
            const int src = nS - 1 - c;
            h.h_lamp[c] = lp[src];
            for (int k = 0; k < nS; ++k) h.h_Wp[k + (size_t)nS * c] = Ap[k + (size_t)nS * src] * isq[k];
        }
    }
    h.Wp.upload(h.h_Wp, s);
}

// the coarse matrix E_c = W^T (E - K+) W in band form, factored (Sec. 5.4), with the
// bandwidth-reducing order of the P1 unknowns that the banded E_0 factors share
void Asm::coarse() {
    {
        const int dN = h.dNp;
        // (A_n W+)[(k,m), a] = 2 T_k(n, m) W+[k, a]  [nSm x dN], and with the odd eigenbasis
        // P_n = W_full^T (A_n W+)
        std::vector<Vec> AWn(d, Vec((size_t)nSm * dN));
        std::vector<Vec> Pn(odd_eig ? d : 0, Vec((size_t)nSm * dN, 0.0));
        for (int n = 0; n < d; ++n) {
            Vec& AW = AWn[n];
            for (int k = 0; k < nS; ++k)
                for (int m = 0; m < 3; ++m)
                    for (int a = 0; a < dN; ++a)
                        AW[(3 * k + m) + (size_t)nSm * a] = 2.0 * h.h_T[9 * k + 3 * n + m] * h.h_Wp[k + (size_t)nS * a];
            if (!odd_eig) continue;
            for (int c = 0; c < nSm; ++c)
                for (int a = 0; a < dN; ++a) {
                    double v = 0;
                    const double* wc = &Wfull[(size_t)nSm * c];
                    const double* aw = &AW[(size_t)nSm * a];
                    for (int r = 0; r < nSm; ++r) v += wc[r] * aw[r];
                    Pn[n][c + (size_t)nSm * a] = v;
                }
        }
        // G_nm(delta) = (A_n W+)^T (M_S- - delta S-)^{-1} (A_m W+) for each distinct delta:
        // P_n^T diag(1/(1 - delta lam)) P_m with the eigenbasis, else (uniform delta) through H
        std::map<double, Vec> Gcache;     // key delta -> [d*d*dN*dN]
        auto Gfor = [&](double delta) -> const Vec& {
            auto it = Gcache.find(delta);
            if (it != Gcache.end()) return it->second;
            Vec G((size_t)d * d * dN * dN, 0.0);
            if (odd_eig) {
                Vec f(nSm);
                for (int c = 0; c < nSm; ++c) f[c] = 1.0 / (1.0 - delta * h.h_lamm_full[c]);
                for (int n = 0; n < d; ++n)
                    for (int m = 0; m < d; ++m)
                        for (int a = 0; a < dN; ++a)
                            for (int b = 0; b < dN; ++b) {
                                double v = 0;
                                for (int c = 0; c < nSm; ++c)
                                    v += Pn[n][c + (size_t)nSm * a] * f[c] * Pn[m][c + (size_t)nSm * b];
                                G[((size_t)(n * d + m) * dN + a) * dN + b] = v;
                            }
            } else {
                Vec HA((size_t)nSm * dN);
                for (int m = 0; m < d; ++m) {
                    for (int b = 0; b < dN; ++b)       // HA = H (A_m W+), H symmetric
                        for (int r = 0; r < nSm; ++r) {
                            double v = 0;
                            const double* hr = &Hh[(size_t)nSm * r];
                            const double* aw = &AWn[m][(size_t)nSm * b];
                            for (int c = 0; c < nSm; ++c) v += hr[c] * aw[c];
                            HA[r + (size_t)nSm * b] = v;
                        }
                    for (int n = 0; n < d; ++n)
                        for (int a = 0; a < dN; ++a)
                            for (int b = 0; b < dN; ++b) {
                                double v = 0;
                                for (int r = 0; r < nSm; ++r)
                                    v += AWn[n][r + (size_t)nSm * a] * HA[r + (size_t)nSm * b];
                                G[((size_t)(n * d + m) * dN + a) * dN + b] = v;
                            }
                }
            }
            return Gcache.emplace(delta, std::move(G)).first->second;
        };
        // ordering: the given vertex order unless reverse Cuthill-McKee narrows the band by
        // more than 3% (host.cpp)
        std::vector<int> perm;
        bool natural = false;
        const int sbw = band_order(nRp, rp, ci, perm, &natural);
        h.perm_identity = natural;
        std::vector<int> iperm(nRp);
        for (int i = 0; i < nRp; ++i) iperm[perm[i]] = i;
        h.sbw = sbw;
        const int nc = dN * nRp;
        const int bw = dN * sbw + dN - 1;
        const size_t w1 = (size_t)bw + 1;
        if ((double)nc * w1 > 4.0e9) fail(RTE_E_ARG, "coarse band too large for the host factorisation");
        Vec band((size_t)nc * w1, 0.0);
        auto addE = [&](int i, int a, int i2, int b, double v) {
            const int r = a + dN * perm[i], c = b + dN * perm[i2];
            if (c > r) return;   // lower band only (the matrix is symmetric)
            band[(size_t)r * w1 + bw + c - r] += v;
        };
        // Omega_ab[cb] = sum_k W(k,a) W(k,b) omega[cb, k]
        Vec Om((size_t)dN * dN * nb, 0.0);
        for (int a = 0; a < dN; ++a)
            for (int b = 0; b < dN; ++b)
                for (int c = 0; c < nb; ++c) {
                    double v = 0;
                    for (int k = 0; k < nS; ++k)
                        v += h.h_Wp[k + (size_t)nS * a] * h.h_Wp[k + (size_t)nS * b] * omega[(size_t)c * nS + k];
                    Om[((size_t)a * dN + b) * nb + c] = v;
                }
        for (int i = 0; i < nRp; ++i)
            for (int e = rp[i]; e < rp[i + 1]; ++e) {
                const int i2 = ci[e];
                for (int a = 0; a < dN; ++a)
                    for (int b = 0; b < dN; ++b) {
                        double v = 0;
                        if (a == b) v += cls[(size_t)nstiff * nnz + e] - h.h_lamp[a] * Msv[e];
                        for (int c = 0; c < nb; ++c) v += Om[((size_t)a * dN + b) * nb + c] * cls[(size_t)(nstiff + 1 + c) * nnz + e];
                        if (v != 0.0) addE(i, a, i2, b, v);
                    }
            }
        for (int j = 0; j < nRm; ++j) {
            const Vec& G = Gfor(D->sigma_s[j] / D->sigma_t[j]);
            const int* cj = D->cell + nv * j;
            for (int pa = 0; pa < nv; ++pa)
                for (int pb = 0; pb < nv; ++pb) {
                    const double* Da = &Dc[((size_t)j * nv + pa) * d];
                    const double* Db = &Dc[((size_t)j * nv + pb) * d];
                    for (int a = 0; a < dN; ++a)
                        for (int b = 0; b < dN; ++b) {
                            double v = 0;
                            for (int n = 0; n < d; ++n)
                                for (int m = 0; m < d; ++m)
                                    v += Da[n] * Db[m] * G[((size_t)(n * d + m) * dN + a) * dN + b];
                            addE(cj[pa], a, cj[pb], b, v / mt[j]);
                        }
                }
        }
        h.nc = nc;
        h.cbw = bw;
        // A single band solve is one wave walking nc rows in sequence, so the coarse solve
        // uses the explicit inverse where it fits (dense Cholesky and inverse on the GPU, once),
        // applied as a bandwidth-bound matrix-vector product; else the band solve where the
        // band fits it; else the block-tridiagonal Cholesky on the device.
        const bool inv_fits = (double)nc * nc * sizeof(double) <= kEcinvMaxBytes;
        const bool band_fits = k::band_groups(bw, 2) != 0;
        int how = o->coarse_solver;
        if (how == RTE_COARSE_QUICK) how = (band_fits && k::band_factor_fits(bw)) ? RTE_COARSE_BAND : RTE_COARSE_BLOCK;
        if (how == RTE_COARSE_AUTO) how = inv_fits ? RTE_COARSE_INVERSE : band_fits ? RTE_COARSE_BAND : RTE_COARSE_BLOCK;
        if (how == RTE_COARSE_INVERSE) {
            if (!inv_fits) fail(RTE_E_ARG, "the explicit coarse inverse exceeds its memory budget");
            dense_spd_inverse(*rb, s, band, nc, bw, h.Ecinv, "the coarse matrix E_c");
        } else if (how == RTE_COARSE_BAND) {
            if (!band_fits) fail(RTE_E_ARG, "coarse band too wide for the band solve");
            if (k::band_factor_fits(bw)) {
                // factored on the device, in place, by the E_0 factor kernel
                h.Lc.upload(band_to_blocked(band, nc, bw, false), s);
                h.LcU.upload(Vec(h.Lc.n, 0.0), s);
                DBuf<int> bad(1);
                RTE_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
                k::band_factor_one(nc, bw, h.Lc.p, h.LcU.p, bad.p, s);
                int hb = 0;
                RTE_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
                RTE_HIP(hipStreamSynchronize(s));
                if (hb) fail(RTE_E_ARG, "coarse matrix is not positive definite");
            } else {
                band_cholesky(band, nc, bw);
                h.Lc.upload(band_to_blocked(band, nc, bw, false), s);
                h.LcU.upload(band_to_blocked(band, nc, bw, true), s);
                k::band_invert_diag(h.Lc.p, h.LcU.p, nc, bw, 1, 0, s);
            }
        } else {
            DBuf<double> dband;
            dband.upload(band, s);
            coarse_block_factor(h, dband.p, nc, bw, s);
            RTE_HIP(hipStreamSynchronize(s));
        }
        h.perm.upload(perm, s);
        h.iperm.upload(iperm, s);
    }
    h.h_Sp.clear();
    h.h_Sp.shrink_to_fit();
}

// E_0 data (Sec. 5.3): the banded Cholesky factors of every direction block, or the explicit
// block values of the CG
void Asm::e0_data() {
    if (o->e0_solver == RTE_E0_BANDED) {
        if (k::band_groups(h.sbw, 2) == 0 || k::band_groups(h.sbw, 4) == 0)
            fail(RTE_E_ARG, "E_0 band too wide for the band solve");
        h.e0_stride = k::band_blk_size(nRp, h.sbw, 2);
        h.e0_g64 = (int)k::band_groups(h.sbw, 2);
        h.L0.alloc(h.e0_stride * nS);
        h.L0U.alloc(h.e0_stride * nS);
        DBuf<int> bad(1);
        RTE_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
        k::e0_band_factor(&h, h.sbw, h.perm.p, h.iperm.p, h.L0.p, h.L0U.p, h.e0_stride, bad.p, s);
        int hb = 0;
        RTE_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
        RTE_HIP(hipStreamSynchronize(s));
        if (hb) fail(RTE_E_ARG, "an E_0 block lost positive definiteness in the band factorisation");
        h.have_e0_banded = true;
    } else if (o->e0_solver == RTE_E0_CG || o->e0_solver == RTE_E0_MG) {
        // the explicit block values of the CG: FP64 unless only the mixed form is wanted
        // (mixed = 2; an FP64 CG then builds them on first use), FP32 with mixed != 0
        if (o->e0_solver == RTE_E0_MG) mg_hierarchy();
        if (o->mixed != 2) sv::cg_prepare(&h, false, s);
        if (o->mixed) sv::cg_prepare(&h, true, s);
        if (o->e0_solver == RTE_E0_MG) {
            if (o->mixed != 2) sv::mg_prepare(&h, false, s);
            if (o->mixed) sv::mg_prepare(&h, true, s);
        }
    } else {
        fail(RTE_E_ARG, "unknown e0_solver");
    }
}

// the multigrid hierarchy of the E_0 blocks (RTE_E0_MG): lattice meshes only; levels 1.. by
// Galerkin products of the value classes (host), their sliced-ELL patterns and class values
// uploaded (the per-direction values follow in mg_prepare)
void Asm::mg_hierarchy() {
    const int m = lattice_m(D);
    if (!m) fail(RTE_E_ARG, "e0_solver RTE_E0_MG needs a lattice mesh (Freudenthal triangulation of a box)");
    const std::vector<int> sizes = mg_level_sizes(m);
    h.mgl.clear();
    h.mgl.resize(sizes.size());
    h.mgl[0].m = m;
    h.mgl[0].n = nRp;
    h.mgl[0].nnz = nnz;
    std::vector<int> prp = rp, pci = ci;
    Vec pcls = cls;
    for (size_t l = 1; l < sizes.size(); ++l) {
        MgHostLevel L = mg_coarsen(d, sizes[l - 1], h.ncls, prp, pci, pcls);
        Handle::MgLevel& g = h.mgl[l];
        g.m = L.m;
        g.n = L.n;
        g.nnz = L.rp[L.n];
        std::vector<int> sptr, ecol, epos;
        g.len = sliced_ell(L.n, L.rp, L.ci, &sptr, &ecol, &epos);
        g.nslice = (L.n + 63) / 64;
        for (int sl = 0; sl < g.nslice; ++sl) g.wmax = std::max(g.wmax, sptr[sl + 1] - sptr[sl]);
        g.sptr.upload(sptr, s);
        g.col.upload(ecol, s);
        g.e.upload(epos, s);
        g.cls.upload(L.cls, s);
        prp = std::move(L.rp);
        pci = std::move(L.ci);
        pcls = std::move(L.cls);
    }
    h.mg_m = m;
}

// reduced-precision copies of the mixed-precision path, and the handle's small buffers
void Asm::reduced_precision() {
    if (o->mixed) {
        // FP32 scattering matrices for the FP32 MFMA scatter GEMMs of the preconditioner
        h.Sp_f.alloc(h.Sp.n);
        h.Sm_f.alloc(h.Sm.n);
        k::cvt_f64_f32(h.Sp.p, h.Sp_f.p, h.Sp.n, s);
        k::cvt_f64_f32(h.Sm.p, h.Sm_f.p, h.Sm.n, s);
        if (h.Gc.p) {
            // the BF16 transport operator without its diagonal d x d blocks, which are nearly
            // singular for small sphere triangles and go to the A^T kernel exactly instead (see
            // kernels_mixed.hip)
            const size_t dn = (size_t)h.d * nS;
            h.Gc_bf.alloc(dn * dn);
            k::cvt_f64_bf16_offdiag(h.Gc.p, h.Gc_bf.p, dn, nS, s);
        }
        if (h.have_e0_banded) {
            h.e0_stride32 = k::band_blk_size(nRp, h.sbw, 4);
            h.e0_g32 = (int)k::band_groups(h.sbw, 4);
            h.L0f.alloc(h.e0_stride32 * nS);
            h.L0Uf.alloc(h.e0_stride32 * nS);
            k::band_to_f32(h.L0.p, h.L0f.p, nRp, h.sbw, nS, h.e0_stride, h.e0_stride32, s, h.e0_g64, h.e0_g32);
            k::band_to_f32(h.L0U.p, h.L0Uf.p, nRp, h.sbw, nS, h.e0_stride, h.e0_stride32, s, h.e0_g64, h.e0_g32);
            if (o->mixed == 2) {
                RTE_HIP(hipStreamSynchronize(s));
                h.L0.release();
                h.L0U.release();
            }
        }
        h.have_mixed = true;
    }    h.red.alloc(k::kRedBlocks);
    h.scal.alloc(64);
    RTE_HIP(hipHostMalloc(reinterpret_cast<void**>(&h.pinned), 64 * sizeof(double), hipHostMallocDefault));
    RTE_HIP(hipStreamSynchronize(s));
}

}  // namespace

Handle* assemble(const rte_problem_desc* D, const rte_assemble_opts* o, hipStream_t s) {
    auto H = std::make_unique<Handle>();
    Asm a(D, o, s, *H);
    a.init();
    a.trace("validation");
    a.sphere();
    a.trace("sphere pairing");
    a.quadrature();
    a.trace("angular quadrature");
    a.geometry();
    a.trace("spatial geometry");
    a.pattern();
    a.trace("P1 pattern");
    a.boundary();
    a.trace("boundary facets");
    a.classes();
    a.incidence_and_source();
    a.trace("value classes");
    a.upload();
    a.trace("uploads");
    a.scattering();
    a.trace("scattering matrices");
    a.rb = std::make_unique<RocblasCtx>(s);
    a.odd_basis();
    a.even_basis();
    a.trace("eigen-bases");
    a.coarse();
    a.trace("coarse matrix");
    a.e0_data();
    a.trace("E_0 band factors");
    a.reduced_precision();
    a.trace("reduced-precision copies");
    return H.release();
}

}  // namespace rte
