// Internal declarations of librte: the handle, device buffers, error handling and the
// kernel launchers shared by the host orchestration code.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>
#include <shared_mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/rte.h"
#include "host.h"

namespace rte {

#define RTE_HIP(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            ::rte::fail(e_ == hipErrorOutOfMemory ? RTE_E_NOMEM : RTE_E_HIP,             \
                        std::string(#call) + ": " + hipGetErrorString(e_));              \
    } while (0)

#define RTE_CHECK_LAUNCH() RTE_HIP(hipGetLastError())

// ----------------------------------------------------------------------------- capture
// Stream capture (the batch's graphs) and rocBLAS / rocSOLVER calls exclude each other
// across threads: the libraries touch the legacy null stream (handle set-up, workspace),
// which HIP rejects while a stream of the process is being captured.  Library calls take
// the lock shared, a capture takes it exclusively; neither holds it across a wait for
// device work.
inline std::shared_mutex& capture_mutex() {
    static std::shared_mutex m;
    return m;
}

// The rocSOLVER factorisations of concurrent assemblies (worker threads of the server) run
// one at a time: each holds this lock from upload to read-back.
inline std::mutex& solver_library_mutex() {
    static std::mutex m;
    return m;
}

// ----------------------------------------------------------------------------- buffers
// The first failed hipFree of the calling thread since the last take_free_error() (a destructor
// cannot throw, so releases record their error here; re-allocation and rte_destroy report it).
inline hipError_t& free_error() {
    static thread_local hipError_t e = hipSuccess;
    return e;
}
inline hipError_t take_free_error() {
    const hipError_t e = free_error();
    free_error() = hipSuccess;
    return e;
}

// Owning device buffer (hipMalloc / hipFree); movable, not copyable.
template <typename T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DBuf& operator=(DBuf&& o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t count) {
        release();
        const hipError_t fe = take_free_error();
        if (fe != hipSuccess) fail(RTE_E_HIP, std::string("hipFree failed: ") + hipGetErrorString(fe));
        if (count) RTE_HIP(hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(T)));
        n = count;
    }
    void release() {
        if (p) {
            const hipError_t e = hipFree(p);
            if (e != hipSuccess && free_error() == hipSuccess) free_error() = e;
        }
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
    // blocking: the host vector may be a temporary
    void upload(const std::vector<T>& h, hipStream_t s) {
        alloc(h.size());
        if (n) {
            RTE_HIP(hipMemcpyAsync(p, h.data(), bytes(), hipMemcpyHostToDevice, s));
            RTE_HIP(hipStreamSynchronize(s));
        }
    }
    std::vector<T> download(hipStream_t s) const {
        std::vector<T> h(n);
        if (n) {
            RTE_HIP(hipMemcpyAsync(h.data(), p, bytes(), hipMemcpyDeviceToHost, s));
            RTE_HIP(hipStreamSynchronize(s));
        }
        return h;
    }
};

// ----------------------------------------------------------------------------- handle

struct Handle {
    // sizes
    int d = 0, nRp = 0, nRm = 0, nS = 0, nSm = 0;
    int dNp = 1, dNm = 21;         // sizes of the even correction / odd PCG eigen-bases
    int n_even = 0, n_odd = 5;
    double g = 0, c = 0;           // anisotropy and max sigma_s / sigma_t
    bool uniform_delta = false;    // sigma_s / sigma_t is the same in every cell
    double delta0 = 0;             // that ratio when uniform
    hipStream_t stream = nullptr;  // stream the handle was assembled on

    // ---- angular (Sec. 4)
    DBuf<double> Sp, Sm;           // [nS x nS], [nSm x nSm] symmetric, dense
    DBuf<double> m;                // [nS]   (M_S+)_kk = 2|K_k|
    DBuf<double> T;                // [nS*9] T_k row-major
    DBuf<double> MSinv;            // [nS*9] inverse of the 3x3 block 2 T_k of M_S-
    DBuf<double> Wm, lamm;         // odd eigenvectors [nSm x dNm] col-major, eigenvalues [dNm]
    DBuf<double> Wp;               // even eigenvectors [nS x dNp] col-major
    std::vector<double> h_m, h_T, h_lamp, h_Wp, h_lamm_full, h_Sp, h_Sm;

    // ---- exact odd inverse (RTE_ODD_EXACT)
    bool have_exact = false;
    bool have_odd_eig = false;     // odd eigenpairs present (PCG odd solve, per-cell exact)
    DBuf<double> Hodd;             // [nSm x nSm] (M_S- - delta0 S-)^{-1} when uniform_delta
    DBuf<double> Wfull, WfullT;    // full odd eigenvectors and transpose (both row-major K x N)
    DBuf<double> lam_full;         // [nSm]
    DBuf<double> Gc;               // [(d nS)^2] condensed transport matrix (uniform ratio only)
    DBuf<double> vcD;              // [n_incidences * d] |T_j| d_n phi_v per vertex-cell incidence
    DBuf<double> MtMs;             // [2 nnz] (sigma_t mass, sigma_s mass) per pattern entry
    DBuf<int> bnd_row;             // [nRp] 1 if the row has boundary-mass entries

    // ---- spatial (Sec. 4)
    DBuf<int> cell;                // [nRm*(d+1)]
    DBuf<double> Dc;               // [nRm*(d+1)*d] |T_j| d_n phi_v on T_j
    DBuf<double> mt, ms;           // [nRm] sigma_t|T|, sigma_s|T|
    DBuf<int> rowptr, col;         // P1 pattern (CSR, nRp rows, sorted columns)
    int nnz = 0;
    DBuf<double> Msv;              // [nnz] sigma_s-weighted P1 mass values
    int ncls = 0;                  // value classes of the pattern:
    DBuf<double> cls;              //   [ncls*nnz]: d(d+1)/2 stiffness terms
                                   //   D_n^T Mt-^{-1} D_m (+ transpose), Mt+, then one
                                   //   boundary facet mass per normal class
    int ncls_stiff = 0, nbcls = 0;
    DBuf<double> coefE0;           // [nS*ncls] E_0 block k = sum_c coefE0[k,c] cls_c
    DBuf<double> coefE;            // [nS*ncls] (M+ + R) block k = sum_c coefE[k,c] cls_c
    DBuf<double> diagE0;           // [nRp*nS] diagonal of every E_0 block (Jacobi)
    DBuf<int> vc_ptr, vc_cell, vc_loc;   // vertex -> incident cells (for A^T)
    // E_0 by CG (kernels_cg.hip): the pattern in sliced ELL form (slices of 64 rows, as many
    // slots as the slice's longest row), its entries' positions in the CSR pattern (-1 on
    // padding), and the explicit values of every direction's block with the inverse diagonal,
    // in FP64 and (mixed) FP32, built at assembly for e0_solver = RTE_E0_CG, else on first use
    int ell_nslice = 0, ell_wmax = 0;
    size_t ell_len = 0;
    DBuf<int> ell_sptr, ell_col, ell_e;
    DBuf<double> ell_v64, ell_dinv64;
    DBuf<float> ell_v32, ell_dinv32;
    DBuf<double> cg_part, cg_scal;   // per-tile partials [4 nS ntiles]; rz [2 nS] and stop [nS]
    DBuf<int> cg_state;             // done [nS], active [1]
    // E_0 by CG preconditioned by a geometric multigrid V-cycle (RTE_E0_MG; lattice meshes,
    // kernels_mg.hip).  Level 0 is the fine pattern above; levels 1.. have their own sliced-ELL
    // pattern and Galerkin class values.  The cycle works on every level's explicit values
    // rounded to the smoother precision: FP32 (s32) for FP64 solves, BF16 (s16) for mixed ones
    // (the CG's own products use the full-precision level-0 values above).  Per precision:
    // inverse diagonals and per direction the Chebyshev interval (theta, delta), both from the
    // rounded values; then the cycle's work vectors x, r, b, d0, d1 per level.
    struct MgLevel {
        int m = 0, n = 0, nnz = 0, nslice = 0, wmax = 0;
        size_t len = 0;
        DBuf<int> sptr, col, e;
        DBuf<double> cls;
        DBuf<float> s32;
        DBuf<uint16_t> s16;
        DBuf<double> dinv64, cheb64;
        DBuf<float> dinv32;
        DBuf<double> cheb32;
        DBuf<unsigned char> work;
        size_t bytes() const {
            return sptr.bytes() + col.bytes() + e.bytes() + cls.bytes() + s32.bytes() + s16.bytes() +
                   dinv64.bytes() + cheb64.bytes() + dinv32.bytes() + cheb32.bytes() + work.bytes();
        }
    };
    int mg_m = 0;                  // lattice vertices per axis when the hierarchy exists, else 0
    std::vector<MgLevel> mgl;
    DBuf<double> q;                // [nRp*nS] even load l+
    double qnorm = 0;

    // ---- coarse (Sec. 5.4): banded Cholesky of E_c in the order a + dNp * perm[i]
    int nc = 0, cbw = 0;
    DBuf<double> Lc, LcU;          // blocked band factor, rows of L and of L^T (kernels_band.hip)
    DBuf<double> Ecinv;            // explicit E_c^{-1} (nc x nc, band order) when it fits its budget
    // block-tridiagonal Cholesky of E_c (coarse_block.hip) for wide coarse bands: cnb blocks
    // of cbs rows; inverses of the diagonal factors and their transposes, the two folded
    // coupling blocks per block boundary and two work vectors of the solve
    int cbs = 0, cnb = 0;
    DBuf<double> CLinv, CLinvT, CB, CG, cwork;
    DBuf<int> perm, iperm;         // [nRp] spatial reordering (reverse Cuthill-McKee) and inverse
    int sbw = 0;                   // spatial band width in that order
    bool perm_identity = false;    // that order is the given vertex order (perm = identity)

    // ---- banded E_0 (RTE_E0_BANDED): one blocked band factor per direction
    bool have_e0_banded = false;
    size_t e0_stride = 0;
    int e0_g64 = 0;                // groups per row block of the FP64 factors' layout
    DBuf<double> L0, L0U;          // [nS * e0_stride], rows of L and of L^T

    // ---- reduced-precision copies (mixed precision)
    bool have_mixed = false;
    DBuf<float> Sp_f, Sm_f;        // FP32 S+ and S- (mixed-precision scatter GEMMs)
    DBuf<uint16_t> Gc_bf;          // condensed transport matrix in BF16 without its diagonal blocks
    DBuf<double> coefD;            // [nS * ncls_stiff] those blocks G_kk(n, m) as stiffness-class
                                   //   coefficients (applied exactly by the A^T kernel)
    size_t e0_stride32 = 0;
    int e0_g32 = 0;                // groups per row block of the FP32 factors' layout
    DBuf<float> L0f, L0Uf;         // FP32 copies of the banded E_0 factors ([nS * e0_stride32])

    // ---- workspace (allocated lazily, sized for one solve)
    std::vector<DBuf<double>> ws;
    DBuf<int> cg_iters;            // per-direction CG counts of the last E_0 application
    DBuf<double> red;              // reduction scratch
    DBuf<double> scal;             // device scalars
    std::vector<double> hscal;
    double* pinned = nullptr;      // small pinned host buffer for scalar readback

    // ---- optional kernel timers (rte_solve_opts.profile): HIP events around launches
    struct ProfRec { int kind; hipEvent_t a, b; double flops; };
    bool prof_on = false;
    std::vector<ProfRec> prof;
    std::vector<hipEvent_t> evpool;

    ~Handle();
    size_t footprint() const;
};

// Assembly (assemble.cpp)
Handle* assemble(const rte_problem_desc* desc, const rte_assemble_opts* opts, hipStream_t s);

// Solver (solver.cpp)
void apply_scatter(Handle* h, int parity, int dtin, const void* X, int dtout, void* Y,
                   hipStream_t s);
void apply_E(Handle* h, const rte_solve_opts* o, const double* X, double* Y, hipStream_t s,
             int64_t* pcg_iters);
void apply_E0(Handle* h, const double* X, double* Y, hipStream_t s);
void apply_mg(Handle* h, const double* X, double* Y, hipStream_t s);
void apply_E0inv(Handle* h, const rte_solve_opts* o, const double* X, double* Y, hipStream_t s,
                 int64_t* cg_total, int* cg_max);
void precond(Handle* h, const rte_solve_opts* o, int which, const double* r, double* out,
             hipStream_t s);
rte_status solve(Handle* h, const rte_solve_opts* o, const double* U0, double* U, double* U_odd,
                 rte_solve_info* info, hipStream_t s);

size_t estimate_footprint(const rte_problem_desc* D, const rte_assemble_opts* o, size_t* peak);

// lockstep batch of solves (solver_batch.cpp)
struct Batch;
Batch* batch_create(int max_slots, size_t budget);
void batch_destroy(Batch* B);
int batch_admit(Batch* B, Handle* h, const rte_solve_opts* o, const double* U0, double* U, hipStream_t s);
int batch_step(Batch* B, int outer_iters, hipStream_t s);
void batch_set_graphs(Batch* B, bool on);
// band layout autotuning of the E_0 factors (autotune.cpp)
void derived_outputs(Handle* h, const double* U, double* phi, double* balance, hipStream_t s);
// scattering operator without device allocation (noalloc.hip): its intermediates live in a
// fixed per-device array whose address noalloc_setup looks up on the current device
void noalloc_setup();
void apply_scatter_noalloc(Handle* h, int parity, int dtin, const void* X, int dtout, void* Y, hipStream_t s);
void coarse_block_factor(Handle& h, const double* dband, int n, int bw, hipStream_t s);
void coarse_block_solve(Handle* h, const double* rhs, double* x, hipStream_t s);
void autotune(Handle* h, int flags, hipStream_t s, rte_tune_report* rep);
void set_band_layout(Handle* h, int precision, int H, int P, hipStream_t s);
int batch_poll(Batch* B, int max_out, int32_t* slots, rte_solve_info* infos, int32_t* statuses);
void batch_usage(const Batch* B, int32_t* n_live, int32_t* n_done, size_t* used_bytes);

// ----------------------------------------------------------------------------- GEMM tile maps
// The tile map of a GEMM launch: bit 0 drops the XCD swizzle of the work-group ids, bit 1 flips
// the traversal order of the tile grid (the shorter dimension fastest by default).  Both only
// reorder whole output tiles, so the result is the same bits.  rte_autotune times the four maps
// of a handle's GEMM shapes and records the fastest per (kind, M, N, K) (autotune.cpp, with an
// on-disk cache); launches look it up (0 when none was recorded).
enum GemmKind { kGemmF64 = 1, kGemmF32 = 2, kGemmF32in = 3, kGemmBF16 = 4 };
int gemm_map(int kind, int M, int N, int K);

// ----------------------------------------------------------------------------- launchers
namespace k {
// Dense scattering matrices by double quadrature of the HG kernel.
void hg_scatter(const double* pts, const double* wts, int nS, int Q, double g, double* Sp,
                double* Sm, hipStream_t s);
// C[MxN] = alpha * A[MxK] (col-major, lda) * B (row-major KxN, ldb) + beta * C (col-major).
// ws (nullable, ws_elems elements, contents overwritten): scratch that lets a lightly loaded
// last round of tiles be split over K.
void gemm_f64(int M, int N, int K, double alpha, const double* A, int lda, const double* B,
              int ldb, double beta, double* C, int ldc, hipStream_t s, double* ws = nullptr,
              size_t ws_elems = 0);
// The same in FP32 MFMA arithmetic (FP32 products, FP32 accumulation); an FP64 A is rounded
// to FP32 as it is loaded, an FP64 C receives the FP32 result.
void gemm_f32(int M, int N, int K, float alpha, const double* A, int lda, const float* B, int ldb,
              float beta, double* C, int ldc, hipStream_t s, float* ws = nullptr, size_t ws_elems = 0);
void gemm_f32(int M, int N, int K, float alpha, const float* A, int lda, const float* B, int ldb,
              float beta, double* C, int ldc, hipStream_t s, float* ws = nullptr, size_t ws_elems = 0);
// BF16 inputs, FP32 accumulate; A row-major bf16 (k contiguous, lda), B column-major bf16
// (k contiguous, ldb), C col-major f32.
void gemm_bf16(int M, int N, int K, float alpha, const uint16_t* A, int lda, const uint16_t* B,
               int ldb, float beta, float* C, int ldc, hipStream_t s);
void cvt_f64_bf16(const double* x, uint16_t* y, size_t n, hipStream_t s);
void cvt_f32_bf16(const float* x, uint16_t* y, size_t n, hipStream_t s);
void cvt_f64_f32(const double* x, float* y, size_t n, hipStream_t s);
// Y = bf16(X) for an n x n matrix whose index is (component, direction) with nb directions,
// except that the entries coupling a direction with itself (r mod nb == c mod nb, the d x d
// diagonal blocks) are zero
void cvt_f64_bf16_offdiag(const double* X, uint16_t* Y, size_t n, size_t nb, hipStream_t s);
void cvt_f32_f64(const float* x, double* y, size_t n, hipStream_t s);
}  // namespace k

}  // namespace rte
