// Launchers of the sparse / Kronecker glue kernels (kernels_ops.hip) and of the
// per-direction E_0 solvers (kernels_e0.hip).
#pragma once
#include <memory>

#include "rte_internal.h"

namespace rte {
namespace k {

constexpr int kRedBlocks = 1024;        // partial sums per deterministic reduction

// B = A X  (B: nRm x 3nS, X: nRp x nS)        [Sec. 4: A = sum_n A_n (x) D_n]
void apply_A(const Handle* h, const double* X, double* B, hipStream_t s);
// Y = A^T Z + (M+ + R) X  [- Ms+ G - q]  (Y, X, G: nRp x nS, Z: nRm x 3nS).
// G and q may be null (no scattering / source term).  Alg. 1, last line; with G = X S+
// and q it is the residual (E - K+) X - q of Alg. 3.
void apply_At_E(const Handle* h, const double* Z, const double* X, const double* G,
                const double* q, double* Y, hipStream_t s, bool condensed = false);
// Yc = Mt-^{-1} [D_1 X, .., D_d X]  (nRm x d nS), the input of the condensed E
void apply_grad(const Handle* h, const double* X, double* Yc, hipStream_t s);
// W = (M- - K-) P given G = P S-:  W = Mt- P M_S- - Ms- G;  red <- partials of P.W
void odd_apply(const Handle* h, const double* P, const double* G, double* W, double* red,
               hipStream_t s);
// scal[out] = sum of kRedBlocks partials (fixed order)
void reduce(const double* red, double* scal, int out, hipStream_t s);
// scal[out] = scal[a] / scal[b]  (0 if scal[b] == 0)
void sdiv(double* scal, int out, int a, int b, hipStream_t s);
// z += a p ; r -= a w ; Cpart <- per-chunk projections r W_N ; red <- partials of r.r
// (a = scal[ia])
void pcg_update(const Handle* h, double* z, double* r, const double* p, const double* w,
                const double* scal, int ia, double* Cpart, double* red, hipStream_t s);
// y = (M- - K-_N)^{-1} r  (Lemma of Sec. 5.1) from r and the chunked projections;
// red <- partials of r.y
void odd_precond(const Handle* h, const double* r, const double* Cpart, double* Cfin, double* y,
                 double* red, hipStream_t s);
// p = y + b p  (b = scal[ib]); with ib < 0: p = y
void xpby(const double* y, double* p, const double* scal, int ib, size_t n, hipStream_t s);
// y = x + a z  (a = scal[ia] * sign)
void axpy_s(double* y, const double* x, const double* z, const double* scal, int ia, double sign,
            size_t n, hipStream_t s);
// red <- partials of x.y
void dot(const double* x, const double* y, size_t n, double* red, hipStream_t s);
void fill(double* x, double v, size_t n, hipStream_t s);
void copy(const double* x, double* y, size_t n, hipStream_t s);
// y = a x + b y (host scalars)
void axpby(double a, const double* x, double b, double* y, size_t n, hipStream_t s);
// Z = Mt-^{-1} (C) row scaling: Z[j, :] = C[j, :] / mt_j
void row_scale_inv_mt(const Handle* h, const double* C, double* Z, int ncols, hipStream_t s);
// C[j, a] /= mt_j (1 - Delta_j lam_a)   (exact odd inverse in the eigenbasis)
void scale_eigbasis(const Handle* h, double* C, hipStream_t s);

// ---- coarse correction (Sec. 5.4)
// rhs[a + dN*perm[i]] = sum_k T[i,k] Wp[k,a]
void coarse_project(const Handle* h, const double* T, double* rhs, hipStream_t s);
// The blocked band layout and its size arithmetic (BandShape, band_groups, band_blk_size, ...)
// are in host.h.
// x = L^{-T} L^{-1} b for nsys systems with blocked band factors BL (rows of L) and BU
// (rows of L^T) in the layout of G groups per row block (G = 0: the default layout)
// (kernels_band.hip); b and x are read / written at iperm[band row] when iperm is given
void band_solve_blk(const double* BL, const double* BU, int n, int bw, int nsys, size_t stride_sys,
                    const double* b, double* x, size_t stride_vec, const int* iperm, hipStream_t s, int G = 0);
// Whether the band factors of half-bandwidth bw hold each 64 x 64 diagonal block as its inverse
// (bw >= 63: the band then holds the whole inverse; the solve applies it as a product)
constexpr bool band_diag_inverted(int bw) { return bw >= 63; }
// Replace every diagonal block of the factors (default FP64 layout) by its inverse when
// band_diag_inverted(bw); the factorisations below call it, a host factor uploaded into the
// layout must too
void band_invert_diag(double* BL, double* BU, int n, int bw, int nsys, size_t stride_sys, hipStream_t s);
// Cholesky factorisation of one SPD band matrix on the device (the E_0 factor kernel with one
// work-group): BL holds the lower band in the blocked layout on entry (offset t = c - r + bw),
// and L on exit, BU (zeroed by the caller) rows of L^T; the diagonal entries become
// 1 / L(i,i).  *bad (zeroed by the caller) is set if a pivot is not positive.
void band_factor_one(int n, int bw, double* BL, double* BU, int* bad, hipStream_t s);
// same with FP32 factors (the reduced-precision preconditioner); FP64 vectors and sums
void band_solve_blk_f32(const float* BL, const float* BU, int n, int bw, int nsys, size_t stride_sys,
                        const double* b, double* x, size_t stride_vec, const int* iperm, hipStream_t s, int G = 0);
// One job of a grouped band solve: nsys systems with factors at BL/BU + stride_sys * sys (FP64 or
// FP32 elements, per launch) in the layout of G groups per row block (0: default) and
// right-hand sides / solutions in band order at b/x + stride_vec * sys.  W and first are
// filled in by band_group_plan.
struct BandJob {
    const void* BL;
    const void* BU;
    const double* b;
    double* x;
    size_t stride_sys, stride_vec;
    int n, bw, nsys, W, first, G;
};
// the launches of a set of jobs, one per band shape, and the jobs in device memory
struct BandGroupPlan {
    struct Launch {
        int H, P, first_job, njobs, nwg;
        size_t lds;
    };
    std::vector<Launch> launches;
    DBuf<BandJob> jobs;
    bool f32 = false;
};
// sort the jobs by band shape, number their work-groups and upload them (blocking)
void band_group_plan(std::vector<BandJob>& jobs, bool f32, BandGroupPlan& plan, hipStream_t s);
// all jobs' solves, one launch per band shape
void band_group_run(const BandGroupPlan& plan, hipStream_t s);
// FP64 blocked factors (G64 groups per row block) -> FP32 blocked factors (G32 groups of 4)
void band_to_f32(const double* src, float* dst, int n, int bw, int nsys, size_t stride64, size_t stride32,
                 hipStream_t s, int G64, int G32);
// the same factors from a layout of Gsrc groups to one of Gdst groups (same element type)
void band_relayout(const double* src, int Gsrc, double* dst, int Gdst, int n, int bw, int nsys,
                   size_t stride_src, size_t stride_dst, hipStream_t s);
void band_relayout(const float* src, int Gsrc, float* dst, int Gdst, int n, int bw, int nsys,
                   size_t stride_src, size_t stride_dst, hipStream_t s);
// whether the solve kernel can run a band of width bw in the layout of G groups of vec
bool band_layout_ok(int bw, int vec, int G);
// lower band (row-major, band[r (bw+1) + bw + c - r]) -> lower triangle of a dense
// column-major n x n matrix; and the copy of that lower triangle to the upper one
void band_to_dense(const double* band, int n, int bw, double* A, hipStream_t s);
void symmetrize_lower(double* A, int n, hipStream_t s);
// column-wise permutation of an n x ncols column-major matrix (src != dst):
// gather dst[r, c] = src[iperm[r], c], or scatter dst[iperm[r], c] = src[r, c]
void permute_cols(const int* iperm, int n, int ncols, const double* src, double* dst, bool gather, hipStream_t s);
// Y = A X for a dense n x n matrix stored by rows
void gemv_rows(int n, const double* A, const double* X, double* Y, hipStream_t s);
// factor every E_0 block (one work-group per direction); *bad |= 1 on a non-positive pivot
void e0_band_factor(const Handle* h, int bw, const int* perm, const int* iperm, double* BL, double* BU,
                    size_t stride_sys, int* bad, hipStream_t s);
// U = U - S + sum_a uc[a + dN*perm[i]] Wp[k, a]
void richardson_update(const Handle* h, double* U, const double* S, const double* uc,
                       hipStream_t s);

// ---- E_0 by CG over a sliced-ELL layout (kernels_cg.hip, Sec. 5.3)
struct CgArgs {
    int n = 0, nS = 0, nslice = 0;   // rows per block, directions, slices of 64 rows
    size_t len = 0;                  // ELL entries per direction (64 per slot of every slice)
    int wmax = 0;                    // slots of the widest slice
    const int* sptr = nullptr;       // [nslice + 1] first slot group of each slice
    const int* col = nullptr;        // [len] column of every entry (shared by the directions)
    const double* B = nullptr;       // right-hand sides, n x nS column-major
    double* X = nullptr;             // solutions (FP64 whatever the vector type)
    double tol = 1e-10;              // stop direction k once ||r_k|| <= tol ||b_k||
    int maxit = 1000, check_every = 16;   // host reads the live count every check_every iterations
    double* part = nullptr;          // [4 nS ntiles] per-tile partial sums
    double* rz = nullptr;            // [2 nS] r.z of consecutive iterations
    double* stop = nullptr;          // [nS] tol^2 b.b
    int* done = nullptr;             // [nS] iteration of convergence (INT_MAX while running)
    int* iters = nullptr;            // [nS] iterations taken
    int* active = nullptr;           // [1] directions still running
    int* host_active = nullptr;      // pinned host copy of *active
};
// val[k len + q] = explicit value of entry q of block k from the pattern classes; dinv = 1/diag
void cg_fill_values(const Handle* h, const int* ell_e, size_t len, double* val, hipStream_t s);
void cg_fill_values(const Handle* h, const int* ell_e, size_t len, float* val, hipStream_t s);
// the same from explicit class values cls [ncls * nnz] and coefficients coef [nS * ncls]
void fill_block_values(int nS, size_t len, int nnz, int ncls, const int* ell_e, const double* cls,
                       const double* coef, double* val, hipStream_t s);
void fill_block_values(int nS, size_t len, int nnz, int ncls, const int* ell_e, const double* cls,
                       const double* coef, float* val, hipStream_t s);
void cg_fill_dinv(const double* diag, size_t n, double* dinv, hipStream_t s);
void cg_fill_dinv(const double* diag, size_t n, float* dinv, hipStream_t s);
// X = E_0^{-1} B, Jacobi-preconditioned CG on every direction block at once (vectors R, P, Q
// of the value type, n x nS); blocking (reads the live count every check_every iterations)
void cg_solve(const CgArgs& a, const double* val, const double* dinv, double* R, double* P, double* Q, hipStream_t s);
void cg_solve(const CgArgs& a, const float* val, const float* dinv, float* R, float* P, float* Q, hipStream_t s);
// pieces the multigrid-preconditioned CG shares with the Jacobi CG: the SpMV Y = E_0 X of the
// directions still running at iteration it with its partials p.q (a.part), and the live count
// with its copy to a.host_active (waited for by the caller)
void cg_spmv_it(const CgArgs& a, int it, const double* val, const double* X, double* Y, hipStream_t s);
void cg_spmv_it(const CgArgs& a, int it, const float* val, const float* X, float* Y, hipStream_t s);
void cg_count(const CgArgs& a, int it, hipStream_t s);
// per direction from the tile partials part ([nS ntiles] b.b, then [nS ntiles] r.z of the
// start): rz_0, the stopping threshold tol^2 b.b and the running state
void cg_setup(const CgArgs& a, const double* part, hipStream_t s);

// ---- geometric multigrid V-cycle for the E_0 blocks (kernels_mg.hip)
constexpr int kMgMaxLevels = 12;
constexpr int kMgNu = 4;              // Chebyshev steps before and after the coarse correction
constexpr int kMgNuCoarse = 8;        // Chebyshev steps on the coarsest level
constexpr double kMgLo = 0.02;        // smoothing interval [lo lam, lam]
constexpr double kMgLoCoarse = 0.02;
static_assert(kMgChebSteps >= kMgNu && kMgChebSteps >= kMgNuCoarse, "Chebyshev coefficient table too short");
struct MgLevelArgs {
    int m = 0, n = 0, nslice = 0, wmax = 0;   // lattice vertices per axis, rows, slices, widest slice
    size_t len = 0;                           // ELL entries per direction
    const int *sptr = nullptr, *col = nullptr;
    // [nS * len] the level's values in the smoother precision (FP32 for FP64 vectors, BF16 for
    // FP32 vectors); [nS * n] inverse diagonals of the vector type
    const void *val = nullptr, *dinv = nullptr;
    // [2 nS]: theta, delta of every direction, then [nS][kMgChebSteps][2]: c1, c2 of step j
    const double* cheb = nullptr;
    void *x = nullptr, *r = nullptr, *b = nullptr, *d0 = nullptr, *d1 = nullptr;   // [nS * n] each
};
struct MgArgs {
    int d = 0, nS = 0, L = 0;
    bool f32 = false;
    MgLevelArgs lev[kMgMaxLevels];
};
// z = B r for every direction still running at iteration it (done[k] >= it, all when done is
// null): r is lev[0].b; returns the buffer d of level 0 with z = lev[0].x + d (the last
// smoothing step's sum is left to the caller, which fuses it).  Enqueue only.
const void* mg_vcycle(const MgArgs& g, int it, const int* done, hipStream_t s);
// Y = B X (FP64 vectors), one V-cycle per direction, through the cycle's buffers
void mg_apply(const MgArgs& g, const double* X, double* Y, hipStream_t s);
// the inverse diagonals and Chebyshev intervals of level l from its smoother values
// (lo = the level's interval fraction); part is scratch of [nS * ceil(n / 256)] doubles
void mg_level_setup(const MgArgs& g, int l, double lo, double* part, hipStream_t s);
// smoother values of a coarse level from its class values (formed in FP64, rounded to FP32,
// then for BF16 to BF16, ties to even), and of level 0 by rounding the CG's values
void mg_fill_smoother(int nS, size_t len, int nnz, int ncls, const int* ell_e, const double* cls, const double* coef,
                      float* val, hipStream_t s);
void mg_fill_smoother(int nS, size_t len, int nnz, int ncls, const int* ell_e, const double* cls, const double* coef,
                      uint16_t* val, hipStream_t s);
void mg_round(const double* src, float* dst, size_t n, hipStream_t s);
void mg_round(const float* src, uint16_t* dst, size_t n, hipStream_t s);

// one CG solve driven in phases, Jacobi (kernels_cg.hip) or multigrid (kernels_mg.hip)
struct CgJob;
struct CgPhases {
    virtual ~CgPhases() = default;
    virtual void start() = 0;
    virtual void iterate(int it) = 0;
    // after iteration it: a check point (every check_every iterations, and the last)
    bool check_point(int it) const { return (it + 1) % a.check_every == 0 || it + 1 == a.maxit; }
    void count(int it) { cg_count(a, it, s); }
    const CgArgs& a;
    hipStream_t s;
    CgPhases(const CgArgs& a_, hipStream_t s_) : a(a_), s(s_) {}
};
// Several such solves (different handles) advanced in lockstep, each on its own stream, with
// one host synchronisation per check interval for all of them; each solve's launches and
// arithmetic are exactly those of its solo run on its stream
struct CgJob {
    CgArgs a;
    bool f32 = false;                 // value and vector type: FP32 (else FP64)
    const void* val = nullptr;
    const void* dinv = nullptr;
    void *R = nullptr, *P = nullptr, *Q = nullptr;
    const MgArgs* mg = nullptr;       // multigrid preconditioner (else Jacobi with dinv)
    hipStream_t s = nullptr;
};
std::unique_ptr<CgPhases> mg_phases(const CgJob& j);
void cg_solve_many(std::vector<CgJob>& jobs);
// Y = E_0 X on every direction (FP64), the CG's own SpMV kernel
void cg_spmv(const CgArgs& a, const double* val, const double* X, double* Y, hipStream_t s);

}  // namespace k
}  // namespace rte

namespace rte {
namespace k {
// Y = M X column by column for a matrix with the P1 pattern and values vals[nnz]
void spmm_pattern(const Handle* h, const double* vals, const double* X, double* Y, hipStream_t s);
// Ycb = bf16(Mt-^{-1} [D_1 X, .., D_d X]), row-major nRm x d nS (angular index contiguous)
void apply_grad_bf16(const Handle* h, const double* X, uint16_t* Ycb, hipStream_t s);
// apply_At_E with the condensed components Z row-major (Z[j (d nS) + n nS + k]), FP64 or FP32;
// the FP32 form (the mixed-precision GEMM, whose operator leaves out the diagonal d x d blocks)
// adds those blocks exactly, sum_{n,m} G_kk(n,m) D_n^T Mt-^{-1} D_m X[:, k] (Handle::coefD)
void apply_At_E_rm(const Handle* h, const double* Z, const double* X, const double* G, const double* q, double* Y,
                   hipStream_t s);
void apply_At_E_rm_f32(const Handle* h, const float* Z, const double* X, const double* G, const double* q, double* Y,
                       hipStream_t s);
// Y[j, c] = v[j] X[j, c]   (nrow x ncol, col-major)
void row_scale(const double* v, int nrow, int ncol, const double* X, double* Y, hipStream_t s);
}  // namespace k
}  // namespace rte
