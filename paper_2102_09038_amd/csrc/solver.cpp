// Host orchestration of the preconditioned Richardson iteration (paper Sec. 5):
// ApplyE (Alg. 1), E_0^{-1} (Sec. 5.3), P_1^l (Alg. 2), the subspace correction P_2
// (Sec. 5.4) and the outer loop (Alg. 3).  Every arithmetic step is a HIP kernel on the
// caller's stream; the host only sequences launches and reads back one scalar per PCG
// or outer iteration for the convergence tests.
#include <chrono>
#include <cmath>

#include "solver_detail.h"

namespace rte {
namespace sv {

double* ws(Handle* h, int id) {
    if (h->ws.size() < W_COUNT) h->ws.resize(W_COUNT);
    DBuf<double>& b = h->ws[id];
    if (!b.p) {
        size_t n = 0;
        const size_t odd = (size_t)h->nRm * h->nSm, even = (size_t)h->nRp * h->nS;
        if (id <= W_OG) n = odd;
        else if (id == W_CPART) n = (size_t)h->nRm * h->dNm * std::min(8, h->nSm);
        else if (id == W_CFIN) n = (size_t)h->nRm * h->dNm;
        else if (id <= W_BX) n = even;
        else n = (size_t)h->nc;
        b.alloc(n);
    }
    return b.p;
}

void cg_prepare(Handle* h, bool f32, hipStream_t s) {
    const size_t even = (size_t)h->nRp * h->nS;
    if (f32 ? !h->ell_v32.p : !h->ell_v64.p) {
        if (f32) {
            h->ell_v32.alloc(h->ell_len * h->nS);
            h->ell_dinv32.alloc(even);
            k::cg_fill_values(h, h->ell_e.p, h->ell_len, h->ell_v32.p, s);
            k::cg_fill_dinv(h->diagE0.p, even, h->ell_dinv32.p, s);
        } else {
            h->ell_v64.alloc(h->ell_len * h->nS);
            h->ell_dinv64.alloc(even);
            k::cg_fill_values(h, h->ell_e.p, h->ell_len, h->ell_v64.p, s);
            k::cg_fill_dinv(h->diagE0.p, even, h->ell_dinv64.p, s);
        }
    }
    const size_t ntiles = ((size_t)h->nRp + 255) / 256;
    if (!h->cg_part.p) {
        h->cg_part.alloc(4 * (size_t)h->nS * ntiles);
        h->cg_scal.alloc(3 * (size_t)h->nS);
        h->cg_state.alloc((size_t)h->nS + 1);
    }
    if (h->cg_iters.n < (size_t)h->nS) h->cg_iters.alloc(h->nS);
}

// ----------------------------------------------------------------------------- timers
enum ProfKind { P_E0 = 0, P_GEMM = 1, P_GEMM_BF16 = 2, P_GEMM_SCATTER = 3, P_GEMM_SCATTER_F32 = 4 };

hipEvent_t take_event(Handle* h) {
    if (h->evpool.empty()) {
        hipEvent_t e;
        RTE_HIP(hipEventCreate(&e));
        return e;
    }
    hipEvent_t e = h->evpool.back();
    h->evpool.pop_back();
    return e;
}

// RAII: records an event pair around the enclosed launches when profiling is on
struct Timed {
    Handle* h;
    hipStream_t s;
    int kind;
    double flops;
    hipEvent_t a = nullptr;
    Timed(Handle* h_, hipStream_t s_, int kind_, double flops_ = 0) : h(h_), s(s_), kind(kind_), flops(flops_) {
        if (h->prof_on) {
            a = take_event(h);
            RTE_HIP(hipEventRecord(a, s));
        }
    }
    ~Timed() {
        if (a) {
            hipEvent_t b = take_event(h);
            (void)hipEventRecord(b, s);
            h->prof.push_back({kind, a, b, flops});
        }
    }
};

void gemm(Handle* h, int M, int N, int K, const double* A, int lda, const double* B, int ldb, double* C, int ldc,
          hipStream_t s) {
    Timed t(h, s, P_GEMM, 2.0 * M * N * (double)K);
    k::gemm_f64(M, N, K, 1.0, A, lda, B, ldb, 0.0, C, ldc, s);
}

void collect_profile(Handle* h, rte_solve_info* inf) {
    for (auto& r : h->prof) {
        float ms = 0.f;
        RTE_HIP(hipEventSynchronize(r.b));
        RTE_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        if (r.kind == P_E0) { inf->t_e0inv += ms * 1e-3; inf->n_e0inv += 1; }
        else if (r.kind == P_GEMM) { inf->t_gemm += ms * 1e-3; inf->n_gemm += 1; inf->gemm_flops += r.flops; }
        else if (r.kind == P_GEMM_SCATTER) {
            inf->t_scatter += ms * 1e-3;
            inf->n_scatter += 1;
            inf->scatter_flops += r.flops;
        }
        else if (r.kind == P_GEMM_SCATTER_F32) {
            inf->t_scatter_f32 += ms * 1e-3;
            inf->n_scatter_f32 += 1;
            inf->scatter_f32_flops += r.flops;
        }
        else { inf->t_gemm_bf16 += ms * 1e-3; inf->n_gemm_bf16 += 1; inf->gemm_bf16_flops += r.flops; }
        h->evpool.push_back(r.a);
        h->evpool.push_back(r.b);
    }
    h->prof.clear();
}

double read_scalar(Handle* h, int slot, hipStream_t s) {
    RTE_HIP(hipMemcpyAsync(h->pinned, h->scal.p + slot, sizeof(double), hipMemcpyDeviceToHost, s));
    RTE_HIP(hipStreamSynchronize(s));
    return h->pinned[0];
}

double dot_dev(Handle* h, const double* x, const double* y, size_t n, int slot, hipStream_t s) {
    k::dot(x, y, n, h->red.p, s);
    k::reduce(h->red.p, h->scal.p, slot, s);
    return read_scalar(h, slot, s);
}

// ----------------------------------------------------------------------------- odd solves
// (M- - K-) Z = B by PCG preconditioned with (M- - K-_N)^{-1} (Alg. 1, lemma of Sec. 5.1).
int odd_pcg(Handle* h, const double* B, double* Z, double tol, int maxit, hipStream_t s) {
    const size_t n = (size_t)h->nRm * h->nSm;
    double* R = ws(h, W_OR);
    double* P = ws(h, W_OP);
    double* W = ws(h, W_OW);
    double* Y = ws(h, W_OY);
    double* G = ws(h, W_OG);
    double* Cp = ws(h, W_CPART);
    double* Cf = ws(h, W_CFIN);
    k::fill(Z, 0.0, n, s);
    const double bb = dot_dev(h, B, B, n, S_BB, s);
    if (!std::isfinite(bb)) fail(RTE_E_NONFINITE, "non-finite right-hand side in the odd solve");
    if (bb == 0.0) return 0;
    k::copy(B, R, n, s);
    // projections of r onto the truncated eigenbasis: pcg_update with a = 0 computes them
    k::fill(h->scal.p + S_ALPHA, 0.0, 1, s);
    k::pcg_update(h, Z, R, R, R, h->scal.p, S_ALPHA, Cp, h->red.p, s);
    int rz = S_RZ0, rzn = S_RZ1;
    k::odd_precond(h, R, Cp, Cf, Y, h->red.p, s);
    k::reduce(h->red.p, h->scal.p, rz, s);
    k::copy(Y, P, n, s);
    int it = 0;
    const double stop = tol * tol * bb;
    while (it < maxit) {
        gemm(h, h->nRm, h->nSm, h->nSm, P, h->nRm, h->Sm.p, h->nSm, G, h->nRm, s);
        k::odd_apply(h, P, G, W, h->red.p, s);
        k::reduce(h->red.p, h->scal.p, S_PW, s);
        k::sdiv(h->scal.p, S_ALPHA, rz, S_PW, s);
        k::pcg_update(h, Z, R, P, W, h->scal.p, S_ALPHA, Cp, h->red.p, s);
        k::reduce(h->red.p, h->scal.p, S_RR, s);
        ++it;
        const double rr = read_scalar(h, S_RR, s);
        if (!std::isfinite(rr)) fail(RTE_E_NONFINITE, "non-finite residual in the odd PCG");
        if (rr <= stop) break;
        k::odd_precond(h, R, Cp, Cf, Y, h->red.p, s);
        k::reduce(h->red.p, h->scal.p, rzn, s);
        k::sdiv(h->scal.p, S_BETA, rzn, rz, s);
        k::xpby(Y, P, h->scal.p, S_BETA, n, s);
        std::swap(rz, rzn);
    }
    return it;
}

// (M- - K-) Z = B exactly via the eigen-decomposition of (S-, M_S-).
void odd_exact(Handle* h, const double* B, double* Z, hipStream_t s) {
    const int nRm = h->nRm, nSm = h->nSm;
    if (h->uniform_delta) {
        double* G = ws(h, W_OG);
        gemm(h, nRm, nSm, nSm, B, nRm, h->Hodd.p, nSm, G, nRm, s);
        k::row_scale_inv_mt(h, G, Z, nSm, s);
    } else {
        double* C = ws(h, W_OG);
        gemm(h, nRm, nSm, nSm, B, nRm, h->Wfull.p, nSm, C, nRm, s);
        k::scale_eigbasis(h, C, s);
        gemm(h, nRm, nSm, nSm, C, nRm, h->WfullT.p, nSm, Z, nRm, s);
    }
}

// Y = E X  [- Ms+ G - q]   (Alg. 1; G and q optional)
// lowp: reduced precision (the condensed transport GEMM in BF16 with FP32 accumulation)
void apply_E_core(Handle* h, const rte_solve_opts* o, const double* X, const double* G,
                  const double* q, double* Y, double tol, hipStream_t s, int64_t* pcg, bool lowp) {
    double* B = ws(h, W_OB);
    double* Z = ws(h, W_OZ);
    if (o->odd_solver == RTE_ODD_CONDENSED) {
        if (!h->Gc.p) fail(RTE_E_ARG, "the condensed odd solve needs a uniform sigma_s / sigma_t");
        const int dn = h->d * h->nS;
        if (lowp) {
            if (!h->have_mixed) fail(RTE_E_ARG, "mixed precision needs a handle assembled with mixed != 0");
            uint16_t* Ycb = reinterpret_cast<uint16_t*>(B);
            float* Zf = reinterpret_cast<float*>(Z);
            k::apply_grad_bf16(h, X, Ycb, s);
            {
                Timed t(h, s, P_GEMM_BF16, 2.0 * h->nRm * (double)dn * dn);
                // Z^T = G_off Y^T (G symmetric): Z comes out row-major (cell-major, directions
                // contiguous); the diagonal blocks of G are added by the A^T kernel
                k::gemm_bf16(dn, h->nRm, dn, 1.0f, h->Gc_bf.p, dn, Ycb, dn, 0.0f, Zf, dn, s);
            }
            k::apply_At_E_rm_f32(h, Zf, X, G, q, Y, s);
            return;
        }
        k::apply_grad(h, X, B, s);
        // Z^T = G Yc^T (G symmetric): Z comes out row-major (cell-major, directions contiguous)
        gemm(h, dn, h->nRm, dn, h->Gc.p, dn, B, h->nRm, Z, dn, s);
        k::apply_At_E_rm(h, Z, X, G, q, Y, s);
        return;
    }
    k::apply_A(h, X, B, s);
    if (o->odd_solver == RTE_ODD_EXACT) {
        odd_exact(h, B, Z, s);
    } else {
        if (!h->have_odd_eig) fail(RTE_E_ARG, "the PCG odd solve needs the odd eigenpairs (assembly with odd_eig = 1)");
        const int it = odd_pcg(h, B, Z, tol, o->pcg_max_iter, s);
        if (pcg) *pcg += it;
    }
    k::apply_At_E(h, Z, X, G, q, Y, s);
}

// Y = (E - K+) X - q0 with q0 = q (residual) or any vector (nullable)
void residual_like(Handle* h, const rte_solve_opts* o, const double* X, const double* q0, double* Y,
                   double tol, hipStream_t s, int64_t* pcg, bool lowp) {
    double* G = ws(h, W_EG);
    // the odd workspace is free until apply_E_core: scratch for the GEMM's split last round
    double* scratch = ws(h, W_OZ);
    const size_t nscratch = (size_t)h->nRm * h->nSm;
    const double flops = 2.0 * h->nRp * (double)h->nS * h->nS;
    if (lowp) {
        // inside the preconditioner: FP32 MFMA arithmetic on the FP32 copy of S+
        if (!h->Sp_f.p) fail(RTE_E_ARG, "mixed precision needs a handle assembled with mixed != 0");
        Timed t(h, s, P_GEMM_SCATTER_F32, flops);
        k::gemm_f32(h->nRp, h->nS, h->nS, 1.0f, X, h->nRp, h->Sp_f.p, h->nS, 0.0f, G, h->nRp, s,
                    reinterpret_cast<float*>(scratch), 2 * nscratch);
    } else {
        Timed t(h, s, P_GEMM_SCATTER, flops);
        k::gemm_f64(h->nRp, h->nS, h->nS, 1.0, X, h->nRp, h->Sp.p, h->nS, 0.0, G, h->nRp, s, scratch, nscratch);
    }
    apply_E_core(h, o, X, G, q0, Y, tol, s, pcg, lowp);
}

// the per-precision data of the multigrid hierarchy: values of levels 1.., inverse diagonals
// and Chebyshev intervals of every level, the cycle's work vectors (built once)
void mg_prepare(Handle* h, bool f32, hipStream_t s) {
    if (!h->mg_m || h->mgl.empty())
        fail(RTE_E_ARG, "e0_solver RTE_E0_MG needs a handle assembled with e0_solver = RTE_E0_MG");
    if ((int)h->mgl.size() > k::kMgMaxLevels) fail(RTE_E_ARG, "multigrid: too many levels");
    cg_prepare(h, f32, s);
    const size_t nS = (size_t)h->nS;
    const int L = (int)h->mgl.size();
    bool fresh = false;
    for (int l = 0; l < L; ++l) {
        Handle::MgLevel& g = h->mgl[l];
        if (f32 ? !g.dinv32.p : !g.dinv64.p) {
            fresh = true;
            // the smoother's values: BF16 for FP32 vectors, FP32 for FP64 vectors; level 0 by
            // rounding the CG's values, coarse levels from their class values
            const size_t len = l == 0 ? h->ell_len : g.len;
            if (f32) {
                g.s16.alloc(nS * len);
                if (l == 0) k::mg_round(h->ell_v32.p, g.s16.p, nS * len, s);
                else k::mg_fill_smoother(h->nS, len, g.nnz, h->ncls, g.e.p, g.cls.p, h->coefE0.p, g.s16.p, s);
            } else {
                g.s32.alloc(nS * len);
                if (l == 0) k::mg_round(h->ell_v64.p, g.s32.p, nS * len, s);
                else k::mg_fill_smoother(h->nS, len, g.nnz, h->ncls, g.e.p, g.cls.p, h->coefE0.p, g.s32.p, s);
            }
            if (f32) {
                g.dinv32.alloc(nS * g.n);
                g.cheb32.alloc(2 * nS * (1 + rte::kMgChebSteps));
            } else {
                g.dinv64.alloc(nS * g.n);
                g.cheb64.alloc(2 * nS * (1 + rte::kMgChebSteps));
            }
        }
        if (!g.work.p) g.work.alloc(5 * (size_t)g.n * nS * sizeof(double));
    }
    if (fresh) {
        const k::MgArgs a = mg_args(h, f32);
        DBuf<double> part(nS * (((size_t)h->mgl[0].n + 255) / 256));
        for (int l = 0; l < L; ++l) k::mg_level_setup(a, l, l == L - 1 ? k::kMgLoCoarse : k::kMgLo, part.p, s);
        RTE_HIP(hipStreamSynchronize(s));
    }
}

k::MgArgs mg_args(Handle* h, bool f32) {
    k::MgArgs a;
    a.d = h->d;
    a.nS = h->nS;
    a.L = (int)h->mgl.size();
    a.f32 = f32;
    for (int l = 0; l < a.L; ++l) {
        Handle::MgLevel& g = h->mgl[l];
        k::MgLevelArgs& A = a.lev[l];
        A.m = g.m;
        A.n = g.n;
        if (l == 0) {
            A.nslice = h->ell_nslice;
            A.wmax = h->ell_wmax;
            A.len = h->ell_len;
            A.sptr = h->ell_sptr.p;
            A.col = h->ell_col.p;
        } else {
            A.nslice = g.nslice;
            A.wmax = g.wmax;
            A.len = g.len;
            A.sptr = g.sptr.p;
            A.col = g.col.p;
        }
        A.val = f32 ? static_cast<const void*>(g.s16.p) : static_cast<const void*>(g.s32.p);
        A.dinv = f32 ? static_cast<const void*>(g.dinv32.p) : static_cast<const void*>(g.dinv64.p);
        A.cheb = f32 ? g.cheb32.p : g.cheb64.p;
        const size_t vb = (size_t)g.n * h->nS * (f32 ? sizeof(float) : sizeof(double));
        unsigned char* w = g.work.p;
        A.x = w;
        A.r = w + vb;
        A.b = w + 2 * vb;
        A.d0 = w + 3 * vb;
        A.d1 = w + 4 * vb;
    }
    return a;
}

k::CgJob cg_job(Handle* h, const rte_solve_opts* o, const double* X, double* Y, bool lowp, hipStream_t s,
                k::MgArgs* mg) {
    const bool f32 = lowp;
    if (o->e0_solver == RTE_E0_MG) {
        if (!mg) fail(RTE_E_ARG, "multigrid CG without room for its arguments");
        mg_prepare(h, f32, s);
        *mg = mg_args(h, f32);
    }
    cg_prepare(h, f32, s);
    k::CgJob j;
    k::CgArgs& a = j.a;
    a.n = h->nRp;
    a.nS = h->nS;
    a.nslice = h->ell_nslice;
    a.len = h->ell_len;
    a.wmax = h->ell_wmax;
    a.sptr = h->ell_sptr.p;
    a.col = h->ell_col.p;
    a.B = X;
    a.X = Y;
    a.tol = f32 ? std::max(o->cg_tol, 1e-6) : o->cg_tol;
    a.maxit = o->cg_max_iter;
    a.part = h->cg_part.p;
    a.rz = h->cg_scal.p;
    a.stop = h->cg_scal.p + 2 * (size_t)h->nS;
    a.done = h->cg_state.p;
    a.active = h->cg_state.p + h->nS;
    a.iters = h->cg_iters.p;
    a.host_active = reinterpret_cast<int*>(h->pinned + 32);
    j.f32 = f32;
    j.val = f32 ? static_cast<const void*>(h->ell_v32.p) : static_cast<const void*>(h->ell_v64.p);
    j.dinv = f32 ? static_cast<const void*>(h->ell_dinv32.p) : static_cast<const void*>(h->ell_dinv64.p);
    j.R = ws(h, W_CGR);
    j.P = ws(h, W_CGP);
    j.Q = ws(h, W_CGQ);
    j.s = s;
    if (o->e0_solver == RTE_E0_MG) {
        j.mg = mg;
        j.a.check_every = 4;      // an iteration costs about five SpMVs: read the live count more often
    }
    return j;
}

void e0inv(Handle* h, const rte_solve_opts* o, const double* X, double* Y, hipStream_t s, int64_t* cgt,
           int* cgmax, bool lowp) {
    if (o->e0_solver == RTE_E0_BANDED) {
        if (!h->have_e0_banded) fail(RTE_E_ARG, "banded E_0 factors were not prepared at assembly");
        if (!(lowp && h->L0f.p) && !h->L0.p)
            fail(RTE_E_ARG, "the FP64 band factors were dropped at assembly (mixed = 2)");
        // the factors are in band order: unless that is the given vertex order, permute the
        // columns of X into it and the solution back in coalesced per-column passes, so that
        // the solve itself reads and writes its vectors contiguously (gathering through the
        // permutation inside the solve is slower than the two passes)
        if (h->perm_identity && X != Y) {
            Timed t(h, s, P_E0);
            if (lowp && h->L0f.p)
                k::band_solve_blk_f32(h->L0f.p, h->L0Uf.p, h->nRp, h->sbw, h->nS, h->e0_stride32, X, Y,
                                      (size_t)h->nRp, nullptr, s, h->e0_g32);
            else
                k::band_solve_blk(h->L0.p, h->L0U.p, h->nRp, h->sbw, h->nS, h->e0_stride, X, Y, (size_t)h->nRp,
                                  nullptr, s, h->e0_g64);
            return;
        }
        double* Xb = ws(h, W_BB);
        double* Yb = ws(h, W_BX);
        k::permute_cols(h->iperm.p, h->nRp, h->nS, X, Xb, true, s);
        {
            Timed t(h, s, P_E0);
            if (lowp && h->L0f.p)
                k::band_solve_blk_f32(h->L0f.p, h->L0Uf.p, h->nRp, h->sbw, h->nS, h->e0_stride32, Xb, Yb,
                                      (size_t)h->nRp, nullptr, s, h->e0_g32);
            else
                k::band_solve_blk(h->L0.p, h->L0U.p, h->nRp, h->sbw, h->nS, h->e0_stride, Xb, Yb, (size_t)h->nRp,
                                  nullptr, s, h->e0_g64);
        }
        k::permute_cols(h->iperm.p, h->nRp, h->nS, Yb, Y, false, s);
        return;
    }
    // CG on every direction block at once (kernels_cg.hip), Jacobi- or multigrid-preconditioned
    // (kernels_mg.hip); in mixed precision its vectors and block values are FP32 (dot products
    // FP64) and it stops at a relative residual of max(cg_tol, 1e-6), the FP32 floor of a
    // preconditioner solve
    k::MgArgs g;
    k::CgJob j = cg_job(h, o, X, Y, lowp, s, &g);
    DBuf<int>& iters = h->cg_iters;
    {
        Timed t(h, s, P_E0);
        std::vector<k::CgJob> one{j};
        k::cg_solve_many(one);
    }
    if (cgt || cgmax) {
        std::vector<int> hi(h->nS);
        RTE_HIP(hipMemcpyAsync(hi.data(), iters.p, h->nS * sizeof(int), hipMemcpyDeviceToHost, s));
        RTE_HIP(hipStreamSynchronize(s));
        for (int v : hi) {
            if (cgt) *cgt += v;
            if (cgmax) *cgmax = std::max(*cgmax, v);
        }
    }
}

// z = l steps of CG on E z = r preconditioned by E_0, from z_0 = 0 (the non-stationary
// alternative to P_1^l named in Sec. 5.3).  Inner products are FP64 fixed-order
// reductions into device scalars; alpha = gamma / p.Ep and beta = gamma' / gamma are formed
// on the device (0 when the denominator is 0, so r = 0 gives z = 0), so the l steps run
// without a host synchronisation.  The last step's residual update and E_0 solve are not
// needed for z and are skipped.
void apply_P1_pcg(Handle* h, const rte_solve_opts* o, const double* r, double* z, hipStream_t s,
                  int64_t* pcg, int64_t* cgt, int* cgmax, bool lowp) {
    const size_t n = (size_t)h->nRp * h->nS;
    double* res = ws(h, W_IR);
    double* y = ws(h, W_IY);
    double* p = ws(h, W_IP);
    double* q = ws(h, W_IQ);
    double* scal = h->scal.p;
    k::fill(z, 0.0, n, s);
    k::copy(r, res, n, s);
    e0inv(h, o, res, y, s, cgt, cgmax, lowp);
    int g = S_IG0, gn = S_IG1;
    k::dot(res, y, n, h->red.p, s);
    k::reduce(h->red.p, scal, g, s);
    k::xpby(y, p, scal, -1, n, s);                                  // p = y
    for (int i = 0; i < o->l; ++i) {
        apply_E_core(h, o, p, nullptr, nullptr, q, o->pcg_tol_inner, s, pcg, lowp);   // q = E p
        k::dot(p, q, n, h->red.p, s);
        k::reduce(h->red.p, scal, S_IPQ, s);
        k::sdiv(scal, S_IALPHA, g, S_IPQ, s);
        k::axpy_s(z, z, p, scal, S_IALPHA, 1.0, n, s);              // z += alpha p
        if (i + 1 == o->l) break;
        k::axpy_s(res, res, q, scal, S_IALPHA, -1.0, n, s);         // res -= alpha q
        e0inv(h, o, res, y, s, cgt, cgmax, lowp);
        k::dot(res, y, n, h->red.p, s);
        k::reduce(h->red.p, scal, gn, s);
        k::sdiv(scal, S_IBETA, gn, g, s);
        k::xpby(y, p, scal, S_IBETA, n, s);                         // p = y + beta p
        std::swap(g, gn);
    }
}

// z = P_1^l r  (Alg. 2 with l steps; z_0 = 0 so the first step is E_0^{-1} r), or the inner
// PCG above
void apply_P1(Handle* h, const rte_solve_opts* o, const double* r, double* z, hipStream_t s,
              int64_t* pcg, int64_t* cgt, int* cgmax, bool lowp) {
    if (o->inner == RTE_INNER_PCG) {
        apply_P1_pcg(h, o, r, z, s, pcg, cgt, cgmax, lowp);
        return;
    }
    const size_t n = (size_t)h->nRp * h->nS;
    double* t = ws(h, W_ET2);
    double* t2 = ws(h, W_EZ);
    e0inv(h, o, r, z, s, cgt, cgmax, lowp);
    for (int i = 1; i < o->l; ++i) {
        apply_E_core(h, o, z, nullptr, r, t, o->pcg_tol_inner, s, pcg, lowp);   // t = E z - r
        e0inv(h, o, t, t2, s, cgt, cgmax, lowp);
        k::axpby(-1.0, t2, 1.0, z, n, s);
    }
}

// the correction's right-hand side q_c = W^T ((E - K+) s - r) into W_CRHS (Sec. 5.4; without
// Alg. 3's extra "-q", which would move the fixed point)
void correction_rhs(Handle* h, const rte_solve_opts* o, const double* r, const double* sv, hipStream_t s,
                    int64_t* pcg, bool lowp) {
    double* t = ws(h, W_ET);
    residual_like(h, o, sv, r, t, o->pcg_tol_inner, s, pcg, lowp);
    k::coarse_project(h, t, ws(h, W_CRHS), s);
}

// u_c = E_c^{-1} q_c: W_CRHS -> W_CSOL by the handle's coarse solver
void coarse_solve(Handle* h, hipStream_t s) {
    const double* rhs = ws(h, W_CRHS);
    double* uc = ws(h, W_CSOL);
    if (h->Ecinv.p) k::gemv_rows(h->nc, h->Ecinv.p, rhs, uc, s);
    else if (h->cnb) coarse_block_solve(h, rhs, uc, s);
    else k::band_solve_blk(h->Lc.p, h->LcU.p, h->nc, h->cbw, 1, 0, rhs, uc, 0, nullptr, s);
}

// step = -s + W u_c
void correction_finish(Handle* h, const double* sv, double* step, hipStream_t s) {
    k::fill(step, 0.0, (size_t)h->nRp * h->nS, s);
    k::richardson_update(h, step, sv, ws(h, W_CSOL), s);
}

// step = -s + W E_c^{-1} W^T ((E - K+) s - r)   (Sec. 5.4)
void correction_step(Handle* h, const rte_solve_opts* o, const double* r, const double* sv, double* step,
                     hipStream_t s, int64_t* pcg, bool lowp) {
    correction_rhs(h, o, r, sv, s, pcg, lowp);
    coarse_solve(h, s);
    correction_finish(h, sv, step, s);
}

bool stall_step(const rte_solve_opts* o, double en, double& en_prev, int& stall) {
    if (o->stall_iters <= 0 || en < 0.0) return false;
    if (en_prev > 0.0) stall = en > o->stall_ratio * en_prev ? stall + 1 : 0;
    en_prev = en;
    return stall >= o->stall_iters;
}

}  // namespace sv

using namespace sv;

void apply_E(Handle* h, const rte_solve_opts* o, const double* X, double* Y, hipStream_t s, int64_t* pcg) {
    apply_E_core(h, o, X, nullptr, nullptr, Y, o->pcg_tol_resid, s, pcg, o->precision == RTE_MIXED);
}

void apply_E0(Handle* h, const double* X, double* Y, hipStream_t s) {
    cg_prepare(h, false, s);
    k::CgArgs a;
    a.n = h->nRp;
    a.nS = h->nS;
    a.nslice = h->ell_nslice;
    a.len = h->ell_len;
    a.wmax = h->ell_wmax;
    a.sptr = h->ell_sptr.p;
    a.col = h->ell_col.p;
    a.part = h->cg_part.p;
    k::cg_spmv(a, h->ell_v64.p, X, Y, s);
}

void apply_mg(Handle* h, const double* X, double* Y, hipStream_t s) {
    mg_prepare(h, false, s);
    k::mg_apply(mg_args(h, false), X, Y, s);
}

void apply_E0inv(Handle* h, const rte_solve_opts* o, const double* X, double* Y, hipStream_t s,
                 int64_t* cgt, int* cgmax) {
    e0inv(h, o, X, Y, s, cgt, cgmax, o->precision == RTE_MIXED);
}

void precond(Handle* h, const rte_solve_opts* o, int which, const double* r, double* out, hipStream_t s) {
    const size_t n = (size_t)h->nRp * h->nS;
    if (which == 0) {
        apply_P1(h, o, r, out, s, nullptr, nullptr, nullptr, o->precision == RTE_MIXED);
        return;
    }
    double* sv = ws(h, W_ES);
    apply_P1(h, o, r, sv, s, nullptr, nullptr, nullptr, o->precision == RTE_MIXED);
    correction_step(h, o, r, sv, out, s, nullptr, o->precision == RTE_MIXED);   // out = -s + W uc
    k::axpby(0.0, out, -1.0, out, n, s);             // P2 P1 r = s - W uc
}

rte_status solve(Handle* h, const rte_solve_opts* o, const double* U0, double* U, double* U_odd,
                 rte_solve_info* info, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const size_t n = (size_t)h->nRp * h->nS;
    rte_solve_info inf{};
    const bool lowp = o->precision == RTE_MIXED;   // preconditioner precision; the residual stays FP64
    h->prof_on = o->profile != 0;
    h->prof.clear();
    double* r = ws(h, W_ER);
    double* sv = ws(h, W_ES);
    double* step = ws(h, W_ESTEP);
    if (U0) k::copy(U0, U, n, s);
    else k::fill(U, 0.0, n, s);
    double e1 = -1.0, step_rprev = 0.0, en_prev = -1.0;
    bool have_step = false;
    int stall = 0;
    rte_status st = RTE_E_NOTCONV;
    int it = 0;
    for (;;) {
        residual_like(h, o, U, h->q.p, r, o->pcg_tol_resid, s, &inf.pcg_iters_total, false);   // FP64 always
        const double rr = dot_dev(h, r, r, n, S_DOT0, s);
        if (!std::isfinite(rr)) { st = RTE_E_NONFINITE; break; }
        inf.rel_resid = std::sqrt(rr) / h->qnorm;
        double en = -1.0;
        if (have_step) {
            // ||u_n - u_{n-1}||^2_{E-K} = step^T (r_n - r_{n-1})
            const double sr = dot_dev(h, step, r, n, S_DOT1, s);
            en = std::sqrt(std::max(sr - step_rprev, 0.0));
            if (e1 < 0) e1 = en;
            inf.stop_quantity = e1 > 0 ? en / e1 : 0.0;
        }
        if (inf.rel_resid <= o->tol) { st = RTE_OK; break; }
        if (it >= o->max_iter) { st = RTE_E_NOTCONV; break; }
        if (stall_step(o, en, en_prev, stall)) { st = RTE_E_STALL; break; }
        apply_P1(h, o, r, sv, s, &inf.pcg_iters_total, &inf.cg_iters_total, &inf.cg_iters_max, lowp);
        correction_step(h, o, r, sv, step, s, &inf.pcg_iters_total, lowp);
        step_rprev = dot_dev(h, step, r, n, S_DOT2, s);
        have_step = true;
        k::axpby(1.0, step, 1.0, U, n, s);
        ++it;
    }
    if (U_odd) {
        // the odd part from the second row of the mixed system (Sec. 2.6, eq. mixed_discrete):
        // A u+ + (M- - K-) u- = l- = 0 for an isotropic source, so u- = -(M- - K-)^{-1} A u+
        double* B = ws(h, W_OB);
        k::apply_A(h, U, B, s);
        odd_exact(h, B, U_odd, s);
        const size_t nodd = (size_t)h->nRm * h->nSm;
        k::axpby(0.0, U_odd, -1.0, U_odd, nodd, s);
    }
    RTE_HIP(hipStreamSynchronize(s));
    collect_profile(h, &inf);
    h->prof_on = false;
    inf.iters = it;
    inf.t_solve = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return st;
}

}  // namespace rte
