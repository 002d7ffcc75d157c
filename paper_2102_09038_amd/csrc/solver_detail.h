// Internal pieces of the Richardson solver shared by the single-instance solve
// (solver.cpp) and the lockstep batch (solver_batch.cpp).
#pragma once
#include "ops.h"

namespace rte {
namespace sv {

// device scalar slots of a handle (Handle::scal)
enum Slot { S_BB = 0, S_PW, S_ALPHA, S_RR, S_RZ0, S_RZ1, S_BETA, S_DOT0, S_DOT1, S_DOT2,
            // the inner PCG of P_1: two alternating gammas, p.Ep, alpha, beta
            S_IG0, S_IG1, S_IPQ, S_IALPHA, S_IBETA };

// workspace buffers of a handle (allocated on first use)
enum WsId {
    // odd workspace (nRm x nSm)
    W_OB = 0, W_OZ, W_OR, W_OP, W_OW, W_OY, W_OG,
    // thin odd workspace
    W_CPART, W_CFIN,
    // even workspace (nRp x nS)
    W_EG, W_ET, W_ER, W_ES, W_ESTEP, W_EZ, W_ET2, W_CGR, W_CGP, W_CGQ,
    // the inner PCG of P_1: residual, preconditioned residual, direction, E times direction
    W_IR, W_IY, W_IP, W_IQ,
    // right-hand side and solution of the band solves in band order
    W_BB, W_BX,
    // coarse
    W_CRHS, W_CSOL,
    W_COUNT
};

double* ws(Handle* h, int id);
// the stagnation test of rte_solve_opts on the energy-norm step en of this iteration (< 0 before
// the first step): true once the step has failed to shrink by stall_ratio stall_iters times in
// a row; en_prev and stall carry the state between iterations
bool stall_step(const rte_solve_opts* o, double en, double& en_prev, int& stall);
// the explicit E_0 block values and inverse diagonals of the CG solve, FP64 or FP32 (built once)
void cg_prepare(Handle* h, bool f32, hipStream_t s);
// Y = E X [- q0] (q0 nullable), or with G = X S+ given: Y = (E - K+) X - q0  (Alg. 1)
void apply_E_core(Handle* h, const rte_solve_opts* o, const double* X, const double* G, const double* q0, double* Y,
                  double tol, hipStream_t s, int64_t* pcg, bool lowp);
// the CG solve Y = E_0^{-1} X of a handle (its arguments and buffers, on stream s); lowp: FP32
// vectors and block values, stopping at a relative residual of max(cg_tol, 1e-6).  With
// o->e0_solver == RTE_E0_MG the multigrid preconditioner's arguments go to *mg, which must
// outlive the solve
k::CgJob cg_job(Handle* h, const rte_solve_opts* o, const double* X, double* Y, bool lowp, hipStream_t s,
                k::MgArgs* mg);
// the multigrid hierarchy's per-precision data (built once) and its launch arguments
void mg_prepare(Handle* h, bool f32, hipStream_t s);
k::MgArgs mg_args(Handle* h, bool f32);
// Y = E_0^{-1} X by the handle's banded factors or its CG (o->e0_solver); lowp: FP32 factors / CG
void e0inv(Handle* h, const rte_solve_opts* o, const double* X, double* Y, hipStream_t s, int64_t* cgt,
           int* cgmax, bool lowp);
// Y = (E - K+) X - q0 (FP64 scatter GEMM, then apply_E_core)
void residual_like(Handle* h, const rte_solve_opts* o, const double* X, const double* q0, double* Y, double tol,
                   hipStream_t s, int64_t* pcg, bool lowp);
// the correction in three parts (a batch groups the coarse band solves of its slots):
// q_c = W^T ((E - K+) s - r) into W_CRHS; u_c = E_c^{-1} q_c into W_CSOL; step = -s + W u_c
void correction_rhs(Handle* h, const rte_solve_opts* o, const double* r, const double* sv, hipStream_t s,
                    int64_t* pcg, bool lowp);
void coarse_solve(Handle* h, hipStream_t s);
void correction_finish(Handle* h, const double* sv, double* step, hipStream_t s);
// step = -s + W E_c^{-1} W^T ((E - K+) s - r)   (Sec. 5.4)
void correction_step(Handle* h, const rte_solve_opts* o, const double* r, const double* sv, double* step,
                     hipStream_t s, int64_t* pcg, bool lowp);

}  // namespace sv
}  // namespace rte
