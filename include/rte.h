/*
 * rte.h - C ABI of librte, an MI355X (gfx950) solver for the even-parity
 * discretisation of the anisotropic radiative transfer equation by the
 * preconditioned Richardson iteration of Doelz, Palii and Schlottbom,
 * "On robustly convergent and efficient iterative methods for anisotropic
 * radiative transfer" (arXiv:2102.09038).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - No C++ exception crosses this boundary.  Every function returns an
 *   rte_status; RTE_OK is 0.  On failure rte_last_error() returns a
 *   thread-local description of the last non-OK status.
 * - Pointers named host_* or passed in rte_problem_desc are host memory.
 *   Pointers documented as "device" are HIP device memory owned by the caller;
 *   the library never frees them and never keeps them after the call returns.
 * - hip_stream is a hipStream_t (NULL = the default stream).  Device work is
 *   enqueued on it; calls documented as blocking also synchronise it.
 * - Even-space vectors are n_R+ x n_S+ matrices U (column-major, spatial index
 *   fastest: U[i + n_R+ * k]); vec(U) stacks the columns (Sec. 4).
 *   Odd-space vectors are n_R- x n_S- matrices, n_S- = 3 n_S+, odd column
 *   3k + m holds the coefficient of psi_(k,m) = s_m mu_k.
 * - The even angular index k is the order, in desc->stri, of the triangles
 *   whose centroid lies in the upper half-sphere (z > 0; ties broken on y,
 *   then x).  Every such triangle must have its antipode in the mesh.
 * - All floating-point inputs are FP64.
 */
#ifndef RTE_H
#define RTE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rte_status {
    RTE_OK = 0,
    RTE_E_ARG = 1,        /* invalid pointer, size, option or descriptor field        */
    RTE_E_PHYS = 2,       /* sigma_t <= 0, sigma_s < 0, max sigma_s/sigma_t >= 1, g not in [0,1) */
    RTE_E_MESH = 3,       /* degenerate simplex, non-antipodal sphere mesh, bad index */
    RTE_E_NOMEM = 4,      /* device allocation failed                                 */
    RTE_E_HIP = 5,        /* a HIP / rocSOLVER call failed                             */
    RTE_E_NOTCONV = 6,    /* iteration cap reached; the last iterate is returned      */
    RTE_E_NONFINITE = 7,  /* a residual became NaN or Inf                              */
    RTE_E_STALL = 8       /* the iteration stopped contracting (rte_solve_opts.stall_*);
                             the last iterate is returned                              */
} rte_status;

typedef enum rte_precision {
    RTE_FP64 = 0,         /* every step in FP64                                        */
    RTE_MIXED = 1         /* inside the preconditioner: condensed transport GEMM with BF16
                             inputs and FP32 accumulation (the operator's nearly singular
                             d x d diagonal blocks applied exactly in FP64 beside it),
                             scatter GEMM in FP32 MFMA, E_0 factors (or CG vectors) FP32;
                             outer residual, all dot products and the coarse solve FP64 */
} rte_precision;

typedef enum rte_dtype { RTE_DT_F64 = 0, RTE_DT_F32 = 1, RTE_DT_BF16 = 2 } rte_dtype;

/* How (M- - K-)^{-1} is applied inside E (Sec. 5.1, Alg. 1). */
typedef enum rte_odd_solver {
    RTE_ODD_PCG = 0,      /* PCG preconditioned by (M- - K-_N)^{-1} (Lemma in Sec. 5.1) */
    RTE_ODD_EXACT = 1,    /* exact: per-cell inverse through the full eigendecomposition
                             of (S-, M_S-); one GEMM when sigma_s/sigma_t is uniform,
                             two otherwise                                            */
    RTE_ODD_CONDENSED = 2 /* exact, condensed onto the d spatial directions: with a
                             uniform ratio delta, A^T (M- - K-)^{-1} A X =
                             sum_{n,n'} D_n^T Mt-^{-1} D_n' X G_{n'n}, where
                             G_{n'n} = A_n'^T (M_S- - delta S-)^{-1} A_n is precomputed
                             (one GEMM with N = K = d n_S+); RTE_E_ARG if the ratio
                             varies between cells                                    */
} rte_odd_solver;

/* How each block of E_0^{-1} is applied (Sec. 5.3). */
typedef enum rte_e0_solver {
    RTE_E0_CG = 0,        /* Jacobi-preconditioned CG on every direction block at once
                             (sliced-ELL storage, per-direction early exit); with
                             precision RTE_MIXED its vectors and values are FP32 (dot
                             products FP64) and it stops at max(cg_tol, 1e-6)          */
    RTE_E0_BANDED = 1,    /* banded Cholesky factors per direction, factored once      */
    RTE_E0_MG = 2         /* CG on every direction block at once, preconditioned by one
                             geometric multigrid V-cycle per iteration (Sec. 5.5 names
                             multigrid as the E_0 solver): lattice meshes only (the
                             Freudenthal triangulation of a box, vertex i + m (j + m k),
                             else RTE_E_ARG at assembly); nested lattices with the P1
                             interpolant, Galerkin coarse blocks, four Jacobi-scaled
                             Chebyshev steps before and after the coarse correction on
                             [0.02 lam, lam], lam = Gershgorin's bound of D^-1 E_0, eight
                             on the coarsest level on the same interval.  Levels are added
                             while the cells per axis are even and at least 4.  The cycle
                             reads the level matrices rounded to FP32 (FP64 solves) or BF16
                             (mixed solves); the CG's own products use the full-precision
                             E_0.  Precision and stopping as RTE_E0_CG; the hierarchy is
                             built at assembly (e0_solver = RTE_E0_MG)                */
} rte_e0_solver;

/* How P_1 approximates E^{-1} (Sec. 5.3).  The paper takes l steps of the preconditioned
 * Richardson iteration with E_0 and remarks that a non-stationary preconditioned conjugate
 * gradient method with the same E_0 does better. */
typedef enum rte_inner {
    RTE_INNER_RICHARDSON = 0, /* P_1^l (eq. applyP1, Alg. 2): z_0 = 0, z_{i+1} = z_i -
                                 E_0^{-1} (E z_i - r), l steps; a fixed SPD matrix (Lemma
                                 preconditioner_pl); l - 1 E and l E_0^{-1} applications */
    RTE_INNER_PCG = 1         /* l steps of CG on E z = r preconditioned by E_0, z_0 = 0:
                                 z_l is the E-orthogonal projection of E^{-1} r onto the
                                 Krylov space span{(E_0^{-1} E)^j E_0^{-1} r, j < l}, so
                                 its E-norm error is never larger than P_1^l r's; it
                                 depends on r nonlinearly.  l E and l E_0^{-1}
                                 applications; the step sizes stay on the device (no
                                 host synchronisation).  Four more even-sized FP64
                                 work vectors are allocated on first use.  Single
                                 solves only (the batch refuses it with RTE_E_ARG)    */
} rte_inner;

/* How the coarse system E_c u_c = q_c of the subspace correction is solved (Sec. 5.4). */
typedef enum rte_coarse_solver {
    RTE_COARSE_AUTO = 0,      /* the first of the three below that fits                      */
    RTE_COARSE_INVERSE = 1,   /* explicit E_c^{-1} (dense Cholesky and inverse on the device,
                                 once), applied as a matrix-vector product; needs n_c^2 * 8
                                 bytes <= 12 GiB                                             */
    RTE_COARSE_BAND = 2,      /* banded Cholesky (on the device when the half-bandwidth is
                                 <= 143, else on the host), the band solve on the device;
                                 needs the half-bandwidth d_N (b + 1) - 1 within the band
                                 solve's reach (b: spatial bandwidth)                        */
    RTE_COARSE_QUICK = 4,     /* for a short set-up (served requests): the band solve when its
                                 band fits the device band factorisation (half-bandwidth
                                 <= 143; set-up in milliseconds, about 3 ms per solve at
                                 16641 unknowns against 0.5 ms for the explicit inverse),
                                 else the block-tridiagonal Cholesky (a 32^3 lattice: 0.6 s
                                 and 5.8 GB per handle against 2.2 s and 14.9 GB for the
                                 explicit inverse, the same solve time)                  */
    RTE_COARSE_BLOCK = 3      /* block-tridiagonal Cholesky on the device (blocks of one
                                 half-bandwidth: dense factor, triangular solve and rank
                                 update per block, then inverses of the diagonal factors
                                 folded into the coupling blocks); a solve is two
                                 block-diagonal products and two chains of n_c / bw
                                 matrix-vector products (kernels of this library
                                 only, so a batch may capture them)                       */
} rte_coarse_solver;

typedef struct rte_handle rte_handle;   /* opaque; owns all device memory it allocates */

/* Problem statement (Sec. 1, RTE with Henyey-Greenstein scattering and vacuum or
 * inflow boundary; Sec. 2.2 parameter assumptions; Sec. 4 meshes).  Host pointers,
 * copied by rte_assemble; the caller may free them after it returns. */
typedef struct rte_problem_desc {
    int32_t dim;                 /* spatial dimension d, 2 or 3                              */
    int32_t n_vert;              /* number of spatial vertices (P1 dofs, n_R+)               */
    const double* vert;          /* [n_vert * dim] coordinates, vertex-major                 */
    int32_t n_cell;              /* number of simplices (P0 dofs, n_R-)                      */
    const int32_t* cell;         /* [n_cell * (dim+1)] vertex indices                        */
    const double* sigma_t;       /* [n_cell] total attenuation, > 0, piecewise constant      */
    const double* sigma_s;       /* [n_cell] scattering rate, 0 <= sigma_s < sigma_t         */
    double g;                    /* HG anisotropy factor, 0 <= g < 1                         */
    int32_t n_svert;             /* number of sphere-mesh vertices                           */
    const double* svert;         /* [n_svert * 3] unit vectors                               */
    int32_t n_stri;              /* number of sphere triangles (even, antipodally symmetric) */
    const int32_t* stri;         /* [n_stri * 3] vertex indices                              */
    const double* q_nodal;       /* [n_vert] isotropic volume source at the vertices; the
                                    even load is l+[:,k] = 2|K_k| (P1 mass) q_nodal          */
    const double* g_inflow;      /* must be NULL (vacuum boundary); reserved for inflow data */
} rte_problem_desc;

typedef struct rte_assemble_opts {
    int32_t quad_level;          /* each sphere triangle's flat image is cut into 4^quad_level
                                    parts with a 7-point degree-5 rule on each (0..6)        */
    int32_t n_even;              /* N+ >= 0: correction space = top (N+1)(N+2)/2 eigenvectors
                                    of (S+, M_S+)  (Sec. 5.4)                                */
    int32_t n_odd;               /* N- >= 1 odd: PCG preconditioner uses the top
                                    (N+1)(N+2)/2 eigenpairs of (S-, M_S-)  (Sec. 5.1)        */
    int32_t e0_solver;           /* rte_e0_solver prepared at assembly (CG is always there;
                                    BANDED and MG need it here)                              */
    int32_t mixed;               /* 1: also prepare BF16/FP32 operator copies; 2: the same,  */
                                 /*    and keep only the FP32 E_0 band factors (FP64 banded */
                                 /*    E_0 solves then fail with RTE_E_ARG; halves the      */
                                 /*    largest allocation for mixed-only use); with the CG  */
                                 /*    E_0 solver only the FP32 block values are built      */
    int32_t odd_eig;             /* 1 (default): eigendecomposition of (S-, M_S-) at assembly
                                    (every odd solver); 0: skipped when sigma_s / sigma_t is
                                    uniform, H = (M_S- - delta S-)^{-1} then comes from a
                                    product of this library's GEMMs, bitwise the same in every
                                    assembly (the exact and condensed odd solves work, the PCG
                                    odd solve fails with RTE_E_ARG; RTE_E_ARG at assembly if
                                    M_S- - delta S- is not positive definite); ignored (the
                                    decomposition is done) when the ratio varies             */
    int32_t coarse_solver;       /* rte_coarse_solver (default RTE_COARSE_AUTO); RTE_E_ARG if
                                    the chosen one does not fit                              */
} rte_assemble_opts;

typedef struct rte_solve_opts {
    int32_t l;                   /* inner Richardson steps of P_1^l (Sec. 5.3), >= 1          */
    double tol;                  /* stop when ||r_n||_2 <= tol ||q||_2                       */
    int32_t max_iter;            /* outer iteration cap                                      */
    int32_t precision;           /* rte_precision                                            */
    int32_t odd_solver;          /* rte_odd_solver                                           */
    int32_t e0_solver;           /* rte_e0_solver (BANDED needs it at assembly)              */
    double pcg_tol_resid;        /* relative PCG tolerance inside the residual's E           */
    double pcg_tol_inner;        /* relative PCG tolerance inside P_1 and the correction     */
    int32_t pcg_max_iter;        /* PCG iteration cap per E application                      */
    double cg_tol;               /* relative CG tolerance per E_0 block                      */
    int32_t cg_max_iter;         /* CG iteration cap per E_0 block                           */
    int32_t profile;             /* nonzero: time the E_0 solves and the scattering GEMMs with
                                    HIP events on hip_stream (rte_solve_info.t_*)            */
    int32_t inner;               /* rte_inner: how P_1 is applied                            */
    /* Stagnation test.  The error of the iteration contracts in the energy norm of E - K+ by
     * at least the factor c per step (Sec. 3; with the preconditioners of Sec. 5 the factor
     * is smaller), and so does the step ||u_{n+1} - u_n||_{E-K}.  With stall_iters > 0 the solve
     * stops with RTE_E_STALL once that step shrinks by less than the factor stall_ratio, i.e.
     * step_n > stall_ratio * step_{n-1}, on stall_iters consecutive iterations (an inexact or
     * broken preconditioner, or a floor of the arithmetic).  0 (the default) disables it. */
    double stall_ratio;          /* default 1.0: no contraction at all                       */
    int32_t stall_iters;         /* default 0: off                                           */
} rte_solve_opts;

typedef struct rte_solve_info {
    int32_t iters;               /* outer iterations taken                                   */
    double rel_resid;            /* final ||r||_2 / ||q||_2 (FP64)                           */
    double stop_quantity;        /* ||u_n - u_{n-1}||_{E-K} / ||u_1||_{E-K}  (Sec. 6.4)     */
    int64_t pcg_iters_total;     /* PCG iterations over all E applications                   */
    int64_t cg_iters_total;      /* sum over directions of E_0 CG iterations                 */
    int32_t cg_iters_max;        /* largest per-direction CG count in one E_0 application    */
    double t_solve;              /* seconds spent in rte_solve                               */
    double t_e0inv;              /* with opts->profile: seconds inside E_0^{-1} kernels      */
    int64_t n_e0inv;             /*   number of E_0^{-1} launches                            */
    double t_gemm;               /*   seconds inside the FP64 GEMMs of ApplyE (odd scatter,  */
    int64_t n_gemm;              /*   odd inverse or condensed transport), their launches    */
    double gemm_flops;           /*   and their algorithmic flops (2 M N K summed)           */
    double t_gemm_bf16;          /*   seconds inside BF16 (mixed-precision) GEMM kernels     */
    int64_t n_gemm_bf16;         /*   number of those launches                               */
    double gemm_bf16_flops;      /*   their algorithmic flops (the method's contraction,     */
                                 /*   2 n_R- (d n_S+)^2)                                     */
    double t_scatter;            /*   seconds inside the FP64 even scatter GEMMs U S+        */
    int64_t n_scatter;           /*   (eq. tpmv), their launches                             */
    double scatter_flops;        /*   and their algorithmic flops                            */
    double t_scatter_f32;        /*   seconds inside the FP32 MFMA even scatter GEMMs of the */
    int64_t n_scatter_f32;       /*   mixed-precision preconditioner, their launches         */
    double scatter_f32_flops;    /*   and their algorithmic flops                            */
} rte_solve_info;

/* Fill opts with the defaults: quad_level 2, N+ 0, N- 5, CG E_0, no mixed copies. */
void rte_default_assemble_opts(rte_assemble_opts* opts);
/* Defaults: l 4, tol 1e-8, max_iter 200, FP64, PCG odd solve, CG E_0, PCG tolerances
 * 1e-12 (residual) / 1e-10 (inner), pcg_max_iter 200, cg_tol 1e-10, cg_max_iter 20000,
 * profile 0, Richardson inner iteration, stagnation test off (stall_ratio 1, stall_iters 0). */
void rte_default_solve_opts(rte_solve_opts* opts);

/* Validate the problem and assemble every operator of the mixed system (Sec. 4) on
 * the device: the spatial P1/P0 matrices, the angular moments, the dense scattering
 * matrices S+ and S- by double quadrature of the HG kernel, the eigenpairs of
 * (S+-, M_S+-) (Secs. 5.1, 5.4), the E_0 block data (Sec. 5.3) and the factored
 * coarse matrix E_c = W^T (E - K+) W (Sec. 5.4).  Blocking.  On success *out owns
 * all device memory; release it with rte_destroy.  Errors: RTE_E_ARG, RTE_E_PHYS,
 * RTE_E_MESH before any device work; RTE_E_NOMEM, RTE_E_HIP after. */
rte_status rte_assemble(const rte_problem_desc* desc, const rte_assemble_opts* opts,
                        void* hip_stream, rte_handle** out);

/* Dimensions: n_R+ (vertices), n_R- (cells), n_S+ (antipodal pairs), n_S- = 3 n_S+. */
rte_status rte_query_dims(const rte_handle* h, int32_t* nRp, int32_t* nRm, int32_t* nSp,
                          int32_t* nSm);

/* Band widths of the factored systems: the E_0 blocks (n_R+ unknowns each; 0 when no
 * banded E_0 factors were prepared) and the coarse matrix E_c (coarse_n unknowns). */
rte_status rte_query_band(const rte_handle* h, int32_t* e0_bw, int32_t* coarse_n, int32_t* coarse_bw);

/* Device bytes the handle holds (operators and solver workspace at full size). */
rte_status rte_footprint(const rte_handle* h, size_t* bytes);

/* Before assembly: the device bytes a handle of this problem will hold once assembled with
 * opts and given the workspace of a solve (or batch slot), and the peak during assembly
 * (*peak_bytes, nullable; larger when mixed = 2 drops the FP64 factors at the end).  Host
 * work only (the P1 pattern and its bandwidth); used to admit requests by memory footprint
 * before they are assembled. */
rte_status rte_estimate_footprint(const rte_problem_desc* desc, const rte_assemble_opts* opts, size_t* bytes,
                                  size_t* peak_bytes);

/* Y = K+ X = Ms+ X S+ (parity +1, X and Y n_R+ x n_S+) or Y = K- X = Ms- X S-
 * (parity -1, n_R- x n_S-); Sec. 4 with the Kronecker identity of Sec. 5.1.
 * X and Y are column-major device arrays of dtype_in / dtype_out, each RTE_DT_F64 or
 * RTE_DT_F32 (other codes: RTE_E_ARG).  The GEMM's arithmetic follows dtype_in: FP64
 * MFMA, or FP32 MFMA (FP32 products and sums) on the FP32 copy of S, which needs a handle
 * assembled with mixed != 0 (else RTE_E_ARG); an FP32 Y is rounded from the FP64 epilogue.
 * Uses the handle's workspace: calls on one handle must not overlap.  Enqueue only. */
rte_status rte_apply_scatter(rte_handle* h, int32_t parity, int32_t dtype_in, const void* X,
                             int32_t dtype_out, void* Y, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops or harnesses that forbid hipMalloc): Y = K+- X exactly as rte_apply_scatter computes
 * it (same arguments, layouts and dtypes), calling no hipMalloc, hipFree or allocating
 * library routine.  Its intermediates live in a fixed scratch array of 64 MiB that the
 * library holds on every device it runs on until the process ends (its address is looked
 * up by rte_assemble, or by the first call on a device): the GEMM product X S+ (parity +1,
 * n_R+ n_S+ FP64 values) and an FP64 copy of the result when dtype_out is FP32 (n_R+- n_S+-
 * values); the GEMM is not split over K.  RTE_E_ARG,
 * before any device work, when those intermediates exceed 64 MiB: parity +1 needs
 * n_R+ n_S+ * 8 bytes (twice that with an FP32 Y), parity -1 needs n_R- n_S- * 8 bytes with
 * an FP32 Y and nothing with an FP64 Y.  All calls on one device share its array: calls
 * that overlap on one GPU (other streams, other threads) race, and the caller must order
 * them.  Enqueue only. */
rte_status rte_apply_scatter_noalloc(rte_handle* h, int32_t parity, int32_t dtype_in, const void* X,
                                     int32_t dtype_out, void* Y, void* hip_stream);

/* Y = E X = A^T (M- - K-)^{-1} A X + M+ X + R X (Sec. 4; Alg. 1).  X, Y device FP64
 * n_R+ x n_S+.  The odd solve follows opts->odd_solver with tolerance
 * opts->pcg_tol_resid.  With opts->precision == RTE_MIXED and the condensed odd solver
 * the transport term is applied in BF16 / FP32 (as inside the preconditioner).
 * Synchronises the stream once per PCG iteration. */
rte_status rte_apply_E(rte_handle* h, const rte_solve_opts* opts, const double* X, double* Y,
                       void* hip_stream);

/* Y = E_0 X, the block-diagonal operator of Sec. 5.3 (block k: (1 - c g)^{-1} sum_{n,m} 2 T_k(n,m)
 * D_n^T Mt-^{-1} D_m + m_k Mt+ + R_k), by the SpMV kernel of the CG solve over its sliced-ELL
 * storage.  Device FP64 n_R+ x n_S+ column-major vectors.  The explicit block values are built
 * on the first call when the handle was not assembled for the CG solver (then it allocates).
 * Enqueue only. */
rte_status rte_apply_E0(rte_handle* h, const double* X, double* Y, void* hip_stream);

/* Y = B X, one multigrid V-cycle per direction block (the preconditioner of RTE_E0_MG; the
 * multigrid remark of Sec. 5.5): four Chebyshev steps from 0, the residual restricted by P^T,
 * the coarser levels' cycle, the correction prolongated by P, four Chebyshev steps; eight on the
 * coarsest level, on the level matrices rounded to FP32 (the FP64 solves' smoother precision).
 * B is symmetric positive definite and fixed (linear in X).  Device FP64
 * n_R+ x n_S+ column-major vectors, not aliased.  The handle must be assembled with
 * e0_solver = RTE_E0_MG (else RTE_E_ARG).  Builds the hierarchy's FP64 data on the first call
 * when the handle was assembled with mixed = 2 (then it allocates); otherwise enqueue only. */
rte_status rte_apply_mg(rte_handle* h, const double* X, double* Y, void* hip_stream);

/* Y = E_0^{-1} X, block by block over the directions (Sec. 5.3).  Device FP64 vectors;
 * with opts->precision == RTE_MIXED the banded solver uses FP32 factors. */
rte_status rte_apply_E0inv(rte_handle* h, const rte_solve_opts* opts, const double* X,
                           double* Y, void* hip_stream);

/* s = P_1^l r (which = 0, Alg. 2) or s = P_2 P_1^l r (which = 1, product
 * preconditioner of Sec. 5).  r, s device FP64 n_R+ x n_S+. */
rte_status rte_precond(rte_handle* h, const rte_solve_opts* opts, int32_t which, const double* r,
                       double* s, void* hip_stream);

/* Preconditioned Richardson iteration (Sec. 5, Alg. 3) from U0 (device, NULL = 0)
 * until ||r_n|| <= tol ||q||.  U_even (device FP64 n_R+ x n_S+) receives the iterate.
 * U_odd (device FP64 n_R- x n_S-, column-major, odd index 3k + m; NULL = not wanted)
 * receives the odd part of the final iterate from the second row of the mixed system
 * (eq. mixed_discrete with l- = 0): u- = -(M- - K-)^{-1} A u+, by the exact per-cell odd
 * inverse.  info may be NULL.  Blocking.  Returns
 * RTE_E_NOTCONV at the iteration cap (U_even still holds the last iterate), RTE_E_STALL when the
 * stagnation test of opts fires (likewise), and RTE_E_NONFINITE if the residual is not finite.
 * The iteration is stationary (u_{n+1} depends on u_n alone), so a solve stopped after n steps
 * and resumed with U0 = its iterate reproduces the uninterrupted run bit for bit. */
rte_status rte_solve(rte_handle* h, const rte_solve_opts* opts, const double* U0, double* U_even,
                     double* U_odd, rte_solve_info* info, void* hip_stream);

/* Derived outputs of an even solution U_even (device FP64 n_R+ x n_S+, column-major), e.g.
 * the iterate rte_solve returns.
 * phi (device FP64 [n_R+], NULL = not wanted): the scalar flux at the vertices, the integral
 *   of the intensity over the sphere, phi = U m with m_k = 2|K_k| (the odd part integrates
 *   to zero).
 * balance (host FP64 [4], NULL = not wanted): the particle balance obtained by testing
 *   (E - K+) u = q with the constant 1, whose transport term vanishes (Sec. 2, eq.
 *   mixed_discrete; A 1 = 0):  [0] source 1^T q,  [1] absorption 1^T (M+ - K+) U,
 *   [2] leakage 1^T R U (the outflow through the vacuum boundary),  [3] source -
 *   absorption - leakage, which equals -1^T r for the residual r = (E - K+) U - q.
 * Sums are FP64 with a fixed order.  Blocking when balance is requested (it allocates a
 * few small device buffers and reads back per-direction sums); otherwise enqueue only. */
rte_status rte_derived_outputs(rte_handle* h, const double* U_even, double* phi, double* balance,
                               void* hip_stream);

/* Copy an assembled array to host memory, for inspection and tests.
 * which: 0 S+ [n_S+ x n_S+], 1 S- [n_S- x n_S-], 2 m_k [n_S+], 3 T_k [n_S+ x 9],
 * 4 q = l+ [n_R+ x n_S+], 5 even eigenvalues [d_N+], 6 even eigenvectors
 * [n_S+ x d_N+], 7 odd eigenvalues [n_S-] (all FP64), 8 the iterations every direction took
 * in the last E_0^{-1} by CG (RTE_E0_CG or RTE_E0_MG; int32 [n_S+], RTE_E_ARG before the first).
 * host_bytes must equal the array size in bytes.  Blocking. */
rte_status rte_get_array(rte_handle* h, int32_t which, void* host_dst, size_t host_bytes);

/* Release the handle (synchronises its stream first).  NULL is accepted.  RTE_E_HIP if a
 * hipFree of its device memory failed (the handle is gone either way). */
rte_status rte_destroy(rte_handle* h);

/* ------------------------------------------------------------------ batched and served solves
 * A batch advances several solves of Alg. 3 in lockstep, one outer iteration of every live
 * slot per step.  In each of the l steps of P_1 (Alg. 2, eq. applyP1), the E_0^{-1} of all
 * slots (Sec. 5.3) is one band-solve launch per band shape, so the direction systems of
 * small problems share the GPU.  Slots can be admitted while others run, and they leave the
 * lockstep as soon as their relative residual reaches their tolerance.  A slot computes
 * exactly what rte_solve computes with the same options and handle, independently of the
 * other slots.
 * Requirements: the handle is assembled with e0_solver = RTE_E0_BANDED (and mixed != 0 for
 * RTE_MIXED slots); odd_solver is RTE_ODD_EXACT or RTE_ODD_CONDENSED; all slots of a batch
 * share precision and l; a handle holds at most one slot at a time.  The batch does not own
 * the handles or the U arrays: both must stay alive until the slot has been polled.  A batch
 * is not thread-safe. */
typedef struct rte_batch rte_batch;

/* max_slots in 1..4096; hbm_budget = device bytes the slots' handles and workspace may hold
 * together (0 = unlimited). */
rte_status rte_batch_create(int32_t max_slots, size_t hbm_budget, rte_batch** out);

/* Admit a solve of h from U0 (device, n_R+ x n_S+ column-major; NULL = zero) into U
 * (device, same shape, caller-owned; holds the iterate and, once the slot is done, the
 * result).  Sets *slot.  Allocates the slot's solver workspace in the handle.  Returns
 * RTE_E_NOMEM, with nothing admitted, when the handle's footprint plus that workspace exceeds
 * the budget that is left; RTE_E_ARG when no slot is free or a requirement above fails.
 * Enqueues the initialisation of U on hip_stream. */
rte_status rte_batch_admit(rte_batch* b, rte_handle* h, const rte_solve_opts* opts, const double* U0,
                           double* U, void* hip_stream, int32_t* slot);

/* Run up to outer_iters lockstep iterations on hip_stream (blocking; one host
 * synchronisation per iteration).  Returns early when no slot is live.  *n_live (nullable)
 * receives the number of slots still iterating. */
rte_status rte_batch_step(rte_batch* b, int32_t outer_iters, void* hip_stream, int32_t* n_live);

/* Report and release up to max_out finished slots: slot ids, their solve infos (iters,
 * rel_resid, stop_quantity, t_solve = seconds from admission to completion) and statuses
 * (RTE_OK, RTE_E_NOTCONV, RTE_E_STALL or RTE_E_NONFINITE).  *n_done receives the count.  The
 * released slot ids and budget become free. */
rte_status rte_batch_poll(rte_batch* b, int32_t max_out, int32_t* slots, rte_solve_info* infos,
                          int32_t* statuses, int32_t* n_done);

/* use_graphs != 0: each lockstep iteration replays two captured HIP graphs (the residuals;
 * the preconditioner, correction and update), recaptured whenever the set of live slots
 * changes, on a stream the batch owns (ordered after the caller's stream's earlier work, and
 * the caller's later work after it).  0 (the default): the same launches are issued one by
 * one on the caller's stream.  The results are identical, also while other threads of the
 * process assemble handles (rte_assemble), whose results do not depend on what else runs when
 * they use none of the rocSOLVER paths (the full odd eigendecomposition, odd_eig = 1; the
 * explicit coarse inverse, RTE_COARSE_INVERSE or RTE_COARSE_AUTO where it fits; the block
 * coarse factorisation, RTE_COARSE_BLOCK or where the band does not fit). */
rte_status rte_batch_set_graphs(rte_batch* b, int32_t use_graphs);

/* Slots still iterating, finished slots not yet polled, device bytes held by admitted slots. */
rte_status rte_batch_usage(const rte_batch* b, int32_t* n_live, int32_t* n_done, size_t* used_bytes);

rte_status rte_batch_destroy(rte_batch* b);

/* ------------------------------------------------------------------ autotuning
 * Layouts of the banded E_0 factors: a factor row block holds G = H P groups of 16 bytes,
 * H the register ring depth of the band solve and P its phase count, over the menu of shapes
 * the solve kernel is built for (H, P) in {(9,1) (17,1) (33,1) (9,2) (17,2) (33,2) (17,3)
 * (33,3) (33,4)}.  Assembly lays them out in the shape with the least padding; the
 * autotuner times the E_0^{-1} launch (all n_S+ directions, HIP events on hip_stream) in
 * every shape that holds the band, re-laying the factors out on the device, and keeps the
 * fastest.  The results do not depend on the layout (padding entries are zero and every
 * product is summed in the same order).
 *
 * The tile map of every GEMM shape the handle launches (the scatter GEMM U S+ of Sec. 5.2 in
 * FP64 and, with mixed precision, FP32; the condensed transport GEMM of Sec. 5.1 in FP64 and,
 * with mixed precision, BF16) is tuned the same way: the four combinations of {XCD swizzle
 * of the work-group ids on, off} x {row-major, column-major traversal of the output tile
 * grid} are timed (three launches each, HIP events) and the fastest kept when it beats the
 * default map 0 by 1%.  A map only reorders whole output tiles: results are bitwise the same.
 * The maps are process-wide by (kind, M, N, K) and apply to every handle.
 *
 * Choices are cached per process by (n_R+, band width, n_S+, element size) and (GEMM kind,
 * M, N, K), and in a text file read on the first call and appended to on each new choice:
 * the path in the environment variable RTE_TUNE_CACHE, else $HOME/.cache/rte/tune.txt
 * (lines for another device architecture or compute-unit count are ignored; an unwritable
 * file only costs the timing in later processes).  A cached key takes the cached choice
 * without timing unless flags has RTE_TUNE_FORCE.  Both precisions of banded factors present
 * in the handle are tuned (the FP64 factors are absent after assembly with mixed = 2).
 * While a candidate layout is timed the device holds one more copy of the factors of that
 * precision.  The handle must not be in use (no solve, no batch slot) during the call, and
 * no other handle may solve during it (the GEMM maps are shared).  Blocking. */
#define RTE_TUNE_FORCE 1
typedef struct rte_tune_report {
    int32_t n_cand[2];           /* candidates timed: [0] FP64 factors, [1] FP32 factors    */
    int32_t H[2][9], P[2][9];    /* their shapes                                            */
    double ms[2][9];             /* average E_0^{-1} launch time of each candidate          */
    int32_t chosen_H[2], chosen_P[2];  /* the shape in place on return (0: precision absent) */
    int32_t default_H[2], default_P[2];/* the shape assembly chose                           */
    int32_t from_cache[2];       /* 1: taken from the cache, nothing timed                  */
    int32_t n_gemm;              /* GEMM shapes tuned (at most 4), in the order above        */
    int32_t gemm_kind[4];        /* 1 FP64, 2 FP32 (FP64 operand A), 4 BF16                  */
    int32_t gemm_m[4], gemm_n[4], gemm_k[4];
    double gemm_ms[4][4];        /* average launch time of maps 0..3 (0 if from the cache)   */
    int32_t gemm_map[4];         /* the map chosen                                           */
    int32_t gemm_from_cache[4];  /* 1: taken from the cache, nothing timed                  */
} rte_tune_report;
rte_status rte_autotune(rte_handle* h, int32_t flags, void* hip_stream, rte_tune_report* report);

/* Lay the banded E_0 factors of one precision (RTE_FP64: the FP64 factors, RTE_MIXED: the
 * FP32 ones) out in the shape (H, P) of the menu above, without timing.  RTE_E_ARG if the
 * shape is not in the menu, cannot hold the band, or the factors are absent.  Same
 * conditions as rte_autotune; blocking. */
rte_status rte_set_band_layout(rte_handle* h, int32_t precision, int32_t H, int32_t P, void* hip_stream);

/* Thread-local text of the last non-OK status ("" if none). */
const char* rte_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RTE_H */
