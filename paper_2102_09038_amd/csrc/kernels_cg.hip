// E_0^{-1} by conjugate gradients on every direction block at once (Sec. 5.3: E_0 is block
// diagonal over the directions, each block an SPD anisotropic diffusion-reaction matrix on
// the P1 space).  Jacobi preconditioning; all directions iterate in the same launches and a
// direction that has converged stops doing work (per-direction early exit).
//
// Storage: the P1 pattern in sliced ELL form.  Rows are cut into slices of 64 (one wave, lane
// = row); a slice holds as many entry slots as its longest row, and entry j of the slice's
// rows sits in one contiguous group of 64, so a wave's loads of values and columns are single
// 256- or 512-byte transactions.  The column pattern is shared by every direction; each
// direction has its own explicit values (formed once from the pattern's value classes).
//
// One CG iteration is three launches over (row tile, direction) work-groups of 256 rows:
//   spmv    q = E_0 p, partial sums of p.q per tile (two directions per work-group);
//   update  alpha = rz / p.q (the tile partials summed in a fixed order by every work-group of
//           the direction, so all of them get the same bits), x += alpha p, r -= alpha q,
//           partials of r.z and r.r (z = D^{-1} r);
//   dir     beta = r.z / rz_old; stop if r.r <= tol^2 b.b; p = z + beta p.
// The two rz of consecutive iterations alternate between two slots, so the work-group that
// stores the new one never overwrites the value the others still read.  Dot products are
// accumulated in FP64 whatever the vector type.  Work-group b runs on XCD b mod 8; the tiles
// of one direction are all given to one XCD, so the neighbour rows their SpMV gathers are in
// that XCD's L2.
#include <climits>

#include "dev_reduce.h"
#include "ops.h"

namespace rte {
namespace {

constexpr int CTB = 256;                 // threads (rows) per work-group: 4 slices of 64

using dev::block_sum;
using dev::partial_sum;
using dev::wave_sum;

__device__ __forceinline__ bool cg_tile(int ntiles, int nS, int& k, int& t) { return dev::dir_tile(ntiles, nS, k, t); }

// explicit values of every direction's block in the sliced ELL layout:
// val[k * len + q] = sum_c coef[k, c] cls[c, e(q)] (0 on padding), dinv = 1 / diag
template <typename T>
__global__ void cg_fill_kernel(int nS, size_t len, int nnz, int ncls, const int* __restrict__ ell_e,
                               const double* __restrict__ cls, const double* __restrict__ coef,
                               T* __restrict__ val) {
    const size_t total = len * nS;
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < total; q += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(q / len);
        const int e = ell_e[q % len];
        double v = 0.0;
        if (e >= 0)
            for (int c = 0; c < ncls; ++c) v = fma(coef[(size_t)k * ncls + c], cls[(size_t)c * nnz + e], v);
        val[q] = (T)v;
    }
}

template <typename T>
__global__ void cg_dinv_kernel(size_t n, const double* __restrict__ diag, T* __restrict__ dinv) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dinv[i] = (T)(1.0 / diag[i]);
}

// x = 0, r = b, p = z = D^{-1} r; partials of b.b and r.z
template <typename T>
__global__ __launch_bounds__(CTB) void cg_init_kernel(int n, int nS, int ntiles, const double* __restrict__ B,
                                                      double* __restrict__ X, T* __restrict__ R, T* __restrict__ P,
                                                      const T* __restrict__ dinv, double* __restrict__ part) {
    __shared__ double sh[8];
    int k, t;
    if (!cg_tile(ntiles, nS, k, t)) return;
    const int i = t * CTB + threadIdx.x;
    double bb = 0.0, rz = 0.0;
    if (i < n) {
        const size_t o = (size_t)n * k + i;
        const double b = B[o];
        X[o] = 0.0;
        const T r = (T)b;
        const T z = r * dinv[o];
        R[o] = r;
        P[o] = z;
        bb = b * b;
        rz = (double)r * (double)z;
    }
    bb = block_sum(bb, sh);
    rz = block_sum(rz, sh);
    if (threadIdx.x == 0) {
        part[(size_t)k * ntiles + t] = bb;
        part[(size_t)(nS + k) * ntiles + t] = rz;
    }
}

// per direction: rz_0, the stopping threshold tol^2 b.b and the state (converged at
// iteration done[k]; INT_MAX while running, -1 for a zero right-hand side)
__global__ __launch_bounds__(CTB) void cg_setup_kernel(int nS, int ntiles, const double* __restrict__ part, double tol,
                                                       double* __restrict__ rz, double* __restrict__ stop,
                                                       int* __restrict__ done, int* __restrict__ iters) {
    __shared__ double sh[8];
    const int k = blockIdx.x;
    const double bb = partial_sum(part + (size_t)k * ntiles, ntiles, sh);
    const double r0 = partial_sum(part + (size_t)(nS + k) * ntiles, ntiles, sh);
    if (threadIdx.x == 0) {
        rz[k] = r0;                      // slot 0 (iteration 0 reads slot 0)
        stop[k] = tol * tol * bb;
        done[k] = bb > 0.0 ? INT_MAX : -1;
        iters[k] = 0;
    }
}

// q = E_0 p on a tile of four 64-row slices (one per wave) for two directions at once, k and
// k + 8 of the XCD's directions, which share the tile's column loads; partials p.q per
// direction and tile.  With WMAX > 0 (the widest slice has at most WMAX slots) all of a slice's
// column and value loads are issued together before the gathers; slots past a slice's width
// re-read its last slot (in bounds) and count zero, so WMAX is instantiated at the exact widths
// of the 2D and 3D P1 patterns.  The values are read once per launch and bypass the caches
// (non-temporal loads), which keeps p, which the gathers re-read, resident.  WMAX = 0: a plain
// loop.  A direction that has converged (done[k] < it) is not computed; its q and partial are
// left as they are.
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
    return __builtin_nontemporal_load(p);
}

template <int WMAX, typename T>
__global__ __launch_bounds__(CTB) void cg_spmv_kernel(int n, int nS, int ntiles_s, int nslice, int it,
                                                      const int* __restrict__ sptr, const int* __restrict__ col,
                                                      const T* __restrict__ val, size_t len,
                                                      const T* __restrict__ P, T* __restrict__ Q,
                                                      const int* __restrict__ done, double* __restrict__ part) {
    __shared__ double sh[8];
    const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3;
    const int jp = local / ntiles_s, t = local % ntiles_s;
    const int kA = xcd + 16 * jp, kB = kA + 8;
    const bool actA = kA < nS && !(done && done[kA] < it);
    const bool actB = kB < nS && !(done && done[kB] < it);
    if (!actA && !actB) return;
    // an inactive direction of the pair computes the active one's rows again, unstored
    const int ka = actA ? kA : kB, kb = actB ? kB : ka;
    const int lane = threadIdx.x & 63;
    const int sl = t * (CTB / 64) + (threadIdx.x >> 6);
    const T* pa = P + (size_t)n * ka;
    const T* pb = P + (size_t)n * kb;
    const T* va = val + len * ka;
    const T* vb = val + len * kb;
    const bool in = sl < nslice;
    const int g0 = in ? sptr[sl] : 0;
    const int wd = in ? sptr[sl + 1] - g0 : 1;
    const size_t base = (size_t)g0 * 64 + lane;
    T accA = (T)0, accB = (T)0;
    if constexpr (WMAX > 0) {
        const int w = in ? wd : 0;
        int c[WMAX];
        T xa[WMAX], xb[WMAX];
#pragma unroll
        for (int j = 0; j < WMAX; ++j) {
            const size_t q = base + 64 * (size_t)min(j, wd - 1);
            c[j] = col[q];
            xa[j] = ld_stream(va + q);
            xb[j] = ld_stream(vb + q);
        }
        T ga[WMAX], gb[WMAX];
#pragma unroll
        for (int j = 0; j < WMAX; ++j) {
            ga[j] = pa[c[j]];
            gb[j] = pb[c[j]];
        }
#pragma unroll
        for (int j = 0; j < WMAX; ++j) {
            accA += (j < w ? xa[j] : (T)0) * ga[j];
            accB += (j < w ? xb[j] : (T)0) * gb[j];
        }
    } else if (in) {
        for (int j = 0; j < wd; ++j) {
            const size_t q = base + 64 * (size_t)j;
            const int cj = col[q];
            accA += ld_stream(va + q) * pa[cj];
            accB += ld_stream(vb + q) * pb[cj];
        }
    }
    const int i = sl * 64 + lane;
    double pqA = 0.0, pqB = 0.0;
    if (in && i < n) {
        if (actA) {
            Q[(size_t)n * kA + i] = accA;
            pqA = (double)pa[i] * (double)accA;
        }
        if (actB) {
            Q[(size_t)n * kB + i] = accB;
            pqB = (double)pb[i] * (double)accB;
        }
    }
    pqA = block_sum(pqA, sh);
    pqB = block_sum(pqB, sh);
    if (threadIdx.x == 0) {
        if (actA) part[(size_t)kA * ntiles_s + t] = pqA;
        if (actB) part[(size_t)kB * ntiles_s + t] = pqB;
    }
}

// alpha = rz / p.q; x += alpha p; r -= alpha q; partials of r.z and r.r
template <typename T>
__global__ __launch_bounds__(CTB) void cg_update_kernel(int n, int nS, int ntiles, int ntiles_pq, int it,
                                                        const T* __restrict__ P,
                                                        const T* __restrict__ Q, T* __restrict__ R,
                                                        double* __restrict__ X, const T* __restrict__ dinv,
                                                        const double* __restrict__ rz, const int* __restrict__ done,
                                                        const double* __restrict__ part_pq,
                                                        double* __restrict__ part) {
    __shared__ double sh[8];
    int k, t;
    if (!cg_tile(ntiles, nS, k, t)) return;
    if (done[k] < it) return;
    const double pq = partial_sum(part_pq + (size_t)k * ntiles_pq, ntiles_pq, sh);
    const double a = pq != 0.0 ? rz[(size_t)(it & 1) * nS + k] / pq : 0.0;
    const int i = t * CTB + threadIdx.x;
    double rzn = 0.0, rr = 0.0;
    if (i < n) {
        const size_t o = (size_t)n * k + i;
        const T p = P[o];
        X[o] = fma(a, (double)p, X[o]);
        const T r = R[o] - (T)a * Q[o];
        R[o] = r;
        const T z = r * dinv[o];
        rzn = (double)r * (double)z;
        rr = (double)r * (double)r;
    }
    rzn = block_sum(rzn, sh);
    rr = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        part[(size_t)k * ntiles + t] = rzn;
        part[(size_t)(nS + k) * ntiles + t] = rr;
    }
}

// convergence test and p = z + beta p
template <typename T>
__global__ __launch_bounds__(CTB) void cg_dir_kernel(int n, int nS, int ntiles, int it, T* __restrict__ P,
                                                     const T* __restrict__ R, const T* __restrict__ dinv,
                                                     double* __restrict__ rz, const double* __restrict__ stop,
                                                     int* __restrict__ done, int* __restrict__ iters,
                                                     const double* __restrict__ part) {
    __shared__ double sh[8];
    int k, t;
    if (!cg_tile(ntiles, nS, k, t)) return;
    if (done[k] < it) return;
    const double rzn = partial_sum(part + (size_t)k * ntiles, ntiles, sh);
    const double rr = partial_sum(part + (size_t)(nS + k) * ntiles, ntiles, sh);
    if (rr <= stop[k]) {
        if (t == 0 && threadIdx.x == 0) {
            done[k] = it;
            iters[k] = it + 1;
        }
        return;
    }
    const double rzo = rz[(size_t)(it & 1) * nS + k];
    const double b = rzo != 0.0 ? rzn / rzo : 0.0;
    const int i = t * CTB + threadIdx.x;
    if (i < n) {
        const size_t o = (size_t)n * k + i;
        P[o] = R[o] * dinv[o] + (T)b * P[o];
    }
    if (t == 0 && threadIdx.x == 0) rz[(size_t)((it + 1) & 1) * nS + k] = rzn;
}

// number of directions still iterating; the directions that ran out of iterations get maxit
__global__ __launch_bounds__(CTB) void cg_count_kernel(int nS, int maxit, int final_pass, int* __restrict__ done,
                                                       int* __restrict__ iters, int* __restrict__ active) {
    __shared__ double sh[8];
    double c = 0.0;
    for (int k = threadIdx.x; k < nS; k += CTB) {
        const bool run = done[k] == INT_MAX;
        c += run ? 1.0 : 0.0;
        if (final_pass && run) iters[k] = maxit;
    }
    c = block_sum(c, sh);
    if (threadIdx.x == 0) *active = (int)c;
}

inline int grid_of(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 65536); }

}  // namespace

namespace k {

void cg_fill_values(const Handle* h, const int* ell_e, size_t len, double* val, hipStream_t s) {
    hipLaunchKernelGGL(cg_fill_kernel<double>, dim3(grid_of(len * h->nS)), dim3(256), 0, s, h->nS, len, h->nnz, h->ncls,
                       ell_e, h->cls.p, h->coefE0.p, val);
    RTE_CHECK_LAUNCH();
}
void cg_fill_values(const Handle* h, const int* ell_e, size_t len, float* val, hipStream_t s) {
    hipLaunchKernelGGL(cg_fill_kernel<float>, dim3(grid_of(len * h->nS)), dim3(256), 0, s, h->nS, len, h->nnz, h->ncls,
                       ell_e, h->cls.p, h->coefE0.p, val);
    RTE_CHECK_LAUNCH();
}
void fill_block_values(int nS, size_t len, int nnz, int ncls, const int* ell_e, const double* cls,
                       const double* coef, double* val, hipStream_t s) {
    hipLaunchKernelGGL(cg_fill_kernel<double>, dim3(grid_of(len * nS)), dim3(256), 0, s, nS, len, nnz, ncls, ell_e, cls,
                       coef, val);
    RTE_CHECK_LAUNCH();
}
void fill_block_values(int nS, size_t len, int nnz, int ncls, const int* ell_e, const double* cls,
                       const double* coef, float* val, hipStream_t s) {
    hipLaunchKernelGGL(cg_fill_kernel<float>, dim3(grid_of(len * nS)), dim3(256), 0, s, nS, len, nnz, ncls, ell_e, cls,
                       coef, val);
    RTE_CHECK_LAUNCH();
}
void cg_fill_dinv(const double* diag, size_t n, double* dinv, hipStream_t s) {
    hipLaunchKernelGGL(cg_dinv_kernel<double>, dim3(grid_of(n)), dim3(256), 0, s, n, diag, dinv);
    RTE_CHECK_LAUNCH();
}
void cg_fill_dinv(const double* diag, size_t n, float* dinv, hipStream_t s) {
    hipLaunchKernelGGL(cg_dinv_kernel<float>, dim3(grid_of(n)), dim3(256), 0, s, n, diag, dinv);
    RTE_CHECK_LAUNCH();
}

// tiles of the SpMV (4 slices each)
int spmv_tiles(const CgArgs& a) { return (a.nslice + 3) / 4; }

template <typename T>
void spmv_launch(const CgArgs& a, int it, const T* val, const T* X, T* Y, const int* done, double* part,
                 hipStream_t s) {
    const int ntiles_s = spmv_tiles(a);
    // direction pairs (k, k + 8) per XCD: XCD x holds directions x, x + 8, ...
    const int npair = ((a.nS + 7) / 8 + 1) / 2;
    const unsigned grid = (unsigned)ntiles_s * 8u * (unsigned)npair;
    auto f = a.wmax <= 7    ? cg_spmv_kernel<7, T>
             : a.wmax <= 8  ? cg_spmv_kernel<8, T>
             : a.wmax <= 15 ? cg_spmv_kernel<15, T>
             : a.wmax <= 16 ? cg_spmv_kernel<16, T>
                            : cg_spmv_kernel<0, T>;
    hipLaunchKernelGGL(f, dim3(grid), dim3(CTB), 0, s, a.n, a.nS, ntiles_s, a.nslice, it, a.sptr, a.col, val, a.len,
                       X, Y, done, part);
    RTE_CHECK_LAUNCH();
}

// the phases of one Jacobi-preconditioned solve: set-up and one iteration
template <typename T>
struct CgRun : CgPhases {
    const T *val, *dinv;
    T *R, *P, *Q;
    int ntiles;
    unsigned grid;
    double *part_a, *part_b;
    CgRun(const CgArgs& a_, const T* v, const T* d, T* r, T* p, T* q, hipStream_t s_)
        : CgPhases(a_, s_), val(v), dinv(d), R(r), P(p), Q(q) {
        ntiles = (a.n + CTB - 1) / CTB;
        grid = (unsigned)ntiles * 8u * (unsigned)((a.nS + 7) / 8);
        part_a = a.part;                                   // [2 nS ntiles]
        part_b = a.part + (size_t)2 * a.nS * ntiles;       // [2 nS ntiles]
    }
    void start() override {
        hipLaunchKernelGGL(cg_init_kernel<T>, dim3(grid), dim3(CTB), 0, s, a.n, a.nS, ntiles, a.B, a.X, R, P, dinv,
                           part_a);
        RTE_CHECK_LAUNCH();
        hipLaunchKernelGGL(cg_setup_kernel, dim3(a.nS), dim3(CTB), 0, s, a.nS, ntiles, part_a, a.tol, a.rz, a.stop,
                           a.done, a.iters);
        RTE_CHECK_LAUNCH();
    }
    void iterate(int it) override {
        spmv_launch<T>(a, it, val, (const T*)P, Q, a.done, part_a, s);
        hipLaunchKernelGGL(cg_update_kernel<T>, dim3(grid), dim3(CTB), 0, s, a.n, a.nS, ntiles, spmv_tiles(a), it,
                           (const T*)P, (const T*)Q, R, a.X, dinv, (const double*)a.rz, (const int*)a.done,
                           (const double*)part_a, part_b);
        RTE_CHECK_LAUNCH();
        hipLaunchKernelGGL(cg_dir_kernel<T>, dim3(grid), dim3(CTB), 0, s, a.n, a.nS, ntiles, it, P, (const T*)R, dinv,
                           a.rz, (const double*)a.stop, a.done, a.iters, (const double*)part_b);
        RTE_CHECK_LAUNCH();
    }
};

std::unique_ptr<CgPhases> phases_of(const CgJob& j) {
    if (j.mg) return mg_phases(j);
    if (j.f32)
        return std::make_unique<CgRun<float>>(j.a, static_cast<const float*>(j.val), static_cast<const float*>(j.dinv),
                                              static_cast<float*>(j.R), static_cast<float*>(j.P),
                                              static_cast<float*>(j.Q), j.s);
    return std::make_unique<CgRun<double>>(j.a, static_cast<const double*>(j.val), static_cast<const double*>(j.dinv),
                                           static_cast<double*>(j.R), static_cast<double*>(j.P),
                                           static_cast<double*>(j.Q), j.s);
}

void run_one(CgPhases& run) {
    run.start();
    for (int it = 0; it < run.a.maxit; ++it) {
        run.iterate(it);
        if (run.check_point(it)) {
            run.count(it);
            RTE_HIP(hipStreamSynchronize(run.s));
            if (*run.a.host_active == 0) break;
        }
    }
}

template <typename T>
void cg_solve_t(const CgArgs& a, const T* val, const T* dinv, T* R, T* P, T* Q, hipStream_t s) {
    CgRun<T> run(a, val, dinv, R, P, Q, s);
    run_one(run);
}

// every running solve takes iteration it on its stream; at a check point of any of them the
// host waits for those that counted and retires the finished ones
void cg_solve_many(std::vector<CgJob>& jobs) {
    std::vector<std::unique_ptr<CgPhases>> runs;
    runs.reserve(jobs.size());
    for (auto& j : jobs) runs.push_back(phases_of(j));
    if (runs.size() == 1) {
        run_one(*runs[0]);
        return;
    }
    std::vector<char> live(runs.size(), 1);
    for (auto& r : runs) r->start();
    for (int it = 0;; ++it) {
        bool any = false;
        for (size_t k = 0; k < runs.size(); ++k) {
            if (!live[k] || it >= runs[k]->a.maxit) {
                live[k] = 0;
                continue;
            }
            any = true;
            runs[k]->iterate(it);
        }
        if (!any) break;
        std::vector<size_t> counted;
        for (size_t k = 0; k < runs.size(); ++k) {
            if (!live[k] || !runs[k]->check_point(it)) continue;
            runs[k]->count(it);
            counted.push_back(k);
        }
        for (size_t k : counted) RTE_HIP(hipStreamSynchronize(runs[k]->s));
        for (size_t k : counted)
            if (*runs[k]->a.host_active == 0) live[k] = 0;
    }
}

void cg_spmv_it(const CgArgs& a, int it, const double* val, const double* X, double* Y, hipStream_t s) {
    spmv_launch<double>(a, it, val, X, Y, a.done, a.part, s);
}
void cg_spmv_it(const CgArgs& a, int it, const float* val, const float* X, float* Y, hipStream_t s) {
    spmv_launch<float>(a, it, val, X, Y, a.done, a.part, s);
}

void cg_setup(const CgArgs& a, const double* part, hipStream_t s) {
    const int ntiles = (a.n + CTB - 1) / CTB;
    hipLaunchKernelGGL(cg_setup_kernel, dim3(a.nS), dim3(CTB), 0, s, a.nS, ntiles, part, a.tol, a.rz, a.stop, a.done,
                       a.iters);
    RTE_CHECK_LAUNCH();
}

void cg_count(const CgArgs& a, int it, hipStream_t s) {
    hipLaunchKernelGGL(cg_count_kernel, dim3(1), dim3(CTB), 0, s, a.nS, a.maxit, it + 1 == a.maxit ? 1 : 0, a.done,
                       a.iters, a.active);
    RTE_CHECK_LAUNCH();
    RTE_HIP(hipMemcpyAsync(a.host_active, a.active, sizeof(int), hipMemcpyDeviceToHost, s));
}

void cg_solve(const CgArgs& a, const double* val, const double* dinv, double* R, double* P, double* Q, hipStream_t s) {
    cg_solve_t<double>(a, val, dinv, R, P, Q, s);
}
void cg_solve(const CgArgs& a, const float* val, const float* dinv, float* R, float* P, float* Q, hipStream_t s) {
    cg_solve_t<float>(a, val, dinv, R, P, Q, s);
}

void cg_spmv(const CgArgs& a, const double* val, const double* X, double* Y, hipStream_t s) {
    spmv_launch<double>(a, 0, val, X, Y, nullptr, a.part, s);
}

}  // namespace k
}  // namespace rte
