// E_0^{-1} by CG preconditioned by a geometric multigrid V-cycle, on every direction block at
// once (Sec. 5.5 names multigrid as the solver of the E_0 blocks, each an anisotropic
// diffusion-reaction problem on the P1 space).
//
// Hierarchy (built at assembly on the host): the mesh is the Freudenthal triangulation of a
// box; the coarse lattices halve the cells per axis, so the coarse P1 spaces are nested and the
// prolongation is the P1 interpolant: fine vertex 2I takes coarse vertex I, a fine vertex with
// odd coordinates on the axis set S takes half of each end of the coarse edge it bisects (ends
// floor(f / 2) and ceil(f / 2)).  Coarse blocks are Galerkin products, stored like the fine
// level in sliced ELL with explicit values per direction.
//
// Smoother: the Chebyshev iteration on D^{-1} A over [lo lam, lam] (lam = Gershgorin's bound of
// D^{-1} A per level and direction), the three-term recurrence
//   x_{j+1} = x_j + d_j,  r_{j+1} = r_j - A d_j,
//   rho_{j+1} = 1 / (2 sigma - rho_j),  d_{j+1} = rho_{j+1} rho_j d_j + 2 rho_{j+1} / delta D^{-1} r_{j+1},
// with sigma = theta / delta, rho_0 = 1 / sigma, d_0 = D^{-1} r_0 / theta.  Each step is one
// launch: the SpMV A d_j fused with the recurrence's vector updates of the same rows (d_j is
// gathered from one buffer, d_{j+1} written to the other).  The residual that the restriction
// reads is the recurrence's r (one more SpMV step); the post-smoothing starts with the SpMV
// r_0 = b - A x; the last x + d of a level is left to the launch that reads it (the prolongation
// of the finer level, or the CG's z = x + d).  The coarse levels, where launches are bound by their
// latency, run in one launch per cycle instead (the fused tail below).
//
// Smoother precision: the cycle reads every level's matrix in a reduced precision, FP32 when
// the vectors are FP64 and BF16 when they are FP32 (values rounded to nearest even; inverse
// diagonals and Gershgorin bounds from the rounded values).  The rounded matrices are
// symmetric, so the cycle is still a fixed symmetric preconditioner; the CG's own SpMV uses
// the full-precision values.  The smoothing launches stream half the value bytes.
//
// CG (Saad's preconditioned CG with one V-cycle as the preconditioner), per direction:
//   spmv     q = A p, partials p.q                                   (the Jacobi CG's kernel)
//   update   alpha = rz / p.q; x += alpha p; r -= alpha q; partials r.r; d_0 of the cycle
//   check    stop the direction once r.r <= tol^2 b.b
//   V-cycle  z = B r
//   rz       partials r.z
//   dir      beta = r.z / rz_old; p = z + beta p
// All directions run in the same launches; a direction that has converged returns at once from
// every launch.  Sums of partials are fixed-order, so every work-group of a direction gets the
// same alpha and beta and a solve repeats bit for bit.
#include <climits>

#include "dev_reduce.h"
#include "ops.h"

namespace rte {
namespace {

constexpr int MTB = 256;                 // threads (rows) per work-group: four 64-row slices

using k::CgJob;
using k::CgPhases;
using k::cg_setup;
using k::cg_spmv_it;
using k::kMgMaxLevels;
using k::kMgNu;
using k::kMgNuCoarse;
using k::MgArgs;
using k::MgLevelArgs;
using dev::block_max;
using dev::block_sum;
using dev::dir_tile;
using dev::partial_sum;

template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
    return __builtin_nontemporal_load(p);
}

// the smoother's value type for a vector type, and its conversion
template <typename T> struct SmoothVal;
template <> struct SmoothVal<double> { typedef float V; };
template <> struct SmoothVal<float> { typedef uint16_t V; };      // BF16 bits
__device__ __forceinline__ double sval(float v, double) { return (double)v; }
__device__ __forceinline__ float sval(uint16_t v, float) { return __uint_as_float((uint32_t)v << 16); }

// round to nearest even: FP64 -> FP32 (the conversion), FP32 -> BF16 (bits)
__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ void round_to(double v, float& out) { out = (float)v; }
__device__ __forceinline__ void round_to(double v, uint16_t& out) { out = to_bf16((float)v); }
__device__ __forceinline__ void round_to(float v, uint16_t& out) { out = to_bf16(v); }

// the Chebyshev coefficients of step j: d_{j+1} = c1 d_j + c2 D^{-1} r_{j+1}
__device__ __forceinline__ void cheb_coef(double theta, double delta, int j, double& c1, double& c2) {
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    c1 = c2 = 0.0;
    for (int i = 0; i <= j; ++i) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        if (i == j) {
            c1 = rn * rho;
            c2 = 2.0 * rn / delta;
        }
        rho = rn;
    }
}

// acc = row i of A g for direction k (lane = row of the slice), the sliced ELL layout of the CG,
// the values in the smoother precision VT
template <int WMAX, typename T, typename VT, bool NT = true>
__device__ __forceinline__ T ell_row(const int* __restrict__ sptr, const int* __restrict__ col, const VT* __restrict__ v,
                                     const T* __restrict__ g, int sl, int lane) {
    const int g0 = sptr[sl];
    const int wd = sptr[sl + 1] - g0;
    const size_t base = (size_t)g0 * 64 + lane;
    T acc = (T)0;
    if constexpr (WMAX > 0) {
        int c[WMAX];
        VT x[WMAX];
#pragma unroll
        for (int j = 0; j < WMAX; ++j) {
            const size_t q = base + 64 * (size_t)min(j, wd - 1);
            c[j] = col[q];
            x[j] = NT ? ld_stream(v + q) : v[q];
        }
        T gv[WMAX];
#pragma unroll
        for (int j = 0; j < WMAX; ++j) gv[j] = g[c[j]];
#pragma unroll
        for (int j = 0; j < WMAX; ++j) acc += (j < wd ? sval(x[j], T()) : (T)0) * gv[j];
    } else {
        for (int j = 0; j < wd; ++j) {
            const size_t q = base + 64 * (size_t)j;
            acc += sval(NT ? ld_stream(v + q) : v[q], T()) * g[col[q]];
        }
    }
    return acc;
}

// The row update of a smoothing step (the vectors of one direction; acc = row i of A G):
// RESID:  r = Rin - acc;  Rout = r;  Dn = D^{-1} r / theta
// step j: r = Rin - acc;  X = (first ? 0 : X) + G;  then, unless last, Rout = r and
//         Dn = c1 G + c2 D^{-1} r; when last, Rout = r only if Rout is given
// (c1, c2: the tabulated coefficients of the step)
template <typename T, bool RESID>
__device__ __forceinline__ void smooth_row(T acc, int i, const T* G, const T* Rin, T* Rout, T* X, int first, int last,
                                           T* Dn, const T* __restrict__ dinv, double theta, double c1, double c2) {
    const T r = Rin[i] - acc;
    if constexpr (RESID) {
        Rout[i] = r;
        Dn[i] = dinv[i] * r / (T)theta;
    } else {
        const T dj = G[i];
        X[i] = (first ? (T)0 : X[i]) + dj;
        if (last) {
            if (Rout) Rout[i] = r;
            return;
        }
        Rout[i] = r;
        Dn[i] = (T)c1 * dj + (T)c2 * (dinv[i] * r);
    }
}

// One smoothing launch on a level, for every direction still running (done[k] >= it):
// RESID:  q = A x;  r = b - q;  d_0 = D^{-1} r / theta                (G = x, Rin = b)
// step j: q = A d_j;  r' = r_j - q;  x_{j+1} = (first ? 0 : x_j) + d_j;  then, unless last,
//         r = r', d_{j+1} = c1 d_j + c2 D^{-1} r'; when last, r = r' only if Rout is given
//                                                                     (G = d_j)
template <int WMAX, typename T, bool RESID, typename VT = typename SmoothVal<T>::V>
__global__ __launch_bounds__(MTB) void mg_smooth_kernel(int n, int nS, int ntiles, int nslice, int it,
                                                        const int* __restrict__ sptr, const int* __restrict__ col,
                                                        const VT* __restrict__ val, size_t len,
                                                        const T* __restrict__ G, const T* Rin, T* Rout, T* X,
                                                        int first, int last, T* __restrict__ Dn,
                                                        const T* __restrict__ dinv, const double* __restrict__ cheb,
                                                        int j, const int* __restrict__ done) {
    int k, t;
    if (!dir_tile(ntiles, nS, k, t)) return;
    if (done && done[k] < it) return;
    const int lane = threadIdx.x & 63;
    const int sl = t * (MTB / 64) + (threadIdx.x >> 6);
    if (sl >= nslice) return;
    const T* g = G + (size_t)n * k;
    const T acc = ell_row<WMAX, T, VT>(sptr, col, val + len * k, g, sl, lane);
    const int i = sl * 64 + lane;
    if (i >= n) return;
    const size_t o = (size_t)n * k;
    const double* cf = cheb + 2 * (size_t)nS + ((size_t)k * kMgChebSteps + j) * 2;
    smooth_row<T, RESID>(acc, i, g, Rin + o, Rout ? Rout + o : nullptr, X ? X + o : nullptr, first, last, Dn + o,
                         dinv + o, cheb[2 * k], cf[0], cf[1]);
}

__device__ __forceinline__ void lattice_coords(int v, int m, int d, int* c) {
    for (int a = 0; a < d; ++a, v /= m) c[a] = v % m;
}
__device__ __forceinline__ int lattice_index(const int* c, int m, int d) {
    int v = 0;
    for (int a = d - 1; a >= 0; --a) v = v * m + c[a];
    return v;
}

// (P^T r)_I for one direction's fine vector r: r at fine 2I, plus half of r at 2I +- e_S for
// every nonempty axis set S, in bounds
template <typename T>
__device__ __forceinline__ T restrict_row(int d, int mf, int mc, const T* r, int I) {
    int c[3];
    lattice_coords(I, mc, d, c);
    int q[3];
    for (int a = 0; a < d; ++a) q[a] = 2 * c[a];
    T acc = r[lattice_index(q, mf, d)];
    const int nsets = (1 << d) - 1;
    for (int S = 1; S <= nsets; ++S)
        for (int sg = -1; sg <= 1; sg += 2) {
            bool in = true;
            for (int a = 0; a < d; ++a) {
                q[a] = 2 * c[a] + ((S >> a) & 1) * sg;
                in = in && q[a] >= 0 && q[a] < mf;
            }
            if (in) acc += (T)0.5 * r[lattice_index(q, mf, d)];
        }
    return acc;
}

// b_c = P^T r_f, and the coarse level's d_0 = D^{-1} b_c / theta
template <typename T>
__global__ __launch_bounds__(MTB) void mg_restrict_kernel(int d, int mf, int mc, int nf, int nc, int nS, int ntiles,
                                                          int it, const T* __restrict__ Rf, T* __restrict__ Bc,
                                                          T* __restrict__ Dc, const T* __restrict__ dinv_c,
                                                          const double* __restrict__ cheb_c,
                                                          const int* __restrict__ done) {
    int k, t;
    if (!dir_tile(ntiles, nS, k, t)) return;
    if (done && done[k] < it) return;
    const int I = t * MTB + threadIdx.x;
    if (I >= nc) return;
    const T acc = restrict_row(d, mf, mc, Rf + (size_t)nf * k, I);
    const size_t o = (size_t)nc * k + I;
    Bc[o] = acc;
    Dc[o] = dinv_c[o] * acc / (T)cheb_c[2 * k];
}

// (P e)_f for one direction, e = x_c + d_c (the coarse level's last smoothing step)
template <typename T>
__device__ __forceinline__ T prolong_row(int d, int mf, int mc, const T* Xc, const T* Dc, int f) {
    int c[3], lo[3], hi[3];
    lattice_coords(f, mf, d, c);
    for (int a = 0; a < d; ++a) {
        lo[a] = c[a] / 2;
        hi[a] = (c[a] + 1) / 2;
    }
    const int il = lattice_index(lo, mc, d), ih = lattice_index(hi, mc, d);
    const T el = Xc[il] + Dc[il];
    T e = el;
    if (ih != il) e = (T)0.5 * (el + (Xc[ih] + Dc[ih]));
    return e;
}

// x_f += P e, e = x_c + d_c
template <typename T>
__global__ __launch_bounds__(MTB) void mg_prolong_kernel(int d, int mf, int mc, int nf, int nc, int nS, int ntiles,
                                                         int it, const T* __restrict__ Xc, const T* __restrict__ Dc,
                                                         T* __restrict__ Xf, const int* __restrict__ done) {
    int k, t;
    if (!dir_tile(ntiles, nS, k, t)) return;
    if (done && done[k] < it) return;
    const int f = t * MTB + threadIdx.x;
    if (f >= nf) return;
    const size_t oc = (size_t)nc * k;
    Xf[(size_t)nf * k + f] += prolong_row(d, mf, mc, Xc + oc, Dc + oc, f);
}

// D = D^{-1} B / theta (the start of a cycle)
template <typename T>
__global__ __launch_bounds__(MTB) void mg_start_kernel(int n, int nS, int ntiles, const T* __restrict__ B,
                                                       T* __restrict__ D, const T* __restrict__ dinv,
                                                       const double* __restrict__ cheb) {
    int k, t;
    if (!dir_tile(ntiles, nS, k, t)) return;
    const int i = t * MTB + threadIdx.x;
    if (i >= n) return;
    const size_t o = (size_t)n * k + i;
    D[o] = dinv[o] * B[o] / (T)cheb[2 * k];
}

// Y = X + D (FP64 output)
template <typename T>
__global__ __launch_bounds__(MTB) void mg_sum_kernel(int n, int nS, int ntiles, const T* __restrict__ X,
                                                     const T* __restrict__ D, double* __restrict__ Y) {
    int k, t;
    if (!dir_tile(ntiles, nS, k, t)) return;
    const int i = t * MTB + threadIdx.x;
    if (i >= n) return;
    const size_t o = (size_t)n * k + i;
    Y[o] = (double)(X[o] + D[o]);
}

template <typename T>
__global__ void mg_cast_kernel(size_t n, const double* __restrict__ X, T* __restrict__ Y) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        Y[i] = (T)X[i];
}

// inverse diagonal of every row and Gershgorin's ratio sum_j |a_ij| / a_ii, its maximum per tile
template <int WMAX, typename T, typename VT = typename SmoothVal<T>::V>
__global__ __launch_bounds__(MTB) void mg_diag_kernel(int n, int nS, int ntiles, int nslice,
                                                      const int* __restrict__ sptr, const int* __restrict__ col,
                                                      const VT* __restrict__ val, size_t len, T* __restrict__ dinv,
                                                      double* __restrict__ part) {
    __shared__ double sh[8];
    int k, t;
    if (!dir_tile(ntiles, nS, k, t)) return;
    const int lane = threadIdx.x & 63;
    const int sl = t * (MTB / 64) + (threadIdx.x >> 6);
    const int i = sl * 64 + lane;
    double ratio = 0.0;
    if (sl < nslice && i < n) {
        const int g0 = sptr[sl];
        const int wd = sptr[sl + 1] - g0;
        const VT* v = val + len * k;
        double dg = 0.0, ab = 0.0;
        for (int j = 0; j < wd; ++j) {
            const size_t q = (size_t)(g0 + j) * 64 + lane;
            const double a = (double)sval(v[q], T());
            if (col[q] == i) dg += a;
            ab += fabs(a);
        }
        dinv[(size_t)n * k + i] = (T)(1.0 / dg);
        ratio = ab / dg;
    }
    ratio = block_max(ratio, sh);
    if (threadIdx.x == 0) part[(size_t)k * ntiles + t] = ratio;
}

// lam = the largest ratio of direction k; theta = (lam + lo lam) / 2, delta = (lam - lo lam) / 2;
// the coefficients c1, c2 of steps 0 .. kMgChebSteps - 1 after them (lane j: step j)
__global__ __launch_bounds__(64) void mg_cheb_kernel(int nS, int ntiles, double lo, const double* __restrict__ part,
                                                     double* __restrict__ cheb) {
    const int k = blockIdx.x;
    double m = 0.0;
    for (int i = threadIdx.x; i < ntiles; i += 64) m = fmax(m, part[(size_t)k * ntiles + i]);
    m = dev::wave_max(m);
    const double theta = 0.5 * (m + lo * m), delta = 0.5 * (m - lo * m);
    if (threadIdx.x == 0) {
        cheb[2 * k] = theta;
        cheb[2 * k + 1] = delta;
    }
    if (threadIdx.x < kMgChebSteps) {
        double c1, c2;
        cheb_coef(theta, delta, threadIdx.x, c1, c2);
        double* cf = cheb + 2 * (size_t)nS + ((size_t)k * kMgChebSteps + threadIdx.x) * 2;
        cf[0] = c1;
        cf[1] = c2;
    }
}

// smoother values of a level from its class values: formed in FP64, then rounded
template <typename VT>
__global__ void mg_fill_kernel(int nS, size_t len, int nnz, int ncls, const int* __restrict__ ell_e,
                               const double* __restrict__ cls, const double* __restrict__ coef, VT* __restrict__ val) {
    const size_t total = len * nS;
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < total; q += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(q / len);
        const int e = ell_e[q % len];
        double v = 0.0;
        if (e >= 0)
            for (int c = 0; c < ncls; ++c) v = fma(coef[(size_t)k * ncls + c], cls[(size_t)c * nnz + e], v);
        round_to(v, val[q]);
    }
}

template <typename TS, typename VT>
__global__ void mg_round_kernel(const TS* __restrict__ src, VT* __restrict__ dst, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        round_to(src[i], dst[i]);
}

inline unsigned grid_elems(size_t n) { return (unsigned)std::min<size_t>((n + 255) / 256, 65536); }

// ---- the CG around the cycle

// x = 0, r = b, the cycle's d_0 = D^{-1} r / theta; partials b.b
template <typename T>
__global__ __launch_bounds__(MTB) void mgcg_init_kernel(int n, int nS, int ntiles, const double* __restrict__ B,
                                                        double* __restrict__ X, T* __restrict__ R, T* __restrict__ D0,
                                                        const T* __restrict__ dinv0, const double* __restrict__ cheb0,
                                                        double* __restrict__ part) {
    __shared__ double sh[8];
    int k, t;
    if (!dir_tile(ntiles, nS, k, t)) return;
    const int i = t * MTB + threadIdx.x;
    double bb = 0.0;
    if (i < n) {
        const size_t o = (size_t)n * k + i;
        const double b = B[o];
        X[o] = 0.0;
        const T r = (T)b;
        R[o] = r;
        D0[o] = dinv0[o] * r / (T)cheb0[2 * k];
        bb = b * b;
    }
    bb = block_sum(bb, sh);
    if (threadIdx.x == 0) part[(size_t)k * ntiles + t] = bb;
}

// z = x_0 + d (the cycle's result); partials r.z into part[(off + k) ntiles + t]; p = z when first
template <typename T>
__global__ __launch_bounds__(MTB) void mgcg_rz_kernel(int n, int nS, int ntiles, int it, const T* __restrict__ X0,
                                                      const T* __restrict__ D, const T* __restrict__ R,
                                                      T* __restrict__ P, int first, const int* __restrict__ done,
                                                      double* __restrict__ part, int off) {
    __shared__ double sh[8];
    int k, t;
    if (!dir_tile(ntiles, nS, k, t)) return;
    if (done && done[k] < it) return;
    const int i = t * MTB + threadIdx.x;
    double rz = 0.0;
    if (i < n) {
        const size_t o = (size_t)n * k + i;
        const T z = X0[o] + D[o];
        rz = (double)R[o] * (double)z;
        if (first) P[o] = z;
    }
    rz = block_sum(rz, sh);
    if (threadIdx.x == 0) part[(size_t)(off + k) * ntiles + t] = rz;
}

// alpha = rz / p.q; x += alpha p; r -= alpha q; the cycle's d_0; partials r.r
template <typename T>
__global__ __launch_bounds__(MTB) void mgcg_update_kernel(int n, int nS, int ntiles, int it, const T* __restrict__ P,
                                                          const T* __restrict__ Q, T* __restrict__ R,
                                                          double* __restrict__ X, T* __restrict__ D0,
                                                          const T* __restrict__ dinv0,
                                                          const double* __restrict__ cheb0,
                                                          const double* __restrict__ rz, const int* __restrict__ done,
                                                          const double* __restrict__ part_pq,
                                                          double* __restrict__ part_rr) {
    __shared__ double sh[8];
    int k, t;
    if (!dir_tile(ntiles, nS, k, t)) return;
    if (done[k] < it) return;
    const double pq = partial_sum(part_pq + (size_t)k * ntiles, ntiles, sh);
    const double a = pq != 0.0 ? rz[(size_t)(it & 1) * nS + k] / pq : 0.0;
    const int i = t * MTB + threadIdx.x;
    double rr = 0.0;
    if (i < n) {
        const size_t o = (size_t)n * k + i;
        X[o] = fma(a, (double)P[o], X[o]);
        const T r = R[o] - (T)a * Q[o];
        R[o] = r;
        D0[o] = dinv0[o] * r / (T)cheb0[2 * k];
        rr = (double)r * (double)r;
    }
    rr = block_sum(rr, sh);
    if (threadIdx.x == 0) part_rr[(size_t)k * ntiles + t] = rr;
}

// stop direction k at iteration it once r.r <= tol^2 b.b
__global__ __launch_bounds__(MTB) void mgcg_check_kernel(int nS, int ntiles, int it, const double* __restrict__ part_rr,
                                                         const double* __restrict__ stop, int* __restrict__ done,
                                                         int* __restrict__ iters) {
    __shared__ double sh[8];
    const int k = blockIdx.x;
    if (done[k] < it) return;
    const double rr = partial_sum(part_rr + (size_t)k * ntiles, ntiles, sh);
    if (threadIdx.x == 0 && rr <= stop[k]) {
        done[k] = it;
        iters[k] = it + 1;
    }
}

// beta = r.z / rz_old; p = z + beta p (z = x_0 + d); rz_new into the other slot
template <typename T>
__global__ __launch_bounds__(MTB) void mgcg_dir_kernel(int n, int nS, int ntiles, int it, T* __restrict__ P,
                                                       const T* __restrict__ X0, const T* __restrict__ D,
                                                       double* __restrict__ rz, const int* __restrict__ done,
                                                       const double* __restrict__ part) {
    __shared__ double sh[8];
    int k, t;
    if (!dir_tile(ntiles, nS, k, t)) return;
    if (done[k] <= it) return;
    const double rzn = partial_sum(part + (size_t)k * ntiles, ntiles, sh);
    const double rzo = rz[(size_t)(it & 1) * nS + k];
    const double b = rzo != 0.0 ? rzn / rzo : 0.0;
    const int i = t * MTB + threadIdx.x;
    if (i < n) {
        const size_t o = (size_t)n * k + i;
        P[o] = (X0[o] + D[o]) + (T)b * P[o];
    }
    if (t == 0 && threadIdx.x == 0) rz[(size_t)((it + 1) & 1) * nS + k] = rzn;
}

inline int tiles_of(int n) { return (n + MTB - 1) / MTB; }
inline dim3 grid_dir(int n, int nS) { return dim3((unsigned)tiles_of(n) * 8u * (unsigned)((nS + 7) / 8)); }

template <typename T, bool RESID>
void smooth_launch(const MgArgs& g, int l, int it, const T* G, const T* Rin, T* Rout, T* X, int first, int last, T* Dn,
                   int j, const int* done, hipStream_t s) {
    const MgLevelArgs& L = g.lev[l];
    const int ntiles = tiles_of(L.n);
    auto f = L.wmax <= 7    ? mg_smooth_kernel<7, T, RESID>
             : L.wmax <= 15 ? mg_smooth_kernel<15, T, RESID>
                            : mg_smooth_kernel<0, T, RESID>;
    typedef typename SmoothVal<T>::V VT;
    hipLaunchKernelGGL(f, grid_dir(L.n, g.nS), dim3(MTB), 0, s, L.n, g.nS, ntiles, L.nslice, it, L.sptr, L.col,
                       static_cast<const VT*>(L.val), L.len, G, Rin, Rout, X, first, last, Dn,
                       static_cast<const T*>(L.dinv), L.cheb, j, done);
    RTE_CHECK_LAUNCH();
}

// ---- the coarse tail of the cycle in one launch
//
// The coarse levels hold a few hundred rows per direction, and their per-level launches are
// bound by launch latency, not by their bytes.  From level t0 down (the coarse levels whose five
// vectors fit in kTailLds bytes of LDS together; level 0 is never among them) one work-group per
// direction runs the rest of the cycle: the restriction from level t0 - 1, the descent, the
// coarsest level, the ascent and the prolongation back into level t0 - 1, with the vectors of
// every tail level in LDS and barriers in place of launch boundaries.  Matrix values, columns and
// inverse diagonals are read from global memory (the coarse levels of all directions stay in
// L2).  Each row's arithmetic is that of the per-level launches (the same row functions).
constexpr int TTB = 1024;                      // threads of a tail work-group
constexpr size_t kTailLds = 64 * 1024;         // LDS bytes for the tail's vectors

template <int WMAX, typename T>
__global__ __launch_bounds__(TTB) void mg_tail_kernel(MgArgs g, int t0, int it, const int* __restrict__ done) {
    typedef typename SmoothVal<T>::V VT;
    extern __shared__ __attribute__((aligned(16))) unsigned char tail_lds[];
    const int k = blockIdx.x;                  // on XCD k mod 8, where the per-level launches put direction k
    if (done && done[k] < it) return;
    const int L = g.L, tid = threadIdx.x;
    T* const lds = reinterpret_cast<T*>(tail_lds);
    // the vectors x, r, b, d0, d1 of tail level l (n_l each) from lds + 5 (n_t0 + ... + n_{l-1})
    auto vec = [&](int l) __attribute__((always_inline)) {
        size_t o = 0;
        for (int j = t0; j < l; ++j) o += 5 * (size_t)g.lev[j].n;
        return lds + o;
    };
    // one smoothing step of level l (smooth_row), then a barrier
    auto step = [&](int l, const T* G, const T* Rin, T* Rout, T* X, int first, int last, T* Dn, int j,
                    bool resid) __attribute__((always_inline)) {
        const MgLevelArgs& V = g.lev[l];
        const VT* val = static_cast<const VT*>(V.val) + V.len * k;
        const T* dinv = static_cast<const T*>(V.dinv) + (size_t)V.n * k;
        const double theta = V.cheb[2 * k];
        const double* cf = V.cheb + 2 * (size_t)g.nS + ((size_t)k * kMgChebSteps + j) * 2;
        const double c1 = cf[0], c2 = cf[1];
        for (int i = tid; i < V.n; i += TTB) {
            const T acc = ell_row<WMAX, T, VT, false>(V.sptr, V.col, val, G, i >> 6, i & 63);
            if (resid) smooth_row<T, true>(acc, i, G, Rin, Rout, X, first, last, Dn, dinv, theta, c1, c2);
            else smooth_row<T, false>(acc, i, G, Rin, Rout, X, first, last, Dn, dinv, theta, c1, c2);
        }
        __syncthreads();
    };
    // b and d_0 of level c from the residual rf of level c - 1, then a barrier
    auto restrict_to = [&](int c, const T* rf) __attribute__((always_inline)) {
        const MgLevelArgs& C = g.lev[c];
        T* v = vec(c);
        const T* dinv = static_cast<const T*>(C.dinv) + (size_t)C.n * k;
        const double theta = C.cheb[2 * k];
        for (int I = tid; I < C.n; I += TTB) {
            const T acc = restrict_row(g.d, g.lev[c - 1].m, C.m, rf, I);
            v[2 * C.n + I] = acc;
            v[3 * C.n + I] = dinv[I] * acc / (T)theta;
        }
        __syncthreads();
    };

    restrict_to(t0, static_cast<const T*>(g.lev[t0 - 1].r) + (size_t)g.lev[t0 - 1].n * k);
    // descent: nu steps from 0, the last forming the residual; restriction to the next level
    for (int l = t0; l + 1 < L; ++l) {
        const int n = g.lev[l].n;
        T* v = vec(l);
        T *x = v, *r = v + n, *b = v + 2 * n, *cur = v + 3 * n, *nxt = v + 4 * n;
        for (int j = 0; j < kMgNu; ++j) {
            step(l, cur, j == 0 ? b : r, r, x, j == 0, j + 1 == kMgNu, nxt, j, false);
            T* t = cur; cur = nxt; nxt = t;
        }
        restrict_to(l + 1, r);
    }
    // coarsest level: nu_c steps from 0, the last one's x + d left to the prolongation
    const T* ec;
    {
        const int n = g.lev[L - 1].n;
        T* v = vec(L - 1);
        T *x = v, *r = v + n, *b = v + 2 * n, *cur = v + 3 * n, *nxt = v + 4 * n;
        for (int j = 0; j + 1 < kMgNuCoarse; ++j) {
            step(L - 1, cur, j == 0 ? b : r, r, x, j == 0, 0, nxt, j, false);
            T* t = cur; cur = nxt; nxt = t;
        }
        ec = cur;
    }
    // ascent: x += P e, residual and d_0, nu - 1 full steps
    for (int l = L - 2; l >= t0; --l) {
        const int n = g.lev[l].n;
        T* v = vec(l);
        T *x = v, *r = v + n, *b = v + 2 * n, *cur = v + 3 * n, *nxt = v + 4 * n;
        const T* xc = vec(l + 1);
        for (int f = tid; f < n; f += TTB) x[f] += prolong_row(g.d, g.lev[l].m, g.lev[l + 1].m, xc, ec, f);
        __syncthreads();
        step(l, x, b, r, nullptr, 0, 0, cur, 0, true);
        for (int j = 0; j + 1 < kMgNu; ++j) {
            step(l, cur, r, r, x, 0, 0, nxt, j, false);
            T* t = cur; cur = nxt; nxt = t;
        }
        ec = cur;
    }
    // x of level t0 - 1 (global) += P e
    const MgLevelArgs& F = g.lev[t0 - 1];
    T* xf = static_cast<T*>(F.x) + (size_t)F.n * k;
    const T* xc = vec(t0);
    for (int f = tid; f < F.n; f += TTB) xf[f] += prolong_row(g.d, F.m, g.lev[t0].m, xc, ec, f);
}

// the first level of the fused tail: the longest run of coarsest levels, level 0 excluded, whose
// five vectors fit in kTailLds bytes; L when there is none
inline int tail_start(const MgArgs& g, size_t elem) {
    size_t rows = 0;
    int t0 = g.L;
    for (int l = g.L - 1; l >= 1; --l) {
        rows += (size_t)g.lev[l].n;
        if (5 * rows * elem > kTailLds) break;
        t0 = l;
    }
    return t0;
}

template <typename T>
void tail_launch(const MgArgs& g, int t0, int it, const int* done, hipStream_t s) {
    int wmax = 0;
    size_t rows = 0;
    for (int l = t0; l < g.L; ++l) {
        wmax = std::max(wmax, g.lev[l].wmax);
        rows += (size_t)g.lev[l].n;
    }
    const size_t lds = 5 * rows * sizeof(T);
    if (t0 < 1 || t0 >= g.L || lds > kTailLds) fail(RTE_E_ARG, "multigrid: bad coarse tail");
    auto f = wmax <= 7 ? mg_tail_kernel<7, T> : wmax <= 15 ? mg_tail_kernel<15, T> : mg_tail_kernel<0, T>;
    hipLaunchKernelGGL(f, dim3(g.nS), dim3(TTB), lds, s, g, t0, it, done);
    RTE_CHECK_LAUNCH();
}

template <typename T>
const T* vcycle_t(const MgArgs& g, int it, const int* done, hipStream_t s) {
    const int L = g.L;
    const int t0 = tail_start(g, sizeof(T));       // levels t0.. run in the fused tail (none when L)
    const T* ecur[kMgMaxLevels] = {};
    // descent: nu Chebyshev steps from 0 (d_0 is in d0), the last also forming the residual;
    // restriction to the next level with its d_0 (into the tail's first level: the tail's own)
    for (int l = 0; l + 1 < L && l < t0; ++l) {
        const MgLevelArgs& V = g.lev[l];
        T* x = static_cast<T*>(V.x);
        T* r = static_cast<T*>(V.r);
        T* cur = static_cast<T*>(V.d0);
        T* nxt = static_cast<T*>(V.d1);
        for (int j = 0; j < kMgNu; ++j) {
            const bool last = j + 1 == kMgNu;
            smooth_launch<T, false>(g, l, it, cur, j == 0 ? static_cast<const T*>(V.b) : r, r, x, j == 0, last, nxt,
                                    j, done, s);
            std::swap(cur, nxt);
        }
        if (l + 1 == t0) break;
        const MgLevelArgs& C = g.lev[l + 1];
        hipLaunchKernelGGL(mg_restrict_kernel<T>, grid_dir(C.n, g.nS), dim3(MTB), 0, s, g.d, V.m, C.m, V.n, C.n, g.nS,
                           tiles_of(C.n), it, (const T*)r, static_cast<T*>(C.b), static_cast<T*>(C.d0),
                           static_cast<const T*>(C.dinv), C.cheb, done);
        RTE_CHECK_LAUNCH();
    }
    if (t0 < L) {
        tail_launch<T>(g, t0, it, done, s);            // ends with x of level t0 - 1 += P e
    } else {   // coarsest level: kMgNuCoarse steps from 0, the last one's x + d left to the prolongation
        const MgLevelArgs& V = g.lev[L - 1];
        T* x = static_cast<T*>(V.x);
        T* r = static_cast<T*>(V.r);
        T* cur = static_cast<T*>(V.d0);
        T* nxt = static_cast<T*>(V.d1);
        for (int j = 0; j + 1 < kMgNuCoarse; ++j) {
            smooth_launch<T, false>(g, L - 1, it, cur, j == 0 ? static_cast<const T*>(V.b) : r, r, x, j == 0, false,
                                    nxt, j, done, s);
            std::swap(cur, nxt);
        }
        ecur[L - 1] = cur;
    }
    // ascent: x += P e (for level t0 - 1 the tail did it), residual and d_0, nu - 1 full steps;
    // the last x + d left to the caller
    for (int l = std::min(L - 2, t0 - 1); l >= 0; --l) {
        const MgLevelArgs& V = g.lev[l];
        const MgLevelArgs& C = g.lev[l + 1];
        T* x = static_cast<T*>(V.x);
        T* r = static_cast<T*>(V.r);
        if (l + 1 < t0) {
            hipLaunchKernelGGL(mg_prolong_kernel<T>, grid_dir(V.n, g.nS), dim3(MTB), 0, s, g.d, V.m, C.m, V.n, C.n,
                               g.nS, tiles_of(V.n), it, static_cast<const T*>(C.x), ecur[l + 1], x, done);
            RTE_CHECK_LAUNCH();
        }
        T* cur = static_cast<T*>(V.d0);
        T* nxt = static_cast<T*>(V.d1);
        smooth_launch<T, true>(g, l, it, x, static_cast<const T*>(V.b), r, nullptr, 0, 0, cur, 0, done, s);
        for (int j = 0; j + 1 < kMgNu; ++j) {
            smooth_launch<T, false>(g, l, it, cur, r, r, x, 0, 0, nxt, j, done, s);
            std::swap(cur, nxt);
        }
        ecur[l] = cur;
    }
    return ecur[0];
}

// the phases of one multigrid-preconditioned CG
template <typename T>
struct MgRun : CgPhases {
    MgArgs g;
    const T* val;
    T *R, *P, *Q;
    int ntiles;
    double *part_a, *part_b;
    MgRun(const CgJob& j)
        : CgPhases(j.a, j.s), g(*j.mg), val(static_cast<const T*>(j.val)), R(static_cast<T*>(j.R)),
          P(static_cast<T*>(j.P)), Q(static_cast<T*>(j.Q)) {
        g.lev[0].b = R;                                    // the cycle's right-hand side is the CG residual
        ntiles = tiles_of(a.n);
        part_a = a.part;                                   // [2 nS ntiles]
        part_b = a.part + (size_t)2 * a.nS * ntiles;       // [2 nS ntiles]
    }
    T* x0() const { return static_cast<T*>(g.lev[0].x); }
    void start() override {
        const MgLevelArgs& V = g.lev[0];
        hipLaunchKernelGGL(mgcg_init_kernel<T>, grid_dir(a.n, a.nS), dim3(MTB), 0, s, a.n, a.nS, ntiles, a.B, a.X, R,
                           static_cast<T*>(V.d0), static_cast<const T*>(V.dinv), V.cheb, part_a);
        RTE_CHECK_LAUNCH();
        const T* d = vcycle_t<T>(g, 0, nullptr, s);
        hipLaunchKernelGGL(mgcg_rz_kernel<T>, grid_dir(a.n, a.nS), dim3(MTB), 0, s, a.n, a.nS, ntiles, 0,
                           (const T*)x0(), d, (const T*)R, P, 1, nullptr, part_a, a.nS);
        RTE_CHECK_LAUNCH();
        cg_setup(a, part_a, s);
    }
    void iterate(int it) override {
        const MgLevelArgs& V = g.lev[0];
        cg_spmv_it(a, it, val, (const T*)P, Q, s);
        hipLaunchKernelGGL(mgcg_update_kernel<T>, grid_dir(a.n, a.nS), dim3(MTB), 0, s, a.n, a.nS, ntiles, it,
                           (const T*)P, (const T*)Q, R, a.X, static_cast<T*>(V.d0), static_cast<const T*>(V.dinv),
                           V.cheb, (const double*)a.rz, (const int*)a.done, (const double*)part_a,
                           part_b + (size_t)a.nS * ntiles);
        RTE_CHECK_LAUNCH();
        hipLaunchKernelGGL(mgcg_check_kernel, dim3(a.nS), dim3(MTB), 0, s, a.nS, ntiles, it,
                           (const double*)(part_b + (size_t)a.nS * ntiles), (const double*)a.stop, a.done, a.iters);
        RTE_CHECK_LAUNCH();
        // the cycle and the rest of the iteration skip the directions that stopped at it
        const T* d = vcycle_t<T>(g, it + 1, a.done, s);
        hipLaunchKernelGGL(mgcg_rz_kernel<T>, grid_dir(a.n, a.nS), dim3(MTB), 0, s, a.n, a.nS, ntiles, it + 1,
                           (const T*)x0(), d, (const T*)R, (T*)nullptr, 0, (const int*)a.done, part_b, 0);
        RTE_CHECK_LAUNCH();
        hipLaunchKernelGGL(mgcg_dir_kernel<T>, grid_dir(a.n, a.nS), dim3(MTB), 0, s, a.n, a.nS, ntiles, it, P,
                           (const T*)x0(), d, a.rz, (const int*)a.done, (const double*)part_b);
        RTE_CHECK_LAUNCH();
    }
};

template <typename T>
void level_setup_t(const MgArgs& g, int l, double lo, double* part, hipStream_t s) {
    const MgLevelArgs& L = g.lev[l];
    const int ntiles = tiles_of(L.n);
    typedef typename SmoothVal<T>::V VT;
    auto f = mg_diag_kernel<0, T>;
    hipLaunchKernelGGL(f, grid_dir(L.n, g.nS), dim3(MTB), 0, s, L.n, g.nS, ntiles, L.nslice, L.sptr, L.col,
                       static_cast<const VT*>(L.val), L.len, static_cast<T*>(const_cast<void*>(L.dinv)), part);
    RTE_CHECK_LAUNCH();
    hipLaunchKernelGGL(mg_cheb_kernel, dim3(g.nS), dim3(64), 0, s, g.nS, ntiles, lo, (const double*)part,
                       const_cast<double*>(L.cheb));
    RTE_CHECK_LAUNCH();
}

template <typename T>
void apply_t(const MgArgs& g0, const double* X, double* Y, hipStream_t s) {
    const MgLevelArgs& V = g0.lev[0];
    const size_t nn = (size_t)V.n * g0.nS;
    T* b = static_cast<T*>(V.b);
    hipLaunchKernelGGL(mg_cast_kernel<T>, dim3((unsigned)std::min<size_t>((nn + 255) / 256, 65536)), dim3(256), 0, s,
                       nn, X, b);
    RTE_CHECK_LAUNCH();
    hipLaunchKernelGGL(mg_start_kernel<T>, grid_dir(V.n, g0.nS), dim3(MTB), 0, s, V.n, g0.nS, tiles_of(V.n),
                       (const T*)b, static_cast<T*>(V.d0), static_cast<const T*>(V.dinv), V.cheb);
    RTE_CHECK_LAUNCH();
    const T* d = vcycle_t<T>(g0, 0, nullptr, s);
    hipLaunchKernelGGL(mg_sum_kernel<T>, grid_dir(V.n, g0.nS), dim3(MTB), 0, s, V.n, g0.nS, tiles_of(V.n),
                       (const T*)static_cast<T*>(V.x), d, Y);
    RTE_CHECK_LAUNCH();
}

}  // namespace

namespace k {

const void* mg_vcycle(const MgArgs& g, int it, const int* done, hipStream_t s) {
    if (g.L < 1 || g.L > kMgMaxLevels) fail(RTE_E_ARG, "multigrid: bad level count");
    return g.f32 ? static_cast<const void*>(vcycle_t<float>(g, it, done, s))
                 : static_cast<const void*>(vcycle_t<double>(g, it, done, s));
}

void mg_apply(const MgArgs& g, const double* X, double* Y, hipStream_t s) {
    if (g.L < 1 || g.L > kMgMaxLevels) fail(RTE_E_ARG, "multigrid: bad level count");
    if (g.f32) apply_t<float>(g, X, Y, s);
    else apply_t<double>(g, X, Y, s);
}

void mg_level_setup(const MgArgs& g, int l, double lo, double* part, hipStream_t s) {
    if (g.f32) level_setup_t<float>(g, l, lo, part, s);
    else level_setup_t<double>(g, l, lo, part, s);
}

void mg_fill_smoother(int nS, size_t len, int nnz, int ncls, const int* ell_e, const double* cls, const double* coef,
                      float* val, hipStream_t s) {
    hipLaunchKernelGGL(mg_fill_kernel<float>, dim3(grid_elems(len * nS)), dim3(256), 0, s, nS, len, nnz, ncls, ell_e,
                       cls, coef, val);
    RTE_CHECK_LAUNCH();
}
void mg_fill_smoother(int nS, size_t len, int nnz, int ncls, const int* ell_e, const double* cls, const double* coef,
                      uint16_t* val, hipStream_t s) {
    hipLaunchKernelGGL(mg_fill_kernel<uint16_t>, dim3(grid_elems(len * nS)), dim3(256), 0, s, nS, len, nnz, ncls,
                       ell_e, cls, coef, val);
    RTE_CHECK_LAUNCH();
}
void mg_round(const double* src, float* dst, size_t n, hipStream_t s) {
    hipLaunchKernelGGL((mg_round_kernel<double, float>), dim3(grid_elems(n)), dim3(256), 0, s, src, dst, n);
    RTE_CHECK_LAUNCH();
}
void mg_round(const float* src, uint16_t* dst, size_t n, hipStream_t s) {
    hipLaunchKernelGGL((mg_round_kernel<float, uint16_t>), dim3(grid_elems(n)), dim3(256), 0, s, src, dst, n);
    RTE_CHECK_LAUNCH();
}

std::unique_ptr<CgPhases> mg_phases(const CgJob& j) {
    if (!j.mg || j.mg->L < 1) fail(RTE_E_ARG, "multigrid CG without a hierarchy");
    if (j.f32) return std::make_unique<MgRun<float>>(j);
    return std::make_unique<MgRun<double>>(j);
}

}  // namespace k
}  // namespace rte
