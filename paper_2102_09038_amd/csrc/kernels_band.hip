// Banded Cholesky factorisation and solves.
//
// E_0 is block diagonal with one sparse SPD block per direction (paper Sec. 5.3); the
// paper applies E_0^{-1} with a sparse direct factorisation (Sec. 6.4).  Here every
// block is factored once, on the GPU, as a band matrix in a bandwidth-reducing vertex
// order, and each application of E_0^{-1} streams the factor twice (forward and
// backward), which makes it HBM bound.  The coarse matrix E_c (Sec. 5.4) uses the same
// solve kernel.
//
// Blocked band layout, coalesced for one 64-lane wave per system: for band width bw and
// row r = 64 B + lane,
//   BL[(B (bw+1) + t) 64 + lane] = L(r, r - bw + t),   t = 0..bw,  t = bw holds 1 / L(r,r);
// entries outside the matrix are zero.
#include "ops.h"

namespace rte {
namespace {

__device__ __forceinline__ size_t blk_idx(int row, int t, int bw) {
    return ((size_t)(row >> 6) * (bw + 1) + t) * 64 + (row & 63);
}

// ----------------------------------------------------------------------------- factor
// One 256-thread work-group per direction.  A (bw+1) x (bw+1) window of the active
// trailing matrix lives in LDS with circular row/column indices (mod bw+1).
// Step j: pivot; scale column j; write row j of L (final now); rank-one update of the
// window's lower triangle; load row j+bw+1 of the block into the slot row j vacated.
__global__ __launch_bounds__(256) void e0_band_factor_kernel(
    int n, int bw, int nnz, int ncls, const int* __restrict__ rowptr, const int* __restrict__ col,
    const double* __restrict__ cls, const double* __restrict__ coefE0, const int* __restrict__ perm,
    const int* __restrict__ iperm, double* __restrict__ BLall, size_t stride_sys, int* __restrict__ bad) {
    extern __shared__ double win[];
    __shared__ double cf[kMaxClasses];
    const int kk = blockIdx.x;
    const int w1 = bw + 1;
    double* BL = BLall + stride_sys * kk;
    if (threadIdx.x < ncls) cf[threadIdx.x] = coefE0[(size_t)kk * ncls + threadIdx.x];
    for (int e = threadIdx.x; e < w1 * w1; e += blockDim.x) win[e] = 0.0;
    __syncthreads();
    auto load_row = [&](int r) {      // lower-triangle entries of band row r, columns [r-bw, r]
        const int slot = r % w1;
        for (int c = threadIdx.x; c < w1; c += blockDim.x) win[slot * w1 + c] = 0.0;
        __syncthreads();
        const int v = iperm[r];
        for (int e = rowptr[v] + threadIdx.x; e < rowptr[v + 1]; e += blockDim.x) {
            const int pc = perm[col[e]];
            if (pc <= r && pc >= r - bw) {
                double val = 0.0;
                for (int c = 0; c < ncls; ++c) val = fma(cf[c], cls[(size_t)c * nnz + e], val);
                win[slot * w1 + pc % w1] = val;
            }
        }
    };
    for (int r = 0; r < min(n, w1); ++r) load_row(r);
    __syncthreads();
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
    int failed = 0;
    for (int j = 0; j < n; ++j) {
        const int sj = j % w1;
        const int s1 = (sj + 1 == w1) ? 0 : sj + 1;         // slot of j+1
        double djj = win[sj * w1 + sj];
        if (!(djj > 0.0)) { failed = 1; djj = 1.0; }
        const double d = sqrt(djj), id = 1.0 / d;
        const int m = min(n - 1, j + bw) - j;               // rows below the pivot in the window
        __syncthreads();
        for (int a = threadIdx.x; a < m; a += blockDim.x) {
            int si = s1 + a; if (si >= w1) si -= w1;
            win[si * w1 + sj] *= id;
        }
        if (threadIdx.x == 0) win[sj * w1 + sj] = d;
        __syncthreads();
        // row j of L is final: write it out (columns j-bw .. j)
        for (int t = threadIdx.x; t <= bw; t += blockDim.x) {
            const int c = j - bw + t;
            double v = 0.0;
            if (c >= 0) {
                int sc = sj - bw + t; if (sc < 0) sc += w1;  // c mod w1
                v = (t == bw) ? id : win[sj * w1 + sc];
            }
            BL[blk_idx(j, t, bw)] = v;
        }
        // trailing update of the lower triangle (j, j+m] x (j, j+m]
        for (int a = ty; a < m; a += 16) {
            int si = s1 + a; if (si >= w1) si -= w1;
            const double lij = win[si * w1 + sj];
            double* rowp = win + si * w1;
            for (int b = tx; b <= a; b += 16) {
                int sc = s1 + b; if (sc >= w1) sc -= w1;
                rowp[sc] = fma(-lij, win[sc * w1 + sj], rowp[sc]);
            }
        }
        __syncthreads();
        if (j + w1 < n) load_row(j + w1);
        __syncthreads();
    }
    // rows of the final partial block beyond n
    const int nb = (n + 63) / 64;
    for (int r = n + threadIdx.x; r < nb * 64; r += blockDim.x)
        for (int t = 0; t <= bw; ++t) BL[blk_idx(r, t, bw)] = 0.0;
    if (failed && threadIdx.x == 0) atomicOr(bad, 1);
}

// ----------------------------------------------------------------------------- solve
// One wave per system: L L^T x = b.  Rows in blocks of 64 (lane = row within the block).
// The contribution of earlier (forward) or later (backward) blocks is a per-lane dot
// product over coalesced band loads; the 64 x 64 triangular diagonal block is solved
// with its coefficients in registers and one broadcast per row.  y and x live in an
// LDS ring of W >= bw + 64 entries (W a power of two); y is also parked in x.
template <typename VT>
__global__ __launch_bounds__(64) void band_solve_blk_kernel(const double* __restrict__ BLall, int n, int bw,
                                                            size_t stride_sys, const VT* __restrict__ ball,
                                                            VT* __restrict__ xall, size_t stride_vec,
                                                            const int* __restrict__ iperm, int W) {
    extern __shared__ double win[];
    const int sys = blockIdx.x;
    const double* BL = BLall + stride_sys * sys;
    const VT* b = ball + stride_vec * sys;
    VT* x = xall + stride_vec * sys;
    const int lane = threadIdx.x;
    const int nblk = (n + 63) / 64;
    const int Wm = W - 1;
    // ---- forward: L y = b
    for (int B = 0; B < nblk; ++B) {
        const int row = 64 * B + lane;
        const bool ok = row < n;
        double s = ok ? (double)b[iperm ? iperm[row] : row] : 0.0;
        const size_t base = (size_t)B * (bw + 1) * 64 + lane;
        const int tmax = bw - lane;          // t < tmax: columns in earlier blocks
        const int tmin = max(0, bw - row);   // columns >= 0
        for (int t = 0; t < bw; ++t)
            if (t >= tmin && t < tmax) s = fma(-BL[base + (size_t)t * 64], win[(row - bw + t) & Wm], s);
        const double invd = BL[base + (size_t)bw * 64];
        double Ld[64];
#pragma unroll
        for (int u = 0; u < 64; ++u) {
            const int t = bw - lane + u;
            Ld[u] = (u < lane && t >= 0) ? BL[base + (size_t)t * 64] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 64; ++u) {
            const double yu = __shfl(s * invd, u, 64);
            s = fma(-Ld[u], yu, s);
        }
        if (ok) {
            win[row & Wm] = s * invd;
            x[iperm ? iperm[row] : row] = (VT)(s * invd);
        }
        __syncthreads();
    }
    // ---- backward: L^T x = y, reading column entries L(row + t, row) from BL
    for (int B = nblk - 1; B >= 0; --B) {
        const int row = 64 * B + lane;
        const bool ok = row < n;
        double s = ok ? (double)x[iperm ? iperm[row] : row] : 0.0;
        const int tmin = 64 - lane;          // t >= tmin: rows in later blocks
        for (int t = 1; t <= bw; ++t) {
            const int r2 = row + t;
            if (t >= tmin && r2 < n) s = fma(-BL[blk_idx(r2, bw - t, bw)], win[r2 & Wm], s);
        }
        const double invd = ok ? BL[blk_idx(row, bw, bw)] : 0.0;
        double Ud[64];
#pragma unroll
        for (int u = 0; u < 64; ++u) {
            const int t = u - lane;
            const int r2 = 64 * B + u;
            Ud[u] = (u > lane && t <= bw && r2 < n) ? BL[blk_idx(r2, bw - t, bw)] : 0.0;
        }
#pragma unroll
        for (int u = 63; u >= 0; --u) {
            const double xu = __shfl(s * invd, u, 64);
            s = fma(-Ud[u], xu, s);
        }
        if (ok) {
            win[row & Wm] = s * invd;
            x[iperm ? iperm[row] : row] = (VT)(s * invd);
        }
        __syncthreads();
    }
}

int pow2_at_least(int v) {
    int w = 64;
    while (w < v) w <<= 1;
    return w;
}

}  // namespace

namespace k {

size_t band_blk_size(int n, int bw) { return (size_t)((n + 63) / 64) * (bw + 1) * 64; }

void e0_band_factor(const Handle* h, int bw, const int* perm, const int* iperm, double* BL, size_t stride_sys,
                    int* bad, hipStream_t s) {
    const size_t lds = (size_t)(bw + 1) * (bw + 1) * sizeof(double);
    if (lds > 150 * 1024) fail(RTE_E_ARG, "E_0 band too wide for the LDS factorisation window");
    RTE_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&e0_band_factor_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(e0_band_factor_kernel, dim3(h->nS), dim3(256), lds, s, h->nRp, bw, h->nnz, h->ncls,
                       h->rowptr.p, h->col.p, h->cls.p, h->coefE0.p, perm, iperm, BL, stride_sys, bad);
    RTE_CHECK_LAUNCH();
}

void band_solve_blk(const double* BL, int n, int bw, int nsys, size_t stride_sys, const double* b, double* x,
                    size_t stride_vec, const int* iperm, hipStream_t s) {
    const int W = pow2_at_least(bw + 128);
    if ((size_t)W * 8 > 64 * 1024) fail(RTE_E_ARG, "band too wide for the solve window");
    hipLaunchKernelGGL(band_solve_blk_kernel<double>, dim3(nsys), dim3(64), (size_t)W * 8, s, BL, n, bw,
                       stride_sys, b, x, stride_vec, iperm, W);
    RTE_CHECK_LAUNCH();
}

}  // namespace k
}  // namespace rte
