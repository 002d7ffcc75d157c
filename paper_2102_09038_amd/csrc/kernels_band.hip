// Banded Cholesky factorisation and solves.
//
// E_0 is block diagonal with one sparse SPD block per direction (paper Sec. 5.3); the
// paper applies E_0^{-1} with a sparse direct factorisation (Sec. 6.4).  Here every
// block is factored once, on the GPU, as a band matrix in a bandwidth-reducing vertex
// order, and each application of E_0^{-1} streams the factor once per sweep (forward,
// backward), which makes it HBM bound.  The coarse matrix E_c (Sec. 5.4) uses the same
// solve kernel.
//
// Blocked band layouts, coalesced for one 64-lane wave per system: for band width bw
// and row r = 64 B + lane, t = 0..bw,
//   BL[(B (bw+1) + t) 64 + lane] = L(r, r - bw + t)   (row r of L;   t = bw: 1 / L(r,r))
//   BU[(B (bw+1) + t) 64 + lane] = L(r + t, r)        (row r of L^T; t = 0:  1 / L(r,r))
// Entries outside the matrix are zero.  Allocations carry band_pad() doubles of padding
// after the last system so the solve can prefetch past a block without clamping.
#include "ops.h"

namespace rte {
namespace {

constexpr int UNR = 32;   // loads per batch in the band solve (one wave per system: the
                          // memory-level parallelism must come from within the wave)

__device__ __forceinline__ size_t blk_idx(int row, int t, int bw) {
    return ((size_t)(row >> 6) * (bw + 1) + t) * 64 + (row & 63);
}

// ----------------------------------------------------------------------------- factor
// One 256-thread work-group per direction.  A (bw+1) x (bw+1) window of the active
// trailing matrix lives in LDS with circular row/column indices (mod bw+1).
// Step j: pivot; scale column j; write row j of L (final now) to BL and BU; rank-one
// update of the window's lower triangle; load row j+bw+1 into the slot row j vacated.
__global__ __launch_bounds__(256) void e0_band_factor_kernel(
    int n, int bw, int nnz, int ncls, const int* __restrict__ rowptr, const int* __restrict__ col,
    const double* __restrict__ cls, const double* __restrict__ coefE0, const int* __restrict__ perm,
    const int* __restrict__ iperm, double* __restrict__ BLall, double* __restrict__ BUall, size_t stride_sys,
    int* __restrict__ bad) {
    extern __shared__ double win[];
    __shared__ double cf[kMaxClasses];
    const int kk = blockIdx.x;
    const int w1 = bw + 1;
    double* BL = BLall + stride_sys * kk;
    double* BU = BUall + stride_sys * kk;
    if (threadIdx.x < ncls) cf[threadIdx.x] = coefE0[(size_t)kk * ncls + threadIdx.x];
    for (int e = threadIdx.x; e < w1 * w1; e += blockDim.x) win[e] = 0.0;
    // BU entries pointing past the last row stay zero
    const int nb = (n + 63) / 64;
    for (size_t e = threadIdx.x; e < stride_sys; e += blockDim.x) BU[e] = 0.0;
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
                BU[blk_idx(c, bw - t, bw)] = v;              // L(j, c): row c of L^T at offset j - c
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
    for (int r = n + threadIdx.x; r < nb * 64; r += blockDim.x)
        for (int t = 0; t <= bw; ++t) BL[blk_idx(r, t, bw)] = 0.0;
    if (failed && threadIdx.x == 0) atomicOr(bad, 1);
}

// ----------------------------------------------------------------------------- solve
// One wave per system: L L^T x = b.  Rows in blocks of 64 (lane = row within the block).
// The contribution of earlier (forward) or later (backward) blocks is a per-lane dot
// product over coalesced band rows, loaded UNR at a time with the next batch issued
// before the current one is consumed.  The same stream carries the 64 x 64 triangular
// diagonal block (the masked-out terms); it is captured, transposed, into LDS and then
// solved in chunks of 16 columns with one uniform-lane broadcast per row.  y and x live
// in an LDS ring of W >= bw + 64 entries (W a power of two); y is also parked in x.
__device__ __forceinline__ double bcast(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// sum over t in [tstart, tend] with mask(t) of -P[t*64] * ring[(o + t) & Wm]; every
// loaded entry is also offered to sink(t, value) (used to capture the diagonal block).
// v holds the first batch (entries tstart..tstart+UNR-1), issued by the caller ahead of
// time; full batches are double-buffered, the remainder is one clamped batch, so no
// entry past tend is loaded except the caller's early batch when the range is short.
template <typename FT, typename Mask, typename Sink>
__device__ __forceinline__ double band_dot(const FT* __restrict__ P, int tstart, int tend, const double* ring,
                                           int o, int Wm, Mask mask, Sink sink, FT (&v)[UNR]) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int nfull = (tend - tstart + 1) / UNR;
    for (int bt = 0; bt < nfull; ++bt) {
        const int t0 = tstart + bt * UNR;
        FT vn[UNR];
        if (bt + 1 < nfull) {
#pragma unroll
            for (int q = 0; q < UNR; ++q) vn[q] = P[(size_t)(t0 + UNR + q) * 64];
        }
        __builtin_amdgcn_sched_barrier(0);
        double y[UNR];
#pragma unroll
        for (int q = 0; q < UNR; ++q) y[q] = ring[(o + t0 + q) & Wm];
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
            const double f = fma(-(double)v[q], y[q], acc[q & 3]);
            acc[q & 3] = mask(t0 + q) ? f : acc[q & 3];
            sink(t0 + q, (double)v[q]);
        }
#pragma unroll
        for (int q = 0; q < UNR; ++q) v[q] = vn[q];
    }
    const int t0 = tstart + nfull * UNR;
    if (t0 <= tend) {
        FT vt[UNR];
        double y[UNR];
#pragma unroll
        for (int q = 0; q < UNR; ++q) vt[q] = P[(size_t)min(t0 + q, tend) * 64];
#pragma unroll
        for (int q = 0; q < UNR; ++q) y[q] = ring[(o + t0 + q) & Wm];
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
            const int t = t0 + q;
            const double f = fma(-(double)vt[q], y[q], acc[q & 3]);
            acc[q & 3] = (t <= tend && mask(t)) ? f : acc[q & 3];
            if (t <= tend) sink(t, (double)vt[q]);
        }
    }
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// Dynamic LDS: the y/x ring (W doubles) followed by the 64 x 64 diagonal block of the
// current row block, stored D[u * 64 + lane] = coefficient of row lane, column u.
template <typename FT, typename VT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void band_solve_blk_kernel(const FT* __restrict__ BLall, const FT* __restrict__ BUall, int n, int bw,
                           size_t stride_sys, const VT* __restrict__ ball, VT* __restrict__ xall,
                           size_t stride_vec, const int* __restrict__ iperm, int W) {
    extern __shared__ double smem[];
    double* win = smem;
    double* D = smem + W;
    const int sys = blockIdx.x;
    const FT* BL = BLall + stride_sys * sys;
    const FT* BU = BUall + stride_sys * sys;
    const VT* b = ball + stride_vec * sys;
    VT* x = xall + stride_vec * sys;
    const int lane = threadIdx.x;
    const int nblk = (n + 63) / 64;
    const int Wm = W - 1;
    const size_t bstride = (size_t)(bw + 1) * 64;
    FT vpre[UNR];
    auto prefetch = [&](const FT* P, int tstart) {
#pragma unroll
        for (int q = 0; q < UNR; ++q) vpre[q] = P[(size_t)(tstart + q) * 64];
    };
    // ---- forward: L y = b
    prefetch(BL + lane, 0);
    for (int B = 0; B < nblk; ++B) {
        const int row = 64 * B + lane;
        const bool ok = row < n;
        double s = ok ? (double)b[iperm ? iperm[row] : row] : 0.0;
        const size_t base = B * bstride + lane;
        const int tmax = bw - lane;          // t < tmax: columns in earlier blocks
        const int tmin = max(0, bw - row);   // columns >= 0
        s += band_dot(BL + base, 0, bw - 1, win, row - bw, Wm, [&](int t) { return t >= tmin && t < tmax; },
                      [&](int t, double v) {
                          const int u = t - tmax;             // column within the block
                          if (u >= 0 && u < lane) D[u * 64 + lane] = v;
                      }, vpre);
        const double invd = (double)BL[base + (size_t)bw * 64];
        if (B + 1 < nblk) prefetch(BL + base + bstride, 0);  // overlaps the triangular solve
        __syncthreads();
#pragma unroll 1
        for (int c = 0; c < 4; ++c) {
            double Lc[16];
#pragma unroll
            for (int uu = 0; uu < 16; ++uu) Lc[uu] = D[(16 * c + uu) * 64 + lane];
#pragma unroll
            for (int uu = 0; uu < 16; ++uu) {
                const int u = 16 * c + uu;
                const double yu = bcast(s * invd, u);
                const double f = fma(-Lc[uu], yu, s);
                s = (u < lane && u >= lane - bw) ? f : s;
            }
        }
        if (ok) {
            win[row & Wm] = s * invd;
            x[iperm ? iperm[row] : row] = (VT)(s * invd);
        }
        __syncthreads();
    }
    // ---- backward: L^T x = y
    prefetch(BU + (nblk - 1) * bstride + lane, 1);
    for (int B = nblk - 1; B >= 0; --B) {
        const int row = 64 * B + lane;
        const bool ok = row < n;
        double s = ok ? (double)x[iperm ? iperm[row] : row] : 0.0;
        const size_t base = B * bstride + lane;
        const int tmin = 64 - lane;          // t >= tmin: rows in later blocks
        s += band_dot(BU + base, 1, bw, win, row, Wm, [&](int t) { return t >= tmin && t <= bw && row + t < n; },
                      [&](int t, double v) {
                          if (t < tmin) D[(lane + t) * 64 + lane] = v;   // row lane + t of the block
                      }, vpre);
        const double invd = ok ? (double)BU[base] : 0.0;
        if (B > 0) prefetch(BU + base - bstride, 1);
        __syncthreads();
#pragma unroll 1
        for (int c = 3; c >= 0; --c) {
            double Uc[16];
#pragma unroll
            for (int uu = 0; uu < 16; ++uu) Uc[uu] = D[(16 * c + uu) * 64 + lane];
#pragma unroll
            for (int uu = 15; uu >= 0; --uu) {
                const int u = 16 * c + uu;
                const double xu = bcast(s * invd, u);
                const double f = fma(-Uc[uu], xu, s);
                s = (u > lane && u - lane <= bw && 64 * B + u < n) ? f : s;
            }
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
size_t band_pad() { return (size_t)(2 * UNR + 2) * 64; }

void e0_band_factor(const Handle* h, int bw, const int* perm, const int* iperm, double* BL, double* BU,
                    size_t stride_sys, int* bad, hipStream_t s) {
    const size_t lds = (size_t)(bw + 1) * (bw + 1) * sizeof(double);
    if (lds > 150 * 1024) fail(RTE_E_ARG, "E_0 band too wide for the LDS factorisation window");
    RTE_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&e0_band_factor_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(e0_band_factor_kernel, dim3(h->nS), dim3(256), lds, s, h->nRp, bw, h->nnz, h->ncls,
                       h->rowptr.p, h->col.p, h->cls.p, h->coefE0.p, perm, iperm, BL, BU, stride_sys, bad);
    RTE_CHECK_LAUNCH();
}

template <typename FT>
void band_solve_launch(const FT* BL, const FT* BU, int n, int bw, int nsys, size_t stride_sys, const double* b,
                       double* x, size_t stride_vec, const int* iperm, hipStream_t s) {
    const int W = pow2_at_least(bw + 128);
    const size_t lds = (size_t)(W + 64 * 64) * 8;
    if (lds > 150 * 1024) fail(RTE_E_ARG, "band too wide for the solve window");
    RTE_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&band_solve_blk_kernel<FT, double>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL((band_solve_blk_kernel<FT, double>), dim3(nsys), dim3(64), lds, s, BL, BU, n, bw, stride_sys, b,
                       x, stride_vec, iperm, W);
    RTE_CHECK_LAUNCH();
}

void band_solve_blk(const double* BL, const double* BU, int n, int bw, int nsys, size_t stride_sys,
                    const double* b, double* x, size_t stride_vec, const int* iperm, hipStream_t s) {
    band_solve_launch<double>(BL, BU, n, bw, nsys, stride_sys, b, x, stride_vec, iperm, s);
}

void band_solve_blk_f32(const float* BL, const float* BU, int n, int bw, int nsys, size_t stride_sys,
                        const double* b, double* x, size_t stride_vec, const int* iperm, hipStream_t s) {
    band_solve_launch<float>(BL, BU, n, bw, nsys, stride_sys, b, x, stride_vec, iperm, s);
}

}  // namespace k
}  // namespace rte
