// Coarse solve of the subspace correction (Sec. 5.4, eq. corr_discrete) for coarse systems
// whose explicit inverse does not fit its memory budget and whose band is wider than the
// band solve takes (a large correction space d_N on a large mesh: N+ = 4 on 128 x 128 squares
// gives 249615 unknowns with half-bandwidth 1949).
//
// In the band (vertex-major) order the coarse matrix E_c has half-bandwidth bw, so cut into
// blocks of bs = bw rows it is block tridiagonal: block row k couples to blocks k-1, k, k+1
// only.  Its Cholesky factor is block lower bidiagonal,
//     E_c = L L^T,  L = [L_0; C_0 L_1; C_1 L_2; ...],
// computed on the device block by block with library dense kernels:
//     L_k = chol(D_k),  C_k = B_k L_k^{-T},  D_{k+1} -= C_k C_k^T,
// where D_k is the k-th diagonal block and B_k the block below it.  The diagonal factors are
// then inverted (triangular inverse) and folded into the coupling blocks,
//     F_k = L_k^{-1} C_{k-1},   G_k = C_k L_k^{-1},
// so that a solve is one block-diagonal product and one chain of matrix-vector products per
// sweep:
//     forward   w = diag(L_k^{-1}) b,     z_k = w_k - F_k z_{k-1}
//     backward  v = diag(L_k^{-T}) z,     x_k = v_k - G_k^T x_{k+1}.
// Every product of the solve is taken as a transposed one, y = A^T x, which reads A's
// columns, contiguous in the column-major blocks (one work-group per column), so the forward
// sweep keeps L_k^{-T} and F_k^T.
// Rows past n (the last block's padding) are an identity block decoupled from the rest.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <mutex>
#include <shared_mutex>
#include <string>

#include "ops.h"

namespace rte {
namespace {

constexpr int TPB = 256;

// D_k (column-major bs x bs, lower triangle) and B_k (rows of block k+1, columns of block k)
// from the row-major lower band band[r (bw+1) + bw + c - r]
__global__ __launch_bounds__(TPB) void band_to_blocks_kernel(const double* __restrict__ band, int n, int bw, int bs,
                                                             int nb, double* __restrict__ D, double* __restrict__ B) {
    const size_t w1 = (size_t)bw + 1, blk = (size_t)bs * bs;
    const size_t nD = (size_t)nb * blk, nB = (size_t)(nb - 1) * blk;
    for (size_t t = blockIdx.x * (size_t)TPB + threadIdx.x; t < nD + nB; t += (size_t)gridDim.x * TPB) {
        const bool isD = t < nD;
        const size_t u = isD ? t : t - nD;
        const int k = (int)(u / blk);
        const int i = (int)(u % blk % bs), j = (int)(u % blk / bs);
        const long r = (long)(isD ? k : k + 1) * bs + i, c = (long)k * bs + j;
        double v = 0.0;
        if (r >= c && r - c <= bw) {
            if (r < n) v = band[(size_t)r * w1 + (size_t)(bw + c - r)];
            else if (r == c) v = 1.0;
        }
        (isD ? D : B)[u] = v;
    }
}

__device__ __forceinline__ double block_sum256(double v, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// y_j = alpha sum_i A[i + lda j] x_i (+ y_j when accumulate) for the n columns of each of
// blockIdx.y blocks (block b at A + b sa, x + b sx, y + b sy).  One work-group per column:
// the threads run down the column 8 entries at a time, all 8 loads issued before the first
// is used (past the column's end a load is skipped and reads as zero), into four partial
// sums; the sums are combined in a fixed order.
__global__ __launch_bounds__(TPB) void gemv_t_kernel(int n, double alpha, const double* __restrict__ A, size_t lda,
                                                     size_t sa, const double* __restrict__ x, size_t sx,
                                                     int accumulate, double* y, size_t sy) {
    constexpr int U = 8;
    __shared__ double sh[4];
    const int j = blockIdx.x;
    const size_t b = blockIdx.y;
    const double* a = A + b * sa + (size_t)j * lda;
    const double* xb = x + b * sx;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i0 = threadIdx.x; i0 < n; i0 += U * TPB) {
        double av[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * TPB;
            av[u] = i < n ? a[i] : 0.0;
            xv[u] = i < n ? xb[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u % 4] = fma(av[u], xv[u], acc[u % 4]);
    }
    const double v = block_sum256((acc[0] + acc[1]) + (acc[2] + acc[3]), sh);
    if (threadIdx.x == 0) {
        double* yj = y + b * sy + j;
        *yj = accumulate ? fma(alpha, v, *yj) : alpha * v;
    }
}

void gemv_t(int n, double alpha, const double* A, size_t sa, const double* x, size_t sx, bool accumulate, double* y,
            size_t sy, int nbat, hipStream_t s) {
    hipLaunchKernelGGL(gemv_t_kernel, dim3(n, nbat), dim3(TPB), 0, s, n, alpha, A, (size_t)n, sa, x, sx,
                       accumulate ? 1 : 0, y, sy);
    RTE_CHECK_LAUNCH();
}

struct LibLock {
    std::lock_guard<std::mutex> serial{solver_library_mutex()};
    std::shared_lock<std::shared_mutex> capture{capture_mutex()};
};

void check_rb(rocblas_status st, const char* what) {
    if (st != rocblas_status_success) fail(RTE_E_HIP, std::string(what) + " failed");
}

}  // namespace

void coarse_block_factor(Handle& h, const double* dband, int n, int bw, hipStream_t s) {
    if (bw < 1) fail(RTE_E_ARG, "the block coarse factorisation needs a band half-width >= 1");
    const int bs = bw, nb = (n + bs - 1) / bs;
    if (nb > 65535) fail(RTE_E_ARG, "the block coarse factorisation takes at most 65535 blocks");
    const size_t blk = (size_t)bs * bs;
    h.cbs = bs;
    h.cnb = nb;
    h.CLinv.alloc((size_t)nb * blk);
    h.CLinvT.alloc((size_t)nb * blk);
    h.CB.alloc((size_t)(nb > 1 ? nb - 1 : 0) * blk);
    h.CG.alloc((size_t)(nb > 1 ? nb - 1 : 0) * blk);
    h.cwork.alloc((size_t)2 * nb * bs);
    {
        const size_t tot = (size_t)(2 * nb - 1) * blk;
        const int grid = (int)std::min<size_t>((tot + TPB - 1) / TPB, 65535u * 8);
        hipLaunchKernelGGL(band_to_blocks_kernel, dim3(grid), dim3(TPB), 0, s, dband, n, bw, bs, nb, h.CLinv.p,
                           h.CB.p);
        RTE_CHECK_LAUNCH();
    }
    LibLock lk;
    rocblas_handle rb = nullptr;
    check_rb(rocblas_create_handle(&rb), "rocblas_create_handle");
    rocblas_set_stream(rb, s);
    DBuf<int> info((size_t)2 * nb);
    try {
        const double one = 1.0, minus_one = -1.0;
        for (int k = 0; k < nb; ++k) {
            double* Dk = h.CLinv.p + (size_t)k * blk;
            check_rb(rocsolver_dpotrf(rb, rocblas_fill_lower, bs, Dk, bs, info.p + k), "rocsolver_dpotrf");
            if (k + 1 < nb) {
                double* Bk = h.CB.p + (size_t)k * blk;
                check_rb(rocblas_dtrsm(rb, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                                       rocblas_diagonal_non_unit, bs, bs, &one, Dk, bs, Bk, bs),
                         "rocblas_dtrsm");
                check_rb(rocblas_dsyrk(rb, rocblas_fill_lower, rocblas_operation_none, bs, bs, &minus_one, Bk, bs,
                                       &one, Dk + blk, bs),
                         "rocblas_dsyrk");
            }
        }
        for (int k = 0; k < nb; ++k)
            check_rb(rocsolver_dtrtri(rb, rocblas_fill_lower, rocblas_diagonal_non_unit, bs,
                                      h.CLinv.p + (size_t)k * blk, bs, info.p + nb + k),
                     "rocsolver_dtrtri");
        // L_k^{-T} into CLinvT; G_k = C_k L_k^{-1} into CG; then F_k^T = C_{k-1}^T L_k^{-T} over
        // C_{k-1} in CB (the strictly upper triangles of the L_k^{-1} blocks are zero)
        const double zero = 0.0;
        for (int k = 0; k < nb; ++k)
            check_rb(rocblas_dgeam(rb, rocblas_operation_transpose, rocblas_operation_transpose, bs, bs, &one,
                                   h.CLinv.p + (size_t)k * blk, bs, &zero, h.CLinv.p + (size_t)k * blk, bs,
                                   h.CLinvT.p + (size_t)k * blk, bs),
                     "rocblas_dgeam");
        for (int k = 0; k + 1 < nb; ++k)
            check_rb(rocblas_dgemm(rb, rocblas_operation_none, rocblas_operation_none, bs, bs, bs, &one,
                                   h.CB.p + (size_t)k * blk, bs, h.CLinv.p + (size_t)k * blk, bs, &zero,
                                   h.CG.p + (size_t)k * blk, bs),
                     "rocblas_dgemm");
        DBuf<double> tmp(nb > 1 ? blk : 0);
        for (int k = 1; k < nb; ++k) {
            check_rb(rocblas_dgemm(rb, rocblas_operation_transpose, rocblas_operation_transpose, bs, bs, bs, &one,
                                   h.CB.p + (size_t)(k - 1) * blk, bs, h.CLinv.p + (size_t)k * blk, bs, &zero,
                                   tmp.p, bs),
                     "rocblas_dgemm");
            RTE_HIP(hipMemcpyAsync(h.CB.p + (size_t)(k - 1) * blk, tmp.p, blk * sizeof(double),
                                   hipMemcpyDeviceToDevice, s));
        }
        RTE_HIP(hipStreamSynchronize(s));
        const std::vector<int> hinfo = info.download(s);
        for (int k = 0; k < nb; ++k)
            if (hinfo[k] != 0)
                fail(RTE_E_ARG, "the coarse matrix E_c is not positive definite (block " + std::to_string(k) +
                                    ", pivot " + std::to_string(hinfo[k]) + ")");
        for (int k = 0; k < nb; ++k)
            if (hinfo[nb + k] != 0) fail(RTE_E_HIP, "rocsolver_dtrtri: singular coarse Cholesky block");
    } catch (...) {
        rocblas_destroy_handle(rb);
        throw;
    }
    rocblas_destroy_handle(rb);
}

void coarse_block_solve(Handle* h, const double* rhs, double* x, hipStream_t s) {
    const int bs = h->cbs, nb = h->cnb, n = h->nc;
    const size_t blk = (size_t)bs * bs, np = (size_t)nb * bs;
    double* y = h->cwork.p;
    double* z = h->cwork.p + np;
    k::fill(y, 0.0, np, s);
    k::copy(rhs, y, (size_t)n, s);
    // forward: z = diag(L_k^{-1}) y, then z_k -= F_k z_{k-1}  (from L_k^{-T} and F_k^T)
    gemv_t(bs, 1.0, h->CLinvT.p, blk, y, bs, false, z, bs, nb, s);
    for (int k = 1; k < nb; ++k)
        gemv_t(bs, -1.0, h->CB.p + (size_t)(k - 1) * blk, 0, z + (size_t)(k - 1) * bs, 0, true, z + (size_t)k * bs,
               0, 1, s);
    // backward: y = diag(L_k^{-T}) z, then y_k -= G_k^T y_{k+1}
    gemv_t(bs, 1.0, h->CLinv.p, blk, z, bs, false, y, bs, nb, s);
    for (int k = nb - 2; k >= 0; --k)
        gemv_t(bs, -1.0, h->CG.p + (size_t)k * blk, 0, y + (size_t)(k + 1) * bs, 0, true, y + (size_t)k * bs, 0, 1,
               s);
    k::copy(y, x, (size_t)n, s);
}

}  // namespace rte
