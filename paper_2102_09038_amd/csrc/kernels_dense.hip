// Dense kernels: Henyey-Greenstein scattering matrices by double quadrature and the
// MFMA GEMMs that apply them (paper Sec. 4 matrices; Sec. 5.1 Kronecker identity
// (B (x) C) vec X = vec(C X B^T), which turns K+ and K- into GEMMs).
#include "rte_internal.h"

#include <map>
#include <mutex>
#include <type_traits>

namespace rte {
namespace {

// ============================================================================ HG quadrature
// S+_{kk'}          = 2 sum_{p in K_k} sum_{p' in K_k'} w_p w_p' [k(s.s') + k(-s.s')]
// S-_{(k,n),(k',m)} = 2 sum sum w_p w_p' s_p,n s_p',m [k(s.s') - k(-s.s')]
// with k(+-s.s') = (1-g^2)/(4 pi) [(1-g)^2 + g |s -+ s'|^2]^{-3/2}.
// One thread per pair (k, k') of a 16 x 16 tile; both triangles' points are staged
// through LDS in chunks.  Tiles below the diagonal exit; tiles above it also write the
// transposed entries.
constexpr int QT = 16;     // pairs per tile side
constexpr int QC = 32;     // points per LDS chunk

// S+ / S- from the split partial sums, added in split order
__global__ void sum_parts_kernel(const double* __restrict__ part, int nsplit, int nS, double* __restrict__ Sp,
                                 double* __restrict__ Sm) {
    const size_t n1 = (size_t)nS * nS, n = 10 * n1;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int sp = 0; sp < nsplit; ++sp) v += part[(size_t)sp * n + i];
        if (i < n1) Sp[i] = v;
        else Sm[i - n1] = v;
    }
}

__global__ __launch_bounds__(256) void hg_scatter_kernel(const double* __restrict__ pts,
                                                         const double* __restrict__ wts,
                                                         int nS, int Q, double g,
                                                         double* __restrict__ Sp,
                                                         double* __restrict__ Sm, double* __restrict__ part) {
    const int nt = (nS + QT - 1) / QT;
    // the row points are split over gridDim.y parts (few sphere pairs: more work-groups);
    // a split's sums go to its slice of part and are added up in a fixed order afterwards
    const int nchunk = (Q + QC - 1) / QC;
    const int c_lo = (int)((long long)nchunk * blockIdx.y / gridDim.y);
    const int c_hi = (int)((long long)nchunk * (blockIdx.y + 1) / gridDim.y);
    const int bi = blockIdx.x % nt, bj = blockIdx.x / nt;
    if (bi > bj) return;
    __shared__ double rowp[QT][QC][4];
    __shared__ double colp[QT][QC][4];
    const int tx = threadIdx.x % QT, ty = threadIdx.x / QT;
    const int k = bi * QT + ty, kp = bj * QT + tx;
    const double c0 = (1.0 - g) * (1.0 - g);
    const double cn = (1.0 - g * g) / (4.0 * M_PI);
    double sp = 0.0;
    double sm[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int p0 = c_lo * QC; p0 < c_hi * QC; p0 += QC) {
        const int pc = min(QC, Q - p0);
        for (int q0 = 0; q0 < Q; q0 += QC) {
            const int qc = min(QC, Q - q0);
            __syncthreads();
            for (int e = threadIdx.x; e < QT * QC; e += blockDim.x) {
                const int t = e / QC, pp = e % QC;
                const int kr = bi * QT + t, kc = bj * QT + t;
                double4 vr = {0, 0, 0, 0}, vc = {0, 0, 0, 0};
                if (kr < nS && pp < pc) {
                    const size_t o = (size_t)kr * Q + p0 + pp;
                    vr = make_double4(pts[3 * o], pts[3 * o + 1], pts[3 * o + 2], wts[o]);
                }
                if (kc < nS && pp < qc) {
                    const size_t o = (size_t)kc * Q + q0 + pp;
                    vc = make_double4(pts[3 * o], pts[3 * o + 1], pts[3 * o + 2], wts[o]);
                }
                rowp[t][pp][0] = vr.x; rowp[t][pp][1] = vr.y; rowp[t][pp][2] = vr.z; rowp[t][pp][3] = vr.w;
                colp[t][pp][0] = vc.x; colp[t][pp][1] = vc.y; colp[t][pp][2] = vc.z; colp[t][pp][3] = vc.w;
            }
            __syncthreads();
            if (k < nS && kp < nS && bi <= bj) {
                for (int a = 0; a < pc; ++a) {
                    const double sx = rowp[ty][a][0], sy = rowp[ty][a][1], sz = rowp[ty][a][2];
                    const double w = rowp[ty][a][3];
                    double accp = 0.0, accm[3] = {0, 0, 0};
                    for (int b = 0; b < qc; ++b) {
                        const double tx_ = colp[tx][b][0], ty_ = colp[tx][b][1], tz_ = colp[tx][b][2];
                        const double wb = colp[tx][b][3];
                        const double dx = sx - tx_, dy = sy - ty_, dz = sz - tz_;
                        const double ex = sx + tx_, ey = sy + ty_, ez = sz + tz_;
                        const double d2 = fma(dx, dx, fma(dy, dy, dz * dz));
                        const double e2 = fma(ex, ex, fma(ey, ey, ez * ez));
                        const double ra = rsqrt(fma(g, d2, c0));
                        const double rb = rsqrt(fma(g, e2, c0));
                        const double kpl = ra * ra * ra, kmi = rb * rb * rb;
                        accp = fma(wb, kpl + kmi, accp);
                        const double t = wb * (kpl - kmi);
                        accm[0] = fma(t, tx_, accm[0]);
                        accm[1] = fma(t, ty_, accm[1]);
                        accm[2] = fma(t, tz_, accm[2]);
                    }
                    sp = fma(w, accp, sp);
                    const double wsx = w * sx, wsy = w * sy, wsz = w * sz;
                    for (int m = 0; m < 3; ++m) {
                        sm[0][m] = fma(wsx, accm[m], sm[0][m]);
                        sm[1][m] = fma(wsy, accm[m], sm[1][m]);
                        sm[2][m] = fma(wsz, accm[m], sm[2][m]);
                    }
                }
            }
        }
    }
    if (k < nS && kp < nS) {
        const double f = 2.0 * cn;
        if (gridDim.y > 1) {
            Sp = part + (size_t)blockIdx.y * 10 * nS * nS;
            Sm = Sp + (size_t)nS * nS;
        }
        Sp[k + (size_t)nS * kp] = f * sp;
        if (bi < bj) Sp[kp + (size_t)nS * k] = f * sp;
        const size_t nSm = 3 * (size_t)nS;
        for (int n = 0; n < 3; ++n)
            for (int m = 0; m < 3; ++m) {
                Sm[(3 * k + n) + nSm * (3 * kp + m)] = f * sm[n][m];
                if (bi < bj) Sm[(3 * kp + m) + nSm * (3 * k + n)] = f * sm[n][m];
            }
    }
}

// ============================================================================ MFMA GEMM
// C = alpha A B + beta C.  A: M x K col-major (lda); B: K x N row-major (ldb); C: col-major.
// Work-group tile 128 x 128, K step 16, 4 waves in 2 x 2, each wave 64 x 64 as 4 x 4
// 16 x 16 x 4 MFMA blocks, in FP64 (v_mfma_f64_16x16x4f64) or FP32 (v_mfma_f32_16x16x4f32;
// A may then be FP64, rounded to FP32 as it is staged).  The MFMA "row" operand is the B
// fragment and the "column" operand the A fragment, so the accumulator's lane-fast index
// runs along M and the column-major stores of C are contiguous.  Register-prefetched global
// loads, double-buffered LDS, one barrier per K step.
//
// A launch may cover a range of K steps only (blockIdx.y selects the range): that is the
// split-K form used for a lightly loaded last round of tiles, whose partial products go to
// a workspace and are summed in split order by gemm_sum_parts_kernel.
typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
// rows padded by 16 elements: the four 16-lane row groups of an operand read fall in
// disjoint LDS banks
constexpr int GBM = 128, GBN = 128, GBK = 16, GPAD = 16;

__device__ __forceinline__ int xcd_swizzle(int b, int nb) {
    // consecutive work-group ids land on different XCDs (round-robin over 8); give every
    // XCD a contiguous range of tiles so that neighbouring tiles share its L2
    const int per = nb / 8, rem = nb % 8;
    const int x = b % 8, i = b / 8;
    if (i >= per) return per * 8 + x;       // leftover ids (b >= 8 * per): identity map
    return x * per + i;
}

template <typename TM> struct Mfma16;
template <> struct Mfma16<double> {
    typedef d4v acc_t;
    static __device__ __forceinline__ acc_t mma(double b, double a, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, c, 0, 0, 0);
    }
    // result element v of a lane: row (along the B operand) lane/16 + 4 v
    static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct Mfma16<float> {
    typedef f4v acc_t;
    static __device__ __forceinline__ acc_t mma(float b, float a, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(b, a, c, 0, 0, 0);
    }
    // result element v of a lane: row 4 (lane/16) + v
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// One work-group's tile over K steps [kt_begin, kt_end) into acc.  CHECK: guard every load
// (edge tiles, or K not a multiple of the step); interior tiles load unconditionally.
template <bool CHECK, typename TM, typename TA>
__device__ __forceinline__ void gemm_tile(int M, int N, int K, int m0, int n0, int kt_begin, int kt_end,
                                          const TA* __restrict__ A, int lda, const TM* __restrict__ B, int ldb,
                                          TM (&As)[2][GBK][GBM + GPAD], TM (&Bs)[2][GBK][GBN + GPAD],
                                          typename Mfma16<TM>::acc_t (&acc)[4][4]) {
    typedef Mfma16<TM> F;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    TM ra[8], rb[8];
    auto gload = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int f = tid + 256 * i;
            const int ka = f / GBM, ma = f % GBM;
            const int gm = m0 + ma, gk = k0 + ka;
            const int kb = f / GBN, nbx = f % GBN;
            const int gn = n0 + nbx, gk2 = k0 + kb;
            if (CHECK) {
                ra[i] = (gm < M && gk < K) ? (TM)A[gm + (size_t)lda * gk] : (TM)0;
                rb[i] = (gn < N && gk2 < K) ? B[(size_t)ldb * gk2 + gn] : (TM)0;
            } else {
                ra[i] = (TM)A[gm + (size_t)lda * gk];
                rb[i] = B[(size_t)ldb * gk2 + gn];
            }
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int f = tid + 256 * i;
            As[buf][f / GBM][f % GBM] = ra[i];
            Bs[buf][f / GBN][f % GBN] = rb[i];
        }
    };
    if (kt_begin < kt_end) {
        gload(kt_begin * GBK);
        sstore(0);
    }
    __syncthreads();
    for (int kt = kt_begin; kt < kt_end; ++kt) {
        const int cur = (kt - kt_begin) & 1;
        if (kt + 1 < kt_end) gload((kt + 1) * GBK);
#pragma unroll
        for (int kk = 0; kk < GBK / 4; ++kk) {
            const int kr = kk * 4 + (lane >> 4);
            TM af[4], bf[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) af[i] = As[cur][kr][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j) bf[j] = Bs[cur][kr][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[j][i] = F::mma(bf[j], af[i], acc[j][i]);
            // FP64: the next step's tile goes to the other buffer half-way through this step's
            // MFMAs (every wave finished reading that buffer before the last barrier), so the
            // stores overlap the matrix pipe instead of following it.  FP32 MFMAs are twice as
            // fast, the loads would not have landed by then: its stores follow the MFMAs.
            if (kk == (sizeof(TM) == 8 ? 2 : GBK / 4 - 1) && kt + 1 < kt_end) sstore(cur ^ 1);
        }
        __syncthreads();
    }
}

// TM: MFMA and LDS type; TA: A's storage type; TC: C's storage type.  kps: K steps per
// split (blockIdx.y); the split's result goes to C + blockIdx.y * split_stride.
template <typename TM, typename TA, typename TC>
__global__ __launch_bounds__(256, 2) void gemm_mfma_kernel(int M, int N, int K, int kps, int map, TM alpha,
                                                           const TA* __restrict__ A, int lda,
                                                           const TM* __restrict__ B, int ldb, TM beta,
                                                           TC* __restrict__ C, int ldc, size_t split_stride) {
    typedef Mfma16<TM> F;
    __shared__ TM As[2][GBK][GBM + GPAD];
    __shared__ TM Bs[2][GBK][GBN + GPAD];
    const int tm = (M + GBM - 1) / GBM, tn = (N + GBN - 1) / GBN;
    const int nb = tm * tn;
    const int b = (map & 1) ? (int)blockIdx.x : xcd_swizzle(blockIdx.x, nb);
    // tile order: along the shorter tile dimension fastest, so that the panel of the other
    // operand is shared by the few consecutive tiles that need it while it is in L2 and the
    // operand re-read across the long dimension is the small one (HBM reads it once)
    const bool mfast = (tm < tn) != ((map & 2) != 0);
    const int bm = mfast ? b % tm : b / tn, bn = mfast ? b / tm : b % tn;
    const int m0 = bm * GBM, n0 = bn * GBN;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int kt_begin = blockIdx.y * kps;
    const int kt_end = min((K + GBK - 1) / GBK, kt_begin + kps);
    C += blockIdx.y * split_stride;

    typename F::acc_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = typename F::acc_t{0, 0, 0, 0};
    if (m0 + GBM <= M && n0 + GBN <= N && K % GBK == 0)
        gemm_tile<false>(M, N, K, m0, n0, kt_begin, kt_end, A, lda, B, ldb, As, Bs, acc);
    else
        gemm_tile<true>(M, N, K, m0, n0, kt_begin, kt_end, A, lda, B, ldb, As, Bs, acc);
    // acc[j][i][v] = C(m = m0 + wm*64 + i*16 + lane%16, n = n0 + wn*64 + j*16 + F::row(lane, v))
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int gm = m0 + wm * 64 + i * 16 + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gn = n0 + wn * 64 + j * 16 + F::row(lane, v);
                if (gm < M && gn < N) {
                    TC* cp = C + gm + (size_t)ldc * gn;
                    const TM val = alpha * acc[j][i][v];
                    *cp = (TC)((beta == (TM)0) ? val : beta * (TM)*cp + val);
                }
            }
        }
}

// FP64 form for shapes made of whole tiles (M, N multiples of 128, K of 16) with 16-byte
// aligned operand rows: the tiles go from global memory straight into LDS
// (global_load_lds_dwordx4: a wave moves one 128-element K row of a tile, 16 bytes a lane),
// so no registers stage them and no LDS stores follow the MFMAs.  The next step's loads are
// issued into the other buffer at the start of a step; the barrier at its end (which waits
// for them) makes them visible.  Same tile order, fragments and summation order as above.
__global__ __launch_bounds__(256, 2) void gemm_f64_dtl_kernel(int M, int N, int K, int map, double alpha,
                                                              const double* __restrict__ A, int lda,
                                                              const double* __restrict__ B, int ldb, double beta,
                                                              double* __restrict__ C, int ldc) {
    typedef Mfma16<double> F;
    __shared__ __attribute__((aligned(16))) double As[2][GBK][GBM + GPAD];
    __shared__ __attribute__((aligned(16))) double Bs[2][GBK][GBN + GPAD];
    const int tm = M / GBM, tn = N / GBN;
    const int b = (map & 1) ? (int)blockIdx.x : xcd_swizzle(blockIdx.x, tm * tn);
    const bool mfast = (tm < tn) != ((map & 2) != 0);
    const int bm = mfast ? b % tm : b / tn, bn = mfast ? b / tm : b % tn;
    const int m0 = bm * GBM, n0 = bn * GBN;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave & 1, wn = wave >> 1;
    const int nk = K / GBK;
    // wave w moves K rows w, w + 4, w + 8, w + 12 of both tiles
    auto issue = [&](int kt, int buf) {
#pragma unroll
        for (int i = 0; i < GBK / 4; ++i) {
            const int kr = wave + 4 * i;
            const size_t gk = (size_t)kt * GBK + kr;
            __builtin_amdgcn_global_load_lds(A + m0 + lda * gk + 2 * lane, &As[buf][kr][0], 16, 0, 0);
            __builtin_amdgcn_global_load_lds(B + ldb * gk + n0 + 2 * lane, &Bs[buf][kr][0], 16, 0, 0);
        }
    };
    typename F::acc_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = typename F::acc_t{0, 0, 0, 0};
    issue(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) issue(kt + 1, cur ^ 1);
#pragma unroll
        for (int kk = 0; kk < GBK / 4; ++kk) {
            const int kr = kk * 4 + (lane >> 4);
            double af[4], bf[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) af[i] = As[cur][kr][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j) bf[j] = Bs[cur][kr][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[j][i] = F::mma(bf[j], af[i], acc[j][i]);
        }
        __builtin_amdgcn_s_waitcnt(0);       // this wave's tile loads have landed in LDS
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int gm = m0 + wm * 64 + i * 16 + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gn = n0 + wn * 64 + j * 16 + F::row(lane, v);
                double* cp = C + gm + (size_t)ldc * gn;
                const double val = alpha * acc[j][i][v];
                *cp = (beta == 0.0) ? val : fma(beta, *cp, val);
            }
        }
}

// C[m, n] = alpha sum_p P[p][m + M n] + beta C[m + ldc n], the parts added in order
template <typename TM, typename TC>
__global__ void gemm_sum_parts_kernel(int M, int N, int nsplit, const TM* __restrict__ P, TM alpha, TM beta,
                                      TC* __restrict__ C, int ldc) {
    const size_t total = (size_t)M * N;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        TM acc = P[i];
        for (int p = 1; p < nsplit; ++p) acc += P[(size_t)p * total + i];
        const size_t m = i % M, n = i / M;
        TC* cp = C + m + (size_t)ldc * n;
        const TM val = alpha * acc;
        *cp = (TC)((beta == (TM)0) ? val : beta * (TM)*cp + val);
    }
}

// ============================================================================ conversions
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__global__ void cvt_f64_bf16_kernel(const double* x, uint16_t* y, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = f32_to_bf16_rne((float)x[i]);
}
__global__ void cvt_f64_bf16_offdiag_kernel(const double* X, uint16_t* Y, size_t n, size_t nb) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n * n; i += (size_t)gridDim.x * blockDim.x) {
        const size_t c = i / n, r = i % n;
        Y[i] = (r % nb == c % nb) ? (uint16_t)0 : f32_to_bf16_rne((float)X[i]);
    }
}
__global__ void cvt_f32_bf16_kernel(const float* x, uint16_t* y, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = f32_to_bf16_rne(x[i]);
}
__global__ void cvt_f64_f32_kernel(const double* x, float* y, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = (float)x[i];
}
__global__ void cvt_f32_f64_kernel(const float* x, double* y, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = (double)x[i];
}

inline int grid_for(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 16384); }

}  // namespace

namespace k {
void hg_scatter(const double* pts, const double* wts, int nS, int Q, double g, double* Sp,
                double* Sm, hipStream_t s) {
    const int nt = (nS + QT - 1) / QT;
    const int tiles = nt * (nt + 1) / 2, nchunk = (Q + QC - 1) / QC;
    const int nsplit = std::max(1, std::min(nchunk, (2048 + tiles - 1) / tiles));
    DBuf<double> part;
    if (nsplit > 1) part.alloc((size_t)nsplit * 10 * nS * nS);
    hipLaunchKernelGGL(hg_scatter_kernel, dim3(nt * nt, nsplit), dim3(256), 0, s, pts, wts, nS, Q, g, Sp, Sm,
                       part.p);
    RTE_CHECK_LAUNCH();
    if (nsplit > 1) {
        const size_t n = (size_t)10 * nS * nS;
        hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)std::min<size_t>((n + 255) / 256, 65536)), dim3(256), 0,
                           s, part.p, nsplit, nS, Sp, Sm);
        RTE_CHECK_LAUNCH();
        RTE_HIP(hipStreamSynchronize(s));     // part is freed on return
    }
}

namespace {
// work-groups of a kernel resident on the whole current device (compute units x occupancy)
template <typename Kern>
int resident_groups(Kern kern) {
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, int> cache;
    int dev = 0;
    RTE_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    const auto key = std::make_pair(reinterpret_cast<const void*>(kern), dev);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int cus = 0, occ = 0;
    RTE_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    RTE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 256, 0));
    const int n = std::max(1, cus) * std::max(1, occ);
    cache[key] = n;
    return n;
}

template <typename TM, typename TA, typename TC>
void gemm_mfma(int M, int N, int K, TM alpha, const TA* A, int lda, const TM* B, int ldb, TM beta, TC* C,
               int ldc, TM* ws, size_t ws_elems, hipStream_t s, int kind) {
    // the tile map the autotuner chose for this shape (XCD swizzle, traversal order; both only
    // reorder whole tiles, so the result does not depend on it)
    const int map = gemm_map(kind, M, N, K);
    if (M <= 0 || N <= 0) return;
    const int tm = (M + GBM - 1) / GBM, tn = (N + GBN - 1) / GBN, nk = (K + GBK - 1) / GBK;
    const int tiles = tm * tn;
    const int slots = resident_groups(gemm_mfma_kernel<TM, TA, TC>);
    const int rounds = tiles / slots, tail = tiles % slots;
    // A last round filled to a quarter or less leaves most of the device idle: its whole row
    // blocks are split over K instead (partial products in ws, summed in split order).
    const int trb = (tail + tn - 1) / tn;
    if (ws && rounds >= 1 && tail > 0 && 4 * tail <= slots && trb < tm && nk >= 2) {
        const int units = trb * tn;
        int nsplit = std::min(nk, std::max(1, slots / units));
        const int kps = (nk + nsplit - 1) / nsplit;
        nsplit = (nk + kps - 1) / kps;
        const int Mm = (tm - trb) * GBM, Mt = M - Mm;
        const size_t part = (size_t)Mt * N;
        if (nsplit >= 2 && (size_t)nsplit * part <= ws_elems) {
            hipLaunchKernelGGL((gemm_mfma_kernel<TM, TA, TC>), dim3((tm - trb) * tn, 1), dim3(256), 0, s, Mm, N, K,
                               nk, map, alpha, A, lda, B, ldb, beta, C, ldc, (size_t)0);
            RTE_CHECK_LAUNCH();
            hipLaunchKernelGGL((gemm_mfma_kernel<TM, TA, TM>), dim3(units, nsplit), dim3(256), 0, s, Mt, N, K, kps,
                               map, (TM)1, A + Mm, lda, B, ldb, (TM)0, ws, Mt, part);
            RTE_CHECK_LAUNCH();
            const int g = (int)std::min<size_t>((part + 255) / 256, 4096);
            hipLaunchKernelGGL((gemm_sum_parts_kernel<TM, TC>), dim3(g), dim3(256), 0, s, Mt, N, nsplit,
                               (const TM*)ws, alpha, beta, C + Mm, ldc);
            RTE_CHECK_LAUNCH();
            return;
        }
    }
    if constexpr (std::is_same<TM, double>::value && std::is_same<TA, double>::value &&
                  std::is_same<TC, double>::value) {
        const bool aligned = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (reinterpret_cast<uintptr_t>(B) % 16 == 0) &&
                             lda % 2 == 0 && ldb % 2 == 0;
        if (aligned && M % GBM == 0 && N % GBN == 0 && K % GBK == 0 && K > 0) {
            hipLaunchKernelGGL(gemm_f64_dtl_kernel, dim3(tiles), dim3(256), 0, s, M, N, K, map, alpha, A, lda, B,
                               ldb, beta, C, ldc);
            RTE_CHECK_LAUNCH();
            return;
        }
    }
    hipLaunchKernelGGL((gemm_mfma_kernel<TM, TA, TC>), dim3(tiles, 1), dim3(256), 0, s, M, N, K, nk, map, alpha, A,
                       lda, B, ldb, beta, C, ldc, (size_t)0);
    RTE_CHECK_LAUNCH();
}
}  // namespace

void gemm_f64(int M, int N, int K, double alpha, const double* A, int lda, const double* B, int ldb, double beta,
              double* C, int ldc, hipStream_t s, double* ws, size_t ws_elems) {
    gemm_mfma<double, double, double>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, ws_elems, s, kGemmF64);
}

void gemm_f32(int M, int N, int K, float alpha, const double* A, int lda, const float* B, int ldb, float beta,
              double* C, int ldc, hipStream_t s, float* ws, size_t ws_elems) {
    gemm_mfma<float, double, double>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, ws_elems, s, kGemmF32);
}

void gemm_f32(int M, int N, int K, float alpha, const float* A, int lda, const float* B, int ldb, float beta,
              double* C, int ldc, hipStream_t s, float* ws, size_t ws_elems) {
    gemm_mfma<float, float, double>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, ws_elems, s, kGemmF32in);
}

void cvt_f64_bf16(const double* x, uint16_t* y, size_t n, hipStream_t s) {
    if (!n) return;
    hipLaunchKernelGGL(cvt_f64_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, y, n);
    RTE_CHECK_LAUNCH();
}
void cvt_f64_bf16_offdiag(const double* X, uint16_t* Y, size_t n, size_t nb, hipStream_t s) {
    if (!n) return;
    hipLaunchKernelGGL(cvt_f64_bf16_offdiag_kernel, dim3(grid_for(n * n)), dim3(256), 0, s, X, Y, n, nb);
    RTE_CHECK_LAUNCH();
}
void cvt_f32_bf16(const float* x, uint16_t* y, size_t n, hipStream_t s) {
    if (!n) return;
    hipLaunchKernelGGL(cvt_f32_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, y, n);
    RTE_CHECK_LAUNCH();
}
void cvt_f64_f32(const double* x, float* y, size_t n, hipStream_t s) {
    if (!n) return;
    hipLaunchKernelGGL(cvt_f64_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, y, n);
    RTE_CHECK_LAUNCH();
}
void cvt_f32_f64(const float* x, double* y, size_t n, hipStream_t s) {
    if (!n) return;
    hipLaunchKernelGGL(cvt_f32_f64_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, y, n);
    RTE_CHECK_LAUNCH();
}
}  // namespace k
}  // namespace rte
