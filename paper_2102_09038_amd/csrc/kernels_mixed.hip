// Mixed-precision kernels: the BF16-input / FP32-accumulate MFMA GEMM that applies the
// condensed transport operator inside the preconditioner, the BF16 producer of its input,
// and the A^T + M+ + R kernel reading its FP32 output.  The outer residual, every dot
// product and the coarse solve stay FP64 (the Richardson iteration then acts as
// iterative refinement of the reduced-precision preconditioner; Sec. 5's convergence
// argument only needs P_1 to stay symmetric positive definite).
#include "ops.h"

namespace rte {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);    // round to nearest even
    return (uint16_t)(u >> 16);
}

// ============================================================================ BF16 GEMM
// C (f32, col-major, ldc) = alpha A B + beta C with A (bf16, M x K, row-major: k contiguous,
// lda) and B (bf16, K x N, column-major: k contiguous, ldb).  K, lda, ldb multiples of 8.
// Tile 128 x 128 x 64, 4 waves in 2 x 2, each wave 64 x 64 as 4 x 4 blocks of
// v_mfma_f32_16x16x32_bf16 (operand lanes: row l%16, k = 8 (l/16) + e; result rows
// 4 (l/16) + v, column l%16).  The MFMA row operand is the B fragment (n) and the column
// operand the A fragment (m), so the result's lane-fast index runs along m and the
// column-major stores of C are contiguous.  16-byte global loads, double-buffered LDS, one
// barrier per K step.  LDS rows are not padded: the 16-byte chunk c of tile row r sits at
// chunk c ^ ((r / 2) % 8) of the row, so that the 16 lanes of a 16-byte access, which read
// one chunk of 16 consecutive rows or write two whole rows, cover all 64 banks once.
//
// A K step is short (32 MFMAs per wave), shorter than a global load's latency, so interior
// tiles run the loads two steps ahead of the MFMAs (two register sets) in a loop without
// branches: the loads past the last step re-read the last step (in bounds, unused) and the
// store after the last step fills a buffer nobody reads, so the compiler's waits for a
// register set never cover the younger set's loads.  Edge tiles, and K not a multiple of
// two steps, take a guarded loop with one step of prefetch.
constexpr int HBM_ = 128, HBN = 128, HBK = 64;

__device__ __forceinline__ int xcd_swz(int b, int nb) {
    const int per = nb / 8, x = b % 8, i = b / 8;
    if (i >= per) return per * 8 + x;
    return x * per + i;
}

typedef uint16_t BTile[HBM_][HBK];

// element offset of 16-byte chunk c of tile row r within that row (the bank swizzle)
__device__ __forceinline__ int swz(int r, int c) { return (c ^ ((r >> 1) & 7)) * 8; }

// the MFMAs of one K step from LDS buffers As / Bs
__device__ __forceinline__ void bf16_step_mfma(const BTile& As, const BTile& Bs, int lane, int wm, int wn,
                                               f4v (&acc)[4][4]) {
#pragma unroll
    for (int kk = 0; kk < HBK / 32; ++kk) {
        const int c = kk * 4 + (lane >> 4);           // 16-byte chunk: k = 8 c .. 8 c + 7
        bf8v af[4], bfr[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = wm * 64 + i * 16 + (lane & 15);
            af[i] = *reinterpret_cast<const bf8v*>(&As[r][swz(r, c)]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = wn * 64 + j * 16 + (lane & 15);
            bfr[j] = *reinterpret_cast<const bf8v*>(&Bs[r][swz(r, c)]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                acc[j][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j], af[i], acc[j][i], 0, 0, 0);
    }
}

// Large-tile form for whole tiles (M, N multiples of 256, K of 64, 16-byte aligned operand
// rows): tile 256 x 256 x 64, eight waves in 2 x 4 (two per SIMD), each 128 x 64 as 4 x 8
// blocks of v_mfma_f32_16x16x32_bf16.  The tiles go from global memory straight into LDS
// (global_load_lds_dwordx4: one wave moves 1 KiB, eight tile rows of 64 k, lane l into slot
// l % 8 of row l / 8); the bank swizzle above is kept by letting lane l fetch the global chunk
// that belongs in its slot, (l % 8) ^ ((row / 2) % 8).  The next step's loads go into the
// other buffer at the start of a step; the wait and barrier at its end make them visible.
// Same fragments and K order as the 128 x 128 kernel, so the same bits, with half the operand
// bytes per MFMA (the 128 x 128 tiles re-read their panels from L2 and the Infinity Cache).
constexpr int LBM = 256, LBN = 256;
typedef uint16_t LTile[LBM][HBK];

__global__ __launch_bounds__(512, 1) void gemm_bf16_l_kernel(int M, int N, int K, float alpha,
                                                             const uint16_t* __restrict__ A, int lda,
                                                             const uint16_t* __restrict__ B, int ldb, float beta,
                                                             float* __restrict__ C, int ldc, int map) {
    __shared__ __attribute__((aligned(16))) LTile As[2];
    __shared__ __attribute__((aligned(16))) LTile Bs[2];
    const int tm = M / LBM, tn = N / LBN;
    const int b = (map & 1) ? (int)blockIdx.x : xcd_swz(blockIdx.x, tm * tn);
    const bool mfast = (tm < tn) != ((map & 2) != 0);
    const int bm = mfast ? b % tm : b / tn, bn = mfast ? b / tm : b % tn;
    const int m0 = bm * LBM, n0 = bn * LBN;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave & 1, wn = wave >> 1;
    const int nk = K / HBK;
    // wave w moves tile rows 8 q .. 8 q + 7 of both tiles, q = w + 8 i, i = 0..3; lane l takes
    // row 8 q + l / 8, whose swizzle ((row / 2) % 8 = (4 w + l / 16) % 8) is the same for every
    // i, so one base address per lane and operand serves all four loads
    const int lr = lane >> 3;
    const int c = (lane & 7) ^ ((4 * wave + (lr >> 1)) & 7);
    const uint16_t* Al = A + (size_t)(m0 + 8 * wave + lr) * lda + 8 * c;
    const uint16_t* Bl = B + (size_t)(n0 + 8 * wave + lr) * ldb + 8 * c;
    const size_t sa = (size_t)64 * lda, sb = (size_t)64 * ldb;
    auto issue = [&](int kt, int buf) {
        const size_t k0 = (size_t)kt * HBK;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int q = wave + 8 * i;
            __builtin_amdgcn_global_load_lds(Al + i * sa + k0, &As[buf][8 * q][0], 16, 0, 0);
            __builtin_amdgcn_global_load_lds(Bl + i * sb + k0, &Bs[buf][8 * q][0], 16, 0, 0);
        }
    };
    f4v acc[4][8];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[j][i] = f4v{0, 0, 0, 0};
    issue(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) issue(kt + 1, cur ^ 1);
#pragma unroll
        for (int kk = 0; kk < HBK / 32; ++kk) {
            const int ch = kk * 4 + (lane >> 4);
            bf8v af[8], bfr[4];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int r = wm * 128 + i * 16 + (lane & 15);
                af[i] = *reinterpret_cast<const bf8v*>(&As[cur][r][swz(r, ch)]);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = wn * 64 + j * 16 + (lane & 15);
                bfr[j] = *reinterpret_cast<const bf8v*>(&Bs[cur][r][swz(r, ch)]);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    acc[j][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j], af[i], acc[j][i], 0, 0, 0);
        }
        __builtin_amdgcn_s_waitcnt(0);       // this wave's tile loads have landed in LDS
        __syncthreads();
    }
    // acc[j][i][v] = C(m = m0 + wm*128 + i*16 + lane%16, n = n0 + wn*64 + j*16 + 4*(lane/16) + v)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int gm = m0 + wm * 128 + i * 16 + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gn = n0 + wn * 64 + j * 16 + 4 * (lane >> 4) + v;
                float* cp = C + gm + (size_t)ldc * gn;
                const float val = alpha * acc[j][i][v];
                *cp = (beta == 0.0f) ? val : fmaf(beta, *cp, val);
            }
        }
}

__global__ __launch_bounds__(256, 2) void gemm_bf16_kernel(int M, int N, int K, float alpha,
                                                           const uint16_t* __restrict__ A, int lda,
                                                           const uint16_t* __restrict__ B, int ldb, float beta,
                                                           float* __restrict__ C, int ldc, int map) {
    __shared__ __attribute__((aligned(16))) BTile As[2];
    __shared__ __attribute__((aligned(16))) BTile Bs[2];
    const int tm = (M + HBM_ - 1) / HBM_, tn = (N + HBN - 1) / HBN;
    const int b = (map & 1) ? (int)blockIdx.x : xcd_swz(blockIdx.x, tm * tn);
    // the shorter tile dimension fastest by default: consecutive tiles share the other
    // operand's panel (in L2), and the operand re-read across the long dimension is the small
    // one; the tuned map may flip it (map & 2) or drop the XCD swizzle (map & 1)
    const bool mfast = (tm < tn) != ((map & 2) != 0);
    const int bm = mfast ? b % tm : b / tn, bn = mfast ? b / tm : b % tn;
    const int m0 = bm * HBM_, n0 = bn * HBN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int nk = (K + HBK - 1) / HBK;
    // thread tid moves 16-byte chunk ch of rows r = tid / 8 + 32 i of both tiles
    const int r0 = tid >> 3, ch = tid & 7;

    f4v acc[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[j][i] = f4v{0, 0, 0, 0};

    if (m0 + HBM_ <= M && n0 + HBN <= N && K % (2 * HBK) == 0) {
        const uint16_t* Ab = A + (size_t)(m0 + r0) * lda + ch * 8;
        const uint16_t* Bb = B + (size_t)(n0 + r0) * ldb + ch * 8;
        // one K step's share of this thread: 4 chunks of A and 4 of B (kept as named values:
        // arrays passed to the helpers would be placed in scratch memory)
        struct Stage { uint4 a0, a1, a2, a3, b0, b1, b2, b3; };
        auto load = [&](int kt) {
            const size_t ko = (size_t)kt * HBK;
            const size_t la = (size_t)32 * lda, lb = (size_t)32 * ldb;
            Stage t;
            t.a0 = *reinterpret_cast<const uint4*>(Ab + ko);
            t.a1 = *reinterpret_cast<const uint4*>(Ab + la + ko);
            t.a2 = *reinterpret_cast<const uint4*>(Ab + 2 * la + ko);
            t.a3 = *reinterpret_cast<const uint4*>(Ab + 3 * la + ko);
            t.b0 = *reinterpret_cast<const uint4*>(Bb + ko);
            t.b1 = *reinterpret_cast<const uint4*>(Bb + lb + ko);
            t.b2 = *reinterpret_cast<const uint4*>(Bb + 2 * lb + ko);
            t.b3 = *reinterpret_cast<const uint4*>(Bb + 3 * lb + ko);
            return t;
        };
        // rows r0 + 32 i share (r / 2) % 8, hence the chunk position
        const int cs = swz(r0, ch);
        auto store = [&](const Stage& t, BTile& as, BTile& bs) {
            *reinterpret_cast<uint4*>(&as[r0][cs]) = t.a0;
            *reinterpret_cast<uint4*>(&as[r0 + 32][cs]) = t.a1;
            *reinterpret_cast<uint4*>(&as[r0 + 64][cs]) = t.a2;
            *reinterpret_cast<uint4*>(&as[r0 + 96][cs]) = t.a3;
            *reinterpret_cast<uint4*>(&bs[r0][cs]) = t.b0;
            *reinterpret_cast<uint4*>(&bs[r0 + 32][cs]) = t.b1;
            *reinterpret_cast<uint4*>(&bs[r0 + 64][cs]) = t.b2;
            *reinterpret_cast<uint4*>(&bs[r0 + 96][cs]) = t.b3;
        };
        Stage s0 = load(0);
        store(s0, As[0], Bs[0]);
        Stage s1 = load(1);
        __syncthreads();
        for (int kt = 0; kt < nk; kt += 2) {
            // step kt from buffer 0; step kt + 1's data (s1) goes to buffer 1
            s0 = load(min(kt + 2, nk - 1));
            __builtin_amdgcn_sched_barrier(0);     // the loads stay ahead of the MFMAs
            bf16_step_mfma(As[0], Bs[0], lane, wm, wn, acc);
            store(s1, As[1], Bs[1]);
            __syncthreads();
            // step kt + 1 from buffer 1; step kt + 2's data (s0) goes to buffer 0
            s1 = load(min(kt + 3, nk - 1));
            __builtin_amdgcn_sched_barrier(0);
            bf16_step_mfma(As[1], Bs[1], lane, wm, wn, acc);
            store(s0, As[0], Bs[0]);
            __syncthreads();
        }
    } else {
        uint4 ra[4], rb[4];
        auto gload = [&](int k0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = r0 + 32 * i;
                const int gk = k0 + ch * 8;
                const int gm = m0 + r, gn = n0 + r;
                ra[i] = (gm < M && gk < K) ? *reinterpret_cast<const uint4*>(A + (size_t)gm * lda + gk)
                                           : make_uint4(0, 0, 0, 0);
                rb[i] = (gn < N && gk < K) ? *reinterpret_cast<const uint4*>(B + (size_t)gn * ldb + gk)
                                           : make_uint4(0, 0, 0, 0);
            }
        };
        const int cs = swz(r0, ch);
        auto sstore = [&](int buf) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                *reinterpret_cast<uint4*>(&As[buf][r0 + 32 * i][cs]) = ra[i];
                *reinterpret_cast<uint4*>(&Bs[buf][r0 + 32 * i][cs]) = rb[i];
            }
        };
        gload(0);
        sstore(0);
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            const int cur = kt & 1;
            if (kt + 1 < nk) gload((kt + 1) * HBK);
            bf16_step_mfma(As[cur], Bs[cur], lane, wm, wn, acc);
            if (kt + 1 < nk) sstore(cur ^ 1);
            __syncthreads();
        }
    }
    // acc[j][i][v] = C(m = m0 + wm*64 + i*16 + lane%16, n = n0 + wn*64 + j*16 + 4*(lane/16) + v)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int gm = m0 + wm * 64 + i * 16 + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gn = n0 + wn * 64 + j * 16 + 4 * (lane >> 4) + v;
                if (gm < M && gn < N) {
                    float* cp = C + gm + (size_t)ldc * gn;
                    const float val = alpha * acc[j][i][v];
                    *cp = (beta == 0.0f) ? val : fmaf(beta, *cp, val);
                }
            }
        }
}

// ============================================================================ glue
// Ycb[j * dn + n nS + k] = bf16((D_n X)[j, k] / mt_j): the condensed GEMM's B operand, row-major
// (angular index contiguous).
template <int D>
__global__ __launch_bounds__(256) void apply_grad_bf16_kernel(int nRm, int nRp, int nS, const int* __restrict__ cell,
                                                              const double* __restrict__ Dc,
                                                              const double* __restrict__ mt,
                                                              const double* __restrict__ X,
                                                              uint16_t* __restrict__ Ycb) {
    // Rounding the data Y to BF16 only adds a small error to each product.  The operator's
    // d x d diagonal blocks (the odd moments 2 T_k of the sphere triangles plus their own
    // scattering part) are nearly singular for small triangles (s_x and s_y almost
    // proportional over the triangle), and rounding them to 8 bits can make the transport
    // term indefinite; they are therefore left out of the BF16 operator and applied exactly
    // in FP64 by the A^T kernel.
    //
    // A work-group takes 32 cells x 64 directions.  First each thread computes 8 directions
    // of one cell (consecutive threads on consecutive cells, so the reads of X run along its
    // columns) into an LDS tile; then the threads turn to write the tile's rows, 128
    // contiguous bytes per cell and component, instead of one 16-byte piece per cell.
    constexpr int TC = 32, TKD = 64;
    __shared__ __attribute__((aligned(16))) uint16_t T[TC][D][TKD + 8];
    const int j0 = blockIdx.x * TC, k0 = blockIdx.y * TKD;
    {
        const int c = threadIdx.x % TC, kg = threadIdx.x / TC;       // 8 groups of 8 directions
        const int j = j0 + c, kb = k0 + 8 * kg;
        if (j < nRm && kb < nS) {
            int cv[D + 1];
            double dc[D + 1][D];
#pragma unroll
            for (int v = 0; v < D + 1; ++v) {
                cv[v] = cell[j * (D + 1) + v];
#pragma unroll
                for (int n = 0; n < D; ++n) dc[v][n] = Dc[(j * (D + 1) + v) * D + n];
            }
            const double inv = 1.0 / mt[j];
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                double gn[D];
#pragma unroll
                for (int n = 0; n < D; ++n) gn[n] = 0.0;
#pragma unroll
                for (int v = 0; v < D + 1; ++v) {
                    const double xv = X[cv[v] + (size_t)nRp * (kb + kk)];
#pragma unroll
                    for (int n = 0; n < D; ++n) gn[n] = fma(dc[v][n], xv, gn[n]);
                }
#pragma unroll
                for (int n = 0; n < D; ++n) T[c][n][8 * kg + kk] = f32_to_bf16((float)(gn[n] * inv));
            }
        }
    }
    __syncthreads();
    // rows out: (cell, component) pairs, 8 chunks of 16 bytes each
    const size_t dn = (size_t)D * nS;
    for (int e = threadIdx.x; e < TC * D * 8; e += 256) {
        const int ch = e % 8, row = e / 8;
        const int c = row / D, n = row % D;
        const int j = j0 + c, k = k0 + 8 * ch;
        if (j >= nRm || k >= nS) continue;
        const uint4 w = *reinterpret_cast<const uint4*>(&T[c][n][8 * ch]);
        *reinterpret_cast<uint4*>(Ycb + (size_t)j * dn + (size_t)n * nS + k) = w;
    }
}

}  // namespace

namespace k {

void gemm_bf16(int M, int N, int K, float alpha, const uint16_t* A, int lda, const uint16_t* B, int ldb,
               float beta, float* C, int ldc, hipStream_t s) {
    if (M <= 0 || N <= 0) return;
    if (K % 8 || lda % 8 || ldb % 8) fail(RTE_E_ARG, "BF16 GEMM needs K, lda, ldb multiples of 8");
    const bool aligned = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (reinterpret_cast<uintptr_t>(B) % 16 == 0);
    if (M % LBM == 0 && N % LBN == 0 && K % HBK == 0 && aligned) {
        hipLaunchKernelGGL(gemm_bf16_l_kernel, dim3((M / LBM) * (N / LBN)), dim3(512), 0, s, M, N, K, alpha, A, lda, B,
                           ldb, beta, C, ldc, gemm_map(kGemmBF16, M, N, K));
        RTE_CHECK_LAUNCH();
        return;
    }
    const int nb = ((M + HBM_ - 1) / HBM_) * ((N + HBN - 1) / HBN);
    hipLaunchKernelGGL(gemm_bf16_kernel, dim3(nb), dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                       gemm_map(kGemmBF16, M, N, K));
    RTE_CHECK_LAUNCH();
}

void apply_grad_bf16(const Handle* h, const double* X, uint16_t* Ycb, hipStream_t s) {
    if (h->nS % 8) fail(RTE_E_ARG, "the BF16 transport path needs a multiple of 8 sphere pairs");
    const dim3 g((unsigned)((h->nRm + 31) / 32), (unsigned)((h->nS + 63) / 64));
    auto* f = h->d == 2 ? apply_grad_bf16_kernel<2> : apply_grad_bf16_kernel<3>;
    hipLaunchKernelGGL(f, g, dim3(256), 0, s, h->nRm, h->nRp, h->nS, h->cell.p, h->Dc.p, h->mt.p, X, Ycb);
    RTE_CHECK_LAUNCH();
}


}  // namespace k
}  // namespace rte
