// Banded Cholesky factorisation and solves.
//
// E_0 is block diagonal with one sparse SPD block per direction (paper Sec. 5.3); the
// paper applies E_0^{-1} with a sparse direct factorisation (Sec. 6.4).  Here every
// block is factored once, on the GPU, as a band matrix in a bandwidth-reducing vertex
// order, and each application of E_0^{-1} streams the factor once per sweep (forward,
// backward), which makes it HBM bound.  The coarse matrix E_c (Sec. 5.4) uses the same
// solve kernel.
//
// Blocked band layout (band_blk_index in ops.h), coalesced for one 64-lane wave per
// system: rows in blocks of 64 (lane = row within the block), and for each row of a block
// the band offsets t = 0..bw in groups of VEC = 16 bytes / element consecutive entries, so
// that one group of the whole block is a single 1 KiB load:
//   BL at (r, t) = L(r, r - bw + t)   (row r of L;   t = bw: 1 / L(r,r))
//   BU at (r, t) = L(r + t, r)        (row r of L^T; t = 0:  1 / L(r,r))
// Entries outside the matrix, and the padding of the last group, are zero.
#include <algorithm>

#include "ops.h"

namespace rte {
namespace {


__device__ __forceinline__ size_t blk_idx(int row, int t, int bw) { return k::band_blk_index(row, t, bw, 2); }

// ----------------------------------------------------------------------------- factor
// The lower band of every direction's E_0 block, in band order, is first written into the
// blocked layout of BL by a fully parallel pass (e0_band_fill_kernel: one thread per row,
// BL and BU zeroed around it).  The factorisation then streams its input rows from there
// with plain coalesced loads, ahead of use, instead of walking the sparse pattern row by row.
__global__ __launch_bounds__(256) void e0_band_fill_kernel(int n, int bw, int nnz, int ncls,
                                                           const int* __restrict__ rowptr,
                                                           const int* __restrict__ col,
                                                           const double* __restrict__ cls,
                                                           const double* __restrict__ coefE0,
                                                           const int* __restrict__ perm,
                                                           const int* __restrict__ iperm, double* __restrict__ BLall,
                                                           double* __restrict__ BUall, size_t stride_sys) {
    const int kk = blockIdx.y;
    const int r = blockIdx.x * 256 + threadIdx.x;
    const int rows = (n + 63) / 64 * 64;             // the layout's rows, padding included
    if (r >= rows) return;
    double* BL = BLall + stride_sys * kk;
    double* BU = BUall + stride_sys * kk;
    const int G2 = (int)k::band_groups(bw, 2) * 2;   // offsets per row in the layout
    for (int t = 0; t < G2; ++t) {
        BL[blk_idx(r, t, bw)] = 0.0;
        BU[blk_idx(r, t, bw)] = 0.0;
    }
    if (r >= n) return;
    const double* cf = coefE0 + (size_t)kk * ncls;
    const int v = iperm[r];
    for (int e = rowptr[v]; e < rowptr[v + 1]; ++e) {
        const int pc = perm[col[e]];
        if (pc <= r && pc >= r - bw) {
            double val = 0.0;
            for (int c = 0; c < ncls; ++c) val = fma(cf[c], cls[(size_t)c * nnz + e], val);
            BL[blk_idx(r, pc - (r - bw), bw)] = val;
        }
    }
}

// One work-group of 512 or 1024 threads (wide bands) per direction.  A (bw+1) x (bw+1) window of the active
// trailing matrix lives in LDS with circular row and column indices (mod bw+1).  Step j:
// pivot and scale column j; write row j of L (final now) to BL and BU; rank-one update of
// the window's lower triangle; store row j+bw+1 of the input (read from BL one step ahead)
// into the slot row j vacated.  Thread t owns offset t of the row leaving and of the row
// arriving: column j-bw+t and column j+1+t share one window position (mod bw+1), so the
// thread reads the old entry before it writes the new one and no other thread touches it.

// Work-group barrier for LDS traffic only: this thread's LDS operations complete
// (lgkmcnt(0)), then s_barrier.  __syncthreads would also wait for every global load and
// store in flight, which here are the prefetched input row and the output rows of L.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);       // vmcnt and expcnt at their maxima, lgkmcnt 0
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}
__global__ __launch_bounds__(1024) void e0_band_factor_kernel(int n, int bw, double* __restrict__ BLall,
                                                             double* __restrict__ BUall, size_t stride_sys,
                                                             int* __restrict__ bad) {
    extern __shared__ double win[];
    const int kk = blockIdx.x;
    const int w1 = bw + 1;
    double* BL = BLall + stride_sys * kk;
    double* BU = BUall + stride_sys * kk;
    const int t = threadIdx.x;                       // offset owned (t <= bw)
    const bool own = t <= bw;
    // rows 0 .. min(n, w1) - 1 of the input into the window: row r, offset t is column
    // r - bw + t, at position (r + 1 + t) mod w1
    for (int r = 0; r < min(n, w1); ++r)
        if (own) win[(r % w1) * w1 + (r + 1 + t) % w1] = BL[blk_idx(r, t, bw)];
    // the input row that arrives at step j is row j + w1, loaded one step ahead
    double next = (own && w1 < n) ? BL[blk_idx(w1, t, bw)] : 0.0;
    __syncthreads();
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15, nty = blockDim.x >> 4;
    int failed = 0;
    for (int j = 0; j < n; ++j) {
        const int sj = j % w1;
        const int s1 = (sj + 1 == w1) ? 0 : sj + 1;         // slot of j+1
        double djj = win[sj * w1 + sj];
        if (!(djj > 0.0)) { failed = 1; djj = 1.0; }
        const double d = sqrt(djj), id = 1.0 / d;
        const int m = min(n - 1, j + bw) - j;               // rows below the pivot in the window
        const double arriving = next;
        if (own && j + w1 + 1 < n) next = BL[blk_idx(j + w1 + 1, t, bw)];
        if (t < m) {
            int si = s1 + t; if (si >= w1) si -= w1;
            win[si * w1 + sj] *= id;
        }
        lds_barrier();
        // row j of L is final: offset t is column c = j - bw + t (t = bw: 1 / L(j,j))
        const int pos = (j + 1 + t) % w1;
        if (own) {
            const int c = j - bw + t;
            const double v = (t == bw) ? id : win[sj * w1 + pos];
            if (c >= 0) {
                BU[blk_idx(c, bw - t, bw)] = v;              // L(j, c): row c of L^T at offset j - c
                BL[blk_idx(j, t, bw)] = v;
            }
            // the arriving row j + w1 takes the slot (offset t: column j + 1 + t, same position)
            if (j + w1 < n) win[sj * w1 + pos] = arriving;
        }
        // trailing update of the lower triangle (j, j+m] x (j, j+m]: this thread's columns
        // b = tx + 16 k (their column-j entries held in registers) of rows a = ty + (blockDim.x / 16) i; a
        // row's entries are read together, then written, so the LDS reads overlap
        int scol[kFacCols];
        double lb[kFacCols];
#pragma unroll
        for (int q = 0; q < kFacCols; ++q) {
            const int b = tx + 16 * q;
            int sc = s1 + b; if (sc >= w1) sc -= w1;
            scol[q] = b < w1 ? sc : 0;
            lb[q] = b < m ? win[sc * w1 + sj] : 0.0;
        }
        for (int a = ty; a < m; a += nty) {
            int si = s1 + a; if (si >= w1) si -= w1;
            const double lij = win[si * w1 + sj];
            double* rowp = win + si * w1;
            double val[kFacCols];
#pragma unroll
            for (int q = 0; q < kFacCols; ++q)
                if (tx + 16 * q <= a) val[q] = rowp[scol[q]];
#pragma unroll
            for (int q = 0; q < kFacCols; ++q)
                if (tx + 16 * q <= a) rowp[scol[q]] = fma(-lij, lb[q], val[q]);
        }
        lds_barrier();
    }
    if (failed && threadIdx.x == 0) atomicOr(bad, 1);
}

// ----------------------------------------------------------------------------- diagonal blocks
// After the factorisation, the 64 x 64 diagonal block of every row block (rows and columns
// 64B .. 64B+63, lower triangle; in BL at (r, t = bw + c - r), in BU at (c, t = r - c)) is
// replaced by its inverse, which the solve applies as a product of independent broadcasts
// instead of a 64-step substitution.  With bw >= 63 every entry of the block's lower triangle
// lies in the band, so the inverse (dense below its diagonal) fits the same slots; the
// diagonal keeps 1 / L(r,r), the inverse's own diagonal.  One work-group of 64 threads per
// (row block, system): the block in LDS, thread j forms column j of the inverse by forward
// substitution (L x = e_j) in FP64, four partial sums per dot product.
__global__ __launch_bounds__(64) void band_diag_invert_kernel(int n, int bw, double* __restrict__ BLall,
                                                              double* __restrict__ BUall, size_t stride_sys) {
    __shared__ double Lb[64 * 64];    // Lb[i * 64 + k] = L(r0 + i, r0 + k), k < i; Lb[i * 65] = 1 / L(i, i)
    __shared__ double X[64 * 64];     // X[i * 64 + j] = inverse entry (i, j), j <= i
    const int B = blockIdx.x, lane = threadIdx.x;
    double* BL = BLall + stride_sys * blockIdx.y;
    double* BU = BUall + stride_sys * blockIdx.y;
    const int r0 = 64 * B;
    const int nb = min(64, n - r0);
    for (int j = 0; j < 64; ++j) {
        double v = 0.0;
        if (lane < nb && j <= lane) v = BL[blk_idx(r0 + lane, bw + j - lane, bw)];
        Lb[lane * 64 + j] = v;
        X[lane * 64 + j] = 0.0;
    }
    __syncthreads();
    if (lane < nb) {
        const int j = lane;
        X[j * 65] = Lb[j * 65];
        for (int i = j + 1; i < nb; ++i) {
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            int k = j;
            for (; k + 3 < i; k += 4) {
                a0 = fma(Lb[i * 64 + k], X[k * 64 + j], a0);
                a1 = fma(Lb[i * 64 + k + 1], X[(k + 1) * 64 + j], a1);
                a2 = fma(Lb[i * 64 + k + 2], X[(k + 2) * 64 + j], a2);
                a3 = fma(Lb[i * 64 + k + 3], X[(k + 3) * 64 + j], a3);
            }
            for (; k < i; ++k) a0 = fma(Lb[i * 64 + k], X[k * 64 + j], a0);
            X[i * 64 + j] = -((a0 + a1) + (a2 + a3)) * Lb[i * 65];
        }
    }
    __syncthreads();
    if (lane < nb) {
        for (int j = 0; j <= lane; ++j) BL[blk_idx(r0 + lane, bw + j - lane, bw)] = X[lane * 64 + j];
        for (int i = lane; i < nb; ++i) BU[blk_idx(r0 + lane, i - lane, bw)] = X[i * 64 + lane];
    }
}

// ----------------------------------------------------------------------------- solve
// One wave per system: L L^T x = b.  Rows in blocks of 64 (lane = row within the block).
// A row block of a factor is G = ceil((bw+1)/VEC) groups of 16 bytes per lane; each group
// is one coalesced 1 KiB load for the wave.  The wave is the only one on its SIMD, so the
// memory-level parallelism has to come from inside it: the groups land in a ring of kRing
// registers (132 VGPRs) that is refilled as soon as a slot is consumed, from the same row
// block (phase p + 1) or, after the slot's last use, from the next row block of the sweep
// (or the first block of the backward sweep).  The loads in flight therefore never drain
// at a block boundary or at the turn between the sweeps; the compiler's own waitcnt
// tracking orders every use after its load.
//
// Per block, the dot product with the already-solved neighbours uses the LDS ring of
// y (forward) or x (backward) values; the 64 x 64 triangular diagonal block comes from the
// same stream, is captured transposed into LDS, and is solved with one uniform-lane
// broadcast per row.  The right-hand side is fetched one block ahead.
__device__ __forceinline__ double bcast(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

template <typename FT> struct Vec16;
template <> struct Vec16<double> { typedef double T __attribute__((ext_vector_type(2))); static constexpr int N = 2; };
template <> struct Vec16<float> { typedef float T __attribute__((ext_vector_type(4))); static constexpr int N = 4; };

// Dynamic LDS: the y/x ring, mirrored (entry k at k and k + W, so that a window of up to W
// consecutive entries is contiguous), followed by the 64 x 64 diagonal block of the current
// row block, stored D[u * 64 + lane] = coefficient of row lane, column u, and 64 dump
// slots (one per lane) for the stores of entries outside that block.
// The dot products carry no masks: before a block is processed, the ring entries of its own
// rows are set to zero, and every other entry a band row can touch is either a solved
// neighbour or is paired with a zero factor entry (columns outside the matrix, padding), so
// it only has to be finite (the ring starts zeroed).
// A row block is P phases of H groups (the layout pads the group count to P H), all
// unrolled, so every ring slot, band offset and load source is known at compile time; the
// only loop that carries the ring is the one over row blocks.
// The solve's memory is global device memory, said explicitly in the pointer types: a
// pointer read from memory (the grouped launch's job table) is otherwise generic to the
// compiler, and generic (flat) loads are also counted as LDS operations, so waiting for one
// would drain the whole ring.
#define GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLOBAL T* as_global(T* p) {
    return (GLOBAL T*)p;
}

template <typename FT, int H, int P>
__device__ __forceinline__ void band_solve_system(const GLOBAL FT* __restrict__ BLs,
                                                  const GLOBAL FT* __restrict__ BUs, int n, int bw,
                                                  const GLOBAL double* __restrict__ b, GLOBAL double* __restrict__ x,
                                                  const int* __restrict__ iperm, int W) {
    typedef typename Vec16<FT>::T V;
    constexpr int VEC = Vec16<FT>::N;
    constexpr int G = H * P;
    constexpr size_t bs = (size_t)G * 64 * VEC;      // elements per row block
    extern __shared__ double smem[];
    // the y ring and the captured diagonal block hold the factor's type: FP64 factors keep
    // every product and sum in FP64; FP32 factors (the mixed-precision preconditioner) take
    // the band rows' dot products in FP32 (products and four partial sums, added to the FP64
    // right-hand side), which spares a conversion per entry, and solve the diagonal block
    // in FP64
    FT* win = reinterpret_cast<FT*>(smem);              // 2 W entries
    FT* D = reinterpret_cast<FT*>(smem + 2 * W);
    const int lane = threadIdx.x;
    const int nblk = (n + 63) / 64;
    const int Wm = W - 1;
    const int nstep = 2 * nblk;
    for (int e = lane; e < 2 * W; e += 64) win[e] = (FT)0;
    // step st: forward row block st (st < nblk), else backward row block 2 nblk - 1 - st
    auto block_ptr = [&](int st) -> const GLOBAL FT* {
        return st < nblk ? BLs + (size_t)st * bs : BUs + (size_t)(nstep - 1 - st) * bs;
    };
    auto step_row = [&](int st) -> int { return 64 * (st < nblk ? st : nstep - 1 - st) + lane; };
    // where the right-hand side of step st lives (clamped into the matrix; the value of a
    // row outside it is discarded)
    auto src_index = [&](int st) -> int {
        const int row = min(step_row(min(st, nstep - 1)), n - 1);
        return iperm ? iperm[row] : row;
    };
    V ring[H];
    {
        const GLOBAL V* p0 = reinterpret_cast<const GLOBAL V*>(block_ptr(0));
#pragma unroll
        for (int i = 0; i < H; ++i) ring[i] = p0[(size_t)i * 64 + lane];
    }
    int cidx = src_index(0);
    double sval = b[cidx];
    int nidx = src_index(1);
    double ylast = 0.0;
    // Drain the prologue's loads once: the loop header then sees only the steady-state
    // pending loads of the previous step, and the compiler's waits stay partial (a merge
    // with the prologue's fresher loads would make every step wait for almost all of them).
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const bool inv = k::band_diag_inverted(bw);
    for (int st = 0; st < nstep; ++st) {
        const bool fwd = st < nblk;
        const int B = fwd ? st : nstep - 1 - st;
        const int row = 64 * B + lane;
        const bool ok = row < n;
        double s = (st == nblk) ? ylast : sval;
        s = ok ? s : 0.0;
        const int myidx = cidx;
        // prefetch, ahead of this step's ring loads: the right-hand side of the next step and
        // the source index of the one after.  Backward steps read the y parked in x (the first
        // one is served from ylast instead); all addresses stay inside the matrix.
        {
            const int s1 = min(st + 1, nstep - 1);
            sval = (s1 > nblk) ? x[nidx] : b[nidx];
            cidx = nidx;
            nidx = src_index(st + 2);
        }
        const GLOBAL V* cur = reinterpret_cast<const GLOBAL V*>(block_ptr(st));
        const GLOBAL V* nxt = reinterpret_cast<const GLOBAL V*>(block_ptr(min(st + 1, nstep - 1)));
        // the ring entries of this block's own rows are not known yet: zero
        win[row & Wm] = (FT)0;
        win[(row & Wm) + W] = (FT)0;
        // band offset t of this row touches ring entry yoff + t; it is part of the
        // diagonal block for t in [clo, clo + span) and is then stored at D[dbase + 64 t].
        // The range includes the stored 1 / L(r,r) (t = bw forward, 0 backward), which lands
        // on the tile's diagonal D[65 lane].
        const int yoff = fwd ? row - bw : row;
        const int clo = fwd ? bw - lane : 0;
        const unsigned span = fwd ? (unsigned)lane + 1 : (unsigned)(64 - lane);
        const int dbase = fwd ? lane - 64 * (bw - lane) : 65 * lane;
        const int dump = 64 * 64 + lane;
        FT acc[4] = {(FT)0, (FT)0, (FT)0, (FT)0};
        constexpr int Q = 4;   // ring entries are read Q slots before their use
        const FT* yw = win + (yoff & Wm);
        FT yq[Q][VEC];
#pragma unroll
        for (int j = 0; j < Q; ++j)
#pragma unroll
            for (int e = 0; e < VEC; ++e) yq[j][e] = yw[j * VEC + e];
#pragma unroll
        for (int c = 0; c < G; ++c) {
            const int i = c % H;
            const V v = ring[i];
            FT yc[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) yc[e] = yq[c % Q][e];
            if (c + Q < G) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) yq[c % Q][e] = yw[(c + Q) * VEC + e];
            }
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const int t = c * VEC + e;
                const FT val = v[e];
                acc[t & 3] = fma(-val, yc[e], acc[t & 3]);
                // branch-free capture: lanes outside the diagonal block write their dump slot
                D[((unsigned)(t - clo) < span) ? dbase + 64 * t : dump] = val;
            }
            // the slot's old value is dead from here on (the empty asm pins this slot's
            // products here, so the compiler cannot defer them and keep the value live): reload
            // it in place
            asm volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]));
            __builtin_amdgcn_sched_barrier(0);
            ring[i] = (c + H < G) ? cur[(size_t)(c + H) * 64 + lane] : nxt[(size_t)i * 64 + lane];
        }
        s += ((double)acc[0] + (double)acc[1]) + ((double)acc[2] + (double)acc[3]);
        __syncthreads();
        double res;
        if (inv) {
            // the block's inverse (captured like the block): y = D^{-1} s over the rows of the
            // block, 64 independent broadcasts
            double y = 0.0;
            if (fwd) {
#pragma unroll 1
                for (int c = 0; c < 4; ++c) {
                    double Dc[16];
#pragma unroll
                    for (int uu = 0; uu < 16; ++uu) Dc[uu] = (double)D[(16 * c + uu) * 64 + lane];
#pragma unroll
                    for (int uu = 0; uu < 16; ++uu) {
                        const int u = 16 * c + uu;
                        const double f = fma(Dc[uu], bcast(s, u), y);
                        y = (u <= lane) ? f : y;
                    }
                }
            } else {
#pragma unroll 1
                for (int c = 0; c < 4; ++c) {
                    double Dc[16];
#pragma unroll
                    for (int uu = 0; uu < 16; ++uu) Dc[uu] = (double)D[(16 * c + uu) * 64 + lane];
#pragma unroll
                    for (int uu = 0; uu < 16; ++uu) {
                        const int u = 16 * c + uu;
                        const double f = fma(Dc[uu], bcast(s, u), y);
                        y = (u >= lane && 64 * B + u < n) ? f : y;
                    }
                }
            }
            res = ok ? y : 0.0;
        } else {
        const double dinv = ok ? (double)D[65 * lane] : 0.0;
        if (fwd) {
#pragma unroll 1
            for (int c = 0; c < 4; ++c) {
                double Lc[16];
#pragma unroll
                for (int uu = 0; uu < 16; ++uu) Lc[uu] = (double)D[(16 * c + uu) * 64 + lane];
#pragma unroll
                for (int uu = 0; uu < 16; ++uu) {
                    const int u = 16 * c + uu;
                    const double yu = bcast(s * dinv, u);
                    const double f = fma(-Lc[uu], yu, s);
                    s = (u < lane && u >= lane - bw) ? f : s;
                }
            }
        } else {
#pragma unroll 1
            for (int c = 3; c >= 0; --c) {
                double Uc[16];
#pragma unroll
                for (int uu = 0; uu < 16; ++uu) Uc[uu] = (double)D[(16 * c + uu) * 64 + lane];
#pragma unroll
                for (int uu = 15; uu >= 0; --uu) {
                    const int u = 16 * c + uu;
                    const double xu = bcast(s * dinv, u);
                    const double f = fma(-Uc[uu], xu, s);
                    s = (u > lane && u - lane <= bw && 64 * B + u < n) ? f : s;
                }
            }
        }
        res = s * dinv;
        }
        ylast = res;
        if (ok) {
            win[row & Wm] = (FT)res;
            win[(row & Wm) + W] = (FT)res;
            x[myidx] = res;
        }
        __syncthreads();
    }
}

// one system per work-group: factors and vectors at fixed strides
template <typename FT, int H, int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void band_solve_kernel(const FT* __restrict__ BLall, const FT* __restrict__ BUall, int n, int bw,
                       size_t stride_sys, const double* __restrict__ ball, double* __restrict__ xall,
                       size_t stride_vec, const int* __restrict__ iperm, int W) {
    const int sys = blockIdx.x;
    band_solve_system<FT, H, P>(as_global(BLall + stride_sys * sys), as_global(BUall + stride_sys * sys), n, bw,
                                as_global(ball + stride_vec * sys), as_global(xall + stride_vec * sys), iperm, W);
}

// the systems of several jobs (problem instances of one band shape) in one launch: the
// work-group finds its job by binary search over the jobs' first work-group indices
template <typename FT, int H, int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void band_solve_group_kernel(const k::BandJob* __restrict__ jobs, int njobs) {
    const int wg = blockIdx.x;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].first <= wg) lo = mid;
        else hi = mid - 1;
    }
    const k::BandJob& J = jobs[lo];
    const size_t sys = (size_t)(wg - J.first);
    band_solve_system<FT, H, P>(as_global(static_cast<const FT*>(J.BL) + J.stride_sys * sys),
                                as_global(static_cast<const FT*>(J.BU) + J.stride_sys * sys), J.n, J.bw,
                                as_global(J.b + J.stride_vec * sys), as_global(J.x + J.stride_vec * sys), nullptr, J.W);
}

// lower band (row-major, band[r (bw+1) + bw + c - r]) -> lower triangle of a dense
// column-major n x n matrix (the rest untouched)
__global__ void band_to_dense_kernel(const double* __restrict__ band, int n, int bw, double* __restrict__ A) {
    const size_t total = (size_t)n * (bw + 1);
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / (bw + 1));
        const int c = r - bw + (int)(e % (bw + 1));
        if (c >= 0) A[(size_t)c * n + r] = band[e];
    }
}

// A(c, r) = A(r, c) for r > c (copy the lower triangle of a column-major matrix to the upper),
// through 32 x 32 LDS tiles
__global__ __launch_bounds__(256) void symmetrize_lower_kernel(double* __restrict__ A, int n) {
    __shared__ double tile[32][33];
    const int bi = blockIdx.y, bj = blockIdx.x;     // tile row / column (lower: bi >= bj)
    if (bi < bj) return;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int k = ty; k < 32; k += 8) {
        const int r = 32 * bi + tx, c = 32 * bj + k;
        tile[k][tx] = (r < n && c < n) ? A[(size_t)c * n + r] : 0.0;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int r = 32 * bj + tx, c = 32 * bi + k;       // upper entry (r, c) = lower (c, r)
        if (r < n && c < n && c > r) A[(size_t)c * n + r] = tile[tx][k];
    }
}

// column-wise permutation of an n x ncols column-major matrix: gather (dst[r] = src[iperm[r]])
// or scatter (dst[iperm[r]] = src[r]); one work-group per column, so the scattered side of a
// column is touched by one work-group in a short time and its cache lines are reused
// one thread per element: column blockIdx.y, rows of the 256-row chunk blockIdx.x
__global__ __launch_bounds__(256) void permute_cols_kernel(const int* __restrict__ iperm, int n,
                                                           const double* __restrict__ src,
                                                           double* __restrict__ dst, int gather) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    const size_t off = (size_t)blockIdx.y * n;
    const int p = iperm[r];
    if (gather) dst[off + r] = src[off + p];
    else dst[off + p] = src[off + r];
}

// Y[i] = sum_j A[i * n + j] X[j] for a dense n x n matrix stored by rows (one wave per row,
// fixed summation order)
__global__ __launch_bounds__(256) void gemv_rows_kernel(int n, const double* __restrict__ A,
                                                        const double* __restrict__ X, double* __restrict__ Y) {
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    const double* a = A + (size_t)i * n;
    double acc0 = 0.0, acc1 = 0.0;
    int j = lane;
    for (; j + 64 < n; j += 128) {
        acc0 = fma(a[j], X[j], acc0);
        acc1 = fma(a[j + 64], X[j + 64], acc1);
    }
    if (j < n) acc0 = fma(a[j], X[j], acc0);
    double v = acc0 + acc1;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) Y[i] = v;
}

constexpr int kBandMaxLds = 150 * 1024;   // largest dynamic LDS window of a band solve

int pow2_at_least(int v) {
    int w = 64;
    while (w < v) w <<= 1;
    return w;
}

// FP64 blocked factor (VEC 2, G64 groups) -> FP32 blocked factor (VEC 4, G32 groups) of
// the same band
__global__ void band_to_f32_kernel(const double* __restrict__ src, float* __restrict__ dst, int n, int bw,
                                   int nsys, size_t stride64, size_t stride32, int G64, int G32) {
    const size_t per = k::band_blk_size_g(n, G32, 4);
    const size_t total = per * nsys;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const size_t sys = e / per, q = e % per;
        // q = ((B G32 + g) 64 + lane) 4 + k
        const int k = (int)(q & 3), lane = (int)((q >> 2) & 63);
        const size_t bg = q >> 8;
        const int B = (int)(bg / G32), g = (int)(bg % G32);
        const int t = 4 * g + k;
        const int r = 64 * B + lane;
        float v = 0.0f;
        if (t <= bw && r < n) v = (float)src[stride64 * sys + k::band_blk_index_g(r, t, G64, 2)];
        dst[stride32 * sys + q] = v;
    }
}

// the same band from a layout of Gs groups to one of Gd groups, VEC entries per group
template <typename T, int VEC>
__global__ void band_relayout_kernel(const T* __restrict__ src, int Gs, T* __restrict__ dst, int Gd, int n, int bw,
                                     int nsys, size_t stride_src, size_t stride_dst) {
    const size_t per = k::band_blk_size_g(n, Gd, VEC);
    const size_t total = per * nsys;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const size_t sys = e / per, q = e % per;
        // q = ((B Gd + g) 64 + lane) VEC + k
        const int k = (int)(q % VEC), lane = (int)((q / VEC) & 63);
        const size_t bg = q / (64 * VEC);
        const int B = (int)(bg / Gd), g = (int)(bg % Gd);
        const int t = VEC * g + k;
        const int r = 64 * B + lane;
        T v = (T)0;
        if (t <= bw && r < n) v = src[stride_src * sys + k::band_blk_index_g(r, t, Gs, VEC)];
        dst[stride_dst * sys + q] = v;
    }
}

}  // namespace

namespace k {

template <typename FT, int H, int P>
void band_launch_hp(const FT* BL, const FT* BU, int n, int bw, int nsys, size_t stride_sys, const double* b,
                    double* x, size_t stride_vec, const int* iperm, int W, size_t lds, hipStream_t s) {
    // the window limit is raised once per kernel to the largest window any band may use
    // (so that no attribute call happens while a caller captures a graph)
    static const bool attr = [] {
        RTE_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&band_solve_kernel<FT, H, P>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, kBandMaxLds));
        return true;
    }();
    (void)attr;
    hipLaunchKernelGGL((band_solve_kernel<FT, H, P>), dim3(nsys), dim3(64), lds, s, BL, BU, n, bw, stride_sys, b, x,
                       stride_vec, iperm, W);
    RTE_CHECK_LAUNCH();
}

// ring: the rows a block reads (bw before it, or after it, its own 64 and up to a group of
// padding) fit in W; W >= 256 also covers the window of ring reads ahead
int band_ring(int bw, int vec, int G) {
    return std::max(256, pow2_at_least(std::max(bw + 64 + vec * 8, G * vec)));
}
size_t band_lds(int W) { return (size_t)(2 * W + 64 * 65) * 8; }

bool band_layout_ok(int bw, int vec, int G) {
    const BandShape sh = band_shape_of_groups(G);
    return sh.H > 0 && G >= (bw + vec) / vec && band_lds(band_ring(bw, vec, G)) <= (size_t)kBandMaxLds;
}

template <typename FT>
void band_solve_launch(const FT* BL, const FT* BU, int n, int bw, int nsys, size_t stride_sys, const double* b,
                       double* x, size_t stride_vec, const int* iperm, hipStream_t s, int G) {
    if (nsys <= 0 || n <= 0) return;
    constexpr int VEC = 16 / (int)sizeof(FT);
    if (G == 0) G = (int)band_groups(bw, VEC);
    if (!band_layout_ok(bw, VEC, G)) fail(RTE_E_ARG, "band too wide for the solve kernel");
    const BandShape sh = band_shape_of_groups(G);
    const int W = band_ring(bw, VEC, G);
    const size_t lds = band_lds(W);
#define RTE_BAND_CASE(HH, PP)                                                                             \
    if (sh.H == HH && sh.P == PP) {                                                                       \
        band_launch_hp<FT, HH, PP>(BL, BU, n, bw, nsys, stride_sys, b, x, stride_vec, iperm, W, lds, s); \
        return;                                                                                           \
    }
    RTE_BAND_CASE(9, 1) RTE_BAND_CASE(17, 1) RTE_BAND_CASE(33, 1)
    RTE_BAND_CASE(9, 2) RTE_BAND_CASE(17, 2) RTE_BAND_CASE(33, 2)
    RTE_BAND_CASE(17, 3) RTE_BAND_CASE(33, 3) RTE_BAND_CASE(33, 4)
#undef RTE_BAND_CASE
    fail(RTE_E_ARG, "band too wide for the solve kernel");
}

template <typename FT, int H, int P>
void band_group_launch_hp(const BandJob* jobs, int njobs, int nwg, size_t lds, hipStream_t s) {
    static const bool attr = [] {
        RTE_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&band_solve_group_kernel<FT, H, P>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, kBandMaxLds));
        return true;
    }();
    (void)attr;
    hipLaunchKernelGGL((band_solve_group_kernel<FT, H, P>), dim3(nwg), dim3(64), lds, s, jobs, njobs);
    RTE_CHECK_LAUNCH();
}

void band_group_plan(std::vector<BandJob>& jobs, bool f32, BandGroupPlan& plan, hipStream_t s) {
    const int vec = f32 ? 4 : 2;
    for (auto& j : jobs) {
        if (j.G == 0) j.G = (int)band_groups(j.bw, vec);
        if (!band_layout_ok(j.bw, vec, j.G)) fail(RTE_E_ARG, "band too wide for the solve kernel");
        const BandShape sh = band_shape_of_groups(j.G);
        j.W = band_ring(j.bw, vec, j.G);
        j.first = sh.H * 16 + sh.P;                 // sort key for now
    }
    std::stable_sort(jobs.begin(), jobs.end(), [](const BandJob& a, const BandJob& b) { return a.first < b.first; });
    plan.launches.clear();
    for (size_t i = 0; i < jobs.size();) {
        const int key = jobs[i].first;
        BandGroupPlan::Launch L{};
        L.H = key / 16;
        L.P = key % 16;
        L.first_job = (int)i;
        int wg = 0, wmax = 0;
        size_t e = i;
        for (; e < jobs.size() && jobs[e].first == key; ++e) {
            wmax = std::max(wmax, jobs[e].W);
            const int nsys = jobs[e].nsys;
            jobs[e].first = wg;
            wg += nsys;
        }
        L.njobs = (int)(e - i);
        L.nwg = wg;
        L.lds = band_lds(wmax);
        if (wg > 0) plan.launches.push_back(L);
        i = e;
    }
    plan.f32 = f32;
    plan.jobs.alloc(std::max<size_t>(jobs.size(), 1));
    if (!jobs.empty())
        RTE_HIP(hipMemcpyAsync(plan.jobs.p, jobs.data(), jobs.size() * sizeof(BandJob), hipMemcpyHostToDevice, s));
    RTE_HIP(hipStreamSynchronize(s));
}

void band_group_run(const BandGroupPlan& plan, hipStream_t s) {
    for (const auto& L : plan.launches) {
        const BandJob* jp = plan.jobs.p + L.first_job;
#define RTE_GROUP_CASE(FT, HH, PP)                                                 \
    if (L.H == HH && L.P == PP) {                                                  \
        band_group_launch_hp<FT, HH, PP>(jp, L.njobs, L.nwg, L.lds, s);            \
        continue;                                                                  \
    }
        if (plan.f32) {
            RTE_GROUP_CASE(float, 9, 1) RTE_GROUP_CASE(float, 17, 1) RTE_GROUP_CASE(float, 33, 1)
            RTE_GROUP_CASE(float, 9, 2) RTE_GROUP_CASE(float, 17, 2) RTE_GROUP_CASE(float, 33, 2)
            RTE_GROUP_CASE(float, 17, 3) RTE_GROUP_CASE(float, 33, 3) RTE_GROUP_CASE(float, 33, 4)
        } else {
            RTE_GROUP_CASE(double, 9, 1) RTE_GROUP_CASE(double, 17, 1) RTE_GROUP_CASE(double, 33, 1)
            RTE_GROUP_CASE(double, 9, 2) RTE_GROUP_CASE(double, 17, 2) RTE_GROUP_CASE(double, 33, 2)
            RTE_GROUP_CASE(double, 17, 3) RTE_GROUP_CASE(double, 33, 3) RTE_GROUP_CASE(double, 33, 4)
        }
#undef RTE_GROUP_CASE
        fail(RTE_E_ARG, "band too wide for the solve kernel");
    }
}

// The factorisation's LDS window limit is raised once per process, to the largest window any
// band may use (150 KiB), and never per call: concurrent assemblies on other threads launch
// the same kernel with windows of their own size, and a per-call attribute write by one of
// them could lower the limit under another's launch (or land inside a graph capture).
void raise_factor_window() {
    static const bool attr = [] {
        RTE_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&e0_band_factor_kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024));
        return true;
    }();
    (void)attr;
}

void e0_band_factor(const Handle* h, int bw, const int* perm, const int* iperm, double* BL, double* BU,
                    size_t stride_sys, int* bad, hipStream_t s) {
    const size_t lds = (size_t)(bw + 1) * (bw + 1) * sizeof(double);
    if (lds > 150 * 1024 || bw + 1 > 16 * kFacCols)
        fail(RTE_E_ARG, "E_0 band too wide for the LDS factorisation window");
    const int rows = (h->nRp + 63) / 64 * 64;
    hipLaunchKernelGGL(e0_band_fill_kernel, dim3((rows + 255) / 256, h->nS), dim3(256), 0, s, h->nRp, bw, h->nnz,
                       h->ncls, h->rowptr.p, h->col.p, h->cls.p, h->coefE0.p, perm, iperm, BL, BU, stride_sys);
    RTE_CHECK_LAUNCH();
    raise_factor_window();
    hipLaunchKernelGGL(e0_band_factor_kernel, dim3(h->nS), dim3(bw >= 120 ? 1024 : 512), lds, s, h->nRp, bw, BL, BU,
                       stride_sys, bad);
    RTE_CHECK_LAUNCH();
    band_invert_diag(BL, BU, h->nRp, bw, h->nS, stride_sys, s);
}

void band_factor_one(int n, int bw, double* BL, double* BU, int* bad, hipStream_t s) {
    const size_t lds = (size_t)(bw + 1) * (bw + 1) * sizeof(double);
    if (lds > 150 * 1024 || bw + 1 > 16 * kFacCols) fail(RTE_E_ARG, "band too wide for the LDS factorisation window");
    raise_factor_window();
    hipLaunchKernelGGL(e0_band_factor_kernel, dim3(1), dim3(bw >= 120 ? 1024 : 512), lds, s, n, bw, BL, BU,
                       (size_t)0, bad);
    RTE_CHECK_LAUNCH();
    band_invert_diag(BL, BU, n, bw, 1, 0, s);
}

void band_invert_diag(double* BL, double* BU, int n, int bw, int nsys, size_t stride_sys, hipStream_t s) {
    if (!band_diag_inverted(bw) || n <= 0 || nsys <= 0) return;
    hipLaunchKernelGGL(band_diag_invert_kernel, dim3((n + 63) / 64, nsys), dim3(64), 0, s, n, bw, BL, BU, stride_sys);
    RTE_CHECK_LAUNCH();
}


void band_solve_blk(const double* BL, const double* BU, int n, int bw, int nsys, size_t stride_sys,
                    const double* b, double* x, size_t stride_vec, const int* iperm, hipStream_t s, int G) {
    band_solve_launch<double>(BL, BU, n, bw, nsys, stride_sys, b, x, stride_vec, iperm, s, G);
}

void band_solve_blk_f32(const float* BL, const float* BU, int n, int bw, int nsys, size_t stride_sys,
                        const double* b, double* x, size_t stride_vec, const int* iperm, hipStream_t s, int G) {
    band_solve_launch<float>(BL, BU, n, bw, nsys, stride_sys, b, x, stride_vec, iperm, s, G);
}

void band_to_f32(const double* src, float* dst, int n, int bw, int nsys, size_t stride64, size_t stride32,
                 hipStream_t s, int G64, int G32) {
    const size_t total = band_blk_size_g(n, G32, 4) * nsys;
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(band_to_f32_kernel, dim3(blocks), dim3(256), 0, s, src, dst, n, bw, nsys, stride64, stride32,
                       G64, G32);
    RTE_CHECK_LAUNCH();
}

void band_relayout(const double* src, int Gsrc, double* dst, int Gdst, int n, int bw, int nsys, size_t stride_src,
                   size_t stride_dst, hipStream_t s) {
    const size_t total = band_blk_size_g(n, Gdst, 2) * nsys;
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL((band_relayout_kernel<double, 2>), dim3(blocks), dim3(256), 0, s, src, Gsrc, dst, Gdst, n, bw,
                       nsys, stride_src, stride_dst);
    RTE_CHECK_LAUNCH();
}

void band_relayout(const float* src, int Gsrc, float* dst, int Gdst, int n, int bw, int nsys, size_t stride_src,
                   size_t stride_dst, hipStream_t s) {
    const size_t total = band_blk_size_g(n, Gdst, 4) * nsys;
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL((band_relayout_kernel<float, 4>), dim3(blocks), dim3(256), 0, s, src, Gsrc, dst, Gdst, n, bw,
                       nsys, stride_src, stride_dst);
    RTE_CHECK_LAUNCH();
}

void band_to_dense(const double* band, int n, int bw, double* A, hipStream_t s) {
    const size_t total = (size_t)n * (bw + 1);
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(band_to_dense_kernel, dim3(blocks), dim3(256), 0, s, band, n, bw, A);
    RTE_CHECK_LAUNCH();
}

void symmetrize_lower(double* A, int n, hipStream_t s) {
    const int nt = (n + 31) / 32;
    hipLaunchKernelGGL(symmetrize_lower_kernel, dim3(nt, nt), dim3(256), 0, s, A, n);
    RTE_CHECK_LAUNCH();
}

void permute_cols(const int* iperm, int n, int ncols, const double* src, double* dst, bool gather, hipStream_t s) {
    if (n <= 0 || ncols <= 0) return;
    hipLaunchKernelGGL(permute_cols_kernel, dim3((n + 255) / 256, ncols), dim3(256), 0, s, iperm, n, src, dst,
                       gather ? 1 : 0);
    RTE_CHECK_LAUNCH();
}

void gemv_rows(int n, const double* A, const double* X, double* Y, hipStream_t s) {
    hipLaunchKernelGGL(gemv_rows_kernel, dim3((n + 3) / 4), dim3(256), 0, s, n, A, X, Y);
    RTE_CHECK_LAUNCH();
}

}  // namespace k
}  // namespace rte
