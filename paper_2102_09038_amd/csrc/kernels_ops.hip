// Sparse and Kronecker "glue" kernels of the even-parity operators (paper Sec. 4), the
// pieces of the odd PCG of Alg. 1 with the explicit preconditioner of the lemma in
// Sec. 5.1, the coarse-space transfer of Sec. 5.4 and deterministic reductions.
//
// Layouts: even vectors U[i + nRp*k]; odd vectors V[j + nRm*(3k+m)]; every kernel maps
// consecutive threads to consecutive spatial indices so global accesses coalesce.
#include <type_traits>

#include "ops.h"

namespace rte {
namespace {

constexpr int TPB = 256;
constexpr int kAtEK = 8;   // directions per thread in the A / A^T kernels

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Sum over a 256-thread block in a fixed order; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

inline int blocks_for(size_t n) { return (int)std::min<size_t>((n + TPB - 1) / TPB, 65535u * 8); }

// ----------------------------------------------------------------------------- A and A^T
template <int D>
__global__ __launch_bounds__(TPB) void apply_A_kernel(int nRm, int nRp, int nS,
                                                      const int* __restrict__ cell,
                                                      const double* __restrict__ Dc,
                                                      const double* __restrict__ T,
                                                      const double* __restrict__ X,
                                                      double* __restrict__ B) {
    const size_t t = blockIdx.x * (size_t)TPB + threadIdx.x;
    if (t >= (size_t)nRm * nS) return;
    const int j = (int)(t % nRm), kk = (int)(t / nRm);
    double gn[D];
#pragma unroll
    for (int n = 0; n < D; ++n) gn[n] = 0.0;
#pragma unroll
    for (int v = 0; v < D + 1; ++v) {
        const double xv = X[cell[j * (D + 1) + v] + (size_t)nRp * kk];
#pragma unroll
        for (int n = 0; n < D; ++n) gn[n] = fma(Dc[(j * (D + 1) + v) * D + n], xv, gn[n]);
    }
    const double* Tk = T + 9 * kk;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        double b = 0.0;
#pragma unroll
        for (int n = 0; n < D; ++n) b = fma(gn[n], Tk[3 * n + m], b);
        B[j + (size_t)nRm * (3 * kk + m)] = 2.0 * b;
    }
}

// Y = A^T Z + (M+ + R) X [- Ms+ G] [- q] for the even vectors (n_R+ x n_S+, column-major).
// COND = false: Z holds the odd coefficients of Alg. 1 (3 per pair, Z[j + nRm (3k + m)]),
// contracted with 2 T_k; COND = true: Z holds the d condensed components per pair
// (Z[j + nRm (n nS + k)]), in FP64 or FP32 (ZT).  One thread per vertex and KC consecutive
// directions: the vertex's incidence, derivative and P1-row data are loaded once and reused
// for all KC outputs, while every access to the big arrays stays coalesced along the
// vertex index across the wave.
template <int D, bool COND, typename ZT, int KC>
__global__ __launch_bounds__(TPB) void at_e_kernel(
    int nRm, int nRp, int nS, int nnz, int ncls, int nstiff, int nb, const int* __restrict__ vc_ptr,
    const int* __restrict__ vc_cell, const double* __restrict__ vcD, const double* __restrict__ T,
    const int* __restrict__ rowptr, const int* __restrict__ col, const double* __restrict__ MtMs,
    const double* __restrict__ cls, const int* __restrict__ bnd_row, const double* __restrict__ coefE,
    const ZT* __restrict__ Z, const double* __restrict__ X, const double* __restrict__ G,
    const double* __restrict__ q, double* __restrict__ Y) {
    const int nkc = (nS + KC - 1) / KC;
    const size_t t = blockIdx.x * (size_t)TPB + threadIdx.x;
    if (t >= (size_t)nRp * nkc) return;
    const int i = (int)(t % nRp);
    const int k0 = (int)(t / nRp) * KC;
    double acc[KC];
    int kq[KC];                       // direction of slot kk, clamped into range
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        acc[kk] = 0.0;
        kq[kk] = min(k0 + kk, nS - 1);
    }
    if (Z) {
        for (int e = vc_ptr[i]; e < vc_ptr[i + 1]; ++e) {
            const int j = vc_cell[e];
            double dv[D];
#pragma unroll
            for (int n = 0; n < D; ++n) dv[n] = vcD[(size_t)e * D + n];
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                const int k = kq[kk];
                if (COND) {
#pragma unroll
                    for (int n = 0; n < D; ++n)
                        acc[kk] = fma(dv[n], (double)Z[j + (size_t)nRm * (n * (size_t)nS + k)], acc[kk]);
                } else {
                    const double z0 = (double)Z[j + (size_t)nRm * (3 * (size_t)k)];
                    const double z1 = (double)Z[j + (size_t)nRm * (3 * (size_t)k + 1)];
                    const double z2 = (double)Z[j + (size_t)nRm * (3 * (size_t)k + 2)];
                    const double* Tk = T + 9 * (size_t)k;
#pragma unroll
                    for (int n = 0; n < D; ++n)
                        acc[kk] = fma(dv[n], 2.0 * fma(Tk[3 * n], z0, fma(Tk[3 * n + 1], z1, Tk[3 * n + 2] * z2)),
                                      acc[kk]);
                }
            }
        }
    }
    double mk[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) mk[kk] = coefE[(size_t)kq[kk] * ncls + nstiff];
    const int e0 = rowptr[i], e1 = rowptr[i + 1];
    for (int e = e0; e < e1; ++e) {
        const int c = col[e];
        const double a = MtMs[2 * (size_t)e], bm = MtMs[2 * (size_t)e + 1];
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            const size_t o = c + (size_t)nRp * kq[kk];
            acc[kk] = fma(mk[kk] * a, X[o], acc[kk]);
            if (G) acc[kk] = fma(-bm, G[o], acc[kk]);
        }
    }
    if (bnd_row[i]) {
        for (int e = e0; e < e1; ++e) {
            const int c = col[e];
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                const double* cf = coefE + (size_t)kq[kk] * ncls + nstiff + 1;
                double val = 0.0;
                for (int b = 0; b < nb; ++b) val = fma(cf[b], cls[(size_t)(nstiff + 1 + b) * nnz + e], val);
                acc[kk] = fma(val, X[c + (size_t)nRp * kq[kk]], acc[kk]);
            }
        }
    }
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        if (k0 + kk >= nS) break;
        const size_t o = i + (size_t)nRp * (k0 + kk);
        Y[o] = q ? acc[kk] - q[o] : acc[kk];
    }
}

// Y = A^T Z + (M+ + R) X [- Ms+ G] [- q] with the condensed components in row-major layout,
// Z[j (d nS) + n nS + k] (cell j, component n, direction k), FP64 or FP32.  A work-group
// takes a tile of 32 vertices x 64 directions: first each wave gathers A^T Z for its vertices
// with the lanes along the directions (the vertex's incidence data is wave-uniform and each
// cell's 64 directions are one contiguous read), into an LDS tile; then the threads turn to
// run along the vertices for the mass, boundary and source terms, whose vectors are
// column-major, and write Y coalesced.
//
// Both phases load their index data first and then issue all the dependent loads of a
// batch at once (KI incidences of a vertex; the RMAX entries of a pattern row, kept in
// registers for all of the thread's directions), so that a vertex costs one or two memory
// round trips instead of one per entry.  The sums run in the same order as entry by entry.
template <int D, typename ZT>
__global__ __launch_bounds__(256) void at_e_rm_kernel(
    int nRp, int nS, int nnz, int ncls, int nstiff, int nb, const int* __restrict__ vc_ptr,
    const int* __restrict__ vc_cell, const double* __restrict__ vcD, const int* __restrict__ rowptr,
    const int* __restrict__ col, const double* __restrict__ MtMs, const double* __restrict__ cls,
    const int* __restrict__ bnd_row, const double* __restrict__ coefE, const double* __restrict__ coefD,
    const ZT* __restrict__ Z, const double* __restrict__ X, const double* __restrict__ G, const double* __restrict__ q,
    double* __restrict__ Y) {
    constexpr int TI = 32, TK = 64;
    constexpr int KI = D == 2 ? 6 : 8;       // incidences per batch (six triangles meet at an
                                             // interior vertex of the 2D meshes)
    constexpr int RMAX = D == 2 ? 7 : 16;    // pattern entries held in registers (a vertex and
                                             // its six neighbours in 2D; longer rows loop)
    __shared__ double T[TI][TK + 1];
    const int i0 = blockIdx.x * TI, k0 = blockIdx.y * TK;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const size_t dn = (size_t)D * nS;
    {
        // lanes past the last direction read direction nS - 1 (in bounds) and their sums are
        // never used; a batch's missing incidences re-read the vertex's last one and are
        // skipped in the sum, so every load is unconditional and the batch's loads are in
        // flight together
        const int k = min(k0 + lane, nS - 1);
        // two vertices per pass (il and il + 4), so that both vertices' loads are in flight
        for (int il = wave; il < TI; il += 8) {
            int e0[2], e1[2];
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const int i = i0 + il + 4 * v;
                e0[v] = i < nRp ? vc_ptr[i] : 0;
                e1[v] = i < nRp ? vc_ptr[i + 1] : 0;
            }
            double acc[2] = {0.0, 0.0};
            const int nbat = max((e1[0] - e0[0] + KI - 1) / KI, (e1[1] - e0[1] + KI - 1) / KI);
            for (int bt = 0; bt < nbat; ++bt) {
                int cj[2][KI];
                double w[2][KI][D];
                ZT z[2][KI][D];        // converted only when summed
#pragma unroll
                for (int v = 0; v < 2; ++v) {
                    // a vertex whose incidences are used up re-reads its last one (skipped in
                    // the sum); a vertex past the end reads incidence 0 of the mesh
                    const int last = e1[v] > e0[v] ? e1[v] - 1 : 0;
#pragma unroll
                    for (int t = 0; t < KI; ++t) {
                        const int e = min(e0[v] + bt * KI + t, last);
                        cj[v][t] = vc_cell[e];
#pragma unroll
                        for (int n = 0; n < D; ++n) w[v][t][n] = vcD[(size_t)e * D + n];
                    }
                }
#pragma unroll
                for (int v = 0; v < 2; ++v)
#pragma unroll
                    for (int t = 0; t < KI; ++t) {
                        const ZT* zr = Z + (size_t)cj[v][t] * dn + k;
#pragma unroll
                        for (int n = 0; n < D; ++n) z[v][t][n] = zr[(size_t)n * nS];
                    }
#pragma unroll
                for (int v = 0; v < 2; ++v)
#pragma unroll
                    for (int t = 0; t < KI; ++t) {
                        if (e0[v] + bt * KI + t < e1[v]) {
#pragma unroll
                            for (int n = 0; n < D; ++n) acc[v] = fma(w[v][t][n], (double)z[v][t][n], acc[v]);
                        }
                    }
            }
            T[il][lane] = acc[0];
            T[il + 4][lane] = acc[1];
        }
    }
    __syncthreads();
    const int il = threadIdx.x & (TI - 1);
    const int i = i0 + il;
    const bool valid = i < nRp;
    const int e0 = valid ? rowptr[i] : 0, e1 = valid ? rowptr[i + 1] : 0;
    const bool bnd = valid && bnd_row[i] != 0;
    const bool inreg = e1 - e0 <= RMAX;
    // 2D with coefD: the three stiffness-class values of the row's entries, staged in LDS once
    // per vertex (they are the same for every direction)
    constexpr int NSR = D == 2 ? 3 : 1, RSR = D == 2 ? RMAX : 1;
    __shared__ double Sv[NSR][RSR][TI];
    constexpr bool DIAG = std::is_same<ZT, float>::value;   // only the mixed-precision form has coefD
    if (DIAG && D == 2 && coefD) {
        const int c = threadIdx.x / TI;
        if (c < NSR && inreg)
            for (int t = 0; t < RSR; ++t) Sv[c][t][il] = e0 + t < e1 ? cls[(size_t)c * nnz + e0 + t] : 0.0;
        __syncthreads();
    }
    if (!valid) return;
    int rc[RMAX];
    double ra[RMAX], rb[RMAX];
#pragma unroll
    for (int t = 0; t < RMAX; ++t) {
        const bool ok = inreg && e0 + t < e1;
        rc[t] = ok ? col[e0 + t] : 0;
        ra[t] = ok ? MtMs[2 * (size_t)(e0 + t)] : 0.0;
        rb[t] = ok ? MtMs[2 * (size_t)(e0 + t) + 1] : 0.0;
    }
    for (int kl = threadIdx.x / TI; kl < TK; kl += 256 / TI) {
        const int k = k0 + kl;
        if (k >= nS) break;
        const double* cf = coefE + (size_t)k * ncls;
        const double mk = cf[nstiff];
        const double* xk = X + (size_t)nRp * k;
        double acc = T[il][kl];
        if (inreg) {
            double xv[RMAX], gv[RMAX];
#pragma unroll
            for (int t = 0; t < RMAX; ++t) {
                const bool ok = e0 + t < e1;
                xv[t] = ok ? xk[rc[t]] : 0.0;
                gv[t] = (ok && G) ? G[rc[t] + (size_t)nRp * k] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < RMAX; ++t) {
                if (e0 + t < e1) {
                    acc = fma(mk * ra[t], xv[t], acc);
                    if (G) acc = fma(-rb[t], gv[t], acc);
                }
            }
            if (DIAG && D == 2 && coefD) {
                // the diagonal d x d blocks of the condensed operator (see below), in FP64
                const double c0 = coefD[(size_t)k * NSR], c1 = coefD[(size_t)k * NSR + 1],
                             c2 = coefD[(size_t)k * NSR + 2];
#pragma unroll
                for (int t = 0; t < RSR; ++t)
                    if (e0 + t < e1) acc = fma(fma(c0, Sv[0][t][il], fma(c1, Sv[1][t][il], c2 * Sv[2][t][il])), xv[t], acc);
            }
        } else {
            for (int e = e0; e < e1; ++e) {
                const int c = col[e];
                acc = fma(mk * MtMs[2 * (size_t)e], xk[c], acc);
                if (G) acc = fma(-MtMs[2 * (size_t)e + 1], G[c + (size_t)nRp * k], acc);
            }
        }
        if (bnd) {
            for (int e = e0; e < e1; ++e) {
                double val = 0.0;
                for (int b2 = 0; b2 < nb; ++b2)
                    val = fma(cf[nstiff + 1 + b2], cls[(size_t)(nstiff + 1 + b2) * nnz + e], val);
                acc = fma(val, xk[col[e]], acc);
            }
        }
        if (DIAG && coefD && !(D == 2 && inreg)) {
            // the diagonal d x d blocks of the condensed operator, kept out of the BF16 GEMM:
            // sum_{n,m} G_kk(n,m) D_n^T Mt-^{-1} D_m x_k over the stiffness classes, in FP64
            // (2D rows held in registers take the LDS-staged form above)
            const double* cd = coefD + (size_t)k * nstiff;
            for (int e = e0; e < e1; ++e) {
                double val = 0.0;
                for (int c = 0; c < nstiff; ++c) val = fma(cd[c], cls[(size_t)c * nnz + e], val);
                acc = fma(val, xk[col[e]], acc);
            }
        }
        const size_t o = i + (size_t)nRp * k;
        Y[o] = q ? acc - q[o] : acc;
    }
}

// Yc[j + nRm (n nS + k)] = (D_n X)[j, k] / mt_j   (input of the condensed transport GEMM).
// One thread per cell and KC consecutive directions (cell data loaded once).
template <int D, int KC>
__global__ __launch_bounds__(TPB) void apply_grad_kernel(int nRm, int nRp, int nS, const int* __restrict__ cell,
                                                         const double* __restrict__ Dc,
                                                         const double* __restrict__ mt,
                                                         const double* __restrict__ X, double* __restrict__ Yc) {
    const int nkc = (nS + KC - 1) / KC;
    const size_t t = blockIdx.x * (size_t)TPB + threadIdx.x;
    if (t >= (size_t)nRm * nkc) return;
    const int j = (int)(t % nRm);
    const int k0 = (int)(t / nRm) * KC;
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
    for (int kk = 0; kk < KC; ++kk) {
        const int k = k0 + kk;
        if (k >= nS) break;
        double gn[D];
#pragma unroll
        for (int n = 0; n < D; ++n) gn[n] = 0.0;
#pragma unroll
        for (int v = 0; v < D + 1; ++v) {
            const double xv = X[cv[v] + (size_t)nRp * k];
#pragma unroll
            for (int n = 0; n < D; ++n) gn[n] = fma(dc[v][n], xv, gn[n]);
        }
#pragma unroll
        for (int n = 0; n < D; ++n) Yc[j + (size_t)nRm * (n * (size_t)nS + k)] = gn[n] * inv;
    }
}

// ----------------------------------------------------------------------------- odd PCG
__global__ __launch_bounds__(TPB) void odd_apply_kernel(int nRm, int nS, const double* __restrict__ mt,
                                                        const double* __restrict__ ms,
                                                        const double* __restrict__ T,
                                                        const double* __restrict__ P,
                                                        const double* __restrict__ G,
                                                        double* __restrict__ W, double* __restrict__ red) {
    __shared__ double sh[4];
    double part = 0.0;
    const size_t total = (size_t)nRm * nS;
    for (size_t t = blockIdx.x * (size_t)TPB + threadIdx.x; t < total; t += (size_t)gridDim.x * TPB) {
        const int j = (int)(t % nRm), kk = (int)(t / nRm);
        const double* Tk = T + 9 * kk;
        double p[3], w[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) p[m] = P[j + (size_t)nRm * (3 * kk + m)];
        const double a = mt[j], b = ms[j];
#pragma unroll
        for (int n = 0; n < 3; ++n) {
            const double mp = 2.0 * fma(Tk[3 * n], p[0], fma(Tk[3 * n + 1], p[1], Tk[3 * n + 2] * p[2]));
            const size_t o = j + (size_t)nRm * (3 * kk + n);
            w[n] = fma(a, mp, -b * G[o]);
            W[o] = w[n];
        }
        part += p[0] * w[0] + p[1] * w[1] + p[2] * w[2];
    }
    const double s = block_sum(part, sh);
    if (threadIdx.x == 0) red[blockIdx.x] = s;
}

__global__ __launch_bounds__(TPB) void reduce_kernel(const double* __restrict__ red, double* scal, int out) {
    __shared__ double sh[4];
    double v = 0.0;
    for (int i = threadIdx.x; i < k::kRedBlocks; i += TPB) v += red[i];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) scal[out] = v;
}

__global__ void sdiv_kernel(double* scal, int out, int a, int b) {
    const double den = scal[b];
    scal[out] = (den != 0.0) ? scal[a] / den : 0.0;
}

template <int DN>
__global__ __launch_bounds__(TPB) void pcg_update_kernel(int nRm, int nSm, int nch,
                                                         double* __restrict__ z, double* __restrict__ r,
                                                         const double* __restrict__ p,
                                                         const double* __restrict__ w,
                                                         const double* __restrict__ scal, int ia,
                                                         const double* __restrict__ Wm,
                                                         double* __restrict__ Cpart,
                                                         double* __restrict__ red) {
    __shared__ double sh[4];
    const double a = scal[ia];
    const int cw = (nSm + nch - 1) / nch;
    double rr = 0.0;
    const size_t total = (size_t)nRm * nch;
    for (size_t t = blockIdx.x * (size_t)TPB + threadIdx.x; t < total; t += (size_t)gridDim.x * TPB) {
        const int j = (int)(t % nRm), ch = (int)(t / nRm);
        double acc[DN];
#pragma unroll
        for (int q = 0; q < DN; ++q) acc[q] = 0.0;
        const int c1 = min(nSm, (ch + 1) * cw);
        for (int c = ch * cw; c < c1; ++c) {
            const size_t o = j + (size_t)nRm * c;
            z[o] = fma(a, p[o], z[o]);
            const double rn = fma(-a, w[o], r[o]);
            r[o] = rn;
            rr = fma(rn, rn, rr);
#pragma unroll
            for (int q = 0; q < DN; ++q) acc[q] = fma(rn, Wm[c + (size_t)nSm * q], acc[q]);
        }
#pragma unroll
        for (int q = 0; q < DN; ++q) Cpart[j + (size_t)nRm * (q + (size_t)DN * ch)] = acc[q];
    }
    const double s = block_sum(rr, sh);
    if (threadIdx.x == 0) red[blockIdx.x] = s;
}

// Cfin[j, a] = (sum_ch Cpart) * (1/(mt_j - lam_a ms_j) - 1/mt_j)
__global__ __launch_bounds__(TPB) void odd_coarse_scale_kernel(int nRm, int dN, int nch,
                                                               const double* __restrict__ mt,
                                                               const double* __restrict__ ms,
                                                               const double* __restrict__ lam,
                                                               const double* __restrict__ Cpart,
                                                               double* __restrict__ Cfin) {
    const size_t t = blockIdx.x * (size_t)TPB + threadIdx.x;
    if (t >= (size_t)nRm * dN) return;
    const int j = (int)(t % nRm), q = (int)(t / nRm);
    double s = 0.0;
    for (int ch = 0; ch < nch; ++ch) s += Cpart[j + (size_t)nRm * (q + (size_t)dN * ch)];
    const double a = mt[j];
    Cfin[t] = s * (1.0 / (a - lam[q] * ms[j]) - 1.0 / a);
}

template <int DN>
__global__ __launch_bounds__(TPB) void odd_precond_kernel(int nRm, int nS, const double* __restrict__ mt,
                                                          const double* __restrict__ MSinv,
                                                          const double* __restrict__ Wm,
                                                          const double* __restrict__ Cfin,
                                                          const double* __restrict__ r,
                                                          double* __restrict__ y,
                                                          double* __restrict__ red) {
    __shared__ double sh[4];
    const int nSm = 3 * nS;
    double part = 0.0;
    const size_t total = (size_t)nRm * nS;
    for (size_t t = blockIdx.x * (size_t)TPB + threadIdx.x; t < total; t += (size_t)gridDim.x * TPB) {
        const int j = (int)(t % nRm), kk = (int)(t / nRm);
        double rv[3], out[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) rv[m] = r[j + (size_t)nRm * (3 * kk + m)];
        const double inv = 1.0 / mt[j];
        const double* Mi = MSinv + 9 * kk;
#pragma unroll
        for (int n = 0; n < 3; ++n)
            out[n] = inv * fma(Mi[3 * n], rv[0], fma(Mi[3 * n + 1], rv[1], Mi[3 * n + 2] * rv[2]));
#pragma unroll
        for (int q = 0; q < DN; ++q) {
            const double cq = Cfin[j + (size_t)nRm * q];
#pragma unroll
            for (int n = 0; n < 3; ++n) out[n] = fma(cq, Wm[3 * kk + n + (size_t)nSm * q], out[n]);
        }
#pragma unroll
        for (int n = 0; n < 3; ++n) {
            y[j + (size_t)nRm * (3 * kk + n)] = out[n];
            part = fma(rv[n], out[n], part);
        }
    }
    const double s = block_sum(part, sh);
    if (threadIdx.x == 0) red[blockIdx.x] = s;
}

// ----------------------------------------------------------------------------- vectors
__global__ void xpby_kernel(const double* __restrict__ y, double* __restrict__ p,
                            const double* __restrict__ scal, int ib, size_t n) {
    const double b = ib >= 0 ? scal[ib] : 0.0;
    for (size_t i = blockIdx.x * (size_t)TPB + threadIdx.x; i < n; i += (size_t)gridDim.x * TPB)
        p[i] = ib >= 0 ? fma(b, p[i], y[i]) : y[i];
}
// y may be x (in-place update): no restrict on those two
__global__ void axpy_s_kernel(double* y, const double* x, const double* __restrict__ z,
                              const double* __restrict__ scal, int ia, double sign, size_t n) {
    const double a = sign * scal[ia];
    for (size_t i = blockIdx.x * (size_t)TPB + threadIdx.x; i < n; i += (size_t)gridDim.x * TPB)
        y[i] = fma(a, z[i], x[i]);
}
__global__ __launch_bounds__(TPB) void dot_kernel(const double* __restrict__ x,
                                                  const double* __restrict__ y, size_t n,
                                                  double* __restrict__ red) {
    __shared__ double sh[4];
    double v = 0.0;
    for (size_t i = blockIdx.x * (size_t)TPB + threadIdx.x; i < n; i += (size_t)gridDim.x * TPB)
        v = fma(x[i], y[i], v);
    v = block_sum(v, sh);
    if (threadIdx.x == 0) red[blockIdx.x] = v;
}
__global__ void fill_kernel(double* x, double v, size_t n) {
    for (size_t i = blockIdx.x * (size_t)TPB + threadIdx.x; i < n; i += (size_t)gridDim.x * TPB) x[i] = v;
}
__global__ void copy_kernel(const double* __restrict__ x, double* __restrict__ y, size_t n) {
    for (size_t i = blockIdx.x * (size_t)TPB + threadIdx.x; i < n; i += (size_t)gridDim.x * TPB) y[i] = x[i];
}
__global__ void axpby_kernel(double a, const double* __restrict__ x, double b, double* __restrict__ y, size_t n) {
    for (size_t i = blockIdx.x * (size_t)TPB + threadIdx.x; i < n; i += (size_t)gridDim.x * TPB)
        y[i] = fma(a, x[i], b * y[i]);
}
__global__ void row_scale_inv_mt_kernel(int nRm, int ncols, const double* __restrict__ mt,
                                        const double* __restrict__ C, double* __restrict__ Z) {
    const size_t n = (size_t)nRm * ncols;
    for (size_t t = blockIdx.x * (size_t)TPB + threadIdx.x; t < n; t += (size_t)gridDim.x * TPB)
        Z[t] = C[t] / mt[t % nRm];
}
__global__ void scale_eigbasis_kernel(int nRm, int nSm, const double* __restrict__ mt,
                                      const double* __restrict__ ms, const double* __restrict__ lam,
                                      double* __restrict__ C) {
    const size_t n = (size_t)nRm * nSm;
    for (size_t t = blockIdx.x * (size_t)TPB + threadIdx.x; t < n; t += (size_t)gridDim.x * TPB) {
        const int j = (int)(t % nRm), a = (int)(t / nRm);
        C[t] = C[t] / (mt[j] - lam[a] * ms[j]);
    }
}

// ----------------------------------------------------------------------------- coarse
// rhs[a + DN perm[i]] = sum_k T[i, k] W+[k, a].  A work-group takes 32 vertices; its 8
// groups of 32 threads sum interleaved eighths of the directions (k = g, g + 8, ...), and the
// eight partial sums are added in group order, so each vertex's long sum is split over 8
// threads instead of walked by one.
template <int DN>
__global__ __launch_bounds__(TPB) void coarse_project_kernel(int nRp, int nS, const double* __restrict__ T,
                                                             const double* __restrict__ Wp,
                                                             const int* __restrict__ perm,
                                                             double* __restrict__ rhs) {
    constexpr int VB = 32, NG = TPB / VB;
    __shared__ double part[NG][DN][VB];
    const int v = threadIdx.x % VB, grp = threadIdx.x / VB;
    const int i = blockIdx.x * VB + v;
    double acc[DN];
#pragma unroll
    for (int a = 0; a < DN; ++a) acc[a] = 0.0;
    if (i < nRp) {
        for (int kk = grp; kk < nS; kk += NG) {
            const double t = T[i + (size_t)nRp * kk];
#pragma unroll
            for (int a = 0; a < DN; ++a) acc[a] = fma(t, Wp[kk + (size_t)nS * a], acc[a]);
        }
    }
#pragma unroll
    for (int a = 0; a < DN; ++a) part[grp][a][v] = acc[a];
    __syncthreads();
    if (grp == 0 && i < nRp) {
        const int pi = perm[i];
#pragma unroll
        for (int a = 0; a < DN; ++a) {
            double sum = part[0][a][v];
            for (int g2 = 1; g2 < NG; ++g2) sum += part[g2][a][v];
            rhs[a + (size_t)DN * pi] = sum;
        }
    }
}

template <int DN>
__global__ __launch_bounds__(TPB) void richardson_update_kernel(int nRp, int nS, double* __restrict__ U,
                                                                const double* __restrict__ S,
                                                                const double* __restrict__ uc,
                                                                const double* __restrict__ Wp,
                                                                const int* __restrict__ perm) {
    const size_t t = blockIdx.x * (size_t)TPB + threadIdx.x;
    if (t >= (size_t)nRp * nS) return;
    const int i = (int)(t % nRp), kk = (int)(t / nRp);
    const int pi = perm[i];
    double v = U[t] - S[t];
#pragma unroll
    for (int a = 0; a < DN; ++a) v = fma(uc[a + (size_t)DN * pi], Wp[kk + (size_t)nS * a], v);
    U[t] = v;
}

// compile-time dispatch over the eigen-basis sizes d_N = (N+1)(N+2)/2, N = 0..8
template <template <int> class F, typename... Args>
void dispatch_dn(int dn, Args&&... args) {
    switch (dn) {
        case 1: F<1>::run(args...); break;
        case 3: F<3>::run(args...); break;
        case 6: F<6>::run(args...); break;
        case 10: F<10>::run(args...); break;
        case 15: F<15>::run(args...); break;
        case 21: F<21>::run(args...); break;
        case 28: F<28>::run(args...); break;
        case 36: F<36>::run(args...); break;
        case 45: F<45>::run(args...); break;
        default: fail(RTE_E_ARG, "eigen-basis size " + std::to_string(dn) + " not supported");
    }
}

template <int DN> struct PcgUpdateL {
    static void run(const Handle* h, double* z, double* r, const double* p, const double* w,
                    const double* scal, int ia, double* Cpart, double* red, int nch, hipStream_t s) {
        hipLaunchKernelGGL(pcg_update_kernel<DN>, dim3(k::kRedBlocks), dim3(TPB), 0, s, h->nRm, h->nSm, nch,
                           z, r, p, w, scal, ia, h->Wm.p, Cpart, red);
    }
};
template <int DN> struct OddPrecondL {
    static void run(const Handle* h, const double* r, const double* Cfin, double* y, double* red, hipStream_t s) {
        hipLaunchKernelGGL(odd_precond_kernel<DN>, dim3(k::kRedBlocks), dim3(TPB), 0, s, h->nRm, h->nS,
                           h->mt.p, h->MSinv.p, h->Wm.p, Cfin, r, y, red);
    }
};
template <int DN> struct CoarseProjectL {
    static void run(const Handle* h, const double* T, double* rhs, hipStream_t s) {
        hipLaunchKernelGGL(coarse_project_kernel<DN>, dim3((h->nRp + 31) / 32), dim3(TPB), 0, s,
                           h->nRp, h->nS, T, h->Wp.p, h->perm.p, rhs);
    }
};
template <int DN> struct RichUpdateL {
    static void run(const Handle* h, double* U, const double* S, const double* uc, hipStream_t s) {
        const size_t n = (size_t)h->nRp * h->nS;
        hipLaunchKernelGGL(richardson_update_kernel<DN>, dim3((n + TPB - 1) / TPB), dim3(TPB), 0, s,
                           h->nRp, h->nS, U, S, uc, h->Wp.p, h->perm.p);
    }
};

inline int pcg_chunks(const Handle* h) { return std::min(8, h->nSm); }

}  // namespace

namespace k {

void apply_A(const Handle* h, const double* X, double* B, hipStream_t s) {
    const size_t n = (size_t)h->nRm * h->nS;
    const dim3 g((unsigned)((n + TPB - 1) / TPB));
    if (h->d == 2)
        hipLaunchKernelGGL(apply_A_kernel<2>, g, dim3(TPB), 0, s, h->nRm, h->nRp, h->nS, h->cell.p, h->Dc.p, h->T.p, X, B);
    else
        hipLaunchKernelGGL(apply_A_kernel<3>, g, dim3(TPB), 0, s, h->nRm, h->nRp, h->nS, h->cell.p, h->Dc.p, h->T.p, X, B);
    RTE_CHECK_LAUNCH();
}

void apply_At_E(const Handle* h, const double* Z, const double* X, const double* G, const double* q,
                double* Y, hipStream_t s, bool condensed) {
    const size_t n = (size_t)h->nRp * ((h->nS + kAtEK - 1) / kAtEK);
    const dim3 g((unsigned)((n + TPB - 1) / TPB));
    decltype(&at_e_kernel<2, false, double, kAtEK>) f;
    if (h->d == 2) f = condensed ? at_e_kernel<2, true, double, kAtEK> : at_e_kernel<2, false, double, kAtEK>;
    else f = condensed ? at_e_kernel<3, true, double, kAtEK> : at_e_kernel<3, false, double, kAtEK>;
    hipLaunchKernelGGL(f, g, dim3(TPB), 0, s, h->nRm, h->nRp, h->nS, h->nnz, h->ncls, h->ncls_stiff, h->nbcls,
                       h->vc_ptr.p, h->vc_cell.p, h->vcD.p, h->T.p, h->rowptr.p, h->col.p, h->MtMs.p, h->cls.p,
                       h->bnd_row.p, h->coefE.p, Z, X, G, q, Y);
    RTE_CHECK_LAUNCH();
}

template <typename ZT>
void at_e_rm_launch(const Handle* h, const ZT* Z, const double* X, const double* G, const double* q, double* Y,
                    const double* coefD, hipStream_t s) {
    const dim3 g((unsigned)((h->nRp + 31) / 32), (unsigned)((h->nS + 63) / 64));
    auto* f = h->d == 2 ? at_e_rm_kernel<2, ZT> : at_e_rm_kernel<3, ZT>;
    hipLaunchKernelGGL(f, g, dim3(256), 0, s, h->nRp, h->nS, h->nnz, h->ncls, h->ncls_stiff, h->nbcls, h->vc_ptr.p,
                       h->vc_cell.p, h->vcD.p, h->rowptr.p, h->col.p, h->MtMs.p, h->cls.p, h->bnd_row.p, h->coefE.p,
                       coefD, Z, X, G, q, Y);
    RTE_CHECK_LAUNCH();
}

void apply_At_E_rm(const Handle* h, const double* Z, const double* X, const double* G, const double* q, double* Y,
                   hipStream_t s) {
    at_e_rm_launch<double>(h, Z, X, G, q, Y, nullptr, s);
}

void apply_At_E_rm_f32(const Handle* h, const float* Z, const double* X, const double* G, const double* q, double* Y,
                       hipStream_t s) {
    at_e_rm_launch<float>(h, Z, X, G, q, Y, h->coefD.p, s);
}

void apply_grad(const Handle* h, const double* X, double* Yc, hipStream_t s) {
    constexpr int KC = 16;   // directions per thread
    const size_t n = (size_t)h->nRm * ((h->nS + KC - 1) / KC);
    const dim3 g((unsigned)((n + TPB - 1) / TPB));
    auto* f = h->d == 2 ? apply_grad_kernel<2, KC> : apply_grad_kernel<3, KC>;
    hipLaunchKernelGGL(f, g, dim3(TPB), 0, s, h->nRm, h->nRp, h->nS, h->cell.p, h->Dc.p, h->mt.p, X, Yc);
    RTE_CHECK_LAUNCH();
}

void odd_apply(const Handle* h, const double* P, const double* G, double* W, double* red, hipStream_t s) {
    hipLaunchKernelGGL(odd_apply_kernel, dim3(kRedBlocks), dim3(TPB), 0, s, h->nRm, h->nS, h->mt.p,
                       h->ms.p, h->T.p, P, G, W, red);
    RTE_CHECK_LAUNCH();
}

void reduce(const double* red, double* scal, int out, hipStream_t s) {
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(TPB), 0, s, red, scal, out);
    RTE_CHECK_LAUNCH();
}

void sdiv(double* scal, int out, int a, int b, hipStream_t s) {
    hipLaunchKernelGGL(sdiv_kernel, dim3(1), dim3(1), 0, s, scal, out, a, b);
    RTE_CHECK_LAUNCH();
}

void pcg_update(const Handle* h, double* z, double* r, const double* p, const double* w,
                const double* scal, int ia, double* Cpart, double* red, hipStream_t s) {
    dispatch_dn<PcgUpdateL>(h->dNm, h, z, r, p, w, scal, ia, Cpart, red, pcg_chunks(h), s);
    RTE_CHECK_LAUNCH();
}

void odd_precond(const Handle* h, const double* r, const double* Cpart, double* Cfin, double* y,
                 double* red, hipStream_t s) {
    const size_t n = (size_t)h->nRm * h->dNm;
    hipLaunchKernelGGL(odd_coarse_scale_kernel, dim3((unsigned)((n + TPB - 1) / TPB)), dim3(TPB), 0, s,
                       h->nRm, h->dNm, pcg_chunks(h), h->mt.p, h->ms.p, h->lamm.p, Cpart, Cfin);
    RTE_CHECK_LAUNCH();
    dispatch_dn<OddPrecondL>(h->dNm, h, r, (const double*)Cfin, y, red, s);
    RTE_CHECK_LAUNCH();
}

void xpby(const double* y, double* p, const double* scal, int ib, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(xpby_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, y, p, scal, ib, n);
    RTE_CHECK_LAUNCH();
}
void axpy_s(double* y, const double* x, const double* z, const double* scal, int ia, double sign,
            size_t n, hipStream_t s) {
    hipLaunchKernelGGL(axpy_s_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, y, x, z, scal, ia, sign, n);
    RTE_CHECK_LAUNCH();
}
void dot(const double* x, const double* y, size_t n, double* red, hipStream_t s) {
    hipLaunchKernelGGL(dot_kernel, dim3(kRedBlocks), dim3(TPB), 0, s, x, y, n, red);
    RTE_CHECK_LAUNCH();
}
void fill(double* x, double v, size_t n, hipStream_t s) {
    if (!n) return;
    hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, x, v, n);
    RTE_CHECK_LAUNCH();
}
void copy(const double* x, double* y, size_t n, hipStream_t s) {
    if (!n) return;
    hipLaunchKernelGGL(copy_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, x, y, n);
    RTE_CHECK_LAUNCH();
}
void axpby(double a, const double* x, double b, double* y, size_t n, hipStream_t s) {
    if (!n) return;
    hipLaunchKernelGGL(axpby_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, a, x, b, y, n);
    RTE_CHECK_LAUNCH();
}
void row_scale_inv_mt(const Handle* h, const double* C, double* Z, int ncols, hipStream_t s) {
    const size_t n = (size_t)h->nRm * ncols;
    hipLaunchKernelGGL(row_scale_inv_mt_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, h->nRm, ncols, h->mt.p, C, Z);
    RTE_CHECK_LAUNCH();
}
void scale_eigbasis(const Handle* h, double* C, hipStream_t s) {
    const size_t n = (size_t)h->nRm * h->nSm;
    hipLaunchKernelGGL(scale_eigbasis_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, h->nRm, h->nSm,
                       h->mt.p, h->ms.p, h->lam_full.p, C);
    RTE_CHECK_LAUNCH();
}

void coarse_project(const Handle* h, const double* T, double* rhs, hipStream_t s) {
    dispatch_dn<CoarseProjectL>(h->dNp, h, T, rhs, s);
    RTE_CHECK_LAUNCH();
}

void richardson_update(const Handle* h, double* U, const double* S, const double* uc, hipStream_t s) {
    dispatch_dn<RichUpdateL>(h->dNp, h, U, S, uc, s);
    RTE_CHECK_LAUNCH();
}

}  // namespace k
}  // namespace rte

namespace rte {
namespace {
__global__ __launch_bounds__(256) void spmm_pattern_kernel(int nRp, int nS, const int* __restrict__ rowptr,
                                                           const int* __restrict__ col,
                                                           const double* __restrict__ vals,
                                                           const double* __restrict__ X, double* __restrict__ Y) {
    const size_t t = blockIdx.x * (size_t)256 + threadIdx.x;
    if (t >= (size_t)nRp * nS) return;
    const int i = (int)(t % nRp), kk = (int)(t / nRp);
    const double* xk = X + (size_t)nRp * kk;
    double acc = 0.0;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) acc = fma(vals[e], xk[col[e]], acc);
    Y[t] = acc;
}
__global__ void row_scale_kernel(const double* __restrict__ v, int nrow, size_t n, const double* __restrict__ X,
                                 double* __restrict__ Y) {
    for (size_t t = blockIdx.x * (size_t)256 + threadIdx.x; t < n; t += (size_t)gridDim.x * 256)
        Y[t] = v[t % nrow] * X[t];
}
}  // namespace
namespace k {
void spmm_pattern(const Handle* h, const double* vals, const double* X, double* Y, hipStream_t s) {
    const size_t n = (size_t)h->nRp * h->nS;
    hipLaunchKernelGGL(spmm_pattern_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, h->nRp, h->nS,
                       h->rowptr.p, h->col.p, vals, X, Y);
    RTE_CHECK_LAUNCH();
}
void row_scale(const double* v, int nrow, int ncol, const double* X, double* Y, hipStream_t s) {
    const size_t n = (size_t)nrow * ncol;
    if (!n) return;
    hipLaunchKernelGGL(row_scale_kernel, dim3((unsigned)std::min<size_t>((n + 255) / 256, 65535)), dim3(256), 0, s,
                       v, nrow, n, X, Y);
    RTE_CHECK_LAUNCH();
}
}  // namespace k
}  // namespace rte
