// Derived outputs of an even-parity solution (Sec. 2): the scalar flux at the vertices and
// the terms of the particle balance.
//
// The odd part of the intensity integrates to zero over the sphere, so the scalar flux is
// the integral of the even part: phi_i = sum_k m_k U[i, k] with m_k = 2|K_k| (the even basis
// function of direction k is one on K_k and on its antipode).
//
// Testing the even equation (E - K+) u = q with the constant function 1 removes the transport
// term (A 1 = 0: constants have no gradient), which leaves the balance
//     1^T q  =  1^T (M+ - K+) U  +  1^T R U
//     source    absorption          leakage (outflow through the vacuum boundary)
// with M+ U = Mt+ U M_S+, K+ U = Ms+ U S+ and (R U)[:, k] = sum_c omega_k(nu_c) B_c U[:, k]
// (B_c the facet mass of the boundary facets of normal class c).  Each term is a weighted
// sum of the columns of U:
//     absorption = sum_k (a_t . U[:, k]) m_k - (a_s . U[:, k]) (S+ 1)_k
//     leakage    = sum_k sum_c omega_k(nu_c) (b_c . U[:, k])
// with a_t = Mt+ 1, a_s = Ms+ 1, b_c = B_c 1 (row sums of the symmetric pattern matrices).
// The device forms the column moments in one pass over U (fixed-order block reductions);
// the host adds them up in FP64 in a fixed order.
#include "ops.h"

namespace rte {
namespace {

constexpr int TPB = 256;

__device__ __forceinline__ double block_sum256(double v, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

// V[i + nRp c]: row sums of the sigma_t mass (c = 0), of the sigma_s mass (c = 1) and of
// each boundary facet-mass class (c = 2 + b)
__global__ __launch_bounds__(TPB) void balance_weights_kernel(int nRp, int nnz, const int* __restrict__ rowptr,
                                                              const double* __restrict__ cls, int nstiff, int nb,
                                                              const double* __restrict__ Msv, double* __restrict__ V) {
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i >= nRp) return;
    const int e0 = rowptr[i], e1 = rowptr[i + 1];
    for (int c = 0; c < 2 + nb; ++c) {
        const double* vals = c == 0 ? cls + (size_t)nstiff * nnz : c == 1 ? Msv : cls + (size_t)(nstiff + c - 1) * nnz;
        double acc = 0.0;
        for (int e = e0; e < e1; ++e) acc += vals[e];
        V[i + (size_t)nRp * c] = acc;
    }
}

// T[c + nv k] = sum_i V[i + nrows c] X[i + ldx k], c < nv (V == nullptr: nv = 1, V = 1);
// one block per column k
__global__ __launch_bounds__(TPB) void col_moments_kernel(int nrows, int nv, const double* __restrict__ V,
                                                          const double* __restrict__ X, size_t ldx,
                                                          double* __restrict__ T) {
    __shared__ double sh[4];
    const int k = blockIdx.x;
    const double* x = X + ldx * k;
    for (int c = 0; c < nv; ++c) {
        double acc = 0.0;
        if (V) {
            const double* v = V + (size_t)nrows * c;
            for (int i = threadIdx.x; i < nrows; i += TPB) acc = fma(v[i], x[i], acc);
        } else {
            for (int i = threadIdx.x; i < nrows; i += TPB) acc += x[i];
        }
        acc = block_sum256(acc, sh);
        if (threadIdx.x == 0) T[c + (size_t)nv * k] = acc;
    }
}

// phi[i] = sum_k m[k] U[i + nRp k]
__global__ __launch_bounds__(TPB) void scalar_flux_kernel(int nRp, int nS, const double* __restrict__ U,
                                                          const double* __restrict__ m, double* __restrict__ phi) {
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i >= nRp) return;
    double acc = 0.0;
    for (int k = 0; k < nS; ++k) acc = fma(m[k], U[i + (size_t)nRp * k], acc);
    phi[i] = acc;
}

}  // namespace

void derived_outputs(Handle* h, const double* U, double* phi, double* out, hipStream_t s) {
    const int nRp = h->nRp, nS = h->nS;
    if (phi) {
        hipLaunchKernelGGL(scalar_flux_kernel, dim3((nRp + TPB - 1) / TPB), dim3(TPB), 0, s, nRp, nS, U, h->m.p, phi);
        RTE_CHECK_LAUNCH();
    }
    if (!out) return;
    const int nb = h->nbcls, nv = 2 + nb;
    DBuf<double> V((size_t)nRp * nv), T((size_t)nv * nS), Ts(nS), Tq(nS);
    hipLaunchKernelGGL(balance_weights_kernel, dim3((nRp + TPB - 1) / TPB), dim3(TPB), 0, s, nRp, h->nnz,
                       h->rowptr.p, h->cls.p, h->ncls_stiff, nb, h->Msv.p, V.p);
    RTE_CHECK_LAUNCH();
    hipLaunchKernelGGL(col_moments_kernel, dim3(nS), dim3(TPB), 0, s, nRp, nv, V.p, U, (size_t)nRp, T.p);
    RTE_CHECK_LAUNCH();
    // S+ 1 (column sums of the symmetric S+) and the column sums of q
    hipLaunchKernelGGL(col_moments_kernel, dim3(nS), dim3(TPB), 0, s, nS, 1, nullptr, h->Sp.p, (size_t)nS, Ts.p);
    RTE_CHECK_LAUNCH();
    hipLaunchKernelGGL(col_moments_kernel, dim3(nS), dim3(TPB), 0, s, nRp, 1, nullptr, h->q.p, (size_t)nRp, Tq.p);
    RTE_CHECK_LAUNCH();
    const std::vector<double> t = T.download(s), ts = Ts.download(s), tq = Tq.download(s);
    const std::vector<double> m = h->m.download(s), coef = h->coefE.download(s);
    const int ncls = h->ncls, b0 = h->ncls_stiff + 1;
    double source = 0.0, absorption = 0.0, leakage = 0.0;
    for (int k = 0; k < nS; ++k) {
        source += tq[k];
        absorption += t[0 + (size_t)nv * k] * m[k] - t[1 + (size_t)nv * k] * ts[k];
        double lk = 0.0;
        for (int c = 0; c < nb; ++c) lk += coef[(size_t)k * ncls + b0 + c] * t[2 + c + (size_t)nv * k];
        leakage += lk;
    }
    out[0] = source;
    out[1] = absorption;
    out[2] = leakage;
    out[3] = source - absorption - leakage;
}

}  // namespace rte
