// rte_apply_scatter_noalloc: Y = K+- X (the Kronecker form of the scattering operator,
// Sec. 4 with the identity of Sec. 5.1) without any device allocation, for callers that
// cannot allocate (code under HIP graph capture, serving loops that forbid it).
//
// rte_apply_scatter keeps its intermediates (the GEMM product X S+-, an FP64 staging copy
// for an FP32 result, the split last round of GEMM tiles) in the handle's workspace, which
// it allocates on first use.  This variant keeps the first two in one fixed array per device,
// `scratch`, of kScratchBytes.  The array's device address is looked up once per device,
// with that device current (by rte_assemble, or by this entry point on a device it has not
// seen), and only that address is used on the host; the array's own name is a host-side
// stand-in and is never passed to a kernel or a copy.
//
// Every call on a device shares its array: calls that overlap on one GPU race.  Nothing in
// the array is read before the same call has written it (the GEMM writes every entry of its
// product, beta = 0), so no clearing is needed between calls.  The GEMM runs unsplit: a split
// last round only pays off on shapes whose product alone exceeds the array.
#include <mutex>

#include "ops.h"
#include "rte_internal.h"

namespace rte {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;              // 64 MiB per device
constexpr size_t kScratchElems = kScratchBytes / sizeof(double);
__device__ __align__(256) double scratch[kScratchElems];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

// the array's address on the current device (looked up once per device)
double* scratch_on_current_device() {
    int dev = 0;
    RTE_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(RTE_E_ARG, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        RTE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(RTE_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch[dev] = static_cast<double*>(p);
    }
    return g_scratch[dev];
}

}  // namespace

void noalloc_setup() { (void)scratch_on_current_device(); }

void apply_scatter_noalloc(Handle* h, int parity, int dtin, const void* X, int dtout, void* Y, hipStream_t s) {
    if ((dtin != RTE_DT_F64 && dtin != RTE_DT_F32) || (dtout != RTE_DT_F64 && dtout != RTE_DT_F32))
        fail(RTE_E_ARG, "scatter operands are FP64 or FP32");
    const bool f32 = dtin == RTE_DT_F32;
    if (f32 && !(parity == 1 ? h->Sp_f.p : h->Sm_f.p))
        fail(RTE_E_ARG, "FP32 scatter operands need a handle assembled with mixed != 0");
    const int n = parity == 1 ? h->nRp : h->nRm, m = parity == 1 ? h->nS : h->nSm;
    const size_t nm = (size_t)n * m;
    // FP64 intermediates: the product X S+ before the mass matrix (parity +1), and the
    // result before its rounding to FP32 (dtype_out FP32)
    const size_t need = (parity == 1 ? nm : 0) + (dtout == RTE_DT_F32 ? nm : 0);
    if (need > kScratchElems)
        fail(RTE_E_ARG, "the no-allocation scatter needs " + std::to_string(need * sizeof(double)) +
                            " bytes of scratch for this problem, more than the " + std::to_string(kScratchBytes) +
                            " bytes it holds per device");
    double* base = scratch_on_current_device();
    if (parity == 1) {
        double* G = base;
        double* T = dtout == RTE_DT_F64 ? static_cast<double*>(Y) : base + nm;
        if (f32) k::gemm_f32(n, m, m, 1.0f, static_cast<const float*>(X), n, h->Sp_f.p, m, 0.0f, G, n, s);
        else k::gemm_f64(n, m, m, 1.0, static_cast<const double*>(X), n, h->Sp.p, m, 0.0, G, n, s);
        k::spmm_pattern(h, h->Msv.p, G, T, s);
        if (dtout == RTE_DT_F32) k::cvt_f64_f32(T, static_cast<float*>(Y), nm, s);
    } else {
        double* T = dtout == RTE_DT_F64 ? static_cast<double*>(Y) : base;
        if (f32) k::gemm_f32(n, m, m, 1.0f, static_cast<const float*>(X), n, h->Sm_f.p, m, 0.0f, T, n, s);
        else k::gemm_f64(n, m, m, 1.0, static_cast<const double*>(X), n, h->Sm.p, m, 0.0, T, n, s);
        k::row_scale(h->ms.p, n, m, T, T, s);
        if (dtout == RTE_DT_F32) k::cvt_f64_f32(T, static_cast<float*>(Y), nm, s);
    }
}

}  // namespace rte
