// Allocation-free form of the full direct-adjoint gradient: the same
// launches as pxp_gradient, with the workspace taken from a fixed device
// array of the library instead of a caller buffer.
//
// The array is a file-scope __device__ symbol: each GPU the library runs on
// holds its own copy at its own address for the life of the process.  Host
// code never passes the symbol's name to a kernel or a copy (on the host it
// is only a stand-in, not a device address); the device address is looked
// up once per device with hipGetSymbolAddress and kept in a per-device
// table.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/paraexp.h"
#include "pxp_internal.hpp"

static __device__ __align__(256) unsigned char scratch[PXP_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};

// Device address of this GPU's copy of `scratch` (looked up on the first
// call on the device, with that device current).
pxp_status scratch_ptr(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PXP_EHIP;
    if (dev < 0 || dev >= MAX_DEVICES) return PXP_EHIP;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return PXP_EHIP;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return PXP_OK;
}

// dst[0..n) = src[0..n) as raw 64-bit words (the status block holds flags and
// counters, not values).
__global__ void k_copy_words(const unsigned long long* __restrict__ src,
                             unsigned long long* __restrict__ dst, int n) {
    const int i = threadIdx.x;
    if (i < n) dst[i] = src[i];
}

}  // namespace

extern "C" pxp_status pxp_gradient_noalloc(const pxp_problem* pb, int32_t batch,
                                           int32_t method, const double* ctrl,
                                           const double* basis, const double* q0,
                                           const double* u_tgt, double* J, double* grad,
                                           double* qT, double* lam_out, void* status_out,
                                           void* stream) {
    size_t need = 0;
    pxp_status st = pxp_workspace_size(pb, batch, &need);
    if (st != PXP_OK) return st;
    if (need > (size_t)PXP_NOALLOC_SCRATCH_BYTES) return PXP_EWORKSPACE;
    if (batch == 0) return PXP_OK;
    void* ws = nullptr;
    st = scratch_ptr(&ws);
    if (st != PXP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the status block (flags, largest estimate, counters) starts at zero
    // for every call; nothing else of the array is read before written
    constexpr int words = (int)(sizeof(pxp::DevStatus) / sizeof(double));
    if (pxp::launch_zero(static_cast<double*>(ws), words, s) != hipSuccess) return PXP_EHIP;
    st = pxp_gradient(pb, batch, method, ctrl, basis, q0, u_tgt, J, grad, qT, lam_out, ws,
                      (size_t)PXP_NOALLOC_SCRATCH_BYTES, stream);
    if (st != PXP_OK) return st;
    if (status_out) {
        k_copy_words<<<1, 64, 0, s>>>(static_cast<const unsigned long long*>(ws),
                                      static_cast<unsigned long long*>(status_out), words);
        if (hipGetLastError() != hipSuccess) return PXP_EHIP;
    }
    return PXP_OK;
}
