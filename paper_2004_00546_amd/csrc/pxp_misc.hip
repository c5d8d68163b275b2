// Small kernels of the direct-adjoint loop: control -> forcing/initial state,
// cost and adjoint final condition (eq. adjFinalTime), gradient reductions
// (eqs. paramupdate, initupdate) and the superposition of the Paraexp pieces
// (eq. fullsol0).  All reductions are deterministic (fixed order).
#include "pxp_internal.hpp"
#include "pxp_device.hpp"

#include <cstring>

namespace pxp {
namespace {

__global__ void k_combine_basis(const double* __restrict__ a,
                                const double* __restrict__ basis,
                                const double* __restrict__ base,
                                double* __restrict__ out, int K, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // four independent partial sums (fixed order) keep several loads in
    // flight instead of one dependent chain
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    int k = 0;
    for (; k + 4 <= K; k += 4)
#pragma unroll
        for (int u = 0; u < 4; ++u) s[u] += a[k + u] * basis[(size_t)(k + u) * n + i];
    for (; k < K; ++k) s[0] += a[k] * basis[(size_t)k * n + i];
    out[i] = (base ? base[i] : 0.0) + ((s[0] + s[1]) + (s[2] + s[3]));
}

__global__ void k_apply_tri(const double* __restrict__ x, double* __restrict__ out,
                            int n, Tri op) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xm = x[i == 0 ? n - 1 : i - 1];
    const double xp = x[i == n - 1 ? 0 : i + 1];
    out[i] = op.lo * xm + op.d * x[i] + op.up * xp;
}

// One workgroup: lamT = qT - tgt, J = 1/2 |lamT|^2 + beta |a|^2.
__global__ void __launch_bounds__(256)
k_cost(const double* __restrict__ qT, const double* __restrict__ tgt,
       const double* __restrict__ a, int n, int K, double beta,
       double* __restrict__ lamT, double* __restrict__ J, DevStatus* st) {
    __shared__ double red[8];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double d = qT[i] - tgt[i];
        if (lamT) lamT[i] = d;
        s += d * d;
    }
    double r = 0.0;
    for (int k = threadIdx.x; k < K; k += blockDim.x) r += a[k] * a[k];
    s = block_sum(s, red);
    r = block_sum(r, red);
    if (threadIdx.x == 0) {
        *J = 0.5 * s + beta * r;
        // every method's q(T) passes through here
        if (st && !isfinite(s + r)) atomicOr(&st->flags, ST_NONFINITE);
    }
}

// One workgroup per control k: grad[k] = <basis_k, v> + 2 beta a[k].
__global__ void __launch_bounds__(256)
k_grad(const double* __restrict__ basis, const double* __restrict__ v,
       const double* __restrict__ a, int n, double beta,
       double* __restrict__ grad, DevStatus* st) {
    __shared__ double red[8];
    const int k = blockIdx.x;
    const double* b = basis + (size_t)k * n;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += b[i] * v[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        grad[k] = s + 2.0 * beta * a[k];
        if (st && !isfinite(grad[k])) atomicOr(&st->flags, ST_NONFINITE);
    }
}

__global__ void k_recombine(const double* __restrict__ q0,
                            const double* __restrict__ vlast,
                            const double* __restrict__ Y, int np, int n,
                            double* __restrict__ out, DevStatus* st) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    int p = 0;
    for (; p + 4 <= np; p += 4)
#pragma unroll
        for (int u = 0; u < 4; ++u) t[u] += Y[(size_t)(p + u) * n + i];
    for (; p < np; ++p) t[0] += Y[(size_t)p * n + i];
    double s = q0 ? q0[i] : 0.0;
    if (vlast) s += vlast[i];
    s += (t[0] + t[1]) + (t[2] + t[3]);
    out[i] = s;
    if (st && !isfinite(s)) atomicOr(&st->flags, ST_NONFINITE);
}

__global__ void k_add(const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ out, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = (a ? a[i] : 0.0) + b[i];
}

inline int blocks(int n, int b) { return (n + b - 1) / b; }

__device__ __forceinline__ int red_entry(const RedDesc* tab, int count, int b, bool grad) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((grad ? tab[mid].blk0_grad : tab[mid].blk0_cost) <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Batched cost, phase 1: block (instance, chunk) forms lamT = qT - tgt on
// its chunk of RED_CHUNK points and the partial sum of lamT^2.
__global__ void __launch_bounds__(256)
k_cost_part(const RedDesc* __restrict__ tab, int count, double* __restrict__ part) {
    __shared__ double red[8];
    const RedDesc& d = tab[red_entry(tab, count, blockIdx.x, false)];
    const int c = blockIdx.x - d.blk0_cost;
    const int i0 = c * RED_CHUNK, i1 = min(d.n, i0 + RED_CHUNK);
    double s0 = 0.0, s1 = 0.0;
    int i = i0 + threadIdx.x;
    for (; i + 256 < i1; i += 512) {
        const double a = d.qT[i] - d.tgt[i], b = d.qT[i + 256] - d.tgt[i + 256];
        if (d.lamT) {
            d.lamT[i] = a;
            d.lamT[i + 256] = b;
        }
        s0 += a * a;
        s1 += b * b;
    }
    if (i < i1) {
        const double a = d.qT[i] - d.tgt[i];
        if (d.lamT) d.lamT[i] = a;
        s0 += a * a;
    }
    const double s = block_sum(s0 + s1, red);
    if (threadIdx.x == 0) part[d.part0 + c] = s;
}

// Batched cost, phase 2: one wave per instance; lane l sums partials l,
// l+64, ... in order, then the lanes combine in a fixed pattern.
__global__ void __launch_bounds__(64)
k_cost_fin(const RedDesc* __restrict__ tab, const double* __restrict__ part) {
    const RedDesc& d = tab[blockIdx.x];
    const int l = threadIdx.x;
    double s = 0.0, r = 0.0;
    if (d.ipart) {
        for (int c = l; c < d.ichunks; c += WAVE) s += d.ipart[c];
        s = wave_sum(s);
    } else {
        for (int c = l; c < d.chunks; c += WAVE) s += part[d.part0 + c];
        s = 0.5 * wave_sum(s);
    }
    if (l != 0) return;
    for (int k = 0; k < d.K; ++k) r += d.a[k] * d.a[k];
    *d.J = s + d.beta * r;
    // every method's q(T) passes through here
    if (d.st && !isfinite(s + r)) atomicOr(&d.st->flags, ST_NONFINITE);
}

// Batched gradient, phase 1: block (instance, k, chunk) forms the partial
// <basis_k, v> over its chunk.
__global__ void __launch_bounds__(256)
k_grad_part(const RedDesc* __restrict__ tab, int count, double* __restrict__ part) {
    __shared__ double red[8];
    const RedDesc& d = tab[red_entry(tab, count, blockIdx.x, true)];
    const int local = blockIdx.x - d.blk0_grad;
    const int k = local / d.chunks, c = local - k * d.chunks;
    const double* b = d.basis + (size_t)k * d.n;
    const int i0 = c * RED_CHUNK, i1 = min(d.n, i0 + RED_CHUNK);
    double s0 = 0.0, s1 = 0.0;
    int i = i0 + threadIdx.x;
    for (; i + 256 < i1; i += 512) {
        s0 += b[i] * d.v[i];
        s1 += b[i + 256] * d.v[i + 256];
    }
    if (i < i1) s0 += b[i] * d.v[i];
    const double s = block_sum(s0 + s1, red);
    if (threadIdx.x == 0) part[d.gpart0 + (size_t)k * d.chunks + c] = s;
}

// Batched gradient, phase 2: grad_k = sum of the partials + 2 beta a_k.
__global__ void __launch_bounds__(256)
k_grad_fin(const RedDesc* __restrict__ tab, const double* __restrict__ part) {
    const RedDesc& d = tab[blockIdx.x];
    bool bad = false;
    for (int k = threadIdx.x; k < d.K; k += blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < d.chunks; ++c) s += part[d.gpart0 + (size_t)k * d.chunks + c];
        const double g = s + 2.0 * d.beta * d.a[k];
        d.grad[k] = g;
        bad |= !isfinite(g);
    }
    if (d.st && bad) atomicOr(&d.st->flags, ST_NONFINITE);
}

}  // namespace

hipError_t launch_cost_batch(const RedDesc* tab, int count, int blocks_cost, double* part,
                             hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (blocks_cost > 0) {
        k_cost_part<<<blocks_cost, 256, 0, s>>>(tab, count, part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_cost_fin<<<count, 64, 0, s>>>(tab, part);
    return hipGetLastError();
}

hipError_t launch_grad_batch(const RedDesc* tab, int count, int blocks_grad, double* part,
                             hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (blocks_grad > 0) {
        k_grad_part<<<blocks_grad, 256, 0, s>>>(tab, count, part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_grad_fin<<<count, 256, 0, s>>>(tab, part);
    return hipGetLastError();
}

hipError_t launch_combine_basis(const double* a, const double* basis,
                                const double* base, double* out, int K, int n,
                                hipStream_t s) {
    k_combine_basis<<<blocks(n, 64), 64, 0, s>>>(a, basis, base, out, K, n);
    return hipGetLastError();
}

hipError_t launch_apply_tri(const double* x, double* out, int n, Tri op,
                            hipStream_t s) {
    k_apply_tri<<<blocks(n, 256), 256, 0, s>>>(x, out, n, op);
    return hipGetLastError();
}

hipError_t launch_cost(const double* qT, const double* tgt, const double* a,
                       int n, int K, double beta, double* lamT, double* J,
                       hipStream_t s, DevStatus* st) {
    k_cost<<<1, 256, 0, s>>>(qT, tgt, a, n, K, beta, lamT, J, st);
    return hipGetLastError();
}

hipError_t launch_grad(const double* basis, const double* v, const double* a,
                       int K, int n, double beta, double* grad, hipStream_t s,
                       DevStatus* st) {
    if (K <= 0) return hipSuccess;
    k_grad<<<K, 256, 0, s>>>(basis, v, a, n, beta, grad, st);
    return hipGetLastError();
}

// One block per instance: the Richardson estimate of each sampled Magnus
// step, sums in a fixed order.
__global__ void __launch_bounds__(256) k_magnus_check(const MagnusCheck* __restrict__ tab) {
    __shared__ double red[80];
    const MagnusCheck& d = tab[blockIdx.x];
    double est = 0.0;
    int slot = 0;
    for (int k = 0; k < d.nsamp; ++k) {
        const double* a = d.y + (size_t)(2 * k) * d.n;
        const double* b = a + d.n;
        double dd = 0.0, bb = 0.0;
        for (int i = threadIdx.x; i < d.n; i += blockDim.x) {
            const double e = a[i] - b[i];
            dd += e * e;
            bb += b[i] * b[i];
        }
        block_sum2(dd, bb, red, slot);
        const double e = bb > 0.0 ? d.scale * sqrt(dd / bb) : 0.0;
        est = fmax(est, e);
    }
    if (threadIdx.x != 0) return;
    bool bad = !isfinite(est);
    if (bad) est = INFINITY;
    const unsigned long long eb = (unsigned long long)__double_as_longlong(est);
    if (d.st) {
        atomicMax(&d.st->max_est, eb);
        if (bad) atomicOr(&d.st->flags, ST_NONFINITE);
        else if (est > d.tol) atomicOr(&d.st->flags, ST_NOCONV);
    }
    if (d.irep) atomicMax(&d.irep->max_est, eb);
}

hipError_t launch_magnus_check(const MagnusCheck* tab, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    k_magnus_check<<<count, 256, 0, s>>>(tab);
    return hipGetLastError();
}

__global__ void k_scaled_diff(const double* __restrict__ x, const double* __restrict__ y,
                              double a, double* __restrict__ out, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a * (x[i] - y[i]);
}

hipError_t launch_scaled_diff(const double* x, const double* y, double a, double* out, int n,
                              hipStream_t s) {
    k_scaled_diff<<<blocks(n, 256), 256, 0, s>>>(x, y, a, out, n);
    return hipGetLastError();
}

hipError_t launch_recombine(const double* q0, const double* vlast,
                            const double* Y, int np, int n, double* out,
                            DevStatus* st, hipStream_t s) {
    k_recombine<<<blocks(n, 64), 64, 0, s>>>(q0, vlast, Y, np, n, out, st);
    return hipGetLastError();
}

hipError_t launch_add(const double* a, const double* b, double* out, int n,
                      hipStream_t s) {
    k_add<<<blocks(n, 256), 256, 0, s>>>(a, b, out, n);
    return hipGetLastError();
}

}  // namespace pxp

namespace pxp {
namespace {
__global__ void k_zero(double* __restrict__ p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}
}  // namespace

struct UploadChunk {
    unsigned char b[3072];
};

__global__ void k_upload(unsigned char* __restrict__ dst, UploadChunk c, int bytes) {
    for (int i = threadIdx.x; i < bytes; i += blockDim.x) dst[i] = c.b[i];
}

hipError_t launch_upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
    unsigned char* d = static_cast<unsigned char*>(dst);
    const unsigned char* h = static_cast<const unsigned char*>(src);
    while (bytes > 0) {
        const size_t nb = bytes > sizeof(UploadChunk) ? sizeof(UploadChunk) : bytes;
        UploadChunk c;
        memcpy(c.b, h, nb);
        k_upload<<<1, 256, 0, s>>>(d, c, (int)nb);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        d += nb;
        h += nb;
        bytes -= nb;
    }
    return hipSuccess;
}

hipError_t launch_zero(double* p, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_zero<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
    return hipGetLastError();
}
}  // namespace pxp
