// Device helpers shared by the Paraexp kernels (gfx950, wave64).
//
//  - block reductions: a scalar sum, and a "transpose" multi-sum that reduces
//    up to 64 partial dot products per thread with 63 shuffles per wave
//    (recursive halving) instead of 6 shuffles per value;
//  - small dense matrices held in LDS (row-major, leading dimension ld):
//    product, Gauss-Jordan solve, exponential by Taylor series with scaling
//    and squaring (Paterson-Stockmeyer evaluation).  These act on the
//    m x m Hessenberg matrices of the Arnoldi process (paper section 4.1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pxp {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }
__device__ __forceinline__ int num_waves() { return (blockDim.x + WAVE - 1) >> 6; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// Sum over the block; `red` is LDS scratch of at least num_waves() doubles.
// Every thread returns the total.  Begins and ends with a barrier so `red`
// may be reused immediately.
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    __syncthreads();
    if (lane_id() == 0) red[wave_id()] = v;
    __syncthreads();
    double s = 0.0;
    const int nw = num_waves();
    for (int w = 0; w < nw; ++w) s += red[w];
    return s;
}

// Two sums over the block with a single barrier.  `red` is LDS scratch of
// at least 80 doubles; the sums go to one of two slots (red + 16 and
// red + 48, 32 doubles each, so at most 16 waves), and `slot` alternates
// between calls: a call never overwrites the slot that a slower thread may
// still be reading from the previous call, and neither slot overlaps the
// first 16 doubles that block_sum uses.  Every thread gets both totals.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red, int& slot) {
    a = wave_sum(a);
    b = wave_sum(b);
    double* r = red + 16 + 32 * slot;
    if (lane_id() == 0) {
        r[wave_id()] = a;
        r[16 + wave_id()] = b;
    }
    __syncthreads();
    double sa = 0.0, sb = 0.0;
    const int nw = num_waves();
    for (int w = 0; w < nw; ++w) {
        sa += r[w];
        sb += r[16 + w];
    }
    a = sa;
    b = sb;
    slot ^= 1;
}

__device__ __forceinline__ double block_max(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    __syncthreads();
    if (lane_id() == 0) red[wave_id()] = v;
    __syncthreads();
    double s = red[0];
    const int nw = num_waves();
    for (int w = 1; w < nw; ++w) s = fmax(s, red[w]);
    return s;
}

// One recursive-halving stage of block_multi_sum: lanes whose bit O is set
// keep the upper half of their values, the others the lower half, each
// adding the partner lane's matching half.  Compile-time indices only.
template <int KMAX, int ST>
__device__ __forceinline__ void multi_sum_stage(double (&part)[KMAX], int lane) {
    constexpr int HALF = KMAX >> (ST + 1);
    if constexpr (HALF >= 1) {
        constexpr int O = 32 >> ST;
        const bool up = (lane & O) != 0;
#pragma unroll
        for (int q = 0; q < HALF; ++q) {
            const double send = up ? part[q] : part[q + HALF];
            const double keep = up ? part[q + HALF] : part[q];
            part[q] = keep + __shfl_xor(send, O, WAVE);
        }
        multi_sum_stage<KMAX, ST + 1>(part, lane);
    }
}

// Reduce part[0..KMAX) over every thread of the block (blockDim.x must be a
// multiple of 64).  out[k] (LDS) holds the sum for k < cnt on return.
// red: LDS scratch of num_waves()*KMAX doubles.  KMAX: power of two <= 64.
// Within a wave this costs KMAX-1 shuffles instead of 6 per value.
template <int KMAX>
__device__ __forceinline__ void block_multi_sum(double (&part)[KMAX], int cnt,
                                                double* red, double* out) {
    static_assert(KMAX >= 1 && KMAX <= 64 && (KMAX & (KMAX - 1)) == 0, "KMAX");
    const int lane = lane_id();
    multi_sum_stage<KMAX, 0>(part, lane);
    // log2(KMAX) stages used offsets 32 .. 64/KMAX; finish the lower bits.
    constexpr int LOG = (KMAX == 1) ? 0 : (KMAX == 2) ? 1 : (KMAX == 4) ? 2
                      : (KMAX == 8) ? 3 : (KMAX == 16) ? 4 : (KMAX == 32) ? 5 : 6;
    double v = part[0];
#pragma unroll
    for (int o = 32 >> LOG; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
    const int k = lane >> (6 - LOG);
    __syncthreads();
    if ((lane & ((1 << (6 - LOG)) - 1)) == 0) red[wave_id() * KMAX + k] = v;
    __syncthreads();
    const int nw = num_waves();
    if ((int)threadIdx.x < cnt) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[w * KMAX + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// ---- small dense matrices in LDS (n <= 64 rows) -----------------------

// Visits the (row, col) pairs of an n x ncol index space, this thread's
// share in the order o = threadIdx.x + i * blockDim.x, without a division
// per element.
template <class F>
__device__ __forceinline__ void for_rc(int n, int ncol, F&& f) {
    const int B = blockDim.x;
    int r = threadIdx.x / ncol, c = threadIdx.x - r * ncol;
    const int dr = B / ncol, dc = B - dr * ncol;
    while (r < n) {
        f(r, c);
        c += dc;
        r += dr;
        if (c >= ncol) {
            c -= ncol;
            ++r;
        }
    }
}

// C = A * B (n x n, leading dimension ld).  C must not alias A or B.
// FP64 matrix-core tiles: each wave takes 16 x 16 tiles of C in turn and
// accumulates them over k in steps of 4 with v_mfma_f64_16x16x4f64 (lane l
// supplies A[row0 + l%16][k + l/16] and B[k + l/16][col0 + l%16] and holds
// C[row0 + 4j + l/16][col0 + l%16], j < 4).  Entries past n are read as
// zero and not written.  Every operand is read from LDS once per tile
// instead of once per output element.
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void sm_matmul(double* C, const double* A, const double* B,
                                 int n, int ld) {
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    const int nt = (n + 15) >> 4;
    const int li = lane & 15, lk = lane >> 4;
    for (int q = threadIdx.x >> 6; q < nt * nt; q += nw) {
        const int r0 = (q / nt) * 16, c0 = (q % nt) * 16;
        const int ra = r0 + li, cb = c0 + li;
        mfma_d4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < n; k0 += 4) {
            const int kk = k0 + lk;
            const double av = (ra < n && kk < n) ? A[ra * ld + kk] : 0.0;
            const double bv = (kk < n && cb < n) ? B[kk * ld + cb] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + 4 * j + lk;
            if (r < n && cb < n) C[r * ld + cb] = acc[j];
        }
    }
    __syncthreads();
}

// Y = alpha * X + beta * I + Z*gamma (elementwise combination helper).
__device__ __forceinline__ void sm_comb(double* Y, int n, int ld, double a,
                               const double* X, double g, const double* Z,
                               double dI) {
    for_rc(n, n, [&](int r, int c) {
        double v = a * X[r * ld + c];
        if (Z) v += g * Z[r * ld + c];
        if (r == c) v += dI;
        Y[r * ld + c] = v;
    });
    __syncthreads();
}

__device__ __forceinline__ double sm_norm1(const double* A, int n, int ld, double* red) {
    double mx = 0.0;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        double s = 0.0;
        for (int r = 0; r < n; ++r) s += fabs(A[r * ld + c]);
        mx = fmax(mx, s);
    }
    return block_max(mx, red);
}

// Gauss-Jordan elimination with partial pivoting on the augmented matrix
// [A | B] (n rows, ncol = n + nrhs columns, leading dimension ld).  On
// return the last nrhs columns hold A^{-1} B.  Returns false (uniformly) if a
// pivot is exactly zero.  piv: LDS scratch of 2 ints; red: LDS scratch.
__device__ __forceinline__ bool sm_gauss_jordan(double* Ab, int n, int ncol, int ld,
                                       double* red, int* piv) {
    bool ok = true;
    for (int k = 0; k < n; ++k) {
        // pivot search in column k (one wave suffices for n <= 64 rows).
        if (threadIdx.x < WAVE) {
            double best = -1.0;
            int bi = k;
            for (int r = k + threadIdx.x; r < n; r += WAVE) {
                double v = fabs(Ab[r * ld + k]);
                if (v > best) { best = v; bi = r; }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                double ob = __shfl_xor(best, o, WAVE);
                int oi = __shfl_xor(bi, o, WAVE);
                if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
            }
            if (threadIdx.x == 0) piv[0] = bi;
        }
        __syncthreads();
        const int p = piv[0];
        if (p != k) {
            for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
                double t = Ab[k * ld + c];
                Ab[k * ld + c] = Ab[p * ld + c];
                Ab[p * ld + c] = t;
            }
            __syncthreads();
        }
        const double d = Ab[k * ld + k];
        if (d == 0.0) { ok = false; break; }
        const double inv = 1.0 / d;
        // eliminate column k from every other row, then scale the pivot row
        const int w = ncol - k - 1;
        if (w > 0)
            for_rc(n, w, [&](int r, int cc) {
                const int c = k + 1 + cc;
                if (r != k) Ab[r * ld + c] -= Ab[r * ld + k] * inv * Ab[k * ld + c];
            });
        __syncthreads();
        for (int c = threadIdx.x; c < ncol; c += blockDim.x)
            if (c > k) Ab[k * ld + c] *= inv;
        for (int r = threadIdx.x; r < n; r += blockDim.x)
            Ab[r * ld + k] = (r == k) ? 1.0 : 0.0;
        __syncthreads();
    }
    (void)red;
    return ok;
}

// Solves the complex upper-Hessenberg system (Mr + i Mi) x = (xr + i xi)
// in place (n x n, leading dimension n; the right-hand side is overwritten
// by the solution).  Gaussian elimination with partial pivoting: column j
// has one entry below the diagonal, so step j only compares, swaps and
// combines rows j and j+1 (columns j+1.. and the right-hand side; the pivot
// goes to dr/di, so no thread writes what another may still be reading);
// then back substitution, one column per step.  All threads take the same
// pivot decisions from the same LDS values.  dr, di: n doubles of scratch.
__device__ __forceinline__ void sm_hess_solve_c(double* Mr, double* Mi, double* xr,
                                                double* xi, double* dr, double* di,
                                                int n) {
    const int t = threadIdx.x, B = blockDim.x;
    for (int j = 0; j + 1 < n; ++j) {
        const double ar = Mr[j * n + j], ai = Mi[j * n + j];
        const double br = Mr[(j + 1) * n + j], bi = Mi[(j + 1) * n + j];
        const bool swap = (br * br + bi * bi) > (ar * ar + ai * ai);
        const double pr = swap ? br : ar, pi = swap ? bi : ai;
        const double qr = swap ? ar : br, qi = swap ? ai : bi;
        const double den = pr * pr + pi * pi;
        const double lr = (qr * pr + qi * pi) / den, li = (qi * pr - qr * pi) / den;
        if (t == 0) {
            dr[j] = pr;
            di[j] = pi;
        }
        for (int c = j + 1 + t; c <= n; c += B) {
            // column n stands for the right-hand side
            double* R0 = (c < n) ? Mr + j * n + c : xr + j;
            double* I0 = (c < n) ? Mi + j * n + c : xi + j;
            double* R1 = (c < n) ? Mr + (j + 1) * n + c : xr + j + 1;
            double* I1 = (c < n) ? Mi + (j + 1) * n + c : xi + j + 1;
            const double ur = swap ? *R1 : *R0, ui = swap ? *I1 : *I0;
            const double vr = swap ? *R0 : *R1, vi = swap ? *I0 : *I1;
            *R0 = ur;
            *I0 = ui;
            *R1 = vr - (lr * ur - li * ui);
            *I1 = vi - (lr * ui + li * ur);
        }
        __syncthreads();
    }
    if (t == 0) {
        dr[n - 1] = Mr[(n - 1) * n + n - 1];
        di[n - 1] = Mi[(n - 1) * n + n - 1];
    }
    __syncthreads();
    for (int i = n - 1; i >= 0; --i) {
        const double ddr = dr[i], ddi = di[i];
        const double den = ddr * ddr + ddi * ddi;
        const double sr = xr[i], si = xi[i];
        const double yr = (sr * ddr + si * ddi) / den, yi = (si * ddr - sr * ddi) / den;
        for (int r = t; r < i; r += B) {
            const double mr = Mr[r * n + i], mi = Mi[r * n + i];
            xr[r] -= mr * yr - mi * yi;
            xi[r] -= mr * yi + mi * yr;
        }
        __syncthreads();
        if (t == 0) {
            xr[i] = yr;
            xi[i] = yi;
        }
    }
    __syncthreads();
}

// X = H^{-1} for an n x n upper-Hessenberg H (leading dimension ldh, read
// only).  U (n x n) and D (n) are scratch; X has leading dimension n.
// Elimination of [H | I] with partial pivoting between neighbouring rows
// (one barrier per column; the pivots go to D so no thread overwrites what
// another may still read), then back substitution with one thread per
// column of X.
__device__ __forceinline__ void sm_hess_inverse(const double* H, int ldh, int n,
                                                double* U, double* D, double* X) {
    const int t = threadIdx.x, B = blockDim.x;
    for_rc(n, n, [&](int r, int c) {
        U[r * n + c] = H[r * ldh + c];
        X[r * n + c] = (r == c) ? 1.0 : 0.0;
    });
    __syncthreads();
    for (int j = 0; j + 1 < n; ++j) {
        const double a = U[j * n + j], b = U[(j + 1) * n + j];
        const bool swap = fabs(b) > fabs(a);
        const double p = swap ? b : a, l = (swap ? a : b) / p;
        if (t == 0) D[j] = p;
        const int wu = n - j - 1;  // columns j+1.. of U, then the n of X
        for (int c = t; c < wu + n; c += B) {
            double* R0 = (c < wu) ? U + j * n + j + 1 + c : X + j * n + (c - wu);
            double* R1 = (c < wu) ? U + (j + 1) * n + j + 1 + c : X + (j + 1) * n + (c - wu);
            const double u = swap ? *R1 : *R0, v = swap ? *R0 : *R1;
            *R0 = u;
            *R1 = v - l * u;
        }
        __syncthreads();
    }
    if (t == 0) D[n - 1] = U[(n - 1) * n + n - 1];
    __syncthreads();
    for (int c = t; c < n; c += B) {
        for (int i = n - 1; i >= 0; --i) {
            double s = X[i * n + c];
            for (int q = i + 1; q < n; ++q) s -= U[i * n + q] * X[q * n + c];
            X[i * n + c] = s / D[i];
        }
    }
    __syncthreads();
}

// E = exp(M) for an n x n matrix in LDS (M is overwritten).  Taylor
// polynomial of degree 16 evaluated by the Paterson-Stockmeyer scheme on
// A = M / 2^s with ||A||_1 <= 1/2, followed by s squarings (Moler & Van Loan,
// "Nineteen dubious ways to compute the exponential of a matrix": scaling and
// squaring with a truncated Taylor series).  The truncation error is below
// 2^-17/17! ~ 2e-20 relative to the scaled exponential.
// Scratch W must hold 4 matrices of n x ld.  Returns the number of squarings.
__device__ __forceinline__ int sm_expm(double* E, double* M, int n, int ld, double* W,
                              double* red) {
    const int sz = n * ld;
    double* A = M;
    double* A2 = W;
    double* A3 = W + sz;
    double* A4 = W + 2 * sz;
    double* T = W + 3 * sz;
    const double nrm = sm_norm1(M, n, ld, red);
    int s = 0;
    if (nrm > 0.5) s = (int)ceil(log2(nrm / 0.5));
    if (!(s <= 1000)) s = 1000;  // also catches NaN norms
    const double sc = ldexp(1.0, -s);
    sm_comb(A, n, ld, sc, M, 0.0, nullptr, 0.0);
    sm_matmul(A2, A, A, n, ld);
    sm_matmul(A3, A2, A, n, ld);
    sm_matmul(A4, A3, A, n, ld);
    double f[17];
    f[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= 16; ++k) f[k] = f[k - 1] / (double)k;
    // T = f16 I; then T = B_j + A4 T for j = 3..0 with
    // B_j = f_{4j} I + f_{4j+1} A + f_{4j+2} A^2 + f_{4j+3} A^3.
    sm_comb(T, n, ld, 0.0, A, 0.0, nullptr, f[16]);
#pragma unroll
    for (int j = 3; j >= 0; --j) {
        sm_matmul(E, A4, T, n, ld);
        const int b = 4 * j;
        for_rc(n, n, [&](int r, int c) {
            const int ix = r * ld + c;
            double v = E[ix] + f[b + 1] * A[ix] + f[b + 2] * A2[ix] + f[b + 3] * A3[ix];
            if (r == c) v += f[b];
            T[ix] = v;
        });
        __syncthreads();
    }
    double* src = T;
    double* dst = E;
    for (int q = 0; q < s; ++q) {
        sm_matmul(dst, src, src, n, ld);
        double* t = src;
        src = dst;
        dst = t;
    }
    if (src != E) {
        for_rc(n, n, [&](int r, int c) { E[r * ld + c] = src[r * ld + c]; });
        __syncthreads();
    }
    return s;
}

}  // namespace pxp
