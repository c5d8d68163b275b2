// Classical RK4 marches for the 1D operators (paper section 4.2/4.3).
//
// Layout: one workgroup marches one state vector of n points; thread t owns
// the contiguous chunk [t*PT, (t+1)*PT) in registers for the whole march, so
// a step touches HBM only for checkpoints.  A stencil needs one neighbour on
// each side of a chunk: the chunk edges are exchanged through LDS with one
// barrier per stage (double-buffered, so no second barrier is needed).
//
// Used for
//  - the P inhomogeneous sub-problems of the Paraexp direct solve, one
//    workgroup per slice, each from zero data (section 3.1, eq.
//    linInhomEqus);
//  - the serial march (P = 1) that Paraexp is compared with;
//  - the reverse sweep of the exact discrete adjoint of that march;
//  - the serial Burgers direct march with checkpoints (section 3.3, 3.5).
#include "pxp_internal.hpp"
#include "pxp_device.hpp"

namespace pxp {
namespace {

// Largest workgroup for PT points per thread: keeps the register arrays of
// the march (about 6 PT doubles) inside the VGPR budget without spills.
template <int PT>
constexpr int max_block() {
    return PT <= 4 ? 1024 : (PT <= 16 ? 512 : 256);
}

// Exchange the chunk edges of NA arrays with one barrier.  edge is LDS of
// 2 buffers of NB x 2 x B values (NB >= NA: the same buffer stride must be
// used by every exchange of a kernel so the two buffers never overlap).
template <int PT, int NA, int NB = NA, typename R>
__device__ __forceinline__ void exch(const R* const (&arrs)[NA], R* edge, int& buf,
                                     R (&left)[NA], R (&right)[NA]) {
    static_assert(NB >= NA, "buffer stride");
    const int t = threadIdx.x, B = blockDim.x;
    R* e = edge + buf * 2 * NB * B;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        e[(2 * a) * B + t] = arrs[a][0];
        e[(2 * a + 1) * B + t] = arrs[a][PT - 1];
    }
    __syncthreads();
    const int tl = (t == 0) ? B - 1 : t - 1;
    const int tr = (t == B - 1) ? 0 : t + 1;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        left[a] = e[(2 * a + 1) * B + tl];
        right[a] = e[(2 * a) * B + tr];
    }
    buf ^= 1;
}

// Compensated accumulation s += inc (Kahan) in FP32; plain in FP64.
template <typename R>
__device__ __forceinline__ void kadd(R& s, R& c, R inc) {
    if constexpr (sizeof(R) == 4) {
        const R yk = inc - c;
        const R t = s + yk;
        c = (t - s) - yk;
        s = t;
    } else {
        (void)c;
        s += inc;
    }
}

// value of a compensated pair in FP64
template <typename R>
__device__ __forceinline__ double hilo(R s, R c) {
    return (double)s - (double)c;
}
// split an FP64 value into a compensated pair (exact for FP32 pairs)
template <typename R>
__device__ __forceinline__ void split_hilo(double v, R& s, R& c) {
    s = (R)v;
    c = (sizeof(R) == 4) ? (R)((double)s - v) : (R)0;
}

// Coefficients of a tridiagonal operator split for accuracy:
// lo x_{i-1} + d x_i + up x_{i+1} = cs ((x_{i+1} + x_{i-1}) - 2 x_i)
//                                  + cdf (x_{i+1} - x_{i-1}) + cc x_i
struct TriSplit {
    double cs, cdf, cc;
};
__host__ __device__ inline TriSplit split(Tri a) {
    TriSplit s;
    s.cs = 0.5 * (a.lo + a.up);
    s.cdf = 0.5 * (a.up - a.lo);
    s.cc = a.d + 2.0 * s.cs;
    return s;
}

// The forcing sin(omega t) (and the integral weight sin(ia + ib t)) at the
// three stage times t_s, t_s + dt/2, t_s + dt of a step is the same for
// every point: a block of SINE_BLK steps is tabulated into LDS by the whole
// workgroup, one sine per thread instead of three per thread per step.  Two
// tables alternate between blocks: a table is rewritten two blocks after it
// was read, with at least one barrier per step in between.  The values are
// the very expressions the march would evaluate.
constexpr int SINE_BLK = 64;
constexpr int SINE_LDS_DOUBLES = 2 * SINE_BLK * 6;

// Fill the table of block `blk` (steps blk*SINE_BLK .. of the march whose
// step s starts at time (step0 + s) dt), NV = 3 (forcing) or 6 (forcing and
// integral weights); ends with a barrier.
template <int NV>
__device__ __forceinline__ const double* sine_block(double* tabs, int64_t blk, int64_t n_s,
                                                    int64_t step0, double dt, double omega,
                                                    double ia, double ib) {
    double* tab = tabs + (blk & 1) * SINE_BLK * 6;
    for (int e = threadIdx.x; e < SINE_BLK * NV; e += blockDim.x) {
        const int ls = e / NV, v = e - ls * NV;
        const int64_t s = blk * SINE_BLK + ls;
        if (s >= n_s) continue;
        const double tn = (double)(step0 + s) * dt;
        double val;
        switch (v) {
            case 0: val = sin(omega * tn); break;
            case 1: val = sin(omega * (tn + 0.5 * dt)); break;
            case 2: val = sin(omega * (tn + dt)); break;
            case 3: val = sin(ia + ib * tn); break;
            case 4: val = sin(ia + ib * (tn + 0.5 * dt)); break;
            default: val = sin(ia + ib * (tn + dt)); break;
        }
        tab[ls * 6 + v] = val;
    }
    __syncthreads();
    return tab;
}

// CC = false: the operator has cc == 0 (central advection-diffusion, where
// lo + d + up = 0 exactly), and the term, exactly zero, is not formed.
template <int PT, typename R, bool CC = true>
__device__ __forceinline__ void tri_rhs(const R (&Y)[PT], R l, R r, R cs, R cdf,
                                        R cc, R (&k)[PT]) {
#pragma unroll
    for (int q = 0; q < PT; ++q) {
        const R ym = (q == 0) ? l : Y[q - 1];
        const R yp = (q == PT - 1) ? r : Y[q + 1];
        if constexpr (CC)
            k[q] = cs * ((yp + ym) - (R)2 * Y[q]) + cdf * (yp - ym) + cc * Y[q];
        else
            k[q] = cs * ((yp + ym) - (R)2 * Y[q]) + cdf * (yp - ym);
    }
}

// G = false: no constant source (g0 is null), the term is not formed.
template <int PT, typename R, bool INT, bool CC = true, bool G = true>
__device__ __forceinline__ void
dev_rk4_lin1d(const double* __restrict__ F, const double* __restrict__ g0,
              const double* __restrict__ y0, double* __restrict__ out, int n,
              int64_t n_s, double dt, double omega, TriSplit A, SliceIntegral si) {
    extern __shared__ double lds_d[];
    R* lds = reinterpret_cast<R*>(lds_d);
    const int t = threadIdx.x;
    const int p = blockIdx.x;
    const int base = t * PT;
    const R cs = (R)A.cs, cdf = (R)A.cdf, cc = (R)A.cc;
    R f[PT], g[PT], y[PT], yc[PT], acc[PT], Y[PT], k[PT];
#pragma unroll
    for (int q = 0; q < PT; ++q) {
        f[q] = F ? (R)F[base + q] : (R)0;
        g[q] = (G && g0) ? (R)g0[base + q] : (R)0;
        split_hilo<R>(y0 ? y0[base + q] : 0.0, y[q], yc[q]);
    }
    int buf = 0;
    const int64_t step0 = (int64_t)p * n_s;
    const R h2 = (R)(0.5 * dt), h6 = (R)(dt / 6.0), h1 = (R)dt;
    // optional time integral I = int sin(ia + ib t) y(t) dt over the slice,
    // integrated as the extra equation I' = sin(ia + ib t) y with the same
    // RK4 stages (fourth order)
    double I[PT];
#pragma unroll
    for (int q = 0; q < PT; ++q) I[q] = 0.0;
    double* tabs = lds_d + 4 * (size_t)blockDim.x;
    const double* tab = nullptr;
    for (int64_t s = 0; s < n_s; ++s) {
        if (s % SINE_BLK == 0)
            tab = sine_block<INT ? 6 : 3>(tabs, s / SINE_BLK, n_s, step0, dt, omega, si.ia, si.ib);
        const double* sv = tab + (s % SINE_BLK) * 6;
        const R s1 = (R)sv[0];
        const R s2 = (R)sv[1];
        const R s4 = (R)sv[2];
        double w1 = 0.0, w2 = 0.0, w4 = 0.0;
        if constexpr (INT) {
            w1 = dt / 6.0 * sv[3];
            w2 = dt / 3.0 * sv[4];
            w4 = dt / 6.0 * sv[5];
#pragma unroll
            for (int q = 0; q < PT; ++q) I[q] += w1 * hilo<R>(y[q], yc[q]);
        }
        R l[1], r[1];
        {
            const R* arr[1] = {y};
            exch<PT, 1>(arr, lds, buf, l, r);
        }
        tri_rhs<PT, R, CC>(y, l[0], r[0], cs, cdf, cc, k);
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            if constexpr (G) k[q] += s1 * f[q] + g[q];
            else k[q] += s1 * f[q];
            acc[q] = k[q];
            Y[q] = y[q] + h2 * k[q];
        }
        if constexpr (INT) {
#pragma unroll
            for (int q = 0; q < PT; ++q) I[q] += w2 * ((double)y[q] - (double)yc[q] + (double)(h2 * k[q]));
        }
        {
            const R* arr[1] = {Y};
            exch<PT, 1>(arr, lds, buf, l, r);
        }
        tri_rhs<PT, R, CC>(Y, l[0], r[0], cs, cdf, cc, k);
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            if constexpr (G) k[q] += s2 * f[q] + g[q];
            else k[q] += s2 * f[q];
            acc[q] += (R)2 * k[q];
            Y[q] = y[q] + h2 * k[q];
        }
        if constexpr (INT) {
#pragma unroll
            for (int q = 0; q < PT; ++q) I[q] += w2 * ((double)y[q] - (double)yc[q] + (double)(h2 * k[q]));
        }
        {
            const R* arr[1] = {Y};
            exch<PT, 1>(arr, lds, buf, l, r);
        }
        tri_rhs<PT, R, CC>(Y, l[0], r[0], cs, cdf, cc, k);
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            if constexpr (G) k[q] += s2 * f[q] + g[q];
            else k[q] += s2 * f[q];
            acc[q] += (R)2 * k[q];
            Y[q] = y[q] + h1 * k[q];
        }
        if constexpr (INT) {
#pragma unroll
            for (int q = 0; q < PT; ++q) I[q] += w4 * ((double)y[q] - (double)yc[q] + (double)(h1 * k[q]));
        }
        {
            const R* arr[1] = {Y};
            exch<PT, 1>(arr, lds, buf, l, r);
        }
        tri_rhs<PT, R, CC>(Y, l[0], r[0], cs, cdf, cc, k);
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            if constexpr (G) k[q] += s4 * f[q] + g[q];
            else k[q] += s4 * f[q];
            kadd<R>(y[q], yc[q], h6 * (acc[q] + k[q]));
        }
    }
    double* o = out + (size_t)p * n;
#pragma unroll
    for (int q = 0; q < PT; ++q) o[base + q] = hilo<R>(y[q], yc[q]);
    if constexpr (INT) {
        double* io = si.iout + (size_t)p * n;
#pragma unroll
        for (int q = 0; q < PT; ++q)
            io[base + q] = I[q] + ((p == 0 && si.v0) ? si.c0 * si.v0[base + q] : 0.0);
    }
}

// The slice march without and with the slice integral (separate code, so
// the plain march keeps its register budget).
template <int PT, typename R>
__global__ void __launch_bounds__(max_block<PT>())
k_rk4_lin1d_plain(const double* __restrict__ F, const double* __restrict__ g0,
                  const double* __restrict__ y0, double* __restrict__ out, int n,
                  int64_t n_s, double dt, double omega, TriSplit A, SliceIntegral si) {
    dev_rk4_lin1d<PT, R, false>(F, g0, y0, out, n, n_s, dt, omega, A, si);
}
template <int PT, typename R>
__global__ void __launch_bounds__(max_block<PT>())
k_rk4_lin1d_int(const double* __restrict__ F, const double* __restrict__ g0,
                const double* __restrict__ y0, double* __restrict__ out, int n,
                int64_t n_s, double dt, double omega, TriSplit A, SliceIntegral si) {
    dev_rk4_lin1d<PT, R, true>(F, g0, y0, out, n, n_s, dt, omega, A, si);
}
// plain march of an operator with cc == 0 (see tri_rhs), with and without
// the constant source
template <int PT, typename R>
__global__ void __launch_bounds__(max_block<PT>())
k_rk4_lin1d_nocc(const double* __restrict__ F, const double* __restrict__ g0,
                 const double* __restrict__ y0, double* __restrict__ out, int n,
                 int64_t n_s, double dt, double omega, TriSplit A, SliceIntegral si) {
    dev_rk4_lin1d<PT, R, false, false>(F, g0, y0, out, n, n_s, dt, omega, A, si);
}
template <int PT, typename R>
__global__ void __launch_bounds__(max_block<PT>())
k_rk4_lin1d_nocc_nog(const double* __restrict__ F, const double* __restrict__ g0,
                     const double* __restrict__ y0, double* __restrict__ out, int n,
                     int64_t n_s, double dt, double omega, TriSplit A, SliceIntegral si) {
    dev_rk4_lin1d<PT, R, false, false, false>(F, g0, y0, out, n, n_s, dt, omega, A, si);
}

// Reverse sweep: y_{s+1} = y_s + dt sum_i b_i k_i with k_i = A Y_i + ...
// gives kbar_i = dt b_i lam (+ the chain through later stages), Ybar_i =
// A^T kbar_i, lam_s = lam_{s+1} + sum_i Ybar_i, Lambda += s(t_i) kbar_i.
template <int PT, typename R, bool CC>
__device__ __forceinline__ void
dev_rk4_rev_lin1d(const double* __restrict__ lamT, double* __restrict__ lam0,
                  double* __restrict__ Lambda, int n, int64_t n_t, double dt,
                  double omega, TriSplit AT) {
    extern __shared__ double lds_d[];
    R* lds = reinterpret_cast<R*>(lds_d);
    const int t = threadIdx.x;
    const int base = t * PT;
    const R cs = (R)AT.cs, cdf = (R)AT.cdf, cc = (R)AT.cc;
    R lam[PT], lamc[PT], Lam[PT], Lamc[PT], kb[PT], Yb[PT], nl[PT];
#pragma unroll
    for (int q = 0; q < PT; ++q) {
        split_hilo<R>(lamT[base + q], lam[q], lamc[q]);
        Lam[q] = (R)0;
        Lamc[q] = (R)0;
    }
    int buf = 0;
    const R d6 = (R)(dt / 6.0), d3 = (R)(dt / 3.0), d2 = (R)(0.5 * dt), d1 = (R)dt;
    double* tabs = lds_d + 4 * (size_t)blockDim.x;
    const double* tab = nullptr;
    for (int64_t s = n_t - 1; s >= 0; --s) {
        if (s == n_t - 1 || s % SINE_BLK == SINE_BLK - 1)
            tab = sine_block<3>(tabs, s / SINE_BLK, n_t, 0, dt, omega, 0.0, 0.0);
        const double* sv = tab + (s % SINE_BLK) * 6;
        const R s1 = (R)sv[0];
        const R s2 = (R)sv[1];
        const R s4 = (R)sv[2];
        R l[1], r[1];
        // stage 4
#pragma unroll
        for (int q = 0; q < PT; ++q) kb[q] = d6 * lam[q];
        {
            const R* arr[1] = {kb};
            exch<PT, 1>(arr, lds, buf, l, r);
        }
        tri_rhs<PT, R, CC>(kb, l[0], r[0], cs, cdf, cc, Yb);
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            nl[q] = Yb[q];
            kadd<R>(Lam[q], Lamc[q], s4 * kb[q]);
            kb[q] = d3 * lam[q] + d1 * Yb[q];
        }
        // stage 3
        {
            const R* arr[1] = {kb};
            exch<PT, 1>(arr, lds, buf, l, r);
        }
        tri_rhs<PT, R, CC>(kb, l[0], r[0], cs, cdf, cc, Yb);
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            nl[q] += Yb[q];
            kadd<R>(Lam[q], Lamc[q], s2 * kb[q]);
            kb[q] = d3 * lam[q] + d2 * Yb[q];
        }
        // stage 2
        {
            const R* arr[1] = {kb};
            exch<PT, 1>(arr, lds, buf, l, r);
        }
        tri_rhs<PT, R, CC>(kb, l[0], r[0], cs, cdf, cc, Yb);
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            nl[q] += Yb[q];
            kadd<R>(Lam[q], Lamc[q], s2 * kb[q]);
            kb[q] = d6 * lam[q] + d2 * Yb[q];
        }
        // stage 1
        {
            const R* arr[1] = {kb};
            exch<PT, 1>(arr, lds, buf, l, r);
        }
        tri_rhs<PT, R, CC>(kb, l[0], r[0], cs, cdf, cc, Yb);
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            kadd<R>(Lam[q], Lamc[q], s1 * kb[q]);
            kadd<R>(lam[q], lamc[q], nl[q] + Yb[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < PT; ++q) {
        if (lam0) lam0[base + q] = hilo<R>(lam[q], lamc[q]);
        if (Lambda) Lambda[base + q] = hilo<R>(Lam[q], Lamc[q]);
    }
}

template <int PT, typename R>
__global__ void __launch_bounds__(max_block<PT>())
k_rk4_rev_lin1d(const double* __restrict__ lamT, double* __restrict__ lam0,
                double* __restrict__ Lambda, int n, int64_t n_t, double dt,
                double omega, TriSplit AT) {
    dev_rk4_rev_lin1d<PT, R, true>(lamT, lam0, Lambda, n, n_t, dt, omega, AT);
}
template <int PT, typename R>
__global__ void __launch_bounds__(max_block<PT>())
k_rk4_rev_lin1d_nocc(const double* __restrict__ lamT, double* __restrict__ lam0,
                     double* __restrict__ Lambda, int n, int64_t n_t, double dt,
                     double omega, TriSplit AT) {
    dev_rk4_rev_lin1d<PT, R, false>(lamT, lam0, Lambda, n, n_t, dt, omega, AT);
}

// ---- Burgers: N(u)_i = -u_i (u_{i+1} - u_{i-1})/(2h) + nu lap(u)_i -------

struct BurgersC {
    double inv2h, nuh2;
};

template <int PT, typename R>
__device__ __forceinline__ void burgers_rhs(const R (&Y)[PT], R l, R r, R inv2h,
                                            R nuh2, R (&k)[PT]) {
#pragma unroll
    for (int q = 0; q < PT; ++q) {
        const R ym = (q == 0) ? l : Y[q - 1];
        const R yp = (q == PT - 1) ? r : Y[q + 1];
        k[q] = -Y[q] * ((yp - ym) * inv2h) + nuh2 * ((yp + ym) - (R)2 * Y[q]);
    }
}

// One Burgers RK4 step in registers; the state is the compensated pair
// (y, yc).  With 8 or more points per thread the chunk edges are exchanged
// once per step: each thread takes four points of y from either neighbour
// and evaluates the stages on its own points plus a halo that shrinks by
// one point per stage (own +-3, +-2, +-1, own), in the LDS region after
// the exchange buffers (8 B .. 24 B values, two slots in turn); every value
// is computed as the stage-by-stage exchange computes it, so the result is
// the same bit for bit with one barrier per step instead of four.  Fewer
// points per thread exchange every stage.
template <int PT, int NB, typename R>
__device__ __forceinline__ void burgers_step(R (&y)[PT], R (&yc)[PT], R dt,
                                             R inv2h, R nuh2, R* lds, int& buf) {
    if constexpr (PT >= 8) {
        constexpr int H = 4, E = PT + 2 * H;  // extended index i <-> point i - H
        const int t = threadIdx.x, B = blockDim.x;
        R* e = lds + 8 * B + buf * 8 * B;
#pragma unroll
        for (int j = 0; j < H; ++j) {
            e[j * B + t] = y[j];
            e[(H + j) * B + t] = y[PT - H + j];
        }
        __syncthreads();
        const int tl = (t == 0) ? B - 1 : t - 1;
        const int tr = (t == B - 1) ? 0 : t + 1;
        R y0[E], Y[E], k[E], acc[PT];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            y0[j] = e[(H + j) * B + tl];
            y0[H + PT + j] = e[j * B + tr];
        }
#pragma unroll
        for (int q = 0; q < PT; ++q) y0[H + q] = y[q];
        buf ^= 1;
        // the right-hand side at extended indices [a, b) from Y
        auto rhs = [&](const R (&Z)[E], int a, int b) {
#pragma unroll
            for (int i = 0; i < E; ++i) {
                if (i < a || i >= b) continue;
                k[i] = -Z[i] * ((Z[i + 1] - Z[i - 1]) * inv2h) +
                       nuh2 * ((Z[i + 1] + Z[i - 1]) - (R)2 * Z[i]);
            }
        };
        rhs(y0, 1, E - 1);
#pragma unroll
        for (int i = 1; i < E - 1; ++i) {
            if (i >= H && i < H + PT) acc[i - H] = k[i];
            Y[i] = y0[i] + (R)0.5 * dt * k[i];
        }
        rhs(Y, 2, E - 2);
#pragma unroll
        for (int i = 2; i < E - 2; ++i) {
            if (i >= H && i < H + PT) acc[i - H] += (R)2 * k[i];
            Y[i] = y0[i] + (R)0.5 * dt * k[i];
        }
        rhs(Y, 3, E - 3);
#pragma unroll
        for (int i = 3; i < E - 3; ++i) {
            if (i >= H && i < H + PT) acc[i - H] += (R)2 * k[i];
            Y[i] = y0[i] + dt * k[i];
        }
        rhs(Y, H, H + PT);
#pragma unroll
        for (int q = 0; q < PT; ++q) kadd<R>(y[q], yc[q], (dt / (R)6) * (acc[q] + k[H + q]));
    } else {
        R acc[PT], Y[PT], k[PT], l[1], r[1];
        {
            const R* arr[1] = {y};
            exch<PT, 1, NB>(arr, lds, buf, l, r);
        }
        burgers_rhs<PT, R>(y, l[0], r[0], inv2h, nuh2, k);
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            acc[q] = k[q];
            Y[q] = y[q] + (R)0.5 * dt * k[q];
        }
        {
            const R* arr[1] = {Y};
            exch<PT, 1, NB>(arr, lds, buf, l, r);
        }
        burgers_rhs<PT, R>(Y, l[0], r[0], inv2h, nuh2, k);
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            acc[q] += (R)2 * k[q];
            Y[q] = y[q] + (R)0.5 * dt * k[q];
        }
        {
            const R* arr[1] = {Y};
            exch<PT, 1, NB>(arr, lds, buf, l, r);
        }
        burgers_rhs<PT, R>(Y, l[0], r[0], inv2h, nuh2, k);
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            acc[q] += (R)2 * k[q];
            Y[q] = y[q] + dt * k[q];
        }
        {
            const R* arr[1] = {Y};
            exch<PT, 1, NB>(arr, lds, buf, l, r);
        }
        burgers_rhs<PT, R>(Y, l[0], r[0], inv2h, nuh2, k);
#pragma unroll
        for (int q = 0; q < PT; ++q) kadd<R>(y[q], yc[q], (dt / (R)6) * (acc[q] + k[q]));
    }
}

// The march over steps [rg.s0, rg.s1) from y0 (the state at s0) to yT
// (in place allowed: every thread reads its own points before it writes
// them), checkpoints every c steps, and the integral-cost share of J where
// rg.tgt is set.
template <int PT, typename R>
__device__ __forceinline__ void dev_burgers_direct(const double* y0,
                                                   double* yT,
                                                   double* __restrict__ ckpt, int n,
                                                   int64_t n_t, int64_t c, double dt,
                                                   BurgersC bc, double* lds_d,
                                                   const BurgersRange& rg) {
    R* lds = reinterpret_cast<R*>(lds_d);
    const int base = threadIdx.x * PT;
    const R inv2h = (R)bc.inv2h, nuh2 = (R)bc.nuh2, rdt = (R)dt;
    R y[PT], yc[PT];
#pragma unroll
    for (int q = 0; q < PT; ++q) split_hilo<R>(y0[base + q], y[q], yc[q]);
    if (ckpt && rg.s0 == 0) {
#pragma unroll
        for (int q = 0; q < PT; ++q) ckpt[base + q] = hilo<R>(y[q], yc[q]);
    }
    // the share of J: sum w_s (q_s - tgt)^2, w_s = gw c_s / 2
    double js = 0.0, tg[PT];
    if (rg.tgt) {
#pragma unroll
        for (int q = 0; q < PT; ++q) tg[q] = rg.tgt[base + q];
    }
    auto emit = [&](int64_t st) {
        const double cs = rg.gw * ((st == 0 || st == n_t) ? 0.5 : 1.0);
        double e = 0.0;
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            const double d = hilo<R>(y[q], yc[q]) - tg[q];
            e += d * d;
        }
        js += 0.5 * cs * e;
    };
    int buf = 0;
    for (int64_t s = rg.s0; s < rg.s1; ++s) {
        if (rg.tgt) emit(s);
        burgers_step<PT, 1, R>(y, yc, rdt, inv2h, nuh2, lds, buf);
        if (ckpt && ((s + 1) % c) == 0) {
            double* o = ckpt + (size_t)((s + 1) / c) * n;
#pragma unroll
            for (int q = 0; q < PT; ++q) o[base + q] = hilo<R>(y[q], yc[q]);
        }
    }
    if (rg.tgt && rg.s1 == n_t) emit(n_t);
#pragma unroll
    for (int q = 0; q < PT; ++q) yT[base + q] = hilo<R>(y[q], yc[q]);
    if (rg.cpart) {
        // the march is done with the LDS exchange buffers (block_sum
        // begins with a barrier)
        const double t = block_sum(js, lds_d);
        if (threadIdx.x == 0) *rg.cpart = t;
    }
}

template <int PT, typename R>
__global__ void __launch_bounds__(max_block<PT>())
k_rk4_burgers_direct(const double* y0, double* yT,
                     double* __restrict__ ckpt, int n, int64_t n_t, int64_t c,
                     double dt, BurgersC bc, BurgersRange rg) {
    extern __shared__ double lds_d[];
    dev_burgers_direct<PT, R>(y0, yT, ckpt, n, n_t, c, dt, bc, lds_d, rg);
}

// (J(U)^T v)_i = ((U v)_{i+1} - (U v)_{i-1})/(2h) - (U_{i+1} - U_{i-1}) v_i/(2h)
//               + nu lap(v)_i
template <int PT, typename R>
__device__ __forceinline__ void burgers_jt(const R (&U)[PT], R Ul, R Ur,
                                           const R (&v)[PT], R inv2h, R nuh2,
                                           R* lds, int& buf, R (&out)[PT]) {
    R uv[PT];
#pragma unroll
    for (int q = 0; q < PT; ++q) uv[q] = U[q] * v[q];
    R l[2], r[2];
    {
        const R* arr[2] = {v, uv};
        exch<PT, 2>(arr, lds, buf, l, r);
    }
#pragma unroll
    for (int q = 0; q < PT; ++q) {
        const R vm = (q == 0) ? l[0] : v[q - 1];
        const R vp = (q == PT - 1) ? r[0] : v[q + 1];
        const R wm = (q == 0) ? l[1] : uv[q - 1];
        const R wp = (q == PT - 1) ? r[1] : uv[q + 1];
        const R Um = (q == 0) ? Ul : U[q - 1];
        const R Up = (q == PT - 1) ? Ur : U[q + 1];
        out[q] = (wp - wm) * inv2h - (Up - Um) * inv2h * v[q] + nuh2 * ((vp + vm) - (R)2 * v[q]);
    }
}

// The exact discrete adjoint over steps [rg.s0, rg.s1) (multiples of c)
// from lamT (nullable: zero) at s1, with the step sources where rg.tgt is
// set; lambda at s0 to lam0.
template <int PT, typename R>
__device__ __forceinline__ void dev_burgers_reverse(const double* __restrict__ ckpt,
                                                    const double* __restrict__ lamT,
                                                    double* __restrict__ lam0,
                                                    double* __restrict__ seg, int n,
                                                    int64_t n_t, int64_t c, double dt,
                                                    BurgersC bc, double* lds_d,
                                                    const BurgersRange& rg) {
    R* lds = reinterpret_cast<R*>(lds_d);
    const int base = threadIdx.x * PT;
    const R inv2h = (R)bc.inv2h, nuh2 = (R)bc.nuh2, rdt = (R)dt;
    R lam[PT], lamc[PT];
#pragma unroll
    for (int q = 0; q < PT; ++q) split_hilo<R>(lamT ? lamT[base + q] : 0.0, lam[q], lamc[q]);
    // step sources g_s = gw c_s (q_s - tgt) from the states at hand
    double tg[PT];
    if (rg.tgt) {
#pragma unroll
        for (int q = 0; q < PT; ++q) tg[q] = rg.tgt[base + q];
    }
    auto source = [&](const double* ys, int64_t st) {
        const double cs = rg.gw * ((st == 0 || st == n_t) ? 0.5 : 1.0);
#pragma unroll
        for (int q = 0; q < PT; ++q) kadd<R>(lam[q], lamc[q], (R)(cs * (ys[base + q] - tg[q])));
    };
    if (rg.tgt && rg.src_start) source(ckpt + (size_t)(rg.s1 / c) * n, rg.s1);
    int buf = 0;
    for (int64_t g = rg.s1 / c - 1; g >= rg.s0 / c; --g) {
        // recompute the segment's step states from its checkpoint (stored
        // exactly as FP64 values of the compensated pairs)
        R y[PT], yc[PT];
        const double* ck = ckpt + (size_t)g * n;
#pragma unroll
        for (int q = 0; q < PT; ++q) split_hilo<R>(ck[base + q], y[q], yc[q]);
        for (int64_t q2 = 0; q2 < c; ++q2) {
            double* o = seg + (size_t)q2 * n;
#pragma unroll
            for (int q = 0; q < PT; ++q) o[base + q] = hilo<R>(y[q], yc[q]);
            if (q2 + 1 < c) burgers_step<PT, 2, R>(y, yc, rdt, inv2h, nuh2, lds, buf);
        }
        // reverse over the segment
        for (int64_t q2 = c - 1; q2 >= 0; --q2) {
            const double* ys = seg + (size_t)q2 * n;
            R Y1[PT], Y2[PT], Y3[PT], Y4[PT], k[PT];
            R Ul[4], Ur[4], l[1], r[1];
#pragma unroll
            for (int q = 0; q < PT; ++q) Y1[q] = (R)ys[base + q];
            {
                const R* arr[1] = {Y1};
                exch<PT, 1, 2>(arr, lds, buf, l, r);
            }
            Ul[0] = l[0]; Ur[0] = r[0];
            burgers_rhs<PT, R>(Y1, l[0], r[0], inv2h, nuh2, k);
#pragma unroll
            for (int q = 0; q < PT; ++q) Y2[q] = Y1[q] + (R)0.5 * rdt * k[q];
            {
                const R* arr[1] = {Y2};
                exch<PT, 1, 2>(arr, lds, buf, l, r);
            }
            Ul[1] = l[0]; Ur[1] = r[0];
            burgers_rhs<PT, R>(Y2, l[0], r[0], inv2h, nuh2, k);
#pragma unroll
            for (int q = 0; q < PT; ++q) Y3[q] = Y1[q] + (R)0.5 * rdt * k[q];
            {
                const R* arr[1] = {Y3};
                exch<PT, 1, 2>(arr, lds, buf, l, r);
            }
            Ul[2] = l[0]; Ur[2] = r[0];
            burgers_rhs<PT, R>(Y3, l[0], r[0], inv2h, nuh2, k);
#pragma unroll
            for (int q = 0; q < PT; ++q) Y4[q] = Y1[q] + rdt * k[q];
            {
                const R* arr[1] = {Y4};
                exch<PT, 1, 2>(arr, lds, buf, l, r);
            }
            Ul[3] = l[0]; Ur[3] = r[0];
            // adjoint stages
            R kb[PT], Yb[PT], nl[PT];
#pragma unroll
            for (int q = 0; q < PT; ++q) kb[q] = (rdt / (R)6) * lam[q];
            burgers_jt<PT, R>(Y4, Ul[3], Ur[3], kb, inv2h, nuh2, lds, buf, Yb);
#pragma unroll
            for (int q = 0; q < PT; ++q) {
                nl[q] = Yb[q];
                kb[q] = (rdt / (R)3) * lam[q] + rdt * Yb[q];
            }
            burgers_jt<PT, R>(Y3, Ul[2], Ur[2], kb, inv2h, nuh2, lds, buf, Yb);
#pragma unroll
            for (int q = 0; q < PT; ++q) {
                nl[q] += Yb[q];
                kb[q] = (rdt / (R)3) * lam[q] + (R)0.5 * rdt * Yb[q];
            }
            burgers_jt<PT, R>(Y2, Ul[1], Ur[1], kb, inv2h, nuh2, lds, buf, Yb);
#pragma unroll
            for (int q = 0; q < PT; ++q) {
                nl[q] += Yb[q];
                kb[q] = (rdt / (R)6) * lam[q] + (R)0.5 * rdt * Yb[q];
            }
            burgers_jt<PT, R>(Y1, Ul[0], Ur[0], kb, inv2h, nuh2, lds, buf, Yb);
#pragma unroll
            for (int q = 0; q < PT; ++q) kadd<R>(lam[q], lamc[q], nl[q] + Yb[q]);
            if (rg.tgt) source(ys, g * c + q2);
        }
    }
#pragma unroll
    for (int q = 0; q < PT; ++q) lam0[base + q] = hilo<R>(lam[q], lamc[q]);
}

template <int PT, typename R>
__global__ void __launch_bounds__(max_block<PT>())
k_rk4_burgers_reverse(const double* __restrict__ ckpt,
                      const double* __restrict__ lamT, double* __restrict__ lam0,
                      double* __restrict__ seg, int n, int64_t n_t, int64_t c,
                      double dt, BurgersC bc, BurgersRange rg) {
    extern __shared__ double lds_d[];
    dev_burgers_reverse<PT, R>(ckpt, lamT, lam0, seg, n, n_t, c, dt, bc, lds_d, rg);
}

// Hybrid adjoint slices: workgroup b runs slice s_first + b from zero.
template <int PT, typename R>
__global__ void __launch_bounds__(max_block<PT>())
k_burgers_adj_slices(const double* __restrict__ ckpt, const double* __restrict__ tgt,
                     double gw, double* __restrict__ seg, double* __restrict__ mu,
                     const int64_t* __restrict__ bounds, int s_first, int n, int64_t n_t,
                     int64_t c, double dt, BurgersC bc) {
    extern __shared__ double lds_d[];
    const int sl = s_first + (int)blockIdx.x;
    BurgersRange rg{};
    rg.s0 = bounds[sl];
    rg.s1 = bounds[sl + 1];
    rg.tgt = tgt;
    rg.gw = gw;
    dev_burgers_reverse<PT, R>(ckpt, nullptr, mu + (size_t)sl * n,
                               seg + (size_t)sl * (size_t)c * n, n, n_t, c, dt, bc, lds_d, rg);
}

// Per-macro-step recompute for the time-varying adjoint (one workgroup per
// macro step q, all in parallel): march from the checkpoint preceding the
// step's Gauss nodes, interpolate U at the two nodes by cubic Hermite
// interpolation between step states (fourth order in dt), and store the
// effective states of the two commutator-free Magnus factors,
// W_first = 2(a2 U1 + a1 U2), W_second = 2(a1 U1 + a2 U2),
// so that each factor is exp((D/2) J(W)^T).  In tau = T - t the macro step q
// covers [qD, (q+1)D]; U1 = U(T - qD - c1 D), U2 = U(T - qD - c2 D).
template <int PT, typename R>
__device__ __forceinline__ void dev_burgers_nodes(const double* __restrict__ ckpt,
                                                  double* __restrict__ Wout, int n,
                                                  int64_t n_t, int64_t c, int64_t S,
                                                  double dt, BurgersC bc, int q, int qw,
                                                  double* lds_d) {
    R* lds = reinterpret_cast<R*>(lds_d);
    const int base = threadIdx.x * PT;
    const R inv2h = (R)bc.inv2h, nuh2 = (R)bc.nuh2, rdt = (R)dt;
    const double r3 = sqrt(3.0);
    const double c1 = 0.5 - r3 / 6.0, c2 = 0.5 + r3 / 6.0;
    const double a1 = 0.25 - r3 / 6.0, a2 = 0.25 + r3 / 6.0;
    // node times as step index + fraction; t1 > t2
    const double f1 = (double)(n_t - (int64_t)q * S) - c1 * (double)S;
    const double f2 = (double)(n_t - (int64_t)q * S) - c2 * (double)S;
    int64_t s1 = (int64_t)floor(f1), s2 = (int64_t)floor(f2);
    if (s1 > n_t - 1) s1 = n_t - 1;
    if (s2 > n_t - 1) s2 = n_t - 1;
    if (s2 < 0) s2 = 0;
    if (s1 < s2) s1 = s2;
    const double th1 = f1 - (double)s1, th2 = f2 - (double)s2;
    const int64_t start = (s2 / c) * c;
    R y[PT], yc[PT], y0[PT], k0[PT], k1[PT];
    double U1[PT], U2[PT];
    const double* ck = ckpt + (size_t)(start / c) * n;
#pragma unroll
    for (int i = 0; i < PT; ++i) split_hilo<R>(ck[base + i], y[i], yc[i]);
    int buf = 0;
    for (int64_t s = start; s < s2; ++s) burgers_step<PT, 1, R>(y, yc, rdt, inv2h, nuh2, lds, buf);
    auto hermite = [&](double th, double (&out)[PT]) {
        const double h00 = 2 * th * th * th - 3 * th * th + 1;
        const double h10 = th * th * th - 2 * th * th + th;
        const double h01 = -2 * th * th * th + 3 * th * th;
        const double h11 = th * th * th - th * th;
#pragma unroll
        for (int i = 0; i < PT; ++i)
            out[i] = h00 * (double)y0[i] + h10 * dt * (double)k0[i] +
                     h01 * hilo<R>(y[i], yc[i]) + h11 * dt * (double)k1[i];
    };
    auto rhs = [&](R (&out)[PT]) {
        R l[1], r[1];
        const R* arr[1] = {y};
        exch<PT, 1>(arr, lds, buf, l, r);
        burgers_rhs<PT, R>(y, l[0], r[0], inv2h, nuh2, out);
    };
    R y0c[PT];
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        y0[i] = y[i];
        y0c[i] = yc[i];
    }
    rhs(k0);
    burgers_step<PT, 1, R>(y, yc, rdt, inv2h, nuh2, lds, buf);  // y = state at s2 + 1
    rhs(k1);
#pragma unroll
    for (int i = 0; i < PT; ++i) y0[i] = (R)hilo<R>(y0[i], y0c[i]);
    hermite(th2, U2);
    if (s1 == s2) {
        hermite(th1, U1);
    } else {
        for (int64_t s = s2 + 1; s < s1; ++s) burgers_step<PT, 1, R>(y, yc, rdt, inv2h, nuh2, lds, buf);
#pragma unroll
        for (int i = 0; i < PT; ++i) y0[i] = (R)hilo<R>(y[i], yc[i]);
        rhs(k0);
        burgers_step<PT, 1, R>(y, yc, rdt, inv2h, nuh2, lds, buf);
        rhs(k1);
        hermite(th1, U1);
    }
    double* w1 = Wout + (size_t)(2 * qw) * n;
    double* w2 = Wout + (size_t)(2 * qw + 1) * n;
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        w1[base + i] = 2.0 * (a2 * U1[i] + a1 * U2[i]);
        w2[base + i] = 2.0 * (a1 * U1[i] + a2 * U2[i]);
    }
}

template <int PT, typename R>
__global__ void __launch_bounds__(max_block<PT>())
k_burgers_nodes(const double* __restrict__ ckpt, double* __restrict__ Wout, int n,
                int64_t n_t, int64_t c, int64_t S, double dt, BurgersC bc, int qbase) {
    extern __shared__ double lds_d[];
    // macro step qbase + b into output slot b
    dev_burgers_nodes<PT, R>(ckpt, Wout, n, n_t, c, S, dt, bc, qbase + (int)blockIdx.x,
                             (int)blockIdx.x, lds_d);
}

// ---- Burgers: the iterative nonlinear Paraexp (section 3.2) ----------------
// Burgers as y' = A y + N(y), A = nu lap (linear), N(y) = -y Dy.  Iterate
// i+1 on slice p solves the linear problem (eq. nonlinTrans)
//   y' = (A + J_p) y + N(O) - J_p O,   J_p = J(ubar_p) = -ubar_p D - diag(D ubar_p)
// (J is linear in the state, so the slice-averaged Jacobian of eq.
// Jacobians is the Jacobian at the slice-averaged state), where O are the
// previous iterate's RK4 stage states: at the fixed point every stage's
// source is N at that stage's own state, the nonlinear RK4 stage.  The
// right-hand side of a stage with state Y and previous stage state O:
//   F = nu lap Y - ubar (DY - DO) - (D ubar)(Y - O) - O DO.

// Stage states st[(s * 4 + k) * n], k = 0..3 (Y1 = the step state).
template <int PT>
__device__ __forceinline__ void nl_rhs(const double (&Y)[PT], const double (&O)[PT],
                                       double yl, double yr, double ol, double orr,
                                       const double (&ub)[PT], const double (&dub)[PT],
                                       double inv2h, double nuh2, double (&F)[PT]) {
#pragma unroll
    for (int q = 0; q < PT; ++q) {
        const double ym = (q == 0) ? yl : Y[q - 1], yp = (q == PT - 1) ? yr : Y[q + 1];
        const double om = (q == 0) ? ol : O[q - 1], op = (q == PT - 1) ? orr : O[q + 1];
        const double dy = (yp - ym) * inv2h, dO = (op - om) * inv2h;
        F[q] = nuh2 * ((yp + ym) - 2.0 * Y[q]) - ub[q] * (dy - dO) - dub[q] * (Y[q] - O[q]) -
               O[q] * dO;
    }
}

// Slice p (one workgroup) of iterate i+1: RK4 over steps [p S, (p+1) S)
// from q0 (p = 0, when q0 is set), E + (p-1) n (p > 0, the corrected
// start, when E is set) or zero, with the stage sources of the previous stages st_old; writes the
// new stage states (st_new, nullable), the end state reversed for the
// chain (vend + (P-1-p) n, nullable) and, for the last slice, q(T) (qT,
// nullable).
template <int PT>
__device__ __forceinline__ void dev_burgers_nl_march(
    const double* __restrict__ st_old, double* __restrict__ st_new, double* __restrict__ vend,
    const double* __restrict__ E, const double* __restrict__ q0, double* __restrict__ qT,
    const double* __restrict__ W, int n, int64_t S, int P, double dt, BurgersC bc,
    const NlState* __restrict__ ns, double* lds_d) {
    if (ns && ns->done) return;
    const int p = blockIdx.x;
    const int base = threadIdx.x * PT;
    double* lds = lds_d;
    int buf = 0;
    const double inv2h = bc.inv2h, nuh2 = bc.nuh2;
    // the slice's averaged state and its central difference
    double ub[PT], dub[PT];
    {
        const double* w = W + (size_t)p * n;
#pragma unroll
        for (int q = 0; q < PT; ++q) ub[q] = w[base + q];
        double l[1], r[1];
        const double* arr[1] = {ub};
        exch<PT, 1, 2>(arr, lds, buf, l, r);
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            const double um = (q == 0) ? l[0] : ub[q - 1], up = (q == PT - 1) ? r[0] : ub[q + 1];
            dub[q] = (up - um) * inv2h;
        }
    }
    double y[PT];
    const double* y0 = (p == 0) ? q0 : (E ? E + (size_t)(p - 1) * n : nullptr);
#pragma unroll
    for (int q = 0; q < PT; ++q) y[q] = y0 ? y0[base + q] : 0.0;
    const int64_t a = (int64_t)p * S;
    const double cf[4] = {0.0, 0.5, 0.5, 1.0};
    double Y[PT], F[PT], acc[PT];
    // stage k of step s from y with the previous iterate's stage state O
    auto stage = [&](int64_t s, int k, const double (&O)[PT]) {
        // stage state from the previous stage's slope
#pragma unroll
        for (int q = 0; q < PT; ++q) Y[q] = (k == 0) ? y[q] : y[q] + cf[k] * dt * F[q];
        if (st_new) {
            double* w = st_new + (size_t)(s * 4 + k) * n;
#pragma unroll
            for (int q = 0; q < PT; ++q) w[base + q] = Y[q];
        }
        double l[2], r[2];
        const double* arr[2] = {Y, O};
        exch<PT, 2, 2>(arr, lds, buf, l, r);
        nl_rhs<PT>(Y, O, l[0], r[0], l[1], r[1], ub, dub, inv2h, nuh2, F);
#pragma unroll
        for (int q = 0; q < PT; ++q) acc[q] = (k == 0) ? F[q] : acc[q] + ((k == 3) ? 1.0 : 2.0) * F[q];
    };
    auto finish = [&]() {
#pragma unroll
        for (int q = 0; q < PT; ++q) y[q] += (dt / 6.0) * acc[q];
    };
    auto load_step = [&](int64_t s, double (&O)[4][PT]) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double* o = st_old + (size_t)(s * 4 + k) * n + base;
#pragma unroll
            for (int q = 0; q < PT; ++q) O[k][q] = o[q];
        }
    };
    if constexpr (PT <= 8) {
        // the previous stage states are loaded one step ahead, issued after
        // the first stage's exchange: the workgroup barriers wait for LDS
        // only, so the loads of step s + 1 are in flight during stages 1-3
        double Oc[4][PT], On[4][PT];
        load_step(a, Oc);
        for (int64_t s = a; s < a + S; ++s) {
            stage(s, 0, Oc[0]);
            if (s + 1 < a + S) load_step(s + 1, On);
            stage(s, 1, Oc[1]);
            stage(s, 2, Oc[2]);
            stage(s, 3, Oc[3]);
            finish();
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int q = 0; q < PT; ++q) Oc[k][q] = On[k][q];
        }
    } else {
        // (more points per thread: two steps of stage states do not fit in
        // registers; each step's are loaded at its start)
        for (int64_t s = a; s < a + S; ++s) {
            double Oc[4][PT];
            load_step(s, Oc);
#pragma unroll
            for (int k = 0; k < 4; ++k) stage(s, k, Oc[k]);
            finish();
        }
    }
    if (vend) {
        double* v = vend + (size_t)(P - 1 - p) * n;
#pragma unroll
        for (int q = 0; q < PT; ++q) v[base + q] = y[q];
    }
    if (qT && p == P - 1) {
#pragma unroll
        for (int q = 0; q < PT; ++q) qT[base + q] = y[q];
    }
}

template <int PT, typename R>
__global__ void __launch_bounds__(max_block<PT>())
k_burgers_nl_march(const double* __restrict__ st_old, double* __restrict__ st_new,
                   double* __restrict__ vend, const double* __restrict__ E,
                   const double* __restrict__ q0, double* __restrict__ qT,
                   const double* __restrict__ W, int n, int64_t S, int P, double dt,
                   BurgersC bc, const NlState* __restrict__ ns) {
    extern __shared__ double lds_d[];
    dev_burgers_nl_march<PT>(st_old, st_new, vend, E, q0, qT, W, n, S, P, dt, bc, ns, lds_d);
}

// ubar_p = time average of the previous iterate over slice p by the
// trapezoidal rule on the step grid: the step states pS .. (p+1)S (stage 0
// of each step; the last slice ends on that iterate's q(T), qlast); grid
// (n / 256, P).
__global__ void k_nl_slice_mean(const double* __restrict__ st, const double* __restrict__ qlast,
                                double* __restrict__ W, int n, int64_t S, int P,
                                const NlState* __restrict__ ns) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = blockIdx.y;
    if (i >= n || ns->done) return;
    const int64_t s0 = (int64_t)p * S, s1 = s0 + S;
    double a = 0.5 * st[(size_t)(s0 * 4) * n + i];
    for (int64_t s = s0 + 1; s < s1; ++s) a += st[(size_t)(s * 4) * n + i];
    a += 0.5 * ((p == P - 1) ? qlast[i] : st[(size_t)(s1 * 4) * n + i]);
    W[(size_t)p * n + i] = a / (double)S;
}

// The first guess: every stage state of every step equals q0; the change
// check's previous q(T) is q0; the iteration state is reset.
__global__ void k_nl_fill(const double* __restrict__ q0, double* __restrict__ st,
                          double* __restrict__ qprev, NlState* __restrict__ ns, int n,
                          int64_t nst) {
    const size_t tot = (size_t)nst * n;
    const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = i0; k < tot; k += stride) st[k] = q0[k % n];
    for (size_t k = i0; k < (size_t)n; k += stride) qprev[k] = q0[k];
    if (i0 == 0) {
        ns->done = 0;
        ns->last = 0;
        ns->change = INFINITY;
    }
}

// One workgroup: the relative change of q(T) in the iteration that wrote
// stage-state generation gen; within tol it stops the iteration.  Every
// thread reads done before the reduction's barrier, thread 0 writes it
// after; qprev takes the new q(T) for the next iteration's change.
__global__ void __launch_bounds__(256) k_nl_change(const double* __restrict__ qT,
                                                   double* __restrict__ qprev, int n,
                                                   double tol, NlState* __restrict__ ns,
                                                   int gen, InstStat* irep) {
    __shared__ double red[80];
    if (ns->done) return;
    double dd = 0.0, qq = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double e = qT[i] - qprev[i];
        dd += e * e;
        qq += qT[i] * qT[i];
    }
    int slot = 0;
    block_sum2(dd, qq, red, slot);
    for (int i = threadIdx.x; i < n; i += blockDim.x) qprev[i] = qT[i];
    if (threadIdx.x == 0) {
        double c = qq > 0.0 ? sqrt(dd / qq) : (dd > 0.0 ? INFINITY : 0.0);
        if (!isfinite(c)) c = INFINITY;
        ns->change = c;
        ns->last = gen;
        ns->done = (c <= tol) ? 1 : 0;
        if (irep) atomicAdd(&irep->nl_iters, 1ull);
    }
}

__global__ void k_nl_final(const NlState* __restrict__ ns, double tol, DevStatus* st,
                           InstStat* irep) {
    if (threadIdx.x != 0) return;
    const double est = ns->change;
    const bool bad = !isfinite(est);
    const unsigned long long eb = (unsigned long long)__double_as_longlong(bad ? INFINITY : est);
    if (st) {
        atomicMax(&st->max_est, eb);
        if (bad) atomicOr(&st->flags, ST_NONFINITE);
        else if (est > tol) atomicOr(&st->flags, ST_NOCONV);
    }
    if (irep) atomicMax(&irep->max_est, eb);
}

// Checkpoints of the final iterate: the step states every c steps, and q(T).
__global__ void k_nl_ckpt(const double* __restrict__ st0, const double* __restrict__ st1,
                          const NlState* __restrict__ ns, const double* __restrict__ qT,
                          double* __restrict__ ckpt, int n, int64_t n_t, int64_t c) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t j = blockIdx.y;
    if (i >= n) return;
    const double* st = ns->last ? st1 : st0;
    const int64_t s = j * c;
    ckpt[(size_t)j * n + i] = (s == n_t) ? qT[i] : st[(size_t)(s * 4) * n + i];
}

// ---- ragged batches: one launch over all instances -------------------------
// Every workgroup reads its instance from the descriptor table and runs the
// march for that instance's points per thread (256 threads per workgroup,
// n = 256 * pt).

#define PXP_BATCH_SWITCH(FN, R, ...)                                           \
    switch (d.pt) {                                                            \
        case 1: FN<1, R>(__VA_ARGS__); break;                                  \
        case 2: FN<2, R>(__VA_ARGS__); break;                                  \
        case 4: FN<4, R>(__VA_ARGS__); break;                                  \
        case 8: FN<8, R>(__VA_ARGS__); break;                                  \
        case 16: FN<16, R>(__VA_ARGS__); break;                                \
        case 32: FN<32, R>(__VA_ARGS__); break;                                \
        default: break;                                                        \
    }

template <typename R>
__global__ void __launch_bounds__(256) k_burgers_direct_batch(const BurgersDesc* tab) {
    extern __shared__ double lds_d[];
    const BurgersDesc d = tab[blockIdx.x];
    const BurgersC bc{d.inv2h, d.nuh2};
    const BurgersRange rg{0, d.n_t, nullptr, 0.0, nullptr, 0, 0};
    PXP_BATCH_SWITCH(dev_burgers_direct, R, d.y0, d.yT, d.ckpt, d.n, d.n_t, d.c, d.dt,
                     bc, lds_d, rg)
}

template <typename R>
__global__ void __launch_bounds__(256) k_burgers_reverse_batch(const BurgersDesc* tab) {
    extern __shared__ double lds_d[];
    const BurgersDesc d = tab[blockIdx.x];
    const BurgersC bc{d.inv2h, d.nuh2};
    const BurgersRange rg{0, d.n_t, nullptr, 0.0, nullptr, 0, 0};
    PXP_BATCH_SWITCH(dev_burgers_reverse, R, d.ckpt, d.lamT, d.lam0, d.seg, d.n, d.n_t,
                     d.c, d.dt, bc, lds_d, rg)
}

// The serial reverse sweep at 512 threads per instance (every instance of
// the launch has pt_rev points per thread, pt_rev * 512 = n).
#define PXP_BATCH_SWITCH_REV(FN, R, ...)                                       \
    switch (d.pt_rev) {                                                        \
        case 2: FN<2, R>(__VA_ARGS__); break;                                  \
        case 4: FN<4, R>(__VA_ARGS__); break;                                  \
        case 8: FN<8, R>(__VA_ARGS__); break;                                  \
        case 16: FN<16, R>(__VA_ARGS__); break;                                \
        default: break;                                                        \
    }

template <typename R>
__global__ void __launch_bounds__(512) k_burgers_reverse_batch512(const BurgersDesc* tab) {
    extern __shared__ double lds_d[];
    const BurgersDesc d = tab[blockIdx.x];
    const BurgersC bc{d.inv2h, d.nuh2};
    const BurgersRange rg{0, d.n_t, nullptr, 0.0, nullptr, 0, 0};
    PXP_BATCH_SWITCH_REV(dev_burgers_reverse, R, d.ckpt, d.lamT, d.lam0, d.seg, d.n, d.n_t,
                         d.c, d.dt, bc, lds_d, rg)
}

// grid = sum of the instances' macro-step counts; the instance of a
// workgroup is found by a scan of the table's prefix counts
template <typename R>
__global__ void __launch_bounds__(256) k_burgers_nodes_batch(const BurgersDesc* tab,
                                                             int count) {
    extern __shared__ double lds_d[];
    int i = 0;
    while (i + 1 < count && (int)blockIdx.x >= tab[i + 1].q0) ++i;
    const BurgersDesc d = tab[i];
    const BurgersC bc{d.inv2h, d.nuh2};
    const int q = (int)blockIdx.x - d.q0;
    PXP_BATCH_SWITCH(dev_burgers_nodes, R, d.ckpt, d.nodes, d.n, d.n_t, d.c, d.S, d.dt,
                     bc, d.qbase + q, q, lds_d)
}

// Threads per workgroup and points per thread for an n-point march: by
// default 256 threads (one wave per SIMD, full register budget) with n/256
// points each; small grids use fewer threads.
int max_block_rt(int pt) { return pt <= 4 ? 1024 : (pt <= 16 ? 512 : 256); }

bool valid_pt(int p) { return p == 1 || p == 2 || p == 4 || p == 8 || p == 16 || p == 32; }

bool pick_shape(int n, int block_hint, int* block, int* pt) {
    if (n < 2) return false;
    if (block_hint > 0) {
        if (n % block_hint) return false;
        const int p = n / block_hint;
        if (!valid_pt(p) || block_hint > max_block_rt(p)) return false;
        *block = block_hint;
        *pt = p;
        return true;
    }
    if (n % 256 == 0 && valid_pt(n / 256) && n / 256 <= 16) {
        *block = 256;
        *pt = n / 256;
        return true;
    }
    static const int cands[] = {64, 128, 512, 1024};
    for (int b : cands) {
        if (n % b == 0 && valid_pt(n / b) && b <= max_block_rt(n / b)) {
            *block = b;
            *pt = n / b;
            return true;
        }
    }
    if (n <= 1024) {
        *block = n;
        *pt = 1;
        return true;
    }
    return false;
}

// One-workgroup marches (the serial comparison method) wait on a barrier per
// RK4 stage.  Measured: at N = 4096 the linear forward march plus reverse
// sweep took 105 ms with 512 threads of 8 points against 124 ms with 256 of
// 16, and at N = 2048 the Burgers reverse sweep ran 9% faster with 512 of 4.
// The Paraexp slice batch (many workgroups) keeps the 256-thread default.
int serial_block_hint(int n, int block_hint) {
    if (block_hint > 0) return block_hint;
    return (n == 4 * 512 || n == 8 * 512) ? 512 : 0;
}

}  // namespace

#define PXP_DISPATCH_PT(pt, KERNEL, R, ...)                                    \
    switch (pt) {                                                              \
        case 1: KERNEL<1, R> __VA_ARGS__; break;                               \
        case 2: KERNEL<2, R> __VA_ARGS__; break;                               \
        case 4: KERNEL<4, R> __VA_ARGS__; break;                               \
        case 8: KERNEL<8, R> __VA_ARGS__; break;                               \
        case 16: KERNEL<16, R> __VA_ARGS__; break;                             \
        case 32: KERNEL<32, R> __VA_ARGS__; break;                             \
        default: return hipErrorInvalidValue;                                  \
    }
#define PXP_DISPATCH(fp32, pt, KERNEL, ...)                                    \
    if (fp32) {                                                                \
        PXP_DISPATCH_PT(pt, KERNEL, float, __VA_ARGS__)                        \
    } else {                                                                   \
        PXP_DISPATCH_PT(pt, KERNEL, double, __VA_ARGS__)                       \
    }

bool march_shape(int n, int block_hint, int* block, int* pt) {
    return pick_shape(n, block_hint, block, pt);
}

hipError_t launch_rk4_lin1d(const double* F, const double* g0, const double* y0,
                            double* out, int n, int P, int64_t n_s, double dt,
                            double omega, Tri A, int block_hint, int fp32,
                            hipStream_t s, SliceIntegral si) {
    int block, pt;
    if (!pick_shape(n, P == 1 ? serial_block_hint(n, block_hint) : block_hint, &block, &pt))
        return hipErrorInvalidValue;
    const size_t lds = sizeof(double) * (4 * block + SINE_LDS_DOUBLES);
    const TriSplit sp = split(A);
    if (si.iout) {
        PXP_DISPATCH(fp32, pt, k_rk4_lin1d_int,
                     <<<P, block, lds, s>>>(F, g0, y0, out, n, n_s, dt, omega, sp, si))
    } else if (sp.cc == 0.0 && !g0) {
        PXP_DISPATCH(fp32, pt, k_rk4_lin1d_nocc_nog,
                     <<<P, block, lds, s>>>(F, g0, y0, out, n, n_s, dt, omega, sp, si))
    } else if (sp.cc == 0.0) {
        PXP_DISPATCH(fp32, pt, k_rk4_lin1d_nocc,
                     <<<P, block, lds, s>>>(F, g0, y0, out, n, n_s, dt, omega, sp, si))
    } else {
        PXP_DISPATCH(fp32, pt, k_rk4_lin1d_plain,
                     <<<P, block, lds, s>>>(F, g0, y0, out, n, n_s, dt, omega, sp, si))
    }
    return hipGetLastError();
}

hipError_t launch_rk4_rev_lin1d(const double* lamT, double* lam0,
                                double* Lambda, int n, int64_t n_t, double dt,
                                double omega, Tri AT, int block_hint, int fp32,
                                hipStream_t s) {
    int block, pt;
    if (!pick_shape(n, serial_block_hint(n, block_hint), &block, &pt))
        return hipErrorInvalidValue;
    const size_t lds = sizeof(double) * (4 * block + SINE_LDS_DOUBLES);
    const TriSplit sp = split(AT);
    if (sp.cc == 0.0) {
        PXP_DISPATCH(fp32, pt, k_rk4_rev_lin1d_nocc,
                     <<<1, block, lds, s>>>(lamT, lam0, Lambda, n, n_t, dt, omega, sp))
    } else {
        PXP_DISPATCH(fp32, pt, k_rk4_rev_lin1d,
                     <<<1, block, lds, s>>>(lamT, lam0, Lambda, n, n_t, dt, omega, sp))
    }
    return hipGetLastError();
}

hipError_t launch_rk4_burgers_direct(const double* y0, double* yT, double* ckpt,
                                     int n, int64_t n_t, int64_t c, double dt,
                                     double nu, double L, int block_hint, int fp32,
                                     hipStream_t s, const BurgersRange* rgp) {
    int block, pt;
    if (!pick_shape(n, block_hint, &block, &pt)) return hipErrorInvalidValue;
    const double h = L / n;
    BurgersC bc{1.0 / (2.0 * h), nu / (h * h)};
    const size_t lds = sizeof(double) * (pt >= 8 ? 24 : 4) * block;
    BurgersRange rg{0, n_t, nullptr, 0.0, nullptr, 0, 0};
    if (rgp) rg = *rgp;
    if (rg.s0 < 0 || rg.s1 > n_t || rg.s0 >= rg.s1) return hipErrorInvalidValue;
    PXP_DISPATCH(fp32, pt, k_rk4_burgers_direct,
                 <<<1, block, lds, s>>>(y0, yT, ckpt, n, n_t, c, dt, bc, rg))
    return hipGetLastError();
}

hipError_t launch_burgers_nodes(const double* ckpt, double* W, int n, int64_t n_t,
                                int64_t c, int64_t S, double dt, double nu, double L,
                                int block_hint, int fp32, hipStream_t s, int qbase,
                                int count) {
    int block, pt;
    if (!pick_shape(n, block_hint, &block, &pt)) return hipErrorInvalidValue;
    if (S <= 0 || n_t % S) return hipErrorInvalidValue;
    const double h = L / n;
    BurgersC bc{1.0 / (2.0 * h), nu / (h * h)};
    const size_t lds = sizeof(double) * (pt >= 8 ? 24 : 4) * block;
    const int Q = (int)(n_t / S);
    if (count < 0) count = Q - qbase;
    if (qbase < 0 || count <= 0 || qbase + count > Q) return hipErrorInvalidValue;
    PXP_DISPATCH(fp32, pt, k_burgers_nodes,
                 <<<count, block, lds, s>>>(ckpt, W, n, n_t, c, S, dt, bc, qbase))
    return hipGetLastError();
}

hipError_t launch_rk4_burgers_reverse(const double* ckpt, const double* lamT,
                                      double* lam0, double* seg, int n,
                                      int64_t n_t, int64_t c, double dt,
                                      double nu, double L, int block_hint, int fp32,
                                      hipStream_t s, const BurgersRange* rgp) {
    int block, pt;
    if (!pick_shape(n, serial_block_hint(n, block_hint), &block, &pt))
        return hipErrorInvalidValue;
    const double h = L / n;
    BurgersC bc{1.0 / (2.0 * h), nu / (h * h)};
    const size_t lds = sizeof(double) * (pt >= 8 ? 24 : 8) * block;
    BurgersRange rg{0, n_t, nullptr, 0.0, nullptr, 0, 0};
    if (rgp) rg = *rgp;
    if (rg.s0 < 0 || rg.s1 > n_t || rg.s0 >= rg.s1 || rg.s0 % c || rg.s1 % c)
        return hipErrorInvalidValue;
    PXP_DISPATCH(fp32, pt, k_rk4_burgers_reverse,
                 <<<1, block, lds, s>>>(ckpt, lamT, lam0, seg, n, n_t, c, dt, bc, rg))
    return hipGetLastError();
}

hipError_t launch_burgers_nl_march(const double* st_old, double* st_new, double* vend,
                                   const double* E, const double* q0, double* qT,
                                   const double* W, int n, int64_t S, int P, double dt,
                                   double nu, double L, int block_hint, const NlState* ns,
                                   hipStream_t s) {
    int block, pt;
    if (!pick_shape(n, block_hint, &block, &pt)) return hipErrorInvalidValue;
    const double h = L / n;
    BurgersC bc{1.0 / (2.0 * h), nu / (h * h)};
    const size_t lds = sizeof(double) * 8 * block;
    PXP_DISPATCH_PT(pt, k_burgers_nl_march, double,
                    <<<P, block, lds, s>>>(st_old, st_new, vend, E, q0, qT, W, n, S, P, dt, bc,
                                           ns))
    return hipGetLastError();
}

hipError_t launch_nl_slice_mean(const double* st, const double* qlast, double* W, int n,
                                int64_t S, int P, const NlState* ns, hipStream_t s) {
    dim3 g((unsigned)((n + 255) / 256), (unsigned)P);
    k_nl_slice_mean<<<g, 256, 0, s>>>(st, qlast, W, n, S, P, ns);
    return hipGetLastError();
}

hipError_t launch_nl_fill(const double* q0, double* st, double* qprev, NlState* ns, int n,
                          int64_t nst, hipStream_t s) {
    k_nl_fill<<<1024, 256, 0, s>>>(q0, st, qprev, ns, n, nst);
    return hipGetLastError();
}

hipError_t launch_nl_change(const double* qT, double* qprev, int n, double tol, NlState* ns,
                            int gen, InstStat* irep, hipStream_t s) {
    k_nl_change<<<1, 256, 0, s>>>(qT, qprev, n, tol, ns, gen, irep);
    return hipGetLastError();
}

hipError_t launch_nl_final(const NlState* ns, double tol, DevStatus* st, InstStat* irep,
                           hipStream_t s) {
    k_nl_final<<<1, 64, 0, s>>>(ns, tol, st, irep);
    return hipGetLastError();
}

hipError_t launch_nl_ckpt(const double* st0, const double* st1, const NlState* ns,
                          const double* qT, double* ckpt, int n, int64_t n_t, int64_t c,
                          hipStream_t s) {
    dim3 g((unsigned)((n + 255) / 256), (unsigned)(n_t / c + 1));
    k_nl_ckpt<<<g, 256, 0, s>>>(st0, st1, ns, qT, ckpt, n, n_t, c);
    return hipGetLastError();
}

hipError_t launch_burgers_adj_slices(const double* ckpt, const double* tgt, double gw,
                                     double* seg, double* mu, const int64_t* bounds,
                                     int s_first, int count, int n, int64_t n_t, int64_t c,
                                     double dt, double nu, double L, int block_hint,
                                     hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int block, pt;
    if (!pick_shape(n, serial_block_hint(n, block_hint), &block, &pt))
        return hipErrorInvalidValue;
    const double h = L / n;
    BurgersC bc{1.0 / (2.0 * h), nu / (h * h)};
    const size_t lds = sizeof(double) * (pt >= 8 ? 24 : 8) * block;
    PXP_DISPATCH_PT(pt, k_burgers_adj_slices, double,
                    <<<count, block, lds, s>>>(ckpt, tgt, gw, seg, mu, bounds, s_first, n,
                                               n_t, c, dt, bc))
    return hipGetLastError();
}

hipError_t launch_burgers_batch(int which, const BurgersDesc* tab, int count,
                                int total_blocks, int fp32, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * 24 * 256;
    const int grid = (which == 2) ? total_blocks : count;
    if (which == 0) {
        if (fp32) k_burgers_direct_batch<float><<<grid, 256, lds, s>>>(tab);
        else k_burgers_direct_batch<double><<<grid, 256, lds, s>>>(tab);
    } else if (which == 1) {
        if (fp32) k_burgers_reverse_batch<float><<<grid, 256, lds, s>>>(tab);
        else k_burgers_reverse_batch<double><<<grid, 256, lds, s>>>(tab);
    } else if (which == 3) {
        const size_t lds512 = sizeof(double) * 24 * 512;
        if (fp32) k_burgers_reverse_batch512<float><<<grid, 512, lds512, s>>>(tab);
        else k_burgers_reverse_batch512<double><<<grid, 512, lds512, s>>>(tab);
    } else {
        if (fp32) k_burgers_nodes_batch<float><<<grid, 256, lds, s>>>(tab, count);
        else k_burgers_nodes_batch<double><<<grid, 256, lds, s>>>(tab, count);
    }
    return hipGetLastError();
}

}  // namespace pxp
