// RK4 marches of the 2D periodic advection-diffusion problem (paper section
// 4.2) with the first-order upwind, five-point operator:
//   - the P inhomogeneous slices from zero data (eq. linInhomEqus), all
//     instances and slices of a call in one launch;
//   - the serial comparison march and its exact discrete adjoint.
//
// Workgroup layout: one workgroup advances a band of grid rows of one march
// by up to BAND_MAX_STEPS steps.  Rows are periodic in x, so the band only
// needs a halo in y: every stage application of the stencil consumes one
// halo row on each side, so a band of nsteps steps loads 4*nsteps extra rows
// above and below, recomputes them redundantly, and writes back only its own
// rows.  State, stage input and stage accumulator live in registers.
#include "pxp_internal.hpp"
#include "pxp_device.hpp"
#include "pxp_band.hpp"

namespace pxp {
namespace {

// Band layout (shared with the uniformised exponentials): 8 waves, wave w
// holds region rows 8w .. 8w+7 of a 64-row region, lane l columns
// l*CPL .. l*CPL+CPL-1 (CPL = NX/64), so a wave row is a whole periodic grid
// row: x neighbours are the adjacent lanes (wrapping), y neighbours the same
// lane's registers except at the wave's first and last rows, which go
// through LDS once per stage.  Output rows are region rows off .. off+R-1
// (R = d.rows, 16 or 32; off = (64 - R) / 2); every stage application
// consumes one halo row on each side, and at most 16 are needed (four steps
// of four stages).  Waves whose rows are no longer needed skip the
// arithmetic.  The forcing pattern of the needed rows is staged in LDS once
// per launch (it enters every stage); the four stages are unrolled, each
// with its own update, and the forcing sines of the launch are evaluated by
// one lane each and broadcast.
// One classical RK4 step of y' = A y + s(t) F with constant A is, exactly
// (up to rounding), the polynomial step
//   y_{n+1} = R(Z) y_n + phi(Z) F,   Z = dt A,
//   R(Z) = 1 + Z + Z^2/2 + Z^3/6 + Z^4/24,
//   phi(Z) = dt/6 [s1 (1 + Z + Z^2/2 + Z^3/4) + s2 (4 + 2Z + Z^2/2) + s4],
// s1, s2, s4 the forcing modulation at t_n, t_n + dt/2, t_n + dt: expand the
// four stages with y = 0 and with F = 0.  The marches evaluate it by Horner
// in Z (four stencil applications per step, as the stages), keeping two
// arrays in registers instead of three; the forcing pattern comes from LDS.
// Its exact discrete adjoint is lambda_n = R(Z^T) lambda_{n+1} with the
// forcing gradient phi(Z^T) lambda_{n+1}, formed from the powers
// (Z^T)^j lambda_{n+1}, j <= 4.

// One Horner level of the forward step: v = rj y + fj F + Z v, with
// (rj, fj) = (1/6, f3), (1/2, f2), (1, f1), (1, f0) for the levels in turn.
template <int NX, int CPL, bool FORCED>
__device__ __forceinline__ void fwd_level(const double (&y)[BRW][CPL], double (&v)[BRW][CPL],
                                          const double (*fl)[NX], double (*xch)[2][NX],
                                          const Sten5& A, double rj, double fj, double dt,
                                          int w, int l, int cb, bool active) {
    double prev[CPL], dn[CPL];
    exchange_edges<NX, CPL>(xch, v, w, cb, prev, dn);
    if (!active) return;
#pragma unroll
    for (int i = 0; i < BRW; ++i) {
        double cur[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) cur[c] = v[i][c];
        const double wv = from_west(cur[CPL - 1]);
        const double ev = from_east(cur[0]);
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const double xw = (c > 0) ? cur[c - 1] : wv;
            const double xe = (c < CPL - 1) ? cur[c + 1] : ev;
            const double xn = (i < BRW - 1) ? v[i + 1][c] : dn[c];
            const double av = A.c * cur[c] + A.w * xw + A.e * xe + A.s * prev[c] + A.n * xn;
            double r = rj * y[i][c] + dt * av;
            if (FORCED) r += fj * fl[w * BRW + i][cb + c];
            v[i][c] = r;
            prev[c] = cur[c];
        }
        // one row at a time: the scheduler would otherwise hoist later rows'
        // LDS reads and shuffles and push the register use past 256
        __builtin_amdgcn_sched_barrier(0);
    }
}

// rows of the wave still needed after stencil application `app` of H
__device__ __forceinline__ bool wave_active(int w, int off, int R, int H, int app) {
    const int keep = H - 1 - app;
    return !(w * BRW + BRW <= off - keep || w * BRW >= off + R + keep);
}

// Step s of a launch of ns steps (H = 4 ns stencil applications).
template <int NX, bool FORCED>
__device__ __forceinline__ void fwd_step(double (&y)[BRW][NX / WAVE], const Sten5& A, double dt,
                                         const double (*fl)[NX], double (*xch)[2][NX], int s,
                                         int H, double snv, int w, int l, int cb, int off, int R) {
    constexpr int CPL = NX / WAVE;
    const double h6 = dt / 6.0;
    // modulation at t_n, t_n + dt/2, t_n + dt (lanes 3s .. 3s+2)
    const double s1 = __shfl(snv, 3 * s, WAVE), s2 = __shfl(snv, 3 * s + 1, WAVE),
                 s4 = __shfl(snv, 3 * s + 2, WAVE);
    const double f0 = h6 * (s1 + 4.0 * s2 + s4), f1 = h6 * (s1 + 2.0 * s2),
                 f2 = h6 * 0.5 * (s1 + s2), f3 = h6 * 0.25 * s1;
    double v[BRW][CPL];
#pragma unroll
    for (int i = 0; i < BRW; ++i)
#pragma unroll
        for (int c = 0; c < CPL; ++c) v[i][c] = y[i][c] * (1.0 / 24.0);
#pragma unroll 1
    for (int j = 0; j < 4; ++j) {
        const double rj = (j == 0) ? 1.0 / 6.0 : ((j == 1) ? 0.5 : 1.0);
        const double fj = (j == 0) ? f3 : ((j == 1) ? f2 : ((j == 2) ? f1 : f0));
        fwd_level<NX, CPL, FORCED>(y, v, fl, xch, A, rj, fj, dt, w, l, cb,
                                   wave_active(w, off, R, H, 4 * s + j));
    }
#pragma unroll
    for (int i = 0; i < BRW; ++i)
#pragma unroll
        for (int c = 0; c < CPL; ++c) y[i][c] = v[i][c];
}

template <int NX, bool FORCED>
__device__ __forceinline__ void fwd_march(double (&y)[BRW][NX / WAVE], const Band2D& d,
                                          const double (*fl)[NX], double (*xch)[2][NX], int ns,
                                          double snv, int w, int l, int cb, int off, int R) {
    const Sten5 A = d.A;
    for (int s = 0; s < ns; ++s)
        fwd_step<NX, FORCED>(y, A, d.dt, fl, xch, s, 4 * ns, snv, w, l, cb, off, R);
}

template <int NX>
__global__ void __launch_bounds__(BNT)
k_band2d_fwd(const Band2D* __restrict__ tab, int count, int serial, int L) {
    constexpr int CPL = NX / WAVE;
    __shared__ double xch[BW][2][NX];
    __shared__ double fl[BROWS][NX];
    const Band2D& d = tab[find_entry(tab, count, blockIdx.x)];
    const int ny = d.ny, R = d.rows, nb = ny / R, off = (BROWS - R) / 2;
    const int local = blockIdx.x - d.blk0;
    const int item = local / nb, band = local - item * nb;
    int ns;
    int64_t first;
    const double* in;
    double* out;
    const size_t nn = (size_t)NX * ny;
    if (serial) {
        const int64_t left = d.n_t - 4 * (int64_t)L;
        if (left <= 0) return;
        ns = left < 4 ? (int)left : 4;
        first = 4 * (int64_t)L;
        in = (L == 0) ? d.y0 : d.buf[L & 1];
        out = d.buf[(L + 1) & 1];
    } else {
        if (item >= d.items) return;
        ns = d.nsteps;
        first = d.step0 + (int64_t)item * d.item_steps;
        // the initial state belongs to the first slice, the others start
        // from zero (eq. linInhomEqus)
        in = (item == 0) ? d.y0 : nullptr;
        out = d.out + (size_t)item * nn;
    }
    const int H = 4 * ns;
    const int w = wave_id(), l = lane_id(), cb = l * CPL;
    const int base = band * R - off + w * BRW;
    const double dt = d.dt;
    // lane j < 3 ns: the forcing modulation at stage time j of the launch
    double snv = 0.0;
    if (l < 3 * ns) {
        const int st = l / 3, v = l - 3 * (l / 3);
        const double tn = (double)(first + st) * dt;
        snv = sin(d.omega * (tn + (v == 0 ? 0.0 : (v == 2 ? dt : 0.5 * dt))));
    }
    // every region row is a grid row, so all loads are in bounds and issued
    // together; rows beyond the halo the launch needs never reach the output
    int g[BRW];
    wave_rows(band_grow(base, 0, ny), ny, g);
    double y[BRW][CPL];
    if (in) {
#pragma unroll
        for (int i = 0; i < BRW; ++i) row_load<CPL>(in + (size_t)g[i] * NX + cb, y[i]);
    } else {
#pragma unroll
        for (int i = 0; i < BRW; ++i)
#pragma unroll
            for (int c = 0; c < CPL; ++c) y[i][c] = 0.0;
    }
    if (d.F) {
        double f[BRW][CPL];
#pragma unroll
        for (int i = 0; i < BRW; ++i) row_load<CPL>(d.F + (size_t)g[i] * NX + cb, f[i]);
#pragma unroll
        for (int i = 0; i < BRW; ++i) row_store<CPL>(&fl[w * BRW + i][cb], f[i]);
        fwd_march<NX, true>(y, d, fl, xch, ns, snv, w, l, cb, off, R);
    } else {
        fwd_march<NX, false>(y, d, fl, xch, ns, snv, w, l, cb, off, R);
    }
    (void)H;
#pragma unroll
    for (int i = 0; i < BRW; ++i) {
        const int r = w * BRW + i;
        if (r >= off && r < off + R) row_store<CPL>(out + (size_t)g[i] * NX + cb, y[i]);
    }
}

// One power of the reverse step: w <- Z^T w, lam_n += rj w and (output
// rows) Lambda += fj w, with (rj, fj) = (1, f1), (1/2, f2), (1/6, f3),
// (1/24, 0) for the powers 1..4.
template <int NX, int CPL, bool TRACK>
__device__ __forceinline__ void rev_power(double (&w_)[BRW][CPL], double (&ln)[BRW][CPL],
                                          double (*lm)[NX], double (*xch)[2][NX],
                                          const Sten5& A, double rj, double fj, double dt,
                                          int w, int l, int cb, int off, int R, bool active) {
    double prev[CPL], dn[CPL];
    exchange_edges<NX, CPL>(xch, w_, w, cb, prev, dn);
    if (!active) return;
#pragma unroll
    for (int i = 0; i < BRW; ++i) {
        const int r = w * BRW + i;
        double cur[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) cur[c] = w_[i][c];
        const double wv = from_west(cur[CPL - 1]);
        const double ev = from_east(cur[0]);
        const bool orow = TRACK && r >= off && r < off + R;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const double xw = (c > 0) ? cur[c - 1] : wv;
            const double xe = (c < CPL - 1) ? cur[c + 1] : ev;
            const double xn = (i < BRW - 1) ? w_[i + 1][c] : dn[c];
            const double z =
                dt * (A.c * cur[c] + A.w * xw + A.e * xe + A.s * prev[c] + A.n * xn);
            ln[i][c] += rj * z;
            if (orow) lm[r - off][cb + c] += fj * z;
            w_[i][c] = z;
            prev[c] = cur[c];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// One reverse step (step s of the launch, a = stencil applications done so
// far of H): lam_n = R(Z^T) lam_{n+1}, Lambda += phi(Z^T) lam_{n+1}.  The
// Lambda increments build in LDS for the output rows.
template <int NX, bool TRACK>
__device__ __forceinline__ void rev_step(double (&lam)[BRW][NX / WAVE], const Sten5& A,
                                         double dt, double (*lm)[NX], double (*xch)[2][NX],
                                         int s, int a, int H, double snv, int w, int l, int cb,
                                         int off, int R) {
    constexpr int CPL = NX / WAVE;
    const double h6 = dt / 6.0;
    const double s1 = __shfl(snv, 3 * s, WAVE), s2 = __shfl(snv, 3 * s + 1, WAVE),
                 s4 = __shfl(snv, 3 * s + 2, WAVE);
    const double f0 = h6 * (s1 + 4.0 * s2 + s4), f1 = h6 * (s1 + 2.0 * s2),
                 f2 = h6 * 0.5 * (s1 + s2), f3 = h6 * 0.25 * s1;
    double ln[BRW][CPL];
    // power 0: lam_n starts as lam_{n+1}, Lambda takes f0 lam_{n+1}
#pragma unroll
    for (int i = 0; i < BRW; ++i) {
        const int r = w * BRW + i;
        const bool orow = TRACK && r >= off && r < off + R;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            ln[i][c] = lam[i][c];
            if (orow) lm[r - off][cb + c] += f0 * lam[i][c];
        }
    }
#pragma unroll 1
    for (int j = 1; j <= 4; ++j) {
        const double rj = (j == 1) ? 1.0 : ((j == 2) ? 0.5 : ((j == 3) ? 1.0 / 6.0 : 1.0 / 24.0));
        const double fj = (j == 1) ? f1 : ((j == 2) ? f2 : ((j == 3) ? f3 : 0.0));
        rev_power<NX, CPL, TRACK>(lam, ln, lm, xch, A, rj, fj, dt, w, l, cb, off, R,
                                  wave_active(w, off, R, H, a + j - 1));
    }
#pragma unroll
    for (int i = 0; i < BRW; ++i)
#pragma unroll
        for (int c = 0; c < CPL; ++c) lam[i][c] = ln[i][c];
}

// Exact discrete adjoint of the RK4 march, backwards over the steps of the
// launch.
template <int NX, bool TRACK>
__device__ __forceinline__ void rev_march(double (&lam)[BRW][NX / WAVE], const Band2D& d,
                                          double (*lm)[NX], double (*xch)[2][NX], int ns,
                                          double snv, int w, int l, int cb, int off, int R) {
    const Sten5 A = d.A;
    int a = 0;
    for (int s = ns - 1; s >= 0; --s, a += 4)
        rev_step<NX, TRACK>(lam, A, d.dt, lm, xch, s, a, 4 * ns, snv, w, l, cb, off, R);
}

template <int NX>
__global__ void __launch_bounds__(BNT)
k_band2d_rev(const Band2D* __restrict__ tab, int count, int L) {
    constexpr int CPL = NX / WAVE;
    __shared__ double xch[BW][2][NX];
    __shared__ double lm[32][NX];
    const Band2D& d = tab[find_entry(tab, count, blockIdx.x)];
    const int ny = d.ny, R = d.rows, off = (BROWS - R) / 2;
    const int band = blockIdx.x - d.blk0;
    const int64_t left = d.n_t - 4 * (int64_t)L;
    if (left <= 0) return;
    const int ns = left < 4 ? (int)left : 4;
    const int64_t first = left - ns;
    const double* in = (L == 0) ? d.y0 : d.buf[L & 1];
    double* out = d.buf[(L + 1) & 1];
    const int H = 4 * ns;
    const int t = threadIdx.x, w = wave_id(), l = lane_id(), cb = l * CPL;
    const int base = band * R - off + w * BRW;
    const double dt = d.dt;
    double snv = 0.0;
    if (l < 3 * ns) {
        const int st = l / 3, v = l - 3 * (l / 3);
        const double tn = (double)(first + st) * dt;
        snv = sin(d.omega * (tn + (v == 0 ? 0.0 : (v == 2 ? dt : 0.5 * dt))));
    }
    const bool track = d.Lam != nullptr;
    if (track)
        for (int q = t; q < R * NX; q += BNT) lm[q / NX][q % NX] = 0.0;
    int g[BRW];
    wave_rows(band_grow(base, 0, ny), ny, g);
    double lam[BRW][CPL];
#pragma unroll
    for (int i = 0; i < BRW; ++i) row_load<CPL>(in + (size_t)g[i] * NX + cb, lam[i]);
    (void)H;
    __syncthreads();  // the Lambda buffer is cleared
    if (track)
        rev_march<NX, true>(lam, d, lm, xch, ns, snv, w, l, cb, off, R);
    else
        rev_march<NX, false>(lam, d, lm, xch, ns, snv, w, l, cb, off, R);
#pragma unroll
    for (int i = 0; i < BRW; ++i) {
        const int r = w * BRW + i;
        if (r < off || r >= off + R) continue;
        const size_t o = (size_t)g[i] * NX + cb;
        row_store<CPL>(out + o, lam[i]);
        if (track) {
            double L[CPL], m[CPL];
            row_load<CPL>(d.Lam + o, L);
            row_load<CPL>(&lm[r - off][cb], m);
#pragma unroll
            for (int c = 0; c < CPL; ++c) L[c] += m[c];
            row_store<CPL>(d.Lam + o, L);
        }
    }
}

// ---- integral cost (section 4.2, eq. cost) ----------------------------------
// J = 1/T int_0^T |q - tgt|^2 dt by the trapezoidal rule over the RK4 step
// states: J = sum_n w_n |q_n - tgt|^2, w_n = dt c_n / T, c_n = 1/2 at n = 0
// and n = n_t, 1 between.  Every step state is then an argument of J, and
// the discrete adjoint takes dJ/dq_n = 2 w_n (q_n - tgt) after each reverse
// step (the step form of the adjoint source of eq. adjEquation).

__device__ __forceinline__ double trap_c(int64_t n, int64_t n_t) {
    return (n == 0 || n == n_t) ? 0.5 : 1.0;
}

// g_n = gw c_n (q_n - tgt) on the output rows (gw = 2 dt / T); the lane's
// share of w_n |q_n - tgt|^2 is added to js.
template <int NX>
__device__ __forceinline__ void emit_src(const double (&y)[BRW][NX / WAVE], const Band2D& d,
                                         int64_t n, const int (&gr)[BRW], int w, int cb,
                                         int off, int R, double& js) {
    constexpr int CPL = NX / WAVE;
    const double c = d.gw * trap_c(n, d.n_t);
    double* gn = d.g + (size_t)n * ((size_t)NX * d.ny);
#pragma unroll
    for (int i = 0; i < BRW; ++i) {
        const int r = w * BRW + i;
        if (r < off || r >= off + R) continue;
        const size_t o = (size_t)gr[i] * NX + cb;
        double t[CPL], e[CPL];
        row_load<CPL>(d.tgt + o, t);
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            const double dq = y[i][k] - t[k];
            e[k] = c * dq;
            s += dq * dq;
        }
        row_store<CPL>(gn + o, e);
        js += 0.5 * c * s;
    }
}

template <int NX, bool FORCED>
__device__ __forceinline__ void src_march(double (&y)[BRW][NX / WAVE], const Band2D& d,
                                          const double (*fl)[NX], double (*xch)[2][NX],
                                          int64_t first, int ns, bool last, double snv,
                                          const int (&gr)[BRW], int w, int l, int cb, int off,
                                          int R, double& js) {
    const Sten5 A = d.A;
    emit_src<NX>(y, d, first, gr, w, cb, off, R, js);
    for (int s = 0; s < ns; ++s) {
        fwd_step<NX, FORCED>(y, A, d.dt, fl, xch, s, 4 * ns, snv, w, l, cb, off, R);
        if (s + 1 < ns || last) emit_src<NX>(y, d, first + s + 1, gr, w, cb, off, R, js);
    }
}

// Forward source march: the states of every step of a slice (from its
// corrected start state) or of a serial launch, their sources and the cost.
template <int NX>
__global__ void __launch_bounds__(BNT)
k_band2d_src(const Band2D* __restrict__ tab, int count, int serial, int L) {
    constexpr int CPL = NX / WAVE;
    __shared__ double xch[BW][2][NX];
    __shared__ double fl[BROWS][NX];
    const Band2D& d = tab[find_entry(tab, count, blockIdx.x)];
    const int ny = d.ny, R = d.rows, nb = ny / R, off = (BROWS - R) / 2;
    const int local = blockIdx.x - d.blk0;
    const int item = local / nb, band = local - item * nb;
    const size_t nn = (size_t)NX * ny;
    int ns;
    int64_t first;
    const double* in;
    double* out = nullptr;
    bool last;
    if (serial) {
        const int64_t left = d.n_t - 4 * (int64_t)L;
        if (left <= 0) return;
        ns = left < 4 ? (int)left : 4;
        first = 4 * (int64_t)L;
        in = (L == 0) ? d.y0 : d.buf[L & 1];
        out = d.buf[(L + 1) & 1];
        last = first + ns == d.n_t;
    } else {
        if (item >= d.items) return;
        ns = d.nsteps;
        first = d.step0 + (int64_t)item * d.item_steps;
        in = (item == 0) ? d.y0 : d.ys + (size_t)(item - 1) * nn;
        last = item == d.items - 1;
    }
    const int w = wave_id(), l = lane_id(), cb = l * CPL;
    const double dt = d.dt;
    double snv = 0.0;
    if (l < 3 * ns) {
        const int st = l / 3, v = l - 3 * (l / 3);
        const double tn = (double)(first + st) * dt;
        snv = sin(d.omega * (tn + (v == 0 ? 0.0 : (v == 2 ? dt : 0.5 * dt))));
    }
    int gr[BRW];
    wave_rows(band_grow(band * R - off + w * BRW, 0, ny), ny, gr);
    double y[BRW][CPL];
    if (in) {
#pragma unroll
        for (int i = 0; i < BRW; ++i) row_load<CPL>(in + (size_t)gr[i] * NX + cb, y[i]);
    } else {
#pragma unroll
        for (int i = 0; i < BRW; ++i)
#pragma unroll
            for (int c = 0; c < CPL; ++c) y[i][c] = 0.0;
    }
    double js = 0.0;
    if (d.F) {
        double f[BRW][CPL];
#pragma unroll
        for (int i = 0; i < BRW; ++i) row_load<CPL>(d.F + (size_t)gr[i] * NX + cb, f[i]);
#pragma unroll
        for (int i = 0; i < BRW; ++i) row_store<CPL>(&fl[w * BRW + i][cb], f[i]);
        src_march<NX, true>(y, d, fl, xch, first, ns, last, snv, gr, w, l, cb, off, R, js);
    } else {
        src_march<NX, false>(y, d, fl, xch, first, ns, last, snv, gr, w, l, cb, off, R, js);
    }
    if (out) {
#pragma unroll
        for (int i = 0; i < BRW; ++i) {
            const int r = w * BRW + i;
            if (r >= off && r < off + R) row_store<CPL>(out + (size_t)gr[i] * NX + cb, y[i]);
        }
    }
    // the workgroup's cost partial, summed in wave order (deterministic);
    // a serial march adds its launches into one slot per band
    js = wave_sum(js);
    double* red = &xch[0][0][0];
    __syncthreads();
    if (l == 0) red[w] = js;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < BW; ++q) t += red[q];
        double* slot = d.cpart + (serial ? (size_t)band : (size_t)item * nb + band);
        *slot = (serial && L > 0) ? *slot + t : t;
    }
}

// lam += g_n on the rows that `keep` more stencil applications still read
template <int NX>
__device__ __forceinline__ void add_src(double (&lam)[BRW][NX / WAVE], const double* gn,
                                        const int (&gr)[BRW], int w, int cb, int off, int R,
                                        int keep) {
    constexpr int CPL = NX / WAVE;
#pragma unroll
    for (int i = 0; i < BRW; ++i) {
        const int r = w * BRW + i;
        if (r < off - keep || r >= off + R + keep) continue;
        double q[CPL];
        row_load<CPL>(gn + (size_t)gr[i] * NX + cb, q);
#pragma unroll
        for (int c = 0; c < CPL; ++c) lam[i][c] += q[c];
    }
}

template <int NX, bool TRACK>
__device__ __forceinline__ void rsrc_march(double (&lam)[BRW][NX / WAVE], const Band2D& d,
                                           double (*lm)[NX], double (*xch)[2][NX],
                                           int64_t first, int ns, double snv,
                                           const int (&gr)[BRW], int w, int l, int cb, int off,
                                           int R) {
    const Sten5 A = d.A;
    const size_t nn = (size_t)NX * d.ny;
    int a = 0;
    for (int s = ns - 1; s >= 0; --s, a += 4) {
        rev_step<NX, TRACK>(lam, A, d.dt, lm, xch, s, a, 4 * ns, snv, w, l, cb, off, R);
        add_src<NX>(lam, d.g + (size_t)(first + s) * nn, gr, w, cb, off, R, 4 * s);
    }
}

// Reverse source march: the discrete adjoint with the step sources, over
// each slice from zero (the last slice from y0 + g_{n_t}), or a serial
// launch.
template <int NX>
__global__ void __launch_bounds__(BNT)
k_band2d_rsrc(const Band2D* __restrict__ tab, int count, int serial, int L) {
    constexpr int CPL = NX / WAVE;
    __shared__ double xch[BW][2][NX];
    __shared__ double lm[32][NX];
    const Band2D& d = tab[find_entry(tab, count, blockIdx.x)];
    const int ny = d.ny, R = d.rows, nb = ny / R, off = (BROWS - R) / 2;
    const int local = blockIdx.x - d.blk0;
    const int item = local / nb, band = local - item * nb;
    const size_t nn = (size_t)NX * ny;
    int ns;
    int64_t first;
    const double* in;
    double *out, *Lo;
    bool start;
    if (serial) {
        const int64_t left = d.n_t - 4 * (int64_t)L;
        if (left <= 0) return;
        ns = left < 4 ? (int)left : 4;
        first = left - ns;
        in = (L == 0) ? d.y0 : d.buf[L & 1];
        out = d.buf[(L + 1) & 1];
        Lo = d.Lam;
        start = L == 0;
    } else {
        if (item >= d.items) return;
        ns = d.nsteps;
        first = d.step0 + (int64_t)item * d.item_steps;
        start = item == d.items - 1;
        in = start ? d.y0 : nullptr;
        out = d.out + (size_t)item * nn;
        Lo = d.Lam ? d.Lam + (size_t)item * nn : nullptr;
    }
    const int H = 4 * ns;
    const int t = threadIdx.x, w = wave_id(), l = lane_id(), cb = l * CPL;
    const double dt = d.dt;
    double snv = 0.0;
    if (l < 3 * ns) {
        const int st = l / 3, v = l - 3 * (l / 3);
        const double tn = (double)(first + st) * dt;
        snv = sin(d.omega * (tn + (v == 0 ? 0.0 : (v == 2 ? dt : 0.5 * dt))));
    }
    const bool track = Lo != nullptr;
    if (track)
        for (int q = t; q < R * NX; q += BNT) lm[q / NX][q % NX] = 0.0;
    int gr[BRW];
    wave_rows(band_grow(band * R - off + w * BRW, 0, ny), ny, gr);
    double lam[BRW][CPL];
    if (in) {
#pragma unroll
        for (int i = 0; i < BRW; ++i) row_load<CPL>(in + (size_t)gr[i] * NX + cb, lam[i]);
    } else {
#pragma unroll
        for (int i = 0; i < BRW; ++i)
#pragma unroll
            for (int c = 0; c < CPL; ++c) lam[i][c] = 0.0;
    }
    // the final state takes the last step state's source
    if (start) add_src<NX>(lam, d.g + (size_t)d.n_t * nn, gr, w, cb, off, R, H);
    __syncthreads();  // the Lambda buffer is cleared
    if (track)
        rsrc_march<NX, true>(lam, d, lm, xch, first, ns, snv, gr, w, l, cb, off, R);
    else
        rsrc_march<NX, false>(lam, d, lm, xch, first, ns, snv, gr, w, l, cb, off, R);
#pragma unroll
    for (int i = 0; i < BRW; ++i) {
        const int r = w * BRW + i;
        if (r < off || r >= off + R) continue;
        const size_t o = (size_t)gr[i] * NX + cb;
        row_store<CPL>(out + o, lam[i]);
        if (track) {
            double Lv[CPL], m[CPL];
            row_load<CPL>(&lm[r - off][cb], m);
            if (serial) {
                row_load<CPL>(Lo + o, Lv);
#pragma unroll
                for (int c = 0; c < CPL; ++c) Lv[c] += m[c];
                row_store<CPL>(Lo + o, Lv);
            } else {
                row_store<CPL>(Lo + o, m);
            }
        }
    }
}

__global__ void k_apply5(const double* __restrict__ x, double* __restrict__ out, int nx,
                         int ny, Sten5 A) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nx * ny) return;
    const int r = i / nx, c = i - r * nx;
    const int base = r * nx;
    const double xw = x[base + (c == 0 ? nx - 1 : c - 1)];
    const double xe = x[base + (c == nx - 1 ? 0 : c + 1)];
    const double xs = x[(r == 0 ? ny - 1 : r - 1) * nx + c];
    const double xn = x[(r == ny - 1 ? 0 : r + 1) * nx + c];
    out[i] = A.c * x[i] + A.w * xw + A.e * xe + A.s * xs + A.n * xn;
}

template <int NX>
hipError_t band_fwd(const Band2D* tab, int count, int total_blocks, int serial, int L,
                    hipStream_t s) {
    k_band2d_fwd<NX><<<total_blocks, BNT, 0, s>>>(tab, count, serial, L);
    return hipGetLastError();
}

template <int NX>
hipError_t band_rev(const Band2D* tab, int count, int total_blocks, int L,
                    hipStream_t s) {
    k_band2d_rev<NX><<<total_blocks, BNT, 0, s>>>(tab, count, L);
    return hipGetLastError();
}

template <int NX>
hipError_t band_src(const Band2D* tab, int count, int total_blocks, int serial, int L,
                    int rev, hipStream_t s) {
    if (rev)
        k_band2d_rsrc<NX><<<total_blocks, BNT, 0, s>>>(tab, count, serial, L);
    else
        k_band2d_src<NX><<<total_blocks, BNT, 0, s>>>(tab, count, serial, L);
    return hipGetLastError();
}

}  // namespace

// Every entry of one launch has the same row length nx.
hipError_t launch_band2d(const Band2D* tab, int count, int total_blocks, int nx,
                         int serial, int L, hipStream_t s) {
    if (count <= 0 || total_blocks <= 0) return hipSuccess;
    switch (nx) {
        case 64: return band_fwd<64>(tab, count, total_blocks, serial, L, s);
        case 128: return band_fwd<128>(tab, count, total_blocks, serial, L, s);
        case 256: return band_fwd<256>(tab, count, total_blocks, serial, L, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_band2d_rev(const Band2D* tab, int count, int total_blocks, int nx,
                             int L, hipStream_t s) {
    if (count <= 0 || total_blocks <= 0) return hipSuccess;
    switch (nx) {
        case 64: return band_rev<64>(tab, count, total_blocks, L, s);
        case 128: return band_rev<128>(tab, count, total_blocks, L, s);
        case 256: return band_rev<256>(tab, count, total_blocks, L, s);
        default: return hipErrorInvalidValue;
    }
}

static hipError_t launch_src(const Band2D* tab, int count, int total_blocks, int nx,
                             int serial, int L, int rev, hipStream_t s) {
    if (count <= 0 || total_blocks <= 0) return hipSuccess;
    switch (nx) {
        case 64: return band_src<64>(tab, count, total_blocks, serial, L, rev, s);
        case 128: return band_src<128>(tab, count, total_blocks, serial, L, rev, s);
        case 256: return band_src<256>(tab, count, total_blocks, serial, L, rev, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_band2d_src(const Band2D* tab, int count, int total_blocks, int nx,
                             int serial, int L, hipStream_t s) {
    return launch_src(tab, count, total_blocks, nx, serial, L, 0, s);
}

hipError_t launch_band2d_rsrc(const Band2D* tab, int count, int total_blocks, int nx,
                              int serial, int L, hipStream_t s) {
    return launch_src(tab, count, total_blocks, nx, serial, L, 1, s);
}

hipError_t launch_apply5(const double* x, double* out, int nx, int ny, Sten5 op,
                         hipStream_t s) {
    const int n = nx * ny;
    if (n <= 0) return hipSuccess;
    k_apply5<<<(n + 255) / 256, 256, 0, s>>>(x, out, nx, ny, op);
    return hipGetLastError();
}

}  // namespace pxp
