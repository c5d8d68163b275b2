// Action of the matrix exponential on the homogeneous pieces (paper section
// 4.1): Arnoldi projection onto the Krylov space, exponential of the small
// Hessenberg matrix, exp(tau A) v ~ beta V_m exp(tau H_m) e_1.
//
// One workgroup owns one piece.  Thread t owns the strided points
// i = t + r*B (r < PT), so every read of a basis vector is coalesced and each
// thread only ever reads back basis entries it wrote itself.  The basis lives
// in HBM (streamed through L2/MALL); the Hessenberg matrix and all small dense
// work live in LDS.
//
// Two Krylov flavours:
//  - polynomial: K_m(A, v); the time is cut into substeps accepted by the
//    a-posteriori estimate beta h_{m+1,m} |e_m^T exp(ts H_m) e_1|; a rejected
//    substep only re-evaluates the small exponential;
//  - shift-and-invert: K_m((I - gamma A)^{-1}, v), gamma = gamma_frac * tau,
//    with A ~ (I - H_m^{-1}) / gamma on the space; the periodic tridiagonal
//    solve is parallel cyclic reduction in LDS (uniform coefficients, n a
//    power of two) or chunk elimination plus cyclic reduction of the chunk
//    interfaces (the Burgers Jacobian).  From about m/2 on, checks compare
//    the approximation with the previous check's and extrapolate the
//    error from the observed contraction; the process stops once that is
//    below the tolerance, and the next check is placed where the
//    contraction predicts convergence.
//
// Optional time integral of the piece against sin(a + b s):
//   int_0^tau sin(a + b s) exp(s A) v ds ~ beta V_m Im(e^{ia} x),
//   (Hop + i b I) x = e^{i b tau} exp(tau Hop) e_1 - e_1,
// one real 2m x 2m solve in LDS after the exponential (Hop = H_m or the
// shift-and-invert image).
#include "pxp_internal.hpp"
#include "pxp_device.hpp"

namespace pxp {
namespace {

constexpr int M_MAX_1D = 48;

// Table of the uniform shift-and-invert solve (Ctx::ui_setup), in doubles:
// Thomas pivots piv_l and ratios cp_l of a chunk's interior block, the
// interior's responses g_l, h_l to the chunk's first point and to the next
// chunk's first point (l < 32 each), the cyclic-reduction multipliers of
// the chunk-interface system (two per level, at most 16 levels), then the
// final 2 x 2 elimination and the row coefficients.
constexpr int UT_PIV = 0, UT_CP = 32, UT_G = 64, UT_H = 96, UT_LVL = 128, UT_FIN = 160;
constexpr int UT_DOUBLES = 168;
// Chebyshev flavour: most series coefficients kept in LDS
constexpr int CHEB_KMAX = 320;

// Gram-Schmidt: the second classical pass runs when the first removed all
// but a fraction eta of the vector's norm, |w_1| < eta |w_0| (Daniel, Gragg,
// Kaufman & Stewart's criterion), with eta = 0.1: the exponential's
// approximation tolerates the orthogonality lost at milder cancellation.
constexpr double DGKS_ETA2 = 0.01;  // eta^2

// Basis vectors per batch of the Gram-Schmidt sweeps: a batch holds at most
// 32 doubles per thread in flight (sixteen 16-byte loads), so threads with
// many points take fewer vectors at a time and stay within their registers.
template <int PT>
constexpr int sweep_batch(int cap) {
    return (32 / PT) < 1 ? 1 : ((32 / PT) > cap ? cap : (32 / PT));
}

__host__ __device__ inline size_t big_doubles(int n, int m, int block) {
    size_t vec = 2 * (size_t)n;
    // variable-coefficient solve: padded chunks (n + B) and 8 B for the
    // interface reduction
    if ((size_t)n + 9 * (size_t)block > vec) vec = (size_t)n + 9 * (size_t)block;
    const size_t part = (size_t)(m + 1) * ((block + 63) / 64);
    const size_t sm = 6 * (size_t)m * m + 5 * (size_t)m + 8;
    size_t b = vec > sm ? vec : sm;
    return b > part ? b : part;
}

// Largest workgroup a kernel instance with PT points per thread is compiled
// for: the register budget per thread halves each time the wave count per
// SIMD doubles.
__host__ __device__ constexpr int krylov_max_block(int pt) {
    return pt <= 8 ? 512 : 256;
}

struct Smem {
    double* red;   // 128: block reductions (block_sum, block_sum2)
    double* hcol;  // ldr + 8
    double* H;     // (m+1) x m, ld = m
    double* yprev; // m: the previous shift-and-invert check's approximation
    double* ut;    // UT_DOUBLES: factors of the uniform shift-and-invert solve
    double* big;   // vector buffers (2n) or small matrices
    // small-matrix region (inside big)
    double* Mt;    // m x m
    double* E;     // m x m
    double* W;     // 4 m^2 + 2 m + 8
    double* vy;    // m
    double* vy2;   // m
    double* vc;    // m
};

struct Tsplit {
    double cs, cdf, cc;
};

// Shared part of the Krylov contexts: LDS layout, the small dense phase
// (Hessenberg exponential, shift-and-invert image, time integral), status
// reporting and the substep control of exp(tau Op) v.  D supplies the vector
// side: arnoldi(), combine() and before_space().
template <class D, bool SI>
struct Core {
    const KrylovArgs a;
    Smem S;
    int n, m, B, t, ldr;
    unsigned nre = 0;  // second Gram-Schmidt passes since the last report
    // Shift-and-invert early exit, state of the current Arnoldi process:
    // dimension of the last check (0: none yet), the difference of that
    // check's approximation to the one before it (negative: none) and the
    // gap in dimensions between those two checks.
    int si_kc = 0, si_gp = 0;
    double si_dp = -1.0;
    // Error of an approximation: the extrapolated difference to the previous
    // check (si_extrapolate), or, with si_plain, the difference itself.
    bool si_plain = false;

    __device__ Core(const KrylovArgs& a_, double* lds)
        : a(a_), n(a_.n), m(a_.m), B(blockDim.x), t(threadIdx.x) {
        ldr = ((m + 1 + 7) / 8) * 8;
        S.red = lds;
        S.hcol = S.red + 128;
        S.H = S.hcol + ldr + 8;
        S.yprev = S.H + (size_t)(m + 1) * m;
        S.ut = S.yprev + ldr;
        S.big = S.ut + UT_DOUBLES;
        S.Mt = S.big;
        S.E = S.Mt + (size_t)m * m;
        S.W = S.E + (size_t)m * m;
        S.vy = S.W + 4 * (size_t)m * m + 2 * m + 8;
        S.vy2 = S.vy + m;
        S.vc = S.vy2 + m;
    }
    __device__ __forceinline__ D& self() { return *static_cast<D*>(this); }

    // Mt = scale * (I - H_k^{-1}) / gamma for the leading k x k block.
    __device__ __forceinline__ void si_image(int k, double gamma, double scale) {
        double* X = S.W;
        double* U = X + (size_t)k * k;
        double* piv = U + (size_t)k * k;
        sm_hess_inverse(S.H, m, k, U, piv, X);
        const double f = scale / gamma;
        for_rc(k, k, [&](int r, int c) {
            S.Mt[r * k + c] = f * (((r == c) ? 1.0 : 0.0) - X[r * k + c]);
        });
        __syncthreads();
    }

    // |vy - yprev| over the first k coefficients (yprev holds the
    // approximation of the last check, dimension si_kc, zero-extended).
    __device__ __forceinline__ double si_diff(int k) const {
        double d2 = 0.0;
        for (int q = 0; q < k; ++q) {
            const double d = S.vy[q] - (q < si_kc ? S.yprev[q] : 0.0);
            d2 += d * d;
        }
        return sqrt(d2);
    }

    // Error of the dimension-k approximation.  d = |y_k - y_kc| (gap
    // g = k - kc) measures the error of the older y_kc; with the previous
    // difference dp over gap gp the per-dimension contraction is
    // (d/dp)^(1/gp), and geometric convergence carries d over the g
    // dimensions to k.  Without a previous difference d itself is returned
    // (an over-estimate).
    __device__ __forceinline__ static double si_extrapolate(double d, double dp, int g, int gp) {
        if (!(dp > 0.0) || gp <= 0) return d;
        const double r = fmin(1.0, d / dp);
        return d * pow(r, (double)g / (double)gp);
    }

    // vec = exp(ts Hop) e_1 (leading k x k block); returns |vec[k-1]|.
    __device__ __forceinline__ double small_exp(int k, double ts, double gamma, double* vec) {
        if (SI) {
            si_image(k, gamma, ts);
        } else {
            for_rc(k, k, [&](int r, int c) { S.Mt[r * k + c] = ts * S.H[r * m + c]; });
            __syncthreads();
        }
        sm_expm(S.E, S.Mt, k, k, S.W, S.red);
        for (int r = t; r < k; r += B) vec[r] = S.E[r * k];
        __syncthreads();
        return fabs(vec[k - 1]);
    }

    // vc = coefficients of int_0^ts sin(ia + ib s) exp(s Hop) e_1 ds, given
    // vy = exp(ts Hop) e_1: Im(e^{i ia} x) with
    //   (Hop + i ib I) x = e^{i ib ts} vy - e_1.
    // Polynomial: Hop = H_k is upper Hessenberg.  Shift-and-invert:
    // Hop = (I - H_k^{-1}) / gamma; multiplying by gamma H_k gives the
    // Hessenberg system ((1 + i ib gamma) H_k - I) x = gamma H_k (rhs).
    __device__ __forceinline__ void small_integral(int k, double ts, double ia, double ib,
                                                   double gamma) {
        double* Mr = S.W;
        double* Mi = Mr + (size_t)k * k;
        double* xr = Mi + (size_t)k * k;
        double* xi = xr + k;
        double* dr = xi + k;
        double* di = dr + k;
        const double cb = cos(ib * ts), sb = sin(ib * ts);
        for_rc(k, k, [&](int r, int c) {
            const double h = S.H[r * m + c];
            if (SI) {
                Mr[r * k + c] = h - ((r == c) ? 1.0 : 0.0);
                Mi[r * k + c] = ib * gamma * h;
            } else {
                Mr[r * k + c] = h;
                Mi[r * k + c] = (r == c) ? ib : 0.0;
            }
        });
        for (int r = t; r < k; r += B) {
            if (SI) {
                double sr = 0.0, si = 0.0;
                for (int c = (r > 0 ? r - 1 : 0); c < k; ++c) {
                    const double h = S.H[r * m + c];
                    sr += h * (cb * S.vy[c] - ((c == 0) ? 1.0 : 0.0));
                    si += h * (sb * S.vy[c]);
                }
                xr[r] = gamma * sr;
                xi[r] = gamma * si;
            } else {
                xr[r] = cb * S.vy[r] - ((r == 0) ? 1.0 : 0.0);
                xi[r] = sb * S.vy[r];
            }
        }
        __syncthreads();
        sm_hess_solve_c(Mr, Mi, xr, xi, dr, di, k);
        const double sa = sin(ia), ca = cos(ia);
        for (int r = t; r < k; r += B) S.vc[r] = sa * xr[r] + ca * xi[r];
        __syncthreads();
    }

    // A NaN or infinite norm of a start vector ends the exponential early
    // (nothing to propagate); it is recorded here so the caller learns of it.
    __device__ __forceinline__ void flag_nonfinite(double x) {
        if (t == 0 && a.status && !isfinite(x)) atomicOr(&a.status->flags, ST_NONFINITE);
    }

    __device__ __forceinline__ void report(double est_rel, bool noconv, unsigned substeps,
                           unsigned iters) {
        if (t == 0 && a.status) {
            if (noconv) atomicOr(&a.status->flags, ST_NOCONV);
            if (!(est_rel == est_rel)) atomicOr(&a.status->flags, ST_NONFINITE);
            const double e = fabs(est_rel);
            if (e == e)
                atomicMax(&a.status->max_est, (unsigned long long)__double_as_longlong(e));
            // the forward time-varying chain (the nonlinear direct) counts
            // with the direct class
            const int cls =
                (a.adj || a.mode == KM_SINGLE || (a.mode == KM_LTV && !a.ltv_fwd)) ? 1 : 0;
            atomicAdd(&a.status->substeps[cls], (unsigned long long)substeps);
            atomicAdd(&a.status->krylov_iters[cls], (unsigned long long)iters);
            atomicAdd(&a.status->reorth[cls], (unsigned long long)nre);
            if (a.irep) {
                atomicAdd(&a.irep->substeps, (unsigned long long)substeps);
                atomicAdd(&a.irep->iters, (unsigned long long)iters);
                if (e == e)
                    atomicMax(&a.irep->max_est, (unsigned long long)__double_as_longlong(e));
            }
        }
        nre = 0;
    }

    // V_0 <- exp(tau Op) V_0; if iout, iout += int_0^tau sin(ia + ib s)
    // exp(s Op) V_0 ds.
    // Weight of the k-th Taylor term (hOp)^k u / k! in the integral
    // int_0^h sin(ph + ib s) exp(s Op) u ds:
    //   J_k = h Im(e^{i ph} int_0^1 x^k e^{i ib h x} dx),
    // the inner integral as the series sum_j (i ib h)^j / (j! (k + j + 1)).
    __device__ __forceinline__ static double taylor_weight(int k, double h, double ph,
                                                           double ib) {
        const double beta = ib * h;
        double re = 0.0, im = 0.0, tr = 1.0, ti = 0.0;
        for (int j = 0; j < 60; ++j) {
            const double c = 1.0 / (double)(k + j + 1);
            re += tr * c;
            im += ti * c;
            const double nr = -ti * beta / (j + 1), ni = tr * beta / (j + 1);
            tr = nr;
            ti = ni;
            if (fabs(tr) + fabs(ti) < 1e-18 * (fabs(re) + fabs(im))) break;
        }
        return h * (sin(ph) * re + cos(ph) * im);
    }

    __device__ __forceinline__ void expv(double tau, double ia, double ib, double* iout) {
        if (!(tau > 0.0)) return;
        if (!SI && a.taylor) {
            self().expv_taylor(tau, ia, ib, iout);
            return;
        }
        const double tol = a.tol;
        if (SI) {
            const double gamma = a.gamma_frac * tau;
            self().before_space(gamma);
            double beta;
            bool bd, conv = false;
            double est = 0.0;
            const int me = self().arnoldi(gamma, beta, bd, tau, tol, &conv, &est);
            if (me == 0) return;
            if (!conv) {
                // full dimension: extrapolated from the checks when there
                // were any, else the difference of dimensions m and m - 1;
                // after a breakdown the space is exact
                if (!bd && si_kc > 0 && si_kc < me) {
                    small_exp(me, tau, gamma, S.vy);
                    est = si_plain ? si_diff(me)
                                   : si_extrapolate(si_diff(me), si_dp, me - si_kc, si_gp);
                    __syncthreads();
                } else if (!bd && me > 1) {
                    small_exp(me - 1, tau, gamma, S.vy2);
                    small_exp(me, tau, gamma, S.vy);
                    double s = 0.0;
                    for (int q = 0; q < me; ++q) {
                        const double d = S.vy[q] - (q < me - 1 ? S.vy2[q] : 0.0);
                        s += d * d;
                    }
                    est = sqrt(s);  // relative to beta
                } else {
                    small_exp(me, tau, gamma, S.vy);
                }
            }
            if (iout) small_integral(me, tau, ia, ib, gamma);
            self().combine(me, beta, iout);
            report(est, est > tol, 1, me);
            __syncthreads();
            return;
        }
        // polynomial Krylov with substeps
        double left = tau, sigma0 = 0.0, ts = tau;
        double worst = 0.0;
        bool noconv = false;
        unsigned nsub = 0, iters = 0;
        while (left > 0.0) {
            double beta;
            bool bd, conv = false;
            if (ts > left) ts = left;
            double est = 0.0, tolb = 0.0;
            const int me = self().arnoldi(0.0, beta, bd, ts, tol * (ts / tau), &conv, &est);
            iters += me;
            if (me == 0) break;
            const double hnext = bd ? 0.0 : S.H[me * m + (me - 1)];
            int tries = 0;
            if (conv) tolb = tol * beta * (ts / tau);
            for (; !conv;) {
                if (ts > left) ts = left;
                const double e1 = small_exp(me, ts, 0.0, S.vy);
                est = bd ? 0.0 : beta * hnext * e1;
                tolb = tol * beta * (ts / tau);
                if (est <= tolb) break;
                if (tries >= 40 || ts <= 1e-10 * tau || !(est == est)) {
                    noconv = true;
                    break;
                }
                double f = 0.9 * pow(tolb / est, 1.0 / (double)me);
                f = fmin(0.9, fmax(0.1, f));
                ts *= f;
                ++tries;
            }
            if (beta > 0.0) worst = fmax(worst, est / beta / (ts / tau));
            if (iout) small_integral(me, ts, ia + ib * sigma0, ib, 0.0);
            self().combine(me, beta, iout);
            ++nsub;
            sigma0 += ts;
            left = tau - sigma0;
            if (left <= 1e-13 * tau) left = 0.0;
            if (nsub >= 20000 && left > 0.0) {  // give up: flagged, not hidden
                noconv = true;
                break;
            }
            // grow the next substep when the estimate allows it
            double g = (est > 0.0) ? 0.9 * pow(tolb / est, 1.0 / (double)me) : 2.0;
            g = fmin(2.0, fmax(1.0, g));
            ts *= g;
            __syncthreads();
        }
        report(worst, noconv, nsub, iters);
    }
};

template <int PT, bool SI, bool VAR>
struct Ctx : Core<Ctx<PT, SI, VAR>, SI> {
    using Base = Core<Ctx<PT, SI, VAR>, SI>;
    using Base::a;
    using Base::S;
    using Base::n;
    using Base::m;
    using Base::B;
    using Base::t;
    using Base::small_exp;
    using Base::nre;
    // Points owned by thread t: R groups of VW consecutive points, group r
    // at (t + r*B)*VW, so every basis read is a coalesced 16-byte load.
    static constexpr int VW = (PT >= 2) ? 2 : 1;
    static constexpr int R = PT / VW;
    double* V;
    Tsplit op;
    const double* Wcur = nullptr;  // VAR: state W of the operator J(W)^T
    // VAR && SI: factors of (I - gamma J(W)^T), or of (I - gamma J(W)) with
    // ltv_fwd, for the current W, in global
    // memory after the basis: lo, piv, cp, g, h ([l][chunk], 5n doubles),
    // then the interface rows RA, RB, RC and lo, up at the chunk starts (5B)
    double* aux = nullptr;

    __device__ Ctx(const KrylovArgs& a_, double* lds, double* V_) : Base(a_, lds), V(V_) {
        op.cs = 0.5 * (a.op.lo + a.op.up);
        op.cdf = 0.5 * (a.op.up - a.op.lo);
        op.cc = a.op.d + 2.0 * op.cs;
    }

    __device__ __forceinline__ void before_space(double gamma) {
        if (VAR && SI) si_setup(gamma);
        if (!VAR && SI) ui_setup(gamma);
    }

    // Shift-and-invert solve with constant coefficients, rows
    // lo x_{i-1} + dd x_i + up x_{i+1} of the periodic system (I - gamma A):
    // thread k owns the chunk of PT consecutive points k*PT .. k*PT+PT-1.
    // The chunk's interior 1..PT-1 is a tridiagonal block coupled only to
    // the chunk's first point x_k and the next chunk's first point x_{k+1},
    //   interior = y + g x_k + h x_{k+1},
    // y the block's solve of the right-hand side (Thomas, in registers).
    // Substituting into the chunks' first rows leaves a periodic system in
    // the B values x_k whose rows are again uniform, solved by cyclic
    // reduction with one value per thread.  Everything that depends only
    // on gamma (pivots, g, h, the reduction's multipliers) is computed here
    // once per Krylov space, by one thread, into the LDS table.
    __device__ __attribute__((noinline)) void ui_setup(double gamma) {
        if (t == 0) {
            double* T = S.ut;
            const double lo = -gamma * a.op.lo, dd = 1.0 - gamma * a.op.d, up = -gamma * a.op.up;
            double ca = lo, cb = dd, cc = up;
            if (PT > 1) {
                // forward sweep: pivots, ratios, and the response to x_k
                // (kept in the g slots until the backward sweep)
                T[UT_PIV + 1] = 1.0 / dd;
                T[UT_CP + 1] = up * T[UT_PIV + 1];
                T[UT_G + 1] = -lo * T[UT_PIV + 1];
                for (int l = 2; l < PT; ++l) {
                    T[UT_PIV + l] = 1.0 / (dd - lo * T[UT_CP + l - 1]);
                    T[UT_CP + l] = up * T[UT_PIV + l];
                    T[UT_G + l] = -lo * T[UT_G + l - 1] * T[UT_PIV + l];
                }
                T[UT_H + PT - 1] = -up * T[UT_PIV + PT - 1];
                for (int l = PT - 2; l >= 1; --l) {
                    T[UT_G + l] -= T[UT_CP + l] * T[UT_G + l + 1];
                    T[UT_H + l] = -T[UT_CP + l] * T[UT_H + l + 1];
                }
                ca = lo * T[UT_G + PT - 1];
                cb = dd + lo * T[UT_H + PT - 1] + up * T[UT_G + 1];
                cc = up * T[UT_H + 1];
            }
            int lvl = 0;
            for (int sft = 1; 2 * sft < B; sft <<= 1, ++lvl) {
                const double k1 = ca / cb, k2 = cc / cb;
                T[UT_LVL + 2 * lvl] = k1;
                T[UT_LVL + 2 * lvl + 1] = k2;
                const double na = -ca * k1, nc = -cc * k2, nb = cb - cc * k1 - ca * k2;
                ca = na;
                cb = nb;
                cc = nc;
            }
            // rows k and k + B/2 now couple only to each other
            const double e = ca + cc;
            T[UT_FIN] = cb;
            T[UT_FIN + 1] = e;
            T[UT_FIN + 2] = 1.0 / (cb * cb - e * e);
            T[UT_FIN + 3] = lo;
            T[UT_FIN + 4] = up;
        }
        __syncthreads();
    }

    __device__ __forceinline__ void ui_solve(double (&z)[PT]) {
        const int k = t, Bm = B - 1;
        const double* T = S.ut;
        double* X = S.big;          // chunk c at c * (PT + 1): one pad per chunk
        double* Q = X + n + B;      // two buffers of B interface values
        __syncthreads();            // previous users of `big` are done
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int i = gidx(r) + v;
                X[(i / PT) * (PT + 1) + (i % PT)] = z[r * VW + v];
            }
        __syncthreads();
        const double lo = T[UT_FIN + 3], up = T[UT_FIN + 4];
        double rr[PT], y[PT];
#pragma unroll
        for (int l = 0; l < PT; ++l) rr[l] = X[k * (PT + 1) + l];
        double rhs = rr[0];
        if constexpr (PT > 1) {
            y[1] = rr[1] * T[UT_PIV + 1];
#pragma unroll
            for (int l = 2; l < PT; ++l) y[l] = (rr[l] - lo * y[l - 1]) * T[UT_PIV + l];
            // the previous chunk's last interior value: its forward sweep
            // (the last point needs no back substitution)
            const double* P = X + ((k - 1) & Bm) * (PT + 1);
            double yp = P[1] * T[UT_PIV + 1];
#pragma unroll
            for (int l = 2; l < PT; ++l) yp = (P[l] - lo * yp) * T[UT_PIV + l];
#pragma unroll
            for (int l = PT - 2; l >= 1; --l) y[l] -= T[UT_CP + l] * y[l + 1];
            rhs = rr[0] - lo * yp - up * y[1];
        }
        // cyclic reduction on the B interface values: level s removes the
        // couplings to k - s and k + s using rows k - s and k + s
        int buf = 0, lvl = 0;
        for (int sft = 1; 2 * sft < B; sft <<= 1, ++lvl) {
            double* Rb = Q + buf * B;
            Rb[k] = rhs;
            __syncthreads();
            rhs = rhs - T[UT_LVL + 2 * lvl] * Rb[(k - sft) & Bm] -
                  T[UT_LVL + 2 * lvl + 1] * Rb[(k + sft) & Bm];
            buf ^= 1;
        }
        double* Rb = Q + buf * B;
        Rb[k] = rhs;
        __syncthreads();
        const double cb = T[UT_FIN], e = T[UT_FIN + 1], idet = T[UT_FIN + 2];
        const int kn = (k + 1) & Bm, hb = B >> 1;
        const double xk = (cb * rhs - e * Rb[(k + hb) & Bm]) * idet;
        // the next chunk's first point, from the same two reduced rows
        const double xn = (cb * Rb[kn] - e * Rb[(kn + hb) & Bm]) * idet;
        X[k * (PT + 1)] = xk;
#pragma unroll
        for (int l = 1; l < PT; ++l)
            X[k * (PT + 1) + l] = y[l] + T[UT_G + l] * xk + T[UT_H + l] * xn;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int i = gidx(r) + v;
                z[r * VW + v] = X[(i / PT) * (PT + 1) + (i % PT)];
            }
    }

    // first point of group r, and whether the group lies inside the grid
    __device__ __forceinline__ int gidx(int r) const { return (t + r * B) * VW; }
    __device__ __forceinline__ bool own(int r) const { return gidx(r) < n; }

    // x[r*VW + v] = src[gidx(r) + v] (global, 16-byte loads when VW == 2).
    // Groups past the grid read point 0 and yield zero: the loads carry no
    // branches, so a caller's loads of several vectors are all in flight
    // together.
    __device__ __forceinline__ void gload(const double* __restrict__ src,
                                          double (&x)[PT]) const {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool o = own(r);
            const int g = o ? gidx(r) : 0;
            if (VW == 2) {
                const double2 v = *reinterpret_cast<const double2*>(src + g);
                x[2 * r] = o ? v.x : 0.0;
                x[2 * r + 1] = o ? v.y : 0.0;
            } else {
                const double v = src[g];
                x[r] = o ? v : 0.0;
            }
        }
    }
    __device__ __forceinline__ void gstore(double* __restrict__ dst,
                                           const double (&x)[PT]) const {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!own(r)) continue;
            if (VW == 2)
                *reinterpret_cast<double2*>(dst + gidx(r)) = make_double2(x[2 * r], x[2 * r + 1]);
            else
                dst[gidx(r)] = x[r];
        }
    }

    // z <- Op z (polynomial) or (I - gamma Op)^{-1} z (shift-and-invert).
    __device__ __forceinline__ void apply(double (&z)[PT], double gamma) {
        if constexpr (SI && !VAR) {
            (void)gamma;
            ui_solve(z);
            return;
        }
        double* b0 = S.big;
        __syncthreads();  // previous users of `big` are done
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int v = 0; v < VW; ++v)
                if (own(r)) b0[gidx(r) + v] = z[r * VW + v];
        __syncthreads();
        if (VAR && SI) {
            var_solve(z);
        } else if (VAR) {
            // (J(W)^T x)_i = ((W x)_{i+1} - (W x)_{i-1})/(2h)
            //               - (W_{i+1} - W_{i-1}) x_i/(2h) + nu lap(x)_i
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (!own(r)) continue;
#pragma unroll
                for (int v = 0; v < VW; ++v) {
                    const int i = gidx(r) + v;
                    const int im = i == 0 ? n - 1 : i - 1, ip = i == n - 1 ? 0 : i + 1;
                    const double xm = b0[im], xp = b0[ip], x0 = b0[i];
                    const double Wm = Wcur[im], Wp = Wcur[ip];
                    if (a.ltv_fwd) {
                        // (J(W) x)_i = nu lap(x)_i - W_i (x_{i+1} - x_{i-1})/(2h)
                        //             - x_i (W_{i+1} - W_{i-1})/(2h)
                        z[r * VW + v] = a.nuh2 * ((xp + xm) - 2.0 * x0)
                                        - a.inv2h * (Wcur[i] * (xp - xm) + x0 * (Wp - Wm));
                    } else if (a.fp32) {
                        const float fxm = (float)xm, fxp = (float)xp, fx0 = (float)x0;
                        const float fWm = (float)Wm, fWp = (float)Wp;
                        z[r * VW + v] = (double)((float)a.nuh2 * ((fxp + fxm) - 2.0f * fx0)
                                        + (float)a.inv2h * ((fWp * fxp - fWm * fxm) - (fWp - fWm) * fx0));
                    } else {
                        z[r * VW + v] = a.nuh2 * ((xp + xm) - 2.0 * x0)
                                        + a.inv2h * ((Wp * xp - Wm * xm) - (Wp - Wm) * x0);
                    }
                }
            }
        } else if (!SI) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (!own(r)) continue;
#pragma unroll
                for (int v = 0; v < VW; ++v) {
                    const int i = gidx(r) + v;
                    const double xm = b0[i == 0 ? n - 1 : i - 1];
                    const double xp = b0[i == n - 1 ? 0 : i + 1];
                    const double x0 = b0[i];
                    if (a.fp32) {
                        const float fxm = (float)xm, fxp = (float)xp, fx0 = (float)x0;
                        z[r * VW + v] = (double)((float)op.cs * ((fxp + fxm) - 2.0f * fx0)
                                        + (float)op.cdf * (fxp - fxm) + (float)op.cc * fx0);
                    } else {
                        z[r * VW + v] = op.cs * ((xp + xm) - 2.0 * x0) + op.cdf * (xp - xm) + op.cc * x0;
                    }
                }
            }
        }
    }

    // Row i of (I - gamma J(W)^T): lo x_{i-1} + d x_i + up x_{i+1}, with
    // (J(W)^T x)_i = (W_{i+1} x_{i+1} - W_{i-1} x_{i-1})/(2h)
    //               - (W_{i+1} - W_{i-1}) x_i/(2h) + nu (x_{i+1} - 2x_i + x_{i-1})/h^2.
    // With ltv_fwd, row i of (I - gamma J(W)) from
    // (J(W) x)_i = nu lap(x)_i - W_i (x_{i+1} - x_{i-1})/(2h) - (W_{i+1} - W_{i-1}) x_i/(2h).
    __device__ __forceinline__ void var_row(int i, double gamma, double& lo, double& d,
                                            double& up) const {
        const int im = i == 0 ? n - 1 : i - 1, ip = i == n - 1 ? 0 : i + 1;
        const double Wm = Wcur[im], Wp = Wcur[ip];
        if (a.ltv_fwd) {
            lo = -gamma * (a.nuh2 + a.inv2h * Wcur[i]);
            up = -gamma * (a.nuh2 - a.inv2h * Wcur[i]);
        } else {
            lo = -gamma * (a.nuh2 - a.inv2h * Wm);
            up = -gamma * (a.nuh2 + a.inv2h * Wp);
        }
        d = 1.0 + gamma * (2.0 * a.nuh2 + a.inv2h * (Wp - Wm));
    }

    // Partitioned solve of the periodic tridiagonal system (I - gamma J^T):
    // thread k owns the PT consecutive points of chunk k (B * PT = n).  The
    // chunk's interior points 1..PT-1 are a tridiagonal block coupled only to
    // the chunk's first point x_k and the next chunk's first point x_{k+1}:
    //   interior = y + g x_k + h x_{k+1},
    // y the block solve of the right-hand side, g and h its responses to the
    // two couplings.  Substituting into the rows of the chunk starts leaves a
    // periodic tridiagonal system in the B values x_k, solved by parallel
    // cyclic reduction in LDS.  si_setup factors everything that depends only
    // on W and gamma (Thomas pivots of the blocks, g, h, the interface rows)
    // once per Krylov space.
    __device__ __forceinline__ void si_setup(double gamma) {
        const int k = t, Bn = B;
        double* ex = S.big + n + B;  // 2B exchange slots
        double lo[PT], dd[PT], up[PT];
#pragma unroll
        for (int l = 0; l < PT; ++l) var_row(k * PT + l, gamma, lo[l], dd[l], up[l]);
        double g1 = 0.0, h1 = 0.0, glast = 0.0, hlast = 0.0;
        if constexpr (PT > 1) {
            double piv[PT], cp[PT], gp[PT], g[PT], h[PT];
            piv[1] = 1.0 / dd[1];
            cp[1] = up[1] * piv[1];
            gp[1] = -lo[1] * piv[1];
#pragma unroll
            for (int l = 2; l < PT; ++l) {
                piv[l] = 1.0 / (dd[l] - lo[l] * cp[l - 1]);
                cp[l] = up[l] * piv[l];
                gp[l] = -lo[l] * gp[l - 1] * piv[l];
            }
            g[PT - 1] = gp[PT - 1];
            h[PT - 1] = -up[PT - 1] * piv[PT - 1];
#pragma unroll
            for (int l = PT - 2; l >= 1; --l) {
                g[l] = gp[l] - cp[l] * g[l + 1];
                h[l] = -cp[l] * h[l + 1];
            }
#pragma unroll
            for (int l = 1; l < PT; ++l) {
                aux[(size_t)l * Bn + k] = lo[l];
                aux[(size_t)n + (size_t)l * Bn + k] = piv[l];
                aux[2 * (size_t)n + (size_t)l * Bn + k] = cp[l];
                aux[3 * (size_t)n + (size_t)l * Bn + k] = g[l];
                aux[4 * (size_t)n + (size_t)l * Bn + k] = h[l];
            }
            g1 = g[1];
            h1 = h[1];
            glast = g[PT - 1];
            hlast = h[PT - 1];
        }
        __syncthreads();
        ex[k] = glast;
        ex[Bn + k] = hlast;
        __syncthreads();
        const int km = k == 0 ? Bn - 1 : k - 1;
        double* RI = aux + 5 * (size_t)n;
        if (PT > 1) {
            RI[k] = lo[0] * ex[km];
            RI[Bn + k] = dd[0] + lo[0] * ex[Bn + km] + up[0] * g1;
            RI[2 * Bn + k] = up[0] * h1;
        } else {
            RI[k] = lo[0];
            RI[Bn + k] = dd[0];
            RI[2 * Bn + k] = up[0];
        }
        RI[3 * Bn + k] = lo[0];
        RI[4 * Bn + k] = up[0];
        __syncthreads();
    }

    __device__ __forceinline__ void var_solve(double (&z)[PT]) {
        const int k = t, Bn = B;
        double* X = S.big;          // chunk k at k * (PT + 1), one pad per chunk
        double* Q = X + n + Bn;     // two buffers of a, b, c, d (8B)
        // the caller's barrier at the top of apply() has freed `big`
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int i = gidx(r) + v;
                X[(i / PT) * (PT + 1) + (i % PT)] = z[r * VW + v];
            }
        __syncthreads();
        double rr[PT], y[PT];
#pragma unroll
        for (int l = 0; l < PT; ++l) rr[l] = X[k * (PT + 1) + l];
        const double* RI = aux + 5 * (size_t)n;
        double ca = RI[k], cb = RI[Bn + k], cc = RI[2 * Bn + k];
        double rhs = rr[0];
        if constexpr (PT > 1) {
            y[1] = rr[1] * aux[(size_t)n + Bn + k];
#pragma unroll
            for (int l = 2; l < PT; ++l)
                y[l] = (rr[l] - aux[(size_t)l * Bn + k] * y[l - 1]) *
                       aux[(size_t)n + (size_t)l * Bn + k];
#pragma unroll
            for (int l = PT - 2; l >= 1; --l)
                y[l] -= aux[2 * (size_t)n + (size_t)l * Bn + k] * y[l + 1];
            Q[k] = y[PT - 1];
            __syncthreads();
            const int km = k == 0 ? Bn - 1 : k - 1;
            rhs = rr[0] - RI[3 * Bn + k] * Q[km] - RI[4 * Bn + k] * y[1];
            __syncthreads();
        }
        // parallel cyclic reduction on the B interface rows: level s removes
        // the couplings to k - s and k + s using rows k - s and k + s
        int buf = 0;
        for (int sft = 1; 2 * sft < Bn; sft <<= 1) {
            double* A4 = Q + buf * 4 * Bn;
            A4[k] = ca;
            A4[Bn + k] = cb;
            A4[2 * Bn + k] = cc;
            A4[3 * Bn + k] = rhs;
            __syncthreads();
            const int km = (k - sft) & (Bn - 1), kp = (k + sft) & (Bn - 1);
            const double al = -ca / A4[Bn + km], be = -cc / A4[Bn + kp];
            const double na = al * A4[km], nc = be * A4[2 * Bn + kp];
            cb = cb + al * A4[2 * Bn + km] + be * A4[kp];
            rhs = rhs + al * A4[3 * Bn + km] + be * A4[3 * Bn + kp];
            ca = na;
            cc = nc;
            buf ^= 1;
        }
        // rows k and k + B/2 now couple only to each other
        double* A4 = Q + buf * 4 * Bn;
        const double e = ca + cc;
        A4[k] = e;
        A4[Bn + k] = cb;
        A4[3 * Bn + k] = rhs;
        __syncthreads();
        const int kh = (k + Bn / 2) & (Bn - 1);
        const double xk = (A4[Bn + kh] * rhs - e * A4[3 * Bn + kh]) /
                          (cb * A4[Bn + kh] - e * A4[kh]);
        // back-substitution into the chunk interiors
        double* xs = Q + (buf ^ 1) * 4 * Bn;
        xs[k] = xk;
        __syncthreads();
        const double xn = xs[(k + 1) & (Bn - 1)];
        X[k * (PT + 1)] = xk;
#pragma unroll
        for (int l = 1; l < PT; ++l)
            X[k * (PT + 1) + l] = y[l] + aux[3 * (size_t)n + (size_t)l * Bn + k] * xk +
                                  aux[4 * (size_t)n + (size_t)l * Bn + k] * xn;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int i = gidx(r) + v;
                z[r * VW + v] = X[(i / PT) * (PT + 1) + (i % PT)];
            }
    }

    // Taylor flavour (see KrylovArgs): V_0 <- exp(tau Op) V_0 in registers,
    // iout += the time integral.  The Burgers Jacobian bounds its own norm
    // (largest absolute row sum of J(W)^T).
    __device__ __forceinline__ void expv_taylor(double tau, double ia, double ib,
                                                double* iout) {
        if constexpr (!SI) {
            double u[PT];
            gload(V, u);
            double anorm = a.anorm;
            if (VAR) {
                double mx = 0.0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (!own(r)) continue;
#pragma unroll
                    for (int v = 0; v < VW; ++v) {
                        const int i = gidx(r) + v;
                        const double Wm = Wcur[i == 0 ? n - 1 : i - 1];
                        const double Wp = Wcur[i == n - 1 ? 0 : i + 1];
                        // absolute row sum of J(W)^T (or of J(W))
                        const double rs =
                            a.ltv_fwd ? 2.0 * a.nuh2 + fabs(a.nuh2 - a.inv2h * Wcur[i]) +
                                            fabs(a.nuh2 + a.inv2h * Wcur[i]) +
                                            fabs(a.inv2h * (Wp - Wm))
                                      : 2.0 * a.nuh2 + fabs(a.nuh2 + a.inv2h * Wp) +
                                            fabs(a.nuh2 - a.inv2h * Wm) +
                                            fabs(a.inv2h * (Wp - Wm));
                        mx = fmax(mx, rs);
                    }
                }
                anorm = block_max(mx, S.red);
            }
            double nu = sqrt(block_sum(sumsq(u), S.red));
            if (!(nu > 0.0)) {
                this->flag_nonfinite(nu);
                return;
            }
            int ns = (int)ceil(tau * anorm / a.theta);
            if (ns < 1) ns = 1;
            const double h = tau / ns;
            double I[PT];
#pragma unroll
            for (int q = 0; q < PT; ++q) I[q] = 0.0;
            bool noconv = false;
            double worst = 0.0;
            unsigned terms = 0;
            for (int sub = 0; sub < ns; ++sub) {
                const double ph = ia + ib * (sub * h);
                double tk[PT], sum[PT];
                const double J0 = iout ? Base::taylor_weight(0, h, ph, ib) : 0.0;
#pragma unroll
                for (int q = 0; q < PT; ++q) {
                    tk[q] = u[q];
                    sum[q] = u[q];
                    I[q] += J0 * u[q];
                }
                // terms in pairs: both norms in one reduction.  The stop
                // test of each term is the one of the single-term loop
                // (two consecutive term norms below tol |u|); stopping at
                // the first of a pair keeps its second term as well.
                double prev = nu;
                bool conv = false;
                int slot = 0;
                for (int k = 1; k <= a.tdeg; k += 2) {
                    const bool two = k + 1 <= a.tdeg;
                    double s1, s2 = 0.0;
                    for (int e = 0; e < (two ? 2 : 1); ++e) {
                        apply(tk, 0.0);
                        const double f = h / (k + e);
                        const double Jk = iout ? Base::taylor_weight(k + e, h, ph, ib) : 0.0;
#pragma unroll
                        for (int q = 0; q < PT; ++q) {
                            tk[q] *= f;
                            sum[q] += tk[q];
                            I[q] += Jk * tk[q];
                        }
                        (e == 0 ? s1 : s2) = sumsq(tk);
                    }
                    block_sum2(s1, s2, S.red, slot);
                    const double n1 = sqrt(s1), n2 = sqrt(s2);
                    terms += two ? 2 : 1;
                    if (prev + n1 <= a.tol * nu) {
                        conv = true;
                        worst = fmax(worst, (prev + n1) / nu);
                        break;
                    }
                    if (two && n1 + n2 <= a.tol * nu) {
                        conv = true;
                        worst = fmax(worst, (n1 + n2) / nu);
                        break;
                    }
                    prev = two ? n2 : n1;
                }
                if (!conv) noconv = true;
#pragma unroll
                for (int q = 0; q < PT; ++q) u[q] = sum[q];
                nu = sqrt(block_sum(sumsq(u), S.red));
            }
            gstore(V, u);
            if (iout) {
                double o[PT];
                gload(iout, o);
#pragma unroll
                for (int q = 0; q < PT; ++q) o[q] += I[q];
                gstore(iout, o);
            }
            this->report(worst, noconv, (unsigned)ns, terms);
            __syncthreads();
        }
    }

    // hcol[k] = <V_k, z> for k <= j, KD basis vectors at a time (at most
    // 8, and at most 32 doubles per thread: sweep_batch).  The KD per-thread partial sums
    // are reduced inside the wave by recursive halving (log2 KD exchange
    // stages leave lane group g = lane / (64/KD) holding vector g, the
    // remaining stages sum within the group); one lane per group writes the
    // wave's partial to LDS (layout [k][wave]) and the waves' partials are
    // added in a fixed order at the end, so the loads of the next vectors
    // never wait for a barrier.
    template <int KD, int O>
    __device__ __forceinline__ void halve(double (&part)[KD], int lane) const {
        if constexpr (KD > 1) {
            constexpr int H = KD / 2;
            const bool up = (lane & O) != 0;
            double nxt[H];
#pragma unroll
            for (int q = 0; q < H; ++q) {
                const double send = up ? part[q] : part[q + H];
                const double keep = up ? part[q + H] : part[q];
                nxt[q] = keep + __shfl_xor(send, O, WAVE);
            }
#pragma unroll
            for (int q = 0; q < H; ++q) part[q] = nxt[q];
            halve<H, O / 2>(reinterpret_cast<double(&)[H]>(part), lane);
        }
    }

    __device__ __forceinline__ void dots(const double (&z)[PT], int j) {
        constexpr int KD = sweep_batch<PT>(8);
        constexpr int GS = WAVE / KD;  // lanes per group after the exchanges
        double* P = S.big;
        const int nw = num_waves(), w = wave_id(), lane = lane_id();
        const int g = lane / GS;
        __syncthreads();
        for (int k0 = 0; k0 <= j; k0 += KD) {
            // all KD vectors' loads are issued before the first is used;
            // past V_j the index is clamped to j and the sum discarded
            double x[KD][PT];
#pragma unroll
            for (int q = 0; q < KD; ++q) gload(V + (size_t)(k0 + q <= j ? k0 + q : j) * n, x[q]);
            double part[KD];
#pragma unroll
            for (int q = 0; q < KD; ++q) {
                double s = 0.0;
#pragma unroll
                for (int u = 0; u < PT; ++u) s += x[q][u] * z[u];
                part[q] = (k0 + q <= j) ? s : 0.0;
            }
            halve<KD, 32>(part, lane);
            double s = part[0];
#pragma unroll
            for (int o = GS / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, WAVE);
            if ((lane % GS) == 0 && k0 + g <= j) P[(k0 + g) * nw + w] = s;
        }
        __syncthreads();
        for (int k = t; k <= j; k += B) {
            double s = 0.0;
            for (int u = 0; u < nw; ++u) s += P[k * nw + u];
            S.hcol[k] = s;
        }
        __syncthreads();
    }

    // z -= sum_{k<=j} hcol[k] V_k, UK vectors' loads in flight at a time
    // (past V_j the index is clamped and the coefficient is zero)
    __device__ __forceinline__ void subtract(double (&z)[PT], int j) {
        constexpr int UK = sweep_batch<PT>(4);
        for (int k0 = 0; k0 <= j; k0 += UK) {
            double x[UK][PT];
#pragma unroll
            for (int q = 0; q < UK; ++q) gload(V + (size_t)(k0 + q <= j ? k0 + q : j) * n, x[q]);
#pragma unroll
            for (int q = 0; q < UK; ++q) {
                const double h = (k0 + q <= j) ? S.hcol[k0 + q] : 0.0;
#pragma unroll
                for (int u = 0; u < PT; ++u) z[u] -= h * x[q][u];
            }
        }
    }

    __device__ __forceinline__ double sumsq(const double (&z)[PT]) const {
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < PT; ++u) s += z[u] * z[u];
        return s;
    }

    // Arnoldi from the (unnormalised) vector held in V_0.  Returns the
    // dimension reached; beta = |v|; bd = happy breakdown.  Polynomial
    // flavour with ts > 0: at dimensions 8, 12, 16, ... the a-posteriori
    // estimate beta h_{k+1,k} |e_k^T exp(ts H_k) e_1| is checked against
    // tolb_rel * beta and the process stops early (conv = true, vy holds
    // exp(ts H_k) e_1) once it is met.
    __device__ __forceinline__ int arnoldi(double gamma, double& beta, bool& bd,
                                           double ts = 0.0, double tolb_rel = 0.0,
                                           bool* conv = nullptr, double* est_out = nullptr) {
        double z[PT];
        gload(V, z);
        beta = sqrt(block_sum(sumsq(z), S.red));
        bd = false;
        for (int o = t; o < (m + 1) * m; o += B) S.H[o] = 0.0;
        if (!(beta > 0.0)) {
            this->flag_nonfinite(beta);
            __syncthreads();
            return 0;
        }
        const double ib = 1.0 / beta;
#pragma unroll
        for (int u = 0; u < PT; ++u) z[u] *= ib;
        gstore(V, z);
        int me = m;
        this->si_kc = 0;
        this->si_gp = 0;
        this->si_dp = -1.0;
        int knext = (m / 8 > 1 ? m / 8 : 1) * 4;  // first check, about m/2
        for (int j = 0; j < m; ++j) {
            apply(z, gamma);
            // classical Gram-Schmidt; the second pass runs only when the
            // first left less than eta^2 of |Op v_j|^2 (DGKS_ETA2)
            double nrm2 = 0.0, col = 0.0;
            for (int pass = 0; pass < 2; ++pass) {
                dots(z, j);
                if (t <= j) S.H[t * m + j] += S.hcol[t];
                subtract(z, j);
                nrm2 = block_sum(sumsq(z), S.red);
                double hh = 0.0;
                for (int k = 0; k <= j; ++k) hh += S.H[k * m + j] * S.H[k * m + j];
                // |Op v_j|^2 = sum_k h_kj^2 + nrm^2 (the Gram-Schmidt column)
                col = hh + nrm2;
                if (pass == 0 && !(nrm2 < DGKS_ETA2 * col)) break;
                if (pass == 0) ++nre;
            }
            const double nrm = sqrt(nrm2);
            __syncthreads();
            if (t == 0) S.H[(j + 1) * m + j] = nrm;
            if (!(nrm > 1e-12 * sqrt(col))) {
                // happy breakdown: K_{j+1} is invariant under Op
                me = j + 1;
                bd = true;
                break;
            }
            const int k = j + 1;
            if (!SI && conv && ts > 0.0 && k < m && k >= 8 && (k % 4) == 0) {
                const double e1 = small_exp(k, ts, 0.0, S.vy);
                const double est = beta * nrm * e1;
                if (est <= tolb_rel * beta) {
                    *conv = true;
                    if (est_out) *est_out = est;
                    me = k;
                    break;
                }
            }
            if (SI && conv && ts > 0.0 && k < m && k == knext) {
                // Compare with the previous check's approximation (yprev)
                // and extrapolate the error to dimension k (si_extrapolate);
                // converged when that is below tol.  The next check goes
                // where the observed contraction predicts the tolerance,
                // at least 4 dimensions on and at most at m - 4.
                small_exp(k, ts, gamma, S.vy);
                int step = 4;
                if (this->si_kc > 0) {
                    const double d = this->si_diff(k);
                    const int g = k - this->si_kc;
                    const double est = this->si_extrapolate(d, this->si_dp, g, this->si_gp);
                    __syncthreads();
                    if (est <= tolb_rel) {
                        *conv = true;
                        if (est_out) *est_out = est;
                        me = k;
                        break;
                    }
                    if (this->si_dp > 0.0 && d < this->si_dp && est > 0.0) {
                        const double r4 = pow(d / this->si_dp, 4.0 / (double)this->si_gp);
                        const double blocks = ceil(log(tolb_rel / est) / log(r4));
                        if (blocks > 1.0) step = 4 * (int)fmin(blocks, (double)m);
                    }
                    this->si_dp = d;
                    this->si_gp = g;
                }
                // the last check before the full dimension sits at most 4
                // below it, so the final extrapolation spans few dimensions
                knext = k + step < m - 4 ? k + step : m - 4;
                if (knext < k + 4) knext = k + 4;
                this->si_kc = k;
                for (int q = t; q < k; q += B) S.yprev[q] = S.vy[q];
                __syncthreads();
            }
            const double inv = 1.0 / nrm;
#pragma unroll
            for (int u = 0; u < PT; ++u) z[u] *= inv;
            gstore(V + (size_t)(j + 1) * n, z);
        }
        __syncthreads();
        return me;
    }

    // V_0 <- beta * V_k vy  and, when iout, iout += beta * V_k vc.
    __device__ __forceinline__ void combine(int k, double beta, double* iout) {
        double y[PT], I[PT];
#pragma unroll
        for (int u = 0; u < PT; ++u) {
            y[u] = 0.0;
            I[u] = 0.0;
        }
        constexpr int UK = (PT >= 16) ? 2 : 4;
#pragma unroll UK
        for (int q = 0; q < k; ++q) {
            const double cy = beta * S.vy[q];
            const double ci = iout ? beta * S.vc[q] : 0.0;
            double x[PT];
            gload(V + (size_t)q * n, x);
#pragma unroll
            for (int u = 0; u < PT; ++u) {
                y[u] += cy * x[u];
                I[u] += ci * x[u];
            }
        }
        gstore(V, y);
        if (iout) {
            double o[PT];
            gload(iout, o);
#pragma unroll
            for (int u = 0; u < PT; ++u) o[u] += I[u];
            gstore(iout, o);
        }
    }

};

template <int PT, bool SI, bool VAR>
__device__ __forceinline__ void dev_krylov1d(const KrylovArgs& a, int piece, double* lds) {
    if (a.skip && *a.skip) return;  // the same value for the whole workgroup
    const int n = a.n;
    double* V = a.basis + (size_t)piece * (a.m + 1) * n;
    Ctx<PT, SI, VAR> c(a, lds, V);
    // The current vector of the piece lives in V_0 (global memory); every
    // thread only reads and writes its own points of it.
    const double* vin = (a.mode == KM_CLASSIC) ? a.vin + (size_t)piece * n : a.vin;
    // time integral: the single piece, or each classic piece into its own
    // vector (phase a.ia per unit of the piece's time, see KrylovArgs)
    double* iout = (a.mode == KM_SINGLE) ? a.iout
                 : (a.mode == KM_CLASSIC && a.iout) ? a.iout + (size_t)piece * n : nullptr;
    {
        double x[PT];
        c.gload(vin, x);
        c.gstore(V, x);
        if (iout) {
#pragma unroll
            for (int u = 0; u < PT; ++u) x[u] = 0.0;
            c.gstore(iout, x);
        }
    }
    // classic: one exponential of (npieces - piece) slice lengths;
    // chain: npieces - 1 exponentials of one slice length, adding the next
    // slice end state after each; single: one exponential with integral.
    // ltv: 2 * npieces exponentials, each with its own operator state.
    const int nexp = (a.mode == KM_CHAIN) ? a.npieces - 1
                   : (a.mode == KM_LTV) ? (a.ltv_one ? a.npieces : 2 * a.npieces) : 1;
    const double tau = (a.mode == KM_CLASSIC) ? (double)(a.npieces - piece) * a.tau : a.tau;
    const double ia = (a.mode == KM_CLASSIC) ? a.ia * tau : a.ia;
    if (VAR && SI) c.aux = V + (size_t)(a.m + 1) * n;
    int nextadd = 0;
    for (int q = 0; q < nexp; ++q) {
        if (VAR) c.Wcur = a.wop + (size_t)q * n;
        c.expv(tau, ia, a.ib, iout);
        if (a.mode == KM_CHAIN) {
            double x[PT], w[PT];
            c.gload(a.vin + (size_t)(q + 1) * n, x);
            c.gload(V, w);
#pragma unroll
            for (int u = 0; u < PT; ++u) w[u] += x[u];
            c.gstore(V, w);
        }
        // time-varying chain: after a macro step (two factors, or one) that
        // ends on a slice start, add that slice's end state
        const bool mend = a.ltv_one || (q & 1);
        const int mstep = a.ltv_one ? q : (q >> 1);
        if (VAR && a.vadd && mend && nextadd < a.nadd && a.addq[nextadd] == mstep) {
            double x[PT], w[PT];
            c.gload(a.vadd + (size_t)(a.nadd - 1 - nextadd) * n, x);
            c.gload(V, w);
#pragma unroll
            for (int u = 0; u < PT; ++u) w[u] += x[u];
            c.gstore(V, w);
            if (a.vsnap) c.gstore(a.vsnap + (size_t)nextadd * n, w);
            ++nextadd;
        }
    }
    double* y = (a.mode == KM_CLASSIC) ? a.yout + (size_t)piece * n : a.yout;
    if (y) {
        double x[PT];
        c.gload(V, x);
        c.gstore(y, x);
    }
}

template <int PT, bool SI, bool VAR>
__global__ void __launch_bounds__(krylov_max_block(PT)) k_krylov1d(KrylovArgs a) {
    extern __shared__ double lds[];
    dev_krylov1d<PT, SI, VAR>(a, blockIdx.x, lds);
}

// ---- the Chebyshev flavour: its own chain kernel ---------------------------
// Each factor exp(tau Op) v of a time-varying chain (Op = J(W)^T, or J(W)
// with ltv_fwd) by the Chebyshev series of exp on a real interval that
// holds the real parts of tau Op's spectrum (the focal interval of the
// ReLPM of section 4.1, here the Gershgorin bounds of the current operator),
// in the Chebyshev basis instead of Newton form at Leja points:
//   exp(c + g x) = e^{c+g} (e_0 + 2 sum_{k>=1} e_k T_k(x)),
//   e_k = e^{-g} I_k(g)  (modified Bessel functions, scaled),
// c, g the interval's centre and half-width, T_k(Ah) v by the three-term
// recurrence with Ah = (tau Op - c)/g.  No inner products until the a priori
// degree (e_k + e_{k+1} <= tol/16, k >= g); from there the terms are checked
// in pairs until two consecutive ones are below tol |v|.  Substeps keep the
// series within the coefficient table.
//
// A chain runs in one workgroup whose B threads cover the grid in whole
// chunks (B PT = n): thread t keeps points t PT .. t PT + PT - 1 of the
// chain vector in registers from the start vector to the result, each
// factor's operator state W beside it (its two halo values loaded once per
// factor, the next factor's during the current one), and each series term
// exchanges only the chunk edges through LDS (two slots in turn, one
// barrier per term).  LDS: 128 doubles for reductions, 4 B for the edges,
// the coefficients and the a priori degree.
constexpr int CHEB_CHAIN_LDS = 128 + 4 * 512 + CHEB_KMAX + 2;

bool cheb_chain_shape(int n, int* B, int* pt) {
    if (n <= 256 && n % 64 == 0) {
        *B = n;
        *pt = 1;
        return true;
    }
    for (int b : {256, 512}) {
        if (n % b) continue;
        const int p = n / b;
        if ((p & (p - 1)) == 0 && p <= (b == 256 ? 8 : 16)) {
            *B = b;
            *pt = p;
            return true;
        }
    }
    return false;
}

struct ChebStats {
    double worst = 0.0;
    unsigned terms = 0, substeps = 0;
    bool noconv = false, nonfinite = false;
};

// u <- exp(tau Op) u for Op = J(W)^T (or J(W) with ltv_fwd), the chunk's
// W in w with halos wl, wr.
template <int PT>
__device__ __forceinline__ void cheb_factor(const KrylovArgs& a, double (&u)[PT],
                                            const double (&w)[PT], double wl, double wr,
                                            double tau, double* red, double* xch,
                                            double* coef, ChebStats& st) {
    const int t = threadIdx.x, B = blockDim.x;
    auto coefs = [&](int q, double& lw, double& d, double& up) {
        const double Wm = q == 0 ? wl : w[q - 1], Wp = q == PT - 1 ? wr : w[q + 1];
        lw = a.ltv_fwd ? a.nuh2 + a.inv2h * w[q] : a.nuh2 - a.inv2h * Wm;
        up = a.ltv_fwd ? a.nuh2 - a.inv2h * w[q] : a.nuh2 + a.inv2h * Wp;
        d = -2.0 * a.nuh2 - a.inv2h * (Wp - Wm);
    };
    double lo = INFINITY, hi = -INFINITY, ss = 0.0;
#pragma unroll
    for (int q = 0; q < PT; ++q) {
        double lw, d, up;
        coefs(q, lw, d, up);
        const double o = fabs(lw) + fabs(up);
        lo = fmin(lo, d - o);
        hi = fmax(hi, d + o);
        ss += u[q] * u[q];
    }
    hi = block_max(hi, red);
    lo = -block_max(-lo, red);
    double nu = sqrt(block_sum(ss, red));
    if (!(nu > 0.0) || !isfinite(lo) || !isfinite(hi)) {
        // a zero vector stays zero; a non-finite one is recorded
        if (!isfinite(nu) || !isfinite(lo) || !isfinite(hi)) st.nonfinite = true;
        return;
    }
    const double room = (double)(CHEB_KMAX - 40);
    const double gmax = fmax(1.0, room - 6.0 * sqrt(room));
    int ns = (int)ceil(0.5 * tau * (hi - lo) / gmax);
    if (ns < 1) ns = 1;
    const double ts = tau / ns;
    const double c = 0.5 * ts * (hi + lo);
    const double g = fmax(0.5 * ts * (hi - lo), 0.5);
    const int kc = (int)fmin((double)(CHEB_KMAX - 1), g + 6.0 * sqrt(g) + 40.0);
    // every thread has read the previous factor's coefficients: the
    // reductions above passed barriers since
    if (t == 0) {
        // Miller's backward recurrence I_{k-1} = I_{k+1} + (2k/g) I_k, from
        // above kc (where the scaled values are below 1e-20), normalised by
        // e^g = I_0 + 2 sum I_k; then the a priori degree into the slot
        // after the table
        const double r2 = 2.0 / g;
        const int top = kc + 24;
        double ip = 0.0, ik = 1e-200, sum = 0.0;
        for (int k = top; k >= 1; --k) {
            if (k <= kc + 1) coef[k] = ik;
            sum += 2.0 * ik;
            const double im = ip + (k * r2) * ik;
            ip = ik;
            ik = im;
            if (ik > 1e200) {
                for (int j = k; j <= kc + 1; ++j) coef[j] *= 1e-200;
                ip *= 1e-200;
                ik *= 1e-200;
                sum *= 1e-200;
            }
        }
        coef[0] = ik;
        sum += ik;
        const double inv = 1.0 / sum;
        for (int k = 0; k <= kc + 1; ++k) coef[k] *= inv;
        int kd = kc - 1;
        for (int k = (int)ceil(g) > 1 ? (int)ceil(g) : 1; k < kc; ++k)
            if (coef[k] + coef[k + 1] <= a.tol * 0.0625) {
                kd = k;
                break;
            }
        coef[CHEB_KMAX + 1] = (double)kd;
    }
    __syncthreads();
    const int ka = (int)coef[CHEB_KMAX + 1];
    const double scale = exp(c + g), ig = 1.0 / g;
    int slotx = 0;
    auto ahat = [&](const double (&x)[PT], double (&z)[PT]) {
        double* e = xch + slotx * 2 * B;
        e[t] = x[0];
        e[B + t] = x[PT - 1];
        __syncthreads();
        const double xl = e[B + (t == 0 ? B - 1 : t - 1)];
        const double xr = e[t == B - 1 ? 0 : t + 1];
        slotx ^= 1;
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            double lw, d, up;
            coefs(q, lw, d, up);
            const double xm = q == 0 ? xl : x[q - 1], xp = q == PT - 1 ? xr : x[q + 1];
            z[q] = (ts * (lw * xm + d * x[q] + up * xp) - c * x[q]) * ig;
        }
    };
    for (int sub = 0; sub < ns; ++sub) {
        double t0[PT], t1[PT], acc[PT], z[PT];
#pragma unroll
        for (int q = 0; q < PT; ++q) t0[q] = u[q];
        ahat(u, t1);
        ++st.terms;
#pragma unroll
        for (int q = 0; q < PT; ++q) acc[q] = coef[0] * u[q] + 2.0 * coef[1] * t1[q];
        double prev = INFINITY;
        bool conv = false;
        int slot = 0;
        int k = 2;
        while (k <= kc) {
            const bool two = k + 1 <= kc;
            double s1 = 0.0, s2 = 0.0;
            for (int e = 0; e < (two ? 2 : 1); ++e) {
                ahat(t1, z);
                ++st.terms;
                const double ck = 2.0 * coef[k + e];
                double sq = 0.0;
#pragma unroll
                for (int q = 0; q < PT; ++q) {
                    const double tn = 2.0 * z[q] - t0[q];
                    t0[q] = t1[q];
                    t1[q] = tn;
                    acc[q] += ck * tn;
                    sq += tn * tn;
                }
                (e == 0 ? s1 : s2) = ck * ck * sq;
            }
            if (k + 1 >= ka) {
                block_sum2(s1, s2, red, slot);
                const double n1 = scale * sqrt(s1), n2 = scale * sqrt(s2);
                if (prev + n1 <= a.tol * nu) {
                    conv = true;
                    st.worst = fmax(st.worst, (prev + n1) / nu);
                    break;
                }
                if (two && n1 + n2 <= a.tol * nu) {
                    conv = true;
                    st.worst = fmax(st.worst, (n1 + n2) / nu);
                    break;
                }
                prev = two ? n2 : n1;
            }
            k += two ? 2 : 1;
        }
        if (!conv) {
            st.noconv = true;
            st.worst = fmax(st.worst, isfinite(prev) ? prev / nu : 1.0);
        }
        double s2 = 0.0;
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            u[q] = scale * acc[q];
            s2 += u[q] * u[q];
        }
        if (sub + 1 < ns) nu = sqrt(block_sum(s2, red));
    }
    st.substeps += ns;
}

template <int PT>
__device__ __forceinline__ void dev_cheb_chain(const KrylovArgs& a, double* lds) {
    if (a.skip && *a.skip) return;
    const int n = a.n, t = threadIdx.x, B = blockDim.x, base = t * PT;
    double* red = lds;
    double* xch = lds + 128;
    double* coef = xch + 4 * B;
    double u[PT];
#pragma unroll
    for (int q = 0; q < PT; ++q) u[q] = a.vin[base + q];
    const int nexp = a.ltv_one ? a.npieces : 2 * a.npieces;
    ChebStats st;
    int nextadd = 0;
    // each factor's operator state, loaded one factor ahead (the series'
    // barriers wait for LDS only)
    double w[PT], wl, wr;
    auto load_w = [&](int q, double (&x)[PT], double& xl, double& xr) {
        const double* W = a.wop + (size_t)q * n;
#pragma unroll
        for (int k = 0; k < PT; ++k) x[k] = W[base + k];
        xl = W[base == 0 ? n - 1 : base - 1];
        xr = W[base + PT == n ? 0 : base + PT];
    };
    load_w(0, w, wl, wr);
    for (int q = 0; q < nexp; ++q) {
        double wn[PT], wnl = 0.0, wnr = 0.0;
        if (q + 1 < nexp) load_w(q + 1, wn, wnl, wnr);
        cheb_factor<PT>(a, u, w, wl, wr, a.tau, red, xch, coef, st);
#pragma unroll
        for (int k = 0; k < PT; ++k) w[k] = wn[k];
        wl = wnl;
        wr = wnr;
        // after a macro step (two factors, or one) that ends on a slice
        // start, add that slice's end state
        const bool mend = a.ltv_one || (q & 1);
        const int mstep = a.ltv_one ? q : (q >> 1);
        if (a.vadd && mend && nextadd < a.nadd && a.addq[nextadd] == mstep) {
            const double* x = a.vadd + (size_t)(a.nadd - 1 - nextadd) * n + base;
#pragma unroll
            for (int k = 0; k < PT; ++k) u[k] += x[k];
            if (a.vsnap) {
                double* y = a.vsnap + (size_t)nextadd * n + base;
#pragma unroll
                for (int k = 0; k < PT; ++k) y[k] = u[k];
            }
            ++nextadd;
        }
    }
    if (a.yout) {
#pragma unroll
        for (int q = 0; q < PT; ++q) a.yout[base + q] = u[q];
    }
    if (t == 0 && a.status) {
        if (st.noconv) atomicOr(&a.status->flags, ST_NOCONV);
        if (st.nonfinite || !(st.worst == st.worst)) atomicOr(&a.status->flags, ST_NONFINITE);
        const double e = fabs(st.worst);
        if (e == e) atomicMax(&a.status->max_est, (unsigned long long)__double_as_longlong(e));
        const int cls = a.ltv_fwd ? 0 : 1;  // the nonlinear direct's chain: direct
        atomicAdd(&a.status->substeps[cls], (unsigned long long)st.substeps);
        atomicAdd(&a.status->krylov_iters[cls], (unsigned long long)st.terms);
        if (a.irep) {
            atomicAdd(&a.irep->substeps, (unsigned long long)st.substeps);
            atomicAdd(&a.irep->iters, (unsigned long long)st.terms);
            if (e == e)
                atomicMax(&a.irep->max_est, (unsigned long long)__double_as_longlong(e));
        }
    }
}

template <int PT>
__global__ void __launch_bounds__(512) k_cheb_chain(KrylovArgs a) {
    __shared__ double lds[CHEB_CHAIN_LDS];
    dev_cheb_chain<PT>(a, lds);
}

// Ragged batch: workgroup i runs the chain of entry i; all entries of a
// launch share the workgroup size and PT (the host groups them so).
template <int PT>
__global__ void __launch_bounds__(512) k_cheb_chain_batch(const KrylovArgs* tab) {
    __shared__ double lds[CHEB_CHAIN_LDS];
    const KrylovArgs a = tab[blockIdx.x];
    if (a.pt != PT || a.n != PT * (int)blockDim.x) return;
    dev_cheb_chain<PT>(a, lds);
}

// Ragged batch of time-varying chains: workgroup i runs instance i; all
// instances of one launch share the workgroup size, compiled for at most NT.
template <int PT, int NT>
__device__ __forceinline__ void ltv_if(const KrylovArgs& a, double* lds) {
    if constexpr (krylov_max_block(PT) >= NT) {
        if (a.si)
            dev_krylov1d<PT, true, true>(a, 0, lds);
        else
            dev_krylov1d<PT, false, true>(a, 0, lds);
    }
}

template <int NT>
__global__ void __launch_bounds__(NT) k_krylov_ltv_batch(const KrylovArgs* tab) {
    extern __shared__ double lds[];
    const KrylovArgs a = tab[blockIdx.x];
    switch (a.pt) {
        case 1: ltv_if<1, NT>(a, lds); break;
        case 2: ltv_if<2, NT>(a, lds); break;
        case 4: ltv_if<4, NT>(a, lds); break;
        case 8: ltv_if<8, NT>(a, lds); break;
        case 16: ltv_if<16, NT>(a, lds); break;
        case 32: ltv_if<32, NT>(a, lds); break;
        default: break;
    }
}

// ---- 2D: basis vectors streamed from global memory ------------------------
// A 2D instance has n = nx * ny points, too many to keep a vector in
// registers; thread t owns the 16-byte groups g = t + r*B (points 2g, 2g+1),
// r < n / (2B), of every vector, and each Arnoldi step streams them: the
// five-point stencil writes the new vector, the Gram-Schmidt passes read the
// basis (8 vectors per exchange round for the dots) and update the new vector
// in place.  Polynomial and Taylor flavours, and shift-and-invert (below).
template <int KD, int O>
__device__ __forceinline__ void wave_halve(double (&part)[KD], int lane) {
    if constexpr (KD > 1) {
        constexpr int H = KD / 2;
        const bool up = (lane & O) != 0;
        double nxt[H];
#pragma unroll
        for (int q = 0; q < H; ++q) {
            const double send = up ? part[q] : part[q + H];
            const double keep = up ? part[q + H] : part[q];
            nxt[q] = keep + __shfl_xor(send, O, WAVE);
        }
        wave_halve<H, O / 2>(nxt, lane);
        part[0] = nxt[0];
    }
}

// ---- 2D shift-and-invert: (I - gamma A)^{-1} by Fourier diagonalisation ----
// The five-point operator has constant coefficients on a periodic grid, so
// the Fourier mode exp(i(thx col + thy row)) (thx = 2 pi kx / nx, thy =
// 2 pi ky / ny) is an eigenvector with eigenvalue
//   lam = c + w e^{-i thx} + e e^{i thx} + s e^{-i thy} + n e^{i thy},
// and the solve divides each mode by 1 - gamma lam.  It runs in place on
// the output vector in three passes of one workgroup:
//   rows:    the real DFT of every row (radix-2 in LDS, one wave per row),
//            packed into the row's nx doubles: slot 0 the mode kx = 0, slot
//            1 the mode kx = nx/2 (both real for real data), slots 2kx,
//            2kx + 1 the complex mode 0 < kx < nx/2;
//   columns: for each kx (one wave per kx), the DFT along y of that slot's
//            column, the division, the inverse DFT along y; the kx = 0 and
//            nx/2 columns have real y-operators and stay real;
//   rows:    the inverse real DFT of every row.
// nx and ny are powers of two of at most FFT2_MAX; the twiddle table
// e^{-2 pi i k / FFT2_MAX} stays in LDS for the whole launch.
constexpr int FFT2_MAX = 256;

// Doubles of the Krylov layout in LDS: Core's regions for dimension m up to
// its small dense scratch S.big, then that scratch (shared with the dot
// partials of KRYLOV2D_BLOCK threads).
__host__ __device__ constexpr size_t krylov2d_big_doubles(int m) {
    return (size_t)(m + 1) * (KRYLOV2D_BLOCK / 64) > 6 * (size_t)m * m + 5 * (size_t)m + 8
               ? (size_t)(m + 1) * (KRYLOV2D_BLOCK / 64)
               : 6 * (size_t)m * m + 5 * (size_t)m + 8;
}
__host__ __device__ constexpr size_t krylov2d_core_doubles(int m) {
    return 128 + (size_t)(((m + 1 + 7) / 8) * 8) * 2 + 8 + (size_t)(m + 1) * m + UT_DOUBLES +
           krylov2d_big_doubles(m);
}
// Shift-and-invert: the per-wave FFT buffers share S.big (the solve runs
// between the small dense phases, and nothing in S.big outlives a solve: the
// checks keep their coefficients in S.yprev, and the final coefficients are
// formed after the last solve); the twiddle table follows the larger of the
// two.
constexpr size_t FFT2_BUF_DOUBLES = (size_t)(KRYLOV2D_BLOCK / WAVE) * 2 * FFT2_MAX;
__host__ __device__ constexpr size_t krylov2d_si_doubles(int m) {
    return krylov2d_core_doubles(m) - krylov2d_big_doubles(m) +
           (krylov2d_big_doubles(m) > FFT2_BUF_DOUBLES ? krylov2d_big_doubles(m)
                                                       : FFT2_BUF_DOUBLES) +
           2 * FFT2_MAX;
}

__device__ __forceinline__ int bitrev(int j, int lb) {
    return lb == 0 ? 0 : (int)(__brev((unsigned)j) >> (32 - lb));
}

__device__ __forceinline__ double2 cmul(double2 u, double2 v) {
    return make_double2(u.x * v.x - u.y * v.y, u.x * v.y + u.y * v.x);
}

// Orders one wave's LDS accesses: the wave's LDS operations complete in
// issue order, so a compiler fence at wavefront scope is all a transform
// stage needs between writing points and reading other lanes' points.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// In-place radix-2 transform of the L points in buf (L a power of two,
// L <= FFT2_MAX) by the lanes of one wave.  dit: the input is in bit-reversed
// order and the output in natural order (decimation in time); otherwise the
// reverse (decimation in frequency).  inv: e^{+2 pi i jk / L} (unscaled).
// Wave-local: the caller orders the buffer's writes before the call.
__device__ __forceinline__ void wave_fft(double2* buf, const double2* tw, int L, bool dit,
                                         bool inv, int lane) {
    const int nb = L >> 1;
    for (int s = 0; (1 << s) < L; ++s) {
        const int len = dit ? (2 << s) : (L >> s), half = len >> 1;
        const int ts = FFT2_MAX / len;
        for (int b = lane; b < nb; b += WAVE) {
            const int grp = b / half, pos = b - grp * half;
            const int i0 = grp * len + pos, i1 = i0 + half;
            double2 w = tw[pos * ts];
            if (inv) w.y = -w.y;
            const double2 u = buf[i0], v = buf[i1];
            if (dit) {
                const double2 tv = cmul(v, w);
                buf[i0] = make_double2(u.x + tv.x, u.y + tv.y);
                buf[i1] = make_double2(u.x - tv.x, u.y - tv.y);
            } else {
                buf[i0] = make_double2(u.x + v.x, u.y + v.y);
                buf[i1] = cmul(make_double2(u.x - v.x, u.y - v.y), w);
            }
        }
        wave_sync();
    }
}

template <bool SI>
struct Ctx2 : Core<Ctx2<SI>, SI> {
    using Base = Core<Ctx2<SI>, SI>;
    using Base::a;
    using Base::S;
    using Base::n;
    using Base::m;
    using Base::B;
    using Base::t;
    using Base::small_exp;
    using Base::nre;
    double* V;
    int G, nx, ny;
    double2* fbuf;  // shift-and-invert: this wave's FFT buffer
    double2* tw;    // shift-and-invert: twiddle table

    __device__ Ctx2(const KrylovArgs& a_, double* lds, double* V_)
        : Base(a_, lds), V(V_), G(a_.n / (2 * blockDim.x)), nx(a_.nx), ny(a_.ny) {
        if constexpr (SI) {
            // the 2D spaces' differences need not contract geometrically
            // (advection): the error is taken as the difference itself
            this->si_plain = true;
            tw = reinterpret_cast<double2*>(lds + krylov2d_si_doubles(a_.m) - 2 * FFT2_MAX);
            fbuf = reinterpret_cast<double2*>(S.big) + (size_t)wave_id() * FFT2_MAX;
            for (int k = t; k < FFT2_MAX; k += B) {
                double sn, cs;
                sincospi(-2.0 * (double)k / (double)FFT2_MAX, &sn, &cs);
                tw[k] = make_double2(cs, sn);
            }
            __syncthreads();
        }
    }

    __device__ __forceinline__ void before_space(double) {}

    // dst = (I - gamma A)^{-1} src (all of src visible to the workgroup; dst
    // complete on return).  src and dst are distinct.  Each wave takes rows
    // (or x-wavenumbers) on its own; the workgroup meets only between passes.
    __device__ void solve(const double* __restrict__ src, double* __restrict__ dst,
                          double gamma) {
        const int lane = lane_id(), wv = wave_id(), nw = num_waves();
        const int lx = 31 - __clz(nx), ly = 31 - __clz(ny), hx = nx >> 1;
        // rows: real DFT, packed
        for (int r = wv; r < ny; r += nw) {
            for (int j = lane; j < nx; j += WAVE)
                fbuf[bitrev(j, lx)] = make_double2(src[(size_t)r * nx + j], 0.0);
            wave_sync();
            wave_fft(fbuf, tw, nx, true, false, lane);
            double* row = dst + (size_t)r * nx;
            for (int k = lane; k <= hx; k += WAVE) {
                const double2 X = fbuf[k];
                if (k == 0)
                    row[0] = X.x;
                else if (k == hx)
                    row[1] = X.x;
                else
                    *reinterpret_cast<double2*>(row + 2 * k) = X;
            }
            wave_sync();
        }
        __syncthreads();
        // columns: DFT along y, division by 1 - gamma lam, inverse DFT
        const Sten5 o = a.op5;
        const double scale = 1.0 / ((double)nx * (double)ny);
        for (int kx = wv; kx <= hx; kx += nw) {
            const bool real = kx == 0 || kx == hx;
            const int slot = kx == 0 ? 0 : (kx == hx ? 1 : 2 * kx);
            for (int j = lane; j < ny; j += WAVE) {
                const double* p = dst + (size_t)j * nx + slot;
                fbuf[bitrev(j, ly)] =
                    real ? make_double2(p[0], 0.0) : *reinterpret_cast<const double2*>(p);
            }
            wave_sync();
            wave_fft(fbuf, tw, ny, true, false, lane);
            // with E = e^{-i th} (a table entry), w E + e conj(E) has real
            // part (w + e) Re E and imaginary part (w - e) Im E
            const double2 ex = tw[kx * (FFT2_MAX / nx)];
            const double lxr = o.c + (o.w + o.e) * ex.x;
            const double lxi = (o.w - o.e) * ex.y;
            for (int ky = lane; ky < ny; ky += WAVE) {
                const double2 ey = tw[ky * (FFT2_MAX / ny)];
                // mr + i mi = 1 - gamma lam
                const double mr = 1.0 - gamma * (lxr + (o.s + o.n) * ey.x);
                const double mi = -gamma * (lxi + (o.s - o.n) * ey.y);
                const double d = scale / (mr * mr + mi * mi);
                const double2 z = fbuf[ky];
                fbuf[ky] = make_double2((z.x * mr + z.y * mi) * d, (z.y * mr - z.x * mi) * d);
            }
            wave_sync();
            wave_fft(fbuf, tw, ny, false, true, lane);
            for (int j = lane; j < ny; j += WAVE) {
                double* p = dst + (size_t)j * nx + slot;
                const double2 z = fbuf[bitrev(j, ly)];
                if (real)
                    p[0] = z.x;
                else
                    *reinterpret_cast<double2*>(p) = z;
            }
            wave_sync();
        }
        __syncthreads();
        // rows: inverse real DFT (Hermitian completion of the packed modes)
        for (int r = wv; r < ny; r += nw) {
            double* row = dst + (size_t)r * nx;
            for (int k = lane; k < nx; k += WAVE) {
                double2 X;
                if (k == 0)
                    X = make_double2(row[0], 0.0);
                else if (k == hx)
                    X = make_double2(row[1], 0.0);
                else if (k < hx)
                    X = *reinterpret_cast<const double2*>(row + 2 * k);
                else {
                    X = *reinterpret_cast<const double2*>(row + 2 * (nx - k));
                    X.y = -X.y;
                }
                fbuf[k] = X;
            }
            wave_sync();
            wave_fft(fbuf, tw, nx, false, true, lane);
            for (int j = lane; j < nx; j += WAVE) row[j] = fbuf[bitrev(j, lx)].x;
            wave_sync();
        }
        __syncthreads();
    }

    __device__ __forceinline__ double2 ld2(const double* p, int g) const {
        return *reinterpret_cast<const double2*>(p + 2 * (size_t)g);
    }
    __device__ __forceinline__ void st2(double* p, int g, double2 v) const {
        *reinterpret_cast<double2*>(p + 2 * (size_t)g) = v;
    }

    // dst = Op src (all of src must be visible to the workgroup)
    __device__ __forceinline__ void apply(const double* __restrict__ src,
                                          double* __restrict__ dst) const {
        const Sten5 o = a.op5;
#pragma unroll 4
        for (int r = 0; r < G; ++r) {
            const int g = t + r * B, i = 2 * g;
            const int row = i / nx, col = i - row * nx, rc = row * nx;
            const int rs = (row == 0 ? ny - 1 : row - 1) * nx;
            const int rn = (row == ny - 1 ? 0 : row + 1) * nx;
            const double2 x = ld2(src, g);
            const double xw = src[rc + (col == 0 ? nx - 1 : col - 1)];
            const double xe = src[rc + (col + 2 == nx ? 0 : col + 2)];
            const double2 xs = *reinterpret_cast<const double2*>(src + rs + col);
            const double2 xn = *reinterpret_cast<const double2*>(src + rn + col);
            double2 y;
            y.x = o.c * x.x + o.w * xw + o.e * x.y + o.s * xs.x + o.n * xn.x;
            y.y = o.c * x.y + o.w * x.x + o.e * xe + o.s * xs.y + o.n * xn.y;
            st2(dst, g, y);
        }
    }

    __device__ __forceinline__ double sumsq(const double* v) const {
        double s = 0.0;
#pragma unroll 4
        for (int r = 0; r < G; ++r) {
            const double2 x = ld2(v, t + r * B);
            s += x.x * x.x + x.y * x.y;
        }
        return s;
    }

    __device__ __forceinline__ void scale(double* v, double f) const {
#pragma unroll 4
        for (int r = 0; r < G; ++r) {
            const int g = t + r * B;
            double2 x = ld2(v, g);
            x.x *= f;
            x.y *= f;
            st2(v, g, x);
        }
    }

    // hcol[k] = <V_k, w>, k <= j (see Ctx::dots for the reduction layout)
    __device__ __forceinline__ void dots(const double* w, int j) {
        constexpr int KD = 8, GS = WAVE / KD;
        double* Pp = S.big;
        const int nw = num_waves(), wv = wave_id(), lane = lane_id();
        __syncthreads();
        for (int k0 = 0; k0 <= j; k0 += KD) {
            double part[KD];
#pragma unroll
            for (int q = 0; q < KD; ++q) part[q] = 0.0;
            for (int r = 0; r < G; ++r) {
                const int g = t + r * B;
                const double2 x = ld2(w, g);
#pragma unroll
                for (int q = 0; q < KD; ++q) {
                    if (k0 + q <= j) {
                        const double2 v = ld2(V + (size_t)(k0 + q) * n, g);
                        part[q] += x.x * v.x + x.y * v.y;
                    }
                }
            }
            wave_halve<KD, 32>(part, lane);
            double s = part[0];
#pragma unroll
            for (int o = GS / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, WAVE);
            const int gq = lane / GS;
            if ((lane % GS) == 0 && k0 + gq <= j) Pp[(k0 + gq) * nw + wv] = s;
        }
        __syncthreads();
        for (int k = t; k <= j; k += B) {
            double s = 0.0;
            for (int u = 0; u < nw; ++u) s += Pp[k * nw + u];
            S.hcol[k] = s;
        }
        __syncthreads();
    }

    // w -= sum_{k<=j} hcol[k] V_k; returns this thread's part of |w|^2
    __device__ __forceinline__ double subtract(double* w, int j) const {
        double ss = 0.0;
        for (int r = 0; r < G; ++r) {
            const int g = t + r * B;
            double2 x = ld2(w, g);
#pragma unroll 4
            for (int k = 0; k <= j; ++k) {
                const double h = S.hcol[k];
                const double2 v = ld2(V + (size_t)k * n, g);
                x.x -= h * v.x;
                x.y -= h * v.y;
            }
            st2(w, g, x);
            ss += x.x * x.x + x.y * x.y;
        }
        return ss;
    }

    // Arnoldi from the (unnormalised) vector in V_0; same contract as
    // Ctx::arnoldi (both flavours: the shift-and-invert space from the
    // Fourier solve, with the same extrapolated checks from about m/2 on).
    __device__ __forceinline__ int arnoldi(double gamma, double& beta, bool& bd,
                                           double ts = 0.0, double tolb_rel = 0.0,
                                           bool* conv = nullptr, double* est_out = nullptr) {
        beta = sqrt(block_sum(sumsq(V), S.red));
        bd = false;
        for (int o = t; o < (m + 1) * m; o += B) S.H[o] = 0.0;
        if (!(beta > 0.0)) {
            this->flag_nonfinite(beta);
            __syncthreads();
            return 0;
        }
        scale(V, 1.0 / beta);
        int me = m;
        this->si_kc = 0;
        this->si_gp = 0;
        this->si_dp = -1.0;
        int knext = (m / 8 > 1 ? m / 8 : 1) * 4;  // first shift-and-invert check
        for (int j = 0; j < m; ++j) {
            double* w = V + (size_t)(j + 1) * n;
            __syncthreads();  // V_j complete: the stencil reads neighbours
            if constexpr (SI)
                solve(V + (size_t)j * n, w, gamma);
            else
                apply(V + (size_t)j * n, w);
            // classical Gram-Schmidt, second pass by the DGKS criterion
            double nrm2 = 0.0, col = 0.0;
            for (int pass = 0; pass < 2; ++pass) {
                dots(w, j);
                if (t <= j) S.H[t * m + j] += S.hcol[t];
                nrm2 = block_sum(subtract(w, j), S.red);
                double hh = 0.0;
                for (int k = 0; k <= j; ++k) hh += S.H[k * m + j] * S.H[k * m + j];
                col = hh + nrm2;
                if (pass == 0 && !(nrm2 < DGKS_ETA2 * col)) break;
                if (pass == 0) ++nre;
            }
            const double nrm = sqrt(nrm2);
            __syncthreads();
            if (t == 0) S.H[(j + 1) * m + j] = nrm;
            if (!(nrm > 1e-12 * sqrt(col))) {
                me = j + 1;
                bd = true;
                break;
            }
            const int k = j + 1;
            if (!SI && conv && ts > 0.0 && k < m && k >= 8 && (k % 4) == 0) {
                const double e1 = small_exp(k, ts, 0.0, S.vy);
                const double est = beta * nrm * e1;
                if (est <= tolb_rel * beta) {
                    *conv = true;
                    if (est_out) *est_out = est;
                    me = k;
                    break;
                }
            }
            if (SI && conv && ts > 0.0 && k < m && k == knext) {
                // as in Ctx::arnoldi, with the difference to the previous
                // check's approximation itself as the error (si_plain)
                small_exp(k, ts, gamma, S.vy);
                int step = 4;
                if (this->si_kc > 0) {
                    const double d = this->si_diff(k);
                    const int g = k - this->si_kc;
                    const double est = d;
                    __syncthreads();
                    if (est <= tolb_rel) {
                        *conv = true;
                        if (est_out) *est_out = est;
                        me = k;
                        break;
                    }
                    if (this->si_dp > 0.0 && d < this->si_dp && est > 0.0) {
                        const double r4 = pow(d / this->si_dp, 4.0 / (double)this->si_gp);
                        const double blocks = ceil(log(tolb_rel / est) / log(r4));
                        if (blocks > 1.0) step = 4 * (int)fmin(blocks, (double)m);
                    }
                    this->si_dp = d;
                    this->si_gp = g;
                }
                knext = k + step < m - 4 ? k + step : m - 4;
                if (knext < k + 4) knext = k + 4;
                this->si_kc = k;
                for (int q = t; q < k; q += B) S.yprev[q] = S.vy[q];
                __syncthreads();
            }
            scale(w, 1.0 / nrm);
        }
        __syncthreads();
        return me;
    }

    // V_0 <- beta * V_k vy and, when iout, iout += beta * V_k vc.
    __device__ __forceinline__ void combine(int k, double beta, double* iout) {
        for (int r = 0; r < G; ++r) {
            const int g = t + r * B;
            double2 y = make_double2(0.0, 0.0), I = make_double2(0.0, 0.0);
#pragma unroll 4
            for (int q = 0; q < k; ++q) {
                const double2 v = ld2(V + (size_t)q * n, g);
                const double cy = beta * S.vy[q];
                y.x += cy * v.x;
                y.y += cy * v.y;
                if (iout) {
                    const double ci = beta * S.vc[q];
                    I.x += ci * v.x;
                    I.y += ci * v.y;
                }
            }
            st2(V, g, y);
            if (iout) {
                double2 o = ld2(iout, g);
                o.x += I.x;
                o.y += I.y;
                st2(iout, g, o);
            }
        }
    }

    // One Taylor term with the running sum updated every other term:
    // dst = f Op src; when acc, the sum takes both the previous term (src,
    // read anyway for the stencil) and the new one, sum = (base or sum) +
    // src + dst, and iout += Jb base + Js src + Jd dst (base: the substep's
    // start vector, folded in at the substep's first update).  Without acc
    // only dst is written.  Returns the local |dst|^2.
    __device__ __forceinline__ double taylor_pass2(const double* __restrict__ src,
                                                   double* __restrict__ dst,
                                                   double* __restrict__ sum,
                                                   const double* __restrict__ base,
                                                   double* __restrict__ iout, double f,
                                                   double Jb, double Js, double Jd,
                                                   bool acc) const {
        const Sten5 o = a.op5;
        double ss = 0.0;
#pragma unroll 2
        for (int r = 0; r < G; ++r) {
            const int g = t + r * B, i = 2 * g;
            const int row = i / nx, col = i - row * nx, rc = row * nx;
            const int rs = (row == 0 ? ny - 1 : row - 1) * nx;
            const int rn = (row == ny - 1 ? 0 : row + 1) * nx;
            const double2 x = ld2(src, g);
            const double xw = src[rc + (col == 0 ? nx - 1 : col - 1)];
            const double xe = src[rc + (col + 2 == nx ? 0 : col + 2)];
            const double2 xs = *reinterpret_cast<const double2*>(src + rs + col);
            const double2 xn = *reinterpret_cast<const double2*>(src + rn + col);
            double2 y;
            y.x = f * (o.c * x.x + o.w * xw + o.e * x.y + o.s * xs.x + o.n * xn.x);
            y.y = f * (o.c * x.y + o.w * x.x + o.e * xe + o.s * xs.y + o.n * xn.y);
            st2(dst, g, y);
            if (acc) {
                const double2 b = ld2(base ? base : sum, g);
                if (iout) {
                    double2 io = ld2(iout, g);
                    if (base) {
                        io.x += Jb * b.x;
                        io.y += Jb * b.y;
                    }
                    io.x += Js * x.x + Jd * y.x;
                    io.y += Js * x.y + Jd * y.y;
                    st2(iout, g, io);
                }
                st2(sum, g, make_double2(b.x + x.x + y.x, b.y + x.y + y.y));
            }
            ss += y.x * y.x + y.y * y.y;
        }
        return ss;
    }

    // sum = (base or sum) + src and iout += Jb base + Js src: the last term
    // of a substep when it is still pending.
    __device__ __forceinline__ void taylor_flush(const double* __restrict__ src,
                                                 double* __restrict__ sum,
                                                 const double* __restrict__ base,
                                                 double* __restrict__ iout, double Jb,
                                                 double Js) const {
        for (int r = 0; r < G; ++r) {
            const int g = t + r * B;
            const double2 x = ld2(src, g);
            const double2 b = ld2(base ? base : sum, g);
            if (iout) {
                double2 io = ld2(iout, g);
                if (base) {
                    io.x += Jb * b.x;
                    io.y += Jb * b.y;
                }
                io.x += Js * x.x;
                io.y += Js * x.y;
                st2(iout, g, io);
            }
            st2(sum, g, make_double2(b.x + x.x, b.y + x.y));
        }
    }

    // Taylor flavour (see KrylovArgs) on streamed vectors: the current
    // vector and the running sum alternate between V_0 and V_1, the terms
    // between V_2 and V_3.
    __device__ __forceinline__ void expv_taylor(double tau, double ia, double ib,
                                                double* iout) {
        double* u = V;
        double* sm = V + n;
        double* tA = V + 2 * (size_t)n;
        double* tB = V + 3 * (size_t)n;
        double nu = sqrt(block_sum(sumsq(u), S.red));
        if (!(nu > 0.0)) {
            this->flag_nonfinite(nu);
            return;
        }
        int ns = (int)ceil(tau * a.anorm / a.theta);
        if (ns < 1) ns = 1;
        const double h = tau / ns;
        bool noconv = false;
        double worst = 0.0;
        unsigned terms = 0;
        for (int sub = 0; sub < ns; ++sub) {
            const double ph = ia + ib * (sub * h);
            const double J0 = iout ? this->taylor_weight(0, h, ph, ib) : 0.0;
            __syncthreads();  // u complete: the stencil reads neighbours
            // term 1 from u; the sum (started from u) is updated every
            // other term, so a term is pending after each odd one
            double prev = sqrt(block_sum(
                taylor_pass2(u, tA, sm, nullptr, nullptr, h, 0.0, 0.0, 0.0, false), S.red));
            ++terms;
            bool conv = false, started = false;
            double Jprev = iout ? this->taylor_weight(1, h, ph, ib) : 0.0;
            const double* src = tA;
            double* dst = tB;
            int k = 2;
            for (; k <= a.tdeg; ++k) {
                const double Jk = iout ? this->taylor_weight(k, h, ph, ib) : 0.0;
                const bool acc = (k % 2) == 0;
                const double nt = sqrt(block_sum(
                    taylor_pass2(src, dst, sm, started ? nullptr : u, iout, h / k, J0, Jprev, Jk,
                                 acc), S.red));
                if (acc) started = true;
                ++terms;
                Jprev = Jk;
                const double* tmp = src;
                src = dst;
                dst = const_cast<double*>(tmp);
                if (prev + nt <= a.tol * nu) {
                    conv = true;
                    worst = fmax(worst, (prev + nt) / nu);
                    break;
                }
                prev = nt;
            }
            // the last term (now in src) is pending after an odd term, and
            // so is u when no update has run yet (term 1 only)
            const int last = (k <= a.tdeg) ? k : a.tdeg;
            if ((last % 2) == 1) taylor_flush(src, sm, started ? nullptr : u, iout, J0, Jprev);
            if (!conv) noconv = true;
            double* tmp = u;
            u = sm;
            sm = tmp;
            nu = sqrt(block_sum(sumsq(u), S.red));
        }
        if (u != V) copy(u, V);
        this->report(worst, noconv, (unsigned)ns, terms);
        __syncthreads();
    }

    __device__ __forceinline__ void copy(const double* src, double* dst) const {
#pragma unroll 4
        for (int r = 0; r < G; ++r) st2(dst, t + r * B, ld2(src, t + r * B));
    }
    __device__ __forceinline__ void add(const double* src, double* dst) const {
#pragma unroll 4
        for (int r = 0; r < G; ++r) {
            const int g = t + r * B;
            double2 x = ld2(dst, g);
            const double2 v = ld2(src, g);
            x.x += v.x;
            x.y += v.y;
            st2(dst, g, x);
        }
    }
};

template <bool SI>
__device__ __forceinline__ void dev_krylov2d(const KrylovArgs& a, int piece, double* lds) {
    const int n = a.n;
    double* V = a.basis + (size_t)piece * (a.m + 1) * n;
    Ctx2<SI> c(a, lds, V);
    const double* vin = (a.mode == KM_CLASSIC) ? a.vin + (size_t)piece * n : a.vin;
    c.copy(vin, V);
    double* iout = (a.mode == KM_SINGLE) ? a.iout : nullptr;
    if (iout) {
#pragma unroll 4
        for (int r = 0; r < c.G; ++r)
            c.st2(iout, c.t + r * c.B, make_double2(0.0, 0.0));
    }
    const int nexp = (a.mode == KM_CHAIN) ? a.npieces - 1 : 1;
    const double tau = (a.mode == KM_CLASSIC) ? (double)(a.npieces - piece) * a.tau : a.tau;
    for (int q = 0; q < nexp; ++q) {
        c.expv(tau, a.ia, a.ib, iout);
        if (a.mode == KM_CHAIN) c.add(a.vin + (size_t)(q + 1) * n, V);
    }
    double* y = (a.mode == KM_CLASSIC) ? a.yout + (size_t)piece * n : a.yout;
    if (y) c.copy(V, y);
}

template <bool SI>
__global__ void __launch_bounds__(KRYLOV2D_BLOCK) k_krylov2d(const KrylovArgs* tab, int count) {
    extern __shared__ double lds[];
    const int b = blockIdx.x;
    int e = 0;
    while (e + 1 < count && tab[e + 1].blk0 <= b) ++e;
    const KrylovArgs a = tab[e];
    const int piece = b - a.blk0;
    if (a.mode != KM_CLASSIC && piece > 0) return;
    if (a.mode == KM_CLASSIC && piece >= a.npieces) return;
    dev_krylov2d<SI>(a, piece, lds);
}

template <bool SI, bool VAR>
hipError_t launch_pt(const KrylovArgs& a, int B, int pt, int grid, size_t lds,
                     hipStream_t s) {
    switch (pt) {
#define PXP_K(PTV)                                                               \
    case PTV: {                                                                \
        auto kern = k_krylov1d<PTV, SI, VAR>;                                 \
        (void)hipFuncSetAttribute((const void*)kern,                                 \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        kern<<<grid, B, lds, s>>>(a);                                          \
        break;                                                                 \
    }
        PXP_K(1)
        PXP_K(2)
        PXP_K(4)
        PXP_K(8)
        PXP_K(16)
        PXP_K(32)
#undef PXP_K
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

bool pow2_pt(int p) { return p == 1 || p == 2 || p == 4 || p == 8 || p == 16 || p == 32; }

// Workgroup size B and points per thread pt for n points.  With a hint the
// hint is the workgroup size (a multiple of 64, at most 512, cut to n);
// without one, 512 threads where that shape exists (more waves in flight per
// compute unit for the basis streams), else 256.
bool krylov_shape(int n, int block_hint, int* B, int* pt) {
    if (block_hint <= 0)
        return krylov_shape(n, 512, B, pt) || krylov_shape(n, 256, B, pt);
    int b = block_hint;
    if (b > n) b = ((n + 63) / 64) * 64;
    if (b % 64 || b > 512) return false;
    const int p = (n + b - 1) / b;
    if (!pow2_pt(p) || b > krylov_max_block(p)) return false;
    *B = b;
    *pt = p;
    return true;
}

}  // namespace

size_t krylov1d_lds_bytes(int n, int m, int block, int si) {
    (void)si;
    const int ldr = ((m + 1 + 7) / 8) * 8;
    const size_t d = 128 + ldr + 8 + (size_t)(m + 1) * m + ldr + UT_DOUBLES +
                     big_doubles(n, m, block);
    return d * sizeof(double);
}

size_t krylov2d_lds_bytes(int m, int si) {
    return (si ? krylov2d_si_doubles(m) : krylov2d_core_doubles(m)) * sizeof(double);
}

bool fft2_grid(int nx, int ny) {
    auto p2 = [](int v) { return v >= 2 && (v & (v - 1)) == 0; };
    return p2(nx) && p2(ny) && nx <= FFT2_MAX && ny <= FFT2_MAX;
}

hipError_t launch_krylov2d(const KrylovArgs* tab, int count, int total_blocks,
                           size_t lds, int si, hipStream_t s) {
    if (count <= 0 || total_blocks <= 0) return hipSuccess;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const void* kern = si ? (const void*)k_krylov2d<true> : (const void*)k_krylov2d<false>;
    (void)hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (si)
        k_krylov2d<true><<<total_blocks, KRYLOV2D_BLOCK, lds, s>>>(tab, count);
    else
        k_krylov2d<false><<<total_blocks, KRYLOV2D_BLOCK, lds, s>>>(tab, count);
    return hipGetLastError();
}

hipError_t launch_krylov_ltv_batch(const KrylovArgs* tab, int block, int count,
                                   size_t lds, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (lds > 160 * 1024 || block % 64 || block <= 0 || block > 512)
        return hipErrorInvalidValue;
#define PXP_LTV(NTV)                                                               \
    {                                                                            \
        (void)hipFuncSetAttribute((const void*)k_krylov_ltv_batch<NTV>,                \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        k_krylov_ltv_batch<NTV><<<count, block, lds, s>>>(tab);                   \
    }
    if (block <= 256)
        PXP_LTV(256)
    else
        PXP_LTV(512)
#undef PXP_LTV
    return hipGetLastError();
}

bool krylov_shape_pub(int n, int block_hint, int* B, int* pt) {
    return krylov_shape(n, block_hint, B, pt);
}

bool cheb_chain_shape_pub(int n, int* B, int* pt) { return cheb_chain_shape(n, B, pt); }

hipError_t launch_cheb_chain_batch(const KrylovArgs* tab, int block, int pt, int count,
                                   hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (block % 64 || block <= 0 || block > 512) return hipErrorInvalidValue;
    switch (pt) {
        case 1: k_cheb_chain_batch<1><<<count, block, 0, s>>>(tab); break;
        case 2: k_cheb_chain_batch<2><<<count, block, 0, s>>>(tab); break;
        case 4: k_cheb_chain_batch<4><<<count, block, 0, s>>>(tab); break;
        case 8: k_cheb_chain_batch<8><<<count, block, 0, s>>>(tab); break;
        case 16: k_cheb_chain_batch<16><<<count, block, 0, s>>>(tab); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_krylov1d(const KrylovArgs& a, int block_hint, hipStream_t s) {
    if (a.m < 1 || a.m > M_MAX_1D || a.n < 2) return hipErrorInvalidValue;
    if (a.si && a.mode != KM_LTV && (a.n & (a.n - 1))) return hipErrorInvalidValue;
    int B, pt;
    if (!krylov_shape(a.n, block_hint, &B, &pt)) return hipErrorInvalidValue;
    if (a.si && pt * B != a.n) return hipErrorInvalidValue;
    // two consecutive points per 16-byte load when pt >= 2
    if (pt >= 2 && (a.n & 1)) return hipErrorInvalidValue;
    const size_t lds = krylov1d_lds_bytes(a.n, a.m, B, a.si);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const int grid = (a.mode == KM_CLASSIC) ? a.npieces : 1;
    if (grid <= 0) return hipSuccess;
    if (a.mode == KM_LTV) {
        if (!a.wop) return hipErrorInvalidValue;
        if (a.si && (B & (B - 1))) return hipErrorInvalidValue;
        int cB, cpt;
        if (a.cheb) {
            // the Chebyshev flavour runs in its own kernel only (problems
            // whose grid it does not cover are refused at validation)
            if (a.si || a.iout || !cheb_chain_shape(a.n, &cB, &cpt)) return hipErrorInvalidValue;
            switch (cpt) {
                case 1: k_cheb_chain<1><<<1, cB, 0, s>>>(a); break;
                case 2: k_cheb_chain<2><<<1, cB, 0, s>>>(a); break;
                case 4: k_cheb_chain<4><<<1, cB, 0, s>>>(a); break;
                case 8: k_cheb_chain<8><<<1, cB, 0, s>>>(a); break;
                case 16: k_cheb_chain<16><<<1, cB, 0, s>>>(a); break;
                default: return hipErrorInvalidValue;
            }
            return hipGetLastError();
        }
        return a.si ? launch_pt<true, true>(a, B, pt, grid, lds, s)
                    : launch_pt<false, true>(a, B, pt, grid, lds, s);
    }
    return a.si ? launch_pt<true, false>(a, B, pt, grid, lds, s)
                : launch_pt<false, false>(a, B, pt, grid, lds, s);
}

}  // namespace pxp
