// Exponential actions of the 2D five-point operator by uniformisation, split
// over row bands (the homogeneous solves of paper section 3.1, eqs. hom and
// adjHomNormal, for the 2D problem of section 4.2).
//
// With mu >= -A.c and nonnegative off-diagonal coefficients (upwind
// advection with nonnegative velocities and the five-point Laplacian, and
// the transposes of both), N = I + A / mu is a nonnegative matrix whose rows
// and columns sum to one, and
//     exp(tau A) x = sum_k p_k N^k x,   p_k = e^{-lam} lam^k / k!,  lam = mu tau.
// Every term N^k x is bounded by |x| in the max norm and the weights are
// positive with unit sum, so the series has no cancellation, and the part
// left out after D terms is bounded a priori by the Poisson tail P(X >= D).
// The number of terms is therefore fixed before the launch, and a band of
// output rows can compute its part of D terms from its own rows plus D halo
// rows on each side, recomputed redundantly: no workgroup waits for another.
//
// Workgroup layout: the row bands of pxp_band.hpp (8 waves of 8 rows, whole
// grid rows per wave row, edge rows through LDS once per term).  Output rows
// are region rows off .. off+R-1 (R = 16 or 32 rows per band, off =
// (64 - R) / 2); a pass of d stencil applications needs d <= off halo rows,
// and rows further out never reach the output.  N has a zero diagonal
// (mu = -A.c), so a term costs four multiply-adds per point.
//
// A pass covers terms k0 .. k1-1 of one or two weighted sums of the same
// terms: the first (weights p_k, or a table) for exp(tau A) x, the second (a
// table) for a time integral of the exponential (the adjoint's Lambda).
#include "pxp_internal.hpp"
#include "pxp_device.hpp"
#include "pxp_band.hpp"

namespace pxp {
namespace {

static_assert(POIS_PASS_TERMS <= 16, "a pass needs at most 16 halo rows");

// Poisson weight e^{-lam} lam^k / k! in log form (no underflow of e^{-lam}
// for large lam; terms far below the peak flush to zero harmlessly).
__device__ __forceinline__ double pois_pmf(double lam, int k) {
    if (lam <= 0.0) return k == 0 ? 1.0 : 0.0;
    return exp((double)k * log(lam) - lam - lgamma((double)k + 1.0));
}

__device__ __forceinline__ int pois_entry(const PoisEntry* tab, int count, int b) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].blk0 <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <int NX, bool TWO>
__global__ void __launch_bounds__(BNT)
k_pois2d(const PoisEntry* __restrict__ tab, int count, int pass) {
    constexpr int CPL = NX / WAVE;
    __shared__ double xch[BW][2][NX];
    __shared__ double wt[POIS_PASS_TERMS], wt2[POIS_PASS_TERMS];
    const PoisEntry& E = tab[pois_entry(tab, count, blockIdx.x)];
    const int ny = E.ny, R = E.rows, nb = ny / R;
    const int local = blockIdx.x - E.blk0;
    const int vec = local / nb, band = local - vec * nb;
    const int off = (BROWS - R) / 2;
    const int k0 = pass * POIS_PASS_TERMS, k1 = min(E.D, k0 + POIS_PASS_TERMS);
    const bool final_pass = k1 == E.D;
    const int nterm = k1 - k0;
    const int napp = final_pass ? nterm - 1 : nterm;
    const size_t nn = (size_t)NX * ny;
    const int t = threadIdx.x, w = wave_id(), l = lane_id(), cb = l * CPL;
    if (t < nterm) {
        const int k = k0 + t;
        if (E.wtab) {
            wt[t] = E.wtab[k];
        } else {
            // p_k = p_{k0} lam^(k-k0) k0! / k!: one log-form weight per
            // pass, then a short product (k - k0 < 16)
            double pk = pois_pmf(E.lam, k0);
            for (int q = k0 + 1; q <= k; ++q) pk *= E.lam / q;
            wt[t] = pk;
        }
        if (TWO) {
            if (E.wtab2i) {
                const double ph = E.ph0 + (double)vec * E.dph;
                wt2[t] = sin(ph) * E.wtab2[k] + cos(ph) * E.wtab2i[k];
            } else {
                wt2[t] = E.wtab2[k];
            }
        }
    }
    // region row r <-> grid row band*R - off + r (periodic); every region
    // row is a grid row, so the loads are in bounds and issued together, and
    // rows beyond the pass's halo never reach the output
    int g[BRW];
    wave_rows(band_grow(band * R - off + w * BRW, 0, ny), ny, g);
    const size_t vof = (size_t)vec;
    // pass 0 reads the input vectors, later passes the previous pass's terms
    const double* tin = pass == 0 ? E.x + vof * E.sx : E.tb[(pass - 1) & 1] + vof * nn;
    double tv[BRW][CPL], acc[BRW][CPL], acc2[TWO ? BRW : 1][CPL];
    // rows of the term vector this pass needs (the halo of its napp
    // applications); a wave row is uniform, so the skip is a uniform branch
#pragma unroll
    for (int i = 0; i < BRW; ++i) {
        const int r = w * BRW + i;
        if (r >= off - napp && r < off + R + napp) {
            row_load<CPL>(tin + (size_t)g[i] * NX + cb, tv[i]);
        } else {
#pragma unroll
            for (int c = 0; c < CPL; ++c) tv[i][c] = 0.0;
        }
    }
    // the sums start from the previous pass's (or zero) plus, in the final
    // pass, the vectors added to them: those loads then overlap the term
    // loads instead of trailing the arithmetic
    const bool cont = k0 > 0;
    const double* add1 = final_pass ? E.partner : nullptr;
    const double* add2 = (TWO && final_pass) ? E.out2_add : nullptr;
    const double* add3 = (TWO && final_pass) ? E.out2_add2 : nullptr;
#pragma unroll
    for (int i = 0; i < BRW; ++i) {
        const int r = w * BRW + i;
        const bool orow = r >= off && r < off + R;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            acc[i][c] = 0.0;
            if (TWO) acc2[i][c] = 0.0;
        }
        if (!orow) continue;
        const size_t o = (size_t)g[i] * NX + cb;
        if (cont) {
            row_load<CPL>(E.acc + vof * E.s_acc + o, acc[i]);
            if (TWO) row_load<CPL>(E.acc2 + vof * E.s_acc + o, acc2[i]);
        }
        if (add1) {
            double q[CPL];
            row_load<CPL>(add1 + vof * E.s_partner + o, q);
#pragma unroll
            for (int c = 0; c < CPL; ++c) acc[i][c] += q[c];
        }
        if (add2) {
            double q[CPL];
            row_load<CPL>(add2 + vof * E.s_add + o, q);
#pragma unroll
            for (int c = 0; c < CPL; ++c) acc2[i][c] += q[c];
        }
        if (add3) {
            double q[CPL];
            row_load<CPL>(add3 + vof * E.s_add + o, q);
#pragma unroll
            for (int c = 0; c < CPL; ++c) acc2[i][c] += q[c];
        }
    }
    // N = I + A/mu has a zero diagonal for mu = -A.c
    const double Nw = E.N.w, Ne = E.N.e, Ns = E.N.s, Nn = E.N.n;
    __syncthreads();  // weights visible
    for (int j = 0; j < nterm; ++j) {
        const double pj = wt[j];
        const double qj = TWO ? wt2[j] : 0.0;
#pragma unroll
        for (int i = 0; i < BRW; ++i)
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                acc[i][c] += pj * tv[i][c];
                if (TWO) acc2[i][c] += qj * tv[i][c];
            }
        if (j >= napp) break;
        // tv <- N tv; waves whose rows are no longer needed skip it
        double prev[CPL], dn[CPL];
        exchange_edges<NX, CPL>(xch, tv, w, cb, prev, dn);
        const int keep = napp - 1 - j;
        if (w * BRW + BRW <= off - keep || w * BRW >= off + R + keep) continue;
#pragma unroll
        for (int i = 0; i < BRW; ++i) {
            double cur[CPL];
#pragma unroll
            for (int c = 0; c < CPL; ++c) cur[c] = tv[i][c];
            const double wv = from_west(cur[CPL - 1]);
            const double ev = from_east(cur[0]);
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const double xw = (c > 0) ? cur[c - 1] : wv;
                const double xe = (c < CPL - 1) ? cur[c + 1] : ev;
                const double xn = (i < BRW - 1) ? tv[i + 1][c] : dn[c];
                tv[i][c] = Nw * xw + Ne * xe + Ns * prev[c] + Nn * xn;
                prev[c] = cur[c];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // write back: output rows only
    bool bad = false;
#pragma unroll
    for (int i = 0; i < BRW; ++i) {
        const int r = w * BRW + i;
        if (r < off || r >= off + R) continue;
        const size_t o = (size_t)g[i] * NX + cb;
        if (final_pass) {
            if (E.out) {
#pragma unroll
                for (int c = 0; c < CPL; ++c) bad |= !isfinite(acc[i][c]);
                row_store<CPL>(E.out + vof * E.s_out + o, acc[i]);
            }
            if (TWO) {
#pragma unroll
                for (int c = 0; c < CPL; ++c) bad |= !isfinite(acc2[i][c]);
                row_store<CPL>(E.out2 + vof * E.s_out + o, acc2[i]);
            }
        } else {
            row_store<CPL>(E.tb[pass & 1] + vof * nn + o, tv[i]);
            row_store<CPL>(E.acc + vof * E.s_acc + o, acc[i]);
            if (TWO) row_store<CPL>(E.acc2 + vof * E.s_acc + o, acc2[i]);
        }
    }
    if (final_pass && E.status) {
        if (__any(bad) && l == 0) atomicOr(&E.status->flags, ST_NONFINITE);
        if (local == 0 && t == 0) {
            const unsigned long long eb = (unsigned long long)__double_as_longlong(E.est);
            atomicMax(&E.status->max_est, eb);
            if (E.irep) {
                // one exponential per vector of the entry, k1 terms each
                atomicAdd(&E.irep->substeps, (unsigned long long)E.nvec);
                atomicAdd(&E.irep->iters, (unsigned long long)E.nvec * (unsigned long long)k1);
                atomicMax(&E.irep->max_est, eb);
            }
        }
    }
}

// Weights of the time integral int_0^h sin(phi - omega s) exp(s A) x ds of
// one uniformised exponential (lam = mu h), in the form sum_k w_k N^k x:
//   w_k = scale * Im( e^{i phi} alpha^{-(k+1)} R_k ),  alpha = 1 + i omega / mu,
//   R_k = sum_{j > k} e^{-alpha lam} (alpha lam)^j / j!,  scale = 1 / mu,
// which is int_0^lam of e^{-u} u^k / k! against the modulation, written with
// the regularised incomplete gamma function of complex argument alpha lam.
// R_k is summed from the far tail down (no cancellation).  One workgroup per
// table, one thread.
__global__ void k_pois_weights(const PoisWeights* __restrict__ tab) {
    const PoisWeights& P = tab[blockIdx.x];
    if (threadIdx.x != 0) return;
    const int D = P.D;
    const double beta = P.omega / P.mu;
    const double zr = P.lam, zi = P.lam * beta;  // z = alpha lam
    // E_j by the forward recurrence from E_0 = e^{-z}, up to J well past D
    const int J = D + 64 + (int)(8.0 * sqrt(P.lam));
    double er = exp(-zr) * cos(zi), ei = -exp(-zr) * sin(zi);
    // E_j = e^{-z} z^j / j!: by the recurrence E_j = E_{j-1} z / j from E_0
    // while e^{-lam} is a normal double.  Beyond, e^{-lam} underflows: E_j is
    // formed in log form at the peak j0 = floor|z|, |E_j0| = exp(j0 log|z| -
    // lam - lgamma(j0+1)), arg E_j0 = j0 arg z - Im z, and the same
    // recurrence runs from there both ways (down: E_{j-1} = E_j j / z), the
    // magnitudes falling away from the peak (terms far from it flush to zero
    // harmlessly).  E_j, j < D, go into the output table; the tail beyond D
    // is summed on the way.
    double tr = 0.0, ti = 0.0;  // sum_{j >= D} E_j
    auto put = [&](int j, double a, double b) {
        if (j < D) {
            P.w[j] = a;
            P.wi[j] = b;
        } else {
            tr += a;
            ti += b;
        }
    };
    if (P.lam <= 600.0) {
        for (int j = 0; j <= J; ++j) {
            if (j > 0) {
                const double nr = (er * zr - ei * zi) / j, ni = (er * zi + ei * zr) / j;
                er = nr;
                ei = ni;
            }
            put(j, er, ei);
        }
    } else {
        const double az2 = zr * zr + zi * zi;
        const int j0 = min(J, (int)floor(sqrt(az2)));
        const double m0 = exp((double)j0 * 0.5 * log(az2) - zr - lgamma((double)j0 + 1.0));
        const double ph0 = (double)j0 * atan2(zi, zr) - zi;
        const double e0r = m0 * cos(ph0), e0i = m0 * sin(ph0);
        // down to 0: E_{j-1} = E_j j conj(z) / |z|^2
        er = e0r;
        ei = e0i;
        put(j0, er, ei);
        for (int j = j0; j > 0; --j) {
            const double f = (double)j / az2;
            const double nr = (er * zr + ei * zi) * f, ni = (ei * zr - er * zi) * f;
            er = nr;
            ei = ni;
            put(j - 1, er, ei);
        }
        er = e0r;
        ei = e0i;
        for (int j = j0 + 1; j <= J; ++j) {
            const double nr = (er * zr - ei * zi) / j, ni = (er * zi + ei * zr) / j;
            er = nr;
            ei = ni;
            put(j, er, ei);
        }
    }
    // R_k = sum_{j > k} E_j, downwards from k = D-1; alpha^{-(k+1)} upwards
    // is replaced by its value at D-1 carried down by multiplying with alpha
    const double an = 1.0 + beta * beta;
    // alpha^{-D} by repeated multiplication with 1/alpha
    double pr = 1.0, pi = 0.0;
    const double ir = 1.0 / an, ii = -beta / an;  // 1 / alpha
    for (int k = 0; k < D; ++k) {
        const double nr = pr * ir - pi * ii, ni = pr * ii + pi * ir;
        pr = nr;
        pi = ni;
    }
    const double cph = cos(P.phi), sph = sin(P.phi);
    double Rr = tr, Ri = ti;  // R_{D-1}
    for (int k = D - 1; k >= 0; --k) {
        // c_k = scale Im(e^{i phi} alpha^{-(k+1)} R_k); here p = alpha^{-(k+1)}
        const double ar = pr * Rr - pi * Ri, ai = pr * Ri + pi * Rr;
        const double Ej_r = P.w[k], Ej_i = P.wi[k];
        if (P.split) {
            P.w[k] = P.scale * ar;
            P.wi[k] = P.scale * ai;
        } else {
            P.w[k] = P.scale * (sph * ar + cph * ai);
        }
        // R_{k-1} = R_k + E_k; alpha^{-k} = alpha^{-(k+1)} * alpha
        Rr += Ej_r;
        Ri += Ej_i;
        const double nr = pr * 1.0 - pi * beta, ni = pr * beta + pi * 1.0;
        pr = nr;
        pi = ni;
    }
}

template <int NX, bool TWO>
hipError_t pois_launch(const PoisEntry* tab, int count, int blocks, int pass, hipStream_t s) {
    k_pois2d<NX, TWO><<<blocks, BNT, 0, s>>>(tab, count, pass);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_pois2d(const PoisEntry* tab, int count, int total_blocks, int nx, int two,
                         int pass, hipStream_t s) {
    if (count <= 0 || total_blocks <= 0) return hipSuccess;
    switch (nx) {
        case 64: return two ? pois_launch<64, true>(tab, count, total_blocks, pass, s)
                            : pois_launch<64, false>(tab, count, total_blocks, pass, s);
        case 128: return two ? pois_launch<128, true>(tab, count, total_blocks, pass, s)
                             : pois_launch<128, false>(tab, count, total_blocks, pass, s);
        case 256: return two ? pois_launch<256, true>(tab, count, total_blocks, pass, s)
                             : pois_launch<256, false>(tab, count, total_blocks, pass, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pois_weights(const PoisWeights* tab, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    k_pois_weights<<<count, 64, 0, s>>>(tab);
    return hipGetLastError();
}

}  // namespace pxp
