// RK4 marches of the 2D periodic advection-diffusion problem (paper section
// 4.2) with the first-order upwind, five-point operator:
//   - the P inhomogeneous slices from zero data (eq. linInhomEqus), all
//     instances and slices of a call in one launch;
//   - the serial comparison march and its exact discrete adjoint.
//
// Workgroup layout: one workgroup advances BAND_ROWS full grid rows of one
// march by up to BAND_MAX_STEPS steps.  Rows are periodic in x, so the band
// only needs a halo in y: every stage application of the stencil consumes
// one halo row on each side, so a band of nsteps steps loads 4*nsteps extra
// rows above and below, recomputes them redundantly, and writes back only
// its own rows.  The stage input lives in LDS (neighbour reads), the state
// and the stage accumulators in registers.
#include "pxp_internal.hpp"
#include "pxp_device.hpp"

namespace pxp {
namespace {

constexpr int NT2 = 512;  // threads per band workgroup
// region points per thread: (16 + 2*16 rows) * 256 columns / 512 threads
constexpr int KPT = (BAND_ROWS + 4 * BAND_MAX_STEPS * 2) * 256 / NT2;

struct Region {
    int nx, rows, np, lnx;
    __device__ __forceinline__ int row(int p) const { return p >> lnx; }
    __device__ __forceinline__ int col(int p) const { return p & (nx - 1); }
};

// Five-point stencil at region point p from the stage input in LDS; rows
// outside the region repeat the edge row (those points are discarded).
__device__ __forceinline__ double sten(const double* X, const Region& R, int p,
                                       const Sten5& A) {
    const int r = R.row(p), c = R.col(p);
    const int base = p - c;
    const double xw = X[base + (c == 0 ? R.nx - 1 : c - 1)];
    const double xe = X[base + (c == R.nx - 1 ? 0 : c + 1)];
    const double xs = X[r == 0 ? p : p - R.nx];
    const double xn = X[r == R.rows - 1 ? p : p + R.nx];
    return A.c * X[p] + A.w * xw + A.e * xe + A.s * xs + A.n * xn;
}

__device__ __forceinline__ int find_entry(const Band2D* tab, int count, int b) {
    int e = 0;
    while (e + 1 < count && tab[e + 1].blk0 <= b) ++e;
    return e;
}

__device__ __forceinline__ int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

__global__ void __launch_bounds__(NT2)
k_band2d_fwd(const Band2D* __restrict__ tab, int count, int serial, int L) {
    extern __shared__ double X[];
    const int b = blockIdx.x, t = threadIdx.x;
    const Band2D d = tab[find_entry(tab, count, b)];
    const int nx = d.nx, ny = d.ny, nb = ny / BAND_ROWS;
    const int local = b - d.blk0;
    const int item = local / nb, band = local - item * nb;
    int ns;
    int64_t first;
    const double* in;
    double* out;
    const size_t nn = (size_t)nx * ny;
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
        in = d.y0;
        out = d.out + (size_t)item * nn;
    }
    const int H = 4 * ns;
    Region R{nx, BAND_ROWS + 2 * H, (BAND_ROWS + 2 * H) * nx, ilog2(nx)};
    const int row0 = band * BAND_ROWS - H;
    // global index of region point p
    auto gidx = [&](int p) {
        int gr = row0 + R.row(p);
        gr = ((gr % ny) + ny) % ny;
        return gr * nx + R.col(p);
    };
    double y[KPT], acc[KPT], Y[KPT];
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
        const int p = t + q * NT2;
        y[q] = (p < R.np && in) ? in[gidx(p)] : 0.0;
        acc[q] = 0.0;
        Y[q] = y[q];
    }
    const Sten5 A = d.A;
    const double dt = d.dt, h2 = 0.5 * dt, h6 = dt / 6.0;
    for (int s = 0; s < ns; ++s) {
        const double tn = (double)(first + s) * dt;
#pragma unroll 1
        for (int st = 0; st < 4; ++st) {
            const double sv = sin(d.omega * (tn + (st == 0 ? 0.0 : (st == 3 ? dt : h2))));
            const double cw = (st == 0) ? 1.0 : 2.0;
            const double cy = (st == 2) ? dt : h2;
            __syncthreads();  // previous readers of X are done
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                const int p = t + q * NT2;
                if (p < R.np) X[p] = (st == 0) ? y[q] : Y[q];
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                const int p = t + q * NT2;
                if (p >= R.np) continue;
                double k = sten(X, R, p, A);
                if (d.F || d.g0) {
                    const int g = gidx(p);
                    if (d.F) k += sv * d.F[g];
                    if (d.g0) k += d.g0[g];
                }
                if (st < 3) {
                    acc[q] += cw * k;
                    Y[q] = y[q] + cy * k;
                } else {
                    y[q] += h6 * (acc[q] + k);
                    acc[q] = 0.0;
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
        const int p = t + q * NT2;
        if (p >= R.np) continue;
        const int r = R.row(p);
        if (r >= H && r < H + BAND_ROWS) out[gidx(p)] = y[q];
    }
}

// Exact discrete adjoint of the RK4 march, backwards over the steps of
// launch L: per step, kbar_4 = dt/6 lam, Ybar_i = A^T kbar_i, kbar_{i-1} =
// b_{i-1} dt lam + c_i dt Ybar_i, lam += sum_i Ybar_i, Lam += s(t_i) kbar_i.
__global__ void __launch_bounds__(NT2)
k_band2d_rev(const Band2D* __restrict__ tab, int count, int L) {
    extern __shared__ double X[];
    const int b = blockIdx.x, t = threadIdx.x;
    const Band2D d = tab[find_entry(tab, count, b)];
    const int nx = d.nx, ny = d.ny;
    const int band = b - d.blk0;
    const int64_t left = d.n_t - 4 * (int64_t)L;
    if (left <= 0) return;
    const int ns = left < 4 ? (int)left : 4;
    const int64_t first = left - ns;
    const double* in = (L == 0) ? d.y0 : d.buf[L & 1];
    double* out = d.buf[(L + 1) & 1];
    const int H = 4 * ns;
    Region R{nx, BAND_ROWS + 2 * H, (BAND_ROWS + 2 * H) * nx, ilog2(nx)};
    const int row0 = band * BAND_ROWS - H;
    auto gidx = [&](int p) {
        int gr = row0 + R.row(p);
        gr = ((gr % ny) + ny) % ny;
        return gr * nx + R.col(p);
    };
    double lam[KPT], kb[KPT], nl[KPT], Lm[KPT];
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
        const int p = t + q * NT2;
        lam[q] = (p < R.np) ? in[gidx(p)] : 0.0;
        Lm[q] = 0.0;
        nl[q] = 0.0;
        kb[q] = 0.0;
    }
    const Sten5 A = d.A;
    const double dt = d.dt, d6 = dt / 6.0, d3 = dt / 3.0, d2 = 0.5 * dt;
    for (int s = ns - 1; s >= 0; --s) {
        const double tn = (double)(first + s) * dt;
#pragma unroll
        for (int q = 0; q < KPT; ++q) kb[q] = d6 * lam[q];
        // stages 4, 3, 2, 1
#pragma unroll 1
        for (int st = 0; st < 4; ++st) {
            const double sv = sin(d.omega * (tn + (st == 0 ? dt : (st == 3 ? 0.0 : d2))));
            const double bl = (st == 2) ? d6 : d3;  // weight of lam in the next kbar
            const double cy = (st == 0) ? dt : d2;  // weight of Ybar in the next kbar
            __syncthreads();
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                const int p = t + q * NT2;
                if (p < R.np) X[p] = kb[q];
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                const int p = t + q * NT2;
                if (p >= R.np) continue;
                const double yb = sten(X, R, p, A);
                Lm[q] += sv * kb[q];
                if (st < 3) {
                    nl[q] += yb;
                    kb[q] = bl * lam[q] + cy * yb;
                } else {
                    lam[q] += nl[q] + yb;
                    nl[q] = 0.0;
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
        const int p = t + q * NT2;
        if (p >= R.np) continue;
        const int r = R.row(p);
        if (r >= H && r < H + BAND_ROWS) {
            const int g = gidx(p);
            out[g] = lam[q];
            if (d.Lam) d.Lam[g] += Lm[q];
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

size_t band_lds(const Band2D* host_max_nx) {
    (void)host_max_nx;
    return (size_t)(BAND_ROWS + 8 * BAND_MAX_STEPS) * 256 * sizeof(double);
}

}  // namespace

hipError_t launch_band2d(const Band2D* tab, int count, int total_blocks, int serial,
                         int L, hipStream_t s) {
    if (count <= 0 || total_blocks <= 0) return hipSuccess;
    const size_t lds = band_lds(nullptr);
    (void)hipFuncSetAttribute((const void*)k_band2d_fwd,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    k_band2d_fwd<<<total_blocks, NT2, lds, s>>>(tab, count, serial, L);
    return hipGetLastError();
}

hipError_t launch_band2d_rev(const Band2D* tab, int count, int total_blocks, int L,
                             hipStream_t s) {
    if (count <= 0 || total_blocks <= 0) return hipSuccess;
    const size_t lds = band_lds(nullptr);
    (void)hipFuncSetAttribute((const void*)k_band2d_rev,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    k_band2d_rev<<<total_blocks, NT2, lds, s>>>(tab, count, L);
    return hipGetLastError();
}

hipError_t launch_apply5(const double* x, double* out, int nx, int ny, Sten5 op,
                         hipStream_t s) {
    const int n = nx * ny;
    if (n <= 0) return hipSuccess;
    k_apply5<<<(n + 255) / 256, 256, 0, s>>>(x, out, nx, ny, op);
    return hipGetLastError();
}

}  // namespace pxp
