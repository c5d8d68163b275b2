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
// region points per thread for rows of NX points: (16 + 2*16 rows) * NX / NT2
template <int NX>
constexpr int kpt() {
    return (BAND_ROWS + 4 * BAND_MAX_STEPS * 2) * NX / NT2;
}

// Band region of `rows` rows x NX columns; thread t owns column t % NX and
// rows t / NX + q * (NT2 / NX), q < KPT.  In LDS, region row r sits at row
// r + 1 with stride NX + 2: a zeroed pad row above and below, and the two
// periodic neighbour columns stored beside each row, so the stencil reads
// five fixed offsets from every point (the rows next to the pads are halo
// rows, whose results are discarded).
template <int NX>
struct Region {
    static constexpr int LD = NX + 2;
    static constexpr int RSTEP = NT2 / NX;
    int rows, col, r0;
    __device__ __forceinline__ int row(int q) const { return r0 + q * RSTEP; }
    __device__ __forceinline__ int idx(int q) const { return (row(q) + 1) * LD + col + 1; }
    // store v at region point q, with its periodic copy when on an edge
    __device__ __forceinline__ void put(double* X, int q, double v) const {
        const int i = idx(q);
        X[i] = v;
        if (col == 0) X[i + NX] = v;
        if (col == NX - 1) X[i - NX] = v;
    }
};

template <int NX>
__device__ __forceinline__ Region<NX> make_region(int H) {
    Region<NX> R;
    R.rows = BAND_ROWS + 2 * H;
    R.col = threadIdx.x % NX;
    R.r0 = threadIdx.x / NX;
    return R;
}

template <int NX>
__device__ __forceinline__ void zero_pads(double* X, const Region<NX>& R) {
    for (int c = threadIdx.x; c < Region<NX>::LD; c += NT2) {
        X[c] = 0.0;
        X[(R.rows + 1) * Region<NX>::LD + c] = 0.0;
    }
}

// Five-point stencil at LDS index i.
template <int NX>
__device__ __forceinline__ double sten(const double* X, int i, const Sten5& A) {
    constexpr int LD = Region<NX>::LD;
    return A.c * X[i] + A.w * X[i - 1] + A.e * X[i + 1] + A.s * X[i - LD] + A.n * X[i + LD];
}

// global row of band row r (periodic in y)
__device__ __forceinline__ int grow(int row0, int r, int ny) {
    int g = row0 + r;
    if (g < 0) g += ny;
    if (g >= ny) g -= ny;
    return g;
}

__device__ __forceinline__ int find_entry(const Band2D* tab, int count, int b) {
    int e = 0;
    while (e + 1 < count && tab[e + 1].blk0 <= b) ++e;
    return e;
}

template <int NX>
__global__ void __launch_bounds__(NT2)
k_band2d_fwd(const Band2D* __restrict__ tab, int count, int serial, int L) {
    extern __shared__ double X[];
    constexpr int KPT = kpt<NX>();
    const int b = blockIdx.x;
    const Band2D& d = tab[find_entry(tab, count, b)];
    constexpr int nx = NX;
    const int ny = d.ny, nb = ny / BAND_ROWS;
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
        // the initial state belongs to the first slice, the others start
        // from zero (eq. linInhomEqus)
        in = (item == 0) ? d.y0 : nullptr;
        out = d.out + (size_t)item * nn;
    }
    const int H = 4 * ns;
    const Region<NX> R = make_region<NX>(H);
    const int row0 = band * BAND_ROWS - H;
    zero_pads(X, R);
    double y[KPT], acc[KPT], Y[KPT], f[KPT];
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
        const int r = R.row(q);
        const int g = grow(row0, r, ny) * nx + R.col;
        y[q] = (r < R.rows && in) ? in[g] : 0.0;
        f[q] = (r < R.rows && d.F) ? d.F[g] : 0.0;
        acc[q] = 0.0;
        Y[q] = y[q];
    }
    const Sten5 A = d.A;
    const double dt = d.dt, h2 = 0.5 * dt, h6 = dt / 6.0;
    // the forcing sines of the block's steps at the stage times t, t + dt/2,
    // t + dt: one evaluation per value instead of one per thread and stage
    __shared__ double sn[12];
    if ((int)threadIdx.x < 3 * ns) {
        const int s = threadIdx.x / 3, v = threadIdx.x - 3 * (threadIdx.x / 3);
        const double tn = (double)(first + s) * dt;
        sn[threadIdx.x] = sin(d.omega * (tn + (v == 0 ? 0.0 : (v == 2 ? dt : h2))));
    }
    __syncthreads();
    for (int s = 0; s < ns; ++s) {
#pragma unroll 1
        for (int st = 0; st < 4; ++st) {
            const double sv = sn[3 * s + (st == 0 ? 0 : (st == 3 ? 2 : 1))];
            const double cw = (st == 0) ? 1.0 : 2.0;
            const double cy = (st == 2) ? dt : h2;
            __syncthreads();  // previous readers of X are done
#pragma unroll
            for (int q = 0; q < KPT; ++q)
                if (R.row(q) < R.rows) R.put(X, q, (st == 0) ? y[q] : Y[q]);
            __syncthreads();
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                const int r = R.row(q);
                if (r >= R.rows) continue;
                const double k = sten<NX>(X, R.idx(q), A) + sv * f[q];
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
        const int r = R.row(q);
        if (r >= H && r < H + BAND_ROWS) out[grow(row0, r, ny) * nx + R.col] = y[q];
    }
}

// Exact discrete adjoint of the RK4 march, backwards over the steps of
// launch L: per step, kbar_4 = dt/6 lam, Ybar_i = A^T kbar_i, kbar_{i-1} =
// b_{i-1} dt lam + c_i dt Ybar_i, lam += sum_i Ybar_i, Lam += s(t_i) kbar_i.
template <int NX>
__global__ void __launch_bounds__(NT2)
k_band2d_rev(const Band2D* __restrict__ tab, int count, int L) {
    extern __shared__ double X[];
    constexpr int KPT = kpt<NX>();
    const int b = blockIdx.x;
    const Band2D& d = tab[find_entry(tab, count, b)];
    constexpr int nx = NX;
    const int ny = d.ny;
    const int band = b - d.blk0;
    const int64_t left = d.n_t - 4 * (int64_t)L;
    if (left <= 0) return;
    const int ns = left < 4 ? (int)left : 4;
    const int64_t first = left - ns;
    const double* in = (L == 0) ? d.y0 : d.buf[L & 1];
    double* out = d.buf[(L + 1) & 1];
    const int H = 4 * ns;
    const Region<NX> R = make_region<NX>(H);
    const int row0 = band * BAND_ROWS - H;
    zero_pads(X, R);
    double lam[KPT], kb[KPT], nl[KPT], Lm[KPT];
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
        const int r = R.row(q);
        lam[q] = (r < R.rows) ? in[grow(row0, r, ny) * nx + R.col] : 0.0;
        Lm[q] = 0.0;
        nl[q] = 0.0;
        kb[q] = 0.0;
    }
    const Sten5 A = d.A;
    const double dt = d.dt, d6 = dt / 6.0, d3 = dt / 3.0, d2 = 0.5 * dt;
    // the forcing sines at the stage times, as in k_band2d_fwd
    __shared__ double sn[12];
    if ((int)threadIdx.x < 3 * ns) {
        const int s = threadIdx.x / 3, v = threadIdx.x - 3 * (threadIdx.x / 3);
        const double tn = (double)(first + s) * dt;
        sn[threadIdx.x] = sin(d.omega * (tn + (v == 0 ? 0.0 : (v == 2 ? dt : d2))));
    }
    __syncthreads();
    for (int s = ns - 1; s >= 0; --s) {
#pragma unroll
        for (int q = 0; q < KPT; ++q) kb[q] = d6 * lam[q];
        // stages 4, 3, 2, 1
#pragma unroll 1
        for (int st = 0; st < 4; ++st) {
            const double sv = sn[3 * s + (st == 0 ? 2 : (st == 3 ? 0 : 1))];
            const double bl = (st == 2) ? d6 : d3;  // weight of lam in the next kbar
            const double cy = (st == 0) ? dt : d2;  // weight of Ybar in the next kbar
            __syncthreads();
#pragma unroll
            for (int q = 0; q < KPT; ++q)
                if (R.row(q) < R.rows) R.put(X, q, kb[q]);
            __syncthreads();
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                const int r = R.row(q);
                if (r >= R.rows) continue;
                const double yb = sten<NX>(X, R.idx(q), A);
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
        const int r = R.row(q);
        if (r >= H && r < H + BAND_ROWS) {
            const int g = grow(row0, r, ny) * nx + R.col;
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

size_t band_lds(int nx) {
    return (size_t)(BAND_ROWS + 8 * BAND_MAX_STEPS + 2) * (nx + 2) * sizeof(double);
}

template <int NX>
hipError_t band_fwd(const Band2D* tab, int count, int total_blocks, int serial, int L,
                    hipStream_t s) {
    const size_t lds = band_lds(NX);
    (void)hipFuncSetAttribute((const void*)k_band2d_fwd<NX>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    k_band2d_fwd<NX><<<total_blocks, NT2, lds, s>>>(tab, count, serial, L);
    return hipGetLastError();
}

template <int NX>
hipError_t band_rev(const Band2D* tab, int count, int total_blocks, int L,
                    hipStream_t s) {
    const size_t lds = band_lds(NX);
    (void)hipFuncSetAttribute((const void*)k_band2d_rev<NX>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    k_band2d_rev<NX><<<total_blocks, NT2, lds, s>>>(tab, count, L);
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

hipError_t launch_apply5(const double* x, double* out, int nx, int ny, Sten5 op,
                         hipStream_t s) {
    const int n = nx * ny;
    if (n <= 0) return hipSuccess;
    k_apply5<<<(n + 255) / 256, 256, 0, s>>>(x, out, nx, ny, op);
    return hipGetLastError();
}

}  // namespace pxp
