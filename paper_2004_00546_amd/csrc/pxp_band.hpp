// Row-band layout shared by the 2D band kernels (RK4 marches and
// uniformised exponentials): 8 waves, wave w holds region rows 8w .. 8w+7
// of a 64-row region, lane l columns l*CPL .. l*CPL+CPL-1 (CPL = NX/64), so a
// wave row is a whole periodic grid row: x neighbours are the adjacent lanes
// (wrapping; wave-wide DPP rotates), y neighbours the same lane's registers
// except at the wave's first and last rows, which go through LDS.
#pragma once
#include "pxp_internal.hpp"
#include "pxp_device.hpp"

namespace pxp {
namespace {

constexpr int BW = 8;            // waves per workgroup
constexpr int BNT = BW * WAVE;   // threads per workgroup
constexpr int BRW = 8;           // region rows per wave
constexpr int BROWS = BW * BRW;  // region rows

__device__ __forceinline__ int find_entry(const Band2D* tab, int count, int b) {
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

// grid row of region row r of a band (periodic in y)
__device__ __forceinline__ int band_grow(int base, int r, int ny) {
    int g = (base + r) % ny;
    return g < 0 ? g + ny : g;
}

// The wave's BRW grid rows from its first one: consecutive, wrapping once
// at most (ny >= 16 > BRW).
__device__ __forceinline__ void wave_rows(int g0, int ny, int (&g)[BRW]) {
#pragma unroll
    for (int i = 0; i < BRW; ++i) {
        const int r = g0 + i;
        g[i] = r >= ny ? r - ny : r;
    }
}

// x neighbours of a lane's edge columns across the wave (the row is periodic
// and spans the wave): wave-wide DPP rotates, two 32-bit moves per double,
// every lane active.  wave_ror:1 hands lane l the value of lane l-1 (lane 0:
// lane 63), wave_rol:1 that of lane l+1 (lane 63: lane 0).
__device__ __forceinline__ double dpp_rot(double v, bool from_west) {
    const long long b = __double_as_longlong(v);
    const int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
    int rlo, rhi;
    if (from_west) {
        rlo = __builtin_amdgcn_update_dpp(0, lo, 0x13C, 0xF, 0xF, false);
        rhi = __builtin_amdgcn_update_dpp(0, hi, 0x13C, 0xF, 0xF, false);
    } else {
        rlo = __builtin_amdgcn_update_dpp(0, lo, 0x134, 0xF, 0xF, false);
        rhi = __builtin_amdgcn_update_dpp(0, hi, 0x134, 0xF, 0xF, false);
    }
    return __longlong_as_double((long long)(unsigned)rlo | ((long long)rhi << 32));
}
__device__ __forceinline__ double from_west(double v) { return dpp_rot(v, true); }
__device__ __forceinline__ double from_east(double v) { return dpp_rot(v, false); }

// CPL consecutive doubles of one grid row (16-byte loads and stores where
// CPL is even).
template <int CPL>
__device__ __forceinline__ void row_load(const double* __restrict__ p, double (&v)[CPL]) {
    if constexpr (CPL % 2 == 0) {
#pragma unroll
        for (int c = 0; c < CPL; c += 2) {
            const double2 x = *reinterpret_cast<const double2*>(p + c);
            v[c] = x.x;
            v[c + 1] = x.y;
        }
    } else {
#pragma unroll
        for (int c = 0; c < CPL; ++c) v[c] = p[c];
    }
}
template <int CPL>
__device__ __forceinline__ void row_store(double* __restrict__ p, const double (&v)[CPL]) {
    if constexpr (CPL % 2 == 0) {
#pragma unroll
        for (int c = 0; c < CPL; c += 2)
            *reinterpret_cast<double2*>(p + c) = make_double2(v[c], v[c + 1]);
    } else {
#pragma unroll
        for (int c = 0; c < CPL; ++c) p[c] = v[c];
    }
}

// Edge rows of the stage input through LDS (one slot: a barrier before the
// writes keeps them behind the previous stage's reads); returns the rows
// above the wave's first row and below its last row.
template <int NX, int CPL>
__device__ __forceinline__ void exchange_edges(double (*xch)[2][NX], const double (&Y)[BRW][CPL],
                                               int w, int cb, double (&up)[CPL],
                                               double (&dn)[CPL]) {
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        xch[w][0][cb + c] = Y[0][c];
        xch[w][1][cb + c] = Y[BRW - 1][c];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        up[c] = (w > 0) ? xch[w - 1][1][cb + c] : 0.0;
        dn[c] = (w < BW - 1) ? xch[w + 1][0][cb + c] : 0.0;
    }
}

}  // namespace
}  // namespace pxp
