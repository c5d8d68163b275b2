// C ABI and host engine: argument validation, workspace layout and the order
// of the launches that make up the direct solve, the adjoint solve and the
// full direct-adjoint loop (paper sections 2 and 3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/paraexp.h"
#include "pxp_internal.hpp"

namespace pxp {
namespace {

constexpr size_t ALIGN = 256;
constexpr int M_MAX_1D = 48;

inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
    size_t status;             // DevStatus
    size_t btab, ktab, t2d;    // batch tables: Burgers, Krylov, 2D marches
    size_t kchk, mtab;         // Magnus check: chains, estimate descriptors
    size_t ptab, pwt;          // uniformised exponentials: pass entries, weights
    size_t ptab_entries;       // capacity of the pass-entry table
    size_t rtab, rpart;        // batched cost/gradient: descriptors, partial sums
    size_t irep;               // per-instance statistics
    std::vector<size_t> base;  // per-instance region offset
    size_t total;
};

// Per-instance buffers (offsets relative to the instance region).
struct Inst {
    size_t F, g0, q0eff, slices, pieces, basis, qT, lamT, lam0, Lam, chain,
        ckpt, seg, nodes, sbuf0, sbuf1, aint, J, tbuf, wtab, ubuf;
    // integral cost: step sources, kept tree levels, corrected slice-start
    // states, Lambda shares (slices then tree pairs), cost partials, weight
    // tables of the adjoint tree
    size_t gsrc, lev, ebuf, islot, cpart, iwtab;
    // Burgers integral cost: hybrid scheme buffers
    size_t hstate, hmu, hseg, hbnd, haddq;
    // Burgers nonlinear Paraexp iteration
    size_t nst[2], nW, nv, nE, nq, naddq, ndesc;
    // Burgers: Magnus check node states (two samples x two half steps x two
    // vectors) and results (one step, two half steps per sample)
    size_t mnodes, mout, mdesc;
    size_t size;
};

int64_t grid_n(const pxp_problem& p) { return (int64_t)p.nx * (int64_t)p.ny; }

bool is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

Tri advdiff_tri(const pxp_problem& p) {
    const double h = p.L / p.nx;
    Tri A;
    A.lo = p.vx / (2.0 * h) + p.nu / (h * h);
    A.d = -2.0 * p.nu / (h * h);
    A.up = -p.vx / (2.0 * h) + p.nu / (h * h);
    return A;
}
Tri transpose(Tri A) {
    Tri B;
    B.lo = A.up;
    B.d = A.d;
    B.up = A.lo;
    return B;
}

// First-order upwind advection (vx, vy >= 0) and the five-point Laplacian.
Sten5 advdiff2d_sten(const pxp_problem& p) {
    const double hx = p.L / p.nx, hy = p.L / p.ny;
    Sten5 A;
    A.w = p.vx / hx + p.nu / (hx * hx);
    A.e = p.nu / (hx * hx);
    A.s = p.vy / hy + p.nu / (hy * hy);
    A.n = p.nu / (hy * hy);
    A.c = -p.vx / hx - p.vy / hy - 2.0 * p.nu / (hx * hx) - 2.0 * p.nu / (hy * hy);
    return A;
}
double sten_norm(const Sten5& A) {
    return std::fabs(A.c) + std::fabs(A.w) + std::fabs(A.e) + std::fabs(A.s) + std::fabs(A.n);
}
Sten5 transpose5(Sten5 A) {
    Sten5 B = A;
    B.w = A.e;
    B.e = A.w;
    B.s = A.n;
    B.n = A.s;
    return B;
}

// max |R(dt lambda)| <= 1 for RK4 over the exact eigenvalues of the 2D
// upwind operator (block circulant).
bool rk4_stable_advdiff2d(const pxp_problem& p) {
    const double hx = p.L / p.nx, hy = p.L / p.ny, dt = p.T / (double)p.n_steps;
    for (int ky = 0; ky < p.ny; ++ky) {
        const double ph = 2.0 * M_PI * ky / p.ny;
        for (int kx = 0; kx < p.nx; ++kx) {
            const double th = 2.0 * M_PI * kx / p.nx;
            const std::complex<double> lam =
                -p.vx / hx * (1.0 - std::polar(1.0, -th)) -
                p.vy / hy * (1.0 - std::polar(1.0, -ph)) +
                p.nu * (2.0 * std::cos(th) - 2.0) / (hx * hx) +
                p.nu * (2.0 * std::cos(ph) - 2.0) / (hy * hy);
            const std::complex<double> z = dt * lam;
            const std::complex<double> R = 1.0 + z + z * z / 2.0 + z * z * z / 6.0 +
                                           z * z * z * z / 24.0;
            if (std::abs(R) > 1.0 + 1e-12) return false;
        }
    }
    return true;
}

// max_k |R(dt lambda_k)| for RK4 over the exact eigenvalues of the 1D
// central advection-diffusion operator (circulant).
bool rk4_stable_advdiff1d(const pxp_problem& p) {
    const double h = p.L / p.nx, dt = p.T / (double)p.n_steps;
    for (int k = 0; k < p.nx; ++k) {
        const double th = 2.0 * M_PI * k / p.nx;
        const std::complex<double> lam(p.nu * (2.0 * std::cos(th) - 2.0) / (h * h),
                                       -p.vx * std::sin(th) / h);
        const std::complex<double> z = dt * lam;
        const std::complex<double> R = 1.0 + z + z * z / 2.0 + z * z * z / 6.0 +
                                       z * z * z * z / 24.0;
        if (std::abs(R) > 1.0 + 1e-12) return false;
    }
    return true;
}

// Krylov flavour of a problem.  AUTO takes shift-and-invert where a
// polynomial method would need many terms or substeps: when tau * rho,
// rho = 4 nu / h^2 + |c| / h the spectral radius bound of the diffusion and
// advection stencil and tau the longest exponential the call takes (the
// horizon for the linear pieces, half a slice for the Magnus factors),
// exceeds 64, and the grid allows the cyclic-reduction shape; otherwise the
// Taylor flavour.
bool use_si(const pxp_problem& p) {
    // 2D: named only (the Fourier solve; AUTO takes uniformisation)
    if (p.op == PXP_OP_ADVDIFF2D_UPWIND) return p.krylov == PXP_KRYLOV_SHIFT_INVERT;
    if (p.krylov == PXP_KRYLOV_SHIFT_INVERT) return true;
    if (p.krylov != PXP_KRYLOV_AUTO) return false;
    // Burgers: the Chebyshev chain kernel wherever it covers the grid (it
    // beats shift-and-invert also on the stiffest ragged instances, tau rho
    // about 1600)
    {
        int cb, cp;
        if (p.op == PXP_OP_BURGERS1D && cheb_chain_shape_pub(p.nx, &cb, &cp)) return false;
    }
    const double h = p.L / p.nx;
    const double rho = 4.0 * p.nu / (h * h) + std::fabs(p.vx) / h;
    const double tau = p.op == PXP_OP_BURGERS1D ? 0.5 * p.T / p.P : p.T;
    if (!(tau * rho > 64.0)) return false;
    int B, pt;
    if (!krylov_shape_pub(p.nx, p.kblock, &B, &pt)) return false;
    if (pt * B != p.nx || (B & (B - 1))) return false;
    return p.op == PXP_OP_BURGERS1D || (is_pow2(p.nx) && p.nx >= 64);
}

// 2D exponentials by uniformisation: named, or AUTO for the adjoint piece and
// for the chain and tree schedules of the direct pieces (the classic
// schedule's independent long pieces stay with the Taylor flavour).
bool uniform_direct(const pxp_problem& p) {
    if (p.op != PXP_OP_ADVDIFF2D_UPWIND) return false;
    if (p.krylov == PXP_KRYLOV_UNIFORM) return true;
    return p.krylov == PXP_KRYLOV_AUTO && p.sched != PXP_SCHED_CLASSIC;
}
bool uniform_adjoint(const pxp_problem& p) {
    if (p.op != PXP_OP_ADVDIFF2D_UPWIND) return false;
    return p.krylov == PXP_KRYLOV_UNIFORM || p.krylov == PXP_KRYLOV_AUTO;
}

// The RK4 stability checks above visit every Fourier mode of the grid
// (65536 for a 256 x 256 grid): their results are remembered per operator,
// grid, horizon and step count, so repeated calls on the same problem pay
// for the check once.  The cache is process-wide and bounded.
using StabKey = std::tuple<int, int, int, double, double, double, double, double, int64_t>;
std::mutex g_stab_mu;
std::map<StabKey, bool> g_stab;

bool rk4_stable_cached(const pxp_problem& p) {
    const StabKey k{p.op, p.nx, p.ny, p.L, p.vx, p.vy, p.nu, p.T, p.n_steps};
    {
        std::lock_guard<std::mutex> lock(g_stab_mu);
        auto it = g_stab.find(k);
        if (it != g_stab.end()) return it->second;
    }
    const bool ok = p.op == PXP_OP_ADVDIFF2D_UPWIND ? rk4_stable_advdiff2d(p)
                                                    : rk4_stable_advdiff1d(p);
    std::lock_guard<std::mutex> lock(g_stab_mu);
    if (g_stab.size() >= 4096) g_stab.clear();
    g_stab[k] = ok;
    return ok;
}

// Taylor flavour: named, or AUTO where neither shift-and-invert nor
// uniformisation is taken.
// Chebyshev flavour: the time-varying Burgers chains on the grids its
// chain kernel covers, named or AUTO.
bool use_cheb(const pxp_problem& p) {
    if (p.op != PXP_OP_BURGERS1D) return false;
    int cb, cp;
    if (!cheb_chain_shape_pub(p.nx, &cb, &cp)) return false;
    return p.krylov == PXP_KRYLOV_CHEBYSHEV || p.krylov == PXP_KRYLOV_AUTO;
}

bool use_taylor(const pxp_problem& p) {
    if (p.krylov == PXP_KRYLOV_TAYLOR) return true;
    return p.krylov == PXP_KRYLOV_AUTO && !use_si(p) && !uniform_direct(p) && !use_cheb(p);
}

// The Krylov kernels' workgroup shape for this problem exists, fits in LDS,
// reads two consecutive points per 16-byte load (even n once a thread owns
// more than one point) and, for shift-and-invert, covers the grid exactly.
bool krylov_fits(const pxp_problem& p, bool si) {
    int B, pt;
    if (!krylov_shape_pub(p.nx, p.kblock, &B, &pt)) return false;
    if (pt >= 2 && (p.nx & 1)) return false;
    if (si && (pt * B != p.nx || (B & (B - 1)))) return false;
    return krylov1d_lds_bytes(p.nx, p.m, B, si) <= 160 * 1024;
}

pxp_status validate(const pxp_problem& p) {
    if (p.nx < 2 || p.ny < 1 || p.n_steps < 1 || p.P < 1 || p.T <= 0.0 ||
        p.L <= 0.0 || p.nu < 0.0 || p.K < 0 || !std::isfinite(p.T) ||
        !std::isfinite(p.nu) || !std::isfinite(p.vx))
        return PXP_EINVAL;
    if (p.n_steps % p.P != 0) return PXP_EINVAL;
    if (p.ctrl != PXP_CTRL_FORCING && p.ctrl != PXP_CTRL_IC) return PXP_EINVAL;
    if (p.krylov != PXP_KRYLOV_POLY && p.krylov != PXP_KRYLOV_SHIFT_INVERT &&
        p.krylov != PXP_KRYLOV_AUTO && p.krylov != PXP_KRYLOV_TAYLOR &&
        p.krylov != PXP_KRYLOV_UNIFORM && p.krylov != PXP_KRYLOV_CHEBYSHEV)
        return PXP_EINVAL;
    if (p.sched != PXP_SCHED_CLASSIC && p.sched != PXP_SCHED_CHAIN && p.sched != PXP_SCHED_TREE)
        return PXP_EINVAL;
    if (p.krylov == PXP_KRYLOV_UNIFORM && p.op != PXP_OP_ADVDIFF2D_UPWIND) return PXP_EUNSUPPORTED;
    if (p.krylov == PXP_KRYLOV_CHEBYSHEV) {
        // the flavour's chain kernel: Burgers grids it covers in whole chunks
        int cb, cp;
        if (p.op != PXP_OP_BURGERS1D || !cheb_chain_shape_pub(p.nx, &cb, &cp))
            return PXP_EUNSUPPORTED;
    }
    if (p.sched == PXP_SCHED_TREE && !uniform_direct(p)) return PXP_EUNSUPPORTED;
    if (p.prec != PXP_FP64 && p.prec != PXP_FP32_BULK) return PXP_EINVAL;
    if ((p.flags & ~(PXP_FLAG_ABSORBED_ADJOINT | PXP_FLAG_INTEGRAL_COST |
                     PXP_FLAG_NL_PARAEXP)) ||
        p.kblock < 0 || p.block < 0)
        return PXP_EINVAL;
    if ((p.flags & PXP_FLAG_ABSORBED_ADJOINT) && p.op != PXP_OP_ADVDIFF1D) return PXP_EUNSUPPORTED;
    if (p.op == PXP_OP_ADVDIFF1D) {
        if (p.ny != 1) return PXP_EINVAL;
        if (p.m < 1 || p.m > M_MAX_1D) return PXP_EUNSUPPORTED;
        int b, pt;
        if (!march_shape(p.nx, p.block, &b, &pt)) return PXP_EUNSUPPORTED;
        // cyclic reduction: n a power of two, every thread of a 64-wide
        // multiple owning whole points
        if (use_si(p) && (!is_pow2(p.nx) || p.nx < 64)) return PXP_EUNSUPPORTED;
        if (!(p.krylov_tol > 0.0)) return PXP_EINVAL;
        if (!krylov_fits(p, use_si(p))) return PXP_EUNSUPPORTED;
        if (!rk4_stable_cached(p)) return PXP_EUNSTABLE_DT;
        return PXP_OK;
    }
    if (p.op == PXP_OP_BURGERS1D) {
        if (p.ny != 1) return PXP_EINVAL;
        if (p.ctrl != PXP_CTRL_IC) return PXP_EUNSUPPORTED;
        int b, pt;
        if (!march_shape(p.nx, p.block, &b, &pt)) return PXP_EUNSUPPORTED;
        if (p.ckpt_every < 1 || p.n_steps % p.ckpt_every) return PXP_EINVAL;
        if (p.m < 1 || p.m > M_MAX_1D) return PXP_EUNSUPPORTED;
        if (!(p.krylov_tol > 0.0)) return PXP_EINVAL;
        if (!krylov_fits(p, use_si(p))) return PXP_EUNSUPPORTED;
        // diffusion part of the spectrum on the negative real axis
        const double h = p.L / p.nx, dt = p.T / (double)p.n_steps;
        if (dt * 4.0 * p.nu / (h * h) > 2.785) return PXP_EUNSTABLE_DT;
        return PXP_OK;
    }
    if (p.op == PXP_OP_ADVDIFF2D_UPWIND) {
        // band marches and uniformised exponentials: power-of-two rows of
        // 64..256 points, whole bands of 16 rows (at most 4 steps per slice:
        // checked per method); streamed Krylov: 2048-point multiples,
        // polynomial, Taylor or shift-and-invert flavour (the last on
        // power-of-two grids of at most 256 x 256, for the Fourier solve); FP64
        if (p.nx < 64 || p.nx > 256 || !is_pow2(p.nx)) return PXP_EUNSUPPORTED;
        if (p.ny < BAND_ROWS || p.ny % BAND_ROWS) return PXP_EUNSUPPORTED;
        if (p.vx < 0.0 || p.vy < 0.0 || !std::isfinite(p.vy)) return PXP_EUNSUPPORTED;
        if (p.prec != PXP_FP64) return PXP_EUNSUPPORTED;
        if (use_si(p) && !fft2_grid(p.nx, p.ny)) return PXP_EUNSUPPORTED;
        if (p.krylov == PXP_KRYLOV_UNIFORM && p.sched == PXP_SCHED_CLASSIC)
            return PXP_EUNSUPPORTED;
        if (!uniform_direct(p) || !uniform_adjoint(p)) {
            if (grid_n(p) % (2 * KRYLOV2D_BLOCK)) return PXP_EUNSUPPORTED;
            if (p.m < 1 || krylov2d_lds_bytes(p.m, use_si(p)) > 160 * 1024)
                return PXP_EUNSUPPORTED;
            // the Taylor flavour keeps four vectors in the basis region
            if (use_taylor(p) && p.m < 3) return PXP_EUNSUPPORTED;
        }
        if (!(p.krylov_tol > 0.0)) return PXP_EINVAL;
        if (!rk4_stable_cached(p)) return PXP_EUNSTABLE_DT;
        return PXP_OK;
    }
    return PXP_EINVAL;
}

// ---- uniformisation: terms, Poisson tails, plans ---------------------------

// Smallest D with the Poisson tail P(X >= D) <= tol (X of mean lam); *est
// receives that tail.  Weights in log form, tail summed from the far end.
int pois_terms_uncached(double lam, double tol, double* est);

// pois_terms is called for every job of every call; its result depends on
// (lam, tol) only and is remembered (process-wide, bounded).
std::mutex g_pois_mu;
std::map<std::pair<double, double>, std::pair<int, double>> g_pois;

int pois_terms(double lam, double tol, double* est) {
    const std::pair<double, double> k{lam, tol};
    {
        std::lock_guard<std::mutex> lock(g_pois_mu);
        auto it = g_pois.find(k);
        if (it != g_pois.end()) {
            if (est) *est = it->second.second;
            return it->second.first;
        }
    }
    double e = 0.0;
    const int D = pois_terms_uncached(lam, tol, &e);
    std::lock_guard<std::mutex> lock(g_pois_mu);
    if (g_pois.size() >= 4096) g_pois.clear();
    g_pois[k] = {D, e};
    if (est) *est = e;
    return D;
}

int pois_terms_uncached(double lam, double tol, double* est) {
    if (!(lam > 0.0)) {
        if (est) *est = 0.0;
        return 1;
    }
    const int K = (int)(lam + 40.0 * std::sqrt(lam) + 80.0);
    std::vector<long double> pk(K + 1);
    const long double ll = std::log((long double)lam);
    for (int k = 0; k <= K; ++k)
        pk[k] = std::exp((long double)k * ll - (long double)lam - std::lgamma((long double)k + 1.0L));
    long double tail = 0.0L;
    int D = K + 1;
    double e = 0.0;
    for (int k = K; k >= 1; --k) {
        tail += pk[k];  // P(X >= k)
        if (tail > (long double)tol) break;
        D = k;
        e = (double)tail;
    }
    if (est) *est = e;
    return D;
}

// Largest Poisson parameter of one uniformised adjoint exponential of the
// terminal-cost piece, split into substeps beyond (its integral weights are
// formed by a recurrence from e^{-lam} up to this size).
constexpr double POIS_LMAX = 600.0;
// Largest Poisson parameter of one piece of the integral-cost adjoint tree
// (weights in log form beyond POIS_LMAX; their table is formed by one thread
// in time proportional to lam).
constexpr double POIS_LMAX_TREE = 4096.0;

double uniform_mu(const Sten5& A) { return -A.c; }
Sten5 uniform_N(const Sten5& A, double mu) {
    Sten5 N;
    N.c = 1.0 + A.c / mu;
    N.w = A.w / mu;
    N.e = A.e / mu;
    N.s = A.s / mu;
    N.n = A.n / mu;
    return N;
}
double uniform_tail_tol(const pxp_problem& p) { return 1e-2 * p.krylov_tol; }

// The adjoint piece over [0, T] by uniformisation: nsub equal substeps of
// Poisson parameter lam <= POIS_LMAX, D terms each.
struct AdjPlan {
    int nsub, D;
    double h, lam, est;
};
AdjPlan adj_plan(const pxp_problem& p) {
    AdjPlan a{};
    const double mu = uniform_mu(advdiff2d_sten(p));
    a.nsub = std::max(1, (int)std::ceil(mu * p.T / POIS_LMAX));
    a.h = p.T / a.nsub;
    a.lam = mu * a.h;
    a.D = pois_terms(a.lam, uniform_tail_tol(p), &a.est);
    return a;
}

// ---- the pairwise tree over the slice ranges --------------------------------

// Level 0 holds the P slices; level l pairs ranges 2j and 2j+1 of level l-1
// (an odd last range is carried up alone); the last level holds the root.
// Every range of a level but its last spans 2^l slices, so the pairs of a
// level have at most two shapes.
struct TNode {
    int start, size;  // slice range [start, start + size)
};
using TShape = std::vector<std::vector<TNode>>;

TShape tree_shape(int P) {
    TShape lv(1);
    for (int q = 0; q < P; ++q) lv[0].push_back({q, 1});
    while (lv.back().size() > 1) {
        std::vector<TNode> nx;
        {
            const std::vector<TNode>& c = lv.back();
            const size_t pairs = c.size() / 2;
            for (size_t j = 0; j < pairs; ++j)
                nx.push_back({c[2 * j].start, c[2 * j].size + c[2 * j + 1].size});
            if (c.size() & 1) nx.push_back(c.back());
        }
        lv.push_back(nx);
    }
    return lv;
}

// vectors of levels 1 .. depth kept one after the other
size_t tree_kept_vectors(const TShape& sh) {
    size_t v = 0;
    for (size_t l = 1; l < sh.size(); ++l) v += sh[l].size();
    return v;
}

bool icost(const pxp_problem& p) { return (p.flags & PXP_FLAG_INTEGRAL_COST) != 0; }
bool nlpx(const pxp_problem& p) { return (p.flags & PXP_FLAG_NL_PARAEXP) != 0; }
int nl_iters(const pxp_problem& p) { return p.nl_iters > 0 ? p.nl_iters : 8; }
int nl_slices(const pxp_problem& p) { return p.nl_slices > 0 ? p.nl_slices : p.P; }

// Largest Poisson parameter of the integral-cost adjoint tree: the pair at
// the root, whose left half spans the most slices.
double icost_max_lam(const pxp_problem& p) {
    if (p.P < 2) return 0.0;
    const TShape sh = tree_shape(p.P);
    const int left = sh[sh.size() - 2][0].size;
    return uniform_mu(transpose5(advdiff2d_sten(p))) * (p.T / p.P) * left;
}

// Weight tables of the adjoint tree: at most two pair shapes per level, two
// tables of D doubles each, D at most that of the largest piece.
size_t icost_wtab_doubles(const pxp_problem& p) {
    if (p.P < 2) return 1;
    const size_t depth = tree_shape(p.P).size() - 1;
    const int D = pois_terms(icost_max_lam(p), uniform_tail_tol(p), nullptr);
    return 2 * depth * 2 * (size_t)D;
}
size_t icost_wtab_count(const pxp_problem& p) {
    return p.P < 2 ? 0 : 2 * (tree_shape(p.P).size() - 1);
}

// Adjoint slices of the hybrid scheme for the Burgers integral cost
// (section 3.3): bounds T_n = T (1 - r^n) / (1 - r^N), r = k / (k + 1)
// (eq. nonEquiP; k = 0: equal slices), in steps rounded to multiples of
// L = lcm(S, c) (S = n_steps / P the Magnus macro step, c the checkpoint
// interval: the slices start on checkpoints, the chain adds their end states
// between macro steps); bounds that coincide after rounding merge.  Returns
// 0 = a_0 < a_1 < ... < a_N = n_steps.
int64_t gcd64(int64_t a, int64_t b) { return b == 0 ? a : gcd64(b, a % b); }
std::vector<int64_t> hyb_bounds(const pxp_problem& p) {
    const int64_t S = p.n_steps / p.P, c = p.ckpt_every;
    const int64_t L = S / gcd64(S, c) * c, U = p.n_steps / L;
    const int64_t N = std::min<int64_t>(p.hyb_slices > 0 ? p.hyb_slices : p.P, U);
    const double r = p.hyb_k / (p.hyb_k + 1.0);
    std::vector<int64_t> b{0};
    for (int64_t i = 1; i < N; ++i) {
        const double f = p.hyb_k > 0.0 ? (1.0 - std::pow(r, (double)i)) / (1.0 - std::pow(r, (double)N))
                                        : (double)i / (double)N;
        const int64_t a = std::llround(f * (double)U) * L;
        if (a > b.back() && a < p.n_steps) b.push_back(a);
    }
    b.push_back(p.n_steps);
    return b;
}
int hyb_group(const pxp_problem& p) { return p.hyb_group > 0 ? p.hyb_group : 4; }

pxp_status validate_icost(const pxp_problem& p) {
    if (p.hyb_slices < 0 || p.hyb_group < 0 || !(p.hyb_k >= 0.0) || !std::isfinite(p.hyb_k))
        return PXP_EINVAL;
    if (p.nl_iters < 0 || p.nl_slices < 0 || !(p.nl_tol >= 0.0) || !std::isfinite(p.nl_tol))
        return PXP_EINVAL;
    if (p.n_steps % nl_slices(p)) return PXP_EINVAL;
    if (nlpx(p)) {
        // the iteration of section 3.2: Burgers, FP64, terminal cost, at
        // least four steps (the march's stage layout)
        if (p.op != PXP_OP_BURGERS1D || p.prec != PXP_FP64 || icost(p)) return PXP_EUNSUPPORTED;
    }
    if (!icost(p)) return PXP_OK;
    if (p.op == PXP_OP_BURGERS1D) {
        // the serial march's state passes between launches as FP64
        if (p.prec != PXP_FP64) return PXP_EUNSUPPORTED;
        return PXP_OK;
    }
    if (p.op != PXP_OP_ADVDIFF2D_UPWIND) return PXP_EUNSUPPORTED;
    if (!uniform_direct(p) || !uniform_adjoint(p) || p.sched != PXP_SCHED_TREE)
        return PXP_EUNSUPPORTED;
    if (icost_max_lam(p) > POIS_LMAX_TREE) return PXP_EUNSUPPORTED;
    return PXP_OK;
}

Inst inst_layout(const pxp_problem& p) {
    const size_t n = (size_t)grid_n(p), d = sizeof(double);
    const size_t P = (size_t)p.P, m = (size_t)p.m;
    Inst L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes);
        return o;
    };
    L.F = take(n * d);
    L.g0 = take(n * d);
    L.q0eff = take(n * d);
    L.qT = take(n * d);
    L.lamT = take(n * d);
    L.lam0 = take(n * d);
    L.Lam = take(n * d);
    L.chain = take(n * d);
    L.J = take(d);
    if (p.op == PXP_OP_ADVDIFF1D) {
        const bool absorbed = (p.flags & PXP_FLAG_ABSORBED_ADJOINT) != 0;
        L.slices = take(P * n * d);
        L.pieces = take((P > 1 ? P - 1 : 1) * n * d);
        const size_t npar = ((p.sched == PXP_SCHED_CLASSIC || absorbed) && P > 1) ? P - 1 : 1;
        L.basis = take(npar * (m + 1) * n * d);
        // absorbed adjoint: the slices' and the pieces' integrals
        if (absorbed) L.aint = take((2 * P - 1) * n * d);
    }
    if (p.op == PXP_OP_ADVDIFF2D_UPWIND) {
        L.slices = take(P * n * d);
        const bool ud = uniform_direct(p), ua = uniform_adjoint(p);
        const bool classic = p.sched == PXP_SCHED_CLASSIC && P > 1;
        // tree: the levels alternate between the slices and these (P+1)/2
        // vectors; chain: two vectors in turn
        const size_t half = (P + 1) / 2;
        const size_t np = ud ? (p.sched == PXP_SCHED_TREE ? half : 2) : (classic ? P - 1 : 1);
        L.pieces = take(np * n * d);
        if (!ud || !ua) L.basis = take(((!ud && classic) ? P - 1 : 1) * (m + 1) * n * d);
        // term vectors of multi-pass exponentials, two per job (the
        // adjoint's single piece needs two)
        L.tbuf = take(2 * (ud ? std::max(np, (size_t)1) : 1) * n * d);
        if (ua) {
            const AdjPlan ap = adj_plan(p);
            L.wtab = take((size_t)ap.nsub * 2 * ap.D * d);
            L.ubuf = take(3 * n * d);
        }
        L.sbuf0 = take(n * d);
        L.sbuf1 = take(n * d);
        if (icost(p)) {
            L.gsrc = take(((size_t)p.n_steps + 1) * n * d);
            L.lev = take(std::max(tree_kept_vectors(tree_shape(p.P)), (size_t)1) * n * d);
            L.ebuf = take((P > 1 ? P - 1 : 1) * n * d);
            L.islot = take((2 * P - 1) * n * d);
            L.cpart = take(P * (size_t)(p.ny / BAND_ROWS) * d);
            L.iwtab = take(icost_wtab_doubles(p) * d);
        }
    }
    if (p.op == PXP_OP_BURGERS1D) {
        const size_t c = (size_t)p.ckpt_every;
        L.ckpt = take(((size_t)p.n_steps / c + 1) * n * d);
        L.seg = take(c * n * d);
        L.nodes = take(2 * P * n * d);
        L.mnodes = take(8 * n * d);
        L.mout = take(4 * n * d);
        L.mdesc = take(sizeof(MagnusCheck));
        if (nlpx(p)) {
            // two generations of stage states, the slices' averaged states,
            // their end states, the corrected slice starts, the
            // previous q(T), the chain's addition table, the change check
            L.nst[0] = take(4 * (size_t)p.n_steps * n * d);
            L.nst[1] = take(4 * (size_t)p.n_steps * n * d);
            const size_t Pn = (size_t)nl_slices(p);
            L.nW = take(Pn * n * d);
            L.nv = take(Pn * n * d);
            L.nE = take(Pn * n * d);
            L.nq = take(n * d);
            L.naddq = take(Pn * sizeof(int));
            L.ndesc = take(sizeof(NlState));
        }
        if (icost(p)) {
            // the march's running state, the hybrid adjoint slices' end
            // states and segment scratch, cost partials, and the slice
            // bounds and chain additions (device tables); the step sources
            // are formed from the states the reverse sweeps recompute
            const size_t ns = hyb_bounds(p).size() - 1;
            L.hstate = take(n * d);
            L.hmu = take(ns * n * d);
            L.hseg = take(ns * c * n * d);
            L.cpart = take(std::max(ns, (size_t)1) * d);
            L.hbnd = take((ns + 1) * sizeof(int64_t));
            L.haddq = take(ns * sizeof(int));
        }
        // basis, then the shift-and-invert factors of the time-varying
        // operator (5 n + 5 B doubles, B <= 512)
        L.basis = take(((m + 6) * n + 5 * 512) * d);
    }
    L.size = off;
    return L;
}

Layout layout(const pxp_problem* pb, int batch) {
    Layout Ly;
    size_t off = 0;
    Ly.status = off;
    off += align_up(sizeof(DevStatus));
    // Burgers descriptors: the instances, then two Magnus-check node jobs
    // per instance
    Ly.btab = off;
    off += align_up((size_t)batch * 3 * sizeof(BurgersDesc));
    Ly.ktab = off;
    off += align_up((size_t)batch * sizeof(KrylovArgs));
    Ly.kchk = off;
    off += align_up((size_t)batch * 4 * sizeof(KrylovArgs));
    Ly.mtab = off;
    off += align_up((size_t)batch * sizeof(MagnusCheck));
    Ly.t2d = off;
    off += align_up((size_t)batch * sizeof(Band2D));
    // at most four entries per instance in one pass launch (pairs of two
    // lengths, a pass-through, or the adjoint's piece)
    Ly.ptab = off;
    Ly.ptab_entries = (size_t)batch * 8;
    off += align_up(Ly.ptab_entries * sizeof(PoisEntry));
    size_t nw = 0;
    for (int i = 0; i < batch; ++i) {
        if (uniform_adjoint(pb[i])) nw += (size_t)adj_plan(pb[i]).nsub;
        if (icost(pb[i])) nw += icost_wtab_count(pb[i]);
    }
    Ly.pwt = off;
    off += align_up(nw * sizeof(PoisWeights));
    Ly.rtab = off;
    off += align_up((size_t)batch * sizeof(RedDesc));
    size_t np = 0;
    for (int i = 0; i < batch; ++i)
        np += (size_t)(pb[i].K + 1) * (size_t)((grid_n(pb[i]) + RED_CHUNK - 1) / RED_CHUNK);
    Ly.rpart = off;
    off += align_up(np * sizeof(double));
    Ly.irep = off;
    off += align_up((size_t)batch * sizeof(InstStat));
    for (int i = 0; i < batch; ++i) {
        Ly.base.push_back(off);
        off += inst_layout(pb[i]).size;
    }
    Ly.total = off;
    return Ly;
}

// The Paraexp path marches each 2D slice in one band launch of at most
// BAND_MAX_STEPS steps.
pxp_status check_method(const pxp_problem* pb, int batch, int method) {
    if (method != PXP_METHOD_PARAEXP) return PXP_OK;
    for (int i = 0; i < batch; ++i)
        if (pb[i].op == PXP_OP_ADVDIFF2D_UPWIND && pb[i].n_steps / pb[i].P > BAND_MAX_STEPS)
            return PXP_EUNSUPPORTED;
    return PXP_OK;
}

pxp_status check_all(const pxp_problem* pb, int batch) {
    if (batch < 0 || (batch > 0 && !pb)) return PXP_EINVAL;
    for (int i = 0; i < batch; ++i) {
        pxp_status s = validate(pb[i]);
        if (s == PXP_OK) s = validate_icost(pb[i]);
        if (s != PXP_OK) return s;
    }
    return PXP_OK;
}

#define HIPCHK(x)                               \
    do {                                        \
        if ((x) != hipSuccess) return PXP_EHIP; \
    } while (0)

// ---- side stream: independent launch groups of one phase run concurrently --
// One non-blocking stream (default priority) and two events per device,
// created by pxp_workspace_init, outside any stream capture.  A call forks
// onto the side stream with an event recorded on its own stream and joins
// back with another; a stream capture records both as graph dependencies.
// The enqueue of a fork/join is serialised by a mutex so that concurrent
// host threads never interleave the event records and waits.
struct SideStream {
    hipStream_t st = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
constexpr int MAX_DEVICES = 64;
static std::mutex g_side_mu;
static SideStream g_side[MAX_DEVICES];

static void side_init() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return;
    std::lock_guard<std::mutex> lock(g_side_mu);
    SideStream& ss = g_side[dev];
    if (ss.st) return;
    hipStream_t st = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
    if (hipEventCreateWithFlags(&a, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b, hipEventDisableTiming) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        (void)hipStreamDestroy(st);
        return;
    }
    ss.st = st;
    ss.fork = a;
    ss.join = b;
}

// Optional launch timing: when enabled, every launch of a kernel class is
// bracketed by two events recorded on the launch stream.  Host-side state,
// not thread-safe; meant for benchmarks and profiling runs only.
struct Profiler {
    bool on = false;
    struct Rec {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};
Profiler g_prof;

struct ProfScope {
    int cls;
    hipStream_t s;
    hipEvent_t b = nullptr;
    ProfScope(int c, hipStream_t st) : cls(c), s(st) {
        if (!g_prof.on) return;
        hipEvent_t a = g_prof.get();
        b = g_prof.get();
        if (!a || !b) return;
        hipEventRecord(a, s);
        g_prof.recs.push_back({cls, a, b});
    }
    ~ProfScope() {
        if (g_prof.on && b) hipEventRecord(b, s);
    }
};

struct Ctx {
    const pxp_problem& p;
    char* base;
    Inst L;
    DevStatus* st;
    hipStream_t s;
    InstStat* irep;
    double* at(size_t off) const { return reinterpret_cast<double*>(base + off); }
    int n() const { return (int)grid_n(p); }
    double dt() const { return p.T / (double)p.n_steps; }
    int fp32() const { return p.prec == PXP_FP32_BULK ? 1 : 0; }
};

// Largest scaled norm theta for which the Taylor remainder bound
// theta^(d+1) e^theta / (d+1)! stays below tol (bisection in log form).
double taylor_theta(int d, double tol) {
    const double lt = std::log(tol), lf = std::lgamma((double)d + 2.0);
    double lo = 1e-6, hi = 100.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if ((d + 1) * std::log(mid) + mid - lf <= lt)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

constexpr int TAYLOR_DEG = 40;

KrylovArgs kargs(const Ctx& c, Tri op) {
    KrylovArgs a{};
    a.taylor = use_taylor(c.p) ? 1 : 0;
    a.cheb = use_cheb(c.p) ? 1 : 0;
    a.tdeg = TAYLOR_DEG;
    a.theta = taylor_theta(TAYLOR_DEG, c.p.krylov_tol);
    a.anorm = std::fabs(op.lo) + std::fabs(op.d) + std::fabs(op.up);
    a.si = use_si(c.p) ? 1 : 0;
    a.n = c.n();
    a.m = c.p.m;
    a.tol = c.p.krylov_tol;
    // shift gamma = gamma_frac tau: 0.2 in 1D; the 2D upwind operator's
    // advection reaches further into the complex plane and its spaces
    // converge fastest near 0.05 (a random vector on a 64 x 64 grid,
    // tau = 0.7: relative error 6e-11 at dimension 28, against 4e-6 at 0.2)
    a.gamma_frac = (c.p.si_gamma > 0.0) ? c.p.si_gamma
                                        : (c.p.op == PXP_OP_ADVDIFF2D_UPWIND ? 0.05 : 0.2);
    a.op = op;
    a.basis = c.at(c.L.basis);
    a.status = c.st;
    a.irep = c.irep;
    a.fp32 = c.fp32();
    return a;
}

// Direct solve of one linear 1D instance: q0 (device, nullable), F
// (nullable) -> qT.
pxp_status direct_lin1d(const Ctx& c, const double* q0, const double* F,
                        double* qT, int method) {
    const int n = c.n();
    const Tri A = advdiff_tri(c.p);
    const double* g0 = nullptr;
    if (q0) {
        // IC shift q~ = q - q0: the source gains A q0 (eq. linzero)
        HIPCHK(launch_apply_tri(q0, c.at(c.L.g0), n, A, c.s));
        g0 = c.at(c.L.g0);
    }
    if (method == PXP_METHOD_SERIAL) {
        ProfScope ps(PXP_K_SERIAL_DIRECT, c.s);
        HIPCHK(launch_rk4_lin1d(F, nullptr, q0, qT, n, 1, c.p.n_steps, c.dt(),
                                c.p.omega, A, c.p.block, c.fp32(), c.s));
        return PXP_OK;
    }
    const int P = c.p.P;
    const int64_t n_s = c.p.n_steps / P;
    double* slices = c.at(c.L.slices);
    // (1) P inhomogeneous sub-problems from zero data, one batch
    {
        ProfScope ps(PXP_K_SLICES, c.s);
        HIPCHK(launch_rk4_lin1d(F, g0, nullptr, slices, n, P, n_s, c.dt(),
                                c.p.omega, A, c.p.block, c.fp32(), c.s));
    }
    if (P == 1) {
        HIPCHK(launch_recombine(q0, slices, nullptr, 0, n, qT, c.st, c.s));
        return PXP_OK;
    }
    const double dT = c.p.T / P;
    KrylovArgs a = kargs(c, A);
    a.vin = slices;
    a.tau = dT;
    if (c.p.sched == PXP_SCHED_CLASSIC) {
        // (2) P-1 independent homogeneous pieces exp((T - T_{p+1}) A) v_p
        a.mode = KM_CLASSIC;
        a.npieces = P - 1;
        a.yout = c.at(c.L.pieces);
        {
            ProfScope ps(PXP_K_KRYLOV_DIRECT, c.s);
            HIPCHK(launch_krylov1d(a, c.p.kblock, c.s));
        }
        // (3) superposition q(T) = q0 + v_{P-1} + sum_p pieces
        HIPCHK(launch_recombine(q0, slices + (size_t)(P - 1) * n, c.at(c.L.pieces),
                                P - 1, n, qT, c.st, c.s));
    } else {
        // nested form of the same sum: w <- exp(dT A) w + v_p
        a.mode = KM_CHAIN;
        a.npieces = P;
        a.yout = c.at(c.L.chain);
        {
            ProfScope ps(PXP_K_KRYLOV_DIRECT, c.s);
            HIPCHK(launch_krylov1d(a, c.p.kblock, c.s));
        }
        HIPCHK(launch_recombine(q0, nullptr, c.at(c.L.chain), 1, n, qT, c.st, c.s));
    }
    return PXP_OK;
}

// Absorbed form of the adjoint (section 3.3, eq. hybadjinhom with the final
// condition absorbed): lam = lamT + q~ with q~(T) = 0.  In tau = T - t,
//   q~' = A^T q~ + A^T lamT,
// cut into P slices marched from zero as one batch (slice p covers
// tau in [p dT, (p+1) dT]); the end state w_p of slice p propagates
// homogeneously over the remaining (P-1-p) dT (classic pieces).  Then
//   lam(0) = lamT + w_{P-1} + sum_p exp((P-1-p) dT A^T) w_p,
//   Lambda = (1 - cos omega T)/omega lamT + sum_p (slice integrals)
//            + sum_p (piece integrals),
// every integral of sin(omega (T - tau)) against its part of q~.
pxp_status adjoint_lin1d_absorbed(const Ctx& c, const double* lamT, double* lam0,
                                  double* Lam) {
    const int n = c.n(), P = c.p.P;
    const int64_t n_s = c.p.n_steps / P;
    const Tri AT = transpose(advdiff_tri(c.p));
    const double w = c.p.omega, T = c.p.T;
    double* g = c.at(c.L.g0);
    double* sl = c.at(c.L.slices);
    double* aint = c.at(c.L.aint);
    HIPCHK(launch_apply_tri(lamT, g, n, AT, c.s));
    {
        // (1) the P adjoint slices, one batch; their integrals, with the
        // lamT term added to slice 0's
        SliceIntegral si{Lam ? aint : nullptr, w * T, -w,
                         (w != 0.0) ? (1.0 - std::cos(w * T)) / w : 0.0, lamT};
        ProfScope ps(PXP_K_SLICES, c.s);
        HIPCHK(launch_rk4_lin1d(nullptr, g, nullptr, sl, n, P, n_s, c.dt(), 0.0, AT,
                                c.p.block, c.fp32(), c.s, si));
    }
    {
        // (2) P-1 homogeneous pieces exp((P-1-p) dT A^T) w_p with integrals
        KrylovArgs a = kargs(c, AT);
        a.mode = KM_CLASSIC;
        a.adj = 1;
        a.npieces = P - 1;
        a.vin = sl;
        a.yout = c.at(c.L.pieces);
        a.iout = Lam ? aint + (size_t)P * n : nullptr;
        a.tau = T / P;
        a.ia = w;  // piece p: phase omega * tau_p
        a.ib = -w;
        ProfScope ps(PXP_K_KRYLOV_ADJOINT, c.s);
        HIPCHK(launch_krylov1d(a, c.p.kblock, c.s));
    }
    // (3) superposition
    if (lam0)
        HIPCHK(launch_recombine(lamT, sl + (size_t)(P - 1) * n, c.at(c.L.pieces), P - 1, n,
                                lam0, c.st, c.s));
    if (Lam)
        HIPCHK(launch_recombine(nullptr, nullptr, aint, 2 * P - 1, n, Lam, c.st, c.s));
    return PXP_OK;
}

// Adjoint of one linear 1D instance from lamT: lam0 and/or Lambda.
pxp_status adjoint_lin1d(const Ctx& c, const double* lamT, double* lam0,
                         double* Lam, int method) {
    const int n = c.n();
    const Tri AT = transpose(advdiff_tri(c.p));
    if (method == PXP_METHOD_SERIAL) {
        ProfScope ps(PXP_K_SERIAL_REVERSE, c.s);
        HIPCHK(launch_rk4_rev_lin1d(lamT, lam0, Lam, n, c.p.n_steps, c.dt(),
                                    c.p.omega, AT, c.p.block, c.fp32(), c.s));
        return PXP_OK;
    }
    if ((c.p.flags & PXP_FLAG_ABSORBED_ADJOINT) && c.p.P > 1)
        return adjoint_lin1d_absorbed(c, lamT, lam0, Lam);
    // The terminal-cost adjoint is one homogeneous piece from q^dagger(T)
    // over [T, 0] (eq. adjhomfinal); in tau = T - t it reads
    // d lam / d tau = A^T lam, and Lambda = int_0^T sin(omega (T - tau))
    // lam(tau) d tau is formed inside the Krylov space.
    KrylovArgs a = kargs(c, AT);
    a.mode = KM_SINGLE;
    a.npieces = 1;
    a.vin = lamT;
    a.yout = lam0;
    a.iout = Lam;
    a.tau = c.p.T;
    a.ia = c.p.omega * c.p.T;
    a.ib = -c.p.omega;
    if (!lam0 && !Lam) return PXP_OK;
    ProfScope ps(PXP_K_KRYLOV_ADJOINT, c.s);
    HIPCHK(launch_krylov1d(a, c.p.kblock, c.s));
    return PXP_OK;
}

pxp_status direct_burgers_nl(const Ctx& c, const double* q0, double* qT);

pxp_status direct_burgers(const Ctx& c, const double* q0, double* qT, int method) {
    if (nlpx(c.p) && method == PXP_METHOD_PARAEXP) return direct_burgers_nl(c, q0, qT);
    ProfScope ps(PXP_K_SERIAL_DIRECT, c.s);
    HIPCHK(launch_rk4_burgers_direct(q0, qT, c.at(c.L.ckpt), c.n(), c.p.n_steps,
                                     c.p.ckpt_every, c.dt(), c.p.nu, c.p.L,
                                     c.p.block, c.fp32(), c.s));
    return PXP_OK;
}

// The Magnus steps' own error is estimated on two sampled macro steps (the
// first and the last in reversed time) by one step against two half steps
// of lamT; the half steps need an even number of RK4 steps per slice (no
// estimate otherwise).
bool magnus_checkable(const pxp_problem& p) {
    const int64_t S = p.n_steps / p.P;
    return S >= 2 && S % 2 == 0;
}

// Sampled macro step k (0, 1) of the check.
int magnus_sample(const pxp_problem& p, int k) { return k == 0 ? 0 : p.P - 1; }

// The four check chains of one instance from its main chain's arguments a
// (kind 2k: one step of sample k, kind 2k+1: its two half steps).
KrylovArgs magnus_check_args(const Ctx& c, const KrylovArgs& a, int kind) {
    const int64_t n = c.n();
    const int k = kind / 2, q = magnus_sample(c.p, k);
    const double D = (double)(c.p.n_steps / c.p.P) * c.dt();
    KrylovArgs b = a;
    // in FP64 also for FP32-bulk problems: the difference of the two
    // propagations is then the Magnus error, not the FP32 stencil's rounding
    b.fp32 = 0;
    // the check propagates the start vector alone
    b.vadd = nullptr;
    b.addq = nullptr;
    b.nadd = 0;
    b.yout = c.at(c.L.mout) + (size_t)kind * n;
    if (kind % 2 == 0) {
        b.npieces = 1;
        b.wop = c.at(c.L.nodes) + (size_t)(2 * q) * n;
        b.tau = 0.5 * D;
    } else {
        b.npieces = 2;
        b.wop = c.at(c.L.mnodes) + (size_t)(4 * k) * n;
        b.tau = 0.25 * D;
    }
    return b;
}

MagnusCheck magnus_check_desc(const Ctx& c) {
    MagnusCheck m{};
    m.y = c.at(c.L.mout);
    m.n = c.n();
    m.nsamp = 2;
    m.tol = c.p.krylov_tol;
    m.scale = 16.0 / 15.0;
    m.st = c.st;
    m.irep = c.irep;
    return m;
}

pxp_status adjoint_burgers(const Ctx& c, const double* lamT, double* lam0,
                           int method, const double* vadd = nullptr,
                           const int* addq = nullptr, int nadd = 0) {
    if (method == PXP_METHOD_SERIAL) {
        ProfScope ps(PXP_K_SERIAL_REVERSE, c.s);
        HIPCHK(launch_rk4_burgers_reverse(c.at(c.L.ckpt), lamT, lam0, c.at(c.L.seg),
                                          c.n(), c.p.n_steps, c.p.ckpt_every, c.dt(),
                                          c.p.nu, c.p.L, c.p.block, c.fp32(), c.s));
        return PXP_OK;
    }
    // The adjoint of the serial direct march is linear and time-varying
    // (section 3.3).  With a terminal cost only it is the single
    // homogeneous piece from q^dagger(T) (eq. adjhomfinal), propagated over
    // the P slices by fourth-order commutator-free Magnus steps; each factor
    // is the exponential of the Burgers Jacobian transpose at an effective
    // state, recomputed for all slices at once from the checkpoints.
    const int64_t S = c.p.n_steps / c.p.P;
    const double h = c.p.L / c.p.nx;
    {
        ProfScope ps(PXP_K_LTV_NODES, c.s);
        HIPCHK(launch_burgers_nodes(c.at(c.L.ckpt), c.at(c.L.nodes), c.n(),
                                    c.p.n_steps, c.p.ckpt_every, S, c.dt(), c.p.nu,
                                    c.p.L, c.p.block, c.fp32(), c.s));
    }
    KrylovArgs a = kargs(c, Tri{0.0, 0.0, 0.0});
    a.si = use_si(c.p) ? 1 : 0;
    a.mode = KM_LTV;
    a.npieces = c.p.P;
    a.vin = lamT;
    a.yout = lam0;
    a.tau = 0.5 * (double)S * c.dt();
    a.wop = c.at(c.L.nodes);
    a.inv2h = 1.0 / (2.0 * h);
    a.nuh2 = c.p.nu / (h * h);
    a.vadd = vadd;
    a.addq = addq;
    a.nadd = nadd;
    {
        ProfScope ps(PXP_K_LTV_ADJOINT, c.s);
        HIPCHK(launch_krylov1d(a, c.p.kblock, c.s));
    }
    if (!magnus_checkable(c.p)) return PXP_OK;
    // the a posteriori Magnus check: half-step nodes of the two sampled
    // macro steps, one and two steps from lamT, the Richardson estimate
    ProfScope ps(PXP_K_LTV_CHECK, c.s);
    for (int k = 0; k < 2; ++k)
        HIPCHK(launch_burgers_nodes(c.at(c.L.ckpt), c.at(c.L.mnodes) + (size_t)(4 * k) * c.n(),
                                    c.n(), c.p.n_steps, c.p.ckpt_every, S / 2, c.dt(), c.p.nu,
                                    c.p.L, c.p.block, c.fp32(), c.s,
                                    2 * magnus_sample(c.p, k), 2));
    for (int kind = 0; kind < 4; ++kind)
        HIPCHK(launch_krylov1d(magnus_check_args(c, a, kind), c.p.kblock, c.s));
    const MagnusCheck m = magnus_check_desc(c);
    auto* dm = reinterpret_cast<MagnusCheck*>(c.at(c.L.mdesc));
    HIPCHK(launch_upload(dm, &m, sizeof(m), c.s));
    HIPCHK(launch_magnus_check(dm, 1, c.s));
    return PXP_OK;
}

// The iterative nonlinear Paraexp direct for Burgers (section 3.2): the
// first iterate q0 at every stage; per iteration the slice averages, the
// zero-start slices, the chain of the slices' linearised exponentials with
// their end states added (the corrected slice starts kept), and every slice
// again from its corrected start for the new stage states, and the change
// of q(T), which ends the iteration once within tolerance.  The last
// change is the estimate; the checkpoints come from the last iterate.
pxp_status direct_burgers_nl(const Ctx& c, const double* q0, double* qT) {
    const pxp_problem& p = c.p;
    const int n = c.n(), P = nl_slices(p);
    const int64_t n_t = p.n_steps, S = n_t / P;
    const double h = p.L / p.nx;
    const double tol = p.nl_tol > 0.0 ? p.nl_tol : p.krylov_tol;
    double* st[2] = {c.at(c.L.nst[0]), c.at(c.L.nst[1])};
    double* qprev = c.at(c.L.nq);
    auto* ns = reinterpret_cast<NlState*>(c.at(c.L.ndesc));
    std::vector<int> addq(P);
    for (int k = 0; k < P; ++k) addq[k] = k;
    auto* daddq = reinterpret_cast<int*>(c.at(c.L.naddq));
    for (size_t o = 0; o < addq.size() * sizeof(int); o += 3072)
        HIPCHK(launch_upload(reinterpret_cast<char*>(daddq) + o,
                             reinterpret_cast<const char*>(addq.data()) + o,
                             std::min((size_t)3072, addq.size() * sizeof(int) - o), c.s));
    HIPCHK(launch_nl_fill(q0, st[0], qprev, ns, n, 4 * n_t, c.s));
    // the chain of the linearised slice exponentials: the operator is
    // constant over a slice, so a macro step is the single factor
    // exp((T_{p+1} - T_p)(A + J_p))
    KrylovArgs a = kargs(c, Tri{0.0, 0.0, 0.0});
    a.mode = KM_LTV;
    a.ltv_one = 1;
    a.npieces = P;
    a.vin = q0;
    a.yout = nullptr;  // q(T) comes from the last slice's march
    a.tau = (double)S * c.dt();
    a.wop = c.at(c.L.nW);
    a.inv2h = 1.0 / (2.0 * h);
    a.nuh2 = p.nu / (h * h);
    a.vadd = c.at(c.L.nv);
    a.addq = daddq;
    a.nadd = P;
    a.ltv_fwd = 1;
    a.vsnap = c.at(c.L.nE);
    a.adj = 0;
    a.skip = &ns->done;
    // up to nl_iters iterations; once an iteration's change of q(T) is
    // within tol the remaining launches return at once (algorithm 2's
    // while loop without a host synchronisation)
    const int K = nl_iters(p);
    for (int it = 0; it < K; ++it) {
        const double* so = st[it & 1];
        double* sn = st[(it + 1) & 1];
        {
            // the slices' Jacobians and the slices from zero (every slice,
            // slice 0 too: the chain carries q0)
            ProfScope ps(PXP_K_SLICES, c.s);
            HIPCHK(launch_nl_slice_mean(so, it == 0 ? q0 : qT, c.at(c.L.nW), n, S, P, ns, c.s));
            HIPCHK(launch_burgers_nl_march(so, nullptr, c.at(c.L.nv), nullptr, nullptr, nullptr,
                                           c.at(c.L.nW), n, S, P, c.dt(), p.nu, p.L, p.block,
                                           ns, c.s));
        }
        {
            ProfScope ps(PXP_K_KRYLOV_DIRECT, c.s);
            HIPCHK(launch_krylov1d(a, p.kblock, c.s));
        }
        {
            // the new iterate at the stage points, and its change
            ProfScope ps(PXP_K_NL_ITER, c.s);
            HIPCHK(launch_burgers_nl_march(so, sn, nullptr, c.at(c.L.nE), q0, qT, c.at(c.L.nW),
                                           n, S, P, c.dt(), p.nu, p.L, p.block, ns, c.s));
            HIPCHK(launch_nl_change(qT, qprev, n, tol, ns, (it + 1) & 1, c.irep, c.s));
        }
    }
    HIPCHK(launch_nl_final(ns, tol, c.st, c.irep, c.s));
    HIPCHK(launch_nl_ckpt(st[0], st[1], ns, qT, c.at(c.L.ckpt), n, n_t, p.ckpt_every, c.s));
    return PXP_OK;
}

// Integral cost, Burgers: the serial march forms one cost partial per
// launch (the step sources come later, from the recomputed states).  Paraexp: the hybrid scheme of section 3.3
// (algorithm 3) -- one march launch per adjoint slice on the caller's
// stream; after every hyb_group slices the library's side stream (when it
// exists; else the caller's) waits for the march and runs those slices'
// adjoint batch.  *nparts receives the number of cost partials.
pxp_status direct_burgers_icost(const Ctx& c, const double* q0, const double* tgt,
                                double* qT, int method, int* nparts) {
    const int64_t n_t = c.p.n_steps;
    const int n = c.n();
    BurgersRange rg{};
    rg.tgt = tgt;
    rg.gw = 2.0 * c.dt() / c.p.T;
    if (method == PXP_METHOD_SERIAL) {
        rg.s0 = 0;
        rg.s1 = n_t;
        rg.cpart = c.at(c.L.cpart);
        ProfScope ps(PXP_K_SERIAL_DIRECT, c.s);
        HIPCHK(launch_rk4_burgers_direct(q0, qT, c.at(c.L.ckpt), n, n_t, c.p.ckpt_every,
                                         c.dt(), c.p.nu, c.p.L, c.p.block, 0, c.s, &rg));
        *nparts = 1;
        return PXP_OK;
    }
    const std::vector<int64_t> b = hyb_bounds(c.p);
    const int ns = (int)b.size() - 1;
    const int64_t S = n_t / c.p.P;
    // the chain adds slice ns-1-k's end state after macro step addq[k]
    // (reversed time), where it reaches the slice's start
    std::vector<int> addq(ns);
    for (int k = 0; k < ns; ++k) addq[k] = (int)((n_t - b[ns - 1 - k]) / S) - 1;
    auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
        for (size_t o = 0; o < bytes; o += 3072) {
            hipError_t e = launch_upload(static_cast<char*>(dst) + o,
                                         static_cast<const char*>(src) + o,
                                         std::min((size_t)3072, bytes - o), c.s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    auto* dbnd = reinterpret_cast<int64_t*>(c.at(c.L.hbnd));
    HIPCHK(up(dbnd, b.data(), b.size() * sizeof(int64_t)));
    HIPCHK(up(c.at(c.L.haddq), addq.data(), addq.size() * sizeof(int)));
    int dev = 0;
    SideStream side;
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < MAX_DEVICES) {
        std::lock_guard<std::mutex> copy(g_side_mu);
        side = g_side[dev];
    }
    std::unique_lock<std::mutex> lock(g_side_mu, std::defer_lock);
    const bool forked = side.st != nullptr;
    if (forked) lock.lock();
    const int G = hyb_group(c.p);
    double* st = c.at(c.L.hstate);
    for (int sl = 0; sl < ns; ++sl) {
        rg.s0 = b[sl];
        rg.s1 = b[sl + 1];
        rg.cpart = c.at(c.L.cpart) + sl;
        const double* in = sl == 0 ? q0 : st;
        double* out = sl == ns - 1 ? qT : st;
        {
            ProfScope ps(PXP_K_SERIAL_DIRECT, c.s);
            HIPCHK(launch_rk4_burgers_direct(in, out, c.at(c.L.ckpt), n, n_t, c.p.ckpt_every,
                                             c.dt(), c.p.nu, c.p.L, c.p.block, 0, c.s, &rg));
        }
        if ((sl + 1) % G != 0 && sl != ns - 1) continue;
        const int g0 = (sl / G) * G;
        hipStream_t sg = c.s;
        if (forked) {
            HIPCHK(hipEventRecord(side.fork, c.s));
            HIPCHK(hipStreamWaitEvent(side.st, side.fork, 0));
            sg = side.st;
        }
        ProfScope ps(PXP_K_ADJ_SLICES, sg);
        HIPCHK(launch_burgers_adj_slices(c.at(c.L.ckpt), tgt, rg.gw, c.at(c.L.hseg),
                                         c.at(c.L.hmu), dbnd, g0, sl + 1 - g0, n, n_t,
                                         c.p.ckpt_every, c.dt(), c.p.nu, c.p.L, c.p.block, sg));
    }
    if (forked) {
        HIPCHK(hipEventRecord(side.join, side.st));
        HIPCHK(hipStreamWaitEvent(c.s, side.join, 0));
    }
    *nparts = ns;
    return PXP_OK;
}

// Its adjoint: serial, the discrete adjoint with the sources from
// dJ/dq(T); Paraexp, the Magnus chain from dJ/dq(T) = gw / 2 (q(T) - tgt)
// adding the hybrid slices' end states.
pxp_status adjoint_burgers_icost(const Ctx& c, const double* qT, const double* tgt,
                                 double* lam0, int method) {
    const int64_t n_t = c.p.n_steps;
    const int n = c.n();
    const double gw = 2.0 * c.dt() / c.p.T;
    if (method == PXP_METHOD_SERIAL) {
        BurgersRange rg{};
        rg.s0 = 0;
        rg.s1 = n_t;
        rg.tgt = tgt;
        rg.gw = gw;
        rg.src_start = 1;
        ProfScope ps(PXP_K_SERIAL_REVERSE, c.s);
        HIPCHK(launch_rk4_burgers_reverse(c.at(c.L.ckpt), nullptr, lam0, c.at(c.L.seg), n,
                                          n_t, c.p.ckpt_every, c.dt(), c.p.nu, c.p.L,
                                          c.p.block, 0, c.s, &rg));
        return PXP_OK;
    }
    const int ns = (int)hyb_bounds(c.p).size() - 1;
    double* gT = c.at(c.L.lamT);
    HIPCHK(launch_scaled_diff(qT, tgt, 0.5 * gw, gT, n, c.s));
    return adjoint_burgers(c, gT, lam0, method, c.at(c.L.hmu),
                           reinterpret_cast<const int*>(c.at(c.L.haddq)), ns);
}

// Burgers instances that the ragged batch kernels take: 256 threads with a
// supported number of points per thread.
bool burgers_batchable(const pxp_problem& p) {
    if (p.op != PXP_OP_BURGERS1D || p.nx % 256 || icost(p) || nlpx(p)) return false;
    const int pt = p.nx / 256;
    return pt == 1 || pt == 2 || pt == 4 || pt == 8 || pt == 16 || pt == 32;
}

// Burgers instances of a call go through one launch per phase when there is
// more than one of them and all have the same precision.
struct BurgersBatch {
    std::vector<int> idx;  // instance indices
    int fp32 = 0;
    bool on = false;
};

BurgersBatch burgers_batch(const pxp_problem* pb, int batch) {
    BurgersBatch b;
    for (int i = 0; i < batch; ++i)
        if (burgers_batchable(pb[i])) b.idx.push_back(i);
    if (b.idx.size() < 2) {
        b.idx.clear();
        return b;
    }
    b.fp32 = pb[b.idx[0]].prec == PXP_FP32_BULK;
    for (int i : b.idx)
        if ((pb[i].prec == PXP_FP32_BULK) != (b.fp32 != 0)) {
            b.idx.clear();
            return b;
        }
    b.on = true;
    return b;
}

bool in_batch(const BurgersBatch& b, int i) {
    for (int j : b.idx)
        if (j == i) return true;
    return false;
}

// Device arrays handed to the kernels that use 16-byte loads must be
// 16-byte aligned at every instance offset.
bool aligned16(const double* base, size_t off) {
    return !base || (reinterpret_cast<uintptr_t>(base + off) % 16) == 0;
}

pxp_status ws_check(const pxp_problem* pb, int batch, void* ws, size_t ws_bytes,
                    Layout* Ly) {
    *Ly = layout(pb, batch);
    if (!ws || ws_bytes < Ly->total) return PXP_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % ALIGN) return PXP_EWORKSPACE;
    return PXP_OK;
}

Ctx make_ctx(const pxp_problem& p, void* ws, const Layout& Ly, int i,
             hipStream_t s) {
    char* w = static_cast<char*>(ws);
    return Ctx{p, w + Ly.base[i], inst_layout(p),
               reinterpret_cast<DevStatus*>(w + Ly.status), s,
               reinterpret_cast<InstStat*>(w + Ly.irep) + i};
}

BurgersDesc burgers_desc(const pxp_problem& p, const Ctx& c) {
    BurgersDesc d{};
    const double h = p.L / p.nx;
    d.n = p.nx;
    d.pt = p.nx / 256;
    const int pr = p.nx / 512;
    d.pt_rev = (p.nx % 512 == 0 && (pr == 2 || pr == 4 || pr == 8 || pr == 16)) ? pr : 0;
    d.n_t = p.n_steps;
    d.c = p.ckpt_every;
    d.S = p.n_steps / p.P;
    d.dt = c.dt();
    d.inv2h = 1.0 / (2.0 * h);
    d.nuh2 = p.nu / (h * h);
    d.ckpt = c.at(c.L.ckpt);
    d.seg = c.at(c.L.seg);
    d.nodes = c.at(c.L.nodes);
    return d;
}

pxp_status burgers_batch_direct(const pxp_problem* pb, const BurgersBatch& bb,
                                void* ws, const Layout& Ly,
                                const std::vector<const double*>& init,
                                const std::vector<double*>& qT, hipStream_t s) {
    std::vector<BurgersDesc> tab;
    for (size_t j = 0; j < bb.idx.size(); ++j) {
        const int i = bb.idx[j];
        Ctx c = make_ctx(pb[i], ws, Ly, i, s);
        BurgersDesc d = burgers_desc(pb[i], c);
        d.y0 = init[j];
        d.yT = qT[j];
        tab.push_back(d);
    }
    auto* dtab = reinterpret_cast<BurgersDesc*>(static_cast<char*>(ws) + Ly.btab);
    HIPCHK(launch_upload(dtab, tab.data(), tab.size() * sizeof(BurgersDesc), s));
    ProfScope ps(PXP_K_SERIAL_DIRECT, s);
    HIPCHK(launch_burgers_batch(0, dtab, (int)tab.size(), 0, bb.fp32, s));
    return PXP_OK;
}

pxp_status burgers_batch_adjoint(const pxp_problem* pb, const BurgersBatch& bb,
                                 void* ws, const Layout& Ly,
                                 const std::vector<double*>& lamT,
                                 const std::vector<double*>& lam0, int method,
                                 hipStream_t s) {
    std::vector<BurgersDesc> tab;
    std::vector<KrylovArgs> ktab;
    std::vector<int> kB;
    std::vector<char> kcheb;  // the Chebyshev flavour's own chain kernel
    int q0 = 0;
    size_t lds = 0;
    for (size_t j = 0; j < bb.idx.size(); ++j) {
        const int i = bb.idx[j];
        const pxp_problem& p = pb[i];
        Ctx c = make_ctx(p, ws, Ly, i, s);
        BurgersDesc d = burgers_desc(p, c);
        d.lamT = lamT[j];
        d.lam0 = lam0[j];
        d.q0 = q0;
        q0 += p.P;
        tab.push_back(d);
        KrylovArgs a = kargs(c, Tri{0.0, 0.0, 0.0});
        a.si = use_si(p) ? 1 : 0;
        a.mode = KM_LTV;
        a.npieces = p.P;
        a.vin = lamT[j];
        a.yout = lam0[j];
        a.tau = 0.5 * (double)d.S * c.dt();
        a.wop = d.nodes;
        a.inv2h = d.inv2h;
        a.nuh2 = d.nuh2;
        int B = 0, pt = 0;
        const bool ch = a.cheb && !a.si && cheb_chain_shape_pub(p.nx, &B, &pt);
        if (!ch) {
            krylov_shape_pub(p.nx, p.kblock, &B, &pt);  // validated
            const size_t l = krylov1d_lds_bytes(p.nx, p.m, B, 0);
            if (l > lds) lds = l;
        }
        a.pt = pt;
        ktab.push_back(a);
        kB.push_back(B);
        kcheb.push_back(ch ? 1 : 0);
    }
    // one launch per kernel and workgroup size, the instances of one
    // contiguous
    auto key = [&](int j) { return (kcheb[j] ? 1 << 20 : 0) + 64 * kB[j] + ktab[j].pt; };
    std::vector<int> order(ktab.size());
    for (size_t j = 0; j < order.size(); ++j) order[j] = (int)j;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return key(x) < key(y); });
    std::vector<KrylovArgs> ksorted;
    for (int j : order) ksorted.push_back(ktab[j]);
    auto* dtab = reinterpret_cast<BurgersDesc*>(static_cast<char*>(ws) + Ly.btab);
    HIPCHK(launch_upload(dtab, tab.data(), tab.size() * sizeof(BurgersDesc), s));
    if (method == PXP_METHOD_SERIAL) {
        // the sweep is barrier-latency bound: 512 threads with half the
        // points each when every instance of the launch allows it
        bool rev512 = true;
        for (const BurgersDesc& d : tab) rev512 = rev512 && d.pt_rev != 0;
        ProfScope ps(PXP_K_SERIAL_REVERSE, s);
        HIPCHK(launch_burgers_batch(rev512 ? 3 : 1, dtab, (int)tab.size(), 0, bb.fp32, s));
        return PXP_OK;
    }
    auto* kt = reinterpret_cast<KrylovArgs*>(static_cast<char*>(ws) + Ly.ktab);
    HIPCHK(launch_upload(kt, ksorted.data(), ksorted.size() * sizeof(KrylovArgs), s));
    {
        ProfScope ps(PXP_K_LTV_NODES, s);
        HIPCHK(launch_burgers_batch(2, dtab, (int)tab.size(), q0, bb.fp32, s));
    }
    // Magnus check of the instances that allow it: half-step nodes of the
    // two sampled macro steps (one job each, after the instances' own
    // descriptors), then per workgroup-size group and kind one chain launch
    // right after the group's main chains (the same basis), then the
    // estimates
    std::vector<int> chk(order.size(), 0);
    std::vector<BurgersDesc> ctab;
    std::vector<KrylovArgs> cks;  // group-major, then kind, then instance
    std::vector<MagnusCheck> mt;
    struct CLaunch {
        size_t first;
        int count, block;
        size_t group;
        bool cheb;
        int pt;
    };
    std::vector<CLaunch> cl;
    {
        int cq0 = 0;
        for (size_t j = 0; j < bb.idx.size(); ++j) {
            const pxp_problem& p = pb[bb.idx[j]];
            if (!magnus_checkable(p)) continue;
            Ctx c = make_ctx(p, ws, Ly, bb.idx[j], s);
            for (int k = 0; k < 2; ++k) {
                BurgersDesc d = tab[j];
                d.S = tab[j].S / 2;
                d.nodes = c.at(c.L.mnodes) + (size_t)(4 * k) * c.n();
                d.qbase = 2 * magnus_sample(p, k);
                d.q0 = cq0;
                cq0 += 2;
                ctab.push_back(d);
            }
            mt.push_back(magnus_check_desc(c));
        }
        size_t g = 0;
        for (size_t j0 = 0; j0 < order.size(); ++g) {
            size_t j1 = j0;
            while (j1 < order.size() && key(order[j1]) == key(order[j0])) ++j1;
            for (int kind = 0; kind < 4; ++kind) {
                const size_t first = cks.size();
                for (size_t e = j0; e < j1; ++e) {
                    const int j = order[e];
                    const pxp_problem& p = pb[bb.idx[j]];
                    if (!magnus_checkable(p)) continue;
                    Ctx c = make_ctx(p, ws, Ly, bb.idx[j], s);
                    cks.push_back(magnus_check_args(c, ktab[j], kind));
                }
                if (cks.size() > first)
                    cl.push_back({first, (int)(cks.size() - first), kB[order[j0]], g,
                                  kcheb[order[j0]] != 0, ktab[order[j0]].pt});
            }
            j0 = j1;
        }
        if (!ctab.empty()) {
            auto* dc = dtab + tab.size();
            HIPCHK(launch_upload(dc, ctab.data(), ctab.size() * sizeof(BurgersDesc), s));
            auto* kc = reinterpret_cast<KrylovArgs*>(static_cast<char*>(ws) + Ly.kchk);
            const size_t bytes = cks.size() * sizeof(KrylovArgs);
            for (size_t o = 0; o < bytes; o += 3072)
                HIPCHK(launch_upload(reinterpret_cast<char*>(kc) + o,
                                     reinterpret_cast<const char*>(cks.data()) + o,
                                     std::min((size_t)3072, bytes - o), s));
            auto* dm = reinterpret_cast<MagnusCheck*>(static_cast<char*>(ws) + Ly.mtab);
            HIPCHK(launch_upload(dm, mt.data(), mt.size() * sizeof(MagnusCheck), s));
            ProfScope ps(PXP_K_LTV_CHECK, s);
            HIPCHK(launch_burgers_batch(2, dc, (int)ctab.size(), cq0, bb.fp32, s));
        }
    }
    auto* kc = reinterpret_cast<KrylovArgs*>(static_cast<char*>(ws) + Ly.kchk);
    ProfScope ps(PXP_K_LTV_ADJOINT, s);
    // the first group on the caller's stream, the others on the side stream
    // (when it exists) so that the groups' chains run concurrently
    int dev = 0;
    SideStream side;
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < MAX_DEVICES) {
        std::lock_guard<std::mutex> copy(g_side_mu);
        side = g_side[dev];
    }
    std::unique_lock<std::mutex> lock(g_side_mu, std::defer_lock);
    const bool groups = !order.empty() && key(order.front()) != key(order.back());
    const bool forked = groups && side.st;
    if (forked) {
        // the side stream starts where the caller's stream is now: before
        // the first group is enqueued
        lock.lock();
        HIPCHK(hipEventRecord(side.fork, s));
        HIPCHK(hipStreamWaitEvent(side.st, side.fork, 0));
    }
    size_t g = 0;
    for (size_t j0 = 0; j0 < order.size(); ++g) {
        size_t j1 = j0;
        while (j1 < order.size() && key(order[j1]) == key(order[j0])) ++j1;
        const hipStream_t sg = (j0 > 0 && forked) ? side.st : s;
        if (kcheb[order[j0]])
            HIPCHK(launch_cheb_chain_batch(kt + j0, kB[order[j0]], ktab[order[j0]].pt,
                                           (int)(j1 - j0), sg));
        else
            HIPCHK(launch_krylov_ltv_batch(kt + j0, kB[order[j0]], (int)(j1 - j0), lds, sg));
        for (const CLaunch& x : cl) {
            if (x.group != g) continue;
            if (x.cheb)
                HIPCHK(launch_cheb_chain_batch(kc + x.first, x.block, x.pt, x.count, sg));
            else
                HIPCHK(launch_krylov_ltv_batch(kc + x.first, x.block, x.count, lds, sg));
        }
        j0 = j1;
    }
    if (forked) {
        HIPCHK(hipEventRecord(side.join, side.st));
        HIPCHK(hipStreamWaitEvent(s, side.join, 0));
    }
    if (!mt.empty()) {
        auto* dm = reinterpret_cast<MagnusCheck*>(static_cast<char*>(ws) + Ly.mtab);
        HIPCHK(launch_magnus_check(dm, (int)mt.size(), s));
    }
    return PXP_OK;
}


// ---- 2D instances: every 2D instance of a call in one launch per phase ----

std::vector<int> batch2d(const pxp_problem* pb, int batch) {
    std::vector<int> v;
    for (int i = 0; i < batch; ++i)
        if (pb[i].op == PXP_OP_ADVDIFF2D_UPWIND) v.push_back(i);
    return v;
}

bool contains(const std::vector<int>& v, int i) {
    for (int j : v)
        if (j == i) return true;
    return false;
}

// Launches of one batched 2D phase, one per row length: entries of `tab`
// are ordered by nx, and blk0 counts from zero within each group.
struct Group2D {
    int first, count, blocks, nx;
};

// Output rows per band workgroup for a launch: 32 when every grid allows
// it and the launch still has a few workgroups per CU, else 16 (more,
// shorter workgroups for the latency-bound serial marches).
void band_rows(std::vector<Band2D>& tab) {
    size_t blocks32 = 0;
    bool all32 = true;
    for (const Band2D& d : tab) {
        blocks32 += (size_t)d.items * (size_t)(d.ny / 32);
        all32 = all32 && d.ny % 32 == 0;
    }
    const int rows = (all32 && blocks32 >= 1024) ? 32 : BAND_ROWS;
    for (Band2D& d : tab) d.rows = rows;
}

std::vector<Group2D> group2d(std::vector<Band2D>& tab) {
    band_rows(tab);
    std::vector<Group2D> g;
    for (int j = 0; j < (int)tab.size(); ++j) {
        const int nb = tab[j].items * (tab[j].ny / tab[j].rows);
        if (g.empty() || g.back().nx != tab[j].nx) g.push_back({j, 0, 0, tab[j].nx});
        tab[j].blk0 = g.back().blocks;
        g.back().blocks += nb;
        ++g.back().count;
    }
    return g;
}

// Serial march of every instance: launch L advances each instance by up to
// four steps (entries ordered by nx).
// src: the integral-cost marches (sources written forward, added in reverse).
pxp_status serial2d(std::vector<Band2D>& tab, Band2D* dtab, bool rev, bool src, hipStream_t s) {
    const std::vector<Group2D> groups = group2d(tab);
    HIPCHK(launch_upload(dtab, tab.data(), tab.size() * sizeof(Band2D), s));
    for (const Group2D& g : groups) {
        int64_t lmax = 0;
        for (int j = g.first; j < g.first + g.count; ++j)
            lmax = std::max(lmax, (tab[j].n_t + 3) / 4);
        for (int64_t L = 0; L < lmax; ++L) {
            const Band2D* t = dtab + g.first;
            if (src && rev)
                HIPCHK(launch_band2d_rsrc(t, g.count, g.blocks, g.nx, 1, (int)L, s));
            else if (src)
                HIPCHK(launch_band2d_src(t, g.count, g.blocks, g.nx, 1, (int)L, s));
            else if (rev)
                HIPCHK(launch_band2d_rev(t, g.count, g.blocks, g.nx, (int)L, s));
            else
                HIPCHK(launch_band2d(t, g.count, g.blocks, g.nx, 1, (int)L, s));
        }
    }
    return PXP_OK;
}

// Instances ordered by row length (stable), for the per-nx band launches.
std::vector<int> by_nx(const pxp_problem* pb, const std::vector<int>& idx) {
    std::vector<int> o(idx.size());
    for (size_t j = 0; j < o.size(); ++j) o[j] = (int)j;
    std::stable_sort(o.begin(), o.end(),
                     [&](int x, int y) { return pb[idx[x]].nx < pb[idx[y]].nx; });
    return o;
}

const double* serial2d_result(const Band2D& d) {
    const int64_t L = (d.n_t + 3) / 4;
    return d.buf[L & 1];
}

// ---- uniformised exponentials: jobs, stages and pass launches ---------------

// nvec independent exponentials of one instance with the same Poisson
// parameter: out_v = sum_{k<D} w_k N^k x_v + partner_v and, for two-sum jobs,
// out2_v = sum_k w2_k N^k x_v + out2_add_v.  Vectors are s* doubles apart.
struct PJob {
    const double* x = nullptr;
    int64_t sx = 0;
    const double* partner = nullptr;
    int64_t sp = 0;
    double* out = nullptr;
    int64_t so = 0;
    const double* wtab = nullptr;
    double* acc2 = nullptr;
    double* out2 = nullptr;
    const double* out2_add = nullptr;
    const double* out2_add2 = nullptr;
    int64_t sa = 0;  // stride of the added vectors
    const double* wtab2 = nullptr;
    const double* wtab2i = nullptr;  // phase form of the second sum's weights
    double ph0 = 0.0, dph = 0.0;
    double* tb[2] = {nullptr, nullptr};  // term vectors of later passes
    int nvec = 1, D = 1, nx = 0, ny = 0;
    double lam = 0.0, est = 0.0;
    Sten5 N{};
    DevStatus* st = nullptr;
    InstStat* irep = nullptr;
};

int pois_passes(int D) { return (D + POIS_PASS_TERMS - 1) / POIS_PASS_TERMS; }

// One stage: independent jobs (any instances), run pass by pass; every pass
// is one launch per (row length, one or two sums).  Each such group's table
// is uploaded once per stage, its entries ordered by falling term count, so
// the entries still running at a pass are a prefix of the table and the
// kernel derives the pass's terms and term vectors from the pass index.
// Output rows per band: 32 when that still gives a few workgroups per CU,
// else 16.
pxp_status run_stage(const std::vector<PJob>& jobs, PoisEntry* dtab, size_t cap,
                     hipStream_t s) {
    if (jobs.empty()) return PXP_OK;
    // at most a few jobs per instance and stage (two pair shapes, a carried
    // range, a copy); the table holds eight per instance
    if (jobs.size() > cap) return PXP_EWORKSPACE;
    int maxp = 0;
    size_t blocks32 = 0;
    bool all32 = true;
    for (const PJob& j : jobs) {
        maxp = std::max(maxp, pois_passes(j.D));
        blocks32 += (size_t)j.nvec * (size_t)(j.ny / 32);
        all32 = all32 && (j.ny % 32 == 0);
    }
    const int rows = (all32 && blocks32 >= 1024) ? 32 : 16;
    struct Group {
        int nx, two;
        PoisEntry* dev;
        std::vector<PoisEntry> tab;
        std::vector<int> passes;  // per entry
    };
    std::vector<Group> groups;
    size_t used = 0;
    for (int two = 0; two < 2; ++two)
        for (int nx : {64, 128, 256}) {
            Group g{nx, two, dtab + used, {}, {}};
            std::vector<const PJob*> js;
            for (const PJob& j : jobs)
                if (j.nx == nx && (j.out2 != nullptr) == (two != 0)) js.push_back(&j);
            if (js.empty()) continue;
            std::stable_sort(js.begin(), js.end(), [](const PJob* x, const PJob* y) {
                return pois_passes(x->D) > pois_passes(y->D);
            });
            int blk = 0;
            for (const PJob* jp : js) {
                const PJob& j = *jp;
                PoisEntry e{};
                e.x = j.x;
                e.sx = j.sx;
                e.tb[0] = j.tb[0];
                e.tb[1] = j.tb[1];
                e.partner = j.partner;
                e.s_partner = j.sp;
                e.acc = j.out;
                e.out = j.out;
                e.s_acc = e.s_out = j.so;
                e.wtab = j.wtab;
                e.acc2 = j.acc2;
                e.out2 = j.out2;
                e.out2_add = j.out2_add;
                e.out2_add2 = j.out2_add2;
                e.s_add = j.sa;
                e.wtab2 = j.wtab2;
                e.wtab2i = j.wtab2i;
                e.ph0 = j.ph0;
                e.dph = j.dph;
                e.lam = j.lam;
                e.est = j.est;
                e.N = j.N;
                e.D = j.D;
                e.nvec = j.nvec;
                e.nx = j.nx;
                e.ny = j.ny;
                e.rows = rows;
                e.blk0 = blk;
                e.status = j.st;
                e.irep = j.irep;
                blk += j.nvec * (j.ny / rows);
                g.tab.push_back(e);
                g.passes.push_back(pois_passes(j.D));
            }
            used += g.tab.size();
            const size_t bytes = g.tab.size() * sizeof(PoisEntry);
            for (size_t o = 0; o < bytes; o += 3072)
                HIPCHK(launch_upload(reinterpret_cast<char*>(g.dev) + o,
                                     reinterpret_cast<const char*>(g.tab.data()) + o,
                                     std::min((size_t)3072, bytes - o), s));
            groups.push_back(std::move(g));
        }
    for (int pass = 0; pass < maxp; ++pass)
        for (const Group& g : groups) {
            int cnt = 0;
            while (cnt < (int)g.tab.size() && g.passes[cnt] > pass) ++cnt;
            if (cnt == 0) continue;
            const PoisEntry& last = g.tab[cnt - 1];
            const int blocks = last.blk0 + last.nvec * (last.ny / rows);
            HIPCHK(launch_pois2d(g.dev, cnt, blocks, g.nx, g.two, pass, s));
        }
    return PXP_OK;
}

// Tree schedule of one instance's direct pieces: the levels of pairwise
// combinations, each a list of jobs.  Level l reads bufs[l-1] (bufs[0] =
// slices) and writes bufs[l]; the root goes to qT.  A pair of ranges
// [a, b), [b, c) gives exp((T_c - T_b) A) w_ab + w_bc.
void tree_up_levels(const pxp_problem& p, const Ctx& c, const TShape& sh,
                    const std::vector<double*>& bufs, double* qT,
                    std::vector<std::vector<PJob>>& levels) {
    const int64_t n = c.n();
    const Sten5 A = advdiff2d_sten(p);
    const double mu = uniform_mu(A), dT = p.T / p.P, tol = uniform_tail_tol(p);
    double* tb0 = c.at(c.L.tbuf);
    double* tb1 = tb0 + (size_t)((p.P + 1) / 2) * n;
    const size_t depth = sh.size() - 1;
    for (size_t l = 1; l <= depth; ++l) {
        const std::vector<TNode>& ch = sh[l - 1];
        const int cnt = (int)ch.size(), pairs = cnt / 2;
        const double* src = bufs[l - 1];
        double* dst = l == depth ? qT : bufs[l];
        std::vector<PJob> lv;
        int j = 0;
        while (j < pairs) {
            // a run of pairs whose right-hand ranges have the same length
            int j1 = j + 1;
            while (j1 < pairs && ch[2 * j1 + 1].size == ch[2 * j + 1].size) ++j1;
            PJob b;
            b.nvec = j1 - j;
            b.x = src + (size_t)(2 * j) * n;
            b.sx = 2 * n;
            b.partner = src + (size_t)(2 * j + 1) * n;
            b.sp = 2 * n;
            b.out = dst + (size_t)j * n;
            b.so = n;
            b.tb[0] = tb0 + (size_t)j * n;
            b.tb[1] = tb1 + (size_t)j * n;
            b.lam = mu * dT * ch[2 * j + 1].size;
            b.D = pois_terms(b.lam, tol, &b.est);
            b.nx = p.nx;
            b.ny = p.ny;
            b.N = uniform_N(A, mu);
            b.st = c.st;
            b.irep = c.irep;
            lv.push_back(b);
            j = j1;
        }
        if (cnt & 1) {  // the last range has no partner: carried over as is
            PJob b;
            b.x = src + (size_t)(cnt - 1) * n;
            b.out = dst + (size_t)pairs * n;
            b.so = b.sx = n;
            b.tb[0] = tb0;
            b.tb[1] = tb1;
            b.lam = 0.0;
            b.D = 1;
            b.nx = p.nx;
            b.ny = p.ny;
            b.N = uniform_N(A, mu);
            b.st = c.st;
            b.irep = c.irep;
            lv.push_back(b);
        }
        levels.push_back(lv);
    }
}

// The tree with its levels alternating between the slices and the pieces
// buffer ((P+1)/2 vectors).
void tree_levels(const pxp_problem& p, const Ctx& c, double* qT,
                 std::vector<std::vector<PJob>>& levels) {
    const TShape sh = tree_shape(p.P);
    std::vector<double*> bufs;
    for (size_t l = 0; l < sh.size(); ++l)
        bufs.push_back((l & 1) ? c.at(c.L.pieces) : c.at(c.L.slices));
    tree_up_levels(p, c, sh, bufs, qT, levels);
}

// Buffers of the kept levels (integral cost): level 0 the slices, level l
// >= 1 one after the other in the lev region.
std::vector<double*> kept_bufs(const Ctx& c, const TShape& sh) {
    const int64_t n = c.n();
    std::vector<double*> bufs{c.at(c.L.slices)};
    size_t v = 0;
    for (size_t l = 1; l < sh.size(); ++l) {
        bufs.push_back(c.at(c.L.lev) + v * n);
        v += sh[l].size();
    }
    return bufs;
}

// Corrected slice-start states q(T_m), m = 1..P-1, into ebuf slot m-1, from
// the kept up-sweep levels, top down: a pair of ranges [s, m), [m, e) gives
// q(T_m) = exp((T_m - T_s) A) q(T_s) + w_sm (w_sm: the left range's sum,
// which for s = 0 already holds the initial state and is q(T_m) itself).
void tree_down_levels(const pxp_problem& p, const Ctx& c, const TShape& sh,
                      const std::vector<double*>& bufs,
                      std::vector<std::vector<PJob>>& levels) {
    const int64_t n = c.n();
    const Sten5 A = advdiff2d_sten(p);
    const double mu = uniform_mu(A), dT = p.T / p.P, tol = uniform_tail_tol(p);
    double* E = c.at(c.L.ebuf);
    double* tb0 = c.at(c.L.tbuf);
    double* tb1 = tb0 + (size_t)((p.P + 1) / 2) * n;
    for (size_t l = sh.size() - 1; l >= 1; --l) {
        const std::vector<TNode>& ch = sh[l - 1];
        const int pairs = (int)ch.size() / 2;
        const double* left = bufs[l - 1];
        std::vector<PJob> lv;
        int j = 0;
        while (j < pairs) {
            const int s0 = ch[2 * j].start, Ls = ch[2 * j].size, Rs = ch[2 * j + 1].size;
            PJob b;
            b.nx = p.nx;
            b.ny = p.ny;
            b.N = uniform_N(A, mu);
            b.st = c.st;
            b.irep = c.irep;
            b.tb[0] = tb0 + (size_t)j * n;
            b.tb[1] = tb1 + (size_t)j * n;
            if (s0 == 0) {  // the leftmost pair: a copy
                b.x = left + (size_t)(2 * j) * n;
                b.out = E + (size_t)(Ls - 1) * n;
                b.sx = b.so = n;
                b.lam = 0.0;
                b.D = 1;
                lv.push_back(b);
                ++j;
                continue;
            }
            int j1 = j + 1;
            while (j1 < pairs && ch[2 * j1].size == Ls && ch[2 * j1 + 1].size == Rs) ++j1;
            b.nvec = j1 - j;
            b.x = E + (size_t)(s0 - 1) * n;
            b.sx = (int64_t)(Ls + Rs) * n;
            b.partner = left + (size_t)(2 * j) * n;
            b.sp = 2 * n;
            b.out = E + (size_t)(s0 + Ls - 1) * n;
            b.so = (int64_t)(Ls + Rs) * n;
            b.lam = mu * dT * Ls;
            b.D = pois_terms(b.lam, tol, &b.est);
            lv.push_back(b);
            j = j1;
        }
        levels.push_back(lv);
    }
}

// Tree of the integral-cost adjoint pieces over the adjoint slices' end
// states (bufs[0]): a pair of ranges [s, m), [m, e) gives the adjoint at
// T_s, exp((T_m - T_s) A^T) u_me + u_sm, and (Lam_out non-null) its share of
// Lambda, int_{T_s}^{T_m} sin(omega t) exp((T_m - t) A^T) u_me dt plus the
// shares of both halves (the slices' own shares in islot slots 0..P-1 at
// level 0; later levels' shares in the slots after them; a carried range
// keeps its share).  The root's state goes to root_out, its share (Lambda)
// to Lam_out.  Weight tables (phase form) are appended to wt.
void adj_tree_levels(const pxp_problem& p, const Ctx& c, const TShape& sh,
                     const std::vector<double*>& bufs, double* root_out, double* Lam_out,
                     std::vector<PoisWeights>& wt, std::vector<std::vector<PJob>>& levels) {
    const int64_t n = c.n();
    const Sten5 AT = transpose5(advdiff2d_sten(p));
    const double mu = uniform_mu(AT), dT = p.T / p.P, tol = uniform_tail_tol(p);
    double* tb0 = c.at(c.L.tbuf);
    double* tb1 = tb0 + (size_t)((p.P + 1) / 2) * n;
    double* islot = c.at(c.L.islot);
    double* wbase = c.at(c.L.iwtab);
    size_t wofs = 0;
    size_t slot = (size_t)p.P;
    std::vector<double*> share;  // shares of the ranges of the level below
    for (int q = 0; q < p.P; ++q) share.push_back(islot + (size_t)q * n);
    const size_t depth = sh.size() - 1;
    for (size_t l = 1; l <= depth; ++l) {
        const std::vector<TNode>& ch = sh[l - 1];
        const int cnt = (int)ch.size(), pairs = cnt / 2;
        const double* src = bufs[l - 1];
        double* dst = l == depth ? root_out : bufs[l];
        double* shl = l == depth ? Lam_out : islot + slot * n;
        std::vector<double*> nshare;
        std::vector<PJob> lv;
        int j = 0;
        while (j < pairs) {
            const int Ls = ch[2 * j].size, Rs = ch[2 * j + 1].size;
            // a run: equal shapes, and (shares) halves' shares 2n apart
            int j1 = j + 1;
            while (j1 < pairs && ch[2 * j1].size == Ls && ch[2 * j1 + 1].size == Rs &&
                   (!Lam_out || (share[2 * j1] == share[2 * j] + 2 * (j1 - j) * n &&
                                 share[2 * j1 + 1] == share[2 * j + 1] + 2 * (j1 - j) * n)))
                ++j1;
            PJob b;
            b.nvec = j1 - j;
            b.x = src + (size_t)(2 * j + 1) * n;
            b.sx = 2 * n;
            b.partner = src + (size_t)(2 * j) * n;
            b.sp = 2 * n;
            b.out = dst + (size_t)j * n;
            b.so = n;
            b.tb[0] = tb0 + (size_t)j * n;
            b.tb[1] = tb1 + (size_t)j * n;
            b.lam = mu * dT * Ls;
            b.D = pois_terms(b.lam, tol, &b.est);
            b.nx = p.nx;
            b.ny = p.ny;
            b.N = uniform_N(AT, mu);
            b.st = c.st;
            b.irep = c.irep;
            if (Lam_out) {
                PoisWeights pw{};
                pw.w = wbase + wofs;
                pw.wi = pw.w + b.D;
                pw.D = b.D;
                pw.split = 1;
                pw.lam = b.lam;
                pw.mu = mu;
                pw.omega = p.omega;
                pw.scale = 1.0 / mu;
                wofs += 2 * (size_t)b.D;
                wt.push_back(pw);
                b.wtab2 = pw.w;
                b.wtab2i = pw.wi;
                b.ph0 = p.omega * dT * (ch[2 * j].start + Ls);
                b.dph = p.omega * dT * (Ls + Rs);
                b.out2 = shl + (size_t)j * n;
                b.acc2 = b.out2;
                b.out2_add = share[2 * j];
                b.out2_add2 = share[2 * j + 1];
                b.sa = 2 * n;
                for (int v = j; v < j1; ++v) nshare.push_back(shl + (size_t)v * n);
            }
            lv.push_back(b);
            j = j1;
        }
        if (cnt & 1) {  // carried: the state is copied, the share kept
            PJob b;
            b.x = src + (size_t)(cnt - 1) * n;
            b.out = dst + (size_t)pairs * n;
            b.so = b.sx = n;
            b.tb[0] = tb0;
            b.tb[1] = tb1;
            b.lam = 0.0;
            b.D = 1;
            b.nx = p.nx;
            b.ny = p.ny;
            b.N = uniform_N(AT, mu);
            b.st = c.st;
            b.irep = c.irep;
            lv.push_back(b);
            if (Lam_out) nshare.push_back(share[cnt - 1]);
        }
        slot += (size_t)pairs;
        share.swap(nshare);
        levels.push_back(lv);
    }
}

// Chain schedule by uniformisation: w <- exp(dT A) w + v_{p+1}, p = 0..P-2.
void chain_levels(const pxp_problem& p, const Ctx& c, double* qT,
                  std::vector<std::vector<PJob>>& levels) {
    const int64_t n = c.n();
    const Sten5 A = advdiff2d_sten(p);
    const double mu = uniform_mu(A), dT = p.T / p.P;
    const double* sl = c.at(c.L.slices);
    double* cb[2] = {c.at(c.L.pieces), c.at(c.L.pieces) + n};
    double* tb0 = c.at(c.L.tbuf);
    PJob b;
    b.lam = mu * dT;
    b.D = pois_terms(b.lam, uniform_tail_tol(p), &b.est);
    b.nx = p.nx;
    b.ny = p.ny;
    b.N = uniform_N(A, mu);
    b.st = c.st;
    b.irep = c.irep;
    b.tb[0] = tb0;
    b.tb[1] = tb0 + n;
    b.sx = b.sp = b.so = n;
    for (int q = 0; q + 1 < p.P; ++q) {
        b.x = q == 0 ? sl : cb[(q - 1) & 1];
        b.partner = sl + (size_t)(q + 1) * n;
        b.out = (q + 2 == p.P) ? qT : cb[q & 1];
        levels.push_back({b});
    }
}

// Stages of every instance run together: stage l holds level l of each.
pxp_status run_levels(const std::vector<std::vector<std::vector<PJob>>>& per, PoisEntry* dtab,
                      size_t cap, hipStream_t s) {
    size_t depth = 0;
    for (const auto& v : per) depth = std::max(depth, v.size());
    for (size_t l = 0; l < depth; ++l) {
        std::vector<PJob> stage;
        for (const auto& v : per)
            if (l < v.size()) stage.insert(stage.end(), v[l].begin(), v[l].end());
        pxp_status st = run_stage(stage, dtab, cap, s);
        if (st != PXP_OK) return st;
    }
    return PXP_OK;
}

// Direct solve of the 2D instances idx: init (nullable) and F (nullable)
// per instance -> qT.  tgt (nullable; per instance, nullable): for the
// integral-cost instances, also the step sources and the cost partials
// (nparts[j] receives their count).
// Launches the 2D Krylov entries of kt: the shift-and-invert entries (a.si)
// and the others as separate launches (the kernel is specialised on the
// flavour); each group's table goes to its own part of dk, its entries'
// first workgroups numbered from zero.
pxp_status launch_krylov2d_groups(const std::vector<KrylovArgs>& kt, KrylovArgs* dk,
                                  hipStream_t s) {
    size_t off = 0;
    for (int si = 0; si < 2; ++si) {
        std::vector<KrylovArgs> g;
        int blk = 0;
        size_t lds = 0;
        for (KrylovArgs a : kt) {
            if ((a.si != 0) != (si != 0)) continue;
            a.blk0 = blk;
            blk += a.mode == KM_CLASSIC ? a.npieces : 1;
            lds = std::max(lds, krylov2d_lds_bytes(a.m, si));
            g.push_back(a);
        }
        if (g.empty()) continue;
        HIPCHK(launch_upload(dk + off, g.data(), g.size() * sizeof(KrylovArgs), s));
        HIPCHK(launch_krylov2d(dk + off, (int)g.size(), blk, lds, si, s));
        off += g.size();
    }
    return PXP_OK;
}

pxp_status direct_2d_batch(const pxp_problem* pb, const std::vector<int>& idx, void* ws,
                           const Layout& Ly, const std::vector<const double*>& init,
                           const std::vector<const double*>& F,
                           const std::vector<double*>& qT, int method, hipStream_t s,
                           const std::vector<const double*>* tgt = nullptr,
                           std::vector<int>* nparts = nullptr) {
    if (idx.empty()) return PXP_OK;
    auto* dtab = reinterpret_cast<Band2D*>(static_cast<char*>(ws) + Ly.t2d);
    const std::vector<int> ord = by_nx(pb, idx);
    auto with_src = [&](int j) { return tgt && (*tgt)[j] && icost(pb[idx[j]]); };
    auto src_fields = [&](Band2D& d, const Ctx& c, int j) {
        d.g = c.at(c.L.gsrc);
        d.tgt = (*tgt)[j];
        d.cpart = c.at(c.L.cpart);
        d.gw = 2.0 * c.dt() / c.p.T;
        d.n_t = c.p.n_steps;
    };
    if (method == PXP_METHOD_SERIAL) {
        // plain instances, then the integral-cost ones (their march also
        // writes the sources)
        for (int pass = 0; pass < 2; ++pass) {
            std::vector<Band2D> tab;
            std::vector<int> who;
            for (int j : ord) {
                if (with_src(j) != (pass == 1)) continue;
                const pxp_problem& p = pb[idx[j]];
                Ctx c = make_ctx(p, ws, Ly, idx[j], s);
                Band2D d{};
                d.F = F[j];
                d.nx = p.nx;
                d.ny = p.ny;
                d.dt = c.dt();
                d.omega = p.omega;
                d.A = advdiff2d_sten(p);
                d.y0 = init[j];
                d.buf[0] = c.at(c.L.sbuf0);
                d.buf[1] = c.at(c.L.sbuf1);
                d.n_t = p.n_steps;
                d.items = 1;
                if (pass == 1) src_fields(d, c, j);
                tab.push_back(d);
                who.push_back(j);
            }
            if (tab.empty()) continue;
            {
                ProfScope ps(PXP_K_SERIAL_DIRECT, s);
                pxp_status st = serial2d(tab, dtab, false, pass == 1, s);
                if (st != PXP_OK) return st;
            }
            for (size_t e = 0; e < who.size(); ++e) {
                HIPCHK(launch_add(nullptr, serial2d_result(tab[e]), qT[who[e]],
                                  (int)grid_n(pb[idx[who[e]]]), s));
                if (pass == 1 && nparts) (*nparts)[who[e]] = tab[e].ny / tab[e].rows;
            }
        }
        return PXP_OK;
    }
    std::vector<Band2D> tab;
    for (int j : ord) {
        const pxp_problem& p = pb[idx[j]];
        Ctx c = make_ctx(p, ws, Ly, idx[j], s);
        Band2D d{};
        d.F = F[j];
        d.nx = p.nx;
        d.ny = p.ny;
        d.dt = c.dt();
        d.omega = p.omega;
        d.A = advdiff2d_sten(p);
        // the initial state is the first slice's initial data, so the
        // superposition below needs no q0 term
        d.y0 = init[j];
        d.out = c.at(c.L.slices);
        d.items = p.P;
        d.nsteps = (int)(p.n_steps / p.P);
        d.item_steps = p.n_steps / p.P;
        tab.push_back(d);
    }
    // (1) the P inhomogeneous slices of every instance, one launch per row
    // length
    const std::vector<Group2D> groups = group2d(tab);
    HIPCHK(launch_upload(dtab, tab.data(), tab.size() * sizeof(Band2D), s));
    {
        ProfScope ps(PXP_K_SLICES, s);
        for (const Group2D& g : groups)
            HIPCHK(launch_band2d(dtab + g.first, g.count, g.blocks, g.nx, 0, 0, s));
    }
    // (2) homogeneous pieces.  Uniformised: tree or chain stages of pass
    // launches over every instance; their last stage writes q(T).
    {
        std::vector<std::vector<std::vector<PJob>>> per;
        for (size_t j = 0; j < idx.size(); ++j) {
            const pxp_problem& p = pb[idx[j]];
            if (!uniform_direct(p) || p.P == 1) continue;
            Ctx c = make_ctx(p, ws, Ly, idx[j], s);
            per.emplace_back();
            if (with_src((int)j)) {
                // integral cost: the levels kept, then walked back down for
                // the corrected state at every slice start
                const TShape sh = tree_shape(p.P);
                const std::vector<double*> bufs = kept_bufs(c, sh);
                tree_up_levels(p, c, sh, bufs, qT[j], per.back());
                tree_down_levels(p, c, sh, bufs, per.back());
            } else if (p.sched == PXP_SCHED_TREE) {
                tree_levels(p, c, qT[j], per.back());
            } else {
                chain_levels(p, c, qT[j], per.back());
            }
        }
        if (!per.empty()) {
            auto* dp = reinterpret_cast<PoisEntry*>(static_cast<char*>(ws) + Ly.ptab);
            ProfScope ps(PXP_K_KRYLOV_DIRECT, s);
            pxp_status st = run_levels(per, dp, Ly.ptab_entries, s);
            if (st != PXP_OK) return st;
        }
    }
    // integral cost: every slice again from its corrected start, writing the
    // sources of its steps and the cost partials
    {
        std::vector<Band2D> st;
        std::vector<int> who;
        for (int j : ord) {
            if (!with_src(j)) continue;
            const pxp_problem& p = pb[idx[j]];
            Ctx c = make_ctx(p, ws, Ly, idx[j], s);
            Band2D d{};
            d.F = F[j];
            d.nx = p.nx;
            d.ny = p.ny;
            d.dt = c.dt();
            d.omega = p.omega;
            d.A = advdiff2d_sten(p);
            d.y0 = init[j];
            d.ys = c.at(c.L.ebuf);
            d.items = p.P;
            d.nsteps = (int)(p.n_steps / p.P);
            d.item_steps = p.n_steps / p.P;
            src_fields(d, c, j);
            st.push_back(d);
            who.push_back(j);
        }
        if (!st.empty()) {
            const std::vector<Group2D> sg = group2d(st);
            HIPCHK(launch_upload(dtab, st.data(), st.size() * sizeof(Band2D), s));
            ProfScope ps(PXP_K_SOURCES, s);
            for (const Group2D& g : sg)
                HIPCHK(launch_band2d_src(dtab + g.first, g.count, g.blocks, g.nx, 0, 0, s));
            if (nparts)
                for (size_t e = 0; e < who.size(); ++e)
                    (*nparts)[who[e]] = st[e].items * (st[e].ny / st[e].rows);
        }
    }
    // Krylov pieces: classic (P-1 workgroups) or chain (one); the
    // workgroups are numbered per flavour group at launch
    std::vector<KrylovArgs> kt;
    for (size_t j = 0; j < idx.size(); ++j) {
        const pxp_problem& p = pb[idx[j]];
        if (p.P == 1 || uniform_direct(p)) continue;
        Ctx c = make_ctx(p, ws, Ly, idx[j], s);
        KrylovArgs a = kargs(c, Tri{0.0, 0.0, 0.0});
        a.op5 = advdiff2d_sten(p);
        a.anorm = sten_norm(a.op5);
        a.nx = p.nx;
        a.ny = p.ny;
        a.vin = c.at(c.L.slices);
        a.tau = p.T / p.P;
        if (p.sched == PXP_SCHED_CLASSIC) {
            a.mode = KM_CLASSIC;
            a.npieces = p.P - 1;
            a.yout = c.at(c.L.pieces);
        } else {
            a.mode = KM_CHAIN;
            a.npieces = p.P;
            a.yout = c.at(c.L.chain);
        }
        kt.push_back(a);
    }
    if (!kt.empty()) {
        auto* dk = reinterpret_cast<KrylovArgs*>(static_cast<char*>(ws) + Ly.ktab);
        ProfScope ps(PXP_K_KRYLOV_DIRECT, s);
        const pxp_status st = launch_krylov2d_groups(kt, dk, s);
        if (st != PXP_OK) return st;
    }
    // (3) superposition
    for (size_t j = 0; j < idx.size(); ++j) {
        const pxp_problem& p = pb[idx[j]];
        Ctx c = make_ctx(p, ws, Ly, idx[j], s);
        const int n = c.n();
        const double* sl = c.at(c.L.slices);
        if (p.P == 1)
            HIPCHK(launch_recombine(nullptr, sl, nullptr, 0, n, qT[j], c.st, s));
        else if (uniform_direct(p))
            continue;  // written by the last stage
        else if (p.sched == PXP_SCHED_CLASSIC)
            HIPCHK(launch_recombine(nullptr, sl + (size_t)(p.P - 1) * n,
                                    c.at(c.L.pieces), p.P - 1, n, qT[j], c.st, s));
        else
            HIPCHK(launch_recombine(nullptr, nullptr, c.at(c.L.chain), 1, n, qT[j], c.st,
                                    s));
    }
    return PXP_OK;
}

// Adjoint of the 2D instances idx from lamT: lam0 and/or Lambda.  src
// (nullable; per instance, nullable): the step sources of an integral cost
// ([n_steps + 1][n], added after each reverse step; lamT may then be null).
pxp_status adjoint_2d_batch(const pxp_problem* pb, const std::vector<int>& idx, void* ws,
                            const Layout& Ly, const std::vector<const double*>& lamT,
                            const std::vector<double*>& lam0,
                            const std::vector<double*>& Lam, int method, hipStream_t s,
                            const std::vector<const double*>* src = nullptr) {
    if (idx.empty()) return PXP_OK;
    auto has_src = [&](int j) { return src && (*src)[j] != nullptr; };
    auto* dtab = reinterpret_cast<Band2D*>(static_cast<char*>(ws) + Ly.t2d);
    const std::vector<int> ord = by_nx(pb, idx);
    if (method == PXP_METHOD_SERIAL) {
        for (int pass = 0; pass < 2; ++pass) {
            std::vector<Band2D> tab;
            std::vector<int> who;
            for (int j : ord) {
                if (has_src(j) != (pass == 1)) continue;
                const pxp_problem& p = pb[idx[j]];
                Ctx c = make_ctx(p, ws, Ly, idx[j], s);
                Band2D d{};
                d.y0 = lamT[j];
                d.buf[0] = c.at(c.L.sbuf0);
                d.buf[1] = c.at(c.L.sbuf1);
                d.Lam = Lam[j];
                d.n_t = p.n_steps;
                d.nx = p.nx;
                d.ny = p.ny;
                d.dt = c.dt();
                d.omega = p.omega;
                d.A = transpose5(advdiff2d_sten(p));
                d.items = 1;
                if (pass == 1) d.g = const_cast<double*>((*src)[j]);
                tab.push_back(d);
                who.push_back(j);
                if (Lam[j]) HIPCHK(launch_zero(Lam[j], (size_t)grid_n(p), s));
            }
            if (tab.empty()) continue;
            {
                ProfScope ps(PXP_K_SERIAL_REVERSE, s);
                pxp_status st = serial2d(tab, dtab, true, pass == 1, s);
                if (st != PXP_OK) return st;
            }
            for (size_t e = 0; e < who.size(); ++e)
                if (lam0[who[e]])
                    HIPCHK(launch_add(nullptr, serial2d_result(tab[e]), lam0[who[e]],
                                      (int)grid_n(pb[idx[who[e]]]), s));
        }
        return PXP_OK;
    }
    // integral cost: the adjoint slices with their sources (zero data at
    // each slice end; the last slice from lamT), one batch, then the tree of
    // their homogeneous pieces, each pair adding its share of Lambda to its
    // halves' shares up to the root
    {
        std::vector<Band2D> at;
        for (int j : ord) {
            if (!has_src(j) || (!lam0[j] && !Lam[j])) continue;
            const pxp_problem& p = pb[idx[j]];
            Ctx c = make_ctx(p, ws, Ly, idx[j], s);
            Band2D d{};
            d.y0 = lamT[j];
            d.g = const_cast<double*>((*src)[j]);
            d.out = c.at(c.L.slices);
            // each slice's share of Lambda (a single slice: Lambda itself)
            d.Lam = Lam[j] ? (p.P == 1 ? Lam[j] : c.at(c.L.islot)) : nullptr;
            d.items = p.P;
            d.nsteps = (int)(p.n_steps / p.P);
            d.item_steps = p.n_steps / p.P;
            d.n_t = p.n_steps;
            d.nx = p.nx;
            d.ny = p.ny;
            d.dt = c.dt();
            d.omega = p.omega;
            d.A = transpose5(advdiff2d_sten(p));
            at.push_back(d);
        }
        if (!at.empty()) {
            const std::vector<Group2D> ag = group2d(at);
            HIPCHK(launch_upload(dtab, at.data(), at.size() * sizeof(Band2D), s));
            ProfScope ps(PXP_K_ADJ_SLICES, s);
            for (const Group2D& g : ag)
                HIPCHK(launch_band2d_rsrc(dtab + g.first, g.count, g.blocks, g.nx, 0, 0, s));
        }
        std::vector<std::vector<std::vector<PJob>>> per;
        std::vector<PoisWeights> wt;
        for (size_t j = 0; j < idx.size(); ++j) {
            const pxp_problem& p = pb[idx[j]];
            if (!has_src((int)j) || (!lam0[j] && !Lam[j]) || p.P < 2) continue;
            Ctx c = make_ctx(p, ws, Ly, idx[j], s);
            const TShape sh = tree_shape(p.P);
            per.emplace_back();
            adj_tree_levels(p, c, sh, kept_bufs(c, sh), lam0[j] ? lam0[j] : c.at(c.L.lam0),
                            Lam[j], wt, per.back());
        }
        if (!per.empty()) {
            ProfScope ps(PXP_K_KRYLOV_ADJOINT, s);
            if (!wt.empty()) {
                auto* dw = reinterpret_cast<PoisWeights*>(static_cast<char*>(ws) + Ly.pwt);
                const size_t bytes = wt.size() * sizeof(PoisWeights);
                for (size_t o = 0; o < bytes; o += 3072)
                    HIPCHK(launch_upload(reinterpret_cast<char*>(dw) + o,
                                         reinterpret_cast<const char*>(wt.data()) + o,
                                         std::min((size_t)3072, bytes - o), s));
                HIPCHK(launch_pois_weights(dw, (int)wt.size(), s));
            }
            auto* dp = reinterpret_cast<PoisEntry*>(static_cast<char*>(ws) + Ly.ptab);
            pxp_status st = run_levels(per, dp, Ly.ptab_entries, s);
            if (st != PXP_OK) return st;
        }
        for (size_t j = 0; j < idx.size(); ++j) {
            const pxp_problem& p = pb[idx[j]];
            if (!has_src((int)j) || (!lam0[j] && !Lam[j])) continue;
            Ctx c = make_ctx(p, ws, Ly, idx[j], s);
            if (p.P == 1 && lam0[j])
                HIPCHK(launch_add(nullptr, c.at(c.L.slices), lam0[j], c.n(), s));
        }
    }
    // one homogeneous piece per instance from q^dagger(T) over [T, 0]
    // (eq. adjhomfinal).  Uniformised: substeps of at most POIS_LMAX, the
    // time integral Lambda by the exact integral weights of every term.
    {
        std::vector<std::vector<std::vector<PJob>>> per;
        std::vector<PoisWeights> wt;
        for (size_t j = 0; j < idx.size(); ++j) {
            const pxp_problem& p = pb[idx[j]];
            if (!uniform_adjoint(p) || (!lam0[j] && !Lam[j]) || has_src((int)j)) continue;
            Ctx c = make_ctx(p, ws, Ly, idx[j], s);
            const int64_t n = c.n();
            const AdjPlan ap = adj_plan(p);
            const Sten5 AT = transpose5(advdiff2d_sten(p));
            const double mu = uniform_mu(AT);
            double* wbase = c.at(c.L.wtab);
            double* ub = c.at(c.L.ubuf);
            per.emplace_back();
            for (int q = 0; q < ap.nsub; ++q) {
                double* w = wbase + (size_t)q * 2 * ap.D;
                if (Lam[j]) {
                    PoisWeights pw{};
                    pw.w = w;
                    pw.wi = w + ap.D;
                    pw.D = ap.D;
                    pw.lam = ap.lam;
                    pw.mu = mu;
                    pw.omega = p.omega;
                    pw.phi = p.omega * (p.T - q * ap.h);
                    pw.scale = 1.0 / mu;
                    wt.push_back(pw);
                }
                PJob b;
                b.lam = ap.lam;
                b.D = ap.D;
                b.est = ap.est;
                b.nx = p.nx;
                b.ny = p.ny;
                b.N = uniform_N(AT, mu);
                b.st = c.st;
                b.irep = c.irep;
                b.tb[0] = c.at(c.L.tbuf);
                b.tb[1] = b.tb[0] + n;
                b.sx = b.sp = b.so = n;
                b.x = q == 0 ? lamT[j] : ub + (size_t)((q - 1) & 1) * n;
                const bool last = q + 1 == ap.nsub;
                if (ap.nsub == 1 && !lam0[j]) {
                    // Lambda only: one sum with the integral weights
                    b.out = Lam[j];
                    b.wtab = w;
                } else {
                    b.out = (last && lam0[j]) ? lam0[j] : ub + (size_t)(q & 1) * n;
                    if (Lam[j]) {
                        b.wtab2 = w;
                        b.out2 = Lam[j];
                        // the second sum of later substeps builds beside
                        // Lambda and is added to it at the end
                        b.acc2 = q == 0 ? Lam[j] : ub + 2 * (size_t)n;
                        b.out2_add = q == 0 ? nullptr : Lam[j];
                    }
                }
                per.back().push_back({b});
            }
        }
        if (!per.empty()) {
            ProfScope ps(PXP_K_KRYLOV_ADJOINT, s);
            if (!wt.empty()) {
                auto* dw = reinterpret_cast<PoisWeights*>(static_cast<char*>(ws) + Ly.pwt);
                const size_t bytes = wt.size() * sizeof(PoisWeights);
                for (size_t o = 0; o < bytes; o += 3072)
                    HIPCHK(launch_upload(reinterpret_cast<char*>(dw) + o,
                                         reinterpret_cast<const char*>(wt.data()) + o,
                                         std::min((size_t)3072, bytes - o), s));
                HIPCHK(launch_pois_weights(dw, (int)wt.size(), s));
            }
            auto* dp = reinterpret_cast<PoisEntry*>(static_cast<char*>(ws) + Ly.ptab);
            pxp_status st = run_levels(per, dp, Ly.ptab_entries, s);
            if (st != PXP_OK) return st;
        }
    }
    std::vector<KrylovArgs> kt;
    for (size_t j = 0; j < idx.size(); ++j) {
        const pxp_problem& p = pb[idx[j]];
        if (!lam0[j] && !Lam[j]) continue;
        if (uniform_adjoint(p)) continue;
        Ctx c = make_ctx(p, ws, Ly, idx[j], s);
        KrylovArgs a = kargs(c, Tri{0.0, 0.0, 0.0});
        a.op5 = transpose5(advdiff2d_sten(p));
        a.anorm = sten_norm(a.op5);
        a.nx = p.nx;
        a.ny = p.ny;
        a.mode = KM_SINGLE;
        a.npieces = 1;
        a.vin = lamT[j];
        a.yout = lam0[j];
        a.iout = Lam[j];
        a.tau = p.T;
        a.ia = p.omega * p.T;
        a.ib = -p.omega;
        kt.push_back(a);
    }
    if (kt.empty()) return PXP_OK;
    auto* dk = reinterpret_cast<KrylovArgs*>(static_cast<char*>(ws) + Ly.ktab);
    ProfScope ps(PXP_K_KRYLOV_ADJOINT, s);
    return launch_krylov2d_groups(kt, dk, s);
}

}  // namespace
}  // namespace pxp

using namespace pxp;

extern "C" {

const char* pxp_version(void) { return "paraexp-mi355x 0.1"; }

const char* pxp_status_str(pxp_status s) {
    switch (s) {
        case PXP_OK: return "ok";
        case PXP_EINVAL: return "invalid argument";
        case PXP_EUNSUPPORTED: return "unsupported problem";
        case PXP_EWORKSPACE: return "workspace missing, misaligned or too small";
        case PXP_EUNSTABLE_DT: return "time step outside the RK4 stability bound";
        case PXP_EKRYLOV_NOCONV: return "Krylov error estimate above tolerance";
        case PXP_ENONFINITE: return "non-finite value";
        case PXP_EHIP: return "HIP runtime error";
    }
    return "unknown status";
}

pxp_status pxp_workspace_size(const pxp_problem* pb, int32_t batch,
                              size_t* bytes) {
    if (!bytes) return PXP_EINVAL;
    pxp_status st = check_all(pb, batch);
    if (st != PXP_OK) return st;
    *bytes = layout(pb, batch).total;
    return PXP_OK;
}

pxp_status pxp_workspace_init(void* ws, size_t ws_bytes, void* stream) {
    if (!ws || ws_bytes < sizeof(DevStatus)) return PXP_EWORKSPACE;
    side_init();
    // the whole workspace starts at zero: the status block and the
    // per-instance statistics accumulate from there
    if (launch_zero(static_cast<double*>(ws), ws_bytes / sizeof(double),
                    static_cast<hipStream_t>(stream)) != hipSuccess)
        return PXP_EHIP;
    return PXP_OK;
}

// Flavour of the direct and of the adjoint exponentials as they run.
int flavour_direct(const pxp_problem& p) {
    // Burgers: the direct march is serial, except in the nonlinear iteration
    if (p.op == PXP_OP_BURGERS1D && !nlpx(p)) return -1;
    if (uniform_direct(p)) return PXP_KRYLOV_UNIFORM;
    if (use_si(p)) return PXP_KRYLOV_SHIFT_INVERT;
    if (use_cheb(p)) return PXP_KRYLOV_CHEBYSHEV;
    return use_taylor(p) ? PXP_KRYLOV_TAYLOR : PXP_KRYLOV_POLY;
}
int flavour_adjoint(const pxp_problem& p) {
    if (uniform_adjoint(p)) return PXP_KRYLOV_UNIFORM;
    if (use_si(p)) return PXP_KRYLOV_SHIFT_INVERT;
    if (use_cheb(p)) return PXP_KRYLOV_CHEBYSHEV;
    return use_taylor(p) ? PXP_KRYLOV_TAYLOR : PXP_KRYLOV_POLY;
}

pxp_status pxp_last_report(const pxp_problem* pb, int32_t batch, void* ws, size_t ws_bytes,
                           void* stream, pxp_report* out) {
    pxp_status st = check_all(pb, batch);
    if (st != PXP_OK) return st;
    if (batch == 0) return PXP_OK;
    if (!out) return PXP_EINVAL;
    Layout Ly;
    st = ws_check(pb, batch, ws, ws_bytes, &Ly);
    if (st != PXP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipStreamSynchronize(s) != hipSuccess) return PXP_EHIP;
    std::vector<InstStat> h(batch);
    char* w = static_cast<char*>(ws);
    if (hipMemcpy(h.data(), w + Ly.irep, batch * sizeof(InstStat), hipMemcpyDeviceToHost) !=
        hipSuccess)
        return PXP_EHIP;
    for (int i = 0; i < batch; ++i) {
        const pxp_problem& p = pb[i];
        pxp_report& r = out[i];
        r.P = p.P;
        r.sched = (p.op == PXP_OP_BURGERS1D) ? (nlpx(p) ? PXP_SCHED_CHAIN : -1) : p.sched;
        r.krylov_direct = flavour_direct(p);
        r.krylov_adjoint = flavour_adjoint(p);
        r.substeps = h[i].substeps;
        r.iterations = h[i].iters;
        std::memcpy(&r.max_est, &h[i].max_est, sizeof(double));
        r.nl_iterations = (int32_t)h[i].nl_iters;
        r.pad = 0;
    }
    if (launch_zero(reinterpret_cast<double*>(w + Ly.irep),
                    batch * sizeof(InstStat) / sizeof(double), s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return PXP_EHIP;
    return PXP_OK;
}

static pxp_status direct_impl(const pxp_problem* pb, int32_t batch,
                              const double* q0, const double* F, double* qT,
                              void* ws, size_t ws_bytes, void* stream,
                              int method) {
    pxp_status st = check_all(pb, batch);
    if (st == PXP_OK) st = check_method(pb, batch, method);
    if (st != PXP_OK) return st;
    if (batch == 0) return PXP_OK;
    if (!qT) return PXP_EINVAL;
    Layout Ly;
    st = ws_check(pb, batch, ws, ws_bytes, &Ly);
    if (st != PXP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    size_t off = 0;
    // the 2D kernels move whole rows with 16-byte accesses
    for (int i = 0; i < batch; ++i) {
        if (pb[i].op == PXP_OP_ADVDIFF2D_UPWIND &&
            (!aligned16(q0, off) || !aligned16(F, off) || !aligned16(qT, off)))
            return PXP_EINVAL;
        off += (size_t)grid_n(pb[i]);
    }
    off = 0;
    const std::vector<int> idx2 = batch2d(pb, batch);
    std::vector<const double*> i2, f2;
    std::vector<double*> o2;
    for (int i = 0; i < batch; ++i) {
        const pxp_problem& p = pb[i];
        Ctx c = make_ctx(p, ws, Ly, i, s);
        const double* q0i = q0 ? q0 + off : nullptr;
        const double* Fi = F ? F + off : nullptr;
        if (p.op == PXP_OP_ADVDIFF2D_UPWIND) {
            i2.push_back(q0i);
            f2.push_back(Fi);
            o2.push_back(qT + off);
        } else if (p.op == PXP_OP_ADVDIFF1D) {
            st = direct_lin1d(c, q0i, Fi, qT + off, method);
        } else {
            if (!q0i) return PXP_EINVAL;
            st = direct_burgers(c, q0i, qT + off, method);
        }
        if (st != PXP_OK) return st;
        off += (size_t)grid_n(p);
    }
    return direct_2d_batch(pb, idx2, ws, Ly, i2, f2, o2, method, s);
}

pxp_status paraexp_direct(const pxp_problem* pb, int32_t batch,
                          const double* q0, const double* F, double* qT,
                          void* ws, size_t ws_bytes, void* stream) {
    return direct_impl(pb, batch, q0, F, qT, ws, ws_bytes, stream,
                       PXP_METHOD_PARAEXP);
}

static pxp_status adjoint_impl(const pxp_problem* pb, int32_t batch,
                               const double* lamT, const double* jI_src, double* lam0,
                               double* Lambda, void* ws, size_t ws_bytes, void* stream,
                               int method) {
    pxp_status st = check_all(pb, batch);
    if (st != PXP_OK) return st;
    // step sources: the integral-cost path of the 2D problems only (its
    // workspace holds the adjoint slices' buffers)
    if (jI_src)
        for (int i = 0; i < batch; ++i)
            if (pb[i].op != PXP_OP_ADVDIFF2D_UPWIND || !icost(pb[i])) return PXP_EUNSUPPORTED;
    if (batch == 0) return PXP_OK;
    if (!lamT && !jI_src) return PXP_EINVAL;
    Layout Ly;
    st = ws_check(pb, batch, ws, ws_bytes, &Ly);
    if (st != PXP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    size_t off = 0;
    size_t goff = 0;
    for (int i = 0; i < batch; ++i) {
        if (!aligned16(lamT, off) || !aligned16(lam0, off) || !aligned16(Lambda, off))
            return PXP_EINVAL;
        if (jI_src && !aligned16(jI_src, goff)) return PXP_EINVAL;
        off += (size_t)grid_n(pb[i]);
        goff += ((size_t)pb[i].n_steps + 1) * (size_t)grid_n(pb[i]);
    }
    off = 0;
    goff = 0;
    const std::vector<int> idx2 = batch2d(pb, batch);
    std::vector<const double*> l2, g2;
    std::vector<double*> z2, L2;
    for (int i = 0; i < batch; ++i) {
        const pxp_problem& p = pb[i];
        Ctx c = make_ctx(p, ws, Ly, i, s);
        if (p.op == PXP_OP_ADVDIFF2D_UPWIND) {
            g2.push_back(jI_src ? jI_src + goff : nullptr);
            goff += ((size_t)p.n_steps + 1) * (size_t)grid_n(p);
            l2.push_back(lamT ? lamT + off : nullptr);
            z2.push_back(lam0 ? lam0 + off : nullptr);
            L2.push_back(Lambda ? Lambda + off : nullptr);
        } else if (p.op == PXP_OP_ADVDIFF1D) {
            st = adjoint_lin1d(c, lamT + off, lam0 ? lam0 + off : nullptr,
                               Lambda ? Lambda + off : nullptr, method);
        } else {
            if (Lambda) return PXP_EINVAL;  // no forcing control for Burgers
            if (!lam0) return PXP_EINVAL;
            st = adjoint_burgers(c, lamT + off, lam0 + off, method);
        }
        if (st != PXP_OK) return st;
        off += (size_t)grid_n(p);
    }
    return adjoint_2d_batch(pb, idx2, ws, Ly, l2, z2, L2, method, s, &g2);
}

pxp_status paraexp_adjoint(const pxp_problem* pb, int32_t batch,
                           const double* lamT, const double* jI_src, double* lam0,
                           double* Lambda, void* ws, size_t ws_bytes, void* stream) {
    return adjoint_impl(pb, batch, lamT, jI_src, lam0, Lambda, ws, ws_bytes, stream,
                        PXP_METHOD_PARAEXP);
}

pxp_status pxp_gradient(const pxp_problem* pb, int32_t batch, int32_t method,
                        const double* ctrl, const double* basis,
                        const double* q0, const double* u_tgt, double* J,
                        double* grad, double* qT, double* lam_out, void* ws,
                        size_t ws_bytes, void* stream) {
    pxp_status st = check_all(pb, batch);
    if (st != PXP_OK) return st;
    if (method != PXP_METHOD_PARAEXP && method != PXP_METHOD_SERIAL)
        return PXP_EINVAL;
    st = check_method(pb, batch, method);
    if (st != PXP_OK) return st;
    if (batch == 0) return PXP_OK;
    if (!u_tgt || !J || !grad) return PXP_EINVAL;
    Layout Ly;
    st = ws_check(pb, batch, ws, ws_bytes, &Ly);
    if (st != PXP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // per-instance pointers
    struct IP {
        const double *a, *G, *q0, *F, *init, *tgt;
        double *qT, *lamT, *lam0, *Lam;
        int n, K;
        size_t off, koff;
    };
    std::vector<IP> ip(batch);
    {
        size_t off = 0, koff = 0, boff = 0;
        for (int i = 0; i < batch; ++i) {
            const pxp_problem& p = pb[i];
            const int n = (int)grid_n(p), K = p.K;
            if (K > 0 && (!ctrl || !basis)) return PXP_EINVAL;
            // the 2D kernels move whole rows with 16-byte accesses
            if (p.op == PXP_OP_ADVDIFF2D_UPWIND &&
                (!aligned16(q0, off) || !aligned16(qT, off) || !aligned16(u_tgt, off)))
                return PXP_EINVAL;
            Ctx c = make_ctx(p, ws, Ly, i, s);
            IP& x = ip[i];
            x.a = ctrl ? ctrl + koff : nullptr;
            x.G = basis ? basis + boff : nullptr;
            x.q0 = q0 ? q0 + off : nullptr;
            x.tgt = u_tgt + off;
            x.qT = qT ? qT + off : c.at(c.L.qT);
            x.lamT = c.at(c.L.lamT);
            x.lam0 = c.at(c.L.lam0);
            x.Lam = c.at(c.L.Lam);
            x.F = (p.ctrl == PXP_CTRL_FORCING) ? c.at(c.L.F) : nullptr;
            x.init = (p.ctrl == PXP_CTRL_FORCING) ? x.q0 : c.at(c.L.q0eff);
            if (p.op == PXP_OP_BURGERS1D && !x.init) return PXP_EINVAL;
            x.n = n;
            x.K = K;
            x.off = off;
            x.koff = koff;
            off += (size_t)n;
            koff += (size_t)K;
            boff += (size_t)K * n;
        }
    }
    const BurgersBatch bb = burgers_batch(pb, batch);
    std::vector<int> npart(batch, 0);  // integral cost: cost partials per instance
    // (a1) controls -> forcing pattern or initial state
    for (int i = 0; i < batch; ++i) {
        const pxp_problem& p = pb[i];
        Ctx c = make_ctx(p, ws, Ly, i, s);
        if (p.ctrl == PXP_CTRL_FORCING)
            HIPCHK(launch_combine_basis(ip[i].a, ip[i].G, nullptr, c.at(c.L.F),
                                        ip[i].K, ip[i].n, s));
        else
            HIPCHK(launch_combine_basis(ip[i].a, ip[i].G, ip[i].q0, c.at(c.L.q0eff),
                                        ip[i].K, ip[i].n, s));
    }
    // (a2-a4, a10) direct
    std::vector<const double*> binit;
    std::vector<double*> bqT, blamT, blam0;
    const std::vector<int> idx2 = batch2d(pb, batch);
    std::vector<const double*> i2, f2;
    std::vector<double*> o2;
    for (int i = 0; i < batch; ++i) {
        const pxp_problem& p = pb[i];
        if (p.op == PXP_OP_ADVDIFF2D_UPWIND) {
            i2.push_back(ip[i].init);
            f2.push_back(ip[i].F);
            o2.push_back(ip[i].qT);
            continue;
        }
        if (bb.on && in_batch(bb, i)) {
            binit.push_back(ip[i].init);
            bqT.push_back(ip[i].qT);
            blamT.push_back(ip[i].lamT);
            blam0.push_back(ip[i].lam0);
            continue;
        }
        Ctx c = make_ctx(p, ws, Ly, i, s);
        if (p.op == PXP_OP_BURGERS1D && icost(p))
            st = direct_burgers_icost(c, ip[i].init, ip[i].tgt, ip[i].qT, method, &npart[i]);
        else
            st = (p.op == PXP_OP_ADVDIFF1D)
                     ? direct_lin1d(c, ip[i].init, ip[i].F, ip[i].qT, method)
                     : direct_burgers(c, ip[i].init, ip[i].qT, method);
        if (st != PXP_OK) return st;
    }
    if (bb.on) {
        st = burgers_batch_direct(pb, bb, ws, Ly, binit, bqT, s);
        if (st != PXP_OK) return st;
    }
    // integral-cost instances: their targets, for the step sources
    std::vector<const double*> t2(idx2.size(), nullptr);
    std::vector<int> np2(idx2.size(), 0);
    for (size_t j = 0; j < idx2.size(); ++j)
        if (icost(pb[idx2[j]])) t2[j] = ip[idx2[j]].tgt;
    st = direct_2d_batch(pb, idx2, ws, Ly, i2, f2, o2, method, s, &t2, &np2);
    if (st != PXP_OK) return st;
    for (size_t j = 0; j < idx2.size(); ++j) npart[idx2[j]] = np2[j];
    // (a5) cost and adjoint final condition, every instance in two launches
    // (integral cost: the partials of the source march; no final condition)
    auto* dst = reinterpret_cast<DevStatus*>(static_cast<char*>(ws) + Ly.status);
    std::vector<RedDesc> rd(batch);
    int bcost = 0, bgrad = 0;
    {
        int64_t po = 0;
        for (int i = 0; i < batch; ++i) {
            RedDesc& d = rd[i];
            const bool forcing = (pb[i].ctrl == PXP_CTRL_FORCING);
            d.qT = ip[i].qT;
            d.tgt = ip[i].tgt;
            d.lamT = ip[i].lamT;
            d.a = ip[i].a;
            d.J = J + i;
            d.basis = ip[i].G;
            d.v = forcing ? ip[i].Lam : ip[i].lam0;
            d.grad = grad + ip[i].koff;
            d.beta = pb[i].beta;
            d.st = dst;
            d.n = ip[i].n;
            d.K = ip[i].K;
            d.chunks = (d.n + RED_CHUNK - 1) / RED_CHUNK;
            d.blk0_cost = bcost;
            d.blk0_grad = bgrad;
            d.part0 = po;
            d.gpart0 = po + d.chunks;
            po += (int64_t)(d.K + 1) * d.chunks;
            if (icost(pb[i])) {
                Ctx c = make_ctx(pb[i], ws, Ly, i, s);
                d.ipart = c.at(c.L.cpart);
                d.ichunks = npart[i];
                d.lamT = nullptr;
            } else {
                bcost += d.chunks;
            }
            bgrad += d.K * d.chunks;
        }
    }
    auto* drd = reinterpret_cast<RedDesc*>(static_cast<char*>(ws) + Ly.rtab);
    double* rpart = reinterpret_cast<double*>(static_cast<char*>(ws) + Ly.rpart);
    HIPCHK(launch_upload(drd, rd.data(), rd.size() * sizeof(RedDesc), s));
    HIPCHK(launch_cost_batch(drd, batch, bcost, rpart, s));
    // (a6-a8) adjoint
    std::vector<const double*> l2, g2;
    std::vector<double*> z2, L2;
    for (int i = 0; i < batch; ++i) {
        const pxp_problem& p = pb[i];
        const bool forcing = (p.ctrl == PXP_CTRL_FORCING);
        if (p.op == PXP_OP_ADVDIFF2D_UPWIND) {
            Ctx c = make_ctx(p, ws, Ly, i, s);
            l2.push_back(icost(p) ? nullptr : ip[i].lamT);
            g2.push_back(icost(p) ? c.at(c.L.gsrc) : nullptr);
            z2.push_back(forcing ? nullptr : ip[i].lam0);
            L2.push_back(forcing ? ip[i].Lam : nullptr);
            continue;
        }
        if (bb.on && in_batch(bb, i)) continue;
        Ctx c = make_ctx(p, ws, Ly, i, s);
        if (p.op == PXP_OP_BURGERS1D && icost(p))
            st = adjoint_burgers_icost(c, ip[i].qT, ip[i].tgt, ip[i].lam0, method);
        else
            st = (p.op == PXP_OP_ADVDIFF1D)
                     ? adjoint_lin1d(c, ip[i].lamT, forcing ? nullptr : ip[i].lam0,
                                     forcing ? ip[i].Lam : nullptr, method)
                     : adjoint_burgers(c, ip[i].lamT, ip[i].lam0, method);
        if (st != PXP_OK) return st;
    }
    if (bb.on) {
        st = burgers_batch_adjoint(pb, bb, ws, Ly, blamT, blam0, method, s);
        if (st != PXP_OK) return st;
    }
    st = adjoint_2d_batch(pb, idx2, ws, Ly, l2, z2, L2, method, s, &g2);
    if (st != PXP_OK) return st;
    // (a9) gradient, every instance in two launches
    HIPCHK(launch_grad_batch(drd, batch, bgrad, rpart, s));
    if (lam_out)
        for (int i = 0; i < batch; ++i)
            HIPCHK(launch_add(nullptr, rd[i].v, lam_out + ip[i].off, ip[i].n, s));
    return PXP_OK;
}

pxp_status gradient(const pxp_problem* pb, int32_t batch, const double* ctrl,
                    const double* basis, const double* q0, const double* u_tgt,
                    double* J, double* grad, double* qT, void* ws,
                    size_t ws_bytes, void* stream) {
    return pxp_gradient(pb, batch, PXP_METHOD_PARAEXP, ctrl, basis, q0, u_tgt,
                        J, grad, qT, nullptr, ws, ws_bytes, stream);
}

pxp_status pxp_assemble(const pxp_problem* pb, int32_t batch, const double* ctrl,
                        const double* basis, const double* base, double* out,
                        void* stream) {
    pxp_status st = check_all(pb, batch);
    if (st != PXP_OK) return st;
    if (batch > 0 && !out) return PXP_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    size_t off = 0, koff = 0, boff = 0;
    for (int i = 0; i < batch; ++i) {
        const int n = (int)grid_n(pb[i]), K = pb[i].K;
        if (K > 0 && (!ctrl || !basis)) return PXP_EINVAL;
        HIPCHK(launch_combine_basis(ctrl ? ctrl + koff : nullptr,
                                    basis ? basis + boff : nullptr,
                                    base ? base + off : nullptr, out + off, K, n, s));
        off += (size_t)n;
        koff += (size_t)K;
        boff += (size_t)K * n;
    }
    return PXP_OK;
}

pxp_status pxp_cost(const pxp_problem* pb, int32_t batch, const double* qT,
                    const double* u_tgt, const double* ctrl, double* J,
                    double* lamT, void* stream) {
    pxp_status st = check_all(pb, batch);
    if (st != PXP_OK) return st;
    // the integral cost needs the trajectory: pxp_gradient forms it
    for (int i = 0; i < batch; ++i)
        if (icost(pb[i])) return PXP_EUNSUPPORTED;
    if (batch > 0 && (!qT || !u_tgt || !J)) return PXP_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    size_t off = 0, koff = 0;
    for (int i = 0; i < batch; ++i) {
        const int n = (int)grid_n(pb[i]), K = pb[i].K;
        if (K > 0 && !ctrl) return PXP_EINVAL;
        HIPCHK(launch_cost(qT + off, u_tgt + off, ctrl ? ctrl + koff : nullptr, n,
                           ctrl ? K : 0, pb[i].beta, lamT ? lamT + off : nullptr,
                           J + i, s));
        off += (size_t)n;
        koff += (size_t)K;
    }
    return PXP_OK;
}

pxp_status pxp_reduce_gradient(const pxp_problem* pb, int32_t batch,
                               const double* basis, const double* v,
                               const double* ctrl, double* grad, void* stream) {
    pxp_status st = check_all(pb, batch);
    if (st != PXP_OK) return st;
    if (batch > 0 && (!basis || !v || !ctrl || !grad)) return PXP_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    size_t off = 0, koff = 0, boff = 0;
    for (int i = 0; i < batch; ++i) {
        const int n = (int)grid_n(pb[i]), K = pb[i].K;
        HIPCHK(launch_grad(basis + boff, v + off, ctrl + koff, K, n, pb[i].beta,
                           grad + koff, s));
        off += (size_t)n;
        koff += (size_t)K;
        boff += (size_t)K * n;
    }
    return PXP_OK;
}

pxp_status pxp_device_status(void* ws, size_t ws_bytes, void* stream,
                             double* max_est) {
    if (!ws || ws_bytes < sizeof(DevStatus)) return PXP_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipStreamSynchronize(s) != hipSuccess) return PXP_EHIP;
    DevStatus h{};
    if (hipMemcpy(&h, ws, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
        return PXP_EHIP;
    if (max_est) {
        double e;
        std::memcpy(&e, &h.max_est, sizeof(e));
        *max_est = e;
    }
    if (launch_zero(static_cast<double*>(ws), sizeof(DevStatus) / sizeof(double), s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return PXP_EHIP;
    if (h.flags & ST_NONFINITE) return PXP_ENONFINITE;
    if (h.flags & ST_NOCONV) return PXP_EKRYLOV_NOCONV;
    return PXP_OK;
}

pxp_status pxp_device_counters(void* ws, size_t ws_bytes, void* stream,
                               uint64_t* substeps, uint64_t* krylov_iters,
                               uint64_t* reorth_passes) {
    if (!ws || ws_bytes < sizeof(DevStatus)) return PXP_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipStreamSynchronize(s) != hipSuccess) return PXP_EHIP;
    DevStatus h{};
    if (hipMemcpy(&h, ws, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
        return PXP_EHIP;
    if (substeps) *substeps = h.substeps[0] + h.substeps[1];
    if (krylov_iters) *krylov_iters = h.krylov_iters[0] + h.krylov_iters[1];
    if (reorth_passes) *reorth_passes = h.reorth[0] + h.reorth[1];
    return PXP_OK;
}

pxp_status pxp_device_counters_class(void* ws, size_t ws_bytes, void* stream, int32_t cls,
                                     uint64_t* substeps, uint64_t* krylov_iters,
                                     uint64_t* reorth_passes) {
    if (cls != 0 && cls != 1) return PXP_EINVAL;
    if (!ws || ws_bytes < sizeof(DevStatus)) return PXP_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipStreamSynchronize(s) != hipSuccess) return PXP_EHIP;
    DevStatus h{};
    if (hipMemcpy(&h, ws, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
        return PXP_EHIP;
    if (substeps) *substeps = h.substeps[cls];
    if (krylov_iters) *krylov_iters = h.krylov_iters[cls];
    if (reorth_passes) *reorth_passes = h.reorth[cls];
    return PXP_OK;
}

pxp_status pxp_profile_enable(int32_t on) {
    g_prof.on = (on != 0);
    return PXP_OK;
}

pxp_status pxp_profile_read(int32_t kernel_class, double* total_ms,
                            int32_t* count) {
    if (!total_ms || !count) return PXP_EINVAL;
    double tot = 0.0;
    int cnt = 0;
    std::vector<Profiler::Rec> keep;
    for (auto& r : g_prof.recs) {
        if (r.cls != kernel_class) {
            keep.push_back(r);
            continue;
        }
        if (hipEventSynchronize(r.b) != hipSuccess) return PXP_EHIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return PXP_EHIP;
        tot += ms;
        ++cnt;
        g_prof.pool.push_back(r.a);
        g_prof.pool.push_back(r.b);
    }
    g_prof.recs.swap(keep);
    *total_ms = tot;
    *count = cnt;
    return PXP_OK;
}

}  // extern "C"
