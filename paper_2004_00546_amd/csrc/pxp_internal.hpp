// Internal launcher interface between the C ABI / host engine and the HIP
// kernels.  Every launcher enqueues on the given stream and returns the HIP
// launch status; none allocates or synchronises.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pxp {

// Periodic tridiagonal operator (Op x)_i = lo x_{i-1} + d x_i + up x_{i+1}.
struct Tri {
    double lo, d, up;
};

// Periodic 2D five-point operator on a row-major grid (x fastest):
// (Op x)_{j,i} = c x_{j,i} + w x_{j,i-1} + e x_{j,i+1} + s x_{j-1,i} + n x_{j+1,i}
struct Sten5 {
    double c, w, e, s, n;
};

// Device-side status block at the start of every workspace.
struct DevStatus {
    unsigned int flags;          // bit 0: Krylov estimate above tolerance,
                                 // bit 1: non-finite value met
    unsigned int pad;
    unsigned long long max_est;  // bit pattern of the largest relative est.
    // per class: [0] direct pieces, [1] adjoint pieces
    unsigned long long substeps[2];      // accepted Krylov substeps
    unsigned long long krylov_iters[2];  // Arnoldi steps (Taylor: terms)
    unsigned long long reorth[2];        // Arnoldi steps that took a second
                                         // Gram-Schmidt pass
};
static_assert(sizeof(DevStatus) == 64, "status block layout");
// Per-instance statistics beside the status block: Krylov substeps and
// iterations (Arnoldi steps, or series terms) and the largest error estimate
// (bit pattern) of one instance's exponentials, and the iterations of the
// nonlinear Paraexp direct that ran, since the last read.
struct InstStat {
    unsigned long long substeps, iters, max_est, nl_iters;
};
constexpr unsigned int ST_NOCONV = 1u;
constexpr unsigned int ST_NONFINITE = 2u;

// ---- RK4 marches (1D, one workgroup per slice) ---------------------------
// fp32 != 0: stencil and RK arithmetic in FP32 with compensated (Kahan)
// accumulation of the state and adjoint sums; inputs, outputs and
// checkpoints stay FP64 (an FP32 compensated pair is exact in FP64).
// Optional time integral of each slice's march: iout[p] = int over the
// slice of sin(ia + ib t) y(t) dt (RK4 stages of the extra equation), plus
// c0 * v0 for slice 0 when v0 is given.  iout null: none.
struct SliceIntegral {
    double* iout;
    double ia, ib, c0;
    const double* v0;
};
// Slices p = 0..P-1 of a linear 1D problem, each from zero (or from y0 when
// given, P must then be 1) over n_s steps starting at global step p*n_s:
//   y' = A y + sin(omega t) F + g0.
hipError_t launch_rk4_lin1d(const double* F, const double* g0, const double* y0,
                            double* out, int n, int P, int64_t n_s, double dt,
                            double omega, Tri A, int block, int fp32, hipStream_t s,
                            SliceIntegral si = SliceIntegral{nullptr, 0.0, 0.0, 0.0, nullptr});

// Reverse sweep of the exact discrete adjoint of the linear RK4 march:
// from lamT to lam0 and Lambda = sum s(t_stage) kbar_stage.
hipError_t launch_rk4_rev_lin1d(const double* lamT, double* lam0,
                                double* Lambda, int n, int64_t n_t, double dt,
                                double omega, Tri AT, int block, int fp32,
                                hipStream_t s);

// Burgers 1D direct march with checkpoints every c steps (ckpt[k] = state at
// step k*c, k = 0..n_t/c).
// Step range and integral-cost terms of a Burgers march (the cost of
// section 4.2 on the problem of section 4.3): steps [s0, s1) of n_t, the
// states at step s0 in / at s1 out.  With tgt set, the step sources are
// g_s = gw c_s (q_s - tgt), c_s = 1/2 at both ends and 1 inside.  Forward:
// the workgroup's share of J, sum over s0 <= s < s1 (and s = n_t when
// s1 = n_t) of w_s |q_s - tgt|^2 (w_s = gw c_s / 2), into *cpart.  Reverse:
// g_s added after the step that produces lambda_s, formed from the step
// states the sweep recomputes from the checkpoints (g_{s1} added to the
// start vector when src_start, from the checkpoint at s1).  Ranges of the
// reverse sweep start and end on checkpoints.
struct BurgersRange {
    int64_t s0, s1;
    const double* tgt;
    double gw;
    double* cpart;
    int src_start, pad;
};
// Iterative nonlinear Paraexp for Burgers (section 3.2).  Device state of
// one call's iteration (in the workspace): done = an iteration's change of
// q(T) was within the tolerance, after which every launch of the call that
// takes the state returns at once; last = the stage-state generation that
// holds the last iterate; change = the last iteration's relative change.
struct NlState {
    int done, last;
    double change;
};
// One workgroup per slice p of P (S steps each): the linearised march of
// iterate i+1 with the previous stage states st_old ([n_t][4][n]) as
// sources and J at W + p n, from q0 (p = 0, when set), E + (p-1) n (p > 0,
// when set) or zero; writes st_new (nullable), the end states reversed
// (vend + (P-1-p) n, nullable) and q(T) (last slice, nullable).
hipError_t launch_burgers_nl_march(const double* st_old, double* st_new, double* vend,
                                   const double* E, const double* q0, double* qT,
                                   const double* W, int n, int64_t S, int P, double dt,
                                   double nu, double L, int block, const NlState* ns,
                                   hipStream_t s);
// W + p n = trapezoidal time average of slice p's step states (the last
// slice ends on qlast)
hipError_t launch_nl_slice_mean(const double* st, const double* qlast, double* W, int n,
                                int64_t S, int P, const NlState* ns, hipStream_t s);
// every stage state of nst = 4 n_t stages = q0, qprev = q0, the state reset
hipError_t launch_nl_fill(const double* q0, double* st, double* qprev, NlState* ns, int n,
                          int64_t nst, hipStream_t s);
// the change |qT - qprev| / |qT| of an iteration that wrote generation gen:
// sets done when within tol, then qprev = qT (skipped once done)
hipError_t launch_nl_change(const double* qT, double* qprev, int n, double tol, NlState* ns,
                            int gen, InstStat* irep, hipStream_t s);
// the last change into the status block (estimate; NOCONV above tol)
hipError_t launch_nl_final(const NlState* ns, double tol, DevStatus* st, InstStat* irep,
                           hipStream_t s);
// checkpoints every c steps from the last iterate's step states, q(T) at n_t
hipError_t launch_nl_ckpt(const double* st0, const double* st1, const NlState* ns,
                          const double* qT, double* ckpt, int n, int64_t n_t, int64_t c,
                          hipStream_t s);
// out = a (x - y) on n points
hipError_t launch_scaled_diff(const double* x, const double* y, double a, double* out, int n,
                              hipStream_t s);
hipError_t launch_rk4_burgers_direct(const double* y0, double* yT, double* ckpt,
                                     int n, int64_t n_t, int64_t c, double dt,
                                     double nu, double L, int block, int fp32,
                                     hipStream_t s, const BurgersRange* rg = nullptr);
// The adjoint slices of the hybrid scheme (section 3.3, eq. hybadjinhom with
// the step sources of target tgt and weight gw): workgroup b runs slice
// s = s_first + b, steps [bounds[s], bounds[s+1]) backwards from zero,
// recomputing the states from the checkpoints (its own segment scratch
// seg + s c n), and writes the slice's end state to mu + s n.
hipError_t launch_burgers_adj_slices(const double* ckpt, const double* tgt, double gw,
                                     double* seg, double* mu, const int64_t* bounds,
                                     int s_first, int count, int n, int64_t n_t, int64_t c,
                                     double dt, double nu, double L, int block, hipStream_t s);

// Burgers reverse sweep, serial, over segments between checkpoints: each
// segment's step states are recomputed into `seg` (c x n) first.
hipError_t launch_rk4_burgers_reverse(const double* ckpt, const double* lamT,
                                      double* lam0, double* seg, int n,
                                      int64_t n_t, int64_t c, double dt,
                                      double nu, double L, int block, int fp32,
                                      hipStream_t s, const BurgersRange* rg = nullptr);

// Effective states of the two commutator-free Magnus factors of each macro
// step of S steps (W[2q], W[2q+1], q < n_t / S), recomputed from the
// checkpoints (every c steps) in parallel over macro steps.
// Macro steps qbase .. qbase+count-1 (count < 0: all from qbase) into
// slots 0 .. count-1 of W (two vectors per slot).
hipError_t launch_burgers_nodes(const double* ckpt, double* W, int n, int64_t n_t,
                                int64_t c, int64_t S, double dt, double nu, double L,
                                int block, int fp32, hipStream_t s, int qbase = 0,
                                int count = -1);
// A posteriori error of the commutator-free Magnus steps: per instance, for
// nsamp sampled macro steps, y[2k] = one step and y[2k+1] = two half steps
// of the same vector; est = 16/15 |y[2k] - y[2k+1]| / |y[2k+1]| (the
// fourth-order Richardson estimate of the one-step error, relative), the
// largest over the samples raises max_est and, above tol, ST_NOCONV.
struct MagnusCheck {
    const double* y;
    int n, nsamp;
    double tol;
    double scale;  // 16/15 (Richardson, fourth order); 1: a plain relative change
    DevStatus* st;
    InstStat* irep;
};
hipError_t launch_magnus_check(const MagnusCheck* tab, int count, hipStream_t s);

// ---- ragged Burgers batches ----------------------------------------------------
// One descriptor per instance (device table in the workspace, written by
// launch_upload).  Every instance uses 256 threads with pt = n / 256.
struct BurgersDesc {
    int n, pt, q0, pt_rev;   // q0: prefix count of macro steps (nodes grid);
                             // pt_rev: points per thread of the 512-thread
                             // reverse sweep (0: not available)
    int qbase, pad;          // nodes: first macro step (its slot is 0)
    int64_t n_t, c, S;
    double dt, inv2h, nuh2;
    const double* y0;
    double* yT;
    double* ckpt;
    double* seg;
    double* nodes;
    const double* lamT;
    double* lam0;
};
// which: 0 direct march with checkpoints, 1 serial reverse sweep,
// 2 Magnus node recompute (grid = total macro steps), 3 serial reverse sweep
// at 512 threads (every descriptor's pt_rev set)
hipError_t launch_burgers_batch(int which, const BurgersDesc* tab, int count,
                                int total_blocks, int fp32, hipStream_t s);
// Copy `bytes` (<= 3072) host bytes, passed by value as kernel arguments, to
// dst (device): graph-capturable table upload.
hipError_t launch_upload(void* dst, const void* src, size_t bytes, hipStream_t s);

// ---- Krylov exponential pieces (1D tridiagonal operator) -------------------
// KM_LTV: chain of 2*npieces exponentials exp(tau J(W_e)^T) with the Burgers
// Jacobian transpose at the effective states W_e = wop + e*n, in order.
enum KrylovMode { KM_CLASSIC = 0, KM_CHAIN = 1, KM_SINGLE = 2, KM_LTV = 3 };

struct KrylovArgs {
    int mode;            // KrylovMode
    int si;              // 0 polynomial, 1 shift-and-invert
    int n, m;
    int npieces;         // classic: P-1 pieces; chain: P slices; single: 1
    const double* vin;   // classic/chain: slice end states [P][n]; single: [n]
    double* yout;        // classic: [P-1][n]; chain/single: [n]
    double* iout;        // single: integral output [n]; classic (1D):
                         // [npieces][n], piece p integrating over its own
                         // [0, tau_p] with phase ia * tau_p (nullable)
    double tau;          // single: time; chain: slice length; classic: slice
                         // length dT (piece p uses tau_p = (npieces - p) * dT)
    double ia, ib;       // integral weight sin(ia + ib * sigma)
    double tol;          // relative tolerance
    double gamma_frac;   // shift-and-invert shift = gamma_frac * time
    Tri op;
    int fp32;            // operator stencil in FP32 (polynomial flavour)
    int pt;              // batched launches: points per thread
    const double* wop;   // KM_LTV: effective states [2*npieces][n]
    double inv2h, nuh2;  // KM_LTV: 1/(2h), nu/h^2
    // KM_LTV: vectors added to the chain (nullable): after macro step
    // addq[k] (increasing), vadd + (nadd - 1 - k) n
    const double* vadd;
    const int* addq;
    int nadd;
    // KM_LTV: the operator J(W) itself instead of J(W)^T (the nonlinear
    // direct iteration), and (nullable) the chain's vector after its k-th
    // addition into vsnap + k n
    int ltv_fwd;
    double* vsnap;
    // KM_LTV: one factor exp(tau J(W_k)) per macro step k (wop [npieces][n],
    // additions after macro step addq[k]) instead of two half-step factors
    int ltv_one;
    // nullable: the launch returns at once when *skip is set
    const int* skip;
    double* basis;       // [gridDim][m+1][n] workspace
    Sten5 op5;           // 2D: five-point operator
    int nx, ny;          // 2D: grid
    int blk0;            // batched launches: first workgroup of the entry
    // Taylor flavour: exp(tau Op) v by the truncated Taylor series in
    // substeps of at most theta / anorm time units, terms until two
    // consecutive term norms are below tol |v| (at most tdeg terms); anorm
    // is a bound of |Op| (0: computed in the kernel for the Burgers
    // Jacobian)
    int taylor, tdeg;
    double anorm, theta;
    // Chebyshev flavour (time-varying Burgers chains without a time
    // integral): exp(tau Op) v by the Chebyshev series on the Gershgorin
    // interval of the real parts, computed in the kernel
    int cheb;
    DevStatus* status;
    int adj;             // counters of the adjoint class (absorbed pieces;
                         // KM_SINGLE and KM_LTV count there anyway)
    InstStat* irep;      // this instance's statistics (nullable)
};
hipError_t launch_krylov1d(const KrylovArgs& a, int block, hipStream_t s);
// Batched time-varying chains: workgroup i runs tab[i] (KM_LTV, polynomial),
// `block` threads each (every entry's shape has that workgroup size);
// lds = the largest krylov1d_lds_bytes of the batch.
hipError_t launch_krylov_ltv_batch(const KrylovArgs* tab, int block, int count,
                                   size_t lds, hipStream_t s);
// The Chebyshev flavour's own chain kernel: the grids it covers in whole
// chunks (B threads of pt points, B pt = n), and a ragged batch of such
// chains (all entries of workgroup size block and a.pt == pt).
bool cheb_chain_shape_pub(int n, int* B, int* pt);
hipError_t launch_cheb_chain_batch(const KrylovArgs* tab, int block, int pt, int count,
                                   hipStream_t s);
size_t krylov1d_lds_bytes(int n, int m, int block, int si);
bool krylov_shape_pub(int n, int block_hint, int* B, int* pt);

// ---- 2D five-point operators (row-major, x fastest, periodic) -------------

// One entry of a batched 2D RK4 march: `items` independent marches of one
// instance (the slices, or the single serial march), each of nsteps steps of
//   y' = A y + sin(omega t) F,
// item q starting at global step step0 + q * item_steps, item 0 from y0
// (null: zero) and the others from zero.
// Workgroups blk0 .. blk0 + items * ny / 16 - 1 of the launch belong to the
// entry.  Serial sweeps: launch number L of the sweep advances the state in
// buf[L & 1] (y0 when L == 0) by min(4, n_t - 4L) steps into buf[(L+1) & 1];
// reverse sweeps run the exact discrete adjoint backwards the same way,
// adding sum s(t_stage) kbar_stage to Lam.
struct Band2D {
    const double* y0;
    const double* F;
    double* out;
    double* buf[2];
    double* Lam;
    // integral cost J = 1/T int |q - tgt|^2 dt (trapezoidal over the step
    // states): the source marches write g_n = dJ/dq_n = gw c_n (q_n - tgt),
    // c_n = 1/2 at both ends, 1 inside, into g ([n_t + 1][n]) and one cost
    // partial per (item, band) into cpart; the reverse source marches add
    // g_n after each step.  Forward items p >= 1 start from ys + (p-1) n.
    double* g;
    const double* tgt;
    const double* ys;
    double* cpart;
    double gw;
    int64_t step0, item_steps, n_t;
    double dt, omega;
    Sten5 A;
    int nx, ny, nsteps, items, blk0;
    int rows;  // output rows per workgroup: 16 or 32 (a divisor of ny)
};
constexpr int BAND_ROWS = 16;  // smallest band: ny must be a multiple
constexpr int BAND_MAX_STEPS = 4;
// Forward: slices (serial == 0) or launch L of a serial sweep.  Every
// entry of one launch has row length nx (64, 128 or 256).
hipError_t launch_band2d(const Band2D* tab, int count, int total_blocks, int nx,
                         int serial, int L, hipStream_t s);
// Reverse launch L of the serial discrete-adjoint sweep (A holds A^T).
hipError_t launch_band2d_rev(const Band2D* tab, int count, int total_blocks, int nx,
                             int L, hipStream_t s);
// Integral-cost marches.  Forward: the step sources g_n and the cost
// partials of every step of the slices (serial == 0: item p from y0 (p = 0)
// or ys, the corrected slice-start states) or of launch L of the serial
// march (which also advances buf as launch_band2d does).  Reverse: the
// discrete adjoint with the sources added after each step, from zero (the
// last item: from y0 + g_{n_t}) over each slice, writing the slice's end
// state to out + p n and its share of Lambda to Lam + p n (serial == 0), or
// launch L of the serial sweep (Lambda accumulated).
hipError_t launch_band2d_src(const Band2D* tab, int count, int total_blocks, int nx,
                             int serial, int L, hipStream_t s);
hipError_t launch_band2d_rsrc(const Band2D* tab, int count, int total_blocks, int nx,
                              int serial, int L, hipStream_t s);
// out = Op x for a five-point operator
hipError_t launch_apply5(const double* x, double* out, int nx, int ny, Sten5 op,
                         hipStream_t s);

// 2D Krylov pieces, vectors streamed from global memory, one workgroup per
// piece: KM_CLASSIC (npieces workgroups), KM_CHAIN or KM_SINGLE (one).
// Entries of `tab` own workgroups blk0 .. (next entry's blk0) - 1.
// si: every entry is a shift-and-invert entry (the Fourier solve; the grid
// passes fft2_grid), else none is.
hipError_t launch_krylov2d(const KrylovArgs* tab, int count, int total_blocks,
                           size_t lds, int si, hipStream_t s);
size_t krylov2d_lds_bytes(int m, int si);
bool fft2_grid(int nx, int ny);
constexpr int KRYLOV2D_BLOCK = 1024;

// ---- 2D exponential actions by uniformisation -------------------------------
// exp(tau A) x = sum_k p_k N^k x with N = I + A / mu (mu >= -A.c, off-diagonal
// coefficients >= 0, so N is nonnegative with unit row and column sums) and
// p_k the Poisson weights of lam = mu tau.  One entry of a pass launch covers
// `nvec` vectors (stride s_* doubles apart) of one row length; workgroups
// blk0 .. blk0 + nvec * ny / rows - 1 of the launch belong to it.  A pass
// covers terms k0 .. k1-1 (at most POIS_PASS_TERMS): the first pass starts
// the sums from zero, later ones read them from acc / acc2; a non-final pass
// writes N^{k1} x to tout and the sums back in place, the final one writes
// out = sum + partner and out2 = sum2 + out2_add.
constexpr int POIS_PASS_TERMS = 16;
struct PoisEntry {
    const double* x;         // input vectors (vector v at x + v sx)
    double* tb[2];           // term vectors N^k x between passes (+ v n)
    const double* partner;   // added to the final first sum (nullable)
    double* acc;             // first sum between passes
    double* out;             // final first sum (nullable: not wanted)
    const double* wtab;      // weights of the first sum (null: Poisson of lam)
    double* acc2;            // second sum between passes (two-sum launches)
    double* out2;            // final second sum
    const double* out2_add;  // added to the final second sum (nullable)
    const double* out2_add2; // a second vector added to it (nullable)
    int64_t s_add;           // vector stride of both added vectors
    const double* wtab2;     // weights of the second sum
    // phase form of the second sum's weights (nullable): vector v of the
    // entry weighs term k by sin(ph_v) wtab2[k] + cos(ph_v) wtab2i[k],
    // ph_v = ph0 + v dph (integrals of pieces that start at different times)
    const double* wtab2i;
    double ph0, dph;
    int64_t sx, s_partner, s_acc, s_out;
    double lam;              // Poisson parameter mu * tau
    double est;              // a priori truncation bound (reported)
    Sten5 N;                 // I + A / mu
    int D, nvec;             // terms; vectors of the entry
    int nx, ny, rows, blk0;  // rows: output rows per band (16 or 32)
    DevStatus* status;
    InstStat* irep;          // the instance's statistics (nullable)
};
// Pass `pass` (terms 16 pass .. 16 pass + 15) of the first `count` entries
// of a table (the entries still running: a table lists its entries by
// falling term count, blk0 their prefix sums).
hipError_t launch_pois2d(const PoisEntry* tab, int count, int total_blocks, int nx, int two,
                         int pass, hipStream_t s);
// Weight table of the time integral int_0^h sin(phi - omega s) exp(s A) x ds
// of one uniformised exponential: w[k], k < D, so that the integral is
// sum_k w_k N^k x (lam = mu h); wi is scratch of D doubles.  split != 0:
// the phase is left open, w and wi receive the two tables whose combination
// sin(phi) w + cos(phi) wi gives the weights for any phi.
struct PoisWeights {
    double* w;
    double* wi;
    int D, split;
    double lam, mu, omega, phi, scale;
};
hipError_t launch_pois_weights(const PoisWeights* tab, int count, hipStream_t s);

// ---- small kernels ---------------------------------------------------------
// out[i] = base[i] (or 0) + sum_k a[k] basis[k*n + i]
hipError_t launch_combine_basis(const double* a, const double* basis,
                                const double* base, double* out, int K, int n,
                                hipStream_t s);
// out = Op x (tridiagonal, periodic)
hipError_t launch_apply_tri(const double* x, double* out, int n, Tri op,
                            hipStream_t s);
// lamT = qT - tgt;  J = 1/2 |lamT|^2 + beta |a|^2 (one workgroup); a
// non-finite J sets ST_NONFINITE in st (nullable)
hipError_t launch_cost(const double* qT, const double* tgt, const double* a,
                       int n, int K, double beta, double* lamT, double* J,
                       hipStream_t s, DevStatus* st = nullptr);
// grad[k] = <basis_k, v> + 2 beta a[k] (one workgroup per k); a non-finite
// component sets ST_NONFINITE in st (nullable)
hipError_t launch_grad(const double* basis, const double* v, const double* a,
                       int K, int n, double beta, double* grad, hipStream_t s,
                       DevStatus* st = nullptr);
// Batched cost and gradient reductions over every instance of a call, in
// two deterministic phases: blocks of RED_CHUNK points write partial sums,
// then one block per instance adds them in chunk order.
//   cost: lamT = qT - tgt, J = 1/2 |lamT|^2 + beta |a|^2
//   grad: grad_k = <basis_k, v> + 2 beta a_k
// Non-finite J or gradient components set ST_NONFINITE in st (nullable).
constexpr int RED_CHUNK = 8192;
struct RedDesc {
    const double* qT;
    const double* tgt;
    double* lamT;
    const double* a;
    double* J;
    const double* basis;
    const double* v;
    double* grad;
    double beta;
    DevStatus* st;
    // integral cost (nullable): J = sum of ipart[0..ichunks) + beta |a|^2,
    // the partials written by the source march; the instance then has no
    // terminal-cost blocks
    const double* ipart;
    int n, K, chunks, blk0_cost, blk0_grad, ichunks;
    int64_t part0, gpart0;  // this instance's partials in the cost / gradient areas
};
hipError_t launch_cost_batch(const RedDesc* tab, int count, int blocks_cost, double* part,
                             hipStream_t s);
hipError_t launch_grad_batch(const RedDesc* tab, int count, int blocks_grad, double* part,
                             hipStream_t s);
// out = q0 (or 0) + vlast + sum_{p<np} Y[p]   (checks finiteness)
hipError_t launch_recombine(const double* q0, const double* vlast,
                            const double* Y, int np, int n, double* out,
                            DevStatus* st, hipStream_t s);
// p[0..n) = 0 (a kernel, so it may be captured in a graph)
hipError_t launch_zero(double* p, size_t n, hipStream_t s);
// Threads per workgroup and points per thread of the register-resident
// 1D marches (false if n has no supported shape).
bool march_shape(int n, int block_hint, int* block, int* pt);
// out = (a or 0) + b
hipError_t launch_add(const double* a, const double* b, double* out, int n,
                      hipStream_t s);

}  // namespace pxp
