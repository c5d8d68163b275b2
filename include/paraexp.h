/*
 * paraexp.h -- C ABI of the MI355X Paraexp direct-adjoint gradient library.
 *
 * The library computes one gradient of a PDE-constrained cost per instance,
 * following the direct-adjoint loop of Skene, Eggl & Schmid, "A
 * parallel-in-time approach for accelerating direct-adjoint studies"
 * (section 2) with the Paraexp time decomposition of section 3:
 *
 *  - the direct equation is split over P equal time slices; the P
 *    inhomogeneous sub-problems start from zero data and run as one batch
 *    (section 3.1, eq. linInhomEqus) with fixed-step classical RK4;
 *  - their end states are propagated to the final time by the action of
 *    the matrix exponential (eq. hom), computed with Arnoldi/Krylov
 *    projection and a small dense exponential of the Hessenberg matrix
 *    (section 4.1), either polynomial Krylov or shift-and-invert Krylov;
 *  - the solution is the superposition of all pieces (eq. fullsol0);
 *  - the adjoint (eq. adjEquation) starts from q^dagger(T) = dJ/dq(T)
 *    (eq. adjFinalTime) and, being linear, is propagated the same way
 *    (eq. adjHomNormal, adjhomfinal), with its time integral against the
 *    forcing modulation evaluated inside the Krylov space;
 *  - the gradient follows eq. paramupdate (forcing amplitudes) or
 *    eq. initupdate (initial-condition amplitudes).
 *
 * Conventions
 *  - Every array argument is a DEVICE pointer (HIP global memory) unless
 *    stated otherwise; `pb` and scalars are host memory read during the
 *    call only.  The caller owns every buffer.
 *  - A batch of `batch` instances is described by `pb[0..batch-1]`.  Arrays
 *    of grid size are packed instance after instance: instance i occupies
 *    elements [off_i, off_i + nx_i*ny_i) with off_i the prefix sum of the
 *    sizes; control-sized arrays are packed the same way with K_i.  2D grids
 *    are row-major with x fastest.
 *  - The calls never allocate device memory and never synchronise the
 *    stream: work is enqueued on `stream` (a hipStream_t; NULL = default
 *    stream) and uses only the caller's workspace `ws` of `ws_bytes`
 *    bytes (query with pxp_workspace_size).  Calls that share a workspace
 *    must not overlap.
 *  - Argument errors are detected on the host before anything is enqueued
 *    and nothing is written in that case.  Conditions found on the device
 *    (Krylov non-convergence, non-finite values) are recorded in the
 *    workspace and read back with pxp_device_status after the stream has
 *    been synchronised.
 *  - Double precision is used at the boundary in all modes.
 */
#ifndef PARAEXP_H
#define PARAEXP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PXP_OK = 0,
    PXP_EINVAL = 1,          /* malformed argument (sizes, nulls, steps)      */
    PXP_EUNSUPPORTED = 2,    /* valid but not implemented for this operator   */
    PXP_EWORKSPACE = 3,      /* workspace missing or too small                */
    PXP_EUNSTABLE_DT = 4,    /* dt outside the RK4 stability region bound     */
    PXP_EKRYLOV_NOCONV = 5,  /* device: Krylov estimate above tolerance       */
    PXP_ENONFINITE = 6,      /* device: NaN/Inf met                           */
    PXP_EHIP = 7             /* a HIP runtime call failed                     */
} pxp_status;

/* Operators (paper section 4.2 and 4.3; periodic grids, spacing L/n). */
enum {
    PXP_OP_ADVDIFF1D = 0,        /* -c u_x + nu u_xx, central differences     */
    PXP_OP_ADVDIFF2D_UPWIND = 1, /* -vx u_x - vy u_y + nu lap u, upwind adv.  */
    PXP_OP_BURGERS1D = 2         /* -u u_x + nu u_xx, central differences     */
};
enum { PXP_FP64 = 0, PXP_FP32_BULK = 1 };
/* Controls: forcing amplitudes a_k of f(x,t) = sin(omega t) sum_k a_k G_k(x)
 * (eq. paramupdate), or initial-condition amplitudes q0 = sum_k a_k phi_k
 * (eq. initupdate). */
enum { PXP_CTRL_FORCING = 0, PXP_CTRL_IC = 1 };
/* Krylov flavour for the homogeneous exponentials. */
/* POLY: Arnoldi on A; time substeps accepted by the a-posteriori estimate
 * beta h_{k+1,k} |e_k^T exp(ts H_k) e_1| <= krylov_tol beta ts/tau, with an
 * early exit every 4 dimensions from 8 on. */
/* SHIFT_INVERT: Arnoldi on (I - gamma A)^{-1}, gamma = si_gamma times the
 * exponential's time, one step over the whole time.  The solve: periodic
 * tridiagonal (1D, the Burgers Jacobian with variable coefficients), or, in
 * 2D (named only; power-of-two grids of at most 256 x 256, terminal cost),
 * the constant-coefficient five-point operator divided out mode by mode in
 * the 2D Fourier basis.  From about m/2 the
 * approximation is compared with the previous check's; the error is
 * extrapolated from the contraction of those differences and the space stops
 * once it is below krylov_tol (relative to |v|).  Both Arnoldi flavours use
 * classical Gram-Schmidt with a second pass only on tenfold cancellation. */
/* AUTO: 1D linear: shift-and-invert when tau * rho > 64 (rho = 4 nu/h^2 +
 * |vx|/h, tau the horizon) and the grid has the cyclic-reduction shape,
 * else TAYLOR.  Burgers: CHEBYSHEV where its chain kernel covers the grid
 * (see CHEBYSHEV); elsewhere shift-and-invert when half a slice times rho
 * exceeds 64, else TAYLOR.
 * 2D: UNIFORM, except for the CLASSIC schedule of the direct pieces, which
 * takes TAYLOR. */
/* TAYLOR: no Arnoldi process; exp(tau Op) v by the truncated Taylor series
 * in substeps of at most theta/|Op| (theta from the remainder bound for 40
 * terms at krylov_tol), terms added until two consecutive term norms fall
 * below krylov_tol |v|; the time integral is accumulated term by term.  Its
 * traffic is a few vectors per term and it needs no inner products. */
/* UNIFORM (2D only): no Arnoldi process; exp(tau A) x by uniformisation,
 * sum_k p_k N^k x with N = I + A/mu, mu = -A_ii the diagonal magnitude of
 * the five-point operator (N is nonnegative with unit row and column sums
 * for nonnegative velocities) and p_k the Poisson weights of mu tau.  The
 * number of terms D is fixed before the launch as the smallest with Poisson
 * tail P(X >= D) <= krylov_tol / 100, a bound of the truncation error in the
 * max norm; it is the value reported as the estimate.  Each exponential is
 * split over bands of grid rows, every band recomputing up to 16 halo rows
 * per pass of 16 terms, so one exponential spreads over many workgroups.
 * The adjoint's time integral uses the exact integral of every term's
 * weight against the forcing modulation. */
/* CHEBYSHEV (Burgers only, on grids its chain kernel covers in whole chunks:
 * n a multiple of 64 up to 256, or 256 threads of 1, 2, 4 or 8 points, or
 * 512 threads of 1, 2, 4, 8 or 16 points; PXP_EUNSUPPORTED elsewhere): no
 * Arnoldi process; each exponential of the
 * time-varying chains, exp(tau J) v, by the Chebyshev series of exp on the
 * real interval of the Gershgorin bounds of tau J's real parts (the focal
 * interval of section 4.1's ReLPM; Chebyshev basis, coefficients the scaled
 * modified Bessel functions of the half-width), taken in substeps where
 * the half-width exceeds what the kernel's coefficient table holds.  Terms
 * are added up to the a priori degree of the coefficients' decay and then
 * until two consecutive term norms are below krylov_tol |v|, which is the
 * reported estimate.  About a fifth of the Taylor flavour's stencil
 * applications for the diffusion-dominated Burgers Jacobian. */
enum { PXP_KRYLOV_POLY = 0, PXP_KRYLOV_SHIFT_INVERT = 1, PXP_KRYLOV_AUTO = 2,
       PXP_KRYLOV_TAYLOR = 3, PXP_KRYLOV_UNIFORM = 4, PXP_KRYLOV_CHEBYSHEV = 5 };
/* Schedule of the direct homogeneous pieces: CLASSIC = P-1 independent
 * pieces exp((T - T_{p+1}) A) v_p (eq. hom); CHAIN = nested sum
 * w <- exp(dT A) w + v_p, one piece after the other; TREE (2D, UNIFORM) =
 * the same sum combined pairwise: adjacent partial sums over slice ranges
 * [a, b) and [b, c) give exp((T_c - T_b) A) w_ab + w_bc, all pairs of one
 * level independent, log2(P) levels. */
enum { PXP_SCHED_CLASSIC = 0, PXP_SCHED_CHAIN = 1, PXP_SCHED_TREE = 2 };
/* Problem flags.  ABSORBED_ADJOINT (1D linear problems): the Paraexp
 * adjoint runs in the absorbed form of section 3.3 (eq. hybadjinhom with the
 * final condition absorbed): lambda = lambda_T + q~, q~(T) = 0, with the P
 * inhomogeneous adjoint slices q~' = A^T q~ + A^T lambda_T from zero (in
 * reversed time) as one batch and the P-1 homogeneous pieces of their end
 * states by Krylov, each with its share of Lambda.  Default (0): the
 * unabsorbed form, one homogeneous piece from lambda_T (eq. adjhomfinal). */
enum { PXP_FLAG_ABSORBED_ADJOINT = 1, PXP_FLAG_INTEGRAL_COST = 2, PXP_FLAG_NL_PARAEXP = 4 };
/* NL_PARAEXP (Burgers, FP64, terminal cost): the Paraexp direct solves the
 * nonlinear equation by the iteration of section 3.2 (eqs. nlIter,
 * nonlinTrans, Jacobians, nlHomIter, fullsolIter) instead of the serial
 * march: with A = nu lap and N(y) = -y Dy, iterate i+1 on each of the P
 * slices is the linear problem y' = (A + J_p) y + N(O) - J_p O, J_p the
 * Jacobian of N at the time average of iterate i over the slice (the
 * trapezoidal rule on the step grid; J is linear in the state, so this is
 * the slice-averaged Jacobian), O the previous iterate's RK4 stage states;
 * the slices from zero as one batch, the chain of one exponential
 * exp((T_{p+1} - T_p)(A + J_p)) per slice (the krylov flavour as for the
 * adjoint's factors) with each slice's end state added for the corrected
 * slice starts, and every slice again from its corrected start for the new
 * stage states.  The first iterate is q0 at all times; after every
 * iteration the relative change of q(T), and once it is within nl_tol the
 * remaining launches of the call return at once (at most nl_iters
 * iterations; no host synchronisation); the last
 * iteration's relative change of q(T) is reported as the estimate and
 * raises PXP_EKRYLOV_NOCONV above nl_tol.  The checkpoints for the adjoint
 * come from the last iterate.  The workspace then holds 8 n_steps n stage
 * states. */
/* INTEGRAL_COST (2D problems with UNIFORM or AUTO exponentials and the TREE
 * schedule; Burgers problems in FP64):
 * pxp_gradient minimises the integral cost of section 4.2 (eq. cost),
 *   J = 1/T int_0^T |q(t) - u_tgt|^2 dt + beta |a|^2,
 * the time integral taken by the trapezoidal rule over the RK4 step states
 * (weights dt/T inside, dt/(2T) at both ends).  Every step state is then an
 * argument of J, so the adjoint is driven by the sources dJ/dq_n after each
 * step (eq. adjEquation) instead of a final condition.  The Paraexp path:
 * the slices as usual, the tree of their homogeneous pieces kept level by
 * level and walked back down for the corrected state at every slice start,
 * one more batched march of every slice from its corrected start that writes
 * the sources (the dense direct trajectory) and the cost, the adjoint slices
 * with those sources as one batch (the genuinely inhomogeneous adjoint of
 * eq. adjInhom), and the tree of their homogeneous pieces, each carrying its
 * exact share of Lambda.  The workspace then holds (n_steps + 1) n sources
 * per instance.  The largest adjoint piece, mu T_left with T_left the
 * horizon of the tree's left half, must stay within 4096 (PXP_EUNSUPPORTED
 * otherwise; mu = -diagonal of A).
 * Burgers (section 3.3, the hybrid serial-direct-parallel-adjoint scheme of
 * algorithm 3): the serial direct march writes the step sources; it runs as
 * one launch per adjoint slice, and every hyb_group slices the adjoint
 * slices of the march so far (the exact discrete adjoint of each slice from
 * zero with its sources, eq. hybadjinhom) start on the library's side stream
 * while the march goes on.  The slice bounds follow eq. nonEquiP with
 * k = hyb_k, rounded to multiples of lcm(n_steps/P, ckpt_every) steps; the
 * P Magnus steps of the time-varying adjoint chain then start from
 * dJ/dq(T) and add each slice's end state where it starts (eq.
 * fullAdjSolHyb as a nested sum).
 * The paraexp_direct and paraexp_adjoint calls on their own ignore the
 * flag, except that paraexp_adjoint accepts jI_src only for 2D problems
 * that carry it; pxp_cost refuses it. */
/* Method: PARAEXP = the time-parallel path; SERIAL = plain RK4 stepping of
 * the direct equation and its exact discrete adjoint (the comparison). */
enum { PXP_METHOD_PARAEXP = 0, PXP_METHOD_SERIAL = 1 };

typedef struct {
    int32_t op, prec, ctrl, krylov;  /* enums above                           */
    int32_t sched, nx, ny, P;        /* ny = 1 in 1D; P = number of slices     */
    int32_t m, K, ckpt_every, block; /* Krylov dimension, #controls, Burgers
                                        checkpoint interval (steps), threads
                                        per workgroup for the 1D marches
                                        (0 = library default)                 */
    int32_t kblock, flags;           /* threads per workgroup of the Krylov
                                        kernels (multiple of 64, <= 512;
                                        0 = library default); PXP_FLAG_*      */
    int64_t n_steps;                 /* RK4 steps; n_steps % P == 0            */
    double L, vx, vy, nu;            /* box [0,L)^d, velocity, viscosity       */
    double T, omega, beta;           /* horizon, s(t) = sin(omega t), weight   */
    double krylov_tol;               /* relative a-posteriori tolerance        */
    double si_gamma;                 /* shift-and-invert shift as a fraction of
                                        the exponential's time (0 = 0.2 in
                                        1D, 0.05 in 2D)                       */
    int32_t hyb_slices;              /* integral cost, Burgers: adjoint slices
                                        of the hybrid scheme (0 = P)          */
    int32_t hyb_group;               /* slices per adjoint launch (0 = 4)      */
    double hyb_k;                    /* their partition (eq. nonEquiP): adjoint
                                        over direct time per unit of time
                                        (0 = equal slices)                    */
    int32_t nl_iters;                /* NL_PARAEXP: most iterations (0 = 8)    */
    int32_t nl_slices;               /* NL_PARAEXP: slices of the iteration
                                        (0 = P; must divide n_steps); the
                                        adjoint's Magnus steps stay P        */
    double nl_tol;                   /* NL_PARAEXP: relative change of q(T)
                                        that ends the iteration
                                        (0 = krylov_tol)                      */
} pxp_problem;

/* Bytes of device workspace the calls below need for this batch.
 * Returns PXP_EINVAL/PXP_EUNSUPPORTED for problems the calls would reject. */
pxp_status pxp_workspace_size(const pxp_problem* pb, int32_t batch,
                              size_t* bytes);

/* Zero a fresh workspace (status block, per-instance statistics and the
 * rest; enqueued on `stream` as a kernel).  Call once after allocating `ws`, outside any
 * stream capture: on its first call on a device it also creates the
 * library's side stream there (default priority, non-blocking) and two
 * events, which the compute calls use to run independent launch groups of
 * one phase concurrently (fork and join by events on the caller's stream).
 * Without it the groups run one after the other on the caller's stream. */
pxp_status pxp_workspace_init(void* ws, size_t ws_bytes, void* stream);

/* Direct solve (section 3.1, eqs. linInhomEqus, hom, fullsol0):
 *   q0  [sum n]  initial state (device)
 *   F   [sum n]  forcing pattern f(x), modulated by sin(omega t) (nullable:
 *                no forcing)
 *   qT  [sum n]  output q(T)
 * For PXP_OP_BURGERS1D the direct march is serial (section 3.3) and writes
 * the checkpoints every ckpt_every steps into the workspace for the
 * adjoint. */
pxp_status paraexp_direct(const pxp_problem* pb, int32_t batch,
                          const double* q0, const double* F, double* qT,
                          void* ws, size_t ws_bytes, void* stream);

/* Adjoint solve (eqs. adjEquation, adjFinalTime, adjHomNormal,
 * adjhomfinal) from the final condition lamT (= dJ/dq(T)).  lamT, lam0
 * and Lambda must be 16-byte aligned at every instance offset (PXP_EINVAL
 * otherwise):
 *   jI_src  [sum (n_steps+1) n]  sources of an integral cost term J_I =
 *           int_0^T j(q, t) dt (section 2, eq. adjEquation), nullable: row n
 *           of instance i (at sum_{j<i} (n_steps_j + 1) n_j + n n_i) holds
 *           dJ_I/dq_n of the discrete cost, added to the adjoint after the
 *           reverse step that produces lambda_n (row n_steps: added to lamT).
 *           Non-null requires every instance to be 2D with
 *           PXP_FLAG_INTEGRAL_COST (PXP_EUNSUPPORTED otherwise, before
 *           anything is enqueued); lamT may then be NULL (no terminal
 *           cost).  16-byte aligned rows.
 *   lam0    [sum n]  output q^dagger(0) (nullable)
 *   Lambda  [sum n]  output int_0^T sin(omega t) q^dagger(t) dt (nullable)
 * Burgers instances read the checkpoints that the preceding paraexp_direct
 * call left in the same workspace (the workspace holds them, not a caller
 * array: a second direct call on that workspace replaces them).  Their
 * time-varying adjoint is propagated by fourth-order commutator-free Magnus
 * steps, one per slice; where a slice has an even number of RK4 steps the
 * call also estimates the steps' own error a posteriori: on the first and
 * the last slice (in reversed time) one step and two half steps of lamT,
 * 16/15 |difference| / |two half steps| (the Richardson estimate of a
 * fourth-order step, in FP64 whatever prec says).  It enters the device
 * status like the Krylov estimates: the largest estimate, and
 * PXP_EKRYLOV_NOCONV above krylov_tol. */
pxp_status paraexp_adjoint(const pxp_problem* pb, int32_t batch,
                           const double* lamT, const double* jI_src, double* lam0,
                           double* Lambda, void* ws, size_t ws_bytes, void* stream);

/* Full direct-adjoint loop (section 2): control -> J and dJ/da.
 *   ctrl   [sum K]      control amplitudes a
 *   basis  [sum K*n]    G_k (forcing) or phi_k (initial condition), row k of
 *                       instance i at koff_i*n_i + k*n_i
 *   q0     [sum n]      base initial state (nullable = zero)
 *   u_tgt  [sum n]      target state of J = 1/2 |q(T) - u_tgt|^2 + beta |a|^2
 *                       (PXP_FLAG_INTEGRAL_COST: of the integral cost)
 *   J      [batch]      output cost
 *   grad   [sum K]      output dJ/da
 *   qT     [sum n]      output q(T) (nullable)
 *   lam_out [sum n]     output Lambda (forcing) or lambda_0 (IC) (nullable)
 * method selects PXP_METHOD_PARAEXP or PXP_METHOD_SERIAL. */
pxp_status pxp_gradient(const pxp_problem* pb, int32_t batch, int32_t method,
                        const double* ctrl, const double* basis,
                        const double* q0, const double* u_tgt, double* J,
                        double* grad, double* qT, double* lam_out, void* ws,
                        size_t ws_bytes, void* stream);

/* Same as pxp_gradient with method = PXP_METHOD_PARAEXP, without the
 * lam_out output: the one-call form of the time-parallel gradient. */
pxp_status gradient(const pxp_problem* pb, int32_t batch, const double* ctrl,
                    const double* basis, const double* q0,
                    const double* u_tgt, double* J, double* grad, double* qT,
                    void* ws, size_t ws_bytes, void* stream);

/* The three short steps of the loop on their own, for callers that drive
 * the direct and adjoint solves separately (e.g. an autograd wrapper):
 *   pxp_assemble         out = base + sum_k ctrl_k basis_k per instance
 *                        (forcing pattern or initial state; base nullable)
 *   pxp_cost             J_i = 1/2 |qT - u_tgt|^2 + beta |ctrl|^2 and
 *                        lamT = qT - u_tgt (eq. adjFinalTime; lamT nullable);
 *                        terminal cost only (PXP_EUNSUPPORTED for
 *                        PXP_FLAG_INTEGRAL_COST problems)
 *   pxp_reduce_gradient  grad_k = <basis_k, v> + 2 beta ctrl_k with v the
 *                        adjoint integral Lambda (forcing, eq. paramupdate)
 *                        or lambda_0 (initial condition, eq. initupdate)
 * Device arrays packed as for pxp_gradient; enqueued on `stream`. */
pxp_status pxp_assemble(const pxp_problem* pb, int32_t batch, const double* ctrl,
                        const double* basis, const double* base, double* out,
                        void* stream);
pxp_status pxp_cost(const pxp_problem* pb, int32_t batch, const double* qT,
                    const double* u_tgt, const double* ctrl, double* J,
                    double* lamT, void* stream);
pxp_status pxp_reduce_gradient(const pxp_problem* pb, int32_t batch,
                               const double* basis, const double* v,
                               const double* ctrl, double* grad, void* stream);

/* Synchronises `stream` and returns the device-side status recorded in the
 * workspace (its first 64 bytes) by the last calls (PXP_OK, PXP_EKRYLOV_NOCONV, PXP_ENONFINITE);
 * `max_est` (host, nullable) receives the largest relative Krylov error
 * estimate seen.  Clears the recorded status. */
pxp_status pxp_device_status(void* ws, size_t ws_bytes, void* stream,
                             double* max_est);

/* Synchronises `stream` and reads the accumulated Krylov counters of the
 * workspace: accepted substeps, Arnoldi iterations, and Arnoldi iterations
 * that took a second Gram-Schmidt pass (classical Gram-Schmidt reruns only
 * when the first pass left less than a tenth of the vector's norm),
 * over all pieces since the workspace was initialised (host outputs,
 * nullable). */
pxp_status pxp_device_counters(void* ws, size_t ws_bytes, void* stream,
                               uint64_t* substeps, uint64_t* krylov_iters,
                               uint64_t* reorth_passes);

/* The same counters for one class of exponentials: cls = 0 the direct
 * pieces (eq. hom, and the nonlinear iteration's chain), cls = 1 the
 * adjoint pieces (eqs. adjHomNormal, adjhomfinal, the absorbed adjoint's
 * pieces and the time-varying Magnus chains).  For the Taylor and
 * Chebyshev flavours the iteration counter holds series terms.
 * The uniformised 2D exponentials fix their terms before the launch and do
 * not count.  PXP_EINVAL for another cls. */
pxp_status pxp_device_counters_class(void* ws, size_t ws_bytes, void* stream, int32_t cls,
                                     uint64_t* substeps, uint64_t* krylov_iters,
                                     uint64_t* reorth_passes);

/* Per-instance report of the exponentials since the workspace was
 * initialised or last reported on (host output `out`, one entry per
 * instance of the same batch and workspace as the compute calls).
 * Synchronises `stream`, then clears the statistics.  P and the schedule are
 * the problem's (sched -1: the direct march is serial, Burgers without
 * NL_PARAEXP, whose chain reports CHAIN); the flavours
 * are the ones that ran, AUTO resolved (-1: no exponential).  substeps counts
 * Krylov substeps (uniformised exponentials: one per exponential);
 * iterations counts Arnoldi steps or series terms; max_est is the largest
 * error estimate, relative to |v| (Krylov: a posteriori; uniformisation: the
 * a priori Poisson tail); nl_iterations counts the iterations of the
 * nonlinear Paraexp direct that ran (NL_PARAEXP; 0 otherwise). */
typedef struct {
    int32_t P, sched, krylov_direct, krylov_adjoint;
    uint64_t substeps, iterations;
    double max_est;
    int32_t nl_iterations, pad;
} pxp_report;
pxp_status pxp_last_report(const pxp_problem* pb, int32_t batch, void* ws, size_t ws_bytes,
                           void* stream, pxp_report* out);

/* Launch timing for benchmarks and profiling.  While enabled, every launch
 * of a kernel class is bracketed by two HIP events recorded on the launch
 * stream.  pxp_profile_read waits for the recorded events of one class and
 * returns their summed elapsed time (host outputs) and count, then forgets
 * them.  Process-wide host state: not thread-safe. */
enum {
    PXP_K_SLICES = 0,          /* batched inhomogeneous RK4 slices          */
    PXP_K_KRYLOV_DIRECT = 1,   /* direct homogeneous pieces (Arnoldi+expm)  */
    PXP_K_KRYLOV_ADJOINT = 2,  /* adjoint homogeneous piece and integral    */
    PXP_K_SERIAL_DIRECT = 3,   /* serial RK4 march                          */
    PXP_K_SERIAL_REVERSE = 4,  /* serial reverse (discrete adjoint) sweep   */
    PXP_K_LTV_ADJOINT = 5,     /* time-varying adjoint Magnus chain         */
    PXP_K_LTV_NODES = 6,       /* per-slice recompute of the Magnus states  */
    PXP_K_SOURCES = 7,         /* integral cost: march of every slice from its
                                  corrected start writing the step sources   */
    PXP_K_ADJ_SLICES = 8,      /* integral cost: adjoint slices with sources */
    PXP_K_LTV_CHECK = 9,       /* a posteriori error of the Magnus steps    */
    PXP_K_NL_ITER = 10         /* iterations of the nonlinear Paraexp direct */
};
pxp_status pxp_profile_enable(int32_t on);
pxp_status pxp_profile_read(int32_t kernel_class, double* total_ms,
                            int32_t* count);

/* Autotuner (host-driven: synchronises `stream`, not for graph capture).
 * Instances that share op, grid, precision and control kind form a group;
 * for each group the gradient of its longest instance is timed over
 * candidate settings and the fastest candidate whose gradient agrees with
 * the serial method's gradient (the exact discrete adjoint of the same RK4
 * march) to `rtol` (relative L2) is kept.  Candidates: first the problem
 * as given (so tuning never loses to the untuned settings), then slice
 * counts P among the divisors of n_steps in [p_min, p_max] (at most six,
 * spread geometrically; 0 = 8 and 256), polynomial, shift-and-invert or
 * Taylor, classic or chain schedule (linear problems), 256 or 512 Krylov
 * threads (1D).  Candidates slower than four times the best so far in their
 * warm-up run are not timed further; `reps` timed runs each (0 = 2).  When
 * the problem as given wins, every instance of the group keeps its own
 * settings.  Otherwise the other instances of the group take the tuned
 * krylov, sched and kblock, and the slice count whose slices last about as
 * long as the tuned ones; each is checked against its own serial gradient
 * and its slice count doubled (to the next divisor of n_steps) until it
 * passes, at most four times.  Arrays
 * are packed as for pxp_gradient; ws must hold pxp_tune_workspace_size bytes
 * (256-byte aligned); report (host, nullable) receives one entry per
 * instance (rel_err = -1 when no setting passed: the instance then keeps
 * its own settings). */
typedef struct {
    int32_t P, krylov, sched, kblock;
    int32_t candidates;  /* candidates tried for the group                */
    int32_t group;       /* index of the group's timed instance           */
    double ms;           /* Paraexp gradient time of that instance        */
    double serial_ms;    /* serial-method gradient time of that instance  */
    double rel_err;      /* its gradient vs the serial gradient           */
} pxp_tune_report;
pxp_status pxp_tune_workspace_size(const pxp_problem* pb, int32_t batch,
                                   int32_t p_min, int32_t p_max, size_t* bytes);
pxp_status pxp_autotune(pxp_problem* pb, int32_t batch, const double* ctrl,
                        const double* basis, const double* q0,
                        const double* u_tgt, int32_t p_min, int32_t p_max,
                        double rtol, int32_t reps, void* ws, size_t ws_bytes,
                        pxp_tune_report* report, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as pxp_gradient, with its workspace in a fixed device array of
 * the library (PXP_NOALLOC_SCRATCH_BYTES per GPU, held by each GPU the
 * library runs on until the process ends) instead of a caller buffer.  The
 * call allocates nothing.  Arguments as for pxp_gradient; problems whose
 * pxp_workspace_size exceeds PXP_NOALLOC_SCRATCH_BYTES are rejected with
 * PXP_EWORKSPACE before anything is enqueued.  The device status block is
 * cleared at the start of every call; status_out (device, nullable, at least
 * 64 bytes, 8-byte aligned) receives it at the end, to be read with
 * pxp_device_status(status_out, 64, stream, ...).  Every call on a GPU uses
 * that GPU's one array: calls that overlap on one GPU (two streams, two host
 * threads) race and give wrong results; serialise them. */
#define PXP_NOALLOC_SCRATCH_BYTES (64u << 20)
pxp_status pxp_gradient_noalloc(const pxp_problem* pb, int32_t batch,
                                int32_t method, const double* ctrl,
                                const double* basis, const double* q0,
                                const double* u_tgt, double* J, double* grad,
                                double* qT, double* lam_out, void* status_out,
                                void* stream);

/* Human-readable text for a status code (static storage). */
const char* pxp_status_str(pxp_status s);

/* Library version string (static storage). */
const char* pxp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PARAEXP_H */
