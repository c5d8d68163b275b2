/*
 * Oracle: plain serial FP64 reference for one direct-adjoint loop.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this code; the product path
 * never does.  It shares no source, header or helper with the HIP library.
 *
 * What it computes (paper section 2, equations state, adjEquation,
 * adjFinalTime, paramupdate, initupdate; section 4.2/4.3 for the operators):
 *
 *   direct   dq/dt = N(q) + s(t) F,  q(0) = q0,  s(t) = sin(omega t),
 *            marched by classical fourth-order Runge-Kutta with a fixed step
 *            dt = T / n_steps (the time integrator the paper's inhomogeneous
 *            solves use, section 4.2, here without step adaptation);
 *   cost     J = 1/2 ||q(T) - q_tgt||^2 + beta ||a||^2, with the unweighted
 *            discrete inner product [a, b] = a^H b (section 2); or the
 *            integral cost of section 4.2, J = 1/T int_0^T ||q - q_tgt||^2 dt
 *            + beta ||a||^2, with the time integral taken by the trapezoidal
 *            rule over the RK4 step states (orc_gradient_icost);
 *   adjoint  the exact discrete adjoint of the RK4 march (the adjoint of the
 *            discretised direct map, section 2: the adjoint operator of a
 *            discrete problem is its transpose), started from the final
 *            condition lambda_T = dJ/dq(T) = q(T) - q_tgt (eq. adjFinalTime);
 *            for the integral cost every step state q_n is a cost argument,
 *            so the reverse sweep adds dJ/dq_n after each step and starts
 *            from dJ/dq_{n_t} (the discrete form of the source -dJ_I/dq of
 *            eq. adjEquation);
 *   gradient forcing amplitudes:  dJ/da_k = <G_k, Lambda> + 2 beta a_k,
 *            Lambda = sum over steps/stages of s(t_stage) * kbar_stage, the
 *            discrete counterpart of int_0^T s(t) lambda(t) dt
 *            (eq. paramupdate, eq. update);
 *            initial-condition amplitudes: dJ/da_k = <phi_k, lambda_0>
 *            + 2 beta a_k (eq. initupdate).
 *
 * Operators (periodic grids, spacing h = L / n):
 *   OP 0  1D advection-diffusion, second-order central differences:
 *         (A u)_i = -c (u_{i+1} - u_{i-1}) / (2h) + nu (u_{i+1} - 2u_i + u_{i-1}) / h^2
 *   OP 1  2D advection-diffusion, first-order upwind advection for positive
 *         velocities and the five-point Laplacian (row-major, x fastest)
 *   OP 2  1D viscous Burgers in advective form, central differences
 *         (section 4.3):  N(u)_i = -u_i (u_{i+1} - u_{i-1}) / (2h) + nu lap(u)_i
 * Transposes are written out from the definition (A^T)_{ij} = A_{ji}.
 *
 * Built with -O2 -ffp-contract=off so no fused multiply-add is introduced.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int op;            /* 0 advdiff1d, 1 advdiff2d upwind, 2 burgers1d */
    int nx, ny;        /* ny = 1 in 1D */
    double L, vx, vy, nu;
    double T, omega, beta;
    long n_steps;
} orc_problem;

static long orc_n(const orc_problem* p) { return (long)p->nx * (long)p->ny; }

/* ---- right-hand side operators -------------------------------------- */

/* out = A u (linear operators) or N(u) (Burgers). */
void orc_rhs(const orc_problem* p, const double* u, double* out)
{
    if (p->op == 0 || p->op == 2) {
        int n = p->nx;
        double h = p->L / n;
        for (int i = 0; i < n; ++i) {
            double um = u[(i - 1 + n) % n], u0 = u[i], up = u[(i + 1) % n];
            double adv_speed = (p->op == 0) ? p->vx : u0;
            double adv = -adv_speed * (up - um) / (2.0 * h);
            double dif = p->nu * (up - 2.0 * u0 + um) / (h * h);
            out[i] = adv + dif;
        }
    } else {
        int nx = p->nx, ny = p->ny;
        double hx = p->L / nx, hy = p->L / ny;
        for (int j = 0; j < ny; ++j) {
            for (int i = 0; i < nx; ++i) {
                double c = u[(long)j * nx + i];
                double w = u[(long)j * nx + (i - 1 + nx) % nx];
                double e = u[(long)j * nx + (i + 1) % nx];
                double s = u[(long)((j - 1 + ny) % ny) * nx + i];
                double nn = u[(long)((j + 1) % ny) * nx + i];
                double adv = -p->vx * (c - w) / hx - p->vy * (c - s) / hy;
                double dif = p->nu * ((e - 2.0 * c + w) / (hx * hx)
                                      + (nn - 2.0 * c + s) / (hy * hy));
                out[(long)j * nx + i] = adv + dif;
            }
        }
    }
}

/* out = J(U)^T lam, J = dRHS/du at state U (U ignored for linear ops).
 * Written as the transpose of the row-wise Jacobian entries. */
void orc_rhs_adjoint(const orc_problem* p, const double* U, const double* lam,
                     double* out)
{
    long n = orc_n(p);
    for (long i = 0; i < n; ++i) out[i] = 0.0;
    if (p->op == 0 || p->op == 2) {
        int nx = p->nx;
        double h = p->L / nx;
        for (int r = 0; r < nx; ++r) {          /* row r of J */
            int rm = (r - 1 + nx) % nx, rp = (r + 1) % nx;
            double jm, j0, jp;                  /* J[r][rm], J[r][r], J[r][rp] */
            if (p->op == 0) {
                jm = p->vx / (2.0 * h) + p->nu / (h * h);
                j0 = -2.0 * p->nu / (h * h);
                jp = -p->vx / (2.0 * h) + p->nu / (h * h);
            } else {
                jm = U[r] / (2.0 * h) + p->nu / (h * h);
                j0 = -(U[rp] - U[rm]) / (2.0 * h) - 2.0 * p->nu / (h * h);
                jp = -U[r] / (2.0 * h) + p->nu / (h * h);
            }
            out[rm] += jm * lam[r];
            out[r] += j0 * lam[r];
            out[rp] += jp * lam[r];
        }
    } else {
        int nx = p->nx, ny = p->ny;
        double hx = p->L / nx, hy = p->L / ny;
        double cw = p->vx / hx + p->nu / (hx * hx);  /* coefficient of west */
        double cs = p->vy / hy + p->nu / (hy * hy);  /* coefficient of south */
        double ce = p->nu / (hx * hx), cn = p->nu / (hy * hy);
        double cc = -p->vx / hx - p->vy / hy
                    - 2.0 * p->nu / (hx * hx) - 2.0 * p->nu / (hy * hy);
        for (int j = 0; j < ny; ++j) {
            for (int i = 0; i < nx; ++i) {
                long r = (long)j * nx + i;
                long w = (long)j * nx + (i - 1 + nx) % nx;
                long e = (long)j * nx + (i + 1) % nx;
                long s = (long)((j - 1 + ny) % ny) * nx + i;
                long nn = (long)((j + 1) % ny) * nx + i;
                out[w] += cw * lam[r];
                out[s] += cs * lam[r];
                out[e] += ce * lam[r];
                out[nn] += cn * lam[r];
                out[r] += cc * lam[r];
            }
        }
    }
}

/* ---- one RK4 step ------------------------------------------------------ */

/* Stage states Y1..Y4 and slopes k1..k4 of the step from y at time t. */
static void rk4_stages(const orc_problem* p, const double* y, double t,
                       const double* F, double* Y /* 4n */, double* k /* 4n */)
{
    long n = orc_n(p);
    double dt = p->T / (double)p->n_steps;
    double c[4] = {0.0, 0.5, 0.5, 1.0};
    for (int st = 0; st < 4; ++st) {
        double* Ys = Y + st * n;
        double* ks = k + st * n;
        if (st == 0) {
            memcpy(Ys, y, n * sizeof(double));
        } else {
            const double* kp = k + (st - 1) * n;
            double a = (st == 3) ? dt : 0.5 * dt;
            for (long i = 0; i < n; ++i) Ys[i] = y[i] + a * kp[i];
        }
        orc_rhs(p, Ys, ks);
        if (F) {
            double sv = sin(p->omega * (t + c[st] * dt));
            for (long i = 0; i < n; ++i) ks[i] += sv * F[i];
        }
    }
}

/* March the direct problem; traj (n_steps+1 states) is optional. */
int orc_direct(const orc_problem* p, const double* q0, const double* F,
               double* qT, double* traj)
{
    long n = orc_n(p);
    double dt = p->T / (double)p->n_steps;
    double* y = malloc(n * sizeof(double));
    double* Y = malloc(4 * n * sizeof(double));
    double* k = malloc(4 * n * sizeof(double));
    if (!y || !Y || !k) { free(y); free(Y); free(k); return 1; }
    memcpy(y, q0, n * sizeof(double));
    if (traj) memcpy(traj, y, n * sizeof(double));
    for (long s = 0; s < p->n_steps; ++s) {
        rk4_stages(p, y, s * dt, F, Y, k);
        for (long i = 0; i < n; ++i)
            y[i] = y[i] + dt / 6.0 * (k[i] + 2.0 * k[n + i] + 2.0 * k[2 * n + i]
                                      + k[3 * n + i]);
        if (traj) memcpy(traj + (s + 1) * n, y, n * sizeof(double));
    }
    memcpy(qT, y, n * sizeof(double));
    free(y); free(Y); free(k);
    return 0;
}

/*
 * Reverse sweep of the RK4 march: from lam = dJ/dq(T) to lam0 = dJ/dq0,
 * accumulating Lambda = sum_steps sum_stages s(t_stage) * kbar_stage.
 * traj holds all step states (needed for the nonlinear Jacobian; unused by
 * the linear operators but always supplied by orc_gradient).
 */
int orc_adjoint(const orc_problem* p, const double* traj, const double* F,
                const double* lamT, double* lam0, double* Lambda)
{
    long n = orc_n(p);
    double dt = p->T / (double)p->n_steps;
    double* lam = malloc(n * sizeof(double));
    double* Y = malloc(4 * n * sizeof(double));
    double* k = malloc(4 * n * sizeof(double));
    double* kb = malloc(4 * n * sizeof(double));
    double* Yb = malloc(n * sizeof(double));
    double* nl = malloc(n * sizeof(double));
    if (!lam || !Y || !k || !kb || !Yb || !nl) {
        free(lam); free(Y); free(k); free(kb); free(Yb); free(nl); return 1;
    }
    memcpy(lam, lamT, n * sizeof(double));
    if (Lambda) for (long i = 0; i < n; ++i) Lambda[i] = 0.0;
    double c[4] = {0.0, 0.5, 0.5, 1.0};
    double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    /* The linear operators have a state-independent Jacobian, so their
     * reverse sweep needs no stored trajectory (traj may be NULL). */
    int linear = (p->op != 2);
    for (long s = p->n_steps - 1; s >= 0; --s) {
        double t = s * dt;
        if (!linear) rk4_stages(p, traj + s * n, t, F, Y, k);
        /* y_{s+1} = y_s + dt sum_i b_i k_i  =>  kbar_i = dt b_i lam. */
        for (int st = 0; st < 4; ++st)
            for (long i = 0; i < n; ++i) kb[st * n + i] = dt * b[st] * lam[i];
        for (long i = 0; i < n; ++i) nl[i] = lam[i];   /* ybar_s, direct term */
        for (int st = 3; st >= 0; --st) {
            /* k_st = RHS(Y_st): Ybar_st = J(Y_st)^T kbar_st. */
            orc_rhs_adjoint(p, Y + st * n, kb + st * n, Yb);
            for (long i = 0; i < n; ++i) nl[i] += Yb[i];
            /* Y_st = y_s + a_st k_{st-1}: kbar_{st-1} += a_st Ybar_st. */
            if (st > 0) {
                double a = (st == 3) ? dt : 0.5 * dt;
                for (long i = 0; i < n; ++i) kb[(st - 1) * n + i] += a * Yb[i];
            }
        }
        if (Lambda) {
            for (int st = 0; st < 4; ++st) {
                double sv = sin(p->omega * (t + c[st] * dt));
                for (long i = 0; i < n; ++i) Lambda[i] += sv * kb[st * n + i];
            }
        }
        memcpy(lam, nl, n * sizeof(double));
    }
    memcpy(lam0, lam, n * sizeof(double));
    free(lam); free(Y); free(k); free(kb); free(Yb); free(nl);
    return 0;
}

/*
 * One full direct-adjoint loop.
 *   control 0 (forcing amplitudes): F = sum_k a_k basis_k, q(0) = q0.
 *   control 1 (initial-condition amplitudes): q(0) = q0 + sum_k a_k basis_k,
 *             no forcing.
 * Outputs (any may be NULL except J): qT, J, grad (K), lam0, Lambda.
 */
int orc_gradient(const orc_problem* p, int control, int K,
                 const double* basis, const double* a, const double* q0,
                 const double* q_tgt, double* qT, double* J, double* grad,
                 double* lam0_out, double* Lambda_out)
{
    long n = orc_n(p);
    double* traj = (p->op == 2)
        ? malloc((p->n_steps + 1) * n * sizeof(double)) : malloc(sizeof(double));
    double* F = calloc(n, sizeof(double));
    double* init = malloc(n * sizeof(double));
    double* fin = malloc(n * sizeof(double));
    double* lamT = malloc(n * sizeof(double));
    double* lam0 = malloc(n * sizeof(double));
    double* Lam = malloc(n * sizeof(double));
    int rc = 1;
    if (!traj || !F || !init || !fin || !lamT || !lam0 || !Lam) goto done;
    for (long i = 0; i < n; ++i) init[i] = q0 ? q0[i] : 0.0;
    if (control == 0) {
        for (int kk = 0; kk < K; ++kk)
            for (long i = 0; i < n; ++i) F[i] += a[kk] * basis[kk * n + i];
    } else {
        for (int kk = 0; kk < K; ++kk)
            for (long i = 0; i < n; ++i) init[i] += a[kk] * basis[kk * n + i];
    }
    const double* Fp = (control == 0) ? F : NULL;
    if (orc_direct(p, init, Fp, fin, (p->op == 2) ? traj : NULL)) goto done;
    double jt = 0.0, jr = 0.0;
    for (long i = 0; i < n; ++i) {
        double d = fin[i] - q_tgt[i];
        jt += 0.5 * d * d;
        lamT[i] = d;              /* conj(dJ_T/dq(T)), real problem */
    }
    for (int kk = 0; kk < K; ++kk) jr += p->beta * a[kk] * a[kk];
    *J = jt + jr;
    if (orc_adjoint(p, traj, Fp, lamT, lam0, Lam)) goto done;
    if (grad) {
        for (int kk = 0; kk < K; ++kk) {
            const double* v = (control == 0) ? Lam : lam0;
            double g = 0.0;
            for (long i = 0; i < n; ++i) g += basis[kk * n + i] * v[i];
            grad[kk] = g + 2.0 * p->beta * a[kk];
        }
    }
    if (qT) memcpy(qT, fin, n * sizeof(double));
    if (lam0_out) memcpy(lam0_out, lam0, n * sizeof(double));
    if (Lambda_out) memcpy(Lambda_out, Lam, n * sizeof(double));
    rc = 0;
done:
    free(traj); free(F); free(init); free(fin); free(lamT); free(lam0);
    free(Lam);
    return rc;
}

/*
 * Integral cost (section 4.2, eq. cost):
 *   J = sum_{n=0}^{n_t} w_n ||q_n - q_tgt||^2 + beta ||a||^2,
 *   w_n = dt c_n / T, c_0 = c_{n_t} = 1/2, c_n = 1 otherwise
 * (the trapezoidal rule for 1/T int_0^T ||q - q_tgt||^2 dt on the RK4 step
 * states).  Every q_n enters J, so the exact discrete adjoint is the reverse
 * sweep of orc_adjoint with dJ/dq_n = 2 w_n (q_n - q_tgt) added to the
 * adjoint after the step that produces lambda_n, starting from
 * lambda_{n_t} = dJ/dq_{n_t}.  Written out here rather than folded into
 * orc_adjoint so that the terminal-cost path stays as it is.
 */
static double icost_weight(const orc_problem* p, long s)
{
    double dt = p->T / (double)p->n_steps;
    double c = (s == 0 || s == p->n_steps) ? 0.5 : 1.0;
    return dt * c / p->T;
}

static int orc_adjoint_icost(const orc_problem* p, const double* traj, const double* F,
                             const double* q_tgt, double* lam0, double* Lambda)
{
    long n = orc_n(p);
    double dt = p->T / (double)p->n_steps;
    double* lam = malloc(n * sizeof(double));
    double* Y = malloc(4 * n * sizeof(double));
    double* k = malloc(4 * n * sizeof(double));
    double* kb = malloc(4 * n * sizeof(double));
    double* Yb = malloc(n * sizeof(double));
    double* nl = malloc(n * sizeof(double));
    if (!lam || !Y || !k || !kb || !Yb || !nl) {
        free(lam); free(Y); free(k); free(kb); free(Yb); free(nl); return 1;
    }
    {
        double w = icost_weight(p, p->n_steps);
        const double* qn = traj + p->n_steps * n;
        for (long i = 0; i < n; ++i) lam[i] = 2.0 * w * (qn[i] - q_tgt[i]);
    }
    if (Lambda) for (long i = 0; i < n; ++i) Lambda[i] = 0.0;
    double c[4] = {0.0, 0.5, 0.5, 1.0};
    double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    int linear = (p->op != 2);
    for (long s = p->n_steps - 1; s >= 0; --s) {
        double t = s * dt;
        if (!linear) rk4_stages(p, traj + s * n, t, F, Y, k);
        for (int st = 0; st < 4; ++st)
            for (long i = 0; i < n; ++i) kb[st * n + i] = dt * b[st] * lam[i];
        for (long i = 0; i < n; ++i) nl[i] = lam[i];
        for (int st = 3; st >= 0; --st) {
            orc_rhs_adjoint(p, Y + st * n, kb + st * n, Yb);
            for (long i = 0; i < n; ++i) nl[i] += Yb[i];
            if (st > 0) {
                double a = (st == 3) ? dt : 0.5 * dt;
                for (long i = 0; i < n; ++i) kb[(st - 1) * n + i] += a * Yb[i];
            }
        }
        if (Lambda) {
            for (int st = 0; st < 4; ++st) {
                double sv = sin(p->omega * (t + c[st] * dt));
                for (long i = 0; i < n; ++i) Lambda[i] += sv * kb[st * n + i];
            }
        }
        /* q_s is a cost argument too: add dJ/dq_s */
        double w = icost_weight(p, s);
        const double* qs = traj + s * n;
        for (long i = 0; i < n; ++i) lam[i] = nl[i] + 2.0 * w * (qs[i] - q_tgt[i]);
    }
    memcpy(lam0, lam, n * sizeof(double));
    free(lam); free(Y); free(k); free(kb); free(Yb); free(nl);
    return 0;
}

/* One direct-adjoint loop with the integral cost; arguments as for
 * orc_gradient. */
int orc_gradient_icost(const orc_problem* p, int control, int K,
                       const double* basis, const double* a, const double* q0,
                       const double* q_tgt, double* qT, double* J, double* grad,
                       double* lam0_out, double* Lambda_out)
{
    long n = orc_n(p);
    double* traj = malloc((p->n_steps + 1) * n * sizeof(double));
    double* F = calloc(n, sizeof(double));
    double* init = malloc(n * sizeof(double));
    double* fin = malloc(n * sizeof(double));
    double* lam0 = malloc(n * sizeof(double));
    double* Lam = malloc(n * sizeof(double));
    int rc = 1;
    if (!traj || !F || !init || !fin || !lam0 || !Lam) goto done;
    for (long i = 0; i < n; ++i) init[i] = q0 ? q0[i] : 0.0;
    if (control == 0) {
        for (int kk = 0; kk < K; ++kk)
            for (long i = 0; i < n; ++i) F[i] += a[kk] * basis[kk * n + i];
    } else {
        for (int kk = 0; kk < K; ++kk)
            for (long i = 0; i < n; ++i) init[i] += a[kk] * basis[kk * n + i];
    }
    const double* Fp = (control == 0) ? F : NULL;
    if (orc_direct(p, init, Fp, fin, traj)) goto done;
    double ji = 0.0, jr = 0.0;
    for (long s = 0; s <= p->n_steps; ++s) {
        double w = icost_weight(p, s), acc = 0.0;
        const double* qs = traj + s * n;
        for (long i = 0; i < n; ++i) {
            double d = qs[i] - q_tgt[i];
            acc += d * d;
        }
        ji += w * acc;
    }
    for (int kk = 0; kk < K; ++kk) jr += p->beta * a[kk] * a[kk];
    *J = ji + jr;
    if (orc_adjoint_icost(p, traj, Fp, q_tgt, lam0, Lam)) goto done;
    if (grad) {
        for (int kk = 0; kk < K; ++kk) {
            const double* v = (control == 0) ? Lam : lam0;
            double g = 0.0;
            for (long i = 0; i < n; ++i) g += basis[kk * n + i] * v[i];
            grad[kk] = g + 2.0 * p->beta * a[kk];
        }
    }
    if (qT) memcpy(qT, fin, n * sizeof(double));
    if (lam0_out) memcpy(lam0_out, lam0, n * sizeof(double));
    if (Lambda_out) memcpy(Lambda_out, Lam, n * sizeof(double));
    rc = 0;
done:
    free(traj); free(F); free(init); free(fin); free(lam0); free(Lam);
    return rc;
}
