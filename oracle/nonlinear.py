"""Oracle: the iterative nonlinear Paraexp direct solve (section 3.2).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  The HIP
library never imports or calls it, and it imports nothing from the HIP
package.  Dense n x n operators: small grids only.

Burgers (section 4.3, periodic grid, spacing h = L/n, central differences)
split as in eq. nl into its linear part and its genuine nonlinearity:
    dq/dt = A q + N(q),   A = nu lap,   N(q) = -q * (D q).

One iteration i -> i+1 in the paper's shifted variable q~ = q - q0
(eqs. nonlinTrans, Jacobians, nlHomIter, fullsolIter, algorithm 2):
  * J_{i,p}: the time average of dN/dq at the iterate q_i over
    [T_p, T_{p+1}] -- the Jacobian matrices themselves averaged by the
    trapezoidal rule on the RK4 step grid;
  * inhomogeneous problem of slice p, from zero at T_p:
        dq~/dt = (A + J_{i,p}) q~ + A q0 + N(q_i) - J_{i,p} (q_i - q0),
    marched by classical RK4 with q_i taken at the stage points;
  * homogeneous problems: slice p carries q_{I,p-1}(T_p) (j = 0) and every
    piece of slice p-1 (j >= 1), each propagated over slice p on its own by
    the matrix exponential of (T_{p+1} - T_p)(A + J_{i,p});
  * the new iterate: q0 + q_I + the sum of slice p's homogeneous pieces
    (eq. fullsolIter).
Readings where the paper leaves the discrete form open:
  * the iterate at the RK4 stage points of slice p (the next iteration's
    N(q_i) and q_i, and its step states) is the stage values of the slice's
    inhomogeneous equation marched by RK4 from the sum of the homogeneous
    pieces at T_p; q(T) is the end of the last slice's march;
  * the first guess is q0 at every point (algorithm 2 leaves it open);
  * the error after an iteration is the relative change of q(T).
At a fixed point every stage source is N at that stage's own state, so the
iterate is the nonlinear RK4 march inside every slice; the slice starts
come from exact exponentials, which differ from RK4's propagation by RK4's
own time error.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm


def burgers_split(inst: dict):
    """Dense A = nu lap and D (central first difference), periodic."""
    n = int(inst["nx"])
    h = float(inst["L"]) / n
    D = np.zeros((n, n))
    lap = np.zeros((n, n))
    for i in range(n):
        D[i, (i + 1) % n] += 1.0 / (2.0 * h)
        D[i, (i - 1) % n] -= 1.0 / (2.0 * h)
        lap[i, (i + 1) % n] += 1.0 / (h * h)
        lap[i, (i - 1) % n] += 1.0 / (h * h)
        lap[i, i] -= 2.0 / (h * h)
    return float(inst["nu"]) * lap, D


def n_of(q, D):
    """N(q) = -q * (D q)."""
    return -q * (D @ q)


def jac_n(q, D):
    """dN/dq at q: -diag(q) D - diag(D q)."""
    return -(q[:, None] * D) - np.diag(D @ q)


def initial_state(inst: dict) -> np.ndarray:
    """q0 of an initial-condition-control instance: q0 + sum_k a_k phi_k."""
    n = int(inst["nx"])
    q0 = np.asarray(inst.get("q0", np.zeros(n)), dtype=np.float64)
    if inst["control"] == "ic":
        q0 = q0 + np.asarray(inst["a"]) @ np.asarray(inst["basis"])
    return q0


_C = (0.0, 0.5, 0.5, 1.0)
_W = (1.0, 2.0, 2.0, 1.0)


def _march(M, src, y, dt):
    """RK4 of dy/dt = M y + src[s, k] (the source at stage k of step s) from
    y; returns the stage values [S, 4, n] and the end value."""
    S = src.shape[0]
    stages = np.empty_like(src)
    for s in range(S):
        acc = np.zeros_like(y)
        slope = None
        for k in range(4):
            Y = y if k == 0 else y + _C[k] * dt * slope
            stages[s, k] = Y
            slope = M @ Y + src[s, k]
            acc += _W[k] * slope
        y = y + (dt / 6.0) * acc
    return stages, y


def nl_paraexp_direct(inst: dict, iters: int, P: int | None = None) -> dict:
    """``iters`` iterations from the first guess q0.  Returns q(T) after
    every iteration (``qT_iters``), the final iterate's step states
    (``traj``, [n_steps + 1, n]) and the relative change of q(T) in every
    iteration (``change``)."""
    A, D = burgers_split(inst)
    q0 = initial_state(inst)
    n = q0.size
    n_t = int(inst["n_steps"])
    P = int(inst["P"] if P is None else P)
    if n_t % P:
        raise ValueError("n_steps must be a multiple of P")
    S = n_t // P
    dt = float(inst["T"]) / n_t
    # the previous iterate at the stage points and at T (first guess: q0)
    O = np.broadcast_to(q0, (n_t, 4, n)).copy()
    qT_prev = q0.copy()
    tw = np.ones(S + 1)
    tw[0] = tw[-1] = 0.5
    qT_iters, change = [], []
    for _ in range(iters):
        Mp, src = [], []
        for p in range(P):
            steps = [O[s, 0] for s in range(p * S, (p + 1) * S)]
            steps.append(qT_prev if p == P - 1 else O[(p + 1) * S, 0])
            Jp = sum(w * jac_n(q, D) for w, q in zip(tw, steps)) / S
            M = A + Jp
            b = np.empty((S, 4, n))
            for s in range(S):
                for k in range(4):
                    o = O[p * S + s, k]
                    b[s, k] = A @ q0 + n_of(o, D) - Jp @ (o - q0)
            Mp.append(M)
            src.append(b)
        # inhomogeneous problems from zero, every slice independently
        q_I = [_march(Mp[p], src[p], np.zeros(n), dt)[1] for p in range(P)]
        # homogeneous pieces at each slice start, then the dense slices
        O_new = np.empty_like(O)
        pieces = []
        qT = None
        for p in range(P):
            if p > 0:
                E = expm((S * dt) * Mp[p - 1])
                pieces = [q_I[p - 1]] + [E @ v for v in pieces]
            start = sum(pieces) if pieces else np.zeros(n)
            st, end = _march(Mp[p], src[p], start, dt)
            O_new[p * S:(p + 1) * S] = st + q0
            if p == P - 1:
                qT = end + q0
        change.append(float(np.linalg.norm(qT - qT_prev) / np.linalg.norm(qT)))
        O, qT_prev = O_new, qT
        qT_iters.append(qT)
    traj = np.concatenate([O[:, 0], qT_prev[None, :]], axis=0)
    return dict(qT_iters=qT_iters, qT=qT_prev, traj=traj, change=change)
