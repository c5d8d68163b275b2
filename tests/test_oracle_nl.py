"""Pins of the oracle's iterative nonlinear Paraexp direct (section 3.2).

Each pin ties the oracle to something other than itself:
  - the split A q + N(q) against the C oracle's Burgers right-hand side, and
    A + dN/dq against the C oracle's transposed Jacobian (written row by row
    from the definition there);
  - dN/dq against central differences of N, exact for a quadratic map;
  - one slice (P = 1): no exponential is involved, the fixed point is the
    serial nonlinear RK4 march, to rounding, at every step;
  - the first iteration (guess q0 everywhere) solves the linearisation
    about q0, whose solution is q0 + T phi_1(T M0) f(q0) (M0 = A + J(q0),
    f the full right-hand side), evaluated by the exponential of the
    augmented matrix [[M0, f], [0, 0]]; the oracle reaches it at RK4's
    fourth order in dt;
  - several slices: the fixed point differs from the serial RK4 march only
    by the slice starts, propagated by exact exponentials instead of RK4
    steps, so the gap falls at fourth order in dt;
  - the iterates' changes shrink until rounding (the scheme converges).
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm

import oracle
from oracle import nonlinear as onl
from paper_2004_00546_amd import workloads


def rel(x, r):
    return float(np.linalg.norm(np.asarray(x) - r) / np.linalg.norm(r))


def burgers(n=64, T=0.5, nt=256, P=8, nu=0.05, K=6, seed=11, amp=0.9):
    rng = np.random.default_rng(seed)
    phases = rng.uniform(0, 2 * math.pi, K)
    return dict(op="burgers1d", control="ic", nx=n, ny=1, L=2 * math.pi, vx=0.0, vy=0.0,
                nu=nu, T=T, omega=1.0, beta=1e-3, n_steps=nt, P=P, m=30, ckpt_every=16,
                basis=workloads.burgers_ic_modes(n, 2 * math.pi, phases),
                a=amp * rng.standard_normal(K) / np.arange(1, K + 1),
                u_tgt=rng.standard_normal(n), q0=np.zeros(n))


def test_split_matches_c_oracle():
    inst = burgers()
    A, D = onl.burgers_split(inst)
    rng = np.random.default_rng(3)
    q, lam = rng.standard_normal(64), rng.standard_normal(64)
    assert rel(A @ q + onl.n_of(q, D), oracle.rhs(inst, q)) < 1e-14
    full = A + onl.jac_n(q, D)
    assert rel(full.T @ lam, oracle.rhs_adjoint(inst, q, lam)) < 1e-14


def test_jacobian_is_exact_central_difference():
    inst = burgers()
    _, D = onl.burgers_split(inst)
    rng = np.random.default_rng(4)
    q, x = rng.standard_normal(64), rng.standard_normal(64)
    fd = 0.5 * (onl.n_of(q + x, D) - onl.n_of(q - x, D))
    assert rel(onl.jac_n(q, D) @ x, fd) < 1e-14


def test_one_slice_fixed_point_is_the_serial_march():
    inst = burgers(P=1, nt=128)
    q0 = onl.initial_state(inst)
    qT, traj = oracle.direct(inst, q0, traj=True)
    r = onl.nl_paraexp_direct(inst, 12)
    assert rel(r["qT"], qT) < 1e-13
    assert rel(r["traj"], traj) < 1e-13


def test_first_iteration_is_the_linearisation_about_q0():
    errs = []
    for nt in (64, 128, 256):
        inst = burgers(P=4, nt=nt)
        q0 = onl.initial_state(inst)
        A, D = onl.burgers_split(inst)
        f0 = oracle.rhs(inst, q0)
        n = q0.size
        aug = np.zeros((n + 1, n + 1))
        aug[:n, :n] = A + onl.jac_n(q0, D)
        aug[:n, n] = f0
        closed = q0 + expm(inst["T"] * aug)[:n, n]
        r = onl.nl_paraexp_direct(inst, 1)
        errs.append(rel(r["qT"], closed))
        # far from the nonlinear solution: the pin separates the two
        assert rel(r["qT"], oracle.direct(inst, q0)) > 1e-3
    assert errs[-1] < 1e-10
    for coarse, fine in zip(errs, errs[1:]):
        assert 12.0 < coarse / fine < 20.0, errs


def test_fixed_point_gap_is_fourth_order():
    gaps = []
    for nt in (128, 256, 512):
        inst = burgers(nt=nt)
        q0 = onl.initial_state(inst)
        r = onl.nl_paraexp_direct(inst, 10)
        gaps.append(rel(r["qT"], oracle.direct(inst, q0)))
    assert gaps[-1] < 1e-11
    for coarse, fine in zip(gaps, gaps[1:]):
        assert 12.0 < coarse / fine < 20.0, gaps


def test_iteration_converges():
    r = onl.nl_paraexp_direct(burgers(), 8)
    ch = r["change"]
    assert ch[0] > 1e-2 and ch[-1] < 1e-14
    k = next(i for i, c in enumerate(ch) if c < 1e-14)
    assert all(b < a for a, b in zip(ch[:k], ch[1:k + 1])), ch


def test_rejects_ragged_slices():
    with pytest.raises(ValueError):
        onl.nl_paraexp_direct(burgers(nt=100, P=8), 1)
