"""Seeded synthetic workloads for the direct-adjoint gradient.

This module only draws random numbers and evaluates the input shapes
(forcing pulses, initial-condition modes, target fields).  It holds none of
the method's arithmetic, so both the HIP path and the CPU oracle may consume
what it produces.

The paper's experiments (section 4.2, 4.3) use periodic advection-diffusion
and viscous Burgers problems on [0, 2*pi]^d with forcing f(x) sin(omega t);
the five workloads below are concrete instances of that family:

* ``advdiff1d_n128``  1D advection-diffusion, N=128, T=1, 8 slices, 4 pulses
* ``advdiff1d_n4096`` 1D advection-diffusion, N=4096, T=4, 64 slices, 64 pulses
* ``burgers1d_n2048`` 1D viscous Burgers, N=2048, T=2, 128 slices, IC control
* ``advdiff2d_256``   2D upwind advection-diffusion 256^2, 16 instances
* ``burgers1d_ragged`` 64 Burgers instances of uneven N, nu and T
* ``advdiff2d_icost`` the integral-cost experiment of section 4.2 (eq. cost):
  2D forced advection-diffusion 128^2, a = 1, omega = 1, T = 10, four
  diffusivities D in {0.01, 0.02, 0.05, 0.1}, forcing control on the
  patterns {1, sin x sin y}; the paper recovers f_true = sin x sin y from
  the guess f = 1 against the observed trajectory q_true(t).  The problem is
  linear with zero initial state, so q_f(t) - q_true(t) = q_{f - f_true}(t):
  the instances hold the difference amplitudes a = (1, -1) and a zero
  target, which gives the same cost and gradient.
* ``burgers1d_icost`` the N=2048 Burgers instance above with the integral
  cost (the hybrid serial-direct-parallel-adjoint scheme of section 3.3):
  128 Magnus steps and 128 equal adjoint slices, four per launch.
* ``burgers1d_nl``    the N=2048 Burgers instance above with the direct
  solved by the iterative nonlinear Paraexp of section 3.2 (64 slices of
  the iteration, at most 8 iterations, ended by the change of q(T); the
  adjoint keeps its 128 Magnus steps).

Every instance is a plain dict of numbers and float64 numpy arrays.  Random
draws come from ``numpy.random.default_rng([1000 + cfg, instance])`` in the
order documented in each builder.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi

# RK4's stability interval on the negative real axis ends at about -2.785.
RK4_REAL_LIMIT = 2.785

WORKLOADS = ("advdiff1d_n128", "advdiff1d_n4096", "burgers1d_n2048",
             "advdiff2d_256", "burgers1d_ragged", "advdiff2d_icost", "burgers1d_icost",
             "burgers1d_nl")
CFG_INDEX = {name: i + 1 for i, name in enumerate(WORKLOADS)}


def _rng(cfg: int, instance: int) -> np.random.Generator:
    return np.random.default_rng([1000 + cfg, instance])


def _periodic_dist(x: np.ndarray, c: float, L: float) -> np.ndarray:
    d = np.abs(x - c) % L
    return np.minimum(d, L - d)


def gaussian_pulses_1d(n: int, L: float, centres: np.ndarray,
                       sigma: float) -> np.ndarray:
    """G_k(x_i) = exp(-d(x_i, c_k)^2 / (2 sigma^2)), periodic distance d."""
    x = np.arange(n) * (L / n)
    G = np.empty((len(centres), n))
    for k, c in enumerate(centres):
        d = _periodic_dist(x, c, L)
        G[k] = np.exp(-d * d / (2.0 * sigma * sigma))
    return G


def gaussian_blobs_2d(nx: int, ny: int, L: float, centres: np.ndarray,
                      sigma: float) -> np.ndarray:
    """Isotropic periodic Gaussian blobs, flattened row-major (y, x)."""
    x = np.arange(nx) * (L / nx)
    y = np.arange(ny) * (L / ny)
    G = np.empty((len(centres), ny * nx))
    for k, (cx, cy) in enumerate(centres):
        dx = _periodic_dist(x, cx, L)[None, :]
        dy = _periodic_dist(y, cy, L)[:, None]
        G[k] = np.exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma)).ravel()
    return G


def _fd_dirs(rng: np.random.Generator, K: int, count: int = 8) -> np.ndarray:
    d = rng.standard_normal((count, K))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def _target_1d(rng, n, L):
    b = rng.standard_normal(4)
    th = rng.uniform(0.0, TWO_PI, 4)
    x = np.arange(n) * (L / n)
    j = np.arange(1, 5)
    return (b[:, None] * np.sin(j[:, None] * (TWO_PI / L) * x[None, :]
                                + th[:, None])).sum(0)


def _advdiff1d(cfg: int, n: int, T: float, dt: float, P: int, K: int,
               m: int) -> dict:
    """Draw order: pulse centres (K), amplitudes (K), target amplitudes (4),
    target phases (4), finite-difference directions (8 x K)."""
    rng = _rng(cfg, 0)
    L = TWO_PI
    centres = L * rng.uniform(0.0, 1.0, K)
    a = rng.standard_normal(K)
    u_tgt = _target_1d(rng, n, L)
    fd = _fd_dirs(rng, K)
    n_steps = int(round(T / dt))
    return dict(op="advdiff1d", control="forcing", nx=n, ny=1, L=L,
                vx=1.0, vy=0.0, nu=0.01, T=T, omega=1.0, beta=1e-3,
                n_steps=n_steps, P=P, m=m,
                basis=gaussian_pulses_1d(n, L, centres, 0.05 * L),
                a=a, u_tgt=u_tgt, q0=np.zeros(n), fd_dirs=fd)


def burgers_ic_modes(n: int, L: float, phases: np.ndarray) -> np.ndarray:
    """phi_k(x) = sin(k x + theta_k), k = 1..K (x scaled to [0, 2 pi))."""
    x = np.arange(n) * (TWO_PI / n)
    k = np.arange(1, len(phases) + 1)
    return np.sin(k[:, None] * x[None, :] + phases[:, None])


def _burgers_instance(cfg: int, inst: int, n: int, nu: float, T: float,
                      n_steps: int, P: int, K: int, m: int, rng) -> dict:
    """Continues an rng: mode phases (K), amplitudes N(0, 0.1/k) (K),
    target amplitudes (4), target phases (4), FD directions (8 x K)."""
    L = TWO_PI
    phases = rng.uniform(0.0, TWO_PI, K)
    a = rng.standard_normal(K) * (0.1 / np.arange(1, K + 1))
    u_tgt = _target_1d(rng, n, L)
    fd = _fd_dirs(rng, K)
    return dict(op="burgers1d", control="ic", nx=n, ny=1, L=L, vx=0.0,
                vy=0.0, nu=nu, T=T, omega=1.0, beta=1e-3, n_steps=n_steps,
                P=P, m=m, ckpt_every=64,
                basis=burgers_ic_modes(n, L, phases), a=a, u_tgt=u_tgt,
                q0=np.zeros(n), fd_dirs=fd)


def burgers_dt_bound(n: int, nu: float, L: float = TWO_PI) -> float:
    """Largest RK4 step for the diffusion part: dt * 4 nu / h^2 <= 2.785."""
    h = L / n
    return RK4_REAL_LIMIT / (4.0 * nu / (h * h))


def make(name: str) -> list[dict]:
    """Return the list of instances of a named workload."""
    cfg = CFG_INDEX[name]
    if name == "advdiff1d_n128":
        return [_advdiff1d(cfg, 128, 1.0, 1e-3, 8, 4, 30)]
    if name == "advdiff1d_n4096":
        return [_advdiff1d(cfg, 4096, 4.0, 1e-4, 64, 64, 40)]
    if name == "burgers1d_n2048":
        rng = _rng(cfg, 0)
        return [_burgers_instance(cfg, 0, 2048, 5e-3, 2.0, 8192, 128, 32, 30,
                                  rng)]
    if name == "advdiff2d_256":
        out = []
        for i in range(16):
            rng = _rng(cfg, i)
            # Draw order: horizon T, blob centres (8 x 2), amplitudes (8),
            # target amplitudes (4), phases (4), wave numbers (4 x 2), FD dirs.
            T = float(rng.uniform(0.5, 2.0))
            L = TWO_PI
            K = 8
            centres = L * rng.uniform(0.0, 1.0, (K, 2))
            a = rng.standard_normal(K)
            b = rng.standard_normal(4)
            th = rng.uniform(0.0, TWO_PI, 4)
            pq = rng.integers(1, 5, (4, 2))
            nx = ny = 256
            x = np.arange(nx) * (L / nx)
            y = np.arange(ny) * (L / ny)
            u_tgt = np.zeros((ny, nx))
            for j in range(4):
                u_tgt += b[j] * np.sin(pq[j, 0] * x[None, :]
                                       + pq[j, 1] * y[:, None] + th[j])
            n_steps = 256 * int(math.ceil(T / (256 * 2e-3)))
            out.append(dict(op="advdiff2d_upwind", control="forcing", nx=nx,
                            ny=ny, L=L, vx=1.0, vy=0.5, nu=1e-3, T=T,
                            omega=1.0, beta=1e-3, n_steps=n_steps, P=256,
                            m=50,
                            basis=gaussian_blobs_2d(nx, ny, L, centres,
                                                    0.05 * L),
                            a=a, u_tgt=u_tgt.ravel(), q0=np.zeros(nx * ny),
                            fd_dirs=_fd_dirs(rng, K)))
        return out
    if name == "burgers1d_ragged":
        out = []
        for i in range(64):
            rng = _rng(cfg, i)
            # Draw order: N, nu, T, then as _burgers_instance.
            n = int(rng.choice([1024, 2048, 4096, 8192]))
            nu = float(rng.uniform(2e-3, 1e-2))
            T = float(rng.uniform(1.0, 3.0))
            dt = 0.9 * burgers_dt_bound(n, nu)
            n_steps = 256 * int(math.ceil(T / (256 * dt)))
            out.append(_burgers_instance(cfg, i, n, nu, T, n_steps, 64, 32,
                                         30, rng))
        return out
    if name == "burgers1d_nl":
        inst = make("burgers1d_n2048")[0]
        return [dict(inst, nl_paraexp=True, nl_iters=8, nl_slices=64)]
    if name == "burgers1d_icost":
        inst = make("burgers1d_n2048")[0]
        return [dict(inst, cost="integral", hyb_slices=128, hyb_k=0.0, hyb_group=4)]
    if name == "advdiff2d_icost":
        out = []
        nx = ny = 128
        L = TWO_PI
        x = np.arange(nx) * (L / nx)
        y = np.arange(ny) * (L / ny)
        patterns = np.stack([np.ones((ny, nx)),
                             np.sin(x[None, :]) * np.sin(y[:, None])])
        for i, D in enumerate((0.01, 0.02, 0.05, 0.1)):
            rng = _rng(cfg, i)  # draws: FD directions only
            out.append(dict(op="advdiff2d_upwind", control="forcing", cost="integral",
                            nx=nx, ny=ny, L=L, vx=1.0, vy=1.0, nu=D, T=10.0,
                            omega=1.0, beta=0.0, n_steps=2048, P=512, m=50,
                            basis=patterns.reshape(2, nx * ny).copy(),
                            a=np.array([1.0, -1.0]), u_tgt=np.zeros(nx * ny),
                            q0=np.zeros(nx * ny), fd_dirs=_fd_dirs(rng, 2)))
        return out
    raise KeyError(name)


def scaled(inst: dict, n_steps: int | None = None, T: float | None = None,
           P: int | None = None) -> dict:
    """Copy of an instance with a shorter horizon (same dt unless given)."""
    out = dict(inst)
    if T is not None:
        dt = inst["T"] / inst["n_steps"]
        out["T"] = T
        out["n_steps"] = int(round(T / dt)) if n_steps is None else n_steps
    elif n_steps is not None:
        out["n_steps"] = n_steps
    if P is not None:
        out["P"] = P
    return out
