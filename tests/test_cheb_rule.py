"""Host checks of the numerical rules behind the Chebyshev flavour of the
Burgers chains (the focal-interval polynomial of section 4.1 in the
Chebyshev basis), independent of the GPU:

  - the scaled modified Bessel coefficients e_k = e^{-g} I_k(g) from
    Miller's backward recurrence, started 24 orders above the table and
    normalised by e^g = I_0 + 2 sum I_k, against scipy.special.ive;
  - the a priori degree (the first k >= g with e_k + e_{k+1} <= tol/16)
    leaves a truncation error of exp on the interval below tol;
  - the series reproduces exp(tau M) v for a diffusion-dominated
    nonsymmetric matrix (a small periodic Burgers Jacobian) on the
    Gershgorin interval of its real parts.

The recurrence here is written from its definition for this test; the
kernel's arithmetic is checked end to end against the oracle on the GPU."""
import math

import numpy as np
import pytest
from scipy.linalg import expm
from scipy.special import ive

CHEB_KMAX = 320


def table(g):
    """e_0 .. e_{kc+1} for half-width g (kc as the kernel chooses it)."""
    kc = int(min(CHEB_KMAX - 1, g + 6.0 * math.sqrt(g) + 40.0))
    top = kc + 24
    ip, ik, s = 0.0, 1e-200, 0.0
    e = np.zeros(kc + 2)
    for k in range(top, 0, -1):
        if k <= kc + 1:
            e[k] = ik
        s += 2.0 * ik
        ip, ik = ik, ip + (2.0 * k / g) * ik
        if ik > 1e200:
            e[k:] *= 1e-200
            ip *= 1e-200
            ik *= 1e-200
            s *= 1e-200
    e[0] = ik
    s += ik
    return e / s, kc


def apriori(e, g, kc, tol):
    for k in range(max(1, math.ceil(g)), kc):
        if e[k] + e[k + 1] <= tol / 16:
            return k
    return kc - 1


@pytest.mark.parametrize("g", [0.5, 1.0, 3.7, 8.3, 16.6, 40.0, 120.0, 200.0])
def test_coefficients_match_scaled_bessel(g):
    e, kc = table(g)
    ref = ive(np.arange(kc + 2), g)
    # absolute error relative to e_0 (the coefficients span many decades)
    assert np.max(np.abs(e - ref)) <= 1e-14 * max(1.0, ref[0])


@pytest.mark.parametrize("g", [0.5, 2.0, 8.3, 16.6, 60.0, 150.0])
@pytest.mark.parametrize("tol", [1e-6, 1e-9, 1e-12])
def test_apriori_degree_bounds_the_tail(g, tol):
    """|exp(c + g x) - series_K(x)| <= e^{c+g} 2 sum_{k>K} e_k on [-1, 1]:
    the tail beyond the a priori degree is below tol (relative to the
    largest value e^{c+g})."""
    e, kc = table(g)
    K = apriori(e, g, kc, tol)
    tail = 2.0 * ive(np.arange(K + 1, K + 400), g).sum()
    assert tail <= tol
    # and the truncated series on a grid of x
    x = np.linspace(-1.0, 1.0, 201)
    T = np.cos(np.outer(np.arange(K + 1), np.arccos(x)))
    s = e[0] * T[0] + 2.0 * (e[1:K + 1, None] * T[1:]).sum(axis=0)
    assert np.max(np.abs(s - np.exp(g * (x - 1.0)))) <= 2 * tol


def test_series_on_burgers_jacobian():
    """exp(tau J(W)^T) v by the series on the Gershgorin interval equals the
    dense exponential for a 128-point periodic Burgers Jacobian with a
    moderate advecting state (skew part a small fraction of the interval)."""
    n, L, nu = 128, 2 * math.pi, 0.02
    h = L / n
    x = np.arange(n) * h
    W = 0.8 * np.sin(x) + 0.3 * np.cos(3 * x)
    J = np.zeros((n, n))
    for i in range(n):
        im, ip = (i - 1) % n, (i + 1) % n
        J[i, im] += nu / h**2 + W[i] / (2 * h)
        J[i, ip] += nu / h**2 - W[i] / (2 * h)
        J[i, i] += -2 * nu / h**2 - (W[ip] - W[im]) / (2 * h)
    M = J.T
    tau = 0.05
    d = np.diag(M)
    off = np.abs(M).sum(axis=1) - np.abs(d)
    lo, hi = tau * np.min(d - off), tau * np.max(d + off)
    c, g = 0.5 * (hi + lo), 0.5 * (hi - lo)
    tol = 1e-11
    e, kc = table(g)
    K = apriori(e, g, kc, tol)
    v = np.exp(-((x - 2.0) ** 2) / 0.3)
    A = (tau * M - c * np.eye(n)) / g
    t0, t1 = v, A @ v
    acc = e[0] * t0 + 2 * e[1] * t1
    for k in range(2, K + 3):
        t0, t1 = t1, 2 * (A @ t1) - t0
        acc = acc + 2 * e[k] * t1
    got = math.exp(c + g) * acc
    want = expm(tau * M) @ v
    assert np.linalg.norm(got - want) <= 10 * tol * np.linalg.norm(v)
