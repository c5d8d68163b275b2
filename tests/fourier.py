"""Closed forms for constant-coefficient periodic operators (test-only).

Every operator of the advection-diffusion problems (paper section 4.2) is
circulant, so Fourier modes diagonalise it.  These helpers evaluate, mode by
mode, (i) the exact RK4 recurrence for y' = lambda y + sin(omega t) f and
(ii) the exact semi-discrete solution, independently of the oracle's stencil
and RK4 code.  They pin the oracle; they are not part of it.
"""
import numpy as np


def eig_advdiff1d(n, L, c, nu):
    h = L / n
    th = 2.0 * np.pi * np.arange(n) / n
    return -1j * c * np.sin(th) / h + nu * (2.0 * np.cos(th) - 2.0) / h ** 2


def eig_advdiff2d_upwind(nx, ny, L, vx, vy, nu):
    hx, hy = L / nx, L / ny
    th = 2.0 * np.pi * np.arange(nx) / nx
    ph = 2.0 * np.pi * np.arange(ny) / ny
    TH, PH = th[None, :], ph[:, None]
    return (-vx * (1.0 - np.exp(-1j * TH)) / hx - vy * (1.0 - np.exp(-1j * PH)) / hy
            + nu * ((2.0 * np.cos(TH) - 2.0) / hx ** 2
                    + (2.0 * np.cos(PH) - 2.0) / hy ** 2))


def eigenvalues(inst):
    if inst["op"] == "advdiff1d":
        return eig_advdiff1d(inst["nx"], inst["L"], inst["vx"], inst["nu"])
    if inst["op"] == "advdiff2d_upwind":
        return eig_advdiff2d_upwind(inst["nx"], inst["ny"], inst["L"],
                                    inst["vx"], inst["vy"], inst["nu"])
    raise ValueError(inst["op"])


def _fft(inst, v):
    if inst.get("ny", 1) > 1:
        return np.fft.fft2(np.asarray(v).reshape(inst["ny"], inst["nx"]))
    return np.fft.fft(v)


def _ifft(inst, v):
    if inst.get("ny", 1) > 1:
        return np.fft.ifft2(v).real.ravel()
    return np.fft.ifft(v).real


def rk4_transfer(inst, lam=None):
    """Per-mode factor t(lambda) with yhat(T) = t * fhat for y(0) = 0.

    One RK4 step of y' = lam y + s(t) f from y_n gives
    y_{n+1} = R(z) y_n + dt/6 [s1 p1(z) + s2 p2(z) + s4] f,  z = dt lam,
    R = 1 + z + z^2/2 + z^3/6 + z^4/24, p1 = 1 + z + z^2/2 + z^3/4,
    p2 = 4 + 2 z + z^2/2, s1, s2, s4 = s at t_n, t_n + dt/2, t_n + dt
    (obtained by expanding the four stages by hand)."""
    if lam is None:
        lam = eigenvalues(inst)
    nt = int(inst["n_steps"])
    dt = inst["T"] / nt
    w = inst.get("omega", 1.0)
    z = dt * lam
    R = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    p1 = 1 + z + z ** 2 / 2 + z ** 3 / 4
    p2 = 4 + 2 * z + z ** 2 / 2
    x = np.zeros_like(lam)
    for k in range(nt):
        t = k * dt
        s1, s2, s4 = np.sin(w * t), np.sin(w * (t + dt / 2)), np.sin(w * (t + dt))
        x = R * x + dt / 6 * (s1 * p1 + s2 * p2 + s4)
    return x


def exact_transfer(inst, lam=None):
    """Semi-discrete exact: int_0^T sin(w t) e^{lam (T-t)} dt per mode."""
    if lam is None:
        lam = eigenvalues(inst)
    T, w = inst["T"], inst.get("omega", 1.0)
    return (w * np.exp(lam * T) - lam * np.sin(w * T) - w * np.cos(w * T)) / (
        lam ** 2 + w ** 2)


def apply_transfer(inst, tr, F):
    return _ifft(inst, tr * _fft(inst, F))


def gradient_closed_form(inst, tr, a=None):
    """g = M^T (u(T) - u_tgt) + 2 beta a with M's columns from the per-mode
    transfer factor (linear problem, u0 = 0, forcing control)."""
    a = inst["a"] if a is None else a
    G = inst["basis"]
    F = a @ G
    uT = apply_transfer(inst, tr, F)
    r = uT - inst["u_tgt"]
    M = np.stack([apply_transfer(inst, tr, G[k]) for k in range(G.shape[0])])
    J = 0.5 * r @ r + inst["beta"] * a @ a
    return uT, J, M @ r + 2 * inst["beta"] * a


def exp_action(inst, tau, v, lam=None):
    """exp(tau A) v exactly, through the Fourier diagonalisation."""
    if lam is None:
        lam = eigenvalues(inst)
    return _ifft(inst, np.exp(tau * lam) * _fft(inst, v))


def exp_action_T(inst, tau, v, lam=None):
    """exp(tau A^T) v: A^T is circulant with conjugated eigenvalues for a
    real operator."""
    if lam is None:
        lam = eigenvalues(inst)
    return _ifft(inst, np.exp(tau * np.conj(lam)) * _fft(inst, v))
