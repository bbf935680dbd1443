"""TEST INFRASTRUCTURE ONLY: an independent high-accuracy solution of the
periodic 2-D KGS equations, against which the oracle's discretisation error
is measured.

The equations (sec. 1 of arXiv 2502.09537) in the real form of sec. 2, with
psi = p + i q and v = u_t:

    psi_t = i (kappa1/2 Lap psi + gamma u psi)
    u_t   = v
    v_t   = kappa2 Lap u - mu^2 u + gamma |psi|^2

Space is Fourier pseudo-spectral on [lo, hi)^2 (exact derivatives of the
trigonometric interpolant); time is the classical fourth-order Runge-Kutta
method.  This shares nothing with the oracle or with the GPU library: it is
a different discretisation of the same PDE, standing in for the sixth-order
spectral reference solution that the paper computes for its 2-D accuracy
table (sec. 5.1), which is not published.
"""
from __future__ import annotations

import numpy as np


def grid_axis(n: int, lo: float, hi: float) -> np.ndarray:
    """x_j = lo + j h, j = 0..n-1 (the paper's x_j = a + (j-1) h)."""
    return lo + (hi - lo) / n * np.arange(n)


def _wavenumbers(n: int, lo: float, hi: float) -> np.ndarray:
    return 2.0 * np.pi * np.fft.fftfreq(n, d=(hi - lo) / n)


def solve(psi, u, v, lo: float, hi: float, t_end: float, steps: int,
          kappa1=1.0, kappa2=1.0, mu=1.0, gamma=1.0):
    """(psi, u, v) at t_end from the initial fields on an n x n periodic grid,
    with `steps` classical Runge-Kutta steps."""
    n = psi.shape[0]
    k = _wavenumbers(n, lo, hi)
    minus_k2 = -(k[:, None] ** 2 + k[None, :] ** 2)

    def lap(f):
        return np.fft.ifft2(minus_k2 * np.fft.fft2(f))

    def rhs(p, a, b):
        dp = 1j * (0.5 * kappa1 * lap(p) + gamma * a * p)
        db = kappa2 * lap(a).real - mu * mu * a + gamma * (p.real ** 2 + p.imag ** 2)
        return dp, b, db

    dt = t_end / steps
    p = np.asarray(psi, dtype=complex).copy()
    a = np.asarray(u, dtype=float).copy()
    b = np.asarray(v, dtype=float).copy()
    for _ in range(steps):
        k1 = rhs(p, a, b)
        k2 = rhs(p + 0.5 * dt * k1[0], a + 0.5 * dt * k1[1], b + 0.5 * dt * k1[2])
        k3 = rhs(p + 0.5 * dt * k2[0], a + 0.5 * dt * k2[1], b + 0.5 * dt * k2[2])
        k4 = rhs(p + dt * k3[0], a + dt * k3[1], b + dt * k3[2])
        p = p + dt / 6.0 * (k1[0] + 2.0 * k2[0] + 2.0 * k3[0] + k4[0])
        a = a + dt / 6.0 * (k1[1] + 2.0 * k2[1] + 2.0 * k3[1] + k4[1])
        b = b + dt / 6.0 * (k1[2] + 2.0 * k2[2] + 2.0 * k3[2] + k4[2])
    return p, a, b


def energy(psi, u, v, lo: float, hi: float, kappa1=1.0, kappa2=1.0, mu=1.0, gamma=1.0):
    """The continuous energy of sec. 2 with spectral gradients and the
    trapezoidal (exact for trigonometric polynomials) quadrature."""
    n = psi.shape[0]
    h = (hi - lo) / n
    k = _wavenumbers(n, lo, hi)

    def grad2(f):
        F = np.fft.fft2(f)
        gx = np.fft.ifft2(1j * k[:, None] * F)
        gy = np.fft.ifft2(1j * k[None, :] * F)
        return np.abs(gx) ** 2 + np.abs(gy) ** 2

    dens = (0.5 * (kappa1 * grad2(psi) + kappa2 * grad2(u) + v ** 2 + mu * mu * u ** 2)
            - gamma * np.abs(psi) ** 2 * u)
    return h * h * float(np.sum(dens))


def _pad_axis(F, m: int, axis: int):
    """Spectrum F of n samples along `axis` as the spectrum of m samples of
    the same trigonometric interpolant: frequencies |k| < n/2 are kept, the
    Nyquist coefficient (k = -n/2) is split evenly between k = +n/2 and
    k = -n/2, and the new frequencies are zero."""
    F = np.moveaxis(F, axis, 0)
    n = F.shape[0]
    h = n // 2
    G = np.zeros((m,) + F.shape[1:], dtype=complex)
    G[:h] = F[:h]
    G[h] = 0.5 * F[h]
    G[m - h] = 0.5 * F[h]
    G[m - h + 1:] = F[h + 1:]
    return np.moveaxis(G, 0, axis)


def resample(f, m: int):
    """The trigonometric interpolant of the n x n periodic samples f at an
    m x m grid over the same box (m >= n, both even)."""
    n = f.shape[0]
    if m == n:
        return np.asarray(f).copy()
    G = _pad_axis(_pad_axis(np.fft.fft2(f), m, 0), m, 1)
    out = np.fft.ifft2(G) * (m / n) ** 2
    return out if np.iscomplexobj(f) else out.real
