"""Complex Ginzburg-Landau in a doubly periodic square (oracle; test infrastructure only).

Sec. 6: u_t = u + (1 + i b) lap u - (1 + i c) |u|^2 u on [-L/2, L/2)^2 with
Fourier x Fourier bases (the paper's case is b = 0, c = 1.5, L = 100).  The
Fourier-Galerkin form (eq. Ginz_var) has a diagonal left-hand side, so the
spectral right-hand side is
    rhs(u_hat) = (1 - (1 + i b)|k|^2) u_hat - F_trunc[(1 + i c) |u_p|^2 u_p],
with k = (2 pi / L) * integer wavenumbers and u_p the 3/2-padded backward
transform (retained modes evaluated on the Mp = floor(3N/2) grid, every other
padded coefficient zero), and F_trunc the forward transform on that grid
(1/Mp per axis) truncated to the retained modes (Sec. 6, padded transforms).

Time steppers:
  rk4_step   -- the classical four-stage scheme exactly as in Sec. 6
                (a = [1/6, 1/3, 1/3, 1/6], b = [1/2, 1/2, 1])
  ifrk4_step -- the same RK4 applied after the integrating-factor change of
                variables v = exp(-Lhat t) u_hat (Lawson 1967), which treats the
                stiff linear part exactly; used where the explicit scheme's
                stability limit is exceeded.
"""
import numpy as np

from . import fourier


def kgrid(N, L):
    k = fourier.wavenumbers(N) * (2 * np.pi / L)
    return k[:, None], k[None, :]


def padded_size(N):
    return (3 * N) // 2


def linear_symbol(N, L, b):
    kx, ky = kgrid(N, L)
    return 1.0 - (1.0 + 1j * b) * (kx**2 + ky**2)


def nonlinear(uh, c):
    """F_trunc[(1 + i c)|u_p|^2 u_p] for the N x N spectrum uh."""
    N = uh.shape[0]
    up = fourier.padded_backward(uh, padded_size(N))
    w = (1.0 + 1j * c) * np.abs(up) ** 2 * up
    return fourier.padded_forward_truncate(w, N)


def rhs(uh, L, b, c):
    N = uh.shape[0]
    return linear_symbol(N, L, b) * uh - nonlinear(uh, c)


def rk4_step(uh, dt, L, b, c):
    a = [1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0]
    bb = [0.5, 0.5, 1.0]
    u0 = uh.copy()
    u1 = uh.copy()
    u = uh.copy()
    for rk in range(4):
        du = rhs(u, L, b, c)
        if rk < 3:
            u = u0 + bb[rk] * dt * du
        u1 = u1 + a[rk] * dt * du
    return u1


def ifrk4_step(uh, dt, L, b, c):
    """One Lawson IF-RK4 step; E = exp(Lhat dt / 2), Nl(v) = -nonlinear(v)."""
    N = uh.shape[0]
    E = np.exp(linear_symbol(N, L, b) * (dt / 2))
    E2 = E * E
    k1 = -nonlinear(uh, c)
    k2 = -nonlinear(E * (uh + 0.5 * dt * k1), c)
    k3 = -nonlinear(E * uh + 0.5 * dt * k2, c)
    k4 = -nonlinear(E2 * uh + dt * E * k3, c)
    return E2 * uh + (dt / 6.0) * (E2 * k1 + 2.0 * E * (k2 + k3) + k4)


def grid(N, L):
    return -L / 2 + L * np.arange(N) / N


def forward(u):
    """2D forward transform (1/N^2) of a physical N x N field."""
    return fourier.forward(fourier.forward(u, axis=0), axis=1)


def backward(uh):
    return fourier.backward(fourier.backward(uh, axis=0), axis=1)
