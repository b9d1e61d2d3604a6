"""Fourier bases by plain summation (oracle; test infrastructure only).

Sec. 3.4.1 (periodic boundary conditions): grid x_j = 2 pi j / M, wavenumbers
l = -M/2 .. M/2-1 (eq. wavenumber_even), forward transform
u_hat_l = (1/M) sum_j u_j exp(-i l x_j), backward u_j = sum_l u_hat_l exp(i l x_j)
(eq. ufourier).  Arrays are kept in FFT order (index q = l mod M).  R2C keeps
q = 0..M/2 and uses u_hat_{M-q} = conj(u_hat_q) (end of Sec. 3.4.1).

Each phase exp(+-2 pi i l j / M) is computed from the exactly reduced integer
(l*j) mod M, so no phase error grows with l*j.  The sums are matrix products
with those exact-phase DFT matrices.
"""
from functools import lru_cache

import numpy as np

# 2 pi to the full x87 extended precision
TWO_PI_LD = 2 * np.arccos(np.longdouble(-1))


def wavenumbers(M):
    """Integer wavenumbers in FFT order: 0..ceil(M/2)-1, then -floor(M/2)..-1.

    For even M the index M/2 holds -M/2, as in eq. wavenumber_even."""
    q = np.arange(M)
    return np.where(q < (M + 1) // 2, q, q - M)


def dft_matrix(M, sign, rows=None):
    """E[q, j] = exp(sign * 2 pi i ((q*j) mod M) / M) for q in rows (default all)."""
    q = np.arange(M) if rows is None else np.asarray(rows)
    r = np.mod(np.outer(q, np.arange(M)), M).astype(np.longdouble)
    ang = sign * TWO_PI_LD * r / M
    return (np.cos(ang) + 1j * np.sin(ang)).astype(np.complex128)


def _apply(mat, a, axis):
    a = np.moveaxis(np.asarray(a), axis, 0)
    sh = a.shape
    out = mat @ a.reshape(sh[0], -1)
    return np.moveaxis(out.reshape((mat.shape[0],) + sh[1:]), 0, axis)


def forward(u, axis=-1):
    """C2C forward: u_hat_q = (1/M) sum_j u_j exp(-2 pi i q j / M)."""
    M = np.shape(u)[axis]
    return _apply(dft_matrix(M, -1), np.asarray(u, dtype=np.complex128), axis) / M


def backward(uh, axis=-1):
    """C2C backward (unnormalised): u_j = sum_q u_hat_q exp(2 pi i q j / M)."""
    M = np.shape(uh)[axis]
    return _apply(dft_matrix(M, +1), np.asarray(uh, dtype=np.complex128), axis)


def rforward(u, axis=-1):
    """R2C forward of real data: the first M//2+1 coefficients of `forward`."""
    M = np.shape(u)[axis]
    E = dft_matrix(M, -1, rows=np.arange(M // 2 + 1))
    return _apply(E, np.asarray(u, dtype=np.float64).astype(np.complex128), axis) / M


def hermitian_extend(uh, M, axis=-1):
    """Rebuild the full FFT-order spectrum from the R2C half using
    u_hat_{M-q} = conj(u_hat_q).  The imaginary parts of q = 0 and (even M)
    q = M/2 are discarded: those coefficients of real data are real."""
    uh = np.moveaxis(np.asarray(uh, dtype=np.complex128), axis, 0)
    full = np.zeros((M,) + uh.shape[1:], dtype=np.complex128)
    h = M // 2 + 1
    full[:h] = uh[:h]
    full[0] = full[0].real
    if M % 2 == 0:
        full[M // 2] = full[M // 2].real
    for q in range(1, (M + 1) // 2):
        full[M - q] = np.conj(full[q])
    return np.moveaxis(full, 0, axis)


def rbackward(uh, M, axis=-1):
    """C2R backward: real part of `backward` of the Hermitian-extended spectrum."""
    return backward(hermitian_extend(uh, M, axis), axis).real


def padded_backward(uh, Mp, axes=(0, 1)):
    """Backward transform of the retained modes evaluated on a finer grid of Mp
    points per axis (the padded transform of Sec. 6): every retained FFT-order
    coefficient keeps its wavenumber l, all other padded modes are zero.
    u_p(x_j) = sum_{l retained} u_hat_l exp(i l 2 pi j / Mp)."""
    out = np.asarray(uh, dtype=np.complex128)
    for ax in axes:
        out = _apply(_padded_matrix(Mp, out.shape[ax], +1), out, ax)
    return out


def padded_forward_truncate(w, N, axes=(0, 1)):
    """Forward transform on the fine grid (1/Mp per axis) followed by truncation
    to the N retained wavenumbers of the coarse grid (FFT order)."""
    out = np.asarray(w, dtype=np.complex128)
    for ax in axes:
        Mp = out.shape[ax]
        out = _apply(_padded_matrix(Mp, N, -1), out, ax) / Mp
    return out


@lru_cache(maxsize=64)
def _padded_matrix(Mp, N, sign):
    """Exact-phase matrix between the N retained wavenumbers l and the Mp fine
    grid points j: exp(+i l 2 pi j / Mp) as Mp x N (sign +1, padded backward) or
    exp(-i l 2 pi j / Mp) as N x Mp (sign -1, forward before truncation).  Kept
    per size (read-only), since every Runge-Kutta stage uses the same ones."""
    l = wavenumbers(N)
    j = np.arange(Mp)
    r = np.mod(np.outer(j, l) if sign > 0 else np.outer(l, j), Mp).astype(np.longdouble)
    ang = sign * TWO_PI_LD * r / Mp
    E = (np.cos(ang) + 1j * np.sin(ang)).astype(np.complex128)
    E.setflags(write=False)
    return E
