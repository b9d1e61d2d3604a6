"""Legendre and Shen-Legendre bases by direct evaluation (oracle; test infrastructure only).

Sec. 3.1 lists Legendre versions of every Chebyshev basis; Sec. 3.4.2 gives the
Legendre-Gauss quadrature: x_j the zeros of L_N, w_j = 2 / ((1 - x_j^2) L_N'(x_j)^2),
and the Dirichlet basis L_l - L_{l+2} (eq. shen_legendre_basis, eq. legdirichlet).
The transforms are the plain O(N^2) sums the paper says the Legendre bases use.

Bases (phi_l = sum_k P[k, l] L_k):
  "legendre":       phi_l = L_l,                                        l = 0..N-1
  "leg_dirichlet":  phi_l = L_l - L_{l+2},                              l = 0..N-3
  "leg_neumann":    phi_l = L_l - l(l+1)/((l+2)(l+3)) L_{l+2},          l = 0..N-3
  "leg_biharmonic": phi_l = L_l - 2(2l+5)/(2l+7) L_{l+2} + (2l+3)/(2l+7) L_{l+4},
                                                                        l = 0..N-5
The paper names the Neumann basis without a formula and prints the biharmonic
one garbled (eq. legbiharmonic: k for l and the L_{l+4} factor missing); these
are the standard Shen-Legendre bases, the ones whose functions satisfy
phi'(+-1) = 0, resp. phi(+-1) = phi'(+-1) = 0 (pinned by the tests).

Points are stored in descending order (x_0 nearest +1), as the Chebyshev points
x_j = cos((2j+1) pi / (2N)) are.  L_k(x_j) comes from the three-term recurrence
(k+1) L_{k+1} = (2k+1) x L_k - k L_{k-1} in extended precision; the points from
Newton's method on L_N started at the Chebyshev-Gauss points.

Forward transform: the weighted least-squares projection min sum_j w_j |u_j -
sum_l u_hat_l phi_l(x_j)|^2 (B^{-1} S(u), eq. projection), by a dense Householder
QR in extended precision; backward: u(x_j) = sum_l u_hat_l phi_l(x_j).

Galerkin matrices (Sec. 3.4, eq. cheb_poisson with the Legendre weight 1): mass
B_ml = (phi_l, phi_m), stiffness A_ml = (phi_l'', phi_m) and, for the biharmonic
problem, S_ml = (phi_l^(4), phi_m) by Legendre-Gauss
quadrature in extended precision (exact: the integrands have degree <= 2N - 2);
derivatives of the basis functions from the exact Legendre derivative relation
(numpy.polynomial.legendre.legder on extended-precision coefficients).
"""
import functools

import numpy as np
from numpy.polynomial import legendre as nplegendre

from .linalg import householder_qr, lstsq_qr

LD = np.longdouble
PI_LD = np.arccos(LD(-1))
BASES = ("legendre", "leg_dirichlet", "leg_neumann", "leg_biharmonic")


def nbasis(basis, N):
    return {"legendre": N, "leg_dirichlet": N - 2, "leg_neumann": N - 2, "leg_biharmonic": N - 4}[basis]


def _legendre_and_derivative(n, x):
    """(L_n(x), L_n'(x)) by the three-term recurrence (extended precision)."""
    p0, p1 = np.ones_like(x), x.copy()
    if n == 0:
        return p0, np.zeros_like(x)
    for k in range(1, n):
        p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
    # (1 - x^2) L_n' = n (L_{n-1} - x L_n)
    return p1, n * (p0 - x * p1) / (1 - x * x)


@functools.lru_cache(maxsize=32)
def nodes_weights(N):
    """Legendre-Gauss points (descending) and weights, extended precision."""
    j = np.arange(N)
    x = np.cos(PI_LD * (4 * j + 3) / (4 * N + 2))   # standard initial guesses
    for _ in range(100):
        p, dp = _legendre_and_derivative(N, x)
        dx = p / dp
        x = x - dx
        if np.abs(dx).max() < LD(1e-30):
            break
    _, dp = _legendre_and_derivative(N, x)
    w = 2 / ((1 - x * x) * dp * dp)
    return x, w


def points(N):
    return nodes_weights(N)[0].astype(np.float64)


def weights(N):
    return nodes_weights(N)[1].astype(np.float64)


@functools.lru_cache(maxsize=32)
def lmatrix(N, K=None):
    """L[j, k] = L_k(x_j), k = 0..K-1 (default N), extended precision."""
    K = N if K is None else K
    x = nodes_weights(N)[0]
    out = np.zeros((N, K), dtype=LD)
    out[:, 0] = 1
    if K > 1:
        out[:, 1] = x
    for k in range(1, K - 1):
        out[:, k + 1] = ((2 * k + 1) * x * out[:, k] - k * out[:, k - 1]) / (k + 1)
    return out


@functools.lru_cache(maxsize=32)
def recombination(basis, N):
    """P[k, l]: Legendre coefficient k of basis function l."""
    nb = nbasis(basis, N)
    P = np.zeros((N, nb), dtype=LD)
    for l in range(nb):
        P[l, l] = 1
        if basis == "leg_dirichlet":
            P[l + 2, l] = -1
        elif basis == "leg_neumann":
            P[l + 2, l] = -LD(l * (l + 1)) / LD((l + 2) * (l + 3))
        elif basis == "leg_biharmonic":
            P[l + 2, l] = -LD(2 * (2 * l + 5)) / LD(2 * l + 7)
            P[l + 4, l] = LD(2 * l + 3) / LD(2 * l + 7)
    return P


@functools.lru_cache(maxsize=32)
def synthesis(basis, N):
    """Phi[j, l] = phi_l(x_j) (extended precision)."""
    return lmatrix(N) @ recombination(basis, N)


@functools.lru_cache(maxsize=32)
def derivative_synthesis(basis, N, order):
    """Phi^(order)[j, l] = phi_l^(order)(x_j) (extended precision)."""
    P = recombination(basis, N)
    D = np.zeros_like(P)
    for l in range(P.shape[1]):
        d = nplegendre.legder(P[:, l], order)
        D[: len(d), l] = d
    return lmatrix(N) @ D


def _apply_left(mat, a, axis):
    a = np.moveaxis(np.asarray(a), axis, 0)
    sh = a.shape
    flat = a.reshape(sh[0], -1)
    if np.iscomplexobj(flat):
        out = (mat @ flat.real.astype(LD)).astype(np.float64) + 1j * (mat @ flat.imag.astype(LD)).astype(np.float64)
    else:
        out = (mat @ flat.astype(LD)).astype(np.float64)
    return np.moveaxis(out.reshape((mat.shape[0],) + sh[1:]), 0, axis)


def scalar_product(basis, u, axis=0):
    """S_m(u) = sum_j u(x_j) phi_m(x_j) w_j along `axis` (nb outputs)."""
    N = np.shape(u)[axis]
    w = nodes_weights(N)[1]
    return _apply_left(synthesis(basis, N).T * w[None, :], u, axis)


@functools.lru_cache(maxsize=32)
def mass_matrix(basis, N):
    Phi = synthesis(basis, N)
    w = nodes_weights(N)[1]
    return Phi.T @ (Phi * w[:, None])


@functools.lru_cache(maxsize=32)
def stiffness_matrix(basis, N):
    """A[m, l] = (phi_l'', phi_m) by Legendre-Gauss quadrature."""
    w = nodes_weights(N)[1]
    return synthesis(basis, N).T @ (derivative_synthesis(basis, N, 2) * w[:, None])


@functools.lru_cache(maxsize=32)
def bilaplace_matrix(basis, N):
    """S[m, l] = (phi_l^(4), phi_m) by Legendre-Gauss quadrature (Sec. 4, biharmonic problem)."""
    w = nodes_weights(N)[1]
    return synthesis(basis, N).T @ (derivative_synthesis(basis, N, 4) * w[:, None])


@functools.lru_cache(maxsize=16)
def _projection_qr(basis, N):
    w = nodes_weights(N)[1]
    return householder_qr(synthesis(basis, N) * np.sqrt(w)[:, None])


def forward(basis, u, axis=0):
    """u_hat = B^{-1} S(u) as the weighted least-squares problem (extended-precision QR)."""
    N = np.shape(u)[axis]
    V, R = _projection_qr(basis, N)
    wh = np.sqrt(nodes_weights(N)[1])[:, None]
    a = np.moveaxis(np.asarray(u), axis, 0)
    sh = a.shape
    flat = a.reshape(sh[0], -1)
    x = lstsq_qr(V, R, flat.real.astype(LD) * wh).astype(np.float64)
    if np.iscomplexobj(flat):
        x = x + 1j * lstsq_qr(V, R, flat.imag.astype(LD) * wh).astype(np.float64)
    return np.moveaxis(x.reshape((x.shape[0],) + sh[1:]), 0, axis)


def backward(basis, uh, axis=0):
    """u(x_j) = sum_l u_hat_l phi_l(x_j) along `axis` (N outputs)."""
    nb = np.shape(uh)[axis]
    N = nb + {"legendre": 0, "leg_dirichlet": 2, "leg_neumann": 2, "leg_biharmonic": 4}[basis]
    return _apply_left(synthesis(basis, N), uh, axis)
