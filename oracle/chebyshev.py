"""Chebyshev and Shen bases by direct evaluation (oracle; test infrastructure only).

Sec. 3.4.2 (Dirichlet boundary conditions): Gauss-Chebyshev points
x_j = cos((2j+1) pi / (2N)) and weights w_j = pi/N; the discrete weighted
inner product (u, v)^N_w = sum_j u(x_j) v(x_j) w_j (eq. quadrature, Sec. 2).

Bases (recombinations of T_k, stored as an N x nb matrix P with phi_l = sum_k P[k,l] T_k):
  "dirichlet":  phi_l = T_l - T_{l+2},                 l = 0..N-3   (eq. chebdirichlet)
  "biharmonic": phi_l = T_l - 2(l+2)/(l+3) T_{l+2} + (l+1)/(l+3) T_{l+4},
                                                       l = 0..N-5   (eq. chebbiharmonic, Sec. 4)
  "chebyshev":  phi_l = T_l,                           l = 0..N-1   (regular basis, Sec. 3.1)
  "neumann":    phi_l = T_l - (l/(l+2))^2 T_{l+2},     l = 0..N-3   (Shen's Neumann basis; Sec. 3.1
                names it without a formula, this is the standard one with phi_l'(+-1) = 0)

T_k(x_j) = cos(k (2j+1) pi / (2N)) is evaluated from the exactly reduced integer
k(2j+1) mod 4N in extended precision.  Matrices are assembled by Gauss
quadrature in extended precision: mass B_ml = (phi_l, phi_m), stiffness
A_ml = (phi_l'', phi_m) (eq. cheb_poisson) and the fourth-derivative matrix
S_ml = (phi_l'''', phi_m) (Sec. 4, biharmonic problem); derivatives of the
basis functions come from the exact Chebyshev derivative recurrence
(numpy.polynomial.chebyshev.chebder on extended-precision coefficients).

Forward transform (Sec. 3.4.2, eq. projection and the lines after it):
u_hat = B^{-1} S(u) with the Shen scalar product S_m(u) = (u, phi_m)^N_w;
backward transform u(x_j) = sum_l u_hat_l phi_l(x_j) (eq. fast_shen).
"""
import functools

import numpy as np
from numpy.polynomial import chebyshev as npcheb

from .linalg import householder_qr, lstsq_qr, solve_refined

LD = np.longdouble
# pi to the full x87 extended precision (np.pi is a binary64 constant)
PI_LD = np.arccos(LD(-1))
BASES = ("dirichlet", "biharmonic", "chebyshev", "neumann")


def points(N):
    j = np.arange(N)
    return np.cos((2 * j + 1) * np.pi / (2 * N))


def weights(N):
    return np.full(N, np.pi / N)


def nbasis(basis, N):
    return {"dirichlet": N - 2, "biharmonic": N - 4, "chebyshev": N, "neumann": N - 2}[basis]


@functools.lru_cache(maxsize=32)
def tmatrix(N, K=None):
    """T[j, k] = T_k(x_j), k = 0..K-1 (default N), longdouble."""
    K = N if K is None else K
    r = np.mod(np.outer(2 * np.arange(N) + 1, np.arange(K)), 4 * N).astype(LD)
    return np.cos(PI_LD * r / (2 * N))


@functools.lru_cache(maxsize=32)
def recombination(basis, N, K=None):
    """P[k, l]: Chebyshev coefficient k of basis function l (K rows, default N)."""
    K = N if K is None else K
    nb = nbasis(basis, N)
    P = np.zeros((K, nb), dtype=LD)
    for l in range(nb):
        P[l, l] = 1
        if basis == "dirichlet":
            P[l + 2, l] = -1
        elif basis == "biharmonic":
            P[l + 2, l] = -LD(2 * (l + 2)) / LD(l + 3)
            P[l + 4, l] = LD(l + 1) / LD(l + 3)
        elif basis == "neumann":
            P[l + 2, l] = -(LD(l) / LD(l + 2)) ** 2
    return P


@functools.lru_cache(maxsize=32)
def synthesis(basis, N):
    """Phi[j, l] = phi_l(x_j) (longdouble)."""
    return tmatrix(N) @ recombination(basis, N)


@functools.lru_cache(maxsize=32)
def derivative_synthesis(basis, N, order):
    """Phi^(order)[j, l] = phi_l^(order)(x_j) (longdouble)."""
    P = recombination(basis, N)
    D = np.zeros_like(P)
    for l in range(P.shape[1]):
        d = npcheb.chebder(P[:, l], order)
        D[: len(d), l] = d
    return tmatrix(N) @ D


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
    """S_m(u) = sum_j u(x_j) phi_m(x_j) pi/N along `axis` (nb outputs)."""
    N = np.shape(u)[axis]
    Phi = synthesis(basis, N)
    return _apply_left(Phi.T * (PI_LD / N), u, axis)


@functools.lru_cache(maxsize=32)
def mass_matrix(basis, N):
    Phi = synthesis(basis, N)
    return (Phi.T @ Phi) * (PI_LD / N)


@functools.lru_cache(maxsize=32)
def stiffness_matrix(basis, N):
    """A[m, l] = (phi_l'', phi_m)^N_w."""
    return (synthesis(basis, N).T @ derivative_synthesis(basis, N, 2)) * (PI_LD / N)


@functools.lru_cache(maxsize=32)
def bilaplace_matrix(basis, N):
    """S[m, l] = (phi_l'''', phi_m)^N_w."""
    return (synthesis(basis, N).T @ derivative_synthesis(basis, N, 4)) * (PI_LD / N)


@functools.lru_cache(maxsize=16)
def _projection_qr(basis, N):
    """Householder QR (extended precision) of the weighted synthesis matrix
    W^{1/2} Phi, W = diag(pi/N)."""
    return householder_qr(synthesis(basis, N) * np.sqrt(PI_LD / N))


def forward(basis, u, axis=0):
    """u_hat = B^{-1} S(u) along `axis`.

    B u_hat = S(u) are the normal equations of the weighted least-squares
    problem  min_u_hat sum_j w_j |u(x_j) - sum_l u_hat_l phi_l(x_j)|^2  (the
    projection of eq. projection); the oracle solves that least-squares
    problem with a dense Householder QR in extended precision.  B itself is
    ill-conditioned for the biharmonic basis (cond ~ 1e8 at N = 512), so
    forming and solving the normal equations directly would lose digits; the
    small-N test pins both forms against each other."""
    N = np.shape(u)[axis]
    V, R = _projection_qr(basis, N)
    wh = np.sqrt(PI_LD / N)
    a = np.moveaxis(np.asarray(u), axis, 0)
    sh = a.shape
    flat = a.reshape(sh[0], -1)
    x = lstsq_qr(V, R, flat.real.astype(LD) * wh).astype(np.float64)
    if np.iscomplexobj(flat):
        x = x + 1j * lstsq_qr(V, R, flat.imag.astype(LD) * wh).astype(np.float64)
    return np.moveaxis(x.reshape((x.shape[0],) + sh[1:]), 0, axis)


def forward_normal_equations(basis, u):
    """u_hat = B^{-1} S(u) for a 1D u by dense LU on the assembled mass matrix
    (refined); the literal form of the projection, used as a cross-check."""
    N = len(u)
    S = (synthesis(basis, N).T * (PI_LD / N)) @ np.asarray(u, dtype=LD)
    return solve_refined(mass_matrix(basis, N), S)


def backward(basis, uh, axis=0):
    """u(x_j) = sum_l u_hat_l phi_l(x_j) along `axis` (N outputs)."""
    nb = np.shape(uh)[axis]
    N = {"dirichlet": nb + 2, "biharmonic": nb + 4, "chebyshev": nb, "neumann": nb + 2}[basis]
    return _apply_left(synthesis(basis, N), uh, axis)
