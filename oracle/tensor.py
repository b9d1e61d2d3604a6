"""Tensor-product spaces W = V(x) x V^p(y) [x V^p(z)] (oracle; test infrastructure only).

Sec. 4: the non-periodic direction is axis 0 (x) with a Chebyshev-family basis
(oracle.chebyshev) or a Legendre-family one (oracle.legendre, Sec. 3.1); the periodic
directions are Fourier with period 2 pi.  Physical arrays are indexed
[x][y] or [x][y][z]; spectral arrays [l][m] or [l][m][n] keep N rows along x
(rows l >= nb are zero) and FFT order along every periodic axis.  The last
periodic axis is R2C (M/2+1 coefficients, real physical data) or C2C.

Forward transform: the Fourier transforms first (last axis first), then the
Shen forward transform along x (eq. laplace and the right-hand side formula
after it, where the paper applies F along the periodic axis and then S along
x).  The scalar product f_tilde = S_x(F_y F_z f) drops the (2 pi)^(d-1)
factor that appears on both sides of every periodic-direction Galerkin
system.

Solves, one dense system per Fourier wavenumber pair (m, n) with
kappa^2 = m^2 + n^2 (Sec. 4, eq. laplace; Sec. 4 biharmonic problem):
  Helmholtz   alpha u - lap u = f :  (-A + (kappa^2 + alpha) B) u_hat = f_tilde
  Biharmonic  lap^2 u = f        :  (S - 2 kappa^2 A + kappa^4 B) u_hat = f_tilde
"""
import numpy as np

from . import chebyshev as _chebyshev
from . import fourier
from . import legendre as _legendre
from .linalg import solve_refined


def _xmod(basis):
    return _legendre if basis in _legendre.BASES else _chebyshev


cheb = _chebyshev


def spectral_shape(phys_shape, kind_last="r2c"):
    s = list(phys_shape)
    if kind_last == "r2c":
        s[-1] = s[-1] // 2 + 1
    return tuple(s)


def _fourier_forward(u, kind_last):
    nd = np.ndim(u)
    out = fourier.rforward(u, axis=nd - 1) if kind_last == "r2c" else fourier.forward(u, axis=nd - 1)
    for ax in range(nd - 2, 0, -1):
        out = fourier.forward(out, axis=ax)
    return out


def _fourier_backward(uh, M_last, kind_last):
    nd = np.ndim(uh)
    out = uh
    for ax in range(1, nd - 1):
        out = fourier.backward(out, axis=ax)
    if kind_last == "r2c":
        return fourier.rbackward(out, M_last, axis=nd - 1)
    return fourier.backward(out, axis=nd - 1)


def _pad_rows(a, N):
    out = np.zeros((N,) + a.shape[1:], dtype=np.complex128)
    out[: a.shape[0]] = a
    return out


def scalar_product(basis, f, kind_last="r2c"):
    """f_tilde[l, m, n] = S_l(F(f)) (nb nonzero rows, N rows stored)."""
    N = f.shape[0]
    return _pad_rows(_xmod(basis).scalar_product(basis, _fourier_forward(f, kind_last), axis=0), N)


def forward(basis, u, kind_last="r2c"):
    N = u.shape[0]
    return _pad_rows(_xmod(basis).forward(basis, _fourier_forward(u, kind_last), axis=0), N)


def backward(basis, uh, M_last, kind_last="r2c"):
    N = uh.shape[0]
    nb = _xmod(basis).nbasis(basis, N)
    return _fourier_backward(_xmod(basis).backward(basis, uh[:nb], axis=0), M_last, kind_last)


def kappa2(spec_shape, M_last, kind_last="r2c"):
    """kappa^2 = sum of squared integer wavenumbers over the periodic axes,
    broadcast to spec_shape[1:] (FFT order; R2C axis holds 0..M/2)."""
    k2 = np.zeros(spec_shape[1:])
    nd = len(spec_shape)
    for ax in range(1, nd):
        M = spec_shape[ax] if (ax < nd - 1 or kind_last == "c2c") else M_last
        k = fourier.wavenumbers(M)[: spec_shape[ax]]
        sh = [1] * (nd - 1)
        sh[ax - 1] = spec_shape[ax]
        k2 = k2 + (k.astype(np.float64) ** 2).reshape(sh)
    return k2


def _solve_columns(ftilde, k2, build, nb, cols):
    """Solve build(kappa^2) u = f_tilde for each selected spectral column."""
    N = ftilde.shape[0]
    flat = ftilde.reshape(N, -1)
    k2f = k2.reshape(-1)
    cols = np.arange(flat.shape[1]) if cols is None else np.asarray(cols)
    out = np.zeros((N, len(cols)), dtype=np.complex128)
    groups = {}
    for i, c in enumerate(cols):
        groups.setdefault(float(k2f[c]), []).append(i)
    for kk, idx in groups.items():
        M = build(kk)
        rhs = flat[:nb, cols[idx]]
        out[:nb, idx] = solve_refined(M, rhs)
    return out


def helmholtz_solve(basis, ftilde, alpha, M_last, kind_last="r2c", cols=None):
    """Solve (-A + (kappa^2+alpha) B) u_hat = f_tilde per wavenumber column
(Chebyshev-Dirichlet with the Chebyshev weight, Legendre-Dirichlet with weight 1).

    Returns the full spectral array, or an N x len(cols) array if `cols`
    (flat column indices into spectral dims 1..) is given."""
    N = ftilde.shape[0]
    nb = _xmod(basis).nbasis(basis, N)
    A = _xmod(basis).stiffness_matrix(basis, N)
    B = _xmod(basis).mass_matrix(basis, N)
    k2 = kappa2(ftilde.shape, M_last, kind_last)
    out = _solve_columns(ftilde, k2, lambda kk: -A + (np.longdouble(kk) + np.longdouble(alpha)) * B, nb, cols)
    return out.reshape(ftilde.shape) if cols is None else out


def biharmonic_solve(basis, ftilde, M_last, kind_last="r2c", cols=None):
    """Solve (S - 2 kappa^2 A + kappa^4 B) u_hat = f_tilde per wavenumber column."""
    N = ftilde.shape[0]
    nb = _xmod(basis).nbasis(basis, N)
    S = _xmod(basis).bilaplace_matrix(basis, N)
    A = _xmod(basis).stiffness_matrix(basis, N)
    B = _xmod(basis).mass_matrix(basis, N)
    k2 = kappa2(ftilde.shape, M_last, kind_last)
    LD = np.longdouble
    out = _solve_columns(ftilde, k2, lambda kk: S - 2 * LD(kk) * A + LD(kk) ** 2 * B, nb, cols)
    return out.reshape(ftilde.shape) if cols is None else out


def fourier_columns(u, cols, kind_last="r2c"):
    """Fourier coefficients F_y F_z u for selected spectral columns only.

    Returns an N x len(cols) complex array: for flat column c = (m, n) of the
    spectral dims 1.., (1/prod M) sum_{y,z} u[:, y, z] exp(-2 pi i (m y/M1 + n z/M2)).
    This is the same sum as the full transform restricted to those outputs."""
    N = u.shape[0]
    phys = u.shape[1:]
    spec = spectral_shape(u.shape, kind_last)[1:]
    idx = np.unravel_index(np.asarray(cols), spec)
    out = np.zeros((N, len(cols)), dtype=np.complex128)
    flat = u.reshape(N, -1)
    for i in range(len(cols)):
        phase = np.ones(phys, dtype=np.complex128)
        for ax, M in enumerate(phys):
            q = idx[ax][i]
            r = np.mod(q * np.arange(M), M).astype(np.longdouble)
            e = (np.cos(fourier.TWO_PI_LD * r / M) - 1j * np.sin(fourier.TWO_PI_LD * r / M)).astype(np.complex128) / M
            sh = [1] * len(phys)
            sh[ax] = M
            phase = phase * e.reshape(sh)
        out[:, i] = flat @ phase.reshape(-1)
    return out


def forward_columns(basis, u, cols, kind_last="r2c"):
    """forward() restricted to the selected spectral columns (N x len(cols))."""
    N = u.shape[0]
    return _pad_rows(_xmod(basis).forward(basis, fourier_columns(u, cols, kind_last), axis=0), N)


def scalar_product_columns(basis, f, cols, kind_last="r2c"):
    N = f.shape[0]
    return _pad_rows(_xmod(basis).scalar_product(basis, fourier_columns(f, cols, kind_last), axis=0), N)


def backward_rows(basis, uh, rows, M_last, kind_last="r2c"):
    """backward() restricted to the physical x-rows `rows` (3D spectral input):
    for each x_j, c_mn = sum_l u_hat[l, m, n] phi_l(x_j), then the Fourier
    backward transforms along y and z."""
    N = uh.shape[0]
    nb = _xmod(basis).nbasis(basis, N)
    Phi = _xmod(basis).synthesis(basis, N)
    flat = uh[:nb].reshape(nb, -1)
    re = flat.real.astype(np.longdouble)
    im = flat.imag.astype(np.longdouble)
    out = []
    for j in rows:
        cj = ((Phi[j] @ re).astype(np.float64) + 1j * (Phi[j] @ im).astype(np.float64)).reshape(uh.shape[1:])
        out.append(_fourier_backward(cj[None], M_last, kind_last)[0])
    return np.array(out)
