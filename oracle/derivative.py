"""Spectral derivatives projected onto a space (oracle; test infrastructure only).

Sec. 5 (other functionality): Dx(u, axis, k) is the k-th partial derivative
along one axis (nested Dx calls give mixed derivatives), and
project(expr, space, uh_hat=u_hat) returns the coefficients, in `space`, of the
weighted L2 projection of expr, where expr is evaluated from the coefficients
u_hat of a Function.  For a tensor-product Function with coefficients u_hat in
W = V(x) x V^p(y) [x V^p(z)] this is, axis by axis:

  x (Chebyshev/Shen axis): the values of d^k u / dx^k at the Gauss-Chebyshev
      points, sum_l u_hat_l phi_l^(k)(x_j), followed by the target space's
      forward transform (its weighted least-squares projection, Sec. 3.4.2).
      A Legendre-family space does the same at its Legendre-Gauss points with
      the Legendre weight 1, onto a Legendre-family target.
      Gauss quadrature with N points is exact for the degree <= 2N - 2 products
      involved, so this equals the paper's route through the spectral matrix
      (phi_l^(k), psi_m)^N_w and the target mass matrix.  A regular Chebyshev
      target reproduces the derivative exactly; a Shen-Dirichlet target is the
      projection the paper recommends when the derivative vanishes at x = +-1.
  periodic axes: coefficient m times (i m 2 pi / L)^k (eq. ufourier
      differentiated term by term).

Reading where the paper is silent: for even M the Nyquist coefficient (m = -M/2
on a C2C axis, n = M/2 on an R2C axis) stands for cos(M y / 2) on the grid; its
odd derivatives are set to zero (the derivative sin(M y / 2) vanishes at every
grid point) and its even derivatives are multiplied by (-(M/2)^2)^(k/2).
"""
import numpy as np

from . import chebyshev as cheb
from . import fourier
from . import legendre as leg


def fourier_factor(M, n_coef, order, L=0.0):
    """(i k)^order for the n_coef stored coefficients of an axis of M points and
    period L (0 means 2 pi): FFT order for C2C (n_coef = M), k = 0..M/2 for R2C
    (n_coef = M/2 + 1); Nyquist rule as above."""
    L = 2 * np.pi if L == 0.0 else L
    q = np.arange(n_coef)
    k = q if n_coef < M else fourier.wavenumbers(M)
    f = (k * (2 * np.pi / L)) ** order * (1, 1j, -1, -1j)[order % 4]
    f = np.asarray(f, dtype=np.complex128)
    if M % 2 == 0 and order % 2 == 1:
        f[q == M // 2] = 0.0
    return f


def _axis_factors(order, spec_shape, M_last, kind_last, Ly, Lz):
    """Per periodic axis (1..): the factor array (or None for order 0)."""
    nd = len(spec_shape)
    out = []
    for ax in range(1, nd):
        o = order[ax] if ax < len(order) else 0
        if o == 0:
            out.append(None)
            continue
        last = ax == nd - 1
        n_coef = spec_shape[ax]
        M = M_last if last else n_coef
        L = (Lz if nd == 3 else Ly) if last else Ly
        out.append(fourier_factor(M, n_coef, o, L))
    return out


def _x_part(basis, target, cols, ox):
    """Target coefficients of d^ox/dx^ox along axis 0 of an N x k array of columns."""
    N = cols.shape[0]
    mod = leg if basis in leg.BASES else cheb
    if (target in leg.BASES) != (mod is leg):
        raise ValueError("source and target bases must be of one family (Chebyshev or Legendre)")
    nb = mod.nbasis(basis, N)
    D = mod.derivative_synthesis(basis, N, ox) if ox > 0 else mod.synthesis(basis, N)
    g = mod._apply_left(D, cols[:nb], 0)
    res = mod.forward(target, g, axis=0)
    out = np.zeros(cols.shape, dtype=np.complex128)
    out[: res.shape[0]] = res
    return out


def project_dx(basis, uh, order, target, M_last, kind_last="r2c", Ly=0.0, Lz=0.0):
    """Coefficients in the `target` basis ("chebyshev", "dirichlet" or "neumann";
    "legendre", "leg_dirichlet" or "leg_neumann" for a Legendre-family source) of the
    projection of d^(ox+oy[+oz]) u / dx^ox dy^oy [dz^oz], where u has the
    spectral coefficients uh ([N][M1] or [N][M1][M2c], rows >= nbasis zero) in
    `basis`.  order = (ox, oy) or (ox, oy, oz).  Returns an array shaped like uh
    with the target's rows beyond its basis size zero."""
    uh = np.asarray(uh, dtype=np.complex128)
    N = uh.shape[0]
    full = _x_part(basis, target, uh.reshape(N, -1), order[0]).reshape(uh.shape)
    for ax, f in enumerate(_axis_factors(order, uh.shape, M_last, kind_last, Ly, Lz), start=1):
        if f is not None:
            sh = [1] * uh.ndim
            sh[ax] = f.size
            full = full * f.reshape(sh)
    return full


def project_dx_columns(basis, uh_cols, order, target, col_index, spec_shape, M_last, kind_last="r2c",
                       Ly=0.0, Lz=0.0):
    """project_dx restricted to selected spectral columns: uh_cols is N x k (the
    columns of the flattened spectral dims 1.. at flat indices col_index).  The x
    operation acts per column and the Fourier factors are per column, so this is
    the full result at those columns."""
    out = _x_part(basis, target, np.asarray(uh_cols, dtype=np.complex128), order[0])
    idx = np.unravel_index(np.asarray(col_index), tuple(spec_shape[1:]))
    for ax, f in enumerate(_axis_factors(order, spec_shape, M_last, kind_last, Ly, Lz), start=1):
        if f is not None:
            out = out * f[idx[ax - 1]][None, :]
    return out
