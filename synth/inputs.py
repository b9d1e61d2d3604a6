"""Seeded input generators (numpy only, float64 / complex128).

Every generator takes an explicit integer seed and uses numpy's PCG64
(``numpy.random.default_rng``), so a (function, arguments, seed) triple always
gives the same arrays.  Grids follow the paper's conventions: the
Gauss-Chebyshev points x_j = cos((2j+1)pi/(2N)) (descending) on the
non-periodic axis and y_k = 2 pi k / M on each periodic axis of period 2 pi.
"""
import numpy as np

__all__ = [
    "cheb_points", "periodic_points", "smooth_profile", "random_smooth_field",
    "poisson2d_manufactured", "biharmonic3d_manufactured", "gl_noise",
    "gl_ragged_sizes", "gl_gaussian_ic", "random_spectral",
]


def cheb_points(N):
    """Gauss-Chebyshev points x_j = cos((2j+1)pi/(2N)), j = 0..N-1."""
    j = np.arange(N)
    return np.cos((2 * j + 1) * np.pi / (2 * N))


def periodic_points(M, length=2 * np.pi, start=0.0):
    """Uniform periodic grid start + length*k/M, k = 0..M-1."""
    return start + length * np.arange(M) / M


def smooth_profile(x, rng, nterms=12, decay=3.0, amp=1.0):
    """A random smooth, generally non-polynomial function of x in [-1, 1].

    sum_q a_q cos(q*pi*(x+1)/2 + phi_q) with a_q ~ N(0,1)*(1+q)^-decay.
    It does not vanish at x = +-1, so it is not in any Shen space.
    """
    q = np.arange(nterms)
    a = rng.standard_normal(nterms) * (1.0 + q) ** (-decay) * amp
    phi = rng.uniform(0, 2 * np.pi, nterms)
    return (a[None, :] * np.cos(np.outer((x + 1) * np.pi / 2, q) + phi[None, :])).sum(axis=1)


def _periodic_profile(y, rng, nmodes, decay):
    m = np.arange(nmodes)
    a = rng.standard_normal(nmodes) * (1.0 + m) ** (-decay)
    phi = rng.uniform(0, 2 * np.pi, nmodes)
    return (a[None, :] * np.cos(np.outer(y, m) + phi[None, :])).sum(axis=1)


def random_smooth_field(shape, seed, rank=6, decay=3.0, modes=16, complex_last=False):
    """Smooth random field on the tensor grid (Chebyshev x) x (periodic ...).

    f = sum_{r<rank} X_r(x) Y_r(y) [Z_r(z)], each factor a random trig series
    with N(0,1)*(1+k)^-decay amplitudes over its lowest `modes` modes.  The
    field is real unless `complex_last` (then the last factor gets a random
    complex phase series and the field is complex128).
    """
    rng = np.random.default_rng(seed)
    N = shape[0]
    x = cheb_points(N)
    grids = [periodic_points(M) for M in shape[1:]]
    out = np.zeros(shape, dtype=np.complex128 if complex_last else np.float64)
    for _ in range(rank):
        fx = smooth_profile(x, rng, nterms=modes, decay=decay)
        facs = [_periodic_profile(g, rng, min(modes, max(1, len(g) // 2)), decay) for g in grids]
        if complex_last:
            g = grids[-1]
            facs[-1] = facs[-1] + 1j * _periodic_profile(g, rng, min(modes, max(1, len(g) // 2)), decay)
        term = fx
        for f in facs:
            term = np.multiply.outer(term, f)
        out += term
    return out


def poisson2d_manufactured(N, M, seed=1, nrand=4):
    """2D manufactured Poisson case on [-1,1] x [0,2pi).

    u = (1-x^2) sin(2y) cos(pi x/2) + u_r, u_r = sum_{l,m<nrand} a_lm (T_l - T_{l+2})(x) e^{imy} + c.c.
    with a_lm ~ N(0,1) max(1, sqrt(l^2+m^2))^-2 (real for m = 0).  Returns
    (x, y, u, f) with f = -lap(u) in closed form, all float64 on the N x M grid.
    """
    rng = np.random.default_rng(seed)
    x = cheb_points(N)
    y = periodic_points(M)
    X, Y = np.meshgrid(x, y, indexing="ij")
    h = np.pi / 2
    u = (1 - X**2) * np.sin(2 * Y) * np.cos(h * X)
    # d2/dx2 of (1-x^2)cos(hx) = -2cos(hx) + 4hx sin(hx) - h^2 (1-x^2) cos(hx)
    uxx = (-2 * np.cos(h * X) + 4 * h * X * np.sin(h * X) - h * h * (1 - X**2) * np.cos(h * X)) * np.sin(2 * Y)
    uyy = -4 * u
    theta = np.arccos(np.clip(X, -1, 1))
    for l in range(nrand):
        for m in range(nrand):
            amp = max(1.0, np.hypot(l, m)) ** -2
            a = rng.standard_normal() * amp
            if m > 0:
                a = a + 1j * rng.standard_normal() * amp
            # phi_l(x) = T_l - T_{l+2} = cos(l t) - cos((l+2) t), t = arccos x
            phi = np.cos(l * theta) - np.cos((l + 2) * theta)
            # second derivative of T_n(x) in closed form via sin t:
            # T_n''(x) = n (n cos(nt) sin t - sin(nt) cos t) / sin^3 t ... use polynomial form instead
            d2 = _cheb_d2(l, X) - _cheb_d2(l + 2, X)
            e = np.exp(1j * m * Y)
            if m == 0:
                u = u + a.real * phi
                uxx = uxx + a.real * d2
            else:
                u = u + 2 * np.real(a * e) * phi
                uxx = uxx + 2 * np.real(a * e) * d2
                uyy = uyy - m * m * 2 * np.real(a * e) * phi
    f = -(uxx + uyy)
    return x, y, u, f


def _cheb_d2(n, x):
    """Second derivative of the degree-n Chebyshev polynomial evaluated by numpy's
    polynomial module (used only to build manufactured right-hand sides)."""
    c = np.zeros(n + 1)
    c[n] = 1.0
    return np.polynomial.chebyshev.chebval(x, np.polynomial.chebyshev.chebder(c, 2))


def biharmonic3d_manufactured(N, M1, M2):
    """u = (1-x^2)^2 sin(y) cos(3z) and f = u'''' (x derivs) + ... = lap^2 u in closed form.

    lap^2 u = (d4x + 2 d2x (d2y + d2z) + (d2y+d2z)^2) u with d2y + d2z -> -(1 + 9) = -10.
    Returns (x, y, z, u, f) on the N x M1 x M2 tensor grid.
    """
    x = cheb_points(N)
    y = periodic_points(M1)
    z = periodic_points(M2)
    X, Y, Z = np.meshgrid(x, y, z, indexing="ij")
    p = (1 - X**2) ** 2          # x^4 - 2x^2 + 1
    p2 = 12 * X**2 - 4           # p''
    p4 = 24.0                    # p''''
    s = np.sin(Y) * np.cos(3 * Z)
    u = p * s
    f = (p4 - 20 * p2 + 100 * p) * s
    return x, y, z, u, f


def gl_ragged_sizes(count=64, sizes=(128, 192, 256, 384, 512)):
    """Grid sizes N_i = sizes[i mod len(sizes)] for a ragged batch of GL problems."""
    return [sizes[i % len(sizes)] for i in range(count)]


def gl_noise(N, seed, amp=0.01):
    """Complex uniform(-amp, amp) + i uniform(-amp, amp) noise on an N x N grid."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, (N, N)) + 1j * rng.uniform(-amp, amp, (N, N))


def gl_gaussian_ic(N, L=100.0, kind=1):
    """The Ginzburg-Landau initial conditions on [-L/2, L/2)^2 (Sec. 6):
    kind 0: (i x + y) exp(-0.03 (x^2+y^2));  kind 1: (x + y) exp(-0.03 (x^2+y^2))."""
    x = periodic_points(N, L, -L / 2)
    X, Y = np.meshgrid(x, x, indexing="ij")
    g = np.exp(-0.03 * (X**2 + Y**2))
    if kind == 0:
        return (1j * X + Y) * g
    return ((X + Y) * g).astype(np.complex128)


def random_spectral(shape, seed, decay=3.0, nrows=None):
    """Random complex spectral array: N(0,1) (re, im) * (1 + |k|)^-decay with
    |k| = sqrt(l^2 + m^2 + n^2) from the array indices (FFT-order indices are
    folded to |wavenumber|).  Rows l >= nrows are zero."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    k2 = np.zeros(shape)
    for ax, M in enumerate(shape):
        q = np.arange(M)
        if ax > 0:
            q = np.minimum(q, M - q)
        sh = [1] * len(shape)
        sh[ax] = M
        k2 = k2 + (q.astype(float) ** 2).reshape(sh)
    a = a * (1.0 + np.sqrt(k2)) ** (-decay)
    if nrows is not None:
        a[nrows:] = 0
    return a
