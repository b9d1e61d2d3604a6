"""Pins for oracle.derivative (Sec. 5, Dx and project): Chebyshev derivative values
against the Chebyshev differential equation, closed-form derivatives of
polynomials in the Shen spaces, spectral accuracy on the paper's 1D example,
nesting, and Fourier derivatives (with the Nyquist reading) on closed forms."""
import numpy as np
import pytest

from oracle import chebyshev as cheb
from oracle import derivative as D
from oracle import fourier, tensor


def _col(basis, vals):
    """One column of N spectral rows (Shen rows beyond the basis zero) from grid values."""
    N = len(vals)
    out = np.zeros((N, 1), complex)
    c = cheb.forward(basis, vals)
    out[: len(c), 0] = c
    return out


def _cheb_derivs_by_ode(N, kmax):
    """T_n^(k)(x_j) for n < N, k <= kmax from T_n = cos(n t), T_n' = n sin(n t) / sin t
    (x = cos t) and the differentiated Chebyshev equation
    (1 - x^2) y^(k+2) - (2k + 1) x y^(k+1) + (n^2 - k^2) y^(k) = 0."""
    LD = np.longdouble
    j = np.arange(N)
    t = (2 * j + 1) * np.arccos(LD(-1)) / (2 * N)
    x = np.cos(t)
    out = []
    for n in range(N):
        ys = [np.cos(n * t), n * np.sin(n * t) / np.sin(t)]
        for k in range(kmax - 1):
            ys.append(((2 * k + 1) * x * ys[k + 1] - (n * n - k * k) * ys[k]) / (1 - x * x))
        out.append(ys)
    return [np.array([out[n][k] for n in range(N)]).T for k in range(kmax + 1)]


@pytest.mark.parametrize("N", [9, 12])
def test_chebyshev_derivative_values_satisfy_the_ode(N):
    ode = _cheb_derivs_by_ode(N, 4)
    for k in range(1, 5):
        got = cheb.derivative_synthesis("chebyshev", N, k)
        ref = ode[k]
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), k


def test_closed_form_derivatives_of_shen_polynomials():
    N = 16
    x = cheb.points(N)
    # u = (1 - x^2) x^3 lies in the Dirichlet space:
    #   u'  = 3x^2 - 5x^4 = -3/8 T0 - T2 - 5/8 T4,   u'' = 6x - 20x^3 = -9 T1 - 5 T3
    uh = _col("dirichlet", (1 - x**2) * x**3)
    d1 = D.project_dx("dirichlet", uh, (1, 0), "chebyshev", 1, "c2c")[:, 0]
    d2 = D.project_dx("dirichlet", uh, (2, 0), "chebyshev", 1, "c2c")[:, 0]
    ref1 = np.zeros(N); ref1[[0, 2, 4]] = [-3 / 8, -1, -5 / 8]
    ref2 = np.zeros(N); ref2[[1, 3]] = [-9, -5]
    assert np.abs(d1 - ref1).max() < 1e-13 and np.abs(d2 - ref2).max() < 1e-13
    # u = (1 - x^2)^2 (the biharmonic space): u' = 4x^3 - 4x = -T1 + T3 vanishes at
    # x = +-1, so its Dirichlet projection reproduces it exactly
    bh = _col("biharmonic", (1 - x**2) ** 2)
    c1 = D.project_dx("biharmonic", bh, (1, 0), "chebyshev", 1, "c2c")[:, 0]
    ref = np.zeros(N); ref[[1, 3]] = [-1, 1]
    assert np.abs(c1 - ref).max() < 1e-13
    dd = D.project_dx("biharmonic", bh, (1, 0), "dirichlet", 1, "c2c")[:, 0]
    vals = cheb.backward("dirichlet", dd[: N - 2])
    assert np.abs(vals - (4 * x**3 - 4 * x)).max() < 1e-13


def test_paper_1d_example_derivative_is_spectrally_accurate():
    # Sec. 3.4.2 example u = sin(pi x)(1 - x^2), N = 32: the derivative of its
    # Dirichlet projection, projected onto the regular Chebyshev space, evaluated at
    # the Gauss points, against u' = pi cos(pi x)(1 - x^2) - 2x sin(pi x)
    N = 32
    x = cheb.points(N)
    uh = _col("dirichlet", np.sin(np.pi * x) * (1 - x**2))
    du = D.project_dx("dirichlet", uh, (1, 0), "chebyshev", 1, "c2c")[:, 0]
    vals = cheb.backward("chebyshev", du)
    exact = np.pi * np.cos(np.pi * x) * (1 - x**2) - 2 * x * np.sin(np.pi * x)
    assert np.abs(vals - exact).max() < 1e-12


@pytest.mark.parametrize("basis", ["dirichlet", "biharmonic", "chebyshev"])
def test_nested_first_derivatives_equal_second_derivative(basis):
    rng = np.random.default_rng(4)
    N = 14
    nb = cheb.nbasis(basis, N)
    uh = np.zeros((N, 3), complex)
    uh[:nb] = rng.standard_normal((nb, 3)) + 1j * rng.standard_normal((nb, 3))
    once = D.project_dx(basis, uh, (1, 0), "chebyshev", 3, "c2c")
    twice = D.project_dx("chebyshev", once, (1, 0), "chebyshev", 3, "c2c")
    direct = D.project_dx(basis, uh, (2, 0), "chebyshev", 3, "c2c")
    assert np.abs(twice - direct).max() < 1e-11 * np.abs(direct).max()


def test_fourier_derivatives_on_closed_forms_and_nyquist():
    M = 8
    y = 2 * np.pi * np.arange(M) / M
    u = np.sin(2 * y) + np.cos(3 * y)
    for kind, fwd, bwd in (("c2c", fourier.forward, fourier.backward),
                           ("r2c", fourier.rforward, lambda a: fourier.rbackward(a, M))):
        uh = fwd(u)
        d1 = bwd(uh * D.fourier_factor(M, uh.size, 1))
        d2 = bwd(uh * D.fourier_factor(M, uh.size, 2))
        assert np.abs(np.real(d1) - (2 * np.cos(2 * y) - 3 * np.sin(3 * y))).max() < 1e-13, kind
        assert np.abs(np.real(d2) - (-4 * np.sin(2 * y) - 9 * np.cos(3 * y))).max() < 1e-13, kind
        # the Nyquist mode cos(4y): odd derivatives vanish on the grid, even ones are -16 cos(4y)
        nq = fwd(np.cos(4 * y))
        assert np.abs(bwd(nq * D.fourier_factor(M, nq.size, 1))).max() < 1e-14, kind
        assert np.abs(np.real(bwd(nq * D.fourier_factor(M, nq.size, 2))) + 16 * np.cos(4 * y)).max() < 1e-12, kind
    # period L scales the wavenumbers by 2 pi / L
    assert np.allclose(D.fourier_factor(6, 6, 1, L=4.0), 1j * fourier.wavenumbers(6) * (2 * np.pi / 4.0) *
                       np.array([1, 1, 1, 0, 1, 1]))


def test_mixed_derivative_2d_closed_form():
    # u(x, y) = (1 - x^2) x^3 sin(2y): d2u/dxdy = (3x^2 - 5x^4) 2 cos(2y)
    N, M = 12, 10
    x = cheb.points(N)
    y = 2 * np.pi * np.arange(M) / M
    u = ((1 - x**2) * x**3)[:, None] * np.sin(2 * y)[None, :]
    uh = tensor.forward("dirichlet", u, "r2c")
    d = D.project_dx("dirichlet", uh, (1, 1), "chebyshev", M, "r2c")
    vals = tensor.backward("chebyshev", d, M, "r2c")
    exact = (3 * x**2 - 5 * x**4)[:, None] * 2 * np.cos(2 * y)[None, :]
    assert np.abs(vals - exact).max() < 1e-13


def test_columns_form_matches_full_form():
    rng = np.random.default_rng(7)
    N, M1, M2 = 10, 6, 8
    sh = (N, M1, M2 // 2 + 1)
    uh = rng.standard_normal(sh) + 1j * rng.standard_normal(sh)
    uh[N - 4:] = 0
    full = D.project_dx("biharmonic", uh, (2, 1, 3), "dirichlet", M2, "r2c", Ly=3.0, Lz=5.0)
    cols = np.array([0, 5, 7, 13, sh[1] * sh[2] - 1])
    part = D.project_dx_columns("biharmonic", uh.reshape(N, -1)[:, cols], (2, 1, 3), "dirichlet", cols, sh, M2,
                                "r2c", Ly=3.0, Lz=5.0)
    assert np.array_equal(part, full.reshape(N, -1)[:, cols])


# ---- Legendre family (same Dx / project, Legendre-Gauss points, weight 1) ----
from oracle import legendre as L  # noqa: E402


def _lcol(basis, vals):
    N = len(vals)
    out = np.zeros((N, 1), complex)
    c = L.forward(basis, vals)
    out[: len(c), 0] = c
    return out


def test_legendre_derivative_values_satisfy_the_ode():
    # L_n^(k) from L_n, L_n' = n (L_{n-1} - x L_n) / (1 - x^2) and the differentiated
    # Legendre equation (1 - x^2) y^(k+2) - 2(k+1) x y^(k+1) + (n(n+1) - k(k+1)) y^(k) = 0
    N = 11
    x = L.points(N).astype(np.longdouble)
    P = [np.ones_like(x), x]
    for n in range(1, N):
        P.append(((2 * n + 1) * x * P[n] - n * P[n - 1]) / (n + 1))
    for n in range(N):
        ys = [P[n], n * ((P[n - 1] if n > 0 else 0 * x) - x * P[n]) / (1 - x * x)]
        for k in range(3):
            ys.append((2 * (k + 1) * x * ys[k + 1] - (n * (n + 1) - k * (k + 1)) * ys[k]) / (1 - x * x))
        for k in range(1, 5):
            got = L.derivative_synthesis("legendre", N, k)[:, n]
            assert np.abs(got - ys[k]).max() <= 1e-12 * max(1.0, float(np.abs(ys[k]).max())), (n, k)


def test_legendre_closed_form_derivatives():
    N = 14
    x = L.points(N)
    # u = (1 - x^2) x^3 in the Dirichlet space: u' = 3x^2 - 5x^4 = -(6/7) L2 - (8/7) L4,
    # u'' = 6x - 20x^3 = -6 L1 - 8 L3
    uh = _lcol("leg_dirichlet", (1 - x**2) * x**3)
    d1 = D.project_dx("leg_dirichlet", uh, (1, 0), "legendre", 1, "c2c")[:, 0]
    d2 = D.project_dx("leg_dirichlet", uh, (2, 0), "legendre", 1, "c2c")[:, 0]
    ref1 = np.zeros(N); ref1[[2, 4]] = [-6 / 7, -8 / 7]
    ref2 = np.zeros(N); ref2[[1, 3]] = [-6, -8]
    assert np.abs(d1 - ref1).max() < 1e-13 and np.abs(d2 - ref2).max() < 1e-13
    # u = (1 - x^2)^2 (biharmonic space): u' = 4x^3 - 4x vanishes at +-1, so its
    # Dirichlet projection reproduces it exactly
    bh = _lcol("leg_biharmonic", (1 - x**2) ** 2)
    dd = D.project_dx("leg_biharmonic", bh, (1, 0), "leg_dirichlet", 1, "c2c")[:, 0]
    assert np.abs(L.backward("leg_dirichlet", dd[: N - 2]) - (4 * x**3 - 4 * x)).max() < 1e-13
    # u = x - 2x^3/3 + x^5/5 (regular space): u' = (1 - x^2)^2 has u''(+-1) = 0, so its
    # Neumann projection reproduces it exactly
    rg = _lcol("legendre", x - 2 * x**3 / 3 + x**5 / 5)
    dn = D.project_dx("legendre", rg, (1, 0), "leg_neumann", 1, "c2c")[:, 0]
    assert np.abs(L.backward("leg_neumann", dn[: N - 2]) - (1 - x**2) ** 2).max() < 1e-13


@pytest.mark.parametrize("target", ["leg_dirichlet", "leg_neumann"])
def test_legendre_projection_residual_is_orthogonal_to_the_target(target):
    # the L2 (weight 1) projection f -> Pf leaves f - Pf orthogonal to every basis
    # function of the target: sum_j w_j (f - Pf)(x_j) phi_m(x_j) = 0, and Pf satisfies
    # the target's boundary conditions
    rng = np.random.default_rng(11)
    N = 16
    uh = np.zeros((N, 2), complex)
    nb = L.nbasis("leg_biharmonic", N)
    uh[:nb] = rng.standard_normal((nb, 2)) + 1j * rng.standard_normal((nb, 2))
    f = L.backward("legendre", D.project_dx("leg_biharmonic", uh, (1, 0), "legendre", 2, "c2c"))
    Pf = D.project_dx("leg_biharmonic", uh, (1, 0), target, 2, "c2c")[: N - 2]
    r = f - L.backward(target, Pf)
    w = L.weights(N)
    G = L.synthesis(target, N).astype(np.float64)
    assert np.abs(G.T @ (w[:, None] * r)).max() < 1e-12 * np.abs(f).max()
    ends = np.array([1.0, -1.0])
    from numpy.polynomial import legendre as npl
    for c in range(2):
        coef = L.recombination(target, N).astype(np.float64) @ Pf[:, c]
        vals = npl.legval(ends, coef) if target == "leg_dirichlet" else npl.legval(ends, npl.legder(coef))
        assert np.abs(vals).max() < 1e-12 * np.abs(f).max()


def test_legendre_and_chebyshev_families_do_not_mix():
    uh = np.zeros((8, 1), complex)
    with pytest.raises(ValueError):
        D.project_dx("leg_dirichlet", uh, (1, 0), "chebyshev", 1, "c2c")
    with pytest.raises(ValueError):
        D.project_dx("dirichlet", uh, (1, 0), "leg_dirichlet", 1, "c2c")
