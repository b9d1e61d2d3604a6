"""Pins for oracle.legendre (Sec. 3.1 Legendre bases, Sec. 3.4.2 Legendre-Gauss
quadrature): points and weights against numpy's Gauss-Legendre rule and the
paper's weight formula, exact quadrature (discrete orthogonality), boundary
conditions of every Shen basis, closed-form Dirichlet mass and stiffness
matrices, round trips, the least-squares form against a library solver, and
the paper's 1D Poisson example with the Legendre basis."""
import numpy as np
import pytest

from oracle import legendre as L

PI = np.pi


@pytest.mark.parametrize("N", [5, 16, 33, 64])
def test_points_and_weights(N):
    x, w = L.nodes_weights(N)
    xr, wr = np.polynomial.legendre.leggauss(N)
    # descending order; same rule as numpy's
    assert np.all(np.diff(x.astype(float)) < 0)
    assert np.abs(x.astype(float)[::-1] - xr).max() < 1e-15
    assert np.abs(w.astype(float)[::-1] - wr).max() < 1e-14
    # the paper's formula w_j = 2 / ((1 - x_j^2) L_N'(x_j)^2) with L_N' from
    # numpy's Legendre-series derivative
    c = np.zeros(N + 1)
    c[N] = 1
    dLN = np.polynomial.legendre.legval(xr, np.polynomial.legendre.legder(c))
    assert np.abs(2 / ((1 - xr**2) * dLN**2) - wr).max() < 1e-13


@pytest.mark.parametrize("N", [8, 21])
def test_discrete_orthogonality(N):
    # Gauss quadrature is exact to degree 2N - 1: sum_j w_j L_k L_m = 2/(2k+1) delta_km
    Lm = L.lmatrix(N)
    w = L.nodes_weights(N)[1]
    G = Lm.T @ (Lm * w[:, None])
    ref = np.diag([2.0 / (2 * k + 1) for k in range(N)])
    assert np.abs(np.asarray(G, dtype=float) - ref).max() < 1e-15
    # against numpy's legvander
    x = L.points(N)
    assert np.abs(np.asarray(Lm, dtype=float) - np.polynomial.legendre.legvander(x, N - 1)).max() < 1e-13


def test_boundary_conditions_of_the_shen_bases():
    # L_k(1) = 1, L_k(-1) = (-1)^k, L_k'(1) = k(k+1)/2, L_k'(-1) = (-1)^(k+1) k(k+1)/2
    N = 20
    k = np.arange(N, dtype=np.longdouble)
    val_p, val_m = np.ones(N, dtype=np.longdouble), (-1) ** k
    der_p, der_m = k * (k + 1) / 2, (-1) ** (k + 1) * k * (k + 1) / 2
    for basis, conds in (("leg_dirichlet", (val_p, val_m)), ("leg_neumann", (der_p, der_m)),
                         ("leg_biharmonic", (val_p, val_m, der_p, der_m))):
        P = L.recombination(basis, N)
        for c in conds:
            assert np.abs(c @ P).max() < 1e-15, basis


def test_dirichlet_mass_and_stiffness_closed_forms():
    # (phi_k, phi_k) = 2/(2k+1) + 2/(2k+5), (phi_k, phi_{k+2}) = -2/(2k+5);
    # (phi_l', phi_m') = (4l + 6) delta_lm (Legendre weight 1, by parts)
    N = 18
    nb = N - 2
    B = np.asarray(L.mass_matrix("leg_dirichlet", N), dtype=float)
    k = np.arange(nb)
    ref = np.diag(2 / (2 * k + 1) + 2 / (2 * k + 5))
    off = -2 / (2 * k[: nb - 2] + 5)
    ref += np.diag(off, 2) + np.diag(off, -2)
    assert np.abs(B - ref).max() < 1e-15
    # derivative values from numpy's Legendre derivative, quadrature with the oracle's rule
    x, w = L.points(N), L.weights(N)
    P = np.asarray(L.recombination("leg_dirichlet", N), dtype=float)
    D = np.stack([np.polynomial.legendre.legval(x, np.polynomial.legendre.legder(P[:, l])) for l in range(nb)], 1)
    A = D.T @ (D * w[:, None])
    assert np.abs(A - np.diag(4 * k + 6.0)).max() < 1e-11


@pytest.mark.parametrize("basis", L.BASES)
@pytest.mark.parametrize("N", [8, 13, 40])
def test_round_trip_and_least_squares(basis, N):
    rng = np.random.default_rng(N)
    nb = L.nbasis(basis, N)
    uh = rng.standard_normal(nb) + 1j * rng.standard_normal(nb)
    assert np.allclose(L.forward(basis, L.backward(basis, uh)), uh, atol=1e-13)
    u = rng.standard_normal(N)
    Phi = np.asarray(L.synthesis(basis, N), dtype=float)
    sw = np.sqrt(L.weights(N))
    ref = np.linalg.lstsq(Phi * sw[:, None], u * sw, rcond=None)[0]
    assert np.allclose(L.forward(basis, u), ref, atol=1e-11)
    # the scalar product is Phi^T W u
    assert np.allclose(L.scalar_product(basis, u), Phi.T @ (L.weights(N) * u), atol=1e-13)


def test_poisson_1d_legendre_dirichlet_paper_example():
    # Sec. 3.4.2 example with the Legendre basis: u = sin(pi x)(1 - x^2), -u'' = f;
    # (phi_l', phi_m') u_hat = (f, phi_m) with the diagonal stiffness 4l + 6
    N = 32
    x = L.points(N)
    u = np.sin(PI * x) * (1 - x**2)
    f = PI**2 * np.sin(PI * x) * (1 - x**2) + 4 * PI * x * np.cos(PI * x) + 2 * np.sin(PI * x)
    ft = L.scalar_product("leg_dirichlet", f)
    uh = ft / (4 * np.arange(N - 2) + 6.0)
    assert np.abs(L.backward("leg_dirichlet", uh) - u).max() < 1e-13


@pytest.mark.parametrize("N", [6, 17, 64])
def test_stiffness_matrix_is_minus_the_diagonal_closed_form(N):
    # A_ml = (phi_l'', phi_m) = -(phi_l', phi_m') = -(4l + 6) delta_lm: by parts (phi_m
    # vanishes at +-1) and phi_l' = -(2l + 3) L_{l+1}, (L_k, L_k) = 2 / (2k + 1)
    A = np.asarray(L.stiffness_matrix("leg_dirichlet", N), dtype=float)
    assert np.abs(A + np.diag(4 * np.arange(N - 2) + 6.0)).max() < 1e-12


@pytest.mark.parametrize("alpha", [0.0, 1.5])
def test_helmholtz_2d_legendre_manufactured_exact_coefficients(alpha):
    # u = (1 - x^2)(x^3 + 2x - 0.5) cos(2y) lies in the Legendre-Dirichlet x Fourier
    # space, so the Galerkin solution of -lap u + alpha u = f is u itself:
    # the solve must return the projection of u (its exact coefficients)
    from oracle import tensor as T
    N, M = 12, 8
    x = L.points(N)
    y = 2 * PI * np.arange(M) / M
    p = (1 - x**2) * (x**3 + 2 * x - 0.5)
    # p'' = d2/dx2 of -x^5 - x^3 + 0.5 x^2 + 2x - 0.5
    p2 = -20 * x**3 - 6 * x + 1.0
    u = p[:, None] * np.cos(2 * y)[None, :]
    f = (-p2 + (4 + alpha) * p)[:, None] * np.cos(2 * y)[None, :]
    ft = T.scalar_product("leg_dirichlet", f)
    uh = T.helmholtz_solve("leg_dirichlet", ft, alpha, M)
    assert np.abs(uh - T.forward("leg_dirichlet", u)).max() < 1e-13
    assert np.abs(T.backward("leg_dirichlet", uh, M) - u).max() < 1e-13


def test_neumann_galerkin_closed_forms():
    # phi_k = L_k - s_k L_{k+2}, s_k = k(k+1)/((k+2)(k+3)): phi_k'(+-1) = 0, so by parts
    # A_mk = -(phi_k', phi_m'); with L_{n+1}' - L_{n-1}' = (2n+1) L_n this is diagonal,
    # -A_kk = (4k+6) s_k; B_kk = 2/(2k+1) + s_k^2 2/(2k+5), B_{k,k+2} = -s_k 2/(2k+5)
    N = 20
    nb = N - 2
    k = np.arange(nb, dtype=float)
    s = k * (k + 1) / ((k + 2) * (k + 3))
    A = np.asarray(L.stiffness_matrix("leg_neumann", N), dtype=float)
    B = np.asarray(L.mass_matrix("leg_neumann", N), dtype=float)
    assert np.abs(A + np.diag((4 * k + 6) * s)).max() < 1e-12
    Bref = np.diag(2 / (2 * k + 1) + s**2 * 2 / (2 * k + 5))
    off = -s[: nb - 2] * 2 / (2 * k[: nb - 2] + 5)
    Bref += np.diag(off, 2) + np.diag(off, -2)
    assert np.abs(B - Bref).max() < 1e-15


def test_biharmonic_galerkin_matrices():
    # S = (phi_l'''', phi_m) is diagonal, 2 (2k+3)^2 (2k+5) (by parts twice: (phi_l'', phi_m'')
    # with phi_k'' proportional to L_{k+2}); A and B against numpy's own Gauss-Legendre rule
    # and Legendre-series derivative (an independent implementation)
    from numpy.polynomial import legendre as npl
    N = 18
    nb = N - 4
    k = np.arange(nb, dtype=float)
    S = np.asarray(L.bilaplace_matrix("leg_biharmonic", N), dtype=float)
    assert np.abs(S - np.diag(2 * (2 * k + 3) ** 2 * (2 * k + 5))).max() < 1e-12 * S.max()
    P = np.asarray(L.recombination("leg_biharmonic", N), dtype=float)
    x, w = npl.leggauss(N + 2)
    Phi = np.stack([npl.legval(x, P[:, l]) for l in range(nb)], 1)
    D2 = np.stack([npl.legval(x, npl.legder(P[:, l], 2)) for l in range(nb)], 1)
    A = np.asarray(L.stiffness_matrix("leg_biharmonic", N), dtype=float)
    B = np.asarray(L.mass_matrix("leg_biharmonic", N), dtype=float)
    assert np.abs(A - Phi.T @ (D2 * w[:, None])).max() < 1e-12 * np.abs(A).max()
    assert np.abs(B - Phi.T @ (Phi * w[:, None])).max() < 1e-14


def test_neumann_and_biharmonic_2d_manufactured():
    from oracle import tensor as T
    N, M = 40, 16
    x = L.points(N)
    y = 2 * PI * np.arange(M) / M
    # Neumann: alpha u - lap u = f, u = cos(pi x) sin(2y) (u'(+-1) = 0): spectral accuracy
    alpha = 0.5
    u = np.cos(PI * x)[:, None] * np.sin(2 * y)[None, :]
    uh = T.helmholtz_solve("leg_neumann", T.scalar_product("leg_neumann", (alpha + PI**2 + 4) * u), alpha, M)
    assert np.abs(T.backward("leg_neumann", uh, M) - u).max() < 1e-12
    # biharmonic: lap^2 u = f, u = (1 - x^2)^2 sin(y) lies in the space: exact coefficients
    g = (1 - x**2) ** 2
    g2 = 12 * x**2 - 4
    u = g[:, None] * np.sin(y)[None, :]
    f = (24 - 2 * g2 + g)[:, None] * np.sin(y)[None, :]
    uh = T.biharmonic_solve("leg_biharmonic", T.scalar_product("leg_biharmonic", f), M)
    assert np.abs(uh - T.forward("leg_biharmonic", u)).max() < 1e-13
    assert np.abs(T.backward("leg_biharmonic", uh, M) - u).max() < 1e-13
