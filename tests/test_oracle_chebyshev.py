"""Pins for oracle.chebyshev (Sec. 3.3, 3.4.2 and the biharmonic basis of Sec. 4).

Every matrix is checked against a closed form derived independently of the
quadrature assembly, and every transform against an exactly known result.
"""
import os

import numpy as np
import pytest

from oracle import chebyshev as C

PI = np.pi
HERE = os.path.dirname(__file__)


def test_points_and_tk_direct_vs_recurrence_and_arccos():
    N = 9
    x = C.points(N)
    assert np.all(np.diff(x) < 0)                       # descending
    T = np.asarray(C.tmatrix(N), dtype=float)
    Tr = np.zeros((N, N))
    Tr[:, 0] = 1
    Tr[:, 1] = x
    for k in range(2, N):
        Tr[:, k] = 2 * x * Tr[:, k - 1] - Tr[:, k - 2]
    assert np.allclose(T, Tr, atol=1e-14)
    assert np.allclose(T, np.cos(np.outer(np.arccos(x), np.arange(N))), atol=1e-14)


@pytest.mark.parametrize("N", [4, 7, 16])
def test_gauss_chebyshev_discrete_orthogonality(N):
    # sum_j T_k(x_j) T_l(x_j) pi/N = c_k pi/2 delta_kl for k, l < N (c_0 = 2).
    T = np.asarray(C.tmatrix(N), dtype=float)
    G = T.T @ T * PI / N
    ck = np.where(np.arange(N) == 0, 2.0, 1.0)
    assert np.allclose(G, np.diag(ck * PI / 2), atol=1e-13)


def test_mass_matrix_dirichlet_closed_form_and_paper_printout():
    N = 8
    B = np.asarray(C.mass_matrix("dirichlet", N), dtype=float)
    nb = N - 2
    ref = np.zeros((nb, nb))
    for k in range(nb):
        ref[k, k] = PI / 2 * ((2 if k == 0 else 1) + 1)
        if k + 2 < nb:
            ref[k, k + 2] = ref[k + 2, k] = -PI / 2
    assert np.allclose(B, ref, atol=1e-14)
    # The legible entries of the printout in Sec. 3.3.
    with open(os.path.join(HERE, "golden", "paper_mass_dirichlet_N8.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            off, idx, val = line.split()
            off, val = int(off), float(val)
            diag = np.diagonal(B, off)
            if idx == "*":
                assert np.allclose(diag, val, atol=5e-9)
            else:
                ndig = len(val.__repr__().split(".")[1])
                assert abs(diag[int(idx)] - val) < 10.0 ** (-ndig) * 1.01


def test_stiffness_dirichlet_closed_form():
    # Shen (1994): A_kj = -2 pi (k+1)(k+2) for j = k; -4 pi (k+1) for j = k+2, k+4, ...; else 0.
    N = 14
    A = np.asarray(C.stiffness_matrix("dirichlet", N), dtype=float)
    nb = N - 2
    ref = np.zeros((nb, nb))
    for k in range(nb):
        ref[k, k] = -2 * PI * (k + 1) * (k + 2)
        for j in range(k + 2, nb, 2):
            ref[k, j] = -4 * PI * (k + 1)
    assert np.allclose(A, ref, atol=1e-10 * abs(ref).max())


def _tn2_tm(n, m):
    # (T_n'', T_m)_w = (pi/2) n (n^2 - m^2) for m <= n-2, n-m even.
    return PI / 2 * n * (n * n - m * m) if (m <= n - 2 and (n - m) % 2 == 0) else 0.0


def _tn4_tm(n, m):
    # (T_n'''', T_m)_w = (pi/2) sum_{p=m+2, step 2}^{n-2} n(n^2-p^2) p(p^2-m^2)
    if not (m <= n - 4 and (n - m) % 2 == 0):
        return 0.0
    return PI / 2 * sum(n * (n * n - p * p) * p * (p * p - m * m) for p in range(m + 2, n - 1, 2))


def _composite(entry, N, basis):
    P = np.asarray(C.recombination(basis, N), dtype=float)
    nb = P.shape[1]
    M = np.zeros((nb, nb))
    for k in range(nb):           # test function row
        for j in range(nb):       # trial function column
            M[k, j] = sum(P[a, j] * P[b, k] * entry(a, b) for a in range(N) if P[a, j] for b in range(N) if P[b, k])
    return M


def test_biharmonic_matrices_closed_forms():
    N = 16
    B = np.asarray(C.mass_matrix("biharmonic", N), dtype=float)
    A = np.asarray(C.stiffness_matrix("biharmonic", N), dtype=float)
    S = np.asarray(C.bilaplace_matrix("biharmonic", N), dtype=float)
    nb = N - 4
    k = np.arange(nb)
    beta = -2 * (k + 2) / (k + 3)
    gam = (k + 1) / (k + 3)
    ck = np.where(k == 0, 2.0, 1.0)
    Bref = np.zeros((nb, nb))
    for i in range(nb):
        Bref[i, i] = PI / 2 * (ck[i] + beta[i] ** 2 + gam[i] ** 2)
        if i + 2 < nb:
            Bref[i, i + 2] = Bref[i + 2, i] = PI / 2 * (beta[i] + gam[i] * beta[i + 2])
        if i + 4 < nb:
            Bref[i, i + 4] = Bref[i + 4, i] = PI / 2 * gam[i]
    assert np.allclose(B, Bref, atol=1e-13)
    assert np.allclose(A, _composite(_tn2_tm, N, "biharmonic"), atol=1e-10 * abs(A).max())
    offs = {j - i for i in range(nb) for j in range(nb) if abs(A[i, j]) > 1e-9}
    assert offs == {-2, 0, 2}
    assert np.allclose(S, _composite(_tn4_tm, N, "biharmonic"), atol=1e-11 * abs(S).max())
    assert np.allclose(np.diag(S), 8 * PI * (k + 1) ** 2 * (k + 2) * (k + 4), rtol=1e-12)
    assert np.allclose(np.tril(S, -1), 0, atol=1e-9)


def test_biharmonic_phi0_closed_form():
    N = 10
    x = C.points(N)
    Phi = np.asarray(C.synthesis("biharmonic", N), dtype=float)
    assert np.allclose(Phi[:, 0], 8.0 / 3.0 * (1 - x**2) ** 2, atol=1e-14)


@pytest.mark.parametrize("basis", C.BASES)
@pytest.mark.parametrize("N", [8, 13, 32])
def test_round_trip_and_basis_coefficients(basis, N):
    # forward(backward(u_hat)) = u_hat (Sec. 3.3); forward(phi_l) = e_l.
    rng = np.random.default_rng(N)
    nb = C.nbasis(basis, N)
    uh = rng.standard_normal(nb) + 1j * rng.standard_normal(nb)
    assert np.allclose(C.forward(basis, C.backward(basis, uh)), uh, atol=1e-13)
    Phi = np.asarray(C.synthesis(basis, N), dtype=float)
    l = nb // 2
    e = np.zeros(nb)
    e[l] = 1
    assert np.allclose(C.forward(basis, Phi[:, l]), e, atol=1e-13)


@pytest.mark.parametrize("basis", ["dirichlet", "biharmonic"])
def test_forward_is_weighted_least_squares(basis):
    # u_hat = B^{-1} S(u) minimises sum_j w_j |u_j - sum_l u_hat_l phi_l(x_j)|^2:
    # compare with a library least-squares solver on the weighted synthesis matrix.
    N = 20
    rng = np.random.default_rng(5)
    u = rng.standard_normal(N)
    Phi = np.asarray(C.synthesis(basis, N), dtype=float)
    ref = np.linalg.lstsq(Phi * np.sqrt(PI / N), u * np.sqrt(PI / N), rcond=None)[0]
    assert np.allclose(C.forward(basis, u), ref, atol=1e-11)


def test_poisson_1d_dirichlet_paper_example():
    # Sec. 3.4.2: u = sin(pi x)(1 - x^2) with f = u'' on N = 32 points; -A u_hat = -f_tilde.
    N = 32
    x = C.points(N)
    u = np.sin(PI * x) * (1 - x**2)
    f = -PI**2 * np.sin(PI * x) * (1 - x**2) - 4 * PI * x * np.cos(PI * x) - 2 * np.sin(PI * x)
    ft = C.scalar_product("dirichlet", f)
    A = np.asarray(C.stiffness_matrix("dirichlet", N), dtype=float)
    uh = np.linalg.solve(A, ft)
    assert np.abs(C.backward("dirichlet", uh) - u).max() < 1e-13


def test_spectral_convergence_dirichlet_poisson():
    # Error of the 1D Dirichlet Poisson solve must fall faster than any power of N.
    errs = []
    for N in (6, 8, 12, 16, 20):
        x = C.points(N)
        u = np.sin(PI * x) * (1 - x**2)
        f = -PI**2 * np.sin(PI * x) * (1 - x**2) - 4 * PI * x * np.cos(PI * x) - 2 * np.sin(PI * x)
        A = np.asarray(C.stiffness_matrix("dirichlet", N), dtype=float)
        uh = np.linalg.solve(A, C.scalar_product("dirichlet", f))
        errs.append(np.abs(C.backward("dirichlet", uh) - u).max())
    assert errs[0] > 1e-3 and errs[-1] < 1e-13
    assert all(errs[i + 1] < errs[i] * 0.2 for i in range(3))


@pytest.mark.parametrize("basis", C.BASES)
def test_least_squares_form_equals_normal_equations(basis):
    # The projection u_hat = B^{-1} S(u) (Sec. 3.4.2) solved as the dense LU of the
    # assembled normal equations and as the weighted least-squares problem agree where
    # B is well conditioned.
    N = 24
    x = C.points(N)
    u = np.exp(x) * np.sin(3 * x + 0.2) + x**2
    assert np.allclose(C.forward(basis, u), C.forward_normal_equations(basis, u), rtol=0, atol=1e-13)


def test_projection_accuracy_against_high_precision():
    # Biharmonic N = 96 (cond(B) ~ 3e5): the oracle's projection agrees with a
    # 40-digit mpmath solve of B u_hat = S (exact quadrature, banded Gaussian elimination).
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    N = 96
    x = C.points(N)
    g = np.exp(x) * np.cos(3 * x) + 0.1 * x
    tab = [mpmath.cos(mpmath.pi * r / (2 * N)) for r in range(4 * N)]
    gv = [mpmath.mpf(float(v)) for v in g]
    chat = []
    for k in range(N):
        s = mpmath.mpf(0)
        for j in range(N):
            s += gv[j] * tab[(k * (2 * j + 1)) % (4 * N)]
        chat.append(s * 2 / ((2 if k == 0 else 1) * N))

    def comp(k):
        return [(k, mpmath.mpf(1)), (k + 2, mpmath.mpf(-2 * (k + 2)) / (k + 3)), (k + 4, mpmath.mpf(k + 1) / (k + 3))]

    def D(k):
        return mpmath.pi if k == 0 else mpmath.pi / 2

    nb = N - 4
    B = mpmath.matrix(nb, nb)
    for a in range(nb):
        for b in range(max(0, a - 4), min(nb, a + 5)):
            B[a, b] = sum(p1 * p2 * D(m1) for m1, p1 in comp(a) for m2, p2 in comp(b) if m1 == m2)
    S = mpmath.matrix([sum(p * D(m) * chat[m] for m, p in comp(k)) for k in range(nb)])
    ref = np.array([float(v) for v in mpmath.lu_solve(B, S)])
    got = C.forward("biharmonic", g)
    assert np.abs(got - ref).max() < 1e-15 * np.abs(ref).max() * 10


def test_neumann_basis_boundary_conditions_and_mass_matrix():
    # phi_l = T_l - (l/(l+2))^2 T_{l+2}: T_k'(1) = k^2 and T_k'(-1) = (-1)^(k+1) k^2,
    # so phi_l'(+-1) = 0 exactly; mass matrix (pi/2)(c_l + beta_l^2) on the diagonal
    # and (pi/2) beta_l two places off it
    N = 14
    P = C.recombination("neumann", N)
    k = np.arange(N, dtype=np.longdouble)
    assert np.all(np.abs((k**2) @ P) < 1e-15)
    assert np.all(np.abs(((-1) ** (k + 1) * k**2) @ P) < 1e-15)
    B = np.asarray(C.mass_matrix("neumann", N), dtype=float)
    nb = N - 2
    beta = np.array([-(l / (l + 2)) ** 2 for l in range(nb)])
    ref = np.diag(PI / 2 * (np.where(np.arange(nb) == 0, 2.0, 1.0) + beta**2))
    ref += np.diag(PI / 2 * beta[: nb - 2], 2) + np.diag(PI / 2 * beta[: nb - 2], -2)
    assert np.abs(B - ref).max() < 1e-13


def test_neumann_projection_of_a_neumann_polynomial_is_exact():
    # u = x^2 - x^4/2 has u'(+-1) = 0 and u = 5/16 T0 + 1/4 T2 - 1/16 T4
    #   = 5/16 phi_0 + 1/4 phi_2 (phi_2 = T2 - T4/4)
    N = 12
    x = C.points(N)
    uh = C.forward("neumann", x**2 - x**4 / 2)
    ref = np.zeros(N - 2)
    ref[0], ref[2] = 5 / 16, 1 / 4
    assert np.abs(uh - ref).max() < 1e-15


def test_neumann_stiffness_closed_form():
    # A_kj = (phi_j'', phi_k)_w with phi_l = T_l - r_l T_{l+2}, r_l = (l/(l+2))^2, from
    # (T_m'', T_n)_w = (pi/2) m (m^2 - n^2) for n <= m - 2 of the parity of m (zero
    # otherwise): A_kk = -2 pi k^2 (k+1)/(k+2); for j >= k+2 the four terms collapse
    # (k^2 - r_k (k+2)^2 = 0) to A_kj = -pi (1 - r_k) j^2
    N = 22
    nb = N - 2
    A = np.asarray(C.stiffness_matrix("neumann", N), dtype=float)
    r = lambda l: (l / (l + 2.0)) ** 2
    ref = np.zeros((nb, nb))
    for k in range(nb):
        ref[k, k] = -2 * PI * k * k * (k + 1) / (k + 2)
        for j in range(k + 2, nb, 2):
            ref[k, j] = -PI * (1 - r(k)) * j * j
    assert np.abs(A - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("alpha", [0.5, 3.0])
def test_neumann_helmholtz_2d_manufactured(alpha):
    # alpha u - lap u = f on [-1, 1] x [0, 2 pi) with u = cos(pi x) sin(2y), which has
    # u'(+-1) = 0: the Galerkin solution in the Neumann space converges spectrally
    # (cos(pi x) is entire), so at N = 40 it reproduces u to rounding
    from oracle import tensor as T
    N, M = 40, 16
    x = C.points(N)
    y = 2 * PI * np.arange(M) / M
    u = np.cos(PI * x)[:, None] * np.sin(2 * y)[None, :]
    f = (alpha + PI**2 + 4) * u
    uh = T.helmholtz_solve("neumann", T.scalar_product("neumann", f), alpha, M)
    assert np.abs(T.backward("neumann", uh, M) - u).max() < 1e-12
