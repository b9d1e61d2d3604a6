"""Pins for oracle.tensor (Sec. 4 tensor-product spaces, Helmholtz and biharmonic solves)."""
import numpy as np
import pytest

import synth
from oracle import chebyshev as C
from oracle import tensor as T


def test_manufactured_poisson_2d_32x32():
    # -lap u = f on [-1,1] x [0, 2 pi) with u in the Dirichlet x Fourier space: exact up to rounding.
    x, y, u, f = synth.poisson2d_manufactured(32, 32, seed=1)
    uh = T.helmholtz_solve("dirichlet", T.scalar_product("dirichlet", f), 0.0, 32)
    assert np.abs(T.backward("dirichlet", uh, 32) - u).max() < 1e-13 * np.abs(u).max() * 10


def test_paper_poisson_2d_listing():
    # Sec. 4 listing: u = (cos 4y + sin 2x)(1 - x^2), f = lap u; solved with -lap u = -f.
    N, M = 32, 33
    x = C.points(N)
    y = 2 * np.pi * np.arange(M) / M
    X, Y = np.meshgrid(x, y, indexing="ij")
    u = (np.cos(4 * Y) + np.sin(2 * X)) * (1 - X**2)
    uxx = -2 * np.cos(4 * Y) + (-4 * np.sin(2 * X) * (1 - X**2) - 8 * X * np.cos(2 * X) - 2 * np.sin(2 * X))
    uyy = -16 * np.cos(4 * Y) * (1 - X**2)
    f = uxx + uyy
    uh = T.helmholtz_solve("dirichlet", T.scalar_product("dirichlet", -f), 0.0, M)
    assert np.abs(T.backward("dirichlet", uh, M) - u).max() < 1e-13


def test_helmholtz_alpha1_manufactured():
    N, M = 24, 16
    x = C.points(N)
    y = 2 * np.pi * np.arange(M) / M
    X, Y = np.meshgrid(x, y, indexing="ij")
    u = (1 - X**2) * np.exp(X) * np.cos(3 * Y)
    uxx = (-2 * np.exp(X) - 4 * X * np.exp(X) + (1 - X**2) * np.exp(X)) * np.cos(3 * Y)
    f = u - (uxx - 9 * u)
    uh = T.helmholtz_solve("dirichlet", T.scalar_product("dirichlet", f), 1.0, M)
    assert np.abs(T.backward("dirichlet", uh, M) - u).max() < 1e-13


def test_biharmonic_3d_manufactured_exact_coefficients():
    # u = (1-x^2)^2 sin y cos 3z = (3/8) phi_0(x) sin y cos 3z; f = lap^2 u in closed form.
    N, M1, M2 = 16, 8, 8
    _, _, _, u, f = synth.biharmonic3d_manufactured(N, M1, M2)
    ref = np.zeros((N, M1, M2 // 2 + 1), complex)
    ref[0, 1, 3] = 3 / 8 / 4j
    ref[0, M1 - 1, 3] = -3 / 8 / 4j
    assert np.allclose(T.forward("biharmonic", u), ref, atol=1e-15)
    uh = T.biharmonic_solve("biharmonic", T.scalar_product("biharmonic", f), M2)
    assert np.allclose(uh, ref, atol=1e-15)
    assert np.allclose(T.backward("biharmonic", uh, M2), u, atol=1e-14)


@pytest.mark.parametrize("kind", ["r2c", "c2c"])
def test_round_trip_3d_paper_sizes(kind):
    # The 3D space of Sec. 4 with N = (32, 33, 34): odd C2C axis, even last axis.
    rng = np.random.default_rng(7)
    shape = (32, 33, 34)
    u = rng.standard_normal(shape) if kind == "r2c" else rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    for basis in ("dirichlet", "biharmonic"):
        uh = T.forward(basis, u, kind)
        u2 = T.backward(basis, uh, 34, kind)
        assert np.allclose(T.forward(basis, u2, kind), uh, atol=1e-12)


def test_column_restricted_forms_match_full():
    rng = np.random.default_rng(3)
    shape = (12, 8, 10)
    f = synth.random_smooth_field(shape, seed=3)
    cols = rng.choice(8 * 6, 7, replace=False)
    full = T.forward("dirichlet", f).reshape(12, -1)[:, cols]
    assert np.allclose(T.forward_columns("dirichlet", f, cols), full, atol=1e-14)
    sp = T.scalar_product("biharmonic", f).reshape(12, -1)[:, cols]
    assert np.allclose(T.scalar_product_columns("biharmonic", f, cols), sp, atol=1e-14)
    ft = T.scalar_product("dirichlet", f)
    hs = T.helmholtz_solve("dirichlet", ft, 1.0, 10).reshape(12, -1)[:, cols]
    assert np.allclose(T.helmholtz_solve("dirichlet", ft, 1.0, 10, cols=cols), hs, atol=1e-15)


def test_backward_rows_matches_full():
    rng = np.random.default_rng(4)
    vh = synth.random_spectral((12, 8, 5), seed=4, nrows=10)
    full = T.backward("dirichlet", vh, 8)
    rows = [0, 5, 11]
    assert np.allclose(T.backward_rows("dirichlet", vh, rows, 8), full[rows], atol=1e-14)
