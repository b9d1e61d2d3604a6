"""Pins for oracle.gl (Sec. 6, complex Ginzburg-Landau with 3/2-rule dealiasing)."""
import numpy as np
import pytest

import synth
from oracle import gl


def _uniform_exact(u0, t, c):
    r0 = abs(u0)
    g = 1 + r0**2 * (np.exp(2 * t) - 1)
    return np.sqrt(r0**2 * np.exp(2 * t) / g) * np.exp(1j * (np.angle(u0) - c / 2 * np.log(g)))


@pytest.mark.parametrize("step", [gl.rk4_step, gl.ifrk4_step])
def test_uniform_solution_fourth_order(step):
    # Spatially uniform u: r' = r - r^3, theta' = -c r^2 (closed form); error ~ dt^4.
    N, L, b, c = 8, 100.0, 1.5, -2.0
    u0 = 0.3 * np.exp(0.7j)
    errs = []
    for dt, n in ((0.1, 20), (0.05, 40)):
        uh = np.zeros((N, N), complex)
        uh[0, 0] = u0
        for _ in range(n):
            uh = step(uh, dt, L, b, c)
        errs.append(abs(uh[0, 0] - _uniform_exact(u0, 2.0, c)))
        assert np.abs(uh).sum() - abs(uh[0, 0]) < 1e-14
    assert 12 < errs[0] / errs[1] < 20


@pytest.mark.parametrize("step", [gl.rk4_step, gl.ifrk4_step])
def test_plane_wave_exact_solution(step):
    # u = A exp(i k.x - i w t), |A|^2 = 1 - |k|^2, w = b|k|^2 + c(1 - |k|^2): a single mode,
    # so the padded product is alias-free and the scheme error is pure time error.
    N, L, b, c = 8, 2 * np.pi * 4, 1.5, -2.0
    mx, my = 1, 2
    k2 = (mx**2 + my**2) * (2 * np.pi / L) ** 2
    A = np.sqrt(1 - k2)
    w = b * k2 + c * (1 - k2)
    uh = np.zeros((N, N), complex)
    uh[mx, my] = A
    dt, n = 0.01, 50
    for _ in range(n):
        uh = step(uh, dt, L, b, c)
    assert abs(uh[mx, my] - A * np.exp(-1j * w * n * dt)) < 1e-9
    uh[mx, my] = 0
    assert np.abs(uh).max() < 1e-13


def test_linear_limit_ifrk4_exact_rk4_stability_polynomial():
    # Amplitude 1e-9: the cubic term is ~1e-27, so the flow is linear.  IF-RK4 is exact
    # for it; RK4 multiplies by R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 per step.
    N, L, b, c, dt = 8, 30.0, 1.5, -2.0, 0.05
    rng = np.random.default_rng(0)
    uh = 1e-9 * (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    Lh = gl.linear_symbol(N, L, b)
    v = uh.copy()
    w = uh.copy()
    for _ in range(10):
        v = gl.ifrk4_step(v, dt, L, b, c)
        w = gl.rk4_step(w, dt, L, b, c)
    assert np.allclose(v, np.exp(Lh * 10 * dt) * uh, rtol=1e-12, atol=1e-23)
    z = Lh * dt
    R = 1 + z + z**2 / 2 + z**3 / 6 + z**4 / 24
    assert np.allclose(w, R**10 * uh, rtol=1e-12, atol=1e-23)


def test_real_symmetric_ic_keeps_xy_symmetry():
    # Sec. 6: the real initial condition (x + y) exp(-0.03(x^2+y^2)) is symmetric under
    # x <-> y, and so is the equation; the dealiased solution keeps that symmetry.
    N, L = 32, 100.0
    u0 = synth.gl_gaussian_ic(N, L, kind=1)
    uh = gl.forward(u0)
    for _ in range(5):
        uh = gl.rk4_step(uh, 0.025, L, 0.0, 1.5)
    u = gl.backward(uh)
    assert np.linalg.norm(u - u.T) < 1e-12 * np.linalg.norm(u)


def test_rhs_of_paper_equation_matches_direct_pseudospectral_form():
    # rhs for b = 0: lap u + u - (1+1.5i)|u|^2 u with the product on the padded grid,
    # recomputed here with numpy.fft and explicit zero padding (independent route).
    N, L, c = 10, 100.0, 1.5
    rng = np.random.default_rng(2)
    uh = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) * 0.1
    from oracle.fourier import wavenumbers
    l = wavenumbers(N)
    Mp = 15
    pad = np.zeros((Mp, Mp), complex)
    pad[np.ix_(l % Mp, l % Mp)] = uh
    up = np.fft.ifft2(pad) * Mp * Mp
    wh = np.fft.fft2((1 + 1j * c) * np.abs(up) ** 2 * up)[np.ix_(l % Mp, l % Mp)] / Mp**2
    k = l * 2 * np.pi / L
    k2 = k[:, None] ** 2 + k[None, :] ** 2
    ref = -k2 * uh + uh - wh
    assert np.allclose(gl.rhs(uh, L, 0.0, c), ref, atol=1e-14)
