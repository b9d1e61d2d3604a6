"""Pins for oracle.fno: finite-difference gradients, identity at zero output weights,
the truncated DFT against numpy.fft, and bf16 rounding."""
import numpy as np
import pytest

from oracle import fno


def _small(seed=0, B=2, H=8, W=8, C=3, K=2, P=4, nl=2):
    p = fno.init_params(C, K, P, nl, seed, scale_spec=0.5)
    rng = np.random.default_rng(seed + 1)
    for k in list(p):
        if k.startswith("b"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((B, H, W, 2))
    t = x + 0.3 * rng.standard_normal((B, H, W, 2))
    return p, x, t, K


def test_gradients_match_central_differences():
    p, x, t, K = _small()
    pred, cache = fno.forward(p, x, K, keep=True)
    g = fno.backward(p, x, K, cache, fno.loss_grad(pred, t))
    rng = np.random.default_rng(3)
    h = 1e-6
    for name in p:
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, min(4, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = fno.loss(fno.forward(p, x, K), t)
            flat[idx] = old - h
            lm = fno.loss(fno.forward(p, x, K), t)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (name, idx, fd, an)


def test_zero_output_layer_is_identity():
    p, x, t, K = _small()
    p["W2"][:] = 0
    p["b2"][:] = 0
    assert np.array_equal(fno.forward(p, x, K), x)


def test_truncated_dft_matches_numpy_fft():
    rng = np.random.default_rng(5)
    H, W, K = 16, 12, 3
    a = rng.standard_normal((H, W))
    Ey, Ex = fno.dft_mats(H, W, K)
    X = Ey @ a @ Ex.T / (H * W)
    ref = np.fft.rfft2(a) / (H * W)
    assert np.allclose(X, ref[fno.ky_modes(H, K)][:, :K], atol=1e-15)


def test_spectral_layer_with_all_modes_is_a_projection():
    # With every mode retained and R = identity, s reproduces the (real) input exactly
    # when the retained set covers the full spectrum (odd W, K = (W+1)/2, H = 2K).
    H, W, K, C = 6, 5, 3, 1
    rng = np.random.default_rng(1)
    a = rng.standard_normal((1, H, W, C))
    Ey, Ex = fno.dft_mats(H, W, K)
    wk = np.where(np.arange(K) == 0, 1.0, 2.0)
    X = np.einsum("byxc,jy,kx->bjkc", a, Ey, Ex) / (H * W)
    s = np.einsum("bjkc,jy,kx,k->byxc", X, np.conj(Ey), np.conj(Ex), wk).real
    assert np.allclose(s, a, atol=1e-14)


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.14159, 0.0])
    r = fno.round_bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7
    assert abs(r[3] - (-3.140625)) < 1e-12 and r[4] == 0.0
