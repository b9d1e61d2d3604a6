"""Pins for oracle.fno: finite-difference gradients, identity at zero output weights,
the truncated DFT against numpy.fft, the whole forward map on a case with a known
answer (circular shift), the GELU against normal-distribution table values, and
bf16 rounding."""
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


@pytest.mark.parametrize("sy,sx", [(0, 0), (1, 2), (-2, 1)])
def test_forward_with_shift_mixing_is_a_circular_shift(sy, sx):
    # fno.forward itself, one spectral layer with every mode retained (H = 2K, odd
    # W = 2K - 1) and mixing R[ky, kx] = exp(-2 pi i (ky sy / H + kx sx / W)) M: the
    # spectral branch is then the input circularly shifted by (sy, sx) and mixed by
    # M, so z = roll(a) M + a Wp + bp exactly.  The head is made the identity on z:
    # gelu(t) = t for t >= 30 in binary64 (erf saturates), so W1 = I, b1 = 40,
    # W2 = I, b2 = -40 gives out = z.  A wrong DFT sign, inverse weight or
    # normalisation moves the shift or scales the result.
    H, W, K, C = 6, 5, 3, 2
    rng = np.random.default_rng(11)
    x = rng.standard_normal((2, H, W, 2))
    M = rng.standard_normal((C, C))
    ky = fno.ky_modes(H, K)
    kx = np.arange(K)
    ph = np.exp(-2j * np.pi * (np.outer(ky, np.ones(K)) * sy / H + np.outer(np.ones(2 * K), kx) * sx / W))
    R = ph[:, :, None, None] * M[None, None]
    p = {"Wl": rng.standard_normal((2, C)), "bl": rng.standard_normal(C),
         "Rr0": R.real.copy(), "Ri0": R.imag.copy(),
         "Wp0": rng.standard_normal((C, C)), "bp0": rng.standard_normal(C),
         "W1": np.eye(C), "b1": np.full(C, 40.0), "W2": np.eye(C), "b2": np.full(2, -40.0)}
    a = x @ p["Wl"] + p["bl"]
    z = np.roll(a, (sy, sx), axis=(1, 2)) @ M + a @ p["Wp0"] + p["bp0"]
    assert np.abs(z).max() < 10.0   # keeps z + 40 in the saturated range of erf
    got = fno.forward(p, x, K)
    assert np.abs(got - (x + z)).max() < 1e-12


def test_gelu_at_normal_table_values():
    # gelu(z) = z Phi(z); Phi(1) = 0.8413447460685429, Phi(2) = 0.9772498680518208,
    # Phi(-1) = 0.15865525393145707 (standard normal distribution tables)
    z = np.array([0.0, 1.0, 2.0, -1.0, 50.0, -50.0])
    ref = np.array([0.0, 0.8413447460685429, 2 * 0.9772498680518208, -0.15865525393145707, 50.0, 0.0])
    assert np.allclose(fno.gelu(z), ref, rtol=1e-15, atol=1e-300)


def test_reflections_form_the_square_symmetry_group():
    # the eight reflections of ENSEMBLES[8] are distinct, each is undone by its
    # unreflect, and the 2- and 4-member sets are closed under composition
    rng = np.random.default_rng(3)
    u = rng.standard_normal((1, 6, 6, 2))
    outs = [fno.reflect(u, *op) for op in fno.ENSEMBLES[8]]
    assert len({o.tobytes() for o in outs}) == 8
    for op in fno.ENSEMBLES[8]:
        assert np.array_equal(fno.unreflect(fno.reflect(u, *op), *op), u)
    for m in (2, 4):
        images = {fno.reflect(u, *op).tobytes() for op in fno.ENSEMBLES[m]}
        for a in fno.ENSEMBLES[m]:
            for b in fno.ENSEMBLES[m]:
                assert fno.reflect(fno.reflect(u, *a), *b).tobytes() in images


@pytest.mark.parametrize("members", [2, 4, 8])
def test_ensemble_is_equivariant_and_reduces_to_the_network(members):
    # E(x) = (1/m) sum_R R^-1 net(R x) over a group commutes with every R of the
    # group (a wrong inverse would break it); one member is the network itself
    p, x, _, _ = _small(seed=4)  # an 8 x 8 grid, square for the transposes
    assert np.array_equal(fno.forward_ensemble(p, x, 2, 1), fno.forward(p, x, 2))
    e = fno.forward_ensemble(p, x, 2, members)
    for op in fno.ENSEMBLES[members]:
        lhs = fno.forward_ensemble(p, fno.reflect(x, *op), 2, members)
        assert np.abs(lhs - fno.reflect(e, *op)).max() < 1e-12
    # the network alone is not equivariant, so the pin has teeth
    assert np.abs(fno.forward(p, fno.reflect(x, *fno.ENSEMBLES[members][1]), 2) -
                  fno.reflect(fno.forward(p, x, 2), *fno.ENSEMBLES[members][1])).max() > 1e-6
