"""Host-side logic of the surrogate weight files (no GPU)."""
import numpy as np
import torch

from paper_1708_03188_amd import surrogate as S


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    a = (rng.standard_normal(100000) * np.exp(rng.uniform(-20, 20, 100000))).astype(np.float32)
    a[:4] = [0.0, -0.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8]  # ties to even both ways
    bits = S._to_bf16_bits(a)
    ref = torch.from_numpy(a).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(bits, ref)


class _FakeFNO:
    H, W, C, K, nl, P = 8, 8, 4, 2, 2, 6

    def __init__(self):
        self.p = None

    def param_shapes(self):
        C, K, P = self.C, self.K, self.P
        sh = [("Wl", (2, C)), ("bl", (C,))]
        for l in range(self.nl):
            sh += [(f"Rr{l}", (2 * K, K, C, C)), (f"Ri{l}", (2 * K, K, C, C)), (f"Wp{l}", (C, C)), (f"bp{l}", (C,))]
        return sh + [("W1", (C, P)), ("b1", (P,)), ("W2", (P, 2)), ("b2", (2,))]

    def get_params(self):
        rng = np.random.default_rng(1)
        return {k: rng.standard_normal(s).astype(np.float32) for k, s in self.param_shapes()}

    def set_params(self, params):
        self.p = params


def test_weight_file_roundtrip(tmp_path):
    f = _FakeFNO()
    orig = f.get_params()
    path = tmp_path / "w.npz"
    S.export_weights(f, path)
    g = _FakeFNO()
    S.import_weights(g, path)
    for k, v in orig.items():
        got = g.p[k]
        assert got.dtype == np.float32 and got.shape == v.shape
        if S._is_fp32(k):
            assert np.array_equal(got, v)
        else:  # bf16-representable and within half an ulp of bf16
            assert np.array_equal(got, torch.from_numpy(v).to(torch.bfloat16).float().numpy())
