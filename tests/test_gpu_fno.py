"""GPU FNO surrogate kernels against the FP64 oracle (bf16 weights/inputs on both sides)."""
import os
import tempfile

import numpy as np
import pytest

from oracle import fno as ofno

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def FNO():
    from paper_1708_03188_amd.api import FNO
    return FNO


CFG = dict(H=32, W=32, width=8, modes=4, layers=2, hidden=16)
# width 32 with 16 x-modes runs the fused row kernels (lift + x-DFT, layer, projection);
# H != W to catch axis mix-ups, three layers so the middle-layer variant runs twice
CFG32 = dict(H=32, W=64, width=32, modes=16, layers=3, hidden=64)
# fused kernels at ragged sizes: H * B = 34 rows (the last work-group has two waves past
# the end), W = 288 (the lift stages its input in a 256-pixel and a 32-pixel chunk)
CFG32R = dict(H=34, W=288, width=32, modes=16, layers=2, hidden=32)
# the surrogate's full shape: 256 x 256, width 32, 16 modes, 4 layers, hidden 128
CFG_C5 = dict(H=256, W=256, width=32, modes=16, layers=4, hidden=128)
# gradient cases large enough for the split-K weight-gradient products (one split
# per 1024 pixels, partial products accumulated atomically): 12 splits for the
# general-GEMM network (3 x 64 x 64 pixels), 16 for the fused one (4 x 64 x 64)
CFG_SK = dict(H=64, W=64, width=8, modes=4, layers=2, hidden=16)
CFG32_SK = dict(H=64, W=64, width=32, modes=16, layers=2, hidden=64)
# fused row kernels with the hidden widths of the fused projection backward (32, 128)
# and one it does not take (96: the projection runs as separate products)
CFG32_P128 = dict(H=32, W=64, width=32, modes=16, layers=2, hidden=128)
CFG32_P96 = dict(H=32, W=32, width=32, modes=16, layers=2, hidden=96)


def _setup(FNO, B=3, seed=0, cfg=CFG):
    f = FNO(cfg["H"], cfg["W"], cfg["width"], cfg["modes"], cfg["layers"], cfg["hidden"], max_batch=max(B, 4), seed=seed)
    p = ofno.init_params(cfg["width"], cfg["modes"], cfg["hidden"], cfg["layers"], seed, scale_spec=0.3)
    rng = np.random.default_rng(seed + 7)
    for k in p:
        if k.startswith("b"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    p = {k: ofno.round_bf16(v) for k, v in p.items()}
    f.set_params(p)
    x = ofno.round_bf16(rng.standard_normal((B, cfg["H"], cfg["W"], 2)) * 0.5)
    t = x + 0.2 * rng.standard_normal(x.shape)
    return f, p, x, t


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("cfg,B", [(CFG, 3), (CFG32, 3), (CFG32R, 1), (CFG_C5, 1)],
                         ids=["gemm", "fused", "fused-ragged", "surrogate-256"])
def test_forward_matches_oracle(FNO, cfg, B):
    print(f"[case] fno forward {cfg} B={B}", flush=True)
    f, p, x, t = _setup(FNO, B=B, cfg=cfg)
    got = f.infer(_dev(x)).cpu().numpy().astype(np.float64)
    ref = ofno.forward(p, x, cfg["modes"])
    # bf16 activations: compare the network output (pred - x) relative to its size
    e = np.linalg.norm(got - ref) / np.linalg.norm(ref - x)
    print("fno forward rel err (net output)", e)
    assert e < 3e-2
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-2


@pytest.mark.parametrize("cfg,B,members", [(CFG, 3, 2), (CFG, 3, 8), (CFG32, 3, 4), (CFG32R, 1, 4), (CFG_C5, 1, 8)],
                         ids=["gemm-2", "gemm-8", "fused-4", "fused-ragged-4", "surrogate-256-8"])
def test_ensemble_forward_matches_oracle(FNO, cfg, B, members):
    # inference averaged over reflections of the grid against the oracle's average
    # of the FP64 network over the same reflections
    print(f"[case] fno ensemble {members} {cfg} B={B}", flush=True)
    f, p, x, t = _setup(FNO, B=B, cfg=cfg)
    f.set_ensemble(members)
    got = f.infer(_dev(x)).cpu().numpy().astype(np.float64)
    ref = ofno.forward_ensemble(p, x, cfg["modes"], members)
    e = np.linalg.norm(got - ref) / np.linalg.norm(ref - x)
    print("fno ensemble rel err (net output)", e)
    assert e < 3e-2
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-2
    # back to the plain network: the same numbers as before any ensemble
    f.set_ensemble(1)
    plain = f.infer(_dev(x)).cpu().numpy().astype(np.float64)
    assert np.linalg.norm(plain - ofno.forward(p, x, cfg["modes"])) / np.linalg.norm(ref) < 1e-2


def test_ensemble_arguments(FNO):
    from paper_1708_03188_amd._lib import SgmError
    f, p, x, t = _setup(FNO, B=1, cfg=CFG32)  # 32 x 64: no transposes
    for m in (2, 8):
        with pytest.raises(SgmError, match="square"):
            f.set_ensemble(m)
    for m in (0, 3, 16):
        with pytest.raises(SgmError, match="members"):
            f.set_ensemble(m)
    f.set_ensemble(4)
    xd = _dev(x)
    with pytest.raises(SgmError, match="alias"):
        f.infer(xd, out=xd)


@pytest.mark.parametrize("cfg,B", [(CFG, 3), (CFG32, 3), (CFG_SK, 3), (CFG32_SK, 4), (CFG32R, 1), (CFG32_P128, 3),
                                   (CFG32_P96, 2)],
                         ids=["gemm", "fused", "gemm-splitk", "fused-splitk", "fused-hidden32-ragged", "fused-hidden128",
                              "fused-hidden96"])
def test_gradients_match_oracle(FNO, cfg, B):
    print(f"[case] fno gradients {cfg} B={B}", flush=True)
    f, p, x, t = _setup(FNO, B=B, seed=1, cfg=cfg)
    g, loss = f.grads(_dev(x), _dev(t))
    pred, cache = ofno.forward(p, x, cfg["modes"], keep=True)
    ref_loss = ofno.loss(pred, t)
    gr = ofno.backward(p, x, cfg["modes"], cache, ofno.loss_grad(pred, t))
    assert abs(loss - ref_loss) < 1e-2 * ref_loss
    worst = 0.0
    for k in gr:
        e = np.linalg.norm(g[k] - gr[k]) / max(np.linalg.norm(gr[k]), 1e-30)
        worst = max(worst, e)
        print(f"grad {k}: rel {e:.3e}")
        assert e < 2e-2, k
    print("worst grad rel err", worst)


def test_training_reduces_loss_and_checkpoint_roundtrip(FNO):
    # a learnable target: the output of a teacher network of the same architecture
    f, p, x, _ = _setup(FNO, B=4, seed=2)
    teacher = ofno.init_params(CFG["width"], CFG["modes"], CFG["hidden"], CFG["layers"], 99, scale_spec=0.3)
    teacher["W2"] *= 10.0
    t = ofno.forward(teacher, x, CFG["modes"])
    xd, td = _dev(x), _dev(t)
    l0 = f.train_step(xd, td, 3e-3)
    for _ in range(80):
        l = f.train_step(xd, td, 3e-3)
    assert l < 0.5 * l0, (l0, l)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ck.bin")
        f.save(path)
        before = f.infer(xd).cpu().numpy()
        f.train_step(xd, td, 1e-3)
        f.load(path)
        after = f.infer(xd).cpu().numpy()
        assert np.array_equal(before, after)


def test_zero_output_layer_gives_identity(FNO):
    f, p, x, t = _setup(FNO, seed=3)
    p["W2"][:] = 0
    p["b2"][:] = 0
    f.set_params(p)
    assert np.array_equal(f.infer(_dev(x)).cpu().numpy(), x.astype(np.float32))


def test_pack_unpack_states():
    from paper_1708_03188_amd.api import pack_states, unpack_states
    u = torch.randn(3, 8, 8, dtype=torch.complex128, device="cuda")
    x = pack_states(u)
    assert torch.allclose(x[..., 0].double(), u.real, atol=1e-6)
    assert torch.allclose(x[..., 1].double(), u.imag, atol=1e-6)
    back = unpack_states(x)
    assert torch.allclose(back, u, atol=1e-6)
