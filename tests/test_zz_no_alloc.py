"""The allocation-free backward transform (static device workspace) against the
ordinary backward transform, through the C ABI: identical results on two calls in
a row (the second on a smaller space), no device allocation by the call, and the
size limit rejected before any device work."""
import ctypes
import gc

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _mem_free():
    free = ctypes.c_size_t()
    total = ctypes.c_size_t()
    hip = ctypes.CDLL("libamdhip64.so")
    assert hip.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    return free.value


def _case(basis, N, M1, M2=None, kind="r2c", seed=0):
    from paper_1708_03188_amd.api import Plan
    p = Plan(basis, N, M1, M2, kind_last=kind)
    nb = {"dirichlet": N - 2, "neumann": N - 2, "leg_dirichlet": N - 2, "biharmonic": N - 4}.get(basis, N)
    uh = torch.from_numpy(synth.random_spectral(p.spec_shape, seed=seed, nrows=nb)).cuda()
    return p, uh


def test_noalloc_backward_matches_backward_on_two_calls():
    # a 3D space spanning several column tiles with ragged tails, then a smaller 2D one
    print("[case] sgm_backward_noalloc 3D 64x48x40 r2c, then 2D 32x20 c2c", flush=True)
    for basis, shape, kind, seed in (("dirichlet", (64, 48, 40), "r2c", 1), ("biharmonic", (32, 20), "c2c", 2)):
        p, uh = _case(basis, *shape, kind=kind, seed=seed)
        ref = p.backward(uh)
        got = p.backward_noalloc(uh)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (basis, shape)
    # the call allocates nothing: free device memory is unchanged across a call
    # (objects of earlier tests are collected first, and the collector is held off
    # meanwhile, so no release of theirs lands inside the measured interval)
    p, uh = _case("dirichlet", 48, 36, 24, seed=3)
    out = torch.empty(p.phys_shape, dtype=p.phys_dtype, device="cuda")
    p.backward_noalloc(uh, out=out)
    torch.cuda.synchronize()
    gc.collect()
    torch.cuda.synchronize()
    gc.disable()
    try:
        before = _mem_free()
        p.backward_noalloc(uh, out=out)
        torch.cuda.synchronize()
        after = _mem_free()
    finally:
        gc.enable()
    assert after == before
    assert torch.equal(out, p.backward(uh))


@pytest.mark.parametrize("basis", ["chebyshev", "neumann", "legendre", "leg_dirichlet", "leg_biharmonic"])
def test_noalloc_backward_every_basis_family(basis):
    # the other x-pass kinds (table-driven Chebyshev backward, the dense Legendre pass)
    # into the static workspace, twice in a row with the second space smaller
    print(f"[case] sgm_backward_noalloc {basis}", flush=True)
    for shape, seed in (((40, 24, 18), 11), ((24, 10), 12)):
        p, uh = _case(basis, *shape, seed=seed)
        ref = p.backward(uh)
        got = p.backward_noalloc(uh)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (basis, shape)


def test_noalloc_backward_rejects_oversized_space():
    from paper_1708_03188_amd.api import Plan
    from paper_1708_03188_amd._lib import SgmError
    print("[case] sgm_backward_noalloc size limit", flush=True)
    p = Plan("dirichlet", 256, 128, 128)   # 256*128*65 complex elements > 2^21
    uh = torch.zeros(p.spec_shape, dtype=torch.complex128, device="cuda")
    with pytest.raises(SgmError, match="allocation-free workspace"):
        p.backward_noalloc(uh)
