"""GPU parity of the derivative/projection pass (Sec. 5: Dx, project) against the
oracle, through the C ABI: every source basis onto the regular, Shen-Dirichlet and
Shen-Neumann spaces of its family (Chebyshev or Legendre), x / y / z derivative orders, 2D and 3D, R2C and C2C, sizes
spanning several 16-column tiles with ragged tails and the chunk-length classes,
sampled columns of the full-size fields, and the paper's Sec. 5 use (derivative
of the biharmonic solution projected onto a Dirichlet space) on a closed form.

Tolerance: relative 1e-12 (transform class), normwise and max-wise."""
import numpy as np
import pytest

import synth
from conftest import rel_err
from oracle import chebyshev as C
from oracle import derivative as D
from oracle import legendre as OL

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
TOL = 1e-12


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def Plan():
    from paper_1708_03188_amd.api import Plan
    return Plan


SHAPES = [(12, 10), (33, 7), (3, 6), (5, 9), (64, 40), (100, 18), (512, 6),
          (20, 6, 8), (40, 5, 6), (17, 9, 14), (130, 12, 10)]
ORDERS = [(0, 0, 0), (1, 0, 0), (2, 1, 0), (4, 0, 2), (3, 2, 1)]


@pytest.mark.parametrize("kind", ["r2c", "c2c"])
@pytest.mark.parametrize("target", ["chebyshev", "dirichlet", "neumann"])
@pytest.mark.parametrize("basis", ["dirichlet", "biharmonic", "chebyshev", "neumann"])
@pytest.mark.parametrize("shape", SHAPES)
def test_project_derivative_small(Plan, basis, target, kind, shape):
    N = shape[0]
    if basis == "biharmonic" and N < 5:
        pytest.skip("biharmonic needs N >= 5")
    print(f"[case] derivative {basis}->{target} {kind} {shape}", flush=True)
    Ly, Lz = (3.0, 5.0) if N == 17 else (0.0, 0.0)
    p = Plan(basis, *shape, kind_last=kind, Ly=Ly, Lz=Lz)
    t = Plan(target, *shape, kind_last=kind, Ly=Ly, Lz=Lz)
    nb = C.nbasis(basis, N)
    uh = synth.random_spectral(p.spec_shape, seed=sum(shape) + N, nrows=nb)
    ud = dev(uh)
    for order in ORDERS:
        o = order if len(shape) == 3 else (order[0], order[1] + order[2], 0)
        got = host(p.project_derivative(ud, o, target=t))
        ref = D.project_dx(basis, uh, o[: len(shape)], target, shape[-1], kind, Ly, Lz)
        # relative to the size of the derivative itself (its Chebyshev coefficients):
        # a projection can be exactly zero (e.g. an odd derivative onto an even space)
        scale = np.abs(D.project_dx(basis, uh, o[: len(shape)], "chebyshev", shape[-1], kind, Ly, Lz)).max()
        if scale == 0:
            assert np.abs(got).max() == 0, order
            continue
        d = got - ref
        err = max(np.abs(d).max() / max(np.abs(ref).max(), scale),
                  np.linalg.norm(d) / max(np.linalg.norm(ref), scale))
        assert err < TOL, (order, err)


LEG_SHAPES = [(12, 10), (33, 7), (3, 6), (5, 9), (100, 18), (257, 6), (512, 4), (20, 6, 8), (17, 9, 14), (130, 12, 10)]


@pytest.mark.parametrize("kind", ["r2c", "c2c"])
@pytest.mark.parametrize("target", ["legendre", "leg_dirichlet", "leg_neumann"])
@pytest.mark.parametrize("basis", ["leg_dirichlet", "leg_biharmonic", "legendre", "leg_neumann"])
@pytest.mark.parametrize("shape", LEG_SHAPES)
def test_project_derivative_legendre(Plan, basis, target, kind, shape):
    N = shape[0]
    if basis == "leg_biharmonic" and N < 5:
        pytest.skip("the Legendre-biharmonic basis needs N >= 5")
    print(f"[case] derivative {basis}->{target} {kind} {shape}", flush=True)
    Ly, Lz = (3.0, 5.0) if N == 17 else (0.0, 0.0)
    p = Plan(basis, *shape, kind_last=kind, Ly=Ly, Lz=Lz)
    t = Plan(target, *shape, kind_last=kind, Ly=Ly, Lz=Lz)
    nb = OL.nbasis(basis, N)
    uh = synth.random_spectral(p.spec_shape, seed=sum(shape) + 3 * N, nrows=nb)
    ud = dev(uh)
    for order in ORDERS:
        o = order if len(shape) == 3 else (order[0], order[1] + order[2], 0)
        got = host(p.project_derivative(ud, o, target=t))
        ref = D.project_dx(basis, uh, o[: len(shape)], target, shape[-1], kind, Ly, Lz)
        scale = np.abs(D.project_dx(basis, uh, o[: len(shape)], "legendre", shape[-1], kind, Ly, Lz)).max()
        if scale == 0:
            assert np.abs(got).max() == 0, order
            continue
        d = got - ref
        err = max(np.abs(d).max() / max(np.abs(ref).max(), scale),
                  np.linalg.norm(d) / max(np.linalg.norm(ref), scale))
        assert err < TOL, (order, err)


def test_project_derivative_legendre_default_target_and_closed_form(Plan):
    # u = (1 - x^2)^2 sin y cos 3z in the Legendre-biharmonic space: du/dx vanishes at
    # x = +-1, so onto the Legendre-Dirichlet space it is reproduced on the grid; the
    # default target of a Legendre plan is the regular Legendre space
    print("[case] derivative Legendre closed form", flush=True)
    N, M1, M2 = 40, 16, 12
    p = Plan("leg_biharmonic", N, M1, M2)
    t = Plan("leg_dirichlet", N, M1, M2)
    x = p.points()
    y = 2 * np.pi * np.arange(M1) / M1
    z = 2 * np.pi * np.arange(M2) / M2
    s = np.sin(y)[None, :, None] * np.cos(3 * z)[None, None, :]
    u = ((1 - x**2) ** 2)[:, None, None] * s
    uh = p.forward(dev(u))
    du = t.backward(p.project_derivative(uh, (1, 0, 0), target=t))
    exact = (-4 * x * (1 - x**2))[:, None, None] * s
    assert np.abs(host(du) - exact).max() < 1e-12
    d2 = p.project_derivative(uh, (2, 0, 0))
    reg = Plan("legendre", N, M1, M2)
    exact2 = (12 * x**2 - 4)[:, None, None] * s
    assert np.abs(host(reg.backward(d2)) - exact2).max() < 1e-11


def test_project_derivative_rejects_bad_arguments(Plan):
    from paper_1708_03188_amd._lib import SgmError
    p = Plan("dirichlet", 16, 8, 6)
    uh = torch.zeros(p.spec_shape, dtype=torch.complex128, device="cuda")
    with pytest.raises(SgmError, match="target basis"):
        p.project_derivative(uh, (1, 0, 0), target=Plan("biharmonic", 16, 8, 6))
    with pytest.raises(SgmError, match="target basis"):
        p.project_derivative(uh, (1, 0, 0), target=Plan("leg_dirichlet", 16, 8, 6))
    lp = Plan("leg_dirichlet", 16, 8, 6)
    with pytest.raises(SgmError, match="target basis"):
        lp.project_derivative(uh, (1, 0, 0), target=Plan("chebyshev", 16, 8, 6))
    with pytest.raises(SgmError, match="target basis"):
        lp.project_derivative(uh, (1, 0, 0), target=Plan("leg_biharmonic", 16, 8, 6))
    with pytest.raises(SgmError, match="same grid"):
        p.project_derivative(uh, (1, 0, 0), target=Plan("chebyshev", 16, 8, 8))
    with pytest.raises(SgmError, match="order"):
        p.project_derivative(uh, (9, 0, 0))
    q = Plan("dirichlet", 16, 8)
    with pytest.raises(SgmError, match="order\\[2\\]"):
        q.project_derivative(torch.zeros(q.spec_shape, dtype=torch.complex128, device="cuda"), (1, 0, 1))


def test_biharmonic_solution_derivative_onto_dirichlet_closed_form(Plan):
    # Sec. 5: d/dx of the biharmonic problem's solution, projected onto a Dirichlet
    # space (it vanishes at x = +-1): u = (1 - x^2)^2 sin y cos 3z,
    # du/dx = -4x (1 - x^2) sin y cos 3z, exact on the grid
    print("[case] derivative of the manufactured biharmonic solution", flush=True)
    N, M1, M2 = 40, 16, 12
    x, y, z, u, _ = synth.biharmonic3d_manufactured(N, M1, M2)
    p = Plan("biharmonic", N, M1, M2)
    t = Plan("dirichlet", N, M1, M2)
    du = t.backward(p.project_derivative(p.forward(dev(u)), (1, 0, 0), target=t))
    exact = (-4 * x * (1 - x**2))[:, None, None] * np.sin(y)[None, :, None] * np.cos(3 * z)[None, None, :]
    assert np.abs(host(du) - exact).max() < 1e-12


@pytest.mark.parametrize("case", ["dirichlet256-cheb-x", "biharmonic512-dir-x", "dirichlet256-cheb-xyz",
                                  "legdirichlet256-legneumann-xyz"])
def test_project_derivative_full_size_sampled(Plan, case):
    # the full-size fields: every column computed on the GPU, sampled columns (and
    # the first and last) against the column-restricted oracle
    print(f"[case] derivative full size {case}", flush=True)
    basis, N, target, order = {"dirichlet256-cheb-x": ("dirichlet", 256, "chebyshev", (1, 0, 0)),
                               "biharmonic512-dir-x": ("biharmonic", 512, "dirichlet", (1, 0, 0)),
                               "dirichlet256-cheb-xyz": ("dirichlet", 256, "chebyshev", (2, 1, 1)),
                               "legdirichlet256-legneumann-xyz": ("leg_dirichlet", 256, "leg_neumann",
                                                                  (1, 1, 1))}[case]
    M1 = M2 = 256
    p = Plan(basis, N, M1, M2)
    t = Plan(target, N, M1, M2)
    nb = (OL if basis.startswith("leg") else C).nbasis(basis, N)
    uh = synth.random_spectral(p.spec_shape, seed=N, nrows=nb)
    got = host(p.project_derivative(dev(uh), order, target=t)).reshape(N, -1)
    ncols = got.shape[1]
    rng = np.random.default_rng(1)
    cols = np.unique(np.concatenate([[0, ncols - 1, 128, 129 * 128], rng.choice(ncols, 40, replace=False)]))
    ref = D.project_dx_columns(basis, uh.reshape(N, -1)[:, cols], order, target, cols, p.spec_shape, M2, "r2c")
    assert rel_err(got[:, cols], ref) < TOL
