"""Fourier-neural-operator surrogate, FP64 reference (oracle; test infrastructure only).

Architecture (an FNO-style map u(t) -> u(t + s dt) for the Ginzburg-Landau
state, complex split into two real channels, residual form):
  a_0  = x W_l + b_l                                        (lift, 2 -> C)
  for layer l = 0..nl-1:
    X    = (1/(H W)) sum_{y,x} a(y,x) exp(-2 pi i (ky y/H + kx x/W))   retained modes:
           ky in {0..K-1} u {H-K..H-1}, kx in {0..K-1}
    Y    = X R_l                      (complex C x C mixing per retained mode)
    s    = sum_{ky,kx} w_kx Re(Y exp(+2 pi i (ky y/H + kx x/W))),  w_0 = 1, w_kx>0 = 2
    z_l  = s + a W_l + b_l ;  a = gelu(z_l) (l < nl-1) or z_l (last layer)
  h    = gelu(a W_1 + b_1)  (C -> P) ;  out = h W_2 + b_2  (P -> 2) ;  pred = x + out
gelu(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2.
Loss: mean over samples of ||pred - target||_2 / ||target||_2.

All sums are plain contractions (exact-phase DFT matrices, einsum, evaluated
through BLAS products); the backward pass is
written out by hand and pinned against central finite differences.
"""
import numpy as np
from math import sqrt

import scipy.special as sps

TWO_PI_LD = 2 * np.arccos(np.longdouble(-1))


def round_bf16(a):
    """Round float64/float32 values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def ky_modes(H, K):
    return np.concatenate([np.arange(K), np.arange(H - K, H)])


def _phase(n, idx, sign):
    r = np.mod(np.outer(idx, np.arange(n)), n).astype(np.longdouble)
    ang = sign * TWO_PI_LD * r / n
    return (np.cos(ang) + 1j * np.sin(ang)).astype(np.complex128)


def dft_mats(H, W, K):
    """Ey[j, y] = exp(-2 pi i ky_j y / H), Ex[k, x] = exp(-2 pi i k x / W)."""
    return _phase(H, ky_modes(H, K), -1), _phase(W, np.arange(K), -1)


def init_params(C, K, P, nl, seed, scale_spec=None):
    """Seeded FP64 parameters (Glorot-like scales)."""
    rng = np.random.default_rng(seed)
    p = {"Wl": rng.standard_normal((2, C)) / sqrt(2), "bl": np.zeros(C)}
    sspec = (1.0 / (C * C)) if scale_spec is None else scale_spec
    for l in range(nl):
        p[f"Rr{l}"] = sspec * rng.random((2 * K, K, C, C))
        p[f"Ri{l}"] = sspec * rng.random((2 * K, K, C, C))
        p[f"Wp{l}"] = rng.standard_normal((C, C)) / sqrt(C)
        p[f"bp{l}"] = np.zeros(C)
    p["W1"] = rng.standard_normal((C, P)) / sqrt(C)
    p["b1"] = np.zeros(P)
    p["W2"] = rng.standard_normal((P, 2)) / sqrt(P) * 0.1
    p["b2"] = np.zeros(2)
    return p


def gelu(z):
    return 0.5 * z * (1.0 + sps.erf(z / sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + sps.erf(z / sqrt(2.0))) + z * np.exp(-0.5 * z * z) / sqrt(2 * np.pi)


def nlayers(p):
    return len([k for k in p if k.startswith("Wp")])


def forward(p, x, K, keep=False):
    """pred = x + net(x) for x of shape [B, H, W, 2]; keep=True also returns the
    intermediates the backward pass needs."""
    B, H, W, _ = x.shape
    Ey, Ex = dft_mats(H, W, K)
    wk = np.where(np.arange(K) == 0, 1.0, 2.0)
    nl = nlayers(p)
    a = x @ p["Wl"] + p["bl"]
    acts, zs, Xs = [a], [], []
    for l in range(nl):
        X = np.einsum("byxc,jy,kx->bjkc", a, Ey, Ex, optimize=True) / (H * W)
        R = p[f"Rr{l}"] + 1j * p[f"Ri{l}"]
        Y = np.einsum("bjkc,jkco->bjko", X, R, optimize=True)
        s = np.einsum("bjko,jy,kx,k->byxo", Y, np.conj(Ey), np.conj(Ex), wk, optimize=True).real
        z = s + a @ p[f"Wp{l}"] + p[f"bp{l}"]
        a = gelu(z) if l < nl - 1 else z
        zs.append(z)
        Xs.append(X)
        acts.append(a)
    hp = a @ p["W1"] + p["b1"]
    h = gelu(hp)
    out = h @ p["W2"] + p["b2"]
    pred = x + out
    if keep:
        return pred, dict(acts=acts, zs=zs, Xs=Xs, hp=hp, h=h, Ey=Ey, Ex=Ex, wk=wk)
    return pred


def reflect(u, t, fx, fy):
    """(R u)[b, i, j] for the reflection R = (transpose if t) after (flip rows if fx,
    flip columns if fy) of the H x W grid: the flips first, then the transpose."""
    v = u
    if fx:
        v = v[:, ::-1, :]
    if fy:
        v = v[:, :, ::-1]
    if t:
        v = np.swapaxes(v, 1, 2)
    return np.ascontiguousarray(v)


def unreflect(u, t, fx, fy):
    """R^{-1} u: the steps of reflect undone in reverse order."""
    v = u
    if t:
        v = np.swapaxes(v, 1, 2)
    if fy:
        v = v[:, :, ::-1]
    if fx:
        v = v[:, ::-1, :]
    return np.ascontiguousarray(v)


ENSEMBLES = {1: [(0, 0, 0)], 2: [(0, 0, 0), (1, 0, 0)],
             4: [(0, 0, 0), (0, 1, 0), (0, 0, 1), (0, 1, 1)],
             8: [(t, fx, fy) for t in (0, 1) for fx in (0, 1) for fy in (0, 1)]}


def forward_ensemble(p, x, K, members):
    """(1/m) sum_R R^{-1} forward(R x) over the m reflections of ENSEMBLES[m]: the
    network averaged over symmetries of the periodic square, which the
    Ginzburg-Landau equation (isotropic Laplacian, square periodic domain) has."""
    ops = ENSEMBLES[members]
    return sum(unreflect(forward(p, reflect(x, *op), K), *op) for op in ops) / len(ops)


def loss(pred, tgt):
    """mean_b ||pred_b - tgt_b|| / ||tgt_b||."""
    B = pred.shape[0]
    d = (pred - tgt).reshape(B, -1)
    n = tgt.reshape(B, -1)
    return float(np.mean(np.linalg.norm(d, axis=1) / np.linalg.norm(n, axis=1)))


def loss_grad(pred, tgt):
    B = pred.shape[0]
    d = (pred - tgt).reshape(B, -1)
    nd = np.linalg.norm(d, axis=1)
    nt = np.linalg.norm(tgt.reshape(B, -1), axis=1)
    g = d / (nd * nt)[:, None] / B
    return g.reshape(pred.shape)


def backward(p, x, K, cache, dpred):
    """Gradients of a scalar loss with d loss / d pred = dpred, for every parameter."""
    B, H, W, _ = x.shape
    Ey, Ex, wk = cache["Ey"], cache["Ex"], cache["wk"]
    nl = nlayers(p)
    g = {}
    dout = dpred
    g["W2"] = np.einsum("byxp,byxo->po", cache["h"], dout, optimize=True)
    g["b2"] = dout.sum(axis=(0, 1, 2))
    dh = dout @ p["W2"].T
    dhp = dh * gelu_grad(cache["hp"])
    a = cache["acts"][nl]
    g["W1"] = np.einsum("byxc,byxp->cp", a, dhp, optimize=True)
    g["b1"] = dhp.sum(axis=(0, 1, 2))
    da = dhp @ p["W1"].T
    for l in range(nl - 1, -1, -1):
        z = cache["zs"][l]
        dz = da * gelu_grad(z) if l < nl - 1 else da
        aprev = cache["acts"][l]
        g[f"Wp{l}"] = np.einsum("byxc,byxo->co", aprev, dz, optimize=True)
        g[f"bp{l}"] = dz.sum(axis=(0, 1, 2))
        da = dz @ p[f"Wp{l}"].T
        # spectral branch: s = Re(sum w Y e^{+i theta})  =>  gY = w sum dz e^{-i theta}
        gY = np.einsum("byxo,jy,kx,k->bjko", dz, Ey, Ex, wk, optimize=True)
        R = p[f"Rr{l}"] + 1j * p[f"Ri{l}"]
        X = cache["Xs"][l]
        gR = np.einsum("bjkc,bjko->jkco", np.conj(X), gY, optimize=True)
        g[f"Rr{l}"] = gR.real
        g[f"Ri{l}"] = gR.imag
        gX = np.einsum("bjko,jkco->bjkc", gY, np.conj(R), optimize=True)
        # X = (1/HW) sum a e^{-i theta}, a real  =>  da += (1/HW) Re(sum gX e^{+i theta})
        da = da + np.einsum("bjkc,jy,kx->byxc", gX, np.conj(Ey), np.conj(Ex), optimize=True).real / (H * W)
    g["Wl"] = np.einsum("byxi,byxc->ic", x, da, optimize=True)
    g["bl"] = da.sum(axis=(0, 1, 2))
    return g
