"""Surrogate pipeline: trajectories from the GL solver, training, evaluation.

Orchestration only: trajectories come from GLBatch (HIP solver kernels), states are
converted with the library's pack kernel, and training/inference run in the FNO
kernels.  Sample selection uses torch indexing on device tensors.
"""
import math

import numpy as np
import torch

from .api import FNO, GLBatch, pack_states


def generate_trajectories(n_traj, n_snap, N, L=100.0, b=1.5, c=-2.0, dt=0.05, spinup=200, stride=10, seed=5000,
                          noise=None):
    """Run n_traj independent N x N problems (IF-RK4) from seeded noise initial states,
    discard `spinup` steps, then record n_snap + 1 snapshots `stride` steps apart.
    Returns fp32 physical snapshots [n_snap + 1, n_traj, N, N, 2] on the device."""
    if noise is None:
        import synth
        noise = [synth.gl_noise(N, seed + i) for i in range(n_traj)]
    g = GLBatch([N] * n_traj, L=L, b=b, c=c, dt=dt, scheme="ifrk4", graph=True)
    u = g.pack(noise)
    uh = g.forward(u)
    g.step(uh, spinup)
    out = torch.empty((n_snap + 1, n_traj, N, N, 2), dtype=torch.float32, device="cuda")
    phys = torch.empty_like(uh)
    for k in range(n_snap + 1):
        if k:
            g.step(uh, stride)
        g.backward(uh, out=phys)
        pack_states(phys.view(n_traj, N, N), out=out[k])
    torch.cuda.synchronize()
    return out


def identity_error(data):
    """Relative L2 of the no-surrogate guess u(t + s dt) ~ u(t) over all pairs."""
    x = data[:-1].reshape(-1, *data.shape[2:])
    y = data[1:].reshape(-1, *data.shape[2:])
    d = (x - y).reshape(x.shape[0], -1).norm(dim=1) / y.reshape(y.shape[0], -1).norm(dim=1)
    return float(d.mean()), float(d.max())


def train(fno, data, steps, batch, lr=3e-3, lr_min=1e-5, seed=0, log_every=0, start=0, total=None):
    """Adam with cosine learning-rate decay on random (snapshot, trajectory) pairs.
    start/total place these steps inside a longer schedule (default: one decay
    over these steps)."""
    total = total or steps
    gen = torch.Generator(device="cpu").manual_seed(seed)
    ns, nt = data.shape[0] - 1, data.shape[1]
    losses = []
    for it in range(steps):
        k = torch.randint(0, ns, (batch,), generator=gen)
        i = torch.randint(0, nt, (batch,), generator=gen)
        x = data[k, i].contiguous()
        y = data[k + 1, i].contiguous()
        a = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * (start + it) / max(1, total)))
        want = log_every and (it % log_every == 0 or it == steps - 1)
        l = fno.train_step(x, y, a, want_loss=bool(want))
        if want:
            losses.append((it, l))
    torch.cuda.synchronize()
    return losses


def evaluate(fno, data, batch=None):
    """Per-sample relative L2 of the surrogate on every (snapshot, trajectory) pair."""
    batch = batch or fno.max_batch
    x = data[:-1].reshape(-1, *data.shape[2:])
    y = data[1:].reshape(-1, *data.shape[2:])
    rels = []
    for b0 in range(0, x.shape[0], batch):
        xb = x[b0:b0 + batch].contiguous()
        yb = y[b0:b0 + batch].contiguous()
        rels.append(fno.rel_l2(fno.infer(xb), yb))
    r = torch.cat(rels)
    return float(r.mean()), float(r.max())


# Parameters the kernels read in fp32 (lift and biases); the rest are only ever
# used through their bf16 mirrors, so storing them as bf16 (round to nearest
# even, as the device mirrors are made) reproduces inference bit for bit.
_FP32_KEYS = ("Wl", "bl", "b1", "b2")


def _is_fp32(name):
    return name in _FP32_KEYS or name.startswith("bp")


def _to_bf16_bits(a):
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)
    rounded = u + 0x7FFF + ((u >> 16) & 1)
    return (rounded >> 16).astype(np.uint16)


def export_weights(fno, path):
    """Write the inference weights of `fno` to an .npz file (no pickled objects)."""
    params = fno.get_params()
    arrays = {}
    for k, v in params.items():
        arrays[k] = np.asarray(v, dtype=np.float32) if _is_fp32(k) else _to_bf16_bits(v)
    meta = np.array([fno.H, fno.W, fno.C, fno.K, fno.nl, fno.P], dtype=np.int64)
    np.savez(path, _shape=meta, **arrays)


def import_weights(fno, path):
    """Load weights written by export_weights into `fno` (same architecture)."""
    with np.load(path, allow_pickle=False) as z:
        meta = [int(x) for x in z["_shape"]]
        if meta != [fno.H, fno.W, fno.C, fno.K, fno.nl, fno.P]:
            raise ValueError(f"weights are for shape {meta}")
        params = {}
        for k, shp in fno.param_shapes():
            a = z[k]
            params[k] = a if _is_fp32(k) else (a.astype(np.uint32) << 16).view(np.float32)
            params[k] = params[k].reshape(shp)
    fno.set_params(params)
