"""The autotuner's persisted choices: a tuned plan and a tuned GL batch write their
choice to the cache file; with the in-process memory cleared, new objects take the
file's choice (edited here to a different compiled variant, which proves the read),
give results equal to the oracle's, and ignore a stored choice that names no
compiled kernel."""
import os

import numpy as np
import pytest

import synth
from conftest import rel_err
from oracle import gl as ogl
from oracle import tensor as T

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _lines(path, head):
    with open(path) as fh:
        return [l for l in fh.read().splitlines() if l.startswith(head)]


def _rewrite(path, head, values):
    keep = [l for l in open(path).read().splitlines() if not l.startswith(head)]
    key = _lines(path, head)[-1].split(" =")[0]
    with open(path, "w") as fh:
        fh.write("\n".join(keep + [key + " = " + " ".join(str(v) for v in values)]) + "\n")


def test_plan_choices_persist_and_reload(tmp_path, monkeypatch):
    from paper_1708_03188_amd.api import Plan, autotune_forget, autotune_cache_path
    print("[case] autotune plan cache", flush=True)
    path = str(tmp_path / "tune.txt")
    monkeypatch.setenv("SGM_TUNE_CACHE", path)
    assert autotune_cache_path() == path
    autotune_forget()
    shape = (128, 128, 256)
    p = Plan("dirichlet", *shape, autotune=True)
    first = p.variants() + [p.solve_layout()[1]]
    assert first[3] in (8, 16)
    lines = _lines(path, "plan ")
    assert len(lines) == 1 and [int(v) for v in lines[0].split("=")[1].split()] == first
    # another compiled choice in the file (register variants per axis, rows per lane of
    # the solves): the next tuned plan takes it
    _rewrite(path, "plan ", [6, 7, 2, 8])
    autotune_forget()
    q = Plan("dirichlet", *shape, autotune=True)
    assert q.variants() == [6, 7, 2] and q.solve_layout() == (8, 8)
    ft = synth.random_spectral(q.spec_shape, seed=32, nrows=shape[0] - 2)
    sol = q.helmholtz_solve(torch.from_numpy(ft).cuda(), 1.0)
    torch.cuda.synchronize()
    scols = np.array([0, 7, 129 * 5 + 3, 128 * 129 - 1])
    ref = T.helmholtz_solve("dirichlet", ft, 1.0, shape[-1], cols=scols)
    assert rel_err(sol.cpu().numpy().reshape(shape[0], -1)[:, scols], ref) < 1e-10
    # an entry from before the solve was tuned (three values): 16 rows per lane
    _rewrite(path, "plan ", [6, 7, 2])
    autotune_forget()
    assert Plan("dirichlet", *shape, autotune=True).solve_layout() == (4, 16)
    u = synth.random_smooth_field(shape, seed=31)
    uh = q.forward(torch.from_numpy(u).cuda())
    torch.cuda.synchronize()
    N = shape[0]
    cols = np.array([0, 5, 129 * 3 + 17, 128 * 129 - 1])
    assert rel_err(uh.cpu().numpy().reshape(N, -1)[:, cols], T.forward_columns("dirichlet", u, cols)) < 1e-12
    vh = synth.random_spectral(q.spec_shape, seed=3, nrows=N - 2)
    rows = np.array([0, 77, N - 1])
    back = q.backward(torch.from_numpy(vh).cuda())
    torch.cuda.synchronize()
    assert rel_err(back.cpu().numpy()[rows], T.backward_rows("dirichlet", vh, rows, shape[-1])) < 1e-12
    # a stored choice naming no compiled kernel (variant 4 does not exist at 128) is ignored
    _rewrite(path, "plan ", [4, 4, 4, 16])
    autotune_forget()
    r = Plan("dirichlet", *shape, autotune=True)
    assert 4 not in r.variants()[:2]


def test_gl_choice_persists_and_reloads(tmp_path, monkeypatch):
    from paper_1708_03188_amd.api import GLBatch, autotune_forget
    print("[case] autotune gl cache", flush=True)
    path = str(tmp_path / "tune.txt")
    monkeypatch.setenv("SGM_TUNE_CACHE", path)
    autotune_forget()
    sizes = [64, 96, 64, 128]
    g = GLBatch(sizes, L=100.0, b=1.5, c=-2.0, dt=0.05, scheme="ifrk4", tune=True)
    lines = _lines(path, "gl ")
    assert len(lines) == 1 and int(lines[0].split("=")[1]) == g.variant
    other = (g.variant + 1) % 2 + 2 * (g.variant // 2)   # the other grid mode of the same tiling
    _rewrite(path, "gl ", [other])
    autotune_forget()
    h = GLBatch(sizes, L=100.0, b=1.5, c=-2.0, dt=0.05, scheme="ifrk4", tune=True)
    assert h.variant == other
    us = [synth.gl_noise(n, 60 + i) for i, n in enumerate(sizes)]
    st = h.forward(h.pack(us))
    h.step(st, 1)
    out = h.unpack(st)
    for i, n in enumerate(sizes):
        ref = ogl.ifrk4_step(ogl.forward(us[i]), 0.05, 100.0, 1.5, -2.0)
        assert rel_err(out[i].cpu().numpy(), ref) < 1e-12, n


def test_creation_on_a_side_stream(tmp_path, monkeypatch):
    # plan and batch creation (uploads and tuning runs) enqueued on the caller's
    # stream: results on that stream equal the oracle's
    from paper_1708_03188_amd.api import GLBatch, Plan, autotune_forget
    print("[case] creation on a side stream", flush=True)
    monkeypatch.setenv("SGM_TUNE_CACHE", str(tmp_path / "tune.txt"))
    autotune_forget()
    shape = (24, 16, 12)
    u = synth.random_smooth_field(shape, seed=8)
    st = torch.cuda.Stream()
    us = [synth.gl_noise(16, 1), synth.gl_noise(24, 2)]
    with torch.cuda.stream(st):
        p = Plan("dirichlet", *shape, autotune=True)
        g = GLBatch([16, 24], L=20.0, b=0.5, c=-1.0, dt=0.01, scheme="ifrk4", tune=True)
        uh = p.forward(torch.from_numpy(u).cuda())
        state = g.forward(g.pack(us))
        g.step(state, 1)
        out = g.unpack(state)
    st.synchronize()
    assert rel_err(uh.cpu().numpy(), T.forward("dirichlet", u)) < 1e-12
    for i in range(2):
        ref = ogl.ifrk4_step(ogl.forward(us[i]), 0.01, 20.0, 0.5, -1.0)
        assert rel_err(out[i].cpu().numpy(), ref) < 1e-12
