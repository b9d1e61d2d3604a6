"""Benchmark of the spectral-Galerkin hot path on one MI355X.

Workload: 3D Poisson/Helmholtz space, Shen-Dirichlet N = 256 along x times
Fourier 256 x 256 (R2C) along y, z, float64, a seeded smooth random field
(synthetic; no dataset).  One step = one forward transform (Fourier R2C + C2C,
DCT-II, Shen projection) plus one backward transform of the whole field;
value = N*M1*M2 / (t_fwd + t_bwd) in Gdof/s.  Also reported: full 3D
Helmholtz solves per second (solve kernel alone and the Poisson pipeline
scalar product -> solve -> backward), the dominant kernel's roofline
fraction from per-pass hipEvents, and the CPU oracle on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calib", action="store_true", help="also run a plain 1 GiB device copy (counter calibration)")
    return ap.parse_args()


def pass_bytes(N, M1, M2, nb):
    """Algorithmic HBM bytes per launch of each pass kind at this shape."""
    M2r = M2 // 2 + 1
    dof = N * M1 * M2
    spec = N * M1 * M2r * 16
    specnb = nb * M1 * M2r * 16
    return {
        "last_fwd": dof * 8 + spec,        # read real field, write half spectrum
        "last_bwd": spec + dof * 8,
        "mid_fwd": 2 * spec,
        "mid_bwd": 2 * spec,
        "cheb_fwd": 2 * spec,
        "cheb_scalar": 2 * spec,
        "cheb_bwd": specnb + spec,         # rows >= nb are not read
        "solve": specnb + spec,
    }


def cpu_baseline(N, M1, M2):
    """Time the oracle on a bounded sample of the same workload and extrapolate."""
    import synth
    from oracle import tensor as T
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    u = synth.random_smooth_field((N, M1, M2), seed=2)
    M2r = M2 // 2 + 1
    ncols = M1 * M2r
    rng = np.random.default_rng(0)
    kc, kr = 48, 8
    cols = rng.choice(ncols, kc, replace=False)
    t0 = time.perf_counter()
    T.forward_columns("dirichlet", u, cols)
    t_cols = time.perf_counter() - t0
    vh = synth.random_spectral((N, M1, M2r), seed=3, nrows=N - 2)
    rows = rng.choice(N, kr, replace=False)
    t0 = time.perf_counter()
    T.backward_rows("dirichlet", vh, rows, M2)
    t_rows = time.perf_counter() - t0
    t_full = t_cols * ncols / kc + t_rows * N / kr
    return {
        "value": N * M1 * M2 / t_full / 1e9,
        "unit": "Gdof/s",
        "cores": int(cores),
        "kind": "oracle",
        "sample": f"oracle forward on {kc} of {ncols} spectral columns ({t_cols:.1f} s) and backward on "
                  f"{kr} of {N} x-rows ({t_rows:.1f} s) of the same 256^3 field, extrapolated linearly "
                  f"to the full transform pair ({t_full:.0f} s)",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "requested_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import synth
    from paper_1708_03188_amd.api import Plan

    torch.cuda.set_device(0)
    N = M1 = M2 = 256
    p = Plan("dirichlet", N, M1, M2, autotune=True)
    u = torch.from_numpy(synth.random_smooth_field((N, M1, M2), seed=2)).cuda()
    uh = torch.empty(p.spec_shape, dtype=torch.complex128, device="cuda")
    v = torch.empty_like(u)

    def step():
        p.forward(u, out=uh)
        p.backward(uh, out=v)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    p.pass_times(reset=True)
    p.set_timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    times = p.pass_times(reset=True)
    p.set_timing(False)

    # secondary figures: Helmholtz solve kernel alone and the Poisson pipeline
    ft = p.scalar_product(u)
    sol = torch.empty_like(ft)
    for _ in range(3):
        p.helmholtz_solve(ft, 0.0, out=sol)
    torch.cuda.synchronize()
    ks = max(10, args.steps)
    e0.record()
    for _ in range(ks):
        p.helmholtz_solve(ft, 0.0, out=sol)
    e1.record()
    torch.cuda.synchronize()
    ms_solve = e0.elapsed_time(e1) / ks
    e0.record()
    for _ in range(ks):
        p.scalar_product(u, out=ft)
        p.helmholtz_solve(ft, 0.0, out=sol)
        p.backward(sol, out=v)
    e1.record()
    torch.cuda.synchronize()
    ms_poisson = e0.elapsed_time(e1) / ks

    if args.copy_calib:
        a = torch.empty(2**27, dtype=torch.float64, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    dof = N * M1 * M2
    gdofs = dof / (ms * 1e-3) / 1e9
    nbytes = pass_bytes(N, M1, M2, N - 2)
    per_pass = {k: {"avg_us": 1e3 * t / c, "launches": c,
                    "GBps": nbytes[k] / (t / c * 1e-3) / 1e9} for k, (t, c) in times.items()}
    dom = max(times, key=lambda k: times[k][0])
    avg_s = times[dom][0] / times[dom][1] * 1e-3
    achieved = nbytes[dom] / avg_s / 1e9
    out = {
        "metric": "FP64 fwd+bwd transform Gdof/s; Poisson solves/s; GL steps/s surrogate vs plain",
        "value": round(gdofs, 3),
        "unit": "Gdof/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D Poisson/Helmholtz space, Shen-Dirichlet N=256 x Fourier 256x256 R2C, "
                               "float64; step = forward + backward transform",
                   "N": N, "M1": M1, "M2": M2, "basis": "shen_dirichlet", "kind_last": "r2c"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
        "passes": {k: {kk: round(vv, 2) for kk, vv in d.items()} for k, d in per_pass.items()},
        "helmholtz_solves_per_s": round(1e3 / ms_solve, 1),
        "poisson_pipeline_solves_per_s": round(1e3 / ms_poisson, 1),
        "transform_pair_algorithmic_GBps": round((2 * dof * 8 + 2 * N * M1 * (M2 // 2 + 1) * 16) / (ms * 1e-3) / 1e9, 1),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(N, M1, M2)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
