"""Train the Ginzburg-Landau FNO surrogate on trajectories of the FP64 solver.

    python -m paper_1708_03188_amd.train_surrogate --out fno_gl256.bin

Trajectories come from GLBatch (IF-RK4, 256^2, L = 100, b = 1.5, c = -2, dt = 0.05,
200 spin-up steps, snapshots 10 steps apart) started from seeded uniform noise;
training runs the library's forward/backward/Adam kernels with one cosine
learning-rate decay, optionally continuing from a checkpoint.  Held-out
trajectories use a disjoint seed range.  Progress (held-out relative L2) is
printed every --eval-every steps and the checkpoint is written at each
evaluation and at the end.
"""
import argparse
import json
import time

from . import surrogate as S
from .api import FNO


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--traj", type=int, default=512)
    ap.add_argument("--snaps", type=int, default=24)
    ap.add_argument("--test-traj", type=int, default=16)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval-every", type=int, default=2000)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--init", default=None, help="checkpoint to continue from")
    ap.add_argument("--export", default=None, help="also write the inference weights (.npz) at the end")
    args = ap.parse_args(argv)
    t0 = time.perf_counter()
    train = S.generate_trajectories(args.traj, args.snaps, args.N, seed=5000)
    test = S.generate_trajectories(args.test_traj, 8, args.N, seed=900000)
    print(json.dumps({"generated_s": round(time.perf_counter() - t0, 1), "train_pairs": args.traj * args.snaps,
                      "persistence_rel_l2": S.identity_error(test)}), flush=True)
    f = FNO(args.N, args.N, width=32, modes=16, layers=4, hidden=128, max_batch=max(16, args.batch), seed=args.seed)
    if args.init:
        f.load(args.init)
    t0 = time.perf_counter()
    done = 0
    while done < args.steps:
        n = min(args.eval_every, args.steps - done)
        S.train(f, train, steps=n, batch=args.batch, lr=args.lr, seed=done, start=done, total=args.steps)
        done += n
        m, mx = S.evaluate(f, test)
        f.save(args.out)
        print(json.dumps({"steps": done, "heldout_rel_l2_mean": round(m, 5), "heldout_rel_l2_max": round(mx, 5),
                          "train_s": round(time.perf_counter() - t0, 1)}), flush=True)
    if args.export:
        S.export_weights(f, args.export)


if __name__ == "__main__":
    main()
