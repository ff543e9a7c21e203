"""Train the learned initial guess on the GPU and evaluate it.

    python -m paper_2001_02327_amd.train_guess --seeds 2000 --out weights.npy

Training data: FP64 nested solves of the seeded multi-Plummer workload (3
levels of 128^3, seeds 0..S-1), each refined level one sample (the network's
input and the error of the interpolated guess, extracted by the library).
Evaluation: validation seeds 100000.. solved with the interpolated and with
the learned guess; V-cycles per level and time are printed as JSON.
"""
import argparse
import json
import sys
import time

import numpy as np
import torch

from . import learned
from . import workloads as W
from .solver import NestedPoissonSolver


def evaluate(theta, seeds, N=128, nlevels=3):
    rows = []
    for seed in seeds:
        wl = W.c4_multi_plummer(seed, N=N, nlevels=nlevels)
        rho, po = W.make_inputs(wl.geom, wl.prob, device="cuda")
        res = {}
        for mode in ("interp", "learned"):
            s = NestedPoissonSolver(wl.geom, guess=mode)
            if mode == "learned":
                s.set_guess_weights(theta)
            s.solve(rho, po)  # warm-up (graph capture)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = s.solve(rho, po)
            torch.cuda.synchronize()
            res[mode] = dict(cycles=st["cycles"], ms=(time.perf_counter() - t0) * 1e3,
                             initial=st["initial_rel_residual"], interp=st["interp_rel_residual"],
                             used=st["learned_used"])
            s.close()
        rows.append(dict(seed=seed, **res))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", type=int, default=2000)
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-final", type=float, default=2e-4)
    ap.add_argument("--eval-seeds", type=int, default=6)
    ap.add_argument("--objective", default="residual", choices=["error", "residual"])
    ap.add_argument("--out", default=learned.DEFAULT_WEIGHTS)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    t0 = time.time()
    net, hist = learned.train(list(range(args.seeds)), N=args.N, lr=args.lr, lr_final=args.lr_final,
                              log=lambda m: print(m, flush=True), objective=args.objective)
    theta = net.params()
    learned.save_weights(theta, args.out)
    print("trained in %.1f s, saved %s" % (time.time() - t0, args.out), flush=True)
    rows = evaluate(theta, [100000 + i for i in range(args.eval_seeds)], N=args.N)
    for r in rows:
        print(json.dumps(r), flush=True)
    ci = sum(sum(r["interp"]["cycles"][1:]) for r in rows)
    cl = sum(sum(r["learned"]["cycles"][1:]) for r in rows)
    ti = sum(r["interp"]["ms"] for r in rows)
    tl = sum(r["learned"]["ms"] for r in rows)
    print(json.dumps(dict(summary=True, refined_cycles_interp=ci, refined_cycles_learned=cl, ms_interp=ti,
                          ms_learned=tl, loss_history=hist[-10:])), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
