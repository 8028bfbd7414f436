"""Warm-start experiment on the m=255, s=128 GBDF3 workload (u0 = 0):

  1. solve the training seeds with the plain method (zero start) on the GPU,
  2. train the network with the library's forward/backward kernels and Adam,
  3. on held-out seeds, compare GMRES iterations and time to rel-res 1e-10 with zero start
     and with the network's x0 (inference included), on the same batched solver.

    python -m paper_1305_6653_amd.train_warmstart --train 20000 --heldout 1000 --out res.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--heldout", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--out", default="warmstart_eval.json")
    ap.add_argument("--checkpoint", default="")
    ap.add_argument("--target", default="lowrank", choices=["solution", "lowrank"],
                    help="solution: predict u; lowrank: predict c = (S - M) u on the boundary rows")
    a = ap.parse_args()

    import workloads as W
    from paper_1305_6653_amd import warmstart as WS

    log = lambda msg: print(msg, flush=True)
    if a.target == "lowrank":
        rows = WS.boundary_rows(2, 3, 128)          # GBDF3: nu = 2, mu = 3
        net = WS.WarmStartNet(max_batch=a.batch, seed=0, nx=255, nt=len(rows))
        net.use_boundary_rows(rows)
    else:
        net = WS.WarmStartNet(max_batch=a.batch, seed=0)
    log(f"network parameters: {net.num_params} (target {a.target})")
    data = WS.build_dataset(list(range(a.train)), net, W.warmstart_instance, batch=a.batch, log=log,
                            target=a.target)
    log(f"dataset: {a.train} instances in {data['seconds']:.1f} s, mean iters {data['iters'].mean():.2f}")
    t0 = time.perf_counter()
    hist = WS.train(net, data, epochs=a.epochs, batch=a.batch, lr=a.lr, log=log)
    t_train = time.perf_counter() - t0
    del data
    seeds = list(range(1_000_000, 1_000_000 + a.heldout))
    res = WS.evaluate(net, seeds, W.warmstart_instance, batch=a.batch, target=a.target)
    res_all = WS.evaluate(net, seeds, W.warmstart_instance, batch=a.batch, target=a.target, gate=0)
    n = len(seeds)
    summary = {
        "workload": "m=255, s=128, GBDF3, u0=0, random alpha/d+-/f (seeds 0..%d train, 1e6.. held out)" % (a.train - 1),
        "target": a.target, "network_params": net.num_params, "train_instances": a.train,
        "heldout_instances": n,
        "epochs": a.epochs, "train_seconds": round(t_train, 2), "loss_history": [float(x) for x in hist],
        "iters_zero_mean": float(np.mean(res["iters_zero"])), "iters_warm_mean": float(np.mean(res["iters_warm"])),
        "iters_zero_max": int(np.max(res["iters_zero"])), "iters_warm_max": int(np.max(res["iters_warm"])),
        "x0_gate": "library default (1e-2 of ||b||)", "x0_kept_fraction": float(np.mean(res["x0_kept"])),
        "iters_warm_mean_every_guess_kept": float(np.mean(res_all["iters_warm"])),
        "ms_per_instance_warm_incl_nn_every_guess_kept": res_all["ms_warm"] / n,
        "x0_rel_err_mean": float(np.mean(res["rel_err_x0"])), "x0_rel_err_median": float(np.median(res["rel_err_x0"])),
        "ms_per_instance_zero": res["ms_zero"] / n, "ms_per_instance_warm_incl_nn": res["ms_warm"] / n,
        "ms_per_instance_nn": res["ms_nn"] / n,
        "max_true_relres_warm": float(np.max(res["relres_warm"])),
        "max_true_relres_zero": float(np.max(res["relres_zero"])),
        "all_converged": bool(max(res["relres_warm"]) <= 1e-10 and max(res["relres_zero"]) <= 1e-10),
    }
    os.makedirs(os.path.dirname(a.out) or ".", exist_ok=True)
    with open(a.out, "w") as fh:
        json.dump(summary, fh, indent=1)
    if a.checkpoint:
        ck = net.checkpoint()
        np.savez(a.checkpoint, **{k: np.asarray(v) for k, v in ck.items()})
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
