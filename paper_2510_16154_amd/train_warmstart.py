"""Train and evaluate the learned warm start.

1. Training pairs: n RGB Voronoi images of size x size, each solved by the
   plain method (batched solve), giving its final multiplier field and
   controls.
2. Training: Adam on the library's network kernels.
3. Evaluation on held-out images: time to a converged solve (Lagrangian-gap
   stop of Sec. 4.1, iteration cap), cold against warm (prediction + solve);
   the warm result counts only at equal or lower final energy (within 1e-4
   relative), otherwise the cold time is added (fallback).

Writes the trained weights (.npy) and a JSON summary into --out.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-train", type=int, default=4000)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--w-eps", type=float, default=1.0)
    ap.add_argument("--n-eval", type=int, default=16)
    ap.add_argument("--eval-size", type=int, default=1024)
    ap.add_argument("--train-seed", type=int, default=50000)
    ap.add_argument("--eval-seed", type=int, default=60000)
    ap.add_argument("--out", default="warmstart_out")
    ap.add_argument("--weights", default=None, help="skip data and training: evaluate these weights (.npy)")
    ap.add_argument("--eval-outer", type=int, default=20, help="multiplier iteration cap of the evaluated solves")
    ap.add_argument("--tol-gap", type=float, default=1e-2, help="Lagrangian-gap stop of the evaluated solves")
    ap.add_argument("--eval-tol-alm", type=float, default=0.0,
                    help="ALM residual stop of the evaluated solves (0: off, the gap stop decides)")
    ap.add_argument("--target-outer", type=int, default=5, help="multiplier iterations of the target solves")
    ap.add_argument("--target-inner", type=int, default=10, help="DAL iterations per multiplier iteration")
    ap.add_argument("--target-tol-alm", type=float, default=0.0,
                    help="ALM residual stop of the target solves (0: run --target-outer iterations)")
    ap.add_argument("--target-tol-gap", type=float, default=0.0,
                    help="Lagrangian-gap stop of the target solves (0: off); with --target-outer 20 and "
                         "--target-inner 10 the targets come from the evaluation's own stopping rule")
    ap.add_argument("--solve-batch", type=int, default=64, help="images per batched target solve")
    ap.add_argument("--chunk", type=int, default=256, help="images solved per data chunk (one progress line each)")
    ap.add_argument("--warm-eps", action="store_true",
                    help="warm solves start from the predicted controls too (default: predicted multiplier only)")
    ap.add_argument("--eval-both", action="store_true",
                    help="also evaluate the other warm-start mode (with / without the predicted controls)")
    args = ap.parse_args(argv)

    import torch

    from . import binding as B
    from .synth import voronoi_image
    from .warmstart import WarmStart, cold_solve, ideal_warm_solve, make_dataset
    from .workloads import VORONOI512

    os.makedirs(args.out, exist_ok=True)
    params = B.Params(K=VORONOI512.K, R=VORONOI512.R, max_outer=args.target_outer, max_inner=args.target_inner,
                      alpha=VORONOI512.alpha, tol_alm=args.target_tol_alm, tol_gap=args.target_tol_gap)
    ws = WarmStart(params.K, params, seed=7)
    logs, t_data = [], 0.0
    if args.weights:
        ws.params.copy_(torch.as_tensor(np.load(args.weights), device="cuda"))
        args.n_train = 0
    t0 = time.perf_counter()
    xs, mus, epss = [], [], []
    chunk = args.chunk
    for s in range(0, args.n_train, chunk):
        x, mu, eps = make_dataset(min(chunk, args.n_train - s), args.size, args.train_seed + s, params,
                                  batch=args.solve_batch)
        xs.append(x)
        mus.append(mu)
        epss.append(eps)
        print(f"[data] {s + x.shape[0]}/{args.n_train} solved ({time.perf_counter() - t0:.0f} s)", flush=True)
    if args.n_train:
        x, mu, eps = torch.cat(xs), torch.cat(mus), torch.cat(epss)
        t_data = time.perf_counter() - t0
    for ep in range(args.epochs if args.n_train else 0):
        lg = ws.train(x, mu, eps, epochs=1, batch=args.batch, lr=args.lr * (0.8 ** ep), w_eps=args.w_eps, seed=ep)
        logs.append(lg.losses[0])
        print(f"[train] epoch {ep + 1}/{args.epochs} loss {lg.losses[0]:.5f} ({lg.seconds:.1f} s)", flush=True)
    if args.n_train:
        np.save(os.path.join(args.out, "wsnet_k50.npy"), ws.params.cpu().numpy())
        del x, mu, eps, xs, mus, epss
        torch.cuda.empty_cache()

    rows = []
    for i in range(args.n_eval):
        seed = args.eval_seed + i
        r = np.random.default_rng(seed)
        regions = int(r.integers(4, 17))
        sigma = float(r.uniform(0.02, 0.1))
        img = torch.as_tensor(voronoi_image(args.eval_size, args.eval_size, 3, regions, sigma, seed), device="cuda")
        pe = params.replace(max_outer=args.eval_outer, max_inner=10, tol_gap=args.tol_gap,
                            tol_alm=args.eval_tol_alm)
        cold = cold_solve(img, pe, keep_state=True)
        warm = ws.solve(img, pe, cold=cold, use_eps=args.warm_eps)
        ideal = ideal_warm_solve(img, pe, cold)
        rows.append({"seed": seed, "cold_K": cold["K"], "cold_outer": cold["outer_iters"], "cold_s": cold["seconds"],
                     "warm_outer": warm["outer_iters"], "warm_s": warm["seconds"], "warm_K": warm["K"],
                     "fallback": warm["fallback"], "ideal_outer": ideal["outer_iters"], "ideal_s": ideal["seconds"],
                     "ideal_K": ideal["K"], "cold_outer_log": cold["outer_log"]})
        if args.eval_both:
            other = ws.solve(img, pe, cold=cold, use_eps=not args.warm_eps)
            rows[-1].update(other_outer=other["outer_iters"], other_s=other["seconds"], other_K=other["K"],
                            other_fallback=other["fallback"])
        print(f"[eval] {i + 1}/{args.n_eval} " + json.dumps(rows[-1]), flush=True)
    sp = [r["cold_s"] / r["warm_s"] for r in rows]
    it = [r["cold_outer"] / max(r["warm_outer"], 1) for r in rows]
    summary = {"train": {"n": args.n_train, "size": args.size, "epochs": args.epochs, "batch": args.batch,
                         "lr": args.lr, "losses": logs, "data_seconds": t_data,
                         "targets": {"max_outer": args.target_outer, "max_inner": args.target_inner,
                                     "tol_alm": args.target_tol_alm, "tol_gap": args.target_tol_gap}},
               "eval": {"n": args.n_eval, "size": args.eval_size, "rows": rows,
                        "speedup_time_median": float(np.median(sp)), "speedup_time_geomean": float(np.exp(np.mean(np.log(sp)))),
                        "speedup_iters_median": float(np.median(it)),
                        "ideal_speedup_time_median": float(np.median([r["cold_s"] / r["ideal_s"] for r in rows])),
                        "fallbacks": int(sum(r["fallback"] for r in rows))}}
    if args.eval_both:
        so = [r["cold_s"] / r["other_s"] for r in rows]
        summary["eval"].update(other_mode="multiplier only" if args.warm_eps else "multiplier and controls",
                               other_speedup_time_median=float(np.median(so)),
                               other_speedup_time_geomean=float(np.exp(np.mean(np.log(so)))),
                               other_fallbacks=int(sum(r["other_fallback"] for r in rows)))
    json.dump(summary, open(os.path.join(args.out, "summary.json"), "w"), indent=1)
    print("[summary] " + json.dumps({k: v for k, v in summary["eval"].items() if k != "rows"}), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
