"""Benchmark of the solver's hot path on one MI355X.

Workload: 512 x 512 RGB Voronoi image (12 regions, colour gradients of
amplitude 0.1, noise sigma 0.08), window radius R = 5, K = 50 Euler steps.

One timed step is one pass over the whole hot path, as one iteration of the
control argmin runs it: terminal condition and objective, adjoint sweep with
the control-gradient reduction (K adjoint steps), the projected control
update, the forward sweep storing the trajectory (K steps), the objective of
the trial, then one shrinkage / multiplier update, each with the host reads
the solver does.  value = agent-steps per second = H * W * K / (step time),
counting one forward and one adjoint sweep per step.

Also reported: forward and adjoint sweep times alone (HIP events on the
stream the kernels run on), the roofline of the dominant kernel (the adjoint
step), the FP64 CPU oracle timed on a bounded sample of the same work (all
host threads and one), and the second half of the metric, time to a
converged solve: the same image solved to ALM residual 1e-5 from the cold
start (with and without the DAL stationarity stop), the oracle's time for it
extrapolated from its own sweep times and the GPU's iteration counts, the
32 x 32 x 3 solve (5 x 50 iterations) timed whole on both sides, and the
learned warm start against the plain solve on held-out 1024 x 1024 images.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_VALU_TFLOPS = 157.3  # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the dominant kernel of each workload, from the rocprofv3
# FETCH_SIZE / WRITE_SIZE passes (scaled by a plain-copy calibration), keyed by the
# SHA-256 of the kernel source they were taken with; reported as null for any other source.
PROFILED_TRAFFIC = {
    "kernel_sha256": "d5bd119be8ef2ddca56872e5b997b50c8b0d976cb59581e891f69d5e04cf42a9",
    "adj_step_kernel<3,5>": 11.53e6,
    "adj_step_wide_kernel<31,2>": 1607.64e6,
}
KERNEL_SRC = os.path.join(ROOT, "paper_2510_16154_amd", "csrc", "abc_kernels.hip")


def kernel_sha() -> str:
    import hashlib
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()


def profiled_traffic(kernel: str):
    return PROFILED_TRAFFIC.get(kernel) if PROFILED_TRAFFIC["kernel_sha256"] == kernel_sha() else None


def window_pairs(H: int, W: int, R: int) -> int:
    """Ordered in-image pairs (i, j), j != i, with |row diff|, |col diff| <= R."""
    rows = sum((H - abs(a)) for a in range(-R, R + 1) if abs(a) < H)
    cols = sum((W - abs(b)) for b in range(-R, R + 1) if abs(b) < W)
    return rows * cols - H * W


def flops_per_pair(C: int, kind: str) -> int:
    # forward: D (C), |D|^2 (2C), r (2), phi (6), accumulation (2C)
    # adjoint: forward terms + phi' + (p_j - p_i), D.dp, two accumulations, two gradient integrands
    return 5 * C + 8 if kind == "fwd" else 12 * C + 18


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 50 for voronoi512, fewer for the longer workloads)")
    # The GPU's clocks settle only after tens of milliseconds of sustained load (per-launch
    # times of the interaction kernels fall by about 12% over the first 10 to 20 sweeps), so
    # the default warm-up of the headline line runs about a quarter of a second of steps.
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed warm-up steps (default: 100 for voronoi512, fewer for the longer workloads)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-min-seconds", type=float, default=10.0,
                    help="repeat the oracle's full forward+adjoint sweep until this much time has passed")
    ap.add_argument("--workload", default="voronoi512", choices=["voronoi512", "batch64", "segment512", "hyper2048", "warmstart1024", "converge512",
                             "transfer1024", "quadratic512", "support128", "sweeps1024"],
                    help="voronoi512: the headline line (default); batch64: the batched form; segment512: "
                         "watershed labels and IRV/IRC/VS scores of a solved 512 x 512 image; hyper2048: the "
                         "differentiable form on 2048 x 2048 x 31 (checkpointed forward + backward); warmstart1024: "
                         "time to a converged solve of held-out 1024 x 1024 images, plain against the packaged "
                         "learned warm start; converge512: time to solve the 512 x 512 image to ALM residual 1e-5; "
                         "transfer1024: controls of the 512 x 512 solve applied to its 2x finer version; "
                         "quadratic512: the DAL with the quadratic cost J (Def. 3.2) on the 512 x 512 image; "
                         "support128: the un-windowed sum (window from the kernel's support) on 128 x 128; "
                         "sweeps1024: the headline sweeps on a 1024 x 1024 version of the image (a grid that fills "
                         "the GPU)")
    ap.add_argument("--images", type=int, default=4, help="warmstart1024: held-out images to solve")
    ap.add_argument("--no-converge", action="store_true",
                    help="voronoi512: skip the time-to-converged part (converged solves, 32 x 32 solve, warm start)")
    ap.add_argument("--tol-dal", type=float, default=TOL_DAL,
                    help="voronoi512: DAL stationarity tolerance of the second converged solve")
    ap.add_argument("--no-graphs", action="store_true",
                    help="batch64: launch every sweep step directly instead of replaying captured graphs")
    ap.add_argument("--persistent", type=int, default=None, choices=[0, 1],
                    help="batch64: persistent sweeps over per-step tile queues (1) or one workgroup per tile (0); "
                         "default: the faster form as measured (see the design notes)")
    ap.add_argument("--autotune", type=int, default=1, choices=[0, 1],
                    help="batch64: tiles timed by the library's tuner on the largest image (1, default) or the "
                         "library's default tiles (0)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times) and exit; used to calibrate "
                         "the HBM byte counters")
    args = ap.parse_args()
    # (steps, warmup) per workload when not given: the longer workloads time whole solves.
    defaults = {"voronoi512": (50, 100), "batch64": (3, 1), "segment512": (20, 3), "hyper2048": (5, 2),
                "warmstart1024": (0, 1), "converge512": (1, 1), "transfer1024": (20, 5), "quadratic512": (3, 1),
                "support128": (5, 2), "sweeps1024": (20, 20)}
    d_steps, d_warm = defaults[args.workload]
    if args.steps is None:
        args.steps = d_steps
    if args.warmup is None:
        args.warmup = d_warm
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the solver runs on a "
              "single device, see the design notes for how it would shard)", file=sys.stderr)
        return 2

    import torch

    if args.copy_probe > 0:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "reps": 5}))
        return 0

    if args.workload == "batch64":
        return bench_batch(args)
    if args.workload == "segment512":
        return bench_segment(args)
    if args.workload == "hyper2048":
        return bench_hyper(args)
    if args.workload == "warmstart1024":
        return bench_warmstart(args)
    if args.workload == "converge512":
        return bench_converge(args)
    if args.workload == "transfer1024":
        return bench_transfer(args)
    if args.workload == "quadratic512":
        return bench_quadratic(args)
    if args.workload == "support128":
        return bench_support(args)
    if args.workload == "sweeps1024":
        return bench_sweeps1024(args)

    import paper_2510_16154_amd as A
    from paper_2510_16154_amd.workloads import VORONOI512 as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    H, W, C, K, R = wl.H, wl.W, wl.C, wl.K, wl.R
    params = wl.params()
    c0n = wl.image()
    c0 = torch.as_tensor(c0n, device=dev)
    eps = torch.full((K, 2), params.eps_init, dtype=torch.float32, device=dev)
    eps_try = eps.clone()
    v = torch.zeros((H, W, 2, C), dtype=torch.float32, device=dev)
    mu = torch.zeros_like(v)
    ws_f = torch.empty(max(A.abc_workspace_bytes(A.ABC_WS_FORWARD, H, W, C, params), 1), dtype=torch.uint8,
                       device=dev)
    ws_a = torch.empty(A.abc_workspace_bytes(A.ABC_WS_ADJOINT, H, W, C, params), dtype=torch.uint8, device=dev)
    traj = torch.empty((K + 1, H, W, C), dtype=torch.float32, device=dev)
    traj2 = torch.empty_like(traj)
    g0 = torch.empty_like(c0)
    geps = torch.empty((K, 2), dtype=torch.float32, device=dev)

    A.abc_forward_dynamics(c0, eps, params, traj=traj, ws=ws_f)
    A.abc_pd_step(traj[-1], c0, v, mu, params, update_mu=False, want_stats=False)
    # As in the library's solver loop: the host keeps the FP64 master controls, the
    # gradient comes back and the trial controls go out through pinned buffers, and
    # the objective at the current controls is known from the previous trial.
    eps_master = np.full((K, 2), float(params.eps_init))
    geps_h = torch.empty((K, 2), dtype=torch.float32, pin_memory=True)
    eps_h = torch.empty((K, 2), dtype=torch.float32, pin_memory=True)
    ws_p = torch.empty(max(A.abc_workspace_bytes(A.ABC_WS_PD, H, W, C, params), 1), dtype=torch.uint8, device=dev)
    gK_buf = torch.empty_like(c0)
    kstream = torch.cuda.current_stream()

    def step():
        gK, _ = A.abc_pd_terminal(traj[-1], c0, v, mu, params, want_objective=False, gK=gK_buf, ws=ws_p)
        A.abc_adjoint_dynamics(traj, eps, params, gK, g0=g0, geps=geps, ws=ws_a)
        geps_h.copy_(geps, non_blocking=True)
        kstream.synchronize()
        G = geps_h.numpy().astype(np.float64) / params.dt
        e_new = np.clip(eps_master - 1.0 * G, params.eps_min[0], params.eps_max[0])
        eps_h.numpy()[:] = e_new
        eps_try.copy_(eps_h, non_blocking=True)
        A.abc_forward_dynamics(c0, eps_try, params, traj=traj2, ws=ws_f)
        _, phit = A.abc_pd_terminal(traj2[-1], c0, v, mu, params, want_gradient=False, ws=ws_p)
        return A.abc_pd_step(traj[-1], c0, v, mu, params, update_mu=True, ws=ws_p)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = step()
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps

    # sweep-only timings with HIP events on the kernels' stream
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    reps = 20
    fwd_ms, adj_ms = [], []
    gK = torch.randn((H, W, C), generator=torch.Generator().manual_seed(0)).to(dev)
    for rep in range(reps + 5):
        ev[0].record(stream)
        A.abc_forward_dynamics(c0, eps, params, traj=traj, ws=ws_f)
        ev[1].record(stream)
        A.abc_adjoint_dynamics(traj, eps, params, gK, g0=g0, geps=geps, ws=ws_a)
        ev[2].record(stream)
        ev[2].synchronize()
        if rep >= 5:  # the first sweep pairs are warm-up
            fwd_ms.append(ev[0].elapsed_time(ev[1]))
            adj_ms.append(ev[1].elapsed_time(ev[2]))
    t_fwd = float(np.median(fwd_ms)) * 1e-3
    t_adj = float(np.median(adj_ms)) * 1e-3

    pairs = window_pairs(H, W, R)
    adj_launch = t_adj / K  # one adjoint-step launch (sweep time / K, launch gaps included)
    adj_flops = pairs * flops_per_pair(C, "adj")
    fwd_flops = pairs * flops_per_pair(C, "fwd")
    achieved = adj_flops / adj_launch / 1e12
    traffic = profiled_traffic("adj_step_kernel<3,5>")
    value = H * W * K / t_step
    out = {
        "metric": "agent-steps/sec (fwd+adjoint)",
        "value": value,
        "unit": "agent-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Voronoi image)",
        "config": {"workload": wl.name, "H": H, "W": W, "C": C, "R": R, "K": K,
                   "step": "terminal+adjoint sweep+control update+forward sweep+objective+pd_step"},
        "sweeps": {"fwd_ms": t_fwd * 1e3, "adj_ms": t_adj * 1e3,
                   "agent_steps_per_s_sweeps_only": H * W * K / (t_fwd + t_adj),
                   "fwd_tflops": fwd_flops * K / t_fwd / 1e12, "adj_tflops": adj_flops * K / t_adj / 1e12},
        "roofline": {"kernel": "adj_step_kernel<3,5>", "bound": "alu", "achieved": achieved,
                     "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU_TFLOPS,
                     "traffic": traffic, "flops_per_launch": adj_flops, "launch_ms": adj_launch * 1e3},
        "last_step_stats": {k: st[k] for k in ("K", "TV", "fid", "r_rel")},
    }
    sweep_s = None
    if not args.no_cpu_baseline:
        out["cpu_baseline"], sweep_s = cpu_baseline(c0n, wl, args.cpu_min_seconds)
    if not args.no_converge:
        out["time_to_converged"] = time_to_converged(c0, wl, sweep_s, args.tol_dal, not args.no_cpu_baseline)
    print(json.dumps(out), flush=True)
    return 0


# Whether the batched line runs its sweeps as persistent launches over per-step tile
# queues (ABC_FLAG_PERSISTENT): the faster of the two forms as measured on the 64-image batch.
BATCH_PERSISTENT = True

# Relative change of the inner objective below which the second converged solve
# ends a control argmin (convergence remark, Sec. 3.2).  The paper's 1e-10 is
# below what FP32 objectives resolve; this is the smallest value measurably
# above their rounding.
TOL_DAL = 1e-5


def _solve_row(A, c0, params, oracle_sweep_s=None) -> dict:
    import torch
    t0 = time.perf_counter()
    res = A.abc_solve(c0, params)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    st = res["stats"]
    row = {"s": t, **{k: st[k] for k in ("status", "outer_iters", "inner_iters", "ls_evals", "K", "L", "r_rel")}}
    if oracle_sweep_s is not None:
        # one adjoint sweep per DAL iteration, one forward sweep per Armijo trial plus the starting one
        f, a = oracle_sweep_s
        row["oracle_s_extrapolated"] = st["inner_iters"] * a + (st["ls_evals"] + 1) * f
    return row


def time_to_converged(c0, wl, oracle_sweep_s, tol_dal: float, with_oracle: bool) -> dict:
    """Second half of the metric.  plain: the bench image solved from the cold start
    until r_rel < 1e-5 (M <= 200, P = 50); plain_dal_stop: the same with each
    control argmin also ended by the stationarity test |dPhi| < tol_dal |Phi|.
    The oracle's time for each is its measured forward and adjoint sweep times
    times the GPU run's sweep counts (labelled extrapolated; its per-pixel
    terminal and shrinkage work is left out).  cfg0: the 32 x 32 x 3 image,
    R = 2, K = 20, 5 x 50 iterations, timed whole on the GPU and in the oracle
    (all host threads and one).  warm_start: held-out 1024 x 1024 images, the
    packaged network's start against the plain solve under the gap stop."""
    import torch

    import paper_2510_16154_amd as A
    from paper_2510_16154_amd.workloads import VORONOI32

    params = wl.params()
    A.abc_solve(c0, params.replace(max_outer=2))  # records the sweep graphs of this shape
    out = {"stop": f"r_rel < {params.tol_alm:g}, M <= {params.max_outer}, P = {params.max_inner}",
           "plain": _solve_row(A, c0, params, oracle_sweep_s)}
    row = _solve_row(A, c0, params.replace(tol_dal=tol_dal), oracle_sweep_s)
    row["tol_dal"] = tol_dal
    out["plain_dal_stop"] = row

    w0 = VORONOI32
    x0n = w0.image()
    x0 = torch.as_tensor(x0n, device=c0.device)
    p0 = w0.params()
    A.abc_solve(x0, p0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r0 = A.abc_solve(x0, p0)
    torch.cuda.synchronize()
    cfg0 = {"workload": w0.name, "gpu_s": time.perf_counter() - t0, "K": r0["stats"]["K"],
            "schedule": f"{p0.max_outer}x{p0.max_inner}"}
    if with_oracle:
        from oracle import oracle as O
        op = O.Params(K=w0.K, R=w0.R, alpha=p0.alpha, max_outer=p0.max_outer, max_inner=p0.max_inner)
        n_all = O.num_threads()
        t1 = time.perf_counter()
        ref = O.solve(x0n, op)
        cfg0.update(oracle_s=time.perf_counter() - t1, oracle_cores=n_all, oracle_K=ref["stats"]["K"])
        O.set_num_threads(1)
        try:
            t1 = time.perf_counter()
            O.solve(x0n, op)
            cfg0["oracle_1thread_s"] = time.perf_counter() - t1
        finally:
            O.set_num_threads(n_all)
    out["cfg0"] = cfg0
    out["warm_start"] = warm_start_rows(4)
    return out


def warm_start_rows(n_images: int) -> dict:
    """Plain against learned warm start on held-out 1024 x 1024 images (seeds 60000+):
    time and iterations to a converged solve under the gap stop of Sec. 4.1."""
    import torch

    import paper_2510_16154_amd as A
    from paper_2510_16154_amd.synth import voronoi_image
    from paper_2510_16154_amd.warmstart import TRAINED_K50, WarmStart, cold_solve

    params = A.Params(K=50, R=5, max_outer=20, max_inner=10, alpha=3000.0, tol_gap=1e-2)
    ws = WarmStart.load(TRAINED_K50, 50, params)
    rows = []
    for i in range(n_images + 1):
        seed = 60000 + i
        r = np.random.default_rng(seed)
        regions, sigma = int(r.integers(4, 17)), float(r.uniform(0.02, 0.1))
        img = torch.as_tensor(voronoi_image(1024, 1024, 3, regions, sigma, seed), device="cuda")
        cold = cold_solve(img, params)
        warm = ws.solve(img, params, cold=cold)
        if i == 0:
            continue  # the first image records the graphs of this shape
        rows.append({"seed": seed, "cold_s": cold["seconds"], "warm_s": warm["seconds"],
                     "cold_outer": cold["outer_iters"], "warm_outer": warm["outer_iters"],
                     "cold_dal": cold["dal_iters"], "warm_dal": warm["dal_iters"], "fallback": warm["fallback"]})
    sp = np.array([r["cold_s"] / r["warm_s"] for r in rows])
    return {"stop": "gap 1e-2, M <= 20, P = 10", "images": len(rows),
            "speedup_geomean": float(np.exp(np.mean(np.log(sp)))), "speedup_median": float(np.median(sp)),
            "fallbacks": int(sum(r["fallback"] for r in rows)), "rows": rows}


def bench_batch(args) -> int:
    """Batched form: 64 uneven images per solve; images/s and per-image latency."""
    import torch

    import paper_2510_16154_amd as A
    from paper_2510_16154_amd.workloads import BATCH64 as wb

    dev = torch.device("cuda:0")
    imgs = [torch.as_tensor(x, device=dev) for x in wb.images()]
    persistent = BATCH_PERSISTENT if args.persistent is None else bool(args.persistent)
    flags = ((A.ABC_FLAG_NO_GRAPHS if args.no_graphs else 0) | (A.ABC_FLAG_PERSISTENT if persistent else 0) |
             (A.ABC_FLAG_AUTOTUNE if args.autotune else 0))
    params = wb.params(flags=flags)
    shapes = [(x.shape[0], x.shape[1]) for x in imgs]
    ws = torch.empty(A.abc_workspace_bytes_batched(shapes, wb.C, params), dtype=torch.uint8, device=dev)
    npx = sum(h * w for h, w in shapes)
    for _ in range(args.warmup):
        A.abc_solve_batched(imgs, params, ws=ws)
    torch.cuda.synchronize()
    times, fins, stats = [], [], None
    for _ in range(args.steps):
        t0 = time.perf_counter()
        _, stats, fin = A.abc_solve_batched(imgs, params, ws=ws)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        fins.append(fin)
    t = float(np.median(times))
    lat = np.concatenate(fins)
    evals = sum(s["ls_evals"] + s["inner_iters"] for s in stats)
    out = {"metric": "images/sec (batched solve)", "value": wb.n / t, "unit": "images/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": t * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded Voronoi images)",
           "config": {"workload": wb.name, "images": wb.n, "pixels": npx, "R": wb.R, "K": wb.K,
                      "schedule": f"{wb.max_outer}x{wb.max_inner}", "graphs": not args.no_graphs,
                      "persistent": persistent, "autotune": bool(args.autotune)},
           "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
           "sweeps_per_solve": evals,
           "agent_steps_per_s": npx * wb.K * evals / len(stats) / t}
    print(json.dumps(out), flush=True)
    return 0


def bench_hyper(args) -> int:
    """Differentiable form on the 2048 x 2048 x 31 smooth-spectrum image (R = 2, K = 100):
    one step = the forward sweep keeping a checkpoint every 10 steps plus the backward of
    l = <w, c^K> (adjoint sweep, each segment recomputed once).  value = H W K / step time.
    Per-launch kernel times come from a 10-step sweep with the full trajectory."""
    import torch

    import paper_2510_16154_amd as A
    from paper_2510_16154_amd.workloads import HYPER2048 as wl

    dev = torch.device("cuda:0")
    H, W, C, K, R = wl.H, wl.W, wl.C, wl.K, wl.R
    c0n = wl.image()
    c0 = torch.as_tensor(c0n, device=dev)
    params = A.Params(K=K, R=R, ckpt_every=10)
    eps = torch.full((K, 2), params.eps_init, dtype=torch.float32, device=dev)
    w = torch.randn((H, W, C), generator=torch.Generator().manual_seed(2003)).to(dev)
    ws_f = torch.empty(max(A.abc_workspace_bytes(A.ABC_WS_FORWARD, H, W, C, params), 1), dtype=torch.uint8,
                       device=dev)
    ws_a = torch.empty(A.abc_workspace_bytes(A.ABC_WS_ADJOINT, H, W, C, params), dtype=torch.uint8, device=dev)
    traj = torch.empty((A.abc_traj_slots(params), H, W, C), dtype=torch.float32, device=dev)
    g0 = torch.empty_like(c0)
    geps = torch.empty((K, 2), dtype=torch.float32, device=dev)

    def step():
        A.abc_forward_dynamics(c0, eps, params, traj=traj, ws=ws_f)
        A.abc_adjoint_dynamics(traj, eps, params, w, g0=g0, geps=geps, ws=ws_a)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    del traj, ws_f, ws_a

    # per-launch times: a 10-step sweep with the full trajectory, HIP events on the kernels' stream
    Ks = 10
    ps = A.Params(K=Ks, R=R)
    es = eps[:Ks].contiguous()
    tr = torch.empty((Ks + 1, H, W, C), dtype=torch.float32, device=dev)
    wf = torch.empty(max(A.abc_workspace_bytes(A.ABC_WS_FORWARD, H, W, C, ps), 1), dtype=torch.uint8, device=dev)
    wa = torch.empty(A.abc_workspace_bytes(A.ABC_WS_ADJOINT, H, W, C, ps), dtype=torch.uint8, device=dev)
    ge = torch.empty((Ks, 2), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fwd_ms, adj_ms = [], []
    for _ in range(5):
        ev[0].record(stream)
        A.abc_forward_dynamics(c0, es, ps, traj=tr, ws=wf)
        ev[1].record(stream)
        A.abc_adjoint_dynamics(tr, es, ps, w, g0=g0, geps=ge, ws=wa)
        ev[2].record(stream)
        ev[2].synchronize()
        fwd_ms.append(ev[0].elapsed_time(ev[1]))
        adj_ms.append(ev[1].elapsed_time(ev[2]))
    t_fwd = float(np.median(fwd_ms)) * 1e-3 / Ks
    t_adj = float(np.median(adj_ms)) * 1e-3 / Ks
    pairs = window_pairs(H, W, R)
    npx = H * W

    def kernel(name, t, flops, nbytes):
        return {"kernel": name, "launch_ms": t * 1e3, "tflops": flops / t / 1e12, "gbs": nbytes / t / 1e9,
                "flops_per_launch": flops, "bytes_per_launch": nbytes,
                "roof_ms": max(nbytes / (PEAK_HBM_GBS * 1e9), flops / (PEAK_FP32_VALU_TFLOPS * 1e12)) * 1e3}

    kf = kernel(f"fwd_step_wide_kernel<31,{R}>", t_fwd, pairs * flops_per_pair(C, "fwd"), 8 * C * npx)
    ka = kernel(f"adj_step_wide_kernel<31,{R}>", t_adj, pairs * flops_per_pair(C, "adj"), 12 * C * npx)
    out = {"metric": "agent-steps/sec (fwd+adjoint), differentiable form", "value": npx * K / t_step,
           "unit": "agent-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": t_step * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic (seeded smooth-spectrum Voronoi image)",
           "config": {"workload": wl.name, "H": H, "W": W, "C": C, "R": R, "K": K, "ckpt_every": 10,
                      "step": "checkpointed forward sweep + backward (adjoint sweep with segment recompute)"},
           "kernels": {"fwd": kf, "adj": ka},
           "roofline": {"kernel": ka["kernel"], "bound": "alu", "achieved": ka["tflops"],
                        "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                        "frac": ka["tflops"] / PEAK_FP32_VALU_TFLOPS, "traffic": profiled_traffic(ka["kernel"])},
           "hbm": {"kernel": kf["kernel"], "achieved_gbs": kf["gbs"], "peak_gbs": PEAK_HBM_GBS,
                   "frac": kf["gbs"] / PEAK_HBM_GBS}}
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        crop = np.ascontiguousarray(c0n[960:1088, 960:1088])
        P = O.Params(K=K, R=R)
        e = np.full((K, 2), 57.0)
        pK = np.random.default_rng(0).normal(size=crop.shape)
        reps, t1 = 0, time.perf_counter()
        while True:
            tr_o = O.forward_sweep(crop, P, e)
            O.adjoint_sweep(tr_o, P, pK, e)
            reps += 1
            dt = time.perf_counter() - t1
            if dt >= args.cpu_min_seconds:
                break
        out["cpu_baseline"] = {"value": crop.shape[0] * crop.shape[1] * K * reps / dt, "unit": "agent-steps/s",
                               "cores": O.num_threads(), "kind": "oracle",
                               "sample": f"{reps} x (forward + adjoint sweep, {K} steps) of a 128x128x31 crop, "
                                         f"R={R}, FP64, {dt:.1f} s"}
    print(json.dumps(out), flush=True)
    return 0


def bench_transfer(args) -> int:
    """Sec. 4.3 control transfer: controls solved on the 512 x 512 x 3 bench image (3 x 5
    iterations) drive one forward sweep of its 2x nearest-neighbour upsampled version
    (1024 x 1024, window 2R = 10, normalisation s/4).  One step = that sweep."""
    import torch

    import paper_2510_16154_amd as A
    from paper_2510_16154_amd.transfer import transfer_params
    from paper_2510_16154_amd.workloads import VORONOI512 as wl

    c_lo = torch.as_tensor(wl.image(), device="cuda")
    p_lo = wl.params(max_outer=3, max_inner=5, tol_alm=0.0)
    eps = torch.full((wl.K, 2), p_lo.eps_init, dtype=torch.float32, device="cuda")
    A.abc_solve(c_lo, p_lo, eps=eps)
    c_hi = c_lo.repeat_interleave(2, dim=0).repeat_interleave(2, dim=1).contiguous()
    ph = transfer_params(p_lo, wl.H, wl.W, 2)
    H, W, C = c_hi.shape
    ws = torch.empty(max(A.abc_workspace_bytes(A.ABC_WS_FORWARD, H, W, C, ph), 1), dtype=torch.uint8, device="cuda")
    traj = torch.empty((A.abc_traj_slots(ph), H, W, C), dtype=torch.float32, device="cuda")
    for _ in range(args.warmup):
        A.abc_forward_dynamics(c_hi, eps, ph, traj=traj, ws=ws)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ms = []
    for _ in range(args.steps):
        ev[0].record(stream)
        A.abc_forward_dynamics(c_hi, eps, ph, traj=traj, ws=ws)
        ev[1].record(stream)
        ev[1].synchronize()
        ms.append(ev[0].elapsed_time(ev[1]))
    t = float(np.median(ms)) * 1e-3
    pairs = window_pairs(H, W, ph.R)
    tflops = pairs * flops_per_pair(C, "fwd") * wl.K / t / 1e12
    out = {"metric": "agent-steps/sec (forward sweep, transferred controls)", "value": H * W * wl.K / t,
           "unit": "agent-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded Voronoi image, 2x upsampled)",
           "config": {"workload": "transfer1024_rgb_r10_k50", "H": H, "W": W, "C": C, "R": ph.R, "K": wl.K},
           "roofline": {"kernel": f"fwd_step_kernel<3,{ph.R if ph.R <= 5 else 0}>", "bound": "alu",
                        "achieved": tflops, "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                        "frac": tflops / PEAK_FP32_VALU_TFLOPS, "traffic": None}}
    print(json.dumps(out), flush=True)
    return 0


def bench_quadratic(args) -> int:
    """Def. 3.2 with Alg. 1 alone: the direct-adjoint loop with the two-way projected
    Armijo search on the quadratic cost J, 512 x 512 x 3 bench image, R = 5, K = 50,
    P = 50 DAL iterations from the cold controls.  One step = one such solve; the
    value counts its sweeps (one adjoint sweep per DAL iteration, one forward sweep per
    Armijo trial plus the starting one).  cpu_baseline: the oracle's same solve on the
    central 256 x 256 crop cut to two DAL iterations, in the same unit."""
    import torch

    import paper_2510_16154_amd as A
    from paper_2510_16154_amd.workloads import VORONOI512 as wl

    c0n = wl.image()
    c0 = torch.as_tensor(c0n, device="cuda")
    params = wl.params(cost=A.ABC_COST_QUADRATIC, max_outer=1, max_inner=50, tol_alm=0.0)
    for _ in range(args.warmup):
        A.abc_solve(c0, params, want_v=False)
    torch.cuda.synchronize()
    times, st = [], None
    for _ in range(args.steps):
        t0 = time.perf_counter()
        st = A.abc_solve(c0, params, want_v=False)["stats"]
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    sweeps = st["inner_iters"] + st["ls_evals"] + 1
    out = {"metric": "agent-steps/sec (DAL, quadratic cost)", "value": wl.H * wl.W * wl.K * sweeps / t,
           "unit": "agent-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": t * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic (seeded Voronoi image)",
           "config": {"workload": "quadratic512_rgb_r5_k50", "H": wl.H, "W": wl.W, "C": wl.C, "R": wl.R,
                      "K": wl.K, "cost": "quadratic J (Def. 3.2)", "schedule": "P = 50 DAL iterations"},
           "stats": {k: st[k] for k in ("inner_iters", "ls_evals", "K", "phi_first", "phi_last")},
           "sweeps_per_solve": sweeps}
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        op = O.Params(K=wl.K, R=wl.R, alpha=params.alpha, cost=1, max_outer=1, max_inner=2)
        crop = np.ascontiguousarray(c0n[128:384, 128:384])
        t0 = time.perf_counter()
        ref = O.solve(crop, op)
        dt = time.perf_counter() - t0
        rs = ref["stats"]
        n = rs["inner_iters"] + rs["ls_evals"] + 1
        out["cpu_baseline"] = {"value": 256 * 256 * wl.K * n / dt, "unit": "agent-steps/s",
                               "cores": O.num_threads(), "kind": "oracle",
                               "sample": f"the same solve on the central 256x256 crop, cut to {rs['inner_iters']} "
                                         f"DAL iterations ({n} sweeps), FP64, {dt:.1f} s"}
    print(json.dumps(out), flush=True)
    return 0


def bench_support(args) -> int:
    """eq. MAsystem summed over every pair inside the kernel's support: a 128 x 128 x 3
    Voronoi image (6 regions, sigma 0.05, seed 1005), R = ABC_RADIUS_SUPPORT with
    eps_x >= 2, which on this image is R* = 127 (all pairs), s = 1/N; K = 20, controls
    eps_init.  One step = one forward and one adjoint sweep (HIP events); these radii
    run the direct kernels.  cpu_baseline: the oracle's forward and adjoint sweeps of
    the same image cut to 10 Euler steps, in the same unit."""
    import torch

    import paper_2510_16154_amd as A
    from paper_2510_16154_amd.synth import voronoi_image

    H = W = 128
    C, K = 3, 20
    c0n = voronoi_image(H, W, C, 6, 0.05, 1005)
    c0 = torch.as_tensor(c0n, device="cuda")
    params = A.Params(K=K, R=A.ABC_RADIUS_SUPPORT)
    R = A.abc_support_radius(H, W, params.eps_min[0])
    eps = torch.full((K, 2), params.eps_init, dtype=torch.float32, device="cuda")
    gKn = np.random.default_rng(5).normal(size=(H, W, C))
    gK = torch.as_tensor(gKn.astype(np.float32), device="cuda")
    traj = torch.empty((K + 1, H, W, C), dtype=torch.float32, device="cuda")
    ws_a = torch.empty(A.abc_workspace_bytes(A.ABC_WS_ADJOINT, H, W, C, params), dtype=torch.uint8, device="cuda")
    g0 = torch.empty_like(c0)
    geps = torch.empty((K, 2), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fwd, adj = [], []
    for rep in range(args.warmup + args.steps):
        ev[0].record(stream)
        A.abc_forward_dynamics(c0, eps, params, traj=traj)
        ev[1].record(stream)
        A.abc_adjoint_dynamics(traj, eps, params, gK, g0=g0, geps=geps, ws=ws_a)
        ev[2].record(stream)
        ev[2].synchronize()
        if rep >= args.warmup:
            fwd.append(ev[0].elapsed_time(ev[1]) * 1e-3)
            adj.append(ev[1].elapsed_time(ev[2]) * 1e-3)
    t_f, t_a = float(np.median(fwd)), float(np.median(adj))
    pairs = window_pairs(H, W, R)
    adj_flops = pairs * flops_per_pair(C, "adj")
    achieved = adj_flops * K / t_a / 1e12
    out = {"metric": "agent-steps/sec (fwd+adjoint, un-windowed sum)", "value": H * W * K / (t_f + t_a),
           "unit": "agent-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": (t_f + t_a) * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic (seeded Voronoi image)",
           "config": {"workload": "support128_rgb_k20", "H": H, "W": W, "C": C, "R": R, "K": K,
                      "window": "support of eps_x >= 2: every pair", "s": "1/N"},
           "sweeps": {"fwd_ms": t_f * 1e3, "adj_ms": t_a * 1e3, "pairs_per_step": pairs,
                      "fwd_tflops": pairs * flops_per_pair(C, "fwd") * K / t_f / 1e12},
           "roofline": {"kernel": "adj_direct_kernel<3>", "bound": "alu", "achieved": achieved,
                        "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU_TFLOPS,
                        "traffic": None, "flops_per_launch": adj_flops, "launch_ms": t_a / K * 1e3}}
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        Ks = 10
        op = O.Params(K=Ks, R=R, s=1.0 / (H * W))
        e = np.full((Ks, 2), float(params.eps_init))
        t0 = time.perf_counter()
        tr = O.forward_sweep(c0n, op, e)
        O.adjoint_sweep(tr, op, gKn, e)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": H * W * Ks / dt, "unit": "agent-steps/s", "cores": O.num_threads(),
                               "kind": "oracle",
                               "sample": f"forward + adjoint sweep of {Ks} Euler steps of the same image, "
                                         f"R = {R}, FP64, {dt:.1f} s"}
    print(json.dumps(out), flush=True)
    return 0


def bench_sweeps1024(args) -> int:
    """The headline image's dynamics (R = 5, K = 50, controls eps_init) on a
    1024 x 1024 x 3 Voronoi image of the same recipe (seed 1006): forward and
    adjoint sweeps timed with HIP events.  At 512 x 512 the 512 tiles of a sweep
    step give each CU two workgroups; here four, which shows what the same
    kernels reach once the grid fills the GPU."""
    import torch

    import paper_2510_16154_amd as A
    from paper_2510_16154_amd.synth import voronoi_image
    from paper_2510_16154_amd.workloads import VORONOI512 as wl

    H = W = 1024
    C, K, R = wl.C, wl.K, wl.R
    c0 = torch.as_tensor(voronoi_image(H, W, C, wl.regions, wl.sigma, 1006, gradient_amp=wl.gradient_amp),
                         device="cuda")
    params = A.Params(K=K, R=R)
    eps = torch.full((K, 2), params.eps_init, dtype=torch.float32, device="cuda")
    gK = torch.as_tensor(np.random.default_rng(6).normal(size=(H, W, C)).astype(np.float32), device="cuda")
    traj = torch.empty((K + 1, H, W, C), dtype=torch.float32, device="cuda")
    ws_a = torch.empty(A.abc_workspace_bytes(A.ABC_WS_ADJOINT, H, W, C, params), dtype=torch.uint8, device="cuda")
    g0 = torch.empty_like(c0)
    geps = torch.empty((K, 2), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fwd, adj = [], []
    for rep in range(args.warmup + args.steps):
        ev[0].record(stream)
        A.abc_forward_dynamics(c0, eps, params, traj=traj)
        ev[1].record(stream)
        A.abc_adjoint_dynamics(traj, eps, params, gK, g0=g0, geps=geps, ws=ws_a)
        ev[2].record(stream)
        ev[2].synchronize()
        if rep >= args.warmup:
            fwd.append(ev[0].elapsed_time(ev[1]) * 1e-3)
            adj.append(ev[1].elapsed_time(ev[2]) * 1e-3)
    t_f, t_a = float(np.median(fwd)), float(np.median(adj))
    pairs = window_pairs(H, W, R)
    adj_flops = pairs * flops_per_pair(C, "adj")
    achieved = adj_flops * K / t_a / 1e12
    out = {"metric": "agent-steps/sec (fwd+adjoint sweeps)", "value": H * W * K / (t_f + t_a),
           "unit": "agent-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": (t_f + t_a) * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic (seeded Voronoi image)",
           "config": {"workload": "voronoi1024_rgb_r5_k50_sweeps", "H": H, "W": W, "C": C, "R": R, "K": K},
           "sweeps": {"fwd_ms": t_f * 1e3, "adj_ms": t_a * 1e3,
                      "fwd_tflops": pairs * flops_per_pair(C, "fwd") * K / t_f / 1e12},
           "roofline": {"kernel": "adj_step_kernel<3,5>", "bound": "alu", "achieved": achieved,
                        "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU_TFLOPS,
                        "traffic": None, "flops_per_launch": adj_flops, "launch_ms": t_a / K * 1e3}}
    print(json.dumps(out), flush=True)
    return 0


def bench_converge(args) -> int:
    """Time to a converged solve of the 512 x 512 x 3 bench image: the method of
    multipliers until r_rel < 1e-5 (at most 200 iterations of at most 50 DAL
    steps each), from the cold start.  One timed call of abc_solve per step."""
    import torch

    import paper_2510_16154_amd as A
    from paper_2510_16154_amd.workloads import VORONOI512 as wl

    c0 = torch.as_tensor(wl.image(), device="cuda")
    params = wl.params()
    for _ in range(args.warmup):
        A.abc_solve(c0, params.replace(max_outer=2))
    torch.cuda.synchronize()
    times, st = [], None
    for _ in range(args.steps):
        t0 = time.perf_counter()
        out = A.abc_solve(c0, params)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        st = out["stats"]
    t = float(np.median(times))
    res = {"metric": "time-to-converged solve (r_rel < 1e-5)", "value": t, "unit": "s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": t * 1e3, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded Voronoi image)",
           "config": {"workload": wl.name, "H": wl.H, "W": wl.W, "C": wl.C, "R": wl.R, "K": wl.K,
                      "stop": "r_rel < 1e-5, M <= 200, P = 50"},
           "stats": {k: st[k] for k in ("status", "outer_iters", "inner_iters", "ls_evals", "K", "r_rel", "gap_rel")}}
    print(json.dumps(res), flush=True)
    return 0


def bench_warmstart(args) -> int:
    """Time to a converged solve (gap stop 1e-2 of Sec. 4.1, at most 20 multiplier x 10 DAL
    iterations, R = 5, K = 50) of held-out 1024 x 1024 RGB Voronoi images, cold start
    against the packaged network's start.  A warm result counts only at the cold solve's
    final energy or below (1e-4 relative); otherwise the cold time is added.  The warm
    time includes the network's forward pass.  value = geometric-mean speedup."""
    import torch

    import paper_2510_16154_amd as A
    from paper_2510_16154_amd.synth import voronoi_image
    from paper_2510_16154_amd.warmstart import TRAINED_K50, WarmStart, cold_solve

    params = A.Params(K=50, R=5, max_outer=20, max_inner=10, alpha=3000.0, tol_gap=1e-2)
    ws = WarmStart.load(TRAINED_K50, 50, params)
    rows = []
    for i in range(args.images + max(args.warmup, 0)):
        seed = 60000 + i
        r = np.random.default_rng(seed)
        regions, sigma = int(r.integers(4, 17)), float(r.uniform(0.02, 0.1))
        img = torch.as_tensor(voronoi_image(1024, 1024, 3, regions, sigma, seed), device="cuda")
        cold = cold_solve(img, params)
        warm = ws.solve(img, params, cold=cold)
        if i < args.warmup:
            continue
        rows.append({"seed": seed, "cold_s": cold["seconds"], "warm_s": warm["seconds"], "cold_K": cold["K"],
                     "warm_K": warm["K"], "cold_outer": cold["outer_iters"], "warm_outer": warm["outer_iters"],
                     "fallback": warm["fallback"]})
    sp = np.array([r["cold_s"] / r["warm_s"] for r in rows])
    out = {"metric": "time-to-converged solve, plain vs warm-start (speedup)",
           "value": float(np.exp(np.mean(np.log(sp)))), "unit": "x", "n_gpus": 1, "steps": len(rows),
           "warmup": args.warmup, "ms_per_step": float(np.mean([r["warm_s"] for r in rows])) * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 solve, bf16 network",
           "data": "synthetic (held-out seeded Voronoi images)",
           "config": {"workload": "warmstart1024_rgb_r5_k50", "H": 1024, "W": 1024, "C": 3, "R": 5, "K": 50,
                      "stop": "gap 1e-2, M <= 20, P = 10", "weights": "wsnet_k50.npy",
                      "warm_start": "predicted multiplier, cold controls"},
           "speedup_median": float(np.median(sp)), "fallbacks": int(sum(r["fallback"] for r in rows)),
           "plain_ms_mean": float(np.mean([r["cold_s"] for r in rows])) * 1e3, "rows": rows}
    print(json.dumps(out), flush=True)
    return 0


def bench_segment(args) -> int:
    """Segmentation scores of Sec. 4.4 on the solved bench image: one step = watershed
    labelling of the processed field plus IRV / IRC / VS against the input."""
    import torch

    import paper_2510_16154_amd as A
    from paper_2510_16154_amd.workloads import VORONOI512 as wl

    dev = torch.device("cuda:0")
    c0n = wl.image()
    c0 = torch.as_tensor(c0n, device=dev)
    solved = A.abc_solve(c0, wl.params(max_outer=3, max_inner=5, tol_alm=0.0))["c"].contiguous()
    H, W, C = solved.shape
    ws = torch.empty(A.abc_segment_workspace_bytes(H, W, C), dtype=torch.uint8, device=dev)
    for _ in range(args.warmup):
        A.abc_segment(solved, c0, 0.02, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st = A.abc_segment(solved, c0, 0.02, ws=ws)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    out = {"metric": "megapixels/sec (watershed + IRV/IRC/VS)", "value": H * W / t / 1e6, "unit": "Mpx/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 relief, f64 scores",
           "data": "synthetic (seeded Voronoi image, solved 3 x 5 iterations)",
           "config": {"workload": "segment512_rgb", "H": H, "W": W, "C": C, "theta": 0.02},
           "scores": {k: st[k] for k in ("k", "rounds", "irv", "irc", "vs")}}
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        cn = solved.cpu().numpy()
        reps, t1 = 0, time.perf_counter()
        while True:
            O.segment(cn, c0n, 0.02)
            reps += 1
            dt = time.perf_counter() - t1
            if dt >= min(args.cpu_min_seconds, 10.0):
                break
        out["cpu_baseline"] = {"value": H * W * reps / dt / 1e6, "unit": "Mpx/s", "cores": 1, "kind": "oracle",
                               "sample": f"{reps} x watershed + scores of the same {H}x{W}x{C} field, {dt:.1f} s"}
    print(json.dumps(out), flush=True)
    return 0


def cpu_baseline(c0n, wl, min_seconds: float):
    """The FP64 oracle on the host cores: full forward + adjoint sweeps (K Euler
    steps each) of the benchmark image, repeated until `min_seconds` passed, then
    the same sweeps on one thread over a 128 x 128 crop.  Returns the baseline
    and the oracle's (forward, adjoint) sweep seconds at all threads."""
    from oracle import oracle as O
    P = O.Params(K=wl.K, R=wl.R)
    eps = np.full((wl.K, 2), 57.0)
    pK = np.random.default_rng(0).normal(size=c0n.shape)
    reps, t_f, t_a = 0, 0.0, 0.0
    t0 = time.perf_counter()
    while True:
        t1 = time.perf_counter()
        traj = O.forward_sweep(c0n, P, eps)
        t2 = time.perf_counter()
        O.adjoint_sweep(traj, P, pK, eps)
        t_f += t2 - t1
        t_a += time.perf_counter() - t2
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
    out = {"value": wl.H * wl.W * wl.K * reps / dt, "unit": "agent-steps/s", "cores": O.num_threads(),
           "kind": "oracle",
           "sample": f"{reps} x (forward + adjoint sweep, {wl.K} Euler steps) of the {wl.H}x{wl.W}x{wl.C} "
                     f"image, R={wl.R}, FP64, {dt:.1f} s"}
    crop = np.ascontiguousarray(c0n[192:320, 192:320])
    pc = pK[192:320, 192:320].copy()
    n_all = O.num_threads()
    O.set_num_threads(1)
    try:
        reps1, t0 = 0, time.perf_counter()
        while True:
            tr = O.forward_sweep(crop, P, eps)
            O.adjoint_sweep(tr, P, pc, eps)
            reps1 += 1
            dt1 = time.perf_counter() - t0
            if dt1 >= min_seconds / 2:
                break
    finally:
        O.set_num_threads(n_all)
    out["single_thread"] = {"value": 128 * 128 * wl.K * reps1 / dt1, "unit": "agent-steps/s", "cores": 1,
                            "sample": f"{reps1} x (forward + adjoint sweep, {wl.K} Euler steps) of a 128x128 crop, "
                                      f"{dt1:.1f} s"}
    return out, (t_f / reps, t_a / reps)


if __name__ == "__main__":
    sys.exit(main())
