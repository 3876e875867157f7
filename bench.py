#!/usr/bin/env python
"""Benchmark: H-LU setup time and truncated updates/s on one MI355X.

A step is one complete H-LU factorisation (all work of the hot path: the
H x thin-dense products, the truncated additions, merges, leaf LUs and solves)
of the 7-point Laplacian on a 32^3 grid (n = 32768, leaf 64, eta 2,
eps = 1e-6).  The headline path is the one the metric names: updates gathered
in accumulators (the paper's method), the dense products and the small-block
truncations' stacked-factor products in split-BF16x3 on the matrix cores
(FP64 storage, cores and leaf LU), independent items batched into one launch
per kind, in the dataflow schedule (launches on four streams, each waiting by
events only for the launches it depends on).  Beside it: the plain FP64
per-update (standard) path in dependency waves, launch by launch; the headline
path in dependency waves replayed from a hipGraph; the accumulated path in
FP64; the standard path with the headline precision and schedule.  The factorised matrix is reset from a device-resident copy
before every step, outside the timed region.

`--config lap2d_batch64` runs 64 independent H-LUs of 2D Laplacians (sides
drawn from 32..128) as one batched plan instead.

Prints one JSON line.  `value` is truncated updates per second of the whole
factorisation (executed truncations / H-LU seconds); the H-LU seconds, the
comparison paths and the per-kernel timings are extra fields.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

KMAX = {2: 64, 3: 96}
HBM_PEAK_GBS = 8000.0
DTYPES = {"fp64": "f64", "fp32": "f32 products, f64 storage and cores",
          "bf16x3": "bf16x3 (MFMA, f32 accumulate) products, f64 storage and cores"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(cfg, mode, eps):
    """The oracle on a bounded sample: H-LU of the leading diagonal block at
    depth 4 of the same matrix (2048 unknowns for the 32^3 grid)."""
    import oracle
    from paper_1703_09085_amd import workloads as W

    if cfg["kind"] == "laplace_batch":
        side = int(W.batch_sides(cfg["count"], cfg["side_lo"], cfg["side_hi"], cfg["seed"])[0])
        dims, depth = (side, side), 0
    else:
        dims, depth = cfg["dims"], 4
    x = W.grid_points(dims)
    rp, ci, v = W.laplacian_csr(dims)
    H = oracle.HMatrix.from_csr(x, rp, ci, v, cfg["leaf"], cfg["eta"])
    t = time.perf_counter()
    size, st = H.lu_sub(depth, eps, mode)
    dt = time.perf_counter() - t
    tr = st["trunc_update"] + st["trunc_accum"] + st["trunc_merge"]
    what = (f"the leading {size}x{size} diagonal block (depth {depth}) of the same matrix" if depth else
            f"the first instance of the batch ({dims[0]}x{dims[1]} grid, n={size})")
    return {"value": tr / dt, "unit": "updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{mode} H-LU of {what}, eps {eps:g}: {tr} truncations in {dt:.2f} s, "
                      f"single-threaded FP64 oracle"}


def train_predictor(hm, ctx, W, eps):
    """Rank predictor trained on the GPU from the features and exact ranks
    that H-LU runs of smaller Laplacians log (outside the timed region)."""
    import numpy as np
    import torch

    g = torch.Generator().manual_seed(1703)
    omega = torch.randn(32, 64, generator=g, dtype=torch.float64).cuda()
    net = hm.MLP(ctx, seed=3)
    os.environ["HM_TRUNC_LOG"] = "1"
    os.environ["HM_FEATURE_LOG"] = "1"
    X, t = [], []
    for dims, leaf in (((64, 64), 32), ((16, 16, 16), 32)):
        for mode in ("standard", "accumulated"):
            x = W.grid_points(dims)
            rp, ci, v = W.laplacian_csr(dims)
            G = hm.HMatrix.from_csr(ctx, x, rp, ci, v, leaf, 2.0, kmax=KMAX[len(dims)])
            plan = hm.Plan.lu(ctx, G, mode).set_predictor(net, omega, 8, 0)
            plan.run(eps)
            f, lg = plan.feature_log(), plan.trunc_log()
            sel = np.isfinite(f[:, 0]) & (lg[:, 0] > 0)
            X.append(f[sel, :8])
            t.append(np.log2(1.0 + lg[sel, 3]).astype(np.float32))
            del plan
    os.environ["HM_TRUNC_LOG"] = "0"
    os.environ["HM_FEATURE_LOG"] = "0"
    X, t = np.concatenate(X), np.concatenate(t)
    perm = np.random.default_rng(0).permutation(len(X))
    losses = net.train(torch.from_numpy(np.ascontiguousarray(X[perm])).cuda(), torch.from_numpy(t[perm]).cuda(),
                       epochs=60, batch=512, lr=2e-3)
    return net, omega, {"samples": int(len(X)), "loss_first_epoch": float(losses[0]),
                        "loss_last_epoch": float(losses[-1])}


def trunc_throughput(hm, W, torch, args):
    """One full batch of identical independent truncations through hm_trunc_batch: the kernels' throughput
    when every CU is busy (the H-LU launches carry tens of items)."""
    m, n, l, count = (int(v) for v in args.trunc_throughput.split(","))
    k1 = l // 2
    k2 = l - k1
    ctx = hm.Context()
    A, B = W.lowrank_factors(m, n, k1, seed=5, decay=0.45)
    C_, D = W.lowrank_factors(m, n, k2, seed=6, decay=0.45, scale=0.7)
    dev = [torch.from_numpy(x.T.copy()).cuda() for x in (A, B, C_, D)]  # column-major storage
    kcap = min(m, n, l)
    Co = torch.zeros((count, kcap, m), dtype=torch.float64, device="cuda")
    Do = torch.zeros((count, kcap, n), dtype=torch.float64, device="cuda")
    rk = torch.zeros(count, dtype=torch.int32, device="cuda")
    descs = [hm.TruncDesc(m=m, n=n, k1=k1, k2=k2, kcap=kcap, lda=m, ldb=n, ldc=m, ldd=n, alpha=-0.9,
                          A=dev[0].data_ptr(), B=dev[1].data_ptr(), C=dev[2].data_ptr(), D=dev[3].data_ptr(),
                          Cout=Co[i].data_ptr(), Dout=Do[i].data_ptr(), rank_out=rk[i:i + 1].data_ptr())
             for i in range(count)]
    ctx.trunc_batch(descs, 1e-6, precision=args.precision)  # warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(max(args.steps, 1)):
        t0 = time.perf_counter()
        ctx.trunc_batch(descs, 1e-6, precision=args.precision)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    k = int(rk[0].item())
    dt = min(times)
    nbytes = 8 * (m + n) * (l + k) * count
    print(json.dumps({"metric": "truncations/s of one full hm_trunc_batch", "value": count / dt, "unit": "truncations/s",
                      "m": m, "n": n, "l": l, "k": k, "count": count, "precision": args.precision, "seconds": dt,
                      "algorithmic_GB_per_s": nbytes / dt / 1e9, "hbm_frac": nbytes / dt / 1e9 / HBM_PEAK_GBS}),
          flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="lap3d_32")
    ap.add_argument("--mode", default="accumulated", choices=["accumulated", "standard"])
    ap.add_argument("--precision", default="bf16x3", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--no-graph", action="store_true", help="run the headline path launch by launch")
    ap.add_argument("--schedule", default="dataflow", choices=["dataflow", "waves"],
                    help="execution order of the headline path: dataflow (four streams, event dependencies) "
                         "or dependency waves (replayed from a hipGraph unless --no-graph)")
    ap.add_argument("--predictor", action="store_true",
                    help="train the rank predictor first and attach it to the headline path")
    ap.add_argument("--no-compare", action="store_true", help="skip the comparison paths")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--trunc-throughput", default="", metavar="M,N,L,COUNT",
                    help="only time one hm_trunc_batch of COUNT independent M x N truncations of stacked rank L "
                         "(two factor pairs of L/2 columns, singular values decaying by 0.45) and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times) and exit: the reference "
                         "kernel for scaling FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the path is built and measured on a "
              "single GPU; its multi-GPU sharding is a design, not code", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "repeats": 5}), flush=True)
        return

    from paper_1703_09085_amd import hm
    from paper_1703_09085_amd import workloads as W

    if args.trunc_throughput:
        trunc_throughput(hm, W, torch, args)
        return

    cfg = W.CONFIGS[args.config]
    if cfg["kind"] not in ("laplace", "laplace_batch"):
        raise SystemExit(f"config {args.config} is not an H-LU workload")
    leaf, eta, eps = cfg["leaf"], cfg["eta"], cfg["eps"]
    ctx = hm.Context()
    if cfg["kind"] == "laplace":
        problems = [tuple(cfg["dims"])]
    else:
        problems = [(int(s), int(s)) for s in W.batch_sides(cfg["count"], cfg["side_lo"], cfg["side_hi"],
                                                            cfg["seed"])]
    n_total = 0
    G0, G = [], []
    for dims in problems:
        x = W.grid_points(dims)
        rp, ci, v = W.laplacian_csr(dims)
        g = hm.HMatrix.from_csr(ctx, x, rp, ci, v, leaf, eta, kmax=KMAX[len(dims)])
        G0.append(g)
        G.append(g.clone())
        n_total += x.shape[0]
    if cfg["kind"] == "laplace":
        dims = problems[0]
        workload = (f"H-LU of the 7-point Laplacian on a {'x'.join(map(str, dims))} grid, n={n_total}, leaf {leaf}, "
                    f"eta {eta:g}, eps {eps:g}" if len(dims) == 3 else
                    f"H-LU of the 5-point Laplacian on a {'x'.join(map(str, dims))} grid, n={n_total}, leaf {leaf}, "
                    f"eta {eta:g}, eps {eps:g}")
    else:
        workload = (f"{len(problems)} independent H-LUs of 5-point Laplacians on NxN grids, N drawn uniformly from "
                    f"{cfg['side_lo']}..{cfg['side_hi']} (seed {cfg['seed']}), total n={n_total}, leaf {leaf}, "
                    f"eta {eta:g}, eps {eps:g}, one batched plan")

    def reset():
        for a, b in zip(G, G0):
            a.copy_from(b)

    net = omega = pred_info = None
    if args.predictor:
        t = time.perf_counter()
        net, omega, pred_info = train_predictor(hm, ctx, W, eps)
        pred_info["train_seconds"] = time.perf_counter() - t
        log(f"[bench] predictor trained on {pred_info['samples']} logged truncations "
            f"in {pred_info['train_seconds']:.1f} s")

    def make_plan(mode, prec, graph, pred, profile, schedule):
        # HIP events around every launch (per-kind kernel times) only in the
        # profiled plan: the timed steps run without them
        os.environ["HM_PROFILE_OPS"] = "1" if profile else "0"
        ctx.set_schedule(schedule)
        t = time.perf_counter()
        plan = hm.Plan.lu(ctx, G[0], mode) if len(G) == 1 else hm.Plan.lu_batch(ctx, G, mode)
        plan.set_precision(prec)
        if graph and not profile:
            plan.use_graph()  # the library replays only wave plans from a graph
        if pred:
            plan.set_predictor(net, omega, 2, 1)
        return plan, time.perf_counter() - t

    def run_path(mode, prec, graph, pred, steps, warmup, schedule, profile=True):
        plan, plan_s = make_plan(mode, prec, graph, pred, False, schedule)
        for _ in range(warmup):
            reset()
            plan.run(eps)
        wall, infos = [], []
        for _ in range(steps):
            reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = plan.run(eps)
            torch.cuda.synchronize()
            wall.append(time.perf_counter() - t0)
            infos.append(info)
            assert info["status_bits"] == 0, info["status_bits"]
        del plan
        prof = None
        if profile:
            # one more run with per-launch events for the kernel times
            plan, _ = make_plan(mode, prec, False, pred, True, schedule)
            reset()
            prof = plan.run(eps)
            torch.cuda.synchronize()
            del plan
        return plan_s, wall, infos, prof

    graph = not args.no_graph
    path = {"mode": args.mode, "precision": args.precision, "batched_launches": True, "schedule": args.schedule,
            "hip_graph": graph, "rank_predictor": args.predictor}
    log(f"[bench] {args.config}: n={n_total} leaf={leaf} eps={eps:g} {path}")
    plan_s, wall, infos, prof = run_path(args.mode, args.precision, graph, args.predictor, args.steps, args.warmup,
                                         args.schedule)
    last = infos[-1]
    # the plan falls back to waves when its temporaries exceed the budget;
    # graph replay applies to wave plans only
    path["schedule"] = last["schedule"]
    path["hip_graph"] = graph and last["schedule"] == "waves"
    trunc = sum(i["truncations"] for i in infos)
    ms_per_step = 1e3 * sum(wall) / args.steps
    value = trunc / sum(wall)
    log(f"[bench] headline: {ms_per_step:.1f} ms/step (steps {', '.join(f'{1e3 * w:.1f}' for w in wall)}), "
        f"{last['truncations']} truncations, plan {plan_s:.1f} s")

    # roofline of the dominant truncation kernel, from the profiled run: the
    # small-block kernel (m, n <= 64) or the register-resident + general kernels
    ops = prof["op_seconds"]
    t_small = prof["small_trunc_seconds"]
    t_general = ops["trunc"] - t_small
    b_small = prof["small_trunc_bytes"]
    b_general = prof["trunc_bytes"] - b_small
    kernels = {
        "trunc_small_kernel": {"seconds": t_small, "bytes": b_small, "launches": prof["small_trunc_launches"]},
        "trunc_tall_kernel+trunc_kernel": {"seconds": t_general, "bytes": b_general,
                                           "launches": prof["general_trunc_launches"]},
    }
    for kv in kernels.values():
        kv["GB_per_s"] = kv["bytes"] / kv["seconds"] / 1e9 if kv["seconds"] > 0 else 0.0
        kv["avg_launch_us"] = 1e6 * kv["seconds"] / kv["launches"] if kv["launches"] else 0.0
        kv["bytes_per_launch"] = kv["bytes"] / kv["launches"] if kv["launches"] else 0.0
    dominant = max(kernels, key=lambda k: kernels[k]["seconds"])
    dk = kernels[dominant]
    roofline = {"kernel": dominant, "bound": "hbm", "achieved": round(dk["GB_per_s"], 3), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": dk["GB_per_s"] / HBM_PEAK_GBS, "traffic": None,
                "algorithmic_bytes_per_launch": dk["bytes_per_launch"], "avg_launch_us": dk["avg_launch_us"],
                "launches_per_step": dk["launches"], "per_unit": "8 (m+n)(l+k) bytes per executed truncation"}

    compare = []
    if not args.no_compare:
        sch = args.schedule
        legs = [("plain FP64 per-update path (standard updates, dependency waves, launch by launch)", "standard",
                 "fp64", False, "waves"),
                ("headline updates and precision, dependency waves replayed from a hipGraph", args.mode,
                 args.precision, True, "waves"),
                ("accumulated updates in FP64, same batching and schedule", args.mode, "fp64", graph, sch),
                ("standard updates with the headline precision, batching and schedule", "standard", args.precision,
                 graph, sch)]
        for name, mode, prec, gr, sc in legs:
            if (mode, prec, gr, sc) == (args.mode, args.precision, graph, sch):
                continue
            p2, w2, inf2, _ = run_path(mode, prec, gr, False, 1, 1, sc, profile=False)
            compare.append({"path": name, "mode": mode, "precision": prec,
                            "hip_graph": gr and inf2[-1]["schedule"] == "waves", "schedule": inf2[-1]["schedule"],
                            "h_lu_seconds": w2[0], "truncations": inf2[-1]["truncations"],
                            "updates_per_s": inf2[-1]["truncations"] / w2[0], "plan_seconds": p2,
                            "headline_speedup": w2[0] / (sum(wall) / args.steps)})
            log(f"[bench] {name}: {1e3 * w2[0]:.1f} ms, {inf2[-1]['truncations']} truncations")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg, args.mode, eps)
        log(f"[bench] cpu baseline: {cpu['value']:.1f} updates/s")

    out = {
        "metric": "H-LU setup s & truncated updates/s at eps=1e-6: mixed+batched vs plain FP64",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[args.precision],
        "data": "synthetic",
        "config": {"workload": workload, "n": n_total, "leaf": leaf, "eta": eta, "eps": eps, **path},
        "h_lu_setup_s": sum(wall) / args.steps,
        "h_lu_setup_s_per_dof": sum(wall) / args.steps / n_total,
        "h_lu_device_s": sum(i["run_seconds"] for i in infos) / args.steps,
        "plan_s": plan_s,
        "h_lu_one_shot_s": plan_s + sum(wall) / args.steps,
        "truncations_per_step": last["truncations"],
        "predicted_truncations": last["predicted"],
        "predicted_fallbacks": last["predicted_fallback"],
        "updates_per_trunc_kernel_second": last["truncations"] / (t_small + t_general) if t_small + t_general else None,
        "waves": last["waves"],
        "launches": last["launches"],
        "temp_bytes": last["temp_bytes"],
        "workspace_bytes": last["workspace_bytes"],
        "kernel_seconds_per_step": ops,
        "trunc_kernels": kernels,
        "dominant_kernel": dominant,
        "roofline": roofline,
        "compare": compare,
        "predictor": pred_info,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
