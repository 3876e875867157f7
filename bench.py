#!/usr/bin/env python
"""Benchmark: H-LU setup time and truncated updates/s on one MI355X.

A step is one complete H-LU factorisation (all work of the hot path: the
H x thin-dense products, the truncated additions, merges, leaf LUs and solves)
of the 7-point Laplacian on a 32^3 grid (n = 32768, leaf 64, eta 2,
eps = 1e-6), with the updates gathered in accumulators (the paper's method)
and executed as level-wise batched launches.  The factorised matrix is reset
from a device-resident copy before every step, outside the timed region.

Prints one JSON line.  `value` is truncated updates per second of the whole
factorisation (executed truncations / H-LU seconds); the H-LU seconds, the
plain per-update (standard) path and the per-kernel timings are extra fields.
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(cfg, mode, eps):
    """The oracle on a bounded sample: H-LU of the leading diagonal block at
    depth 4 of the same matrix (2048 unknowns for the 32^3 grid)."""
    import oracle
    from paper_1703_09085_amd import workloads as W

    x = W.grid_points(cfg["dims"])
    rp, ci, v = W.laplacian_csr(cfg["dims"])
    H = oracle.HMatrix.from_csr(x, rp, ci, v, cfg["leaf"], cfg["eta"])
    depth = 4
    t = time.perf_counter()
    size, st = H.lu_sub(depth, eps, mode)
    dt = time.perf_counter() - t
    tr = st["trunc_update"] + st["trunc_accum"] + st["trunc_merge"]
    return {"value": tr / dt, "unit": "updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{mode} H-LU of the leading {size}x{size} diagonal block (depth {depth}) of the same "
                      f"matrix, eps {eps:g}: {tr} truncations in {dt:.2f} s, single-threaded FP64 oracle"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="lap3d_32")
    ap.add_argument("--mode", default="accumulated", choices=["accumulated", "standard"])
    ap.add_argument("--no-compare", action="store_true", help="skip the standard-path comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    cfg = W.CONFIGS[args.config]
    if cfg["kind"] != "laplace":
        raise SystemExit(f"config {args.config} is not an H-LU workload")
    dims, leaf, eta, eps = cfg["dims"], cfg["leaf"], cfg["eta"], cfg["eps"]
    n = 1
    for d in dims:
        n *= d
    kmax = KMAX[len(dims)]
    ctx = hm.Context()
    x = W.grid_points(dims)
    rp, ci, v = W.laplacian_csr(dims)
    G0 = hm.HMatrix.from_csr(ctx, x, rp, ci, v, leaf, eta, kmax=kmax)
    G = G0.clone()

    def make_plan(mode, profile):
        # HIP events around every launch (per-kind kernel times) only in the
        # profiled plan: the timed steps run without them
        os.environ["HM_PROFILE_OPS"] = "1" if profile else "0"
        t = time.perf_counter()
        plan = hm.Plan.lu(ctx, G, mode)
        return plan, time.perf_counter() - t

    def run_path(mode, steps, warmup):
        plan, plan_s = make_plan(mode, False)
        for _ in range(warmup):
            G.copy_from(G0)
            plan.run(eps)
        wall, infos = [], []
        for _ in range(steps):
            G.copy_from(G0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = plan.run(eps)
            torch.cuda.synchronize()
            wall.append(time.perf_counter() - t0)
            infos.append(info)
        del plan
        # one more run with per-launch events for the kernel times
        plan, _ = make_plan(mode, True)
        G.copy_from(G0)
        prof = plan.run(eps)
        torch.cuda.synchronize()
        del plan
        return plan_s, wall, infos, prof

    log(f"[bench] {args.config}: n={n} leaf={leaf} eps={eps:g} mode={args.mode}")
    plan_s, wall, infos, prof = run_path(args.mode, args.steps, args.warmup)
    last = infos[-1]
    trunc = sum(i["truncations"] for i in infos)
    ms_per_step = 1e3 * sum(wall) / args.steps
    value = trunc / sum(wall)
    log(f"[bench] {args.mode}: {ms_per_step:.1f} ms/step (steps {', '.join(f'{1e3 * w:.1f}' for w in wall)}), "
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

    compare = None
    if not args.no_compare:
        other = "standard" if args.mode == "accumulated" else "accumulated"
        p2, w2, inf2, prof2 = run_path(other, 1, 0)
        compare = {"mode": other, "h_lu_seconds": w2[0], "truncations": inf2[-1]["truncations"],
                   "updates_per_s": inf2[-1]["truncations"] / w2[0], "plan_seconds": p2,
                   "speedup_of_headline_path": w2[0] / (sum(wall) / args.steps),
                   "kernel_seconds": prof2["op_seconds"]}
        log(f"[bench] {other}: {1e3 * w2[0]:.1f} ms, {inf2[-1]['truncations']} truncations")

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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"H-LU ({args.mode} updates, level-batched FP64) of the 7-point Laplacian on a "
                               f"{'x'.join(map(str, dims))} grid, n={n}, leaf {leaf}, eta {eta:g}, eps {eps:g}",
                   "n": n, "leaf": leaf, "eta": eta, "eps": eps, "kmax": kmax, "mode": args.mode,
                   "precision": "fp64"},
        "h_lu_setup_s": sum(wall) / args.steps,
        "h_lu_setup_s_per_dof": sum(wall) / args.steps / n,
        "h_lu_device_s": sum(i["run_seconds"] for i in infos) / args.steps,
        "plan_s": plan_s,
        "truncations_per_step": last["truncations"],
        "updates_per_trunc_kernel_second": last["truncations"] / (t_small + t_general) if t_small + t_general else None,
        "waves": last["waves"],
        "launches": last["launches"],
        "kernel_seconds_per_step": ops,
        "trunc_kernels": kernels,
        "dominant_kernel": dominant,
        "roofline": roofline,
        "compare": compare,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
