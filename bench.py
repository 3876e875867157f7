#!/usr/bin/env python
"""Benchmark: H-LU setup time and truncated updates/s on one MI355X.

Default workload: 64 independent H-LUs of 5-point Laplacians on N x N grids,
N drawn uniformly from 32..128 (seed 4), leaf 32, eta 2, eps 1e-6, total
n = 525,408 -- the largest of the eps = 1e-6 H-LU workloads that runs on one
GPU -- factorised by one batched plan.  `--config lap3d_32` runs the 7-point
Laplacian on 32^3 (n = 32768, leaf 64) instead.

A step is one complete batched H-LU (every item of the hot path: the H x
thin-dense products, the truncated additions, merges, leaf LUs and solves)
with the plan recorded once and replayed; the matrices are reset from
device-resident copies before every step, outside the timed region.  The
headline path is the one the metric names: updates gathered in accumulators
(the paper's method), split-BF16x3 products on the matrix cores (FP64 storage,
cores and leaf LU), independent items batched into one launch per kind.
Beside it (compare): the plain FP64 per-update (standard) path in dependency
waves, launch by launch, and the other mode / precision combinations.

Reported besides `value` (executed truncations per second of the timed
steps): the one-shot H-LU setup time (hm_lu: planning included), the
planning time, per-kernel device times from a profiled run in dependency
waves (each kernel's launches never overlap each other there), the roofline
of the dominant truncation kernel (algorithmic bytes per launch over its
average launch time; HBM traffic per launch from the committed rocprofv3
counter summary when the kernel sources still match it), a roofline per
stacked-rank bucket from full batches of independent truncations, and the
CPU oracle on a sample of the same workload.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

KMAX = {2: 64, 3: 96}
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
DTYPES = {"fp64": "f64", "fp32": "f32 products, f64 storage and cores",
          "bf16x3": "bf16x3 (MFMA, f32 accumulate) products, f64 storage and cores"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")
KERNEL_SOURCES = {
    "trunc_small_kernel": ["trunc_small.hip", "tiny.h", "core.h", "mixed.h", "dev_util.h", "hm_types.h"],
    "trunc_tall_kernel+trunc_kernel": ["trunc_tall.hip", "tall.h", "trunc.hip", "core.h", "dev_util.h",
                                       "hm_types.h"],
    "trunc_thin_kernel": ["trunc_thin.hip", "tiny.h", "core.h", "dev_util.h", "hm_types.h"],
}
# buckets of the per-bucket roofline, (m, n, l, count): the block sizes of the
# batched H-LU's truncations with stacked ranks typical of each (the larger
# blocks' stacked ranks there are at most 16, most of them at most 8), and the
# 128 x 128, l = 40 batch of earlier measurements
BUCKETS = [(32, 32, 24, 16384), (64, 64, 24, 8192), (64, 64, 48, 8192), (128, 128, 6, 8192), (256, 256, 6, 4096),
           (512, 512, 6, 2048), (1024, 1024, 6, 1024), (128, 128, 40, 4096)]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sources_sha(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1703_09085_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(cfg, mode, eps):
    """The oracle (single-threaded FP64) on a bounded sample of the same
    workload, median of three runs: the first instance of the batch, or the
    leading diagonal block at depth 2 of the 3D grid (8192 unknowns)."""
    import oracle
    from paper_1703_09085_amd import workloads as W

    if cfg["kind"] == "laplace_batch":
        sides = [int(s) for s in W.batch_sides(cfg["count"], cfg["side_lo"], cfg["side_hi"], cfg["seed"])[:1]]
        problems, depth = [(s, s) for s in sides], 0
    else:
        problems, depth = [tuple(cfg["dims"])], 2
    runs = []
    for _ in range(3):
        tr, dt, size = 0, 0.0, 0
        for dims in problems:
            x = W.grid_points(dims)
            rp, ci, v = W.laplacian_csr(dims)
            H = oracle.HMatrix.from_csr(x, rp, ci, v, cfg["leaf"], cfg["eta"])
            t = time.perf_counter()
            sz, st = H.lu_sub(depth, eps, mode)
            dt += time.perf_counter() - t
            size += sz
            tr += st["trunc_update"] + st["trunc_accum"] + st["trunc_merge"]
        runs.append((dt, tr, size))
    dts = sorted(r[0] for r in runs)
    dt, tr, size = dts[1], runs[0][1], runs[0][2]
    if depth:
        what = f"the leading {size}x{size} diagonal block (depth {depth}) of the same matrix"
    else:
        what = f"the first instance of the batch ({problems[0][0]}x{problems[0][1]} grid, n={size})"
    return {"value": tr / dt, "unit": "updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{mode} H-LU of {what}, eps {eps:g}: {tr} truncations, median of 3 runs {dt:.2f} s "
                      f"(runs {', '.join(f'{d:.2f}' for d in dts)}), single-threaded FP64 oracle (g++ -O3)",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "seconds": dt, "truncations": tr}


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


def trunc_batch_time(hm, W, torch, ctx, m, n, l, count, precision, steps, shapes=None):
    """Device seconds of one batch of `count` identical independent m x n
    truncations of stacked rank l (two factor pairs, singular values decaying
    by 0.45) through hm_trunc_batch_device, best of `steps`; returns (seconds,
    k).  With shapes, a list of (m, n, l, count), one batch holds all of them
    (k of the first shape)."""
    shapes = shapes or [(m, n, l, count)]
    descs, keep, ranks = [], [], []
    for m, n, l, count in shapes:
        k1 = l // 2
        k2 = l - k1
        A, B = W.lowrank_factors(m, n, k1, seed=5, decay=0.45)
        C_, D = W.lowrank_factors(m, n, k2, seed=6, decay=0.45, scale=0.7)
        # every item reads its own copy of the factors (column-major storage), so
        # that the batch streams its inputs from HBM as the H-LU's items do
        dev = [torch.from_numpy(x.T.copy()).cuda().unsqueeze(0).repeat(count, 1, 1) for x in (A, B, C_, D)]
        kcap = min(m, n, l)
        Co = torch.zeros((count, kcap, m), dtype=torch.float64, device="cuda")
        Do = torch.zeros((count, kcap, n), dtype=torch.float64, device="cuda")
        rk = torch.zeros(count, dtype=torch.int32, device="cuda")
        descs += [hm.TruncDesc(m=m, n=n, k1=k1, k2=k2, kcap=kcap, lda=m, ldb=n, ldc=m, ldd=n, alpha=-0.9,
                               A=dev[0][i].data_ptr(), B=dev[1][i].data_ptr(), C=dev[2][i].data_ptr(),
                               D=dev[3][i].data_ptr(), Cout=Co[i].data_ptr(), Dout=Do[i].data_ptr(),
                               rank_out=rk[i:i + 1].data_ptr())
                  for i in range(count)]
        keep.append((dev, Co, Do))
        ranks.append(rk)
    # the descriptors go to the device once (hm_trunc_batch_device), the
    # batch's buffers come from torch's caching allocator, and HIP events on
    # the context's stream time each call: the figure holds the device's work
    # of one batch (clearing the counters, lowering the descriptors, the
    # truncation kernels), not Python's, hipMalloc's or the descriptor copy's
    arr = hm.Context.desc_array(descs)
    ddev = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).cuda()
    max_rows = max(max(sm, sn) for sm, sn, _, _ in shapes)
    max_stack = max(sl for _, _, sl, _ in shapes)
    bctx = hm.Context(allocator="torch")

    def one():
        bctx.trunc_batch_device(ddev, len(arr), max_rows, max_stack, 1e-6, precision=precision)

    one()  # warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(max(steps, 1)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(bctx.stream)
        one()
        e1.record(bctx.stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    if len(shapes) > 1:
        return min(times), [int(r[0].item()) for r in ranks]
    return min(times), int(ranks[0][0].item())


def bucket_roofline(hm, W, torch, ctx, precision):
    """Roofline per stacked-rank bucket: one full batch of independent
    truncations per (m, n, l); algorithmic bytes 8 (m + n)(l + k) per item and
    flops 2 (m + n) l^2 (the stacks' QR) + 12 q^3 (the core SVD, q =
    min(m, n, l)) + 2 (m + n) l k (the rebuild); attainable = min(FP64 peak,
    HBM peak x flop/byte)."""
    out = []
    for m, n, l, count in BUCKETS:
        dt, k = trunc_batch_time(hm, W, torch, ctx, m, n, l, count, precision, 2)
        nbytes = 8 * (m + n) * (l + k) * count
        q = min(m, n, l)
        flops = (2 * (m + n) * l * l + 12 * q ** 3 + 2 * (m + n) * l * k) * count
        gbs = nbytes / dt / 1e9
        intensity = flops / nbytes
        attainable = min(FP64_PEAK_TFLOPS * 1e3, HBM_PEAK_GBS * intensity)  # GFLOP/s
        out.append({"m": m, "n": n, "l": l, "k": k, "count": count, "precision": precision, "seconds": dt,
                    "truncations_per_s": count / dt, "GB_per_s": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                    "GFLOP_per_s": flops / dt / 1e9, "flop_per_byte": intensity,
                    "attainable_GFLOP_per_s": attainable, "frac_of_attainable": flops / dt / 1e9 / attainable})
        log(f"[bench] bucket {m}x{n} l={l}: {count / dt:,.0f} truncations/s, {gbs:.1f} GB/s "
            f"({100 * gbs / HBM_PEAK_GBS:.2f}% of HBM)")
    return out


def bem_experiments(hm, W, torch, m, modes, precision, steps, ops=None):
    """The arithmetic of the paper's boundary-element experiments (Sect. 7) on
    the GPU: single layer V and double layer K on the refined double pyramid
    (n = 8 m^2), eps 1e-4, leaf 64, rank capacity 128; V V, the inverse and
    the Cholesky factor of V, K K, the inverse and the LU of K, each with a reusable plan (best of `steps`
    runs) and once through the one-shot entry point (planning included)."""
    eps, leaf = 1e-4, 64
    ctx = hm.Context()
    T = W.double_pyramid_mesh(m)
    mats, out = {}, {"n": int(len(T)), "m": m, "eps": eps, "leaf": leaf, "precision": precision, "runs": []}
    for layer in ("single", "double"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        A = hm.HMatrix.from_bem(ctx, T, layer, leaf, 2.0, eps, kmax=128)
        torch.cuda.synchronize()
        b = A.blocks()
        adm = b["kind"] == 1
        out[f"build_{layer}_seconds"] = time.perf_counter() - t0
        out[f"build_{layer}_max_rank"] = int(b["rank"][adm].max())
        mats[layer] = A
        log(f"[bench] BEM {layer} layer n={len(T)}: built in {out[f'build_{layer}_seconds']:.2f} s, "
            f"{int(adm.sum())} admissible blocks, max rank {out[f'build_{layer}_max_rank']}")
    for op, layer in (("mul", "single"), ("inv", "single"), ("chol", "single"), ("mul", "double"),
                      ("inv", "double"), ("lu", "double")):
        if ops and op not in ops:
            continue
        A = mats[layer]
        for mode in modes:
            if op == "mul":
                Z0 = A.zeros_like()
                Z = A.zeros_like()
                target, source = Z, Z0
                make = lambda: hm.Plan.addmul(ctx, 1.0, A, A, Z, mode)  # noqa: E731
                one_shot = lambda: Z.addmul(1.0, A, A, eps, mode)  # noqa: E731
            else:
                G = A.clone()
                target, source = G, A
                make = lambda: getattr(hm.Plan, op)(ctx, G, mode)  # noqa: E731
                one_shot = lambda: getattr(G, op)(eps, mode)  # noqa: E731
            t0 = time.perf_counter()
            plan = make().set_precision(precision)
            plan_s = time.perf_counter() - t0
            best, info = None, None
            for _ in range(max(steps, 1)):
                target.copy_from(source)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = plan.run(eps)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                best = dt if best is None else min(best, dt)
                assert info["status_bits"] == 0, info["status_bits"]
            del plan
            target.copy_from(source)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info1 = one_shot()
            torch.cuda.synchronize()
            once = time.perf_counter() - t0
            rec = {"op": op, "layer": layer, "mode": mode, "plan_seconds": plan_s, "run_seconds": best,
                   "one_shot_seconds": once, "truncations": info["truncations"], "launches": info["launches"],
                   "schedule": info["schedule"], "updates_per_s": info["truncations"] / best}
            out["runs"].append(rec)
            log(f"[bench] BEM {op} {layer} {mode}: run {1e3 * best:.1f} ms, one-shot {once:.2f} s "
                f"(plan {plan_s:.2f} s), {info['truncations']} truncations, {info['launches']} launches")
    return out


def batch_shapes(b):
    """'M x N (l L) x COUNT' for the shapes of a counter batch."""
    shapes = b.get("shapes") or [[b["m"], b["n"], b["l"], b["count"]]]
    return " + ".join(f"{c} x ({m}x{n}, l={l})" for m, n, l, c in shapes)


def traffic_ratio(kernel):
    """HBM bytes over algorithmic bytes of `kernel`, measured by the committed
    counter passes on a full batch of the workload's item shape, or None when
    there is no entry or the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    e = data.get(kernel)
    if not e or e.get("sources_sha") != sources_sha(kernel):
        return None
    return e


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="lap2d_batch64")
    ap.add_argument("--mode", default="accumulated", choices=["accumulated", "standard", "fused"])
    ap.add_argument("--precision", default="bf16x3", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--no-graph", action="store_true", help="run the headline path launch by launch")
    ap.add_argument("--schedule", default="dataflow", choices=["dataflow", "waves"],
                    help="execution order of the headline path: dataflow (four streams, event dependencies; "
                         "plans too large for it run in waves) or dependency waves")
    ap.add_argument("--predictor", action="store_true",
                    help="train the rank predictor first and attach it to the headline path")
    ap.add_argument("--no-compare", action="store_true", help="skip the comparison paths")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-buckets", action="store_true", help="skip the per-bucket roofline")
    ap.add_argument("--profile-only", action="store_true",
                    help="one untimed run of the headline plan in dependency waves and exit (for profilers)")
    ap.add_argument("--trunc-throughput", default="", metavar="M,N,L,COUNT[;M,N,L,COUNT...]",
                    help="only time one hm_trunc_batch of COUNT independent M x N truncations of stacked rank L "
                         "(several shapes separated by ';' go into one batch) and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times) and exit: the reference "
                         "kernel for scaling FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--bem-experiments", type=int, default=0, metavar="M",
                    help="only run the boundary-element experiments (V V, inverse and Cholesky of V, K K, LU of K, "
                         "standard / accumulated / fused) on the double pyramid refined M times (n = 8 M^2) and exit")
    ap.add_argument("--bem-ops", default="mul,inv,chol,lu",
                    help="comma-separated subset of mul, inv, chol, lu for --bem-experiments")
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

    if args.bem_experiments:
        res = bem_experiments(hm, W, torch, args.bem_experiments, ["standard", "accumulated", "fused"],
                              args.precision, args.steps, ops=args.bem_ops.split(","))
        print(json.dumps({"metric": "boundary-element experiments", **res}), flush=True)
        return

    if args.trunc_throughput:
        shapes = [tuple(int(v) for v in part.split(",")) for part in args.trunc_throughput.split(";")]
        ctx = hm.Context()
        if len(shapes) == 1:
            m, n, l, count = shapes[0]
            dt, k = trunc_batch_time(hm, W, torch, ctx, m, n, l, count, args.precision, args.steps)
            nbytes = 8 * (m + n) * (l + k) * count
            print(json.dumps({"metric": "truncations/s of one full hm_trunc_batch", "value": count / dt,
                              "unit": "truncations/s", "m": m, "n": n, "l": l, "k": k, "count": count,
                              "precision": args.precision, "seconds": dt, "algorithmic_GB_per_s": nbytes / dt / 1e9,
                              "hbm_frac": nbytes / dt / 1e9 / HBM_PEAK_GBS}), flush=True)
        else:
            dt, ks = trunc_batch_time(hm, W, torch, ctx, 0, 0, 0, 0, args.precision, args.steps, shapes=shapes)
            nbytes = sum(8 * (m + n) * (l + k) * c for (m, n, l, c), k in zip(shapes, ks))
            count = sum(c for _, _, _, c in shapes)
            print(json.dumps({"metric": "truncations/s of one full hm_trunc_batch", "value": count / dt,
                              "unit": "truncations/s", "shapes": shapes, "k": ks, "count": count,
                              "precision": args.precision, "seconds": dt, "algorithmic_bytes": nbytes,
                              "algorithmic_GB_per_s": nbytes / dt / 1e9,
                              "hbm_frac": nbytes / dt / 1e9 / HBM_PEAK_GBS}), flush=True)
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
        stencil = "7-point" if len(dims) == 3 else "5-point"
        workload = (f"H-LU of the {stencil} Laplacian on a {'x'.join(map(str, dims))} grid, n={n_total}, "
                    f"leaf {leaf}, eta {eta:g}, eps {eps:g}")
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
            plan.use_graph()  # the library replays only wave plans of bounded size from a graph
        if pred:
            plan.set_predictor(net, omega, 2, 1)
        os.environ["HM_PROFILE_OPS"] = "0"
        return plan, time.perf_counter() - t

    def run_path(mode, prec, graph, pred, steps, warmup, schedule):
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
        return plan_s, wall, infos

    graph = not args.no_graph
    path = {"mode": args.mode, "precision": args.precision, "batched_launches": True, "schedule": args.schedule,
            "hip_graph": graph, "rank_predictor": args.predictor}
    log(f"[bench] {args.config}: n={n_total} leaf={leaf} eps={eps:g} {path}")
    if args.profile_only:
        plan, _ = make_plan(args.mode, args.precision, False, args.predictor, False, "waves")
        reset()
        info = plan.run(eps)
        torch.cuda.synchronize()
        log(f"[bench] profile run: {1e3 * info['run_seconds']:.1f} ms, {info['truncations']} truncations, "
            f"schedule {info['schedule']}, {info['launches']} launches")
        print(json.dumps({"profile_run_ms": 1e3 * info["run_seconds"], "truncations": info["truncations"],
                          "launches": info["launches"], "schedule": info["schedule"]}), flush=True)
        return

    plan_s, wall, infos = run_path(args.mode, args.precision, graph, args.predictor, args.steps, args.warmup,
                                   args.schedule)
    last = infos[-1]
    path["schedule"] = last["schedule"]
    path["hip_graph"] = bool(last["graph_replay"])  # replayed, not only requested
    trunc = sum(i["truncations"] for i in infos)
    ms_per_step = 1e3 * sum(wall) / args.steps
    value = trunc / sum(wall)
    log(f"[bench] headline: {ms_per_step:.1f} ms/step (steps {', '.join(f'{1e3 * w:.1f}' for w in wall)}), "
        f"{last['truncations']} truncations, plan {plan_s:.1f} s")

    # one-shot setup: what hm_lu does (recording, scheduling, upload and the
    # run) on the reset matrices, as a caller without a reusable plan sees it
    reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan1, plan1_s = make_plan(args.mode, args.precision, False, args.predictor, False, args.schedule)
    info1 = plan1.run(eps)
    torch.cuda.synchronize()
    one_shot = time.perf_counter() - t0
    del plan1
    phases = info1.get("plan_phase_seconds", [0.0, 0.0, 0.0])
    log(f"[bench] one-shot H-LU (planning included): {one_shot:.2f} s (planning {plan1_s:.2f} s: recording "
        f"{phases[0]:.2f}, scheduling {phases[1]:.2f}, upload {phases[2]:.2f})")

    # profiled run in dependency waves: per-launch HIP events on the launch's
    # own stream; in waves each kernel has at most one launch per wave, so its
    # launches never overlap each other and its summed time is exclusive
    plan, _ = make_plan(args.mode, args.precision, False, args.predictor, True, "waves")
    reset()
    prof = plan.run(eps)
    torch.cuda.synchronize()
    del plan
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
    tr = traffic_ratio(dominant)
    traffic = None if tr is None else tr["traffic_over_algorithmic"] * dk["bytes_per_launch"]
    roofline = {"kernel": dominant, "bound": "hbm", "achieved": round(dk["GB_per_s"], 3), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": dk["GB_per_s"] / HBM_PEAK_GBS, "traffic": traffic,
                "traffic_source": (f"profiles/hbm_traffic.json: FETCH_SIZE + WRITE_SIZE over algorithmic bytes "
                                   f"({tr['traffic_over_algorithmic']}) of a full batch of "
                                   f"{batch_shapes(tr['batch'])}, times this kernel's algorithmic bytes per launch")
                if tr else None,
                "traffic_over_algorithmic": tr["traffic_over_algorithmic"] if tr else None,
                "algorithmic_bytes_per_launch": dk["bytes_per_launch"], "avg_launch_us": dk["avg_launch_us"],
                "launches_per_step": dk["launches"], "per_unit": "8 (m+n)(l+k) bytes per executed truncation",
                "timing": "HIP events per launch in a dependency-wave run (launches of one kernel never overlap)",
                "profiled_run_ms": 1e3 * prof["run_seconds"]}
    log(f"[bench] profiled waves run {1e3 * prof['run_seconds']:.1f} ms; dominant {dominant}: "
        f"{dk['seconds']:.3f} s, {dk['avg_launch_us']:.1f} us/launch, {dk['GB_per_s']:.1f} GB/s")

    buckets = None
    if not args.no_buckets:
        buckets = bucket_roofline(hm, W, torch, ctx, "fp64")

    compare = []
    if not args.no_compare:
        sch = args.schedule
        legs = [("plain FP64 per-update path (standard updates, dependency waves, launch by launch)", "standard",
                 "fp64", False, "waves"),
                ("accumulated updates in FP64, same batching and schedule", "accumulated", "fp64", graph, sch),
                ("fused accumulation with the headline precision, batching and schedule", "fused",
                 args.precision, graph, sch),
                ("standard updates with the headline precision, batching and schedule", "standard", args.precision,
                 graph, sch)]
        for name, mode, prec, gr, sc in legs:
            if (mode, prec, gr, sc) == (args.mode, args.precision, graph, sch):
                continue
            p2, w2, inf2 = run_path(mode, prec, gr, False, 1, 1, sc)
            compare.append({"path": name, "mode": mode, "precision": prec,
                            "hip_graph": bool(inf2[-1]["graph_replay"]),
                            "schedule": inf2[-1]["schedule"], "h_lu_seconds": w2[0],
                            "truncations": inf2[-1]["truncations"], "updates_per_s": inf2[-1]["truncations"] / w2[0],
                            "plan_seconds": p2, "headline_speedup": w2[0] / (sum(wall) / args.steps)})
            log(f"[bench] {name}: {1e3 * w2[0]:.1f} ms, {inf2[-1]['truncations']} truncations")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg, args.mode, eps)
        log(f"[bench] cpu baseline: {cpu['value']:.1f} updates/s ({cpu['sample']})")

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
        "h_lu_setup_s": one_shot,
        "h_lu_setup_s_per_dof": one_shot / n_total,
        "h_lu_setup_planning_s": plan1_s,
        "h_lu_setup_planning_phases_s": {"recording": phases[0], "scheduling": phases[1], "upload": phases[2]},
        "h_lu_run_s": sum(wall) / args.steps,
        "h_lu_device_s": sum(i["run_seconds"] for i in infos) / args.steps,
        "plan_s": plan_s,
        "truncations_per_step": last["truncations"],
        "one_shot_truncations": info1["truncations"],
        "predicted_truncations": last["predicted"],
        "predicted_fallbacks": last["predicted_fallback"],
        "waves": last["waves"],
        "launches": last["launches"],
        "temp_bytes": last["temp_bytes"],
        "workspace_bytes": last["workspace_bytes"],
        "kernel_seconds_per_step": ops,
        "trunc_kernels": kernels,
        "dominant_kernel": dominant,
        "roofline": roofline,
        "roofline_buckets": buckets,
        "compare": compare,
        "predictor": pred_info,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
