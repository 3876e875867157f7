"""Batched execution forms: graph replay, the small-block kernel variants and
the autotuner that chooses between them.

A plan replayed from a captured hipGraph gives the same result as the
launch-by-launch run, on every replay.

Each replay is preceded by eager work on the same stream (resetting the
matrix from a device copy) and followed by a synchronising read-back.  The
kernels are deterministic (fixed summation orders, no atomics in the
arithmetic), so the results must agree bit for bit.  A change of eps makes
the plan capture its launches again.
"""
import numpy as np
import pytest

from paper_1703_09085_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_09085_amd import hm

    return hm, hm.Context()


@pytest.mark.parametrize("mode", ["standard", "accumulated"])
@pytest.mark.parametrize("dims,leaf", [((32, 32), 16), ((12, 12, 12), 16)])
def test_graph_replays_match_eager(ctx, mode, dims, leaf, monkeypatch):
    """A wave plan on two streams replayed from a hipGraph, eps changing
    between replays (each change captures again), equals the plan run launch
    by launch, bit for bit; the run info says that the graph ran."""
    import torch

    hm, c = ctx
    x = W.grid_points(dims)
    rp, ci, v = W.laplacian_csr(dims)
    G0 = hm.HMatrix.from_csr(c, x, rp, ci, v, leaf, 2.0, kmax=64)
    ref = {}
    for eps in (1e-6, 1e-4):
        Ge = G0.clone()
        info = hm.Plan.lu(c, Ge, mode).run(eps)
        ref[eps] = (Ge.to_dense(), info["truncations"])
    G = G0.clone()
    c.set_schedule("waves")  # graph replay is for wave plans on two streams
    monkeypatch.setenv("HM_WAVE_LANES", "2")
    try:
        plan = hm.Plan.lu(c, G, mode).use_graph()
    finally:
        c.set_schedule("dataflow")
    for rep, eps in enumerate([1e-6, 1e-6, 1e-6, 1e-4, 1e-4, 1e-6]):
        G.copy_from(G0)
        info = plan.run(eps)
        torch.cuda.synchronize()
        D = G.to_dense()
        print(f"{mode} {dims} replay {rep} eps {eps:g}: {info['truncations']} truncations", flush=True)
        assert info["graph_replay"] == 1
        assert info["truncations"] == ref[eps][1]
        assert np.array_equal(D, ref[eps][0]), rep


@pytest.mark.parametrize("mode", ["standard", "accumulated"])
def test_small_kernel_8_threads_per_column(ctx, oracle_lib, mode, monkeypatch):
    """The 512-thread variant of the small-block kernel against the oracle."""
    hm, c = ctx
    monkeypatch.setenv("HM_SMALL_TPC", "8")
    dims, leaf, eps = (16, 16), 8, 1e-6
    x = W.grid_points(dims)
    rp, ci, v = W.laplacian_csr(dims)
    G = hm.HMatrix.from_csr(c, x, rp, ci, v, leaf, 2.0, kmax=64)
    H = oracle_lib.HMatrix.from_csr(x, rp, ci, v, leaf, 2.0)
    info = hm.Plan.lu(c, G, mode).run(eps)
    st = H.lu(eps, mode)
    Dg, Do = G.to_dense(), H.to_dense()
    assert np.linalg.norm(Dg - Do) <= 1e-10 * np.linalg.norm(Do)
    assert np.array_equal(G.blocks()["rank"], H.blocks()["rank"])
    assert info["truncations"] == st["trunc_update"] + st["trunc_accum"] + st["trunc_merge"]


@pytest.mark.parametrize("mode", ["standard", "accumulated"])
def test_autotune(ctx, mode):
    """The autotuner leaves the matrix unchanged, chooses a variant for every
    small-block launch, and the tuned plan (also replayed as a graph) agrees
    with the untuned one to rounding."""
    import torch

    hm, c = ctx
    dims, leaf, eps = (12, 12, 12), 16, 1e-6
    x = W.grid_points(dims)
    rp, ci, v = W.laplacian_csr(dims)
    G0 = hm.HMatrix.from_csr(c, x, rp, ci, v, leaf, 2.0, kmax=64)
    Ge = G0.clone()
    ref_info = hm.Plan.lu(c, Ge, mode).run(eps)
    ref = Ge.to_dense()
    G = G0.clone()
    before = G.to_dense()
    plan = hm.Plan.lu(c, G, mode)
    n4, n8 = plan.autotune(eps)
    print(f"{mode}: {n4} launches kept 4 threads per column, {n8} chose 8", flush=True)
    assert n4 + n8 == ref_info["small_trunc_launches"] > 0
    assert np.array_equal(G.to_dense(), before)
    plan.use_graph()
    for _ in range(2):
        G.copy_from(G0)
        info = plan.run(eps)
        torch.cuda.synchronize()
        D = G.to_dense()
        assert np.linalg.norm(D - ref) <= 1e-12 * np.linalg.norm(ref)
        assert abs(info["truncations"] - ref_info["truncations"]) <= 8


@pytest.mark.parametrize("mode", ["standard", "accumulated"])
def test_lu_batch_equals_separate(ctx, oracle_lib, mode):
    """One plan for several independent H-LUs (2D Laplacians of drawn sizes)
    gives every instance the result of its own plan, bit for bit, in fewer
    waves than the separate plans together; the largest instance against the
    oracle; graph replays and the autotuner on the batched plan."""
    import torch

    hm, c = ctx
    sides = [int(s) for s in W.batch_sides(count=8, lo=10, hi=40, seed=4)]
    G0 = []
    for s in sides:
        x = W.grid_points((s, s))
        rp, ci, v = W.laplacian_csr((s, s))
        G0.append(hm.HMatrix.from_csr(c, x, rp, ci, v, 8, 2.0, kmax=64))
    eps = 1e-6
    sep, sep_waves, sep_truncs = [], 0, 0
    for g in G0:
        G = g.clone()
        info = hm.Plan.lu(c, G, mode).run(eps)
        sep.append(G.to_dense())
        sep_waves += info["waves"]
        sep_truncs += info["truncations"]
    Gs = [g.clone() for g in G0]
    plan = hm.Plan.lu_batch(c, Gs, mode)
    info = plan.run(eps)
    print(f"{mode}: sides {sides}: batched {info['waves']} waves, {info['launches']} launches; "
          f"separate {sep_waves} waves", flush=True)
    assert info["status_bits"] == 0
    assert info["truncations"] == sep_truncs
    assert info["waves"] < sep_waves
    for G, D in zip(Gs, sep):
        assert np.array_equal(G.to_dense(), D)
    # the largest instance against the oracle
    i = int(np.argmax(sides))
    s = sides[i]
    H = oracle_lib.HMatrix.from_csr(W.grid_points((s, s)), *W.laplacian_csr((s, s)), 8, 2.0)
    H.lu(eps, mode)
    Do = H.to_dense()
    assert np.linalg.norm(sep[i] - Do) <= 1e-10 * np.linalg.norm(Do)
    # autotuning restores every instance; runs with use_graph set (a dataflow plan
    # still runs launch by launch) reproduce the eager result
    for G, g in zip(Gs, G0):
        G.copy_from(g)
    plan.autotune(eps)
    for G, g in zip(Gs, G0):
        assert np.array_equal(G.to_dense(), g.to_dense())
    plan.use_graph()
    for rep in range(3):
        for G, g in zip(Gs, G0):
            G.copy_from(g)
        plan.run(eps)
        torch.cuda.synchronize()
        ok = all(np.linalg.norm(G.to_dense() - D) <= 1e-10 * np.linalg.norm(D) for G, D in zip(Gs, sep))
        assert ok, rep


def test_lu_batch_rejects_bad_arguments(ctx):
    hm, c = ctx
    x = W.grid_points((8, 8))
    rp, ci, v = W.laplacian_csr((8, 8))
    G = hm.HMatrix.from_csr(c, x, rp, ci, v, 4, 2.0, kmax=64)
    with pytest.raises(hm.HMError):
        hm.Plan.lu_batch(c, [G, G], "standard")
    with pytest.raises(hm.HMError):
        hm.Plan.lu_batch(c, [], "standard")


@pytest.mark.parametrize("mode", ["standard", "accumulated"])
def test_late_schedule_matches(ctx, mode, monkeypatch):
    """The late schedule (operations that only write temporaries placed just
    before their first dependent) gives the earliest-wave schedule's result
    bit for bit, in the same number of waves, with fewer temporary bytes."""
    hm, c = ctx
    x = W.grid_points((12, 12, 12))
    rp, ci, v = W.laplacian_csr((12, 12, 12))
    G0 = hm.HMatrix.from_csr(c, x, rp, ci, v, 16, 2.0, kmax=64)
    res = {}
    for sched in ("early", "late"):
        monkeypatch.setenv("HM_SCHEDULE", "waves" if sched == "early" else "late")
        G = G0.clone()
        info = hm.Plan.lu(c, G, mode).run(1e-6)
        res[sched] = (G.to_dense(), info)
    (De, ie), (Dl, il) = res["early"], res["late"]
    print(f"{mode}: temporaries {ie['temp_bytes']} B early, {il['temp_bytes']} B late; "
          f"{ie['waves']} waves, launches {ie['launches']} / {il['launches']}", flush=True)
    assert il["status_bits"] == 0
    assert np.array_equal(De, Dl)
    assert il["truncations"] == ie["truncations"] and il["waves"] == ie["waves"]
    assert il["temp_bytes"] < ie["temp_bytes"]


@pytest.mark.parametrize("mode", ["standard", "accumulated"])
@pytest.mark.parametrize("dims,leaf", [((32, 32), 8), ((12, 12, 12), 16)])
def test_dataflow_matches_waves(ctx, mode, dims, leaf):
    """The dataflow schedule (launches on four streams, each operation waiting
    only for the operations it conflicts with) gives the wave schedule's H-LU
    and H-multiplication bit for bit, with the same number of truncations:
    every operation sees the same inputs in both."""
    hm, c = ctx
    x = W.grid_points(dims)
    rp, ci, v = W.laplacian_csr(dims)
    G0 = hm.HMatrix.from_csr(c, x, rp, ci, v, leaf, 2.0, kmax=64)
    res = {}
    try:
        for sched in ("waves", "dataflow"):
            c.set_schedule(sched)
            G = G0.clone()
            info = hm.Plan.lu(c, G, mode).run(1e-6)
            assert info["schedule"] == sched and info["status_bits"] == 0
            # the product of the factors with themselves, same schedule
            Z = G.zeros_like()
            zinfo = hm.Plan.addmul(c, 1.0, G, G, Z, mode).run(1e-6)
            assert zinfo["schedule"] == sched and zinfo["status_bits"] == 0
            res[sched] = (G.to_dense(), Z.to_dense(), info, zinfo)
    finally:
        c.set_schedule("dataflow")
    (Gw, Zw, iw, zw), (Gd, Zd, idf, zdf) = res["waves"], res["dataflow"]
    print(f"{mode} {dims}: launches {iw['launches']} (waves) / {idf['launches']} (dataflow); "
          f"temporaries {iw['temp_bytes']} / {idf['temp_bytes']} B", flush=True)
    assert np.array_equal(Gw, Gd) and np.array_equal(Zw, Zd)
    assert iw["truncations"] == idf["truncations"] and zw["truncations"] == zdf["truncations"]


def test_set_schedule_rejects_unknown(ctx):
    hm, c = ctx
    with pytest.raises(KeyError):
        c.set_schedule("sideways")
    from paper_1703_09085_amd.hm import lib

    assert lib().hm_set_schedule(c._h, 7) != 0


@pytest.mark.parametrize("mode", ["standard", "accumulated"])
def test_dataflow_matches_waves_batched(ctx, mode):
    """A batched plan for several independent H-LUs gives every instance the
    same factors, bit for bit, in both schedules."""
    hm, c = ctx
    sides = [int(s) for s in W.batch_sides(count=6, lo=10, hi=30, seed=9)]
    G0 = []
    for s in sides:
        x = W.grid_points((s, s))
        rp, ci, v = W.laplacian_csr((s, s))
        G0.append(hm.HMatrix.from_csr(c, x, rp, ci, v, 8, 2.0, kmax=64))
    res = {}
    try:
        for sched in ("waves", "dataflow"):
            c.set_schedule(sched)
            Gs = [g.clone() for g in G0]
            info = hm.Plan.lu_batch(c, Gs, mode).run(1e-6)
            assert info["schedule"] == sched and info["status_bits"] == 0
            res[sched] = ([G.to_dense() for G in Gs], info["truncations"])
    finally:
        c.set_schedule("dataflow")
    assert res["waves"][1] == res["dataflow"][1]
    for a, b in zip(res["waves"][0], res["dataflow"][0]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("mode", ["standard", "accumulated"])
def test_batch_instances_at_full_size(ctx, oracle_lib, mode):
    """Three instances of the 64-instance benchmark batch, the smallest, median
    and largest grid (sides 37, 87 and 127; leaf 32, eta 2, eps 1e-6), in one
    batched plan against the oracle's H-LU of each: equal ranks in every
    admissible leaf, the truncation counts, every leaf block's Frobenius norm,
    and the product of the packed factors with a seeded vector."""
    from test_gpu_parity import oracle_run_logged, oracle_truncs

    hm, hctx = ctx
    sides = sorted(int(s) for s in W.batch_sides(64, 32, 128, 4))
    pick = [sides[0], sides[len(sides) // 2], sides[-1]]
    G, H = [], []
    for side in pick:
        x = W.grid_points((side, side))
        rp, ci, v = W.laplacian_csr((side, side))
        G.append(hm.HMatrix.from_csr(hctx, x, rp, ci, v, 32, 2.0, kmax=64))
        H.append(oracle_lib.HMatrix.from_csr(x, rp, ci, v, 32, 2.0))
    info = hm.Plan.lu_batch(hctx, G, mode).run(1e-6)
    expected, cancelled = 0, 0
    for side, g, h in zip(pick, G, H):
        st, canc = oracle_run_logged(lambda: h.lu(1e-6, mode))
        expected += oracle_truncs(st)
        cancelled += canc
        b, bo, c = g.blocks(), h.blocks(), g.clusters()
        assert np.array_equal(b["kind"], bo["kind"])
        adm = b["kind"] == 1
        diff = int(np.count_nonzero(b["rank"][adm] != bo["rank"][adm]))
        leaves = np.nonzero(b["kind"] > 0)[0]
        xv = np.random.default_rng(side).standard_normal(g.n)
        y, yo = np.zeros(g.n), np.zeros(g.n)
        norms, norms_o = np.zeros(len(leaves)), np.zeros(len(leaves))
        for j, i in enumerate(leaves):
            t, s = b["t"][i], b["s"][i]
            r0, nr, c0, nc = int(c["off"][t]), int(c["size"][t]), int(c["off"][s]), int(c["size"][s])
            got = g.block_to_dense(int(i), nr, nc)
            ref = h.addeval_block(int(i), np.eye(nc), np.zeros((nr, nc)))
            norms[j], norms_o[j] = np.linalg.norm(got), np.linalg.norm(ref)
            y[r0:r0 + nr] += got @ xv[c0:c0 + nc]
            yo[r0:r0 + nr] += ref @ xv[c0:c0 + nc]
        top = norms_o.max()
        bad = int(np.count_nonzero(np.abs(norms - norms_o) > 1e-9 * norms_o + 1e-13 * top))
        rel = np.linalg.norm(y - yo) / np.linalg.norm(yo)
        print(f"{mode} side {side}: {diff} of {int(adm.sum())} admissible leaves differ in rank, {bad} of "
              f"{len(leaves)} leaf norms off, product relative difference {rel:.2e}", flush=True)
        assert diff == 0 and bad == 0
        assert rel <= 1e-10
    assert abs(info["truncations"] - expected) <= 4 * cancelled
