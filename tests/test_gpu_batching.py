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
def test_graph_replays_match_eager(ctx, mode, dims, leaf):
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
    plan = hm.Plan.lu(c, G, mode).use_graph()
    for rep, eps in enumerate([1e-6, 1e-6, 1e-6, 1e-4, 1e-4, 1e-6]):
        G.copy_from(G0)
        info = plan.run(eps)
        torch.cuda.synchronize()
        D = G.to_dense()
        print(f"{mode} {dims} replay {rep} eps {eps:g}: {info['truncations']} truncations", flush=True)
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
