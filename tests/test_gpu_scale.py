"""GPU checks at the benchmark size (7-point Laplacian on 32^3, leaf 64,
eta 2, eps 1e-6), standard and accumulated H-LU.

* Every truncation item runs exactly once: the device counter of executed
  truncations equals the number of distinct items in the truncation log.  The
  general kernels of a wave are launched on the same items one after the
  other and split them between themselves; an item taken by both would apply
  its update twice.
* Against the oracle's stored results (tests/golden, written by
  tests/golden/make_golden.py from the CPU oracle only): the number of
  executed truncations and the rank of every admissible leaf (both equal to
  the oracle's on this FP64 path), the Frobenius norm of every leaf block of
  the packed L / R factors, their product with a seeded vector, and the
  values of 24 sampled leaf blocks.
"""
import json
import os

import numpy as np
import pytest

from paper_1703_09085_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lap3d_32_lu_eps1e-6")


@pytest.fixture(scope="module")
def lap3d():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_09085_amd import hm

    ctx = hm.Context()
    cfg = W.CONFIGS["lap3d_32"]
    x = W.grid_points(cfg["dims"])
    rp, ci, v = W.laplacian_csr(cfg["dims"])
    G0 = hm.HMatrix.from_csr(ctx, x, rp, ci, v, cfg["leaf"], cfg["eta"], kmax=96)
    golden = np.load(GOLDEN + ".npz")
    with open(GOLDEN + ".json") as f:
        stats = json.load(f)
    return hm, ctx, cfg, G0, golden, stats


@pytest.mark.parametrize("mode", ["accumulated", "standard"])
def test_full_size_lu(lap3d, mode, monkeypatch):
    hm, ctx, cfg, G0, golden, stats = lap3d
    monkeypatch.setenv("HM_TRUNC_LOG", "1")
    G = G0.clone()
    plan = hm.Plan.lu(ctx, G, mode)
    info = plan.run(cfg["eps"])
    log = plan.trunc_log()
    del plan
    executed_items = int(np.count_nonzero(log[:, 0] > 0))
    st = stats[mode]["stats"]
    oracle_truncs = st["trunc_update"] + st["trunc_accum"] + st["trunc_merge"]
    print(f"{mode}: {info['truncations']} executed, {executed_items} distinct items, "
          f"{info['planned_truncations']} planned, oracle {oracle_truncs}", flush=True)
    # each item once
    assert info["status_bits"] == 0
    assert info["truncations"] == executed_items
    assert executed_items <= info["planned_truncations"]
    ex = log[log[:, 0] > 0]
    assert np.all(ex[:, 3] >= 0) and np.all(ex[:, 3] <= np.minimum(ex[:, 0], ex[:, 1]))
    # ranks of the admissible leaves: equal outside rounding ties of the rank rule
    b = G.blocks()
    ro = golden[f"{mode}_rank"].astype(np.int32)
    adm = b["kind"] == 1  # admissible (low-rank) leaves; the oracle stores -1 for the others
    assert np.array_equal(adm, ro >= 0)
    diff = int(np.count_nonzero(b["rank"][adm] != ro[adm]))
    print(f"{mode}: {diff} of {int(adm.sum())} admissible leaves differ in rank", flush=True)
    assert diff == 0
    assert info["truncations"] == oracle_truncs
    # sampled leaf blocks
    c = G.clusters()
    samples = golden[f"{mode}_samples"]
    scale = np.max(np.abs(samples))
    pos = 0
    worst = 0.0
    for i in golden[f"{mode}_pick"]:
        t, s = b["t"][i], b["s"][i]
        nr, nc = int(c["size"][t]), int(c["size"][s])
        ref = samples[pos:pos + nr * nc].reshape((nr, nc), order="F")
        pos += nr * nc
        got = G.block_to_dense(int(i), nr, nc)
        err = np.linalg.norm(got - ref)
        worst = max(worst, err / max(np.linalg.norm(ref), 1e-300))
        assert err <= 1e-9 * np.linalg.norm(ref) + 1e-12 * scale, (int(i), err, np.linalg.norm(ref))
    print(f"{mode}: worst relative difference of the sampled blocks {worst:.2e}", flush=True)
    if f"{mode}_leaf_norm" not in golden:
        pytest.skip("golden file without per-leaf norms")
    # every leaf block: its norm, and y = (packed factors) x for the seeded x
    norms = golden[f"{mode}_leaf_norm"]
    xv = np.random.default_rng(11).standard_normal(G.n)
    y = np.zeros(G.n)
    leaves = np.nonzero(b["kind"] > 0)[0]
    assert np.array_equal(leaves, np.nonzero(norms >= 0)[0])
    top = norms.max()
    bad = 0
    for i in leaves:
        t, s = b["t"][i], b["s"][i]
        r0, nr, c0, nc = int(c["off"][t]), int(c["size"][t]), int(c["off"][s]), int(c["size"][s])
        got = G.block_to_dense(int(i), nr, nc)
        bad += abs(np.linalg.norm(got) - norms[i]) > 1e-9 * norms[i] + 1e-13 * top
        y[r0:r0 + nr] += got @ xv[c0:c0 + nc]
    ref = golden[f"{mode}_product"]
    rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    print(f"{mode}: {bad} of {len(leaves)} leaf norms off; product relative difference {rel:.2e}", flush=True)
    assert bad == 0
    assert rel <= 1e-10
