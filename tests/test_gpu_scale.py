"""GPU checks at the benchmark size (7-point Laplacian on 32^3, leaf 64).

* Every truncation item runs exactly once: the device counter of executed
  truncations equals the number of distinct items in the truncation log.  The
  general kernels of a wave are launched on the same items one after the
  other and split them between themselves; an item taken by both would apply
  its update twice.
* The executed truncations are a subset of the planned ones, and the H-LU is
  finite (no status bits).
"""
import os

import numpy as np
import pytest

from paper_1703_09085_amd import workloads as W

pytestmark = pytest.mark.gpu


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
    return hm, ctx, cfg, G0


@pytest.mark.parametrize("mode", ["accumulated", "standard"])
def test_each_truncation_runs_once(lap3d, mode, monkeypatch):
    hm, ctx, cfg, G0 = lap3d
    monkeypatch.setenv("HM_TRUNC_LOG", "1")
    G = G0.clone()
    plan = hm.Plan.lu(ctx, G, mode)
    info = plan.run(cfg["eps"])
    log = plan.trunc_log()
    executed_items = int(np.count_nonzero(log[:, 0] > 0))
    print(f"{mode}: {info['truncations']} executed, {executed_items} distinct items, "
          f"{info['planned_truncations']} planned", flush=True)
    assert info["status_bits"] == 0
    assert info["truncations"] == executed_items
    assert executed_items <= info["planned_truncations"]
    # every logged item has a rank within its sizes
    ex = log[log[:, 0] > 0]
    assert np.all(ex[:, 3] >= 0) and np.all(ex[:, 3] <= np.minimum(ex[:, 0], ex[:, 1]))
