"""GPU checks of the C ABI beyond the arithmetic: builds from a source
description, options and the rank override, context statistics and the
caller's allocator, truncation batches with device-resident descriptors, and
the error paths (every failing call leaves the device usable: the next call
succeeds).
"""
import numpy as np
import pytest

from paper_1703_09085_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_09085_amd import hm as mod

    return mod


def lap(hm, ctx, dims, leaf, kmax=64):
    x = W.grid_points(dims)
    rp, ci, v = W.laplacian_csr(dims)
    return x, (rp, ci, v), hm.HMatrix.from_csr(ctx, x, rp, ci, v, leaf, 2.0, kmax=kmax)


@pytest.mark.parametrize("dims,leaf", [((20, 17), 8), ((6, 7, 5), 16)])
def test_stencil_source_equals_csr(hm, dims, leaf):
    ctx = hm.Context()
    x, _, G = lap(hm, ctx, dims, leaf)
    S = hm.HMatrix.from_stencil(ctx, x, leaf)
    assert np.array_equal(G.perm(), S.perm())
    assert np.array_equal(G.to_dense(), S.to_dense())


def test_options_and_rank_override(hm, monkeypatch):
    """FP64 ranks imposed on a split-BF16x3 run: identical ranks item by item,
    so the difference of the results is the rounding of the products alone."""
    ctx = hm.Context()
    eps = 1e-6
    _, _, G0 = lap(hm, ctx, (40, 40), 16)
    monkeypatch.setenv("HM_TRUNC_LOG", "1")
    ranks = {}
    results = {}
    for prec in ("fp64", "bf16x3"):
        G = G0.clone()
        plan = hm.Plan.lu(ctx, G, "accumulated").set_precision(prec)
        if prec != "fp64":
            plan.set_rank_override(ranks["fp64"])
        print(f"lu {prec}", flush=True)
        plan.run(eps)
        ranks[prec] = plan.trunc_log()[:, 3].copy()
        del plan
        results[prec] = G.to_dense()
    assert np.array_equal(ranks["fp64"], ranks["bf16x3"])
    ref = results["fp64"]
    assert np.linalg.norm(results["bf16x3"] - ref) <= 10 * eps * np.linalg.norm(ref)
    # the same through hm_lu_opt
    G = G0.clone()
    info = G.lu_opt(eps=eps, mode="accumulated", precision="bf16x3", rank_override=ranks["fp64"])
    assert info["status_bits"] == 0
    assert np.linalg.norm(G.to_dense() - ref) <= 10 * eps * np.linalg.norm(ref)
    with pytest.raises(hm.HMError):
        G0.clone().lu_opt(eps=eps, rank_override=ranks["fp64"][:-1])  # wrong length


def test_lu_opt_matches_lu(hm):
    ctx = hm.Context()
    _, _, G0 = lap(hm, ctx, (32, 32), 16)
    A, B = G0.clone(), G0.clone()
    A.lu(1e-6, "standard")
    B.lu_opt(eps=1e-6, mode="standard", schedule="waves")
    assert np.array_equal(A.to_dense(), B.to_dense())


def test_stats_and_torch_allocator(hm):
    import torch

    ctx = hm.Context(allocator="torch")
    base = torch.cuda.memory_allocated()
    _, _, G = lap(hm, ctx, (48, 48), 16)
    st = ctx.stats()
    assert st["device_bytes_in_use"] > 0 and st["device_allocations"] >= 4
    assert torch.cuda.memory_allocated() - base >= st["device_bytes_in_use"] - 4096
    info = G.lu(1e-6, "accumulated")
    st2 = ctx.stats()
    assert st2["plans"] == 1 and st2["runs"] == 1 and st2["truncations"] == info["truncations"] > 0
    assert st2["device_bytes_peak"] > st["device_bytes_in_use"]  # the plan's arena came and went
    assert st2["device_bytes_in_use"] == st["device_bytes_in_use"]
    del G
    assert ctx.stats()["device_bytes_in_use"] < st["device_bytes_in_use"]


def _items(hm, rng, count, maxmn, kfix=None):
    import torch

    descs, keep = [], []
    for i in range(count):
        m, n = int(rng.integers(1, maxmn)), int(rng.integers(1, maxmn))
        k1, k2 = (int(rng.integers(0, 20)), int(rng.integers(0, 20))) if kfix is None else (kfix, kfix)
        A, B = W.lowrank_factors(m, n, k1, seed=300 + i, decay=0.6)
        C_, D = W.lowrank_factors(m, n, k2, seed=400 + i, decay=0.6)
        t = [torch.from_numpy(np.ascontiguousarray(np.asfortranarray(a).T if a.shape[1] else np.zeros((1, a.shape[0]))))
             .cuda() for a in (A, B, C_, D)]
        kcap = max(min(m, n, k1 + k2), 1)
        Co = torch.zeros((kcap, m), dtype=torch.float64, device="cuda")
        Do = torch.zeros((kcap, n), dtype=torch.float64, device="cuda")
        rk = torch.full((1,), -5, dtype=torch.int32, device="cuda")
        keep.append((t, Co, Do, rk))
        descs.append(hm.TruncDesc(m=m, n=n, k1=k1, k2=k2, kcap=kcap, lda=m, ldb=n, ldc=m, ldd=n, alpha=-0.7,
                                  A=t[0].data_ptr(), B=t[1].data_ptr(), C=t[2].data_ptr(), D=t[3].data_ptr(),
                                  Cout=Co.data_ptr(), Dout=Do.data_ptr(), rank_out=rk.data_ptr()))
    return descs, keep


def _to_device(descs):
    import torch

    arr = (type(descs[0]) * len(descs))(*descs)
    return torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).cuda()


def test_trunc_batch_device_descriptors(hm):
    """Descriptors in device memory give bit-identical results to the same
    descriptors passed from the host (same kernels, classified on the device)."""
    ctx = hm.Context()
    rng = np.random.default_rng(5)
    descs, keep = _items(hm, rng, 48, 200)
    ex_host = ctx.trunc_batch(descs, 1e-6)
    host = [(Co.clone(), Do.clone(), rk.clone()) for _, Co, Do, rk in keep]
    for _, Co, Do, rk in keep:
        Co.zero_()
        Do.zero_()
        rk.fill_(-5)
    ex_dev = ctx.trunc_batch_device(_to_device(descs), len(descs), 200, 40, 1e-6)
    assert ex_dev == ex_host
    for (Ch, Dh, rh), (_, Co, Do, rk) in zip(host, keep):
        assert int(rh.item()) == int(rk.item())
        assert bool((Ch == Co).all()) and bool((Dh == Do).all())
    # an item beyond the caller's bounds: HM_ERR_ARG, the others still run
    with pytest.raises(hm.HMError) as e:
        ctx.trunc_batch_device(_to_device(descs), len(descs), 50, 40, 1e-6)
    assert e.value.status == 1
    assert ctx.trunc_batch_device(_to_device(descs), len(descs), 200, 40, 1e-6) == ex_host


def test_error_nan_factor(hm):
    """A NaN in a factor: HM_ERR_NUMERIC, and the device stays usable."""
    import torch

    ctx = hm.Context()
    rng = np.random.default_rng(9)
    descs, keep = _items(hm, rng, 6, 150)
    for d, (t, *_rest) in zip(descs, keep):
        if d.k1 > 0:
            t[0][0, 0] = float("nan")
    with pytest.raises(hm.HMError) as e:
        ctx.trunc_batch(descs, 1e-6)
    assert e.value.status == 5  # HM_ERR_NUMERIC
    torch.cuda.synchronize()
    _, _, G = lap(hm, ctx, (16, 16), 8)
    assert G.lu(1e-6, "standard")["status_bits"] == 0


def test_error_zero_pivot(hm):
    """A zero diagonal entry in the first leaf: HM_ERR_SINGULAR."""
    ctx = hm.Context()
    dims = (16, 16)
    x = W.grid_points(dims)
    rp, ci, v = W.laplacian_csr(dims)
    v = v.copy()
    perm = hm.HMatrix.from_csr(ctx, x, rp, ci, v, 8, 2.0).perm()
    first = int(perm[0])  # the first unknown in cluster order: pivot 0 of the first leaf LU
    for e in range(rp[first], rp[first + 1]):
        if ci[e] == first:
            v[e] = 0.0
    G = hm.HMatrix.from_csr(ctx, x, rp, ci, v, 8, 2.0)
    for mode in ("standard", "accumulated"):
        with pytest.raises(hm.HMError) as err:
            G.clone().lu(1e-6, mode)
        assert err.value.status == 4  # HM_ERR_SINGULAR
    _, _, H = lap(hm, ctx, dims, 8)
    assert H.lu(1e-6, "standard")["status_bits"] == 0


def test_error_rank_capacity(hm):
    """Ranks above the capacity: HM_ERR_NUMERIC (H-LU with kmax 1, and a
    truncation into a 1-column output)."""
    ctx = hm.Context()
    _, _, G = lap(hm, ctx, (32, 32), 8, kmax=1)
    with pytest.raises(hm.HMError) as e:
        G.lu(1e-10, "standard")
    assert e.value.status == 5
    rng = np.random.default_rng(2)
    descs, keep = _items(hm, rng, 4, 60, kfix=6)
    for d in descs:
        d.kcap = 1  # the outputs hold at least one column
    with pytest.raises(hm.HMError) as e:
        ctx.trunc_batch(descs, 1e-12)
    assert e.value.status == 5
    _, _, H = lap(hm, ctx, (16, 16), 8)
    assert H.lu(1e-6, "standard")["status_bits"] == 0
