"""The allocation-free truncation batch (hm_trunc_batch_device_noalloc)
against the allocating one (hm_trunc_batch_device) through the C ABI: two
calls in a row, the second with fewer and smaller items, each bit-identical
to the allocating entry point on the same descriptors (same kernels; only the
scratch memory differs), and the limits rejected before anything runs."""
import numpy as np
import pytest

from paper_1703_09085_amd import workloads as W

pytestmark = pytest.mark.gpu


def make_items(hm, seed, count, maxmn, maxk):
    import torch

    rng = np.random.default_rng(seed)
    descs, keep = [], []
    for i in range(count):
        m, n = int(rng.integers(1, maxmn)), int(rng.integers(1, maxmn))
        k1, k2 = int(rng.integers(1, maxk)), int(rng.integers(0, maxk))
        A, B = W.lowrank_factors(m, n, k1, seed=seed * 1000 + i, decay=0.6)
        C_, D = W.lowrank_factors(m, n, k2, seed=seed * 1000 + 500 + i, decay=0.6)
        t = [torch.from_numpy(np.ascontiguousarray(a.T if a.shape[1] else np.zeros((1, a.shape[0])))).cuda()
             for a in (A, B, C_, D)]
        kcap = max(min(m, n, k1 + k2), 1)
        outs = [torch.zeros((kcap, m), dtype=torch.float64, device="cuda"),
                torch.zeros((kcap, n), dtype=torch.float64, device="cuda"),
                torch.full((1,), -3, dtype=torch.int32, device="cuda")]
        keep.append((t, outs))
        descs.append(hm.TruncDesc(m=m, n=n, k1=k1, k2=k2, kcap=kcap, lda=m, ldb=n, ldc=m, ldd=n, alpha=-0.6,
                                  A=t[0].data_ptr(), B=t[1].data_ptr(), C=t[2].data_ptr(), D=t[3].data_ptr(),
                                  Cout=outs[0].data_ptr(), Dout=outs[1].data_ptr(), rank_out=outs[2].data_ptr()))
    arr = (hm.TruncDesc * count)(*descs)
    dev = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).cuda()
    return dev, keep


def outputs(keep):
    return [[o.clone() for o in outs] for _, outs in keep]


def reset(keep):
    for _, outs in keep:
        outs[0].zero_()
        outs[1].zero_()
        outs[2].fill_(-3)


@pytest.fixture(scope="module")
def hm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_09085_amd import hm as mod

    return mod


def test_noalloc_matches_allocating_entry_point(hm):
    import torch

    ctx = hm.Context()
    for seed, count, maxmn, maxk in ((1, 100, 200, 30), (2, 40, 100, 12)):
        print(f"no-alloc batch: {count} items, m, n < {maxmn}, k < {maxk}", flush=True)
        dev, keep = make_items(hm, seed, count, maxmn, maxk)
        ex_ref = ctx.trunc_batch_device(dev, count, maxmn, 2 * maxk, 1e-6)
        ref = outputs(keep)
        reset(keep)
        base = torch.cuda.memory_allocated()
        ex = ctx.trunc_batch_device_noalloc(dev, count, maxmn, 2 * maxk, 1e-6)
        assert torch.cuda.memory_allocated() == base
        assert ex == ex_ref == count
        for r, (_, outs) in zip(ref, keep):
            assert int(r[2].item()) == int(outs[2].item())
            assert bool((r[0] == outs[0]).all()) and bool((r[1] == outs[1]).all())


def test_noalloc_asynchronous_call(hm):
    import torch

    ctx = hm.Context()
    dev, keep = make_items(hm, 3, 64, 120, 16)
    ex_ref = ctx.trunc_batch_device(dev, 64, 120, 32, 1e-6)
    ref = outputs(keep)
    reset(keep)
    assert ctx.trunc_batch_device_noalloc(dev, 64, 120, 32, 1e-6, wait=False) is None
    torch.cuda.synchronize()
    for r, (_, outs) in zip(ref, keep):
        assert int(r[2].item()) == int(outs[2].item())
        assert bool((r[0] == outs[0]).all()) and bool((r[1] == outs[1]).all())
    assert ex_ref == 64


def test_noalloc_limits(hm):
    ctx = hm.Context()
    import torch

    dev, _ = make_items(hm, 4, 8, 40, 8)
    big = torch.zeros(5000 * 120, dtype=torch.uint8, device="cuda")  # never read: rejected before any launch
    with pytest.raises(hm.HMError) as e:
        ctx.trunc_batch_device_noalloc(big, 5000, 40, 16, 1e-6)  # more items than the array holds
    assert e.value.status == 1
    with pytest.raises(hm.HMError) as e:
        ctx.trunc_batch_device_noalloc(dev, 8, 20000, 400, 1e-6)  # workspace beyond the array
    assert e.value.status == 1
