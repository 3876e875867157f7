"""GPU checks of the learned rank predictor (network trained on the GPU).

The network is trained, by the library's own kernels, on the features and
exact ranks that H-LU runs of the 2D 5-point Laplacian (64 x 64, leaf 32) and
of the 3D 7-point Laplacian (16^3, leaf 32) log in feature mode.  Then:

* the logged features are what they claim to be (sizes of the truncation);
* the trained network fits the logged ranks;
* per truncation (hm_trunc_batch_predicted against the oracle's truncated
  addition): every result meets the eps bound of the rank rule with a rank at
  least the exact one, whether the range finder was kept or the exact path ran;
* the H-LU of the 3D Laplacian on 32^3 (leaf 64, held out from training) run
  with the predictor agrees with the oracle's stored blocks to 10 eps;
* what the network gains: the truncations whose estimate is kept run a
  narrower core (fewer pivoted QR steps and Jacobi columns), so the mean core
  width of the small truncations falls; the device time of the small-block
  launches with and without the predictor is measured and printed.  (Since
  the exact path became a pivoted QR that stops at the rounding level, the
  time does not fall: a launch lasts as long as its slowest item, and an item
  that falls back runs the narrow core and then the full one.)
"""
import json
import os

import numpy as np
import pytest

from paper_1703_09085_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lap3d_32_lu_eps1e-6")
EPS = 1e-6
OVERSAMPLE = 2
TRAIN_PROBLEMS = [((64, 64), 32), ((16, 16, 16), 32)]


def problem(hm, ctx, dims, leaf):
    x = W.grid_points(dims)
    rp, ci, v = W.laplacian_csr(dims)
    return hm.HMatrix.from_csr(ctx, x, rp, ci, v, leaf, 2.0, kmax=96 if len(dims) == 3 else 64)


class env:
    """Set environment variables for the plans made inside the block."""

    def __init__(self, **kv):
        self.kv = kv

    def __enter__(self):
        self.old = {k: os.environ.get(k) for k in self.kv}
        os.environ.update(self.kv)

    def __exit__(self, *a):
        for k, v in self.old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.fixture(scope="module")
def trained():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_09085_amd import hm

    ctx = hm.Context()
    g = torch.Generator().manual_seed(1703)
    omega = torch.randn(32, 64, generator=g, dtype=torch.float64).cuda()
    net = hm.MLP(ctx, seed=3)
    feats, logs = [], []
    with env(HM_TRUNC_LOG="1", HM_FEATURE_LOG="1"):
        for dims, leaf in TRAIN_PROBLEMS:
            for mode in ("standard", "accumulated"):
                G = problem(hm, ctx, dims, leaf)
                plan = hm.Plan.lu(ctx, G, mode).set_predictor(net, omega, 8, 0)
                info = plan.run(EPS)
                assert info["status_bits"] == 0
                feats.append(plan.feature_log())
                logs.append(plan.trunc_log())
                del plan
    F = np.concatenate(feats)
    L = np.concatenate(logs)
    sel = np.isfinite(F[:, 0]) & (L[:, 0] > 0)
    X = np.ascontiguousarray(F[sel, :8])
    t = np.log2(1.0 + L[sel, 3]).astype(np.float32)
    perm = np.random.default_rng(0).permutation(len(X))
    X, t = X[perm], t[perm]
    Xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    losses = net.train(Xd, td, epochs=60, batch=512, lr=2e-3)
    print(f"trained on {len(X)} logged truncations: loss {losses[0]:.4f} -> {losses[-1]:.4f}", flush=True)
    return hm, ctx, omega, net, F, L, X, t, losses


def test_feature_log(trained):
    """Mode 0 logs the features of every small truncation and keeps it exact."""
    hm, ctx, omega, net, F, L, X, t, losses = trained
    small = (L[:, 0] > 0) & (L[:, 0] <= 64) & (L[:, 1] <= 64)
    logged = np.isfinite(F[:, 0])
    # a small item without features had a zero sum K (a product of exactly
    # cancelling or zero factors): its rank is 0
    assert np.all(L[small & ~logged, 3] == 0)
    print(f"{int(np.count_nonzero(small & logged))} of {int(np.count_nonzero(small))} small items with features",
          flush=True)
    assert not np.any(logged & (L[:, 0] > 64))
    f = F[small & logged]
    lg = L[small & logged]
    assert np.allclose(f[:, 1], np.log2(lg[:, 0]), atol=1e-6)
    assert np.allclose(f[:, 2], np.log2(lg[:, 1]), atol=1e-6)
    assert np.allclose(f[:, 3], np.log2(1.0 + lg[:, 2]), atol=1e-6)
    assert np.all(np.diff(f[:, 4:8], axis=1) <= 1e-6)  # descending
    assert np.all(f[:, 9] == 0)  # outcome: exact path


def test_network_fits_logged_ranks(trained):
    hm, ctx, omega, net, F, L, X, t, losses = trained
    import torch

    assert losses[-1] < losses[0] / 20
    y = net.predict(torch.from_numpy(X).cuda()).cpu().numpy()
    khat = np.ceil(np.exp2(np.minimum(y, 7.0)) - 1.0)
    k = np.exp2(t) - 1.0
    print(f"mean |k^ - k| {np.mean(np.abs(khat - k)):.3f}, within 8: {np.mean(k <= khat + 8):.4f}", flush=True)
    assert np.mean(np.abs(khat - k)) < 2.0
    assert np.mean(k <= khat + 8) > 0.95


def test_predicted_batch_meets_bound(trained, oracle_lib):
    """Every item: eps bound of the rank rule, rank >= the exact rank."""
    import torch

    hm, ctx, omega, net, *_ = trained
    from test_gpu_parity import dev, oracle_margin

    rng = np.random.default_rng(29)
    descs, keep = [], []
    for i in range(96):
        m, n = int(rng.integers(8, 65)), int(rng.integers(8, 65))
        k1, k2 = int(rng.integers(1, 40)), int(rng.integers(0, 40))
        decay = float(rng.uniform(0.3, 0.9))
        A, B = W.lowrank_factors(m, n, k1, seed=300 + i, decay=decay)
        C_, D = W.lowrank_factors(m, n, k2, seed=400 + i, decay=decay, scale=0.7)
        tens = [dev(x) for x in (A, B, C_, D)]
        kcap = max(min(m, n, k1 + k2), 1)
        Co, Do = dev(np.zeros((m, kcap))), dev(np.zeros((n, kcap)))
        rk = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        descs.append(hm.TruncDesc(m=m, n=n, k1=k1, k2=k2, kcap=kcap, lda=m, ldb=n, ldc=m, ldd=n, alpha=-1.0,
                                  A=tens[0].data_ptr(), B=tens[1].data_ptr(), C=tens[2].data_ptr(),
                                  D=tens[3].data_ptr(), Cout=Co.data_ptr(), Dout=Do.data_ptr(),
                                  rank_out=rk.data_ptr()))
        keep.append((tens, Co, Do, rk, (A, B, C_, D)))
    total_acc = total_fb = 0
    for ov in (0, 8):
        executed, acc, fb = ctx.trunc_batch_predicted(descs, EPS, net, omega, oversample=ov, level=6)
        print(f"oversample {ov}: {executed} executed, {acc} range finder kept, {fb} fell back", flush=True)
        assert executed == len(descs) and acc + fb <= executed
        total_acc += acc
        total_fb += fb
        for tens, Co, Do, rk, (A, B, C_, D) in keep:
            K = C_ @ D.T - A @ B.T
            Cr, Dr, sg = oracle_lib.rkadd(-1.0, A, B, C_, D, EPS)
            k = int(rk.item())
            if oracle_margin(sg, EPS) > 1e-8:
                assert k >= Cr.shape[1]
            Cg = Co.cpu().numpy().T[:, :k]
            Dg = Do.cpu().numpy().T[:, :k]
            nk = np.linalg.norm(K)
            assert np.linalg.norm(K - Cg @ Dg.T) <= EPS * nk * (1 + 1e-6) + 1e-14 * nk
            assert np.allclose(Cg.T @ Cg, np.eye(k), atol=1e-12)
    assert total_acc > 0


@pytest.fixture(scope="module")
def lap3d(trained):
    hm, ctx, *_ = trained
    cfg = W.CONFIGS["lap3d_32"]
    G0 = problem(hm, ctx, cfg["dims"], cfg["leaf"])
    golden = np.load(GOLDEN + ".npz")
    with open(GOLDEN + ".json") as f:
        stats = json.load(f)
    return cfg, G0, golden, stats


@pytest.mark.parametrize("mode", ["accumulated", "standard"])
def test_predicted_lu_matches_oracle(trained, lap3d, mode):
    hm, ctx, omega, net, *_ = trained
    cfg, G0, golden, stats = lap3d
    G = G0.clone()
    plan = hm.Plan.lu(ctx, G, mode).set_predictor(net, omega, OVERSAMPLE, 1)
    info = plan.run(cfg["eps"])
    del plan
    assert info["status_bits"] == 0
    acc, fb = info["predicted"], info["predicted_fallback"]
    print(f"{mode}: {info['truncations']} truncations, range finder kept {acc}, fell back {fb}", flush=True)
    assert acc > 0.05 * info["truncations"] and fb < acc
    b = G.blocks()
    c = G.clusters()
    samples = golden[f"{mode}_samples"]
    pos = 0
    worst = 0.0
    for i in golden[f"{mode}_pick"]:
        t, s = b["t"][i], b["s"][i]
        nr, nc = int(c["size"][t]), int(c["size"][s])
        ref = samples[pos:pos + nr * nc].reshape((nr, nc), order="F")
        pos += nr * nc
        got = G.block_to_dense(int(i), nr, nc)
        rel = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
        worst = max(worst, rel)
        assert rel <= 10 * cfg["eps"], (int(i), rel)
    print(f"{mode}: worst relative difference from the oracle's blocks {worst:.2e}", flush=True)
    # ranks never below the oracle's by more than rounding ties
    ro = golden[f"{mode}_rank"].astype(np.int32)
    adm = b["kind"] == 1
    assert int(b["rank"][adm].sum()) >= int(ro[adm].sum()) - 2


def test_predictor_gain(trained, lap3d, monkeypatch):
    """Core widths and device time of the small-block truncations, standard
    H-LU, without and with the predictor."""
    hm, ctx, omega, net, *_ = trained
    cfg, G0, golden, stats = lap3d
    monkeypatch.setenv("HM_PROFILE_OPS", "1")
    monkeypatch.setenv("HM_TRUNC_LOG", "1")
    res = {}
    for name, pred in (("exact", False), ("predicted", True)):
        G = G0.clone()
        plan = hm.Plan.lu(ctx, G, "standard")
        if pred:
            plan.set_predictor(net, omega, OVERSAMPLE, 1)
        best = None
        for _ in range(2):
            G.copy_from(G0)
            info = plan.run(cfg["eps"])
            if best is None or info["small_trunc_seconds"] < best["small_trunc_seconds"]:
                best = info
        log = plan.trunc_log()
        ex = log[(log[:, 0] > 0) & (log[:, 0] <= 64) & (log[:, 1] <= 64) & ((log[:, 4] & 0xFFFF) > 0)]
        best["width"] = float(np.mean(ex[:, 4] >> 16))
        res[name] = best
        del plan
    te, tp = res["exact"]["small_trunc_seconds"], res["predicted"]["small_trunc_seconds"]
    we, wp = res["exact"]["width"], res["predicted"]["width"]
    print(f"small-block truncations: mean core width {we:.2f} exact, {wp:.2f} predicted "
          f"({res['predicted']['predicted']} kept, {res['predicted']['predicted_fallback']} fell back); "
          f"device time {1e3 * te:.1f} ms exact, {1e3 * tp:.1f} ms predicted ({te / tp:.2f}x)", flush=True)
    assert res["predicted"]["predicted"] > 0
    assert wp < we
