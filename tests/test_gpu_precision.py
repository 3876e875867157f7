"""GPU checks of the reduced-precision modes (FP32 and split-BF16x3 on the
matrix cores) against the FP64 oracle.

Storage, the core SVD, the rank rule and the leaf factorisations stay FP64;
the dense products and the small-block truncations' stacked-factor products
run in the reduced precision.  The bound for every result is 10 eps relative
to the oracle's FP64 result (eps = 1e-6, and 1e-4 where stated); each test
prints the error it measured.

* single truncated additions (hm_trunc_batch) against the oracle's rkadd:
  the eps bound up to the FP32 rounding of the products, ranks within two of
  the oracle's;
* H-LU of the 2D 5-point Laplacian (64 x 64, leaf 32): the factors against
  the oracle's, standard and accumulated;
* H-LU of the 3D 7-point Laplacian (32^3, leaf 64): sampled blocks of the
  factors against the oracle's stored blocks (tests/golden), every admissible
  leaf's rank (a few may differ, by at most two), every leaf's norm and the
  product of the packed factors with a seeded vector;
* H-matrix product Z = G G of exact LU factors against the oracle's.
"""
import os

import numpy as np
import pytest

from paper_1703_09085_amd import workloads as W

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "bf16x3"]
MODES = ["standard", "accumulated"]
U32 = 2.0 ** -24
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lap3d_32_lu_eps1e-6")


@pytest.fixture(scope="module")
def ctx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_09085_amd import hm

    return hm, hm.Context()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("eps", [1e-6, 1e-4])
def test_trunc_batch_precision(ctx, oracle_lib, prec, eps):
    import torch
    from test_gpu_parity import dev

    hm, c = ctx
    rng = np.random.default_rng(41)
    descs, keep = [], []
    sizes = [(64, 64, 32, 32), (1, 40, 3, 2), (40, 1, 2, 3), (17, 63, 9, 40), (64, 20, 50, 50), (200, 50, 12, 12)]
    for i in range(40):
        if i < len(sizes):
            m, n, k1, k2 = sizes[i]
        else:
            m, n = int(rng.integers(1, 65)), int(rng.integers(1, 65))
            k1, k2 = int(rng.integers(1, 40)), int(rng.integers(0, 40))
        decay = float(rng.uniform(0.3, 0.9))
        A, B = W.lowrank_factors(m, n, k1, seed=500 + i, decay=decay)
        C_, D = W.lowrank_factors(m, n, k2, seed=600 + i, decay=decay, scale=0.7)
        tens = [dev(x) for x in (A, B, C_, D)]
        kcap = max(min(m, n, k1 + k2), 1)
        Co, Do = dev(np.zeros((m, kcap))), dev(np.zeros((n, kcap)))
        rk = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        descs.append(hm.TruncDesc(m=m, n=n, k1=k1, k2=k2, kcap=kcap, lda=m, ldb=n, ldc=m, ldd=n, alpha=-0.9,
                                  A=tens[0].data_ptr(), B=tens[1].data_ptr(), C=tens[2].data_ptr(),
                                  D=tens[3].data_ptr(), Cout=Co.data_ptr(), Dout=Do.data_ptr(),
                                  rank_out=rk.data_ptr()))
        keep.append((tens, Co, Do, rk, (A, B, C_, D)))
    assert c.trunc_batch(descs, eps, precision=prec) == len(descs)
    worst = 0.0
    for tens, Co, Do, rk, (A, B, C_, D) in keep:
        K = C_ @ D.T - 0.9 * A @ B.T
        Cr, Dr, sg = oracle_lib.rkadd(-0.9, A, B, C_, D, eps)
        k = int(rk.item())
        assert abs(k - Cr.shape[1]) <= 2
        Cg = Co.cpu().numpy().T[:, :k]
        Dg = Do.cpu().numpy().T[:, :k]
        nk = np.linalg.norm(K)
        # products rounded at FP32 level: |alpha| |A| |B| summed over the parts
        rnd = 64 * U32 * (0.9 * np.linalg.norm(A) * np.linalg.norm(B) + np.linalg.norm(C_) * np.linalg.norm(D))
        err = np.linalg.norm(K - Cg @ Dg.T)
        assert err <= 1.01 * eps * nk + rnd, (A.shape, B.shape, err / nk)
        worst = max(worst, err / nk)
        assert np.allclose(Cg.T @ Cg, np.eye(k), atol=1e-12)
    print(f"{prec} eps {eps:g}: worst relative truncation error {worst:.2e}", flush=True)


@pytest.fixture(scope="module")
def lap2d(ctx, oracle_lib):
    hm, c = ctx
    dims = (64, 64)
    x = W.grid_points(dims)
    rp, ci, v = W.laplacian_csr(dims)
    G0 = hm.HMatrix.from_csr(c, x, rp, ci, v, 32, 2.0, kmax=64)
    ref = {}
    for mode in MODES:
        H = oracle_lib.HMatrix.from_csr(x, rp, ci, v, 32, 2.0)
        H.lu(1e-6, mode)
        ref[mode] = H.to_dense()
    return G0, ref


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("prec", PRECS)
def test_lu_precision_lap2d(ctx, lap2d, mode, prec):
    hm, c = ctx
    G0, ref = lap2d
    G = G0.clone()
    info = hm.Plan.lu(c, G, mode).set_precision(prec).run(1e-6)
    assert info["status_bits"] == 0
    Do = ref[mode]
    rel = np.linalg.norm(G.to_dense() - Do) / np.linalg.norm(Do)
    print(f"lap2d_64 {mode} {prec}: relative error of the factors {rel:.2e}", flush=True)
    assert rel <= 10 * 1e-6


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("prec", PRECS)
def test_lu_precision_full_size(ctx, mode, prec):
    hm, c = ctx
    cfg = W.CONFIGS["lap3d_32"]
    x = W.grid_points(cfg["dims"])
    rp, ci, v = W.laplacian_csr(cfg["dims"])
    G = hm.HMatrix.from_csr(c, x, rp, ci, v, cfg["leaf"], cfg["eta"], kmax=96)
    info = hm.Plan.lu(c, G, mode).set_precision(prec).run(cfg["eps"])
    assert info["status_bits"] == 0
    golden = np.load(GOLDEN + ".npz")
    b, cl = G.blocks(), G.clusters()
    samples = golden[f"{mode}_samples"]
    pos, worst = 0, 0.0
    for i in golden[f"{mode}_pick"]:
        nr, nc = int(cl["size"][b["t"][i]]), int(cl["size"][b["s"][i]])
        ref = samples[pos:pos + nr * nc].reshape((nr, nc), order="F")
        pos += nr * nc
        got = G.block_to_dense(int(i), nr, nc)
        worst = max(worst, np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))
    print(f"lap3d_32 {mode} {prec}: {info['truncations']} truncations, worst relative error of the sampled "
          f"blocks {worst:.2e}", flush=True)
    assert worst <= 10 * cfg["eps"]
    # ranks of every admissible leaf against the FP64 oracle's: a singular
    # value within the reduced precision's rounding of the rule's threshold may
    # fall on the other side of it, so a few leaves may differ, by little
    ro = golden[f"{mode}_rank"].astype(np.int64)
    adm = b["kind"] == 1
    d = b["rank"][adm].astype(np.int64) - ro[adm]
    flips = int(np.count_nonzero(d))
    maxd = int(np.abs(d).max()) if d.size else 0
    # every leaf: its norm, and y = (packed factors) x for the seeded x
    norms = golden[f"{mode}_leaf_norm"]
    xv = np.random.default_rng(11).standard_normal(G.n)
    y = np.zeros(G.n)
    dn2 = n2 = 0.0
    worst_leaf = 0.0
    for i in np.nonzero(b["kind"] > 0)[0]:
        t, s = b["t"][i], b["s"][i]
        r0, nr, c0, nc = int(cl["off"][t]), int(cl["size"][t]), int(cl["off"][s]), int(cl["size"][s])
        got = G.block_to_dense(int(i), nr, nc)
        dn = abs(np.linalg.norm(got) - norms[i])
        dn2 += dn * dn
        n2 += norms[i] * norms[i]
        worst_leaf = max(worst_leaf, dn / max(norms[i], 1e-300))
        y[r0:r0 + nr] += got @ xv[c0:c0 + nc]
    ref = golden[f"{mode}_product"]
    rel_prod = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    rel_norms = np.sqrt(dn2 / n2)
    print(f"lap3d_32 {mode} {prec}: {flips} of {int(adm.sum())} admissible leaves differ in rank (at most by "
          f"{maxd}); leaf norms: aggregate {rel_norms:.2e}, worst leaf {worst_leaf:.2e}; product with the seeded "
          f"vector {rel_prod:.2e}", flush=True)
    assert flips <= max(1, int(adm.sum()) // 100) and maxd <= 2
    # |(|A| - |B|)| <= |A - B| leaf by leaf: the aggregate is bounded by the
    # factors' relative difference, as is the product's
    assert rel_norms <= 10 * cfg["eps"]
    assert rel_prod <= 10 * cfg["eps"]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("prec", PRECS)
def test_addmul_precision(ctx, oracle_lib, mode, prec):
    from test_gpu_parity import build_pair

    hm, c = ctx
    G, H = build_pair(c, oracle_lib, (16, 16), 8)
    G.lu(0.0, "standard")
    H.lu(0.0, "standard")
    Zg, Zo = G.zeros_like(), H.zeros_like()
    info = hm.Plan.addmul(c, 1.0, G, G, Zg, mode).set_precision(prec).run(1e-6)
    assert info["status_bits"] == 0
    Zo.addmul(1.0, H, H, 1e-6, mode)
    Do = Zo.to_dense()
    rel = np.linalg.norm(Zg.to_dense() - Do) / np.linalg.norm(Do)
    print(f"addmul {mode} {prec}: relative error {rel:.2e}", flush=True)
    assert rel <= 10 * 1e-6


def test_precision_rejects_unknown(ctx):
    hm, c = ctx
    x = W.grid_points((8, 8))
    rp, ci, v = W.laplacian_csr((8, 8))
    G = hm.HMatrix.from_csr(c, x, rp, ci, v, 4, 2.0, kmax=64)
    with pytest.raises(hm.HMError):
        hm.Plan.lu(c, G, "standard").set_precision(7)
