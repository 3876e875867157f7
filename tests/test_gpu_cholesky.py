"""GPU H-Cholesky G = L L^T through the C ABI against the CPU oracle (the
reading R15 of Sect. 6): the factor's blocks on and below the diagonal agree
to 1e-10 relative (FP64 path), equal ranks in every admissible leaf below the
diagonal (up to noise-level ties), equal truncation counts (up to the effect
of those ties and of exactly cancelling sums); at eps = 0 the dense Cholesky
factor; on the GPU-built sphere kernel matrix, L L^T reproduces G."""
import numpy as np
import pytest

from paper_1703_09085_amd import workloads as W
from test_gpu_parity import build_pair, oracle_run_logged, oracle_truncs

pytestmark = pytest.mark.gpu

MODES = ["standard", "accumulated"]


@pytest.fixture(scope="module")
def ctx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_09085_amd import hm

    return hm.Context()


def lower_ranks(M):
    """Ranks of the admissible leaves below the diagonal (cluster order)."""
    b, c = M.blocks(), M.clusters()
    below = c["off"][b["t"]] > c["off"][b["s"]]
    return np.where((b["kind"] == 1) & below, b["rank"], -1)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("dims,leaf,eps", [((16, 16), 8, 0.0), ((32, 32), 8, 1e-6), ((23, 19), 8, 1e-6),
                                           ((8, 8, 8), 16, 1e-6), ((64, 64), 32, 1e-6)])
def test_cholesky_matches_oracle(ctx, oracle_lib, mode, dims, leaf, eps):
    G, H = build_pair(ctx, oracle_lib, dims, leaf)
    A = G.to_dense()
    print(f"cholesky {mode} {dims} leaf {leaf} eps {eps:g}", flush=True)
    info = G.chol(eps, mode)
    st, cancelled = oracle_run_logged(lambda: H.chol(eps, mode))
    Lg, Lo = np.tril(G.to_dense()), np.tril(H.to_dense())
    rel = np.linalg.norm(Lg - Lo) / np.linalg.norm(Lo)
    print(f"  {info['truncations']} truncations (oracle {oracle_truncs(st)}), relative difference {rel:.2e}",
          flush=True)
    assert rel <= 1e-10
    if eps == 0:
        ref = np.linalg.cholesky(A)
        assert np.linalg.norm(Lg - ref) <= 1e-12 * np.linalg.norm(ref)
        return
    rg, ro = lower_ranks(G), lower_ranks(H)
    bad = np.nonzero(rg != ro)[0]
    c, b = H.clusters(), H.blocks()
    for i in bad:  # only noise-level blocks may differ in rank
        t, s = b["t"][i], b["s"][i]
        blk = Lo[c["off"][t]: c["off"][t] + c["size"][t], c["off"][s]: c["off"][s] + c["size"][s]]
        assert np.linalg.norm(blk) <= 1e-12 * np.linalg.norm(Lo), i
    assert abs(info["truncations"] - oracle_truncs(st)) <= 4 * (len(bad) + cancelled)


@pytest.mark.parametrize("mode", MODES)
def test_cholesky_kernel_matrix(ctx, mode):
    from paper_1703_09085_amd import hm

    x = W.sphere_points(2048, seed=31)
    G = hm.HMatrix.from_kernel(ctx, x, 32, 2.0, 1e3, 1e-8, kmax=64)
    A = G.to_dense()
    print(f"sphere cholesky {mode}", flush=True)
    G.chol(1e-6, mode)
    L = np.tril(G.to_dense())
    err = np.linalg.norm(L @ L.T - A) / np.linalg.norm(A)
    print(f"  |L L^T - G| / |G| = {err:.2e}", flush=True)
    assert err <= 1e-5
