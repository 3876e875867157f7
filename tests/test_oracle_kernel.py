"""Pins of the oracle's kernel-matrix build and of its truncation work.

Kernel build (the sphere workload, a stand-in for the boundary-element
matrices of Sect. 7): inadmissible leaves hold the kernel 1/|x - y| with the
diagonal set to a given value; every admissible leaf holds the best
rank-k approximation of its dense block (Eckart-Young, Sect. 3 "Truncation"),
k from the relative Frobenius rule at the build tolerance.  LAPACK's SVD (via
NumPy) of each dense block is the independent routine the check reduces to.

Truncation work: the Theorem "Complexity" of Sect. 5 bounds the low-rank
update work of the accumulated algorithm by O(n k^2 log n) against
O(n k^2 log^2 n) for the standard one; Sect. 6 carries the same pattern over
to the factorisations.  The oracle's logged work per unknown must therefore
grow at most linearly in log n for accumulated updates and faster than
linearly for standard updates.
"""
import numpy as np
import pytest

from paper_1703_09085_amd import workloads as W
from test_oracle_dense import rank_rule


def kernel_dense(x, diag):
    d = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(axis=2))
    with np.errstate(divide="ignore"):
        G = 1.0 / d
    np.fill_diagonal(G, diag)
    return G


def leaf_blocks(H):
    b, c = H.blocks(), H.clusters()
    for i in range(len(b["kind"])):
        if b["kind"][i] == 0:
            continue
        t, s = b["t"][i], b["s"][i]
        yield (b["kind"][i], b["rank"][i], c["off"][t], c["size"][t], c["off"][s], c["size"][s])


@pytest.mark.parametrize("n,leaf,eps", [(700, 16, 1e-5), (500, 24, 1e-3)])
def test_kernel_build_is_truncated_svd(oracle_lib, n, leaf, eps):
    x = W.sphere_points(n, seed=11 + n)
    H = oracle_lib.HMatrix.from_kernel(x, leaf, 2.0, 1e3, eps)
    perm = H.perm()
    G = kernel_dense(x[perm], 1e3)  # cluster order
    D = H.to_dense()
    nadm = ntie = 0
    for kind, rank, ro, m, co, nn in leaf_blocks(H):
        ref = G[ro:ro + m, co:co + nn]
        got = D[ro:ro + m, co:co + nn]
        if kind == 2:
            # near field: the kernel itself, the diagonal value on the diagonal
            assert np.allclose(got, ref, rtol=1e-15, atol=0), (ro, co)
            if ro == co:
                assert np.all(np.diag(got) == 1e3)
            continue
        nadm += 1
        u, s, vt = np.linalg.svd(ref, full_matrices=False)
        k, margin = rank_rule(s, eps)
        if margin < 1e-8:
            ntie += 1
            continue
        assert rank == k, (ro, co, rank, k)
        assert k > 0
        # the stored block is U_k S_k V_k^T (unique when s_k > s_{k+1})
        best = (u[:, :k] * s[:k]) @ vt[:k]
        assert np.linalg.norm(got - best) <= 1e-11 * s[0], (ro, co)
        err2 = np.linalg.norm(ref - got) ** 2
        tail = float((s[k:] ** 2).sum())
        assert err2 <= eps * eps * float((s ** 2).sum()) * (1 + 1e-8) + 1e-26 * s[0] ** 2
        assert abs(err2 - tail) <= 1e-8 * tail + 1e-24 * s[0] ** 2
    assert nadm >= 20 and ntie <= nadm // 50


def test_kernel_build_eps0_is_exact(oracle_lib):
    x = W.sphere_points(400, seed=5)
    H = oracle_lib.HMatrix.from_kernel(x, 16, 2.0, 1e3, 0.0)
    G = kernel_dense(x[H.perm()], 1e3)
    D = H.to_dense()
    assert np.linalg.norm(D - G) <= 1e-12 * np.linalg.norm(G)
    assert (H.blocks()["kind"] == 1).sum() > 10


@pytest.mark.slow
def test_truncation_work_slope(oracle_lib):
    """Truncation work per unknown, W(n)/n with W = sum (m + n) l^2 over all
    truncations of the H-LU, on 5-point Laplacians of 32^2 ... 256^2 points
    (leaf 16): its second differences in log2 n are positive for standard
    updates (a log^2 n term) and not positive for accumulated updates (at
    most linear in log n), and accumulated updates do more work per unknown
    at the small sizes but gain on standard ones as n grows."""
    w = {"standard": [], "accumulated": []}
    for N in (32, 64, 128, 256):
        x = W.grid_points((N, N))
        rp, ci, v = W.laplacian_csr((N, N))
        for mode in w:
            H = oracle_lib.HMatrix.from_csr(x, rp, ci, v, 16, 2.0)
            st = H.lu(1e-6, mode)
            w[mode].append(st["trunc_flops"] / (N * N))
    ws, wa = np.array(w["standard"]), np.array(w["accumulated"])
    d2s, d2a = np.diff(ws, 2), np.diff(wa, 2)
    assert np.all(d2s > 0.02 * ws[-1]), ws
    assert np.all(d2a <= 0.02 * wa[-1]), wa
    ratio = wa / ws
    assert np.all(np.diff(ratio) < 0), ratio
