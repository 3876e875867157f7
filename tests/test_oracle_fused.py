"""Pins of the oracle's fused accumulation (reading R16: in a split, the
products that reach one accumulator are truncated three at a time together
with it, in one truncation of the stacked sum).

* The stacked truncated addition equals the best rank-k approximation of the
  dense sum (Eckart-Young; LAPACK's SVD via NumPy), k by the relative
  Frobenius rule; updates without columns add nothing.
* eps = 0: the fused multiplication and H-LU reproduce the dense product and
  the dense unpivoted LU to rounding.
* eps > 0: within the truncation bound of the unfused accumulated results,
  with fewer accumulator truncations.
"""
import numpy as np
import pytest

from paper_1703_09085_amd import workloads as W
from test_oracle_dense import rank_rule


@pytest.mark.parametrize("m,n,ks,k2,eps", [(40, 30, [3, 5, 2], 6, 1e-6), (20, 50, [7, 0, 4], 3, 1e-4),
                                            (12, 12, [9, 9], 8, 1e-6), (30, 25, [0, 0], 4, 1e-6)])
def test_rkadd_multi_is_best_approximation(oracle_lib, m, n, ks, k2, eps):
    ups = []
    for q, k in enumerate(ks):
        A, B = W.lowrank_factors(m, n, k, seed=10 + q, decay=0.5)
        ups.append((-0.7 + 0.3 * q, A, B))
    C_, D = W.lowrank_factors(m, n, k2, seed=99, decay=0.5, scale=0.8)
    Co, Do = oracle_lib.rkadd_multi(ups, C_, D, eps)
    if sum(ks) == 0:
        assert np.allclose(Co @ Do.T, C_ @ D.T, atol=1e-15)  # nothing added: unchanged
        return
    S = C_ @ D.T + sum(a * A @ B.T for a, A, B in ups)
    u, s, vt = np.linalg.svd(S)
    k, margin = rank_rule(s, eps)
    assert margin > 1e-8 and Co.shape[1] == k
    best = (u[:, :k] * s[:k]) @ vt[:k]
    assert np.linalg.norm(Co @ Do.T - best) <= 1e-12 * np.linalg.norm(S)
    assert np.allclose(Co.T @ Co, np.eye(k), atol=1e-12)


def lap(oracle_lib, dims, leaf):
    x = W.grid_points(dims)
    rp, ci, v = W.laplacian_csr(dims)
    return oracle_lib.HMatrix.from_csr(x, rp, ci, v, leaf, 2.0)


@pytest.mark.parametrize("dims,leaf", [((16, 16), 4), ((6, 6, 6), 8)])
def test_fused_eps0_exact(oracle_lib, dims, leaf):
    H = lap(oracle_lib, dims, leaf)
    A = H.to_dense()
    H.lu(0.0, "fused")
    F = H.to_dense()
    L = np.tril(F, -1) + np.eye(A.shape[0])
    R = np.triu(F)
    assert np.linalg.norm(L @ R - A) <= 1e-12 * np.linalg.norm(A)
    G = lap(oracle_lib, dims, leaf)
    G.lu(0.0, "standard")  # operands with non-trivial low-rank blocks
    Z = G.zeros_like()
    Z.addmul(1.0, G, G, 0.0, "fused")
    D = G.to_dense()
    assert np.linalg.norm(Z.to_dense() - D @ D) <= 1e-12 * np.linalg.norm(D @ D)


def test_fused_truncated(oracle_lib):
    eps = 1e-6
    out, st = {}, {}
    for mode in ("accumulated", "fused"):
        H = lap(oracle_lib, (48, 48), 8)
        st[mode] = H.lu(eps, mode)
        out[mode] = H.to_dense()
    ref = out["accumulated"]
    depth = 8
    assert np.linalg.norm(out["fused"] - ref) <= (depth + 1) * eps * np.linalg.norm(ref)
    assert st["fused"]["trunc_accum"] < st["accumulated"]["trunc_accum"]
    assert st["fused"]["products"] == st["accumulated"]["products"]
