"""Pins of the oracle's H-matrix arithmetic.

* addeval / addevaltrans equal dense products (Fig. addeval).
* Standard and accumulated multiplication reproduce the dense product exactly
  (up to rounding) at eps = 0, and within the truncation bound at eps > 0.
* Standard and accumulated H-LU reproduce the unique unpivoted LU at eps = 0
  (checked against LAPACK's partial-pivoting LU, which does not pivot on these
  diagonally dominant matrices) and give a small preconditioner error at eps > 0.
"""
import numpy as np
import pytest
import scipy.linalg

from paper_1703_09085_amd import workloads as W

MODES = ["standard", "accumulated"]


def lap(dims, leaf, oracle_lib):
    x = W.grid_points(dims)
    rp, ci, v = W.laplacian_csr(dims)
    H = oracle_lib.HMatrix.from_csr(x, rp, ci, v, leaf, 2.0)
    p = H.perm()
    A = W.csr_to_dense(rp, ci, v, x.shape[0])[np.ix_(p, p)]
    return H, A


@pytest.fixture(scope="module")
def factored(oracle_lib):
    """An H-matrix with non-trivial low-rank blocks: the exact LU factors."""
    H, A = lap((16, 16), 8, oracle_lib)
    G = H.clone()
    G.lu(0.0, "standard")
    return H, A, G


def test_addeval_dense(factored):
    H, A, G = factored
    D = G.to_dense()
    c = G.clusters()
    b = G.blocks()
    rng = np.random.default_rng(0)
    for i in [0, 1, 5, 17, len(b["t"]) - 1]:
        t, s = b["t"][i], b["s"][i]
        rt = slice(c["off"][t], c["off"][t] + c["size"][t])
        rs = slice(c["off"][s], c["off"][s] + c["size"][s])
        w = rng.standard_normal((c["size"][s], 3))
        y = rng.standard_normal((c["size"][t], 3))
        out = G.addeval_block(i, w, y, alpha=-0.5)
        assert np.allclose(out, y - 0.5 * D[rt, rs] @ w, atol=1e-12)
        out = G.addeval_block(i, y, w, alpha=2.0, trans=True)
        assert np.allclose(out, w + 2.0 * D[rt, rs].T @ y, atol=1e-12)


@pytest.mark.parametrize("mode", MODES)
def test_mul_exact_at_eps_zero(factored, mode):
    H, A, G = factored
    D = G.to_dense()
    Z = G.zeros_like()
    Z.addmul(1.0, G, G, 0.0, mode)
    assert np.linalg.norm(Z.to_dense() - D @ D) <= 1e-13 * np.linalg.norm(D @ D)
    Z = G.clone()
    Z.addmul(-1.0, H, G, 0.0, mode)
    ref = D - A @ D
    assert np.linalg.norm(Z.to_dense() - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("eps", [1e-3, 1e-6])
def test_mul_error_bound_and_agreement(factored, eps):
    H, A, G = factored
    D = G.to_dense()
    ref = D @ D
    out = {}
    for mode in MODES:
        Z = G.zeros_like()
        Z.addmul(1.0, G, G, eps, mode)
        out[mode] = Z.to_dense()
        depth = int(G.clusters()["level"].max())
        # each truncation is relative to its own block; the accumulated
        # variant truncates once more per level it passes (bound (p+1) eps)
        assert np.linalg.norm(out[mode] - ref) <= (depth + 1) * eps * np.linalg.norm(ref)
    diff = np.linalg.norm(out["standard"] - out["accumulated"])
    assert diff <= 2 * (depth + 1) * eps * np.linalg.norm(ref)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("dims,leaf", [((16, 16), 8), ((8, 8, 4), 16)])
def test_lu_exact_at_eps_zero(oracle_lib, mode, dims, leaf):
    H, A = lap(dims, leaf, oracle_lib)
    G = H.clone()
    G.lu(0.0, mode)
    D = G.to_dense()
    n = A.shape[0]
    L = np.tril(D, -1) + np.eye(n)
    R = np.triu(D)
    P, Ll, Rl = scipy.linalg.lu(A)
    assert np.array_equal(P, np.eye(n))  # no pivoting needed: the unpivoted LU is unique
    assert np.allclose(L, Ll, atol=1e-12)
    assert np.allclose(R, Rl, atol=1e-12)


def power_error(A, solve, iters=60, seed=0):
    """Estimate ||I - (LR)^{-1} A||_2 by power iteration on M^T M."""
    n = A.shape[0]
    x = np.random.default_rng(seed).standard_normal(n)
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = x - solve(A @ x)
        # M^T y with M = I - S A, M^T = I - A^T S^T; use the dense inverse of S
        lam = np.linalg.norm(y)
        x = y / lam
    return lam


@pytest.mark.parametrize("mode", MODES)
def test_lu_truncated_accuracy(oracle_lib, mode):
    H, A = lap((32, 32), 16, oracle_lib)
    eps = 1e-6
    G = H.clone()
    st = G.lu(eps, mode)
    D = G.to_dense()
    n = A.shape[0]
    L = np.tril(D, -1) + np.eye(n)
    R = np.triu(D)
    rel = np.linalg.norm(L @ R - A) / np.linalg.norm(A)
    assert rel < 50 * eps
    S = np.linalg.inv(L @ R)
    err2 = np.linalg.norm(np.eye(n) - S @ A, 2)
    assert err2 < 1e-2
    # the H-matrix solve agrees with the dense factors
    b = np.random.default_rng(1).standard_normal(n)
    assert np.allclose(G.lu_solve(b)[:, 0] if G.lu_solve(b).ndim == 2 else G.lu_solve(b), S @ b,
                       rtol=1e-9, atol=1e-9)
    assert st["leaf_lu"] == 64


def test_std_acc_lu_agree(oracle_lib):
    H, A = lap((32, 32), 16, oracle_lib)
    eps = 1e-6
    out = {}
    for mode in MODES:
        G = H.clone()
        G.lu(eps, mode)
        D = G.to_dense()
        n = A.shape[0]
        out[mode] = (np.tril(D, -1) + np.eye(n)) @ np.triu(D)
    depth = 6
    diff = np.linalg.norm(out["standard"] - out["accumulated"]) / np.linalg.norm(A)
    assert diff <= (depth + 1) * eps


def test_accumulated_mul_fewer_leaf_updates(oracle_lib):
    """Each accumulator is pushed to its sons once: the final updates of Z
    leaves number at most the leaves of Z (plus merge temporaries)."""
    H, A = lap((16, 16), 8, oracle_lib)
    G = H.clone()
    G.lu(1e-8, "standard")
    Z1 = G.zeros_like()
    s_std = Z1.addmul(1.0, G, G, 1e-8, "standard")
    Z2 = G.zeros_like()
    s_acc = Z2.addmul(1.0, G, G, 1e-8, "accumulated")
    assert s_acc["trunc_update"] < s_std["trunc_update"]
    assert s_acc["dense_updates"] < s_std["dense_updates"]
    b = G.blocks()
    assert s_acc["dense_updates"] <= (b["kind"] == 2).sum()
