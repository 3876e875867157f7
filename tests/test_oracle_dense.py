"""Pins of the oracle's dense kernels and of the truncated addition.

The truncated addition (Fig. rkadd) must return the best rank-k approximation
of the sum (Eckart-Young, Sect. 3 "Truncation"), with k chosen by the relative
Frobenius rule; its singular values are those of the dense sum.  LAPACK (via
NumPy) is the independent library routine these cases reduce to.
"""
import numpy as np
import pytest

from paper_1703_09085_amd import workloads as W


def rank_rule(s, eps):
    """k = smallest j with sum_{i>j} s_i^2 <= eps^2 sum_i s_i^2 (0 for a zero sum),
    with values at or below 1e-13 s_1 counted as zero (numerical rank in FP64)."""
    tail = np.concatenate([np.cumsum((s ** 2)[::-1])[::-1], [0.0]])
    if tail[0] == 0:
        return 0, np.inf
    thr = eps * eps * tail[0]
    k = int(np.nonzero(tail <= thr)[0][0])
    k = min(k, int(np.count_nonzero(s > 1e-13 * s[0])))
    margin = min(abs(tail[k] - thr), abs(tail[k - 1] - thr) if k > 0 else np.inf) / thr if thr > 0 else np.inf
    return k, margin


@pytest.mark.parametrize("m,n", [(7, 3), (3, 7), (6, 6), (40, 12), (1, 5), (5, 1)])
def test_qr_matches_lapack(oracle_lib, m, n):
    M = W.gaussian((m, n), seed=m * 100 + n)
    Q, R = oracle_lib.qr(M)
    q = min(m, n)
    assert np.allclose(Q @ R, M, atol=1e-13)
    assert np.allclose(Q.T @ Q, np.eye(q), atol=1e-13)
    assert np.allclose(np.tril(R, -1)[:, :q], 0)
    Rl = np.linalg.qr(M, mode="r")
    assert np.allclose(np.abs(np.diag(R)), np.abs(np.diag(Rl)), rtol=1e-12)


@pytest.mark.parametrize("m,n", [(7, 3), (3, 7), (9, 9), (50, 20), (1, 1)])
def test_svd_matches_lapack(oracle_lib, m, n):
    M = W.gaussian((m, n), seed=7 * m + n)
    U, S, V = oracle_lib.svd(M)
    r = min(m, n)
    assert np.allclose(S, np.linalg.svd(M, compute_uv=False), rtol=1e-12, atol=1e-14)
    assert np.all(np.diff(S) <= 0)
    assert np.allclose(U.T @ U, np.eye(r), atol=1e-12)
    assert np.allclose(V.T @ V, np.eye(r), atol=1e-12)
    assert np.allclose(U @ np.diag(S) @ V.T, M, atol=1e-12)


def test_svd_graded_and_rank_deficient(oracle_lib):
    rng = np.random.default_rng(3)
    u, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    v, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    s = 10.0 ** (-np.arange(12) * 12.0)  # 1 ... 1e-132
    s[8:] = 0
    M = (u * s) @ v.T
    U, S, V = oracle_lib.svd(M)
    assert np.allclose(U @ np.diag(S) @ V.T, M, atol=1e-15)
    assert abs(S[0] - 1) < 1e-14 and S[1] < 1e-11


CASES = [
    # m, n, k1, k2, eps, decay
    (30, 20, 5, 7, 1e-6, 0.3),
    (64, 48, 16, 16, 1e-6, 0.5),
    (20, 64, 10, 10, 1e-4, 0.6),
    (8, 8, 10, 9, 1e-6, 0.4),   # stacked rank exceeds the block size
    (40, 5, 6, 6, 1e-6, 0.5),   # k1 + k2 > n
    (33, 17, 1, 0, 1e-6, None),
    (50, 50, 12, 0, 1e-3, 0.5),  # k2 = 0: plain truncation of R1
]


@pytest.mark.parametrize("m,n,k1,k2,eps,decay", CASES)
def test_rkadd_is_best_approximation(oracle_lib, m, n, k1, k2, eps, decay):
    A, B = W.lowrank_factors(m, n, k1, seed=1 + m + k1, decay=decay)
    Cf, Df = W.lowrank_factors(m, n, k2, seed=2 + n + k2, decay=decay, scale=0.7)
    alpha = -0.8
    S = Cf @ Df.T + alpha * A @ B.T
    s_ref = np.linalg.svd(S, compute_uv=False)
    Cn, Dn, sg = oracle_lib.rkadd(alpha, A, B, Cf, Df, eps)
    q = min(m, n, k1 + k2)
    assert np.allclose(sg, s_ref[:q], rtol=1e-10, atol=1e-13 * s_ref[0])
    k = Cn.shape[1]
    k_ref, margin = rank_rule(s_ref[:q], eps)
    if margin > 1e-6:
        assert k == k_ref
    # Eckart-Young: the error is the discarded tail exactly
    err = np.linalg.norm(S - Cn @ Dn.T)
    assert err == pytest.approx(np.sqrt(np.sum(s_ref[k:] ** 2)), rel=1e-6, abs=1e-13 * s_ref[0])
    assert err <= eps * np.linalg.norm(S) * (1 + 1e-12) + 1e-14
    # C has orthonormal columns (Fig. rkadd: C = U(:, 1:k))
    assert np.allclose(Cn.T @ Cn, np.eye(k), atol=1e-12)


def test_rkadd_cancellation_gives_zero(oracle_lib):
    """R2 + (-1) R2 = 0: every computed singular value is rounding noise.

    The rule is relative to the block's own sum, so noise of similar size is
    not removed by it; the result is zero up to rounding."""
    A, B = W.lowrank_factors(25, 30, 6, seed=11, decay=0.5)
    Cn, Dn, sg = oracle_lib.rkadd(-1.0, A, B, A, B, 1e-8)
    assert np.all(sg <= 1e-14)
    assert np.linalg.norm(Cn @ Dn.T) <= 1e-14 * np.linalg.norm(A @ B.T)


def test_rkadd_exact_at_eps_zero(oracle_lib):
    A, B = W.lowrank_factors(20, 16, 9, seed=5, decay=0.1)
    C_, D = W.lowrank_factors(20, 16, 9, seed=6, decay=0.2)
    Cn, Dn, _ = oracle_lib.rkadd(1.3, A, B, C_, D, 0.0)
    S = C_ @ D.T + 1.3 * A @ B.T
    assert np.linalg.norm(Cn @ Dn.T - S) <= 1e-14 * np.linalg.norm(S)


@pytest.mark.parametrize("eps", [0.0, 1e-14])
def test_rkadd_numerical_rank(oracle_lib, eps):
    """Singular values at or below 1e-13 sigma_1 are rounding noise in FP64 and
    do not count towards the rank, also at eps = 0 (the sum's singular values
    are fixed by construction: U diag(s) V^T with orthonormal U, V)."""
    rng = np.random.default_rng(3)
    s = np.array([1.0, 1e-6, 1e-12, 5e-14, 1e-16])
    U = np.linalg.qr(rng.standard_normal((30, 5)))[0]
    V = np.linalg.qr(rng.standard_normal((24, 5)))[0]
    A, B = U[:, :3] * s[:3], V[:, :3]
    C_, D = U[:, 3:] * s[3:], V[:, 3:]
    Cn, Dn, sg = oracle_lib.rkadd(1.0, A, B, C_, D, eps)
    assert np.allclose(sg, s, rtol=1e-9, atol=1e-16)
    assert Cn.shape[1] == 3
    assert np.linalg.norm(Cn @ Dn.T - (U[:, :3] * s[:3]) @ V[:, :3].T) <= 1e-15


def test_rkadd_zero_columns_is_noop(oracle_lib):
    C_, D = W.lowrank_factors(10, 12, 4, seed=9, decay=0.5)
    Cn, Dn, _ = oracle_lib.rkadd(1.0, np.zeros((10, 0)), np.zeros((12, 0)), C_, D, 0.5)
    assert np.array_equal(Cn, C_) and np.array_equal(Dn, D)


@pytest.mark.parametrize("eps", [0.0, 1e-6, 1e-3])
def test_rkmerge_recovers_block(oracle_lib, eps):
    rng = np.random.default_rng(4)
    m0, m1, n0, n1 = 9, 7, 8, 11
    # a smooth global low-rank block, cut into four pieces (Sect. 3 "Splitting and merging")
    U, V = W.lowrank_factors(m0 + m1, n0 + n1, 6, seed=21, decay=0.2)
    full = U @ V.T
    pieces = []
    for i, (r0, r1) in enumerate([(0, m0), (m0, m0 + m1)]):
        for j, (c0, c1) in enumerate([(0, n0), (n0, n0 + n1)]):
            k = 6 + i + j  # redundant columns
            extra = rng.standard_normal((r1 - r0, k - 6))
            A = np.hstack([U[r0:r1], extra])
            B = np.hstack([V[c0:c1], np.zeros((c1 - c0, k - 6))])
            pieces.append((A, B))
    A, B = oracle_lib.rkmerge22(m0, m1, n0, n1, pieces, eps)
    err = np.linalg.norm(A @ B.T - full) / np.linalg.norm(full)
    # two truncation stages, each relative to its own input
    assert err <= max(2.0 * eps * 1.01, 1e-14)
    if eps == 0.0:
        assert A.shape[1] == 6 or err < 1e-14
