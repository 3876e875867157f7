"""Pins of the oracle's H-matrix inversion (Sect. 6: the six steps of the
block inversion, standard, and Fig. invert, accumulated).

* eps = 0: no truncation discards anything, so both variants must reproduce
  the dense inverse (LAPACK via NumPy) to rounding, on Laplacians (whose
  admissible blocks start at rank zero and fill in) and on the sphere kernel
  (admissible blocks of full numerical rank).
* eps > 0: the preconditioner error |I - G~^{-1} G|_2 (power iteration) stays
  small, the two variants agree to within the truncation bound, and the
  inverse of the Laplacian is a genuinely hierarchical matrix (its admissible
  blocks acquire rank).
"""
import numpy as np
import pytest

from paper_1703_09085_amd import workloads as W

MODES = ["standard", "accumulated"]


def lap(oracle_lib, dims, leaf):
    x = W.grid_points(dims)
    rp, ci, v = W.laplacian_csr(dims)
    return oracle_lib.HMatrix.from_csr(x, rp, ci, v, leaf, 2.0)


def power_error(G, Xinv, iters=60, seed=3):
    """|I - X G|_2 by power iteration on (I - X G)^T (I - X G)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(G.shape[0])
    v /= np.linalg.norm(v)
    s = 0.0
    for _ in range(iters):
        w = v - Xinv @ (G @ v)
        w = w - G.T @ (Xinv.T @ w)
        s = np.linalg.norm(w)
        if s == 0:
            return 0.0
        v = w / s
    return float(np.sqrt(s))


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("dims,leaf", [((8, 8), 2), ((16, 16), 4), ((12, 9), 4), ((6, 6, 6), 8)])
def test_inverse_eps0_is_dense_inverse(oracle_lib, mode, dims, leaf):
    H = lap(oracle_lib, dims, leaf)
    G = H.to_dense()
    st = H.inv(0.0, mode)
    Xi = H.to_dense()
    ref = np.linalg.inv(G)
    assert np.linalg.norm(Xi - ref) <= 1e-11 * np.linalg.norm(ref)
    assert st["leaf_lu"] == int((H.clusters()["son0"] < 0).sum())  # every diagonal leaf inverted once


@pytest.mark.parametrize("mode", MODES)
def test_inverse_eps0_kernel_matrix(oracle_lib, mode):
    x = W.sphere_points(260, seed=8)
    H = oracle_lib.HMatrix.from_kernel(x, 16, 2.0, 50.0, 0.0)
    G = H.to_dense()
    H.inv(0.0, mode)
    ref = np.linalg.inv(G)
    assert np.linalg.norm(H.to_dense() - ref) <= 1e-11 * np.linalg.norm(ref)


def test_inverse_truncated(oracle_lib):
    eps = 1e-6
    out = {}
    for mode in MODES:
        H = lap(oracle_lib, (32, 32), 8)
        G = H.to_dense()
        st = H.inv(eps, mode)
        X = H.to_dense()
        b = H.blocks()
        out[mode] = X
        err = power_error(G, X)
        print(mode, st, err)
        assert err <= 1e-4
        assert b["rank"][b["kind"] == 1].max() > 0  # the inverse is not sparse
        assert st["trunc_update"] + st["trunc_accum"] > 0
    ref = np.linalg.inv(lap(oracle_lib, (32, 32), 8).to_dense())
    for mode in MODES:
        assert np.linalg.norm(out[mode] - ref) <= 1e-4 * np.linalg.norm(ref)
    depth = 7
    assert np.linalg.norm(out["standard"] - out["accumulated"]) <= (depth + 1) * 1e3 * eps * np.linalg.norm(ref)
