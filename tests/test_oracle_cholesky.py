"""Pins of the oracle's H-Cholesky factorisation G = L L^T (Sect. 6 says it
is treated like the inversion; the reading is the design notes' R15).

* eps = 0: nothing is discarded, so L is the dense Cholesky factor (unique for
  an SPD matrix; LAPACK via NumPy) to rounding, on Laplacians and on the
  sphere kernel, for both variants.
* eps > 0: L L^T reproduces G to within a small multiple of eps, both
  variants agree to within the truncation bound, and the accumulated variant
  does fewer truncations of the factor's blocks (its Schur complements go to
  accumulators).
"""
import numpy as np
import pytest

from paper_1703_09085_amd import workloads as W

MODES = ["standard", "accumulated"]


def lap(oracle_lib, dims, leaf):
    x = W.grid_points(dims)
    rp, ci, v = W.laplacian_csr(dims)
    return oracle_lib.HMatrix.from_csr(x, rp, ci, v, leaf, 2.0)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("dims,leaf", [((8, 8), 2), ((16, 16), 4), ((13, 10), 4), ((6, 6, 6), 8)])
def test_cholesky_eps0_is_dense_cholesky(oracle_lib, mode, dims, leaf):
    H = lap(oracle_lib, dims, leaf)
    G = H.to_dense()
    st = H.chol(0.0, mode)
    L = np.tril(H.to_dense())
    ref = np.linalg.cholesky(G)
    assert np.linalg.norm(L - ref) <= 1e-12 * np.linalg.norm(ref)
    assert st["leaf_lu"] == int((H.clusters()["son0"] < 0).sum())


@pytest.mark.parametrize("mode", MODES)
def test_cholesky_eps0_kernel_matrix(oracle_lib, mode):
    x = W.sphere_points(300, seed=4)
    H = oracle_lib.HMatrix.from_kernel(x, 16, 2.0, 100.0, 0.0)
    G = H.to_dense()
    H.chol(0.0, mode)
    ref = np.linalg.cholesky(G)
    assert np.linalg.norm(np.tril(H.to_dense()) - ref) <= 1e-12 * np.linalg.norm(ref)


def test_cholesky_truncated(oracle_lib):
    eps = 1e-6
    out, st = {}, {}
    for mode in MODES:
        H = lap(oracle_lib, (40, 40), 8)
        G = H.to_dense()
        st[mode] = H.chol(eps, mode)
        L = np.tril(H.to_dense())
        out[mode] = L
        assert np.linalg.norm(L @ L.T - G) <= 20 * eps * np.linalg.norm(G)
        b = H.blocks()
        assert b["rank"][b["kind"] == 1].max() > 0
    ref = np.linalg.cholesky(lap(oracle_lib, (40, 40), 8).to_dense())
    depth = 8
    assert np.linalg.norm(out["standard"] - out["accumulated"]) <= (depth + 1) * 10 * eps * np.linalg.norm(ref)
    assert st["accumulated"]["trunc_update"] < st["standard"]["trunc_update"]
