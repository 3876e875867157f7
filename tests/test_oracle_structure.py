"""Pins of the oracle's cluster tree, block tree and assembly.

Checked against the definitions (Defs. cluster tree / block tree, Sect. 2),
against an independent brute-force bisection written here, and against the
product-tree identity (eq. product_block, Sect. 5).
"""
import numpy as np
import pytest

from paper_1703_09085_amd import workloads as W


def brute_clusters(x, leaf):
    """Independent geometric bisection: list of (indices, level) in pre-order."""
    out = []

    def rec(idx, level):
        pts = x[idx]
        lo, hi = pts.min(axis=0), pts.max(axis=0)
        ext = hi - lo
        axis = int(np.argmax(ext))  # first maximal axis
        me = len(out)
        out.append((idx, level))
        if len(idx) > leaf and ext[axis] > 0:
            mid = 0.5 * (lo[axis] + hi[axis])
            left = idx[pts[:, axis] <= mid]
            right = idx[pts[:, axis] > mid]
            rec(left, level + 1)
            rec(right, level + 1)
        return me

    rec(np.arange(len(x)), 0)
    return out


def build(dims, leaf, oracle_lib):
    x = W.grid_points(dims)
    rp, ci, v = W.laplacian_csr(dims)
    return x, (rp, ci, v), oracle_lib.HMatrix.from_csr(x, rp, ci, v, leaf, 2.0)


@pytest.mark.parametrize("dims,leaf", [((16, 16), 8), ((12, 9), 5), ((6, 5, 4), 8)])
def test_cluster_tree_matches_bruteforce(oracle_lib, dims, leaf):
    x, _, H = build(dims, leaf, oracle_lib)
    c = H.clusters()
    perm = H.perm()
    ref = brute_clusters(x, leaf)
    assert len(ref) == len(c["off"])
    for i, (idx, level) in enumerate(ref):
        got = perm[c["off"][i]: c["off"][i] + c["size"][i]]
        assert np.array_equal(np.sort(got), np.sort(idx)), i
        if c["son0"][i] < 0:  # inside a leaf the original order is kept
            assert np.array_equal(got, idx), i
        assert c["level"][i] == level


@pytest.mark.parametrize("dims,leaf,depth,nleaves", [((64, 64), 32, 7, 128), ((16, 16), 8, 5, 32)])
def test_balanced_depths(oracle_lib, dims, leaf, depth, nleaves):
    _, _, H = build(dims, leaf, oracle_lib)
    c = H.clusters()
    isleaf = c["son0"] < 0
    assert c["level"].max() == depth
    assert isleaf.sum() == nleaves
    assert np.all(c["size"][isleaf] <= leaf)
    assert sorted(np.bincount(c["size"][isleaf]).nonzero()[0]) == [leaf]


def block_info(H):
    c = H.clusters()
    b = H.blocks()
    return c, b


@pytest.mark.parametrize("dims,leaf", [((16, 16), 8), ((64, 64), 32), ((6, 5, 4), 8)])
def test_block_tree_definition(oracle_lib, dims, leaf):
    x, _, H = build(dims, leaf, oracle_lib)
    perm = H.perm()
    c, b = block_info(H)
    n = len(perm)
    cover = np.zeros((n, n), dtype=np.int32)
    kids = {}
    for i, p in enumerate(b["parent"]):
        kids.setdefault(int(p), []).append(i)
    sons = {j: [c["son0"][j], c["son1"][j]] for j in range(len(c["off"])) if c["son0"][j] >= 0}
    for i in range(len(b["t"])):
        t, s, kind = b["t"][i], b["s"][i], b["kind"][i]
        if kind == 0:
            got = [(b["t"][j], b["s"][j]) for j in kids[i]]
            assert got == [(a, bb) for a in sons[t] for bb in sons[s]]  # sons(t) x sons(s), row-major
            continue
        r0, r1 = c["off"][t], c["off"][t] + c["size"][t]
        c0, c1 = c["off"][s], c["off"][s] + c["size"][s]
        cover[r0:r1, c0:c1] += 1
        pt, ps = x[perm[r0:r1]], x[perm[c0:c1]]
        dt = np.sum((pt.max(0) - pt.min(0)) ** 2)
        ds = np.sum((ps.max(0) - ps.min(0)) ** 2)
        gap = np.maximum(0, np.maximum(ps.min(0) - pt.max(0), pt.min(0) - ps.max(0)))
        dist = np.sum(gap ** 2)
        if kind == 1:
            assert dist > 0 and max(dt, ds) <= 4.0 * dist
        else:
            # admissible block tree: an inadmissible leaf has a leaf cluster (Sect. 3)
            assert t not in sons or s not in sons
            assert not (dist > 0 and max(dt, ds) <= 4.0 * dist)
    assert np.all(cover == 1)  # leaves partition I x I


def test_laplacian_assembly_exact(oracle_lib):
    dims = (64, 64)
    x, (rp, ci, v), H = build(dims, 32, oracle_lib)
    n = x.shape[0]
    p = H.perm()
    A = W.csr_to_dense(rp, ci, v, n)[np.ix_(p, p)]
    assert np.array_equal(H.to_dense(), A)
    b = H.blocks()
    assert np.all(b["rank"][b["kind"] == 1] == 0)  # local rank zero (Sect. 3)


def test_product_tree_count(oracle_lib):
    """addproduct is called once per product (t,s,r) with (t,s), (s,r) blocks."""
    x, _, H = build((16, 16), 8, oracle_lib)
    b = H.blocks()
    by_row = {}
    for t, s in zip(b["t"], b["s"]):
        by_row.setdefault(int(t), []).append(int(s))
    blocks = set(zip(b["t"].tolist(), b["s"].tolist()))
    count = sum(1 for (t, s) in blocks for r in by_row.get(s, []) if (s, r) in blocks)
    Z = H.zeros_like()
    st = Z.addmul(1.0, H, H, 1e-6, "accumulated")
    assert st["addproduct"] == count
