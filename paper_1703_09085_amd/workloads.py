"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This module only generates inputs: point sets, sparse stiffness matrices in CSR
form and random low-rank factors.  It contains none of the hierarchical-matrix
arithmetic, so both the GPU library and the CPU oracle can take their inputs
from it without sharing any of the method's code.

The paper's experiments use boundary-element matrices on the unit sphere
(Sect. 7).  The workloads here stand in for them: finite-difference Laplacians
(stiffness matrices of local rank zero, Sect. 3) whose H-LU factors acquire
low-rank blocks, and the kernel 1/|x-y| on random points of the unit sphere.
"""
from __future__ import annotations

import numpy as np

# Workload definitions (cluster tree by geometric bisection, admissibility
# max(diam) <= eta * dist, relative Frobenius truncation eps).
CONFIGS = {
    "lap2d_64": dict(kind="laplace", dims=(64, 64), leaf=32, eta=2.0, eps=1e-6),
    "lap3d_32": dict(kind="laplace", dims=(32, 32, 32), leaf=64, eta=2.0, eps=1e-6),
    "sphere_65536": dict(kind="sphere", n=65536, leaf=64, eta=2.0, eps=1e-5, seed=1703),
    "lap2d_batch64": dict(kind="laplace_batch", count=64, side_lo=32, side_hi=128, seed=4,
                          leaf=32, eta=2.0, eps=1e-6),
    "lap3d_64": dict(kind="laplace", dims=(64, 64, 64), leaf=64, eta=2.0, eps=1e-6),
    # the paper's experiments: Galerkin single / double layer on the refined
    # double pyramid, truncation tolerance 1e-4 (m = 64: n = 32768)
    "bem_single_64": dict(kind="bem", layer="single", m=64, leaf=64, eta=2.0, eps=1e-4),
    "bem_double_64": dict(kind="bem", layer="double", m=64, leaf=64, eta=2.0, eps=1e-4),
}


def grid_points(dims):
    """Integer lattice coordinates 1..N_d of the interior grid points.

    Points are numbered lexicographically with the first axis fastest.
    Returns an (n, dim) float64 array.
    """
    dims = tuple(int(d) for d in dims)
    axes = [np.arange(1, d + 1, dtype=np.float64) for d in dims]
    mesh = np.meshgrid(*axes, indexing="ij")
    # first axis fastest: flatten in Fortran order
    return np.stack([m.ravel(order="F") for m in mesh], axis=1)


def laplacian_csr(dims):
    """(2d+1)-point finite-difference Laplacian with Dirichlet boundary.

    Diagonal 2*dim, -1 for each grid neighbour inside the domain (boundary
    unknowns eliminated, unscaled).  Index numbering as in grid_points.
    Returns (rowptr int64, colind int32, vals float64).
    """
    dims = tuple(int(d) for d in dims)
    dim = len(dims)
    n = int(np.prod(dims))
    idx = np.arange(n).reshape(dims, order="F")
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [np.full(n, 2.0 * dim)]
    for ax in range(dim):
        lo = [slice(None)] * dim
        hi = [slice(None)] * dim
        lo[ax] = slice(0, dims[ax] - 1)
        hi[ax] = slice(1, dims[ax])
        a = idx[tuple(lo)].ravel(order="F")
        b = idx[tuple(hi)].ravel(order="F")
        rows += [a, b]
        cols += [b, a]
        vals += [np.full(a.size, -1.0), np.full(b.size, -1.0)]
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int64)
    return rowptr, c.astype(np.int32), v.astype(np.float64)


def csr_to_dense(rowptr, colind, vals, n):
    a = np.zeros((n, n))
    for i in range(n):
        for e in range(rowptr[i], rowptr[i + 1]):
            a[i, colind[e]] += vals[e]
    return a


def sphere_points(n, seed=1703):
    """n points uniform on the unit sphere: g / |g| with g ~ N(0, I_3), PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def double_pyramid_mesh(m):
    """The surface mesh of the paper's boundary-element experiments: the double
    pyramid (octahedron) with every face refined regularly into m^2 triangles
    and all vertices projected to the unit sphere; n = 8 m^2 flat triangles.
    Returns an (n, 3, 3) float64 array of vertex coordinates, each triangle's
    vertices ordered so that (v1 - v0) x (v2 - v0) points away from the
    origin (outward normals)."""
    m = int(m)
    e = np.eye(3)
    i, j = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    up = i + j < m  # triangles (i, j), (i + 1, j), (i, j + 1)
    dn = i + j < m - 1  # triangles (i + 1, j), (i + 1, j + 1), (i, j + 1)
    iu, ju, idn, jdn = i[up], j[up], i[dn], j[dn]
    out = []
    for sx in (1.0, -1.0):
        for sy in (1.0, -1.0):
            for sz in (1.0, -1.0):
                a, b, c = sx * e[0], sy * e[1], sz * e[2]

                def pt(ii, jj):
                    p = ((m - ii - jj)[:, None] * a + ii[:, None] * b + jj[:, None] * c) / m
                    return p / np.linalg.norm(p, axis=1, keepdims=True)

                t_up = np.stack([pt(iu, ju), pt(iu + 1, ju), pt(iu, ju + 1)], axis=1)
                t_dn = np.stack([pt(idn + 1, jdn), pt(idn + 1, jdn + 1), pt(idn, jdn + 1)], axis=1)
                out += [t_up, t_dn]
    T = np.concatenate(out)
    nrm = np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0])
    flip = (nrm * T.mean(axis=1)).sum(axis=1) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    return np.ascontiguousarray(T)


def batch_sides(count=64, lo=32, hi=128, seed=4):
    """Side lengths of the batched 2D Laplacians, uniform on {lo..hi}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi + 1, size=count)


def lowrank_factors(m, n, k, seed, decay=None, scale=1.0):
    """Random factors A (m x k), B (n x k) with A B^T = U diag(s) V^T.

    U, V have orthonormal columns; s_i = scale * decay**i (decay None gives
    s_i = scale).  Column-major float64 arrays (Fortran order).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if k == 0:
        return np.zeros((m, 0), order="F"), np.zeros((n, 0), order="F")
    u, _ = np.linalg.qr(rng.standard_normal((m, k)))
    v, _ = np.linalg.qr(rng.standard_normal((n, k)))
    u = u[:, :k] if u.shape[1] >= k else np.pad(u, ((0, 0), (0, k - u.shape[1])))
    v = v[:, :k] if v.shape[1] >= k else np.pad(v, ((0, 0), (0, k - v.shape[1])))
    s = scale * (np.ones(k) if decay is None else decay ** np.arange(k))
    return np.asfortranarray(u * s), np.asfortranarray(v)


def gaussian(shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.asfortranarray(rng.standard_normal(shape))
