"""ctypes wrapper of the plain FP64 CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: the oracle is the independent reference the GPU
library is checked against.  Only the tests, the smoke check and the CPU
baseline of the benchmark may import this package.  It shares no code with the
GPU library (paper_1703_09085_amd).

Every function follows the paper (Boerm, "Hierarchical matrix arithmetic with
accumulated updates"); the C++ source cites the section or figure of each step.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hm_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

STAT_NAMES = ["trunc_update", "trunc_accum", "trunc_merge", "dense_updates", "addproduct",
              "pending", "products", "leaf_lu", "merges", "trunc_flops"]


def build(force=False):
    """Compile liboracle.so with g++ (plain -O3, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        d, i, pd = C.c_double, C.c_int, C.POINTER(C.c_double)
        L.or_build.restype = P
        L.or_build.argtypes = [i, i, P, i, d, i, P, P, P, d, d]
        L.or_clone.restype = P
        L.or_clone.argtypes = [P]
        L.or_zeros_like.restype = P
        L.or_zeros_like.argtypes = [P]
        L.or_free.argtypes = [P]
        L.or_n.argtypes = [P]
        L.or_perm.argtypes = [P, P]
        L.or_num_clusters.argtypes = [P]
        L.or_clusters.argtypes = [P, P, P, P, P, P]
        L.or_num_blocks.argtypes = [P]
        L.or_blocks.argtypes = [P, P, P, P, P, P]
        L.or_to_dense.argtypes = [P, P]
        L.or_addmul.argtypes = [d, P, P, P, d, i, P]
        L.or_lu.argtypes = [P, d, i, P]
        L.or_inv.argtypes = [P, d, i, P]
        L.or_chol.argtypes = [P, d, i, P]
        L.or_bem_entry.restype = d
        L.or_bem_entry.argtypes = [i, P, P, i]
        L.or_inv_dist_integral.restype = d
        L.or_inv_dist_integral.argtypes = [P, P]
        L.or_lu_solve.argtypes = [P, P, i]
        L.or_lu_sub.argtypes = [P, i, d, i, P]
        L.or_matvec.argtypes = [P, d, P, P, i]
        L.or_addeval_block.argtypes = [P, i, i, d, P, P, i]
        L.or_rkadd.argtypes = [i, i, i, i, d, P, P, P, P, d, P, P, P]
        L.or_rkmerge22.argtypes = [i, i, i, i, P, P, P, d, P, P]
        L.or_rkadd_multi.argtypes = [i, i, i, P, P, P, P, i, P, P, d, P, P]
        L.or_svd.argtypes = [i, i, P, P, P, P]
        L.or_qr.argtypes = [i, i, P, P, P]
        L.or_last_stats.argtypes = [P]
        L.or_log.argtypes = [P, P]
        L.or_last_error.restype = C.c_char_p
        L.or_set_log.argtypes = [i]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f(a, dtype=np.float64):
    return np.asfortranarray(np.asarray(a, dtype=dtype))


class HMatrix:
    """An oracle H-matrix (cluster tree, block tree, leaf data) on the CPU."""

    def __init__(self, handle):
        if not handle:
            raise RuntimeError("oracle: " + lib().or_last_error().decode())
        self._h = handle

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_free(self._h)
            self._h = None

    @classmethod
    def from_csr(cls, coords, rowptr, colind, vals, leaf, eta):
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        n, dim = coords.shape
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        colind = np.ascontiguousarray(colind, dtype=np.int32)
        vals = np.ascontiguousarray(vals, dtype=np.float64)
        h = lib().or_build(dim, n, _p(coords), leaf, eta, 0, _p(rowptr), _p(colind), _p(vals), 0.0, 0.0)
        return cls(h)

    @classmethod
    def from_kernel(cls, coords, leaf, eta, diag, eps):
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        n, dim = coords.shape
        h = lib().or_build(dim, n, _p(coords), leaf, eta, 1, None, None, None, diag, eps)
        return cls(h)

    @classmethod
    def from_bem(cls, tri, layer, leaf, eta, eps):
        """Galerkin boundary-element matrix on the flat triangles tri (n, 3, 3):
        layer 'single' (V) or 'double' (1/2 M + K); clusters from the centroids,
        admissible blocks by the truncated SVD at eps."""
        tri = np.ascontiguousarray(tri, dtype=np.float64).reshape(-1, 9)
        cen = np.ascontiguousarray(tri.reshape(-1, 3, 3).mean(axis=1))
        kind = {"single": 2, "double": 3}[layer]
        h = lib().or_build(3, cen.shape[0], _p(cen), leaf, eta, kind, None, None, _p(tri), 0.0, eps)
        return cls(h)

    def clone(self):
        return HMatrix(lib().or_clone(self._h))

    def zeros_like(self):
        return HMatrix(lib().or_zeros_like(self._h))

    @property
    def n(self):
        return lib().or_n(self._h)

    def perm(self):
        p = np.zeros(self.n, dtype=np.int32)
        lib().or_perm(self._h, _p(p))
        return p

    def clusters(self):
        nc = lib().or_num_clusters(self._h)
        arrs = [np.zeros(nc, dtype=np.int32) for _ in range(5)]
        lib().or_clusters(self._h, *[_p(a) for a in arrs])
        return dict(zip(["off", "size", "level", "son0", "son1"], arrs))

    def blocks(self):
        nb = lib().or_num_blocks(self._h)
        arrs = [np.zeros(nb, dtype=np.int32) for _ in range(5)]
        lib().or_blocks(self._h, *[_p(a) for a in arrs])
        return dict(zip(["t", "s", "kind", "rank", "parent"], arrs))

    def to_dense(self):
        """Dense matrix in cluster (permuted) order."""
        n = self.n
        out = np.zeros((n, n), order="F")
        lib().or_to_dense(self._h, _p(out))
        return out

    def lu(self, eps, mode):
        """In-place H-LU; mode 'standard' or 'accumulated'.  Returns statistics."""
        st = np.zeros(10, dtype=np.int64)
        rc = lib().or_lu(self._h, eps, _mode(mode), _p(st))
        if rc:
            raise RuntimeError("oracle: " + lib().or_last_error().decode())
        return dict(zip(STAT_NAMES, st.tolist()))

    def inv(self, eps, mode):
        """In-place H-inversion (Sect. 6, Fig. invert); mode 'standard' or
        'accumulated'.  Returns statistics (leaf_lu counts leaf inverses)."""
        st = np.zeros(10, dtype=np.int64)
        rc = lib().or_inv(self._h, eps, _mode(mode), _p(st))
        if rc:
            raise RuntimeError("oracle: " + lib().or_last_error().decode())
        return dict(zip(STAT_NAMES, st.tolist()))

    def chol(self, eps, mode):
        """In-place H-Cholesky G = L L^T (L in the lower blocks, zeros above the
        diagonal of the diagonal leaves); mode 'standard' or 'accumulated'."""
        st = np.zeros(10, dtype=np.int64)
        rc = lib().or_chol(self._h, eps, _mode(mode), _p(st))
        if rc:
            raise RuntimeError("oracle: " + lib().or_last_error().decode())
        return dict(zip(STAT_NAMES, st.tolist()))

    def lu_sub(self, depth, eps, mode):
        """In-place H-LU of the leading diagonal block at `depth`; returns (size, stats)."""
        st = np.zeros(10, dtype=np.int64)
        size = lib().or_lu_sub(self._h, depth, eps, _mode(mode), _p(st))
        if size < 0:
            raise RuntimeError("oracle: " + lib().or_last_error().decode())
        return size, dict(zip(STAT_NAMES, st.tolist()))

    def addmul(self, alpha, X, Y, eps, mode):
        """self <- blocktrunc(self + alpha X Y).  Returns statistics."""
        st = np.zeros(10, dtype=np.int64)
        rc = lib().or_addmul(alpha, X._h, Y._h, self._h, eps, _mode(mode), _p(st))
        if rc:
            raise RuntimeError("oracle: " + lib().or_last_error().decode())
        return dict(zip(STAT_NAMES, st.tolist()))

    def lu_solve(self, x):
        """(L R)^{-1} x for x in cluster order (vector or n x c matrix)."""
        x = _f(x).copy(order="F")
        c = 1 if x.ndim == 1 else x.shape[1]
        lib().or_lu_solve(self._h, _p(x), c)
        return x

    def matvec(self, x, alpha=1.0):
        x = _f(x)
        c = 1 if x.ndim == 1 else x.shape[1]
        y = np.zeros_like(x, order="F")
        lib().or_matvec(self._h, alpha, _p(x), _p(y), c)
        return y

    def addeval_block(self, b, w, y, alpha=1.0, trans=False):
        w = _f(w)
        y = _f(y).copy(order="F")
        rc = lib().or_addeval_block(self._h, b, int(trans), alpha, _p(w), _p(y), w.shape[1])
        if rc:
            raise IndexError(b)
        return y


def _mode(mode):
    return {"standard": 0, "accumulated": 1, "fused": 2, 0: 0, 1: 1, 2: 2}[mode]


def rkadd(alpha, A, B, C_, D, eps):
    """Truncated addition (C, D) <- trunc_eps(C D^T + alpha A B^T) (Fig. rkadd).

    Returns (C_new, D_new, sigma) with sigma the singular values of the sum.
    """
    A, B, C_, D = _f(A), _f(B), _f(C_), _f(D)
    m, k1 = A.shape
    n = B.shape[0]
    k2 = C_.shape[1]
    cap = max(min(m, n, k1 + k2), 1)
    Co = np.zeros((m, cap), order="F")
    Do = np.zeros((n, cap), order="F")
    sg = np.zeros(cap)
    k = lib().or_rkadd(m, n, k1, k2, alpha, _p(A), _p(B), _p(C_), _p(D), eps, _p(Co), _p(Do), _p(sg))
    if k1 == 0:
        return C_.copy(), D.copy(), np.zeros(0)
    q = min(m, n, k1 + k2)
    return Co[:, :k].copy(), Do[:, :k].copy(), sg[:q].copy()


def rkadd_multi(updates, C_, D, eps):
    """Stacked truncated addition: trunc_eps(C D^T + sum alpha A B^T) over the
    updates [(alpha, A, B), ...]; returns (Cout, Dout) with k columns."""
    m, n = C_.shape[0], D.shape[0]
    As = [_f(a) for _, a, _ in updates]
    Bs = [_f(b) for _, _, b in updates]
    ks = np.array([a.shape[1] for a in As], dtype=np.int32)
    al = np.array([u[0] for u in updates], dtype=np.float64)
    Ap = (C.c_void_p * len(As))(*[a.ctypes.data for a in As])
    Bp = (C.c_void_p * len(Bs))(*[b.ctypes.data for b in Bs])
    C_, D = _f(C_), _f(D)
    cap = min(m, n, int(ks.sum()) + C_.shape[1])
    Co = np.zeros((m, max(cap, 1)), order="F")
    Do = np.zeros((n, max(cap, 1)), order="F")
    k = lib().or_rkadd_multi(m, n, len(As), _p(ks), _p(al), C.cast(Ap, C.c_void_p), C.cast(Bp, C.c_void_p),
                             C_.shape[1], _p(C_), _p(D), eps, _p(Co), _p(Do))
    return Co[:, :k], Do[:, :k]


def rkmerge22(m0, m1, n0, n1, pieces, eps):
    """2x2 rkmerge of pieces [(A00,B00),(A01,B01),(A10,B10),(A11,B11)] (Fig. rkmerge)."""
    ks = np.array([p[0].shape[1] for p in pieces], dtype=np.int32)
    As = [_f(p[0]) for p in pieces]
    Bs = [_f(p[1]) for p in pieces]
    Ap = (C.c_void_p * 4)(*[a.ctypes.data for a in As])
    Bp = (C.c_void_p * 4)(*[b.ctypes.data for b in Bs])
    cap = max(min(m0 + m1, n0 + n1, int(ks.sum())), 1)
    Ao = np.zeros((m0 + m1, cap), order="F")
    Bo = np.zeros((n0 + n1, cap), order="F")
    k = lib().or_rkmerge22(m0, m1, n0, n1, _p(ks), C.cast(Ap, C.c_void_p), C.cast(Bp, C.c_void_p),
                           eps, _p(Ao), _p(Bo))
    return Ao[:, :k].copy(), Bo[:, :k].copy()


def bem_entry(layer, ti, tj, same=False):
    """One Galerkin entry between two triangles (3 x 3 vertex arrays)."""
    a = np.ascontiguousarray(ti, dtype=np.float64).reshape(9)
    b = np.ascontiguousarray(tj, dtype=np.float64).reshape(9)
    return lib().or_bem_entry({"single": 2, "double": 3}[layer], _p(a), _p(b), int(same))


def inv_dist_integral(t, x):
    """int_T 1/|x - y| dy for x in the plane of T."""
    a = np.ascontiguousarray(t, dtype=np.float64).reshape(9)
    xx = np.ascontiguousarray(x, dtype=np.float64).reshape(3)
    return lib().or_inv_dist_integral(_p(a), _p(xx))


def svd(M):
    M = _f(M)
    m, n = M.shape
    r = min(m, n)
    U = np.zeros((m, r), order="F")
    S = np.zeros(r)
    V = np.zeros((n, r), order="F")
    lib().or_svd(m, n, _p(M), _p(U), _p(S), _p(V))
    return U, S, V


def qr(M):
    M = _f(M)
    m, n = M.shape
    q = min(m, n)
    Q = np.zeros((m, q), order="F")
    R = np.zeros((q, n), order="F")
    lib().or_qr(m, n, _p(M), _p(Q), _p(R))
    return Q, R


def set_log(enable):
    lib().or_set_log(int(enable))


def last_log():
    n = lib().or_log_size()
    ints = np.zeros((n, 6), dtype=np.int32)
    mg = np.zeros((n, 2))
    if n:
        lib().or_log(_p(ints), _p(mg))
    return ints, mg


def last_stats():
    st = np.zeros(10, dtype=np.int64)
    lib().or_last_stats(_p(st))
    return dict(zip(STAT_NAMES, st.tolist()))
