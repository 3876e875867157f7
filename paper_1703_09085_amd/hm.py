"""Python binding of libhm.so (ctypes; argument marshalling only).

Every computation runs in the library's HIP kernels on the GPU.  PyTorch only
supplies the HIP stream (and device tensors for hm_trunc_batch).  The binding
raises if the library is missing or a call fails; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhm.so")

STANDARD, ACCUMULATED, FUSED = 0, 1, 2
COUNT_NAMES = ["trunc_update", "trunc_accum", "trunc_merge", "dense_updates", "addproduct", "pending",
               "products", "leaf_lu", "merges"]
ITEM_NAMES = ["gemm", "trunc", "lu", "trsm", "copy"]

# Exported C ABI (see include/hm.h); checked by the CPU test suite.
SYMBOLS = ["hm_version", "hm_last_error", "hm_ctx_create", "hm_ctx_destroy", "hm_set_schedule", "hm_schedule_check", "hm_build_csr", "hm_clone",
           "hm_zeros_like", "hm_copy_values", "hm_save", "hm_load", "hm_file_info", "hm_matrix_free", "hm_addmul", "hm_lu", "hm_plan_lu",
           "hm_plan_addmul", "hm_plan_lu_batch", "hm_plan_lu_solve", "hm_lu_solve", "hm_plan_run", "hm_plan_use_graph", "hm_plan_set_precision", "hm_plan_autotune", "hm_plan_set_predictor", "hm_plan_feature_log", "hm_plan_free", "hm_plan_trunc_log", "hm_plan_launch_log", "hm_trunc_batch", "hm_trunc_batch_predicted", "hm_n", "hm_perm",
           "hm_num_clusters", "hm_clusters", "hm_num_blocks", "hm_blocks", "hm_to_dense", "hm_block_to_dense",
           "hm_mlp_create", "hm_mlp_free", "hm_mlp_get", "hm_mlp_predict", "hm_mlp_gradient", "hm_mlp_train",
           "hm_ctx_create_with_allocator", "hm_options_init", "hm_build", "hm_lu_opt", "hm_addmul_opt",
           "hm_plan_set_rank_override", "hm_get_stats", "hm_trunc_batch_device", "hm_trunc_batch_device_noalloc",
           "hm_inv", "hm_plan_inv", "hm_chol", "hm_plan_chol"]


class RunInfo(C.Structure):
    _fields_ = [("plan_seconds", C.c_double), ("run_seconds", C.c_double), ("truncations", C.c_int64),
                ("planned_truncations", C.c_int64), ("items", C.c_int64 * 5), ("waves", C.c_int64),
                ("launches", C.c_int64), ("temp_bytes", C.c_int64), ("workspace_bytes", C.c_int64),
                ("counts", C.c_int64 * 9), ("status_bits", C.c_int32), ("schedule", C.c_int32),
                ("trunc_bytes", C.c_int64), ("op_seconds", C.c_double * 5), ("plan_phase_seconds", C.c_double * 3),
                ("small_trunc_bytes", C.c_int64), ("small_trunc_seconds", C.c_double),
                ("small_trunc_launches", C.c_int64), ("general_trunc_launches", C.c_int64),
                ("predicted", C.c_int64), ("predicted_fallback", C.c_int64), ("graph_replay", C.c_int32),
                ("pad", C.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k in ["plan_seconds", "run_seconds", "truncations", "planned_truncations",
                                            "waves", "launches", "temp_bytes", "workspace_bytes", "status_bits",
                                            "trunc_bytes", "small_trunc_bytes", "small_trunc_seconds",
                                            "small_trunc_launches", "general_trunc_launches", "predicted",
                                            "predicted_fallback", "graph_replay"]}
        d["schedule"] = "dataflow" if self.schedule == 1 else "waves"
        d["op_seconds"] = dict(zip(ITEM_NAMES, list(self.op_seconds)))
        d["plan_phase_seconds"] = list(self.plan_phase_seconds)
        d["items"] = dict(zip(ITEM_NAMES, list(self.items)))
        d["counts"] = dict(zip(COUNT_NAMES, list(self.counts)))
        return d


class TruncDesc(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("k1", C.c_int32), ("k2", C.c_int32), ("kcap", C.c_int32),
                ("lda", C.c_int32), ("ldb", C.c_int32), ("ldc", C.c_int32), ("ldd", C.c_int32), ("pad", C.c_int32),
                ("alpha", C.c_double), ("A", C.c_void_p), ("B", C.c_void_p), ("C", C.c_void_p), ("D", C.c_void_p),
                ("Cout", C.c_void_p), ("Dout", C.c_void_p), ("rank_out", C.c_void_p)]


SRC_CSR, SRC_STENCIL_5PT, SRC_STENCIL_7PT, SRC_KERNEL_INVDIST, SRC_BEM_SINGLE, SRC_BEM_DOUBLE = 0, 1, 2, 3, 4, 5


class Source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad", C.c_int32), ("rowptr", C.c_void_p), ("colind", C.c_void_p),
                ("vals", C.c_void_p), ("diag", C.c_double), ("tri", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("eps", C.c_double), ("eta", C.c_double), ("leaf_size", C.c_int32), ("kmax", C.c_int32),
                ("mode", C.c_int32), ("precision", C.c_int32), ("schedule", C.c_int32), ("use_graph", C.c_int32),
                ("rank_override", C.c_void_p), ("rank_override_count", C.c_int64)]

    @classmethod
    def make(cls, **kw):
        """hm_options_init defaults, then the given fields (mode, precision and
        schedule also by name)."""
        o = cls()
        lib().hm_options_init(C.byref(o))
        for k, v in kw.items():
            if k == "mode":
                v = _mode(v)
            elif k == "precision":
                v = _prec(v)
            elif k == "schedule" and isinstance(v, str):
                v = Context.SCHEDULES[v]
            setattr(o, k, v)
        return o


class Stats(C.Structure):
    _fields_ = [("plans", C.c_int64), ("plan_seconds", C.c_double), ("runs", C.c_int64), ("run_seconds", C.c_double),
                ("truncations", C.c_int64), ("trunc_bytes", C.c_int64), ("builds", C.c_int64),
                ("build_seconds", C.c_double), ("device_bytes_in_use", C.c_int64), ("device_bytes_peak", C.c_int64),
                ("device_allocations", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
# the callbacks must outlive every object allocated through them: kept for
# the life of the process
_CALLBACKS = []


def _torch_allocator(stream):
    """hm_alloc_fn / hm_free_fn bound to torch's caching allocator on `stream`."""
    import torch

    def alloc(nbytes, user):
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), stream=stream))
        except Exception:  # out of memory: the library reports HM_ERR_HIP/ALLOC
            return None

    def free(ptr, user):
        torch.cuda.caching_allocator_delete(int(ptr))

    cb = (_ALLOC_FN(alloc), _FREE_FN(free))
    _CALLBACKS.append(cb)
    return cb


class HMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hm status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libhm.so (built by paper_1703_09085_amd.build); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1703_09085_amd.build")
        L = C.CDLL(LIB_PATH)
        P, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.hm_version.restype = C.c_char_p
        L.hm_last_error.restype = C.c_char_p
        L.hm_ctx_create.argtypes = [P, P]
        L.hm_ctx_destroy.argtypes = [P]
        L.hm_set_schedule.argtypes = [P, i32]
        L.hm_schedule_check.argtypes = [i32, i32, i32, d, i32, i32, i32, P]
        L.hm_build_csr.argtypes = [P, i32, i64, P, P, P, P, i32, d, i32, P]
        L.hm_clone.argtypes = [P, P, P]
        L.hm_zeros_like.argtypes = [P, P, P]
        L.hm_save.argtypes = [P, P, C.c_char_p]
        L.hm_load.argtypes = [P, C.c_char_p, P]
        L.hm_file_info.argtypes = [C.c_char_p, P, P, P]
        L.hm_copy_values.argtypes = [P, P, P]
        L.hm_matrix_free.argtypes = [P]
        L.hm_addmul.argtypes = [P, d, P, P, P, d, i32, P]
        L.hm_lu.argtypes = [P, P, d, i32, P]
        L.hm_plan_lu.argtypes = [P, P, i32, P]
        L.hm_plan_addmul.argtypes = [P, d, P, P, P, i32, P]
        L.hm_plan_lu_batch.argtypes = [P, P, i32, i32, P]
        L.hm_plan_lu_solve.argtypes = [P, P, P, i64, i32, P]
        L.hm_lu_solve.argtypes = [P, P, P, i64, i32]
        L.hm_plan_run.argtypes = [P, P, d, P]
        L.hm_plan_use_graph.argtypes = [P, i32]
        L.hm_plan_autotune.argtypes = [P, P, d, P]
        L.hm_plan_set_predictor.argtypes = [P, P, P, i32, i32]
        L.hm_plan_feature_log.restype = i64
        L.hm_plan_feature_log.argtypes = [P, P, i64]
        L.hm_plan_free.argtypes = [P]
        L.hm_plan_trunc_log.restype = i64
        L.hm_plan_trunc_log.argtypes = [P, P, i64]
        L.hm_plan_launch_log.restype = i64
        L.hm_plan_launch_log.argtypes = [P, P, i64]
        L.hm_trunc_batch.argtypes = [P, i32, P, d, i32, P]
        L.hm_plan_set_precision.argtypes = [P, i32]
        L.hm_trunc_batch_predicted.argtypes = [P, i32, P, d, P, P, i32, i32, P]
        L.hm_n.restype = i64
        L.hm_n.argtypes = [P]
        L.hm_perm.argtypes = [P, P]
        L.hm_num_clusters.argtypes = [P]
        L.hm_clusters.argtypes = [P, P, P, P, P, P]
        L.hm_num_blocks.argtypes = [P]
        L.hm_blocks.argtypes = [P, P, P, P, P, P, P]
        L.hm_to_dense.argtypes = [P, P, P]
        L.hm_block_to_dense.argtypes = [P, P, i64, P, i64]
        L.hm_mlp_create.argtypes = [P, P, C.c_uint64, P]
        L.hm_mlp_free.argtypes = [P]
        L.hm_mlp_get.argtypes = [P, P, P, P]
        L.hm_mlp_predict.argtypes = [P, P, P, i64, P]
        L.hm_mlp_gradient.argtypes = [P, P, P, P, i64, P, P]
        L.hm_mlp_train.argtypes = [P, P, P, P, i64, i32, i32, C.c_float, P]
        L.hm_ctx_create_with_allocator.argtypes = [P, _ALLOC_FN, _FREE_FN, P, P]
        L.hm_options_init.restype = None
        L.hm_options_init.argtypes = [P]
        L.hm_build.argtypes = [P, i32, i64, P, P, P, P]
        L.hm_lu_opt.argtypes = [P, P, P, P]
        L.hm_addmul_opt.argtypes = [P, d, P, P, P, P, P]
        L.hm_plan_set_rank_override.argtypes = [P, P, i64]
        L.hm_get_stats.argtypes = [P, P]
        L.hm_trunc_batch_device.argtypes = [P, i32, P, i32, i32, d, i32, P]
        L.hm_inv.argtypes = [P, P, d, i32, P]
        L.hm_plan_inv.argtypes = [P, P, i32, P]
        L.hm_chol.argtypes = [P, P, d, i32, P]
        L.hm_plan_chol.argtypes = [P, P, i32, P]
        L.hm_trunc_batch_device_noalloc.argtypes = [P, i32, P, i32, i32, d, i32, P]
        _lib = L
    return _lib


def file_info(path):
    """hm_file_info: (n, clusters, blocks) of a checkpoint file, checked on the host."""
    n, nc, nb = C.c_int64(), C.c_int32(), C.c_int32()
    _chk(lib().hm_file_info(os.fsencode(path), C.byref(n), C.byref(nc), C.byref(nb)))
    return n.value, nc.value, nb.value


def _chk(status):
    if status != 0:
        raise HMError(status, lib().hm_last_error().decode())


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


class Context:
    """A library context on a HIP stream (torch's current stream by default)."""

    def __init__(self, stream=None, allocator=None):
        """allocator None: hipMalloc / hipFree; "torch": torch's caching
        allocator on the context's stream."""
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("hm needs a GPU (torch.cuda.is_available() is False)")
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        if allocator is None:
            _chk(lib().hm_ctx_create(C.c_void_p(stream.cuda_stream), C.byref(h)))
        elif allocator == "torch":
            fa, ff = _torch_allocator(stream)
            _chk(lib().hm_ctx_create_with_allocator(C.c_void_p(stream.cuda_stream), fa, ff, None, C.byref(h)))
        else:
            raise ValueError(allocator)
        self._h = h

    def stats(self):
        """hm_get_stats: totals of this context."""
        st = Stats()
        _chk(lib().hm_get_stats(self._h, C.byref(st)))
        return st.as_dict()

    def trunc_batch_device(self, descs, count, max_rows, max_stack, eps, precision="fp64"):
        """hm_trunc_batch_device: descs is a device buffer (a torch uint8
        tensor of count * sizeof(TruncDesc) bytes) holding the descriptors."""
        assert descs.is_cuda and descs.numel() >= count * C.sizeof(TruncDesc)
        ex = C.c_int64(0)
        _chk(lib().hm_trunc_batch_device(self._h, int(count), C.c_void_p(descs.data_ptr()), int(max_rows),
                                         int(max_stack), eps, _prec(precision), C.byref(ex)))
        return ex.value

    def trunc_batch_device_noalloc(self, descs, count, max_rows, max_stack, eps, precision="fp64", wait=True):
        """hm_trunc_batch_device_noalloc: as trunc_batch_device, with the library's
        static scratch array instead of allocations; wait=False only enqueues."""
        assert descs.is_cuda and descs.numel() >= count * C.sizeof(TruncDesc)
        ex = C.c_int64(0)
        _chk(lib().hm_trunc_batch_device_noalloc(self._h, int(count), C.c_void_p(descs.data_ptr()), int(max_rows),
                                                 int(max_stack), eps, _prec(precision),
                                                 C.byref(ex) if wait else None))
        return ex.value if wait else None

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hm_ctx_destroy(self._h)
            self._h = None

    SCHEDULES = {"waves": 0, "dataflow": 1}

    def set_schedule(self, schedule):
        """hm_set_schedule: "waves" or "dataflow" for the plans made from now on."""
        if schedule not in self.SCHEDULES:
            raise KeyError(schedule)
        _chk(lib().hm_set_schedule(self._h, self.SCHEDULES[schedule]))
        return self

    @staticmethod
    def desc_array(descs):
        """A ctypes array of TruncDesc (to pass to trunc_batch more than once)."""
        return (TruncDesc * len(descs))(*descs)

    def trunc_batch(self, descs, eps, precision="fp64"):
        """hm_trunc_batch on a list (or desc_array) of TruncDesc; returns the
        executed count."""
        arr = descs if isinstance(descs, C.Array) else self.desc_array(descs)
        ex = C.c_int64(0)
        _chk(lib().hm_trunc_batch(self._h, len(arr), C.cast(arr, C.c_void_p), eps, _prec(precision),
                                  C.byref(ex)))
        return ex.value

    def trunc_batch_predicted(self, descs, eps, mlp, omega, oversample=2, level=0):
        """hm_trunc_batch_predicted: the rank predictor sizes a range finder for
        the small items.  Returns (executed, accepted, fallbacks)."""
        assert tuple(omega.shape) == (32, 64) and omega.is_contiguous()
        arr = (TruncDesc * len(descs))(*descs)
        counts = np.zeros(3, dtype=np.int64)
        _chk(lib().hm_trunc_batch_predicted(self._h, len(descs), C.cast(arr, C.c_void_p), eps, mlp._h,
                                            C.c_void_p(omega.data_ptr()), int(oversample), int(level), _p(counts)))
        return int(counts[0]), int(counts[1]), int(counts[2])


class HMatrix:
    """A device-resident H-matrix."""

    def __init__(self, ctx, handle):
        self.ctx = ctx
        self._h = handle

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hm_matrix_free(self._h)
            self._h = None

    @classmethod
    def from_csr(cls, ctx, coords, rowptr, colind, vals, leaf, eta=2.0, kmax=64):
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        n, dim = coords.shape
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        colind = np.ascontiguousarray(colind, dtype=np.int32)
        vals = np.ascontiguousarray(vals, dtype=np.float64)
        h = C.c_void_p()
        _chk(lib().hm_build_csr(ctx._h, dim, n, _p(coords), _p(rowptr), _p(colind), _p(vals), leaf, eta, kmax,
                                C.byref(h)))
        return cls(ctx, h)

    @classmethod
    def build(cls, ctx, coords, source, **options):
        """hm_build from a Source with Options fields as keywords."""
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        n, dim = coords.shape
        opt = Options.make(**options)
        h = C.c_void_p()
        _chk(lib().hm_build(ctx._h, dim, n, _p(coords), C.byref(source), C.byref(opt), C.byref(h)))
        return cls(ctx, h)

    @classmethod
    def from_kernel(cls, ctx, coords, leaf, eta=2.0, diag=1e3, eps=1e-5, kmax=64):
        """Kernel matrix 1/|x - y| (diagonal `diag`), admissible blocks
        truncated at eps; assembled and compressed on the GPU."""
        src = Source(kind=SRC_KERNEL_INVDIST, diag=diag)
        return cls.build(ctx, coords, src, leaf_size=leaf, eta=eta, kmax=kmax, eps=eps)

    @classmethod
    def from_bem(cls, ctx, tri, layer, leaf, eta=2.0, eps=1e-4, kmax=64):
        """Galerkin boundary-element matrix on the flat triangles tri (n, 3, 3):
        layer 'single' (V) or 'double' (1/2 M + K); clusters from the
        centroids; assembled and compressed on the GPU."""
        tri = np.ascontiguousarray(tri, dtype=np.float64).reshape(-1, 9)
        cen = tri.reshape(-1, 3, 3).mean(axis=1)
        src = Source(kind={"single": SRC_BEM_SINGLE, "double": SRC_BEM_DOUBLE}[layer], tri=tri.ctypes.data)
        return cls.build(ctx, cen, src, leaf_size=leaf, eta=eta, kmax=kmax, eps=eps)

    @classmethod
    def from_stencil(cls, ctx, coords, leaf, eta=2.0, kmax=64):
        """(2 dim + 1)-point Laplacian of lattice points."""
        coords = np.asarray(coords)
        src = Source(kind=SRC_STENCIL_5PT if coords.shape[1] == 2 else SRC_STENCIL_7PT)
        return cls.build(ctx, coords, src, leaf_size=leaf, eta=eta, kmax=kmax)

    def clone(self):
        h = C.c_void_p()
        _chk(lib().hm_clone(self.ctx._h, self._h, C.byref(h)))
        return HMatrix(self.ctx, h)

    def zeros_like(self):
        h = C.c_void_p()
        _chk(lib().hm_zeros_like(self.ctx._h, self._h, C.byref(h)))
        return HMatrix(self.ctx, h)

    def save(self, path):
        """hm_save: structure, ranks and values to a file."""
        _chk(lib().hm_save(self.ctx._h, self._h, os.fsencode(path)))

    @classmethod
    def load(cls, ctx, path):
        """hm_load: a new matrix from a file written by save()."""
        h = C.c_void_p()
        _chk(lib().hm_load(ctx._h, os.fsencode(path), C.byref(h)))
        return cls(ctx, h)

    def copy_from(self, src):
        _chk(lib().hm_copy_values(self.ctx._h, src._h, self._h))

    @property
    def n(self):
        return lib().hm_n(self._h)

    def perm(self):
        p = np.zeros(self.n, dtype=np.int32)
        _chk(lib().hm_perm(self._h, _p(p)))
        return p

    def clusters(self):
        nc = lib().hm_num_clusters(self._h)
        arrs = [np.zeros(nc, dtype=np.int32) for _ in range(5)]
        _chk(lib().hm_clusters(self._h, *[_p(a) for a in arrs]))
        return dict(zip(["off", "size", "level", "son0", "son1"], arrs))

    def blocks(self):
        nb = lib().hm_num_blocks(self._h)
        arrs = [np.zeros(nb, dtype=np.int32) for _ in range(5)]
        _chk(lib().hm_blocks(self.ctx._h, self._h, *[_p(a) for a in arrs]))
        return dict(zip(["t", "s", "kind", "rank", "parent"], arrs))

    def to_dense(self):
        n = self.n
        out = np.zeros((n, n), order="F")
        _chk(lib().hm_to_dense(self.ctx._h, self._h, _p(out)))
        return out

    def block_to_dense(self, block, rows, cols):
        """Values of leaf block `block` (pre-order index) as a rows x cols array."""
        out = np.zeros((rows, cols), order="F")
        _chk(lib().hm_block_to_dense(self.ctx._h, self._h, int(block), _p(out), rows))
        return out

    def lu(self, eps, mode):
        info = RunInfo()
        _chk(lib().hm_lu(self.ctx._h, self._h, eps, _mode(mode), C.byref(info)))
        return info.as_dict()

    def inv(self, eps, mode):
        """hm_inv: in-place H-matrix inversion (Sect. 6, Fig. invert)."""
        info = RunInfo()
        _chk(lib().hm_inv(self.ctx._h, self._h, eps, _mode(mode), C.byref(info)))
        return info.as_dict()

    def chol(self, eps, mode):
        """hm_chol: in-place H-Cholesky G = L L^T (L in the lower blocks)."""
        info = RunInfo()
        _chk(lib().hm_chol(self.ctx._h, self._h, eps, _mode(mode), C.byref(info)))
        return info.as_dict()

    def lu_solve(self, x):
        """In place x <- (L R)^{-1} x with the H-LU factors held by this matrix.
        x: torch float64 CUDA tensor of shape (n,) or (c, n) (row i of the
        tensor is right-hand side i), in cluster order."""
        n = self.n
        assert x.dtype.is_floating_point and x.element_size() == 8 and x.is_contiguous() and x.shape[-1] == n
        c = 1 if x.dim() == 1 else x.shape[0]
        _chk(lib().hm_lu_solve(self.ctx._h, self._h, C.c_void_p(x.data_ptr()), n, c))
        return x

    def addmul(self, alpha, X, Y, eps, mode):
        info = RunInfo()
        _chk(lib().hm_addmul(self.ctx._h, alpha, X._h, Y._h, self._h, eps, _mode(mode), C.byref(info)))
        return info.as_dict()

    def lu_opt(self, rank_override=None, **options):
        """hm_lu_opt with Options fields as keywords; rank_override an int32
        array (one entry per truncation item) or None."""
        ov = None if rank_override is None else np.ascontiguousarray(rank_override, dtype=np.int32)
        opt = Options.make(**options)
        if ov is not None:
            opt.rank_override, opt.rank_override_count = ov.ctypes.data, len(ov)
        info = RunInfo()
        _chk(lib().hm_lu_opt(self.ctx._h, self._h, C.byref(opt), C.byref(info)))
        return info.as_dict()

    def addmul_opt(self, alpha, X, Y, rank_override=None, **options):
        ov = None if rank_override is None else np.ascontiguousarray(rank_override, dtype=np.int32)
        opt = Options.make(**options)
        if ov is not None:
            opt.rank_override, opt.rank_override_count = ov.ctypes.data, len(ov)
        info = RunInfo()
        _chk(lib().hm_addmul_opt(self.ctx._h, alpha, X._h, Y._h, self._h, C.byref(opt), C.byref(info)))
        return info.as_dict()


class Plan:
    """A recorded, scheduled and uploaded H-LU or multiplication."""

    def __init__(self, ctx, handle, keep):
        self.ctx = ctx
        self._h = handle
        self._keep = keep  # the matrices the plan is bound to

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hm_plan_free(self._h)
            self._h = None

    @classmethod
    def lu(cls, ctx, G, mode):
        h = C.c_void_p()
        _chk(lib().hm_plan_lu(ctx._h, G._h, _mode(mode), C.byref(h)))
        return cls(ctx, h, [G])

    @classmethod
    def lu_batch(cls, ctx, Gs, mode):
        """One plan for the H-LU of several independent matrices."""
        Gs = list(Gs)
        arr = (C.c_void_p * len(Gs))(*[G._h.value for G in Gs])
        h = C.c_void_p()
        _chk(lib().hm_plan_lu_batch(ctx._h, C.cast(arr, C.c_void_p), len(Gs), _mode(mode), C.byref(h)))
        return cls(ctx, h, Gs)

    @classmethod
    def inv(cls, ctx, G, mode):
        h = C.c_void_p()
        _chk(lib().hm_plan_inv(ctx._h, G._h, _mode(mode), C.byref(h)))
        return cls(ctx, h, [G])

    @classmethod
    def chol(cls, ctx, G, mode):
        h = C.c_void_p()
        _chk(lib().hm_plan_chol(ctx._h, G._h, _mode(mode), C.byref(h)))
        return cls(ctx, h, [G])

    @classmethod
    def addmul(cls, ctx, alpha, X, Y, Z, mode):
        h = C.c_void_p()
        _chk(lib().hm_plan_addmul(ctx._h, alpha, X._h, Y._h, Z._h, _mode(mode), C.byref(h)))
        return cls(ctx, h, [X, Y, Z])

    def set_rank_override(self, ranks):
        """Rank of every truncation item (recording order, -1 keeps the rule), or None."""
        if ranks is None:
            _chk(lib().hm_plan_set_rank_override(self._h, None, 0))
            return self
        r = np.ascontiguousarray(ranks, dtype=np.int32)
        _chk(lib().hm_plan_set_rank_override(self._h, _p(r), len(r)))
        return self

    def set_precision(self, precision):
        """'fp64', 'fp32' or 'bf16x3': arithmetic of the dense products and of
        the small-block truncations' stacked-factor products."""
        _chk(lib().hm_plan_set_precision(self._h, _prec(precision)))
        return self

    def use_graph(self, enable=True):
        """Replay the plan's launches from a captured hipGraph."""
        _chk(lib().hm_plan_use_graph(self._h, int(enable)))
        return self

    def autotune(self, eps):
        """Choose, per small-block truncation launch, the faster kernel variant
        (two timed trial runs; the written matrix is left unchanged).
        Returns the number of launches that chose 4 and 8 threads per column."""
        chosen = np.zeros(2, dtype=np.int64)
        _chk(lib().hm_plan_autotune(self.ctx._h, self._h, eps, _p(chosen)))
        return int(chosen[0]), int(chosen[1])

    def set_predictor(self, mlp, omega, oversample=2, mode=1):
        """Attach the rank predictor (mode 1 predicts, mode 0 only computes the
        features); omega: torch float64 tensor (32, 64), i.e. the 64 x 32
        column-major sketch matrix on the device.  None detaches."""
        if mlp is None:
            _chk(lib().hm_plan_set_predictor(self._h, None, None, 0, 0))
            return self
        assert tuple(omega.shape) == (32, 64) and omega.is_contiguous()
        _chk(lib().hm_plan_set_predictor(self._h, mlp._h, omega.data_ptr(), int(oversample), int(mode)))
        self._keep = list(self._keep) + [mlp, omega]
        return self

    def feature_log(self):
        """(items, 10) float32: 8 features, k^, outcome; NaN rows for items that
        did not run the small-block kernel."""
        n = lib().hm_plan_feature_log(self._h, None, 0)
        out = np.full((max(n, 0), 10), np.nan, dtype=np.float32)
        if n > 0:
            lib().hm_plan_feature_log(self._h, _p(out), n)
        return out

    def run(self, eps):
        info = RunInfo()
        _chk(lib().hm_plan_run(self.ctx._h, self._h, eps, C.byref(info)))
        return info.as_dict()

    def launch_log(self):
        """(launches, 5) array: wave, kind, variant, items, device ms of the last
        run (ms only for plans recorded with HM_PROFILE_OPS=1)."""
        n = lib().hm_plan_launch_log(self._h, None, 0)
        out = np.zeros((max(n, 0), 5))
        if n > 0:
            lib().hm_plan_launch_log(self._h, _p(out), n)
        return out

    def trunc_log(self):
        """(items, 9) int array per truncation item in recursion order: m, n,
        l, k, Jacobi sweeps, cycles/16 of the QR, core and rebuild phases
        (-1: skipped), and the item's wave."""
        n = lib().hm_plan_trunc_log(self._h, None, 0)
        out = np.zeros((max(n, 0), 9), dtype=np.int32)
        if n > 0:
            lib().hm_plan_trunc_log(self._h, _p(out), n)
        return out


PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}


def schedule_check(dim, side, leaf, eta=2.0, kmax=64, mode="accumulated", schedule="dataflow"):
    """hm_schedule_check (host only, no GPU needed): schedule the H-LU of a
    side^dim grid and check it against the run rules; returns the counts."""
    out = np.zeros(8, dtype=np.int64)
    _chk(lib().hm_schedule_check(dim, side, leaf, eta, kmax, _mode(mode), Context.SCHEDULES[schedule], _p(out)))
    keys = ["launches", "conflicts", "unordered", "shared_temporaries", "unordered_temporaries", "missing_events",
            "misplaced_items", "dataflow"]
    return dict(zip(keys, (int(v) for v in out)))


def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _mode(mode):
    return {"standard": STANDARD, "accumulated": ACCUMULATED, "fused": FUSED, 0: 0, 1: 1, 2: 2}[mode]


MLP_NPARAM = 4801
MLP_LAYOUT = [("W1", (64, 8)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("w3", (64,)), ("b3", ())]


def mlp_unpack(vec):
    """Split a parameter vector into the named arrays (views, row-major)."""
    out, o = {}, 0
    for name, shape in MLP_LAYOUT:
        size = int(np.prod(shape)) if shape else 1
        out[name] = vec[o:o + size].reshape(shape) if shape else vec[o]
        o += size
    return out


class MLP:
    """The rank-predictor network on the device (BF16 weights, FP32 accumulation)."""

    def __init__(self, ctx, init=None, seed=0):
        self.ctx = ctx
        h = C.c_void_p()
        w = None if init is None else np.ascontiguousarray(init, dtype=np.float32)
        _chk(lib().hm_mlp_create(ctx._h, None if w is None else _p(w), int(seed), C.byref(h)))
        self._h = h.value

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hm_mlp_free(self._h)
            self._h = None

    def weights(self):
        """(master FP32 vector, working vector: BF16 matrices as FP32, FP32 biases)."""
        m = np.zeros(MLP_NPARAM, dtype=np.float32)
        w = np.zeros(MLP_NPARAM, dtype=np.float32)
        _chk(lib().hm_mlp_get(self.ctx._h, self._h, _p(m), _p(w)))
        return m, w

    def predict(self, X):
        """X: torch float32 (B, 8) on the device; returns a torch (B,) tensor."""
        import torch

        y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        _chk(lib().hm_mlp_predict(self.ctx._h, self._h, X.data_ptr(), X.shape[0], y.data_ptr()))
        return y

    def gradient(self, X, t):
        g = np.zeros(MLP_NPARAM, dtype=np.float32)
        loss = C.c_double()
        _chk(lib().hm_mlp_gradient(self.ctx._h, self._h, X.data_ptr(), t.data_ptr(), X.shape[0], _p(g),
                                   C.byref(loss)))
        return g, loss.value

    def train(self, X, t, epochs, batch, lr):
        losses = np.zeros(max(epochs, 1), dtype=np.float32)
        _chk(lib().hm_mlp_train(self.ctx._h, self._h, X.data_ptr(), t.data_ptr(), X.shape[0], epochs, batch,
                                float(lr), _p(losses)))
        return losses[:epochs]
