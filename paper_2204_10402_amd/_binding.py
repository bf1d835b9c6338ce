"""ctypes binding of libvc.so (include/vc.h). Argument marshalling only: every step of the
search runs in the library's HIP kernels. PyTorch, when used, only supplies device memory and
the stream."""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libvc.so")

OK = 0
ERR_INVALID_GRAPH = -1
ERR_INVALID_ARG = -2
ERR_NO_MEMORY = -3
ERR_BUDGET = -4
ERR_DEVICE = -5
ERR_INTERNAL = -6

OPT_NO_DEGREE_ONE = 0x1
OPT_NO_TRIANGLE = 0x2
OPT_NO_HIGH_DEGREE = 0x4
OPT_NO_EDGE_PRUNE = 0x8
OPT_PROFILE = 0x10
OPT_DEGREE_ARRAYS = 0x20
OPT_BITSETS = 0x40
OPT_AUTOTUNE = 0x80
OPT_STACK_ONLY = 0x100
OPT_GLOBAL_NODES = 0x200
OPT_CSR_GLOBAL = 0x400
ACTIVITIES = ("acquire", "reduce", "branch", "donate", "other", "total",
              "reduce_deg1", "reduce_tri", "reduce_high", "reduce_apply")

# Every function include/vc.h declares.
EXPORTS = (
    "vc_create", "vc_destroy", "vc_strerror", "vc_last_error", "vc_version",
    "vc_mvc", "vc_pvc", "vc_mvc_device", "vc_pvc_device", "vc_greedy_device",
    "vc_reduce_device", "vc_mvc_batch", "vc_pvc_batch", "vc_mvc_batch_device",
    "vc_pvc_batch_device", "vc_server_create", "vc_server_submit", "vc_server_poll",
    "vc_server_pending", "vc_server_destroy", "vc_wg_loads", "vc_abort", "vc_workspace_bytes",
    "vc_batch_workspace_bytes", "vc_mvc_device_ws", "vc_pvc_device_ws",
    "vc_mvc_batch_device_ws", "vc_pvc_batch_device_ws", "vc_pvc_device_noalloc",
)

PROBLEM_MVC = 0
PROBLEM_PVC = 1


class _Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


class _Batch(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("n", ctypes.c_void_p), ("nnz", ctypes.c_void_p),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


class _ServerOptions(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("memory_budget", ctypes.c_int64), ("wg_per_request", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 3)]


class _Served(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_int64), ("status", ctypes.c_int32), ("size", ctypes.c_int32),
                ("yes", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("worker", ctypes.c_int32), ("pad", ctypes.c_int32), ("nodes", ctypes.c_int64),
                ("submit_ms", ctypes.c_double), ("start_ms", ctypes.c_double),
                ("done_ms", ctypes.c_double)]


class _Options(ctypes.Structure):
    _fields_ = [("wg_size", ctypes.c_int32), ("num_wg", ctypes.c_int32),
                ("wl_capacity", ctypes.c_int32), ("wl_threshold", ctypes.c_int32),
                ("node_budget", ctypes.c_int64), ("flags", ctypes.c_int32),
                ("grid_share", ctypes.c_int32), ("start_depth", ctypes.c_int32),
                ("stack_depth", ctypes.c_int32), ("timeout_ms", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("nodes", ctypes.c_int64), ("wg_nodes_max", ctypes.c_int64),
                ("wg_nodes_min", ctypes.c_int64), ("stack_pushes", ctypes.c_int64),
                ("stack_pops", ctypes.c_int64), ("wl_enqueues", ctypes.c_int64),
                ("wl_dequeues", ctypes.c_int64), ("max_stack_depth", ctypes.c_int32),
                ("greedy_size", ctypes.c_int32), ("wg_size", ctypes.c_int32),
                ("num_wg", ctypes.c_int32), ("wl_capacity", ctypes.c_int32),
                ("wl_threshold", ctypes.c_int32), ("depth_cap", ctypes.c_int32),
                ("n", ctypes.c_int32), ("bitset_words", ctypes.c_int32),
                ("node_bytes", ctypes.c_int32), ("kernel_ms", ctypes.c_double),
                ("greedy_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("cycles", ctypes.c_int64 * 10), ("hbm_node_bytes", ctypes.c_int64),
                ("lds_node_bytes", ctypes.c_int64), ("graph_bytes", ctypes.c_int64),
                ("stack_lds", ctypes.c_int32), ("launches", ctypes.c_int32)]


@dataclass
class Options:
    """Launch and search knobs of vc_options (0 = automatic)."""
    wg_size: int = 0
    num_wg: int = 0
    wl_capacity: int = 0
    wl_threshold: int = 0
    node_budget: int = 0
    flags: int = 0
    grid_share: int = 0
    start_depth: int = 0
    stack_depth: int = 0
    timeout_ms: int = 0

    def _c(self) -> _Options:
        o = _Options()
        o.wg_size, o.num_wg = self.wg_size, self.num_wg
        o.wl_capacity, o.wl_threshold = self.wl_capacity, self.wl_threshold
        o.node_budget, o.flags = self.node_budget, self.flags
        o.grid_share, o.start_depth = self.grid_share, self.start_depth
        o.stack_depth, o.timeout_ms = self.stack_depth, self.timeout_ms
        return o


@dataclass
class Result:
    size: int               # MVC: minimum cover size; PVC: cover size or -1
    yes: bool               # PVC decision (True for MVC)
    cover: object           # numpy uint8[n] (host calls) or the caller's device tensor
    stats: dict = field(default_factory=dict)


@dataclass
class BatchResult:
    status: np.ndarray      # int32[count]: OK, ERR_INVALID_GRAPH or ERR_BUDGET per graph
    size: np.ndarray        # int32[count]: MVC size / PVC cover size, -1 on PVC no or error
    yes: np.ndarray         # bool[count]: PVC decision (True for MVC answers)
    nodes: np.ndarray       # int64[count]: search-tree nodes per graph
    cover: object           # packed covers: numpy uint8[sum n] or the caller's device tensor
    offsets: np.ndarray     # int64[count + 1]: graph i's cover is cover[offsets[i]:offsets[i+1]]
    stats: dict = field(default_factory=dict)

    def cover_of(self, i: int):
        return self.cover[int(self.offsets[i]):int(self.offsets[i + 1])]


class VCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libvc.so. Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing; build it with `python -m paper_2204_10402_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    i32p = ctypes.POINTER(ctypes.c_int32)
    gp, op, sp = ctypes.POINTER(_Graph), ctypes.POINTER(_Options), ctypes.POINTER(_Stats)
    bp = ctypes.POINTER(_Batch)
    sig = {
        "vc_create": ([ctypes.POINTER(vp), ctypes.c_int, vp], ctypes.c_int),
        "vc_destroy": ([vp], ctypes.c_int),
        "vc_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "vc_last_error": ([vp], ctypes.c_char_p),
        "vc_version": ([], ctypes.c_char_p),
        "vc_mvc": ([vp, gp, op, i32p, vp, sp], ctypes.c_int),
        "vc_pvc": ([vp, gp, i32, op, i32p, i32p, vp, sp], ctypes.c_int),
        "vc_mvc_device": ([vp, gp, op, i32p, vp, sp], ctypes.c_int),
        "vc_pvc_device": ([vp, gp, i32, op, i32p, i32p, vp, sp], ctypes.c_int),
        "vc_greedy_device": ([vp, gp, i32p, vp], ctypes.c_int),
        "vc_reduce_device": ([vp, gp, vp, i32p, i64, i32], ctypes.c_int),
        "vc_mvc_batch": ([vp, bp, op, vp, vp, vp, vp, sp], ctypes.c_int),
        "vc_pvc_batch": ([vp, bp, vp, op, vp, vp, vp, vp, vp, sp], ctypes.c_int),
        "vc_mvc_batch_device": ([vp, bp, op, vp, vp, vp, vp, sp], ctypes.c_int),
        "vc_pvc_batch_device": ([vp, bp, vp, op, vp, vp, vp, vp, vp, sp], ctypes.c_int),
        "vc_server_create": ([ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(_ServerOptions), op],
                             ctypes.c_int),
        "vc_server_submit": ([vp, gp, i32, i32, vp, ctypes.POINTER(i64)], ctypes.c_int),
        "vc_server_poll": ([vp, ctypes.POINTER(_Served), i32, i32, i32p], ctypes.c_int),
        "vc_server_pending": ([vp, i32p, i32p], ctypes.c_int),
        "vc_server_destroy": ([vp], ctypes.c_int),
        "vc_wg_loads": ([vp, vp, vp, i32, i32p], ctypes.c_int),
        "vc_abort": ([vp], ctypes.c_int),
        "vc_workspace_bytes": ([vp, i32, i32, i32, op, ctypes.POINTER(ctypes.c_size_t)],
                               ctypes.c_int),
        "vc_batch_workspace_bytes": ([vp, bp, i32, op, ctypes.POINTER(ctypes.c_size_t)],
                                     ctypes.c_int),
        "vc_mvc_device_ws": ([vp, gp, op, vp, ctypes.c_size_t, i32p, vp, sp], ctypes.c_int),
        "vc_pvc_device_ws": ([vp, gp, i32, op, vp, ctypes.c_size_t, i32p, i32p, vp, sp],
                             ctypes.c_int),
        "vc_mvc_batch_device_ws": ([vp, bp, op, vp, ctypes.c_size_t, vp, vp, vp, vp, sp],
                                   ctypes.c_int),
        "vc_pvc_batch_device_ws": ([vp, bp, vp, op, vp, ctypes.c_size_t, vp, vp, vp, vp, vp, sp],
                                   ctypes.c_int),
        "vc_pvc_device_noalloc": ([vp, gp, i32, op, i32p, i32p, vp, sp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _stats_dict(s: _Stats) -> dict:
    d = {name: getattr(s, name) for name, _ in _Stats._fields_ if name != "cycles"}
    d["cycles"] = dict(zip(ACTIVITIES, list(s.cycles)))
    return d


def _host_graph(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    cg = _Graph(int(g.n), int(ci.size), rp.ctypes.data, ci.ctypes.data if ci.size else None)
    return cg, (rp, ci)


def _device_graph(row_ptr, col_idx):
    import torch
    for t, name in ((row_ptr, "row_ptr"), (col_idx, "col_idx")):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.int32 \
                or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous int32 device tensor")
    n = row_ptr.numel() - 1
    if n < 0:
        raise ValueError("row_ptr must hold n+1 entries")
    return _Graph(n, col_idx.numel(), row_ptr.data_ptr(),
                  col_idx.data_ptr() if col_idx.numel() else None)


def _device_out(t, name, count, dtype_name):
    """A device output tensor the library writes `count` elements of (None passes through):
    on a GPU, of the named dtype, contiguous and long enough."""
    import torch
    if t is None:
        return None
    dtype = getattr(torch, dtype_name)
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype_name}")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    if t.numel() < count:
        raise ValueError(f"{name} holds {t.numel()} elements, the call writes {count}")
    return t.data_ptr()


def _workspace(ws):
    """(pointer, bytes) of a caller workspace: a contiguous uint8 device tensor."""
    import torch
    if not isinstance(ws, torch.Tensor) or not ws.is_cuda or ws.dtype != torch.uint8 \
            or not ws.is_contiguous():
        raise TypeError("workspace must be a contiguous uint8 device tensor")
    if ws.data_ptr() % 256:
        raise ValueError("workspace must be 256-byte aligned")
    return ws.data_ptr(), ws.numel()


def pack_batch(graphs):
    """Pack CSR graphs one after another (vc_batch layout): returns int32 arrays
    (n, nnz, row_ptr, col_idx). Each graph keeps its own row pointers and vertex ids."""
    n = np.array([g.n for g in graphs], np.int32)
    nnz = np.array([len(g.col_idx) for g in graphs], np.int32)
    rp = np.concatenate([np.asarray(g.row_ptr, np.int32) for g in graphs]) if graphs \
        else np.zeros(0, np.int32)
    ci = np.concatenate([np.asarray(g.col_idx, np.int32) for g in graphs]) if graphs \
        else np.zeros(0, np.int32)
    return n, nnz, np.ascontiguousarray(rp), np.ascontiguousarray(ci)


def _ptr(a):
    return a.ctypes.data if a.size else None


class Solver:
    """One library context (device workspace + HIP stream).

    ``stream``: None for a stream owned by the context, or a ``torch.cuda.Stream`` to run on.
    Device-form calls order themselves after the work queued on torch's current stream.
    """

    def __init__(self, device: int = 0, stream=None):
        self._lib = load_library()
        self._ctx = ctypes.c_void_p()
        self._stream = stream
        handle = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
        rc = self._lib.vc_create(ctypes.byref(self._ctx), int(device), handle)
        if rc != OK:
            raise VCError(rc, f"vc_create failed: {self._lib.vc_strerror(rc).decode()}")
        self.device = device

    def close(self):
        if self._ctx:
            self._lib.vc_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, what: str):
        if rc != OK:
            detail = self._lib.vc_last_error(self._ctx).decode()
            raise VCError(rc, f"{what}: {self._lib.vc_strerror(rc).decode()}: {detail}")

    def _order_after_torch(self):
        import torch
        cur = torch.cuda.current_stream(self.device)
        if self._stream is None or self._stream.cuda_stream != cur.cuda_stream:
            cur.synchronize()

    @staticmethod
    def _opts(options):
        return ctypes.byref(options._c()) if options is not None else None

    # ---- host-memory graphs -------------------------------------------------------------

    def mvc(self, g, options: Options | None = None) -> Result:
        cg, keep = _host_graph(g)
        cover = np.zeros(max(g.n, 1), np.uint8)
        size = ctypes.c_int32()
        st = _Stats()
        rc = self._lib.vc_mvc(self._ctx, ctypes.byref(cg), self._opts(options),
                              ctypes.byref(size), cover.ctypes.data, ctypes.byref(st))
        self._check(rc, "vc_mvc")
        return Result(size.value, True, cover[:g.n], _stats_dict(st))

    def pvc(self, g, k: int, options: Options | None = None) -> Result:
        cg, keep = _host_graph(g)
        cover = np.zeros(max(g.n, 1), np.uint8)
        size, yes = ctypes.c_int32(), ctypes.c_int32()
        st = _Stats()
        rc = self._lib.vc_pvc(self._ctx, ctypes.byref(cg), int(k), self._opts(options),
                              ctypes.byref(yes), ctypes.byref(size), cover.ctypes.data,
                              ctypes.byref(st))
        self._check(rc, "vc_pvc")
        return Result(size.value, bool(yes.value), cover[:g.n], _stats_dict(st))

    # ---- device-memory graphs (torch tensors) --------------------------------------------

    def mvc_device(self, row_ptr, col_idx, cover=None, options: Options | None = None) -> Result:
        cg = _device_graph(row_ptr, col_idx)
        self._order_after_torch()
        size = ctypes.c_int32()
        st = _Stats()
        cov = _device_out(cover, "cover", cg.n, "uint8")
        rc = self._lib.vc_mvc_device(self._ctx, ctypes.byref(cg), self._opts(options),
                                     ctypes.byref(size), cov, ctypes.byref(st))
        self._check(rc, "vc_mvc_device")
        return Result(size.value, True, cover, _stats_dict(st))

    def pvc_device(self, row_ptr, col_idx, k: int, cover=None,
                   options: Options | None = None) -> Result:
        cg = _device_graph(row_ptr, col_idx)
        self._order_after_torch()
        size, yes = ctypes.c_int32(), ctypes.c_int32()
        st = _Stats()
        cov = _device_out(cover, "cover", cg.n, "uint8")
        rc = self._lib.vc_pvc_device(self._ctx, ctypes.byref(cg), int(k), self._opts(options),
                                     ctypes.byref(yes), ctypes.byref(size), cov,
                                     ctypes.byref(st))
        self._check(rc, "vc_pvc_device")
        return Result(size.value, bool(yes.value), cover, _stats_dict(st))

    # ---- batches ----------------------------------------------------------------------------

    def _batch_result(self, count, n, status, size, yes, nodes, cover, st, pvc):
        c = count
        return BatchResult(status[:c].copy(), size[:c].copy(),
                           (yes[:c] != 0) if pvc else (status[:c] == OK),
                           nodes[:c].copy(), cover, _offsets(n), _stats_dict(st))

    def mvc_batch(self, graphs, options: Options | None = None) -> BatchResult:
        n, nnz, rp, ci = pack_batch(graphs)
        cover = np.zeros(max(int(n.sum()), 1), np.uint8)
        status, size, yes, nodes = _batch_arrays(len(graphs))
        cb = _Batch(len(graphs), _ptr(n), _ptr(nnz), _ptr(rp), _ptr(ci))
        st = _Stats()
        rc = self._lib.vc_mvc_batch(self._ctx, ctypes.byref(cb), self._opts(options),
                                    status.ctypes.data, size.ctypes.data, cover.ctypes.data,
                                    nodes.ctypes.data, ctypes.byref(st))
        self._check(rc, "vc_mvc_batch")
        return self._batch_result(len(graphs), n, status, size, yes, nodes,
                                  cover[:int(n.sum())], st, False)

    def pvc_batch(self, graphs, ks, options: Options | None = None) -> BatchResult:
        n, nnz, rp, ci = pack_batch(graphs)
        k = np.ascontiguousarray(ks, dtype=np.int32)
        if k.size != len(graphs):
            raise ValueError("one k per graph")
        cover = np.zeros(max(int(n.sum()), 1), np.uint8)
        status, size, yes, nodes = _batch_arrays(len(graphs))
        cb = _Batch(len(graphs), _ptr(n), _ptr(nnz), _ptr(rp), _ptr(ci))
        st = _Stats()
        rc = self._lib.vc_pvc_batch(self._ctx, ctypes.byref(cb), _ptr(k), self._opts(options),
                                    status.ctypes.data, yes.ctypes.data, size.ctypes.data,
                                    cover.ctypes.data, nodes.ctypes.data, ctypes.byref(st))
        self._check(rc, "vc_pvc_batch")
        return self._batch_result(len(graphs), n, status, size, yes, nodes,
                                  cover[:int(n.sum())], st, True)

    def _device_batch(self, n, nnz, row_ptr, col_idx):
        import torch
        n = np.ascontiguousarray(n, dtype=np.int32)
        nnz = np.ascontiguousarray(nnz, dtype=np.int32)
        for t, name in ((row_ptr, "row_ptr"), (col_idx, "col_idx")):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.int32 \
                    or not t.is_contiguous():
                raise TypeError(f"{name} must be a contiguous int32 device tensor")
        if row_ptr.numel() != int(n.sum()) + n.size or col_idx.numel() != int(nnz.sum()):
            raise ValueError("packed row_ptr / col_idx do not match n / nnz")
        cb = _Batch(n.size, _ptr(n), _ptr(nnz), row_ptr.data_ptr() if row_ptr.numel() else None,
                    col_idx.data_ptr() if col_idx.numel() else None)
        return n, nnz, cb

    def mvc_batch_device(self, n, nnz, row_ptr, col_idx, cover=None,
                         options: Options | None = None) -> BatchResult:
        n, nnz, cb = self._device_batch(n, nnz, row_ptr, col_idx)
        self._order_after_torch()
        status, size, yes, nodes = _batch_arrays(n.size)
        st = _Stats()
        cov = _device_out(cover, "cover", int(n.sum()), "uint8")
        rc = self._lib.vc_mvc_batch_device(self._ctx, ctypes.byref(cb), self._opts(options),
                                           status.ctypes.data, size.ctypes.data, cov,
                                           nodes.ctypes.data, ctypes.byref(st))
        self._check(rc, "vc_mvc_batch_device")
        return self._batch_result(n.size, n, status, size, yes, nodes, cover, st, False)

    def pvc_batch_device(self, n, nnz, row_ptr, col_idx, ks, cover=None,
                         options: Options | None = None) -> BatchResult:
        n, nnz, cb = self._device_batch(n, nnz, row_ptr, col_idx)
        k = np.ascontiguousarray(ks, dtype=np.int32)
        if k.size != n.size:
            raise ValueError("one k per graph")
        self._order_after_torch()
        status, size, yes, nodes = _batch_arrays(n.size)
        st = _Stats()
        cov = _device_out(cover, "cover", int(n.sum()), "uint8")
        rc = self._lib.vc_pvc_batch_device(self._ctx, ctypes.byref(cb), _ptr(k),
                                           self._opts(options), status.ctypes.data,
                                           yes.ctypes.data, size.ctypes.data, cov,
                                           nodes.ctypes.data, ctypes.byref(st))
        self._check(rc, "vc_pvc_batch_device")
        return self._batch_result(n.size, n, status, size, yes, nodes, cover, st, True)

    # ---- caller-owned workspace (vc_*_ws) --------------------------------------------------

    def abort(self):
        """Stop the call running on this context (from another thread): it returns
        ERR_BUDGET."""
        self._check(self._lib.vc_abort(self._ctx), "vc_abort")

    def workspace_bytes(self, n: int, nnz: int, depth: int = 0,
                        options: Options | None = None) -> int:
        out = ctypes.c_size_t()
        self._check(self._lib.vc_workspace_bytes(self._ctx, int(n), int(nnz), int(depth),
                                                 self._opts(options), ctypes.byref(out)),
                    "vc_workspace_bytes")
        return out.value

    def batch_workspace_bytes(self, n, nnz, depth: int = 0,
                              options: Options | None = None) -> int:
        n = np.ascontiguousarray(n, dtype=np.int32)
        nnz = np.ascontiguousarray(nnz, dtype=np.int32)
        cb = _Batch(n.size, _ptr(n), _ptr(nnz), None, None)
        out = ctypes.c_size_t()
        self._check(self._lib.vc_batch_workspace_bytes(self._ctx, ctypes.byref(cb), int(depth),
                                                       self._opts(options), ctypes.byref(out)),
                    "vc_batch_workspace_bytes")
        return out.value

    def mvc_device_ws(self, row_ptr, col_idx, workspace, cover=None,
                      options: Options | None = None) -> Result:
        cg = _device_graph(row_ptr, col_idx)
        wp, wb = _workspace(workspace)
        cov = _device_out(cover, "cover", cg.n, "uint8")
        self._order_after_torch()
        size = ctypes.c_int32()
        st = _Stats()
        rc = self._lib.vc_mvc_device_ws(self._ctx, ctypes.byref(cg), self._opts(options), wp, wb,
                                        ctypes.byref(size), cov, ctypes.byref(st))
        self._check(rc, "vc_mvc_device_ws")
        return Result(size.value, True, cover, _stats_dict(st))

    def pvc_device_ws(self, row_ptr, col_idx, k: int, workspace, cover=None,
                      options: Options | None = None) -> Result:
        cg = _device_graph(row_ptr, col_idx)
        wp, wb = _workspace(workspace)
        cov = _device_out(cover, "cover", cg.n, "uint8")
        self._order_after_torch()
        size, yes = ctypes.c_int32(), ctypes.c_int32()
        st = _Stats()
        rc = self._lib.vc_pvc_device_ws(self._ctx, ctypes.byref(cg), int(k), self._opts(options),
                                        wp, wb, ctypes.byref(yes), ctypes.byref(size), cov,
                                        ctypes.byref(st))
        self._check(rc, "vc_pvc_device_ws")
        return Result(size.value, bool(yes.value), cover, _stats_dict(st))

    def mvc_batch_device_ws(self, n, nnz, row_ptr, col_idx, workspace, cover=None,
                            options: Options | None = None) -> BatchResult:
        n, nnz, cb = self._device_batch(n, nnz, row_ptr, col_idx)
        wp, wb = _workspace(workspace)
        cov = _device_out(cover, "cover", int(n.sum()), "uint8")
        self._order_after_torch()
        status, size, yes, nodes = _batch_arrays(n.size)
        st = _Stats()
        rc = self._lib.vc_mvc_batch_device_ws(self._ctx, ctypes.byref(cb), self._opts(options),
                                              wp, wb, status.ctypes.data, size.ctypes.data, cov,
                                              nodes.ctypes.data, ctypes.byref(st))
        self._check(rc, "vc_mvc_batch_device_ws")
        return self._batch_result(n.size, n, status, size, yes, nodes, cover, st, False)

    def pvc_batch_device_ws(self, n, nnz, row_ptr, col_idx, ks, workspace, cover=None,
                            options: Options | None = None) -> BatchResult:
        n, nnz, cb = self._device_batch(n, nnz, row_ptr, col_idx)
        k = np.ascontiguousarray(ks, dtype=np.int32)
        if k.size != n.size:
            raise ValueError("one k per graph")
        wp, wb = _workspace(workspace)
        cov = _device_out(cover, "cover", int(n.sum()), "uint8")
        self._order_after_torch()
        status, size, yes, nodes = _batch_arrays(n.size)
        st = _Stats()
        rc = self._lib.vc_pvc_batch_device_ws(self._ctx, ctypes.byref(cb), _ptr(k),
                                              self._opts(options), wp, wb, status.ctypes.data,
                                              yes.ctypes.data, size.ctypes.data, cov,
                                              nodes.ctypes.data, ctypes.byref(st))
        self._check(rc, "vc_pvc_batch_device_ws")
        return self._batch_result(n.size, n, status, size, yes, nodes, cover, st, True)

    def pvc_device_noalloc(self, row_ptr, col_idx, k: int, cover=None,
                           options: Options | None = None) -> Result:
        """vc_pvc_device_noalloc: PVC in the library's fixed device scratch (no allocation)."""
        cg = _device_graph(row_ptr, col_idx)
        cov = _device_out(cover, "cover", cg.n, "uint8")
        self._order_after_torch()
        size, yes = ctypes.c_int32(), ctypes.c_int32()
        st = _Stats()
        rc = self._lib.vc_pvc_device_noalloc(self._ctx, ctypes.byref(cg), int(k),
                                             self._opts(options), ctypes.byref(yes),
                                             ctypes.byref(size), cov, ctypes.byref(st))
        self._check(rc, "vc_pvc_device_noalloc")
        return Result(size.value, bool(yes.value), cover, _stats_dict(st))

    def wg_loads(self, cycles: bool = False):
        """Nodes visited by each workgroup of the last traversal launch; with cycles=True also
        its activity clocks, an int64 array [workgroups, 10] (see ACTIVITIES)."""
        count = ctypes.c_int32()
        self._check(self._lib.vc_wg_loads(self._ctx, None, None, 0, ctypes.byref(count)),
                    "vc_wg_loads")
        c = count.value
        out = np.zeros(max(c, 1), np.int64)
        cyc = np.zeros((max(c, 1), len(ACTIVITIES)), np.int64)
        self._check(self._lib.vc_wg_loads(self._ctx, out.ctypes.data,
                                          cyc.ctypes.data if cycles else None, c,
                                          ctypes.byref(count)), "vc_wg_loads")
        return (out[:c], cyc[:c]) if cycles else out[:c]

    def greedy_device(self, row_ptr, col_idx, cover=None) -> int:
        cg = _device_graph(row_ptr, col_idx)
        self._order_after_torch()
        size = ctypes.c_int32()
        cov = _device_out(cover, "cover", cg.n, "uint8")
        rc = self._lib.vc_greedy_device(self._ctx, ctypes.byref(cg), ctypes.byref(size), cov)
        self._check(rc, "vc_greedy_device")
        return size.value

    def reduce_device(self, row_ptr, col_idx, deg, s: int, bound: int, flags: int = 0) -> int:
        """Reduction rules in place on the int32 device tensor ``deg``; returns the new s."""
        cg = _device_graph(row_ptr, col_idx)
        self._order_after_torch()
        if deg is None:
            raise TypeError("deg must be a device tensor")
        dp = _device_out(deg, "deg", cg.n, "int32")
        sv = ctypes.c_int32(int(s))
        rc = self._lib.vc_reduce_device(self._ctx, ctypes.byref(cg), dp,
                                        ctypes.byref(sv), int(bound), int(flags))
        self._check(rc, "vc_reduce_device")
        return sv.value


def _batch_arrays(count: int):
    return (np.zeros(max(count, 1), np.int32), np.zeros(max(count, 1), np.int32),
            np.zeros(max(count, 1), np.int32), np.zeros(max(count, 1), np.int64))


def _offsets(n):
    off = np.zeros(len(n) + 1, np.int64)
    np.cumsum(n, out=off[1:])
    return off


class Server:
    """Continuous batching of a request stream (vc_server_*): submit graphs as they arrive,
    poll finished results. Each worker runs batches on its own context and stream."""

    def __init__(self, device: int = 0, workers: int = 0, max_batch: int = 0,
                 memory_budget: int = 0, wg_per_request: int = 0,
                 options: Options | None = None):
        self._lib = load_library()
        self._srv = ctypes.c_void_p()
        so = _ServerOptions(workers, max_batch, memory_budget, wg_per_request)
        rc = self._lib.vc_server_create(ctypes.byref(self._srv), int(device), ctypes.byref(so),
                                        ctypes.byref(options._c()) if options else None)
        if rc != OK:
            raise VCError(rc, f"vc_server_create: {self._lib.vc_strerror(rc).decode()}")
        self._covers = {}
        self._buf = (_Served * 1024)()

    def submit(self, g, problem: str, k: int = 0, cover: bool = True) -> int:
        """Queue graph `g` (host CSR, copied) for "mvc" or "pvc" with parameter k."""
        cg, keep = _host_graph(g)
        code = {"mvc": PROBLEM_MVC, "pvc": PROBLEM_PVC}[problem]
        buf = np.zeros(max(g.n, 1), np.uint8) if cover else None
        ticket = ctypes.c_int64()
        rc = self._lib.vc_server_submit(self._srv, ctypes.byref(cg), code, int(k),
                                        buf.ctypes.data if buf is not None else None,
                                        ctypes.byref(ticket))
        if rc != OK:
            raise VCError(rc, f"vc_server_submit: {self._lib.vc_strerror(rc).decode()}")
        if buf is not None:
            self._covers[ticket.value] = (buf, g.n)
        return ticket.value

    def poll(self, timeout_ms: int = 0, max_results: int = 1024) -> list[dict]:
        """Finished results (waits up to timeout_ms when none is ready)."""
        count = ctypes.c_int32()
        m = min(max_results, len(self._buf))
        rc = self._lib.vc_server_poll(self._srv, self._buf, m, int(timeout_ms),
                                      ctypes.byref(count))
        if rc != OK:
            raise VCError(rc, "vc_server_poll")
        out = []
        for i in range(count.value):
            r = self._buf[i]
            d = {name: getattr(r, name) for name, _ in _Served._fields_ if name != "pad"}
            cov = self._covers.pop(r.ticket, None)
            if cov is not None:
                d["cover"] = cov[0][:cov[1]]
            out.append(d)
        return out

    def pending(self) -> tuple[int, int]:
        q, r = ctypes.c_int32(), ctypes.c_int32()
        self._lib.vc_server_pending(self._srv, ctypes.byref(q), ctypes.byref(r))
        return q.value, r.value

    def close(self):
        if self._srv:
            self._lib.vc_server_destroy(self._srv)
            self._srv = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def version() -> str:
    return load_library().vc_version().decode()
