"""CPU oracle for the vertex-cover search -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package. The product library never calls it, and shares no code with it.

The arithmetic lives in ``vc_oracle.c`` (plain sequential C, one thread); this module only
builds it with gcc and marshals numpy arrays through ctypes.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vc_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

RULE_DEG1 = 1
RULE_TRI = 2
RULE_HIGH = 4
PRUNE_EDGES = 8
ALL = 15

_STATUS = {0: "ok", 1: "node budget exhausted", 2: "bad argument", 3: "out of memory"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.vco_tau_by_definition.argtypes = [ctypes.c_int32, i32p, i32p, u8p]
        lib.vco_tau_by_definition.restype = ctypes.c_int32
        lib.vco_greedy.argtypes = [ctypes.c_int32, i32p, i32p, u8p]
        lib.vco_greedy.restype = ctypes.c_int32
        lib.vco_reduce.argtypes = [ctypes.c_int32, i32p, i32p, i32p, i32p, ctypes.c_int64,
                                   ctypes.c_int32]
        lib.vco_reduce.restype = None
        lib.vco_mvc.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32, ctypes.c_int64,
                                i32p, u8p, i64p, i32p]
        lib.vco_mvc.restype = ctypes.c_int
        lib.vco_pvc.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int64, ctypes.c_int32,
                                ctypes.c_int64, i32p, i32p, u8p, i64p]
        lib.vco_pvc.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    if ci.size == 0:
        ci = np.zeros(1, np.int32)
    return rp, ci


@dataclass
class Result:
    size: int          # MVC: minimum cover size; PVC: cover size, -1 on "no"
    cover: np.ndarray  # uint8[n]
    nodes: int         # search-tree nodes visited
    yes: bool | None = None
    greedy: int | None = None


class BudgetExceeded(RuntimeError):
    pass


def tau_by_definition(g):
    """Minimum cover size by exhaustive subset enumeration (n <= 24)."""
    rp, ci = _csr(g)
    cover = np.zeros(max(g.n, 1), np.uint8)
    t = _load().vco_tau_by_definition(g.n, _p(rp, ctypes.c_int32), _p(ci, ctypes.c_int32),
                                      _p(cover, ctypes.c_uint8))
    if t < 0:
        raise ValueError("graph too large for exhaustive enumeration")
    return int(t), cover[:g.n]


def greedy(g):
    rp, ci = _csr(g)
    cover = np.zeros(max(g.n, 1), np.uint8)
    s = _load().vco_greedy(g.n, _p(rp, ctypes.c_int32), _p(ci, ctypes.c_int32),
                           _p(cover, ctypes.c_uint8))
    return int(s), cover[:g.n]


def reduce(g, deg, s, bound, rules=RULE_DEG1 | RULE_TRI | RULE_HIGH):
    """Reduction rules to a fixpoint on a copy of ``deg``; returns (deg, s)."""
    rp, ci = _csr(g)
    d = np.array(deg, dtype=np.int32, copy=True)
    if d.size == 0:
        d = np.zeros(1, np.int32)
    sv = ctypes.c_int32(int(s))
    _load().vco_reduce(g.n, _p(rp, ctypes.c_int32), _p(ci, ctypes.c_int32),
                       _p(d, ctypes.c_int32), ctypes.byref(sv), int(bound), int(rules))
    return d[:g.n], int(sv.value)


def mvc(g, rules=ALL, node_cap=0):
    rp, ci = _csr(g)
    cover = np.zeros(max(g.n, 1), np.uint8)
    size = ctypes.c_int32(0)
    nodes = ctypes.c_int64(0)
    gr = ctypes.c_int32(0)
    rc = _load().vco_mvc(g.n, _p(rp, ctypes.c_int32), _p(ci, ctypes.c_int32), int(rules),
                         int(node_cap), ctypes.byref(size), _p(cover, ctypes.c_uint8),
                         ctypes.byref(nodes), ctypes.byref(gr))
    if rc == 1:
        raise BudgetExceeded(f"oracle node cap {node_cap} reached")
    if rc != 0:
        raise RuntimeError(f"oracle mvc failed: {_STATUS.get(rc, rc)}")
    return Result(int(size.value), cover[:g.n], int(nodes.value), None, int(gr.value))


def pvc(g, k, rules=ALL, node_cap=0):
    rp, ci = _csr(g)
    cover = np.zeros(max(g.n, 1), np.uint8)
    size = ctypes.c_int32(0)
    yes = ctypes.c_int32(0)
    nodes = ctypes.c_int64(0)
    rc = _load().vco_pvc(g.n, _p(rp, ctypes.c_int32), _p(ci, ctypes.c_int32), int(k),
                         int(rules), int(node_cap), ctypes.byref(yes), ctypes.byref(size),
                         _p(cover, ctypes.c_uint8), ctypes.byref(nodes))
    if rc == 1:
        raise BudgetExceeded(f"oracle node cap {node_cap} reached")
    if rc != 0:
        raise RuntimeError(f"oracle pvc failed: {_STATUS.get(rc, rc)}")
    return Result(int(size.value), cover[:g.n], int(nodes.value), bool(yes.value))


def is_cover(g, cover) -> bool:
    """Every edge has at least one endpoint in ``cover`` (checked edge by edge)."""
    cover = np.asarray(cover).astype(bool)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    return bool(np.all(cover[src] | cover[g.col_idx])) if g.nnz else True
