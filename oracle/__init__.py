"""CPU oracle for batch-dynamic rooted spanning forest updates.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU product
path never touches it.

``oracle.c`` holds the plain single-threaded reference (``oracle_apply``) and
the forest checker (``oracle_check_forest``); this module compiles it with
gcc and wraps it with ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

INSERT, DELETE = 0, 1
OK, E_ARG, E_NOMEM, E_FOREST, E_BATCH = 0, -1, -2, -3, -4


class _Stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "k", "ell", "n_key", "n_cross", "n_repl", "n_tree_deleted",
        "n_parent_changed", "n_label_changed", "m_out")]


@dataclass
class Result:
    keys: np.ndarray      # sorted unique uint64 keys of G'
    parent: np.ndarray    # int32[n]
    label: np.ndarray     # int32[n]
    stats: dict


class OracleError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the oracle library in-tree (plain C, -O2, no threads)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.oracle_apply.restype = ctypes.c_int
    lib.oracle_apply.argtypes = [i32, vp, i64, vp, vp, vp, i64, ctypes.c_int, ctypes.c_int,
                                 vp, vp, vp, vp, ctypes.POINTER(_Stats)]
    lib.oracle_check_forest.restype = ctypes.c_int
    lib.oracle_check_forest.argtypes = [i32, vp, i64, vp, vp, ctypes.c_int, ctypes.c_char_p,
                                        ctypes.c_int]
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data


def apply(n: int, keys: np.ndarray, parent: np.ndarray, batch: np.ndarray, op: int,
          label: np.ndarray | None = None, scan_all: bool = False) -> Result:
    """Apply one batch; raises OracleError on a rejected batch or bad forest."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    batch = np.ascontiguousarray(np.asarray(batch, dtype=np.int32).reshape(-1, 2))
    if label is not None:
        label = np.ascontiguousarray(label, dtype=np.int32)
    b = batch.shape[0]
    out_keys = np.empty(len(keys) + b + 1, dtype=np.uint64)
    m_out = np.zeros(1, dtype=np.int64)
    par = np.empty(n, dtype=np.int32)
    lab = np.empty(n, dtype=np.int32)
    st = _Stats()
    rc = _load().oracle_apply(n, _p(keys), len(keys), _p(parent), _p(label), _p(batch), b,
                              op, int(scan_all), _p(out_keys), _p(m_out), _p(par), _p(lab),
                              ctypes.byref(st))
    if rc != OK:
        raise OracleError(rc)
    stats = {name: int(getattr(st, name)) for name, _ in _Stats._fields_}
    return Result(out_keys[: int(m_out[0])].copy(), par, lab, stats)


def check_forest(n: int, keys: np.ndarray, parent: np.ndarray, label: np.ndarray | None = None,
                 require_min_root: bool = True) -> tuple[int, str]:
    """Validate a rooted spanning forest of the graph given by sorted keys."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    if label is not None:
        label = np.ascontiguousarray(label, dtype=np.int32)
    buf = ctypes.create_string_buffer(512)
    rc = _load().oracle_check_forest(n, _p(keys), len(keys), _p(parent), _p(label),
                                     int(require_min_root), buf, 512)
    return rc, buf.value.decode()
