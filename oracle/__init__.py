"""CPU oracle for the label-propagation sweep -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It is the plain sequential reference the GPU library is
checked against and shares no code with it.  The arithmetic lives in
``lpa_oracle.c`` (plain C, fp64 accumulation); this module only compiles it
with gcc and marshals numpy arrays.

Functions and the passages they follow (paper arXiv 2411.11468):
  lpa_sync          Algorithm 1 (lpa / lpaMove) in synchronous order, Eq. 3,
                    Pick-Less (Sec. 4.1), pruning/tolerance/cap (Sec. 4).
  modularity        Eq. 1, community form.
  modularity_pairs  Eq. 1, pair form over all vertex pairs (tiny graphs).
  local_optimal     Eq. 3 attained by the current label, per vertex.
  mlp_*             the change-predictor network (fp64 on bf16-rounded data).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lpa_oracle.c")
_LIB = os.path.join(_HERE, "liblpa_oracle.so")
_lib = None


class IterStats(ctypes.Structure):
    _fields_ = [("iteration", ctypes.c_int32), ("pick_less", ctypes.c_int32),
                ("changed", ctypes.c_int64), ("processed", ctypes.c_int64),
                ("edges_scanned", ctypes.c_int64)]


def build(force: bool = True) -> str:
    """Compile liblpa_oracle.so with gcc (plain C, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        lib.oracle_lpa_sync.argtypes = [ctypes.c_int64, vp, vp, vp, ctypes.c_double,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        vp, vp, vp, ctypes.c_int32, vp]
        lib.oracle_lpa_sync.restype = ctypes.c_int
        for f in (lib.oracle_modularity, lib.oracle_modularity_pairs):
            f.argtypes = [ctypes.c_int64, vp, vp, vp, vp]
            f.restype = ctypes.c_double
        lib.oracle_local_optimal.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp]
        lib.oracle_local_optimal.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _csr(offsets, targets, weights):
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    tgt = np.ascontiguousarray(targets, dtype=np.int32)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float32)
    return off, tgt, w


@dataclass
class SyncResult:
    labels: np.ndarray
    stats: list  # list of dicts, one per iteration
    iterations: int


def lpa_sync(offsets, targets, weights=None, tolerance: float = 0.05,
             max_iterations: int = 20, pl_period: int = 4, prune: bool = True,
             initial_labels=None) -> SyncResult:
    off, tgt, w = _csr(offsets, targets, weights)
    n = off.shape[0] - 1
    labels = np.empty(max(n, 0), dtype=np.int32)
    init = None if initial_labels is None else np.ascontiguousarray(initial_labels, dtype=np.int32)
    cap = max(int(max_iterations), 0)
    stats = (IterStats * max(cap, 1))()
    iters = ctypes.c_int32(0)
    rc = _load().oracle_lpa_sync(n, _p(off), _p(tgt), _p(w), float(tolerance), cap,
                                 int(pl_period), int(bool(prune)), _p(init), _p(labels),
                                 ctypes.cast(stats, ctypes.c_void_p), cap,
                                 ctypes.cast(ctypes.byref(iters), ctypes.c_void_p))
    if rc != 0:
        raise ValueError("oracle_lpa_sync rejected its arguments")
    k = int(iters.value)
    st = [dict(iteration=s.iteration, pick_less=s.pick_less, changed=s.changed,
               processed=s.processed, edges_scanned=s.edges_scanned) for s in stats[:k]]
    return SyncResult(labels, st, k)


def modularity(offsets, targets, weights, labels) -> float:
    off, tgt, w = _csr(offsets, targets, weights)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    return float(_load().oracle_modularity(off.shape[0] - 1, _p(off), _p(tgt), _p(w), _p(lab)))


def modularity_pairs(offsets, targets, weights, labels) -> float:
    off, tgt, w = _csr(offsets, targets, weights)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    return float(_load().oracle_modularity_pairs(off.shape[0] - 1, _p(off), _p(tgt), _p(w), _p(lab)))


def local_optimal(offsets, targets, weights, labels) -> np.ndarray:
    """Boolean per vertex: current label attains the Eq. 3 maximum."""
    off, tgt, w = _csr(offsets, targets, weights)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    out = np.empty(off.shape[0] - 1, dtype=np.uint8)
    bad = _load().oracle_local_optimal(off.shape[0] - 1, _p(off), _p(tgt), _p(w), _p(lab), _p(out))
    if bad < 0:
        raise MemoryError("oracle_local_optimal")
    return out.astype(bool)
