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
  pl_refusable      Eq. 3's maxima all above the current label (Pick-Less).
  cpu_lpa_async     not the oracle: the multi-core CPU throughput baseline of
                    the benchmark (asynchronous order, OpenMP; cpu_async.c).
  lpa_learned       Algorithm 1 with the learned change predictor: per-vertex
                    state records, features, skipping schedule, guard and
                    fallback, traces (learned_oracle.c; a project addition).
  mlp (module)      the change-predictor network (fp64 on bf16-rounded data).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "lpa_oracle.c"), os.path.join(_HERE, "learned_oracle.c"),
         os.path.join(_HERE, "cpu_async.c")]
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
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               *_SRCS, "-o", tmp, "-lm"])
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
        lib.oracle_lpa_sync_cc.argtypes = [ctypes.c_int64, vp, vp, vp, ctypes.c_double,
                                           ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, vp, vp, vp, ctypes.c_int32, vp]
        lib.oracle_lpa_sync_cc.restype = ctypes.c_int
        for f in (lib.oracle_modularity, lib.oracle_modularity_pairs):
            f.argtypes = [ctypes.c_int64, vp, vp, vp, vp]
            f.restype = ctypes.c_double
        lib.oracle_local_optimal.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp]
        lib.oracle_local_optimal.restype = ctypes.c_int64
        lib.oracle_lpa_learned.argtypes = [
            ctypes.c_int64, vp, vp, vp, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
            ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, vp,
            ctypes.c_double,
            ctypes.c_double, ctypes.c_double, ctypes.c_uint64, vp, vp, vp, vp, ctypes.c_int64,
            vp, vp, vp, vp, ctypes.c_int32, vp, vp]
        lib.oracle_lpa_learned.restype = ctypes.c_int
        lib.cpu_lpa_async_omp.argtypes = [ctypes.c_int64, vp, vp, vp, ctypes.c_double,
                                          ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
        lib.cpu_lpa_async_omp.restype = ctypes.c_int32
        lib.oracle_mlp_logit.argtypes = [vp, vp]
        lib.oracle_mlp_logit.restype = ctypes.c_double
        lib.oracle_features.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp]
        lib.oracle_features.restype = ctypes.c_int
        lib.oracle_lq.argtypes = [ctypes.c_uint64, ctypes.c_float, vp]
        lib.oracle_lq.restype = ctypes.c_int
        lib.oracle_sample_draw.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64]
        lib.oracle_sample_draw.restype = ctypes.c_double
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
             initial_labels=None, cc_period: int = 0) -> SyncResult:
    """Algorithm 1, deterministic synchronous order (lpa_oracle.c); cc_period
    > 0 adds the Cross-Check of Sec. 4.1 in iterations l % cc_period == 0."""
    off, tgt, w = _csr(offsets, targets, weights)
    n = off.shape[0] - 1
    labels = np.empty(max(n, 0), dtype=np.int32)
    init = None if initial_labels is None else np.ascontiguousarray(initial_labels, dtype=np.int32)
    cap = max(int(max_iterations), 0)
    stats = (IterStats * max(cap, 1))()
    iters = ctypes.c_int32(0)
    if cc_period:
        rc = _load().oracle_lpa_sync_cc(n, _p(off), _p(tgt), _p(w), float(tolerance), cap,
                                        int(pl_period), int(cc_period), int(bool(prune)),
                                        _p(init), _p(labels), ctypes.cast(stats, ctypes.c_void_p),
                                        cap, ctypes.cast(ctypes.byref(iters), ctypes.c_void_p))
    else:
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


@dataclass
class AsyncCpuResult:
    labels: np.ndarray
    iterations: int
    changed_last: int
    threads: int


def cpu_lpa_async(offsets, targets, weights=None, tolerance: float = 0.05,
                  max_iterations: int = 20, pl_period: int = 4) -> AsyncCpuResult:
    """The CPU throughput baseline (cpu_async.c; not the oracle): Algorithm 1
    in asynchronous order on all OpenMP threads."""
    off, tgt, w = _csr(offsets, targets, weights)
    n = off.shape[0] - 1
    labels = np.empty(max(n, 0), dtype=np.int32)
    last = ctypes.c_int64(0)
    thr = ctypes.c_int32(0)
    it = _load().cpu_lpa_async_omp(n, _p(off), _p(tgt), _p(w), float(tolerance),
                                   int(max_iterations), int(pl_period), _p(labels),
                                   ctypes.cast(ctypes.byref(last), ctypes.c_void_p),
                                   ctypes.cast(ctypes.byref(thr), ctypes.c_void_p))
    if it < 0:
        raise MemoryError("cpu_lpa_async_omp")
    return AsyncCpuResult(labels, int(it), int(last.value), int(thr.value))


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


def pl_refusable(offsets, targets, weights, labels, verts) -> np.ndarray:
    """Per vertex of verts: True when every label of maximum Eq. 3 weight is
    larger than the vertex's own, i.e. a move that Pick-Less (Sec. 4.1)
    refuses.  With Pick-Less on, an asynchronous run may end with such a
    vertex unflagged and off the maximum (it was refused at its last
    evaluation and no neighbour changed since); any other unflagged vertex
    must attain the maximum.  Plain numpy over the given rows."""
    off, tgt, w = _csr(offsets, targets, weights)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    out = np.zeros(len(verts), dtype=bool)
    for q, i in enumerate(np.asarray(verts, dtype=np.int64)):
        a, b = int(off[i]), int(off[i + 1])
        nb = tgt[a:b]
        keep = nb != i
        if not keep.any():
            continue
        ls, inv = np.unique(lab[nb[keep]], return_inverse=True)
        sums = np.zeros(ls.shape[0])
        ww = np.ones(b - a) if w is None else w[a:b].astype(np.float64)
        np.add.at(sums, inv, ww[keep])
        out[q] = bool(np.all(ls[sums == sums.max()] > lab[i]))
    return out


class LearnedStats(ctypes.Structure):
    _fields_ = [("iteration", ctypes.c_int32), ("pick_less", ctypes.c_int32),
                ("changed", ctypes.c_int64), ("processed", ctypes.c_int64),
                ("edges_scanned", ctypes.c_int64), ("skipped", ctypes.c_int64),
                ("predicted", ctypes.c_int64), ("false_neg", ctypes.c_int64),
                ("skipping", ctypes.c_int32), ("fallback", ctypes.c_int32)]


@dataclass
class LearnedResult:
    labels: np.ndarray
    stats: list
    iterations: int
    records: np.ndarray        # uint8 [n, 8]
    min_margin: float          # smallest |z - z_theta| over all predictions
    trace: dict | None         # X [k, 12], y [k], v [k], l [k] (k = samples kept)
    trace_total: int           # samples drawn (may exceed the capacity)


def lpa_learned(offsets, targets, weights=None, *, params=None, z_theta: float = 0.0,
                tolerance: float = 0.05, max_iterations: int = 20, pl_period: int = 4,
                prune: bool = True, guard: int = 4, max_pred_degree: int = 8192,
                min_pred_degree: int = 1, pred_start: int = 1,
                fn_bound: float = 0.02, sample_rate: float = 0.0, seed: int = 0,
                trace_cap: int = 0) -> LearnedResult:
    """Synchronous LPA with the learned change predictor (learned_oracle.c).
    params: 5,057 fp32 network parameters or None (plain schedule).  Rows of
    min_pred_degree .. max_pred_degree entries are predicted (and keep
    records); the others are always processed.  Predictions (and traces)
    start at iteration pred_start, records one iteration earlier."""
    off, tgt, w = _csr(offsets, targets, weights)
    n = off.shape[0] - 1
    labels = np.empty(max(n, 0), dtype=np.int32)
    rec = np.empty((max(n, 0), 8), dtype=np.uint8)
    cap = max(int(max_iterations), 0)
    stats = (LearnedStats * max(cap, 1))()
    iters = ctypes.c_int32(0)
    margin = ctypes.c_double(0.0)
    P = None if params is None else np.ascontiguousarray(params, dtype=np.float32).ravel()
    if P is not None and P.shape[0] != 5057:
        raise ValueError("params must hold 5057 values")
    tc = max(int(trace_cap), 0)
    tX = np.zeros((max(tc, 1), 12), dtype=np.float32) if tc else None
    ty = np.zeros(max(tc, 1), dtype=np.float32) if tc else None
    tv = np.zeros(max(tc, 1), dtype=np.int32) if tc else None
    tl = np.zeros(max(tc, 1), dtype=np.int32) if tc else None
    tcount = ctypes.c_int64(0)
    rc = _load().oracle_lpa_learned(
        n, _p(off), _p(tgt), _p(w), float(tolerance), cap, int(pl_period), int(bool(prune)),
        int(guard), int(min_pred_degree), int(max_pred_degree), int(pred_start), _p(P),
        float(z_theta),
        float(fn_bound),
        float(sample_rate), int(seed) & 0xFFFFFFFFFFFFFFFF, _p(tX), _p(ty), _p(tv), _p(tl),
        tc, ctypes.cast(ctypes.byref(tcount), ctypes.c_void_p), _p(labels), _p(rec),
        ctypes.cast(stats, ctypes.c_void_p), cap,
        ctypes.cast(ctypes.byref(iters), ctypes.c_void_p),
        ctypes.cast(ctypes.byref(margin), ctypes.c_void_p))
    if rc != 0:
        raise ValueError("oracle_lpa_learned rejected its arguments")
    k = int(iters.value)
    st = [{f: getattr(s, f) for f, _ in LearnedStats._fields_} for s in stats[:k]]
    trace = None
    if tc:
        kept = min(int(tcount.value), tc)
        trace = dict(X=tX[:kept].copy(), y=ty[:kept].copy(), v=tv[:kept].copy(),
                     l=tl[:kept].copy())
    return LearnedResult(labels, st, k, rec, float(margin.value), trace, int(tcount.value))


def mlp_logit(params, features) -> float:
    P = np.ascontiguousarray(params, dtype=np.float32).ravel()
    f = np.ascontiguousarray(features, dtype=np.float32).ravel()
    return float(_load().oracle_mlp_logit(_p(P), _p(f)))


def record_features(record, iteration: int, cap: int, pl_period: int) -> np.ndarray:
    r = np.ascontiguousarray(record, dtype=np.uint8).ravel()
    f = np.zeros(12, dtype=np.float32)
    _load().oracle_features(_p(r), int(iteration), int(cap), int(pl_period), _p(f))
    return f


def log_quant(u: int, x: float) -> tuple:
    """(lq of the integer u >= 1, lq of the fp32 value x >= 1)."""
    out = np.zeros(2, dtype=np.uint8)
    _load().oracle_lq(int(u), float(x), _p(out))
    return int(out[0]), int(out[1])


def sample_draw(seed: int, iteration: int, v: int) -> float:
    return float(_load().oracle_sample_draw(int(seed) & 0xFFFFFFFFFFFFFFFF, int(iteration),
                                            int(v)))
