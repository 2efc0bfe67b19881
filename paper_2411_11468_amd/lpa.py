"""ctypes binding of the C ABI in include/lpa.h (liblpa.so, HIP for gfx950).

Argument marshalling only: every step of the label sweep runs in the HIP
kernels of liblpa.so.  There is no CPU fallback; if the library is missing
the import of a function raises.  torch supplies device memory and the
stream (``torch.cuda.current_stream().cuda_stream``); numpy arrays are
accepted as host memory.

Names follow the C ABI: lpa_create, lpa_run, lpa_modularity, lpa_destroy,
lpa_graph_classes, plus the ``LpaGraph`` convenience wrapper.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblpa.so")

LPA_OK = 0
# lpa_status
OK, ERR_INVALID, ERR_OOM, ERR_HIP, ERR_STATE, ERR_UNSUPPORTED = 0, 1, 2, 3, 4, 5

MODE_DETERMINISTIC = 0
MODE_ASYNC = 1
INDEX_I32 = 0
INDEX_I64 = 1
FLAGS_AUTO = 0
FLAGS_PUSH = 1
FLAGS_PULL = 2
LAUNCH_EAGER = 0
LAUNCH_GRAPH = 1
CLASS_NAMES = ("degree0", "small4", "small16", "wave", "block", "hub")


class LpaError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"lpa status {status}: {detail}")
        self.status = status


class lpa_csr(ctypes.Structure):
    _fields_ = [("num_vertices", ctypes.c_int64), ("num_edges", ctypes.c_int64),
                ("offset_type", ctypes.c_int32), ("on_device", ctypes.c_int32),
                ("offsets", ctypes.c_void_p), ("targets", ctypes.c_void_p),
                ("weights", ctypes.c_void_p), ("validate", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class lpa_tuning(ctypes.Structure):
    _fields_ = [("small4", ctypes.c_int32), ("small16", ctypes.c_int32),
                ("wave", ctypes.c_int32), ("block", ctypes.c_int32),
                ("hub_chunk", ctypes.c_int32), ("max_retries", ctypes.c_int32),
                ("xcd_local", ctypes.c_int32), ("hub_table_cap", ctypes.c_int32),
                ("relabel", ctypes.c_int32), ("probe", ctypes.c_int32),
                ("table_values", ctypes.c_int32), ("batch_queue", ctypes.c_int32),
                ("queue_chunk", ctypes.c_int32), ("queue_group", ctypes.c_int32),
                ("sort_rows", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("table_load", ctypes.c_int32), ("pull_divisor", ctypes.c_int32),
                ("memory_limit_kib", ctypes.c_int32)]


class lpa_options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("max_iterations", ctypes.c_int32),
                ("tolerance", ctypes.c_double), ("pl_period", ctypes.c_int32),
                ("prune", ctypes.c_int32), ("initial_labels", ctypes.c_void_p),
                ("profile", ctypes.c_int32), ("flag_mode", ctypes.c_int32),
                ("launch", ctypes.c_int32), ("learned", ctypes.c_int32),
                ("cc_period", ctypes.c_int32)]


class lpa_learned_options(ctypes.Structure):
    _fields_ = [("threshold", ctypes.c_float), ("fn_bound", ctypes.c_float),
                ("guard_period", ctypes.c_int32), ("predict_small", ctypes.c_int32),
                ("predict_large", ctypes.c_int32), ("first_predicted", ctypes.c_int32)]


class lpa_learned_iter(ctypes.Structure):
    _fields_ = [("iteration", ctypes.c_int32), ("skipping", ctypes.c_int32),
                ("fallback", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("skipped", ctypes.c_int64), ("predicted", ctypes.c_int64),
                ("false_negatives", ctypes.c_int64)]


class lpa_tune_report(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int32), ("runs", ctypes.c_int32),
                ("rounds", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double),
                ("elapsed_ms", ctypes.c_double)]


class lpa_kernel_profile(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double),
                ("edges", ctypes.c_int64), ("vertices", ctypes.c_int64)]


class lpa_train_options(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("pos_weight", ctypes.c_float), ("seed", ctypes.c_uint64)]


class lpa_iter_stats(ctypes.Structure):
    _fields_ = [("iteration", ctypes.c_int32), ("pick_less", ctypes.c_int32),
                ("changed", ctypes.c_int64), ("processed", ctypes.c_int64),
                ("edges_scanned", ctypes.c_int64), ("ms", ctypes.c_float),
                ("skipped", ctypes.c_int32)]


EXPORTED = ("lpa_options_default", "lpa_tuning_default", "lpa_create", "lpa_run",
            "lpa_modularity", "lpa_graph_classes", "lpa_get_flags", "lpa_profile",
            "lpa_profile_reset", "lpa_destroy", "lpa_status_string", "lpa_last_error",
            "lpa_create_batched", "lpa_run_batched", "lpa_predictor_create",
            "lpa_predictor_destroy", "lpa_predictor_set_params", "lpa_predictor_get_params",
            "lpa_predictor_gradient", "lpa_predictor_adam", "lpa_predictor_train",
            "lpa_predictor_predict", "lpa_learned_options_default", "lpa_set_predictor",
            "lpa_learned_history", "lpa_get_records", "lpa_trace", "lpa_autotune",
            "lpa_label_read_rate", "lpa_modularity_noalloc", "lpa_predictor_save",
            "lpa_predictor_load")

_lib = None


def load_library(path: str | None = None):
    """Load liblpa.so (raises if it has not been built).  LPA_LIBRARY in the
    environment names another build of the same ABI."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("LPA_LIBRARY") or LIB_PATH
    # One HIP runtime per process: torch ships its own libamdhip64.so.7 with
    # the same soname as ROCm's.  Importing torch first lets liblpa.so bind
    # to the copy torch uses; loading liblpa.so first would map ROCm's copy
    # as well, and torch's device memory would then belong to another
    # runtime instance than the library's calls.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_2411_11468_amd.build`")
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.lpa_options_default.argtypes = [ctypes.POINTER(lpa_options)]
    lib.lpa_options_default.restype = None
    lib.lpa_tuning_default.argtypes = [ctypes.POINTER(lpa_tuning)]
    lib.lpa_tuning_default.restype = None
    lib.lpa_create.argtypes = [ctypes.POINTER(lpa_csr), vp, ctypes.POINTER(lpa_tuning),
                               ctypes.POINTER(vp)]
    lib.lpa_create.restype = ctypes.c_int
    lib.lpa_run.argtypes = [vp, ctypes.POINTER(lpa_options), vp,
                            ctypes.POINTER(lpa_iter_stats), ctypes.c_int32,
                            ctypes.POINTER(ctypes.c_int32)]
    lib.lpa_run.restype = ctypes.c_int
    lib.lpa_modularity.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double)]
    lib.lpa_modularity.restype = ctypes.c_int
    lib.lpa_modularity_noalloc.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double)]
    lib.lpa_modularity_noalloc.restype = ctypes.c_int
    lib.lpa_label_read_rate.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
    lib.lpa_label_read_rate.restype = ctypes.c_int
    lib.lpa_graph_classes.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.lpa_graph_classes.restype = ctypes.c_int
    lib.lpa_get_flags.argtypes = [vp, vp]
    lib.lpa_get_flags.restype = ctypes.c_int
    lib.lpa_profile.argtypes = [vp, ctypes.POINTER(lpa_kernel_profile), ctypes.c_int32,
                                ctypes.POINTER(ctypes.c_int32)]
    lib.lpa_profile.restype = ctypes.c_int
    lib.lpa_profile_reset.argtypes = [vp]
    lib.lpa_profile_reset.restype = ctypes.c_int
    lib.lpa_create_batched.argtypes = [ctypes.c_int32, vp, ctypes.POINTER(lpa_csr), vp,
                                       ctypes.POINTER(lpa_tuning), ctypes.POINTER(vp)]
    lib.lpa_create_batched.restype = ctypes.c_int
    lib.lpa_run_batched.argtypes = [vp, ctypes.POINTER(lpa_options), vp, vp, vp,
                                    ctypes.POINTER(ctypes.c_int32)]
    lib.lpa_run_batched.restype = ctypes.c_int
    lib.lpa_destroy.argtypes = [vp]
    lib.lpa_destroy.restype = None
    fp = ctypes.POINTER(ctypes.c_float)
    lib.lpa_predictor_create.argtypes = [ctypes.c_uint64, vp, ctypes.POINTER(vp)]
    lib.lpa_predictor_create.restype = ctypes.c_int
    lib.lpa_predictor_destroy.argtypes = [vp]
    lib.lpa_predictor_destroy.restype = None
    lib.lpa_predictor_set_params.argtypes = [vp, vp]
    lib.lpa_predictor_set_params.restype = ctypes.c_int
    lib.lpa_predictor_get_params.argtypes = [vp, vp]
    lib.lpa_predictor_get_params.restype = ctypes.c_int
    lib.lpa_predictor_save.argtypes = [vp, vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.lpa_predictor_save.restype = ctypes.c_int
    lib.lpa_predictor_load.argtypes = [vp, vp, ctypes.c_int64]
    lib.lpa_predictor_load.restype = ctypes.c_int
    lib.lpa_predictor_gradient.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_float, vp,
                                           ctypes.POINTER(ctypes.c_double)]
    lib.lpa_predictor_gradient.restype = ctypes.c_int
    lib.lpa_predictor_adam.argtypes = [vp, vp, ctypes.c_float]
    lib.lpa_predictor_adam.restype = ctypes.c_int
    lib.lpa_predictor_train.argtypes = [vp, vp, vp, ctypes.c_int64,
                                        ctypes.POINTER(lpa_train_options), fp]
    lib.lpa_predictor_train.restype = ctypes.c_int
    lib.lpa_predictor_predict.argtypes = [vp, vp, ctypes.c_int64, vp]
    lib.lpa_predictor_predict.restype = ctypes.c_int
    lib.lpa_learned_options_default.argtypes = [ctypes.POINTER(lpa_learned_options)]
    lib.lpa_learned_options_default.restype = None
    lib.lpa_set_predictor.argtypes = [vp, vp, ctypes.POINTER(lpa_learned_options)]
    lib.lpa_set_predictor.restype = ctypes.c_int
    lib.lpa_learned_history.argtypes = [vp, ctypes.POINTER(lpa_learned_iter), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32)]
    lib.lpa_learned_history.restype = ctypes.c_int
    lib.lpa_get_records.argtypes = [vp, vp]
    lib.lpa_get_records.restype = ctypes.c_int
    lib.lpa_trace.argtypes = [vp, ctypes.POINTER(lpa_options), ctypes.c_double, ctypes.c_uint64,
                              vp, vp, vp, vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.lpa_trace.restype = ctypes.c_int
    lib.lpa_autotune.argtypes = [ctypes.POINTER(lpa_csr), ctypes.c_int32, vp, vp,
                                 ctypes.POINTER(lpa_options), ctypes.c_double,
                                 ctypes.POINTER(lpa_tuning), ctypes.POINTER(lpa_tune_report)]
    lib.lpa_autotune.restype = ctypes.c_int
    lib.lpa_status_string.argtypes = [ctypes.c_int]
    lib.lpa_status_string.restype = ctypes.c_char_p
    lib.lpa_last_error.argtypes = []
    lib.lpa_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int):
    if status != LPA_OK:
        lib = load_library()
        raise LpaError(status, f"{lib.lpa_status_string(status).decode()}: "
                               f"{lib.lpa_last_error().decode()}")


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _addr(x):
    """Data address of a torch tensor or numpy array (None stays None)."""
    if x is None:
        return None
    if _is_torch(x):
        return ctypes.c_void_p(x.data_ptr())
    return x.ctypes.data_as(ctypes.c_void_p)


def _current_stream(device_arrays: bool):
    if not device_arrays:
        return None
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_tuning() -> lpa_tuning:
    t = lpa_tuning()
    load_library().lpa_tuning_default(ctypes.byref(t))
    return t


def default_options() -> lpa_options:
    o = lpa_options()
    load_library().lpa_options_default(ctypes.byref(o))
    return o


# ---- thin wrappers with the C names ---------------------------------------------

def _csr_struct(offsets, targets, weights, validate):
    on_dev = _is_torch(offsets) and offsets.is_cuda
    if on_dev:
        import torch
        assert offsets.dtype in (torch.int32, torch.int64) and targets.dtype == torch.int32
        assert weights is None or weights.dtype == torch.float32
        for t in (offsets, targets, weights):
            assert t is None or t.is_contiguous()
        off_t = INDEX_I64 if offsets.dtype == torch.int64 else INDEX_I32
    else:
        offsets = np.ascontiguousarray(offsets)
        targets = np.ascontiguousarray(targets, dtype=np.int32)
        if weights is not None:
            weights = np.ascontiguousarray(weights, dtype=np.float32)
        assert offsets.dtype in (np.int32, np.int64)
        off_t = INDEX_I64 if offsets.dtype == np.int64 else INDEX_I32
    g = lpa_csr()
    g.num_vertices = int(offsets.shape[0]) - 1
    g.num_edges = int(targets.shape[0])
    g.offset_type = off_t
    g.on_device = int(on_dev)
    g.offsets = _addr(offsets)
    g.targets = _addr(targets)
    g.weights = _addr(weights)
    g.validate = int(validate)
    return g, on_dev, (offsets, targets, weights)


def lpa_create(offsets, targets, weights=None, *, validate: bool = True,
               tuning: lpa_tuning | None = None, stream=None):
    """Create a graph handle.  torch CUDA tensors are borrowed (keep them alive);
    numpy arrays are copied to the device.  Returns an opaque handle."""
    lib = load_library()
    g, on_dev, _keep = _csr_struct(offsets, targets, weights, validate)
    h = ctypes.c_void_p()
    s = stream if stream is not None else _current_stream(on_dev)
    _check(lib.lpa_create(ctypes.byref(g), s, ctypes.byref(tuning) if tuning else None,
                          ctypes.byref(h)))
    return h


def lpa_create_batched(v_off, offsets, targets, weights=None, *, validate: bool = True,
                       tuning: lpa_tuning | None = None, stream=None):
    """Handle over graphs packed in one CSR; v_off (host, G + 1 int64) gives
    each graph's vertex range."""
    lib = load_library()
    vo = np.ascontiguousarray(v_off, dtype=np.int64)
    g, on_dev, _keep = _csr_struct(offsets, targets, weights, validate)
    h = ctypes.c_void_p()
    s = stream if stream is not None else _current_stream(on_dev)
    _check(lib.lpa_create_batched(int(vo.shape[0] - 1), _addr(vo), ctypes.byref(g), s,
                                  ctypes.byref(tuning) if tuning else None, ctypes.byref(h)))
    return h


def _options(mode, tolerance, max_iterations, pl_period, prune, initial_labels, profile,
             flag_mode, launch, learned=False, cc_period=0):
    o = default_options()
    o.learned = int(bool(learned))
    o.cc_period = int(cc_period)
    o.mode = int(mode)
    o.tolerance = float(tolerance)
    o.max_iterations = int(max_iterations)
    o.pl_period = int(pl_period)
    o.prune = int(bool(prune))
    o.initial_labels = _addr(initial_labels)
    o.profile = int(bool(profile))
    o.flag_mode = int(flag_mode)
    o.launch = int(launch)
    return o


def lpa_run_batched(handle, labels, num_graphs: int, *, mode: int = MODE_ASYNC,
                    tolerance: float = 0.05, max_iterations: int = 20, pl_period: int = 4,
                    prune: bool = True, initial_labels=None, flag_mode: int = FLAGS_AUTO,
                    launch: int = LAUNCH_GRAPH):
    """Returns (batch iterations, per-graph iterations, per-graph changed in
    the last iteration)."""
    lib = load_library()
    o = _options(mode, tolerance, max_iterations, pl_period, prune, initial_labels, False,
                 flag_mode, launch)
    iters = np.zeros(num_graphs, dtype=np.int32)
    last = np.zeros(num_graphs, dtype=np.int64)
    it = ctypes.c_int32(0)
    _check(lib.lpa_run_batched(handle, ctypes.byref(o), _addr(labels), _addr(iters),
                               _addr(last), ctypes.byref(it)))
    return int(it.value), iters, last


def lpa_run(handle, labels, *, mode: int = MODE_ASYNC, tolerance: float = 0.05,
            max_iterations: int = 20, pl_period: int = 4, prune: bool = True,
            initial_labels=None, profile: bool = False, flag_mode: int = FLAGS_AUTO,
            launch: int = LAUNCH_EAGER, learned: bool = False, cc_period: int = 0):
    """Run to termination; labels is a preallocated int32 torch tensor or numpy
    array of N entries.  Returns (iterations, list of stats dicts)."""
    lib = load_library()
    o = _options(mode, tolerance, max_iterations, pl_period, prune, initial_labels, profile,
                 flag_mode, launch, learned, cc_period)
    cap = max(int(max_iterations), 1)
    st = (lpa_iter_stats * cap)()
    it = ctypes.c_int32(0)
    _check(lib.lpa_run(handle, ctypes.byref(o), _addr(labels), st, cap, ctypes.byref(it)))
    stats = [dict(iteration=s.iteration, pick_less=s.pick_less, changed=s.changed,
                  processed=s.processed, edges_scanned=s.edges_scanned, ms=s.ms,
                  skipped=s.skipped)
             for s in st[:it.value]]
    return int(it.value), stats


def learned_options(threshold: float = 0.1, fn_bound: float = 0.02,
                    guard_period: int = 4, predict_small: bool = False,
                    predict_large: bool = False,
                    first_predicted: int = 2) -> lpa_learned_options:
    o = lpa_learned_options()
    load_library().lpa_learned_options_default(ctypes.byref(o))
    o.threshold, o.fn_bound, o.guard_period = threshold, fn_bound, guard_period
    o.predict_small = int(bool(predict_small))
    o.predict_large = int(bool(predict_large))
    o.first_predicted = int(first_predicted)
    return o


def lpa_set_predictor(handle, predictor, *, threshold: float = 0.1, fn_bound: float = 0.02,
                      guard_period: int = 4, predict_small: bool = False,
                      predict_large: bool = False, first_predicted: int = 2) -> None:
    o = learned_options(threshold, fn_bound, guard_period, predict_small, predict_large,
                        first_predicted)
    ph = None if predictor is None else predictor.handle
    _check(load_library().lpa_set_predictor(handle, ph, ctypes.byref(o)))


def lpa_learned_history(handle, cap: int = 64) -> list:
    arr = (lpa_learned_iter * cap)()
    cnt = ctypes.c_int32(0)
    _check(load_library().lpa_learned_history(handle, arr, cap, ctypes.byref(cnt)))
    return [{f: getattr(r, f) for f, _ in lpa_learned_iter._fields_ if f != "reserved"}
            for r in arr[:cnt.value]]


def lpa_get_records(handle, n: int) -> np.ndarray:
    out = np.empty((n, 8), dtype=np.uint8)
    _check(load_library().lpa_get_records(handle, _addr(out)))
    return out


def lpa_trace(handle, *, sample_rate: float, seed: int = 0, cap: int = 1 << 20,
              mode: int = MODE_DETERMINISTIC, tolerance: float = 0.05,
              max_iterations: int = 20, pl_period: int = 4, prune: bool = True,
              learned: bool = False, device=None):
    """Training trace of one run (see lpa_trace in the header).  With device
    (a torch device) the buffers are torch tensors there, else numpy arrays.
    Returns (X, y, vertex, iteration, drawn) cut to the samples kept."""
    lib = load_library()
    o = _options(mode, tolerance, max_iterations, pl_period, prune, None, False, FLAGS_AUTO,
                 LAUNCH_EAGER, learned)
    if device is not None:
        import torch
        X = torch.empty((cap, 12), dtype=torch.float32, device=device)
        y = torch.empty(cap, dtype=torch.float32, device=device)
        v = torch.empty(cap, dtype=torch.int32, device=device)
        it = torch.empty(cap, dtype=torch.int32, device=device)
    else:
        X = np.empty((cap, 12), dtype=np.float32)
        y = np.empty(cap, dtype=np.float32)
        v = np.empty(cap, dtype=np.int32)
        it = np.empty(cap, dtype=np.int32)
    cnt = ctypes.c_int64(0)
    _check(lib.lpa_trace(handle, ctypes.byref(o), float(sample_rate),
                         int(seed) & 0xFFFFFFFFFFFFFFFF, _addr(X), _addr(y), _addr(v),
                         _addr(it), int(cap), ctypes.byref(cnt)))
    k = min(int(cnt.value), cap)
    return X[:k], y[:k], v[:k], it[:k], int(cnt.value)


def lpa_autotune(offsets, targets, weights=None, *, v_off=None, mode: int = MODE_ASYNC,
                 budget_ms: float = 60_000.0, launch: int = LAUNCH_GRAPH, stream=None):
    """Search lpa_tuning for this graph (or packed batch with v_off).
    Returns (tuning, report dict)."""
    lib = load_library()
    g, on_dev, _keep = _csr_struct(offsets, targets, weights, True)
    o = _options(mode, 0.05, 20, 4, True, None, False, FLAGS_AUTO, launch)
    best = lpa_tuning()
    rep = lpa_tune_report()
    vo = None if v_off is None else np.ascontiguousarray(v_off, dtype=np.int64)
    ng = 0 if vo is None else int(vo.shape[0] - 1)
    s = stream if stream is not None else _current_stream(on_dev)
    _check(lib.lpa_autotune(ctypes.byref(g), ng, _addr(vo), s, ctypes.byref(o),
                            float(budget_ms), ctypes.byref(best), ctypes.byref(rep)))
    return best, {f: getattr(rep, f) for f, _ in lpa_tune_report._fields_ if f != "reserved"}


MODULARITY_NOALLOC_MAX_VERTICES = 4194304


def lpa_modularity_noalloc(handle, labels) -> float:
    q = ctypes.c_double(0.0)
    _check(load_library().lpa_modularity_noalloc(handle, _addr(labels), ctypes.byref(q)))
    return q.value


def lpa_modularity(handle, labels) -> float:
    q = ctypes.c_double(0.0)
    _check(load_library().lpa_modularity(handle, _addr(labels), ctypes.byref(q)))
    return float(q.value)


def lpa_label_read_rate(handle, reps: int = 3) -> float:
    """CSR entries per second of a pass that only reads each entry's target
    and neighbour label (the sweeps' memory-side ceiling)."""
    r = ctypes.c_double(0.0)
    _check(load_library().lpa_label_read_rate(handle, int(reps), ctypes.byref(r)))
    return float(r.value)


def lpa_graph_classes(handle) -> dict:
    c = (ctypes.c_int64 * 6)()
    _check(load_library().lpa_graph_classes(handle, c))
    return dict(zip(CLASS_NAMES, list(c)))


def lpa_profile(handle) -> list:
    """Accumulated per-kernel records of the runs made with profile=True."""
    lib = load_library()
    cap = 32
    arr = (lpa_kernel_profile * cap)()
    cnt = ctypes.c_int32(0)
    _check(lib.lpa_profile(handle, arr, cap, ctypes.byref(cnt)))
    return [dict(name=r.name.decode(), launches=r.launches, total_ms=r.total_ms,
                 bytes=r.bytes, edges=r.edges, vertices=r.vertices)
            for r in arr[:min(cnt.value, cap)]]


def lpa_profile_reset(handle) -> None:
    _check(load_library().lpa_profile_reset(handle))


def lpa_get_flags(handle, out) -> None:
    _check(load_library().lpa_get_flags(handle, _addr(out)))


def lpa_destroy(handle) -> None:
    if handle:
        load_library().lpa_destroy(handle)


# ---- convenience wrapper -----------------------------------------------------------

@dataclass
class RunResult:
    labels: object          # torch.int32 tensor (device) or numpy array (host)
    iterations: int
    stats: list

    @property
    def gpu_ms(self) -> float:
        return float(sum(s["ms"] for s in self.stats))


class LpaGraph:
    """Owns an lpa_graph handle (and keeps borrowed device arrays alive)."""

    def __init__(self, offsets, targets, weights=None, *, validate: bool = True,
                 tuning: lpa_tuning | None = None):
        self._keep = (offsets, targets, weights)
        self.on_device = _is_torch(offsets) and offsets.is_cuda
        self.num_vertices = int(offsets.shape[0]) - 1
        self.num_edges = int(targets.shape[0])
        self.handle = lpa_create(offsets, targets, weights, validate=validate, tuning=tuning)

    def run(self, mode: str | int = "async", out=None, **kw) -> RunResult:
        """lpa_run; keyword options as lpa_run (launch=LAUNCH_GRAPH replays a
        captured iteration)."""
        m = {"async": MODE_ASYNC, "det": MODE_DETERMINISTIC,
             "deterministic": MODE_DETERMINISTIC}.get(mode, mode)
        if out is None:
            if self.on_device:
                import torch
                out = torch.empty(self.num_vertices, dtype=torch.int32,
                                  device=self._keep[0].device)
            else:
                out = np.empty(self.num_vertices, dtype=np.int32)
        iters, stats = lpa_run(self.handle, out, mode=m, **kw)
        return RunResult(out, iters, stats)

    def modularity(self, labels) -> float:
        return lpa_modularity(self.handle, labels)

    def set_predictor(self, predictor, **kw) -> None:
        """Attach a Predictor (None detaches) for runs with learned=True."""
        lpa_set_predictor(self.handle, predictor, **kw)
        self._pred = predictor     # keep it alive while attached

    def learned_history(self) -> list:
        return lpa_learned_history(self.handle)

    def records(self) -> np.ndarray:
        return lpa_get_records(self.handle, self.num_vertices)

    def trace(self, **kw):
        return lpa_trace(self.handle, **kw)

    def classes(self) -> dict:
        return lpa_graph_classes(self.handle)

    def label_read_rate(self, reps: int = 3) -> float:
        return lpa_label_read_rate(self.handle, reps)

    def profile(self) -> list:
        return lpa_profile(self.handle)

    def profile_reset(self) -> None:
        lpa_profile_reset(self.handle)

    def flags(self) -> np.ndarray:
        out = np.empty(self.num_vertices, dtype=np.uint8)
        lpa_get_flags(self.handle, out)
        return out

    def close(self):
        if getattr(self, "handle", None):
            lpa_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class BatchResult:
    labels: object
    iterations: int            # iterations of the batch (the longest graph)
    iters_per_graph: np.ndarray
    changed_last: np.ndarray


class LpaBatch(LpaGraph):
    """Many graphs packed in one CSR (see lpa_create_batched)."""

    def __init__(self, v_off, offsets, targets, weights=None, *, validate: bool = True,
                 tuning: lpa_tuning | None = None):
        self._keep = (offsets, targets, weights)
        self.on_device = _is_torch(offsets) and offsets.is_cuda
        self.num_vertices = int(offsets.shape[0]) - 1
        self.num_edges = int(targets.shape[0])
        self.v_off = np.ascontiguousarray(v_off, dtype=np.int64)
        self.num_graphs = int(self.v_off.shape[0] - 1)
        self.handle = lpa_create_batched(self.v_off, offsets, targets, weights,
                                         validate=validate, tuning=tuning)

    def run_batched(self, mode: str | int = "async", out=None, **kw) -> BatchResult:
        m = {"async": MODE_ASYNC, "det": MODE_DETERMINISTIC,
             "deterministic": MODE_DETERMINISTIC}.get(mode, mode)
        if out is None:
            if self.on_device:
                import torch
                out = torch.empty(self.num_vertices, dtype=torch.int32,
                                  device=self._keep[0].device)
            else:
                out = np.empty(self.num_vertices, dtype=np.int32)
        it, per, last = lpa_run_batched(self.handle, out, self.num_graphs, mode=m, **kw)
        return BatchResult(out, it, per, last)


PREDICTOR_PARAMS = 5057
PREDICTOR_FEATURES = 12


def _f32(x):
    """fp32 contiguous view: torch tensors stay where they are, the rest
    becomes a numpy array."""
    if _is_torch(x):
        import torch
        return x.detach().to(torch.float32).contiguous()
    return np.ascontiguousarray(x, dtype=np.float32)


class Predictor:
    """Owns an lpa_predictor handle (the change-predictor network)."""

    def __init__(self, seed: int = 0, params=None, device_stream: bool = True):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.lpa_predictor_create(seed, _current_stream(device_stream), ctypes.byref(h)))
        self.handle = h
        if params is not None:
            self.set_params(params)

    def set_params(self, params) -> None:
        p = np.ascontiguousarray(params, dtype=np.float32).ravel()
        if p.shape[0] != PREDICTOR_PARAMS:
            raise ValueError(f"expected {PREDICTOR_PARAMS} parameters")
        _check(load_library().lpa_predictor_set_params(self.handle, _addr(p)))

    def params(self) -> np.ndarray:
        out = np.empty(PREDICTOR_PARAMS, dtype=np.float32)
        _check(load_library().lpa_predictor_get_params(self.handle, _addr(out)))
        return out

    def save_blob(self) -> bytes:
        """Checkpoint (lpa_predictor_save): shape, parameters, Adam state."""
        lib = load_library()
        size = ctypes.c_int64(0)
        _check(lib.lpa_predictor_save(self.handle, None, 0, ctypes.byref(size)))
        buf = (ctypes.c_uint8 * size.value)()
        _check(lib.lpa_predictor_save(self.handle, buf, size.value, ctypes.byref(size)))
        return bytes(buf)

    def load_blob(self, blob: bytes) -> None:
        """Resume from a checkpoint (lpa_predictor_load)."""
        buf = (ctypes.c_uint8 * len(blob)).from_buffer_copy(blob)
        _check(load_library().lpa_predictor_load(self.handle, buf, len(blob)))

    def gradient(self, X, y, pos_weight: float = 1.0):
        X, y = _f32(X), _f32(y)
        g = np.empty(PREDICTOR_PARAMS, dtype=np.float32)
        loss = ctypes.c_double()
        _check(load_library().lpa_predictor_gradient(self.handle, _addr(X), _addr(y),
                                                     int(y.shape[0]), pos_weight, _addr(g),
                                                     ctypes.byref(loss)))
        return g, loss.value

    def adam(self, grad=None, lr: float = 1e-3) -> None:
        g = None if grad is None else np.ascontiguousarray(grad, dtype=np.float32)
        _check(load_library().lpa_predictor_adam(self.handle, _addr(g), lr))

    def train(self, X, y, *, epochs: int = 1, batch: int = 1024, lr: float = 1e-3,
              pos_weight: float = 1.0, seed: int = 0) -> float:
        X, y = _f32(X), _f32(y)
        o = lpa_train_options(epochs=epochs, batch=batch, lr=lr, pos_weight=pos_weight,
                              seed=seed)
        loss = ctypes.c_float()
        _check(load_library().lpa_predictor_train(self.handle, _addr(X), _addr(y),
                                                  int(y.shape[0]), ctypes.byref(o),
                                                  ctypes.byref(loss)))
        return loss.value

    def predict(self, X, out=None):
        X = _f32(X)
        n = int(X.shape[0])
        if out is None:
            if _is_torch(X) and X.is_cuda:
                import torch
                out = torch.empty(n, dtype=torch.float32, device=X.device)
            else:
                out = np.empty(n, dtype=np.float32)
        _check(load_library().lpa_predictor_predict(self.handle, _addr(X), n, _addr(out)))
        return out

    def close(self):
        if getattr(self, "handle", None):
            load_library().lpa_predictor_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
