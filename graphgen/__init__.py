"""Seeded synthetic graph inputs shared by the tests, the oracle and the bench.

Holds no part of the label-propagation method: it only produces symmetric
CSR graphs (rows sorted, no self-loops, no duplicates) and edge weights.  All
randomness is Philox4x32-10 addressed by counters, so outputs are identical
for any thread count.  The native part is ``graphgen.cpp`` (g++ + OpenMP).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


class _GG(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64),
                ("off", ctypes.POINTER(ctypes.c_int64)),
                ("tgt", ctypes.POINTER(ctypes.c_int32))]


def build(force: bool = True) -> str:
    """Compile libgraphgen.so next to its source (g++ -O3 -fopenmp)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC",
                               "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        lib.gg_philox4x32_10.argtypes = [vp, vp, vp]
        lib.gg_sbm.argtypes = [ctypes.c_int64, ctypes.c_int32, vp, vp,
                               ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                               ctypes.POINTER(_GG)]
        lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                ctypes.POINTER(_GG)]
        lib.gg_free.argtypes = [ctypes.POINTER(_GG)]
        lib.gg_copy_out.argtypes = [ctypes.POINTER(_GG), vp, vp, vp]
        lib.gg_pair_weights.argtypes = [ctypes.c_int64, vp, vp, ctypes.c_uint64,
                                        ctypes.c_int32, vp]
        lib.gg_fill_f32.argtypes = [ctypes.c_int64, ctypes.c_float, vp]
        lib.gg_lfr.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, vp, ctypes.POINTER(_GG)]
        lib.gg_sbm_batch.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                     ctypes.c_int32, vp, ctypes.POINTER(_GG)]
        lib.gg_lattice.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                   ctypes.c_uint64, ctypes.POINTER(_GG)]
        lib.gg_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


@dataclass
class Graph:
    """Symmetric CSR on the host: offsets (N+1), targets (M), weights (M or None)."""
    offsets: np.ndarray
    targets: np.ndarray
    weights: np.ndarray | None
    name: str = ""

    @property
    def num_vertices(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def num_edges(self) -> int:
        return int(self.targets.shape[0])

    def degrees(self) -> np.ndarray:
        o = self.offsets.astype(np.int64)
        return o[1:] - o[:-1]


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().gg_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def _take(gg: _GG, offset_dtype) -> tuple[np.ndarray, np.ndarray]:
    lib = _load()
    n, m = int(gg.n), int(gg.m)
    tgt = np.empty(m, dtype=np.int32)
    if offset_dtype == np.int32:
        if m > np.iinfo(np.int32).max:
            lib.gg_free(ctypes.byref(gg))
            raise ValueError("edge count exceeds int32 offsets")
        off = np.empty(n + 1, dtype=np.int32)
        rc = lib.gg_copy_out(ctypes.byref(gg), None, _ptr(off), _ptr(tgt))
    else:
        off = np.empty(n + 1, dtype=np.int64)
        rc = lib.gg_copy_out(ctypes.byref(gg), _ptr(off), None, _ptr(tgt))
    lib.gg_free(ctypes.byref(gg))
    if rc != 0:
        raise RuntimeError("gg_copy_out failed")
    return off, tgt


def sbm(block_sizes, p_in, p_out: float, seed: int, graph_id: int = 0,
        offset_dtype=np.int32) -> tuple[np.ndarray, np.ndarray]:
    """Planted partition with consecutive blocks; p_in scalar or per block."""
    bs = np.ascontiguousarray(block_sizes, dtype=np.int64)
    pin = np.broadcast_to(np.asarray(p_in, dtype=np.float64), bs.shape).copy()
    gg = _GG()
    rc = _load().gg_sbm(int(bs.sum()), int(bs.shape[0]), _ptr(bs), _ptr(pin),
                        float(p_out), int(seed), int(graph_id), ctypes.byref(gg))
    if rc != 0:
        raise RuntimeError(f"gg_sbm failed ({rc})")
    return _take(gg, offset_dtype)


def rmat(scale: int, edge_factor: int = 16, a=0.57, b=0.19, c=0.19, seed=0,
         offset_dtype=np.int32) -> tuple[np.ndarray, np.ndarray]:
    gg = _GG()
    rc = _load().gg_rmat(int(scale), int(edge_factor), float(a), float(b),
                         float(c), int(seed), ctypes.byref(gg))
    if rc != 0:
        raise RuntimeError(f"gg_rmat failed ({rc})")
    return _take(gg, offset_dtype)


def pair_weights(offsets: np.ndarray, targets: np.ndarray, seed: int,
                 wmax: int = 8) -> np.ndarray:
    """Symmetric integer weights 1..wmax hashed from the unordered pair."""
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    w = np.empty(targets.shape[0], dtype=np.float32)
    _load().gg_pair_weights(off.shape[0] - 1, _ptr(off),
                            _ptr(np.ascontiguousarray(targets)), int(seed),
                            int(wmax), _ptr(w))
    return w


def unit_weights(m: int) -> np.ndarray:
    w = np.empty(m, dtype=np.float32)
    _load().gg_fill_f32(int(m), 1.0, _ptr(w))
    return w


# ---- the named workloads ----------------------------------------------------

def planted_partition_10k(seed: int = 1) -> Graph:
    """10,000 vertices in 100 blocks of 100; expected 16 intra-block and 4
    inter-block neighbours per vertex (p_in = 16/99, p_out = 4/9900); unit
    weights; int32 offsets."""
    off, tgt = sbm(np.full(100, 100), 16.0 / 99.0, 4.0 / 9900.0, seed)
    return Graph(off, tgt, unit_weights(tgt.shape[0]), "sbm10k")


def rmat_graph(scale: int, seed: int, weights: str = "int8",
               offset_dtype=None) -> Graph:
    """R-MAT (a,b,c,d = 0.57,0.19,0.19,0.05), edge factor 16, symmetrised.
    weights: "int8" = integers 1..8 hashed per pair, "unit" = 1.0."""
    if offset_dtype is None:
        offset_dtype = np.int32 if scale <= 24 else np.int64
    off, tgt = rmat(scale, 16, 0.57, 0.19, 0.19, seed, offset_dtype)
    if weights == "int8":
        w = pair_weights(off, tgt, seed, 8)
    elif weights == "unit":
        w = unit_weights(tgt.shape[0])
    else:
        raise ValueError(weights)
    return Graph(off, tgt, w, f"rmat{scale}")


def random_graph(n: int, p: float, seed: int, wmax: int = 0) -> Graph:
    """Erdos-Renyi G(n, p) (one block), weights 1..wmax (0 = unit)."""
    off, tgt = sbm(np.array([n]), p, 0.0, seed)
    w = pair_weights(off, tgt, seed, wmax) if wmax > 0 else unit_weights(tgt.shape[0])
    return Graph(off, tgt, w, f"gnp{n}")


def from_edges(n: int, edges, weights=None, offset_dtype=np.int32) -> Graph:
    """Small hand-made symmetric graph from an undirected edge list [(u, v)];
    weights, if given, is a parallel list of floats (the same for both
    directions).  Duplicate edges add up as separate CSR entries; self-loops
    are kept (one CSR entry)."""
    rows = [[] for _ in range(n)]
    for k, (u, v) in enumerate(edges):
        wt = 1.0 if weights is None else float(weights[k])
        rows[u].append((v, wt))
        if u != v:
            rows[v].append((u, wt))
    off = np.zeros(n + 1, dtype=offset_dtype)
    tg, wt = [], []
    for i in range(n):
        r = sorted(rows[i])
        off[i + 1] = off[i] + len(r)
        tg += [x[0] for x in r]
        wt += [x[1] for x in r]
    return Graph(off, np.array(tg, dtype=np.int32), np.array(wt, dtype=np.float32))


def ring_of_cliques(r: int, s: int) -> Graph:
    """r cliques K_s; clique k holds vertices k*s .. k*s+s-1; one edge joins the
    last vertex of clique k to the first vertex of clique k+1 (cyclically)."""
    edges = []
    for k in range(r):
        b = k * s
        edges += [(b + x, b + y) for x in range(s) for y in range(x + 1, s)]
        edges.append((b + s - 1, ((k + 1) % r) * s))
    return from_edges(r * s, edges)


def disjoint_cliques(r: int, s: int) -> Graph:
    edges = []
    for k in range(r):
        b = k * s
        edges += [(b + x, b + y) for x in range(s) for y in range(x + 1, s)]
    return from_edges(r * s, edges)


def complete_bipartite(n: int) -> Graph:
    return from_edges(2 * n, [(x, n + y) for x in range(n) for y in range(n)])


def planted_partition_batch(num_graphs: int, seed: int, n_range=(256, 65536),
                            d_range=(8.0, 32.0), mu_range=(0.1, 0.4),
                            block_range=(32, 256)) -> tuple[Graph, np.ndarray]:
    """num_graphs planted-partition graphs packed into one CSR (int64
    offsets, global target ids, unit weights) and their vertex offsets
    v_off (num_graphs + 1).  Per graph: vertex count log-uniform in n_range,
    expected degree uniform in d_range, mixing uniform in mu_range, block
    sizes uniform in block_range."""
    v_off = np.zeros(num_graphs + 1, dtype=np.int64)
    gg = _GG()
    rc = _load().gg_sbm_batch(int(num_graphs), int(seed), float(n_range[0]), float(n_range[1]),
                              float(d_range[0]), float(d_range[1]), float(mu_range[0]),
                              float(mu_range[1]), int(block_range[0]), int(block_range[1]),
                              _ptr(v_off), ctypes.byref(gg))
    if rc != 0:
        raise RuntimeError(f"gg_sbm_batch failed ({rc})")
    off, tgt = _take(gg, np.int64)
    return Graph(off, tgt, unit_weights(tgt.shape[0]), f"batch{num_graphs}"), v_off


def lattice(rows: int, cols: int, keep: float, seed: int, offset_dtype=np.int32):
    """Road-like lattice: grid vertices r*cols + c, each right and down lattice
    edge kept with probability keep (mean degree 4*keep)."""
    gg = _GG()
    rc = _load().gg_lattice(int(rows), int(cols), float(keep), int(seed), ctypes.byref(gg))
    if rc != 0:
        raise RuntimeError(f"gg_lattice failed ({rc})")
    return _take(gg, offset_dtype)


def lowdeg_graph(side: int, seed: int, keep: float = 0.525, offset_dtype=None) -> Graph:
    """Low-degree road-like workload: a side x side lattice with each edge kept
    with probability 0.525 (mean degree 2.1, as the road and k-mer graphs of
    the paper's Table 1), row-major ids, unit weights."""
    if offset_dtype is None:
        offset_dtype = np.int32 if 4 * side * side < 2 ** 31 else np.int64
    off, tgt = lattice(side, side, keep, seed, offset_dtype)
    return Graph(off, tgt, unit_weights(tgt.shape[0]), f"lattice{side}")


def lfr_graph(n: int, seed: int, mu: float | None = None, tau1: float = 2.5,
              mean_deg: float = 20.0, kmax: float = 1000.0, tau2: float = 2.0,
              cmin: float = 20.0, cmax: float = 5000.0) -> tuple[Graph, np.ndarray]:
    """LFR-like graph (power-law degrees and community sizes, mixing mu) with
    unit weights and int32 offsets; also returns the planted communities.
    mu defaults to a draw from U[0.1, 0.5] keyed by the seed."""
    if mu is None:
        x = philox4x32_10([seed & 0xFFFFFFFF, 0, 0, 0x4D55], [7, 7])
        mu = 0.1 + 0.4 * (int(x[0]) / 2.0 ** 32)
    comm = np.empty(n, dtype=np.int32)
    gg = _GG()
    rc = _load().gg_lfr(int(n), int(seed), float(tau1), float(mean_deg), float(kmax),
                        float(tau2), float(cmin), float(cmax), float(mu), _ptr(comm),
                        ctypes.byref(gg))
    if rc != 0:
        raise RuntimeError(f"gg_lfr failed ({rc})")
    off, tgt = _take(gg, np.int32)
    g = Graph(off, tgt, unit_weights(tgt.shape[0]), f"lfr{n}")
    g.mu = mu
    return g, comm


def pack_graphs(graphs) -> tuple[Graph, np.ndarray]:
    """Concatenate graphs into one CSR with global target ids (int64
    offsets); returns the packed graph and v_off."""
    v_off = np.zeros(len(graphs) + 1, dtype=np.int64)
    offs, tgts, ws = [np.zeros(1, dtype=np.int64)], [], []
    e0 = 0
    for q, g in enumerate(graphs):
        v_off[q + 1] = v_off[q] + g.num_vertices
        o = g.offsets.astype(np.int64)
        offs.append(o[1:] + e0)
        tgts.append(g.targets.astype(np.int64) + v_off[q])
        ws.append(g.weights if g.weights is not None else np.ones(g.num_edges, np.float32))
        e0 += g.num_edges
    tgt = np.concatenate(tgts).astype(np.int32) if tgts else np.zeros(0, np.int32)
    w = np.concatenate(ws).astype(np.float32) if ws else np.zeros(0, np.float32)
    return Graph(np.concatenate(offs), tgt, w, "packed"), v_off


def max_threads() -> int:
    return int(_load().gg_max_threads())


__all__ = ["Graph", "build", "sbm", "rmat", "pair_weights", "unit_weights",
           "planted_partition_10k", "rmat_graph", "random_graph", "from_edges",
           "ring_of_cliques", "disjoint_cliques", "complete_bipartite",
           "philox4x32_10", "max_threads", "planted_partition_batch", "pack_graphs",
           "lfr_graph"]
