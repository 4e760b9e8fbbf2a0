"""Seeded synthetic inputs (graphs, initial forests, update batches).

Thin ctypes wrapper over ``gen.c``.  Nothing here computes any part of the
spanning-forest update: it draws random numbers, builds edge sets, converts
them to CSR, runs a breadth-first search for the initial forest and samples
update batches.  The CPU oracle and the GPU path both take these outputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB_PATH = os.path.join(_HERE, "libdrsfgen.so")
_lib = None

# purposes for seed derivation
P_GRAPH, P_FOREST, P_INSERT, P_DELETE, P_STREAM = 1, 2, 3, 4, 5


def build(force: bool = True) -> str:
    """Compile the generator library in-tree with gcc."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unused-function", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    u64, i64, i32, vp, dbl = (ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32,
                              ctypes.c_void_p, ctypes.c_double)
    lib.drsfgen_seed.restype = u64
    lib.drsfgen_seed.argtypes = [u64, u64, u64]
    lib.drsfgen_splitmix64.restype = u64
    lib.drsfgen_splitmix64.argtypes = [u64]
    lib.drsfgen_gnm.restype = i64
    lib.drsfgen_gnm.argtypes = [i32, i64, u64, vp]
    lib.drsfgen_rmat.restype = i64
    lib.drsfgen_rmat.argtypes = [ctypes.c_int, i64, dbl, dbl, dbl, u64, vp]
    lib.drsfgen_grid.restype = i64
    lib.drsfgen_grid.argtypes = [i32, i32, i64, u64, vp]
    lib.drsfgen_keys_to_csr.restype = None
    lib.drsfgen_keys_to_csr.argtypes = [i32, vp, i64, vp, vp]
    lib.drsfgen_bfs_forest.restype = None
    lib.drsfgen_bfs_forest.argtypes = [i32, vp, vp, vp]
    lib.drsfgen_insert_batches.restype = i64
    lib.drsfgen_insert_batches.argtypes = [i32, vp, i64, i64, i64, u64, vp]
    lib.drsfgen_delete_batches.restype = i64
    lib.drsfgen_delete_batches.argtypes = [i32, vp, i64, vp, i64, i64, i64, u64, vp]
    lib.drsfgen_uniform.restype = None
    lib.drsfgen_uniform.argtypes = [u64, i64, vp]
    lib.drsfgen_below.restype = None
    lib.drsfgen_below.argtypes = [u64, i64, u64, vp]
    lib.drsfgen_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


def seed(config_id: int, instance: int, purpose: int) -> int:
    return int(_load().drsfgen_seed(config_id, instance, purpose))


def splitmix64(x: int) -> int:
    return int(_load().drsfgen_splitmix64(x & (2**64 - 1)))


def uniform(s: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    _load().drsfgen_uniform(s, count, _p(out))
    return out


def below(s: int, count: int, bound: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _load().drsfgen_below(s, count, bound, _p(out))
    return out


def gnm(n: int, m: int, s: int) -> np.ndarray:
    keys = np.empty(max(m, 1), dtype=np.uint64)
    got = _load().drsfgen_gnm(n, m, s, _p(keys))
    if got < 0:
        raise ValueError(f"G(n={n}, m={m}) infeasible")
    return keys[:got]


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, s: int) -> np.ndarray:
    samples = edge_factor << scale
    keys = np.empty(samples, dtype=np.uint64)
    got = _load().drsfgen_rmat(scale, samples, a, b, c, s, _p(keys))
    if got < 0:
        raise ValueError("bad R-MAT parameters")
    return keys[:got].copy()


def grid(rows: int, cols: int, n_remove: int, s: int) -> np.ndarray:
    total = rows * (cols - 1) + (rows - 1) * cols
    keys = np.empty(total, dtype=np.uint64)
    got = _load().drsfgen_grid(rows, cols, n_remove, s, _p(keys))
    if got < 0:
        raise ValueError("bad grid parameters")
    return keys[:got].copy()


def keys_to_csr(n: int, keys: np.ndarray):
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    row_ptr = np.empty(n + 1, dtype=np.int64)
    col = np.empty(max(2 * len(keys), 1), dtype=np.int32)
    _load().drsfgen_keys_to_csr(n, _p(keys), len(keys), _p(row_ptr), _p(col))
    return row_ptr, col[: 2 * len(keys)]


def bfs_forest(n: int, row_ptr: np.ndarray, col: np.ndarray) -> np.ndarray:
    parent = np.empty(n, dtype=np.int32)
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    _load().drsfgen_bfs_forest(n, _p(row_ptr), _p(col), _p(parent))
    return parent


def insert_batches(n: int, keys: np.ndarray, nb: int, b: int, s: int) -> np.ndarray:
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.empty((nb, b, 2), dtype=np.int32)
    if nb * b and _load().drsfgen_insert_batches(n, _p(keys), len(keys), nb, b, s, _p(out)) < 0:
        raise ValueError("not enough non-edges")
    return out


def delete_batches(n: int, keys: np.ndarray, parent: np.ndarray, nb: int, b: int,
                   n_tree: int, s: int) -> np.ndarray:
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    out = np.empty((nb, b, 2), dtype=np.int32)
    if nb * b and _load().drsfgen_delete_batches(n, _p(keys), len(keys), _p(parent), nb, b,
                                                 n_tree, s, _p(out)) < 0:
        raise ValueError("not enough edges to delete")
    return out


@dataclass
class Graph:
    """An undirected simple graph with its canonical initial forest."""
    name: str
    n: int
    keys: np.ndarray              # sorted unique uint64 keys (u << 32 | v, u < v)
    row_ptr: np.ndarray           # int64[n + 1], symmetric CSR
    col: np.ndarray               # int32[2m], ascending rows
    parent: np.ndarray            # int32[n], BFS forest, roots point to themselves
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return len(self.keys)


def make_graph(name: str, n: int, keys: np.ndarray, **meta) -> Graph:
    row_ptr, col = keys_to_csr(n, keys)
    parent = bfs_forest(n, row_ptr, col)
    return Graph(name, n, keys, row_ptr, col, parent, dict(meta))


def keys_of_edges(edges: np.ndarray) -> np.ndarray:
    """Normalised uint64 keys of an int32 [..., 2] pair array."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    lo = np.minimum(e[:, 0], e[:, 1]).astype(np.uint64)
    hi = np.maximum(e[:, 0], e[:, 1]).astype(np.uint64)
    return (lo << np.uint64(32)) | hi


# ---- several independent graphs in one vertex space ---------------------------

@dataclass
class MultiGraph:
    """Independent graphs side by side: graph g owns global vertex ids
    n_off[g] .. n_off[g + 1] - 1.  ``graphs`` hold the local (0-based) views."""
    n_off: np.ndarray             # int32[G + 1]
    graphs: list                  # [Graph] with local ids
    row_ptr: np.ndarray           # int64[N + 1], symmetric CSR over global ids
    col: np.ndarray               # int32[2 sum m]
    parent: np.ndarray            # int32[N], global ids

    @property
    def G(self) -> int:
        return len(self.graphs)

    @property
    def n(self) -> int:
        return int(self.n_off[-1])


def shift_keys(keys: np.ndarray, off: int) -> np.ndarray:
    k = np.asarray(keys, dtype=np.uint64)
    o = np.uint64(off)
    return (((k >> np.uint64(32)) + o) << np.uint64(32)) | ((k & np.uint64(0xffffffff)) + o)


def multi_graph(graphs: list) -> MultiGraph:
    """Concatenate local graphs into one global CSR and forest."""
    ns = [g.n for g in graphs]
    n_off = np.zeros(len(graphs) + 1, dtype=np.int64)
    n_off[1:] = np.cumsum(ns)
    if n_off[-1] >= 2**31:
        raise ValueError("more than 2^31 - 1 vertices in total")
    keys = np.concatenate([shift_keys(g.keys, int(o)) for g, o in zip(graphs, n_off)]
                          + [np.zeros(0, np.uint64)])
    row_ptr, col = keys_to_csr(int(n_off[-1]), keys)
    parent = np.concatenate([g.parent.astype(np.int64) + o for g, o in zip(graphs, n_off)]
                            + [np.zeros(0, np.int64)]).astype(np.int32)
    return MultiGraph(n_off.astype(np.int32), list(graphs), row_ptr, col, parent)


def batched_sizes(G: int, s: int, log_n=(3.0, 6.0), log_b=(1.0, 4.0)):
    """Per-graph recipe of the batched workload: n_g = round(10^U(log_n)),
    m_g = 4 n_g, op_g ~ Bernoulli(1/2) (1 = delete), b_g = round(10^U(log_b))."""
    u = uniform(s, 3 * G).reshape(3, G)
    ns = np.rint(10.0 ** (log_n[0] + (log_n[1] - log_n[0]) * u[0])).astype(np.int64)
    ops = (u[1] < 0.5).astype(np.int8)
    bs = np.rint(10.0 ** (log_b[0] + (log_b[1] - log_b[0]) * u[2])).astype(np.int64)
    return ns, 4 * ns, ops, bs


def multi_step_batches(graph_state: list, ops, bs, s: int):
    """One batch per graph in local ids: inserts of uniform non-edges, deletes
    of half tree and half non-tree edges (capped by what the graph has).
    graph_state[g] = (n, keys, parent).  Returns (list of int32[b_g, 2], ops)."""
    out, ops_out = [], []
    for g, (n, keys, parent) in enumerate(graph_state):
        op, b = int(ops[g]), int(bs[g])
        sg = splitmix64(s ^ (g * 0x9E3779B97F4A7C15))
        if op == 1:
            trees = int((np.asarray(parent) != np.arange(n)).sum())
            nontree = len(keys) - trees
            b = min(b, len(keys))
            nt = min(b // 2, trees)
            nn = min(b - nt, nontree)
            nt = min(b - nn, trees)
            batch = delete_batches(n, keys, parent, 1, nt + nn, nt, sg)[0] if nt + nn else \
                np.zeros((0, 2), np.int32)
        else:
            free = n * (n - 1) // 2 - len(keys)
            b = min(b, free // 2)  # rejection sampling stays fast
            batch = insert_batches(n, keys, 1, b, sg)[0] if b else np.zeros((0, 2), np.int32)
        out.append(batch)
        ops_out.append(op)
    return out, np.array(ops_out, np.int8)


@dataclass
class BatchedWorkload:
    """Several graphs side by side with a batch per graph per step (global ids).
    steps[s] = (edges int32[b, 2], b_off int64[G + 1], ops int8[G])."""
    mg: MultiGraph
    steps: list
    b: np.ndarray                 # int64[G] batch size per graph


def batched_workload(G: int, nsteps: int, s: int, log_n=(3.0, 6.0), log_b=(1.0, 4.0)):
    """The batched workload: G independent G(n_g, 4 n_g) graphs with n_g =
    round(10^U(log_n)), canonical BFS forests, and per step one batch per
    graph: op ~ Bernoulli(1/2) per graph and step, size b_g = round(10^U(log_b))
    per graph.  All batches are drawn from the initial state: inserts are
    non-edges distinct across steps, deletes are initial edges distinct across
    steps with half of each batch initial tree edges (they stay tree edges
    until deleted, since an update keeps every surviving forest edge), so
    every batch stays valid in sequence.  b_g is capped so that all of a
    graph's delete steps fit."""
    ns, ms, _, bs = batched_sizes(G, s, log_n, log_b)
    ops = (uniform(splitmix64(s ^ 0x5151), G * nsteps).reshape(nsteps, G) < 0.5).astype(np.int8)
    graphs = []
    for g in range(G):
        n, m = int(ns[g]), int(ms[g])
        m = min(m, n * (n - 1) // 4)
        keys = gnm(n, m, splitmix64(s + 1 + g)) if m > 0 else np.zeros(0, np.uint64)
        graphs.append(make_graph(f"g{g}", n, keys))
    mg = multi_graph(graphs)
    per_graph = []
    b_eff = np.zeros(G, np.int64)
    for g, gr in enumerate(graphs):
        nd = int((ops[:, g] == 1).sum())
        ni = nsteps - nd
        trees = int((gr.parent != np.arange(gr.n)).sum())
        nontree = gr.m - trees
        b = int(bs[g])
        if nd:
            b = min(b, 2 * (trees // nd), 2 * (nontree // nd) + 1)
        free = gr.n * (gr.n - 1) // 2 - gr.m
        if ni:
            b = min(b, free // (2 * ni))
        b = max(b, 0)
        b_eff[g] = b
        seed_g = splitmix64(s ^ (0xC4 << 40) ^ g)
        dels = delete_batches(gr.n, gr.keys, gr.parent, nd, b, b // 2, seed_g) if nd and b else None
        inss = insert_batches(gr.n, gr.keys, ni, b, seed_g ^ 1) if ni and b else None
        per_graph.append((dels, inss))
    steps = []
    used = [[0, 0] for _ in range(G)]
    for st in range(nsteps):
        parts, b_off = [], [0]
        for g in range(G):
            dels, inss = per_graph[g]
            o = int(mg.n_off[g])
            if ops[st, g] == 1:
                bt = dels[used[g][0]] if dels is not None else np.zeros((0, 2), np.int32)
                used[g][0] += 1
            else:
                bt = inss[used[g][1]] if inss is not None else np.zeros((0, 2), np.int32)
                used[g][1] += 1
            parts.append(bt.astype(np.int32) + o)
            b_off.append(b_off[-1] + len(bt))
        steps.append((np.concatenate(parts).astype(np.int32), np.array(b_off, np.int64),
                      ops[st].copy()))
    return BatchedWorkload(mg, steps, b_eff)


def served_workload(scale, ntenants, nreq, instance=0):
    """Serving workload: a resident R-MAT graph plus tenants G(n_t, 4 n_t),
    n_t = round(10^U(5,6)), arriving staggered over the stream and leaving
    after their last request.  Requests: target uniform over the graphs live
    at the request's (unit-rate) arrival time, op ~ Bernoulli(1/2), size
    round(10^U(2,5)).  Each graph's requests are filled in arrival order:
    inserts take uniform non-edges of the initial graph, distinct across the
    stream; deletes take initial edges (half tree, half non-tree edges,
    interleaved), and once those run out, edges inserted by the graph's
    earlier requests, oldest first.  So every request is valid in any
    interleaving of graphs that keeps each graph's arrival order; a request
    left empty is dropped.  Arrival gaps are unit-mean exponentials, scaled
    per offered load.  Instance 0 is the benchmark's workload; other
    instances draw everything from other seeds."""
    cfg = 5 if instance == 0 else 500 + int(instance)
    keys = rmat(scale, 16, 0.57, 0.19, 0.19, seed(cfg, 0, P_GRAPH))
    graphs = [make_graph(f"rmat{scale}", 1 << scale, keys)]
    u = uniform(seed(cfg, 1, P_GRAPH), ntenants)
    for t in range(ntenants):
        n = int(round(10 ** (5 + u[t])))
        graphs.append(make_graph(f"t{t}", n, gnm(n, 4 * n, seed(cfg, 2 + t, P_GRAPH))))
    r = uniform(seed(cfg, 0, P_STREAM), 4 * nreq).reshape(4, nreq)
    gaps = -np.log1p(-r[0])                  # unit-mean exponential gaps
    t_arr = np.cumsum(gaps)
    span = t_arr[-1]
    # tenant k is live on [k, k + 4) eighths of the stream (staggered, finite)
    win = [(0.0, np.inf)] + [(span * t / (ntenants + 4), span * (t + 4) / (ntenants + 4))
                             for t in range(ntenants)]
    pools = []
    sizes = np.rint(10 ** (2 + 3 * r[2])).astype(np.int64)
    ops = (r[3] < 0.5).astype(np.int64)
    live_idx = [[g for g, (a, b) in enumerate(win) if a <= t < b] for t in t_arr]
    demand = np.zeros((len(graphs), 2), np.int64)
    target = np.zeros(nreq, np.int64)
    for k in range(nreq):
        lv = live_idx[k]
        target[k] = lv[min(int(r[1][k] * len(lv)), len(lv) - 1)]
        demand[target[k], ops[k]] += sizes[k]
    for g, gr in enumerate(graphs):
        ni = int(min(demand[g, 0], gr.n * (gr.n - 1) // 2 - gr.m))
        nd = int(min(demand[g, 1], gr.m))
        trees = int((gr.parent != np.arange(gr.n)).sum())
        nt = min(trees, nd // 2)
        nn = min(nd - nt, gr.m - trees)
        nt = min(trees, nd - nn)
        ins = insert_batches(gr.n, gr.keys, 1, ni, seed(cfg, g, P_INSERT))[0] if ni else \
            np.zeros((0, 2), np.int32)
        dl = delete_batches(gr.n, gr.keys, gr.parent, 1, nt + nn, nt,
                            seed(cfg, g, P_DELETE))[0] if nt + nn else np.zeros((0, 2), np.int32)
        # tree and non-tree edges interleaved so every request mixes both
        dl = dl[np.argsort(uniform(seed(cfg, g, P_STREAM), len(dl)), kind="stable")]
        pools.append([ins, 0, dl, 0, []])  # [inserts, next, initial deletes, next, inserted runs alive]
    reqs = []
    for k in range(nreq):
        g, op, b = int(target[k]), int(ops[k]), int(sizes[k])
        pool = pools[g]
        if op == 0:
            e = pool[0][pool[1]:pool[1] + b]
            pool[1] += len(e)
            if len(e):
                pool[4].append(e)
        else:
            e = pool[2][pool[3]:pool[3] + b]
            pool[3] += len(e)
            parts = [e]
            need = b - len(e)
            while need > 0 and pool[4]:  # edges inserted by earlier requests of this graph
                run = pool[4][0]
                take, rest = run[:need], run[need:]
                parts.append(take)
                need -= len(take)
                if len(rest):
                    pool[4][0] = rest
                else:
                    pool[4].pop(0)
            e = np.concatenate(parts) if len(parts) > 1 else e
        if len(e) == 0:
            continue
        reqs.append((g, np.ascontiguousarray(e, np.int32), op, float(t_arr[k])))
    last = {}
    for i, (g, _, _, _) in enumerate(reqs):
        last[g] = i
    return graphs, reqs, win, last
