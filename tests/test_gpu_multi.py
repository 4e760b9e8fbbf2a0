"""Several graphs in one context (the batched pattern): every graph's parent
and label arrays after each multi-graph update are bit-exact with the oracle
run on that graph alone, in local ids."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2607_20211_amd import drsf
    return drsf


def _case(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


class MultiPair:
    """A MultiForest on the GPU and one oracle state per graph."""

    def __init__(self, graphs, **kw):
        drsf = _lib()
        self.mg = gen.multi_graph(graphs)
        self.gpu = drsf.MultiForest(self.mg.n_off, self.mg.row_ptr, self.mg.col, self.mg.parent, **kw)
        self.state = []
        for g in graphs:
            r = oracle.apply(g.n, g.keys, g.parent, np.zeros((0, 2), np.int32), oracle.DELETE)
            self.state.append([g.n, g.keys, r.parent, r.label])
        self.check("create")

    def check(self, what):
        p, lab = self.gpu.parent(), self.gpu.label()
        m = self.gpu.num_edges()
        for g, (n, keys, par, label) in enumerate(self.state):
            o = int(self.mg.n_off[g])
            gp, gl = p[o:o + n] - o, lab[o:o + n] - o
            assert np.array_equal(gl, label), f"{what}: graph {g} label mismatch"
            assert np.array_equal(gp, par), f"{what}: graph {g} parent mismatch"
            assert m[g] == len(keys), f"{what}: graph {g} edge count {m[g]} != {len(keys)}"

    def _spoil(self, g, bt, op, kind):
        """bt with one invalid entry of the given kind appended: "dup" a
        repeated pair, "exists" an insert of a present edge, "missing" a
        delete of an absent pair, "self" a self-loop, "range" an id outside
        the graph (local id n)."""
        n, keys = self.state[g][0], self.state[g][1]
        if kind == "dup":
            extra = bt[:1]
        elif kind == "exists":
            assert op == 0 and len(keys)
            k = int(keys[len(keys) // 2])
            extra = np.array([[k >> 32, k & 0xffffffff]])
        elif kind == "missing":
            assert op == 1
            have = set(int(k) for k in keys) | set((int(u) << 32) | int(v) for u, v in np.sort(bt, axis=1))
            extra = next(np.array([[u, v]]) for u in range(n) for v in range(u + 1, n) if (u << 32 | v) not in have)
        elif kind == "self":
            extra = np.array([[n - 1, n - 1]])
        else:
            extra = np.array([[0, n]])
        return np.concatenate([bt, extra.astype(np.int32)])

    def step(self, batches, ops, what, bad=()):
        """batches in local ids; graphs in `bad` get an invalid batch (a
        repeated pair, or the kind `bad` maps them to, see _spoil) and must
        come back rejected and unchanged."""
        drsf = _lib()
        kinds = bad if isinstance(bad, dict) else {g: "dup" for g in bad}
        glob = []
        b_off = [0]
        for g, bt in enumerate(batches):
            o = int(self.mg.n_off[g])
            bt = np.asarray(bt, np.int32).reshape(-1, 2)
            if g in kinds and (len(bt) or kinds[g] != "dup"):
                bt = self._spoil(g, bt, int(ops[g]), kinds[g])
            glob.append(bt + o)
            b_off.append(b_off[-1] + len(bt))
        edges = np.concatenate(glob) if glob else np.zeros((0, 2), np.int32)
        st = self.gpu.apply_multi(edges.astype(np.int32), np.array(b_off, np.int64), ops)
        for g, bt in enumerate(batches):
            if g in kinds and (len(bt) or kinds[g] != "dup"):
                assert st[g] == drsf.DRSF_E_BATCH, f"{what}: graph {g} not rejected ({kinds[g]})"
                continue
            assert st[g] == drsf.DRSF_OK, f"{what}: graph {g} status {st[g]}"
            n, keys, par, label = self.state[g]
            opc = oracle.INSERT if ops[g] == drsf.DRSF_INSERT else oracle.DELETE
            r = oracle.apply(n, keys, par, np.asarray(bt, np.int32).reshape(-1, 2), opc, label=label)
            self.state[g] = [n, r.keys, r.parent, r.label]
        self.check(what)

    def local_state(self):
        return [(n, keys, par) for n, keys, par, _ in self.state]


def _graphs(ns, seed):
    out = []
    for g, n in enumerate(ns):
        n = int(n)
        m = min(4 * n, n * (n - 1) // 2 // 2)
        keys = gen.gnm(n, m, gen.seed(40, seed * 1000 + g, gen.P_GRAPH)) if m > 0 else np.zeros(0, np.uint64)
        out.append(gen.make_graph(f"g{g}", n, keys))
    return out


@pytest.mark.parametrize("seed", range(2))
def test_multi_graph_parity(seed):
    """40 graphs of 1 to ~5000 vertices (log-uniform), mixed ops in every
    call, some graphs with empty batches, state carried over 4 calls."""
    drsf = _lib()
    _case(f"multi seed={seed}")
    ns, _, _, _ = gen.batched_sizes(40, gen.seed(41, seed, gen.P_GRAPH), log_n=(0.0, 3.7))
    ns[0], ns[1] = 1, 2
    graphs = _graphs(ns, seed)
    pair = MultiPair(graphs, max_batch=1 << 16)
    for step in range(4):
        _, _, ops, bs = gen.batched_sizes(40, gen.seed(41, seed * 16 + step, gen.P_STREAM),
                                          log_b=(0.0, 3.0))
        bs[step::7] = 0
        batches, ops = gen.multi_step_batches(pair.local_state(), ops, bs,
                                              gen.seed(41, seed * 16 + step, gen.P_INSERT))
        pair.step(batches, ops, f"multi {seed} step {step}")
    pair.gpu.close()


def test_multi_graph_rejects_one_graph_only():
    drsf = _lib()
    _case("multi invalid")
    graphs = _graphs([300, 500, 800, 1200], 7)
    pair = MultiPair(graphs, max_batch=4096)
    for step in range(3):
        ops = np.array([step % 2, 1 - step % 2, 0, 1], np.int8)
        bs = np.array([50, 80, 120, 200])
        batches, ops = gen.multi_step_batches(pair.local_state(), ops, bs, gen.seed(42, step, gen.P_INSERT))
        pair.step(batches, ops, f"multi invalid step {step}", bad={step})
    pair.gpu.close()


def test_multi_graph_same_as_single_contexts():
    """A graph updated inside a multi-graph context ends exactly as in its own
    single-graph context (same batches)."""
    drsf = _lib()
    _case("multi vs single")
    graphs = _graphs([2000, 3000, 700], 9)
    pair = MultiPair(graphs, max_batch=8192)
    singles = [drsf.Forest(g.n, g.row_ptr, g.col, g.parent, max_batch=8192) for g in graphs]
    for step in range(3):
        ops = np.array([step % 2, 0, 1], np.int8)
        batches, ops = gen.multi_step_batches(pair.local_state(), ops, np.array([600, 900, 300]),
                                              gen.seed(43, step, gen.P_INSERT))
        pair.step(batches, ops, f"multi vs single {step}")
        p, lab = pair.gpu.parent(), pair.gpu.label()
        for g, (f, bt) in enumerate(zip(singles, batches)):
            f.apply(bt, int(ops[g]))
            o = int(pair.mg.n_off[g])
            assert np.array_equal(f.parent(), p[o:o + graphs[g].n] - o)
            assert np.array_equal(f.label(), lab[o:o + graphs[g].n] - o)
    for f in singles:
        f.close()
    pair.gpu.close()


def test_multi_create_rejects_cross_graph_edge():
    drsf = _lib()
    _case("multi create errors")
    graphs = _graphs([50, 60], 11)
    mg = gen.multi_graph(graphs)
    # an edge from graph 0 into graph 1
    keys = np.concatenate([gen.shift_keys(graphs[0].keys, 0), gen.shift_keys(graphs[1].keys, 50),
                           np.array([(3 << 32) | 70], np.uint64)])
    keys.sort()
    row_ptr, col = gen.keys_to_csr(mg.n, keys)
    with pytest.raises(drsf.DrsfError) as ei:
        drsf.MultiForest(mg.n_off, row_ptr, col, mg.parent)
    assert ei.value.code == drsf.DRSF_E_ARG
    f = drsf.MultiForest(mg.n_off, mg.row_ptr, mg.col, mg.parent)
    with pytest.raises(drsf.DrsfError) as ei:
        f.apply(np.array([[0, 1]], np.int32), drsf.DRSF_INSERT)
    assert ei.value.code == drsf.DRSF_E_STATE
    # a pair whose ends lie in different graphs is an invalid batch of its graph
    st = f.apply_multi(np.array([[3, 70]], np.int32), np.array([0, 1, 1]), np.array([0, 0], np.int8))
    assert st[0] == drsf.DRSF_E_BATCH and st[1] == drsf.DRSF_OK
    f.close()


def test_multi_context_with_one_graph():
    """A multi-graph context holding a single graph (its block and tile
    lists are not allocated: every block and tile is in play): inserts and
    deletes through the multi-graph call, bit-exact with the oracle."""
    drsf = _lib()
    _case("multi with one graph")
    graphs = _graphs([3000], 7)
    pair = MultiPair(graphs, max_batch=2048)
    for step in range(3):
        (n, keys, par), = pair.local_state()
        ins = gen.insert_batches(n, keys, 1, 500, gen.seed(41, step, gen.P_INSERT))[0]
        pair.step([ins], np.array([drsf.DRSF_INSERT], np.int8), f"one graph insert {step}")
        (n, keys, par), = pair.local_state()
        trees = int((par != np.arange(n)).sum())
        dl = gen.delete_batches(n, keys, par, 1, 400, min(200, trees), gen.seed(41, step, gen.P_DELETE))[0]
        pair.step([dl], np.array([drsf.DRSF_DELETE], np.int8), f"one graph delete {step}")
    pair.step([np.zeros((0, 2), np.int32)], np.array([drsf.DRSF_INSERT], np.int8), "one graph, empty")
    pair.gpu.close()
