"""Pins for the CPU oracle against facts fixed by the paper and by mathematics.

- exhaustive comparison with the independent brute force (tests/brute.py)
  on every graph with 4 vertices and every batch of up to 3 edges, on every
  graph with 5 vertices and every single-edge batch, and on
  seeded random graphs with up to 7 vertices and arbitrary (not necessarily
  canonical) rooted spanning forests;
- the forest checker, including negative cases;
- Theorem 1 invariants (F-hat kept, k - l replacement edges, l roots) and
  textbook minimum-spanning-forest properties (cut and cycle properties);
- closed-form special cases;
- hand-derived golden fixtures under tests/golden/;
- whole-batch rejection of invalid batches.
"""
from __future__ import annotations

import glob
import itertools
import os
import random

import numpy as np
import pytest

import brute
import gen
import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def keys_np(edges) -> np.ndarray:
    ks = sorted({(min(u, v) << 32) | max(u, v) for u, v in edges})
    return np.array(ks, dtype=np.uint64)


def edges_of(keys: np.ndarray):
    return [(int(k >> np.uint64(32)), int(k & np.uint64(0xffffffff))) for k in keys]


def random_spanning_forest(n, edges, rng, canonical=False):
    """Random spanning forest (random-order Kruskal) with random roots."""
    order = list(edges)
    rng.shuffle(order)
    up = list(range(n))

    def find(x):
        while up[x] != x:
            x = up[x]
        return x
    chosen = []
    for u, v in order:
        a, b = find(u), find(v)
        if a != b:
            up[a] = b
            chosen.append((u, v))
    adj = [[] for _ in range(n)]
    for u, v in chosen:
        adj[u].append(v)
        adj[v].append(u)
    parent = [-1] * n
    comp = brute.components(n, chosen)
    for c in sorted(set(comp)):
        members = [v for v in range(n) if comp[v] == c]
        r = min(members) if canonical else rng.choice(members)
        parent[r] = r
        stack = [r]
        while stack:
            x = stack.pop()
            for w in adj[x]:
                if parent[w] < 0:
                    parent[w] = x
                    stack.append(w)
    return parent


def run_both(n, edges, parent, batch, op):
    opc = oracle.INSERT if op == "insert" else oracle.DELETE
    try:
        exp = brute.apply(n, edges, parent, batch, op)
    except brute.Rejected:
        with pytest.raises(oracle.OracleError) as ei:
            oracle.apply(n, keys_np(edges), np.array(parent, np.int32),
                         np.array(batch, np.int32).reshape(-1, 2), opc)
        assert ei.value.code == oracle.E_BATCH
        return None
    got = oracle.apply(n, keys_np(edges), np.array(parent, np.int32),
                       np.array(batch, np.int32).reshape(-1, 2), opc)
    E2, par, lab, repl = exp
    assert edges_of(got.keys) == sorted(E2)
    assert got.parent.tolist() == par, (n, edges, parent, batch, op)
    assert got.label.tolist() == lab
    assert got.stats["n_repl"] == len(repl)
    return got


def test_exhaustive_n4_against_brute_force():
    n = 4
    all_pairs = list(itertools.combinations(range(n), 2))
    rng = random.Random(7)
    cases = 0
    for mask in range(1 << len(all_pairs)):
        edges = [all_pairs[i] for i in range(len(all_pairs)) if mask >> i & 1]
        parent = random_spanning_forest(n, edges, rng)
        non_edges = [p for p in all_pairs if p not in edges]
        for size in (1, 2, 3):
            for batch in itertools.combinations(non_edges, size):
                run_both(n, edges, parent, list(batch), "insert")
                cases += 1
            for batch in itertools.combinations(edges, size):
                # random orientation of each pair exercises normalisation
                b = [(v, u) if rng.random() < 0.5 else (u, v) for u, v in batch]
                run_both(n, edges, parent, b, "delete")
                cases += 1
    assert cases > 1000


def test_exhaustive_n5_single_edge_batches():
    n = 5
    all_pairs = list(itertools.combinations(range(n), 2))
    rng = random.Random(11)
    cases = 0
    for mask in range(1 << len(all_pairs)):
        edges = [all_pairs[i] for i in range(len(all_pairs)) if mask >> i & 1]
        parent = random_spanning_forest(n, edges, rng)
        for e in all_pairs:
            run_both(n, edges, parent, [e], "delete" if e in edges else "insert")
            cases += 1
    assert cases == 1024 * 10


@pytest.mark.parametrize("seed", range(60))
def test_random_small_against_brute_force(seed):
    rng = random.Random(1000 + seed)
    n = rng.randint(2, 7)
    all_pairs = list(itertools.combinations(range(n), 2))
    p = rng.random()
    edges = [e for e in all_pairs if rng.random() < p]
    parent = random_spanning_forest(n, edges, rng)
    for _ in range(4):  # a short sequence of batches; state carries over
        op = rng.choice(["insert", "delete"])
        pool = [e for e in all_pairs if e not in edges] if op == "insert" else list(edges)
        if not pool:
            continue
        batch = rng.sample(pool, rng.randint(1, min(len(pool), 5)))
        got = run_both(n, edges, parent, batch, op)
        edges = edges_of(got.keys)
        parent = got.parent.tolist()


def test_golden_fixtures():
    files = sorted(glob.glob(os.path.join(GOLDEN, "*.txt")))
    assert len(files) >= 3
    for path in files:
        steps, n, edges, parent = [], None, [], None
        cur = None
        with open(path) as f:
            for line in f:
                line = line.strip()
                if not line or line.startswith("#"):
                    continue
                tag, _, rest = line.partition(" ")
                if tag == "n":
                    n = int(rest)
                elif tag == "edges":
                    edges = [tuple(map(int, p.split())) for p in rest.split(";") if p.strip()]
                elif tag == "parent":
                    parent = list(map(int, rest.split()))
                elif tag == "op":
                    cur = {"op": rest}
                    steps.append(cur)
                elif tag == "batch":
                    cur["batch"] = [tuple(map(int, p.split())) for p in rest.split(";")]
                elif tag == "expect_parent":
                    cur["parent"] = list(map(int, rest.split()))
                elif tag == "expect_label":
                    cur["label"] = list(map(int, rest.split()))
        keys = keys_np(edges)
        par = np.array(parent, np.int32)
        for st in steps:
            opc = oracle.INSERT if st["op"] == "insert" else oracle.DELETE
            r = oracle.apply(n, keys, par, np.array(st["batch"], np.int32), opc)
            assert r.parent.tolist() == st["parent"], path
            assert r.label.tolist() == st["label"], path
            keys, par = r.keys, r.parent


def _medium(seed, n=3000, m=2400):
    keys = gen.gnm(n, m, gen.seed(90, seed, gen.P_GRAPH))
    return gen.make_graph("medium", n, keys)


def _roots(parent):
    r = parent.copy()
    while True:
        nr = r[r]
        if np.array_equal(nr, r):
            return r
        r = nr


@pytest.mark.parametrize("seed", range(4))
def test_theorem1_invariants_and_msf_properties(seed):
    g = _medium(seed)
    lab = _roots(g.parent)
    ins = gen.insert_batches(g.n, g.keys, 1, 600, gen.seed(90, seed, gen.P_INSERT))[0]
    r1 = oracle.apply(g.n, g.keys, g.parent, ins, oracle.INSERT, label=lab)
    dl = gen.delete_batches(g.n, r1.keys, r1.parent, 1, 800, 400, gen.seed(90, seed, gen.P_DELETE))[0]
    r2 = oracle.apply(g.n, r1.keys, r1.parent, dl, oracle.DELETE, label=r1.label)
    for (keys0, par0, res, batch, op) in ((g.keys, g.parent, r1, ins, "insert"),
                                          (r1.keys, r1.parent, r2, dl, "delete")):
        assert oracle.check_forest(g.n, res.keys, res.parent, res.label)[0] == 0
        bset = set(gen.keys_of_edges(batch).tolist())
        tf = {(min(v, int(p)) << 32) | max(v, int(p)) for v, p in enumerate(par0) if p != v}
        that = tf - bset if op == "delete" else tf
        tnew = {(min(v, int(p)) << 32) | max(v, int(p)) for v, p in enumerate(res.parent) if p != v}
        assert that <= tnew                                   # F-hat is kept
        er = tnew - that
        st = res.stats
        assert len(er) == st["n_repl"] == st["k"] - st["ell"]  # Theorem 1
        assert st["ell"] == int((res.parent == np.arange(g.n)).sum())
        # labels = breadth-first components of G' (smallest vertex)
        comp = brute.components(g.n, edges_of(res.keys))
        assert res.label.tolist() == comp
        # cut property: each e in E_r is the lowest-key key edge across the
        # cut it closes in Kruskal order; cycle property: every rejected cross
        # key edge is the highest key on the cycle it closes in F'.
        up = list(range(g.n))

        def find(x):
            while up[x] != x:
                up[x] = up[up[x]]
                x = up[x]
            return x
        for k in that:
            a, b = find(k >> 32), find(k & 0xffffffff)
            up[a] = b
        keyset = sorted(bset) if op == "insert" else sorted(set(res.keys.tolist()) - that)
        for k in keyset:
            a, b = find(k >> 32), find(k & 0xffffffff)
            if a != b:
                assert k in er
                up[a] = b
            else:
                assert k not in er


def test_insert_scan_all_mode_agrees():
    for seed in range(3):
        g = _medium(seed)
        ins = gen.insert_batches(g.n, g.keys, 1, 900, gen.seed(91, seed, gen.P_INSERT))[0]
        a = oracle.apply(g.n, g.keys, g.parent, ins, oracle.INSERT)
        b = oracle.apply(g.n, g.keys, g.parent, ins, oracle.INSERT, scan_all=True)
        assert np.array_equal(a.parent, b.parent) and np.array_equal(a.label, b.label)


def test_special_cases():
    g = _medium(11)
    lab = _roots(g.parent)
    # (i) inserting edges that lie inside one tree leaves the forest unchanged
    rng = np.random.default_rng(3)
    inside = []
    seen = set(g.keys.tolist())
    while len(inside) < 50:
        u, v = rng.integers(0, g.n, 2)
        k = (int(min(u, v)) << 32) | int(max(u, v))
        if u != v and lab[u] == lab[v] and k not in seen:
            seen.add(k)
            inside.append((u, v))
    r = oracle.apply(g.n, g.keys, g.parent, np.array(inside, np.int32), oracle.INSERT)
    assert np.array_equal(r.parent, g.parent) and r.stats["n_repl"] == 0
    # (ii) deleting only non-tree edges leaves the forest unchanged
    gd = _medium(12, m=6000)
    dl = gen.delete_batches(gd.n, gd.keys, gd.parent, 1, 300, 0, gen.seed(92, 0, gen.P_DELETE))[0]
    r = oracle.apply(gd.n, gd.keys, gd.parent, dl, oracle.DELETE)
    assert np.array_equal(r.parent, gd.parent)
    # (iii) all singletons: E_r is Kruskal's minimum spanning forest of B by key
    n = 400
    single = np.arange(n, dtype=np.int32)
    bk = gen.gnm(n, 500, gen.seed(92, 1, gen.P_GRAPH))
    batch = np.array(edges_of(bk), np.int32)
    r = oracle.apply(n, np.zeros(0, np.uint64), single, batch, oracle.INSERT)
    up = list(range(n))

    def find(x):
        while up[x] != x:
            x = up[x]
        return x
    msf = set()
    for k in sorted(bk.tolist()):
        a, b = find(k >> 32), find(k & 0xffffffff)
        if a != b:
            up[a] = b
            msf.add(k)
    tnew = {(min(v, int(p)) << 32) | max(v, int(p)) for v, p in enumerate(r.parent) if p != v}
    assert tnew == msf
    # (iv) G is a forest and tree edges are deleted: no replacement edges and
    # every piece is rooted at its smallest vertex
    fk = keys_np([(v, int(p)) for v, p in enumerate(g.parent) if p != v])
    dl = gen.delete_batches(g.n, fk, g.parent, 1, 300, 300, gen.seed(92, 2, gen.P_DELETE))[0]
    r = oracle.apply(g.n, fk, g.parent, dl, oracle.DELETE)
    assert r.stats["n_repl"] == 0
    assert oracle.check_forest(g.n, r.keys, r.parent, r.label)[0] == 0
    # (vi) delete then re-insert the same batch restores the labels
    dl = gen.delete_batches(gd.n, gd.keys, gd.parent, 1, 400, 200, gen.seed(92, 3, gen.P_DELETE))[0]
    r1 = oracle.apply(gd.n, gd.keys, gd.parent, dl, oracle.DELETE)
    r2 = oracle.apply(gd.n, r1.keys, r1.parent, dl, oracle.INSERT)
    assert np.array_equal(r2.keys, gd.keys)
    assert np.array_equal(r2.label, _roots(gd.parent))


def test_invalid_batches_rejected_whole():
    g = _medium(5)
    e0 = edges_of(g.keys[:1])[0]
    nonedge = gen.insert_batches(g.n, g.keys, 1, 1, 1)[0][0].tolist()
    bad = {
        "self_loop": ([(3, 3)], oracle.INSERT),
        "out_of_range": ([(0, g.n)], oracle.INSERT),
        "negative": ([(-1, 2)], oracle.DELETE),
        "duplicate_insert": ([nonedge, nonedge[::-1]], oracle.INSERT),
        "insert_existing": ([e0], oracle.INSERT),
        "delete_missing": ([nonedge], oracle.DELETE),
        "duplicate_delete": ([e0, e0], oracle.DELETE),
    }
    for name, (batch, op) in bad.items():
        with pytest.raises(oracle.OracleError) as ei:
            oracle.apply(g.n, g.keys, g.parent, np.array(batch, np.int32), op)
        assert ei.value.code == oracle.E_BATCH, name
    # an empty batch is valid and changes nothing
    r = oracle.apply(g.n, g.keys, g.parent, np.zeros((0, 2), np.int32), oracle.DELETE)
    assert np.array_equal(r.parent, g.parent)


def test_checker_rejects_broken_forests():
    g = _medium(6)
    assert oracle.check_forest(g.n, g.keys, g.parent)[0] == 0
    lab = _roots(g.parent)
    assert oracle.check_forest(g.n, g.keys, g.parent, lab)[0] == 0
    nonroot = np.flatnonzero(g.parent != np.arange(g.n))
    v = int(nonroot[0])
    # parent edge not in the graph
    p = g.parent.copy()
    cand = [w for w in range(g.n) if w != v and ((min(v, w) << 32) | max(v, w)) not in set(g.keys.tolist())]
    p[v] = cand[0]
    assert oracle.check_forest(g.n, g.keys, p)[0] != 0
    # cut a tree edge: a graph edge now joins two trees
    p = g.parent.copy()
    p[v] = v
    assert oracle.check_forest(g.n, g.keys, p)[0] != 0
    # two-cycle
    p = g.parent.copy()
    u = int(p[v])
    p[u] = v
    assert oracle.check_forest(g.n, g.keys, p)[0] != 0
    # valid forest but a root that is not the smallest vertex
    r = oracle.apply(g.n, g.keys, g.parent, np.zeros((0, 2), np.int32), oracle.INSERT)
    comp_root = int(r.label[v])
    members = np.flatnonzero(r.label == comp_root)
    if len(members) >= 2:
        p = r.parent.copy()
        other = int(members[1])
        path = [other]
        while p[path[-1]] != path[-1]:
            path.append(int(p[path[-1]]))
        for a, b in zip(path[1:], path[:-1]):
            p[a] = b
        p[other] = other
        assert oracle.check_forest(g.n, g.keys, p, require_min_root=False)[0] == 0
        assert oracle.check_forest(g.n, g.keys, p, require_min_root=True)[0] != 0
    # wrong label
    lab2 = lab.copy()
    lab2[v] = (lab2[v] + 1) % g.n
    assert oracle.check_forest(g.n, g.keys, g.parent, lab2)[0] != 0
