"""Paths longer than one thread's walk (drsf_opts.walk_limit, path reversal
Alg. 1 with the vertex-disjoint paths of Lemma 4): the walks leave such a
path untouched and the host turns it by pointer doubling.  Chains (a path
graph, whose breadth-first forest is the chain itself, depth L - 1) give
both kinds of long path:

* closing each chain into a ring and cutting it a quarter of the way down
  re-attaches the far part through the closing edge, from its far end up to
  its old root (about 3L/4 steps);
* cutting the closing edge then leaves the far part as a tree of its own,
  rooted at its far end, which is re-rooted at its smallest vertex, the far
  part's other end (the re-root path of the super-root piece);
* closing the ring again attaches the far part from its far end.

Every update is compared with the oracle element by element (parent,
label, checker, replacement-edge count), and the view reports that the host
finished it with the pass (host_finished bit 2) exactly when a path was
longer than the limit."""
from __future__ import annotations

import numpy as np
import pytest

import gen
from test_gpu_parity import Pair, _case, _lib

pytestmark = pytest.mark.gpu


def _chains(G, L):
    keys = [((c * L + i) << 32) | (c * L + i + 1) for c in range(G) for i in range(L - 1)]
    return gen.make_graph(f"chains{G}x{L}", G * L, np.array(keys, np.uint64))


def _pairs(G, L, f):
    return np.array([f(c * L) for c in range(G)], np.int32)


def _run(pair, G, L, expect_pass):
    drsf = _lib()
    q = L // 4
    steps = [
        ("close the rings", drsf.DRSF_INSERT, _pairs(G, L, lambda o: (o, o + L - 1)), False),
        ("cut a quarter down", drsf.DRSF_DELETE, _pairs(G, L, lambda o: (o + q, o + q + 1)), True),
        ("cut the closing edges", drsf.DRSF_DELETE, _pairs(G, L, lambda o: (o, o + L - 1)), True),
        ("close the rings again", drsf.DRSF_INSERT, _pairs(G, L, lambda o: (o + L - 1, o)), True),
    ]
    for what, op, batch, long in steps:
        st, _ = pair.step(batch, op, what)
        assert bool(st["host_finished"] & 4) == (long and expect_pass), (what, st)


@pytest.mark.parametrize("device,launch_mode", [(False, 0), (True, 0), (True, 1)])
def test_long_attach_and_reroot_paths(device, launch_mode):
    G, L = 4, 1 << 14
    g = _chains(G, L)
    _case(f"long paths: {G} chains of {L}, device inputs {device}, launch mode {launch_mode}")
    pair = Pair(g, device=device, max_batch=64, launch_mode=launch_mode)
    _run(pair, G, L, True)
    pair.gpu.close()


def test_a_path_of_exactly_the_limit_is_walked():
    """The far part's attach path has L - 2 - L/4 steps: walked by one thread
    at that limit, turned by the pass at one step less (both bit-exact)."""
    G, L = 2, 1 << 12
    hops = L - 2 - L // 4
    drsf = _lib()
    for limit, passed in ((hops, False), (hops - 1, True)):
        g = _chains(G, L)
        _case(f"walk limit {limit} for a path of {hops} steps")
        pair = Pair(g, max_batch=8, walk_limit=limit)
        pair.step(_pairs(G, L, lambda o: (o, o + L - 1)), drsf.DRSF_INSERT, "close")
        st, _ = pair.step(_pairs(G, L, lambda o: (o + L // 4, o + L // 4 + 1)), drsf.DRSF_DELETE, "cut")
        assert bool(st["host_finished"] & 4) == passed, (limit, st)
        pair.gpu.close()


def test_one_chain_over_a_million_vertices():
    """One path of about 7.9e5 steps (one thread would take it in dependent
    reads), then the pass again on the same context (its marks from the
    first pass must not count)."""
    G, L = 1, 1 << 20
    g = _chains(G, L)
    _case(f"long paths: one chain of {L}")
    pair = Pair(g, device=True, max_batch=8)
    _run(pair, G, L, True)
    pair.gpu.close()


def test_every_path_of_more_than_one_step_takes_the_pass():
    """walk_limit 1 on R-MAT and grid workloads: every path longer than one
    step goes through the pass, beside the walked ones, over alternating
    insert and delete batches (multi-graph contexts draw walk limits in the
    randomized tests)."""
    drsf = _lib()
    rng = np.random.default_rng(515)
    cases = [gen.make_graph("rmat14", 1 << 14, gen.rmat(14, 8, 0.57, 0.19, 0.19, 77)),
             gen.make_graph("grid", 64 * 64, gen.grid(64, 64, 1500, 78))]
    for g in cases:
        for launch_mode in (0, 1):
            _case(f"walk limit 1: {g.name} n={g.n}, launch mode {launch_mode}")
            pair = Pair(g, device=True, max_batch=2000, walk_limit=1, launch_mode=launch_mode)
            passes = 0
            for step in range(6):
                ins = gen.insert_batches(g.n, pair.keys, 1, 1500, int(rng.integers(1 << 30)))[0]
                st, _ = pair.step(ins, drsf.DRSF_INSERT, f"{g.name} insert {step}")
                passes += bool(st["host_finished"] & 4)
                trees = int((pair.parent != np.arange(g.n)).sum())
                dl = gen.delete_batches(g.n, pair.keys, pair.parent, 1, 1500, min(trees, 900),
                                        int(rng.integers(1 << 30)))[0]
                st, _ = pair.step(dl, drsf.DRSF_DELETE, f"{g.name} delete {step}")
                passes += bool(st["host_finished"] & 4)
            assert passes >= 6, f"{g.name}: only {passes} of 12 updates had a path of two steps or more"
            pair.gpu.close()


def test_create_reroots_a_long_chain():
    """A forest handed over rooted at the wrong end of a chain: create
    re-roots every tree at its smallest vertex, a path of L - 1 steps per
    chain, through the pass."""
    import dataclasses
    G, L = 3, 1 << 13
    g = _chains(G, L)
    par = np.array([v + 1 if (v % L) != L - 1 else v for v in range(G * L)], np.int32)
    g = dataclasses.replace(g, parent=par)
    _case(f"create re-roots {G} chains of {L}")
    for device in (False, True):
        pair = Pair(g, device=device, max_batch=8)  # compares with the oracle's canonical forest
        pair.gpu.close()


def _chain_steps(L):
    """Updates on one chain of L vertices whose chases are long: close the
    ring, cut it a quarter down, cut the closing edge, close it again,
    restore the cut edge, cut it halfway."""
    drsf = _lib()
    q = L // 4
    return [("close the ring", drsf.DRSF_INSERT, [(0, L - 1)]),
            ("cut a quarter down", drsf.DRSF_DELETE, [(q, q + 1)]),
            ("cut the closing edge", drsf.DRSF_DELETE, [(0, L - 1)]),
            ("close the ring again", drsf.DRSF_INSERT, [(L - 1, 0)]),
            ("restore the cut", drsf.DRSF_INSERT, [(q, q + 1)]),
            ("cut halfway", drsf.DRSF_DELETE, [(L // 2, L // 2 + 1)])]


def test_deep_root_finding_queues_jumping_rounds():
    """Root finding on deep forests.  A chain 2^21 deep handed to create is
    found deeper than 2^16 there, so every delete runs pointer-jumping rounds
    before the chase (drsf_view.jump_rounds > 0).  Chains of 2^16 vertices
    (depth just below that bound) start without them; a chase of more than
    1024 steps would add them for later deletes.  Every update is
    bit-exact."""
    drsf = _lib()
    for L, first in ((1 << 21, True), (1 << 16, False)):
        g = _chains(2, L)
        _case(f"deep root finding: two chains of {L}")
        pair = Pair(g, device=True, max_batch=8)
        deletes = []
        for what, op, e in _chain_steps(L):
            e2 = np.array(e + [(u + L, v + L) for u, v in e], np.int32)  # the same on both chains
            st, _ = pair.step(e2, op, what)
            if op == drsf.DRSF_DELETE:
                deletes.append(st["jump_rounds"])
        assert (deletes[0] > 0) == first, (L, deletes)
        if first:
            assert all(j > 0 for j in deletes), deletes
        pair.gpu.close()


def test_deep_chains_queued_two_in_flight():
    """The same updates queued two deep (drsf_apply_async): the context
    switches to jumping rounds while an update is queued behind the one
    that found the forest deep; statuses and final arrays as the oracle's."""
    import torch
    import oracle
    drsf = _lib()
    dev = torch.device("cuda:0")
    L = 1 << 20
    g = _chains(1, L)
    steps = _chain_steps(L)
    r = oracle.apply(g.n, g.keys, g.parent, np.zeros((0, 2), np.int32), oracle.DELETE)
    keys, par, lab = g.keys, r.parent, r.label
    for _, op, e in steps:
        r = oracle.apply(g.n, keys, par, np.array(e, np.int32), oracle.INSERT if op == drsf.DRSF_INSERT
                         else oracle.DELETE, label=lab)
        keys, par, lab = r.keys, r.parent, r.label
    _case(f"deep chains queued: one chain of {L}")
    stream = torch.cuda.Stream(dev)
    with torch.cuda.stream(stream):
        t = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (g.row_ptr, g.col, g.parent)]
        dbat = [torch.tensor(e, dtype=torch.int32, device=dev) for _, _, e in steps]
    f = drsf.Forest(g.n, *t, inputs_on_device=True, stream=stream.cuda_stream, max_batch=8)
    got = []
    f.apply_async(dbat[0], steps[0][1])
    for j in range(1, len(steps)):
        f.apply_async(dbat[j], steps[j][1])
        got.append(f.wait())
    got.append(f.wait())  # each wait raises unless its update succeeded
    assert np.array_equal(f.label(), lab) and np.array_equal(f.parent(), par)
    assert got[-1]["jump_rounds"] > 0, got[-1]
    f.close()


def test_deep_chains_in_a_multi_graph_context():
    """Three chains of 2^19 side by side in one multi-graph context, deleted
    and re-inserted together: jumping rounds over the deleting graphs'
    vertex blocks; every graph bit-exact with the oracle run on it alone."""
    from test_gpu_multi import MultiPair
    drsf = _lib()
    L = 1 << 19
    graphs = [_chains(1, L) for _ in range(3)]
    _case(f"deep chains, multi-graph: 3 chains of {L}")
    pair = MultiPair(graphs, max_batch=32, launch_mode=0)
    for what, op, e in _chain_steps(L):
        pair.step([np.array(e, np.int32)] * 3, np.full(3, op, np.int8), what)
    pair.gpu.close()
