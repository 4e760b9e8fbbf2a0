"""The small-graph engine of multi-graph contexts (drsf_opts.
small_graph_vertices): graphs up to that many vertices are updated whole by
one workgroup each (forest in LDS, taken from a device work queue) beside
the kernel sequence that updates the others.  Every graph bit-exact with
the oracle run on it alone after every call, for several thresholds and
workgroup sizes: mixed ops, empty and invalid batches (each kind, with the
batch's hash set in LDS and in HBM), deep trees, pools that grow, all graphs
small, snapshots and exports."""
from __future__ import annotations

import numpy as np
import pytest

import gen
from test_gpu_multi import MultiPair, _case, _graphs, _lib

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("T,threads", [(4096, 256), (700, 1024), (5000, 512)])
def test_small_graphs_parity(T, threads):
    drsf = _lib()
    _case(f"small T={T} threads={threads}")
    ns, _, _, _ = gen.batched_sizes(40, gen.seed(44, T, gen.P_GRAPH), log_n=(0.0, 3.8))
    ns[0], ns[1], ns[2] = 1, 2, 4096
    graphs = _graphs(ns, 3)
    pair = MultiPair(graphs, max_batch=1 << 16, small_graph_vertices=T, small_threads=threads)
    for step in range(5):
        _, _, ops, bs = gen.batched_sizes(40, gen.seed(44, T * 16 + step, gen.P_STREAM), log_b=(0.0, 3.3))
        bs[step::6] = 0
        batches, ops = gen.multi_step_batches(pair.local_state(), ops, bs,
                                              gen.seed(44, T * 16 + step, gen.P_INSERT))
        bad = {(3 * step + 5) % 40, (7 * step + 1) % 40}
        pair.step(batches, ops, f"small T={T} step {step}", bad=bad)
    keys = np.sort(np.concatenate([gen.shift_keys(k, int(pair.mg.n_off[g]))
                                   for g, (_, k, _) in enumerate(pair.local_state())]))
    assert np.array_equal(pair.gpu.edges(), keys)
    pair.gpu.close()


def test_small_graphs_all_small_and_schedules():
    """Every graph small (the chain has nothing to do), workgroup schedules
    changed between calls, snapshot and restore."""
    drsf = _lib()
    _case("all small")
    graphs = _graphs([300, 1200, 50, 2000, 999, 1], 5)
    pair = MultiPair(graphs, max_batch=1 << 14, small_graph_vertices=2048)
    snap = None
    for step, (threads, wgs) in enumerate([(0, 0), (256, 1), (1024, 3), (512, 0)]):
        pair.gpu.set_small_schedule(threads, wgs)
        ops = np.array([step % 2, 1 - step % 2, 0, 1, step % 2, 0], np.int8)
        batches, ops = gen.multi_step_batches(pair.local_state(), ops, np.array([90, 400, 20, 700, 300, 5]),
                                              gen.seed(45, step, gen.P_INSERT))
        pair.step(batches, ops, f"all small step {step}")
        if step == 1:
            snap = pair.gpu.snapshot()
            saved = [list(x) for x in pair.state]
    pair.gpu.restore(snap)
    drsf.drsf_snapshot_free(snap)
    pair.state = saved
    pair.check("restored")
    pair.gpu.close()


def test_small_graph_deep_trees_and_pool_growth():
    """Paths with chords as small graphs (deep trees: long pointer-jumping
    chains and reversal paths), tree-edge deletes, then inserts that
    outgrow the key buffers (the pool grows; a snapshot from before cannot
    be restored), beside a large graph in the chain."""
    drsf = _lib()
    _case("small deep")
    graphs = []
    for n, sd in ((4000, 1), (2500, 2)):
        path = np.array([(i << 32) | (i + 1) for i in range(n - 1)], np.uint64)
        graphs.append(gen.make_graph(f"path{n}", n, np.union1d(path, gen.gnm(n, n // 20, sd))))
    graphs.append(gen.make_graph("big", 60000, gen.gnm(60000, 200000, 9)))
    pair = MultiPair(graphs, max_batch=1 << 16, small_graph_vertices=4096)
    snap = pair.gpu.snapshot()
    for step in range(3):
        batches = []
        for n, keys, par in pair.local_state():
            trees = int((par != np.arange(n)).sum())
            b = min(300, len(keys))
            nt = max(min(250, trees), b - (len(keys) - trees))  # the rest must be non-tree edges
            batches.append(gen.delete_batches(n, keys, par, 1, b, nt, gen.seed(46, step * 8 + n, gen.P_DELETE))[0])
        pair.step(batches, np.array([1, 1, 1], np.int8), f"deep delete {step}")
    for step in range(4):  # 4 x 3000 inserts into a 4000-vertex graph holding ~4200 edges
        batches = [gen.insert_batches(n, keys, 1, 3000 if g < 2 else 5000, gen.seed(47, step * 8 + g, gen.P_INSERT))[0]
                   for g, (n, keys, par) in enumerate(pair.local_state())]
        pair.step(batches, np.array([0, 0, 0], np.int8), f"grow insert {step}")
    with pytest.raises(drsf.DrsfError) as e:
        pair.gpu.restore(snap)
    assert e.value.code == drsf.DRSF_E_STATE
    drsf.drsf_snapshot_free(snap)
    pair.gpu.close()


@pytest.mark.parametrize("T", [300, 4096])
def test_small_graph_rejections(T):
    """Each kind of invalid batch sent to small graphs, with batches small
    enough for the LDS hash set and too large for it (more than half the
    LDS words after the parents): the graph comes back rejected and
    unchanged, the others in the same call are applied."""
    drsf = _lib()
    _case(f"small rejections T={T}")
    ns = [T, T // 2, T, 3 * T // 4, 20000]
    graphs = _graphs(ns, 11)
    pair = MultiPair(graphs, max_batch=1 << 16, small_graph_vertices=T)
    lds_words = ((T + 1) & ~1) + T
    sizes = [5, lds_words // 2 + 7]  # hash set in LDS / in HBM
    plan = [("dup", 0), ("exists", 0), ("missing", 1), ("self", 0), ("range", 1), ("dup", 1), ("self", 1)]
    for step, (kind, op_bad) in enumerate(plan):
        for size in sizes:
            ops = np.array([op_bad, 1 - op_bad, op_bad, 0, step % 2], np.int8)
            bs = np.array([size, size // 3, size, 40, 300])
            batches, ops = gen.multi_step_batches(pair.local_state(), ops, bs,
                                                  gen.seed(48, step * 4 + size, gen.P_INSERT))
            bad = {0: kind, 2: kind} if len(batches[2]) else {0: kind}
            pair.step(batches, ops, f"rejection {kind} size {size}", bad=bad)
    pair.gpu.close()


@pytest.mark.parametrize("profile", [False, True])
def test_every_graph_small_runs_the_engine_alone(profile):
    """A context whose graphs are all small launches the engine, its commit
    and the cleanup only (no kernel sequence): inserts, deletes, an invalid
    batch, empty batches; bit-exact per graph; profiled, the engine's time
    is the replacement-edge phase and the sequence's phases read 0."""
    drsf = _lib()
    _case(f"engine alone profile={profile}")
    ns, _, _, _ = gen.batched_sizes(60, gen.seed(49, 0, gen.P_GRAPH), log_n=(0.5, 3.3))
    graphs = _graphs(ns, 12)
    pair = MultiPair(graphs, max_batch=1 << 16, small_graph_vertices=2048, profile=profile)
    for step in range(4):
        _, _, ops, bs = gen.batched_sizes(60, gen.seed(49, step + 1, gen.P_STREAM), log_b=(0.0, 2.7))
        bs[step::5] = 0
        batches, ops = gen.multi_step_batches(pair.local_state(), ops, bs, gen.seed(49, step, gen.P_INSERT))
        pair.step(batches, ops, f"engine alone step {step}", bad={(7 * step + 3) % 60: "dup"})
        if profile:
            t = pair.gpu.phase_times()
            assert t["replacement_edges"] > 0, t
            assert all(t[k] == 0.0 for k in ("validate", "update_graph", "root_finding", "orphan_scan",
                                              "superforest_rooting", "reversal_and_labels")), t
    pair.gpu.close()
