"""Two updates in flight: drsf_apply_async queues a batch behind the one
still running on a device-input context.  The queued updates must give the
results of applying them one at a time (Algorithm 1, Theorem 1): each
waited status is that batch's own (a rejected batch changes nothing and the
next one runs on the unchanged state), and at every drain the parent and
label arrays are bit-exact with the oracle's.  With one queued hooking round
and one search level most updates are finished by the host, so the update
queued behind each of them first stands still on the device and is then
queued again.  With a short inserted-edge list every few inserts rebuild the
store, and such an insert waits for the queue and is applied alone between
queued ones.  With a walk limit of one step, an update whose paths are
longer is finished by the host's doubling pass, which also holds the update
queued behind it."""
from __future__ import annotations

import numpy as np
import pytest

import gen
import oracle
from test_gpu_parity import _case, _lib

pytestmark = pytest.mark.gpu


def _plan(g, nbatch, mb, rng):
    """Batches for the oracle's state sequence: inserts, deletes (about half
    tree edges) and now and then a delete of a pair that is no edge (to be
    rejected); each with the oracle state after it."""
    r = oracle.apply(g.n, g.keys, g.parent, np.zeros((0, 2), np.int32), oracle.DELETE)
    keys, par, lab = g.keys, r.parent, r.label
    out = []
    for i in range(nbatch):
        b = int(rng.integers(1, mb + 1))
        seed = int(rng.integers(1 << 30))
        if i % 5 == 3:  # pairs that are not edges: the delete is rejected
            batch = gen.insert_batches(g.n, keys, 1, min(b, 50), seed)[0]
            out.append((batch, oracle.DELETE, False, par, lab))
            continue
        if i % 2 == 0:
            batch = gen.insert_batches(g.n, keys, 1, b, seed)[0]
            op = oracle.INSERT
        else:
            b = min(b, len(keys))
            trees = int((par != np.arange(g.n)).sum())
            nt = max(min(trees, b // 2), b - (len(keys) - trees))
            batch = gen.delete_batches(g.n, keys, par, 1, b, nt, seed)[0]
            op = oracle.DELETE
        r = oracle.apply(g.n, keys, par, batch, op, label=lab)
        keys, par, lab = r.keys, r.parent, r.label
        out.append((batch, op, True, par, lab))
    return out


@pytest.mark.parametrize("walk_limit", [0, 1])
@pytest.mark.parametrize("short_list", [False, True])
@pytest.mark.parametrize("launch_mode", [0, 1])
@pytest.mark.parametrize("host_finished", [False, True])
def test_queued_updates_match_the_oracle(host_finished, launch_mode, short_list, walk_limit):
    import torch
    drsf = _lib()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(31 + int(host_finished))
    g = gen.make_graph("rmat13", 1 << 13, gen.rmat(13, 8, 0.57, 0.19, 0.19, 4242))
    mb = 1500
    plan = _plan(g, 24, mb, rng)
    _case(f"queued updates: R-MAT 13, {len(plan)} batches up to {mb}, host-finished {host_finished}, "
          f"launch mode {launch_mode}, short inserted-edge list {short_list}, walk limit {walk_limit}")
    stream = torch.cuda.Stream(dev)
    with torch.cuda.stream(stream):
        t = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (g.row_ptr, g.col, g.parent)]
        dbat = [torch.from_numpy(np.ascontiguousarray(b, np.int32)).to(dev) for b, *_ in plan]
    f = drsf.Forest(g.n, *t, inputs_on_device=True, stream=stream.cuda_stream, max_batch=mb,
                    launch_mode=launch_mode, delta_capacity=2 * mb if short_list else 0, walk_limit=walk_limit)
    if host_finished:
        f.set_tuning(1, 1, 0)  # one queued round and level: the host finishes most updates
    op_of = {oracle.INSERT: drsf.DRSF_INSERT, oracle.DELETE: drsf.DRSF_DELETE}
    got, finished_by_host = [], 0

    def wait():
        nonlocal finished_by_host
        try:
            st = f.wait()
            finished_by_host += int(st["host_finished"] > 0)
            got.append(drsf.DRSF_OK)
        except drsf.DrsfError as e:
            got.append(e.code)

    chunk = 6
    for c0 in range(0, len(plan), chunk):
        part = plan[c0:c0 + chunk]
        # two deep: queue the next batch, then wait for the one before it
        f.apply_async(dbat[c0], op_of[part[0][1]])
        for j in range(1, len(part)):
            f.apply_async(dbat[c0 + j], op_of[part[j][1]])
            wait()
        wait()
        want = [drsf.DRSF_OK if ok else drsf.DRSF_E_BATCH for _, _, ok, _, _ in part]
        assert got[c0:c0 + len(part)] == want, f"batches {c0}..: statuses {got[c0:]} expected {want}"
        par, lab = part[-1][3], part[-1][4]
        assert np.array_equal(f.label(), lab), f"labels differ after batch {c0 + len(part) - 1}"
        assert np.array_equal(f.parent(), par), f"parents differ after batch {c0 + len(part) - 1}"
    if host_finished:
        assert finished_by_host >= len(plan) // 3, f"only {finished_by_host} updates needed the host"
    f.close()


def test_results_come_back_in_submission_order():
    """A drain on the caller's behalf (a copy-out, an empty batch) keeps the
    drained updates' results for drsf_wait, which returns them in the order
    the batches were queued: a rejected delete, then a valid insert queued
    while that result waits, then an empty batch, each with its own
    status."""
    import torch
    drsf = _lib()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(77)
    g = gen.make_graph("rmat11", 1 << 11, gen.rmat(11, 8, 0.57, 0.19, 0.19, 99))
    plan = _plan(g, 4, 300, rng)  # batch 3 is a rejected delete
    _case("queued results in order: R-MAT 11")
    stream = torch.cuda.Stream(dev)
    with torch.cuda.stream(stream):
        t = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (g.row_ptr, g.col, g.parent)]
        dbat = [torch.from_numpy(np.ascontiguousarray(b, np.int32)).to(dev) for b, *_ in plan]
        empty = torch.zeros((0, 2), dtype=torch.int32, device=dev)
    f = drsf.Forest(g.n, *t, inputs_on_device=True, stream=stream.cuda_stream, max_batch=300)
    op_of = {oracle.INSERT: drsf.DRSF_INSERT, oracle.DELETE: drsf.DRSF_DELETE}
    for j in range(3):
        f.apply(dbat[j], op_of[plan[j][1]])
    f.apply_async(dbat[3], op_of[plan[3][1]])   # rejected
    f.label()                                   # drains it on the caller's behalf
    # an insert of pairs that are still non-edges after the rejected delete
    ins = gen.insert_batches(g.n, _keys_after(g, plan[:3]), 1, 200, 5)[0]
    with torch.cuda.stream(stream):
        dins = torch.from_numpy(np.ascontiguousarray(ins, np.int32)).to(dev)
    got = []

    def wait():
        try:
            f.wait()
            got.append(drsf.DRSF_OK)
        except drsf.DrsfError as e:
            got.append(e.code)

    f.apply_async(dins, drsf.DRSF_INSERT)
    wait()                                      # the rejected delete's result, kept by the drain
    f.apply_async(empty, drsf.DRSF_DELETE)      # drains the insert, then nothing to launch
    wait()
    wait()
    assert got == [drsf.DRSF_E_BATCH, drsf.DRSF_OK, drsf.DRSF_OK], got
    r = oracle.apply(g.n, _keys_after(g, plan[:3]), plan[2][3], ins, oracle.INSERT, label=plan[2][4])
    assert np.array_equal(f.parent(), r.parent) and np.array_equal(f.label(), r.label)
    f.close()


def _keys_after(g, part):
    """Edge keys after the valid batches of part (replayed on the oracle)."""
    r = oracle.apply(g.n, g.keys, g.parent, np.zeros((0, 2), np.int32), oracle.DELETE)
    keys, par, lab = g.keys, r.parent, r.label
    for batch, op, ok, _, _ in part:
        if ok:
            r = oracle.apply(g.n, keys, par, batch, op, label=lab)
            keys, par, lab = r.keys, r.parent, r.label
    return keys
