"""The boundary's contracts on the GPU, through the C ABI.

Ordering: with no stream given, the context's own stream is ordered after
work queued earlier on the null stream (torch's default stream), so device
inputs still being written there — by asynchronous copies queued behind a
long-running kernel — are read only once written: at create and for every
batch read in place.  Allocator hooks: the context's device memory comes
from torch's caching allocator; every block is returned at destroy; an
allocation that fails is reported as DRSF_E_NOMEM with every block already
taken given back (create, snapshot, store rebuild), and a failed rebuild
leaves the forest readable and the context either as it was or refusing
further updates."""
from __future__ import annotations

import numpy as np
import pytest

import gen
import oracle
from test_gpu_parity import Pair, _case, _lib

pytestmark = pytest.mark.gpu

SPIN = 20_000_000  # cycles of torch.cuda._sleep queued ahead of each copy (~10 ms)


def _late_copy(x, dev):
    """A device copy of x that lands only after a long kernel on the current
    (default) stream: pinned source, asynchronous copy, no synchronisation."""
    import torch
    torch.cuda._sleep(SPIN)
    return torch.from_numpy(np.ascontiguousarray(x)).pin_memory().to(dev, non_blocking=True)


def _graphs():
    yield gen.make_graph("gnm", 3000, gen.gnm(3000, 9000, 5))
    n = 499
    path = np.array([(i << 32) | (i + 1) for i in range(n - 1)], np.uint64)
    yield gen.make_graph("path", n, np.union1d(path, gen.gnm(n, 100, 6)))
    yield gen.make_graph("rmat", 1 << 12, gen.rmat(12, 8, 0.57, 0.19, 0.19, 7))


def test_device_inputs_written_late_on_the_default_stream():
    import torch
    drsf = _lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(0)
    assert torch.cuda.current_stream().cuda_stream == 0  # the null stream
    for gi, g in enumerate(_graphs()):
        _case(f"late device inputs, graph {gi} n={g.n} m={g.m}")
        t = [_late_copy(x, dev) for x in (g.row_ptr, g.col, g.parent)]
        f = drsf.Forest(g.n, *t, inputs_on_device=True, max_batch=2048)  # stream: the context's own
        del t
        r = oracle.apply(g.n, g.keys, g.parent, np.zeros((0, 2), np.int32), oracle.DELETE)
        keys, par, lab = r.keys, r.parent, r.label
        assert np.array_equal(f.parent(), par) and np.array_equal(f.label(), lab)
        for step in range(4):
            if step % 2 == 0:
                batch = gen.insert_batches(g.n, keys, 1, 600, 100 * gi + step)[0]
                op, oop = drsf.DRSF_INSERT, oracle.INSERT
            else:
                trees = int((par != np.arange(g.n)).sum())
                batch = gen.delete_batches(g.n, keys, par, 1, 700, min(350, trees), 100 * gi + step)[0]
                op, oop = drsf.DRSF_DELETE, oracle.DELETE
            eb = _late_copy(batch, dev)
            f.apply(eb, op)
            r = oracle.apply(g.n, keys, par, batch, oop, label=lab)
            keys, par, lab = r.keys, r.parent, r.label
            assert np.array_equal(f.label(), lab), (gi, step)
            assert np.array_equal(f.parent(), par), (gi, step)
        f.close()


def test_torch_allocator_hooks_parity_and_release():
    import torch
    drsf = _lib()
    torch.cuda.set_device(0)
    alloc = drsf.TorchAllocator()
    g = gen.make_graph("gnm", 5000, gen.gnm(5000, 15000, 11))
    _case("torch allocator hooks")
    pair = Pair(g, max_batch=1024, delta_capacity=1500, allocator=alloc)
    assert alloc.live and sum(alloc.live.values()) == pair.gpu.device_bytes()
    snap = pair.gpu.snapshot()
    for step in range(6):  # the inserted-edge list fills: store rebuilds through the hooks
        ins = gen.insert_batches(g.n, pair.keys, 1, 900, 40 + step)[0]
        pair.step(ins, drsf.DRSF_INSERT, f"hooks insert {step}")
        trees = int((pair.parent != np.arange(g.n)).sum())
        dl = gen.delete_batches(g.n, pair.keys, pair.parent, 1, 800, min(300, trees), 60 + step)[0]
        pair.step(dl, drsf.DRSF_DELETE, f"hooks delete {step}")
    drsf.drsf_snapshot_free(snap)
    pair.gpu.close()
    assert not alloc.live, f"{len(alloc.live)} blocks not returned"


def test_failing_allocator_reports_nomem_at_create():
    import torch
    drsf = _lib()
    torch.cuda.set_device(0)
    g = gen.make_graph("gnm", 2000, gen.gnm(2000, 5000, 12))
    probe = drsf.TorchAllocator()
    f = drsf.Forest(g.n, g.row_ptr, g.col, g.parent, max_batch=512, allocator=probe)
    total = probe.calls
    f.close()
    assert total > 20 and not probe.live
    _case(f"create with failing allocations, {total} allocations per create")
    for limit in range(total):
        alloc = drsf.TorchAllocator(limit=limit)
        with pytest.raises(drsf.DrsfError) as e:
            drsf.Forest(g.n, g.row_ptr, g.col, g.parent, max_batch=512, allocator=alloc)
        assert e.value.code == drsf.DRSF_E_NOMEM, (limit, str(e.value))
        assert not alloc.live, (limit, len(alloc.live))


def test_failing_allocator_in_snapshot_and_store_rebuild():
    import torch
    drsf = _lib()
    torch.cuda.set_device(0)
    g = gen.make_graph("gnm", 3000, gen.gnm(3000, 9000, 13))
    ins = [gen.insert_batches(g.n, g.keys, 2, 700, 77)]
    ins = ins[0]
    # allocations a rebuild makes, counted on a context that succeeds
    probe = drsf.TorchAllocator()
    f = drsf.Forest(g.n, g.row_ptr, g.col, g.parent, max_batch=1024, delta_capacity=1000, allocator=probe)
    f.apply(ins[0], drsf.DRSF_INSERT)
    before = probe.calls
    f.apply(ins[1], drsf.DRSF_INSERT)  # 1400 > 1000 inserted edges: merged into the store first
    per_rebuild = probe.calls - before
    f.close()
    assert per_rebuild > 5 and not probe.live
    r1 = oracle.apply(g.n, g.keys, g.parent, ins[0], oracle.INSERT)
    r2 = oracle.apply(g.n, r1.keys, r1.parent, ins[1], oracle.INSERT, label=r1.label)
    _case(f"store rebuild with failing allocations ({per_rebuild} allocations)")
    outcomes = set()
    for j in range(per_rebuild):
        alloc = drsf.TorchAllocator()
        f = drsf.Forest(g.n, g.row_ptr, g.col, g.parent, max_batch=1024, delta_capacity=1000, allocator=alloc)
        f.apply(ins[0], drsf.DRSF_INSERT)
        alloc.limit = alloc.calls + j
        with pytest.raises(drsf.DrsfError) as e:
            f.apply(ins[1], drsf.DRSF_INSERT)
        assert e.value.code == drsf.DRSF_E_NOMEM, (j, str(e.value))
        # the forest is the one before the failed batch
        assert np.array_equal(f.parent(), r1.parent) and np.array_equal(f.label(), r1.label), j
        alloc.limit = None
        try:
            f.apply(ins[1], drsf.DRSF_INSERT)
            outcomes.add("usable")
            assert np.array_equal(f.parent(), r2.parent) and np.array_equal(f.label(), r2.label), j
        except drsf.DrsfError as e2:
            assert e2.code == drsf.DRSF_E_STATE, (j, str(e2))
            outcomes.add("refuses")
            assert np.array_equal(f.parent(), r1.parent), j
        f.close()
        assert not alloc.live, (j, len(alloc.live))
    assert "usable" in outcomes
    # snapshots
    alloc = drsf.TorchAllocator()
    f = drsf.Forest(g.n, g.row_ptr, g.col, g.parent, max_batch=1024, allocator=alloc)
    held = len(alloc.live)
    for j in range(7):
        alloc.limit = alloc.calls + j
        with pytest.raises(drsf.DrsfError) as e:
            f.snapshot()
        assert e.value.code == drsf.DRSF_E_NOMEM and len(alloc.live) == held, j
    f.close()
    assert not alloc.live
