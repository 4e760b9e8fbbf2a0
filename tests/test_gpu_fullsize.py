"""Parity at the benchmark's own sizes, through the C ABI (slow).

- R-MAT scale 22 at batch 1e4 and 1e6 (1e5 is test_gpu_parity's
  test_rmat22_full_size_step): insert and delete from the same initial state,
  graph, forest and batches in device memory, full parent and label arrays
  compared with the oracle.
- The batched workload at full size: 256 graphs G(n, 4n), n = 10^U(3,6), one
  batch per graph (op and size per graph) per multi-graph apply, the
  benchmark's first two steps; every graph's arrays compared with the oracle
  run on it alone, every graph's status checked.
- The served workload at full size: resident R-MAT scale 24 plus 8 tenants
  G(n, 4n), n = 10^U(5,6), a Poisson stream of mixed requests of 10^U(2,5)
  edges, requests of different graphs overlapping on the device.  Every
  request's status and its digests of parent and label are checked against
  the oracle replaying the same requests of the same graph (seconds per
  resident request at this size), and the resident graph's requests also
  against the library's single-graph path replaying them; at the end every
  graph's full arrays are compared element by element with the oracle's."""
from __future__ import annotations

import time

import numpy as np
import pytest

import gen
import oracle
from test_gpu_parity import _case, _lib
from test_gpu_server import digest

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _dev_tensors(*arrs):
    import torch
    dev = torch.device("cuda:0")
    return [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in arrs]


def test_rmat22_batch_sizes_1e4_and_1e6():
    import torch
    drsf = _lib()
    torch.cuda.set_device(0)
    keys = gen.rmat(22, 16, 0.57, 0.19, 0.19, gen.seed(2, 0, gen.P_GRAPH))
    g = gen.make_graph("rmat22", 1 << 22, keys)
    row, col, par = _dev_tensors(g.row_ptr, g.col, g.parent)
    torch.cuda.synchronize()
    f = drsf.Forest(g.n, row, col, par, inputs_on_device=True, max_batch=1_000_000,
                    delta_capacity=2_000_000)
    del row, col, par
    snap = f.snapshot()
    r0 = oracle.apply(g.n, g.keys, g.parent, np.zeros((0, 2), np.int32), oracle.DELETE)
    for b in (10_000, 1_000_000):
        ins = gen.insert_batches(g.n, g.keys, 1, b, gen.seed(2, 1, gen.P_INSERT) + b)[0]
        dl = gen.delete_batches(g.n, g.keys, g.parent, 1, b, b // 2, gen.seed(2, 1, gen.P_DELETE) + b)[0]
        for batch, op, oop in ((ins, drsf.DRSF_INSERT, oracle.INSERT), (dl, drsf.DRSF_DELETE, oracle.DELETE)):
            _case(f"rmat22 b={b} op={op}")
            f.restore(snap)
            (eb,) = _dev_tensors(batch)
            torch.cuda.synchronize()
            st = f.apply(eb, op)
            r = oracle.apply(g.n, g.keys, r0.parent, batch, oop, label=r0.label)
            p, lab = f.parent(), f.label()
            assert np.array_equal(lab, r.label), f"b={b} op={op}: labels differ"
            assert np.array_equal(p, r.parent), f"b={b} op={op}: parents differ"
            assert st["num_replacement"] == r.stats["n_repl"]
            assert st["num_edges"] == len(r.keys)
    drsf.drsf_snapshot_free(snap)
    f.close()


@pytest.mark.parametrize("small", [0, 4096])
def test_batched_256_graphs_full_size(small):
    """small: graphs of at most this many vertices go to the one-workgroup
    engine (0: every graph through the kernel sequence)."""
    import torch
    drsf = _lib()
    torch.cuda.set_device(0)
    t0 = time.time()
    wl = gen.batched_workload(256, 2, gen.seed(4, 0, gen.P_GRAPH))  # the benchmark's workload, steps 0-1
    mg = wl.mg
    ups = max(int(e[1][-1]) for e in wl.steps)
    _case(f"batched 256 graphs: n={mg.n} m={len(mg.col) // 2}, {ups} updates per step "
          f"(generated in {time.time() - t0:.1f}s)")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        row, col, par = _dev_tensors(mg.row_ptr, mg.col, mg.parent)
        steps = [_dev_tensors(e)[0] for e, _, _ in wl.steps]
    f = drsf.MultiForest(mg.n_off, row, col, par, max_batch=ups, stream=stream.cuda_stream,
                         inputs_on_device=True, delta_capacity=4 * ups + (1 << 20), small_graph_vertices=small)
    del row, col, par
    state = [[gr.keys, gr.parent, None] for gr in mg.graphs]
    for g, gr in enumerate(mg.graphs):
        r = oracle.apply(gr.n, gr.keys, gr.parent, np.zeros((0, 2), np.int32), oracle.DELETE)
        state[g] = [r.keys, r.parent, r.label]
    for i, (e, b_off, ops) in enumerate(wl.steps):
        st = f.apply_multi(steps[i], b_off, ops)
        assert (st == drsf.DRSF_OK).all(), f"step {i}: graphs rejected {np.flatnonzero(st).tolist()}"
        p, lab = f.parent(), f.label()
        m = f.num_edges()
        for g, gr in enumerate(mg.graphs):
            o = int(mg.n_off[g])
            bl = e[b_off[g]:b_off[g + 1]] - o
            keys, gp, gl = state[g]
            r = oracle.apply(gr.n, keys, gp, bl, oracle.INSERT if ops[g] == 0 else oracle.DELETE, label=gl)
            state[g] = [r.keys, r.parent, r.label]
            assert np.array_equal(lab[o:o + gr.n] - o, r.label), f"step {i} graph {g}: labels differ"
            assert np.array_equal(p[o:o + gr.n] - o, r.parent), f"step {i} graph {g}: parents differ"
            assert m[g] == len(r.keys), f"step {i} graph {g}: edge count"
        _case(f"batched step {i} (small graphs up to {small}): 256 graphs bit-exact")
    f.close()


ORACLE_RESIDENT = 1 << 30  # resident requests replayed by the oracle (all of them)


def test_served_rmat24_with_replay():
    import torch
    drsf = _lib()
    torch.cuda.set_device(0)
    t0 = time.time()
    graphs, reqs, win, last = gen.served_workload(24, 8, 90, 0)
    ups = sum(len(e) for _, e, _, _ in reqs)
    per = np.bincount([g for g, _, _, _ in reqs], minlength=len(graphs))
    _case(f"served R-MAT 24 + 8 tenants: {len(reqs)} requests ({per.tolist()} per graph), {ups} updates "
          f"(generated in {time.time() - t0:.1f}s)")
    opts = drsf.drsf_default_opts()
    opts.max_batch = 100_000
    fps = [drsf.drsf_footprint(g.n, len(g.col), opts) for g in graphs]
    srv = drsf.Server(sum(fps), max_batch=100_000, digests=True)
    rate = 2000.0  # requests per second: requests of several graphs in flight together
    tids = [srv.admit(gr.n, gr.row_ptr, gr.col, gr.parent,
                      arrive_ns=0 if g == 0 else int(win[g][0] * 1e9 / rate)) for g, gr in enumerate(graphs)]
    rids = [srv.submit(tids[g], e, op, arrive_ns=int(t * 1e9 / rate)) for g, e, op, t in reqs]
    srv.start()
    srv.wait_all()
    res = [srv.result(r) for r in rids]
    bad = [k for k, r in enumerate(res) if r["status"] != drsf.DRSF_OK]
    assert not bad, f"requests failed: {[(k, res[k]['status']) for k in bad[:10]]}"
    finals = [srv.copy_out(tids[g], gr.n) for g, gr in enumerate(graphs)]
    srv.close()
    _case(f"served run done ({time.time() - t0:.1f}s); replaying")
    # tenants (and the first resident requests): the oracle
    n_res = 0
    for g, gr in enumerate(graphs):
        r = oracle.apply(gr.n, gr.keys, gr.parent, np.zeros((0, 2), np.int32), oracle.DELETE)
        keys, par, lab = r.keys, r.parent, r.label
        full = True
        for k, (tg, e, op, _) in enumerate(reqs):
            if tg != g:
                continue
            if g == 0:
                if n_res >= ORACLE_RESIDENT:
                    full = False
                    break
                n_res += 1
            r = oracle.apply(gr.n, keys, par, e, oracle.INSERT if op == 0 else oracle.DELETE, label=lab)
            keys, par, lab = r.keys, r.parent, r.label
            assert res[k]["digest"] == digest(par, lab), f"request {k} (graph {g}): digests differ from the oracle"
        if full:
            assert np.array_equal(finals[g][1], lab), f"graph {g}: final labels differ from the oracle"
            assert np.array_equal(finals[g][0], par), f"graph {g}: final parents differ from the oracle"
        _case(f"graph {g}: {int(per[g])} requests checked ({'oracle' if full else 'oracle prefix'})")
    # the resident graph: every request against the single-graph path
    gr = graphs[0]
    f = drsf.Forest(gr.n, gr.row_ptr, gr.col, gr.parent, max_batch=100_000)
    for k, (tg, e, op, _) in enumerate(reqs):
        if tg != 0:
            continue
        f.apply(e, op)
        assert res[k]["digest"] == f.digest(), f"resident request {k}: served digests differ from the plain path"
    assert np.array_equal(finals[0][0], f.parent()) and np.array_equal(finals[0][1], f.label())
    f.close()
