"""Randomized parity: seeded small cases through the C ABI against the oracle.

Each case draws a graph family and size (G(n, m) up to 2·10^4 vertices, R-MAT
scale 6–14, grids with edges removed, paths with chords), a batch capacity,
the delete scan (per batch or whole store), the path reversal (per path or
Euler tour), the replacement-edge method (hooking on every cross edge or on
the supergraph), sometimes a small inserted-edge list (store rebuilds), host
or device-resident inputs, a random launch schedule and walk limit (paths
longer than it go to the doubling pass), then alternates insert and delete batches of random
sizes (deletes with a random share of tree edges).  Every batch: parent and
label arrays bit-exact, checker pass, same replacement-edge count.  Further
tests draw random multi-graph contexts, servers and static rebuilds."""
from __future__ import annotations

import numpy as np
import pytest

import gen
from test_gpu_parity import Pair, _case, _lib

pytestmark = pytest.mark.gpu


def _graph(rng, kind):
    if kind == "gnm":
        n = int(rng.integers(2, 20000))
        m = min(int(rng.integers(0, 4 * n)), n * (n - 1) // 2)
        return gen.make_graph("gnm", n, gen.gnm(n, m, int(rng.integers(1 << 30))))
    if kind == "rmat":
        s = int(rng.integers(6, 15))
        return gen.make_graph("rmat", 1 << s, gen.rmat(s, int(rng.integers(2, 16)), 0.57, 0.19, 0.19,
                                                        int(rng.integers(1 << 30))))
    if kind == "grid":
        a, b = int(rng.integers(2, 50)), int(rng.integers(2, 50))
        total = a * (b - 1) + b * (a - 1)
        return gen.make_graph("grid", a * b, gen.grid(a, b, int(rng.integers(0, total // 3 + 1)),
                                                      int(rng.integers(1 << 30))))
    n = int(rng.integers(2, 3000))
    path = np.array([(i << 32) | (i + 1) for i in range(n - 1)], np.uint64)
    chords = gen.gnm(n, int(rng.integers(0, n // 4 + 1)), int(rng.integers(1 << 30)))
    return gen.make_graph("path", n, np.union1d(path, chords))


@pytest.mark.parametrize("block", range(4))
def test_random_cases(block):
    drsf = _lib()
    for c in range(block * 100, (block + 1) * 100):
        rng = np.random.default_rng(7000 + c)
        kind = ("gnm", "rmat", "grid", "path")[c % 4]
        g = _graph(rng, kind)
        mb = int(rng.integers(1, 3000))
        kw = dict(max_batch=mb, sweep_mode=int(rng.integers(2)), reverse_mode=int(rng.random() < 0.25),
                  replacement_mode=int(rng.random() < 0.25))
        if rng.random() < 0.3:
            kw["delta_capacity"] = int(rng.integers(mb, 3 * mb + 1))  # a batch always fits
        device = bool(rng.random() < 0.3)
        # captured graphs now and then (its own draw: the cases stay as they were)
        kw["launch_mode"] = int(np.random.default_rng(70000 + c).integers(3))
        # and now and then a short walk limit (long paths turned by the doubling pass)
        kw["walk_limit"] = int(np.random.default_rng(80000 + c).choice([0, 0, 0, 1, 2, 5, 40]))
        _case(f"random {c}: {kind} n={g.n} m={g.m} {kw} device={device}")
        pair = Pair(g, device=device, **kw)
        if rng.random() < 0.5:
            pair.gpu.set_tuning(int(rng.integers(1, 7)), int(rng.integers(1, 9)), int(rng.integers(2)))
        for step in range(int(rng.integers(2, 8))):
            b = int(rng.integers(0, mb + 1))
            bi = min(b, g.n * (g.n - 1) // 2 - len(pair.keys))
            if bi > 0:
                ins = gen.insert_batches(g.n, pair.keys, 1, bi, int(rng.integers(1 << 30)))[0]
                pair.step(ins, drsf.DRSF_INSERT, f"random {c} insert {step}")
            trees = int((pair.parent != np.arange(g.n)).sum())
            bd = min(b, len(pair.keys))
            if bd > 0:
                nt = min(trees, int(rng.integers(0, bd + 1)))
                nt = max(nt, bd - (len(pair.keys) - trees))  # the rest must be non-tree edges
                dl = gen.delete_batches(g.n, pair.keys, pair.parent, 1, bd, nt, int(rng.integers(1 << 30)))[0]
                pair.step(dl, drsf.DRSF_DELETE, f"random {c} delete {step}")
        pair.gpu.close()


def test_random_multi_graph_cases():
    """The batched pattern: 60 seeded contexts of 1–40 graphs (1–5000
    vertices each, some edgeless), 3–6 multi-graph updates each with a
    random op and batch size per graph (empty batches included), now and
    then an invalid batch for one graph (rejected, that graph unchanged), a
    random launch schedule and walk limit, and a random small-graph
    threshold and workgroup size (graphs up to it go to the one-workgroup
    engine); every graph
    bit-exact with the oracle run on it alone."""
    from test_gpu_multi import MultiPair
    drsf = _lib()
    for c in range(60):
        rng = np.random.default_rng(9000 + c)
        graphs = []
        for g in range(int(rng.integers(1, 41))):
            n = int(rng.integers(1, 5000))
            m = min(int(rng.integers(0, 4 * n + 1)), n * (n - 1) // 2)
            keys = gen.gnm(n, m, int(rng.integers(1 << 30))) if m > 0 else np.zeros(0, np.uint64)
            graphs.append(gen.make_graph(f"g{g}", n, keys))
        mb = int(rng.integers(1, 2000))
        small = int(rng.choice([0, 0, 300, 2000, 5000]))  # graphs up to this size: the one-workgroup engine
        threads = int(rng.choice([256, 512, 1024]))
        _case(f"random multi {c}: {len(graphs)} graphs, sum n={sum(g.n for g in graphs)}, max_batch {mb}, "
              f"small graphs up to {small} ({threads} threads)")
        pair = MultiPair(graphs, max_batch=mb * len(graphs), sweep_mode=int(rng.integers(2)),
                         small_graph_vertices=small, small_threads=threads,
                         launch_mode=int(np.random.default_rng(90000 + c).integers(3)),
                         walk_limit=int(np.random.default_rng(95000 + c).choice([0, 0, 1, 3])))
        if rng.random() < 0.5:
            pair.gpu.set_tuning(int(rng.integers(1, 7)), int(rng.integers(1, 9)), int(rng.integers(2)))
        if small and rng.random() < 0.5:
            pair.gpu.set_small_schedule(0, int(rng.integers(1, 9)))
        for step in range(int(rng.integers(3, 7))):
            batches, ops = [], []
            for g, (n, keys, par) in enumerate(pair.local_state()):
                op = int(rng.integers(2))
                b = int(rng.integers(0, mb + 1))
                if op == drsf.DRSF_INSERT:
                    b = min(b, n * (n - 1) // 2 - len(keys))
                    bt = gen.insert_batches(n, keys, 1, b, int(rng.integers(1 << 30)))[0] if b > 0 else \
                        np.zeros((0, 2), np.int32)
                else:
                    b = min(b, len(keys))
                    trees = int((par != np.arange(n)).sum())
                    nt = max(min(trees, int(rng.integers(0, b + 1))), b - (len(keys) - trees))
                    bt = gen.delete_batches(n, keys, par, 1, b, nt, int(rng.integers(1 << 30)))[0] if b > 0 else \
                        np.zeros((0, 2), np.int32)
                batches.append(bt)
                ops.append(op)
            bad = {int(rng.integers(len(graphs)))} if rng.random() < 0.3 else set()
            bad = {g for g in bad if len(batches[g]) > 0 and len(batches[g]) < mb}
            pair.step(batches, np.array(ops, np.int8), f"random multi {c} step {step}", bad=bad)
        pair.gpu.close()


def test_random_server_cases():
    """The serving pattern: 24 seeded servers (1–5 tenants of random size,
    20–120 requests with some invalid ones, Poisson or bursty arrivals, a
    budget that sometimes holds only some tenants, and overlapped, serial or
    coalescing mode).  Every request's status and digests match the oracle
    applying the batches the server reports (one request each unless
    coalescing merged them)."""
    from test_gpu_server import _stream, digest
    import oracle
    drsf = _lib()
    for c in range(24):
        rng = np.random.default_rng(11000 + c)
        graphs = []
        for t in range(int(rng.integers(1, 6))):
            # the request stream draws n non-edges and needs 1.5 non-tree
            # edges per tree edge (m >= 3n leaves enough)
            n = int(rng.integers(50, 6000))
            m = int(rng.integers(3 * n, 5 * n + 1))
            graphs.append(gen.make_graph(f"t{t}", n, gen.gnm(n, m, int(rng.integers(1 << 30)))))
        nreq = int(rng.integers(20, 121))
        bad = set(int(x) for x in rng.choice(nreq, size=int(rng.integers(0, 4)), replace=False))
        reqs = _stream(graphs, nreq, int(rng.integers(1 << 20)), bad=bad)
        if rng.random() < 0.5:  # bursts, so that requests wait together
            reqs = [(t, e, op, (k // 10) * 2_000_000) for k, (t, e, op, _) in enumerate(reqs)]
        mode = ("overlap", "serial", "coalesce")[c % 3]
        fps = [drsf.drsf_footprint(g.n, len(g.col), None) for g in graphs]
        budget = max(fps) + (sum(fps) if rng.random() < 0.6 else 0)
        _case(f"random server {c}: {len(graphs)} tenants, {nreq} requests, bad {sorted(bad)}, {mode}, "
              f"budget {'all' if budget > max(fps) else 'one at a time'}")
        srv = drsf.Server(budget, max_batch=512, digests=True, serial=mode == "serial",
                          coalesce=mode == "coalesce", sweep_mode=int(rng.integers(2)))
        ids = [srv.admit(g.n, g.row_ptr, g.col, g.parent, arrive_ns=int(rng.integers(0, 3_000_000)))
               for g in graphs]
        rids = [srv.submit(ids[t], e, op, arrive_ns=a) for t, e, op, a in reqs]
        for tid in ids:
            srv.release(tid)
        srv.start()
        srv.wait_all()
        res = [srv.result(r) for r in rids]
        batch = [srv.batch(r) for r in rids]
        srv.close()
        pos = {r: k for k, r in enumerate(rids)}
        groups = {}
        for k, b in enumerate(batch):
            groups.setdefault(b, []).append(k)
        if mode != "coalesce":
            assert all(len(v) == 1 for v in groups.values())
        st = []
        for g in graphs:
            r = oracle.apply(g.n, g.keys, g.parent, np.zeros((0, 2), np.int32), oracle.DELETE)
            st.append([g.keys, r.parent, r.label])
        for b in sorted(groups, key=lambda x: pos[x]):
            ks = groups[b]
            t, op = reqs[ks[0]][0], reqs[ks[0]][2]
            e = np.concatenate([reqs[k][1] for k in ks]).reshape(-1, 2)
            keys, par, lab = st[t]
            try:
                r = oracle.apply(graphs[t].n, keys, par, e, oracle.INSERT if op == 0 else oracle.DELETE,
                                 label=lab)
            except oracle.OracleError:
                assert len(ks) == 1 and res[ks[0]]["status"] == drsf.DRSF_E_BATCH, (c, b, ks, res[ks[0]])
                continue
            st[t] = [r.keys, r.parent, r.label]
            dg = digest(r.parent, r.label)
            for k in ks:
                assert res[k]["status"] == drsf.DRSF_OK, (c, k, res[k])
                assert res[k]["digest"] == dg, f"server {c}, request {k}: digest differs from the oracle"


def test_random_static_rebuilds():
    """The static rebuild on 40 seeded graphs (the four families, random
    sizes): labels bit-exact, the forest valid by the oracle's checker and
    breadth-first."""
    from test_gpu_static import _run
    for c in range(40):
        rng = np.random.default_rng(13000 + c)
        _run(_graph(rng, ("gnm", "rmat", "grid", "path")[c % 4]), f"random {c}")
