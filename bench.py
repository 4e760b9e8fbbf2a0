"""Benchmark: batch-dynamic rooted spanning forest updates on one MI355X.

Workload: R-MAT scale 22 (4,194,304 vertices, 16 * 2^22 samples with
a/b/c/d = 0.57/0.19/0.19/0.05, self-loops dropped, symmetrised, deduplicated),
initial BFS forest.  One step = one insert batch of 1e5 uniform random
non-edges followed by one delete batch of 1e5 edges (5e4 tree edges and 5e4
non-tree edges).  The batches of all steps are generated up front from the
initial state: inserted edges are non-edges distinct across steps, deleted
edges are initial edges distinct across steps, and tree edges are initial
tree edges, which stay tree edges until deleted because an update keeps
every surviving forest edge.  Graph, forest and every batch are resident in
device memory before the timed region starts.

Prints one JSON line: value = edge updates per second of the whole timed
job (insert + delete) in the production configuration (each update launches
the context's kernel sequence, queued behind the one before it so that two
are in flight); insert and delete latencies as seen by the host from a
pass over the same steps one update at a time; per-phase device times and
the rooflines of the dominant kernels from a pass that launches the kernels
one by one with events between the phases on the stream the kernels run
on; and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def kernel_source_sha(kernel: str) -> str:
    """sha256[:16] of the kernel's own definition in drsf_kernels.hip (from
    its __global__ line to its closing brace)."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_2607_20211_amd", "csrc", "drsf_kernels.hip")).read()
    i = src.find(f" void {kernel}(")
    if i < 0:
        return ""
    i = src.rfind("\n", 0, i) + 1
    j = src.index("{", i)
    depth = 0
    for k in range(j, len(src)):
        depth += {"{": 1, "}": -1}.get(src[k], 0)
        if depth == 0:
            return hashlib.sha256(src[i:k + 1].encode()).hexdigest()[:16]
    return ""


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    runs (profiles/*.counters.json), or None when the kernel's definition
    has changed since the counters were taken."""
    import glob
    h = kernel_source_sha(kernel)
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.counters.json")):
        c = json.load(open(path))
        if c.get("kernel") == kernel and c.get("workload") == workload and c.get("kernel_sha256_16") == h:
            return c["traffic_bytes_per_launch"]
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def pct(xs, q):
    return float(np.percentile(np.asarray(xs, np.float64), q))


# this build's phases grouped as the paper's breakdown (Sec. V results):
# deletion compaction, finding oriented replacement edges (root finding,
# key-edge scans, hooking, super-forest orientation, and any host-driven
# continuation of those), path reversal (here with the new labels)
PAPER_GROUPS = {"validation (not in the paper)": ["validate"],
                "compaction": ["update_graph"],
                "oriented_replacement_edges": ["root_finding", "orphan_list", "orphan_scan", "store_sweep",
                                               "batch_and_inserted_scan", "replacement_edges",
                                               "superforest_rooting", "host_continuation"],
                "path_reversal": ["reversal_and_labels"]}


def paper_shares(phases, bracket):
    """Shares of the profiled device time per group of PAPER_GROUPS (phase
    times less the event bracket; phases that launched nothing count 0)."""
    t = {k: max(v - bracket, 0.0) if (v > 0 and k != "host_continuation") else v for k, v in phases.items()}
    tot = sum(t.values())
    return {grp: round(sum(t.get(k, 0.0) for k in ks) / tot, 3) if tot > 0 else 0.0
            for grp, ks in PAPER_GROUPS.items()}


def run_instances(scale, b, g0, ninst, runs, dev, stream, log):
    """The paper's protocol (Sec. V: several graph instances, several runs
    each): instances 0..ninst-1 of the headline workload (instance 0 is the
    headline graph, the others R-MAT graphs of the same recipe on other
    seeds), each with 2 warm-up steps and `runs` timed steps of one insert
    and one delete batch of b; per-op updates/s as median, mean, p10 and
    p90 over all instance-runs, and per instance."""
    import torch
    import gen
    from paper_2607_20211_amd import drsf
    ins_rates, del_rates, per = [], [], []
    for inst in range(ninst):
        t0 = time.time()
        if inst == 0:
            g = g0
        else:
            g = gen.make_graph(f"rmat{scale}", 1 << scale,
                               gen.rmat(scale, 16, 0.57, 0.19, 0.19, gen.seed(2, inst, gen.P_GRAPH)))
        ins = torch.from_numpy(gen.insert_batches(g.n, g.keys, 2 + runs, b, gen.seed(2, inst, gen.P_INSERT) + 7)).to(dev)
        dl = torch.from_numpy(gen.delete_batches(g.n, g.keys, g.parent, 2 + runs, b, b // 2,
                                                 gen.seed(2, inst, gen.P_DELETE) + 7)).to(dev)
        f = drsf.Forest(g.n, torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                        torch.from_numpy(g.parent).to(dev), max_batch=b, stream=stream.cuda_stream,
                        inputs_on_device=True, delta_capacity=(2 + runs) * b + (1 << 20))
        ri, rd = [], []
        for i in range(2 + runs):
            ta = time.perf_counter()
            f.apply(ins[i], drsf.DRSF_INSERT)
            tb = time.perf_counter()
            f.apply(dl[i], drsf.DRSF_DELETE)
            tc = time.perf_counter()
            if i >= 2:
                ri.append(b / (tb - ta))
                rd.append(b / (tc - tb))
        f.close()
        ins_rates += ri
        del_rates += rd
        per.append({"instance": inst, "m": g.m, "insert_median": round(float(np.median(ri)), 1),
                    "delete_median": round(float(np.median(rd)), 1)})
        log(f"instance {inst}: m={g.m} insert {np.median(ri):.3e} delete {np.median(rd):.3e} updates/s "
            f"({time.time() - t0:.1f}s)")

    def summ(x):
        return {"median": round(float(np.median(x)), 1), "mean": round(float(np.mean(x)), 1),
                "p10": round(pct(x, 10), 1), "p90": round(pct(x, 90), 1)}
    return {"instances": ninst, "runs_per_instance": runs, "batch": b,
            "insert_updates_per_s": summ(ins_rates), "delete_updates_per_s": summ(del_rates),
            "per_instance": per,
            "how": "instance 0 = the headline graph; others: the same R-MAT recipe on other seeds; each "
                   "run = one insert batch then one delete batch, host-observed latency per apply"}


def run_served(scale, nreq, loads, log):
    """Served pattern against the plain path (one request at a time in
    arrival order, same server code in serial mode), and with coalescing
    (the same-op requests waiting at the head of a tenant's queue go out as
    one batch).  Every request's status is collected and failures are
    counted; a verification pass (outside the timed runs) serves the whole
    stream at once in overlapped and in serial mode with digests on and
    compares every request's digests of parent and label between the two."""
    import gen
    from paper_2607_20211_amd import drsf
    t0 = time.time()
    graphs, reqs, win, last = gen.served_workload(scale, 8, nreq, 0)
    ups = sum(len(e) for _, e, _, _ in reqs)
    log(f"served workload: {len(graphs)} graphs, {len(reqs)} requests, {ups} updates "
        f"({time.time() - t0:.1f}s)")
    opts = drsf.drsf_default_opts()
    opts.max_batch = 100_000
    fps = [drsf.drsf_footprint(g.n, len(g.col), opts) for g in graphs]
    budget = fps[0] + sum(sorted(fps[1:])[-3:])

    def serve(serial, rate, coalesce=False, digests=False):
        srv = drsf.Server(budget, max_batch=100_000, serial=serial, coalesce=coalesce, digests=digests)
        scale_ns = 1e9 / rate if rate else 0.0
        tids = []
        for g, gr in enumerate(graphs):
            a = 0 if g == 0 or not rate else int(win[g][0] * scale_ns)
            tids.append(srv.admit(gr.n, gr.row_ptr, gr.col, gr.parent, arrive_ns=a))
        rids = [srv.submit(tids[g], e, op, arrive_ns=int(t * scale_ns) if rate else 0)
                for g, e, op, t in reqs]
        for g in range(1, len(graphs)):
            srv.release(tids[g])
        srv.start()
        srv.wait_all()
        st = srv.stats()
        res = [srv.result(r) for r in rids]
        st["failed"] = sum(r["status"] != drsf.DRSF_OK for r in res)
        st["batches"] = len({srv.batch(r) for r in rids})
        st["digests"] = [r["digest"] for r in res] if digests else None
        srv.close()
        return st

    sat = serve(True, None)  # plain path, every request queued at once: its service rate
    mu = sat["completed"] / (sat["completed"] and (ups / sat["updates_per_s"]))
    log(f"plain path service rate {mu:.1f} requests/s ({sat['updates_per_s']:.3e} updates/s), "
        f"{sat['failed']} failed")
    out = []
    failed = sat["failed"]
    for lam in loads:
        rate = lam * mu
        a = serve(False, rate)
        bb = serve(True, rate)
        c = serve(False, rate, coalesce=True)
        failed += a["failed"] + bb["failed"] + c["failed"]
        log(f"load {lam}: served p50 {a['p50_ms']:.3f} p99 {a['p99_ms']:.3f} ms "
            f"(service {a['service_p50_ms']:.3f} / {a['service_p99_ms']:.3f}); "
            f"plain p50 {bb['p50_ms']:.3f} p99 {bb['p99_ms']:.3f} ms "
            f"(service {bb['service_p50_ms']:.3f} / {bb['service_p99_ms']:.3f}); "
            f"coalesced p50 {c['p50_ms']:.3f} p99 {c['p99_ms']:.3f} ms in {c['batches']} batches; "
            f"failed {a['failed']}/{bb['failed']}/{c['failed']}")
        out.append({"load": lam, "offered_requests_per_s": round(rate, 1),
                    "served_p50_ms": round(a["p50_ms"], 4), "served_p99_ms": round(a["p99_ms"], 4),
                    "served_service_p50_ms": round(a["service_p50_ms"], 4),
                    "served_service_p99_ms": round(a["service_p99_ms"], 4),
                    "served_updates_per_s": round(a["updates_per_s"], 1),
                    "plain_p50_ms": round(bb["p50_ms"], 4), "plain_p99_ms": round(bb["p99_ms"], 4),
                    "plain_service_p50_ms": round(bb["service_p50_ms"], 4),
                    "plain_service_p99_ms": round(bb["service_p99_ms"], 4),
                    "plain_updates_per_s": round(bb["updates_per_s"], 1),
                    "coalesced_p50_ms": round(c["p50_ms"], 4), "coalesced_p99_ms": round(c["p99_ms"], 4),
                    "coalesced_service_p50_ms": round(c["service_p50_ms"], 4),
                    "coalesced_service_p99_ms": round(c["service_p99_ms"], 4),
                    "coalesced_updates_per_s": round(c["updates_per_s"], 1),
                    "coalesced_batches": c["batches"],
                    "failed": {"served": a["failed"], "plain": bb["failed"], "coalesced": c["failed"]},
                    "peak_bytes": a["peak_bytes"]})
    # verification pass: per-request digests, overlapped against serial
    va = serve(False, None, digests=True)
    vb = serve(True, None, digests=True)
    same = va["digests"] == vb["digests"]
    log(f"served verification: {len(reqs)} requests, digests equal overlapped vs serial: {same}; "
        f"failed {va['failed']}/{vb['failed']}")
    assert failed == 0 and va["failed"] == 0 and vb["failed"] == 0, "served requests failed"
    assert same, "served digests differ from the plain path"
    return {"workload": f"resident R-MAT scale {scale} + 8 tenants G(n, 4n), n = 10^U(5,6), "
                        f"staggered; {len(reqs)} requests of 10^U(2,5) edges, Poisson arrivals",
            "requests": len(reqs), "updates": ups, "budget_bytes": budget,
            "plain_service_requests_per_s": round(mu, 1),
            "plain_saturated_updates_per_s": round(sat["updates_per_s"], 1),
            "failed_requests": int(failed),
            "verified": {"requests": len(reqs), "served_equals_plain_digests": bool(same),
                         "how": "every request's parent and label digests, overlapped against serial, "
                                "whole stream at once"},
            "loads": out}


def time_op(f, snap, batch, op, reps, drsf):
    """Median seconds of one apply of `batch` from the snapshot's state."""
    ts = []
    for _ in range(reps):
        f.restore(snap)
        t0 = time.perf_counter()
        f.apply(batch, op)
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


# replacement_mode (0: hooking on every cross edge, HS; 1: supergraph, SG) x
# reverse_mode (0: a thread per path; 1: Euler tour, ET)
METHODS = {"hs_paths": (0, 0), "hs_et": (0, 1), "sg_paths": (1, 0), "sg_et": (1, 1)}


def methods_ab(n, row, col, par, batches, max_batch, stream, drsf, reps=3):
    """The same updates with each replacement-edge method and each path
    reversal (the paper's SG/HS x ET variants beside this build's defaults).
    Wall time per update: median of reps applies from the same state on a
    context in the production configuration (the supergraph reads sizes
    back between its kernels, so it is always launched kernel by kernel).  Phase times: the same updates on a profiled context (kernels
    launched one by one with events), less the event bracket.  Whether every
    method ends in the same forest: digests."""
    res = {}
    for name, (rm, vm) in METHODS.items():
        f = drsf.Forest(n, row, col, par, max_batch=max_batch, stream=stream.cuda_stream,
                        inputs_on_device=True, replacement_mode=rm, reverse_mode=vm)
        snap = f.snapshot()
        walls = []
        for edges, op in batches:
            state = f.snapshot()
            ts = []
            for _ in range(reps):
                f.restore(state)
                t0 = time.perf_counter()
                f.apply(edges, op)
                ts.append(time.perf_counter() - t0)
            walls.append(float(np.median(ts)))
            drsf.drsf_snapshot_free(state)
        digest = [int(x) for x in f.digest()]
        drsf.drsf_snapshot_free(snap)
        f.close()
        fp = drsf.Forest(n, row, col, par, max_batch=max_batch, stream=stream.cuda_stream,
                         inputs_on_device=True, profile=True, replacement_mode=rm, reverse_mode=vm)
        steps = []
        for (edges, op), wall in zip(batches, walls):
            st = fp.apply(edges, op)
            t = fp.phase_times()
            br = t.pop(drsf.EVENT_BRACKET, 0.0)
            steps.append({"op": "insert" if op == drsf.DRSF_INSERT else "delete",
                          "cross_edges": st["num_key_cross"], "paths": st["num_paths"],
                          "host_finished": st["host_finished"],
                          "replacement_phase_ms": round(t["replacement_edges"] - br, 4),
                          "reversal_and_labels_phase_ms": round(t["reversal_and_labels"] - br, 4),
                          "host_continuation_ms": round(t["host_continuation"], 4),
                          "phases_ms": {k: round(max(v - br, 0.0) if (v > 0 and k != "host_continuation")
                                                 else v, 4) for k, v in t.items()},
                          "update_wall_ms": round(wall * 1e3, 4)})
        assert [int(x) for x in fp.digest()] == digest
        fp.close()
        res[name] = {"steps": steps, "digest": digest}
    res["same_result"] = len({tuple(v["digest"]) for k, v in res.items() if k in METHODS}) == 1
    return res


def static_rebuild(n, keys, dev, stream, drsf, reps=3):
    """The static baseline (row f3): a rooted spanning forest of the graph
    with these keys from scratch on the GPU (components by hooking, then a
    breadth-first forest from each component's smallest vertex); median wall
    time of reps runs with the CSR already in device memory."""
    import torch
    import gen
    row_ptr, col = gen.keys_to_csr(n, keys)
    d_row, d_col = torch.from_numpy(row_ptr).to(dev), torch.from_numpy(col).to(dev)
    par = torch.empty(n, dtype=torch.int32, device=dev)
    lab = torch.empty_like(par)
    times, levels = [], 0
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        levels = drsf.drsf_static_forest(n, d_row, d_col, par, lab, stream.cuda_stream)
        times.append(time.perf_counter() - t0)
    return {"ms": round(float(np.median(times)) * 1e3, 3), "levels": levels}


def edge_keys(batch):
    u, v = batch[:, 0].astype(np.uint64), batch[:, 1].astype(np.uint64)
    return (np.minimum(u, v) << np.uint64(32)) | np.maximum(u, v)


def store_rebuild(g, dev, stream, log, drsf, b=100_000, reps=3):
    """Cost of merging the inserted-edge list into the base store (the
    off-path O(|E|) rebuild): an insert batch that overflows a list of b
    entries (rebuild + insert) against the same batch on a context whose
    list has room, both from the same state; amortised over the insert
    batches that fill the default list."""
    import torch
    import gen
    keys2 = gen.insert_batches(g.n, g.keys, 2, b, gen.seed(2, 3, gen.P_INSERT))
    d0, d1 = (torch.from_numpy(k).to(dev) for k in keys2)
    times = {}
    for cap in (b, 4 * b):
        f = drsf.Forest(g.n, torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                        torch.from_numpy(g.parent).to(dev), max_batch=b, stream=stream.cuda_stream,
                        inputs_on_device=True, delta_capacity=cap)
        f.apply(d0, drsf.DRSF_INSERT)  # fills the list when cap == b
        ts = []
        for _ in range(reps):
            snap = f.snapshot()
            t0 = time.perf_counter()
            f.apply(d1, drsf.DRSF_INSERT)
            ts.append(time.perf_counter() - t0)
            if cap == b:  # the rebuild changed the layout: start again from a fresh context
                drsf.drsf_snapshot_free(snap)
                f.close()
                f = drsf.Forest(g.n, torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                                torch.from_numpy(g.parent).to(dev), max_batch=b, stream=stream.cuda_stream,
                                inputs_on_device=True, delta_capacity=cap)
                f.apply(d0, drsf.DRSF_INSERT)
            else:
                f.restore(snap)
                drsf.drsf_snapshot_free(snap)
        f.close()
        times[cap] = float(np.median(ts))
    rb = times[b] - times[4 * b]
    dcap = max(4 * b, g.m // 8, 1 << 20)  # the default inserted-edge list at max_batch b
    out = {"rebuild_ms": round(rb * 1e3, 3), "insert_with_rebuild_ms": round(times[b] * 1e3, 3),
           "insert_ms": round(times[4 * b] * 1e3, 3), "default_list_entries": dcap,
           "insert_batches_per_rebuild": dcap // b,
           "amortised_ms_per_insert_batch": round(rb * 1e3 / (dcap // b), 4),
           "what": f"R-MAT 22 with {2 * b} inserted edges merged into the base store"}
    log(f"store rebuild: {out}")
    return out


def run_configs(g, dev, stream, log, reps=3):
    """Per-op rates from the initial state: R-MAT 22 at b = 1e4, 1e5, 1e6
    (inserts of uniform non-edges; deletes half tree edges), the deep
    4096 x 4096 grid (5% of edges removed): 1e5 tree-edge deletes, then 1e5
    inserts of uniform vertex pairs that are not edges, and deep chains
    (a long path turned by the pass or walked)."""
    import torch
    import gen
    from paper_2607_20211_amd import drsf
    out = {}
    d_row = torch.from_numpy(g.row_ptr).to(dev)
    d_col = torch.from_numpy(g.col).to(dev)
    d_par = torch.from_numpy(g.parent).to(dev)
    f = drsf.Forest(g.n, d_row, d_col, d_par, max_batch=1_000_000, stream=stream.cuda_stream,
                    inputs_on_device=True, delta_capacity=4_000_000)
    del d_row, d_col, d_par
    snap = f.snapshot()
    sweep = []
    for b in (10_000, 100_000, 1_000_000):
        ins = torch.from_numpy(gen.insert_batches(g.n, g.keys, 1, b, gen.seed(2, 1, gen.P_INSERT))[0]).to(dev)
        dl = torch.from_numpy(gen.delete_batches(g.n, g.keys, g.parent, 1, b, b // 2,
                                                 gen.seed(2, 1, gen.P_DELETE))[0]).to(dev)
        f.apply(ins, drsf.DRSF_INSERT)  # warm
        f.restore(snap)
        f.apply(dl, drsf.DRSF_DELETE)
        ti = time_op(f, snap, ins, drsf.DRSF_INSERT, reps, drsf)
        td = time_op(f, snap, dl, drsf.DRSF_DELETE, reps, drsf)
        sweep.append({"batch": b, "insert_updates_per_s": round(b / ti, 1),
                      "delete_updates_per_s": round(b / td, 1),
                      "insert_ms": round(ti * 1e3, 4), "delete_ms": round(td * 1e3, 4)})
        log(f"rmat22 b={b}: insert {ti * 1e3:.3f} ms, delete {td * 1e3:.3f} ms")
    drsf.drsf_snapshot_free(snap)
    f.close()
    out["rmat22_from_initial_state"] = sweep
    out["store_rebuild_rmat22"] = store_rebuild(g, dev, stream, log, drsf)
    # replacement-edge and path-reversal methods (rows f1, f2) on the headline
    # workload: insert then delete 1e5
    ins = torch.from_numpy(gen.insert_batches(g.n, g.keys, 1, 100_000, gen.seed(2, 2, gen.P_INSERT))[0]).to(dev)
    dl = torch.from_numpy(gen.delete_batches(g.n, g.keys, g.parent, 1, 100_000, 50_000,
                                             gen.seed(2, 2, gen.P_DELETE))[0]).to(dev)
    out["methods_ab_rmat22_b1e5"] = methods_ab(
        g.n, torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
        torch.from_numpy(g.parent).to(dev), [(ins, drsf.DRSF_INSERT), (dl, drsf.DRSF_DELETE)],
        100_000, stream, drsf)
    log(f"methods A/B rmat22: {out['methods_ab_rmat22_b1e5']}")
    # static rebuild of the graph after the 1e5-insert batch (row f3), against
    # the dynamic updates at b = 1e5
    st = static_rebuild(g.n, np.union1d(g.keys, edge_keys(ins.cpu().numpy())), dev, stream, drsf)
    b5 = [x for x in sweep if x["batch"] == 100_000][0]
    st["speedup_insert"] = round(st["ms"] / b5["insert_ms"], 1)
    st["speedup_delete"] = round(st["ms"] / b5["delete_ms"], 1)
    out["static_rebuild_rmat22"] = st
    log(f"static rebuild rmat22: {st}")
    # deep trees
    t0 = time.time()
    side = 4096
    total = side * (side - 1) * 2
    keys = gen.grid(side, side, total // 20, gen.seed(3, 0, gen.P_GRAPH))
    gg = gen.make_graph("grid4096", side * side, keys)
    trees = int((gg.parent != np.arange(gg.n)).sum())
    dl = gen.delete_batches(gg.n, gg.keys, gg.parent, 1, 100_000, 100_000, gen.seed(3, 0, gen.P_DELETE))[0]
    ins = gen.insert_batches(gg.n, gg.keys, 1, 100_000, gen.seed(3, 0, gen.P_INSERT))[0]
    log(f"grid {side}x{side}: n={gg.n} m={gg.m} tree edges {trees} ({time.time() - t0:.1f}s)")
    f = drsf.Forest(gg.n, torch.from_numpy(gg.row_ptr).to(dev), torch.from_numpy(gg.col).to(dev),
                    torch.from_numpy(gg.parent).to(dev), max_batch=100_000, stream=stream.cuda_stream,
                    inputs_on_device=True)
    d_dl, d_ins = torch.from_numpy(dl).to(dev), torch.from_numpy(ins).to(dev)
    snap = f.snapshot()
    f.apply(d_dl, drsf.DRSF_DELETE)
    f.apply(d_ins, drsf.DRSF_INSERT)
    td, ti = [], []
    for _ in range(reps):
        f.restore(snap)
        t1 = time.perf_counter()
        st_d = f.apply(d_dl, drsf.DRSF_DELETE)
        t2 = time.perf_counter()
        st_i = f.apply(d_ins, drsf.DRSF_INSERT)
        t3 = time.perf_counter()
        td.append(t2 - t1)
        ti.append(t3 - t2)
    drsf.drsf_snapshot_free(snap)
    f.close()
    td, ti = float(np.median(td)), float(np.median(ti))
    log(f"grid: delete {td * 1e3:.3f} ms, insert {ti * 1e3:.3f} ms")
    out["grid4096_deep"] = {"n": gg.n, "m": gg.m, "delete_tree_edges": 100_000, "insert_pairs": 100_000,
                            "delete_updates_per_s": round(1e5 / td, 1), "delete_ms": round(td * 1e3, 4),
                            "insert_updates_per_s": round(1e5 / ti, 1), "insert_ms": round(ti * 1e3, 4),
                            "delete_stats": st_d, "insert_stats": st_i}
    out["methods_ab_grid4096"] = methods_ab(
        gg.n, torch.from_numpy(gg.row_ptr).to(dev), torch.from_numpy(gg.col).to(dev),
        torch.from_numpy(gg.parent).to(dev), [(d_dl, drsf.DRSF_DELETE), (d_ins, drsf.DRSF_INSERT)],
        100_000, stream, drsf)
    log(f"methods A/B grid: {out['methods_ab_grid4096']}")
    keep = np.ones(len(gg.keys), bool)
    keep[np.searchsorted(gg.keys, edge_keys(dl))] = False
    st = static_rebuild(gg.n, gg.keys[keep], dev, stream, drsf, reps=1)
    st["speedup_delete"] = round(st["ms"] / (td * 1e3), 1)
    out["static_rebuild_grid4096"] = st
    log(f"static rebuild grid: {st}")
    out["deep_chains"] = deep_chains(dev, stream, log, drsf)
    return out


def deep_chains(dev, stream, log, drsf, n=1 << 22, h=65536):
    """Deep forests: two chains of n/2 vertices (a path graph's breadth-first
    forest is the chain itself), each closed into a ring by an insert, then
    cut so that the far part re-attaches through the closing edge: a path of
    h steps to turn, and root finding over chains n/2 deep.  The first cut
    (chain A) flags the forest deep and allocates the long-path pass; the
    second (chain B) is timed.  Once with the default walk limit (the pass
    turns the path; pointer-jumping rounds precede the chase) and once
    with a walk limit above h (one thread walks it); same forest by
    digests."""
    import torch
    import gen
    L = n // 2
    i = np.arange(L - 1, dtype=np.uint64)
    a = (i << np.uint64(32)) | (i + np.uint64(1))
    g = gen.make_graph("chains", n, np.concatenate([a, a + ((np.uint64(L) << np.uint64(32)) | np.uint64(L))]))
    q = L - 2 - h
    res = {"n": n, "path_steps": h, "what": "delete whose attach path has path_steps steps, on a chain n/2 deep"}
    digests = []
    for name, limit in (("pass", 0), ("walk", 1 << 30)):
        with torch.cuda.stream(stream):
            t = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (g.row_ptr, g.col, g.parent)]
            close = torch.tensor([[0, L - 1], [L, 2 * L - 1]], dtype=torch.int32, device=dev)
            cut_a = torch.tensor([[q, q + 1]], dtype=torch.int32, device=dev)
            cut_b = torch.tensor([[L + q, L + q + 1]], dtype=torch.int32, device=dev)
        f = drsf.Forest(n, *t, inputs_on_device=True, stream=stream.cuda_stream, max_batch=8, walk_limit=limit)
        f.apply(close, drsf.DRSF_INSERT)
        first = f.apply(cut_a, drsf.DRSF_DELETE)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = f.apply(cut_b, drsf.DRSF_DELETE)
        wall = time.perf_counter() - t1
        digests.append([int(x) for x in f.digest()])
        f.close()
        res[name] = {"first_delete_host_finished": first["host_finished"], "delete_ms": round(wall * 1e3, 4),
                     "host_finished": st["host_finished"], "jump_rounds": st["jump_rounds"]}
    res["same_result"] = digests[0] == digests[1]
    assert res["same_result"], "deep chains: the pass and the walk gave different forests"
    log(f"deep chains: {res}")
    return res


def run_batched(nsteps, dev, stream, log, tune, small=None):
    """Batched pattern: 256 independent G(n, 4n) graphs (n = 10^U(3,6)) with
    one batch per graph per step (op and size per graph), all graphs updated
    by one multi-graph apply per step.  The schedule is autotuned: the LDS
    threshold of the small-graph engine (graphs up to it updated whole by one
    workgroup each, beside the kernel sequence for the others; 0 = every
    graph through the kernel sequence), its workgroup size and count, then
    the queued rounds/levels and scan mode.  A/B: the same steps through the
    kernel sequence alone (threshold 0, its schedule tuned the same way);
    both end in the same forest (digests).  Against the same batches applied
    one graph at a time through 256 single-graph contexts."""
    import torch
    import gen
    from paper_2607_20211_amd import drsf
    t0 = time.time()
    wl = gen.batched_workload(256, 2 + nsteps, gen.seed(4, 0, gen.P_GRAPH))
    mg = wl.mg
    ups = int(wl.steps[0][1][-1])
    cap = max(int(e[1][-1]) for e in wl.steps)
    log(f"batched workload: {mg.G} graphs, n={mg.n} m={len(mg.col) // 2}, {ups} updates/step "
        f"({time.time() - t0:.1f}s)")
    d_row = torch.from_numpy(mg.row_ptr).to(dev)
    d_col = torch.from_numpy(mg.col).to(dev)
    d_par = torch.from_numpy(mg.parent).to(dev)
    d_steps = [torch.from_numpy(e).to(dev) for e, _, _ in wl.steps]
    torch.cuda.synchronize()

    def make(th):
        return drsf.MultiForest(mg.n_off, d_row, d_col, d_par, max_batch=cap, stream=stream.cuda_stream,
                                inputs_on_device=True, delta_capacity=(2 + nsteps) * cap + (1 << 20),
                                small_graph_vertices=th)

    def sample(fr):
        fr.apply_multi(d_steps[0], wl.steps[0][1], wl.steps[0][2])

    def run(f):
        for i in range(2):
            st = f.apply_multi(d_steps[i], wl.steps[i][1], wl.steps[i][2])
            assert (st == 0).all()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sts = []
        for i in range(2, 2 + nsteps):
            sts.append(f.apply_multi(d_steps[i], wl.steps[i][1], wl.steps[i][2]))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        rejected = int(sum(int((s != 0).sum()) for s in sts))
        assert rejected == 0, f"batched: {rejected} graph batches rejected"
        return wall, [int(x) for x in f.digest()]

    from paper_2607_20211_amd import autotune
    t0 = time.time()
    if small is not None:
        f, tuning = make(small), {"small_graph_vertices": small, "forced": True}
    elif tune:
        f, tuning = autotune.tune_batched(make, sample, "batched_256_gnm")
    else:
        f, tuning = make(4096), None
    log(f"batched tuning ({time.time() - t0:.1f}s): {tuning}")
    wall, dig = run(f)
    small_graphs = sum(1 for g in mg.graphs if 1 <= g.n <= (tuning or {}).get("small_graph_vertices", 4096))
    f.close()
    # A/B: the kernel sequence alone
    fc = make(0)
    chain_tuning = autotune.tune(fc, sample, "batched_256_gnm_chain", use_cache=False) if tune else None
    wall_chain, dig_chain = run(fc)
    fc.close()
    del d_row, d_col
    log(f"batched: {nsteps} steps in {wall * 1e3:.2f} ms (chain alone {wall_chain * 1e3:.2f} ms), "
        f"same forest: {dig == dig_chain}")
    assert dig == dig_chain, "batched: the small-graph engine and the chain alone end in different forests"
    # the same batches one graph at a time (the plain path), on the first steps
    plain_steps = min(nsteps, 2)
    singles = []
    for g, gr in enumerate(mg.graphs):
        singles.append(drsf.Forest(gr.n, gr.row_ptr, gr.col, gr.parent, max_batch=max(int(wl.b[g]), 1),
                                   stream=stream.cuda_stream,
                                   delta_capacity=(2 + nsteps) * max(int(wl.b[g]), 1) + (1 << 16)))
    local = []
    for i in range(2 + plain_steps):
        e, b_off, ops = wl.steps[i]
        local.append([(np.ascontiguousarray(e[b_off[g]:b_off[g + 1]] - mg.n_off[g]), int(ops[g]))
                      for g in range(mg.G)])
    for i in range(2):
        for g, fs in enumerate(singles):
            fs.apply(*local[i][g])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for i in range(2, 2 + plain_steps):
        for g, fs in enumerate(singles):
            fs.apply(*local[i][g])
    torch.cuda.synchronize()
    wall_plain = (time.perf_counter() - t2) / plain_steps * nsteps
    for fs in singles:
        fs.close()
    log(f"batched: {nsteps} steps in {wall * 1e3:.2f} ms; plain {wall_plain / nsteps * 1e3:.2f} ms/step")
    return {"workload": "256 graphs G(n, 4n), n = 10^U(3,6), b = 10^U(1,4) per graph, op per graph "
                        "and step",
            "graphs": mg.G, "n_total": mg.n, "m_total": int(len(mg.col) // 2),
            "updates_per_step": ups, "steps": nsteps,
            "value": round(ups * nsteps / wall, 1), "unit": "edge updates/s",
            "ms_per_step": round(wall / nsteps * 1e3, 4),
            "small_graphs": small_graphs,
            "chain_alone_ms_per_step": round(wall_chain / nsteps * 1e3, 4),
            "chain_alone_value": round(ups * nsteps / wall_chain, 1),
            "same_forest_as_chain_alone": dig == dig_chain,
            "plain_ms_per_step": round(wall_plain / nsteps * 1e3, 4),
            "plain_value": round(ups * nsteps / wall_plain, 1),
            "speedup_vs_plain": round(wall_plain / wall, 2), "tuning": tuning,
            "chain_alone_tuning": chain_tuning}


def run_batched_small(nsteps, dev, stream, log, G=1024):
    """The batched pattern on small graphs only: G graphs G(n, 4n) with
    n = 10^U(2, 3.5) (up to 3162 vertices), batches of 10^U(1,3) edges, op
    per graph and step.  A/B: the small-graph engine alone (threshold 4096:
    every graph updated whole by one workgroup, no kernel sequence) against
    the kernel sequence alone (threshold 0), same steps, both launch
    schedules at their defaults; both end in the same forest (digests)."""
    import torch
    import gen
    from paper_2607_20211_amd import drsf
    t0 = time.time()
    wl = gen.batched_workload(G, 2 + nsteps, gen.seed(4, 1, gen.P_GRAPH), log_n=(2.0, 3.5), log_b=(1.0, 3.0))
    mg = wl.mg
    cap = max(int(e[1][-1]) for e in wl.steps)
    ups = [int(e[1][-1]) for e in wl.steps]
    log(f"batched small graphs: {mg.G} graphs, n={mg.n} m={len(mg.col) // 2}, {ups[0]} updates in the first step "
        f"({time.time() - t0:.1f}s)")
    d_row, d_col, d_par = (torch.from_numpy(x).to(dev) for x in (mg.row_ptr, mg.col, mg.parent))
    d_steps = [torch.from_numpy(e).to(dev) for e, _, _ in wl.steps]
    torch.cuda.synchronize()
    res = {}
    for name, th in (("engine", 4096), ("chain", 0)):
        f = drsf.MultiForest(mg.n_off, d_row, d_col, d_par, max_batch=cap, stream=stream.cuda_stream,
                             inputs_on_device=True, delta_capacity=(2 + nsteps) * cap + (1 << 20),
                             small_graph_vertices=th)
        for i in range(2):
            assert (f.apply_multi(d_steps[i], wl.steps[i][1], wl.steps[i][2]) == 0).all()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sts = [f.apply_multi(d_steps[i], wl.steps[i][1], wl.steps[i][2]) for i in range(2, 2 + nsteps)]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        assert all((x == 0).all() for x in sts), f"batched small graphs ({name}): batches rejected"
        res[name] = (wall, [int(x) for x in f.digest()])
        f.close()
    same = res["engine"][1] == res["chain"][1]
    assert same, "batched small graphs: the engine and the kernel sequence end in different forests"
    tot = sum(ups[2:])
    out = {"workload": f"{G} graphs G(n, 4n), n = 10^U(2,3.5), b = 10^U(1,3) per graph, op per graph and step",
           "graphs": G, "n_total": mg.n, "m_total": len(mg.col) // 2, "updates_per_step": round(tot / nsteps),
           "steps": nsteps, "engine_ms_per_step": round(res["engine"][0] / nsteps * 1e3, 4),
           "engine_updates_per_s": round(tot / res["engine"][0], 1),
           "chain_ms_per_step": round(res["chain"][0] / nsteps * 1e3, 4),
           "chain_updates_per_s": round(tot / res["chain"][0], 1),
           "speedup": round(res["chain"][0] / res["engine"][0], 2), "same_forest": same}
    log(f"batched small graphs: engine {out['engine_ms_per_step']} ms/step, kernel sequence "
        f"{out['chain_ms_per_step']} ms/step, same forest: {same}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--batch", type=int, default=100_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-pattern measurement (256 graphs per launch)")
    ap.add_argument("--batched-steps", type=int, default=6)
    ap.add_argument("--batched-small", type=int, default=None,
                    help="small-graph threshold of the batched context instead of the tuned one")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the per-op rates at other batch sizes and the deep grid")
    # the served measurement is opt-in for its run time (about two minutes:
    # 10^4 requests at four loads in three modes)
    ap.add_argument("--served", action="store_true",
                    help="run the served-pattern measurement (off by default)")
    ap.add_argument("--no-served", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--served-scale", type=int, default=24)
    ap.add_argument("--served-requests", type=int, default=10_000)
    ap.add_argument("--no-instances", action="store_true",
                    help="skip the several-instance protocol (median, mean, p10/p90)")
    ap.add_argument("--instances", type=int, default=5)
    ap.add_argument("--instance-runs", type=int, default=5)
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch schedule instead of autotuning it first")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after timing, run a plain 512 MiB device copy three times (a known "
                         "byte count for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU runs are not "
                                   "part of it (see DESIGN.md for how the path would shard)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import gen
    from paper_2607_20211_amd import drsf

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    K, W, b = args.steps, args.warmup, args.batch
    scale = args.scale
    t0 = time.time()
    keys = gen.rmat(scale, 16, 0.57, 0.19, 0.19, gen.seed(2, 0, gen.P_GRAPH))
    g = gen.make_graph(f"rmat{scale}", 1 << scale, keys)
    log(f"graph: n={g.n} m={g.m} ({time.time() - t0:.1f}s)")
    nsteps = W + K
    ins = gen.insert_batches(g.n, g.keys, nsteps, b, gen.seed(2, 0, gen.P_INSERT))
    dl = gen.delete_batches(g.n, g.keys, g.parent, nsteps, b, b // 2, gen.seed(2, 0, gen.P_DELETE))
    log(f"batches generated ({time.time() - t0:.1f}s)")

    stream = torch.cuda.current_stream()
    d_row = torch.from_numpy(g.row_ptr).to(dev)
    d_col = torch.from_numpy(g.col).to(dev)
    d_par = torch.from_numpy(g.parent).to(dev)
    d_ins = torch.from_numpy(ins).to(dev)
    d_del = torch.from_numpy(dl).to(dev)
    torch.cuda.synchronize()

    def make(profile):
        return drsf.Forest(g.n, d_row, d_col, d_par, max_batch=b, stream=stream.cuda_stream,
                           inputs_on_device=True, profile=profile,
                           delta_capacity=max(nsteps * b + b, 1 << 20))

    # timed pass: the production configuration (two updates in flight, no
    # events)
    f = make(0)
    torch.cuda.synchronize()
    log(f"context created ({time.time() - t0:.1f}s)")
    tuning = None
    if not args.no_tune:
        from paper_2607_20211_amd import autotune

        def sample(fr):  # the warm-up steps' batches (never the timed ones)
            for i in range(max(1, min(W, 3))):
                fr.apply(d_ins[i], drsf.DRSF_INSERT)
                fr.apply(d_del[i], drsf.DRSF_DELETE)
        tuning = autotune.tune(f, sample, f"rmat{scale}_insert{b}_delete{b}", use_cache=False)
        log(f"tuning: {tuning}")
    for i in range(W):
        f.apply(d_ins[i], drsf.DRSF_INSERT)
        f.apply(d_del[i], drsf.DRSF_DELETE)
    torch.cuda.synchronize()
    # the batches as views, taken before the clock starts
    v_ins = [d_ins[i] for i in range(W + K)]
    v_del = [d_del[i] for i in range(W + K)]

    def run_queued(fr):
        """The K steps with each batch queued behind the one before it (two
        in flight: drsf_apply_async, then drsf_wait for the older); returns
        the wall time and the per-batch statistics."""
        si, sd = [], []
        t = time.perf_counter()
        fr.apply_async(v_ins[W], drsf.DRSF_INSERT)
        for i in range(W, W + K):
            fr.apply_async(v_del[i], drsf.DRSF_DELETE)
            si.append(fr.wait())
            if i + 1 < W + K:
                fr.apply_async(v_ins[i + 1], drsf.DRSF_INSERT)
            sd.append(fr.wait())
        torch.cuda.synchronize()
        return time.perf_counter() - t, si, sd

    wall, st_ins, st_del = run_queued(f)
    digest_timed = [int(x) for x in f.digest()]
    f.close()
    log(f"timed {K} steps in {wall * 1e3:.2f} ms")

    # the same steps one update at a time (drsf_apply: each waits for the
    # last), on a fresh context: the per-op latencies, and the same forest
    fs = make(0)
    if tuning:
        fs.set_tuning(tuning["rounds_queued"], tuning["levels_queued"], tuning["sweep_mode"])
    for i in range(W):
        fs.apply(v_ins[i], drsf.DRSF_INSERT)
        fs.apply(v_del[i], drsf.DRSF_DELETE)
    torch.cuda.synchronize()
    lat_ins, lat_del = [], []
    ts0 = time.perf_counter()
    for i in range(W, W + K):
        ta = time.perf_counter()
        fs.apply(v_ins[i], drsf.DRSF_INSERT)
        tb = time.perf_counter()
        fs.apply(v_del[i], drsf.DRSF_DELETE)
        lat_ins.append(tb - ta)
        lat_del.append(time.perf_counter() - tb)
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - ts0
    same_s = [int(x) for x in fs.digest()] == digest_timed
    fs.close()
    assert same_s, "one update at a time ended in a different forest"
    sequential = {"value": round(2 * b * K / wall_s, 1), "ms_per_step": round(wall_s / K * 1e3, 4),
                  "same_forest": same_s,
                  "what": "the timed steps applied one at a time (each update waits for the one before; "
                          "the per-op latencies below come from this pass)"}
    log(f"sequential: {sequential}")

    # the same steps with batch validation off (drsf_opts.validate_batches =
    # 0: the caller guarantees valid batches, as these are): the same forest
    # (digests), and the latency without the checks
    fu = drsf.Forest(g.n, d_row, d_col, d_par, max_batch=b, stream=stream.cuda_stream, inputs_on_device=True,
                     delta_capacity=max(nsteps * b + b, 1 << 20), validate_batches=False)
    if tuning:
        fu.set_tuning(tuning["rounds_queued"], tuning["levels_queued"], tuning["sweep_mode"])
    for i in range(W):
        fu.apply(d_ins[i], drsf.DRSF_INSERT)
        fu.apply(d_del[i], drsf.DRSF_DELETE)
    torch.cuda.synchronize()
    wall_u, _, _ = run_queued(fu)
    same_u = [int(x) for x in fu.digest()] == digest_timed
    fu.close()
    assert same_u, "validate_batches=0 ended in a different forest"
    unvalidated = {"value": round(2 * b * K / wall_u, 1), "ms_per_step": round(wall_u / K * 1e3, 4),
                   "same_forest": same_u,
                   "what": "the timed steps, queued as timed, on a context with validate_batches = 0 (no "
                           "repeated-pair check, no presence search for inserts; the batches are valid)"}
    log(f"unvalidated: {unvalidated}")

    # profiled pass: the same steps on a fresh context that launches the same
    # kernels one by one with an event between phases, on the stream the
    # kernels run on
    fp = make(1)
    phases_ins, phases_del = [], []
    for i in range(W + K):
        fp.apply(d_ins[i], drsf.DRSF_INSERT)
        if i >= W:
            phases_ins.append(fp.phase_times())
        fp.apply(d_del[i], drsf.DRSF_DELETE)
        if i >= W:
            phases_del.append(fp.phase_times())
    torch.cuda.synchronize()
    fp.close()
    del d_row, d_col

    def mean_phases(lst):
        return {k: float(np.mean([p[k] for p in lst])) for k in lst[0]}

    pi, pd = mean_phases(phases_ins), mean_phases(phases_del)
    # every phase time holds one event record's cost: the empty bracket
    ev_ins, ev_del = pi.pop(drsf.EVENT_BRACKET, 0.0), pd.pop(drsf.EVENT_BRACKET, 0.0)
    t_ins_dev = sum(pi.values()) * 1e-3
    t_del_dev = sum(pd.values()) * 1e-3
    # rooflines of the single-kernel phases with a defined algorithmic byte
    # count; the dominant one (largest time) is "roofline"
    sd = {k: float(np.mean([x[k] for x in st_del])) for k in st_del[0]}
    eb = g.m  # undirected edges, held once in the upper-half store
    # one-kernel phases: the kernel's time is the phase time less the bracket
    kernels = {
        "k_rep_chase": (pd["root_finding"] - ev_del, 12 * g.n + g.n // 8,
                        "root finding: read rep and label, write rep (4 B each per vertex), "
                        "orphan bitmap (1 bit per vertex)"),
        "k_orph_scan": (pd["orphan_scan"] - ev_del,
                        int(4 * sd["orphan_slots"] + g.n // 8 + 40 * sd["num_orphans"]),
                        "orphan scan: 4-B column per adjacency slot, the orphan bitmap "
                        "(1 bit per vertex) once, one 40-B list entry per orphan (the piece of "
                        "orphan neighbours, read only for them, is not counted)"),
    }
    if sd["scan_orphans"] < 0.5:
        kernels["k_sweep_base"] = (pd["store_sweep"] - ev_del, 4 * eb + 4 * (g.n + 1),
                                   "store sweep: 4 B per stored edge slot + 4 B per row offset")
    rooflines = {}
    for name, (ms, nbytes, what) in kernels.items():
        ach = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        rooflines[name] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                           "traffic": measured_traffic(name, f"rmat{scale}_insert{b}_delete{b}"),
                           "kernel": name, "algorithmic_bytes_per_launch": int(nbytes),
                           "avg_launch_ms": round(ms, 4), "bytes": what,
                           "timing": "HIP events around the kernel on its stream, mean over the "
                                     "profiled steps, less an empty two-event bracket"}
    # per-launch medians beside the means (one heavy step can pull a mean up)
    med_del = {k: float(np.median([p[k] - p.get(drsf.EVENT_BRACKET, 0.0) for p in phases_del]))
               for k in phases_del[0]}
    for name, ph in (("k_rep_chase", "root_finding"), ("k_orph_scan", "orphan_scan"),
                     ("k_sweep_base", "store_sweep")):
        if name in rooflines:
            rooflines[name]["median_launch_ms"] = round(med_del[ph], 4)
    dom = max(rooflines, key=lambda k: rooflines[k]["avg_launch_ms"])
    roofline = rooflines[dom]
    phase_share = {"insert": paper_shares(pi, ev_ins), "delete": paper_shares(pd, ev_del),
                   "paper": {"compaction": "10-15% (delete)", "oriented_replacement_edges": "~50%",
                             "path_reversal": "~30% (except SG inserts)"},
                   "mapping": PAPER_GROUPS}

    if args.copy_calibration:
        src = torch.empty(128 << 20, dtype=torch.int32, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 536870912-byte device copies")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        # the oracle is single-threaded C; this thread is pinned to one core
        # for the sample (in-process, no re-exec) and unpinned afterwards
        aff = os.sched_getaffinity(0)
        core = min(aff)
        os.sched_setaffinity(0, {core})
        try:
            t1 = time.perf_counter()
            r1 = oracle.apply(g.n, g.keys, g.parent, ins[0], oracle.INSERT)
            t2 = time.perf_counter()
            oracle.apply(g.n, r1.keys, r1.parent, dl[0], oracle.DELETE)
            t3 = time.perf_counter()
        finally:
            os.sched_setaffinity(0, aff)
        cpu = {"value": round(2 * b / (t3 - t1), 1), "unit": "edge updates/s", "cores": 1,
               "kind": "oracle",
               "sample": f"one insert batch and one delete batch of {b} on the same R-MAT "
                         f"scale {scale} graph (insert {t2 - t1:.2f}s, delete {t3 - t2:.2f}s), "
                         f"single-threaded C oracle pinned to core {core}",
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}

    protocol = None if args.no_instances else run_instances(scale, b, g, args.instances, args.instance_runs,
                                                             dev, stream, log)
    configs = None if args.no_configs else run_configs(g, dev, stream, log)
    batched_small = None if args.no_batched else run_batched_small(args.batched_steps, dev, stream, log)
    batched = None if args.no_batched else run_batched(args.batched_steps, dev, stream, log,
                                                       not args.no_tune, args.batched_small)

    served = None if (args.no_served or not args.served) else run_served(args.served_scale, args.served_requests,
                                                     (0.5, 0.8, 0.95, 1.5), log)

    total_updates = 2 * b * K
    out = {
        "metric": "edge updates/sec (insert, delete) RMAT-22 1e5 batch; served p50/p99 latency",
        "value": round(total_updates / wall, 1),
        "unit": "edge updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(wall / K * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"rmat{scale}_insert{b}_delete{b}", "graph": "R-MAT",
                   "scale": scale, "edge_factor": 16, "abcd": [0.57, 0.19, 0.19, 0.05],
                   "n": g.n, "m": g.m, "batch": b,
                   "step": "one insert batch then one delete batch (50% tree edges)"},
        "insert_updates_per_s": round(b / float(np.mean(lat_ins)), 1),
        "delete_updates_per_s": round(b / float(np.mean(lat_del)), 1),
        "insert_ms": {"mean": round(float(np.mean(lat_ins)) * 1e3, 4),
                      "p50": round(float(np.median(lat_ins)) * 1e3, 4),
                      "max": round(float(np.max(lat_ins)) * 1e3, 4)},
        "delete_ms": {"mean": round(float(np.mean(lat_del)) * 1e3, 4),
                      "p50": round(float(np.median(lat_del)) * 1e3, 4),
                      "max": round(float(np.max(lat_del)) * 1e3, 4)},
        "insert_device_ms_profiled": round(t_ins_dev * 1e3, 4),
        "delete_device_ms_profiled": round(t_del_dev * 1e3, 4),
        "steps_ms": {"insert": [round(x * 1e3, 4) for x in lat_ins],
                     "delete": [round(x * 1e3, 4) for x in lat_del]},
        "batch_stats_insert": {k: float(np.mean([x[k] for x in st_ins])) for k in st_ins[0]},
        "batch_stats_delete": {k: float(np.mean([x[k] for x in st_del])) for k in st_del[0]},
        "phase_ms_insert": {k: round(v, 4) for k, v in pi.items()},
        "phase_ms_delete": {k: round(v, 4) for k, v in pd.items()},
        "event_bracket_ms": {"insert": round(ev_ins, 4), "delete": round(ev_del, 4)},
        "phase_share_vs_paper": phase_share,
        "tuning": tuning,
        "timed_as": "each batch queued behind the one before it (two updates in flight); per-op "
                    "latencies from the sequential pass",
        "sequential": sequential,
        "unvalidated": unvalidated,
        "roofline": roofline,
        "rooflines": rooflines,
        "protocol": protocol,
        "configs": configs,
        "batched": batched,
        "batched_small_graphs": batched_small,
        "served": served,
        "cpu_baseline": cpu,
    }
    f.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
