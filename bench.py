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
job (insert + delete) in the production configuration (each update replays
the context's captured HIP graph); insert and delete latencies as seen by
the host; per-phase device times and the roofline of the dominant kernel
(the key-edge sweep of the base edge store) from a second pass over the
same steps that launches the kernels one by one with events between the
phases on the stream the kernels run on; and the CPU oracle timed on a
bounded sample.
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


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    runs (profiles/*.counters.json), or None when the kernel source has
    changed since the counters were taken."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2607_20211_amd", "csrc", "drsf_kernels.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.counters.json")):
        c = json.load(open(path))
        if c.get("kernel") == kernel and c.get("workload") == workload and c.get("source_sha256_16") == h:
            return c["traffic_bytes_per_launch"]
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--batch", type=int, default=100_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    # timed pass: the production configuration (captured update graph, no events)
    f = make(0)
    torch.cuda.synchronize()
    log(f"context created ({time.time() - t0:.1f}s)")
    for i in range(W):
        f.apply(d_ins[i], drsf.DRSF_INSERT)
        f.apply(d_del[i], drsf.DRSF_DELETE)
    torch.cuda.synchronize()
    lat_ins, lat_del = [], []
    t_start = time.perf_counter()
    for i in range(W, W + K):
        ta = time.perf_counter()
        f.apply(d_ins[i], drsf.DRSF_INSERT)
        tb = time.perf_counter()
        f.apply(d_del[i], drsf.DRSF_DELETE)
        tc = time.perf_counter()
        lat_ins.append(tb - ta)
        lat_del.append(tc - tb)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    f.close()
    log(f"timed {K} steps in {wall * 1e3:.2f} ms")

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
    t_ins_dev = sum(pi.values()) * 1e-3
    t_del_dev = sum(pd.values()) * 1e-3
    # dominant kernel: the base key-edge sweep of the delete path
    sweep_ms = pd["key_edge_sweep"]
    eb = g.m  # undirected edges held once in the upper-half store (the base)
    sweep_bytes = 4 * eb + 4 * (g.n + 1)
    achieved = sweep_bytes / (sweep_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic("k_sweep_base", f"rmat{scale}_insert{b}_delete{b}"),
                "kernel": "k_sweep_base", "algorithmic_bytes_per_launch": sweep_bytes,
                "avg_launch_ms": round(sweep_ms, 4)}

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
        t1 = time.perf_counter()
        r1 = oracle.apply(g.n, g.keys, g.parent, ins[0], oracle.INSERT)
        t2 = time.perf_counter()
        oracle.apply(g.n, r1.keys, r1.parent, dl[0], oracle.DELETE)
        t3 = time.perf_counter()
        cpu = {"value": round(2 * b / (t3 - t1), 1), "unit": "edge updates/s", "cores": 1,
               "kind": "oracle",
               "sample": f"one insert batch and one delete batch of {b} on the same R-MAT "
                         f"scale {scale} graph (insert {t2 - t1:.2f}s, delete {t3 - t2:.2f}s), "
                         f"single-threaded C oracle"}

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
        "phase_ms_insert": {k: round(v, 4) for k, v in pi.items()},
        "phase_ms_delete": {k: round(v, 4) for k, v in pd.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    f.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
