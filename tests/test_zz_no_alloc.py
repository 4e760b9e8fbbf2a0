"""The allocation-free static rebuild (drsf_static_forest_noalloc), through
the C ABI, against the allocating entry point on the same inputs: labels
bit-exact, the same number of breadth-first levels, each vertex's depth its
breadth-first distance, and the oracle's checker passing (the parent among
equally near neighbours is not unique).  Two calls in a row on the shared
per-device scratch, the second on a smaller graph, so that what the first
left there must not leak into the second; a graph beyond the scratch is
refused before any work."""
import numpy as np
import pytest

import gen
import oracle
from test_gpu_static import _distances

pytestmark = pytest.mark.gpu


def _both(g, what):
    import torch
    from paper_2607_20211_amd import drsf
    print(f"[case] noalloc {what} n={g.n} m={g.m}", flush=True)
    dev = torch.device("cuda:0")
    row = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    out = {}
    for name, fn in (("alloc", drsf.drsf_static_forest), ("noalloc", drsf.drsf_static_forest_noalloc)):
        par = torch.full((g.n,), -7, dtype=torch.int32, device=dev)
        lab = torch.full((g.n,), -7, dtype=torch.int32, device=dev)
        levels = fn(g.n, row, col, par, lab)
        torch.cuda.synchronize()
        out[name] = (par.cpu().numpy(), lab.cpu().numpy(), levels)
    pa, la, lva = out["alloc"]
    pn, ln, lvn = out["noalloc"]
    assert np.array_equal(ln, la), f"{what}: labels differ from the allocating entry point"
    assert lvn == lva, f"{what}: levels {lvn} != {lva}"
    ref = oracle.apply(g.n, g.keys, g.parent, np.zeros((0, 2), np.int32), oracle.DELETE)
    assert np.array_equal(ln, ref.label)
    rc, msg = oracle.check_forest(g.n, g.keys, pn, ln)
    assert rc == 0, f"{what}: checker: {msg}"
    roots = np.flatnonzero(pn == np.arange(g.n))
    assert np.array_equal(roots, np.flatnonzero(pa == np.arange(g.n)))
    dist = _distances(g.n, g.row_ptr, g.col, roots)
    depth = np.zeros(g.n, np.int64)
    for v in np.argsort(dist, kind="stable"):
        if pn[v] != v:
            depth[v] = depth[pn[v]] + 1
    assert np.array_equal(depth, dist), f"{what}: not breadth-first"


def test_noalloc_matches_allocating_entry_point_twice_shrinking():
    big = gen.make_graph("rmat", 1 << 16, gen.rmat(16, 16, 0.57, 0.19, 0.19, gen.seed(17, 0, gen.P_GRAPH)))
    small = gen.make_graph("grid", 60 * 70, gen.grid(60, 70, 400, gen.seed(17, 1, gen.P_GRAPH)))
    _both(big, "first call, R-MAT 16")
    _both(small, "second call, smaller grid")
    n = 3000
    path = np.array([(i << 32) | (i + 1) for i in range(n - 1)], np.uint64)
    _both(gen.make_graph("path", n, np.union1d(path, gen.gnm(n, 50, 3))), "third call, path with chords")


def test_noalloc_refuses_a_graph_beyond_its_scratch():
    import torch
    from paper_2607_20211_amd import drsf
    dev = torch.device("cuda:0")
    n = 16
    row = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    row[n] = 20_000_000  # 8 nnz bytes alone exceed the 64 MiB scratch; col is never read
    col = torch.zeros(4, dtype=torch.int32, device=dev)
    par = torch.empty(n, dtype=torch.int32, device=dev)
    lab = torch.empty(n, dtype=torch.int32, device=dev)
    with pytest.raises(drsf.DrsfError) as e:
        drsf.drsf_static_forest_noalloc(n, row, col, par, lab)
    assert e.value.code == drsf.DRSF_E_CAPACITY
