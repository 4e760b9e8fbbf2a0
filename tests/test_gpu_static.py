"""Static rebuild (drsf_static_forest) against the oracle: component labels
bit-exact (each component's smallest vertex), the forest valid by the
oracle's checker, and breadth-first (every vertex's depth is its distance
from the root).  The parent among equally near neighbours is not unique, so
only these properties are compared."""
import collections

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2607_20211_amd import drsf
    return drsf


def _distances(n, row_ptr, col, roots):
    dist = np.full(n, -1, np.int64)
    q = collections.deque()
    for r in roots:
        dist[r] = 0
        q.append(r)
    while q:
        v = q.popleft()
        for w in col[row_ptr[v]:row_ptr[v + 1]]:
            if dist[w] < 0:
                dist[w] = dist[v] + 1
                q.append(w)
    return dist


def _run(g, what):
    import torch
    drsf = _lib()
    print(f"[case] static {what} n={g.n} m={g.m}", flush=True)
    dev = torch.device("cuda:0")
    row = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    par = torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)
    lab = torch.empty_like(par)
    levels = drsf.drsf_static_forest(g.n, row, col, par, lab)
    torch.cuda.synchronize()
    p, lab = par.cpu().numpy()[:g.n], lab.cpu().numpy()[:g.n]
    ref = oracle.apply(g.n, g.keys, g.parent, np.zeros((0, 2), np.int32), oracle.DELETE)
    assert np.array_equal(lab, ref.label), f"{what}: labels differ"
    rc, msg = oracle.check_forest(g.n, g.keys, p, lab)
    assert rc == 0, f"{what}: checker: {msg}"
    roots = np.flatnonzero(p == np.arange(g.n))
    dist = _distances(g.n, g.row_ptr, g.col, roots)
    depth = np.zeros(g.n, np.int64)
    # depth by walking parents in distance order (parents are one level up)
    order = np.argsort(dist, kind="stable")
    for v in order:
        if p[v] != v:
            depth[v] = depth[p[v]] + 1
    assert np.array_equal(depth, dist), f"{what}: not breadth-first"
    assert levels == int(dist.max()) + 1 if g.n else levels == 0
    return levels


def test_static_sparse_many_components():
    n = 30011
    _run(gen.make_graph("sparse", n, gen.gnm(n, 26000, gen.seed(16, 0, gen.P_GRAPH))), "sparse")


def test_static_rmat16():
    keys = gen.rmat(16, 16, 0.57, 0.19, 0.19, gen.seed(16, 1, gen.P_GRAPH))
    _run(gen.make_graph("rmat16", 1 << 16, keys), "rmat16")


def test_static_grid_and_path():
    keys = gen.grid(256, 256, 3276, gen.seed(16, 2, gen.P_GRAPH))
    levels = _run(gen.make_graph("grid", 256 * 256, keys), "grid")
    assert levels > 256  # deep: the small-frontier levels dominate
    n = 20000
    keys = np.array([(i << 32) | (i + 1) for i in range(n - 1)], np.uint64)
    assert _run(gen.make_graph("path", n, keys), "path") == n


def test_static_edgeless_and_tiny():
    _run(gen.make_graph("empty", 1000, np.zeros(0, np.uint64)), "edgeless")
    _run(gen.make_graph("one", 2, np.array([1], np.uint64)), "one edge")
