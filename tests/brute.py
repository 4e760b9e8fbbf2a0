"""Exhaustive pure-Python reference for tiny D-RSF instances.

Shares nothing with the C oracle: it enumerates every candidate set of
replacement edges instead of running Kruskal, and orients trees from
breadth-first distances instead of a traversal order.  Used only to pin the
oracle on graphs with at most ~7 vertices.

Definitions (problem statement, Sec. I; notation, Sec. II-A; Theorem 1):
F-hat = F - B (delete) or F (insert); the new forest keeps every edge of
F-hat and adds k - l cross edges; among all such sets the chosen one is the
lexicographically smallest by edge key, i.e. the minimum of sum(2^rank) over
candidate edges in increasing key order (unique because powers of two are
distinct); every tree is rooted at its smallest vertex.
"""
from __future__ import annotations

from itertools import combinations


def key(u: int, v: int) -> tuple[int, int]:
    return (u, v) if u < v else (v, u)


def components(n: int, edges) -> list[int]:
    """Smallest vertex of each vertex's component, by breadth-first search."""
    adj = [[] for _ in range(n)]
    for u, v in edges:
        adj[u].append(v)
        adj[v].append(u)
    comp = [-1] * n
    for s in range(n):
        if comp[s] >= 0:
            continue
        comp[s] = s
        frontier = [s]
        while frontier:
            nxt = []
            for x in frontier:
                for w in adj[x]:
                    if comp[w] < 0:
                        comp[w] = s
                        nxt.append(w)
            frontier = nxt
    return comp


def is_forest(n: int, edges) -> bool:
    """|E| = n - #components  <=>  acyclic (for a simple graph)."""
    comp = components(n, edges)
    return len(edges) == n - len(set(comp))


def orient(n: int, forest_edges) -> list[int]:
    """Parent array with each tree rooted at its smallest vertex: the parent
    of v is its unique forest neighbour one step closer to the root."""
    adj = [[] for _ in range(n)]
    for u, v in forest_edges:
        adj[u].append(v)
        adj[v].append(u)
    comp = components(n, forest_edges)
    dist = [-1] * n
    for r in set(comp):
        dist[r] = 0
        frontier = [r]
        while frontier:
            nxt = []
            for x in frontier:
                for w in adj[x]:
                    if dist[w] < 0:
                        dist[w] = dist[x] + 1
                        nxt.append(w)
            frontier = nxt
    parent = list(range(n))
    for v in range(n):
        if dist[v] > 0:
            closer = [w for w in adj[v] if dist[w] == dist[v] - 1]
            assert len(closer) == 1
            parent[v] = closer[0]
    return parent


class Rejected(Exception):
    pass


def apply(n: int, edges, parent, batch, op: str):
    """Returns (edge set of G', parent', label', replacement edges)."""
    E = {key(u, v) for u, v in edges}
    B = []
    for u, v in batch:
        if not (0 <= u < n and 0 <= v < n) or u == v:
            raise Rejected("bad pair")
        B.append(key(u, v))
    if len(set(B)) != len(B):
        raise Rejected("duplicate")
    if op == "insert":
        if any(e in E for e in B):
            raise Rejected("exists")
        E2 = E | set(B)
    else:
        if any(e not in E for e in B):
            raise Rejected("missing")
        E2 = E - set(B)
    T = {key(v, parent[v]) for v in range(n) if parent[v] != v}
    T_hat = T - set(B) if op == "delete" else set(T)
    k = n - len(T_hat)
    ell = len(set(components(n, E2)))
    cand = sorted(E2 - T_hat)
    rank = {e: i for i, e in enumerate(cand)}
    best, best_w = None, None
    for S in combinations(cand, k - ell):
        if not is_forest(n, list(T_hat) + list(S)):
            continue
        w = sum(1 << rank[e] for e in S)
        if best_w is None or w < best_w:
            best, best_w = S, w
    assert best is not None
    forest = list(T_hat) + list(best)
    par = orient(n, forest)
    lab = components(n, forest)
    return E2, par, lab, sorted(best)
