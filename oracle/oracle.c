/*
 * CPU oracle for batch-dynamic rooted spanning forest (D-RSF).
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  The GPU product path never calls
 * it and shares no code with it.
 *
 * Plain, single-threaded, deliberately unoptimised C.  It computes the
 * deterministic result of one batch update with the rule used throughout
 * this project:
 *   - replacement edges are chosen by Kruskal's rule over the key edges in
 *     increasing key (min(u,v), max(u,v)) order, on top of the surviving
 *     forest edges (so the lowest-key cross edge hooks two trees);
 *   - every tree of the new forest is rooted at the smallest vertex id of
 *     its component, and a root is its own parent.
 * Sources:
 *   - problem statement (D-RSF box, Sec. I): input G, rooted spanning
 *     forest F, batch B, op in {insert, delete}; output a rooted spanning
 *     forest F' of G' = G + B or G - B;
 *   - notation (Sec. II-A): F-hat = F - B for delete and F for insert; key
 *     edges M = B for insert and M = E(G) - E(F) - B for delete; rep[v] is
 *     the root of v's tree in F-hat; (u,v) in M is a cross edge iff
 *     rep[u] != rep[v]; replacement edges are k - l cross edges joining the
 *     k trees of F-hat into the l components of G';
 *   - Algorithm 1 and Theorem 1: F' is F-hat plus the replacement edges, so
 *     every surviving tree edge stays in F' and exactly l roots remain.
 * Any correct method with the same hooking and root rules produces the same
 * parent array, because with distinct keys the spanning forest "F-hat edges
 * first, then key order" is unique, and a tree with a fixed root has exactly
 * one parent array.
 *
 * Edge keys: {u, v} with u < v is (u << 32) | v.  Graphs are passed as
 * sorted arrays of unique keys.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

enum { OR_OK = 0, OR_E_ARG = -1, OR_E_NOMEM = -2, OR_E_FOREST = -3, OR_E_BATCH = -4 };
enum { OR_INSERT = 0, OR_DELETE = 1 };

typedef struct {
    int64_t k;                 /* trees in F-hat */
    int64_t ell;               /* components of G' (= trees of F') */
    int64_t n_key;             /* |M| */
    int64_t n_cross;           /* key edges with rep[u] != rep[v] */
    int64_t n_repl;            /* |E_r| = k - ell */
    int64_t n_tree_deleted;    /* tree edges of F in B (delete) */
    int64_t n_parent_changed;  /* #{v : parent'[v] != parent[v]} */
    int64_t n_label_changed;   /* #{v : label'[v] != label[v]} (if label given) */
    int64_t m_out;             /* |E(G')| */
} oracle_stats;

static uint64_t key_of(int64_t a, int64_t b) {
    uint64_t lo = (uint64_t)(a < b ? a : b), hi = (uint64_t)(a < b ? b : a);
    return (lo << 32) | hi;
}

static int cmp_u64(const void *x, const void *y) {
    uint64_t a = *(const uint64_t *)x, b = *(const uint64_t *)y;
    return a < b ? -1 : a > b;
}

static int has_key(const uint64_t *keys, int64_t m, uint64_t k) {
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (keys[mid] < k) lo = mid + 1; else hi = mid;
    }
    return lo < m && keys[lo] == k;
}

/* ---- union-find (union by size, path halving): a textbook structure ---- */
typedef struct { int32_t *up; int32_t *size; } uf_t;

static int uf_init(uf_t *u, int32_t n) {
    u->up = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    u->size = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!u->up || !u->size) return -1;
    for (int32_t i = 0; i < n; i++) { u->up[i] = i; u->size[i] = 1; }
    return 0;
}
static void uf_free(uf_t *u) { free(u->up); free(u->size); }
static int32_t uf_find(uf_t *u, int32_t x) {
    while (u->up[x] != x) { u->up[x] = u->up[u->up[x]]; x = u->up[x]; }
    return x;
}
/* returns 1 if a and b were in different sets */
static int uf_union(uf_t *u, int32_t a, int32_t b) {
    a = uf_find(u, a); b = uf_find(u, b);
    if (a == b) return 0;
    if (u->size[a] < u->size[b]) { int32_t t = a; a = b; b = t; }
    u->up[b] = a;
    u->size[a] += u->size[b];
    return 1;
}

/* sorted-set difference a \ b into out; returns |out| */
static int64_t set_minus(const uint64_t *a, int64_t na, const uint64_t *b, int64_t nb,
                         uint64_t *out) {
    int64_t i = 0, j = 0, w = 0;
    while (i < na) {
        while (j < nb && b[j] < a[i]) j++;
        if (j < nb && b[j] == a[i]) { i++; continue; }
        out[w++] = a[i++];
    }
    return w;
}

/* sorted-set union (disjoint inputs) into out; returns |out| */
static int64_t set_merge(const uint64_t *a, int64_t na, const uint64_t *b, int64_t nb,
                         uint64_t *out) {
    int64_t i = 0, j = 0, w = 0;
    while (i < na || j < nb) {
        if (j >= nb || (i < na && a[i] < b[j])) out[w++] = a[i++];
        else out[w++] = b[j++];
    }
    return w;
}

/*
 * One batch update.  Inputs: n vertices; G as sorted unique keys (m of
 * them); parent[] of a rooted spanning forest of G whose trees span G's
 * components; the batch as b (u, v) pairs; op.  label may be NULL (then
 * n_label_changed is not computed).  scan_all = 1 makes an insert use
 * M = E(G') - E(F) instead of B (both give the same result when F spans the
 * components of G; this is a self-check).
 * Outputs: gkeys_out (capacity m + b), parent_out, label_out (label = root =
 * smallest vertex of the component), stats (may be NULL).
 * Returns OR_OK, or OR_E_BATCH / OR_E_ARG / OR_E_FOREST / OR_E_NOMEM with
 * outputs untouched.
 */
int oracle_apply(int32_t n, const uint64_t *gkeys, int64_t m, const int32_t *parent,
                 const int32_t *label, const int32_t *batch, int64_t b, int op, int scan_all,
                 uint64_t *gkeys_out, int64_t *m_out, int32_t *parent_out,
                 int32_t *label_out, oracle_stats *st) {
    if (n < 0 || m < 0 || b < 0 || (op != OR_INSERT && op != OR_DELETE)) return OR_E_ARG;
    int rc = OR_OK;
    uint64_t *bk = NULL, *gnew = NULL, *tf = NULL, *that = NULL, *mkeys = NULL;
    int32_t *adj_ptr = NULL, *adj = NULL, *stack = NULL, *rep = NULL;
    int32_t *par2 = NULL, *lab2 = NULL;
    uint64_t *er = NULL;
    uf_t uf = {0, 0};
    oracle_stats s;
    memset(&s, 0, sizeof s);

    /* Step 1: validate and normalise B (the paper assumes a valid batch; a
     * batch with a self-loop, an out-of-range id, a repeated edge, an insert
     * of an existing edge or a delete of a missing edge is rejected whole). */
    bk = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(b > 0 ? b : 1));
    if (!bk) { rc = OR_E_NOMEM; goto done; }
    for (int64_t i = 0; i < b; i++) {
        int32_t u = batch[2 * i], v = batch[2 * i + 1];
        if (u < 0 || v < 0 || u >= n || v >= n || u == v) { rc = OR_E_BATCH; goto done; }
        bk[i] = key_of(u, v);
    }
    qsort(bk, (size_t)b, sizeof(uint64_t), cmp_u64);
    for (int64_t i = 1; i < b; i++)
        if (bk[i] == bk[i - 1]) { rc = OR_E_BATCH; goto done; }
    for (int64_t i = 0; i < b; i++) {
        int present = has_key(gkeys, m, bk[i]);
        if ((op == OR_INSERT && present) || (op == OR_DELETE && !present)) {
            rc = OR_E_BATCH; goto done;
        }
    }

    /* Step 2: G' = G + B or G - B (problem statement). */
    gnew = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m + b > 0 ? m + b : 1));
    if (!gnew) { rc = OR_E_NOMEM; goto done; }
    int64_t mnew = op == OR_INSERT ? set_merge(gkeys, m, bk, b, gnew)
                                   : set_minus(gkeys, m, bk, b, gnew);

    /* Step 3: tree edges of F, and F-hat = F - B (delete) or F (insert). */
    for (int32_t v = 0; v < n; v++)
        if (parent[v] < 0 || parent[v] >= n) { rc = OR_E_FOREST; goto done; }
    int64_t nt = 0;
    for (int32_t v = 0; v < n; v++) nt += parent[v] != v;
    tf = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nt > 0 ? nt : 1));
    that = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nt > 0 ? nt : 1));
    if (!tf || !that) { rc = OR_E_NOMEM; goto done; }
    {
        int64_t w = 0;
        for (int32_t v = 0; v < n; v++)
            if (parent[v] != v) tf[w++] = key_of(v, parent[v]);
    }
    qsort(tf, (size_t)nt, sizeof(uint64_t), cmp_u64);
    for (int64_t i = 1; i < nt; i++)
        if (tf[i] == tf[i - 1]) { rc = OR_E_FOREST; goto done; } /* 2-cycle */
    for (int64_t i = 0; i < nt; i++)
        if (!has_key(gkeys, m, tf[i])) { rc = OR_E_FOREST; goto done; }
    int64_t nthat;
    if (op == OR_DELETE) {
        nthat = set_minus(tf, nt, bk, b, that);
        s.n_tree_deleted = nt - nthat;
    } else {
        memcpy(that, tf, sizeof(uint64_t) * (size_t)nt);
        nthat = nt;
    }

    /* Step 4: key edges M (Sec. II-A): B for insert, E(G') - E(F-hat) for
     * delete, i.e. every surviving non-tree edge. */
    int64_t nm;
    if (op == OR_INSERT && !scan_all) {
        mkeys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(b > 0 ? b : 1));
        if (!mkeys) { rc = OR_E_NOMEM; goto done; }
        memcpy(mkeys, bk, sizeof(uint64_t) * (size_t)b);
        nm = b;
    } else {
        mkeys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(mnew > 0 ? mnew : 1));
        if (!mkeys) { rc = OR_E_NOMEM; goto done; }
        nm = set_minus(gnew, mnew, that, nthat, mkeys);
    }
    s.n_key = nm;

    /* Step 5: union every edge of F-hat; rep[v] is then v's tree in F-hat. */
    if (uf_init(&uf, n)) { rc = OR_E_NOMEM; goto done; }
    for (int64_t i = 0; i < nthat; i++)
        if (!uf_union(&uf, (int32_t)(that[i] >> 32), (int32_t)(uint32_t)that[i])) {
            rc = OR_E_FOREST; goto done; /* F-hat has a cycle */
        }
    s.k = n - nthat;
    rep = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!rep) { rc = OR_E_NOMEM; goto done; }
    for (int32_t v = 0; v < n; v++) rep[v] = uf_find(&uf, v);
    for (int64_t i = 0; i < nm; i++)
        s.n_cross += rep[mkeys[i] >> 32] != rep[(uint32_t)mkeys[i]];

    /* Step 6: Kruskal over M in increasing key order: a key edge joining two
     * different trees becomes a replacement edge and merges them. */
    er = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nm > 0 ? nm : 1));
    if (!er) { rc = OR_E_NOMEM; goto done; }
    int64_t nr = 0;
    for (int64_t i = 0; i < nm; i++)
        if (uf_union(&uf, (int32_t)(mkeys[i] >> 32), (int32_t)(uint32_t)mkeys[i]))
            er[nr++] = mkeys[i];
    s.n_repl = nr;

    /* Step 7: undirected F' = F-hat + E_r (Theorem 1), as adjacency lists. */
    adj_ptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * (nthat + nr) + 1));
    stack = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    par2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    lab2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!adj_ptr || !adj || !stack || !par2 || !lab2) { rc = OR_E_NOMEM; goto done; }
    for (int pass = 0; pass < 2; pass++) {
        const uint64_t *src = pass == 0 ? that : er;
        int64_t cnt = pass == 0 ? nthat : nr;
        for (int64_t i = 0; i < cnt; i++) {
            adj_ptr[(src[i] >> 32) + 1]++;
            adj_ptr[(uint32_t)src[i] + 1]++;
        }
    }
    for (int32_t v = 0; v < n; v++) adj_ptr[v + 1] += adj_ptr[v];
    {
        int32_t *fill = stack; /* reuse as a cursor array */
        for (int32_t v = 0; v < n; v++) fill[v] = adj_ptr[v];
        for (int pass = 0; pass < 2; pass++) {
            const uint64_t *src = pass == 0 ? that : er;
            int64_t cnt = pass == 0 ? nthat : nr;
            for (int64_t i = 0; i < cnt; i++) {
                int32_t u = (int32_t)(src[i] >> 32), v = (int32_t)(uint32_t)src[i];
                adj[fill[u]++] = v;
                adj[fill[v]++] = u;
            }
        }
    }

    /* Step 8: root every tree at its smallest vertex: visit r = 0, 1, ...
     * and, from each unvisited r, give every newly reached vertex the vertex
     * it was reached from as parent (iterative, trees may be deep). */
    for (int32_t v = 0; v < n; v++) par2[v] = -1;
    int64_t roots = 0;
    for (int32_t r = 0; r < n; r++) {
        if (par2[r] >= 0) continue;
        roots++;
        par2[r] = r;
        lab2[r] = r;
        int64_t top = 0;
        stack[top++] = r;
        while (top > 0) {
            int32_t x = stack[--top];
            for (int32_t e = adj_ptr[x]; e < adj_ptr[x + 1]; e++) {
                int32_t w = adj[e];
                if (par2[w] < 0) { par2[w] = x; lab2[w] = r; stack[top++] = w; }
            }
        }
    }
    s.ell = roots;
    if (roots != s.k - nr) { rc = OR_E_FOREST; goto done; } /* Theorem 1 */

    /* Step 9: outputs and statistics. */
    for (int32_t v = 0; v < n; v++) {
        s.n_parent_changed += par2[v] != parent[v];
        if (label) s.n_label_changed += lab2[v] != label[v];
    }
    s.m_out = mnew;
    if (gkeys_out) memcpy(gkeys_out, gnew, sizeof(uint64_t) * (size_t)mnew);
    if (m_out) *m_out = mnew;
    if (parent_out) memcpy(parent_out, par2, sizeof(int32_t) * (size_t)n);
    if (label_out) memcpy(label_out, lab2, sizeof(int32_t) * (size_t)n);
    if (st) *st = s;

done:
    free(bk); free(gnew); free(tf); free(that); free(mkeys); free(rep); free(er);
    free(adj_ptr); free(adj); free(stack); free(par2); free(lab2);
    uf_free(&uf);
    return rc;
}

/*
 * Forest checker (validity of a rooted spanning forest of a graph).
 * Checks, in order: every parent id is in range; every parent edge is an
 * edge of the graph; following parents from any vertex reaches a root
 * (parent[r] == r) without a cycle; no graph edge joins two different
 * trees and every tree is connected through graph edges, so the trees are
 * exactly the components found by a breadth-first search of the graph;
 * optionally every root is the smallest vertex of its component; optionally
 * label[v] equals the root of v's tree.  Returns 0 if valid, else a negative
 * code and a message.
 */
int oracle_check_forest(int32_t n, const uint64_t *gkeys, int64_t m, const int32_t *parent,
                        const int32_t *label, int require_min_root, char *msg, int msglen) {
    int rc = 0;
    int32_t *root = NULL, *path = NULL, *comp = NULL, *queue = NULL, *ptr = NULL, *nbr = NULL;
    int8_t *state = NULL;
#define FAIL(code, ...) do { if (msg) snprintf(msg, (size_t)msglen, __VA_ARGS__); rc = (code); goto out; } while (0)
    for (int32_t v = 0; v < n; v++)
        if (parent[v] < 0 || parent[v] >= n) FAIL(-1, "parent[%d]=%d out of range", v, parent[v]);
    for (int32_t v = 0; v < n; v++)
        if (parent[v] != v && !has_key(gkeys, m, key_of(v, parent[v])))
            FAIL(-2, "parent edge (%d,%d) not in graph", v, parent[v]);
    root = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    path = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    state = (int8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!root || !path || !state) FAIL(-9, "out of memory");
    for (int32_t v = 0; v < n; v++) {
        if (state[v] == 2) continue;
        int64_t len = 0;
        int32_t x = v, r;
        for (;;) {
            if (state[x] == 2) { r = root[x]; break; }
            if (state[x] == 1) FAIL(-3, "cycle through vertex %d", x);
            state[x] = 1;
            path[len++] = x;
            if (parent[x] == x) { r = x; break; }
            x = parent[x];
        }
        for (int64_t i = 0; i < len; i++) { state[path[i]] = 2; root[path[i]] = r; }
    }
    /* components of the graph by breadth-first search from ascending ids */
    ptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    comp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!ptr || !nbr || !comp || !queue) FAIL(-9, "out of memory");
    for (int64_t i = 0; i < m; i++) { ptr[(gkeys[i] >> 32) + 1]++; ptr[(uint32_t)gkeys[i] + 1]++; }
    for (int32_t v = 0; v < n; v++) ptr[v + 1] += ptr[v];
    for (int32_t v = 0; v < n; v++) queue[v] = ptr[v];
    for (int64_t i = 0; i < m; i++) {
        int32_t u = (int32_t)(gkeys[i] >> 32), v = (int32_t)(uint32_t)gkeys[i];
        nbr[queue[u]++] = v;
        nbr[queue[v]++] = u;
    }
    for (int32_t v = 0; v < n; v++) comp[v] = -1;
    for (int32_t s = 0; s < n; s++) {
        if (comp[s] >= 0) continue;
        int64_t h = 0, t = 0;
        comp[s] = s;
        queue[t++] = s;
        while (h < t) {
            int32_t x = queue[h++];
            for (int32_t e = ptr[x]; e < ptr[x + 1]; e++)
                if (comp[nbr[e]] < 0) { comp[nbr[e]] = s; queue[t++] = nbr[e]; }
        }
    }
    /* trees == components: a tree lies inside one component because its
     * edges are graph edges; a component lies inside one tree iff no graph
     * edge joins two trees. */
    for (int64_t i = 0; i < m; i++) {
        int32_t u = (int32_t)(gkeys[i] >> 32), v = (int32_t)(uint32_t)gkeys[i];
        if (root[u] != root[v]) FAIL(-4, "edge (%d,%d) joins trees rooted at %d and %d", u, v, root[u], root[v]);
    }
    for (int32_t v = 0; v < n; v++) {
        if (comp[root[v]] != comp[v]) FAIL(-4, "vertex %d and its root %d in different components", v, root[v]);
        if (require_min_root && root[v] != comp[v])
            FAIL(-5, "vertex %d: root %d is not the smallest vertex %d of its component", v, root[v], comp[v]);
        if (label && label[v] != root[v]) FAIL(-6, "label[%d]=%d but root is %d", v, label[v], root[v]);
    }
out:
    free(root); free(path); free(state); free(ptr); free(nbr); free(comp); free(queue);
    return rc;
#undef FAIL
}
