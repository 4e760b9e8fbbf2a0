/*
 * drsf.h — batch-dynamic rooted spanning forest (D-RSF) on AMD MI355X (gfx950).
 *
 * C ABI of libdrsf.so.  Plain pointers and sizes only.
 *
 * The problem (D-RSF box, Sec. I of "Fully Dynamic Rooted Spanning Tree on
 * GPU"): given an undirected graph G, a rooted spanning forest F of G, a
 * batch B of edges and op in {insert, delete}, produce a rooted spanning
 * forest F' of G' = G + B (insert) or G - B (delete).  The library keeps G
 * and F resident in device memory across calls and repairs F instead of
 * rebuilding it (Algorithm 1): every tree edge that survives the batch stays
 * in F' (Theorem 1).
 *
 * Deterministic rules, so that results are reproducible bit for bit:
 *   - replacement edges: among the cross edges (Sec. II-A) the lowest key
 *     (min(u,v), max(u,v)) hooks two trees, i.e. the replacement edges are
 *     the Kruskal choice in increasing key order on top of F - B;
 *   - roots: every tree is rooted at the smallest vertex id of its
 *     component, and a root is its own parent (parent[r] == r, as in the
 *     cut step of Algorithm 1).
 * label[v] is the root of v's tree, i.e. the smallest vertex of v's
 * connected component; the same call therefore also maintains connected
 * components under insertions and deletions (Sec. I, contributions).
 *
 * Conventions for every call:
 *   - vertex ids are 0-based int32 in [0, n); n < 2^31;
 *   - inputs are owned by the caller and copied; nothing is retained;
 *   - "host" pointers are ordinary CPU memory, "device" pointers are HIP
 *     device memory on the context's device; which one an input is follows
 *     drsf_opts.inputs_on_device;
 *   - outputs exposed through drsf_view are device memory owned by the
 *     context, valid until the next drsf_apply / drsf_restore / drsf_destroy
 *     on that context;
 *   - all device work, create's included, is queued on drsf_opts.stream.
 *     NULL: a stream owned by the context, created blocking, so that its
 *     work is ordered after work queued earlier on the null (legacy
 *     default) stream — torch's default stream is that stream;
 *   - device inputs (inputs_on_device) must be fully written before the
 *     call's first read of them, which is queued on that stream: write them
 *     with work queued earlier on the same stream (or, for a context-owned
 *     stream, on the null stream), or finish their writes (synchronise the
 *     writing stream, or the device) before the call.  Writes on any other
 *     stream are not waited for.  The library never writes caller inputs;
 *     when they may be written again is stated per call;
 *   - every call returns a drsf_status; on failure drsf_last_error() gives a
 *     message, and a rejected batch leaves the state unchanged;
 *   - one context must not be used from two host threads at once; distinct
 *     contexts are independent.
 */
#ifndef DRSF_H
#define DRSF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { DRSF_INSERT = 0, DRSF_DELETE = 1 } drsf_op;

typedef enum {
    DRSF_OK = 0,
    DRSF_E_ARG = -1,      /* bad argument (null pointer, negative size, bad CSR) */
    DRSF_E_NOMEM = -2,    /* device or host allocation failed */
    DRSF_E_FOREST = -3,   /* create: parent[] is not a rooted spanning forest of G */
    DRSF_E_BATCH = -4,    /* apply: invalid batch (self-loop, id out of range,
                             repeated edge, insert of an existing edge, delete of a
                             missing edge); nothing was changed */
    DRSF_E_CAPACITY = -5, /* batch larger than drsf_opts.max_batch, inserts beyond
                             drsf_opts.delta_capacity in one batch, or graph too large */
    DRSF_E_DEVICE = -6,   /* HIP runtime error, or an internal bound was exceeded */
    DRSF_E_STATE = -7,    /* call not valid in the context's current state */
    DRSF_E_BUDGET = -8    /* server: the graph does not fit the memory budget */
} drsf_status;

typedef struct drsf_ctx drsf_ctx;

typedef struct {
    void *stream;            /* hipStream_t for all device work; NULL = context-owned */
    int inputs_on_device;    /* 0: CSR/parent/batch pointers are host memory;
                                1: they are device memory */
    int validate_forest;     /* create: 1 (default) checks that parent[] is a rooted
                                spanning forest whose trees span G's components */
    int profile;             /* 1: launch the update's kernels one by one with an
                                event between phases (drsf_phase_times) */
    int64_t max_batch;       /* largest batch accepted by apply; 0 = 1 << 20 */
    int64_t delta_capacity;  /* inserted edges held in the inserted-edge list; an
                                insert that would overflow it first merges the list
                                into the base store (and drops deleted entries):
                                O(|E|) work, amortised over the list; 0 = automatic
                                (max(4 max_batch, |E| / 8, 2^20)) */
    int sweep_mode;          /* delete key-edge scan: 0 (default) per batch, the
                                orphans' adjacency (each orphan counted with 8
                                extra slots) when it holds at most as many
                                slots as the store, else the whole store; 1:
                                always the whole store (Sec. II-A as written) */
    int rounds_queued;       /* full-grid hooking rounds (Alg. 2, phase 1)
                                queued in the update's kernel sequence; later
                                rounds run in one workgroup while at most 4096
                                cross edges are live, else host-driven
                                launches finish them; 0 = chosen by the
                                library: 2, raised (up to 12) to what an
                                update that the host had to finish needed */
    int levels_queued;       /* super-forest search levels placed in the graph;
                                0 = chosen by the library: 4, raised (up to
                                12) likewise, and once an update needed more
                                than 12 the super-forest's Euler tour is
                                queued after them (it skips itself when the
                                search sufficed) (max 12) */
    int reverse_mode;        /* path reversal: 0 (default) one thread walks each
                                path; 1: Euler tour of F-hat with list ranking,
                                start/finish times and the interval test
                                (Alg. 3, ReversePathsEulerTour; F-hat's child
                                lists come from this library's radix sort);
                                needs about 56 bytes per vertex more device
                                memory.  Results are identical. */
    int replacement_mode;    /* replacement edges: 0 (default) hooking rounds on
                                every cross edge (Alg. 2); 1: on the supergraph
                                (Sec. III-A): the cross edges reduced to the
                                lowest key per pair of trees of F-hat by a radix
                                sort, then the hooking rounds on those; launched
                                kernel by kernel with two host reads of sizes;
                                needs about 24 bytes per cross-edge slot more
                                device memory.  Results are identical. */
    /* Device allocator hooks, so that a caller can route the context's device
     * memory through its own allocator (torch's caching allocator, a pool):
     * when dev_alloc is non-NULL every device allocation of the context and
     * of its snapshots is dev_alloc(bytes, alloc_user) and is released with
     * dev_free(ptr, alloc_user) (dev_free must then be non-NULL).  dev_alloc
     * returns device memory on the context's device, aligned to at least
     * 256 bytes, or NULL on failure, which the calling function reports as
     * DRSF_E_NOMEM after releasing what it had allocated.  A block is
     * released only when no queued work of the context uses it any more
     * (the context's stream has been synchronised), so a stream-ordered
     * allocator may reuse it at once.  Pinned host staging memory is always
     * allocated by the library itself.  NULL (default): hipMalloc/hipFree. */
    void *(*dev_alloc)(size_t bytes, void *alloc_user);
    void (*dev_free)(void *ptr, void *alloc_user);
    void *alloc_user;
    int small_graph_vertices;  /* multi-graph contexts: graphs with at most
                                this many vertices (<= 16384; 0 = none, the
                                default) are kept apart from the edge store
                                and updated whole by one workgroup each, with
                                the forest held in LDS, taken from a device
                                work queue by a persistent kernel that runs
                                beside the kernel sequence updating the other
                                graphs.  Results are identical. */
    int small_threads;       /* workgroup size of that kernel: 256, 512 or
                                1024; 0 = 512 */
    int validate_batches;    /* 1 (default): every batch is checked (ids in
                                range, no self-loop, no repeated pair, insert
                                of an absent / delete of a present edge) and a
                                graph whose batch fails is rejected unchanged
                                (DRSF_E_BATCH).  0: the caller guarantees
                                valid batches; the repeated-pair check and the
                                inserts' presence search are skipped (ids are
                                still range-checked and self-loops and deletes
                                of absent edges still rejected, so no input
                                can make a kernel read out of bounds); an
                                invalid batch then leaves the context in an
                                unspecified but safe state.  The small-graph
                                engine checks its batches either way. */
    int launch_mode;         /* 1: an update replays a HIP graph captured
                                once per update kind (less host time per
                                update, a few microseconds more on the device
                                between updates); 2: its kernels are launched
                                one by one, its control block passed with the
                                first; 0 (default): 2 for a one-graph context,
                                1 for several graphs (whose updates launch
                                more, shorter kernels).  An update queued
                                behind a running one, a profiled one and one
                                on the supergraph are always launched kernel
                                by kernel.  Results are identical. */
    int walk_limit;          /* path reversal (reverse_mode 0): one thread
                                walks a path of at most this many steps; a
                                longer path is turned after the update's
                                kernel sequence by a pointer-doubling pass
                                over all vertices that the host launches
                                (drsf_view.host_finished bit 2), about
                                log2(path length) kernels, with 13 bytes per
                                vertex more device memory allocated at the
                                first such path.  0 = 1024 (default); must be
                                >= 0.  Results are identical. */
} drsf_opts;

/* Fills *opts with the defaults described above. */
void drsf_default_opts(drsf_opts *opts);

/*
 * Result of the last apply.  parent and label are DEVICE pointers owned by
 * the context (int32[n]).  Counters describe the last batch: num_key_cross
 * is the number of cross edges found among the key edges (Sec. II-A),
 * num_replacement = |E_r| = k - l (Theorem 1), num_pieces the trees of
 * F-hat that the batch touched, num_paths the reversed paths (Algorithm 1,
 * ReversePaths).
 */
typedef struct {
    const int32_t *parent;
    const int32_t *label;
    int32_t n;
    int64_t num_edges;        /* |E(G')| */
    int64_t num_key_cross;
    int64_t num_replacement;
    int64_t num_pieces;
    int64_t num_paths;
    int64_t num_orphans;      /* delete: vertices cut off from their old root */
    int64_t orphan_slots;     /* delete: adjacency entries of those vertices */
    int32_t scan_orphans;     /* delete: 1 if the key-edge scan covered only the
                                 orphans' adjacency, 0 if the whole store */
    int32_t host_finished;    /* 0 if the queued kernel sequence finished the
                                 update; else host-driven launches finished it:
                                 bit 0 set when they ran more hooking rounds
                                 (the live cross edges outgrew the
                                 one-workgroup rounds), bit 1 when they ran
                                 more super-forest search levels or the Euler
                                 tour, bit 2 when they turned paths longer
                                 than walk_limit */
    int32_t jump_rounds;      /* delete: pointer-jumping rounds before root
                                 finding's chase that changed an entry; a
                                 context queues such rounds once a chase has
                                 found its forest deep (more than 1024
                                 steps) or create found a tree deeper than
                                 2^16, 0 before */
} drsf_view;

/*
 * Creates a context from G and F.
 *   n        number of vertices (>= 1)
 *   row_ptr  int64[n + 1], symmetric CSR offsets of G (row_ptr[0] == 0)
 *   col      int32[row_ptr[n]], neighbours; every row strictly ascending,
 *            no self-loops, and (u,v) present iff (v,u) present
 *   parent   int32[n], a rooted spanning forest of G (parent[r] == r for
 *            roots) whose trees span the connected components of G — the
 *            precondition the insert path of Algorithm 1 relies on
 *   opts     may be NULL (defaults)
 * Trees whose root is not their smallest vertex are re-rooted there.
 * Device inputs are read on the context's stream (ordering rule above) and
 * are no longer needed when drsf_create returns.
 * Errors: DRSF_E_ARG (bad CSR), DRSF_E_FOREST (parent invalid; checked when
 * validate_forest is set), DRSF_E_NOMEM, DRSF_E_DEVICE.  *out is NULL on error.
 */
int drsf_create(int32_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *parent,
                const drsf_opts *opts, drsf_ctx **out);

/*
 * Applies one batch (Algorithm 1): edges holds b pairs (u, v) interleaved,
 * int32[2b], in either orientation; op is DRSF_INSERT or DRSF_DELETE.
 * Blocks until the result is final on the device and fills *out (may be
 * NULL); updates still queued are waited for first and their results
 * dropped.  b == 0 is a no-op.  With inputs_on_device the batch is read in
 * place on the device (see drsf_apply_async).  Errors: DRSF_E_BATCH (state
 * unchanged), DRSF_E_CAPACITY (b > max_batch, or more inserts than
 * delta_capacity), DRSF_E_ARG, DRSF_E_DEVICE.
 */
int drsf_apply(drsf_ctx *ctx, const int32_t *edges, int64_t b, int op, drsf_view *out);

/*
 * Queues the same work as drsf_apply on the context's stream and returns
 * without waiting.  A host batch is copied into the context before return.
 * A device batch (inputs_on_device) is read in place by the update's first
 * kernel: work queued later on the context's stream is ordered after that
 * read, but any other writer of that memory (another stream, the host, a
 * free that lets another stream reuse it) must wait for drsf_wait.  Call
 * drsf_wait before reading results or queueing host reads; device work
 * queued later on the same stream is ordered after the update.
 *
 * Two updates may be in flight: on a one-graph context with
 * inputs_on_device, without profiling and with the default replacement and
 * reversal modes, a batch is queued behind the one still running, so that
 * the device starts it as soon as the first is done (the host's round trip
 * between them is hidden; the result is the same as applying them one after
 * the other).  A third call first waits for the oldest; an empty batch, one
 * that needs a store rebuild, and every other context wait for all queued
 * updates first.  If the running update needs the host to finish it (see
 * drsf_view.host_finished), the one queued behind it does nothing on the
 * device until drsf_wait has finished the first, then runs.  An error this
 * call returns other than DRSF_E_CAPACITY or DRSF_E_ARG may belong to an
 * earlier update that it waited for.
 */
int drsf_apply_async(drsf_ctx *ctx, const int32_t *edges, int64_t b, int op);

/* Returns the status and figures of the oldest queued update not yet
 * returned, waiting for it if it is still running: one call per
 * drsf_apply_async, in order.  An update that another call of the library
 * waited for on the caller's behalf (a drain before a call that needs the
 * queue empty) keeps its result for this call (the two newest are kept;
 * a multi-graph apply drops them, since it overwrites the per-graph
 * statuses).  With none left, returns the status of the last update waited
 * for. */
int drsf_wait(drsf_ctx *ctx, drsf_view *out);

/*
 * Several independent graphs in one context, each updated by its own batch
 * and op in a single pass of the update path.  The paper runs one graph at a
 * time (Sec. V, experimental setup); the per-graph result is exactly what
 * drsf_apply computes for that graph alone: components never span two
 * graphs, so every step of Algorithm 1 restricted to one graph's vertices is
 * the single-graph step.
 *
 * drsf_multi_create:
 *   G        number of graphs (>= 1)
 *   n_off    host int32[G + 1], vertex offsets: graph g owns global ids
 *            [n_off[g], n_off[g + 1]); n_off[0] == 0, non-decreasing; n =
 *            n_off[G]
 *   row_ptr, col, parent, opts: as drsf_create over the n global ids; every
 *            neighbour of a vertex lies in the vertex's graph (else
 *            DRSF_E_ARG)
 * Labels are global ids (the smallest global id of the component).
 *
 * drsf_multi_apply(_async):
 *   edges    int32[2 * b_off[G]] global-id pairs, graph g's batch at
 *            [b_off[g], b_off[g + 1]) (host or device per inputs_on_device;
 *            a host batch is copied before return, a device batch by a copy
 *            queued on the context's stream, with drsf_apply_async's rule
 *            for other writers)
 *   b_off    host int64[G + 1], b_off[0] == 0, non-decreasing; b_off[G] <=
 *            max_batch
 *   op       host int8[G], DRSF_INSERT or DRSF_DELETE per graph
 *   status   host int32[G] (may be NULL): DRSF_OK, or DRSF_E_BATCH when graph
 *            g's batch was invalid (that graph is left unchanged; the others
 *            are updated)
 * drsf_apply on a context with G > 1 returns DRSF_E_STATE.
 */
int drsf_multi_create(int32_t G, const int32_t *n_off, const int64_t *row_ptr, const int32_t *col,
                      const int32_t *parent, const drsf_opts *opts, drsf_ctx **out);
int drsf_multi_apply(drsf_ctx *ctx, const int32_t *edges, const int64_t *b_off, const int8_t *op,
                     int32_t *status);
int drsf_multi_apply_async(drsf_ctx *ctx, const int32_t *edges, const int64_t *b_off,
                           const int8_t *op);
/* Waits like drsf_wait and fills the per-graph status of the last multi apply. */
int drsf_multi_wait(drsf_ctx *ctx, int32_t *status);
/* Live edges per graph, host int64[G]. */
int drsf_multi_num_edges(drsf_ctx *ctx, int64_t *m);
/* Number of graphs in the context (1 for drsf_create). */
int drsf_num_graphs(const drsf_ctx *ctx);

/*
 * Digests of the current parent and label arrays (out[0], out[1], host):
 * order-independent 64-bit sums of a mix of (vertex, value).  Equal arrays
 * give equal digests; used to compare runs without copying the arrays.
 */
int drsf_digest(drsf_ctx *ctx, uint64_t *out);

/*
 * Static rebuild (the baseline of the dynamic update, Sec. V's static GPU
 * forest; no context): a rooted spanning forest of G from scratch.
 * Connected components by hooking (the larger root of an edge's two
 * components takes the smaller as its root, repeated with pointer jumping
 * until no edge joins two roots), so each component is rooted at its
 * smallest vertex, then a breadth-first forest from all roots at once
 * (a level is expanded top-down from its frontier's rows when they are few
 * and short, else bottom-up: every unvisited vertex takes the first
 * neighbour on the frontier in its row).
 * row_ptr: DEVICE int64[n + 1]; col: DEVICE int32[row_ptr[n]] (may be NULL
 * when row_ptr[n] == 0), a symmetric CSR without self-loops (not checked
 * here).  parent_out, label_out: DEVICE
 * int32[n], written: parent[root] = root, label = the component's smallest
 * vertex.  The breadth-first parent is one of several valid choices (ties
 * between frontier vertices are decided by the hardware).  stream: hipStream_t
 * or NULL.  levels_out (host, may be NULL): breadth-first levels.  Allocates
 * and frees its own scratch (about 12 bytes per vertex and 4 per CSR entry)
 * and returns when the result is final.  Errors: DRSF_E_ARG, DRSF_E_NOMEM,
 * DRSF_E_DEVICE.
 */
int drsf_static_forest(int32_t n, const int64_t *row_ptr, const int32_t *col, int32_t *parent_out,
                       int32_t *label_out, void *stream, int32_t *levels_out);

/*
 * The same static rebuild for callers that cannot allocate memory (code
 * being captured into a HIP graph, tight serving loops, harnesses that
 * forbid allocation): it makes no device or host allocation.  Its scratch
 * is one array of 64 MiB in device memory that the library holds on each
 * device it runs on until the process ends; the graph must fit it:
 * 12 n + 8 nnz bytes plus about 1.5 KB, each of eight arrays rounded up to
 * 256 bytes (for example n = 10^6 with nnz = 6.8 * 10^6), else
 * DRSF_E_CAPACITY and nothing is done.  Arguments, result and the other
 * errors are drsf_static_forest's.  Every call on a device uses that
 * device's one array, so calls that overlap on one device (from two host
 * threads, or queued on two streams) race and give wrong results; calls
 * one after another are independent (every call clears what it reads).
 */
int drsf_static_forest_noalloc(int32_t n, const int64_t *row_ptr, const int32_t *col, int32_t *parent_out,
                               int32_t *label_out, void *stream, int32_t *levels_out);

/* Device bytes the context holds (its own allocations). */
int64_t drsf_device_bytes(const drsf_ctx *ctx);

/*
 * Upper estimate of the device bytes drsf_create would hold at its peak for
 * n vertices and nnz CSR entries (2 |E|) with these options (NULL: defaults);
 * used for admission against a memory budget.
 */
int64_t drsf_footprint(int32_t n, int64_t nnz, const drsf_opts *opts);

/*
 * Changes the tunables of drsf_opts (rounds_queued, levels_queued,
 * sweep_mode; 0 = default for the first two) on a live context (captured
 * update graphs are dropped).  Results do not depend on them (only the split
 * between queued and host-driven work does).  Used by the
 * autotuner.  Errors: DRSF_E_ARG.
 */
int drsf_set_tuning(drsf_ctx *ctx, int rounds_queued, int levels_queued, int sweep_mode);

/*
 * The launch schedule of the small-graph kernel of a multi-graph context
 * (drsf_opts.small_graph_vertices): threads per workgroup (256, 512 or
 * 1024; 0 = keep) and workgroups (0 = as many as fit on the device at once,
 * at most one per small graph).  Results do not depend on it; captured
 * update graphs are dropped.  Used by the autotuner.  Errors:
 * DRSF_E_ARG.
 */
int drsf_set_small_schedule(drsf_ctx *ctx, int threads, int workgroups);

/* Copies parent and/or label (either may be NULL) to host int32[n]. */
int drsf_copy_out(drsf_ctx *ctx, int32_t *parent_host, int32_t *label_host);

/* Current view without applying anything. */
int drsf_get_view(drsf_ctx *ctx, drsf_view *out);

/*
 * Number of edges of the current graph, and its edges as sorted keys
 * (min << 32 | max) in host memory (capacity >= drsf_num_edges).  Together
 * with drsf_copy_out this is a checkpoint that drsf_create can resume from.
 */
int64_t drsf_num_edges(drsf_ctx *ctx);
int drsf_export_edges(drsf_ctx *ctx, uint64_t *keys_host, int64_t capacity, int64_t *m_out);

/* Device-side copy of the whole state; restore returns to it exactly.  A
 * snapshot taken before a store rebuild cannot be restored after it
 * (DRSF_E_STATE). */
typedef struct drsf_snapshot drsf_snapshot;
int drsf_snapshot_take(drsf_ctx *ctx, drsf_snapshot **out);
int drsf_snapshot_restore(drsf_ctx *ctx, const drsf_snapshot *snap);
void drsf_snapshot_free(drsf_snapshot *snap);

/*
 * Per-phase device times of the last apply in milliseconds (needs
 * opts.profile), 11 entries: validate; update-graph (cut, store update,
 * piece registration, and for deletes the start of root finding, rep =
 * parent); root finding (pointer chase, orphan bitmap, orphan staging);
 * orphan list; orphan adjacency scan; whole-store sweep; cross edges of the
 * batch and of the inserted-edge list; replacement edges (the hooking
 * rounds queued with the update); super-forest rooting; path reversal with
 * the new labels (one launch); and the host-driven continuation: when the
 * queued rounds or search levels did not finish the update
 * (drsf_view.host_finished), the time from the first continuation launch to
 * the end of its cleanup, host round trips between launches included (0
 * otherwise; the queued phases then hold only what ran before it).  A phase
 * that launches nothing for the batch's kind (the delete-only phases of an
 * insert batch) reads 0.  Each phase time includes the fixed cost of one
 * event record; a 12th entry (written when cap > 11) is the time of an
 * empty bracket, two events recorded back to back before the update, which
 * measures that cost.  Returns the number of entries written (<= cap).
 */
int drsf_phase_times(drsf_ctx *ctx, float *ms, int cap);

void drsf_destroy(drsf_ctx *ctx);

/* Message for the last error on ctx (ctx may be NULL for create errors). */
const char *drsf_last_error(const drsf_ctx *ctx);

/* Library version string. */
const char *drsf_version(void);

/*
 * Serving: several graphs ("tenants") resident on the GPU under a device
 * memory budget, updated by a stream of requests (the paper's setting
 * applied to many graphs at once; no counterpart in its experiments).
 * A scheduler thread admits tenants in arrival order while their estimated
 * footprint (drsf_footprint) fits the budget, keeps one FIFO per tenant and
 * starts the head request of every ready tenant on that tenant's stream, so
 * updates of different graphs overlap on the device.  Requests of one tenant
 * are applied in arrival order, by default one batch each, so each request's
 * result is the one drsf_apply would give on that graph.
 *
 * Times are nanoseconds from drsf_server_start.  arrive_ns >= 0 schedules an
 * admission or request at that time (a pre-generated arrival stream); < 0
 * means now.  Requests submitted before their tenant is admitted wait for
 * it.  Flags: DRSF_SERVER_DIGESTS computes drsf_digest-equal digests of
 * parent and label after every request; DRSF_SERVER_SERIAL keeps at most one
 * request in flight over all tenants, in arrival order (the plain path);
 * DRSF_SERVER_COALESCE applies the requests of the same op waiting together
 * at the head of an idle tenant's FIFO as one batch (up to max_batch
 * edges).  A merged result is that of drsf_apply on the merged batch (the
 * same components; the replacement edges may differ from one-at-a-time
 * application, as Kruskal over a union of batches differs from Kruskal in
 * sequence); drsf_server_batch tells which batch carried a request.  A
 * merged batch that is rejected changes nothing and its requests are
 * retried one at a time.
 * All inputs are host memory and are copied.  One thread at a time may call
 * a server's functions, besides its own scheduler thread.
 */
typedef struct drsf_server drsf_server;
#define DRSF_SERVER_DIGESTS 1
#define DRSF_SERVER_SERIAL 2
#define DRSF_SERVER_COALESCE 4
int drsf_server_create(int64_t budget_bytes, const drsf_opts *opts, int flags, drsf_server **out);
/* Errors: DRSF_E_BUDGET when the estimate exceeds the whole budget. */
int drsf_server_admit(drsf_server *srv, int32_t n, const int64_t *row_ptr, const int32_t *col,
                      const int32_t *parent, int64_t arrive_ns, int32_t *tenant);
int drsf_server_submit(drsf_server *srv, int32_t tenant, const int32_t *edges, int64_t b, int op,
                       int64_t arrive_ns, int64_t *req);
/* The tenant leaves once its submitted requests are done; its memory is freed. */
int drsf_server_release(drsf_server *srv, int32_t tenant);
int drsf_server_start(drsf_server *srv);
/* Blocks until every submitted request is done. */
int drsf_server_wait_all(drsf_server *srv);
/*
 * Blocks until request req is done: status (drsf_status of its update),
 * t_ns[3] = arrival, start and completion times, digest[2] (with
 * DRSF_SERVER_DIGESTS).  Any output may be NULL.
 */
int drsf_server_result(drsf_server *srv, int64_t req, int32_t *status, uint64_t *t_ns, uint64_t *digest);
/*
 * Blocks until request req is done; *batch = the id of the first request of
 * the device batch that carried it (req itself when it went alone; all
 * requests of one batch complete together with the same status and
 * digests).
 */
int drsf_server_batch(drsf_server *srv, int64_t req, int64_t *batch);
/*
 * out[8]: completed requests, p50 and p99 of (completion - arrival) in ms,
 * edge updates per second from the first arrival to the last completion,
 * peak device bytes of the admitted tenants, the budget, p50 and p99 of
 * (completion - max(arrival, the tenant's admission)) in ms.  Graphs
 * admitted at time 0 are made resident by drsf_server_start, before the
 * clock starts.
 */
int drsf_server_stats(drsf_server *srv, double *out);
/* 0 waiting to arrive, 1 queued for admission, 2 live, 3 released, 4 failed. */
int32_t drsf_server_tenant_state(drsf_server *srv, int32_t tenant);
/*
 * Copies a live tenant's parent and label arrays (host int32[n] each;
 * either may be NULL) once every request submitted for it so far is done:
 * blocks until then, while the scheduler goes on with other tenants.  The
 * arrays are the result of all of those requests, as drsf_copy_out on the
 * tenant's context.  Errors: DRSF_E_ARG (unknown tenant), DRSF_E_STATE (the
 * tenant is not live: not yet admitted, released or failed; a released
 * tenant is destroyed once its queue is empty), or the copy's error.
 */
int drsf_server_copy_out(drsf_server *srv, int32_t tenant, int32_t *parent_host, int32_t *label_host);
const char *drsf_server_error(const drsf_server *srv);
/* Waits for submitted requests, then frees everything. */
void drsf_server_destroy(drsf_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* DRSF_H */
