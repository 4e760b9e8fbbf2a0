// C ABI of libdrsf.so (declared in include/drsf.h): context management,
// create-time build of the device edge store, and the batch update pipeline.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/drsf.h"
#include "drsf_kernels.h"

using namespace drsf;

namespace {

thread_local std::string g_create_error;

constexpr int BFS_CHUNK = 4;   // search levels per host check
constexpr int BFS_MAX = 8;     // deeper super-trees use the Euler tour instead

enum Phase { PH_VALIDATE, PH_UPDATE, PH_ROOTS, PH_SWEEP, PH_SWEEP_DELTA, PH_REPL, PH_ROOTING, PH_REVERSE, PH_LABELS, PH_N };

int ceil_log2(int64_t x) {
    int r = 0;
    while (((int64_t)1 << r) < x) r++;
    return r;
}

}  // namespace

struct drsf_snapshot {
    int32_t n;
    int64_t eb, dcap, ndelta_bound, m_live;
    uint64_t dhmask;
    unsigned long long ndelta;
    int32_t *parent, *label, *bcol, *dhpos;
    uint64_t *dkey, *dhash;
};

struct drsf_ctx {
    drsf_opts opts{};
    int dev = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int32_t n = 0;
    int64_t m_live = 0;
    // edge store
    uint32_t *bptr = nullptr;
    int32_t *bcol = nullptr;
    int64_t eb = 0;
    int32_t *zrow = nullptr;
    uint32_t *zptr = nullptr;
    int64_t nz = 0;
    int32_t *tile_k = nullptr;
    int64_t ntiles = 0;
    uint64_t *dkey = nullptr;
    int64_t dcap = 0;
    int64_t ndelta_bound = 0;
    uint64_t *dhash = nullptr;
    int32_t *dhpos = nullptr;
    uint64_t dhmask = 0;
    // forest
    int32_t *parent = nullptr, *label = nullptr, *rep = nullptr;
    uint64_t *obits = nullptr;
    // pieces
    int32_t *tidx = nullptr, *owner = nullptr, *prt = nullptr, *pmin = nullptr, *comp = nullptr,
            *hook = nullptr;
    uint8_t *pkeep = nullptr;
    int32_t *head = nullptr, *newlab = nullptr, *level = nullptr, *parc = nullptr;
    uint64_t *best = nullptr, *srkey = nullptr;
    int64_t pcap = 0;
    // batch
    int64_t max_batch = 0;
    int32_t *bedges = nullptr, *bchild = nullptr, *bslot = nullptr;
    uint64_t *bkey = nullptr, *bhash = nullptr;
    int64_t *bloc = nullptr;
    uint64_t bhmask = 0;
    // lists
    Cross *x0 = nullptr, *x1 = nullptr;
    int64_t xcap = 0;
    unsigned long long *rcnt = nullptr;
    int4 *er = nullptr;
    int64_t ercap = 0;
    int32_t *arc_nxt = nullptr, *succ0 = nullptr, *succ1 = nullptr, *rank0 = nullptr, *rank1 = nullptr;
    PathReq *paths = nullptr;
    int64_t pathcap = 0;
    int32_t *status = nullptr;
    unsigned long long *cnt = nullptr;
    // pinned host staging
    int32_t *h_edges = nullptr;
    unsigned long long *h_ret = nullptr;  // [0] status, [1..] counters
    // last apply
    bool pending = false;
    int64_t last_b = 0;
    int last_op = 0;
    int last_rc = DRSF_OK;
    drsf_view view{};
    hipEvent_t ev[PH_N + 1]{};
    float phase_ms[PH_N]{};
    bool have_phases = false;
    std::string err;
    std::vector<void *> allocs;
};

namespace {

int fail(drsf_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf; else g_create_error = buf;
    return code;
}

#define HIPCHK(ctx, call)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail((ctx), DRSF_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

template <class T>
int dalloc(drsf_ctx *c, T **p, int64_t count) {
    size_t bytes = sizeof(T) * (size_t)(count > 0 ? count : 1);
    void *q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, DRSF_E_NOMEM, "device allocation of %zu bytes failed", bytes);
    }
    c->allocs.push_back(q);
    *p = (T *)q;
    return DRSF_OK;
}

void dfree(drsf_ctx *c, void *p) {
    if (!p) return;
    auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
    if (it != c->allocs.end()) c->allocs.erase(it);
    (void)hipFree(p);
}

Dev make_dev(drsf_ctx *c, int op, int64_t b) {
    Dev d;
    memset(&d, 0, sizeof d);
    d.n = c->n;
    d.op = op;
    d.bptr = c->bptr; d.bcol = c->bcol; d.eb = c->eb;
    d.zrow = c->zrow; d.zptr = c->zptr; d.nz = c->nz; d.tile_k = c->tile_k; d.ntiles = c->ntiles;
    d.dkey = c->dkey; d.dcap = c->dcap; d.dhash = c->dhash; d.dhpos = c->dhpos; d.dhmask = c->dhmask;
    d.parent = c->parent; d.label = c->label; d.rep = c->rep;
    d.repv = op == DRSF_DELETE ? c->rep : c->label;
    d.obits = c->obits;
    d.tidx = c->tidx; d.owner = c->owner; d.pkeep = c->pkeep; d.prt = c->prt; d.pmin = c->pmin; d.comp = c->comp; d.hook = c->hook;
    d.best = c->best; d.srkey = c->srkey; d.head = c->head; d.newlab = c->newlab;
    d.level = c->level; d.parc = c->parc; d.pcap = c->pcap;
    d.bedges = c->bedges; d.b = b; d.bkey = c->bkey; d.bloc = c->bloc; d.bchild = c->bchild;
    d.bslot = c->bslot; d.bhash = c->bhash; d.bhmask = c->bhmask;
    d.x0 = c->x0; d.x1 = c->x1; d.xcap = c->xcap; d.rcnt = c->rcnt;
    d.nreg = op == DRSF_DELETE ? c->ntiles + delta_tiles(c->ndelta_bound) : insert_regions(b);
    d.er = c->er; d.ercap = c->ercap; d.arc_nxt = c->arc_nxt;
    d.succ0 = c->succ0; d.succ1 = c->succ1; d.rank0 = c->rank0; d.rank1 = c->rank1;
    d.paths = c->paths; d.pathcap = c->pathcap;
    d.status = c->status; d.cnt = c->cnt;
    return d;
}

int read_status(drsf_ctx *c, int32_t *st) {
    HIPCHK(c, hipMemcpyAsync(c->h_ret, c->status, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *st = *(int32_t *)c->h_ret;
    return DRSF_OK;
}

int alloc_state(drsf_ctx *c) {
    int rc;
    const int32_t n = c->n;
    const int64_t mb = c->max_batch;
    if ((rc = dalloc(c, &c->label, n))) return rc;
    if ((rc = dalloc(c, &c->rep, n))) return rc;
    if ((rc = dalloc(c, &c->obits, (n + 63) / 64))) return rc;
    if ((rc = dalloc(c, &c->tidx, n))) return rc;
    if ((rc = dalloc(c, &c->owner, n))) return rc;
    c->pcap = 2 * mb + 16;
    if ((rc = dalloc(c, &c->pkeep, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->prt, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->pmin, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->comp, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->hook, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->head, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->level, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->parc, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->newlab, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->best, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->srkey, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->bedges, 2 * mb))) return rc;
    if ((rc = dalloc(c, &c->bkey, mb))) return rc;
    if ((rc = dalloc(c, &c->bloc, mb))) return rc;
    if ((rc = dalloc(c, &c->bchild, mb))) return rc;
    if ((rc = dalloc(c, &c->bslot, mb))) return rc;
    uint64_t bh = 16;
    while (bh < (uint64_t)(2 * mb)) bh <<= 1;
    c->bhmask = bh - 1;
    if ((rc = dalloc(c, &c->bhash, (int64_t)bh))) return rc;
    c->dcap = c->opts.delta_capacity > 0 ? c->opts.delta_capacity
                                         : std::max<int64_t>({4 * mb, c->eb / 8, 1 << 20});
    if ((rc = dalloc(c, &c->dkey, c->dcap))) return rc;
    uint64_t dh = 16;
    while (dh < (uint64_t)(2 * c->dcap)) dh <<= 1;
    c->dhmask = dh - 1;
    if ((rc = dalloc(c, &c->dhash, (int64_t)dh))) return rc;
    if ((rc = dalloc(c, &c->dhpos, (int64_t)dh))) return rc;
    // x0: one region of TILE entries per producing workgroup (base-store tiles
    // and inserted-edge tiles on delete, batch tiles on insert)
    const int64_t nregmax = std::max<int64_t>(c->ntiles + delta_tiles(c->dcap), insert_regions(mb));
    c->xcap = nregmax * TILE;
    if ((rc = dalloc(c, &c->x0, c->xcap))) return rc;
    if ((rc = dalloc(c, &c->x1, c->xcap))) return rc;
    if ((rc = dalloc(c, &c->rcnt, nregmax))) return rc;
    launch_fill_u64(c->rcnt, nregmax, 0, c->stream);
    c->ercap = c->pcap;
    if ((rc = dalloc(c, &c->er, c->ercap))) return rc;
    if ((rc = dalloc(c, &c->arc_nxt, 2 * c->ercap))) return rc;
    if ((rc = dalloc(c, &c->succ0, 2 * c->ercap))) return rc;
    if ((rc = dalloc(c, &c->succ1, 2 * c->ercap))) return rc;
    if ((rc = dalloc(c, &c->rank0, 2 * c->ercap))) return rc;
    if ((rc = dalloc(c, &c->rank1, 2 * c->ercap))) return rc;
    c->pathcap = std::max<int64_t>(c->ercap + c->pcap, n);
    if ((rc = dalloc(c, &c->paths, c->pathcap))) return rc;
    if (hipHostMalloc((void **)&c->h_edges, sizeof(int32_t) * 2 * (size_t)mb) != hipSuccess)
        return fail(c, DRSF_E_NOMEM, "pinned host allocation failed");
    launch_fill_i32(c->tidx, n, NONE, c->stream);
    launch_fill_u64(c->bhash, (int64_t)bh, HASH_EMPTY, c->stream);
    launch_fill_u64(c->dhash, (int64_t)dh, HASH_EMPTY, c->stream);
    launch_fill_u64(c->obits, (n + 63) / 64, 0, c->stream);
    return DRSF_OK;
}

void destroy_ctx(drsf_ctx *c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (void *p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
    if (c->h_edges) (void)hipHostFree(c->h_edges);
    if (c->h_ret) (void)hipHostFree(c->h_ret);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

// Build the device edge store from a symmetric CSR with ascending rows.
int build_store(drsf_ctx *c, const int64_t *row_ptr_in, const int32_t *col_in, int64_t nnz) {
    int rc;
    const int32_t n = c->n;
    const bool dev_in = c->opts.inputs_on_device != 0;
    int64_t *drow = nullptr;
    int32_t *dcol = nullptr;
    if (dev_in) {
        drow = const_cast<int64_t *>(row_ptr_in);
        dcol = const_cast<int32_t *>(col_in);
    } else {
        if ((rc = dalloc(c, &drow, (int64_t)n + 1))) return rc;
        if ((rc = dalloc(c, &dcol, nnz))) return rc;
        HIPCHK(c, hipMemcpyAsync(drow, row_ptr_in, sizeof(int64_t) * ((size_t)n + 1),
                                 hipMemcpyHostToDevice, c->stream));
        if (nnz > 0)
            HIPCHK(c, hipMemcpyAsync(dcol, col_in, sizeof(int32_t) * (size_t)nnz,
                                     hipMemcpyHostToDevice, c->stream));
    }
    uint32_t *ucnt = nullptr;
    void *tmp = nullptr;
    if ((rc = dalloc(c, &ucnt, n))) return rc;
    if ((rc = dalloc(c, (char **)&tmp, (int64_t)scan_tmp_bytes(n) + 64))) return rc;
    if ((rc = dalloc(c, &c->bptr, (int64_t)n + 1))) return rc;
    unsigned long long *dtotal = (unsigned long long *)((char *)tmp + scan_tmp_bytes(n));
    launch_fill_i32(c->status, 1, 0, c->stream);
    launch_csr_check(n, drow, dcol, ucnt, c->status, c->stream);
    launch_csr_symmetric(n, drow, dcol, c->status, c->stream);
    launch_scan_u32(ucnt, c->bptr, dtotal, n, tmp, c->stream);
    unsigned long long total = 0;
    HIPCHK(c, hipMemcpyAsync(c->h_ret, dtotal, sizeof total, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->h_ret + 1, c->status, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    total = c->h_ret[0];
    int32_t st = *(int32_t *)(c->h_ret + 1);
    if (st & 1) return fail(c, DRSF_E_ARG, "CSR rows must be ascending, without self-loops, ids in [0,n)");
    if (st & 2) return fail(c, DRSF_E_ARG, "CSR is not symmetric");
    if (2 * (int64_t)total != nnz) return fail(c, DRSF_E_ARG, "CSR is not symmetric");
    if (total >= 0xffffffffull) return fail(c, DRSF_E_CAPACITY, "more than 2^32-1 undirected edges");
    c->eb = (int64_t)total;
    if ((rc = dalloc(c, &c->bcol, c->eb))) return rc;
    launch_upper_fill(n, drow, dcol, c->bptr, c->bcol, c->stream);
    // non-empty-row index for the sweep
    launch_nonempty_flags(n, c->bptr, ucnt, c->stream);
    uint32_t *zpos = nullptr;
    if ((rc = dalloc(c, &zpos, (int64_t)n + 1))) return rc;
    launch_scan_u32(ucnt, zpos, dtotal, n, tmp, c->stream);
    HIPCHK(c, hipMemcpyAsync(c->h_ret, dtotal, sizeof total, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->nz = (int64_t)c->h_ret[0];
    if ((rc = dalloc(c, &c->zrow, c->nz))) return rc;
    if ((rc = dalloc(c, &c->zptr, c->nz + 1))) return rc;
    launch_nonempty_fill(n, c->bptr, zpos, c->zrow, c->zptr, c->nz, c->stream);
    c->ntiles = (c->eb + TILE - 1) / TILE;
    if ((rc = dalloc(c, &c->tile_k, c->ntiles + 1))) return rc;
    launch_tile_k(c->zptr, c->nz, c->eb, c->tile_k, c->ntiles, c->stream);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dfree(c, zpos);
    dfree(c, ucnt);
    dfree(c, tmp);
    if (!dev_in) { dfree(c, drow); dfree(c, dcol); }
    c->m_live = c->eb;
    return DRSF_OK;
}

// Check the forest (optional) and root every tree at its smallest vertex.
int canonicalise_forest(drsf_ctx *c) {
    const int32_t n = c->n;
    hipStream_t s = c->stream;
    Dev d = make_dev(c, DRSF_INSERT, 0);
    launch_fill_i32(c->status, 1, 0, s);
    launch_fill_u64(c->cnt, C_TOTAL, 0, s);
    launch_forest_check(n, c->bptr, c->bcol, c->parent, c->status, c->opts.validate_forest, s);
    int32_t st;
    int rc;
    if ((rc = read_status(c, &st))) return rc;
    if (st) return fail(c, DRSF_E_FOREST, "parent[] has an id out of range or an edge not in G");
    // synchronous pointer jumping: after ceil(log2 n) + 1 rounds every vertex
    // of a tree points at its root
    int32_t *a = c->rep, *b = c->label;
    HIPCHK(c, hipMemcpyAsync(a, c->parent, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    const int rounds = ceil_log2(n) + 1;
    for (int r = 0; r < rounds; r++) {
        launch_pointer_jump(n, a, b, s);
        std::swap(a, b);
    }
    int32_t *root = a;
    int32_t *other = b;
    launch_roots_check(n, c->parent, root, c->status, s);
    if (c->opts.validate_forest) launch_span_check(d, root, s);
    if ((rc = read_status(c, &st))) return rc;
    if (st & 4) return fail(c, DRSF_E_FOREST, "parent[] contains a cycle");
    if (st & 8) return fail(c, DRSF_E_FOREST, "a tree does not span its connected component");
    // label <- smallest vertex of each tree; re-root where it is not the root
    int32_t *lab = c->label;
    if (root == c->label) {  // keep roots in rep, labels in label
        HIPCHK(c, hipMemcpyAsync(c->rep, root, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
        root = c->rep;
    }
    (void)other;
    launch_tree_min(n, root, lab, s);
    d = make_dev(c, DRSF_INSERT, 0);
    launch_reroot_requests(d, root, s);
    launch_reverse(d, s);
    if ((rc = read_status(c, &st))) return rc;
    if (st) return fail(c, DRSF_E_DEVICE, "re-rooting failed (status %d)", st);
    launch_fill_u64(c->cnt, C_TOTAL, 0, s);
    HIPCHK(c, hipStreamSynchronize(s));
    return DRSF_OK;
}

}  // namespace

extern "C" {

const char *drsf_version(void) { return "drsf 0.1 (gfx950)"; }

void drsf_default_opts(drsf_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->validate_forest = 1;
    o->max_batch = 1 << 20;
}

const char *drsf_last_error(const drsf_ctx *c) {
    return c ? c->err.c_str() : g_create_error.c_str();
}

int drsf_create(int32_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *parent,
                const drsf_opts *opts, drsf_ctx **out) {
    if (!out) return fail(nullptr, DRSF_E_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || !row_ptr || !parent) return fail(nullptr, DRSF_E_ARG, "bad arguments");
    drsf_ctx *c = new drsf_ctx();
    if (opts) c->opts = *opts; else drsf_default_opts(&c->opts);
    if (c->opts.max_batch <= 0) c->opts.max_batch = 1 << 20;
    c->max_batch = c->opts.max_batch;
    c->n = n;
    int rc = DRSF_OK;
    auto bail = [&](int code) {
        g_create_error = c->err;
        destroy_ctx(c);
        return code;
    };
    {
        hipError_t e = hipGetDevice(&c->dev);
        if (e != hipSuccess) {
            fail(c, DRSF_E_DEVICE, "no HIP device: %s", hipGetErrorString(e));
            return bail(DRSF_E_DEVICE);
        }
    }
    if (c->opts.stream) {
        c->stream = (hipStream_t)c->opts.stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            fail(c, DRSF_E_DEVICE, "stream creation failed");
            return bail(DRSF_E_DEVICE);
        }
        c->own_stream = true;
    }
    if (hipHostMalloc((void **)&c->h_ret, sizeof(unsigned long long) * (C_TOTAL + 16)) != hipSuccess) {
        fail(c, DRSF_E_NOMEM, "pinned host allocation failed");
        return bail(DRSF_E_NOMEM);
    }
    for (auto &e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) { fail(c, DRSF_E_DEVICE, "event creation failed"); return bail(DRSF_E_DEVICE); }
    if ((rc = dalloc(c, &c->status, 4))) return bail(rc);
    if ((rc = dalloc(c, &c->cnt, C_TOTAL))) return bail(rc);
    launch_fill_u64(c->cnt, C_TOTAL, 0, c->stream);
    // row offsets are checked on the host before any kernel reads through them
    std::vector<int64_t> hrow;
    const int64_t *rp = row_ptr;
    if (c->opts.inputs_on_device) {
        hrow.resize((size_t)n + 1);
        if (hipMemcpy(hrow.data(), row_ptr, sizeof(int64_t) * hrow.size(), hipMemcpyDeviceToHost) !=
            hipSuccess) {
            fail(c, DRSF_E_ARG, "cannot read row_ptr");
            return bail(DRSF_E_ARG);
        }
        rp = hrow.data();
    }
    if (rp[0] != 0) { fail(c, DRSF_E_ARG, "row_ptr[0] must be 0"); return bail(DRSF_E_ARG); }
    for (int32_t u = 0; u < n; u++)
        if (rp[u + 1] < rp[u]) { fail(c, DRSF_E_ARG, "row_ptr must be non-decreasing"); return bail(DRSF_E_ARG); }
    const int64_t nnz = rp[n];
    if (nnz > 0 && !col) { fail(c, DRSF_E_ARG, "col is NULL"); return bail(DRSF_E_ARG); }
    if ((rc = build_store(c, row_ptr, col, nnz))) return bail(rc);
    if ((rc = dalloc(c, &c->parent, n))) return bail(rc);
    if (hipMemcpyAsync(c->parent, parent, sizeof(int32_t) * (size_t)n,
                       c->opts.inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                       c->stream) != hipSuccess) {
        fail(c, DRSF_E_ARG, "cannot copy parent[]");
        return bail(DRSF_E_ARG);
    }
    if ((rc = alloc_state(c))) return bail(rc);
    if ((rc = canonicalise_forest(c))) return bail(rc);
    c->view.parent = c->parent;
    c->view.label = c->label;
    c->view.n = n;
    c->view.num_edges = c->m_live;
    *out = c;
    return DRSF_OK;
}

int drsf_apply_async(drsf_ctx *c, const int32_t *edges, int64_t b, int op) {
    if (!c) return DRSF_E_ARG;
    if (c->pending) {
        int rc = drsf_wait(c, nullptr);
        if (rc != DRSF_OK && rc != DRSF_E_BATCH) return rc;
    }
    if (op != DRSF_INSERT && op != DRSF_DELETE) return fail(c, DRSF_E_ARG, "op must be insert or delete");
    if (b < 0 || (b > 0 && !edges)) return fail(c, DRSF_E_ARG, "bad batch");
    if (b > c->max_batch) return fail(c, DRSF_E_CAPACITY, "batch of %lld exceeds max_batch %lld",
                                      (long long)b, (long long)c->max_batch);
    c->last_b = b;
    c->last_op = op;
    c->have_phases = false;
    if (b == 0) {
        c->pending = false;
        c->last_rc = DRSF_OK;
        c->view.num_key_cross = c->view.num_replacement = c->view.num_pieces = c->view.num_paths = 0;
        return DRSF_OK;
    }
    if (op == DRSF_INSERT && c->ndelta_bound + b > c->dcap)
        return fail(c, DRSF_E_CAPACITY, "inserted-edge store full (%lld of %lld)",
                    (long long)c->ndelta_bound, (long long)c->dcap);
    hipStream_t s = c->stream;
    if (c->opts.inputs_on_device) {
        HIPCHK(c, hipMemcpyAsync(c->bedges, edges, sizeof(int32_t) * 2 * (size_t)b,
                                 hipMemcpyDeviceToDevice, s));
    } else {
        // the previous apply has completed (pending was cleared), so the
        // pinned staging buffer is free
        memcpy(c->h_edges, edges, sizeof(int32_t) * 2 * (size_t)b);
        HIPCHK(c, hipMemcpyAsync(c->bedges, c->h_edges, sizeof(int32_t) * 2 * (size_t)b,
                                 hipMemcpyHostToDevice, s));
    }
    const Dev d = make_dev(c, op, b);
    const bool prof = c->opts.profile != 0;
    auto mark = [&](int i) { if (prof) (void)hipEventRecord(c->ev[i], s); };
    const int64_t np_max = std::min<int64_t>(2 * b, c->pcap);
    const int bor_bound = std::min(ceil_log2(np_max + 2) + 2, MAX_ROUNDS);
    const int lr_rounds = std::min(ceil_log2(2 * np_max + 2) + 2, MAX_ROUNDS);
    mark(PH_VALIDATE);
    launch_classify(d, s);
    mark(PH_UPDATE);
    launch_prepare(d, s);
    launch_register(d, s);
    mark(PH_ROOTS);
    if (op == DRSF_DELETE) launch_rep(d, s);
    mark(PH_SWEEP);
    if (op == DRSF_DELETE) launch_sweep_base(d, s);
    else launch_insert_emit(d, s);
    mark(PH_SWEEP_DELTA);
    if (op == DRSF_DELETE) launch_sweep_delta(d, c->ndelta_bound, s);
    mark(PH_REPL);
    // Hooking rounds run in short chunks; the host reads the device's done
    // flag between chunks instead of queueing the worst-case number of
    // rounds.  The first chunk is followed by speculative super-root and
    // search levels that only run if the rounds have finished.
    int r = op == DRSF_DELETE ? 2 : 4;
    r = std::min(r, bor_bound);
    launch_boruvka(d, 0, r, s);
    launch_sf_root(d, s);
    launch_sf_bfs(d, 0, BFS_CHUNK, s);
    int lv = BFS_CHUNK;
    unsigned long long *ctl = c->h_ret + 1 + C_COUNT;  // [status, done, bfs flag]
    auto read_ctl = [&](int bfs_level) -> int {
        HIPCHK(c, hipMemcpyAsync(ctl, c->status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(ctl + 1, c->cnt + C_DONE_BOR, sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(ctl + 2, c->cnt + C_BFS_ROUND + bfs_level - 1,
                                 sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        return DRSF_OK;
    };
    int rc2;
    if ((rc2 = read_ctl(lv))) return rc2;
    bool bad = *(int32_t *)ctl != 0;
    bool done = ctl[1] != 0;
    if (!bad && !done) {
        while (!done && r < bor_bound) {
            const int r1 = std::min(r + 3, bor_bound);
            launch_boruvka(d, r, r1, s);
            r = r1;
            if ((rc2 = read_ctl(lv))) return rc2;
            done = ctl[1] != 0;
            bad = *(int32_t *)ctl != 0;
            if (bad) break;
        }
        if (!bad && done) {
            launch_sf_root(d, s);
            launch_sf_bfs(d, 0, BFS_CHUNK, s);
            if ((rc2 = read_ctl(lv))) return rc2;
            bad = *(int32_t *)ctl != 0;
        }
    }
    mark(PH_ROOTING);
    if (!bad && !done) {
        launch_fill_i32(c->status, 1, ST_ROUND_BOUND, s);  // hooking rounds did not finish
    } else if (!bad) {
        bool bfs_done = ctl[2] == 0;
        while (!bfs_done && lv < BFS_MAX) {
            launch_sf_bfs(d, lv, lv + BFS_CHUNK, s);
            lv += BFS_CHUNK;
            if ((rc2 = read_ctl(lv))) return rc2;
            bfs_done = ctl[2] == 0;
        }
        if (bfs_done) launch_orient_bfs(d, s);
        else launch_superforest_lr(d, lr_rounds, s);  // deep super-trees: Euler tour
    }
    mark(PH_REVERSE);
    launch_reverse(d, s);
    mark(PH_LABELS);
    launch_labels(d, s);
    mark(PH_N);
    HIPCHK(c, hipMemcpyAsync(c->h_ret, c->status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(c->h_ret + 1, c->cnt, sizeof(unsigned long long) * C_COUNT,
                             hipMemcpyDeviceToHost, s));
    launch_cleanup(d, s);
    HIPCHK(c, hipGetLastError());
    if (op == DRSF_INSERT) c->ndelta_bound += b;
    c->pending = true;
    c->have_phases = prof;
    return DRSF_OK;
}

int drsf_wait(drsf_ctx *c, drsf_view *out) {
    if (!c) return DRSF_E_ARG;
    if (c->pending) {
        c->pending = false;
        HIPCHK(c, hipStreamSynchronize(c->stream));
        const int32_t st = *(int32_t *)c->h_ret;
        const unsigned long long *k = c->h_ret + 1;
        if (st == 0) {
            c->m_live += c->last_op == DRSF_INSERT ? c->last_b : -c->last_b;
            c->view.num_key_cross = (int64_t)k[C_NCROSS];
            c->view.num_replacement = (int64_t)k[C_NER];
            c->view.num_pieces = (int64_t)k[C_NP];
            c->view.num_paths = (int64_t)k[C_NR];
            c->last_rc = DRSF_OK;
        } else if (st & ST_BATCH_MASK) {
            if (c->last_op == DRSF_INSERT) c->ndelta_bound -= c->last_b;
            c->last_rc = fail(c, DRSF_E_BATCH, "invalid batch:%s%s%s%s",
                              st & ST_BAD_PAIR ? " self-loop or id out of range;" : "",
                              st & ST_DUPLICATE ? " repeated edge;" : "",
                              st & ST_EXISTS ? " insert of an existing edge;" : "",
                              st & ST_MISSING ? " delete of a missing edge;" : "");
        } else {
            c->last_rc = fail(c, DRSF_E_DEVICE, "internal bound exceeded (status %d)", st);
        }
        if (c->have_phases) {
            for (int i = 0; i < PH_N; i++)
                (void)hipEventElapsedTime(&c->phase_ms[i], c->ev[i], c->ev[i + 1]);
        }
    }
    c->view.parent = c->parent;
    c->view.label = c->label;
    c->view.n = c->n;
    c->view.num_edges = c->m_live;
    if (out) *out = c->view;
    return c->last_rc;
}

int drsf_apply(drsf_ctx *c, const int32_t *edges, int64_t b, int op, drsf_view *out) {
    int rc = drsf_apply_async(c, edges, b, op);
    if (rc != DRSF_OK) return rc;
    return drsf_wait(c, out);
}

int drsf_get_view(drsf_ctx *c, drsf_view *out) {
    if (!c || !out) return DRSF_E_ARG;
    if (c->pending) drsf_wait(c, nullptr);
    *out = c->view;
    return DRSF_OK;
}

int drsf_copy_out(drsf_ctx *c, int32_t *parent_host, int32_t *label_host) {
    if (!c) return DRSF_E_ARG;
    if (c->pending) drsf_wait(c, nullptr);
    if (parent_host)
        HIPCHK(c, hipMemcpyAsync(parent_host, c->parent, sizeof(int32_t) * (size_t)c->n,
                                 hipMemcpyDeviceToHost, c->stream));
    if (label_host)
        HIPCHK(c, hipMemcpyAsync(label_host, c->label, sizeof(int32_t) * (size_t)c->n,
                                 hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DRSF_OK;
}

int64_t drsf_num_edges(drsf_ctx *c) {
    if (!c) return -1;
    if (c->pending) drsf_wait(c, nullptr);
    return c->m_live;
}

int drsf_export_edges(drsf_ctx *c, uint64_t *keys, int64_t capacity, int64_t *m_out) {
    if (!c || !keys || !m_out) return DRSF_E_ARG;
    if (c->pending) drsf_wait(c, nullptr);
    std::vector<uint32_t> bptr((size_t)c->n + 1);
    std::vector<int32_t> bcol((size_t)c->eb);
    unsigned long long nd = 0;
    HIPCHK(c, hipMemcpyAsync(&nd, c->cnt + C_NDELTA, sizeof nd, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(bptr.data(), c->bptr, sizeof(uint32_t) * bptr.size(), hipMemcpyDeviceToHost, c->stream));
    if (c->eb)
        HIPCHK(c, hipMemcpyAsync(bcol.data(), c->bcol, sizeof(int32_t) * bcol.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<uint64_t> dk((size_t)nd);
    if (nd) {
        HIPCHK(c, hipMemcpy(dk.data(), c->dkey, sizeof(uint64_t) * nd, hipMemcpyDeviceToHost));
    }
    int64_t w = 0;
    for (int32_t u = 0; u < c->n; u++)
        for (uint32_t j = bptr[u]; j < bptr[u + 1]; j++)
            if (bcol[j] >= 0) {
                if (w >= capacity) return fail(c, DRSF_E_CAPACITY, "export buffer too small");
                keys[w++] = ((uint64_t)(uint32_t)u << 32) | (uint32_t)bcol[j];
            }
    for (uint64_t k : dk)
        if (k != KEY_DEAD) {
            if (w >= capacity) return fail(c, DRSF_E_CAPACITY, "export buffer too small");
            keys[w++] = k;
        }
    std::sort(keys, keys + w);
    *m_out = w;
    return DRSF_OK;
}

int drsf_snapshot_take(drsf_ctx *c, drsf_snapshot **out) {
    if (!c || !out) return DRSF_E_ARG;
    if (c->pending) drsf_wait(c, nullptr);
    drsf_snapshot *s = new drsf_snapshot();
    memset(s, 0, sizeof *s);
    s->n = c->n; s->eb = c->eb; s->dcap = c->dcap; s->dhmask = c->dhmask;
    s->ndelta_bound = c->ndelta_bound; s->m_live = c->m_live;
    const size_t dh = (size_t)c->dhmask + 1;
    bool ok = hipMalloc(&s->parent, 4 * (size_t)c->n) == hipSuccess &&
              hipMalloc(&s->label, 4 * (size_t)c->n) == hipSuccess &&
              hipMalloc(&s->bcol, 4 * (size_t)std::max<int64_t>(c->eb, 1)) == hipSuccess &&
              hipMalloc(&s->dkey, 8 * (size_t)c->dcap) == hipSuccess &&
              hipMalloc(&s->dhash, 8 * dh) == hipSuccess &&
              hipMalloc(&s->dhpos, 4 * dh) == hipSuccess;
    if (!ok) { drsf_snapshot_free(s); return fail(c, DRSF_E_NOMEM, "snapshot allocation failed"); }
    hipStream_t st = c->stream;
    HIPCHK(c, hipMemcpyAsync(s->parent, c->parent, 4 * (size_t)c->n, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(s->label, c->label, 4 * (size_t)c->n, hipMemcpyDeviceToDevice, st));
    if (c->eb) HIPCHK(c, hipMemcpyAsync(s->bcol, c->bcol, 4 * (size_t)c->eb, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(s->dkey, c->dkey, 8 * (size_t)c->dcap, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(s->dhash, c->dhash, 8 * dh, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(s->dhpos, c->dhpos, 4 * dh, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(&s->ndelta, c->cnt + C_NDELTA, sizeof s->ndelta, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    *out = s;
    return DRSF_OK;
}

int drsf_snapshot_restore(drsf_ctx *c, const drsf_snapshot *s) {
    if (!c || !s) return DRSF_E_ARG;
    if (c->pending) drsf_wait(c, nullptr);
    if (s->n != c->n || s->eb != c->eb || s->dcap != c->dcap || s->dhmask != c->dhmask)
        return fail(c, DRSF_E_STATE, "snapshot does not match the context's layout");
    hipStream_t st = c->stream;
    const size_t dh = (size_t)c->dhmask + 1;
    HIPCHK(c, hipMemcpyAsync(c->parent, s->parent, 4 * (size_t)c->n, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(c->label, s->label, 4 * (size_t)c->n, hipMemcpyDeviceToDevice, st));
    if (c->eb) HIPCHK(c, hipMemcpyAsync(c->bcol, s->bcol, 4 * (size_t)c->eb, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(c->dkey, s->dkey, 8 * (size_t)c->dcap, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(c->dhash, s->dhash, 8 * dh, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(c->dhpos, s->dhpos, 4 * dh, hipMemcpyDeviceToDevice, st));
    c->h_ret[0] = s->ndelta;
    HIPCHK(c, hipMemcpyAsync(c->cnt + C_NDELTA, c->h_ret, sizeof(unsigned long long), hipMemcpyHostToDevice, st));
    HIPCHK(c, hipStreamSynchronize(st));
    c->ndelta_bound = s->ndelta_bound;
    c->m_live = s->m_live;
    c->view.num_edges = c->m_live;
    return DRSF_OK;
}

void drsf_snapshot_free(drsf_snapshot *s) {
    if (!s) return;
    (void)hipFree(s->parent); (void)hipFree(s->label); (void)hipFree(s->bcol);
    (void)hipFree(s->dkey); (void)hipFree(s->dhash); (void)hipFree(s->dhpos);
    delete s;
}

int drsf_phase_times(drsf_ctx *c, float *ms, int cap) {
    if (!c || !ms) return 0;
    if (c->pending) drsf_wait(c, nullptr);
    if (!c->have_phases) return 0;
    int k = std::min(cap, (int)PH_N);
    for (int i = 0; i < k; i++) ms[i] = c->phase_ms[i];
    return k;
}

void drsf_destroy(drsf_ctx *c) { destroy_ctx(c); }

}  // extern "C"
