// C ABI of libdrsf.so (declared in include/drsf.h): contexts, the create-time
// build of the device edge store, and the host driver of the update path.
//
// One update is a fixed kernel sequence (drsf_kernels.hip) whose batch shape
// lives in a small device control block, so the sequence is captured once
// per context into a HIP graph and replayed for every batch.  The graph
// queues a few full-grid hooking rounds, one workgroup that runs the later
// rounds while few cross edges are live, and a few search levels; when a
// batch needs more, the kernels after them skip themselves and drsf_wait
// finishes the update with direct launches (further rounds in short chunks,
// deeper search or the Euler tour).  With opts.profile the same sequence is launched directly,
// with events between the phases (events recorded inside a captured graph
// cannot be timed on this runtime).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/drsf.h"
#include "drsf_kernels.h"

using namespace drsf;

namespace {

thread_local std::string g_create_error;

constexpr int BOR_FAST = 2;    // default full-grid hooking rounds queued before the one-workgroup tail
constexpr int BFS_FAST = 4;    // default search levels queued in the captured sequence
constexpr int BFS_MAX = 12;    // deeper super-trees use the Euler tour instead
constexpr int BOR_CHUNK = 3;   // rounds per host check in the continuation
constexpr int AUTO_ROUNDS_MAX = 12;  // queued rounds the library may grow to by itself
// default steps one thread walks along a path; a longer path is turned by
// the doubling pass (a few kernels over all vertices, about as long as a
// walk of this many dependent reads)
constexpr int64_t WALK_LIMIT = 1024;
// a forest handed to create deeper than 2^CREATE_DEEP_LOG starts with
// jumping rounds before root finding's chase (the 4096 x 4096 grid's
// breadth-first forest, 8191 deep, is faster without them)
constexpr int CREATE_DEEP_LOG = 16;

enum Phase { PH_VALIDATE, PH_UPDATE, PH_ROOT, PH_ORPH_LIST, PH_ORPH_SCAN, PH_SWEEP, PH_SWEEP_DELTA,
             PH_REPL, PH_ROOTING, PH_FINISH, PH_N };

int ceil_log2(int64_t x) {
    int r = 0;
    while (((int64_t)1 << r) < x) r++;
    return r;
}

}  // namespace

struct drsf_snapshot {
    drsf_opts opts{};  // allocator hooks of the context it was taken from
    int32_t n = 0;
    int64_t eb = 0, dcap = 0, ndelta_bound = 0, m_live = 0, rebuilds = 0;
    uint64_t dhmask = 0;
    unsigned long long ndelta = 0;
    std::vector<int64_t> gm;
    int32_t *parent = nullptr, *label = nullptr, *bcol = nullptr, *lcol = nullptr, *dhpos = nullptr;
    uint64_t *dkey = nullptr, *dhash = nullptr;
    // small graphs: their key pool, live counts and current buffers
    int64_t pool_keys = 0;
    int32_t nsg = 0;
    uint32_t *pool = nullptr;
    int32_t *sm = nullptr, *sbuf = nullptr;
};

struct drsf_ctx {
    drsf_opts opts{};
    int dev = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int32_t n = 0;
    int64_t m_live = 0;
    // graphs sharing the context (disjoint vertex ranges)
    int32_t ngraph = 1;
    std::vector<int32_t> goff_h;   // [ngraph + 1] vertex offsets
    std::vector<int64_t> gedge_h;  // [ngraph + 1] base-store offsets of each graph's rows
    std::vector<int64_t> gm_h;     // live edges per graph
    int32_t *goff = nullptr;
    int32_t *gstat = nullptr;
    // edge store
    uint32_t *bptr = nullptr, *lptr = nullptr;
    int32_t *bcol = nullptr, *lcol = nullptr;
    int64_t eb = 0;
    int32_t *zrow = nullptr;
    uint32_t *zptr = nullptr;
    int64_t nz = 0;
    int32_t *tile_k = nullptr;
    int64_t ntiles = 0;
    uint64_t *dkey = nullptr;
    int64_t dcap = 0, dtmax = 0;
    int64_t ndelta_bound = 0;
    uint64_t *dhash = nullptr;
    int32_t *dhpos = nullptr;
    uint64_t dhmask = 0;
    // forest
    int32_t *parent = nullptr, *label = nullptr, *rep = nullptr;
    uint64_t *obits = nullptr;
    // pieces
    int32_t *tidx = nullptr, *owner = nullptr, *prt = nullptr, *pmin = nullptr, *comp = nullptr;
    uint8_t *pkeep = nullptr;
    int32_t *head = nullptr, *newlab = nullptr, *level = nullptr, *parc = nullptr;
    uint64_t *hook = nullptr, *best = nullptr, *srkey = nullptr;
    int64_t pcap = 0;
    // batch
    int64_t max_batch = 0;
    int32_t *bedges = nullptr, *bchild = nullptr, *bslot = nullptr, *bgid = nullptr;
    int8_t *bop = nullptr;
    uint64_t *bkey = nullptr, *bhash = nullptr;
    int64_t *bloc = nullptr;
    uint32_t *twin = nullptr, *ltwin = nullptr;
    uint64_t bhmask = 0;
    int32_t *dslot = nullptr;
    uint64_t dsmask = 0;
    // orphan scan
    int64_t nvb = 0;
    int64_t *bvol = nullptr, *bpre = nullptr;
    unsigned long long *gsum = nullptr;
    int64_t *gpre = nullptr, *gopre = nullptr;
    int32_t *bcnt = nullptr, *opre = nullptr, *rstart = nullptr;
    OrphEnt *olist = nullptr, *ostage = nullptr;
    unsigned long long *xcnt = nullptr;
    int32_t *lists = nullptr;      // vlist | ilist | tlist (several graphs)
    int64_t nvblk = 0;
    // lists
    Cross *x0 = nullptr, *x1 = nullptr;
    int64_t xcap = 0;
    unsigned long long *rcnt = nullptr;
    int4 *er = nullptr;
    int64_t ercap = 0;
    int32_t *arc_nxt = nullptr, *succ0 = nullptr, *succ1 = nullptr, *rank0 = nullptr, *rank1 = nullptr;
    PathReq *paths = nullptr;
    int64_t pathcap = 0;
    // paths longer than walk_k steps: their list, and the buffers of the
    // doubling pass that turns them (allocated when such a path first occurs)
    int32_t *lp_list = nullptr;
    int64_t lpcap = 0, walk_k = 0;
    int32_t *lp_p0 = nullptr, *lp_j0 = nullptr, *lp_j1 = nullptr;
    uint32_t *lp_mark = nullptr;
    uint32_t lp_epoch = 0;
    // path reversal by Euler tour (reverse_mode 1)
    uint64_t *et_keys = nullptr, *et_sorted = nullptr;
    int32_t *et_fc = nullptr, *et_ns = nullptr, *et_opar = nullptr, *et_nxt0 = nullptr,
            *et_nxt1 = nullptr, *et_dst0 = nullptr, *et_dst1 = nullptr, *et_start = nullptr,
            *et_finish = nullptr, *et_support = nullptr;
    uint8_t *et_tmp = nullptr;
    size_t et_tmp_bytes = 0;
    // supergraph replacement edges (replacement_mode 1)
    uint32_t *sg_rcount = nullptr, *sg_rpos = nullptr, *sg_flag = nullptr, *sg_segid = nullptr;
    uint64_t *sg_skeys = nullptr, *sg_svals = nullptr;
    unsigned long long *sg_totals = nullptr;
    uint8_t *sg_scan_tmp = nullptr, *sg_sort_tmp = nullptr;
    size_t sg_sort_bytes = 0;
    int round_base = 0;  // index of the first hooking round of the last update
    // pointer-jumping rounds queued before root finding's chase: 0 until a
    // delete finds the forest deep (a chase of more than DEEP_STEPS steps)
    int jump_rounds = 0;
    // the super-forest's Euler tour queued after the search (it skips itself
    // when the search sufficed), per update kind (bit kind): set once an
    // update of that kind needed it (tuning 0)
    unsigned lr_kinds = 0;
    // status word, counters and per-graph batch status share one allocation
    // so that one copy returns them: status at word 0, counters from word 1,
    // gstat after the counters
    unsigned long long *ctlmem = nullptr;
    int64_t ret_words = 0;
    int32_t *status = nullptr;
    unsigned long long *cnt = nullptr;
    Ctl *ctl = nullptr;
    // pinned host staging
    int32_t *h_edges = nullptr;           // [2 max_batch]
    int8_t *h_bop = nullptr;              // [max_batch]
    int32_t *h_bgid = nullptr;            // [max_batch]
    int32_t *h_lists = nullptr;           // vlist | ilist | tlist
    // Two slots of control block and returned words: an update can be
    // queued while the one before it runs.  Queued updates alternate between
    // the slots, others use slot 0; h_ctl, h_ret and h_gstat point into the
    // slot in use.
    Ctl *h_ctl_ring = nullptr;
    unsigned long long *h_ret_ring = nullptr;
    int slot = 0;
    int last_slot = 1;  // of the last update launched
    Ctl *h_ctl = nullptr;
    uint8_t *h_stage = nullptr;           // pinned staging of device-to-host copies (STAGE_BYTES)
    unsigned long long *h_ret = nullptr;  // copy of ctlmem, then scratch words; the last is the
                                          // completion word (seq of the finished update)
    uint64_t seq = 0;                     // updates launched
    int32_t *h_gstat = nullptr;           // [ngraph] inside h_ret
    // captured update sequences, by slot and kind (1 inserts, 2 deletes, 3 both)
    hipGraph_t graph[2][4] = {};
    hipGraphExec_t gexec[2][4] = {};
    int kind = 0;  // of the update being waited for
    int bor_fast = BOR_FAST, bfs_fast = BFS_FAST;
    // queued updates not yet waited for (the oldest is number seq - npend + 1)
    struct Pend {
        uint64_t seq;
        int kind, op;
        int64_t b;
    } pend[2] = {};
    int npend = 0;
    // results of updates that a call of the library waited for on the
    // caller's behalf (a drain before a call that needs the queue empty),
    // oldest first, until drsf_wait returns them (the two newest are kept)
    struct Done {
        int rc;
        drsf_view view;
    } done[2] = {};
    int ndone = 0;
    bool multi_last = false;
    std::vector<int64_t> last_bg;  // per-graph batch sizes of the last apply
    std::vector<int8_t> last_opg;  // per-graph op of the last apply
    int64_t last_b = 0;
    int last_op = 0;
    int last_rc = DRSF_OK;
    drsf_view view{};
    // phase boundaries [0, PH_N], an empty bracket, then the bracket of the
    // host-driven continuation
    hipEvent_t ev[PH_N + 5]{};
    bool ph_on[PH_N + 1]{};     // the phase recorded its event in the last enqueued update
    float phase_ms[PH_N + 2]{}; // phases, the host-driven continuation, the empty bracket
    bool cont_timed = false;    // the continuation of the last update recorded its events
    bool have_phases = false;
    std::string err;
    std::vector<void *> allocs;
    std::vector<size_t> alloc_bytes;
    int64_t bytes = 0, peak_bytes = 0;  // device bytes held now / at most
    int64_t rebuilds = 0;               // store rebuilds so far
    bool broken = false;                // a store rebuild failed after dropping the old store, or a
                                        // host continuation failed with an update held behind it
    // small graphs of a multi-graph context (drsf_opts.small_graph_vertices):
    // updated whole by one workgroup each, beside the chain, on stream s2
    int32_t nsg = 0, small_T = 0, small_threads = 512, small_grid = 0;
    std::vector<int32_t> g2s;            // graph -> small graph index, or -1
    std::vector<int32_t> sgid_h;
    std::vector<int64_t> scap_h, soff_h, svoff_h;
    int64_t pool_keys = 0, nsv = 0;
    int32_t *sgid = nullptr, *sm = nullptr, *sbuf = nullptr, *sok = nullptr;
    int64_t *soff = nullptr, *scap = nullptr, *svoff = nullptr;
    uint32_t *pool = nullptr, *xk = nullptr, *bkeys = nullptr, *htab = nullptr;
    int32_t *spar = nullptr, *slab = nullptr;
    int2 *ser = nullptr;
    int4 *stasks = nullptr, *h_stasks = nullptr;
    unsigned int *qhead = nullptr;
    hipStream_t s2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
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

#define HIPCHK(ctx, call)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail((ctx), DRSF_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));  \
    } while (0)

// Device memory through the caller's hooks when given, else hipMalloc.
void *raw_dalloc(const drsf_opts &o, size_t bytes) {
    if (o.dev_alloc) {
        void *q = o.dev_alloc(bytes, o.alloc_user);
        if (q && ((uintptr_t)q & 255u)) {  // the kernels' vector loads need aligned arrays
            o.dev_free(q, o.alloc_user);
            q = nullptr;
        }
        return q;
    }
    void *q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return q;
}
void raw_dfree(const drsf_opts &o, void *p) {
    if (!p) return;
    if (o.dev_alloc) o.dev_free(p, o.alloc_user);
    else (void)hipFree(p);
}

template <class T>
int dalloc(drsf_ctx *c, T **p, int64_t count) {
    const size_t bytes = sizeof(T) * (size_t)(count > 0 ? count : 1);
    void *q = raw_dalloc(c->opts, bytes);
    if (!q) return fail(c, DRSF_E_NOMEM, "device allocation of %zu bytes failed", bytes);
    c->allocs.push_back(q);
    c->alloc_bytes.push_back(bytes);
    c->bytes += (int64_t)bytes;
    c->peak_bytes = std::max(c->peak_bytes, c->bytes);
    *p = (T *)q;
    return DRSF_OK;
}

template <class T>
int halloc(drsf_ctx *c, T **p, int64_t count) {
    if (hipHostMalloc((void **)p, sizeof(T) * (size_t)(count > 0 ? count : 1)) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(c, DRSF_E_NOMEM, "pinned host allocation failed");
    }
    return DRSF_OK;
}

// Copies device memory to host memory that need not be pinned (a caller's
// array, a std::vector) through pinned staging, a chunk at a time: each
// chunk is complete in the pinned buffer once the stream is, and reaches the
// destination by a host copy after that.  No pageable destination is handed
// to the copy engine, so nothing can land in it after this returns.
constexpr size_t STAGE_BYTES = (size_t)1 << 20;
int d2h(drsf_ctx *c, void *dst, const void *src, size_t bytes) {
    if (bytes == 0) return DRSF_OK;
    int rc;
    if (!c->h_stage && (rc = halloc(c, &c->h_stage, (int64_t)STAGE_BYTES))) return rc;
    for (size_t off = 0; off < bytes; off += STAGE_BYTES) {
        const size_t len = std::min(STAGE_BYTES, bytes - off);
        HIPCHK(c, hipMemcpyAsync(c->h_stage, static_cast<const char *>(src) + off, len, hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        memcpy(static_cast<char *>(dst) + off, c->h_stage, len);
    }
    return DRSF_OK;
}

void dfree(drsf_ctx *c, void *p) {
    if (!p) return;
    auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
    if (it != c->allocs.end()) {
        const size_t k = (size_t)(it - c->allocs.begin());
        c->bytes -= (int64_t)c->alloc_bytes[k];
        c->alloc_bytes.erase(c->alloc_bytes.begin() + (std::ptrdiff_t)k);
        c->allocs.erase(it);
    }
    raw_dfree(c->opts, p);
}

Dev make_dev(drsf_ctx *c) {
    Dev d;
    memset(&d, 0, sizeof d);
    d.n = c->n;
    d.validate = c->opts.validate_batches != 0;
    d.gate = 1;
    d.lb = c->max_batch;
    d.ltiles = c->dtmax;
    d.ctl = c->ctl;
    d.ctlw = c->ctl;
    d.hctl = c->h_ctl;
    d.ctlmem = c->ctlmem;
    d.hret = c->h_ret;
    d.hdone = c->h_ret + c->ret_words + 7;
    d.ret_words = c->ret_words;
    d.bptr = c->bptr; d.bcol = c->bcol; d.eb = c->eb;
    d.lptr = c->lptr; d.lcol = c->lcol; d.twin = c->twin; d.ltwin = c->ltwin;
    d.nvb = c->nvb; d.bvol = c->bvol; d.bcnt = c->bcnt; d.bpre = c->bpre; d.opre = c->opre;
    d.olist = c->olist; d.rstart = c->rstart; d.xcnt = c->xcnt;
    d.gsum = c->gsum; d.gpre = c->gpre; d.gopre = c->gopre; d.ostage = c->ostage;
    d.zrow = c->zrow; d.zptr = c->zptr; d.nz = c->nz; d.tile_k = c->tile_k; d.ntiles = c->ntiles;
    d.dtmax = c->dtmax;
    d.dkey = c->dkey; d.dcap = c->dcap; d.dhash = c->dhash; d.dhpos = c->dhpos; d.dhmask = c->dhmask;
    d.parent = c->parent; d.label = c->label; d.rep = c->rep;
    d.obits = c->obits;
    d.tidx = c->tidx; d.owner = c->owner; d.pkeep = c->pkeep; d.prt = c->prt; d.pmin = c->pmin;
    d.comp = c->comp; d.hook = c->hook;
    d.best = c->best; d.srkey = c->srkey; d.head = c->head; d.newlab = c->newlab;
    d.level = c->level; d.parc = c->parc; d.pcap = c->pcap;
    d.bedges = c->bedges; d.bop = c->bop;
    d.bgid = c->ngraph > 1 ? c->bgid : nullptr;
    d.goff = c->ngraph > 1 ? c->goff : nullptr;
    d.gstat = c->gstat; d.max_b = c->max_batch;
    d.bkey = c->bkey; d.bloc = c->bloc; d.bchild = c->bchild;
    d.bslot = c->bslot; d.bhash = c->bhash; d.bhmask = c->bhmask;
    d.dslot = c->dslot; d.dsmask = c->dsmask;
    d.vlist = c->lists;
    d.ilist = c->lists ? c->lists + c->nvblk : nullptr;
    d.tlist = c->lists ? c->lists + 2 * c->nvblk : nullptr;
    d.x0 = c->x0; d.x1 = c->x1; d.xcap = c->xcap; d.rcnt = c->rcnt;
    d.er = c->er; d.ercap = c->ercap; d.arc_nxt = c->arc_nxt;
    d.succ0 = c->succ0; d.succ1 = c->succ1; d.rank0 = c->rank0; d.rank1 = c->rank1;
    d.paths = c->paths; d.pathcap = c->pathcap;
    d.lp_list = c->lp_list; d.lpcap = c->lpcap; d.walk_k = c->walk_k;
    d.et_keys = c->et_keys; d.et_sorted = c->et_sorted; d.et_fc = c->et_fc; d.et_ns = c->et_ns;
    d.et_opar = c->et_opar; d.et_nxt0 = c->et_nxt0; d.et_nxt1 = c->et_nxt1;
    d.et_dst0 = c->et_dst0; d.et_dst1 = c->et_dst1; d.et_start = c->et_start;
    d.et_finish = c->et_finish; d.et_support = c->et_support;
    d.status = c->status; d.cnt = c->cnt;
    return d;
}

SmallDev make_small(drsf_ctx *c) {
    SmallDev sd;
    memset(&sd, 0, sizeof sd);
    sd.nsg = c->nsg;
    sd.T = c->small_T;
    sd.sgid = c->sgid;
    sd.soff = c->soff;
    sd.scap = c->scap;
    sd.svoff = c->svoff;
    sd.sm = c->sm;
    sd.sbuf = c->sbuf;
    sd.sok = c->sok;
    sd.pool = c->pool;
    sd.xk = c->xk;
    sd.spar = c->spar;
    sd.slab = c->slab;
    sd.er = c->ser;
    sd.bkeys = c->bkeys;
    sd.htab = c->htab;
    sd.tasks = c->stasks;
    sd.qhead = c->qhead;
    return sd;
}

// live edges of the graphs in the edge store (the small graphs keep theirs apart)
int64_t store_edges(const drsf_ctx *c) {
    int64_t m = c->m_live;
    for (int32_t g = 0; g < c->nsg; g++) m -= c->gm_h[c->sgid_h[g]];
    return m;
}

int read_status(drsf_ctx *c, int32_t *st) {
    HIPCHK(c, hipMemcpyAsync(c->h_ret, c->status, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *st = *(int32_t *)c->h_ret;
    return DRSF_OK;
}

// Points h_ctl, h_ret and h_gstat at slot q.
void select_slot(drsf_ctx *c, int q) {
    c->slot = q;
    if (c->h_ctl_ring) c->h_ctl = c->h_ctl_ring + q;
    if (c->h_ret_ring) {
        c->h_ret = c->h_ret_ring + (size_t)q * (size_t)(c->ret_words + 8);
        c->h_gstat = reinterpret_cast<int32_t *>(c->h_ret + 1 + C_TOTAL);
    }
}

// Arrays sized by the base store's tiles: cross-edge regions (base-store
// tiles, inserted-edge tiles, batch regions), orphan-scan ranges and, with
// several graphs, the block and tile lists.  Called again after a rebuild.
int alloc_tiles(drsf_ctx *c) {
    int rc;
    dfree(c, c->x0); dfree(c, c->x1); dfree(c, c->rcnt); dfree(c, c->rstart); dfree(c, c->xcnt);
    dfree(c, c->sg_rcount); dfree(c, c->sg_rpos); dfree(c, c->sg_flag); dfree(c, c->sg_segid);
    dfree(c, c->sg_skeys); dfree(c, c->sg_svals); dfree(c, c->sg_totals); dfree(c, c->sg_scan_tmp);
    dfree(c, c->sg_sort_tmp);
    dfree(c, c->lists);
    if (c->h_lists) (void)hipHostFree(c->h_lists);
    c->h_lists = nullptr;
    const int64_t nregmax = c->ntiles + c->dtmax + insert_regions(c->max_batch);
    c->xcap = nregmax * TILE;
    if ((rc = dalloc(c, &c->x0, c->xcap))) return rc;
    if ((rc = dalloc(c, &c->x1, c->xcap))) return rc;
    if ((rc = dalloc(c, &c->rcnt, nregmax))) return rc;
    if ((rc = dalloc(c, &c->rstart, 2 * c->ntiles + 1))) return rc;
    if ((rc = dalloc(c, &c->xcnt, c->ntiles + 1))) return rc;
    launch_fill_u64(c->rcnt, nregmax, 0, c->stream);
    if (c->opts.replacement_mode == 1) {  // supergraph scratch, sized by the cross-edge slots
        if ((rc = dalloc(c, &c->sg_rcount, nregmax)) || (rc = dalloc(c, &c->sg_rpos, nregmax)) ||
            (rc = dalloc(c, &c->sg_flag, c->xcap)) || (rc = dalloc(c, &c->sg_segid, c->xcap)) ||
            (rc = dalloc(c, &c->sg_skeys, c->xcap)) || (rc = dalloc(c, &c->sg_svals, c->xcap)) ||
            (rc = dalloc(c, &c->sg_totals, 2)) ||
            (rc = dalloc(c, &c->sg_scan_tmp, (int64_t)scan_tmp_bytes(c->xcap) + 64)))
            return rc;
        c->sg_sort_bytes = sort_pairs_u64_tmp_bytes(c->xcap) + 256;
        if ((rc = dalloc(c, &c->sg_sort_tmp, (int64_t)c->sg_sort_bytes))) return rc;
    }
    if (c->ngraph > 1) {
        // every vertex block and every tile appears at most once per list
        c->nvblk = (c->n + BLOCK - 1) / BLOCK;
        const int64_t nl = 2 * c->nvblk + c->ntiles + 1;
        if ((rc = dalloc(c, &c->lists, nl))) return rc;
        if ((rc = halloc(c, &c->h_lists, nl))) return rc;
    }
    return DRSF_OK;
}

int alloc_state(drsf_ctx *c) {
    int rc;
    const int32_t n = c->n;
    const int64_t mb = c->max_batch;
    hipStream_t s = c->stream;
    if ((rc = dalloc(c, &c->label, n))) return rc;
    if ((rc = dalloc(c, &c->rep, n))) return rc;
    if ((rc = dalloc(c, &c->obits, (n + 63) / 64))) return rc;
    if ((rc = dalloc(c, &c->tidx, n))) return rc;
    if ((rc = dalloc(c, &c->owner, n))) return rc;
    c->pcap = 2 * mb + 16;  // a batch edge registers at most two pieces
    if ((rc = dalloc(c, &c->pkeep, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->prt, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->pmin, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->comp, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->hook, c->pcap))) return rc;  // set per piece at registration
    if ((rc = dalloc(c, &c->head, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->level, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->parc, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->newlab, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->best, 2 * c->pcap))) return rc;
    if ((rc = dalloc(c, &c->srkey, c->pcap))) return rc;
    if ((rc = dalloc(c, &c->bedges, 2 * mb))) return rc;
    if ((rc = dalloc(c, &c->bop, mb))) return rc;
    if ((rc = dalloc(c, &c->bgid, mb))) return rc;
    if ((rc = dalloc(c, &c->bkey, mb))) return rc;
    if ((rc = dalloc(c, &c->bloc, mb))) return rc;
    if ((rc = dalloc(c, &c->bchild, mb))) return rc;
    if ((rc = dalloc(c, &c->bslot, mb))) return rc;
    uint64_t bh = 16;
    while (bh < (uint64_t)(2 * mb)) bh <<= 1;
    c->bhmask = bh - 1;
    if ((rc = dalloc(c, &c->bhash, (int64_t)bh))) return rc;
    // slot table at load <= 1/8: about 1 edge in 16 collides and takes the
    // claim table; never cleared (only slots written by the batch are read)
    uint64_t ds = 16;
    while (ds < (uint64_t)(8 * mb)) ds <<= 1;
    c->dsmask = ds - 1;
    if ((rc = dalloc(c, &c->dslot, (int64_t)ds))) return rc;
    c->dcap = c->opts.delta_capacity > 0 ? c->opts.delta_capacity
                                         : std::max<int64_t>({4 * mb, c->eb / 8, 1 << 20});
    c->dtmax = delta_tiles(c->dcap);
    if ((rc = dalloc(c, &c->dkey, c->dcap))) return rc;
    uint64_t dh = 16;
    while (dh < (uint64_t)(2 * c->dcap)) dh <<= 1;
    c->dhmask = dh - 1;
    if ((rc = dalloc(c, &c->dhash, (int64_t)dh))) return rc;
    if ((rc = dalloc(c, &c->dhpos, (int64_t)dh))) return rc;
    if ((rc = alloc_tiles(c))) return rc;
    c->ercap = c->pcap;
    if ((rc = dalloc(c, &c->er, c->ercap))) return rc;
    if ((rc = dalloc(c, &c->arc_nxt, 2 * c->ercap))) return rc;
    if ((rc = dalloc(c, &c->succ0, 2 * c->ercap))) return rc;
    if ((rc = dalloc(c, &c->succ1, 2 * c->ercap))) return rc;
    if ((rc = dalloc(c, &c->rank0, 2 * c->ercap))) return rc;
    if ((rc = dalloc(c, &c->rank1, 2 * c->ercap))) return rc;
    c->pathcap = std::max<int64_t>(c->ercap + c->pcap, n);
    if ((rc = dalloc(c, &c->paths, c->pathcap))) return rc;
    c->walk_k = c->opts.walk_limit > 0 ? c->opts.walk_limit : WALK_LIMIT;
    c->lpcap = n / (c->walk_k + 2) + 1;
    if ((rc = dalloc(c, &c->lp_list, c->lpcap))) return rc;
    if (c->opts.reverse_mode == 1) {  // path reversal by Euler tour
        if ((rc = dalloc(c, &c->et_keys, n))) return rc;
        if ((rc = dalloc(c, &c->et_sorted, n))) return rc;
        if ((rc = dalloc(c, &c->et_fc, n))) return rc;
        if ((rc = dalloc(c, &c->et_ns, n))) return rc;
        if ((rc = dalloc(c, &c->et_opar, n))) return rc;
        if ((rc = dalloc(c, &c->et_nxt0, 2 * (int64_t)n))) return rc;
        if ((rc = dalloc(c, &c->et_nxt1, 2 * (int64_t)n))) return rc;
        if ((rc = dalloc(c, &c->et_dst0, 2 * (int64_t)n))) return rc;
        if ((rc = dalloc(c, &c->et_dst1, 2 * (int64_t)n))) return rc;
        if ((rc = dalloc(c, &c->et_start, n))) return rc;
        if ((rc = dalloc(c, &c->et_finish, n))) return rc;
        if ((rc = dalloc(c, &c->et_support, n))) return rc;
        c->et_tmp_bytes = sort_u64_tmp_bytes(n) + 256;
        if ((rc = dalloc(c, &c->et_tmp, (int64_t)c->et_tmp_bytes))) return rc;
        launch_fill_i32(c->et_support, n, NONE, s);
    }
    if ((rc = dalloc(c, &c->ctl, 1))) return rc;
    // orphan scan: per-block figures (zero between updates), list, ranges
    c->nvb = (n + BLOCK - 1) / BLOCK;
    if ((rc = dalloc(c, &c->bvol, c->nvb))) return rc;
    if ((rc = dalloc(c, &c->bcnt, c->nvb))) return rc;
    if ((rc = dalloc(c, &c->bpre, c->nvb))) return rc;
    if ((rc = dalloc(c, &c->opre, c->nvb))) return rc;
    if ((rc = dalloc(c, &c->gsum, (c->nvb + BLOCK - 1) / BLOCK))) return rc;
    if ((rc = dalloc(c, &c->gpre, (c->nvb + BLOCK - 1) / BLOCK))) return rc;
    if ((rc = dalloc(c, &c->gopre, (c->nvb + BLOCK - 1) / BLOCK))) return rc;
    if ((rc = dalloc(c, &c->olist, n))) return rc;
    if ((rc = dalloc(c, &c->ostage, c->nvb * BLOCK))) return rc;
    launch_fill_u64(reinterpret_cast<uint64_t *>(c->bvol), c->nvb, 0, s);
    launch_fill_i32(c->bcnt, c->nvb, 0, s);
    if ((rc = halloc(c, &c->h_edges, 2 * mb))) return rc;
    if ((rc = halloc(c, &c->h_bop, mb))) return rc;
    if ((rc = halloc(c, &c->h_bgid, mb))) return rc;
    if ((rc = halloc(c, &c->h_ctl_ring, 2))) return rc;
    select_slot(c, c->slot);
    launch_fill_i32(c->tidx, n, NONE, s);
    launch_fill_i32(c->level, c->pcap, -1, s);  // the search state is reset by each update's cleanup
    launch_fill_i32(c->parc, c->pcap, NONE, s);
    launch_fill_u64(c->bhash, (int64_t)bh, HASH_EMPTY, s);
    launch_fill_u64(c->dhash, (int64_t)dh, HASH_EMPTY, s);
    launch_fill_u64(c->obits, (n + 63) / 64, 0, s);
    return DRSF_OK;
}

// Drops the captured update sequences (the next update captures anew with
// the context's current round and level counts and buffers).
void drop_graphs(drsf_ctx *c) {
    for (int q = 0; q < 2; q++)
        for (int k = 0; k < 4; k++) {
            if (c->gexec[q][k]) (void)hipGraphExecDestroy(c->gexec[q][k]);
            if (c->graph[q][k]) (void)hipGraphDestroy(c->graph[q][k]);
            c->gexec[q][k] = nullptr;
            c->graph[q][k] = nullptr;
        }
}

void destroy_ctx(drsf_ctx *c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->s2) (void)hipStreamSynchronize(c->s2);
    drop_graphs(c);
    for (void *p : c->allocs) raw_dfree(c->opts, p);
    c->allocs.clear();
    void *hosts[] = {c->h_edges, c->h_bop, c->h_bgid, c->h_lists, c->h_ctl_ring, c->h_ret_ring, c->h_stage};
    for (void *p : hosts)
        if (p) (void)hipHostFree(p);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->h_stasks) (void)hipHostFree(c->h_stasks);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->s2) (void)hipStreamDestroy(c->s2);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

// Builds the device edge store from a symmetric CSR with ascending rows.
int build_store(drsf_ctx *c, const int64_t *row_ptr_in, const int32_t *col_in, int64_t nnz, bool dev_in) {
    int rc;
    const int32_t n = c->n;
    hipStream_t s = c->stream;
    int64_t *drow = nullptr;
    int32_t *dcol = nullptr;
    if (dev_in) {
        drow = const_cast<int64_t *>(row_ptr_in);
        dcol = const_cast<int32_t *>(col_in);
    } else {
        if ((rc = dalloc(c, &drow, (int64_t)n + 1))) return rc;
        if ((rc = dalloc(c, &dcol, nnz))) return rc;
        HIPCHK(c, hipMemcpyAsync(drow, row_ptr_in, sizeof(int64_t) * ((size_t)n + 1),
                                 hipMemcpyHostToDevice, s));
        if (nnz > 0)
            HIPCHK(c, hipMemcpyAsync(dcol, col_in, sizeof(int32_t) * (size_t)nnz,
                                     hipMemcpyHostToDevice, s));
    }
    uint32_t *ucnt = nullptr;
    char *tmp = nullptr;
    if ((rc = dalloc(c, &ucnt, n))) return rc;
    if ((rc = dalloc(c, &tmp, (int64_t)scan_tmp_bytes(n) + 64))) return rc;
    if ((rc = dalloc(c, &c->bptr, (int64_t)n + 1))) return rc;
    unsigned long long *dtotal = (unsigned long long *)(tmp + scan_tmp_bytes(n));
    launch_fill_i32(c->status, 1, 0, s);
    launch_csr_check(n, drow, dcol, nnz, ucnt, c->status, c->ngraph > 1 ? c->goff : nullptr, c->ngraph, s);
    launch_scan_u32(ucnt, c->bptr, dtotal, n, tmp, s);
    HIPCHK(c, hipMemcpyAsync(c->h_ret, dtotal, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(c->h_ret + 1, c->status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const unsigned long long total = c->h_ret[0];
    const int32_t st = *(int32_t *)(c->h_ret + 1);
    if (st & 1)
        return fail(c, DRSF_E_ARG, "CSR rows must be strictly ascending, without self-loops, with ids in range%s",
                    c->ngraph > 1 ? " of the row's graph" : "");
    if (2 * (int64_t)total != nnz) return fail(c, DRSF_E_ARG, "CSR is not symmetric");
    if (total >= 0xffffffffull) return fail(c, DRSF_E_CAPACITY, "more than 2^32-1 undirected edges");
    c->eb = (int64_t)total;
    c->ntiles = (c->eb + TILE - 1) / TILE;
    // padded to whole sweep tiles with deleted entries
    if ((rc = dalloc(c, &c->bcol, c->ntiles * TILE))) return rc;
    launch_fill_i32(c->bcol + c->eb, c->ntiles * TILE - c->eb, TOMB, s);
    launch_upper_fill(n, drow, dcol, c->bptr, c->bcol, c->eb, s);
    // lower half (row v holds u < v), for the orphan scan
    launch_lower_counts(n, drow, c->bptr, ucnt, s);
    if ((rc = dalloc(c, &c->lptr, (int64_t)n + 1))) return rc;
    launch_scan_u32(ucnt, c->lptr, dtotal, n, tmp, s);
    if ((rc = dalloc(c, &c->lcol, c->eb))) return rc;
    launch_lower_fill(n, drow, dcol, c->lptr, c->lcol, c->eb, s);
    if ((rc = dalloc(c, &c->twin, c->eb))) return rc;
    if ((rc = dalloc(c, &c->ltwin, c->eb))) return rc;
    // every lower entry finds its mirror in the upper half: with equal halves
    // this is the symmetry check
    launch_twin(n, c->bptr, c->bcol, c->lptr, c->lcol, c->twin, c->ltwin, c->status, c->eb, s);
    {
        int32_t st2;
        if ((rc = read_status(c, &st2))) return rc;
        if (st2 & 2) return fail(c, DRSF_E_ARG, "CSR is not symmetric");
    }
    // non-empty-row index for the sweep
    launch_nonempty_flags(n, c->bptr, ucnt, s);
    uint32_t *zpos = nullptr;
    if ((rc = dalloc(c, &zpos, (int64_t)n + 1))) return rc;
    launch_scan_u32(ucnt, zpos, dtotal, n, tmp, s);
    HIPCHK(c, hipMemcpyAsync(c->h_ret, dtotal, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    c->nz = (int64_t)c->h_ret[0];
    if ((rc = dalloc(c, &c->zrow, c->nz))) return rc;
    if ((rc = dalloc(c, &c->zptr, c->nz + 1))) return rc;
    launch_nonempty_fill(n, c->bptr, zpos, c->zrow, c->zptr, c->nz, s);
    if ((rc = dalloc(c, &c->tile_k, c->ntiles + 1))) return rc;
    launch_tile_k(c->zptr, c->nz, c->eb, c->tile_k, c->ntiles, s);
    // base-store offsets of each graph's rows (host copy, for the tile lists)
    std::vector<uint32_t> bp((size_t)n + 1);
    if ((rc = d2h(c, bp.data(), c->bptr, sizeof(uint32_t) * bp.size()))) return rc;
    c->gedge_h.assign((size_t)c->ngraph + 1, 0);
    c->gm_h.assign((size_t)c->ngraph, 0);
    for (int32_t g = 0; g <= c->ngraph; g++) c->gedge_h[g] = bp[c->goff_h[g]];
    for (int32_t g = 0; g < c->ngraph; g++) c->gm_h[g] = c->gedge_h[g + 1] - c->gedge_h[g];
    dfree(c, zpos);
    dfree(c, ucnt);
    dfree(c, tmp);
    if (!dev_in) { dfree(c, drow); dfree(c, dcol); }
    c->m_live = c->eb;
    return DRSF_OK;
}

// Small graphs of a multi-graph context: graphs with at most small_T
// vertices move out of the edge store into key arrays of their own (see
// drsf_small.hip); their entries in the store are marked deleted.
int setup_small(drsf_ctx *c) {
    int rc;
    hipStream_t s = c->stream;
    c->g2s.assign((size_t)c->ngraph, -1);
    for (int32_t g = 0; g < c->ngraph; g++) {
        const int32_t ng = c->goff_h[g + 1] - c->goff_h[g];
        if (ng >= 1 && ng <= c->small_T) {
            c->g2s[g] = (int32_t)c->sgid_h.size();
            c->sgid_h.push_back(g);
        }
    }
    c->nsg = (int32_t)c->sgid_h.size();
    if (c->nsg == 0) return DRSF_OK;
    c->scap_h.resize((size_t)c->nsg);
    c->soff_h.resize((size_t)c->nsg);
    c->svoff_h.resize((size_t)c->nsg);
    int64_t off = 0, voff = 0;
    for (int32_t k = 0; k < c->nsg; k++) {
        const int32_t g = c->sgid_h[k];
        const int64_t m = c->gm_h[g];
        c->scap_h[k] = std::max<int64_t>(2 * m, m + 4096);  // room for inserts before the pool grows
        c->soff_h[k] = off;
        off += 2 * c->scap_h[k];
        c->svoff_h[k] = voff;
        voff += c->goff_h[g + 1] - c->goff_h[g];
    }
    c->pool_keys = off;
    c->nsv = voff;
    if ((rc = dalloc(c, &c->sgid, c->nsg)) || (rc = dalloc(c, &c->sm, c->nsg)) || (rc = dalloc(c, &c->sbuf, c->nsg)) ||
        (rc = dalloc(c, &c->sok, c->nsg)) || (rc = dalloc(c, &c->soff, c->nsg)) ||
        (rc = dalloc(c, &c->scap, c->nsg)) || (rc = dalloc(c, &c->svoff, c->nsg)) ||
        (rc = dalloc(c, &c->pool, c->pool_keys)) || (rc = dalloc(c, &c->xk, c->pool_keys)) ||
        (rc = dalloc(c, &c->spar, c->nsv)) || (rc = dalloc(c, &c->slab, c->nsv)) ||
        (rc = dalloc(c, &c->ser, c->nsv)) || (rc = dalloc(c, &c->bkeys, c->max_batch)) ||
        (rc = dalloc(c, &c->htab, 2 * c->max_batch + 4 * (int64_t)c->nsg)) || (rc = dalloc(c, &c->stasks, c->nsg)) ||
        (rc = dalloc(c, &c->qhead, 1)))
        return rc;
    if ((rc = halloc(c, &c->h_stasks, c->nsg))) return rc;
    HIPCHK(c, hipMemcpyAsync(c->sgid, c->sgid_h.data(), 4 * (size_t)c->nsg, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->soff, c->soff_h.data(), 8 * (size_t)c->nsg, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->scap, c->scap_h.data(), 8 * (size_t)c->nsg, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->svoff, c->svoff_h.data(), 8 * (size_t)c->nsg, hipMemcpyHostToDevice, s));
    launch_fill_i32(reinterpret_cast<int32_t *>(c->qhead), 1, 0, s);
    launch_small_init(make_dev(c), make_small(c), s);
    HIPCHK(c, hipStreamSynchronize(s));  // the pageable metadata sources
    if (hipStreamCreateWithFlags(&c->s2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, DRSF_E_DEVICE, "stream or event creation failed");
    }
    return DRSF_OK;
}

// Workgroups of the small-graph kernel: as many as fit on the device at once
// (by its LDS), at most one per small graph.
int small_grid_for(drsf_ctx *c) {
    int cus = 256, lds_cu = 160 * 1024;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->dev);
    (void)hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, c->dev);
    const int64_t per = (int64_t)(small_lds_bytes(c->small_T) + small_static_lds());
    const int64_t fit = std::max<int64_t>(1, lds_cu / per) * cus;
    return (int)std::max<int64_t>(1, std::min<int64_t>(fit, c->nsg));
}

// Makes room for more keys in the small graphs' buffers (an insert would
// not fit): every graph's capacity doubles (at least to what it needs), so
// that the next growth is far off for all of them, the live keys move to a
// new pool, and the captured update graphs (which hold the old pool) are
// dropped; snapshots taken before cannot be restored.
int small_grow(drsf_ctx *c, const std::vector<int64_t> &need) {
    int rc;
    hipStream_t s = c->stream;
    std::vector<int64_t> cap = c->scap_h, off((size_t)c->nsg);
    int64_t tot = 0;
    for (int32_t k = 0; k < c->nsg; k++) {
        cap[k] = std::max<int64_t>(need[k], 2 * cap[k]);
        off[k] = tot;
        tot += 2 * cap[k];
    }
    uint32_t *np = nullptr, *nx = nullptr;
    int64_t *noc = nullptr;  // the new offsets, then the new capacities
    if ((rc = dalloc(c, &np, tot)) || (rc = dalloc(c, &nx, tot)) || (rc = dalloc(c, &noc, 2 * (int64_t)c->nsg))) {
        dfree(c, np);
        dfree(c, nx);
        return rc;
    }
    HIPCHK(c, hipMemcpyAsync(noc, off.data(), 8 * off.size(), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(noc + c->nsg, cap.data(), 8 * cap.size(), hipMemcpyHostToDevice, s));
    // one kernel moves every graph's live keys (queued after any update
    // still using the old pool)
    launch_small_regrow(make_dev(c), make_small(c), noc, np, s);
    HIPCHK(c, hipMemcpyAsync(c->soff, noc, 8 * off.size(), hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->scap, noc + c->nsg, 8 * cap.size(), hipMemcpyDeviceToDevice, s));
    launch_fill_i32(c->sbuf, c->nsg, 0, s);
    HIPCHK(c, hipStreamSynchronize(s));
    dfree(c, noc);
    dfree(c, c->pool);
    dfree(c, c->xk);
    c->pool = np;
    c->xk = nx;
    c->scap_h = cap;
    c->soff_h = off;
    c->pool_keys = tot;
    c->rebuilds++;
    drop_graphs(c);
    return DRSF_OK;
}

// Turns the paths that an update's walks left to the doubling pass (nlong
// of them, listed on the device); allocates the pass's buffers the first
// time.
int reverse_long_paths(drsf_ctx *c, const Dev &d, int64_t nlong, hipStream_t s) {
    const int64_t n = c->n;
    int rc;
    if (!c->lp_p0 && (rc = dalloc(c, &c->lp_p0, n))) return rc;
    if (!c->lp_j0 && (rc = dalloc(c, &c->lp_j0, n))) return rc;
    if (!c->lp_j1 && (rc = dalloc(c, &c->lp_j1, n))) return rc;
    if (!c->lp_mark) {
        if ((rc = dalloc(c, &c->lp_mark, n))) return rc;
        c->lp_epoch = 0;
        launch_fill_i32((int32_t *)c->lp_mark, n, 0, s);
    }
    if (++c->lp_epoch == 0) {  // wrapped: clear the marks so that none equals the epoch
        launch_fill_i32((int32_t *)c->lp_mark, n, 0, s);
        c->lp_epoch = 1;
    }
    LongPaths b;
    b.p0 = c->lp_p0; b.j0 = c->lp_j0; b.j1 = c->lp_j1; b.mark = c->lp_mark;
    b.epoch = c->lp_epoch;
    b.nlong = std::min(nlong, c->lpcap);  // more were listed only if the update failed
    launch_long_paths(d, b, s);
    return DRSF_OK;
}

// Checks the forest (optional) and roots every tree at its smallest vertex.
int canonicalise_forest(drsf_ctx *c) {
    const int32_t n = c->n;
    hipStream_t s = c->stream;
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
        // a tree deeper than 2^16: deletes queue jumping rounds before
        // root finding's chase from the first one on
        if (r + 1 == CREATE_DEEP_LOG) launch_deeper_than(n, a, c->cnt + C_DEEP, s);
    }
    int32_t *root = a;
    if (root == c->label) {  // keep roots in rep, labels in label
        HIPCHK(c, hipMemcpyAsync(c->rep, root, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
        root = c->rep;
    }
    launch_roots_check(n, c->parent, root, c->status, s);
    const Dev d = make_dev(c);
    if (c->opts.validate_forest) launch_span_check(d, root, s);
    if ((rc = read_status(c, &st))) return rc;
    if (st & 4) return fail(c, DRSF_E_FOREST, "parent[] contains a cycle");
    if (st & 8) return fail(c, DRSF_E_FOREST, "a tree does not span its connected component");
    // label <- smallest vertex of each tree; re-root where that is not the root
    launch_tree_min(n, root, c->label, s);
    launch_reroot_requests(d, root, s);
    launch_reverse_all(d, s);
    // paths too long for one thread's walk: the doubling pass
    HIPCHK(c, hipMemcpyAsync(c->h_ret + 1, c->cnt + C_NLONG, sizeof(unsigned long long),
                             hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(c->h_ret + 2, c->cnt + C_DEEP, sizeof(unsigned long long),
                             hipMemcpyDeviceToHost, s));
    if ((rc = read_status(c, &st))) return rc;
    if (!st && c->h_ret[2]) c->jump_rounds = std::min(ceil_log2(n) + 1, MAX_JUMP);
    if (!st && c->h_ret[1] > 0 && (rc = reverse_long_paths(c, d, (int64_t)c->h_ret[1], s))) return rc;
    if ((rc = read_status(c, &st))) return rc;
    if (st) return fail(c, DRSF_E_DEVICE, "re-rooting failed (status %d)", st);
    launch_fill_u64(c->cnt, C_TOTAL, 0, s);
    // invariant between updates: rep == label
    HIPCHK(c, hipMemcpyAsync(c->rep, c->label, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return DRSF_OK;
}


// Merges the inserted-edge list into the base store and drops deleted
// entries: the live edges become one symmetric CSR (rows of live base
// entries merged with the sorted inserted pairs), from which the store is
// built as at create.  The forest is untouched.  Captured update graphs
// hold the old arrays and are dropped.
int rebuild_store(drsf_ctx *c) {
    int rc;
    hipStream_t s = c->stream;
    const int32_t n = c->n;
    HIPCHK(c, hipMemcpyAsync(c->h_ret, c->cnt + C_NDELTA, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const int64_t nd = (int64_t)c->h_ret[0];
    const int64_t pcap2 = 2 * nd + 2;
    uint64_t *pairs = nullptr, *sorted = nullptr;
    unsigned long long *npairs = nullptr, *dtot = nullptr;
    uint32_t *ddeg = nullptr, *dstart = nullptr, *bdeg = nullptr, *rowp32 = nullptr;
    uint32_t *flag = nullptr, *LS = nullptr, *US = nullptr;  // live prefix counts of the two halves
    char *stmp = nullptr, *ctmp = nullptr, *etmp = nullptr;
    const int64_t eb = c->eb;
    int64_t *rowp = nullptr;
    int32_t *col = nullptr;
    const size_t sbytes = sort_u64_tmp_bytes(pcap2) + 256;
    // temporaries are released on every return; the old store is kept until
    // the merged CSR exists, so a failure before that leaves the context as
    // it was
    auto release = [&](int code) {
        for (void *p : {(void *)pairs, (void *)sorted, (void *)npairs, (void *)stmp, (void *)ddeg, (void *)dstart,
                        (void *)bdeg, (void *)rowp32, (void *)ctmp, (void *)rowp, (void *)col, (void *)flag,
                        (void *)LS, (void *)US, (void *)etmp})
            dfree(c, p);
        return code;
    };
    if ((rc = dalloc(c, &pairs, pcap2)) || (rc = dalloc(c, &sorted, pcap2)) || (rc = dalloc(c, &npairs, 2)) ||
        (rc = dalloc(c, &stmp, (int64_t)sbytes)) || (rc = dalloc(c, &ddeg, n)) ||
        (rc = dalloc(c, &dstart, (int64_t)n + 1)) || (rc = dalloc(c, &bdeg, n)) ||
        (rc = dalloc(c, &rowp32, (int64_t)n + 1)) || (rc = dalloc(c, &rowp, (int64_t)n + 1)) ||
        (rc = dalloc(c, &ctmp, (int64_t)scan_tmp_bytes(n) + 64)) || (rc = dalloc(c, &flag, eb)) ||
        (rc = dalloc(c, &LS, eb + 1)) || (rc = dalloc(c, &US, eb + 1)) ||
        (rc = dalloc(c, &etmp, (int64_t)scan_tmp_bytes(eb) + 64))) {
        (void)hipStreamSynchronize(s);
        return release(rc);
    }
    dtot = npairs + 1;
    launch_fill_u64(npairs, 2, 0, s);
    launch_rb_pairs(c->dkey, c->cnt + C_NDELTA, pairs, npairs, pcap2, s);
    HIPCHK(c, hipMemcpyAsync(c->h_ret, npairs, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const int64_t np = (int64_t)c->h_ret[0];
    if (np > 0 && launch_sort_u64(pairs, sorted, np, stmp, sbytes, s) != 0) {
        (void)hipStreamSynchronize(s);
        return release(fail(c, DRSF_E_DEVICE, "sort failed during the store rebuild"));
    }
    launch_fill_i32(reinterpret_cast<int32_t *>(ddeg), n, 0, s);
    launch_rb_pair_deg(sorted, npairs, ddeg, pcap2, s);
    launch_scan_u32(ddeg, dstart, dtot, n, ctmp, s);
    launch_rb_live(c->lcol, eb, flag, s);
    launch_scan_u32(flag, LS, dtot, eb, etmp, s);
    launch_rb_live(c->bcol, eb, flag, s);
    launch_scan_u32(flag, US, dtot, eb, etmp, s);
    launch_rb_row_count(n, c->bptr, c->lptr, LS, US, ddeg, bdeg, s);
    launch_scan_u32(bdeg, rowp32, dtot, n, ctmp, s);
    HIPCHK(c, hipMemcpyAsync(c->h_ret, dtot, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const int64_t nnz = (int64_t)c->h_ret[0];
    if (nnz != 2 * store_edges(c))
        return release(fail(c, DRSF_E_DEVICE, "store rebuild counted %lld entries, expected %lld",
                            (long long)nnz, (long long)(2 * store_edges(c))));
    if ((rc = dalloc(c, &col, nnz))) return release(rc);
    launch_u32_to_i64(rowp32, rowp, (int64_t)n + 1, s);
    launch_rb_fill(n, eb, c->bptr, c->bcol, c->lptr, c->lcol, LS, US, sorted, npairs, pcap2, dstart, ddeg, rowp,
                   col, s);
    if (hipStreamSynchronize(s) != hipSuccess)
        return release(fail(c, DRSF_E_DEVICE, "store rebuild: %s", hipGetErrorString(hipGetLastError())));
    for (void *p : {(void *)pairs, (void *)sorted, (void *)npairs, (void *)stmp, (void *)ddeg, (void *)dstart,
                    (void *)bdeg, (void *)rowp32, (void *)ctmp, (void *)flag, (void *)LS, (void *)US,
                    (void *)etmp})
        dfree(c, p);
    // past this point a failure leaves no store: the context only answers
    // reads of its forest (parent, label) until destroyed
    c->broken = true;
    for (void *p : {(void *)c->bptr, (void *)c->bcol, (void *)c->lptr, (void *)c->lcol, (void *)c->twin,
                    (void *)c->ltwin, (void *)c->zrow, (void *)c->zptr, (void *)c->tile_k})
        dfree(c, p);
    c->bptr = c->lptr = nullptr;
    c->bcol = c->lcol = c->zrow = c->tile_k = nullptr;
    c->twin = c->ltwin = c->zptr = nullptr;
    const int64_t old_tiles = c->ntiles;
    rc = build_store(c, rowp, col, nnz, true);
    dfree(c, rowp);
    dfree(c, col);
    if (rc) return rc;
    if (c->ntiles > old_tiles && (rc = alloc_tiles(c))) return rc;
    // empty inserted-edge list
    launch_fill_u64(c->cnt + C_NDELTA, 1, 0, s);
    launch_fill_u64(c->dhash, (int64_t)c->dhmask + 1, HASH_EMPTY, s);
    c->ndelta_bound = 0;
    c->rebuilds++;
    HIPCHK(c, hipStreamSynchronize(s));
    c->broken = false;
    drop_graphs(c);
    return DRSF_OK;
}

// Supergraph mode: reads the orphan-scan mode and the region sizes back,
// then queues the reduction of the first round's cross edges to one per pair
// of pieces (dense in x0 for the rounds from SG_ROUND0).
int sg_reduce(drsf_ctx *c, const Dev &d, hipStream_t s) {
    unsigned long long *f = c->h_ret + c->ret_words + 3;  // [0] status, [1] scan mode, [2] slots
    HIPCHK(c, hipMemcpyAsync(f, c->status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(f + 1, c->cnt + C_OMODE, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(f + 2, c->cnt + C_OVOL, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (*(int32_t *)f != 0) return DRSF_OK;  // failed already: the rounds skip themselves
    const bool om = f[1] != 0;
    const int64_t nr_om = om ? or_regions((int64_t)f[2], c->eb) : 0;
    const Ctl &k = *c->h_ctl;
    const int64_t rlo2 = om ? std::max<int64_t>(k.rlo, c->ntiles) : k.rlo;
    const int64_t nreg = nr_om + std::max<int64_t>(k.rhi - rlo2, 0);
    SgScratch g;
    g.rcount = c->sg_rcount;
    g.rpos = c->sg_rpos;
    g.flag = c->sg_flag;
    g.segid = c->sg_segid;
    g.skeys = c->sg_skeys;
    g.svals = c->sg_svals;
    g.totals = c->sg_totals;
    g.scan_tmp = c->sg_scan_tmp;
    g.sort_tmp = c->sg_sort_tmp;
    g.sort_tmp_bytes = c->sg_sort_bytes;
    launch_sg_regions(d, nr_om, rlo2, nreg, g, s);
    HIPCHK(c, hipMemcpyAsync(f, c->sg_totals, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const int64_t total = (int64_t)f[0];
    if (total > c->xcap) return fail(c, DRSF_E_DEVICE, "supergraph: %lld cross edges", (long long)total);
    if (launch_sg_reduce(d, nr_om, rlo2, nreg, total, g, s))
        return fail(c, DRSF_E_DEVICE, "supergraph: radix sort failed");
    return DRSF_OK;
}

// List-ranking rounds of the super-forest's Euler tour: enough for a tour
// of every piece the context can register.
int tour_rounds(const drsf_ctx *c) { return std::min(ceil_log2(2 * c->pcap + 2) + 2, MAX_ROUNDS); }

// The update sequence (see the file comment) for batches with inserts
// (kind bit 1) and/or deletes (kind bit 2); with events when profiling.
// kc: the control block, passed with the first kernel when the sequence is
// launched kernel by kernel (null while capturing: read from pinned memory).
void enqueue_update(drsf_ctx *c, int kind, bool profile, const Ctl *kc) {
    Dev d = make_dev(c);
    if (kc) {  // launched kernel by kernel: grids sized for this batch and list
        d.lb = std::max<int64_t>(kc->b, 1);
        d.ltiles = delta_tiles(c->ndelta_bound);
    }
    hipStream_t s = c->stream;
    const bool ins = kind & 1, del = kind & 2;
    // a phase that launches nothing for this kind records no event (an
    // event record costs a few microseconds of its own) and reads zero
    auto mark = [&](int i, bool on = true) {
        c->ph_on[i] = on;
        if (profile && on) (void)hipEventRecord(c->ev[i], s);
    };
    if (profile) {  // two events back to back: the fixed cost a phase time includes
        (void)hipEventRecord(c->ev[PH_N + 1], s);
        (void)hipEventRecord(c->ev[PH_N + 2], s);
    }
    const bool small = c->nsg > 0;
    if (small && c->nsg == c->ngraph) {
        // every graph is small: the engine alone, then its commit and the
        // cleanup (no kernel sequence; its time counts as replacement edges)
        for (int i = 0; i < PH_N; i++)
            if (i != PH_REPL) mark(i, false);
        mark(PH_REPL);
        if (launch_small_update(d, make_small(c), c->small_threads, c->small_grid, s))
            launch_fill_i32(c->status, 1, ST_ROUND_BOUND, s);
        mark(PH_N);
        launch_small_commit(d, make_small(c), grid_for(c->nsg, 1, GRID_CAP), true, s);
        launch_cleanup(d, s);
        return;
    }
    if (small) {  // the small graphs' kernel on its own branch
        (void)hipEventRecord(c->ev_fork, s);
        (void)hipStreamWaitEvent(c->s2, c->ev_fork, 0);
        if (launch_small_update(d, make_small(c), c->small_threads, c->small_grid, c->s2))
            launch_fill_i32(c->status, 1, ST_ROUND_BOUND, c->s2);
        (void)hipEventRecord(c->ev_join, c->s2);
    }
    mark(PH_VALIDATE);
    launch_classify(d, kc, s);
    if (c->opts.validate_batches) launch_dedupe(d, s);
    mark(PH_UPDATE);
    launch_prepare(d, del, s);
    launch_register(d, s);
    mark(PH_ROOT, del);
    if (del && c->jump_rounds) launch_rep_jump(d, c->jump_rounds, s);
    if (del) launch_rep_chase(d, s);
    mark(PH_ORPH_LIST, del);
    if (del) {
        launch_orphan_plan(d, s);
        launch_orphan_fill(d, s);
    }
    mark(PH_ORPH_SCAN, del);
    if (del) launch_orphan_scan(d, s);
    mark(PH_SWEEP, del);
    if (del) launch_sweep_base(d, s);
    mark(PH_SWEEP_DELTA);
    // the supergraph reads the insert regions before the rounds; otherwise
    // the first round emits them itself
    const bool sg = c->opts.replacement_mode == 1;
    if (ins && sg) launch_insert_emit(d, s);
    if (del) launch_sweep_delta(d, s);
    mark(PH_REPL);
    const int64_t units = (ins ? insert_regions(d.lb) : 0) + (del ? c->ntiles + d.ltiles : 0);
    if (sg) {  // supergraph, then its rounds
        c->round_base = SG_ROUND0;
        if (sg_reduce(c, d, s)) launch_fill_i32(c->status, 1, ST_ROUND_BOUND, s);
        launch_boruvka(d, SG_ROUND0, SG_ROUND0 + c->bor_fast, units, false, s);
    } else {
        c->round_base = 0;
        launch_boruvka(d, 0, c->bor_fast, units, ins, s);
    }
    mark(PH_ROOTING);
    launch_sf_root(d, s);
    launch_sf_bfs(d, 0, c->bfs_fast, s);
    launch_orient_bfs(d, c->bfs_fast, s);
    if (c->lr_kinds & (1u << kind)) launch_superforest_lr(d, tour_rounds(c), c->bfs_fast, s);
    mark(PH_FINISH);
    const bool et = c->opts.reverse_mode == 1;
    if (et && launch_et_reverse(d, c->et_tmp, c->et_tmp_bytes, s))
        launch_fill_i32(c->status, 1, ST_ROUND_BOUND, s);  // the library sort failed
    launch_finish(d, ins, del, !et, s);
    mark(PH_N);
    if (small) {
        (void)hipStreamWaitEvent(s, c->ev_join, 0);
        launch_small_commit(d, make_small(c), grid_for(c->nsg, 1, GRID_CAP), false, s);
    }
    launch_cleanup(d, s);  // also hands the results to the host
}

int capture_graph(drsf_ctx *c, int kind) {
    const int q = c->slot;
    if (c->gexec[q][kind]) return DRSF_OK;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    enqueue_update(c, kind, false, nullptr);
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamEndCapture(c->stream, &g));
    c->graph[q][kind] = g;
    HIPCHK(c, hipGraphInstantiate(&c->gexec[q][kind], g, nullptr, nullptr, 0));
    return DRSF_OK;
}

// Finishes an update that the queued sequence left unfinished: more
// hooking rounds in short chunks, deeper search or the Euler tour, then
// reversal, labels and cleanup; or, when its sequence ran to the end and
// left only paths too long for one thread's walk, the doubling pass over
// those and cleanup.
int continue_update(drsf_ctx *c) {
    Dev d = make_dev(c);
    d.gate = 0;  // runs while the update's cleanup holds any update queued behind it
    d.lb = std::max<int64_t>(c->last_b, 1);
    d.ltiles = delta_tiles(c->ndelta_bound);
    hipStream_t s = c->stream;
    unsigned long long *f = c->h_ret + c->ret_words;  // [0] status, [1] rounds done, [2] level active
    auto read_flags = [&](int levels) -> int {
        HIPCHK(c, hipMemcpyAsync(f, c->status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(f + 1, c->cnt + C_DONE_BOR, sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(f + 2, c->cnt + C_BFS_ROUND + levels - 1, sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        return DRSF_OK;
    };
    const int64_t np_max = c->pcap;
    // each round at least halves the components that still have a live edge
    const int bor_bound = std::min(c->round_base + ceil_log2(np_max + 2) + 2, MAX_ROUNDS);
    const int lr_rounds = tour_rounds(c);
    // the counters the update handed over: orientation done means only
    // long paths are left (the walks ran, and the labels)
    const unsigned long long *k = c->h_ret + 1;
    const bool oriented = k[C_ORIENTED] != 0;
    int64_t nlong = oriented ? (int64_t)k[C_NLONG] : 0;
    int rc;
    bool bad = false;
    int how = 0;  // the bits of drsf_view.host_finished
    // profiled contexts time the continuation, host round trips included
    c->cont_timed = c->have_phases;
    if (!oriented) {
        if ((rc = read_flags(c->bfs_fast))) return rc;
    }
    if (c->cont_timed) (void)hipEventRecord(c->ev[PH_N + 3], s);
    bad = !oriented && *(int32_t *)f != 0;
    bool done = oriented || f[1] != 0, bfs_done = oriented || f[2] == 0;
    int r = c->round_base + c->bor_fast, lv = c->bfs_fast;
    if (!oriented && !bad && !done) {
        how |= 1;
        while (!done && !bad && r < bor_bound) {
            const int r1 = std::min(r + BOR_CHUNK, bor_bound);
            launch_boruvka(d, r, r1, 4096, false, s);
            r = r1;
            if ((rc = read_flags(lv))) return rc;
            bad = *(int32_t *)f != 0;
            done = f[1] != 0;
        }
        if (!bad && !done) {
            launch_fill_i32(c->status, 1, ST_ROUND_BOUND, s);
            bad = true;
        }
        if (!bad) {
            launch_sf_root(d, s);
            launch_sf_bfs(d, 0, c->bfs_fast, s);
            if ((rc = read_flags(lv))) return rc;
            bad = *(int32_t *)f != 0;
            bfs_done = f[2] == 0;
        }
    }
    if (!oriented && !bad) {
        if (!bfs_done) how |= 2;
        while (!bfs_done && lv < BFS_MAX) {
            launch_sf_bfs(d, lv, lv + 4, s);
            lv += 4;
            if ((rc = read_flags(lv))) return rc;
            bfs_done = f[2] == 0;
        }
        if (bfs_done) launch_orient_bfs(d, lv, s);
        else launch_superforest_lr(d, lr_rounds, lv, s);  // deep super-trees: Euler tour
        const bool et = c->opts.reverse_mode == 1;
        if (et && launch_et_reverse(d, c->et_tmp, c->et_tmp_bytes, s))
            launch_fill_i32(c->status, 1, ST_ROUND_BOUND, s);
        launch_finish(d, c->kind & 1, c->kind & 2, !et, s);
        // the walks may have left long paths
        HIPCHK(c, hipMemcpyAsync(f + 6, c->cnt + C_NLONG, sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        nlong = (int64_t)f[6];
    }
    if (!bad && nlong > 0) {
        how |= 4;
        if ((rc = reverse_long_paths(c, d, nlong, s))) return rc;
    }
    launch_cleanup(d, s);  // hands the results to the host, then resets
    if (c->cont_timed) (void)hipEventRecord(c->ev[PH_N + 4], s);
    HIPCHK(c, hipStreamSynchronize(s));
    c->view.host_finished = how ? how : 1;
    // counts left to the library (tuning 0): later updates queue the rounds
    // and levels this one needed, so that updates like it finish on the
    // device (each queued round or level that finds nothing costs one
    // dispatch); bounded so that one outlier cannot make every update slow
    if (!bad) {
        bool grew = false;
        if ((how & 1) && c->opts.rounds_queued <= 0 && r - c->round_base > c->bor_fast) {
            c->bor_fast = std::min(r - c->round_base, AUTO_ROUNDS_MAX);
            grew = true;
        }
        if ((how & 2) && bfs_done && c->opts.levels_queued <= 0 && lv > c->bfs_fast) {
            c->bfs_fast = std::min(lv, BFS_MAX);
            grew = true;
        }
        // deeper than the levels may grow: queue the tour itself
        if ((how & 2) && !bfs_done && c->opts.levels_queued <= 0 && !(c->lr_kinds & (1u << c->kind))) {
            c->lr_kinds |= 1u << c->kind;
            grew = true;
        }
        if (grew) drop_graphs(c);
    }
    return DRSF_OK;
}

// Updates replay captured graphs (launch_mode 1, or 0 with several graphs)
// rather than launching kernel by kernel.
bool graph_launch(const drsf_ctx *c) {
    return c->opts.launch_mode == 1 || (c->opts.launch_mode == 0 && c->ngraph > 1);
}

// Queues one update whose batch is in the device batch buffers and whose
// control block is in h_ctl.
int launch_update(drsf_ctx *c) {
    hipStream_t s = c->stream;
    // the first kernel takes the control block in h_ctl: as its argument
    // when launched kernel by kernel, from pinned memory in a captured graph
    const bool prof = c->opts.profile != 0;
    c->h_ctl->seq = ++c->seq;  // the caller filled the slot in use
    // clear the completion word: pinned memory may hold any value (a freed
    // context's, or scratch), and the wait must only see this update's
    *(volatile unsigned long long *)(c->h_ret + c->ret_words + 7) = 0;
    c->kind = (c->h_ctl->has_ins ? 1 : 0) | (c->h_ctl->has_del ? 2 : 0);
    if (c->kind == 0) c->kind = 3;  // nothing but rejected or empty batches: run everything
    // the supergraph reads sizes back between its kernels, so it is not
    // captured (the Euler-tour reversal, sort included, is a fixed sequence).
    // An update queued behind a running one is launched kernel by kernel:
    // the device then goes from one update to the next as from one kernel
    // to the next, where a graph launch starts some microseconds after the
    // work before it
    if (prof || c->opts.replacement_mode == 1 || c->npend > 0 || !graph_launch(c)) {
        enqueue_update(c, c->kind, prof, c->h_ctl);
    } else {
        int rc;
        if ((rc = capture_graph(c, c->kind))) return rc;
        HIPCHK(c, hipGraphLaunch(c->gexec[c->slot][c->kind], s));
    }
    HIPCHK(c, hipGetLastError());
    c->pend[c->slot] = drsf_ctx::Pend{c->seq, c->kind, c->last_op, c->last_b};
    c->last_slot = c->slot;
    c->npend++;
    c->have_phases = prof;
    return DRSF_OK;
}

// Queues again an update whose first launch stood still behind an
// unfinished one (its control block is unchanged in its slot).
int relaunch_update(drsf_ctx *c, int q) {
    select_slot(c, q);
    c->kind = c->pend[q].kind;
    if (!graph_launch(c)) {
        enqueue_update(c, c->kind, false, c->h_ctl);
    } else {
        int rc;
        if ((rc = capture_graph(c, c->kind))) return rc;
        HIPCHK(c, hipGraphLaunch(c->gexec[q][c->kind], c->stream));
    }
    HIPCHK(c, hipGetLastError());
    return DRSF_OK;
}

// An update may be queued behind a running one (two in flight) in a
// one-graph context that reads its batches in place, without profiling, on
// the default replacement and reversal paths; otherwise the queue is drained
// first.
bool can_queue(const drsf_ctx *c) {
    return c->ngraph == 1 && c->opts.inputs_on_device && !c->opts.profile && c->opts.replacement_mode == 0 &&
           c->opts.reverse_mode == 0 && c->nsg == 0;
}

// Regions of x0 the first hooking rounds read (see Dev::x0).
void set_regions(drsf_ctx *c, Ctl &k) {
    k.ibase = c->ntiles + c->dtmax;
    const int64_t dreg = c->ntiles + delta_tiles(c->ndelta_bound);
    if (k.has_ins && k.has_del) {
        k.rlo = 0;
        k.rhi = k.ibase + insert_regions(k.b);
    } else if (k.has_del) {
        k.rlo = 0;
        k.rhi = dreg;
    } else {
        k.rlo = k.ibase;
        k.rhi = k.ibase + insert_regions(k.b);
    }
}

int stage_edges(drsf_ctx *c, const int32_t *edges, int64_t b) {
    if (b == 0) return DRSF_OK;
    hipStream_t s = c->stream;
    if (c->opts.inputs_on_device) {
        HIPCHK(c, hipMemcpyAsync(c->bedges, edges, sizeof(int32_t) * 2 * (size_t)b,
                                 hipMemcpyDeviceToDevice, s));
    } else {
        // the previous update has completed, so the pinned staging is free
        memcpy(c->h_edges, edges, sizeof(int32_t) * 2 * (size_t)b);
        HIPCHK(c, hipMemcpyAsync(c->bedges, c->h_edges, sizeof(int32_t) * 2 * (size_t)b,
                                 hipMemcpyHostToDevice, s));
    }
    return DRSF_OK;
}

int wait_oldest(drsf_ctx *c);

// Keeps the result in last_rc and view for a later drsf_wait.
void keep_done(drsf_ctx *c, int rc) {
    if (c->ndone == 2) {
        c->done[0] = c->done[1];
        c->ndone = 1;
    }
    c->done[c->ndone++] = drsf_ctx::Done{rc, c->view};
}

// Waits for every queued update, keeping their results for drsf_wait;
// returns an error other than a rejected batch.
int finish_pending(drsf_ctx *c) {
    while (c->npend > 0) {
        const int rc = wait_oldest(c);
        keep_done(c, rc);
        if (rc != DRSF_OK && rc != DRSF_E_BATCH) return rc;
    }
    return DRSF_OK;
}

}  // namespace

extern "C" {

const char *drsf_version(void) { return "drsf 0.2 (gfx950)"; }

void drsf_default_opts(drsf_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->validate_forest = 1;
    o->validate_batches = 1;
    o->launch_mode = 0;
    o->max_batch = 1 << 20;
}

const char *drsf_last_error(const drsf_ctx *c) {
    return c ? c->err.c_str() : g_create_error.c_str();
}

static int create_impl(int32_t G, const int32_t *n_off, int32_t n, const int64_t *row_ptr,
                       const int32_t *col, const int32_t *parent, const drsf_opts *opts,
                       drsf_ctx **out) {
    *out = nullptr;
    if (n < 1 || !row_ptr || !parent) return fail(nullptr, DRSF_E_ARG, "n must be >= 1; row_ptr and parent non-NULL");
    drsf_ctx *c = new drsf_ctx();
    if (opts) c->opts = *opts; else drsf_default_opts(&c->opts);
    if (c->opts.max_batch <= 0) c->opts.max_batch = 1 << 20;
    c->max_batch = c->opts.max_batch;
    if (c->opts.rounds_queued > 0) c->bor_fast = std::min(c->opts.rounds_queued, MAX_ROUNDS - 1);
    if (c->opts.levels_queued > 0) c->bfs_fast = std::min(c->opts.levels_queued, BFS_MAX);
    c->n = n;
    c->ngraph = G;
    c->goff_h.assign((size_t)G + 1, 0);
    if (n_off) for (int32_t g = 0; g <= G; g++) c->goff_h[g] = n_off[g];
    else c->goff_h[1] = n;
    int rc = DRSF_OK;
    auto bail = [&](int code) {
        g_create_error = c->err;
        destroy_ctx(c);
        return code;
    };
    for (int32_t g = 0; g < G; g++)
        if (c->goff_h[g + 1] < c->goff_h[g]) {
            fail(c, DRSF_E_ARG, "graph vertex offsets must be non-decreasing");
            return bail(DRSF_E_ARG);
        }
    if (c->opts.reverse_mode < 0 || c->opts.reverse_mode > 1) {
        fail(c, DRSF_E_ARG, "reverse_mode must be 0 or 1");
        return bail(DRSF_E_ARG);
    }
    if (c->opts.replacement_mode < 0 || c->opts.replacement_mode > 1) {
        fail(c, DRSF_E_ARG, "replacement_mode must be 0 or 1");
        return bail(DRSF_E_ARG);
    }
    if (c->opts.launch_mode < 0 || c->opts.launch_mode > 2) {
        fail(c, DRSF_E_ARG, "launch_mode must be 0, 1 or 2");
        return bail(DRSF_E_ARG);
    }
    if (c->opts.walk_limit < 0) {
        fail(c, DRSF_E_ARG, "walk_limit must be >= 0");
        return bail(DRSF_E_ARG);
    }
    if (c->opts.dev_alloc && !c->opts.dev_free) {
        fail(c, DRSF_E_ARG, "dev_alloc needs dev_free");
        return bail(DRSF_E_ARG);
    }
    if (c->opts.small_graph_vertices < 0 || c->opts.small_graph_vertices > 16384 ||
        (c->opts.small_threads != 0 && c->opts.small_threads != 256 && c->opts.small_threads != 512 &&
         c->opts.small_threads != 1024)) {
        fail(c, DRSF_E_ARG, "small_graph_vertices must be in [0, 16384] and small_threads 0, 256, 512 or 1024");
        return bail(DRSF_E_ARG);
    }
    c->small_T = G > 1 ? c->opts.small_graph_vertices : 0;
    if (c->opts.small_threads) c->small_threads = c->opts.small_threads;
    {
        const hipError_t e = hipGetDevice(&c->dev);
        if (e != hipSuccess) {
            fail(c, DRSF_E_DEVICE, "no HIP device: %s", hipGetErrorString(e));
            return bail(DRSF_E_DEVICE);
        }
    }
    if (c->opts.stream) {
        c->stream = (hipStream_t)c->opts.stream;
    } else {
        // a blocking stream: its work is ordered after work queued earlier
        // on the null stream, where a caller without a stream of its own
        // (torch's default stream is the null stream) produces device inputs
        if (hipStreamCreateWithFlags(&c->stream, hipStreamDefault) != hipSuccess) {
            fail(c, DRSF_E_DEVICE, "stream creation failed");
            return bail(DRSF_E_DEVICE);
        }
        c->own_stream = true;
    }
    c->ret_words = 1 + C_TOTAL + (G + 1) / 2;
    if ((rc = halloc(c, &c->h_ret_ring, 2 * (c->ret_words + 8)))) return bail(rc);
    select_slot(c, 0);
    if (c->opts.profile)  // phase events exist only for the profiled launch path
        for (auto &e : c->ev)
            if (hipEventCreate(&e) != hipSuccess) {
                fail(c, DRSF_E_DEVICE, "event creation failed");
                return bail(DRSF_E_DEVICE);
            }
    if ((rc = dalloc(c, &c->ctlmem, c->ret_words))) return bail(rc);
    c->status = reinterpret_cast<int32_t *>(c->ctlmem);
    c->cnt = c->ctlmem + 1;
    c->gstat = reinterpret_cast<int32_t *>(c->ctlmem + 1 + C_TOTAL);
    launch_fill_u64(c->ctlmem, c->ret_words, 0, c->stream);
    if ((rc = dalloc(c, &c->goff, (int64_t)G + 1))) return bail(rc);
    // every copy of create runs on the context's stream, after the work the
    // caller queued there (or, for a context-owned stream, on the null stream)
    if (hipMemcpyAsync(c->goff, c->goff_h.data(), sizeof(int32_t) * ((size_t)G + 1), hipMemcpyHostToDevice,
                       c->stream) != hipSuccess) {
        fail(c, DRSF_E_DEVICE, "cannot copy graph offsets");
        return bail(DRSF_E_DEVICE);
    }
    launch_fill_u64(c->cnt, C_TOTAL, 0, c->stream);
    // row offsets are checked on the host before any kernel reads through them
    std::vector<int64_t> hrow;
    const int64_t *rp = row_ptr;
    if (c->opts.inputs_on_device) {
        hrow.resize((size_t)n + 1);
        if (d2h(c, hrow.data(), row_ptr, sizeof(int64_t) * hrow.size()) != DRSF_OK) {
            (void)hipGetLastError();
            fail(c, DRSF_E_ARG, "cannot read row_ptr");
            return bail(DRSF_E_ARG);
        }
        rp = hrow.data();
    } else if (hipStreamSynchronize(c->stream) != hipSuccess) {  // goff's pageable source
        fail(c, DRSF_E_DEVICE, "cannot copy graph offsets");
        return bail(DRSF_E_DEVICE);
    }
    if (rp[0] != 0) {
        fail(c, DRSF_E_ARG, "row_ptr[0] must be 0");
        return bail(DRSF_E_ARG);
    }
    for (int32_t u = 0; u < n; u++)
        if (rp[u + 1] < rp[u]) {
            fail(c, DRSF_E_ARG, "row_ptr must be non-decreasing");
            return bail(DRSF_E_ARG);
        }
    const int64_t nnz = rp[n];
    if (nnz > 0 && !col) {
        fail(c, DRSF_E_ARG, "col is NULL");
        return bail(DRSF_E_ARG);
    }
    if ((rc = build_store(c, row_ptr, col, nnz, c->opts.inputs_on_device != 0))) return bail(rc);
    if ((rc = dalloc(c, &c->parent, n))) return bail(rc);
    if (hipMemcpyAsync(c->parent, parent, sizeof(int32_t) * (size_t)n,
                       c->opts.inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                       c->stream) != hipSuccess) {
        fail(c, DRSF_E_ARG, "cannot copy parent[]");
        return bail(DRSF_E_ARG);
    }
    if ((rc = alloc_state(c))) return bail(rc);
    if ((rc = canonicalise_forest(c))) return bail(rc);
    if (c->small_T > 0) {
        int lds_blk = 64 * 1024;
        (void)hipDeviceGetAttribute(&lds_blk, hipDeviceAttributeMaxSharedMemoryPerBlock, c->dev);
        if ((int64_t)(small_lds_bytes(c->small_T) + small_static_lds()) > lds_blk) {
            fail(c, DRSF_E_ARG, "small_graph_vertices %d needs more LDS than a workgroup may hold (%d bytes)",
                 c->small_T, lds_blk);
            return bail(DRSF_E_ARG);
        }
        if (small_prepare(c->small_T)) {
            (void)hipGetLastError();
            fail(c, DRSF_E_DEVICE, "cannot give the small-graph kernel %zu bytes of LDS", small_lds_bytes(c->small_T));
            return bail(DRSF_E_DEVICE);
        }
        if ((rc = setup_small(c))) return bail(rc);
        c->small_grid = small_grid_for(c);
    }
    c->view.parent = c->parent;
    c->view.label = c->label;
    c->view.n = n;
    c->view.num_edges = c->m_live;
    *out = c;
    return DRSF_OK;
}

int drsf_create(int32_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *parent,
                const drsf_opts *opts, drsf_ctx **out) {
    if (!out) return fail(nullptr, DRSF_E_ARG, "out is NULL");
    return create_impl(1, nullptr, n, row_ptr, col, parent, opts, out);
}

int drsf_multi_create(int32_t G, const int32_t *n_off, const int64_t *row_ptr, const int32_t *col,
                      const int32_t *parent, const drsf_opts *opts, drsf_ctx **out) {
    if (!out) return fail(nullptr, DRSF_E_ARG, "out is NULL");
    *out = nullptr;
    if (G < 1 || !n_off) return fail(nullptr, DRSF_E_ARG, "G must be >= 1 and n_off non-NULL");
    if (n_off[0] != 0) return fail(nullptr, DRSF_E_ARG, "n_off[0] must be 0");
    return create_impl(G, n_off, n_off[G], row_ptr, col, parent, opts, out);
}

int drsf_num_graphs(const drsf_ctx *c) { return c ? c->ngraph : 0; }

int64_t drsf_device_bytes(const drsf_ctx *c) { return c ? c->bytes : -1; }

int drsf_digest(drsf_ctx *c, uint64_t *out) {
    if (!c || !out) return DRSF_E_ARG;
    const int rc = finish_pending(c);
    if (rc) return rc;
    unsigned long long *dd = c->cnt + C_COUNT;  // two spare counter words
    launch_digest(c->n, c->parent, c->label, dd, c->stream);
    HIPCHK(c, hipMemcpyAsync(c->h_ret, dd, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    out[0] = c->h_ret[0];
    out[1] = c->h_ret[1];
    launch_fill_u64(dd, 2, 0, c->stream);
    return DRSF_OK;
}

int64_t drsf_footprint(int32_t n, int64_t nnz, const drsf_opts *opts) {
    // the allocations of create (peak, with the host-input staging) and of
    // the per-context state, as sized in build_store and alloc_state
    drsf_opts o;
    if (opts) o = *opts; else drsf_default_opts(&o);
    const int64_t mb = o.max_batch > 0 ? o.max_batch : (1 << 20);
    const int64_t eb = nnz / 2, N = n;
    const int64_t ntiles = (eb + TILE - 1) / TILE;
    const int64_t nvb = (N + BLOCK - 1) / BLOCK;
    const int64_t pcap = 2 * mb + 16;
    const int64_t dcap = o.delta_capacity > 0 ? o.delta_capacity : std::max<int64_t>({4 * mb, eb / 8, 1 << 20});
    auto pow2 = [](int64_t x) { int64_t p = 16; while (p < x) p <<= 1; return p; };
    const int64_t bh = pow2(2 * mb), dh = pow2(2 * dcap);
    const int64_t xcap = (ntiles + (dcap + TILE - 1) / TILE + (mb + BLOCK - 1) / BLOCK) * TILE;
    int64_t b = 0;
    b += o.inputs_on_device ? 0 : 8 * (N + 1) + 4 * nnz;                 // staged input
    b += 4 * (N + 1) * 3 + 4 * ntiles * TILE + 8 * eb + 4 * (ntiles + 1);  // bptr, lptr, zptr; bcol; lcol, twin
    b += 4 * N * 2;                                                       // zrow, parent
    b += 16 * N + (N + 63) / 64 * 8;                                      // label, rep, tidx, owner; bitmap
    b += 49 * pcap + 40 * pcap + 16 * pcap + 16 * std::max(2 * pcap, N);  // pieces, tour, er, paths
    b += 37 * mb + 8 * bh + 8 * dcap + 12 * dh;                           // batch, tables, inserted list
    b += 32 * xcap + 8 * (xcap / TILE);                                   // cross lists
    b += 24 * nvb + 40 * N + 40 * nvb * BLOCK + 8 * (ntiles + 1) + 4 * (2 * ntiles + 1) +
         24 * ((nvb + BLOCK - 1) / BLOCK);                                // orphan scan
    return b + (1 << 20);
}

int drsf_set_tuning(drsf_ctx *c, int rounds_queued, int levels_queued, int sweep_mode) {
    if (!c) return DRSF_E_ARG;
    if (sweep_mode < 0 || sweep_mode > 1) return fail(c, DRSF_E_ARG, "sweep_mode must be 0 or 1");
    const int rc = finish_pending(c);
    if (rc) return rc;
    c->bor_fast = rounds_queued > 0 ? std::min(rounds_queued, MAX_ROUNDS - 1) : BOR_FAST;
    c->bfs_fast = levels_queued > 0 ? std::min(levels_queued, BFS_MAX) : BFS_FAST;
    c->opts.rounds_queued = rounds_queued;
    c->opts.levels_queued = levels_queued;
    c->opts.sweep_mode = sweep_mode;
    // the captured sequences hold the old round counts
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    return DRSF_OK;
}

static int check_usable(drsf_ctx *c) {
    return c->broken ? fail(c, DRSF_E_STATE, "a failed store rebuild (or host continuation) left the "
                                              "context unusable; only its forest can be read")
                     : DRSF_OK;
}

int drsf_set_small_schedule(drsf_ctx *c, int threads, int workgroups) {
    if (!c) return DRSF_E_ARG;
    if ((threads != 0 && threads != 256 && threads != 512 && threads != 1024) || workgroups < 0)
        return fail(c, DRSF_E_ARG, "threads must be 0, 256, 512 or 1024 and workgroups >= 0");
    const int rc = finish_pending(c);
    if (rc) return rc;
    if (threads) c->small_threads = threads;
    if (c->nsg) c->small_grid = workgroups ? std::min(workgroups, c->nsg) : small_grid_for(c);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    return DRSF_OK;
}

int drsf_apply_async(drsf_ctx *c, const int32_t *edges, int64_t b, int op) {
    if (!c) return DRSF_E_ARG;
    int rc;
    // queued behind at most one running update; an empty batch or one that
    // fills the inserted-edge list (a store rebuild) drains the queue
    const bool queue = can_queue(c) && b > 0 &&
                       !(op == DRSF_INSERT && c->ndelta_bound + b > c->dcap);
    if (!queue) {
        if ((rc = finish_pending(c))) return rc;
    } else if (c->npend >= 2) {
        rc = wait_oldest(c);
        keep_done(c, rc);
        if (rc != DRSF_OK && rc != DRSF_E_BATCH) return rc;
    }
    if ((rc = check_usable(c))) return rc;
    if (c->ngraph != 1) return fail(c, DRSF_E_STATE, "the context holds several graphs: use drsf_multi_apply");
    if (op != DRSF_INSERT && op != DRSF_DELETE) return fail(c, DRSF_E_ARG, "op must be insert or delete");
    if (b < 0 || (b > 0 && !edges)) return fail(c, DRSF_E_ARG, "bad batch");
    if (b > c->max_batch)
        return fail(c, DRSF_E_CAPACITY, "batch of %lld exceeds max_batch %lld", (long long)b,
                    (long long)c->max_batch);
    c->have_phases = false;
    c->multi_last = false;
    if (b == 0) {
        c->last_rc = DRSF_OK;
        c->view.num_key_cross = c->view.num_replacement = c->view.num_pieces = c->view.num_paths = 0;
        c->view.num_orphans = c->view.orphan_slots = 0;
        c->view.scan_orphans = 0;
        c->view.jump_rounds = 0;
        c->view.host_finished = 0;
        keep_done(c, DRSF_OK);
        return DRSF_OK;
    }
    if (op == DRSF_INSERT && c->ndelta_bound + b > c->dcap) {
        if (b > c->dcap)
            return fail(c, DRSF_E_CAPACITY, "batch of %lld inserts exceeds delta_capacity %lld",
                        (long long)b, (long long)c->dcap);
        if ((rc = rebuild_store(c))) return rc;
    }
    // a device batch is read in place by the first kernel (the stream orders
    // it before later work the caller queues there); a host batch is staged
    if (!c->opts.inputs_on_device && (rc = stage_edges(c, edges, b))) return rc;
    c->last_b = b;
    c->last_op = op;
    // queued updates alternate between the two slots; one waited for alone
    // keeps to slot 0 (and to the graphs captured there)
    select_slot(c, queue ? 1 - c->last_slot : 0);
    Ctl &k = *c->h_ctl;
    memset(&k, 0, sizeof k);
    if (c->opts.inputs_on_device) k.edges = edges;
    k.b = b;
    k.op = op;
    k.has_ins = op == DRSF_INSERT;
    k.has_del = op == DRSF_DELETE;
    k.ngraph = 1;
    k.lfast = c->bfs_fast;
    k.smode = c->opts.sweep_mode;
    k.nvl = k.nil = k.ntl = -1;
    if (op == DRSF_INSERT) c->ndelta_bound += b;
    set_regions(c, k);
    return launch_update(c);
}

int drsf_multi_apply_async(drsf_ctx *c, const int32_t *edges, const int64_t *b_off, const int8_t *op) {
    if (!c) return DRSF_E_ARG;
    int rc;
    if ((rc = finish_pending(c))) return rc;
    // per-graph statuses live in the returned words, which this update
    // overwrites: results not yet returned are dropped
    c->ndone = 0;
    if ((rc = check_usable(c))) return rc;
    if (!b_off || !op) return fail(c, DRSF_E_ARG, "b_off and op must be non-NULL");
    const int32_t G = c->ngraph;
    const int64_t b = b_off[G];
    if (b_off[0] != 0 || b < 0 || (b > 0 && !edges)) return fail(c, DRSF_E_ARG, "bad batch offsets");
    for (int32_t g = 0; g < G; g++)
        if (b_off[g + 1] < b_off[g] || (op[g] != DRSF_INSERT && op[g] != DRSF_DELETE))
            return fail(c, DRSF_E_ARG, "bad batch offsets or op for graph %d", g);
    if (b > c->max_batch)
        return fail(c, DRSF_E_CAPACITY, "batch of %lld exceeds max_batch %lld", (long long)b,
                    (long long)c->max_batch);
    // inserts into the edge store's list (small graphs keep their own arrays,
    // which grow when an insert would not fit)
    int64_t nins = 0;
    std::vector<int64_t> need;
    for (int32_t g = 0; g < G; g++) {
        if (op[g] != DRSF_INSERT) continue;
        const int64_t bg = b_off[g + 1] - b_off[g];
        const int32_t k = c->nsg ? c->g2s[g] : -1;
        if (k < 0) {
            nins += bg;
        } else if (c->gm_h[g] + bg > c->scap_h[k]) {
            if (need.empty()) need.assign((size_t)c->nsg, 0);
            need[k] = c->gm_h[g] + bg;
        }
    }
    if (!need.empty() && (rc = small_grow(c, need))) return rc;
    if (c->ndelta_bound + nins > c->dcap) {
        if (nins > c->dcap)
            return fail(c, DRSF_E_CAPACITY, "batch of %lld inserts exceeds delta_capacity %lld",
                        (long long)nins, (long long)c->dcap);
        if ((rc = rebuild_store(c))) return rc;
    }
    c->have_phases = false;
    c->multi_last = true;
    select_slot(c, 0);
    c->last_b = b;
    c->last_bg.assign((size_t)G, 0);
    c->last_opg.assign(op, op + G);
    for (int32_t g = 0; g < G; g++) c->last_bg[g] = b_off[g + 1] - b_off[g];
    if (b == 0) {
        c->last_rc = DRSF_OK;
        for (int32_t g = 0; g < G; g++) c->h_gstat[g] = 0;
        c->view.num_key_cross = c->view.num_replacement = c->view.num_pieces = c->view.num_paths = 0;
        c->view.num_orphans = c->view.orphan_slots = 0;
        c->view.scan_orphans = 0;
        c->view.jump_rounds = 0;
        c->view.host_finished = 0;
        keep_done(c, DRSF_OK);
        return DRSF_OK;
    }
    // per-edge op and graph; vertex-block lists of the deleting and the
    // inserting graphs and the base-store tiles of the deleting ones
    bool any_ins = false, any_del = false;
    int32_t nsmall = 0;
    // every graph small: the engine alone runs, which reads the tasks only
    // (no per-edge op and graph, no block lists)
    const bool alone = c->nsg > 0 && c->nsg == G;
    for (int32_t g = 0; g < G; g++) {
        const int32_t k = c->nsg ? c->g2s[g] : -1;
        // op 2: the edge belongs to a small graph, whose own kernel takes it
        const int8_t eo = k < 0 ? op[g] : (int8_t)2;
        if (!alone)
            for (int64_t i = b_off[g]; i < b_off[g + 1]; i++) {
                c->h_bop[i] = eo;
                c->h_bgid[i] = g;
            }
        if (b_off[g + 1] == b_off[g]) continue;
        if (k < 0) (op[g] == DRSF_DELETE ? any_del : any_ins) = true;
        else c->h_stasks[nsmall++] = make_int4(k, (int)b_off[g], (int)(b_off[g + 1] - b_off[g]), op[g]);
    }
    hipStream_t s = c->stream;
    // lists of -1: every vertex block and tile (one graph: the lists, only
    // allocated for several, would hold them all)
    int64_t nvl = -1, nil = -1, ntl = -1;
    if (c->h_lists && !alone) {
        int32_t *vl = c->h_lists, *il = c->h_lists + c->nvblk, *tl = c->h_lists + 2 * c->nvblk;
        int64_t lastv = -1, lasti = -1, lastt = -1;
        nvl = nil = ntl = 0;
        for (int32_t g = 0; g < G; g++) {
            if (b_off[g + 1] == b_off[g] || c->goff_h[g + 1] == c->goff_h[g]) continue;
            if (c->nsg && c->g2s[g] >= 0) continue;  // a small graph: not in the lists
            const int64_t v0 = c->goff_h[g] / BLOCK, v1 = (c->goff_h[g + 1] - 1) / BLOCK;
            if (op[g] == DRSF_DELETE) {
                for (int64_t j = std::max(v0, lastv + 1); j <= v1; j++) vl[nvl++] = (int32_t)j;
                lastv = std::max(lastv, v1);
                if (c->gedge_h[g + 1] > c->gedge_h[g]) {
                    const int64_t t0 = c->gedge_h[g] / TILE, t1 = (c->gedge_h[g + 1] - 1) / TILE;
                    for (int64_t t = std::max(t0, lastt + 1); t <= t1; t++) tl[ntl++] = (int32_t)t;
                    lastt = std::max(lastt, t1);
                }
            } else {
                for (int64_t j = std::max(v0, lasti + 1); j <= v1; j++) il[nil++] = (int32_t)j;
                lasti = std::max(lasti, v1);
            }
        }
        HIPCHK(c, hipMemcpyAsync(c->lists, c->h_lists,
                                 sizeof(int32_t) * (size_t)(2 * c->nvblk + c->ntiles + 1),
                                 hipMemcpyHostToDevice, s));
    }
    if (nsmall)
        HIPCHK(c, hipMemcpyAsync(c->stasks, c->h_stasks, sizeof(int4) * (size_t)nsmall, hipMemcpyHostToDevice, s));
    if (!alone) {
        HIPCHK(c, hipMemcpyAsync(c->bop, c->h_bop, (size_t)b, hipMemcpyHostToDevice, s));
        HIPCHK(c, hipMemcpyAsync(c->bgid, c->h_bgid, sizeof(int32_t) * (size_t)b, hipMemcpyHostToDevice, s));
    }
    if ((rc = stage_edges(c, edges, b))) return rc;
    Ctl &k = *c->h_ctl;
    memset(&k, 0, sizeof k);
    k.b = b;
    k.op = 2;
    k.has_ins = any_ins;
    k.has_del = any_del;
    k.ngraph = G;
    k.lfast = c->bfs_fast;
    k.smode = c->opts.sweep_mode;
    k.nvl = nvl;
    k.nil = nil;
    k.ntl = ntl;
    k.nsmall = nsmall;
    c->ndelta_bound += nins;
    set_regions(c, k);
    return launch_update(c);
}

}  // extern "C"

namespace {

// Waits for the oldest queued update and finishes it: its status in
// last_rc (returned), its figures in view.
int wait_oldest(drsf_ctx *c) {
    // the oldest queued update, in its slot
    const uint64_t myseq = c->seq - (uint64_t)c->npend + 1;
    const int q = c->pend[0].seq == myseq ? 0 : 1;
    select_slot(c, q);
    c->kind = c->pend[q].kind;
    c->last_b = c->pend[q].b;
    c->last_op = c->pend[q].op;
    c->npend--;
    // the last kernel writes the completion word once the results in
    // h_ret are final: poll it (a stream synchronisation wakes up later),
    // asking the stream now and then so that a failed or idle stream ends
    // the wait; profiling waits for the stream (its events)
    const volatile unsigned long long *done = c->h_ret + c->ret_words + 7;
    bool seen = false;
    if (!c->have_phases) {
        for (uint32_t it = 1;; it++) {
            if (*done == myseq) {
                seen = true;
                break;
            }
            if ((it & 1023) == 0 && hipStreamQuery(c->stream) != hipErrorNotReady) break;
        }
        std::atomic_thread_fence(std::memory_order_acquire);
    }
    if (!seen || *done != myseq) HIPCHK(c, hipStreamSynchronize(c->stream));
    const unsigned long long *k = c->h_ret + 1;
    int32_t st = *(int32_t *)c->h_ret;
    c->view.host_finished = 0;
    c->cont_timed = false;
    // the queued rounds and levels did not finish it, or its walks left long paths
    if (st == 0 && (!k[C_ORIENTED] || k[C_NLONG])) {
        c->view.host_finished = 1;
        int rc = continue_update(c);
        if (!rc && c->npend > 0) {
            // the update queued behind it stood still: queue it again
            rc = relaunch_update(c, 1 - q);
            select_slot(c, q);
            c->kind = c->pend[q].kind;
        }
        if (rc) {
            // a held update would stay held: the context is not usable
            c->npend = 0;
            c->broken = true;
            return c->last_rc = rc;
        }
        st = *(int32_t *)c->h_ret;
    }
    if (c->have_phases &&
        hipEventElapsedTime(&c->phase_ms[PH_N + 1], c->ev[PH_N + 1], c->ev[PH_N + 2]) != hipSuccess) {
        (void)hipGetLastError();
        c->have_phases = false;
    }
    c->phase_ms[PH_N] = 0.f;
    if (c->have_phases && c->cont_timed &&
        hipEventElapsedTime(&c->phase_ms[PH_N], c->ev[PH_N + 3], c->ev[PH_N + 4]) != hipSuccess) {
        (void)hipGetLastError();
        c->have_phases = false;
    }
    if (c->have_phases)
        for (int i = 0; i < PH_N; i++) {
            c->phase_ms[i] = 0.f;
            if (!c->ph_on[i]) continue;
            int j = i + 1;
            while (j < PH_N && !c->ph_on[j]) j++;
            if (hipEventElapsedTime(&c->phase_ms[i], c->ev[i], c->ev[j]) != hipSuccess) {
                (void)hipGetLastError();
                c->have_phases = false;
            }
        }
    // a deep forest: later deletes queue jumping rounds before the chase,
    // as many as a path of n vertices needs (rounds after the last one
    // that changed something exit at once); more if the last queued round
    // still changed entries
    if (st == 0) {
        int want = c->jump_rounds;
        if (k[C_DEEP] && want == 0) want = std::min(ceil_log2(c->n) + 1, MAX_JUMP);
        if (want > 0 && k[C_JUMP_ROUND + want - 1]) want = std::min(want + 4, MAX_JUMP);
        if (want != c->jump_rounds) {
            (void)hipStreamSynchronize(c->stream);  // a queued update may still run a graph
            c->jump_rounds = want;
            drop_graphs(c);
        }
    }
    if (st != 0) {
        c->last_rc = fail(c, DRSF_E_DEVICE, "internal bound exceeded (status %d)", st);
    } else {
        c->view.num_key_cross = (int64_t)(k[C_NCROSS] + k[C_SNCROSS]);
        c->view.num_replacement = (int64_t)(k[C_NER] + k[C_SNER]);
        c->view.num_pieces = (int64_t)k[C_NP];
        c->view.num_paths = (int64_t)(k[C_NR] + k[C_SNR]);
        c->view.scan_orphans = (int32_t)k[C_OMODE];
        c->view.num_orphans = (int64_t)k[C_NORPH];
        c->view.orphan_slots = (int64_t)k[C_OVOL] - (int64_t)OR_PAD * (int64_t)k[C_NORPH];
        c->view.jump_rounds = 0;
        for (int r = 0; r < MAX_JUMP; r++) c->view.jump_rounds += k[C_JUMP_ROUND + r] ? 1 : 0;
        c->last_rc = DRSF_OK;
        if (c->multi_last) {
            for (int32_t g = 0; g < c->ngraph; g++) {
                const int64_t bg = c->last_bg[g];
                if (c->h_gstat[g]) {
                    const bool in_store = c->g2s.empty() || c->g2s[g] < 0;
                    if (c->last_opg[g] == DRSF_INSERT && in_store) c->ndelta_bound -= bg;
                } else {
                    const int64_t dm = c->last_opg[g] == DRSF_INSERT ? bg : -bg;
                    c->gm_h[g] += dm;
                    c->m_live += dm;
                }
            }
        } else if (c->h_gstat[0]) {
            const int32_t bs = c->h_gstat[0];
            if (c->last_op == DRSF_INSERT) c->ndelta_bound -= c->last_b;
            c->last_rc = fail(c, DRSF_E_BATCH, "invalid batch:%s%s%s%s",
                              bs & ST_BAD_PAIR ? " self-loop or id out of range;" : "",
                              bs & ST_DUPLICATE ? " repeated edge;" : "",
                              bs & ST_EXISTS ? " insert of an existing edge;" : "",
                              bs & ST_MISSING ? " delete of a missing edge;" : "");
        } else {
            const int64_t dm = c->last_op == DRSF_INSERT ? c->last_b : -c->last_b;
            c->m_live += dm;
            c->gm_h[0] += dm;
        }
    }
    c->view.parent = c->parent;
    c->view.label = c->label;
    c->view.n = c->n;
    c->view.num_edges = c->m_live;
    return c->last_rc;
}

}  // namespace

extern "C" {

int drsf_wait(drsf_ctx *c, drsf_view *out) {
    if (!c) return DRSF_E_ARG;
    if (c->ndone > 0) {  // waited for on the caller's behalf by an earlier call
        const drsf_ctx::Done d = c->done[0];
        c->done[0] = c->done[1];
        c->ndone--;
        if (out) *out = d.view;
        return d.rc;
    }
    const int rc = c->npend > 0 ? wait_oldest(c) : c->last_rc;
    if (out) *out = c->view;
    return rc;
}

int drsf_multi_wait(drsf_ctx *c, int32_t *status) {
    if (!c) return DRSF_E_ARG;
    const int rc = drsf_wait(c, nullptr);
    if (rc != DRSF_OK) return rc;
    if (status)
        for (int32_t g = 0; g < c->ngraph; g++) status[g] = c->h_gstat[g] ? DRSF_E_BATCH : DRSF_OK;
    return DRSF_OK;
}

int drsf_multi_apply(drsf_ctx *c, const int32_t *edges, const int64_t *b_off, const int8_t *op,
                     int32_t *status) {
    if (!c) return DRSF_E_ARG;
    int rc = finish_pending(c);  // results of earlier queued updates are dropped
    if (rc) return rc;
    c->ndone = 0;
    if ((rc = drsf_multi_apply_async(c, edges, b_off, op)) != DRSF_OK) return rc;
    return drsf_multi_wait(c, status);
}

int drsf_multi_num_edges(drsf_ctx *c, int64_t *m) {
    if (!c || !m) return DRSF_E_ARG;
    const int rc = finish_pending(c);
    if (rc) return rc;
    for (int32_t g = 0; g < c->ngraph; g++) m[g] = c->gm_h[g];
    return DRSF_OK;
}

int drsf_apply(drsf_ctx *c, const int32_t *edges, int64_t b, int op, drsf_view *out) {
    if (!c) return DRSF_E_ARG;
    int rc = finish_pending(c);  // results of earlier queued updates are dropped
    if (rc) return rc;
    c->ndone = 0;
    if ((rc = drsf_apply_async(c, edges, b, op)) != DRSF_OK) return rc;
    return drsf_wait(c, out);
}

int drsf_get_view(drsf_ctx *c, drsf_view *out) {
    if (!c || !out) return DRSF_E_ARG;
    const int rc = finish_pending(c);
    if (rc) return rc;
    *out = c->view;
    return DRSF_OK;
}

int drsf_copy_out(drsf_ctx *c, int32_t *parent_host, int32_t *label_host) {
    if (!c) return DRSF_E_ARG;
    int rc = finish_pending(c);
    if (rc) return rc;
    if (parent_host && (rc = d2h(c, parent_host, c->parent, sizeof(int32_t) * (size_t)c->n))) return rc;
    if (label_host && (rc = d2h(c, label_host, c->label, sizeof(int32_t) * (size_t)c->n))) return rc;
    return DRSF_OK;
}

int64_t drsf_num_edges(drsf_ctx *c) {
    if (!c) return -1;
    if (finish_pending(c)) return -1;
    return c->m_live;
}

int drsf_export_edges(drsf_ctx *c, uint64_t *keys, int64_t capacity, int64_t *m_out) {
    if (!c || !keys || !m_out) return DRSF_E_ARG;
    int rc = finish_pending(c);
    if (rc) return rc;
    if ((rc = check_usable(c))) return rc;
    std::vector<uint32_t> bptr((size_t)c->n + 1);
    std::vector<int32_t> bcol((size_t)c->eb);
    unsigned long long nd = 0;
    HIPCHK(c, hipMemcpyAsync(c->h_ret, c->cnt + C_NDELTA, sizeof nd, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    nd = c->h_ret[0];
    if ((rc = d2h(c, bptr.data(), c->bptr, sizeof(uint32_t) * bptr.size()))) return rc;
    if (c->eb && (rc = d2h(c, bcol.data(), c->bcol, sizeof(int32_t) * bcol.size()))) return rc;
    std::vector<uint64_t> dk((size_t)nd);
    if (nd && (rc = d2h(c, dk.data(), c->dkey, sizeof(uint64_t) * nd))) return rc;
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
    if (c->nsg) {  // small graphs: their own key arrays, in local ids
        std::vector<int32_t> sm((size_t)c->nsg), sb((size_t)c->nsg);
        std::vector<uint32_t> pk((size_t)c->pool_keys);
        if ((rc = d2h(c, sm.data(), c->sm, 4 * sm.size())) || (rc = d2h(c, sb.data(), c->sbuf, 4 * sb.size())) ||
            (rc = d2h(c, pk.data(), c->pool, 4 * pk.size())))
            return rc;
        for (int32_t k = 0; k < c->nsg; k++) {
            const uint64_t o = (uint64_t)c->goff_h[c->sgid_h[k]];
            const uint32_t *E = pk.data() + c->soff_h[k] + (int64_t)sb[k] * c->scap_h[k];
            for (int32_t j = 0; j < sm[k]; j++) {
                if (w >= capacity) return fail(c, DRSF_E_CAPACITY, "export buffer too small");
                keys[w++] = ((o + (E[j] >> 16)) << 32) | (o + (E[j] & 0xffffu));
            }
        }
    }
    std::sort(keys, keys + w);
    *m_out = w;
    return DRSF_OK;
}

void drsf_snapshot_free(drsf_snapshot *s);

int drsf_snapshot_take(drsf_ctx *c, drsf_snapshot **out) {
    if (!c || !out) return DRSF_E_ARG;
    int rc = finish_pending(c);
    if (rc) return rc;
    if ((rc = check_usable(c))) return rc;
    drsf_snapshot *s = new drsf_snapshot();
    s->n = c->n; s->eb = c->eb; s->dcap = c->dcap; s->dhmask = c->dhmask;
    s->ndelta_bound = c->ndelta_bound; s->m_live = c->m_live; s->rebuilds = c->rebuilds;
    s->gm = c->gm_h;
    const size_t dh = (size_t)c->dhmask + 1;
    s->opts = c->opts;
    auto get = [&](auto **p, size_t bytes) {
        *p = static_cast<std::remove_reference_t<decltype(**p)> *>(raw_dalloc(s->opts, bytes));
        return *p != nullptr;
    };
    const bool ok = get(&s->parent, 4 * (size_t)c->n) && get(&s->label, 4 * (size_t)c->n) &&
                    get(&s->bcol, 4 * (size_t)std::max<int64_t>(c->eb, 1)) &&
                    get(&s->lcol, 4 * (size_t)std::max<int64_t>(c->eb, 1)) &&
                    get(&s->dkey, 8 * (size_t)c->dcap) && get(&s->dhash, 8 * dh) && get(&s->dhpos, 4 * dh) &&
                    (c->nsg == 0 || (get(&s->pool, 4 * (size_t)c->pool_keys) && get(&s->sm, 4 * (size_t)c->nsg) &&
                                     get(&s->sbuf, 4 * (size_t)c->nsg)));
    s->pool_keys = c->pool_keys;
    s->nsg = c->nsg;
    if (!ok) {
        drsf_snapshot_free(s);
        return fail(c, DRSF_E_NOMEM, "snapshot allocation failed");
    }
    hipStream_t st = c->stream;
    HIPCHK(c, hipMemcpyAsync(s->parent, c->parent, 4 * (size_t)c->n, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(s->label, c->label, 4 * (size_t)c->n, hipMemcpyDeviceToDevice, st));
    if (c->eb) HIPCHK(c, hipMemcpyAsync(s->bcol, c->bcol, 4 * (size_t)c->eb, hipMemcpyDeviceToDevice, st));
    if (c->eb) HIPCHK(c, hipMemcpyAsync(s->lcol, c->lcol, 4 * (size_t)c->eb, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(s->dkey, c->dkey, 8 * (size_t)c->dcap, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(s->dhash, c->dhash, 8 * dh, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(s->dhpos, c->dhpos, 4 * dh, hipMemcpyDeviceToDevice, st));
    if (c->nsg) {
        HIPCHK(c, hipMemcpyAsync(s->pool, c->pool, 4 * (size_t)c->pool_keys, hipMemcpyDeviceToDevice, st));
        HIPCHK(c, hipMemcpyAsync(s->sm, c->sm, 4 * (size_t)c->nsg, hipMemcpyDeviceToDevice, st));
        HIPCHK(c, hipMemcpyAsync(s->sbuf, c->sbuf, 4 * (size_t)c->nsg, hipMemcpyDeviceToDevice, st));
    }
    HIPCHK(c, hipMemcpyAsync(c->h_ret, c->cnt + C_NDELTA, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    s->ndelta = c->h_ret[0];
    *out = s;
    return DRSF_OK;
}

int drsf_snapshot_restore(drsf_ctx *c, const drsf_snapshot *s) {
    if (!c || !s) return DRSF_E_ARG;
    int rc = finish_pending(c);
    if (rc) return rc;
    if ((rc = check_usable(c))) return rc;
    if (s->n != c->n || s->eb != c->eb || s->dcap != c->dcap || s->dhmask != c->dhmask ||
        s->gm.size() != c->gm_h.size() || s->rebuilds != c->rebuilds || s->nsg != c->nsg ||
        s->pool_keys != c->pool_keys)
        return fail(c, DRSF_E_STATE, "snapshot does not match the context's layout (taken before a "
                                     "store rebuild?)");
    hipStream_t st = c->stream;
    const size_t dh = (size_t)c->dhmask + 1;
    HIPCHK(c, hipMemcpyAsync(c->parent, s->parent, 4 * (size_t)c->n, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(c->label, s->label, 4 * (size_t)c->n, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(c->rep, s->label, 4 * (size_t)c->n, hipMemcpyDeviceToDevice, st));
    if (c->eb) HIPCHK(c, hipMemcpyAsync(c->bcol, s->bcol, 4 * (size_t)c->eb, hipMemcpyDeviceToDevice, st));
    if (c->eb) HIPCHK(c, hipMemcpyAsync(c->lcol, s->lcol, 4 * (size_t)c->eb, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(c->dkey, s->dkey, 8 * (size_t)c->dcap, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(c->dhash, s->dhash, 8 * dh, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(c->dhpos, s->dhpos, 4 * dh, hipMemcpyDeviceToDevice, st));
    if (c->nsg) {
        HIPCHK(c, hipMemcpyAsync(c->pool, s->pool, 4 * (size_t)c->pool_keys, hipMemcpyDeviceToDevice, st));
        HIPCHK(c, hipMemcpyAsync(c->sm, s->sm, 4 * (size_t)c->nsg, hipMemcpyDeviceToDevice, st));
        HIPCHK(c, hipMemcpyAsync(c->sbuf, s->sbuf, 4 * (size_t)c->nsg, hipMemcpyDeviceToDevice, st));
    }
    c->h_ret[0] = s->ndelta;
    HIPCHK(c, hipMemcpyAsync(c->cnt + C_NDELTA, c->h_ret, sizeof(unsigned long long), hipMemcpyHostToDevice, st));
    HIPCHK(c, hipStreamSynchronize(st));
    c->ndelta_bound = s->ndelta_bound;
    c->m_live = s->m_live;
    c->gm_h = s->gm;
    c->view.num_edges = c->m_live;
    return DRSF_OK;
}

void drsf_snapshot_free(drsf_snapshot *s) {
    if (!s) return;
    for (void *p : {(void *)s->parent, (void *)s->label, (void *)s->bcol, (void *)s->lcol, (void *)s->dkey,
                    (void *)s->dhash, (void *)s->dhpos, (void *)s->pool, (void *)s->sm, (void *)s->sbuf})
        raw_dfree(s->opts, p);
    delete s;
}

int drsf_phase_times(drsf_ctx *c, float *ms, int cap) {
    if (!c || !ms) return 0;
    if (finish_pending(c)) return 0;
    if (!c->have_phases) return 0;
    const int k = std::min(cap, (int)PH_N + 2);
    for (int i = 0; i < k; i++) ms[i] = c->phase_ms[i];
    return k;
}

void drsf_destroy(drsf_ctx *c) { destroy_ctx(c); }

}  // extern "C"
