// Internal interface between the host driver and the D-RSF kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "drsf_dev.h"

namespace drsf {

// Shape of one update, read by the kernels from device memory so that one
// captured kernel sequence serves every batch up to the context's maximum.
struct Ctl {
    int64_t b;        // batch entries
    int64_t rlo, rhi; // regions of x0 read by the first two hooking rounds
    int64_t ibase;    // first region written by the insert emitter
    int64_t nvl;      // vertex blocks in vlist (root finding, delete labels); < 0: all
    int64_t nil;      // vertex blocks in ilist (insert labels); < 0: all
    int64_t ntl;      // tiles in tlist (base-store sweep); < 0: all
    int32_t op;       // 0 insert, 1 delete, 2 per-edge op in bop
    int32_t has_ins;  // some edge inserts
    int32_t has_del;  // some edge deletes
    int32_t ngraph;   // graphs in this context (per-graph batch status)
    int32_t lfast;    // search levels queued before the orientation step
    int32_t smode;    // delete sweep: 0 chosen per batch, 1 always the full store
    const int32_t *edges;  // the batch in the caller's device memory, or null: staged copy
    uint64_t seq;          // update number, written to the completion word when done
    int32_t nsmall;        // small graphs with a batch in this update (SmallDev::tasks)
    int32_t pad;
};

// All device pointers one apply needs; passed by value to every kernel.
struct Dev {
    int32_t n;
    int32_t validate;        // 0: batches guaranteed valid (no repeat check, no insert presence search)
    int64_t lb;              // batch size the launch grids are sized for: the batch itself when
                             // launched kernel by kernel, max_batch in a captured graph
    int64_t ltiles;          // tiles of the inserted-edge list the launch covers (at least the
                             // list's length; its capacity in a captured graph)
    int32_t gate;            // 1: an update's own kernels, which stand still while the hold word
                             // is set; 0: the host's continuation of the update that set it
    const Ctl *ctl;          // device copy, written by the first kernel of an update
    Ctl *ctlw;               // the same, writable
    const Ctl *hctl;         // host copy (pinned), read by the first kernel only
    unsigned long long *ctlmem;  // status word, counters, per-graph status (ret_words words)
    unsigned long long *hret;    // pinned host copy of ctlmem, written by the last kernel
    unsigned long long *hdone;   // pinned completion word: the update's seq once hret is final
    int64_t ret_words;
    // edge store: upper-half base CSR (row u holds v > u, ascending; TOMB bit =
    // deleted) plus a list of inserted edges with a hash index
    const uint32_t *bptr;    // [n + 1]
    int32_t *bcol;           // [eb]
    int64_t eb;
    // the same rows without the empty ones (for the sweep): zrow[k] is the k-th
    // non-empty row, its edges are bcol[zptr[k], zptr[k + 1]); tile_k[t] is the
    // non-empty row holding edge t * TILE
    const int32_t *zrow;     // [nz]
    const uint32_t *zptr;    // [nz + 1]
    int64_t nz;
    const int32_t *tile_k;   // [ntiles + 1]
    int64_t ntiles;
    int64_t dtmax;           // tiles of the inserted-edge list at capacity
    uint64_t *dkey;          // [dcap] inserted edge keys, KEY_DEAD when deleted
    int64_t dcap;
    uint64_t *dhash;         // [dhmask + 1] key -> slot, HASH_TOMB_BIT marks a deleted key
    int32_t *dhpos;          // [dhmask + 1] slot -> index in dkey
    uint64_t dhmask;
    // lower half of the same store (row v holds u < v, ascending; TOMB kept
    // in step with the upper copy), so that a vertex's whole adjacency is
    // two contiguous runs
    const uint32_t *lptr;    // [n + 1]
    int32_t *lcol;           // [eb]
    const uint32_t *twin;    // [eb] position in lcol of the mirror of each bcol entry
    const uint32_t *ltwin;   // [eb] position in bcol of the mirror of each lcol entry
    // orphan adjacency scan (delete): per vertex block of BLOCK vertices the
    // listed orphans and their slots, prefixes, the compacted list and, per
    // range of OR_W slots, the list index holding its first slot
    int64_t nvb;             // vertex blocks
    int64_t *bvol;           // [nvb] slots of the block's orphans (zero between updates)
    int32_t *bcnt;           // [nvb] listed orphans of the block (zero between updates)
    int64_t *bpre;           // [nvb] slots before the block within its group of BLOCK blocks
    int32_t *opre;           // [nvb] orphans before the block within its group
    unsigned long long *gsum;  // [ngroups] packed (slots, orphans) per group
    int64_t *gpre;             // [ngroups] slots before the group
    int64_t *gopre;            // [ngroups] orphans before the group
    OrphEnt *olist;          // [n] every orphan, vertex order
    OrphEnt *ostage;         // [nvb * BLOCK] each block's orphans, compacted at the block's start
    int32_t *rstart;         // [2 ntiles + 1]
    unsigned long long *xcnt;  // [ntiles] cross edges found per range
    // forest.  Between updates rep[v] == label[v]; a delete recomputes rep as
    // the root of v in F-hat.
    int32_t *parent;         // [n]
    int32_t *label;          // [n] root of the vertex's tree = smallest vertex of its component
    int32_t *rep;            // [n]
    uint64_t *obits;         // [ceil(n/64)] vertex lies in a piece cut off from its old root
    // touched pieces (trees of F-hat incident to the batch), dense ids
    int32_t *tidx;           // [n] piece root vertex -> dense id, NONE when idle
    int32_t *owner;          // [n] scratch: one registrant per piece, then in a delete each orphan's piece
    uint8_t *pkeep;          // [pcap] piece holds its component's old root (delete)
    int32_t *prt;            // [pcap] dense id -> piece root vertex
    int32_t *pmin;           // [pcap] smallest vertex of the piece
    int32_t *comp;           // [pcap] current component (a dense piece id)
    uint64_t *hook;          // [pcap] (round << 32 | component) the component hooked onto; ~0 before
    uint64_t *best;          // [2 pcap] lowest key of a cross edge leaving the component, in
                             // two buffers by round parity (one is selected into while the
                             // other is cleared)
    uint64_t *srkey;         // [pcap] (smallest vertex << 32 | piece) of the component
    int32_t *head;           // [pcap] first arc of the piece's super-forest arc list
    int32_t *level;          // [pcap] search level of the piece in its super-tree, -1 unreached
    int32_t *parc;           // [pcap] arc from the parent piece (search rooting)
    int32_t *newlab;         // [pcap] new label of the component
    int64_t pcap;
    // batch
    const int32_t *bedges;   // [2 max_b]
    const int8_t *bop;       // [max_b] per-edge op when ctl->op == 2
    const int32_t *bgid;     // [max_b] graph of each edge (several graphs), or null
    const int32_t *goff;     // [ngraph + 1] vertex range of each graph, or null
    int32_t *gstat;          // [ngraph] batch status bits per graph
    int64_t max_b;
    uint64_t *bkey;          // [max_b] normalised key
    int64_t *bloc;           // [max_b] >= 0: position in bcol; < 0: -(hash slot + 1)
    int32_t *bchild;         // [max_b] child endpoint of a deleted tree edge, NONE otherwise
    int32_t *bslot;          // [max_b] slot claimed in the batch duplicate table
    uint64_t *bhash;         // [bhmask + 1] keys claimed by edges whose slot below collided
    uint64_t bhmask;
    int32_t *dslot;          // [dsmask + 1] batch index of the last edge hashed to the slot
    uint64_t dsmask;         // (plain stores; only slots of the current batch are read)
    // vertex-block and tile lists restricting per-vertex and sweep kernels to
    // the graphs that delete or insert (several graphs); see Ctl
    const int32_t *vlist, *ilist, *tlist;
    // cross-edge lists.  x0 is written in regions of TILE entries, one per
    // producing workgroup: region t holds its cross edges at x0[t * TILE ..]
    // and rcnt[t] their number (no global atomics).  Regions [0, ntiles) come
    // from base-store tiles, [ntiles, ntiles + dtmax) from tiles of the
    // inserted-edge list, [ctl->ibase, ...) from the batch.  Later hooking
    // rounds use dense lists alternating between x1 and x0.
    Cross *x0, *x1;
    int64_t xcap;
    unsigned long long *rcnt;  // [regions]
    // replacement edges and super-forest arcs
    int4 *er;                // [ercap] (x, y, piece of x, piece of y)
    int64_t ercap;
    int32_t *arc_nxt;        // [2 ercap]
    int32_t *succ0, *succ1;  // [2 ercap]
    int32_t *rank0, *rank1;  // [2 ercap]
    PathReq *paths;          // [pathcap]
    int64_t pathcap;
    // paths longer than walk_k steps: one thread does not walk them; their
    // indices in paths wait here for the pointer-doubling pass the host
    // launches (vertex-disjoint paths of more than walk_k + 1 vertices, so
    // at most n / (walk_k + 2) of them)
    int32_t *lp_list;        // [lpcap]
    int64_t lpcap;
    int64_t walk_k;
    // path reversal by Euler tour (reverse_mode 1, else null): arc 2v is the
    // down arc from v's parent into v, arc 2v + 1 the up arc back
    uint64_t *et_keys, *et_sorted;  // [n] (F-hat parent << 32 | child), sorted
    int32_t *et_fc, *et_ns;         // [n] first child / next sibling in F-hat (NONE)
    int32_t *et_opar;               // [n] F-hat parents (read before any reversal)
    int32_t *et_nxt0, *et_nxt1;     // [2n] list-ranking successor (NONE past the end)
    int32_t *et_dst0, *et_dst1;     // [2n] arcs after this one in its tour
    int32_t *et_start, *et_finish;  // [n] Euler-tour times of each vertex
    int32_t *et_support;            // [n] support[r] = x for a path (x, r), else NONE
    // control
    int32_t *status;         // internal errors (bounds exceeded); status[1], the other half of
                             // its 8-byte word, is the hold word: set by the cleanup of an
                             // update left unfinished for the host, cleared by the cleanup of
                             // its continuation, so that an update queued behind it on the
                             // stream does nothing in between (the host queues it again)
    unsigned long long *cnt; // [C_TOTAL]
};

// Small graphs of a multi-graph context, updated whole by one workgroup each
// (drsf_small.hip).  Each keeps its edges as an ascending array of 32-bit
// keys u << 16 | v (u < v, local ids) in one of two buffers of scap keys at
// pool + soff; per-vertex scratch at svoff (the graph's first local vertex).
struct SmallDev {
    int32_t nsg;             // small graphs in the context
    int32_t T;               // vertex capacity of the LDS arrays (every small graph's n <= T)
    const int32_t *sgid;     // [nsg] graph id
    const int64_t *soff;     // [nsg] first key of the graph's two buffers
    const int64_t *scap;     // [nsg] keys per buffer
    const int64_t *svoff;    // [nsg] first entry of the graph's per-vertex scratch
    int32_t *sm;             // [nsg] live edges
    int32_t *sbuf;           // [nsg] buffer holding them
    int32_t *sok;            // [nsg] 1: the last update of the graph is staged for commit
    uint32_t *pool;          // edge keys
    uint32_t *xk;            // cross edges, graph s at soff[s]: two halves of scap keys
    int32_t *spar, *slab;    // staged parents and labels (global ids), per vertex
    int2 *er;                // replacement edges (local ids), per vertex slot
    uint32_t *bkeys;         // [max_b] batch keys (a graph's batch range)
    uint32_t *htab;          // [2 max_b + 4 nsg] hash sets of batch keys too large for LDS
    const int4 *tasks;       // [nsmall] (small graph, batch start, batch length, op)
    unsigned int *qhead;     // work queue: next task (reset by the commit kernel)
};
size_t small_lds_bytes(int T);  // dynamic LDS of the small-graph kernel for T vertices
size_t small_static_lds();      // and its static LDS
int small_prepare(int T);  // allows the kernel its LDS (once, before any launch or capture)
int launch_small_update(const Dev &d, const SmallDev &s, int threads, int grid, hipStream_t st);
void launch_small_commit(const Dev &d, const SmallDev &s, int grid, bool alone, hipStream_t st);
void launch_small_init(const Dev &d, const SmallDev &s, hipStream_t st);
// pool growth: live keys to their new regions (new offsets noff[nsg])
void launch_small_regrow(const Dev &d, const SmallDev &s, const int64_t *noff, uint32_t *npool, hipStream_t st);

// slots per range of the orphan adjacency scan (one workgroup pass).  A
// region of x0 (TILE entries, one per base-store tile) takes the cross edges
// of one range, or of two consecutive ranges when the orphans hold more than
// half as many slots as the base store; the scan is used while they hold at
// most as many (so the regions never outnumber the tiles), and a range's
// entries never outnumber its slots.
constexpr int OR_W = 2048;
static_assert(2 * OR_W == TILE, "two orphan ranges fill one x0 region");
constexpr int OR_K = OR_W / BLOCK;  // slots per thread per range
// slots per x0 region of the orphan scan, for V orphan slots and eb stored edges
__host__ __device__ inline int64_t or_region_slots(int64_t V, int64_t eb) {
    return 2 * V <= eb ? OR_W : 2 * OR_W;
}
__host__ __device__ inline int64_t or_regions(int64_t V, int64_t eb) {
    const int64_t r = or_region_slots(V, eb);
    return (V + r - 1) / r;
}
// every orphan also owns OR_PAD empty slots after its adjacency, so a range
// meets at most about OR_W / OR_PAD orphans: one LDS window of BLOCK
constexpr int OR_PAD = OR_W / BLOCK;

constexpr int MAX_ROUNDS = 64;
// hooking rounds in one workgroup (k_bor_tail): its size, and the longest
// live cross-edge list it takes on
constexpr int TAIL_THREADS = 1024;
constexpr int64_t TAIL_MAX = 4096;
// extra counter slots: per-round activity flags
constexpr int C_LR_ROUND = C_COUNT + MAX_ROUNDS;       // [MAX_ROUNDS]
constexpr int C_BFS_ROUND = C_COUNT + 2 * MAX_ROUNDS;  // [MAX_ROUNDS]
// root finding on deep forests: per-round activity flags of the
// pointer-jumping rounds queued before the chase (at most 32: 2^32 > n)
constexpr int MAX_JUMP = 32;
constexpr int C_JUMP_ROUND = C_COUNT + 3 * MAX_ROUNDS;  // [MAX_JUMP]
constexpr int C_TOTAL = C_COUNT + 3 * MAX_ROUNDS + MAX_JUMP;
// statistics of the small-graph engine (it runs beside the chain, whose
// kernels use C_NER and C_NR as list lengths)
constexpr int C_SNER = C_COUNT + 8;
constexpr int C_SNCROSS = C_COUNT + 9;
constexpr int C_SNR = C_COUNT + 10;
// the long-path pass: every long path's start has reached its root
constexpr int C_LP_DONE = C_COUNT + 11;
// root finding: some chase took more than DEEP_STEPS steps (the forest is deep)
constexpr int C_DEEP = C_COUNT + 12;

// Grid sizes.  Workgroups are dispatched at about 200-270 per microsecond
// across the chip, so a kernel of many short workgroups is bound by
// dispatch: grid-stride kernels over vertices are capped near one full wave
// of residency (8 workgroups of 256 threads per CU on 256 CUs).  Kernels
// over pieces, arcs and paths, and the first hooking selections (one
// region per workgroup), have their own caps, set by measurement.
constexpr int GRID_CAP = 2048;
#ifndef DRSF_SMALL_CAP
#define DRSF_SMALL_CAP 2048
#endif
#ifndef DRSF_EDGE_CAP
#define DRSF_EDGE_CAP 4096
#endif
constexpr int SMALL_CAP = DRSF_SMALL_CAP;  // kernels over pieces, arcs and paths
constexpr int EDGE_CAP = DRSF_EDGE_CAP;    // first hooking selections
#ifndef DRSF_FINISH_CAP
#define DRSF_FINISH_CAP 2048
#endif
#ifndef DRSF_COPY_CAP
#define DRSF_COPY_CAP 2048
#endif
constexpr int FINISH_CAP = DRSF_FINISH_CAP;  // each part of path reversal + labels
constexpr int COPY_CAP = DRSF_COPY_CAP;      // rep <- parent beside the store update
#ifndef DRSF_CLEANUP_CAP
#define DRSF_CLEANUP_CAP 128
#endif
constexpr int CLEANUP_CAP = DRSF_CLEANUP_CAP;  // cleanup (its workgroups share one arrival counter)
int grid_for(int64_t items, int64_t per_block, int cap = GRID_CAP);
int64_t delta_tiles(int64_t count);
int64_t insert_regions(int64_t b);

// launchers of the update path (drsf_kernels.hip); grids are sized from the
// context's maxima so that a captured sequence fits every batch
// kc: the control block passed with the launch (a kernel-by-kernel launch),
// or null: read from pinned host memory (a captured one)
void launch_classify(const Dev &d, const Ctl *kc, hipStream_t s);
void launch_dedupe(const Dev &d, hipStream_t s);  // repeated pairs inside the batch
void launch_prepare(const Dev &d, bool del, hipStream_t s);  // with rep <- parent when del
void launch_register(const Dev &d, hipStream_t s);
void launch_insert_emit(const Dev &d, hipStream_t s);
// pointer-jumping rounds over rep before the chase (deep forests); a round
// after one that changed nothing exits at once
void launch_rep_jump(const Dev &d, int rounds, hipStream_t s);
void launch_rep_chase(const Dev &d, hipStream_t s);
void launch_sweep_base(const Dev &d, hipStream_t s);
void launch_orphan_plan(const Dev &d, hipStream_t s);  // block prefixes, totals and scan mode
void launch_orphan_fill(const Dev &d, hipStream_t s);  // the orphan list
void launch_orphan_scan(const Dev &d, hipStream_t s);
void launch_sweep_delta(const Dev &d, hipStream_t s);
// units: regions of x0 the first two rounds may read (sizes their grids)
// rounds [r0, r1); emit: round 0 also emits the insert cross edges
// (k_insert_emit not launched)
void launch_boruvka(const Dev &d, int r0, int r1, int64_t units, bool emit, hipStream_t s);
void launch_sf_root(const Dev &d, hipStream_t s);
void launch_sf_bfs(const Dev &d, int l0, int l1, hipStream_t s);
void launch_orient_bfs(const Dev &d, int levels, hipStream_t s);
// the super-forest's Euler tour when the search of `levels` levels did not
// finish (skips itself otherwise)
void launch_superforest_lr(const Dev &d, int lr_rounds, int levels, hipStream_t s);
// label kernels of the ops present (delete labels run first)
void launch_finish(const Dev &d, bool ins, bool del, bool rev, hipStream_t s);  // path reversal and labels
// Buffers of the pass that turns the paths too long for one thread's walk
// (allocated when such a path first occurs).
struct LongPaths {
    int32_t *p0;        // [n] parents as the pass starts (the orientation to turn)
    int32_t *j0, *j1;   // [n] the ancestor 2^k steps up, capped at the root (two buffers)
    uint32_t *mark;     // [n] == epoch: the vertex lies on a long path
    uint32_t epoch;     // differs from every mark left by an earlier pass
    int64_t nlong;      // long paths listed in lp_list
};
// that pass: rounds of pointer doubling (enough for any path in n vertices),
// then the reversal and the paths' new parents
void launch_long_paths(const Dev &d, const LongPaths &b, hipStream_t s);
// path reversal by Euler tour (Alg. 3); tmp/tmp_bytes: radix-sort scratch
int launch_et_reverse(const Dev &d, void *tmp, size_t tmp_bytes, hipStream_t s);
// Supergraph (Sec. III-A): the first round's cross edges reduced to one per
// pair of pieces (the lowest key), written densely to x0 with its count in
// C_NX0, ready for hooking rounds started at SG_ROUND0.
constexpr int SG_ROUND0 = 3;
struct SgScratch {
    uint32_t *rcount, *rpos;     // [nregmax] cross edges per region, prefix
    uint32_t *flag, *segid;      // [xcap] segment heads, segment index
    uint64_t *skeys, *svals;     // [xcap] sorted (piece pair, edge key)
    unsigned long long *totals;  // [2] device totals (edges, segments)
    void *scan_tmp;              // scan scratch (for xcap items)
    void *sort_tmp;
    size_t sort_tmp_bytes;
};
void launch_sg_regions(const Dev &d, int64_t nr_om, int64_t rlo2, int64_t nreg, const SgScratch &g,
                       hipStream_t s);
int launch_sg_reduce(const Dev &d, int64_t nr_om, int64_t rlo2, int64_t nreg, int64_t total,
                     const SgScratch &g, hipStream_t s);
void launch_cleanup(const Dev &d, hipStream_t s);

// store rebuild: live flags of the base store's halves (scanned into
// prefix counts), the inserted edges as directed pairs (x << 32 | y, both
// directions), their per-row counts, the merged rows' sizes, and the merged
// symmetric CSR
void launch_rb_live(const int32_t *col, int64_t eb, uint32_t *flag, hipStream_t s);
void launch_rb_row_count(int32_t n, const uint32_t *bptr, const uint32_t *lptr, const uint32_t *LS,
                         const uint32_t *US, const uint32_t *ddeg, uint32_t *deg, hipStream_t s);
void launch_rb_pairs(const uint64_t *dkey, const unsigned long long *ndelta, uint64_t *pairs,
                     unsigned long long *npairs, int64_t cap, hipStream_t s);
void launch_rb_pair_deg(const uint64_t *pairs, const unsigned long long *npairs, uint32_t *ddeg,
                        int64_t cap, hipStream_t s);
void launch_add_u32(const uint32_t *a, const uint32_t *b, uint32_t *out, int64_t count, hipStream_t s);
void launch_u32_to_i64(const uint32_t *in, int64_t *out, int64_t count, hipStream_t s);
void launch_rb_fill(int32_t n, int64_t eb, const uint32_t *bptr, const int32_t *bcol, const uint32_t *lptr,
                    const int32_t *lcol, const uint32_t *LS, const uint32_t *US, const uint64_t *pairs,
                    const unsigned long long *npairs, int64_t cap, const uint32_t *dstart, const uint32_t *ddeg,
                    const int64_t *row_ptr, int32_t *col, hipStream_t s);
size_t sort_u64_tmp_bytes(int64_t count);
size_t sort_pairs_u64_tmp_bytes(int64_t count);
int launch_sort_pairs_u64(const uint64_t *kin, uint64_t *kout, const uint64_t *vin, uint64_t *vout,
                          int64_t count, void *tmp, size_t tmp_bytes, hipStream_t s);
int launch_sort_u64(const uint64_t *in, uint64_t *out, int64_t count, void *tmp, size_t tmp_bytes,
                    hipStream_t s);

// digests of parent and label (out: two device words)
void launch_digest(int32_t n, const int32_t *parent, const int32_t *label, unsigned long long *out,
                   hipStream_t s);

// create-time helpers
void launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t s);
void launch_fill_u64(uint64_t *p, int64_t count, uint64_t v, hipStream_t s);
inline void launch_fill_u64(unsigned long long *p, int64_t count, uint64_t v, hipStream_t s) {
    launch_fill_u64(reinterpret_cast<uint64_t *>(p), count, v, s);
}
// entries checked (ids, self-loops, ascending rows) and each row's entries
// above the diagonal counted into ucnt
void launch_csr_check(int32_t n, const int64_t *row_ptr, const int32_t *col, int64_t nnz, uint32_t *ucnt,
                      int32_t *status, const int32_t *goff, int32_t ngraph, hipStream_t s);
void launch_csr_symmetric(int32_t n, const int64_t *row_ptr, const int32_t *col,
                          int32_t *status, hipStream_t s);
// exclusive scan of n uint32 counts into out[n + 1] (64-bit total in *total)
void launch_scan_u32(const uint32_t *in, uint32_t *out, unsigned long long *total, int64_t n,
                     void *tmp, hipStream_t s);
size_t scan_tmp_bytes(int64_t n);
void launch_upper_fill(int32_t n, const int64_t *row_ptr, const int32_t *col,
                       const uint32_t *bptr, int32_t *bcol, int64_t eb, hipStream_t s);
// lower half: counts (row length minus upper count), then the row prefixes
void launch_lower_counts(int32_t n, const int64_t *row_ptr, const uint32_t *bptr, uint32_t *lcnt,
                         hipStream_t s);
void launch_lower_fill(int32_t n, const int64_t *row_ptr, const int32_t *col,
                       const uint32_t *lptr, int32_t *lcol, int64_t eb, hipStream_t s);
void launch_twin(int32_t n, const uint32_t *bptr, const int32_t *bcol, const uint32_t *lptr,
                 const int32_t *lcol, uint32_t *twin, uint32_t *ltwin, int32_t *status, int64_t eb,
                 hipStream_t s);
// non-empty row index: flags -> (scan) -> zrow/zptr, then tile_k
void launch_nonempty_flags(int32_t n, const uint32_t *bptr, uint32_t *flag, hipStream_t s);
void launch_nonempty_fill(int32_t n, const uint32_t *bptr, const uint32_t *zpos, int32_t *zrow,
                          uint32_t *zptr, int64_t nz, hipStream_t s);
void launch_tile_k(const uint32_t *zptr, int64_t nz, int64_t eb, int32_t *tile_k, int64_t ntiles,
                   hipStream_t s);
void launch_forest_check(int32_t n, const uint32_t *bptr, const int32_t *bcol,
                         const int32_t *parent, int32_t *status, int check_edges, hipStream_t s);
void launch_pointer_jump(int32_t n, const int32_t *in, int32_t *out, hipStream_t s);
// flag = 1 if some jump[v] is not a root (jump: the ancestors 2^k steps up)
void launch_deeper_than(int32_t n, const int32_t *jump, unsigned long long *flag, hipStream_t s);
void launch_roots_check(int32_t n, const int32_t *parent, const int32_t *root,
                        int32_t *status, hipStream_t s);
void launch_span_check(const Dev &d, const int32_t *root, hipStream_t s);
void launch_tree_min(int32_t n, const int32_t *root, int32_t *label, hipStream_t s);
void launch_reroot_requests(const Dev &d, const int32_t *root, hipStream_t s);
void launch_reverse_all(const Dev &d, hipStream_t s);

}  // namespace drsf
