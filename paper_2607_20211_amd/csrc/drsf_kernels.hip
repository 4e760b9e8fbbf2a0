// D-RSF kernels for gfx950 (CDNA4, wave64).  One batch update follows
// Algorithm 1 of "Fully Dynamic Rooted Spanning Tree on GPU":
//   classify/validate -> update the edge store and cut deleted tree edges ->
//   root finding (delete) -> key-edge scan (the orphans' adjacency, or the
//   whole store, plus the inserted-edge list) -> replacement edges by
//   hooking rounds (Alg. 2, phase 1) -> super-forest rooting by a
//   level-synchronous search from the super-roots, or an Euler tour with
//   list ranking for deep super-trees (Alg. 2, phase 2) -> path reversal and
//   new parents (ReversePaths, Algorithm 1) -> component labels.
// All integer work; no MFMA.  Every loop over device-side counts is a
// grid-stride loop, every pointer chase is bounded by n and reports
// ST_WALK_BOUND instead of spinning, and every kernel after validation is a
// no-op when the status word is non-zero, so a rejected batch changes nothing.
#include "drsf_kernels.h"

#include <utility>

namespace drsf {

int grid_for(int64_t items, int64_t per_block, int cap) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// ------------------------------------------------------------------ helpers

// Position of column v in the ascending run col[lo, hi) (tombstone bits
// ignored), or -1; *raw receives the stored entry.  Each step loads
// SEARCH_FAN evenly spaced entries at once and keeps the part of the run
// that can hold v, so a run of length L takes about log_{FAN+1}(L)
// dependent loads.
#ifndef DRSF_SEARCH_FAN
#define DRSF_SEARCH_FAN 4
#endif
constexpr int SEARCH_FAN = DRSF_SEARCH_FAN;
__device__ __forceinline__ int64_t find_in_row(const int32_t *col, uint32_t lo, uint32_t hi,
                                               int32_t v, int32_t *raw) {
    constexpr int F = SEARCH_FAN;
    // the first entry >= v lies in [a, b]; cb is col[b] when b < hi
    uint32_t a = lo, b = hi;
    int32_t cb = 0;
    while (b - a > (uint32_t)F) {
        const uint32_t w = (b - a) / (F + 1);
        int32_t c[F];
#pragma unroll
        for (int j = 0; j < F; j++) c[j] = col[a + (uint32_t)(j + 1) * w];
        int cnt = 0;
#pragma unroll
        for (int j = 0; j < F; j++) cnt += (c[j] & COLMASK) < v;
        if (cnt < F) {
#pragma unroll
            for (int j = 0; j < F; j++)
                if (j == cnt) cb = c[j];
            b = a + (uint32_t)(cnt + 1) * w;
        }
        if (cnt > 0) a += (uint32_t)cnt * w + 1;
    }
    int64_t pos = -1;
#pragma unroll
    for (int j = 0; j < F; j++) {
        if (a + (uint32_t)j < b) {
            const int32_t c = col[a + j];
            if ((c & COLMASK) == v) {
                pos = a + j;
                *raw = c;
            }
        }
    }
    if (pos < 0 && b < hi && (cb & COLMASK) == v) {
        pos = b;
        *raw = cb;
    }
    return pos;
}

// slot holding live key k in the inserted-edge index, or -1
__device__ int64_t dhash_find(const Dev &d, uint64_t k) {
    uint64_t h = hmix(k) & d.dhmask;
    for (uint64_t probe = 0; probe <= d.dhmask; probe++) {
        uint64_t s = d.dhash[h];
        if (s == HASH_EMPTY) return -1;
        if (s == k) return (int64_t)h;
        h = (h + 1) & d.dhmask;
    }
    return -1;
}

// insert key k (not live in the index) pointing at list position pos
__device__ void dhash_insert(const Dev &d, uint64_t k, int32_t pos) {
    uint64_t h = hmix(k) & d.dhmask;
    for (uint64_t probe = 0; probe <= 2 * d.dhmask + 2; probe++) {
        uint64_t s = d.dhash[h];
        if (s == HASH_EMPTY || s == (k | HASH_TOMB_BIT)) {
            uint64_t old = atomicCAS((unsigned long long *)&d.dhash[h], (unsigned long long)s,
                                     (unsigned long long)k);
            if (old == s) {
                d.dhpos[h] = pos;
                return;
            }
            continue;  // lost a race for this slot: look at it again
        }
        h = (h + 1) & d.dhmask;
    }
    atomicOr(d.status, ST_CAPACITY);
}

// Row holding slot j of a CSR with offsets ptr[0..n]: the largest u with
// ptr[u] <= j (empty rows share their start with the next row, so the
// largest such u is the row that holds j).
template <class P>
__device__ __forceinline__ int32_t row_of(const P *ptr, int32_t n, int64_t j) {
    int32_t a = 0, b = n - 1;
    while (a < b) {
        const int32_t mid = a + ((b - a + 1) >> 1);
        if ((int64_t)ptr[mid] <= j) a = mid;
        else b = mid - 1;
    }
    return a;
}

__device__ __forceinline__ bool obit(const uint64_t *bits, int32_t v) {
    return (bits[v >> 6] >> (v & 63)) & 1;
}

__device__ __forceinline__ void init_piece(const Dev &d, int64_t id, int32_t v, bool keep) {
    d.prt[id] = v;
    d.pmin[id] = v;
    d.comp[id] = (int32_t)id;
    d.hook[id] = HOOK_NONE;
    d.best[id] = KEY_INF;
    d.best[d.pcap + id] = KEY_INF;
    d.srkey[id] = KEY_INF;
    d.head[id] = NONE;
    d.newlab[id] = v;
    d.pkeep[id] = keep ? 1 : 0;
    d.tidx[v] = (int32_t)id;  // read by later kernels only
}

// Exclusive scan of one int per thread over the block; also returns the total.
// Every thread of the block must call it.
__device__ int block_excl_scan(int x, int *total) {
    __shared__ int wsum[BLOCK / WAVE];
    const int lane = lane_id(), wid = threadIdx.x / WAVE;
    int inc = x;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        int y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == WAVE - 1) wsum[wid] = inc;
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / WAVE; w++) {
        before += w < wid ? wsum[w] : 0;
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return before + inc - x;
}

// 64-bit exclusive scan over the block; also returns the total.  Every
// thread of the block must call it.
__device__ unsigned long long block_excl_scan64(unsigned long long x, unsigned long long *total) {
    __shared__ unsigned long long wsum[BLOCK / WAVE];
    const int lane = lane_id(), wid = threadIdx.x / WAVE;
    unsigned long long inc = x;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const unsigned long long y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == WAVE - 1) wsum[wid] = inc;
    __syncthreads();
    unsigned long long before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / WAVE; w++) {
        before += w < wid ? wsum[w] : 0;
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return before + inc - x;
}

// Sum over the block (one barrier pair).  Every thread must call it.
__device__ unsigned long long block_sum64(unsigned long long x) {
    __shared__ unsigned long long wsum[BLOCK / WAVE];
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (lane_id() == 0) wsum[threadIdx.x / WAVE] = x;
    __syncthreads();
    unsigned long long t = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / WAVE; w++) t += wsum[w];
    __syncthreads();
    return t;
}

// (slots, orphans) packed into one word so that one sum or scan carries both:
// slots below 2^44, orphans in the 20 bits above.  Used only within a group
// of BLOCK vertex blocks (at most 2^16 orphans); the prefixes over the
// groups keep the two apart (the orphans of a whole graph can pass 2^20).
__device__ __forceinline__ unsigned long long opack(unsigned long long vol, unsigned long long c) {
    return (c << 44) | vol;
}
__device__ __forceinline__ unsigned long long ovol(unsigned long long p) { return p & ((1ull << 44) - 1); }
__device__ __forceinline__ unsigned long long ocnt(unsigned long long p) { return p >> 44; }

// Block-aggregated append: each thread reserves k consecutive slots of
// *counter and gets the first; one atomic per workgroup (a counter shared by
// the whole grid is a hot address).  Every thread of the block must call it.
__device__ int64_t block_append(int k, unsigned long long *counter) {
    __shared__ unsigned long long s_base;
    int total;
    const int off = block_excl_scan(k, &total);
    if (threadIdx.x == 0 && total) s_base = atomicAdd(counter, (unsigned long long)total);
    __syncthreads();
    const int64_t r = (int64_t)s_base + off;
    __syncthreads();  // s_base is reused by the next call
    return r;
}

// True in the workgroup that arrives last among the kernel's gridDim.x
// workgroups (every workgroup calls it once, with all its threads); that
// workgroup also resets the counter.  No fence: it orders the workgroups'
// earlier reads (all consumed before the barrier) before the last one's
// writes, and publishes no data between workgroups (a device-wide fence
// writes back the L2 and costs microseconds per workgroup).
__device__ bool last_block_arrives(unsigned long long *arrive) {
    __shared__ bool s_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        s_last = atomicAdd(arrive, 1ull) == (unsigned long long)gridDim.x - 1;
        if (s_last) atomicExch(arrive, 0ull);
    }
    __syncthreads();
    return s_last;
}

// The update has failed, or it is queued behind one that the host has yet
// to finish: status and hold word in one load.
__device__ __forceinline__ uint64_t status_word(const Dev &d) {
    return *reinterpret_cast<const uint64_t *>(d.status);
}
__device__ __forceinline__ bool held(const Dev &d) { return d.gate && (status_word(d) >> 32) != 0; }
__device__ __forceinline__ bool stopped(const Dev &d) {
    const uint64_t w = status_word(d);
    return (uint32_t)w != 0 || (d.gate && (w >> 32) != 0);
}

__device__ __forceinline__ int edge_op(const Dev &d, int64_t i) {
    return d.ctl->op == 2 ? (int)d.bop[i] : d.ctl->op;
}
__device__ __forceinline__ int32_t edge_graph(const Dev &d, int64_t i) {
    return d.bgid ? d.bgid[i] : 0;
}
// the edge's graph accepted its batch
__device__ __forceinline__ bool edge_ok(const Dev &d, int64_t i) {
    return d.gstat[edge_graph(d, i)] == 0;
}
// vertex block (BLOCK vertices) handled by the j-th slot of a list, or -1
__device__ __forceinline__ int64_t list_block(const int32_t *list, int64_t cnt, int64_t j,
                                              int64_t all) {
    if (cnt < 0) return j < all ? j : -1;
    return j < cnt ? list[j] : -1;
}

// -------------------------------------------------- a1: validate + classify

// Normalise each pair, reject self-loops, ids outside the edge's graph and
// pairs repeated inside the batch, check presence against the edge store
// (insert: must be absent; delete: must be present) and, for deletes, find
// the child endpoint of a tree edge (parent[u] == v or parent[v] == u;
// Algorithm 1, the cut step).  Errors mark the edge's graph as rejected;
// nothing but batch scratch is written.
__global__ __launch_bounds__(BLOCK) void k_classify(Dev d, Ctl kc, int from_arg) {
    if (held(d)) return;  // the device copy of the control block still serves the held update
    // the update's control block comes from pinned host memory (a captured
    // launch) or with the launch (a kernel-by-kernel one); the first
    // workgroup publishes it for the later kernels, which read the device copy
    int64_t b;
    int opm;
    const int32_t *edges;
    if (from_arg) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *d.ctlw = kc;
        b = kc.b;
        opm = kc.op;
        edges = kc.edges;
    } else {
        const Ctl *hc = d.hctl;
        if (blockIdx.x == 0 && threadIdx.x < sizeof(Ctl) / 8)
            reinterpret_cast<uint64_t *>(d.ctlw)[threadIdx.x] =
                reinterpret_cast<const uint64_t *>(hc)[threadIdx.x];
        b = hc->b;
        opm = hc->op;
        edges = hc->edges;
    }
    const int32_t *be = edges ? edges : d.bedges;  // caller's device batch, or the staged one
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < b; i += stride) {
        d.bslot[i] = NONE;
        d.bchild[i] = NONE;
        d.bloc[i] = 0;
        if (opm == 2 && d.bop[i] == 2) {  // a small graph's edge: its own kernel takes it
            d.bkey[i] = 0;
            continue;
        }
        const int32_t u = be[2 * i], v = be[2 * i + 1];
        const int32_t g = edge_graph(d, i);
        const int32_t lo_ok = d.goff ? d.goff[g] : 0, hi_ok = d.goff ? d.goff[g + 1] : d.n;
        if (u < lo_ok || v < lo_ok || u >= hi_ok || v >= hi_ok || u == v) {
            atomicOr(&d.gstat[g], ST_BAD_PAIR);
            d.bkey[i] = 0;
            continue;
        }
        const uint64_t k = mkkey((uint32_t)u, (uint32_t)v);
        d.bkey[i] = k;
        if (!d.validate && (opm == 2 ? (int)d.bop[i] : opm) == 0) continue;  // an absent pair, by contract
        const int32_t lo = key_lo(k), hi = key_hi(k);
        // loads that do not depend on the probes below, issued first (the
        // parents only where the batch holds deletes)
        const uint32_t ua = d.bptr[lo], ub = d.bptr[lo + 1], la = d.lptr[hi], lb = d.lptr[hi + 1];
        const int opi = opm == 2 ? (int)d.bop[i] : opm;
        int32_t plo = NONE, phi = NONE;
        if (opm != 0) {
            plo = d.parent[lo];
            phi = d.parent[hi];
        }
        // repeated pairs: every edge stamps its slot (checked by k_dedupe)
        if (d.validate) d.dslot[hmix(k) & d.dsmask] = (int32_t)i;
        // presence: the edge sits in upper row lo and in lower row hi (with
        // mirrored tombstones); search the shorter and map a lower hit up
        int64_t pos;
        int32_t raw = TOMB;
        if (ub - ua <= lb - la) {
            pos = find_in_row(d.bcol, ua, ub, hi, &raw);
        } else {
            const int64_t q = find_in_row(d.lcol, la, lb, lo, &raw);
            pos = q >= 0 ? (int64_t)d.ltwin[q] : -1;
        }
        int64_t loc;
        bool present;
        if (pos >= 0 && raw >= 0) {
            present = true;
            loc = pos;
        } else {
            const int64_t slot = dhash_find(d, k);
            present = slot >= 0;
            loc = -(slot + 1);
        }
        if (opi == 0) {
            if (present) atomicOr(&d.gstat[g], ST_EXISTS);
        } else {
            if (!present) {
                atomicOr(&d.gstat[g], ST_MISSING);
            } else {
                d.bloc[i] = loc;
                d.bchild[i] = plo == hi ? lo : (phi == lo ? hi : NONE);
            }
        }
    }
}

// Repeated pairs inside the batch.  Equal keys hash to one slot and exactly
// one of their stamps survives, so an edge that finds another edge's stamp
// compares keys: equal is a repeat; different is a collision, and such edges
// claim their key in a table with compare-and-swap, where repeats among them
// meet.  Only the colliding edges (about 1 in 16) pay for an atomic.
__global__ __launch_bounds__(BLOCK) void k_dedupe(Dev d) {
    if (held(d)) return;
    const int64_t b = d.ctl->b;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < b; i += stride) {
        const uint64_t k = d.bkey[i];
        if (k == 0) continue;  // rejected pair (its graph is marked already)
        const int32_t j = d.dslot[hmix(k) & d.dsmask];
        if (j == (int32_t)i) continue;
        const int32_t g = edge_graph(d, i);
        if (d.bkey[j] == k) {
            atomicOr(&d.gstat[g], ST_DUPLICATE);
            continue;
        }
        uint64_t h = hmix(k) & d.bhmask;
        for (uint64_t probe = 0; probe <= d.bhmask; probe++) {
            const uint64_t prev = atomicCAS((unsigned long long *)&d.bhash[h],
                                            (unsigned long long)HASH_EMPTY, (unsigned long long)k);
            if (prev == HASH_EMPTY) {
                d.bslot[i] = (int32_t)h;
                break;
            }
            if (prev == k) {
                atomicOr(&d.gstat[g], ST_DUPLICATE);
                break;
            }
            h = (h + 1) & d.bhmask;
        }
    }
}

// ---------------------------- a2 + a3: update the edge store, cut tree edges

// Also nominates the trees of F-hat the batch touches: each touched piece
// root gets owner[root] = (batch index, side) by plain stores; whichever
// store lands last owns the registration in k_register (no contended atomics
// on the roots of big trees).
// Workgroups from gb on (launched for batches with deletes) start root
// finding instead: rep <- parent over the listed vertex blocks, one wave per
// block, four vertices per lane (16-byte accesses).  A cut child may be
// copied before or after its cut; k_register then sets rep[c] = c.
__device__ void rep_init(const Dev &d, int64_t bid, int64_t nblk) {
    typedef int v4i __attribute__((ext_vector_type(4)));
    const int64_t nb = (d.n + BLOCK - 1) / BLOCK;
    const int w = threadIdx.x / WAVE;
    const int64_t nvl_list = d.ctl->nvl;  // read once: stores below may alias it
    for (int64_t j = bid * (BLOCK / WAVE) + w;; j += nblk * (BLOCK / WAVE)) {
        const int64_t blk = list_block(d.vlist, nvl_list, j, nb);
        if (blk < 0) break;
        const int64_t v = blk * BLOCK + lane_id() * 4;
        if (v + 4 <= d.n) {
            *reinterpret_cast<v4i *>(d.rep + v) = *reinterpret_cast<const v4i *>(d.parent + v);
        } else {
            for (int64_t u = v; u < d.n && u < v + 4; u++) d.rep[u] = d.parent[u];
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_prepare(Dev d, int gb) {
    if (stopped(d)) return;
    if ((int)blockIdx.x >= gb) {
        if (d.ctl->has_del) rep_init(d, (int64_t)blockIdx.x - gb, (int64_t)gridDim.x - gb);
        return;
    }
    const int64_t b = d.ctl->b;
    const int64_t stride = (int64_t)gb * BLOCK;
    for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < b; base += stride) {
        const int64_t i = base + threadIdx.x;
        const bool valid = i < b && edge_op(d, i) != 2 && edge_ok(d, i);
        const int op = valid ? edge_op(d, i) : -1;
        if (op == 1) {
            const int64_t loc = d.bloc[i];
            if (loc >= 0) {
                d.bcol[loc] = d.bcol[loc] | TOMB;
                const uint32_t l2 = d.twin[loc];
                d.lcol[l2] = d.lcol[l2] | TOMB;
            } else {
                const int64_t slot = -loc - 1;
                d.dkey[d.dhpos[slot]] = KEY_DEAD;
                d.dhash[slot] = d.bkey[i] | HASH_TOMB_BIT;
            }
            const int32_t c = d.bchild[i];
            if (c != NONE) {
                d.parent[c] = c;  // Algorithm 1: parent[u] <- u
                // orphan piece rooted at c, and the piece keeping the old root
                d.owner[c] = (int32_t)(2 * i);
                d.owner[d.label[c]] = (int32_t)(2 * i + 1);
            }
        }
        const int64_t pos = block_append(op == 0 ? 1 : 0, &d.cnt[C_NDELTA]);
        if (op == 0) {
            const uint64_t k = d.bkey[i];
            if (pos >= d.dcap) {
                atomicOr(d.status, ST_CAPACITY);
            } else {
                d.dkey[pos] = k;
                dhash_insert(d, k, (int32_t)pos);
                const int32_t la = d.label[key_lo(k)], lb = d.label[key_hi(k)];
                if (la != lb) {
                    d.owner[la] = (int32_t)(2 * i);
                    d.owner[lb] = (int32_t)(2 * i + 1);
                }
            }
        }
    }
}

// Dense ids for the nominated pieces: the owning batch entry registers.
__global__ __launch_bounds__(BLOCK) void k_register(Dev d) {
    if (stopped(d)) return;
    const int64_t b = d.ctl->b;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < b; base += stride) {
        const int64_t i = base + threadIdx.x;
        int32_t a = NONE, c2 = NONE;
        bool del = false;
        if (i < b && edge_op(d, i) != 2 && edge_ok(d, i)) {
            del = edge_op(d, i) == 1;
            if (del) {
                const int32_t c = d.bchild[i];
                if (c != NONE) {
                    a = c;
                    c2 = d.label[c];
                    d.rep[c] = c;  // the cut child roots its piece of F-hat
                }
            } else {
                const uint64_t k = d.bkey[i];
                const int32_t la = d.label[key_lo(k)], lb = d.label[key_hi(k)];
                if (la != lb) { a = la; c2 = lb; }
            }
        }
        const bool ga = a != NONE && d.owner[a] == (int32_t)(2 * i);
        const bool gb = c2 != NONE && d.owner[c2] == (int32_t)(2 * i + 1);
        const int64_t ia = block_append((ga ? 1 : 0) + (gb ? 1 : 0), &d.cnt[C_NP]);
        const int64_t ib = ia + (ga ? 1 : 0);
        if (ga) init_piece(d, ia, a, false);
        if (gb) init_piece(d, ib, c2, del);
    }
}

// insert: key edges M = B; cross edges join two different trees (labels).
// Batch entries [t * BLOCK, (t + 1) * BLOCK) go to region ibase + t of x0;
// every thread of the workgroup calls it.  Returns the thread's edge (live
// when it is a cross edge) and, through *total, the region's count.
__device__ bool insert_emit_block(const Dev &d, int64_t t, Cross *e, int *total) {
    const int64_t b = d.ctl->b;
    const int64_t i = t * BLOCK + threadIdx.x;
    bool cross = false;
    uint64_t k = 0;
    int32_t la = 0, lb = 0;
    if (i < b && edge_op(d, i) == 0 && edge_ok(d, i)) {
        k = d.bkey[i];
        la = d.label[key_lo(k)];
        lb = d.label[key_hi(k)];
        cross = la != lb;
    }
    const int off = block_excl_scan(cross ? 1 : 0, total);
    const int64_t reg = d.ctl->ibase + t;
    if (threadIdx.x == 0) d.rcnt[reg] = (unsigned long long)*total;
    e->key = k;
    e->pa = e->pb = 0;
    if (cross) {
        e->pa = d.tidx[la];
        e->pb = d.tidx[lb];
        d.x0[reg * TILE + off] = *e;
    }
    return cross;
}

// The insert emit on its own (the supergraph reads the regions before the
// first round); in the default mode the first hooking round does it.
__global__ __launch_bounds__(BLOCK) void k_insert_emit(Dev d) {
    if (stopped(d) || !d.ctl->has_ins) return;
    const int64_t t = blockIdx.x;
    if (t * BLOCK >= d.ctl->b) return;
    Cross e;
    int total;
    (void)insert_emit_block(d, t, &e, &total);
}

// ----------------------------------------------- a4: root finding (delete)

// rep[v] <- root of v in F-hat.  Each thread chases rep[] upward; entries
// already finished by other threads are roots, so chains shorten as the
// sweep proceeds (pointer jumping, Algorithm 1).  A chase longer than a few
// steps also publishes its progress in rep[v] after every step, so the
// chases of v's descendants jump over what v has covered: on deep trees
// (long paths of vertices chased at the same time) a chain then takes
// about log of its length in steps instead of half of it.  Every value
// read or published is an ancestor of the vertex, so stale reads only cost
// extra steps.  A thread
// can take REP_CH vertex blocks at a time and interleave their chases and
// the loads that follow (on gfx950 one block at a time measures fastest:
// the whole grid is resident, so more chains per thread add no overlap).
// Marks vertices whose root is not their old root (they lie in a
// piece cut off by the batch), stages each block's such orphans, compacted
// at the block's start, with their adjacency runs, their piece and their
// old root's piece for the orphan scan, and lowers each orphan piece's
// smallest vertex.  (Loading the next block's rep and label before the
// chase of the current one measured slower.)
#ifndef DRSF_REP_CH
#define DRSF_REP_CH 1
#endif
constexpr int REP_CH = DRSF_REP_CH;
constexpr int PUBLISH_AFTER = 4;  // steps before a chase publishes its progress (short chains never do)
#ifndef DRSF_DEEP_STEPS
#define DRSF_DEEP_STEPS 1024
#endif
constexpr int64_t DEEP_STEPS = DRSF_DEEP_STEPS;  // a chase longer than this marks the forest deep

// One round of pointer jumping over the listed vertex blocks (Alg. 1's own
// root finding), queued before the chase on a forest found deep: rep[v] <-
// rep[rep[v]], in place (every value read is an ancestor of v, so a value
// another thread has just written only jumps further).  Round k runs only
// if round k - 1 changed some entry; after ceil(log2 depth) rounds every
// entry is a root and the chase takes one step per vertex.
__global__ __launch_bounds__(BLOCK) void k_rep_jump(Dev d, int k) {
    if (stopped(d) || !d.ctl->has_del) return;
    if (k > 0 && !d.cnt[C_JUMP_ROUND + k - 1]) return;
    const int64_t nb = (d.n + BLOCK - 1) / BLOCK;
    const int64_t nvl_list = d.ctl->nvl;  // read once: stores below may alias it
    bool changed = false;
    for (int64_t j = blockIdx.x;; j += gridDim.x) {
        const int64_t blk = list_block(d.vlist, nvl_list, j, nb);
        if (blk < 0) break;
        const int64_t v = blk * BLOCK + threadIdx.x;
        if (v >= d.n) continue;
        const int32_t x = ld_relaxed(&d.rep[v]);
        const int32_t y = ld_relaxed(&d.rep[x]);
        if (y != x) {
            d.rep[v] = y;
            changed = true;
        }
    }
    if (__ballot(changed) != 0 && lane_id() == 0) d.cnt[C_JUMP_ROUND + k] = 1;
}
__global__ __launch_bounds__(BLOCK) void k_rep_chase(Dev d) {
    if (stopped(d) || !d.ctl->has_del) return;
    const int64_t nb = (d.n + BLOCK - 1) / BLOCK;
    const int64_t nvl_list = d.ctl->nvl;  // read once: stores below may alias it
    for (int64_t j0 = (int64_t)blockIdx.x * REP_CH;; j0 += (int64_t)gridDim.x * REP_CH) {
        int64_t blk[REP_CH], v[REP_CH];
        int32_t x[REP_CH], lab[REP_CH];
        bool live[REP_CH], act[REP_CH];
#pragma unroll
        for (int k = 0; k < REP_CH; k++) {
            blk[k] = list_block(d.vlist, nvl_list, j0 + k, nb);
            v[k] = blk[k] >= 0 ? blk[k] * BLOCK + threadIdx.x : d.n;
            live[k] = act[k] = v[k] < d.n;
        }
        if (blk[0] < 0) break;  // the list is exhausted (uniform over the block)
#pragma unroll
        for (int k = 0; k < REP_CH; k++) {
            x[k] = live[k] ? ld_relaxed(&d.rep[v[k]]) : 0;
            lab[k] = live[k] ? d.label[v[k]] : 0;
        }
        int64_t steps = 0;
        for (;; steps++) {
            int32_t y[REP_CH];
#pragma unroll
            for (int k = 0; k < REP_CH; k++) y[k] = act[k] ? ld_relaxed(&d.rep[x[k]]) : x[k];
            bool more = false;
#pragma unroll
            for (int k = 0; k < REP_CH; k++) {
                act[k] = act[k] && y[k] != x[k];
                if (act[k] && steps >= PUBLISH_AFTER) d.rep[v[k]] = y[k];  // progress, for descendants
                x[k] = y[k];
                more |= act[k];
            }
            if (!more) break;
            if (steps > d.n) {
                atomicOr(d.status, ST_WALK_BOUND);
                break;
            }
        }
        // a long chase tells the host that the forest is deep (one store per
        // wave, and only then): its later deletes queue jumping rounds first
        if (__ballot(steps > DEEP_STEPS) != 0 && lane_id() == 0) d.cnt[C_DEEP] = 1;
        bool orphan[REP_CH];
        int32_t t[REP_CH], tk[REP_CH];
        uint32_t us[REP_CH], ls[REP_CH];
        int32_t du[REP_CH], dl[REP_CH];
#pragma unroll
        for (int k = 0; k < REP_CH; k++) {
            orphan[k] = live[k] && x[k] != lab[k];
            if (live[k]) d.rep[v[k]] = x[k];
            const uint64_t word = __ballot(orphan[k]);
            if (lane_id() == 0 && live[k]) d.obits[v[k] >> 6] = word;
            t[k] = tk[k] = NONE;
            us[k] = ls[k] = 0;
            du[k] = dl[k] = 0;
            if (orphan[k]) {
                t[k] = d.tidx[x[k]];
                tk[k] = d.tidx[lab[k]];  // the old root: a piece of its own
                us[k] = d.bptr[v[k]];
                ls[k] = d.lptr[v[k]];
                du[k] = (int32_t)d.bptr[v[k] + 1];
                dl[k] = (int32_t)d.lptr[v[k] + 1];
            }
        }
#pragma unroll
        for (int k = 0; k < REP_CH; k++) {
            if (blk[k] < 0) continue;  // uniform over the block
            if (orphan[k]) {
                if (t[k] < 0 || tk[k] < 0) atomicOr(d.status, ST_WALK_BOUND);
                du[k] -= (int32_t)us[k];
                dl[k] -= (int32_t)ls[k];
            }
            // the block's orphans with their adjacency runs (plus padding)
            // and the block's totals
            unsigned long long tot;
            const unsigned long long off = block_excl_scan64(
                orphan[k] ? opack((unsigned long long)(du[k] + dl[k] + OR_PAD), 1) : 0, &tot);
            if (orphan[k]) {
                OrphEnt o;
                o.pre = (int64_t)ovol(off);
                o.ustart = us[k];
                o.lstart = ls[k];
                o.v = (int32_t)v[k];
                o.du = du[k];
                o.dl = dl[k];
                o.pu = t[k];
                o.ru = x[k];
                o.pk = tk[k];
                d.ostage[blk[k] * BLOCK + (int64_t)ocnt(off)] = o;
            }
            if (threadIdx.x == 0) {
                d.bvol[blk[k]] = (int64_t)ovol(tot);
                d.bcnt[blk[k]] = (int32_t)ocnt(tot);
            }
            // smallest vertex of each orphan piece; consecutive ids often
            // share a piece
            const bool grp = orphan[k] && t[k] >= 0;
            uint64_t rem = __ballot(grp);
            bool pending = grp;
            for (int round = 0; round < GROUP_ROUNDS && rem; round++) {
                const int leader = __ffsll((unsigned long long)rem) - 1;
                const int32_t t0 = __shfl(t[k], leader);
                const bool in = pending && t[k] == t0;
                rem &= ~__ballot(in);
                if (in) pending = false;
                if (lane_id() == leader) min_i32(&d.pmin[t0], (int32_t)v[k]);  // smallest v of the group
            }
            if (pending) min_i32(&d.pmin[t[k]], (int32_t)v[k]);
        }
    }
}

// ------------------------------------------- a5: key-edge sweep (delete)

// Key edges of a delete are all surviving non-tree edges (Sec. II-A); an
// edge is a cross edge iff rep differs at its ends.  An edge whose ends both
// stay in their old root's piece has equal reps (its ends share a component
// of G, hence a tree of F, hence that tree's root piece), so the rep gathers
// are only made when the orphan bitmap flags an end.
//
// One workgroup streams TILE consecutive stored edges.  Each wave reads its
// quarter of the tile with 16-byte non-temporal loads, every instruction
// covering 1 KB of contiguous columns.  The row of each edge comes from a
// map built in LDS: every row starting inside the tile marks its first
// position with its local index, and a max-scan over the tile fills the
// rest; the row vertices sit in LDS beside it.  So the only global gathers
// are the orphan bits of both ends (all of a thread's issued together) and
// rep for the flagged edges.  Cross edges go to the
// tile's own region of x0.
__global__ __launch_bounds__(BLOCK) void k_sweep_base(Dev d) {
    if (stopped(d) || !d.ctl->has_del || d.cnt[C_OMODE]) return;
    typedef int v4i __attribute__((ext_vector_type(4)));
    typedef short v4s __attribute__((ext_vector_type(4)));
    __shared__ v4i s_rowv[TILE / 8];      // int16 local row index per edge
    __shared__ int32_t s_u[TILE + 1];     // row vertex per local row
    __shared__ int16_t s_wmax[BLOCK / WAVE];
    int16_t *s_row = reinterpret_cast<int16_t *>(s_rowv);
    const int64_t ntl_list = d.ctl->ntl;  // read once: stores below may alias it
    for (int64_t jt = blockIdx.x;; jt += gridDim.x) {
        const int64_t tile = list_block(d.tlist, ntl_list, jt, d.ntiles);
        if (tile < 0) break;
        __syncthreads();  // the previous tile is finished with the LDS
        const int64_t base = tile * TILE;
        const int64_t cnt = d.eb - base < TILE ? d.eb - base : TILE;
        const int lane = lane_id(), wid = threadIdx.x / WAVE;
        // thread's edges: local positions pbase + q * 256 + j, q, j < 4
        const int pbase = wid * (TILE / 4) + lane * 4;
        // the store is padded with deleted entries to whole tiles
        int32_t c[EPT];
        {
            const v4i *p = reinterpret_cast<const v4i *>(d.bcol + base + pbase);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const v4i t = __builtin_nontemporal_load(p + q * 64);
                c[4 * q] = t.x; c[4 * q + 1] = t.y; c[4 * q + 2] = t.z; c[4 * q + 3] = t.w;
            }
        }
        // row map: mark row starts
        const v4i zero = {0, 0, 0, 0};
        s_rowv[threadIdx.x] = zero;
        s_rowv[threadIdx.x + BLOCK] = zero;
        __syncthreads();
        // rows in chunks of 4 * BLOCK: all loads of a chunk are issued before use
        const int32_t ka = d.tile_k[tile], kb = d.tile_k[tile + 1];
        for (int32_t k0 = ka; k0 <= kb; k0 += 4 * BLOCK) {
            int32_t zp[4], zr[4];
#pragma unroll
            for (int i = 0; i < 4; i++) {
                int32_t k = k0 + i * BLOCK + (int32_t)threadIdx.x;
                k = k < kb ? k : kb;
                zp[i] = (int32_t)d.zptr[k];
                zr[i] = d.zrow[k];
            }
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int32_t k = k0 + i * BLOCK + (int32_t)threadIdx.x;
                if (k <= kb) {
                    const int64_t p = (int64_t)(uint32_t)zp[i] - base;
                    if (p > 0 && p < cnt) s_row[p] = (int16_t)(k - ka);
                    s_u[k - ka] = zr[i];
                }
            }
        }
        __syncthreads();
        // inclusive max-scan of the marks: thread t owns positions [16 t, 16 t + 16)
        {
            v4s m[4];
            const v4s *src = reinterpret_cast<const v4s *>(s_row + 16 * threadIdx.x);
            int16_t run = 0;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                m[q] = src[q];
                run = m[q].x > run ? m[q].x : run; m[q].x = run;
                run = m[q].y > run ? m[q].y : run; m[q].y = run;
                run = m[q].z > run ? m[q].z : run; m[q].z = run;
                run = m[q].w > run ? m[q].w : run; m[q].w = run;
            }
            int32_t inc = run;
#pragma unroll
            for (int o = 1; o < WAVE; o <<= 1) {
                const int32_t y = __shfl_up(inc, o);
                if (lane >= o && y > inc) inc = y;
            }
            if (lane == WAVE - 1) s_wmax[wid] = (int16_t)inc;
            int32_t before = __shfl_up(inc, 1);
            if (lane == 0) before = 0;
            __syncthreads();
#pragma unroll
            for (int w = 0; w < BLOCK / WAVE; w++)
                if (w < wid && s_wmax[w] > before) before = s_wmax[w];
            const int16_t pre = (int16_t)before;
            v4s *dst = reinterpret_cast<v4s *>(s_row + 16 * threadIdx.x);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                v4s x = m[q];
                x.x = x.x > pre ? x.x : pre; x.y = x.y > pre ? x.y : pre;
                x.z = x.z > pre ? x.z : pre; x.w = x.w > pre ? x.w : pre;
                dst[q] = x;
            }
        }
        __syncthreads();
        // row vertex of each of the thread's edges
        int32_t urow[EPT];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const v4s r = *reinterpret_cast<const v4s *>(s_row + pbase + q * 256);
            urow[4 * q] = s_u[r.x]; urow[4 * q + 1] = s_u[r.y];
            urow[4 * q + 2] = s_u[r.z]; urow[4 * q + 3] = s_u[r.w];
        }
        // every gather of a thread is issued before any result is used: the
        // bitmap words of both ends unconditionally (a deleted entry's masked id
        // is still a vertex; edges of one row share the row's word), then rep
        // only for flagged edges, the others pointed at rep[0]
        uint64_t bu[EPT], bv[EPT];
#pragma unroll
        for (int j = 0; j < EPT; j++) {
            bu[j] = d.obits[urow[j] >> 6];
            bv[j] = d.obits[(c[j] & COLMASK) >> 6];
        }
        uint32_t cand = 0;
#pragma unroll
        for (int j = 0; j < EPT; j++)
            if (c[j] >= 0 && (((bu[j] >> (urow[j] & 63)) | (bv[j] >> (c[j] & 63))) & 1)) cand |= 1u << j;
        int32_t ra[EPT], rb[EPT];
        uint32_t mask = 0;
        if (__ballot(cand != 0)) {
#pragma unroll
            for (int j = 0; j < EPT; j++) {
                const bool k = cand >> j & 1;
                ra[j] = d.rep[k ? urow[j] : 0];
                rb[j] = d.rep[k ? c[j] : 0];
            }
#pragma unroll
            for (int j = 0; j < EPT; j++)
                if ((cand >> j & 1) && ra[j] != rb[j]) mask |= 1u << j;
        }
        int total;
        const int off = block_excl_scan(__popc(mask), &total);
        if (threadIdx.x == 0) d.rcnt[tile] = (unsigned long long)total;
        if (mask) {
            Cross *out = d.x0 + tile * TILE + off;
            int w = 0;
#pragma unroll
            for (int j = 0; j < EPT; j++) {
                if (mask >> j & 1) {
                    Cross x;
                    x.key = ((uint64_t)(uint32_t)urow[j] << 32) | (uint32_t)c[j];
                    x.pa = d.tidx[ra[j]];
                    x.pb = d.tidx[rb[j]];
                    if (x.pa < 0 || x.pb < 0) atomicOr(d.status, ST_WALK_BOUND);
                    out[w++] = x;
                }
            }
        }
    }
}

// The same test over the list of inserted edges: workgroup t takes list
// entries [t * TILE, (t + 1) * TILE) and writes region ntiles + t.  Lane
// layout and gathers as in k_sweep_base.
__global__ __launch_bounds__(BLOCK) void k_sweep_delta(Dev d) {
    if (stopped(d) || !d.ctl->has_del) return;
    const int64_t nd = (int64_t)d.cnt[C_NDELTA];
    const int64_t t = blockIdx.x;
    if (t * TILE >= nd) return;
    const int lane = lane_id(), wid = threadIdx.x / WAVE;
    const int64_t i0 = t * TILE + wid * (TILE / 4) + lane * 4;  // + q * 256 + j
    uint64_t k[EPT];
#pragma unroll
    for (int q = 0; q < 4; q++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int64_t i = i0 + q * 256 + j;
            k[4 * q + j] = i < nd ? d.dkey[i] : KEY_DEAD;
        }
    uint64_t wu[EPT], wv[EPT];
#pragma unroll
    for (int j = 0; j < EPT; j++) {
        const bool live = k[j] != KEY_DEAD;
        wu[j] = d.obits[live ? key_lo(k[j]) >> 6 : 0];
        wv[j] = d.obits[live ? key_hi(k[j]) >> 6 : 0];
    }
    uint32_t cand = 0;
#pragma unroll
    for (int j = 0; j < EPT; j++)
        if (k[j] != KEY_DEAD &&
            (((wu[j] >> (key_lo(k[j]) & 63)) | (wv[j] >> (key_hi(k[j]) & 63))) & 1))
            cand |= 1u << j;
    int32_t ra[EPT], rb[EPT];
    uint32_t mask = 0;
    if (__ballot(cand != 0)) {
#pragma unroll
        for (int j = 0; j < EPT; j++) {
            const bool c = cand >> j & 1;
            ra[j] = d.rep[c ? key_lo(k[j]) : 0];
            rb[j] = d.rep[c ? key_hi(k[j]) : 0];
        }
#pragma unroll
        for (int j = 0; j < EPT; j++)
            if ((cand >> j & 1) && ra[j] != rb[j]) mask |= 1u << j;
    }
    int total;
    const int off = block_excl_scan(__popc(mask), &total);
    const int64_t reg = d.ntiles + t;
    if (threadIdx.x == 0) d.rcnt[reg] = (unsigned long long)total;
    if (mask) {
        Cross *out = d.x0 + reg * TILE + off;
        int w = 0;
#pragma unroll
        for (int j = 0; j < EPT; j++) {
            if (mask >> j & 1) {
                Cross x;
                x.key = k[j];
                x.pa = d.tidx[ra[j]];
                x.pb = d.tidx[rb[j]];
                if (x.pa < 0 || x.pb < 0) atomicOr(d.status, ST_WALK_BOUND);
                out[w++] = x;
            }
        }
    }
}

// ------------------ f4: key-edge scan restricted to the orphans (delete)

// Every cross edge of a delete has an orphan end (ends that both kept their
// old root have equal reps), so scanning the whole adjacency of the orphan
// vertices finds every cross edge of the base store; when the orphans hold
// few slots this replaces the sweep of the whole store.  Root finding left,
// per vertex block, the block's orphans and their slots.  Prefixes over the
// blocks are taken in two levels: within groups of BLOCK blocks here, then
// over the groups in k_orph_total.
__global__ __launch_bounds__(BLOCK) void k_orph_plan(Dev d) {
    if (stopped(d) || !d.ctl->has_del) return;
    const int64_t b = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const unsigned long long x =
        b < d.nvb ? opack((unsigned long long)d.bvol[b], (unsigned long long)d.bcnt[b]) : 0;
    unsigned long long tot;
    const unsigned long long pre = block_excl_scan64(x, &tot);
    if (b < d.nvb) {
        d.bpre[b] = (int64_t)ovol(pre);
        d.opre[b] = (int32_t)ocnt(pre);
    }
    if (threadIdx.x == 0) d.gsum[blockIdx.x] = tot;
}

// Prefix over the groups, the totals and the choice of scan.
__global__ __launch_bounds__(BLOCK) void k_orph_total(Dev d) {
    if (stopped(d) || !d.ctl->has_del) return;
    const int64_t ng = (d.nvb + BLOCK - 1) / BLOCK;
    const int64_t per = (ng + BLOCK - 1) / BLOCK;
    const int64_t g0 = (int64_t)threadIdx.x * per;
    const int64_t g1 = g0 + per < ng ? g0 + per : ng;
    unsigned long long sv = 0, sc = 0;
    for (int64_t g = g0; g < g1; g++) {
        sv += ovol(d.gsum[g]);
        sc += ocnt(d.gsum[g]);
    }
    unsigned long long tv, tc;
    unsigned long long pv = block_excl_scan64(sv, &tv);
    unsigned long long pc = block_excl_scan64(sc, &tc);
    for (int64_t g = g0; g < g1; g++) {
        d.gpre[g] = (int64_t)pv;
        d.gopre[g] = (int64_t)pc;
        pv += ovol(d.gsum[g]);
        pc += ocnt(d.gsum[g]);
    }
    if (threadIdx.x == 0) {
        const int64_t V = (int64_t)tv;
        d.cnt[C_OVOL] = (unsigned long long)V;
        d.cnt[C_NORPH] = tc;
        d.cnt[C_OMODE] = (d.ctl->smode != 1 && V <= d.eb) ? 1ull : 0ull;
    }
}

// Compacted list of all orphans in vertex order (copied from the blocks'
// staging with global prefixes), each orphan's piece in owner[], and for
// each range of OR_W slots the list index of the orphan holding its first
// slot.
__global__ __launch_bounds__(BLOCK) void k_orph_fill(Dev d) {
    if (stopped(d) || !d.ctl->has_del || !d.cnt[C_OMODE]) return;
    // FILL_LANES lanes per vertex block (blocks hold few orphans), so one
    // wave covers WAVE / FILL_LANES blocks with all its loads in flight
    constexpr int FILL_LANES = 8;
    const int64_t per_block = BLOCK / FILL_LANES;
    const int sub = threadIdx.x % FILL_LANES;
    const int64_t nvl_list = d.ctl->nvl;  // read once: stores below may alias it
    for (int64_t j = (int64_t)blockIdx.x * per_block + threadIdx.x / FILL_LANES;;
         j += (int64_t)gridDim.x * per_block) {
        const int64_t blk = list_block(d.vlist, nvl_list, j, d.nvb);
        if (blk < 0) break;
        const int32_t nc = d.bcnt[blk];
        if (nc == 0) continue;
        const int64_t ob = d.gopre[blk / BLOCK] + d.opre[blk];
        const int64_t vb = d.gpre[blk / BLOCK] + d.bpre[blk];
        for (int32_t i = sub; i < nc; i += FILL_LANES) {
            OrphEnt o = d.ostage[blk * BLOCK + i];
            const int64_t idx = ob + i;
            o.pre += vb;
            d.olist[idx] = o;
            d.owner[o.v] = o.pu;  // the orphan's piece, for the orphan scan
            const int64_t end = o.pre + o.du + o.dl + OR_PAD;
            for (int64_t w = (o.pre + OR_W - 1) / OR_W; w * OR_W < end; w++) d.rstart[w] = (int32_t)idx;
        }
    }
}

// One workgroup per region of x0: one range of OR_W consecutive slots, or
// two when the orphans hold more than half as many slots as the base store.
// For each range, the orphans covering it are staged in LDS; each thread
// takes OR_K consecutive slots (one binary search, then a walk), loads their
// columns from the upper or lower run and tests the neighbour.  A neighbour
// that is no orphan kept its old root, which is not the orphan's piece
// root: the edge is a cross edge to the old root's piece (known per
// orphan), so only orphan neighbours need their piece gathered, one load
// from owner[], where the list fill left each orphan's piece (the orphan
// bitmap, one bit per vertex, mostly stays in L2; owner[] does not).  Two
// ends are in one piece iff their piece ids are equal.  Parallel edges
// between two pieces close a cycle with the lowest of them, on which they
// are the largest, so the lowest-key forest holds none of them: the
// old-root edges of an orphan in a range are kept
// as their lowest key alone, and the orphan-neighbour edges as the lowest
// key of each run of equal piece pairs within a thread's slots.  Every cross
// edge (u, v) also takes part in the first hooking round's selection for
// u's piece (an orphan piece, which never holds an old root); edges between
// two orphan pieces are seen from both ends and counted once (from the
// smaller end).
__global__ __launch_bounds__(BLOCK) void k_orph_scan(Dev d) {
    if (stopped(d) || !d.ctl->has_del || !d.cnt[C_OMODE]) return;
    const int64_t V = (int64_t)d.cnt[C_OVOL];
    const int64_t no = (int64_t)d.cnt[C_NORPH];
    const int64_t per = or_region_slots(V, d.eb) / OR_W;  // ranges per region
    const int64_t nreg = or_regions(V, d.eb);
    __shared__ OrphEnt s_o[BLOCK];
    __shared__ int64_t s_pre[BLOCK];
    __shared__ unsigned long long s_min[BLOCK];   // lowest cross key per staged orphan
    __shared__ unsigned long long s_mink[BLOCK];  // lowest key to the old root's piece
    for (int64_t w = blockIdx.x; w < nreg; w += gridDim.x) {
        Cross *const region = d.x0 + w * TILE;
        int64_t emitted = 0;
        int ncross = 0;
        for (int64_t rg = w * per; rg < (w + 1) * per && rg * OR_W < V; rg++) {  // uniform
            const int64_t S1 = (rg + 1) * OR_W < V ? (rg + 1) * OR_W : V;
            int64_t pos = rg * OR_W;
            int64_t i0 = d.rstart[rg];
            // the last orphan that meets this range: the one holding the next
            // range's first slot (a hub alone covers whole ranges)
            const int64_t ilast = S1 < V ? d.rstart[rg + 1] : no - 1;
            while (pos < S1) {  // windows of BLOCK orphans; uniform over the block
                const int64_t lim = ilast - i0 + 1;
                const int wn = lim < BLOCK ? (int)lim : BLOCK;
                __syncthreads();  // the LDS is free
                if (threadIdx.x < wn) {
                    s_o[threadIdx.x] = d.olist[i0 + threadIdx.x];
                    s_pre[threadIdx.x] = s_o[threadIdx.x].pre;
                }
                s_min[threadIdx.x] = KEY_INF;
                s_mink[threadIdx.x] = KEY_INF;
                __syncthreads();
                int64_t we = S1;
                if (wn > 0) {
                    const OrphEnt &last = s_o[wn - 1];
                    const int64_t e = last.pre + last.du + last.dl + OR_PAD;
                    we = e < S1 ? e : S1;
                }
                if (wn <= 0 || we <= pos || s_pre[0] > pos) {  // inconsistent plan
                    if (threadIdx.x == 0) atomicOr(d.status, ST_WALK_BOUND);
                    break;
                }
                // this thread's slots [s0, s0 + cnt)
                const int64_t s0 = pos + (int64_t)threadIdx.x * OR_K;
                const int cnt = s0 >= we ? 0 : (we - s0 < OR_K ? (int)(we - s0) : OR_K);
                int a = 0;
                if (cnt > 0) {
                    int b = wn - 1;
                    while (a < b) {
                        const int mid = (a + b + 1) >> 1;
                        if (s_pre[mid] <= s0) a = mid; else b = mid - 1;
                    }
                }
                int64_t e = cnt > 0 ? s0 - s_pre[a] : 0;
                int32_t col[OR_K], oi[OR_K];
#pragma unroll
                for (int k = 0; k < OR_K; k++) {
                    const int32_t *src = d.bcol;
                    bool real = false;
                    if (k < cnt) {
                        while (e >= (int64_t)s_o[a].du + s_o[a].dl + OR_PAD && a < wn - 1) {
                            e -= (int64_t)s_o[a].du + s_o[a].dl + OR_PAD;
                            a++;
                        }
                        const OrphEnt &o = s_o[a];
                        real = e < (int64_t)o.du + o.dl;  // else a padding slot
                        if (real) src = e < o.du ? d.bcol + o.ustart + e : d.lcol + o.lstart + (e - o.du);
                        e++;
                    }
                    oi[k] = a;
                    col[k] = *src;
                    if (!real) col[k] = TOMB;
                }
                uint64_t vw[OR_K];
#pragma unroll
                for (int k = 0; k < OR_K; k++) vw[k] = d.obits[(col[k] & COLMASK) >> 6];
                uint32_t onb = 0;  // the neighbour is an orphan
#pragma unroll
                for (int k = 0; k < OR_K; k++)
                    if (col[k] >= 0 && ((vw[k] >> (col[k] & 63)) & 1)) onb |= 1u << k;
                // the neighbour's piece: an orphan's from owner[] (one
                // gather), else the old root's
                int32_t pv[OR_K];
#pragma unroll
                for (int k = 0; k < OR_K; k++) pv[k] = (onb >> k & 1) ? d.owner[col[k]] : s_o[oi[k]].pk;
                uint32_t cross = 0;
#pragma unroll
                for (int k = 0; k < OR_K; k++)
                    if (col[k] >= 0 && (!(onb >> k & 1) || pv[k] != s_o[oi[k]].pu)) cross |= 1u << k;
                const uint32_t xo = cross & onb, xk = cross & ~onb;  // to orphans / to old roots
                // count, and the runs of equal piece pairs among the edges to orphans
                int runs = 0;
                {
                    uint64_t cur = ~0ull;
#pragma unroll
                    for (int k = 0; k < OR_K; k++) {
                        if (!(cross >> k & 1)) continue;
                        const OrphEnt &o = s_o[oi[k]];
                        if (pv[k] < 0 || o.pu < 0) atomicOr(d.status, ST_WALK_BOUND);
                        if (!(onb >> k & 1) || o.v < col[k]) ncross++;
                        if (!(xo >> k & 1)) continue;
                        const uint64_t pair = ((uint64_t)(uint32_t)o.pu << 32) | (uint32_t)pv[k];
                        if (pair != cur) { runs++; cur = pair; }
                    }
                }
                // edges to old roots: the lowest key per orphan (a thread's
                // slots meet few orphans, one LDS minimum per orphan met; the
                // last one met is merged across the wave when every lane
                // ends on the same orphan, as in a hub's ranges)
                {
                    int32_t ca = -1;
                    uint64_t mk = ~0ull;
#pragma unroll
                    for (int k = 0; k < OR_K; k++) {
                        if (!(xk >> k & 1)) continue;
                        const uint64_t key = mkkey((uint32_t)s_o[oi[k]].v, (uint32_t)col[k]);
                        if (oi[k] == ca) {
                            mk = key < mk ? key : mk;
                            continue;
                        }
                        if (ca >= 0 && s_mink[ca] > mk) atomicMin(&s_mink[ca], (unsigned long long)mk);
                        ca = oi[k];
                        mk = key;
                    }
                    const bool has = ca >= 0;
                    const uint64_t hm = __ballot(has);
                    if (hm) {
                        const int leader = __ffsll((unsigned long long)hm) - 1;
                        const int32_t c0 = __shfl(ca, leader);
                        if (__ballot(has && ca == c0) == hm) {
                            uint64_t v = has ? mk : ~0ull;
                            for (int o = WAVE / 2; o > 0; o >>= 1) {
                                const uint64_t y = __shfl_xor(v, o);
                                v = y < v ? y : v;
                            }
                            if (lane_id() == leader && s_mink[c0] > v) atomicMin(&s_mink[c0], (unsigned long long)v);
                        } else if (has && s_mink[ca] > mk) {
                            atomicMin(&s_mink[ca], (unsigned long long)mk);
                        }
                    }
                }
                int rtot;
                const int roff = block_excl_scan(runs, &rtot);
                // lowest key of each run: output, and the run's orphan's
                // minimum in LDS (several threads' runs of one orphan meet
                // there; one global atomic per orphan and window follows)
                {
                    Cross *out = region + emitted + roff;
                    int r = 0;
                    uint64_t cur = ~0ull, mk = 0;
                    int32_t cpu = 0, cpv = 0, ca = 0;
#pragma unroll
                    for (int k = 0; k <= OR_K; k++) {
                        bool flush = k == OR_K;
                        uint64_t pair = 0, key = 0;
                        if (!flush && (xo >> k & 1)) {
                            const OrphEnt &o = s_o[oi[k]];
                            pair = ((uint64_t)(uint32_t)o.pu << 32) | (uint32_t)pv[k];
                            key = mkkey((uint32_t)o.v, (uint32_t)col[k]);
                            if (pair == cur) {
                                mk = key < mk ? key : mk;
                                continue;
                            }
                            flush = true;
                        } else if (!flush) {
                            continue;
                        }
                        if (cur != ~0ull) {
                            Cross x;
                            x.key = mk;
                            x.pa = cpu;
                            x.pb = cpv;
                            out[r++] = x;
                            if (s_min[ca] > mk) atomicMin(&s_min[ca], (unsigned long long)mk);
                        }
                        if (k < OR_K) {
                            cur = pair;
                            mk = key;
                            cpu = (int32_t)(pair >> 32);
                            cpv = (int32_t)(uint32_t)pair;
                            ca = oi[k];
                        }
                    }
                }
                __syncthreads();
                // per staged orphan: its edge to the old root's piece, and its
                // lowest cross key into the first round's selection
                bool ek = false;
                Cross xk1;
                xk1.key = 0;
                xk1.pa = xk1.pb = 0;
                if (threadIdx.x < wn) {
                    const unsigned long long mkk = s_mink[threadIdx.x];
                    const unsigned long long mo = s_min[threadIdx.x];
                    const unsigned long long m = mkk < mo ? mkk : mo;
                    const OrphEnt &o = s_o[threadIdx.x];
                    if (m != KEY_INF && o.pu >= 0 && d.best[o.pu] > m)
                        atomicMin((unsigned long long *)&d.best[o.pu], m);
                    ek = mkk != KEY_INF;
                    xk1.key = mkk;
                    xk1.pa = o.pu;
                    xk1.pb = o.pk;
                }
                int ktot;
                const int koff = block_excl_scan(ek ? 1 : 0, &ktot);
                if (ek) region[emitted + rtot + koff] = xk1;
                emitted += rtot + ktot;
                pos = we;
                i0 += wn;
            }
        }
        int ct;
        block_excl_scan(ncross, &ct);
        if (threadIdx.x == 0) {
            d.rcnt[w] = (unsigned long long)emitted;
            d.xcnt[w] = (unsigned long long)ct;
        }
    }
}

// ------------------------------- a6: replacement edges by hooking rounds

// Hooks.  A component hooks at most once per update, so hook[] is written
// once per component and tagged with its round; the components are never
// compressed between rounds.  The root of x's component at the start of
// round r follows the hooks made before round r (a round's own hooks, being
// written meanwhile, are skipped by their tag).
__device__ __forceinline__ uint64_t hook_pack(int r, int32_t other) {
    return ((uint64_t)(uint32_t)r << 32) | (uint32_t)other;
}
__device__ int32_t comp_root(const Dev &d, int32_t x, uint32_t r, int64_t np) {
    for (int64_t steps = 0;; steps++) {
        const uint64_t h = d.hook[x];
        if ((uint32_t)(h >> 32) >= r) return x;  // a root then (HOOK_NONE has the largest tag)
        x = (int32_t)(uint32_t)h;
        if (steps > np) {
            atomicOr(d.status, ST_WALK_BOUND);
            return x;
        }
    }
}
// the buffer of best[] that round r selects into
__device__ __forceinline__ uint64_t *best_of(const Dev &d, int r) { return d.best + (r & 1) * d.pcap; }

// A component selects the lowest key among the cross edges it touches.  In a
// delete, a component that holds an old root piece never selects: every cross
// edge lies inside one old component, whose root piece is unique, so every
// live edge touches a component without one, which selects; each selected
// edge is the lowest key leaving its component (cut property), so the
// chosen set is still the Kruskal one.
__device__ __forceinline__ void select_edge(const Dev &d, bool live, const Cross &e, int32_t ca,
                                            int32_t cb, uint64_t *best) {
    const bool sa = live && !d.pkeep[ca], sb = live && !d.pkeep[cb];
    group_min_u64(sa, ca, e.key, best);
    group_min_u64(sb, cb, e.key, best);
}

// Round 0: every cross edge is live and every component is a single piece.
// Workgroups take the regions [rlo, rhi) of x0 in turn.  With emit, the
// insert regions are not filled yet: a workgroup taking one runs the insert
// emit for its batch entries (writing the region for the next round) and
// selects on the edges it found, and adds its count to the statistic.
// Workgroup 0 sums the other region lengths (the cross edges found).
__global__ __launch_bounds__(BLOCK) void k_bor_round0(Dev d, int emit) {
    if (stopped(d)) return;
    // regions below ntiles hold the orphan scan's output when it ran: those
    // edges took part in this round's selection already
    const bool om = d.cnt[C_OMODE] != 0;
    const int64_t rhi = d.ctl->rhi;
    const int64_t rlo = om ? (d.ctl->rlo > d.ntiles ? d.ctl->rlo : d.ntiles) : d.ctl->rlo;
    const bool ins_here = emit && d.ctl->has_ins;
    const int64_t ib = d.ctl->ibase, ie = ins_here ? ib + (d.ctl->b + BLOCK - 1) / BLOCK : ib;
    for (int64_t t = rlo + blockIdx.x; t < rhi; t += gridDim.x) {
        if (t >= ib && t < ie) {  // uniform over the workgroup
            Cross e;
            int total;
            const bool live = insert_emit_block(d, t - ib, &e, &total);
            select_edge(d, live, e, e.pa, e.pb, d.best);
            if (threadIdx.x == 0 && total) atomicAdd(&d.cnt[C_NCROSS], (unsigned long long)total);
            continue;
        }
        const int64_t cntr = (int64_t)d.rcnt[t];
        const Cross *in = d.x0 + t * TILE;
        for (int64_t base = 0; base < cntr; base += BLOCK) {
            const int64_t i = base + threadIdx.x;
            const bool live = i < cntr;
            Cross e;
            e.pa = e.pb = 0;
            e.key = 0;
            if (live) e = in[i];
            select_edge(d, live, e, e.pa, e.pb, d.best);
        }
    }
    if (blockIdx.x == 0) {
        unsigned long long s = 0;
        for (int64_t r = rlo + threadIdx.x; r < rhi; r += BLOCK)
            if (r < ib || r >= ie) s += d.rcnt[r];
        if (om) {
            const int64_t nr = or_regions((int64_t)d.cnt[C_OVOL], d.eb);
            for (int64_t r = threadIdx.x; r < nr; r += BLOCK) s += d.xcnt[r];
        }
        for (int o = WAVE / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
        if (lane_id() == 0 && s) atomicAdd(&d.cnt[C_NCROSS], s);
    }
}

// Round r >= 1: drop cross edges now inside one component, select again, and
// compact the survivors into a dense list.  Round 1 reads the regions of x0;
// later rounds alternate dense lists (out: x1 on odd rounds, x0 on even).
__global__ __launch_bounds__(BLOCK) void k_bor_select(Dev d, int r) {
    if (stopped(d) || d.cnt[C_DONE_BOR]) return;
    Cross *out = (r & 1) ? d.x1 : d.x0;
    unsigned long long *cout = &d.cnt[(r & 1) ? C_NX1 : C_NX0];
    const int64_t np = (int64_t)d.cnt[C_NP];
    uint64_t *best = best_of(d, r);
    __shared__ unsigned long long obase;
    // work units: regions of x0 (round 1) or BLOCK-sized chunks of a dense list
    int64_t u0, u1;
    const Cross *dense = (r & 1) ? d.x0 : d.x1;
    int64_t dcount = 0;
    if (r == 1) {
        u0 = d.ctl->rlo;
        u1 = d.ctl->rhi;
    } else {
        dcount = (int64_t)d.cnt[(r & 1) ? C_NX0 : C_NX1];
        u0 = 0;
        u1 = (dcount + BLOCK - 1) / BLOCK;
    }
    for (int64_t unit = u0 + blockIdx.x; unit < u1; unit += gridDim.x) {
        const Cross *in;
        int64_t count;
        if (r == 1) {
            in = d.x0 + unit * TILE;
            count = (int64_t)d.rcnt[unit];
        } else {
            in = dense + unit * BLOCK;
            count = dcount - unit * BLOCK < BLOCK ? dcount - unit * BLOCK : BLOCK;
        }
        for (int64_t base = 0; base < count; base += BLOCK) {
            const int64_t i = base + threadIdx.x;
            bool live = false;
            Cross e;
            e.key = 0;
            e.pa = e.pb = 0;
            int32_t ca = 0, cb = 0;
            if (i < count) {
                e = in[i];  // ends: pieces (round 1) or components at the last round's start
                ca = comp_root(d, e.pa, (uint32_t)r, np);
                cb = comp_root(d, e.pb, (uint32_t)r, np);
                live = ca != cb;
            }
            select_edge(d, live, e, ca, cb, best);
            e.pa = ca;
            e.pb = cb;
            int total;
            const int off = block_excl_scan(live ? 1 : 0, &total);
            if (threadIdx.x == 0) obase = total ? atomicAdd(cout, (unsigned long long)total) : 0ull;
            __syncthreads();
            if (live) out[obase + off] = e;
            __syncthreads();
        }
    }
}

// Each selecting component hooks onto the component across its lowest-key
// edge; when two components pick the same edge the smaller id stays a root.
// Distinct keys make the chosen edges a forest (Boruvka).  Round r >= 1 ends
// the rounds when its select found no live edge.  Also clears the other
// buffer of best[] for the next round's selection.
__global__ __launch_bounds__(BLOCK) void k_bor_hook(Dev d, int r) {
    if (stopped(d) || d.cnt[C_DONE_BOR]) return;
    if (r >= 1) {
        const int64_t nout = (int64_t)d.cnt[(r & 1) ? C_NX1 : C_NX0];
        if (nout == 0) {
            if (blockIdx.x == 0 && threadIdx.x == 0) d.cnt[C_DONE_BOR] = 1;
            return;
        }
        if (r >= 2 && blockIdx.x == 0 && threadIdx.x == 0) d.cnt[(r & 1) ? C_NX0 : C_NX1] = 0;
    }
    const int64_t np = (int64_t)d.cnt[C_NP];
    const uint64_t *best = best_of(d, r);
    uint64_t *next = best_of(d, r + 1);
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < np; base += stride) {
        const int64_t p = base + threadIdx.x;
        bool rec = false;
        int4 er = make_int4(0, 0, 0, 0);
        if (p < np) {
            next[p] = KEY_INF;
            // a root at this round's start (only p's own thread writes hook[p])
            const uint64_t k = d.hook[p] == HOOK_NONE ? best[p] : KEY_INF;
            if (k != KEY_INF) {
                const int32_t x = key_lo(k), y = key_hi(k);
                const int32_t px = d.tidx[d.rep[x]], py = d.tidx[d.rep[y]];
                if (px < 0 || py < 0) {
                    atomicOr(d.status, ST_WALK_BOUND);
                } else {
                    const int32_t cx = comp_root(d, px, (uint32_t)r, np);
                    const int32_t cy = comp_root(d, py, (uint32_t)r, np);
                    const int32_t other = (cx == (int32_t)p) ? cy : cx;
                    if (!(best[other] == k && (int32_t)p < other)) {
                        d.hook[p] = hook_pack(r, other);
                        rec = true;
                        er = make_int4(x, y, px, py);
                    }
                }
            }
        }
        const int64_t slot = block_append(rec ? 1 : 0, &d.cnt[C_NER]);
        if (rec) d.er[slot] = er;
    }
}

// The rounds from r0 on in one workgroup, once few cross edges are live: a
// round costs three block barriers instead of two launches (each launch on
// this part costs a few microseconds however little it does).  Each round
// selects as k_bor_select does, then hooks from the edges: a component that
// selected hooks from the live edge holding its key, by the same rule as
// k_bor_hook (a list can hold an edge twice, so the hook is a
// compare-and-swap from "none" and only its winner records the edge).  The
// next round's best[] entries are cleared for the ends of this round's live
// edges, which include every component a later round can reach.  A list
// longer than TAIL_MAX leaves everything untouched (the full-grid rounds
// then go on).  Within one workgroup a barrier makes earlier global writes
// and atomics visible to every thread of it.
__global__ __launch_bounds__(TAIL_THREADS) void k_bor_tail(Dev d, int r0) {
    if (stopped(d) || d.cnt[C_DONE_BOR]) return;
    int64_t cin = (int64_t)d.cnt[(r0 & 1) ? C_NX0 : C_NX1];
    if (cin > TAIL_MAX) return;
    __shared__ int s_nout;
    const int64_t np = (int64_t)d.cnt[C_NP];
    for (int r = r0;; r++) {
        if (r >= MAX_ROUNDS) {
            if (threadIdx.x == 0) atomicOr(d.status, ST_ROUND_BOUND);
            return;
        }
        const Cross *in = (r & 1) ? d.x0 : d.x1;
        Cross *out = (r & 1) ? d.x1 : d.x0;
        uint64_t *best = best_of(d, r), *nbest = best_of(d, r + 1);
        if (threadIdx.x == 0) s_nout = 0;
        __syncthreads();
        for (int64_t base = 0; base < cin; base += TAIL_THREADS) {
            const int64_t i = base + threadIdx.x;
            bool live = false;
            Cross e;
            e.key = 0;
            e.pa = e.pb = 0;
            int32_t ca = 0, cb = 0;
            if (i < cin) {
                e = in[i];
                ca = comp_root(d, e.pa, (uint32_t)r, np);
                cb = comp_root(d, e.pb, (uint32_t)r, np);
                live = ca != cb;
            }
            select_edge(d, live, e, ca, cb, best);
            const uint64_t m = __ballot(live);
            if (m) {
                const int leader = __ffsll((unsigned long long)m) - 1;
                int wb = 0;
                if (lane_id() == leader) wb = atomicAdd(&s_nout, __popcll(m));
                wb = __shfl(wb, leader);
                if (live) {
                    e.pa = ca;
                    e.pb = cb;
                    out[wb + lanes_below(m)] = e;
                }
            }
        }
        __syncthreads();
        const int64_t nout = s_nout;
        if (nout == 0) {
            if (threadIdx.x == 0) d.cnt[C_DONE_BOR] = 1;
            return;
        }
        for (int64_t base = 0; base < nout; base += TAIL_THREADS) {
            const int64_t i = base + threadIdx.x;
            bool rec[2] = {false, false};
            int4 er[2] = {make_int4(0, 0, 0, 0), make_int4(0, 0, 0, 0)};
            if (i < nout) {
                const Cross e = out[i];
                nbest[e.pa] = KEY_INF;
                nbest[e.pb] = KEY_INF;
                for (int side = 0; side < 2; side++) {
                    const int32_t p = side ? e.pb : e.pa, other = side ? e.pa : e.pb;
                    if (best[p] != e.key) continue;
                    const int32_t x = key_lo(e.key), y = key_hi(e.key);
                    const int32_t px = d.tidx[d.rep[x]], py = d.tidx[d.rep[y]];
                    if (px < 0 || py < 0) {
                        atomicOr(d.status, ST_WALK_BOUND);
                        continue;
                    }
                    if (best[other] == e.key && p < other) continue;  // both chose it: the smaller stays
                    if (atomicCAS((unsigned long long *)&d.hook[p], (unsigned long long)HOOK_NONE,
                                  (unsigned long long)hook_pack(r, other)) == HOOK_NONE) {
                        rec[side] = true;
                        er[side] = make_int4(x, y, px, py);
                    }
                }
            }
            for (int side = 0; side < 2; side++) {
                const int64_t slot = wave_append(rec[side], &d.cnt[C_NER]);
                if (rec[side]) d.er[slot] = er[side];
            }
        }
        __syncthreads();
        cin = nout;
    }
}

// ------------------------------------------- a7: super-forest rooting

// Super-root of each merged component: the piece holding its smallest
// vertex (insert: the tree with the smallest root; delete: the piece that
// kept the old root when present, since that root is the component's
// minimum).  Runs only once the hooking rounds have finished.
__global__ __launch_bounds__(BLOCK) void k_sf_root(Dev d) {
    if (stopped(d) || !d.cnt[C_DONE_BOR]) return;
    const int64_t np = (int64_t)d.cnt[C_NP];
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < np; base += stride) {
        const int64_t p = base + threadIdx.x;
        const bool act = p < np;
        // the final component: every hook of every round
        const int32_t c = act ? comp_root(d, (int32_t)p, ~0u, np) : 0;
        if (act) d.comp[p] = c;
        const uint64_t key = act ? (((uint64_t)(uint32_t)d.pmin[p] << 32) | (uint64_t)p) : KEY_INF;
        group_min_u64(act, c, key, d.srkey);
    }
}

// The super-root piece of p's component (after k_sf_root).
__device__ __forceinline__ bool is_super_root(const Dev &d, int32_t p) {
    return (int32_t)(uint32_t)d.srkey[d.comp[p]] == p;
}

// arc i*2 goes from the piece of x to the piece of y, i*2+1 back.  In a tree
// every piece has exactly one neighbour on the previous level, so each
// piece's level and parent arc have a single writer.  A level that reaches no
// new piece ends the search.
__global__ __launch_bounds__(BLOCK) void k_sf_bfs(Dev d, int L) {
    if (stopped(d) || !d.cnt[C_DONE_BOR]) return;
    if (L > 0 && d.cnt[C_BFS_ROUND + L - 1] == 0) return;
    const int64_t na = 2 * (int64_t)d.cnt[C_NER];
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    bool active = false;
    // every level starts at -1 (cleanup of the previous update); level 0 is
    // the super-roots, recognised here and marked on the first level
    for (int64_t a = (int64_t)blockIdx.x * BLOCK + threadIdx.x; a < na; a += stride) {
        const int4 e = d.er[a >> 1];
        const int32_t src = (a & 1) ? e.w : e.z, dst = (a & 1) ? e.z : e.w;
        bool from;
        if (L == 0) {
            from = is_super_root(d, src);
            if (from) d.level[src] = 0;  // same value from every arc of src
        } else {
            from = d.level[src] == L;
        }
        // a super-root's neighbours are on level 1, so level 0 reaches no
        // super-root; later levels never see one at -1 (marked on level 0)
        if (from && d.level[dst] < 0) {
            d.level[dst] = L + 1;
            d.parc[dst] = (int32_t)a;
            active = true;
        }
    }
    if (__ballot(active) && lane_id() == 0) d.cnt[C_BFS_ROUND + L] = 1;
}

// Orientation from the search, once the rounds have finished and the last
// queued level reached nothing new: a piece reached through arc a (from the
// parent piece) reverses the path from a's endpoint in the piece to the
// piece's root and hangs that endpoint below a's other endpoint (Algorithm 1,
// R and new parents).  A super-root piece whose root is not the component's
// smallest vertex m is re-rooted at m; m is the component's new label.
__global__ __launch_bounds__(BLOCK) void k_orient_bfs(Dev d, int levels) {
    if (stopped(d) || !d.cnt[C_DONE_BOR] || d.cnt[C_BFS_ROUND + levels - 1] != 0) return;
    const int64_t np = (int64_t)d.cnt[C_NP];
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    if (blockIdx.x == 0 && threadIdx.x == 0) d.cnt[C_ORIENTED] = 1;
    for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < np; base += stride) {
        const int64_t p = base + threadIdx.x;
        bool e1 = false, e2 = false;
        PathReq q1, q2;
        q1.start = q1.newpar = q1.stop = q1.pad = 0;
        q2 = q1;
        if (p < np) {
            const int32_t a = d.parc[p];
            if (a >= 0) {
                const int4 e = d.er[a >> 1];
                e1 = true;
                if ((a & 1) == 0) { q1.start = e.y; q1.newpar = e.x; q1.stop = d.prt[e.w]; }
                else { q1.start = e.x; q1.newpar = e.y; q1.stop = d.prt[e.z]; }
            } else if (d.level[p] < 0 && !is_super_root(d, (int32_t)p)) {
                atomicOr(d.status, ST_ROUND_BOUND);  // piece not reached: search incomplete
            }
            if (d.comp[p] == (int32_t)p) {
                const uint64_t sk = d.srkey[p];
                const int32_t S = (int32_t)(uint32_t)sk, m = (int32_t)(sk >> 32);
                d.newlab[p] = m;
                if (m != d.prt[S]) {
                    e2 = true;
                    q2.start = m; q2.newpar = m; q2.stop = d.prt[S];
                }
            }
        }
        const int64_t s1 = block_append((e1 ? 1 : 0) + (e2 ? 1 : 0), &d.cnt[C_NR]);
        const int64_t s2 = s1 + (e1 ? 1 : 0);
        if (e1) { if (s1 < d.pathcap) d.paths[s1] = q1; else atomicOr(d.status, ST_CAPACITY); }
        if (e2) { if (s2 < d.pathcap) d.paths[s2] = q2; else atomicOr(d.status, ST_CAPACITY); }
    }
}

// Fallback for deep super-trees: Euler tour of the super-forest and list
// ranking (Alg. 2, Eulerian tour step).  It runs only when the hooking
// rounds have finished and the search's last level (levels - 1) was still
// active (the search did not orient the pieces); the flags it tests do not
// change while it runs, so it can be queued after the search and skips
// itself when the search sufficed.
__device__ __forceinline__ bool tour_needed(const Dev &d, int levels) {
    return d.cnt[C_DONE_BOR] && d.cnt[C_BFS_ROUND + levels - 1] != 0;
}
// Arc lists per piece:
__global__ __launch_bounds__(BLOCK) void k_sf_arcs(Dev d, int levels) {
    if (stopped(d) || !tour_needed(d, levels)) return;
    const int64_t ner = (int64_t)d.cnt[C_NER];
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < ner; base += stride) {
        const int64_t i = base + threadIdx.x;
        const bool act = i < ner;
        int4 e = make_int4(0, 0, 0, 0);
        if (act) e = d.er[i];
        group_push(act, e.z, (int32_t)(2 * i), d.head, d.arc_nxt);
        group_push(act, e.w, (int32_t)(2 * i + 1), d.head, d.arc_nxt);
    }
}

// Euler tour successor: after arc P->Q comes the arc following Q->P in Q's
// cyclic arc list.  The tour of each component is cut open at its super-root.
__global__ __launch_bounds__(BLOCK) void k_sf_succ(Dev d, int levels) {
    if (stopped(d) || !tour_needed(d, levels)) return;
    const int64_t na = 2 * (int64_t)d.cnt[C_NER];
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t a = (int64_t)blockIdx.x * BLOCK + threadIdx.x; a < na; a += stride) {
        const int4 e = d.er[a >> 1];
        const int32_t q = (a & 1) ? e.z : e.w;  // target piece of arc a
        int32_t s = d.arc_nxt[a ^ 1];
        const int32_t hq = d.head[q];
        if (s == NONE) s = hq;
        const int32_t S = (int32_t)(uint32_t)d.srkey[d.comp[q]];
        if (q == S && s == hq) s = NONE;
        d.succ0[a] = s;
        d.rank0[a] = s == NONE ? 0 : 1;
    }
}

// List ranking by pointer jumping (Wyllie): rank = arcs left until the end
// of the tour.  Double-buffered; round r reads buffer r&1.
__global__ __launch_bounds__(BLOCK) void k_lr_round(Dev d, int r, int levels) {
    if (stopped(d) || d.cnt[C_DONE_LR] || !tour_needed(d, levels)) return;
    if (r > 0 && d.cnt[C_LR_ROUND + r - 1] == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            d.cnt[C_LR_FINAL] = (unsigned long long)(r & 1);
            d.cnt[C_DONE_LR] = 1;
        }
        return;
    }
    const int32_t *si = (r & 1) ? d.succ1 : d.succ0;
    const int32_t *ri = (r & 1) ? d.rank1 : d.rank0;
    int32_t *so = (r & 1) ? d.succ0 : d.succ1;
    int32_t *ro = (r & 1) ? d.rank0 : d.rank1;
    const int64_t na = 2 * (int64_t)d.cnt[C_NER];
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    bool active = false;
    for (int64_t a = (int64_t)blockIdx.x * BLOCK + threadIdx.x; a < na; a += stride) {
        const int32_t s = si[a];
        if (s != NONE) {
            const int32_t s2 = si[s];
            ro[a] = ri[a] + ri[s];
            so[a] = s2;
            active |= s2 != NONE;
        } else {
            ro[a] = ri[a];
            so[a] = NONE;
        }
    }
    if (__ballot(active) && lane_id() == 0) d.cnt[C_LR_ROUND + r] = 1;
}

// Orientation from the tour: of the two arcs of a replacement edge the one
// met first (larger rank) points from parent piece to child piece; the rest
// as in k_orient_bfs.
__global__ __launch_bounds__(BLOCK) void k_orient_lr(Dev d, int lr_rounds, int levels) {
    if (stopped(d) || !tour_needed(d, levels)) return;
    const int64_t ner = (int64_t)d.cnt[C_NER];
    const int64_t np = (int64_t)d.cnt[C_NP];
    int fin;
    if (d.cnt[C_DONE_LR]) {
        fin = (int)d.cnt[C_LR_FINAL];
    } else {
        if (ner > 0 && d.cnt[C_LR_ROUND + lr_rounds - 1] != 0) {
            if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(d.status, ST_ROUND_BOUND);
            return;
        }
        fin = lr_rounds & 1;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) d.cnt[C_ORIENTED] = 1;
    const int32_t *rk = fin ? d.rank1 : d.rank0;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    const int64_t total = ner + np;
    for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < total; base += stride) {
        const int64_t t = base + threadIdx.x;
        bool emit = false;
        PathReq q;
        q.start = q.newpar = q.stop = q.pad = 0;
        if (t < ner) {
            const int4 e = d.er[t];
            emit = true;
            if (rk[2 * t] > rk[2 * t + 1]) {  // piece of x is the parent
                q.start = e.y; q.newpar = e.x; q.stop = d.prt[e.w];
            } else {
                q.start = e.x; q.newpar = e.y; q.stop = d.prt[e.z];
            }
        } else if (t < total) {
            const int64_t p = t - ner;
            if (d.comp[p] == (int32_t)p) {
                const uint64_t sk = d.srkey[p];
                const int32_t S = (int32_t)(uint32_t)sk, m = (int32_t)(sk >> 32);
                d.newlab[p] = m;
                if (m != d.prt[S]) {
                    emit = true;
                    q.start = m; q.newpar = m; q.stop = d.prt[S];
                }
            }
        }
        const int64_t slot = block_append(emit ? 1 : 0, &d.cnt[C_NR]);
        if (emit) {
            if (slot < d.pathcap) d.paths[slot] = q;
            else atomicOr(d.status, ST_CAPACITY);
        }
    }
}

// ------------------------------------- a8: path reversal + new parents

// One thread per path.  Paths lie in distinct pieces (at most one per piece:
// the attach path of a non-root piece or the re-root path of a super-root
// piece), so the walks touch disjoint vertices; each thread reads a parent
// before overwriting it (the old orientation is read exactly once).  A walk
// first follows its path read-only for at most walk_k steps: a path that
// does not reach its end by then is listed for the doubling pass below and
// left untouched (the whole path, its new parent included), so one long
// path cannot hold the update for its length in dependent reads.
__device__ void reverse_paths(const Dev &d, int64_t bid, int64_t nblk) {
    const int64_t nr = (int64_t)d.cnt[C_NR];
    const int64_t stride = nblk * BLOCK;
    for (int64_t i = bid * BLOCK + threadIdx.x; i < nr; i += stride) {
        const PathReq q = d.paths[i];
        int32_t cur = q.start;
        for (int64_t steps = 0; cur != q.stop && steps < d.walk_k; steps++) cur = d.parent[cur];
        if (cur != q.stop) {
            const unsigned long long k = atomicAdd(&d.cnt[C_NLONG], 1ull);
            if ((int64_t)k < d.lpcap) d.lp_list[k] = (int32_t)i;
            else atomicOr(d.status, ST_CAPACITY);
            continue;
        }
        int32_t prev = q.newpar;
        cur = q.start;
        for (int64_t steps = 0;; steps++) {
            const int32_t nxt = d.parent[cur];
            d.parent[cur] = prev;
            if (cur == q.stop) break;
            prev = cur;
            cur = nxt;
            if (steps > d.n) { atomicOr(d.status, ST_WALK_BOUND); break; }
        }
    }
}
__global__ __launch_bounds__(BLOCK) void k_reverse_all(Dev d) {
    if (stopped(d)) return;
    reverse_paths(d, blockIdx.x, gridDim.x);
}

// ----------------------------- a8: long paths by pointer doubling
//
// A long path's vertices are the ancestors of its start x up to its piece
// root r, and r is still a root: the walks above turned only the paths of
// other pieces, and an attach writes the parent of its own path's start.
// Marks spread up by doubling.  In round k every vertex's jump pointer goes
// from the ancestor 2^k steps up to the one 2^(k+1) up (both capped at the
// root), and every marked vertex marks the ancestor its jump pointer names;
// so before round k each ancestor of x fewer than 2^k steps up is marked.
// Only ancestors of a start are ever marked, so a mark that another thread
// of the same round reads as soon as it is set does no harm.  Once every
// start's jump pointer names its path's end, the marks are complete: each
// marked vertex below its root turns its parent edge, parent[p0[u]] = u
// (distinct targets along a path, read from the snapshot p0, so no write
// races a read), and each start hangs below its new parent.

__global__ __launch_bounds__(BLOCK) void k_lp_init(Dev d, LongPaths b) {
    if (stopped(d)) return;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t u = (int64_t)blockIdx.x * BLOCK + threadIdx.x; u < d.n; u += stride) {
        const int32_t p = d.parent[u];
        b.p0[u] = p;
        b.j0[u] = p;
    }
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < b.nlong; i += stride)
        b.mark[d.paths[d.lp_list[i]].start] = b.epoch;
}

__global__ __launch_bounds__(BLOCK) void k_lp_round(Dev d, LongPaths b, const int32_t *jin, int32_t *jout) {
    if (stopped(d) || d.cnt[C_LP_DONE]) return;
    if (blockIdx.x == 0) {
        // reads jin only, which no thread of this round writes
        bool reached = true;
        for (int64_t i = threadIdx.x; i < b.nlong; i += BLOCK) {
            const PathReq q = d.paths[d.lp_list[i]];
            reached = reached && jin[q.start] == q.stop;
        }
        if (__syncthreads_and(reached)) {
            if (threadIdx.x == 0) d.cnt[C_LP_DONE] = 1;
            return;
        }
    }
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t u = (int64_t)blockIdx.x * BLOCK + threadIdx.x; u < d.n; u += stride) {
        const int32_t j = jin[u];
        jout[u] = jin[j];
        if (b.mark[u] == b.epoch && b.mark[j] != b.epoch) b.mark[j] = b.epoch;
    }
}

__global__ __launch_bounds__(BLOCK) void k_lp_reverse(Dev d, LongPaths b) {
    if (stopped(d)) return;
    if (!d.cnt[C_LP_DONE]) {  // a start did not reach its path's end: not a forest
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(d.status, ST_WALK_BOUND);
        return;
    }
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t u = (int64_t)blockIdx.x * BLOCK + threadIdx.x; u < d.n; u += stride) {
        if (b.mark[u] != b.epoch) continue;
        const int32_t p = b.p0[u];
        if (p != (int32_t)u) d.parent[p] = (int32_t)u;
    }
    // the loop above never writes a start's parent: it writes the old
    // parent of a marked vertex, which lies above it, and a start is the
    // lowest vertex of its path
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < b.nlong; i += stride) {
        const PathReq q = d.paths[d.lp_list[i]];
        d.parent[q.start] = q.newpar;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) d.cnt[C_NLONG] = 0;  // the update may finish
}

// ------------------------------------------------------------ a9: labels

// Deletes: a vertex cut off from its old root takes its new component's
// label.  Runs before the insert labels (mixed batches).  Restores
// rep == label for the next update.
__device__ void label_delete(const Dev &d, int64_t bid, int64_t nblk) {
    if (d.cnt[C_OMODE]) {
        // the orphan list holds every orphan with its piece (rep and the
        // piece table are unchanged since root finding): relabel them, clear
        // their bitmap words and their blocks' figures (idempotent stores)
        const int64_t no = (int64_t)d.cnt[C_NORPH];
        const int64_t stride = nblk * BLOCK;
        for (int64_t i = bid * BLOCK + threadIdx.x; i < no; i += stride) {
            const int32_t v = d.olist[i].v;
            const int32_t p = d.olist[i].pu;
            if (p >= 0) {
                const int32_t l = d.newlab[d.comp[p]];
                d.label[v] = l;
                d.rep[v] = l;
            } else {
                atomicOr(d.status, ST_WALK_BOUND);
            }
            d.obits[v >> 6] = 0;
            d.bvol[v / BLOCK] = 0;
            d.bcnt[v / BLOCK] = 0;
        }
        return;
    }
    const int64_t nb = (d.n + BLOCK - 1) / BLOCK;
    const int64_t nvl_list = d.ctl->nvl;  // read once: stores below may alias it
    for (int64_t j = bid;; j += nblk) {
        const int64_t blk = list_block(d.vlist, nvl_list, j, nb);
        if (blk < 0) break;
        const int64_t v = blk * BLOCK + threadIdx.x;
        uint64_t w = 0;
        if (v < d.n) w = d.obits[v >> 6];
        // the bitmap is all zero between updates (the sweeps read it for any
        // vertex); the store depends on the loaded word, so it lands after
        // every lane's read
        if (lane_id() == 0 && w != 0) d.obits[v >> 6] = 0;
        if (threadIdx.x == 0) {  // read only by this update's orphan scan
            d.bvol[blk] = 0;
            d.bcnt[blk] = 0;
        }
        if (v < d.n && ((w >> (v & 63)) & 1)) {
            const int32_t p = d.tidx[d.rep[v]];
            if (p >= 0) {
                const int32_t l = d.newlab[d.comp[p]];
                d.label[v] = l;
                d.rep[v] = l;
            } else {
                atomicOr(d.status, ST_WALK_BOUND);
            }
        }
    }
}

// Inserts: every vertex of a tree that merged into another takes the new
// component's label (the tree is found through its old label, its root).
__device__ void label_insert(const Dev &d, int64_t bid, int64_t nblk) {
    if (d.cnt[C_NP] == 0) return;
    typedef int v4i __attribute__((ext_vector_type(4)));
    const int64_t nb = (d.n + BLOCK - 1) / BLOCK;
    const int w = threadIdx.x / WAVE;
    // one wave per vertex block, four vertices per lane
    const int64_t nil_list = d.ctl->nil;  // read once: stores below may alias it
    for (int64_t j = bid * (BLOCK / WAVE) + w;; j += nblk * (BLOCK / WAVE)) {
        const int64_t blk = list_block(d.ilist, nil_list, j, nb);
        if (blk < 0) break;
        const int64_t v = blk * BLOCK + lane_id() * 4;
        int32_t lab[4];
        if (v + 4 <= d.n) {
            const v4i x = *reinterpret_cast<const v4i *>(d.label + v);
            lab[0] = x.x; lab[1] = x.y; lab[2] = x.z; lab[3] = x.w;
        } else {
            for (int k = 0; k < 4; k++) lab[k] = v + k < d.n ? d.label[v + k] : 0;
        }
        int32_t t[4];
#pragma unroll
        for (int k = 0; k < 4; k++) t[k] = d.tidx[lab[k]];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (v + k < d.n && t[k] != NONE) {
                const int32_t l = d.newlab[d.comp[t[k]]];
                if (l != lab[k]) {  // the super-root's tree keeps its label
                    d.label[v + k] = l;
                    d.rep[v + k] = l;
                }
            }
        }
    }
}

// Path reversal and labels touch disjoint data (parent and the paths; label,
// rep and the orphan scratch), so one launch does both: workgroups below
// grev reverse paths, the rest relabel (lab: 1 inserts, 2 deletes).
__global__ __launch_bounds__(BLOCK) void k_finish(Dev d, int lab, int grev) {
    if (stopped(d) || !d.cnt[C_ORIENTED]) return;
    if ((int)blockIdx.x < grev) {
        reverse_paths(d, blockIdx.x, grev);
    } else {
        const int64_t bid = (int64_t)blockIdx.x - grev, nblk = (int64_t)gridDim.x - grev;
        if (lab == 2 && d.ctl->has_del) label_delete(d, bid, nblk);
        if (lab == 1 && d.ctl->has_ins) label_insert(d, bid, nblk);
    }
}

// The insert labels of a mixed batch, after the delete labels.
__global__ __launch_bounds__(BLOCK) void k_label_insert(Dev d) {
    if (stopped(d) || !d.cnt[C_ORIENTED] || !d.ctl->has_ins) return;
    label_insert(d, blockIdx.x, gridDim.x);
}

// ---------------- f2: replacement edges on the supergraph (Sec. III-A)
//
// The supergraph has a vertex per piece and an edge per pair of pieces that
// a cross edge joins.  Its edges are taken from the cross edges of the first
// round by a radix sort on the piece pair and a minimum per run of equal
// pairs (the lowest key of the pair, where the paper keeps whichever edge a
// racy hash write leaves); the hooking rounds then run on these edges only.
// Regions holding the first round's cross edges: the orphan scan's ranges
// [0, nr_om) when it ran, then regions from rlo2.
__device__ __forceinline__ int64_t sg_region(int64_t i, int64_t nr_om, int64_t rlo2) {
    return i < nr_om ? i : rlo2 + (i - nr_om);
}

// cross edges per region, and the cross-edge count statistic (as round 0)
__global__ __launch_bounds__(BLOCK) void k_sg_count(Dev d, int64_t nr_om, int64_t rlo2, int64_t nreg,
                                                    uint32_t *rcount) {
    if (stopped(d)) return;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    unsigned long long st = 0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < nreg; i += stride) {
        const unsigned long long c = d.rcnt[sg_region(i, nr_om, rlo2)];
        rcount[i] = (uint32_t)c;
        st += i < nr_om ? d.xcnt[i] : c;  // the orphan scan counted its edges before merging runs
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) st += __shfl_xor(st, o);
    if (lane_id() == 0 && st) atomicAdd(&d.cnt[C_NCROSS], st);
}

// (smaller piece << 32 | larger piece) and the edge key of every cross edge,
// densely (one workgroup per region)
__global__ __launch_bounds__(BLOCK) void k_sg_gather(Dev d, int64_t nr_om, int64_t rlo2, int64_t nreg,
                                                     const uint32_t *rpos, uint64_t *keys, uint64_t *vals) {
    if (stopped(d)) return;
    for (int64_t i = blockIdx.x; i < nreg; i += gridDim.x) {
        const int64_t t = sg_region(i, nr_om, rlo2);
        const int64_t c = (int64_t)d.rcnt[t], base = rpos[i];
        const Cross *in = d.x0 + t * TILE;
        for (int64_t j = threadIdx.x; j < c; j += BLOCK) {
            const Cross e = in[j];
            const uint32_t lo = (uint32_t)(e.pa < e.pb ? e.pa : e.pb), hi = (uint32_t)(e.pa < e.pb ? e.pb : e.pa);
            keys[base + j] = ((uint64_t)lo << 32) | hi;
            vals[base + j] = e.key;
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_sg_heads(int64_t total, const uint64_t *skeys, uint32_t *flag) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < total; j += stride)
        flag[j] = (j == 0 || skeys[j] != skeys[j - 1]) ? 1u : 0u;
}

// lowest key per run of equal pairs (segid: exclusive count of heads)
__global__ __launch_bounds__(BLOCK) void k_sg_min(int64_t total, const uint32_t *flag, const uint32_t *segid,
                                                  const uint64_t *svals, uint64_t *smin) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < total; j += stride) {
        const int64_t seg = (int64_t)segid[j] + flag[j] - 1;
        const uint64_t v = svals[j];
        if (smin[seg] > v) atomicMin((unsigned long long *)&smin[seg], (unsigned long long)v);
    }
}

// the supergraph's edges, densely in x0, with their count in C_NX0
__global__ __launch_bounds__(BLOCK) void k_sg_emit(Dev d, int64_t total, const uint64_t *skeys,
                                                   const uint32_t *flag, const uint32_t *segid,
                                                   const uint64_t *smin, const unsigned long long *nseg) {
    if (stopped(d)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        d.cnt[C_NX0] = *nseg;
        d.cnt[C_NX1] = 0;
    }
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < total; j += stride) {
        if (!flag[j]) continue;
        const int64_t seg = segid[j];
        Cross e;
        e.key = smin[seg];
        e.pa = (int32_t)(skeys[j] >> 32);
        e.pb = (int32_t)(uint32_t)skeys[j];
        d.x0[seg] = e;
    }
}

// -------------------------- f1: path reversal by Euler tour (Alg. 3)
//
// F-hat is the forest of the parents as they are before any reversal.  Its
// child lists come from sorting (parent << 32 | child) keys, so siblings are
// in increasing id order.  Euler tour of each tree (EulerianTour, first step
// of Alg. 3): the tour enters a child c through its down arc 2c, walks c's
// subtree, leaves through the up arc 2c + 1, then goes down to c's next
// sibling, or else up from c's parent (the tour of a root ends there).  List
// ranking by pointer jumping gives every arc the number of arcs after it in
// its tour; its rank is the tour length - 1 - that number.

// keys for the child lists, and the F-hat parents
__global__ __launch_bounds__(BLOCK) void k_et_keys(Dev d) {
    if (stopped(d) || !d.cnt[C_ORIENTED]) return;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < d.n; v += stride) {
        const int32_t p = d.parent[v];
        d.et_opar[v] = p;
        // roots sort after every child entry and are skipped
        const uint64_t hi = p == (int32_t)v ? 0xffffffffull : (uint64_t)(uint32_t)p;
        d.et_keys[v] = (hi << 32) | (uint32_t)v;
    }
}

// first child and next sibling from the sorted keys
__global__ __launch_bounds__(BLOCK) void k_et_links(Dev d) {
    if (stopped(d) || !d.cnt[C_ORIENTED]) return;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < d.n; j += stride) {
        const uint64_t k = d.et_sorted[j];
        const uint32_t p = (uint32_t)(k >> 32);
        if (p == 0xffffffffu) continue;
        const int32_t c = (int32_t)(uint32_t)k;
        if (j == 0 || (uint32_t)(d.et_sorted[j - 1] >> 32) != p) d.et_fc[p] = c;
        const uint64_t nk = j + 1 < d.n ? d.et_sorted[j + 1] : ~0ull;
        d.et_ns[c] = (uint32_t)(nk >> 32) == p ? (int32_t)(uint32_t)nk : NONE;
    }
}

// successor of every arc, and the ranking's start (1 arc after, or 0 at the end)
__global__ __launch_bounds__(BLOCK) void k_et_succ(Dev d) {
    if (stopped(d) || !d.cnt[C_ORIENTED]) return;
    const int64_t na = 2 * (int64_t)d.n;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t a = (int64_t)blockIdx.x * BLOCK + threadIdx.x; a < na; a += stride) {
        const int32_t v = (int32_t)(a >> 1), pv = d.et_opar[v];
        int32_t nx = NONE;  // a root has no arcs
        if (pv != v) {
            if ((a & 1) == 0) {
                const int32_t c = d.et_fc[v];
                nx = c != NONE ? 2 * c : 2 * v + 1;
            } else {
                const int32_t sb = d.et_ns[v];
                nx = sb != NONE ? 2 * sb : (d.et_opar[pv] == pv ? NONE : 2 * pv + 1);
            }
        }
        d.et_nxt0[a] = nx;
        d.et_dst0[a] = nx == NONE ? 0 : 1;
    }
}

// one pointer-jumping round: every arc adds the count of its successor and
// jumps past it
__global__ __launch_bounds__(BLOCK) void k_et_round(Dev d, const int32_t *nin, const int32_t *din,
                                                    int32_t *nout, int32_t *dout) {
    if (stopped(d) || !d.cnt[C_ORIENTED]) return;
    const int64_t na = 2 * (int64_t)d.n;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t a = (int64_t)blockIdx.x * BLOCK + threadIdx.x; a < na; a += stride) {
        const int32_t nx = nin[a];
        int32_t dn = din[a], nn = NONE;
        if (nx != NONE) {
            dn += din[nx];
            nn = nin[nx];
        }
        nout[a] = nn;
        dout[a] = dn;
    }
}

// start and finish times (Alg. 3): a leaf takes its up arc's rank for both;
// a root the rank of its first arc and its tour's length; any other vertex
// the rank of the down arc to its first child and of its own up arc
__global__ __launch_bounds__(BLOCK) void k_et_times(Dev d, const int32_t *dst) {
    if (stopped(d) || !d.cnt[C_ORIENTED]) return;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < d.n; v += stride) {
        const int32_t r = d.rep[v];  // root of v's tree of F-hat
        const int32_t fr = d.et_fc[r];
        const int32_t L = fr != NONE ? dst[2 * fr] + 1 : 0;  // arcs in r's tour
        const int32_t fc = d.et_fc[v];
        int32_t st, fi;
        if (d.et_opar[v] == (int32_t)v) {
            st = 0;
            fi = L;
        } else if (fc == NONE) {
            st = fi = L - 1 - dst[2 * v + 1];
        } else {
            st = L - 1 - dst[2 * fc];
            fi = L - 1 - dst[2 * v + 1];
        }
        d.et_start[v] = st;
        d.et_finish[v] = fi;
    }
}

// support[r] = x for each path (x, r) of R (at most one path per tree of F-hat)
__global__ __launch_bounds__(BLOCK) void k_et_support(Dev d) {
    if (stopped(d) || !d.cnt[C_ORIENTED]) return;
    const int64_t nr = (int64_t)d.cnt[C_NR];
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < nr; i += stride) {
        const PathReq q = d.paths[i];
        d.et_support[q.stop] = q.start;
    }
}

// Every tree edge (u, parent[u]) whose u lies on the path from x = support[r]
// up to its root r (excluding r: the interval test of Alg. 3) turns around:
// parent[old parent of u] = u.  Then each path's start hangs below its new
// parent (its own parent edge is not on any path, so no write collides).
__global__ __launch_bounds__(BLOCK) void k_et_reverse(Dev d) {
    if (stopped(d) || !d.cnt[C_ORIENTED]) return;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t u = (int64_t)blockIdx.x * BLOCK + threadIdx.x; u < d.n; u += stride) {
        const int32_t pu = d.et_opar[u];
        if (pu == (int32_t)u) continue;
        const int32_t r = d.rep[u];
        const int32_t x = d.et_support[r];
        if (x == NONE) continue;
        const int32_t su = d.et_start[u], fu = d.et_finish[u];
        if (d.et_start[r] < su && su <= d.et_start[x] && d.et_finish[r] > fu && fu >= d.et_finish[x])
            d.parent[pu] = (int32_t)u;
    }
    const int64_t nr = (int64_t)d.cnt[C_NR];
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < nr; i += stride) {
        const PathReq q = d.paths[i];
        d.parent[q.start] = q.newpar;
    }
}

// ------------------------------------------------------------- cleanup

// Resets the per-update scratch once the update has finished (or failed);
// the workgroup that finishes last then hands status, counters and per-graph
// batch status to the host (pinned memory, also when the update is
// unfinished and the host continues it) and resets them once the update has
// finished.
__global__ __launch_bounds__(BLOCK) void k_cleanup(Dev d) {
    if (held(d)) return;  // queued behind an unfinished update: no handoff, no reset
    // else unfinished: the host continues (more rounds or levels, or the
    // paths too long for one thread)
    const bool fin = (d.cnt[C_ORIENTED] && !d.cnt[C_NLONG]) || *d.status;
    if (fin) {
        const int64_t np = (int64_t)d.cnt[C_NP];
        const int64_t b = d.ctl->b;
        const int64_t stride = (int64_t)gridDim.x * BLOCK;
        for (int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x; p < np; p += stride) {
            d.tidx[d.prt[p]] = NONE;
            d.level[p] = -1;  // the super-forest search starts from all -1
            d.parc[p] = NONE;
            if (d.et_support) d.et_support[d.prt[p]] = NONE;  // path ends are piece roots
        }
        for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < b; i += stride)
            if (d.bslot[i] != NONE) d.bhash[d.bslot[i]] = HASH_EMPTY;
        const int64_t rlo = d.ctl->rlo, rhi = d.ctl->rhi;  // read once: the stores may alias them
        for (int64_t t = rlo + (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < rhi; t += stride)
            d.rcnt[t] = 0;
    }
    if (!last_block_arrives(&d.cnt[C_ARRIVE])) return;
    for (int64_t t = threadIdx.x; t < d.ret_words; t += BLOCK) d.hret[t] = d.ctlmem[t];
    __threadfence_system();
    __syncthreads();  // every thread has copied before the completion word and any reset
    if (!fin) {
        // later updates on the stream wait for the host's continuation
        if (threadIdx.x == 0) d.status[1] = 1;
        __syncthreads();
    }
    if (threadIdx.x == 0)
        __hip_atomic_store(d.hdone, (unsigned long long)d.ctl->seq, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_SYSTEM);
    if (!fin) return;
    const int t = threadIdx.x;
    for (int u = t; u < C_TOTAL; u += BLOCK)
        if (u != C_NDELTA) d.cnt[u] = 0;
    for (int64_t g = threadIdx.x; g < d.ctl->ngraph; g += BLOCK) d.gstat[g] = 0;
    if (t == 0) {
        d.status[0] = 0;
        d.status[1] = 0;  // the hold word
    }
}

// ------------------------------------------------------------ launchers

int64_t delta_tiles(int64_t count) { return (count + TILE - 1) / TILE; }
int64_t insert_regions(int64_t b) { return (b + BLOCK - 1) / BLOCK; }

// Pieces an update can register: two per batch edge (a grid over them is
// grid-stride; its size only sets how many workgroups share the work).
static int64_t piece_bound(const Dev &d) { return std::min<int64_t>(d.pcap, 2 * d.lb + 16); }

void launch_classify(const Dev &d, const Ctl *kc, hipStream_t s) {
    const Ctl none{};
    hipLaunchKernelGGL(k_classify, dim3(grid_for(d.lb, BLOCK)), dim3(BLOCK), 0, s, d, kc ? *kc : none,
                       kc ? 1 : 0);
}
void launch_dedupe(const Dev &d, hipStream_t s) {
    hipLaunchKernelGGL(k_dedupe, dim3(grid_for(d.lb, BLOCK)), dim3(BLOCK), 0, s, d);
}
void launch_prepare(const Dev &d, bool del, hipStream_t s) {
    const int gb = grid_for(d.lb, BLOCK);
    const int gi = del ? grid_for(d.nvb, BLOCK / WAVE, COPY_CAP) : 0;
    hipLaunchKernelGGL(k_prepare, dim3(gb + gi), dim3(BLOCK), 0, s, d, gb);
}
void launch_register(const Dev &d, hipStream_t s) {
    hipLaunchKernelGGL(k_register, dim3(grid_for(d.lb, BLOCK)), dim3(BLOCK), 0, s, d);
}
void launch_insert_emit(const Dev &d, hipStream_t s) {
    hipLaunchKernelGGL(k_insert_emit, dim3((unsigned)insert_regions(d.lb)), dim3(BLOCK), 0, s, d);
}
void launch_rep_jump(const Dev &d, int rounds, hipStream_t s) {
    for (int k = 0; k < std::min(rounds, MAX_JUMP); k++)
        hipLaunchKernelGGL(k_rep_jump, dim3(grid_for(d.nvb, 1, GRID_CAP)), dim3(BLOCK), 0, s, d, k);
}
void launch_rep_chase(const Dev &d, hipStream_t s) {
    hipLaunchKernelGGL(k_rep_chase, dim3(grid_for(d.nvb, REP_CH, GRID_CAP)), dim3(BLOCK), 0, s, d);
}
void launch_sweep_base(const Dev &d, hipStream_t s) {
    // persistent: about as many workgroups as fit at once (24 KB of LDS each)
    if (d.ntiles > 0)
        hipLaunchKernelGGL(k_sweep_base, dim3(grid_for(d.ntiles, 1, 6 * 256)), dim3(BLOCK), 0, s, d);
}
void launch_orphan_plan(const Dev &d, hipStream_t s) {
    hipLaunchKernelGGL(k_orph_plan, dim3(grid_for(d.nvb, BLOCK, 1 << 30)), dim3(BLOCK), 0, s, d);
    hipLaunchKernelGGL(k_orph_total, dim3(1), dim3(BLOCK), 0, s, d);
}
void launch_orphan_fill(const Dev &d, hipStream_t s) {
    hipLaunchKernelGGL(k_orph_fill, dim3(grid_for(d.nvb, BLOCK / 8, GRID_CAP)), dim3(BLOCK), 0, s, d);
}
void launch_orphan_scan(const Dev &d, hipStream_t s) {
    hipLaunchKernelGGL(k_orph_scan, dim3(grid_for(d.ntiles, 1, GRID_CAP)), dim3(BLOCK), 0, s, d);
}
void launch_sweep_delta(const Dev &d, hipStream_t s) {
    if (d.ltiles > 0)
        hipLaunchKernelGGL(k_sweep_delta, dim3((unsigned)d.ltiles), dim3(BLOCK), 0, s, d);
}
// The hooking, rooting and reversal kernels index pieces, arcs and paths
// (at most 2 max_batch): grids of one workgroup per CU, grid-stride, so a
// round that finds nothing to do costs little dispatch.
void launch_boruvka(const Dev &d, int r0, int r1, int64_t units, bool emit, hipStream_t s) {
    const int ge = grid_for(units, 1, EDGE_CAP);
    const int gp = grid_for(piece_bound(d), BLOCK, SMALL_CAP);
    for (int r = r0; r < r1; r++) {
        if (r == 0)
            hipLaunchKernelGGL(k_bor_round0, dim3(ge), dim3(BLOCK), 0, s, d, emit ? 1 : 0);
        else
            hipLaunchKernelGGL(k_bor_select, dim3(r == 1 ? ge : gp), dim3(BLOCK), 0, s, d, r);
        hipLaunchKernelGGL(k_bor_hook, dim3(gp), dim3(BLOCK), 0, s, d, r);
    }
    // the tail reads a dense list, which rounds from 2 on have
    if (r1 >= 2 && r1 > r0) hipLaunchKernelGGL(k_bor_tail, dim3(1), dim3(TAIL_THREADS), 0, s, d, r1);
}
void launch_sf_root(const Dev &d, hipStream_t s) {
    const int gp = grid_for(piece_bound(d), BLOCK, SMALL_CAP);
    hipLaunchKernelGGL(k_sf_root, dim3(gp), dim3(BLOCK), 0, s, d);
}
void launch_sf_bfs(const Dev &d, int l0, int l1, hipStream_t s) {
    const int ga = grid_for(2 * std::min<int64_t>(d.ercap, piece_bound(d)), BLOCK, SMALL_CAP);
    for (int L = l0; L < l1; L++) hipLaunchKernelGGL(k_sf_bfs, dim3(ga), dim3(BLOCK), 0, s, d, L);
}
void launch_orient_bfs(const Dev &d, int levels, hipStream_t s) {
    hipLaunchKernelGGL(k_orient_bfs, dim3(grid_for(piece_bound(d), BLOCK, SMALL_CAP)), dim3(BLOCK), 0, s, d,
                       levels);
}
void launch_superforest_lr(const Dev &d, int lr_rounds, int levels, hipStream_t s) {
    const int ga = grid_for(2 * d.ercap, BLOCK, SMALL_CAP);
    hipLaunchKernelGGL(k_sf_arcs, dim3(grid_for(d.ercap, BLOCK, SMALL_CAP)), dim3(BLOCK), 0, s, d, levels);
    hipLaunchKernelGGL(k_sf_succ, dim3(ga), dim3(BLOCK), 0, s, d, levels);
    for (int r = 0; r < lr_rounds; r++)
        hipLaunchKernelGGL(k_lr_round, dim3(ga), dim3(BLOCK), 0, s, d, r, levels);
    hipLaunchKernelGGL(k_orient_lr, dim3(grid_for(d.ercap + d.pcap, BLOCK, SMALL_CAP)), dim3(BLOCK), 0, s,
                       d, lr_rounds, levels);
}
void launch_reverse_all(const Dev &d, hipStream_t s) {
    hipLaunchKernelGGL(k_reverse_all, dim3(grid_for(d.pathcap, BLOCK, 2048)), dim3(BLOCK), 0, s, d);
}
void launch_long_paths(const Dev &d, const LongPaths &b, hipStream_t s) {
    const int gv = grid_for(d.n, BLOCK, GRID_CAP);
    hipLaunchKernelGGL(k_lp_init, dim3(gv), dim3(BLOCK), 0, s, d, b);
    // round k finds every start's jump at its path's end once the path has
    // at most 2^k steps, and a path has fewer than n: rounds 0 .. k with 2^k >= n
    int rounds = 1;
    while ((int64_t(1) << (rounds - 1)) < (int64_t)d.n) rounds++;
    for (int k = 0; k < rounds; k++)
        hipLaunchKernelGGL(k_lp_round, dim3(gv), dim3(BLOCK), 0, s, d, b, (k & 1) ? b.j1 : b.j0,
                           (k & 1) ? b.j0 : b.j1);
    hipLaunchKernelGGL(k_lp_reverse, dim3(gv), dim3(BLOCK), 0, s, d, b);
}
void launch_finish(const Dev &d, bool ins, bool del, bool rev, hipStream_t s) {
    // an update reverses at most one path per piece and per replacement edge
    const int grev = rev ? grid_for(std::min<int64_t>(d.ercap, piece_bound(d)) + piece_bound(d), BLOCK, FINISH_CAP)
                         : 0;
    // deletes relabel per vertex block or per listed orphan, inserts one wave
    // per vertex block
    const int glab = del ? grid_for(d.n, BLOCK, FINISH_CAP) : grid_for(d.nvb, BLOCK / WAVE, FINISH_CAP);
    hipLaunchKernelGGL(k_finish, dim3(grev + glab), dim3(BLOCK), 0, s, d, del ? 2 : 1, grev);
    if (ins && del)
        hipLaunchKernelGGL(k_label_insert, dim3(grid_for(d.nvb, BLOCK / WAVE, GRID_CAP)), dim3(BLOCK), 0,
                           s, d);
}
void launch_sg_regions(const Dev &d, int64_t nr_om, int64_t rlo2, int64_t nreg, const SgScratch &g,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_sg_count, dim3(grid_for(nreg, BLOCK)), dim3(BLOCK), 0, s, d, nr_om, rlo2, nreg,
                       g.rcount);
    launch_scan_u32(g.rcount, g.rpos, g.totals, nreg, g.scan_tmp, s);
}
int launch_sg_reduce(const Dev &d, int64_t nr_om, int64_t rlo2, int64_t nreg, int64_t total,
                     const SgScratch &g, hipStream_t s) {
    // the dense (pair, key) lists use x1, which the rounds overwrite later
    uint64_t *keys = reinterpret_cast<uint64_t *>(d.x1), *vals = keys + d.xcap;
    hipLaunchKernelGGL(k_sg_gather, dim3(grid_for(nreg, 1)), dim3(BLOCK), 0, s, d, nr_om, rlo2, nreg, g.rpos,
                       keys, vals);
    if (total > 0 &&
        launch_sort_pairs_u64(keys, g.skeys, vals, g.svals, total, g.sort_tmp, g.sort_tmp_bytes, s))
        return -1;
    const int gt = grid_for(total, BLOCK);
    hipLaunchKernelGGL(k_sg_heads, dim3(gt), dim3(BLOCK), 0, s, total, g.skeys, g.flag);
    launch_scan_u32(g.flag, g.segid, g.totals + 1, total, g.scan_tmp, s);
    uint64_t *smin = keys;  // the unsorted keys are no longer needed
    launch_fill_u64(smin, total > 0 ? total : 1, KEY_INF, s);
    hipLaunchKernelGGL(k_sg_min, dim3(gt), dim3(BLOCK), 0, s, total, g.flag, g.segid, g.svals, smin);
    hipLaunchKernelGGL(k_sg_emit, dim3(gt), dim3(BLOCK), 0, s, d, total, g.skeys, g.flag, g.segid, smin,
                       g.totals + 1);
    return 0;
}

int launch_et_reverse(const Dev &d, void *tmp, size_t tmp_bytes, hipStream_t s) {
    const int gv = grid_for(d.n, BLOCK, GRID_CAP), ga = grid_for(2 * (int64_t)d.n, BLOCK, GRID_CAP);
    hipLaunchKernelGGL(k_et_keys, dim3(gv), dim3(BLOCK), 0, s, d);
    if (launch_sort_u64(d.et_keys, d.et_sorted, d.n, tmp, tmp_bytes, s)) return -1;
    launch_fill_i32(d.et_fc, d.n, NONE, s);
    hipLaunchKernelGGL(k_et_links, dim3(gv), dim3(BLOCK), 0, s, d);
    hipLaunchKernelGGL(k_et_succ, dim3(ga), dim3(BLOCK), 0, s, d);
    // 2^rounds >= 2n: every arc has jumped past the end of its tour
    int rounds = 0;
    while ((int64_t)1 << rounds < 2 * (int64_t)d.n) rounds++;
    int32_t *n0 = d.et_nxt0, *d0 = d.et_dst0, *n1 = d.et_nxt1, *d1 = d.et_dst1;
    for (int r = 0; r < rounds; r++) {
        hipLaunchKernelGGL(k_et_round, dim3(ga), dim3(BLOCK), 0, s, d, n0, d0, n1, d1);
        std::swap(n0, n1);
        std::swap(d0, d1);
    }
    hipLaunchKernelGGL(k_et_times, dim3(gv), dim3(BLOCK), 0, s, d, d0);
    hipLaunchKernelGGL(k_et_support, dim3(grid_for(d.ercap + d.pcap, BLOCK, GRID_CAP)), dim3(BLOCK), 0,
                       s, d);
    hipLaunchKernelGGL(k_et_reverse, dim3(gv), dim3(BLOCK), 0, s, d);
    return 0;
}
void launch_cleanup(const Dev &d, hipStream_t s) {
    const int64_t m = std::max<int64_t>(piece_bound(d), d.lb);
    // few workgroups: each arrives once on one counter (serialised atomics)
    hipLaunchKernelGGL(k_cleanup, dim3(grid_for(m, BLOCK, CLEANUP_CAP)), dim3(BLOCK), 0, s, d);
}

// ------------------------------------------------------ store rebuild

// live inserted edges as directed pairs in both directions
__global__ __launch_bounds__(BLOCK) void k_rb_pairs(const uint64_t *dkey, const unsigned long long *ndelta,
                                                    uint64_t *pairs, unsigned long long *npairs,
                                                    int64_t cap) {
    const int64_t nd = (int64_t)*ndelta;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < nd; base += stride) {
        const int64_t i = base + threadIdx.x;
        const uint64_t k = i < nd ? dkey[i] : KEY_DEAD;
        const bool live = k != KEY_DEAD;
        const int64_t pos = block_append(live ? 2 : 0, npairs);
        if (live && pos + 1 < cap) {
            const uint64_t lo = k >> 32, hi = k & 0xffffffffull;
            pairs[pos] = k;
            pairs[pos + 1] = (hi << 32) | lo;
        }
    }
}
void launch_rb_pairs(const uint64_t *dkey, const unsigned long long *ndelta, uint64_t *pairs,
                     unsigned long long *npairs, int64_t cap, hipStream_t s) {
    hipLaunchKernelGGL(k_rb_pairs, dim3(grid_for(cap / 2 + 1, BLOCK, 4096)), dim3(BLOCK), 0, s, dkey, ndelta,
                       pairs, npairs, cap);
}
__global__ void k_rb_pair_deg(const uint64_t *pairs, const unsigned long long *npairs, uint32_t *ddeg,
                              int64_t cap) {
    const int64_t np = (int64_t)*npairs < cap ? (int64_t)*npairs : cap;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride)
        atomicAdd(&ddeg[pairs[i] >> 32], 1u);
}
void launch_rb_pair_deg(const uint64_t *pairs, const unsigned long long *npairs, uint32_t *ddeg,
                        int64_t cap, hipStream_t s) {
    hipLaunchKernelGGL(k_rb_pair_deg, dim3(grid_for(cap, BLOCK, 4096)), dim3(BLOCK), 0, s, pairs, npairs,
                       ddeg, cap);
}
__global__ void k_add_u32(const uint32_t *a, const uint32_t *b, uint32_t *out, int64_t count) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        out[i] = a[i] + b[i];
}
void launch_add_u32(const uint32_t *a, const uint32_t *b, uint32_t *out, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_add_u32, dim3(grid_for(count, BLOCK, GRID_CAP)), dim3(BLOCK), 0, s, a, b, out, count);
}
__global__ void k_u32_to_i64(const uint32_t *in, int64_t *out, int64_t count) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        out[i] = (int64_t)in[i];
}
void launch_u32_to_i64(const uint32_t *in, int64_t *out, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_u32_to_i64, dim3(grid_for(count, BLOCK, GRID_CAP)), dim3(BLOCK), 0, s, in, out, count);
}

// The merged symmetric CSR is written slot-parallel (a hub row holds
// hundreds of thousands of entries; a thread or a wave per row leaves it to
// one lane).  Row u of the merge is its live lower entries, then its live
// upper entries (together ascending), merged with its inserted neighbours
// (ascending in the sorted pairs).  With LS / US the exclusive prefix counts
// of live entries over the lower / upper halves, a live base entry's place
// is its live rank in the row plus the inserted neighbours below it, and an
// inserted neighbour's place is its rank among the row's inserted ones plus
// the live base entries below it.
__global__ void k_rb_live(const int32_t *col, int64_t eb, uint32_t *flag) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < eb; i += stride) flag[i] = col[i] >= 0;
}
// live base entries per row plus its inserted neighbours
__global__ void k_rb_row_count(int32_t n, const uint32_t *bptr, const uint32_t *lptr, const uint32_t *LS,
                               const uint32_t *US, const uint32_t *ddeg, uint32_t *deg) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride)
        deg[u] = (LS[lptr[u + 1]] - LS[lptr[u]]) + (US[bptr[u + 1]] - US[bptr[u]]) + ddeg[u];
}
// number of keys in the row's sorted inserted neighbours pairs[q0, q0 + cnt) below x
__device__ __forceinline__ uint32_t ins_below(const uint64_t *pairs, uint64_t q0, uint32_t cnt, int32_t x) {
    uint32_t a = 0, b = cnt;
    while (a < b) {
        const uint32_t mid = (a + b) >> 1;
        if ((int32_t)(uint32_t)pairs[q0 + mid] < x) a = mid + 1;
        else b = mid;
    }
    return a;
}
// live entries of col[lo, hi) (ascending by id, deleted ones included) below y
__device__ __forceinline__ uint32_t live_below(const int32_t *col, const uint32_t *S, uint32_t lo, uint32_t hi,
                                               int32_t y) {
    uint32_t a = lo, b = hi;
    while (a < b) {
        const uint32_t mid = (a + b) >> 1;
        if ((col[mid] & COLMASK) < y) a = mid + 1;
        else b = mid;
    }
    return S[a] - S[lo];
}
__global__ void k_rb_fill_base(int32_t n, int64_t eb, const uint32_t *bptr, const int32_t *bcol,
                               const uint32_t *lptr, const int32_t *lcol, const uint32_t *LS, const uint32_t *US,
                               const uint64_t *pairs, const uint32_t *dstart, const uint32_t *ddeg,
                               const int64_t *row_ptr, int32_t *col) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < 2 * eb; t += stride) {
        const bool lower = t < eb;
        const int64_t j = lower ? t : t - eb;
        const int32_t x = lower ? lcol[j] : bcol[j];
        if (x < 0) continue;  // deleted
        int32_t u;
        uint32_t rank;
        if (lower) {
            u = row_of(lptr, n, j);
            rank = LS[j] - LS[lptr[u]];
        } else {
            u = row_of(bptr, n, j);
            rank = (LS[lptr[u + 1]] - LS[lptr[u]]) + (US[j] - US[bptr[u]]);
        }
        col[row_ptr[u] + rank + ins_below(pairs, dstart[u], ddeg[u], x)] = x;
    }
}
__global__ void k_rb_fill_ins(int32_t n, const uint32_t *bptr, const int32_t *bcol, const uint32_t *lptr,
                              const int32_t *lcol, const uint32_t *LS, const uint32_t *US, const uint64_t *pairs,
                              const unsigned long long *npairs, int64_t cap, const uint32_t *dstart,
                              const int64_t *row_ptr, int32_t *col) {
    const int64_t np = (int64_t)*npairs < cap ? (int64_t)*npairs : cap;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < np; q += stride) {
        const int32_t u = (int32_t)(pairs[q] >> 32), y = (int32_t)(uint32_t)pairs[q];
        const uint32_t below = live_below(lcol, LS, lptr[u], lptr[u + 1], y) +
                               live_below(bcol, US, bptr[u], bptr[u + 1], y);
        col[row_ptr[u] + (q - (int64_t)dstart[u]) + below] = y;
    }
}
void launch_rb_live(const int32_t *col, int64_t eb, uint32_t *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_rb_live, dim3(grid_for(eb, BLOCK, 1 << 16)), dim3(BLOCK), 0, s, col, eb, flag);
}
void launch_rb_row_count(int32_t n, const uint32_t *bptr, const uint32_t *lptr, const uint32_t *LS,
                         const uint32_t *US, const uint32_t *ddeg, uint32_t *deg, hipStream_t s) {
    hipLaunchKernelGGL(k_rb_row_count, dim3(grid_for(n, BLOCK, 1 << 14)), dim3(BLOCK), 0, s, n, bptr, lptr, LS,
                       US, ddeg, deg);
}
void launch_rb_fill(int32_t n, int64_t eb, const uint32_t *bptr, const int32_t *bcol, const uint32_t *lptr,
                    const int32_t *lcol, const uint32_t *LS, const uint32_t *US, const uint64_t *pairs,
                    const unsigned long long *npairs, int64_t cap, const uint32_t *dstart, const uint32_t *ddeg,
                    const int64_t *row_ptr, int32_t *col, hipStream_t s) {
    if (eb > 0)
        hipLaunchKernelGGL(k_rb_fill_base, dim3(grid_for(2 * eb, BLOCK, 1 << 16)), dim3(BLOCK), 0, s, n, eb, bptr,
                           bcol, lptr, lcol, LS, US, pairs, dstart, ddeg, row_ptr, col);
    hipLaunchKernelGGL(k_rb_fill_ins, dim3(grid_for(cap, BLOCK, 1 << 14)), dim3(BLOCK), 0, s, n, bptr, bcol, lptr,
                       lcol, LS, US, pairs, npairs, cap, dstart, row_ptr, col);
}

// ------------------------------------------------------------ digests

// Order-independent 64-bit digests of parent and label: wrap-around sums of
// a mix of (index, value) over the vertices.  out[0..1] must be zero.
__global__ __launch_bounds__(BLOCK) void k_digest(int32_t n, const int32_t *parent,
                                                  const int32_t *label, unsigned long long *out) {
    unsigned long long a = 0, b = 0;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride) {
        a += hmix(((uint64_t)i << 32) | (uint32_t)parent[i]);
        b += hmix(((uint64_t)i << 32) | (uint32_t)label[i]) ^ 0x9E3779B97F4A7C15ull;
    }
    a = block_sum64(a);
    b = block_sum64(b);
    if (threadIdx.x == 0) {
        atomicAdd(&out[0], a);
        atomicAdd(&out[1], b);
    }
}
void launch_digest(int32_t n, const int32_t *parent, const int32_t *label, unsigned long long *out,
                   hipStream_t s) {
    launch_fill_u64(out, 2, 0, s);
    hipLaunchKernelGGL(k_digest, dim3(grid_for(n, BLOCK, 512)), dim3(BLOCK), 0, s, n, parent, label, out);
}

// ======================================================= create-time kernels

__global__ void k_fill_i32(int32_t *p, int64_t count, int32_t v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}
__global__ void k_fill_u64(uint64_t *p, int64_t count, uint64_t v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}
void launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t s) {
    if (count > 0)
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(count, BLOCK, GRID_CAP)), dim3(BLOCK), 0, s, p, count, v);
}
void launch_fill_u64(uint64_t *p, int64_t count, uint64_t v, hipStream_t s) {
    if (count > 0)
        hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(count, BLOCK, GRID_CAP)), dim3(BLOCK), 0, s, p, count, v);
}

// Create-time kernels walk the CSR's entries, not its rows, one thread per
// entry (its row by a search in the offsets): a power-law graph's hub rows
// hold hundreds of thousands of entries, and a wave per row left one wave
// walking a hub alone while the rest of the device idled.

// Every entry: id in range (of the row's graph), no self-loop, row strictly
// ascending.
__global__ __launch_bounds__(BLOCK) void k_csr_check(int32_t n, const int64_t *row_ptr, const int32_t *col,
                                                     int64_t nnz, int32_t *status, const int32_t *goff,
                                                     int32_t ngraph) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    int bad = 0;
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < nnz; j += stride) {
        const int32_t u = row_of(row_ptr, n, j);
        int32_t lo = 0, hi = n;
        if (goff) {  // graph of row u: largest g with goff[g] <= u
            int32_t a = 0, b = ngraph - 1;
            while (a < b) {
                const int32_t mid = a + ((b - a + 1) >> 1);
                if (goff[mid] <= u) a = mid; else b = mid - 1;
            }
            lo = goff[a];
            hi = goff[a + 1];
        }
        const int32_t c = col[j];
        if (c < lo || c >= hi || c == u) bad = 1;
        if (j + 1 < row_ptr[u + 1] && col[j + 1] <= c) bad = 1;
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(status, 1);
}
// Entries above the diagonal per row (rows ascending: one search each).
__global__ __launch_bounds__(BLOCK) void k_upper_counts(int32_t n, const int64_t *row_ptr, const int32_t *col,
                                                        uint32_t *ucnt) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t u = (int64_t)blockIdx.x * BLOCK + threadIdx.x; u < n; u += stride) {
        int64_t a = row_ptr[u], b = row_ptr[u + 1];
        const int64_t e = b;
        while (a < b) {  // first entry > u
            const int64_t mid = (a + b) >> 1;
            if (col[mid] <= (int32_t)u) a = mid + 1;
            else b = mid;
        }
        ucnt[u] = (uint32_t)(e - a);
    }
}
void launch_csr_check(int32_t n, const int64_t *row_ptr, const int32_t *col, int64_t nnz, uint32_t *ucnt,
                      int32_t *status, const int32_t *goff, int32_t ngraph, hipStream_t s) {
    if (nnz > 0)
        hipLaunchKernelGGL(k_csr_check, dim3(grid_for(nnz, BLOCK, 1 << 16)), dim3(BLOCK), 0, s, n, row_ptr, col,
                           nnz, status, goff, ngraph);
    hipLaunchKernelGGL(k_upper_counts, dim3(grid_for(n, BLOCK, 1 << 14)), dim3(BLOCK), 0, s, n, row_ptr, col,
                       ucnt);
}

// Every entry (u, c) must have its mirror (c, u).
__global__ __launch_bounds__(BLOCK) void k_csr_symmetric(int32_t n, const int64_t *row_ptr,
                                                         const int32_t *col, int32_t *status) {
    const int64_t nw = (int64_t)gridDim.x * (BLOCK / WAVE);
    const int lane = lane_id();
    for (int64_t u = (int64_t)blockIdx.x * (BLOCK / WAVE) + threadIdx.x / WAVE; u < n; u += nw) {
        const int64_t s = row_ptr[u], e = row_ptr[u + 1];
        for (int64_t j = s + lane; j < e; j += WAVE) {
            const int32_t c = col[j];
            if (c < 0 || c >= n) continue;  // reported by k_csr_check
            int64_t a = row_ptr[c], b = row_ptr[c + 1];
            while (a < b) {
                int64_t mid = a + ((b - a) >> 1);
                if (col[mid] < u) a = mid + 1; else b = mid;
            }
            if (!(a < row_ptr[c + 1] && col[a] == u)) atomicOr(status, 2);
        }
    }
}
void launch_csr_symmetric(int32_t n, const int64_t *row_ptr, const int32_t *col, int32_t *status,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_csr_symmetric, dim3(grid_for((int64_t)n * WAVE, BLOCK, GRID_CAP)),
                       dim3(BLOCK), 0, s, n, row_ptr, col, status);
}

// ---- exclusive scan of uint32 counts (three passes), with a 64-bit total
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_CHUNK = BLOCK * SCAN_ITEMS;

size_t scan_tmp_bytes(int64_t n) {
    return sizeof(unsigned long long) * (size_t)((n + SCAN_CHUNK - 1) / SCAN_CHUNK + 1);
}

__device__ unsigned long long block_scan_excl(unsigned long long x, unsigned long long *total) {
    __shared__ unsigned long long ws[BLOCK / WAVE];
    const int lane = lane_id(), wid = threadIdx.x / WAVE;
    unsigned long long inc = x;
    for (int o = 1; o < WAVE; o <<= 1) {
        unsigned long long y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == WAVE - 1) ws[wid] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < BLOCK / WAVE; w++) { unsigned long long s2 = ws[w]; ws[w] = t; t += s2; }
        *total = t;
    }
    __syncthreads();
    unsigned long long r = ws[wid] + inc - x;
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(BLOCK) void k_scan_sums(const uint32_t *in, int64_t n,
                                                     unsigned long long *bsum) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_ITEMS;
    unsigned long long s = 0;
    for (int j = 0; j < SCAN_ITEMS; j++)
        if (base + j < n) s += in[base + j];
    __shared__ unsigned long long tot;
    block_scan_excl(s, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}
__global__ __launch_bounds__(BLOCK) void k_scan_top(unsigned long long *bsum, int64_t nb,
                                                    unsigned long long *total) {
    __shared__ unsigned long long tot;
    unsigned long long carry = 0;
    for (int64_t base = 0; base < nb; base += BLOCK) {
        const int64_t i = base + threadIdx.x;
        unsigned long long x = i < nb ? bsum[i] : 0;
        unsigned long long ex = block_scan_excl(x, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}
__global__ __launch_bounds__(BLOCK) void k_scan_apply(const uint32_t *in, uint32_t *out, int64_t n,
                                                      const unsigned long long *bsum,
                                                      const unsigned long long *total) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_ITEMS;
    unsigned long long s = 0;
    uint32_t v[SCAN_ITEMS];
    for (int j = 0; j < SCAN_ITEMS; j++) {
        v[j] = base + j < n ? in[base + j] : 0;
        s += v[j];
    }
    __shared__ unsigned long long tot;
    unsigned long long off = bsum[blockIdx.x] + block_scan_excl(s, &tot);
    for (int j = 0; j < SCAN_ITEMS; j++) {
        if (base + j < n) out[base + j] = (uint32_t)off;
        off += v[j];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = (uint32_t)*total;
}
void launch_scan_u32(const uint32_t *in, uint32_t *out, unsigned long long *total, int64_t n,
                     void *tmp, hipStream_t s) {
    const int64_t nb = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
    unsigned long long *bsum = (unsigned long long *)tmp;
    if (nb > 0) hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(BLOCK), 0, s, in, n, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(BLOCK), 0, s, bsum, nb, total);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(BLOCK), 0, s, in, out,
                       n, bsum, total);
}

// copy the upper-half suffix of every (ascending) row, one thread per stored entry
__global__ __launch_bounds__(BLOCK) void k_upper_fill(int32_t n, const int64_t *row_ptr,
                                                      const int32_t *col, const uint32_t *bptr,
                                                      int32_t *bcol, int64_t eb) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x; p < eb; p += stride) {
        const int32_t u = row_of(bptr, n, p);
        const int64_t cntu = (int64_t)bptr[u + 1] - bptr[u];
        bcol[p] = col[row_ptr[u + 1] - cntu + (p - (int64_t)bptr[u])];
    }
}
void launch_upper_fill(int32_t n, const int64_t *row_ptr, const int32_t *col, const uint32_t *bptr,
                       int32_t *bcol, int64_t eb, hipStream_t s) {
    if (eb > 0)
        hipLaunchKernelGGL(k_upper_fill, dim3(grid_for(eb, BLOCK, 1 << 16)), dim3(BLOCK), 0, s, n, row_ptr, col,
                           bptr, bcol, eb);
}

// lower half: the prefix of every ascending row below the diagonal
__global__ void k_lower_counts(int32_t n, const int64_t *row_ptr, const uint32_t *bptr,
                               uint32_t *lcnt) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride)
        lcnt[u] = (uint32_t)((row_ptr[u + 1] - row_ptr[u]) - (int64_t)(bptr[u + 1] - bptr[u]));
}
void launch_lower_counts(int32_t n, const int64_t *row_ptr, const uint32_t *bptr, uint32_t *lcnt,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_lower_counts, dim3(grid_for(n, BLOCK, GRID_CAP)), dim3(BLOCK), 0, s, n, row_ptr,
                       bptr, lcnt);
}
__global__ __launch_bounds__(BLOCK) void k_lower_fill(int32_t n, const int64_t *row_ptr,
                                                      const int32_t *col, const uint32_t *lptr,
                                                      int32_t *lcol, int64_t eb) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x; q < eb; q += stride) {
        const int32_t v = row_of(lptr, n, q);
        lcol[q] = col[row_ptr[v] + (q - (int64_t)lptr[v])];
    }
}
void launch_lower_fill(int32_t n, const int64_t *row_ptr, const int32_t *col, const uint32_t *lptr,
                       int32_t *lcol, int64_t eb, hipStream_t s) {
    if (eb > 0)
        hipLaunchKernelGGL(k_lower_fill, dim3(grid_for(eb, BLOCK, 1 << 16)), dim3(BLOCK), 0, s, n, row_ptr, col,
                           lptr, lcol, eb);
}
// twin[p]: position in the lower half of the mirror of upper entry p (one
// thread per lower entry q = (v, u), u < v, finds v in upper row u)
__global__ __launch_bounds__(BLOCK) void k_twin(int32_t n, const uint32_t *bptr, const int32_t *bcol,
                                                const uint32_t *lptr, const int32_t *lcol,
                                                uint32_t *twin, uint32_t *ltwin, int32_t *status, int64_t eb) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x; q < eb; q += stride) {
        const int32_t v = row_of(lptr, n, q);
        const int32_t u = lcol[q];
        int32_t raw;
        const int64_t p = find_in_row(bcol, bptr[u], bptr[u + 1], v, &raw);
        if (p < 0) {
            atomicOr(status, 2);
        } else {
            twin[p] = (uint32_t)q;
            ltwin[q] = (uint32_t)p;
        }
    }
}
void launch_twin(int32_t n, const uint32_t *bptr, const int32_t *bcol, const uint32_t *lptr,
                 const int32_t *lcol, uint32_t *twin, uint32_t *ltwin, int32_t *status, int64_t eb, hipStream_t s) {
    if (eb > 0)
        hipLaunchKernelGGL(k_twin, dim3(grid_for(eb, BLOCK, 1 << 16)), dim3(BLOCK), 0, s, n, bptr, bcol, lptr,
                           lcol, twin, ltwin, status, eb);
}

// Non-empty-row index of the upper-half store (used by the sweep).
__global__ void k_nonempty_flags(int32_t n, const uint32_t *bptr, uint32_t *flag) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride)
        flag[u] = bptr[u + 1] > bptr[u] ? 1u : 0u;
}
__global__ void k_nonempty_fill(int32_t n, const uint32_t *bptr, const uint32_t *zpos, int32_t *zrow,
                                uint32_t *zptr, int64_t nz) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride)
        if (bptr[u + 1] > bptr[u]) {
            zrow[zpos[u]] = (int32_t)u;
            zptr[zpos[u]] = bptr[u];
        }
    if (blockIdx.x == 0 && threadIdx.x == 0) zptr[nz] = bptr[n];
}
void launch_nonempty_flags(int32_t n, const uint32_t *bptr, uint32_t *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_nonempty_flags, dim3(grid_for(n, BLOCK, GRID_CAP)), dim3(BLOCK), 0, s, n, bptr,
                       flag);
}
void launch_nonempty_fill(int32_t n, const uint32_t *bptr, const uint32_t *zpos, int32_t *zrow,
                          uint32_t *zptr, int64_t nz, hipStream_t s) {
    hipLaunchKernelGGL(k_nonempty_fill, dim3(grid_for(n, BLOCK, GRID_CAP)), dim3(BLOCK), 0, s, n, bptr,
                       zpos, zrow, zptr, nz);
}

// tile_k[t] = largest k with zptr[k] <= t * TILE; tile_k[ntiles] = nz - 1
__global__ void k_tile_k(const uint32_t *zptr, int64_t nz, int64_t eb, int32_t *tile_k,
                         int64_t ntiles) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t <= ntiles; t += stride) {
        if (t == ntiles) { tile_k[t] = (int32_t)(nz - 1); continue; }
        const int64_t e = t * TILE;
        int64_t a = 0, b = nz - 1;
        while (a < b) {
            const int64_t mid = a + ((b - a + 1) >> 1);
            if ((int64_t)zptr[mid] <= e) a = mid; else b = mid - 1;
        }
        tile_k[t] = (int32_t)a;
    }
}
void launch_tile_k(const uint32_t *zptr, int64_t nz, int64_t eb, int32_t *tile_k, int64_t ntiles,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_tile_k, dim3(grid_for(ntiles + 1, BLOCK)), dim3(BLOCK), 0, s, zptr, nz, eb,
                       tile_k, ntiles);
}

// parent ids in range; every parent edge is an edge of G
__global__ void k_forest_check(int32_t n, const uint32_t *bptr, const int32_t *bcol,
                               const int32_t *parent, int32_t *status, int edges) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const int32_t p = parent[v];
        if (p < 0 || p >= n) { atomicOr(status, 1); continue; }
        if (p == v || !edges) continue;
        const int32_t lo = p < v ? p : (int32_t)v, hi = p < v ? (int32_t)v : p;
        int32_t raw;
        if (find_in_row(bcol, bptr[lo], bptr[lo + 1], hi, &raw) < 0) atomicOr(status, 2);
    }
}
void launch_forest_check(int32_t n, const uint32_t *bptr, const int32_t *bcol, const int32_t *parent,
                         int32_t *status, int check_edges, hipStream_t s) {
    hipLaunchKernelGGL(k_forest_check, dim3(grid_for(n, BLOCK, GRID_CAP)), dim3(BLOCK), 0, s, n, bptr,
                       bcol, parent, status, check_edges);
}

__global__ void k_pointer_jump(int32_t n, const int32_t *in, int32_t *out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        out[v] = in[in[v]];
}
void launch_pointer_jump(int32_t n, const int32_t *in, int32_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_pointer_jump, dim3(grid_for(n, BLOCK, GRID_CAP)), dim3(BLOCK), 0, s, n, in, out);
}

// After k synchronous rounds jump[v] is the ancestor 2^k steps up (capped
// at the root): some jump[v] that is not a root means a vertex deeper than
// 2^k (one store per wave that finds one).
__global__ void k_deeper_than(int32_t n, const int32_t *jump, unsigned long long *flag) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool deep = false;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const int32_t a = jump[v];
        deep = deep || jump[a] != a;
    }
    if (__ballot(deep) != 0 && lane_id() == 0) *flag = 1;
}
void launch_deeper_than(int32_t n, const int32_t *jump, unsigned long long *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_deeper_than, dim3(grid_for(n, BLOCK, GRID_CAP)), dim3(BLOCK), 0, s, n, jump, flag);
}

// after enough jumping rounds every vertex of a tree points at its root; a
// vertex on or below a cycle does not
__global__ void k_roots_check(int32_t n, const int32_t *parent, const int32_t *root,
                              int32_t *status) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const int32_t r = root[v];
        if (parent[r] != r) atomicOr(status, 4);
    }
}
void launch_roots_check(int32_t n, const int32_t *parent, const int32_t *root, int32_t *status,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_roots_check, dim3(grid_for(n, BLOCK, GRID_CAP)), dim3(BLOCK), 0, s, n, parent,
                       root, status);
}

// no edge of G may join two trees (trees span components); one thread per
// stored entry
__global__ __launch_bounds__(BLOCK) void k_span_check(Dev d, const int32_t *root) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    int bad = 0;
    for (int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x; p < d.eb; p += stride) {
        const int32_t c = d.bcol[p];
        if (c < 0) continue;  // deleted (padding)
        if (root[c] != root[row_of(d.bptr, d.n, p)]) bad = 1;
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(d.status, 8);
}
void launch_span_check(const Dev &d, const int32_t *root, hipStream_t s) {
    if (d.eb > 0)
        hipLaunchKernelGGL(k_span_check, dim3(grid_for(d.eb, BLOCK, 1 << 16)), dim3(BLOCK), 0, s, d, root);
}

// label[r] <- smallest vertex of r's tree (label pre-filled with INT32_MAX),
// then every vertex copies its root's value
__global__ void k_tree_min(int32_t n, const int32_t *root, int32_t *label) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        min_i32(&label[root[v]], (int32_t)v);
}
__global__ void k_label_from_root(int32_t n, const int32_t *root, int32_t *label) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        if (root[v] != v) label[v] = label[root[v]];
}
void launch_tree_min(int32_t n, const int32_t *root, int32_t *label, hipStream_t s) {
    launch_fill_i32(label, n, 0x7fffffff, s);
    hipLaunchKernelGGL(k_tree_min, dim3(grid_for(n, BLOCK, GRID_CAP)), dim3(BLOCK), 0, s, n, root, label);
    hipLaunchKernelGGL(k_label_from_root, dim3(grid_for(n, BLOCK, GRID_CAP)), dim3(BLOCK), 0, s, n, root,
                       label);
}

// a tree whose root r is not its smallest vertex m is re-rooted at m
__global__ __launch_bounds__(BLOCK) void k_reroot_requests(Dev d, const int32_t *root) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < d.n; base += stride) {
        const int64_t v = base + threadIdx.x;
        bool emit = false;
        PathReq q;
        if (v < d.n && root[v] == v && d.label[v] != v) {
            emit = true;
            q.start = d.label[v]; q.newpar = d.label[v]; q.stop = (int32_t)v;
        }
        const int64_t slot = block_append(emit ? 1 : 0, &d.cnt[C_NR]);
        if (emit) {
            if (slot < d.pathcap) d.paths[slot] = q;
            else atomicOr(d.status, ST_CAPACITY);
        }
    }
}
void launch_reroot_requests(const Dev &d, const int32_t *root, hipStream_t s) {
    hipLaunchKernelGGL(k_reroot_requests, dim3(grid_for(d.n, BLOCK, GRID_CAP)), dim3(BLOCK), 0, s, d, root);
}

}  // namespace drsf
