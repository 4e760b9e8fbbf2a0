// Small graphs of a multi-graph context, each updated whole by one
// workgroup (the batched pattern).  A persistent kernel takes graphs from a
// device work queue (one atomic per graph); a workgroup runs every step of
// Algorithm 1 for its graph with the forest held in LDS (parent, component
// and a scratch array as 16-bit local ids, the per-component minima as
// 32-bit words: 10 bytes per vertex) while the graph's edges stream from
// HBM, with block barriers between the steps and no grid-wide barrier.
// It runs beside the kernel chain that updates the context's large graphs
// (a separate branch of the captured update); results are staged and
// written into parent/label by a commit kernel after both branches end,
// since the chain's per-vertex kernels read the parents of every vertex in
// the blocks they visit.
//
// A small graph keeps its edges as an array of 32-bit keys (u << 16 | v,
// u < v, local ids; n <= 16384, so bit 31 is free) in no particular order,
// in one of two buffers: an insert appends the batch in place, a delete
// writes the surviving keys into the other buffer and flips.  Steps per
// graph (local ids):
//   1. parents into LDS; the batch normalised to keys; ids in range and no
//      self-loop;
//   2. validation against a hash set of the batch keys (open addressing in
//      LDS, or in HBM when the batch is too large for it): no repeated pair,
//      insert of an absent / delete of a present edge, found by one pass
//      over the edge array that also drops the deleted keys — a rejected
//      batch changes nothing;
//   3. deletes: cut (parent[c] = c for the child end of a deleted tree edge);
//   4. pieces: roots of F-hat by pointer jumping in LDS;
//   5-6. replacement edges: Boruvka rounds over components with LDS atomic
//      minima of the edge keys (lowest key leaving each component; a mutual
//      pair is recorded once), hooks applied after every selection, then
//      pointer jumping — the Kruskal forest, as in the chain.  The first
//      round reads the candidates, the batch (insert) or every surviving
//      edge (delete), and keeps those whose ends lie in different pieces
//      (the cross edges, Sec. II-A); every round keeps the edges still
//      leaving a component for the next;
//   7. labels: smallest vertex per final component;
//   8. orientation: the super-forest of pieces over the replacement edges
//      is searched level by level from each component's super-root piece
//      (the piece holding its smallest vertex), each other piece's path
//      from its attach vertex to its root is reversed (paths are
//      vertex-disjoint, Lemma 4), and the super-root piece is re-rooted at
//      the smallest vertex.
#include <hip/hip_runtime.h>

#include "drsf_kernels.h"

namespace drsf {
namespace {

constexpr uint32_t SK_INF = 0xffffffffu;
constexpr int MAX_WAVES = 16;  // up to 1024 threads per workgroup
constexpr int UNROLL = 8;      // edge-array loads a thread keeps in flight
constexpr int ER_REGS = 4;     // replacement edges a thread holds in registers during the level search

__device__ __forceinline__ int nthreads() { return (int)blockDim.x; }

__device__ __forceinline__ uint32_t skey(int32_t a, int32_t b) {
    return a < b ? ((uint32_t)a << 16) | (uint32_t)b : ((uint32_t)b << 16) | (uint32_t)a;
}
__device__ __forceinline__ int32_t sk_lo(uint32_t k) { return (int32_t)(k >> 16); }
__device__ __forceinline__ int32_t sk_hi(uint32_t k) { return (int32_t)(k & 0xffffu); }

// dynamic LDS for T vertices: P, C, H (int16) then B (uint32, 4-byte aligned)
__host__ __device__ constexpr size_t lds_bytes_for(int T) { return 6 * (size_t)((T + 1) & ~1) + 4 * (size_t)T; }

struct Shared {
    int32_t err;  // a bound was exceeded (corrupt forest): the update fails
    uint32_t wsum[MAX_WAVES];
    int32_t task;
    int32_t flag;
    uint32_t word[4];
};

// Exclusive sum of one count per thread over the block, in thread order;
// every thread calls it.  *total = the sum of all counts.
__device__ uint32_t block_excl_sum(uint32_t x, Shared &sh, uint32_t *total) {
    const int w = threadIdx.x / WAVE, nw = nthreads() / WAVE;
    uint32_t inc = x;
    for (int of = 1; of < WAVE; of <<= 1) {
        const uint32_t y = __shfl_up(inc, of);
        if (lane_id() >= of) inc += y;
    }
    if (lane_id() == WAVE - 1) sh.wsum[w] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int q = 0; q < nw; q++) {
        const uint32_t c = sh.wsum[q];
        before += q < w ? c : 0;
        tot += c;
    }
    __syncthreads();
    *total = tot;
    return before + inc - x;
}

// Appends the keys of this wave's lanes that have `keep` set to out at
// positions claimed from the counter *cnt (one LDS atomic per wave), in no
// particular order.
__device__ __forceinline__ void wave_append(bool keep, uint32_t k, uint32_t *out, uint32_t *cnt) {
    const uint64_t m = __ballot(keep);
    if (m == 0) return;
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(cnt, (uint32_t)__popcll(m));
    base = __shfl(base, 0);
    if (keep) out[base + lanes_below(m)] = k;
}

// Hash set of edge keys by open addressing over nch chunks of 4 slots
// (16-byte aligned): a key's probe sequence starts at the first slot of its
// home chunk (the high half of mix(k) * nch) and runs on slot by slot, so a
// lookup reads whole chunks with one 16-byte load and stops at the first
// chunk that holds the key or an empty slot.  Whole chunks keep the probe
// count of a wave (its slowest lane) low at half load.  The mix is the
// "lowbias32" integer hash (C. Wellons, hash-prospector).  A slot holds
// HS_EMPTY or a key; bit 31 marks the key as found.
constexpr uint32_t HS_EMPTY = 0xffffffffu, HS_FOUND = 0x80000000u, HS_KEY = 0x7fffffffu;
__device__ __forceinline__ uint32_t hs_home(uint32_t k, uint32_t nch) {
    k ^= k >> 16;
    k *= 0x7feb352du;
    k ^= k >> 15;
    k *= 0x846ca68bu;
    k ^= k >> 16;
    return (uint32_t)(((uint64_t)k * nch) >> 32);
}
// Adds k; false when k is already there.  The table never fills (at most
// half its slots are used), so the probe ends; 4 nch probes bound it anyway.
__device__ __forceinline__ bool hs_add(uint32_t *tab, uint32_t nch, uint32_t k) {
    uint32_t h = 4 * hs_home(k, nch);
    for (uint32_t p = 0; p < 4 * nch; p++) {
        const uint32_t old = atomicCAS(&tab[h], HS_EMPTY, k);
        if (old == HS_EMPTY) return true;
        if ((old & HS_KEY) == k) return false;
        h = h + 1 == 4 * nch ? 0 : h + 1;
    }
    return true;
}
// Slot holding k, or -1 (the table is not written meanwhile).  A chunk is
// tested without branches (selects, and a max for "holds an empty slot"):
// the loop body is a few instructions, run by the wave until its slowest
// lane is done.
__device__ __forceinline__ int hs_find(const uint32_t *tab, uint32_t nch, uint32_t k) {
    uint32_t c = hs_home(k, nch);
    int at = -1;
    for (uint32_t p = 0; p < nch; p++) {
        const uint4 q = *reinterpret_cast<const uint4 *>(tab + 4 * c);
        const int base = (int)(4 * c);
        at = (q.w & HS_KEY) == k ? base + 3 : -1;
        at = (q.z & HS_KEY) == k ? base + 2 : at;
        at = (q.y & HS_KEY) == k ? base + 1 : at;
        at = (q.x & HS_KEY) == k ? base : at;
        const uint32_t mx = max(max(q.x, q.y), max(q.z, q.w));  // HS_EMPTY is the largest word
        if (at >= 0 || mx == HS_EMPTY) break;
        c = c + 1 == nch ? 0 : c + 1;
    }
    return at;
}

// Pointer jumping on X[0, n) until every entry is a root (X[X[v]] == X[v]);
// a forest needs at most log2(n) + 1 rounds, so 40 bound it.
__device__ void jump_all(int16_t *X, int n, Shared &sh) {
    for (int round = 0;; round++) {
        if (round == 40) {
            if (threadIdx.x == 0) sh.err = 1;
            __syncthreads();
            break;
        }
        if (threadIdx.x == 0) sh.flag = 0;
        __syncthreads();
        bool changed = false;
        for (int v = threadIdx.x; v < n; v += nthreads()) {
            const int16_t x = X[v], y = X[x];
            if (x != y) {
                X[v] = y;
                changed = true;
            }
        }
        if (changed) sh.flag = 1;
        __syncthreads();
        const int f = sh.flag;
        __syncthreads();
        if (!f) break;
    }
}

// One graph's update (see the file comment).  Every thread of the block
// calls it.  tab_lds: 16-byte aligned LDS after P (lds_chunks chunks of 4
// words), free until step 4; t: the task's position in the queue.
__device__ void small_task(const Dev &d, const SmallDev &s, const int t, const int4 tk, Shared &sh, int16_t *P,
                           int16_t *C, int16_t *H, uint32_t *B, uint32_t *tab_lds, uint32_t lds_chunks) {
    const int sidx = tk.x, op = tk.w;
    const int64_t bstart = tk.y;
    const int blen = tk.z;
    const int nt = nthreads();
    const int32_t g = s.sgid[sidx];
    const int32_t o = d.goff[g];
    const int n = d.goff[g + 1] - o;
    const int64_t cap = s.scap[sidx];
    const int cur = s.sbuf[sidx];
    const int m = s.sm[sidx];
    uint32_t *E = s.pool + s.soff[sidx] + (int64_t)cur * cap;
    uint32_t *E2 = s.pool + s.soff[sidx] + (int64_t)(1 - cur) * cap;
    uint32_t *X = s.xk + s.soff[sidx], *Y = X + cap;  // surviving candidate edges, two lists
    const int64_t vo = s.svoff[sidx];
    int2 *ER = s.er + vo;
    const Ctl *hc = d.hctl;
    const int32_t *be = hc->edges ? hc->edges : d.bedges;
    uint32_t *ka = s.bkeys + bstart;

    // 1. parents, batch keys, range checks
    for (int v = threadIdx.x; v < n; v += nt) P[v] = (int16_t)(d.parent[o + v] - o);
    if (threadIdx.x == 0) {
        sh.flag = 0;
        sh.err = 0;
        sh.word[0] = 0;
    }
    __syncthreads();
    int bad = 0;
    for (int i = threadIdx.x; i < blen; i += nt) {
        const int32_t u = be[2 * (bstart + i)] - o, v = be[2 * (bstart + i) + 1] - o;
        if (u < 0 || v < 0 || u >= n || v >= n || u == v) {
            bad |= ST_BAD_PAIR;
            ka[i] = 0;
        } else {
            ka[i] = skey(u, v);
        }
    }
    if (bad) atomicOr(&sh.flag, bad);
    __syncthreads();

    // 2. validation with a hash set of the batch keys: in LDS when twice
    // the batch fits, else in the task's 2 blen + 4 words of the HBM table
    // (two inlined copies, so that the LDS one uses LDS instructions)
    auto validate = [&](uint32_t *tab, const uint32_t nch) {
        const uint32_t S = 4 * nch;
        for (uint32_t k = threadIdx.x; k < S; k += nt) tab[k] = HS_EMPTY;
        __syncthreads();
        int bad2 = 0;
        for (int i = threadIdx.x; i < blen; i += nt)
            if (!hs_add(tab, nch, ka[i])) bad2 |= ST_DUPLICATE;
        if (bad2) atomicOr(&sh.flag, bad2);
        __syncthreads();
        // one pass over the edge array: inserts must meet no batch key;
        // deletes mark the batch keys they meet and keep the other keys
        bad2 = 0;
        const int span = nt * UNROLL;
        const int mm = (m + span - 1) / span * span;  // whole block rounds: the waves append together
        for (int j0 = threadIdx.x; j0 < mm; j0 += span) {
            uint32_t kk[UNROLL];  // loads issued together, then used
#pragma unroll
            for (int r = 0; r < UNROLL; r++) kk[r] = j0 + r * nt < m ? E[j0 + r * nt] : HS_EMPTY;
#pragma unroll
            for (int r = 0; r < UNROLL; r++) {
                const bool in = j0 + r * nt < m;
                const int at = in ? hs_find(tab, nch, kk[r]) : -1;
                if (op == 0) {
                    if (at >= 0) bad2 |= ST_EXISTS;
                } else {
                    if (at >= 0) atomicOr(&tab[at], HS_FOUND);
                    wave_append(in && at < 0, kk[r], E2, &sh.word[0]);
                }
            }
        }
        if (bad2) atomicOr(&sh.flag, bad2);
        __syncthreads();
        if (op == 1) {  // every batch key must have been met
            bad2 = 0;
            for (uint32_t k = threadIdx.x; k < S; k += nt) {
                const uint32_t x = tab[k];
                if (x != HS_EMPTY && !(x & HS_FOUND)) bad2 |= ST_MISSING;
            }
            if (bad2) atomicOr(&sh.flag, bad2);
            __syncthreads();
        }
    };
    if (sh.flag == 0 && blen > 0) {
        if (2 * (int64_t)blen <= 4 * (int64_t)lds_chunks) {
            validate(tab_lds, lds_chunks);
        } else {  // words [2 bstart + 4 t, 2 (bstart + blen) + 4 (t + 1)) are the task's: tasks come in batch order
            const int64_t w0 = (2 * bstart + 4 * (int64_t)t + 3) & ~(int64_t)3;  // 16-byte aligned
            validate(s.htab + w0, (uint32_t)((2 * (bstart + blen) + 4 * ((int64_t)t + 1) - w0) / 4));
        }
    }
    const int status = sh.flag;
    const int m2 = op == 0 ? m + blen : (blen > 0 ? (int)sh.word[0] : m);
    __syncthreads();
    if (status) {
        if (threadIdx.x == 0) {
            d.gstat[g] = status;
            s.sok[sidx] = 0;
        }
        __syncthreads();
        return;
    }
    if (op == 0 && (int64_t)m + blen > cap) {  // the host grows the buffers first: a corrupt count
        if (threadIdx.x == 0) {
            atomicOr(d.status, ST_WALK_BOUND);
            s.sok[sidx] = 0;
        }
        __syncthreads();
        return;
    }
    // the new edge array: inserts append the batch in place; an empty
    // delete keeps the array where it is
    const bool flip = op == 1 && blen > 0;
    if (op == 0)
        for (int i = threadIdx.x; i < blen; i += nt) E[m + i] = ka[i];

    // 3. cut the deleted tree edges
    if (op == 1) {
        for (int i = threadIdx.x; i < blen; i += nt) {
            const int32_t u = sk_lo(ka[i]), v = sk_hi(ka[i]);
            if (P[u] == v) P[u] = (int16_t)u;
            else if (P[v] == u) P[v] = (int16_t)v;
        }
    }
    __syncthreads();

    // 4. pieces: C = root of each vertex in F-hat
    for (int v = threadIdx.x; v < n; v += nt) C[v] = P[v];
    __syncthreads();
    jump_all(C, n, sh);

    // 5-6. replacement edges: Boruvka rounds (C holds component links,
    // every entry a root at the start of a round; piece roots are the
    // initial components).  A round reads list L, keeps the edges whose
    // ends lie in different components (appended to `out`, the next
    // round's L) and takes each component's lowest such key.
    uint32_t ner = 0, nx = 0;
    const uint32_t *L = op == 0 ? ka : (flip ? E2 : E);
    int live = op == 0 ? blen : m2;
    uint32_t *out = X, *spare = Y;
    for (int round = 0;; round++) {
        // each round at least halves the components with a live edge; err is
        // read by every thread before any can set it again
        const int e = sh.err;
        __syncthreads();
        if (round == 40 || e) {
            if (threadIdx.x == 0) sh.err = 1;
            break;
        }
        for (int v = threadIdx.x; v < n; v += nt) B[v] = SK_INF;
        if (threadIdx.x == 0) sh.word[1] = 0;
        __syncthreads();
        const int span = nt * UNROLL;
        const int lr = (live + span - 1) / span * span;
        for (int j0 = threadIdx.x; j0 < lr; j0 += span) {
            uint32_t kk[UNROLL];
#pragma unroll
            for (int r = 0; r < UNROLL; r++) kk[r] = j0 + r * nt < live ? L[j0 + r * nt] : 0u;
#pragma unroll
            for (int r = 0; r < UNROLL; r++) {
                const uint32_t k = kk[r];
                const int32_t cu = C[sk_lo(k)], cv = C[sk_hi(k)];
                const bool keep = j0 + r * nt < live && cu != cv;
                if (keep) {
                    atomicMin(&B[cu], k);
                    atomicMin(&B[cv], k);
                }
                wave_append(keep, k, out, &sh.word[1]);
            }
        }
        __syncthreads();
        live = (int)sh.word[1];
        if (round == 0) nx = (uint32_t)live;
        // select: H[c] = component c hooks onto (or c); record each chosen edge once
        uint32_t got = 0;
        for (int c = threadIdx.x; c < n; c += nt) {
            H[c] = (int16_t)c;
            const uint32_t k = B[c];
            if (k == SK_INF || C[c] != c) continue;
            const int32_t cx = C[sk_lo(k)], cy = C[sk_hi(k)];
            const int32_t other = cx == c ? cy : cx;
            const bool mutual = B[other] == k;
            if (!mutual || c > other) H[c] = (int16_t)other;
            if (!mutual || c < other) got++;
        }
        // ranks of this thread's recorded edges: record them in a second pass
        uint32_t tot;
        uint32_t before = block_excl_sum(got, sh, &tot);
        for (int c = threadIdx.x; c < n; c += nt) {
            const uint32_t k = B[c];
            if (k == SK_INF || C[c] != c) continue;
            const int32_t cx = C[sk_lo(k)], cy = C[sk_hi(k)];
            const int32_t other = cx == c ? cy : cx;
            if (!(B[other] == k) || c < other) ER[ner + before++] = make_int2(sk_lo(k), sk_hi(k));
        }
        __syncthreads();
        if (tot == 0) break;
        ner += tot;
        for (int c = threadIdx.x; c < n; c += nt)
            if (H[c] != c) C[c] = H[c];
        __syncthreads();
        jump_all(C, n, sh);
        L = out;
        out = spare;
        spare = const_cast<uint32_t *>(L);
    }

    // 7. labels: smallest vertex of each final component (B[root])
    for (int v = threadIdx.x; v < n; v += nt) B[v] = SK_INF;
    __syncthreads();
    for (int v = threadIdx.x; v < n; v += nt) atomicMin(&B[C[v]], (uint32_t)v);
    __syncthreads();
    for (int v = threadIdx.x; v < n; v += nt) s.slab[vo + v] = (int32_t)B[C[v]] + o;

    // 8. orientation, all in LDS.  H = piece root of each vertex (F-hat,
    // unchanged by the hooking); a super-root piece (the piece holding its
    // component's smallest vertex) is marked by H[root] = -root - 1.  Then B
    // and C, no longer needed (the labels are staged), hold each piece
    // root's search level and the replacement edge it was reached through.
    for (int v = threadIdx.x; v < n; v += nt) H[v] = P[v];
    __syncthreads();
    jump_all(H, n, sh);
    for (int v = threadIdx.x; v < n; v += nt)
        if (C[v] == v) {  // a final component: its smallest vertex is B[v]
            const int32_t sr = H[B[v]];
            H[sr] = (int16_t)(-sr - 1);
        }
    __syncthreads();
    int32_t *LV = reinterpret_cast<int32_t *>(B);
    int16_t *PE = C;
    for (int v = threadIdx.x; v < n; v += nt) LV[v] = H[v] < 0 ? 0 : -1;
    __syncthreads();
    // the piece pair of each of this thread's first ER_REGS replacement
    // edges, held in registers across the levels (0: used up)
    auto piece_pair = [&](int e) {
        const int2 xy = ER[e];
        int32_t pa = H[xy.x], pb = H[xy.y];
        if (pa < 0) pa = -pa - 1;
        if (pb < 0) pb = -pb - 1;
        return ((uint32_t)pa << 16) | (uint32_t)pb | 0x80000000u;
    };
    uint32_t pp[ER_REGS];
#pragma unroll
    for (int r = 0; r < ER_REGS; r++) {
        const int e = threadIdx.x + r * nt;
        pp[r] = e < (int)ner ? piece_pair(e) : 0u;
    }
    // one level: an edge with one end at level lvl and the other unreached
    // attaches the other end's piece
    auto visit = [&](uint32_t q, int e, int lvl) {
        const int32_t pa = (int32_t)((q >> 16) & 0x7fffu), pb = (int32_t)(q & 0xffffu);
        const int32_t la = LV[pa], lb = LV[pb];
        if (la == lvl && lb < 0) {
            LV[pb] = lvl + 1;
            PE[pb] = (int16_t)e;  // attach vertex y, new parent x
            return true;
        }
        if (lb == lvl && la < 0) {
            LV[pa] = lvl + 1;
            PE[pa] = (int16_t)(-e - 1);  // attach vertex x, new parent y
            return true;
        }
        return false;
    };
    for (int lvl = 0; lvl <= n; lvl++) {  // a super-tree has fewer levels than vertices
        if (threadIdx.x == 0) sh.flag = 0;
        __syncthreads();
        bool any = false;
#pragma unroll
        for (int r = 0; r < ER_REGS; r++)
            if (pp[r] && visit(pp[r], threadIdx.x + r * nt, lvl)) {
                pp[r] = 0;  // an edge attaches one piece, once
                any = true;
            }
        for (int e = threadIdx.x + ER_REGS * nt; e < (int)ner; e += nt)
            if (visit(piece_pair(e), e, lvl)) any = true;
        if (any) sh.flag = 1;
        __syncthreads();
        const int f = sh.flag;
        __syncthreads();
        if (!f) break;
    }
    // reversals: one thread per attached piece, plus the re-rooting of each
    // super-root piece whose root is not its component's smallest vertex
    uint32_t npaths = 0;
    for (int v = threadIdx.x; v < n; v += nt) {
        if (H[v] != v && H[v] != -v - 1) continue;  // v is a piece root
        int32_t start, newpar;
        if (LV[v] > 0) {
            const int32_t pe = PE[v];
            const int2 xy = ER[pe >= 0 ? pe : -pe - 1];
            start = pe >= 0 ? xy.y : xy.x;
            newpar = pe >= 0 ? xy.x : xy.y;
        } else if (H[v] < 0) {  // super-root piece: re-rooted at the component's smallest vertex
            start = s.slab[vo + v] - o;
            if (start == v) continue;
            newpar = start;
        } else {
            continue;
        }
        npaths++;
        int32_t prev = newpar, x = start;
        for (int k = 0;; k++) {
            if (k > n) {  // no path from the attach vertex to its piece root
                sh.err = 1;
                break;
            }
            const int32_t nx2 = P[x];
            P[x] = (int16_t)prev;
            if (x == v) break;
            prev = x;
            x = nx2;
        }
    }
    __syncthreads();
    if (sh.err) {  // a corrupt forest: the update fails (the graph is not committed)
        if (threadIdx.x == 0) {
            atomicOr(d.status, ST_WALK_BOUND);
            s.sok[sidx] = 0;
        }
        __syncthreads();
        return;
    }
    for (int v = threadIdx.x; v < n; v += nt) s.spar[vo + v] = (int32_t)P[v] + o;
    // counters of the update (all graphs of the context add up)
    // (own counters: the chain running beside uses C_NER and C_NR as list lengths)
    if (npaths) atomicAdd(&d.cnt[C_SNR], (unsigned long long)npaths);
    if (threadIdx.x == 0) {
        s.sok[sidx] = 1;
        s.sm[sidx] = m2;
        s.sbuf[sidx] = flip ? 1 - cur : cur;
        atomicAdd(&d.cnt[C_SNER], (unsigned long long)ner);
        atomicAdd(&d.cnt[C_SNCROSS], (unsigned long long)nx);
    }
    __syncthreads();
}

__global__ __launch_bounds__(1024) void k_small_update(Dev d, SmallDev s) {
    extern __shared__ unsigned char smem[];
    __shared__ Shared sh;
    const int T = s.T;
    int16_t *P = reinterpret_cast<int16_t *>(smem);
    int16_t *C = P + T;
    int16_t *H = C + T;
    uint32_t *B = reinterpret_cast<uint32_t *>(smem + 6 * (size_t)((T + 1) & ~1));
    // after P, 16-byte aligned: C, H and B, free until the pieces are formed
    const size_t tab0 = (2 * (size_t)T + 15) & ~(size_t)15;
    uint32_t *tab = reinterpret_cast<uint32_t *>(smem + tab0);
    const uint32_t tab_chunks = (uint32_t)((lds_bytes_for(T) - tab0) / 16);
    const int ntask = d.hctl->nsmall;
    while (true) {
        if (threadIdx.x == 0) sh.task = (int32_t)atomicAdd(s.qhead, 1u);
        __syncthreads();
        const int t = sh.task;
        __syncthreads();
        if (t >= ntask) break;
        small_task(d, s, t, s.tasks[t], sh, P, C, H, B, tab, tab_chunks);
    }
}

// After both branches: staged parents and labels of the updated small
// graphs into the context's arrays (rep == label between updates), and the
// work queue reset for the next update.  alone: every graph of the context
// is small, so no kernel sequence ran: this kernel also publishes the
// update's control block, clears the batch's hash-slot marks and marks the
// update finished, as the sequence's kernels would, for the cleanup.
__global__ __launch_bounds__(BLOCK) void k_small_commit(Dev d, SmallDev s, int alone) {
    const int ntask = d.hctl->nsmall;
    if (blockIdx.x == 0 && threadIdx.x == 0) *s.qhead = 0;
    if (alone) {
        const Ctl *hc = d.hctl;
        if (blockIdx.x == 0 && threadIdx.x < sizeof(Ctl) / 8)
            reinterpret_cast<uint64_t *>(d.ctlw)[threadIdx.x] = reinterpret_cast<const uint64_t *>(hc)[threadIdx.x];
        if (blockIdx.x == 0 && threadIdx.x == 0) d.cnt[C_ORIENTED] = 1;
        for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < hc->b; i += (int64_t)gridDim.x * BLOCK)
            d.bslot[i] = NONE;
    }
    for (int t = blockIdx.x; t < ntask; t += gridDim.x) {
        const int sidx = s.tasks[t].x;
        if (!s.sok[sidx]) continue;
        const int32_t g = s.sgid[sidx];
        const int32_t o = d.goff[g];
        const int n = d.goff[g + 1] - o;
        const int64_t vo = s.svoff[sidx];
        for (int v = threadIdx.x; v < n; v += BLOCK) {
            const int32_t lab = s.slab[vo + v];
            d.parent[o + v] = s.spar[vo + v];
            d.label[o + v] = lab;
            d.rep[o + v] = lab;
        }
    }
}

// Pool growth: every small graph's live keys (buffer sbuf, sm keys) copied
// to the start of its region in the new pool (new offsets in noff), one
// workgroup per graph.
__global__ __launch_bounds__(BLOCK) void k_small_regrow(SmallDev s, const int64_t *noff, uint32_t *npool) {
    for (int sidx = blockIdx.x; sidx < s.nsg; sidx += gridDim.x) {
        const uint32_t *src = s.pool + s.soff[sidx] + (int64_t)s.sbuf[sidx] * s.scap[sidx];
        uint32_t *dst = npool + noff[sidx];
        const int m = s.sm[sidx];
        for (int j = threadIdx.x; j < m; j += BLOCK) dst[j] = src[j];
    }
}

// Create: a small graph's upper-half rows (u < v, ascending by u then v)
// become its key array in buffer 0; its entries in the context's edge store
// are marked deleted (the store then holds the large graphs only).
__global__ __launch_bounds__(BLOCK) void k_small_init(Dev d, SmallDev s) {
    for (int sidx = blockIdx.x; sidx < s.nsg; sidx += gridDim.x) {
        const int32_t g = s.sgid[sidx];
        const int32_t o = d.goff[g];
        const int n = d.goff[g + 1] - o;
        const uint32_t e0 = d.bptr[o], e1 = d.bptr[o + n];
        uint32_t *E = s.pool + s.soff[sidx];
        for (int u = threadIdx.x; u < n; u += BLOCK) {
            const uint32_t a = d.bptr[o + u], b = d.bptr[o + u + 1];
            for (uint32_t j = a; j < b; j++) {
                E[j - e0] = ((uint32_t)u << 16) | (uint32_t)(d.bcol[j] - o);
                d.bcol[j] = d.bcol[j] | TOMB;
            }
            const uint32_t la = d.lptr[o + u], lb = d.lptr[o + u + 1];
            for (uint32_t j = la; j < lb; j++) d.lcol[j] = d.lcol[j] | TOMB;
        }
        if (threadIdx.x == 0) {
            s.sm[sidx] = (int32_t)(e1 - e0);
            s.sbuf[sidx] = 0;
            s.sok[sidx] = 0;
        }
    }
}

}  // namespace

size_t small_lds_bytes(int T) { return lds_bytes_for(T); }
size_t small_static_lds() { return sizeof(Shared); }

int small_prepare(int T) {
    return hipFuncSetAttribute((const void *)k_small_update, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)small_lds_bytes(T)) == hipSuccess
               ? 0
               : -1;
}
int launch_small_update(const Dev &d, const SmallDev &s, int threads, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_small_update, dim3(grid), dim3(threads), small_lds_bytes(s.T), st, d, s);
    return 0;
}
void launch_small_commit(const Dev &d, const SmallDev &s, int grid, bool alone, hipStream_t st) {
    hipLaunchKernelGGL(k_small_commit, dim3(grid), dim3(BLOCK), 0, st, d, s, alone ? 1 : 0);
}
void launch_small_regrow(const Dev &, const SmallDev &s, const int64_t *noff, uint32_t *npool, hipStream_t st) {
    hipLaunchKernelGGL(k_small_regrow, dim3(grid_for(s.nsg, 1, GRID_CAP)), dim3(BLOCK), 0, st, s, noff, npool);
}
void launch_small_init(const Dev &d, const SmallDev &s, hipStream_t st) {
    hipLaunchKernelGGL(k_small_init, dim3(grid_for(s.nsg, 1, GRID_CAP)), dim3(BLOCK), 0, st, d, s);
}

}  // namespace drsf
