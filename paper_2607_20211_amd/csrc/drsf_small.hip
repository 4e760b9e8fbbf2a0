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
// A small graph keeps its edges as one ascending array of 32-bit keys
// (u << 16 | v, u < v, local ids) in one of two buffers; an update writes
// the new array into the other buffer (merge for inserts, filter for
// deletes) and flips.  Steps per graph (local ids):
//   1. parents into LDS; the batch normalised to keys, sorted (LSD radix,
//      8-bit digits, stable wave-ballot ranking), checked: ids in range, no
//      self-loop, no repeated pair, insert of an absent / delete of a
//      present edge (binary search) — a rejected batch changes nothing;
//   2. new edge array (merge / filter);
//   3. deletes: cut (parent[c] = c for the child end of a deleted tree edge);
//   4. pieces: roots of F-hat by pointer jumping in LDS;
//   5. cross edges: the batch (insert) or every surviving edge (delete)
//      whose ends lie in different pieces (Sec. II-A);
//   6. replacement edges: Boruvka rounds over components with LDS atomic
//      minima of the edge keys (lowest key leaving each component; a mutual
//      pair is recorded once), hooks applied after every selection, then
//      pointer jumping — the Kruskal forest, as in the chain;
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

__device__ __forceinline__ int nthreads() { return (int)blockDim.x; }

__device__ __forceinline__ uint32_t skey(int32_t a, int32_t b) {
    return a < b ? ((uint32_t)a << 16) | (uint32_t)b : ((uint32_t)b << 16) | (uint32_t)a;
}
__device__ __forceinline__ int32_t sk_lo(uint32_t k) { return (int32_t)(k >> 16); }
__device__ __forceinline__ int32_t sk_hi(uint32_t k) { return (int32_t)(k & 0xffffu); }

// lanes of this wave holding the same 8-bit digit (among lanes with valid)
__device__ __forceinline__ uint64_t same_digit(uint32_t dgt, bool valid) {
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
        const uint64_t bal = __ballot((dgt >> b) & 1u);
        same &= ((dgt >> b) & 1u) ? bal : ~bal;
    }
    return same;
}

struct Shared {
    int32_t err;  // a bound was exceeded (corrupt forest): the update fails
    uint32_t hist[256];
    uint32_t wcnt[MAX_WAVES][256];
    uint32_t wsum[MAX_WAVES];
    int32_t task;
    int32_t flag;
    uint32_t word[4];
};

// Exclusive count of set flags over the block (in thread order); every
// thread calls it.  Returns this thread's position; *total = all set flags.
__device__ uint32_t block_rank(bool f, Shared &sh, uint32_t *total) {
    const uint64_t m = __ballot(f);
    const int w = threadIdx.x / WAVE, nw = nthreads() / WAVE;
    if (lane_id() == 0) sh.wsum[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int k = 0; k < nw; k++) {
        const uint32_t c = sh.wsum[k];
        before += k < w ? c : 0;
        tot += c;
    }
    __syncthreads();
    *total = tot;
    return before + (uint32_t)lanes_below(m);
}

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

// Keeps, in order, the keys of src[0, cnt) that `keep` accepts, written to
// dst (dst may be src: every key is read before a key lands at or below
// it); returns how many.  Each thread takes one contiguous share, counts,
// and writes after one block-wide sum (two barriers in all, where a pass
// per block-sized chunk costs two per chunk).  Every thread calls it.
template <class F>
__device__ uint32_t block_compact(const uint32_t *src, uint32_t *dst, int cnt, F keep, Shared &sh) {
    const int nt = nthreads();
    const int s0 = (int)((int64_t)cnt * threadIdx.x / nt), s1 = (int)((int64_t)cnt * (threadIdx.x + 1) / nt);
    uint32_t k = 0;
    for (int j = s0; j < s1; j++) k += keep(src[j]) ? 1u : 0u;
    uint32_t tot;
    uint32_t w = block_excl_sum(k, sh, &tot);
    for (int j = s0; j < s1; j++) {
        const uint32_t x = src[j];
        if (keep(x)) dst[w++] = x;
    }
    __syncthreads();
    return tot;
}

// Stable LSD radix sort of a[0, cnt) by the low `bits` bits, 8 bits a pass,
// with b as the other buffer; returns the buffer holding the result.  A
// pass takes the keys in chunks of SORT_ITEMS per thread: each wave ranks a
// contiguous run of its chunk 64 keys at a time (lanes with the same digit
// found by ballots, per-wave digit counts in LDS carrying the order from
// round to round), then a prefix over the waves gives each (wave, digit)
// its output base.
constexpr int SORT_ITEMS = 8;
__device__ uint32_t *block_sort(uint32_t *a, uint32_t *b, int cnt, int bits, Shared &sh) {
    const int nt = nthreads(), w = threadIdx.x / WAVE, nw = nt / WAVE;
    const uint64_t lt = (1ull << lane_id()) - 1ull;
    const int chunk = nt * SORT_ITEMS;
    for (int shift = 0; shift < bits; shift += 8) {
        for (int k = threadIdx.x; k < 256; k += nt) sh.hist[k] = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < cnt; i += nt) atomicAdd(&sh.hist[(a[i] >> shift) & 255u], 1u);
        __syncthreads();
        {  // exclusive prefix of the 256 digit counts (every thread calls the sum)
            const uint32_t c = threadIdx.x < 256 ? sh.hist[threadIdx.x] : 0u;
            uint32_t tot;
            const uint32_t e = block_excl_sum(c, sh, &tot);
            if (threadIdx.x < 256) sh.hist[threadIdx.x] = e;
        }
        for (int c0 = 0; c0 < cnt; c0 += chunk) {
            for (int k = threadIdx.x; k < MAX_WAVES * 256; k += nt) (&sh.wcnt[0][0])[k] = 0;
            __syncthreads();
            const int run0 = c0 + w * WAVE * SORT_ITEMS;
            uint32_t key[SORT_ITEMS], dr[SORT_ITEMS];  // digit << 16 | rank within the wave's run
#pragma unroll
            for (int r = 0; r < SORT_ITEMS; r++) {
                const int i = run0 + r * WAVE + lane_id();
                const bool valid = i < cnt;
                key[r] = valid ? a[i] : 0u;
                const uint32_t dg = (key[r] >> shift) & 255u;
                const uint64_t same = same_digit(dg, valid);
                const uint32_t before = sh.wcnt[w][dg];  // read by the group before its leader writes
                if (valid && (same & lt) == 0) sh.wcnt[w][dg] = before + (uint32_t)__popcll(same);
                dr[r] = valid ? (dg << 16) | (before + (uint32_t)__popcll(same & lt)) : 0xffffffffu;
            }
            __syncthreads();
            for (int k = threadIdx.x; k < 256; k += nt) {  // digit k: bases per wave, in wave order
                uint32_t run = sh.hist[k];
                for (int q = 0; q < nw; q++) {
                    const uint32_t c = sh.wcnt[q][k];
                    sh.wcnt[q][k] = run;
                    run += c;
                }
                sh.hist[k] = run;
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < SORT_ITEMS; r++)
                if (dr[r] != 0xffffffffu) b[sh.wcnt[w][dr[r] >> 16] + (dr[r] & 0xffffu)] = key[r];
            __syncthreads();
        }
        uint32_t *t = a;
        a = b;
        b = t;
    }
    return a;
}

// First position in a[0, m) holding a key >= k.
__device__ __forceinline__ int lower_bound(const uint32_t *a, int m, uint32_t k) {
    int lo = 0, hi = m;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Root of v under the component links C (16-bit local ids); at most n
// steps (more means a cycle, reported through err).
__device__ __forceinline__ int32_t cfind(const int16_t *C, int32_t v, int n, Shared &sh) {
    int32_t r = C[v];
    for (int k = 0; C[r] != r; k++) {
        if (k > n) {
            sh.err = 1;
            break;
        }
        r = C[r];
    }
    return r;
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
// calls it.
__device__ void small_task(const Dev &d, const SmallDev &s, const int4 tk, Shared &sh, int16_t *P, int16_t *C,
                           int16_t *H, uint32_t *B) {
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
    const uint32_t *E = s.pool + s.soff[sidx] + (int64_t)cur * cap;
    uint32_t *E2 = s.pool + s.soff[sidx] + (int64_t)(1 - cur) * cap;
    uint32_t *X = s.xk + s.soff[sidx] / 2;
    const int64_t vo = s.svoff[sidx];
    int2 *ER = s.er + vo;
    const Ctl *hc = d.hctl;
    const int32_t *be = hc->edges ? hc->edges : d.bedges;
    uint32_t *ka = s.bsort0 + bstart, *kb = s.bsort1 + bstart;
    // key bits: v in [0, lb), u in [16, 16 + lb)
    int lb = 1;
    while ((1 << lb) < n) lb++;
    const int bits = 16 + lb;

    // 1. parents, batch keys, validation
    for (int v = threadIdx.x; v < n; v += nt) P[v] = (int16_t)(d.parent[o + v] - o);
    if (threadIdx.x == 0) {
        sh.flag = 0;
        sh.err = 0;
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
    // the batch sorted, then merged with the edge array (merge path: each
    // thread takes an equal share of the merged order, found by one search,
    // and walks it; ties put the edge array's key first).  Walking the
    // merged order gives, with each key's neighbours there: repeated batch
    // pairs, inserts of present edges, deletes of absent ones, and the new
    // array (insert: the merged order; delete: the edge array's keys that
    // have no equal batch key next to them).
    const uint32_t *K = ka;
    if (sh.flag == 0) K = block_sort(ka, kb, blen, bits, sh);
    const int64_t L = (int64_t)m + blen;
    const int64_t d0 = L * threadIdx.x / nt, d1 = L * (threadIdx.x + 1) / nt;
    auto tE = [&](int i) { return (uint64_t)E[i] << 1; };
    auto tK = [&](int j) { return ((uint64_t)K[j] << 1) | 1u; };
    int i0 = 0;
    if (sh.flag == 0) {  // co-rank of d0: the edge-array keys among the first d0 of the merged order
        int lo = (int)(d0 - blen > 0 ? d0 - blen : 0), hi = (int)(d0 < m ? d0 : m);
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (tE(mid) < tK((int)(d0 - mid) - 1)) lo = mid + 1;
            else hi = mid;
        }
        i0 = lo;
    }
    // one walk of the share; pass 0 checks and counts, pass 1 (deletes) writes
    uint32_t kept = 0, keep_before = 0;
    for (int pass = 0; pass < 2; pass++) {
        if (sh.flag != 0) break;  // uniform: set before the last barrier
        if (pass == 1 && op == 0) break;
        int a = i0, c = (int)(d0 - i0);
        uint64_t prev = ~0ull;  // the element before the share in the merged order
        if (d0 > 0) {
            const uint64_t pe = a > 0 ? tE(a - 1) : 0, pk = c > 0 ? tK(c - 1) : 0;
            prev = pe > pk ? pe : pk;
        }
        bad = 0;
        uint32_t w = keep_before;
        for (int64_t dd = d0; dd < d1; dd++) {
            const bool fromE = c >= blen || (a < m && tE(a) < tK(c));
            const uint64_t x = fromE ? tE(a) : tK(c);
            if (fromE) a++; else c++;
            uint64_t nx = ~0ull;  // the element after x
            if (a < m || c < blen) {
                const uint64_t ne = a < m ? tE(a) : ~0ull, nk = c < blen ? tK(c) : ~0ull;
                nx = ne < nk ? ne : nk;
            }
            const bool eq_next = nx != ~0ull && (nx >> 1) == (x >> 1);
            const bool eq_prev = prev != ~0ull && (prev >> 1) == (x >> 1);
            if (pass == 0) {
                if (!fromE && eq_next && (nx & 1)) bad |= ST_DUPLICATE;
                if (op == 0) {
                    if (fromE && eq_next) bad |= ST_EXISTS;  // a batch key equal to an edge: right after it
                    E2[dd] = (uint32_t)(x >> 1);
                } else {
                    if (!fromE && !(eq_prev && !(prev & 1))) bad |= ST_MISSING;
                    if (fromE && !eq_next) kept++;
                }
            } else if (fromE && !eq_next) {
                E2[w++] = (uint32_t)(x >> 1);
            }
            prev = x;
        }
        if (pass == 0) {
            if (bad) atomicOr(&sh.flag, bad);
            uint32_t tot;  // the kept counts summed in thread order (barriers inside)
            keep_before = block_excl_sum(kept, sh, &tot);
            if (threadIdx.x == 0) sh.word[0] = tot;
            __syncthreads();
        }
    }
    const int status = sh.flag;
    const int m2 = op == 0 ? (int)L : (int)sh.word[0];
    __syncthreads();
    if (status) {
        if (threadIdx.x == 0) {
            d.gstat[g] = status;
            s.sok[sidx] = 0;
        }
        __syncthreads();
        return;
    }
    __syncthreads();

    // 3. cut the deleted tree edges
    if (op == 1) {
        for (int i = threadIdx.x; i < blen; i += nt) {
            const int32_t u = sk_lo(K[i]), v = sk_hi(K[i]);
            if (P[u] == v) P[u] = (int16_t)u;
            else if (P[v] == u) P[v] = (int16_t)v;
        }
        __syncthreads();
    }

    // 4. pieces: C = root of each vertex in F-hat
    for (int v = threadIdx.x; v < n; v += nt) C[v] = P[v];
    __syncthreads();
    jump_all(C, n, sh);

    // 5. cross edges into X
    const uint32_t *src = op == 0 ? K : E2;
    const int ns = op == 0 ? blen : m2;
    const uint32_t nx =
        block_compact(src, X, ns, [&](uint32_t k) { return C[sk_lo(k)] != C[sk_hi(k)]; }, sh);

    // 6. replacement edges: Boruvka rounds (C holds component links; piece
    // roots are the initial components)
    uint32_t ner = 0;
    int live = (int)nx;
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
        if (threadIdx.x == 0) sh.flag = 0;
        __syncthreads();
        for (int j = threadIdx.x; j < live; j += nt) {
            const uint32_t k = X[j];
            const int32_t cu = cfind(C, sk_lo(k), n, sh), cv = cfind(C, sk_hi(k), n, sh);
            if (cu != cv) {
                atomicMin(&B[cu], k);
                atomicMin(&B[cv], k);
            }
        }
        __syncthreads();
        // select: H[c] = component c hooks onto (or c); record each chosen edge once
        uint32_t got = 0;
        for (int c = threadIdx.x; c < n; c += nt) {
            H[c] = (int16_t)c;
            const uint32_t k = B[c];
            if (k == SK_INF || C[c] != c) continue;
            const int32_t cx = cfind(C, sk_lo(k), n, sh), cy = cfind(C, sk_hi(k), n, sh);
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
            const int32_t cx = cfind(C, sk_lo(k), n, sh), cy = cfind(C, sk_hi(k), n, sh);
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
        // drop edges inside one component
        live = (int)block_compact(X, X, live, [&](uint32_t k) { return C[sk_lo(k)] != C[sk_hi(k)]; }, sh);
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
    for (int lvl = 0; lvl <= n; lvl++) {  // a super-tree has fewer levels than vertices
        if (threadIdx.x == 0) sh.flag = 0;
        __syncthreads();
        bool any = false;
        for (int e = threadIdx.x; e < (int)ner; e += nt) {
            const int2 xy = ER[e];
            int32_t pa = H[xy.x], pb = H[xy.y];
            if (pa < 0) pa = -pa - 1;
            if (pb < 0) pb = -pb - 1;
            const int32_t la = LV[pa], lb = LV[pb];
            if (la == lvl && lb < 0) {
                LV[pb] = lvl + 1;
                PE[pb] = (int16_t)e;  // attach vertex y, new parent x
                any = true;
            } else if (lb == lvl && la < 0) {
                LV[pa] = lvl + 1;
                PE[pa] = (int16_t)(-e - 1);  // attach vertex x, new parent y
                any = true;
            }
        }
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
        s.sbuf[sidx] = 1 - cur;
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
    const int ntask = d.hctl->nsmall;
    while (true) {
        if (threadIdx.x == 0) sh.task = (int32_t)atomicAdd(s.qhead, 1u);
        __syncthreads();
        const int t = sh.task;
        __syncthreads();
        if (t >= ntask) break;
        small_task(d, s, s.tasks[t], sh, P, C, H, B);
    }
}

// After both branches: staged parents and labels of the updated small
// graphs into the context's arrays (rep == label between updates), and the
// work queue reset for the next update.
__global__ __launch_bounds__(BLOCK) void k_small_commit(Dev d, SmallDev s) {
    const int ntask = d.hctl->nsmall;
    if (blockIdx.x == 0 && threadIdx.x == 0) *s.qhead = 0;
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

size_t small_lds_bytes(int T) { return 6 * (size_t)((T + 1) & ~1) + 4 * (size_t)T; }

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
void launch_small_commit(const Dev &d, const SmallDev &s, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_small_commit, dim3(grid), dim3(BLOCK), 0, st, d, s);
}
void launch_small_init(const Dev &d, const SmallDev &s, hipStream_t st) {
    hipLaunchKernelGGL(k_small_init, dim3(grid_for(s.nsg, 1, GRID_CAP)), dim3(BLOCK), 0, st, d, s);
}

}  // namespace drsf
