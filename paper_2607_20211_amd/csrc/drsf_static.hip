// Static rebuild of a rooted spanning forest (the baseline the dynamic update
// is measured against, Sec. V's static GPU BFS): connected components by
// hooking, each rooted at its smallest vertex, then a breadth-first forest
// from all roots at once.  Kept apart from the update path; it shares only
// the small fill and grid helpers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <mutex>

#include "../../include/drsf.h"
#include "drsf_kernels.h"

namespace drsf {
namespace {

// Row of every CSR slot: the number of rows u >= 1 whose first slot is at
// or before it.  Each row u >= 1 counts 1 at its first slot (k_st_marks;
// empty rows share the next row's first slot), an exclusive sum over the
// slots follows, and the row of slot s is that sum plus its own count.
__global__ __launch_bounds__(BLOCK) void k_st_marks(int32_t n, const int64_t *row_ptr, int64_t nnz,
                                                    uint32_t *mark) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t u = 1 + (int64_t)blockIdx.x * BLOCK + threadIdx.x; u < n; u += stride) {
        const int64_t a = row_ptr[u];
        if (a < nnz) atomicAdd(&mark[a], 1u);
    }
}
__global__ __launch_bounds__(BLOCK) void k_st_rows(int64_t nnz, const uint32_t *mark, const uint32_t *excl,
                                                   int32_t *erow) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t s = (int64_t)blockIdx.x * BLOCK + threadIdx.x; s < nnz; s += stride)
        erow[s] = (int32_t)(excl[s] + mark[s]);
}

__global__ __launch_bounds__(BLOCK) void k_st_iota(int32_t n, int32_t *comp) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += stride) comp[v] = (int32_t)v;
}

// position of this lane's entry in a list counted by *cnt, one atomic per
// wave (every lane of the wave calls it)
__device__ __forceinline__ int64_t wave_append(bool take, unsigned long long *cnt) {
    const uint64_t m = __ballot(take);
    if (!m) return 0;
    const int leader = __ffsll((unsigned long long)m) - 1;
    unsigned long long base = 0;
    if (lane_id() == leader) base = atomicAdd(cnt, (unsigned long long)__popcll(m));
    base = __shfl(base, leader);
    return (int64_t)base + __popcll(m & ((1ull << lane_id()) - 1ull));
}

// Frontier appends gathered per workgroup: claims go to an LDS buffer (one
// LDS atomic per wave and call) and the workgroup reserves its whole run of
// the next frontier with one global atomic at the end; claims beyond the
// buffer fall back to a global append per wave.  Every atomic on the one
// frontier counter costs a serialised round trip, so per-wave appends from
// thousands of waves were most of a level's time.
constexpr int APP_BUF = 4096;
struct Appender {
    int32_t buf[APP_BUF];
    int n;
    unsigned long long base;
};
__device__ __forceinline__ void app_begin(Appender &a) {
    if (threadIdx.x == 0) a.n = 0;
    __syncthreads();
}
// every lane of the wave calls it
__device__ __forceinline__ void app_push(Appender &a, bool take, int32_t w, int32_t *next,
                                         unsigned long long *ncnt) {
    const uint64_t m = __ballot(take);
    if (!m) return;
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(&a.n, __popcll(m));
    base = __shfl(base, leader);
    const int pos = base + __popcll(m & ((1ull << lane_id()) - 1ull));
    const bool spill = take && pos >= APP_BUF;
    if (take && !spill) a.buf[pos] = w;
    if (base + __popcll(m) > APP_BUF) {  // wave-uniform
        const int64_t g = wave_append(spill, ncnt);
        if (spill) next[g] = w;
    }
}
// every thread of the workgroup calls it
__device__ __forceinline__ void app_end(Appender &a, int32_t *next, unsigned long long *ncnt) {
    __syncthreads();
    const int k = a.n < APP_BUF ? a.n : APP_BUF;
    if (threadIdx.x == 0 && k > 0) a.base = atomicAdd(ncnt, (unsigned long long)k);
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += BLOCK) next[a.base + i] = a.buf[i];
}

// Row lengths of the vertices a workgroup claimed, into the next level's
// degree sum and maximum (stat[0] sum, stat[1] max): each thread accumulates
// over its whole grid-stride loop, then one atomic pair per workgroup (every
// thread calls it once, at the end of the kernel).
__device__ __forceinline__ void block_degree(unsigned long long sum, unsigned long long mx,
                                             unsigned long long *stat) {
    __shared__ unsigned long long s_sum[BLOCK / WAVE], s_max[BLOCK / WAVE];
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        sum += __shfl_xor(sum, o);
        const unsigned long long y = __shfl_xor(mx, o);
        mx = y > mx ? y : mx;
    }
    if (lane_id() == 0) {
        s_sum[threadIdx.x / WAVE] = sum;
        s_max[threadIdx.x / WAVE] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0, m = 0;
        for (int w = 0; w < BLOCK / WAVE; w++) {
            t += s_sum[w];
            m = s_max[w] > m ? s_max[w] : m;
        }
        if (t) {
            atomicAdd(&stat[0], t);
            if (stat[1] < m) atomicMax(&stat[1], m);
        }
    }
}
__device__ __forceinline__ void add_degree(bool take, const int64_t *row_ptr, int32_t w, unsigned long long &sum,
                                           unsigned long long &mx) {
    if (!take) return;
    const unsigned long long dg = (unsigned long long)(row_ptr[w + 1] - row_ptr[w]);
    sum += dg;
    mx = dg > mx ? dg : mx;
}

// Level counters: three groups of four words, level L's in group L % 3
// (frontier size, row-length sum, longest row), then the depth word (the
// number of non-empty levels seen so far).  The kernel of level L reads group
// L % 3, fills group (L + 1) % 3 and clears group (L + 2) % 3 for the level
// after, so levels run back to back with no host step between them.
constexpr int CNT_WORDS = 13;
constexpr int CNT_DEPTH = 12;
__device__ __forceinline__ unsigned long long *level_group(unsigned long long *g, int L) { return g + 4 * (L % 3); }
__device__ __forceinline__ void level_begin(unsigned long long *g, int L, bool nonempty) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        unsigned long long *c = level_group(g, L + 2);
        c[0] = 0;
        c[1] = 0;
        c[2] = 0;
        if (nonempty) g[CNT_DEPTH] = (unsigned long long)(L + 1);
    }
}

__device__ __forceinline__ int32_t st_root(const int32_t *comp, int32_t x) {
    for (int32_t y = comp[x]; y != x; y = comp[x]) x = y;
    return x;
}

// Hooking: for every edge (u, v), u < v, whose ends have different roots, the
// larger root hooks onto the smaller (an atomic minimum), so every root only
// ever decreases and each component ends rooted at its smallest vertex.
__global__ __launch_bounds__(BLOCK) void k_st_hook(int64_t nnz, const int32_t *erow, const int32_t *col,
                                                   int32_t *comp, int32_t *changed) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    bool any = false;
    for (int64_t s = (int64_t)blockIdx.x * BLOCK + threadIdx.x; s < nnz; s += stride) {
        const int32_t u = erow[s], v = col[s];
        if (v <= u) continue;  // each undirected edge once
        const int32_t ru = st_root(comp, u), rv = st_root(comp, v);
        if (ru == rv) continue;
        const int32_t hi = ru > rv ? ru : rv, lo = ru > rv ? rv : ru;
        if (comp[hi] > lo) {
            atomicMin(&comp[hi], lo);
            any = true;
        }
    }
    if (__ballot(any) && lane_id() == 0) *changed = 1;
}

// pointer jumping to the roots
__global__ __launch_bounds__(BLOCK) void k_st_compress(int32_t n, int32_t *comp) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += stride)
        comp[v] = st_root(comp, (int32_t)v);
}

// roots: level 0, their own parents, the first frontier
__global__ __launch_bounds__(BLOCK) void k_st_bfs_init(int32_t n, const int64_t *row_ptr, const int32_t *comp,
                                                       int32_t *level, int32_t *parent, int32_t *front,
                                                       unsigned long long *g) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    unsigned long long *fcnt = level_group(g, 0), *fstat = fcnt + 1;
    __shared__ Appender app;
    app_begin(app);
    unsigned long long dsum = 0, dmax = 0;
    for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < n; base += stride) {
        const int64_t v = base + threadIdx.x;
        const bool root = v < n && comp[v] == (int32_t)v;
        if (v < n) {
            level[v] = root ? 0 : -1;
            parent[v] = root ? (int32_t)v : -1;
        }
        app_push(app, root, (int32_t)v, front, fcnt);
        add_degree(root, row_ptr, (int32_t)v, dsum, dmax);
    }
    app_end(app, front, fcnt);
    block_degree(dsum, dmax, fstat);
}

// Top-down level from a small frontier: each unvisited neighbour is claimed
// by a compare-and-swap on its level.  Rows of up to SHORT_ROW slots are
// walked by four lanes each (sixteen frontier vertices per wave, the wave
// looping to its longest such row); a longer row is walked by the whole wave.
constexpr int SHORT_ROW = 32;
__device__ __forceinline__ bool td_claim(const int32_t *col, int32_t *level, int32_t *parent, int L, int32_t v,
                                         int64_t s, int32_t &w) {
    w = col[s];
    const bool claim = level[w] < 0 && atomicCAS(&level[w], -1, L + 1) == -1;
    if (claim) parent[w] = v;
    return claim;
}
__global__ __launch_bounds__(BLOCK) void k_st_top_down(const int64_t *row_ptr, const int32_t *col,
                                                       int32_t *level, int32_t *parent, int L,
                                                       const int32_t *front, int32_t *next, unsigned long long *g) {
    const int64_t nf = (int64_t)*level_group(g, L);
    unsigned long long *ncnt = level_group(g, L + 1), *nstat = ncnt + 1;
    level_begin(g, L, nf > 0);
    __shared__ Appender app;
    app_begin(app);
    const int sub = lane_id() & 3;
    const int64_t step = (int64_t)gridDim.x * (BLOCK / WAVE) * (WAVE / 4);
    unsigned long long dsum = 0, dmax = 0;
    for (int64_t f0 = ((int64_t)blockIdx.x * (BLOCK / WAVE) + threadIdx.x / WAVE) * (WAVE / 4); f0 < nf;
         f0 += step) {
        const int64_t f = f0 + (lane_id() >> 2);
        int32_t v = 0;
        int64_t a = 0, b = 0;
        if (f < nf) {
            v = front[f];
            a = row_ptr[v];
            b = row_ptr[v + 1];
        }
        const bool big = b - a > SHORT_ROW;
        int rounds = big ? 0 : (int)((b - a + 3) >> 2);
        for (int o = WAVE / 2; o > 0; o >>= 1) {
            const int y = __shfl_xor(rounds, o);
            rounds = y > rounds ? y : rounds;
        }
        for (int r = 0; r < rounds; r++) {
            const int64_t sl = a + 4 * r + sub;
            bool claim = false;
            int32_t w = 0;
            if (!big && sl < b) claim = td_claim(col, level, parent, L, v, sl, w);
            app_push(app, claim, w, next, ncnt);
            add_degree(claim, row_ptr, w, dsum, dmax);
        }
        uint64_t bm = __ballot(big && sub == 0);
        while (bm) {
            const int l = __ffsll((unsigned long long)bm) - 1;
            bm &= bm - 1;
            const int32_t bv = __shfl(v, l);
            const int64_t ba = __shfl(a, l), bb = __shfl(b, l);
            for (int64_t s0 = ba; s0 < bb; s0 += WAVE) {
                const int64_t sl = s0 + lane_id();
                bool claim = false;
                int32_t w = 0;
                if (sl < bb) claim = td_claim(col, level, parent, L, bv, sl, w);
                app_push(app, claim, w, next, ncnt);
                add_degree(claim, row_ptr, w, dsum, dmax);
            }
        }
    }
    app_end(app, next, ncnt);
    block_degree(dsum, dmax, nstat);
}

// Edge-parallel level for a frontier with long rows but few edges: every
// slot (u, w) with u on level L claims w.
__global__ __launch_bounds__(BLOCK) void k_st_edges(int64_t nnz, const int64_t *row_ptr, const int32_t *erow,
                                                    const int32_t *col, int32_t *level, int32_t *parent, int L,
                                                    int32_t *next, unsigned long long *g) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    unsigned long long *ncnt = level_group(g, L + 1), *nstat = ncnt + 1;
    level_begin(g, L, true);
    __shared__ Appender app;
    app_begin(app);
    unsigned long long dsum = 0, dmax = 0;
    for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < nnz; base += stride) {
        const int64_t s = base + threadIdx.x;
        bool claim = false;
        int32_t w = 0;
        if (s < nnz) {
            const int32_t u = erow[s];
            if (level[u] == L) {
                w = col[s];
                claim = level[w] < 0 && atomicCAS(&level[w], -1, L + 1) == -1;
                if (claim) parent[w] = u;
            }
        }
        app_push(app, claim, w, next, ncnt);
        add_degree(claim, row_ptr, w, dsum, dmax);
    }
    app_end(app, next, ncnt);
    block_degree(dsum, dmax, nstat);
}

// Bottom-up level for a large frontier: every unvisited vertex looks along
// its row for a neighbour on level L and takes the first it meets as its
// parent (no atomics: a vertex writes only its own entries; the level L + 1
// it writes is never mistaken for L).
__global__ __launch_bounds__(BLOCK) void k_st_bottom_up(int32_t n, const int64_t *row_ptr, const int32_t *col,
                                                        int32_t *level, int32_t *parent, int L, int32_t *next,
                                                        unsigned long long *g) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    unsigned long long *ncnt = level_group(g, L + 1), *nstat = ncnt + 1;
    level_begin(g, L, true);
    __shared__ Appender app;
    app_begin(app);
    unsigned long long dsum = 0, dmax = 0;
    for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < n; base += stride) {
        const int64_t v = base + threadIdx.x;
        bool claim = false;
        if (v < n && level[v] < 0) {
            const int64_t b = row_ptr[v + 1];
            for (int64_t s = row_ptr[v]; s < b; s++) {
                const int32_t u = col[s];
                if (level[u] == L) {
                    parent[v] = u;
                    level[v] = L + 1;
                    claim = true;
                    break;
                }
            }
        }
        app_push(app, claim, (int32_t)v, next, ncnt);
        add_degree(claim, row_ptr, (int32_t)v, dsum, dmax);
    }
    app_end(app, next, ncnt);
    block_degree(dsum, dmax, nstat);
}

}  // namespace
}  // namespace drsf

using namespace drsf;

namespace {

// Scratch of one static rebuild: the row of every CSR slot and its marks,
// scan partials, breadth-first levels, two frontiers, the hooking flag and
// the level counters.
struct StaticScratch {
    int32_t *erow, *level, *front0, *front1, *flag;
    uint32_t *mark;
    void *stmp;
    unsigned long long *cnt;
};

// Device bytes of each scratch array, in StaticScratch order of carving.
void scratch_sizes(int32_t n, int64_t nnz, size_t sz[8]) {
    sz[0] = sizeof(int32_t) * (size_t)(nnz + 1);                       // erow
    sz[1] = sizeof(uint32_t) * (size_t)std::max<int64_t>(nnz, 1);      // mark
    sz[2] = scan_tmp_bytes(nnz) + 64;                                  // stmp
    sz[3] = sz[4] = sz[5] = sizeof(int32_t) * (size_t)n;              // level, front0, front1
    sz[6] = sizeof(int32_t);                                           // flag
    sz[7] = CNT_WORDS * sizeof(unsigned long long);                    // cnt
}

// The rebuild on given scratch; h: host memory for CNT_WORDS counters
// (pinned or not: every read of it follows a stream synchronisation).
int static_forest_core(int32_t n, const int64_t *row_ptr, const int32_t *col, int64_t nnz, int32_t *parent_out,
                       int32_t *label_out, hipStream_t s, int32_t *levels_out, const StaticScratch &w,
                       unsigned long long *h) {
    int32_t *erow = w.erow, *level = w.level, *front0 = w.front0, *front1 = w.front1, *flag = w.flag;
    uint32_t *mark = w.mark;
    void *stmp = w.stmp;
    unsigned long long *cnt = w.cnt;
    int rc = DRSF_OK;
    auto ok = [&](hipError_t e) {
        if (e != hipSuccess && rc == DRSF_OK) rc = DRSF_E_DEVICE;
        return e == hipSuccess;
    };
    int32_t *comp = label_out;
    const int gv = grid_for(n, BLOCK), ge = grid_for(nnz, BLOCK);
    if (nnz > 0) {  // row of every slot (the exclusive sums land in erow itself)
        launch_fill_i32(reinterpret_cast<int32_t *>(mark), nnz, 0, s);
        hipLaunchKernelGGL(k_st_marks, dim3(gv), dim3(BLOCK), 0, s, n, row_ptr, nnz, mark);
        launch_scan_u32(mark, reinterpret_cast<uint32_t *>(erow), cnt, nnz, stmp, s);
        hipLaunchKernelGGL(k_st_rows, dim3(ge), dim3(BLOCK), 0, s, nnz, mark,
                           reinterpret_cast<const uint32_t *>(erow), erow);
    }
    hipLaunchKernelGGL(k_st_iota, dim3(gv), dim3(BLOCK), 0, s, n, comp);
    // hooking rounds until nothing hooks (each round at least halves the
    // roots that still have an edge to another root)
    for (int round = 0; round < 64 && rc == DRSF_OK; round++) {
        launch_fill_i32(flag, 1, 0, s);
        hipLaunchKernelGGL(k_st_hook, dim3(ge), dim3(BLOCK), 0, s, nnz, erow, col, comp, flag);
        hipLaunchKernelGGL(k_st_compress, dim3(gv), dim3(BLOCK), 0, s, n, comp);
        if (!ok(hipMemcpyAsync(h, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s)) || !ok(hipStreamSynchronize(s)))
            break;
        if (*(int32_t *)h == 0) break;
        if (round == 63) rc = DRSF_E_DEVICE;
    }
    // breadth-first forest from the roots, a level at a time; the host
    // reads level L's counters and picks the kernel.  While the frontier's
    // rows are short and their sum is far below the switch point, up to
    // BATCH_MAX top-down levels are queued at once (the batch length
    // doubles while this keeps holding), so a deep graph with small
    // frontiers pays one host read per batch instead of per level; a
    // top-down level takes its frontier size from the device, so a batch
    // that outgrows its estimate stays correct, only slower.
    constexpr int BATCH_MAX = 64;
    launch_fill_u64(reinterpret_cast<uint64_t *>(cnt), CNT_WORDS, 0, s);
    hipLaunchKernelGGL(k_st_bfs_init, dim3(gv), dim3(BLOCK), 0, s, n, row_ptr, comp, level, parent_out, front0,
                       cnt);
    int32_t *fr[2] = {front0, front1};
    int L = 0, batch = 1;
    while (rc == DRSF_OK) {
        if (!ok(hipMemcpyAsync(h, cnt, CNT_WORDS * sizeof(unsigned long long), hipMemcpyDeviceToHost, s)) ||
            !ok(hipStreamSynchronize(s)))
            break;
        const unsigned long long *hg = h + 4 * (L % 3);
        const int64_t nf = (int64_t)hg[0], dsum = (int64_t)hg[1];
        const uint64_t dmax = hg[2];
        if (nf == 0) break;
        if (L > n) {  // more levels than vertices: the counters are wrong
            rc = DRSF_E_DEVICE;
            break;
        }
        if (dsum * 16 < nnz && dmax <= 4096) {
            // a frontier with few edges and short rows: top-down from its
            // own rows (four lanes per vertex; room for twice the frontier
            // in a batch)
            const int k = dsum * 256 < nnz ? batch : 1;
            const int g = (int)std::min<int64_t>(GRID_CAP, grid_for(std::max<int64_t>(2 * nf, 64) * 4, BLOCK));
            for (int i = 0; i < k; i++, L++)
                hipLaunchKernelGGL(k_st_top_down, dim3(g), dim3(BLOCK), 0, s, row_ptr, col, level, parent_out, L,
                                   fr[L & 1], fr[(L + 1) & 1], cnt);
            batch = k == batch ? std::min(2 * batch, BATCH_MAX) : 1;
        } else {
            // few edges but a long row: one pass over every slot; many
            // edges: bottom-up
            batch = 1;
            if (dsum * 16 < nnz)
                hipLaunchKernelGGL(k_st_edges, dim3(ge), dim3(BLOCK), 0, s, nnz, row_ptr, erow, col, level,
                                   parent_out, L, fr[(L + 1) & 1], cnt);
            else
                hipLaunchKernelGGL(k_st_bottom_up, dim3(gv), dim3(BLOCK), 0, s, n, row_ptr, col, level, parent_out,
                                   L, fr[(L + 1) & 1], cnt);
            L++;
        }
    }
    if (levels_out) *levels_out = rc == DRSF_OK ? (int32_t)h[CNT_DEPTH] : 0;
    if (rc == DRSF_OK && !ok(hipStreamSynchronize(s))) rc = DRSF_E_DEVICE;
    return rc;
}

// Reads row_ptr[n] (the CSR's entry count) on the stream.
int read_nnz(int32_t n, const int64_t *row_ptr, hipStream_t s, int64_t *nnz) {
    *nnz = 0;
    if (hipMemcpyAsync(nnz, row_ptr + n, sizeof *nnz, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        return DRSF_E_DEVICE;
    }
    return DRSF_OK;
}

// Scratch of the allocation-free entry point: one array per device, held
// until the process ends.  In host code its name only stands for the
// symbol; kernels get the device address that hipGetSymbolAddress returns
// for the device that is current.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of this device's scratch array, looked up once per device.
int scratch_address(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        (void)hipGetLastError();
        return DRSF_E_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return DRSF_E_DEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DRSF_OK;
}

}  // namespace

extern "C" int drsf_static_forest(int32_t n, const int64_t *row_ptr, const int32_t *col,
                                  int32_t *parent_out, int32_t *label_out, void *stream,
                                  int32_t *levels_out) {
    if (n < 0 || (n > 0 && (!row_ptr || !parent_out || !label_out))) return DRSF_E_ARG;
    if (n == 0) {
        if (levels_out) *levels_out = 0;
        return DRSF_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    int64_t nnz = 0;
    int rc = read_nnz(n, row_ptr, s, &nnz);
    if (rc) return rc;
    if (nnz < 0 || (nnz > 0 && !col)) return DRSF_E_ARG;
    size_t sz[8];
    scratch_sizes(n, nnz, sz);
    void *p[8] = {};
    unsigned long long *h = nullptr;
    bool got = true;
    for (int k = 0; k < 8 && got; k++) got = hipMalloc(&p[k], sz[k]) == hipSuccess;
    got = got && hipHostMalloc((void **)&h, CNT_WORDS * sizeof(unsigned long long)) == hipSuccess;
    if (!got) {
        (void)hipGetLastError();
        rc = DRSF_E_NOMEM;
    } else {
        const StaticScratch w{(int32_t *)p[0], (int32_t *)p[3], (int32_t *)p[4], (int32_t *)p[5],
                              (int32_t *)p[6], (uint32_t *)p[1], p[2], (unsigned long long *)p[7]};
        rc = static_forest_core(n, row_ptr, col, nnz, parent_out, label_out, s, levels_out, w, h);
    }
    (void)hipStreamSynchronize(s);
    for (void *q : p)
        if (q) (void)hipFree(q);
    if (h) (void)hipHostFree(h);
    return rc;
}

extern "C" int drsf_static_forest_noalloc(int32_t n, const int64_t *row_ptr, const int32_t *col,
                                          int32_t *parent_out, int32_t *label_out, void *stream,
                                          int32_t *levels_out) {
    if (n < 0 || (n > 0 && (!row_ptr || !parent_out || !label_out))) return DRSF_E_ARG;
    if (n == 0) {
        if (levels_out) *levels_out = 0;
        return DRSF_OK;
    }
    void *base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    int64_t nnz = 0;
    if ((rc = read_nnz(n, row_ptr, s, &nnz))) return rc;
    if (nnz < 0 || (nnz > 0 && !col)) return DRSF_E_ARG;
    if (nnz > ((int64_t)1 << 32)) return DRSF_E_CAPACITY;
    size_t sz[8], off[8], total = 0;
    scratch_sizes(n, nnz, sz);
    for (int k = 0; k < 8; k++) {  // each array 256-byte aligned inside the scratch
        off[k] = total;
        total += (sz[k] + 255) & ~(size_t)255;
    }
    if (total > NOALLOC_SCRATCH_BYTES) return DRSF_E_CAPACITY;
    unsigned char *b = static_cast<unsigned char *>(base);
    const StaticScratch w{(int32_t *)(b + off[0]), (int32_t *)(b + off[3]), (int32_t *)(b + off[4]),
                          (int32_t *)(b + off[5]), (int32_t *)(b + off[6]), (uint32_t *)(b + off[1]),
                          (void *)(b + off[2]), (unsigned long long *)(b + off[7])};
    unsigned long long h[CNT_WORDS] = {};  // pageable: each read follows a stream synchronisation
    rc = static_forest_core(n, row_ptr, col, nnz, parent_out, label_out, s, levels_out, w, h);
    (void)hipStreamSynchronize(s);
    return rc;
}
