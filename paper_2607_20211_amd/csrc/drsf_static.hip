// Static rebuild of a rooted spanning forest (the baseline the dynamic update
// is measured against, Sec. V's static GPU BFS): connected components by
// hooking, each rooted at its smallest vertex, then a breadth-first forest
// from all roots at once.  Kept apart from the update path; it shares only
// the small fill and grid helpers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>

#include "../../include/drsf.h"
#include "drsf_kernels.h"

namespace drsf {
namespace {

// row of every CSR slot (one wave per row)
__global__ __launch_bounds__(BLOCK) void k_st_rows(int32_t n, const int64_t *row_ptr, int32_t *erow) {
    const int64_t nw = (int64_t)gridDim.x * (BLOCK / WAVE);
    for (int64_t u = (int64_t)blockIdx.x * (BLOCK / WAVE) + threadIdx.x / WAVE; u < n; u += nw)
        for (int64_t s = row_ptr[u] + lane_id(); s < row_ptr[u + 1]; s += WAVE) erow[s] = (int32_t)u;
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
__global__ __launch_bounds__(BLOCK) void k_st_bfs_init(int32_t n, const int32_t *comp, int32_t *level,
                                                       int32_t *parent, int32_t *front,
                                                       unsigned long long *fcnt) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < n; base += stride) {
        const int64_t v = base + threadIdx.x;
        const bool root = v < n && comp[v] == (int32_t)v;
        if (v < n) {
            level[v] = root ? 0 : -1;
            parent[v] = root ? (int32_t)v : -1;
        }
        const int64_t pos = wave_append(root, fcnt);
        if (root) front[pos] = (int32_t)v;
    }
}

// Top-down level from a small frontier: one wave per frontier vertex claims
// its unvisited neighbours (compare-and-swap on the level).
__global__ __launch_bounds__(BLOCK) void k_st_top_down(const int64_t *row_ptr, const int32_t *col,
                                                       int32_t *level, int32_t *parent, int L,
                                                       const int32_t *front, const unsigned long long *fcnt,
                                                       int32_t *next, unsigned long long *ncnt) {
    const int64_t nf = (int64_t)*fcnt;
    const int64_t nw = (int64_t)gridDim.x * (BLOCK / WAVE);
    for (int64_t f = (int64_t)blockIdx.x * (BLOCK / WAVE) + threadIdx.x / WAVE; f < nf; f += nw) {
        const int32_t v = front[f];
        const int64_t a = row_ptr[v], b = row_ptr[v + 1];
        for (int64_t s0 = a; s0 < b; s0 += WAVE) {
            const int64_t s = s0 + lane_id();
            bool claim = false;
            int32_t w = 0;
            if (s < b) {
                w = col[s];
                claim = level[w] < 0 && atomicCAS(&level[w], -1, L + 1) == -1;
                if (claim) parent[w] = v;
            }
            const int64_t pos = wave_append(claim, ncnt);
            if (claim) next[pos] = w;
        }
    }
}

// Edge-parallel level for a large frontier: every slot (u, w) with u on
// level L claims w.
__global__ __launch_bounds__(BLOCK) void k_st_edges(int64_t nnz, const int32_t *erow, const int32_t *col,
                                                    int32_t *level, int32_t *parent, int L, int32_t *next,
                                                    unsigned long long *ncnt) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < nnz; base += stride) {
        const int64_t s = base + threadIdx.x;
        bool claim = false;
        int32_t w = 0, u = 0;
        if (s < nnz) {
            u = erow[s];
            if (level[u] == L) {
                w = col[s];
                claim = level[w] < 0 && atomicCAS(&level[w], -1, L + 1) == -1;
                if (claim) parent[w] = u;
            }
        }
        const int64_t pos = wave_append(claim, ncnt);
        if (claim) next[pos] = w;
    }
}

}  // namespace
}  // namespace drsf

using namespace drsf;

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
    if (hipMemcpyAsync(&nnz, row_ptr + n, sizeof nnz, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return DRSF_E_DEVICE;
    if (nnz < 0 || (nnz > 0 && !col)) return DRSF_E_ARG;
    int32_t *erow = nullptr, *level = nullptr, *front0 = nullptr, *front1 = nullptr, *flag = nullptr;
    unsigned long long *cnt = nullptr, *h = nullptr;
    int rc = DRSF_OK;
    auto ok = [&](hipError_t e) {
        if (e != hipSuccess && rc == DRSF_OK) rc = (e == hipErrorOutOfMemory) ? DRSF_E_NOMEM : DRSF_E_DEVICE;
        return e == hipSuccess;
    };
    if (ok(hipMalloc(&erow, sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1))) &&
        ok(hipMalloc(&level, sizeof(int32_t) * (size_t)n)) && ok(hipMalloc(&front0, sizeof(int32_t) * (size_t)n)) &&
        ok(hipMalloc(&front1, sizeof(int32_t) * (size_t)n)) && ok(hipMalloc(&flag, sizeof(int32_t))) &&
        ok(hipMalloc(&cnt, 3 * sizeof(unsigned long long))) &&
        ok(hipHostMalloc((void **)&h, 4 * sizeof(unsigned long long)))) {
        int32_t *comp = label_out;
        const int gv = grid_for(n, BLOCK), ge = grid_for(nnz, BLOCK), gw = grid_for((int64_t)n * WAVE, BLOCK);
        hipLaunchKernelGGL(k_st_rows, dim3(gw), dim3(BLOCK), 0, s, n, row_ptr, erow);
        hipLaunchKernelGGL(k_st_iota, dim3(gv), dim3(BLOCK), 0, s, n, comp);
        // hooking rounds until nothing hooks (each round at least halves the
        // roots that still have an edge to another root)
        for (int round = 0; round < 64 && rc == DRSF_OK; round++) {
            launch_fill_i32(flag, 1, 0, s);
            hipLaunchKernelGGL(k_st_hook, dim3(ge), dim3(BLOCK), 0, s, nnz, erow, col, comp, flag);
            hipLaunchKernelGGL(k_st_compress, dim3(gv), dim3(BLOCK), 0, s, n, comp);
            if (!ok(hipMemcpyAsync(h, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s)) ||
                !ok(hipStreamSynchronize(s)))
                break;
            if (*(int32_t *)h == 0) break;
            if (round == 63) rc = DRSF_E_DEVICE;
        }
        // breadth-first forest from the roots; cnt[L % 3] holds level L's
        // frontier size, cnt[(L + 1) % 3] collects the next
        launch_fill_u64(reinterpret_cast<uint64_t *>(cnt), 3, 0, s);
        hipLaunchKernelGGL(k_st_bfs_init, dim3(gv), dim3(BLOCK), 0, s, n, comp, level, parent_out, front0,
                           cnt);
        int32_t *fa = front0, *fb = front1;
        int L = 0;
        for (; rc == DRSF_OK; L++) {
            unsigned long long *fc = cnt + L % 3, *nc = cnt + (L + 1) % 3;
            if (!ok(hipMemcpyAsync(h, fc, sizeof(unsigned long long), hipMemcpyDeviceToHost, s)) ||
                !ok(hipStreamSynchronize(s)))
                break;
            const int64_t nf = (int64_t)h[0];
            if (nf == 0) break;
            launch_fill_u64(reinterpret_cast<uint64_t *>(cnt + (L + 2) % 3), 1, 0, s);
            if (nf * 4 < n) {  // small frontier: its own rows
                hipLaunchKernelGGL(k_st_top_down, dim3(grid_for(nf * WAVE, BLOCK)), dim3(BLOCK), 0, s, row_ptr,
                                   col, level, parent_out, L, fa, fc, fb, nc);
            } else {
                hipLaunchKernelGGL(k_st_edges, dim3(ge), dim3(BLOCK), 0, s, nnz, erow, col, level, parent_out, L,
                                   fb, nc);
            }
            std::swap(fa, fb);
            if (L > n) rc = DRSF_E_DEVICE;
        }
        if (levels_out) *levels_out = L;
        if (rc == DRSF_OK && !ok(hipStreamSynchronize(s))) rc = DRSF_E_DEVICE;
    }
    (void)hipStreamSynchronize(s);
    hipFree(erow);
    hipFree(level);
    hipFree(front0);
    hipFree(front1);
    hipFree(flag);
    hipFree(cnt);
    if (h) hipHostFree(h);
    return rc;
}
