// Stable device radix sort of 64-bit keys, alone or with 64-bit values
// (least significant digit first, 8-bit digits).  Used by the supergraph's
// reduction of cross edges to one per pair of trees (Sec. III-A: its
// parallel sorting step), by the Euler tour's child lists (Algorithm 3), and
// when the edge store is rebuilt.
//
// Every pass is three steps over tiles of SORT_TILE keys: a histogram of
// the pass's digit per tile (LDS atomics), an exclusive scan over
// (digit, tile) in digit-major order, which gives every (digit, tile) its
// first output position, and a stable scatter.  Inside a tile each wave
// takes a contiguous run of keys 64 at a time; lanes holding the same digit
// are found with eight ballots (one per digit bit), their order among
// themselves is their lane order, and a per-wave LDS count per digit
// carries the order across rounds and, by a prefix over the waves, across
// the tile.  Keys therefore keep their input order within a digit, which
// makes the passes compose into a sort.
//
// Before the passes one kernel computes the bits in which the keys differ;
// a pass whose digit is the same in every key does nothing.  Which buffer
// holds the keys after each pass is kept on the device, so the whole sort
// is a fixed kernel sequence without host reads (it can be captured), and a
// last kernel moves the result into the output buffer when the last pass
// that ran left it in the scratch buffer (or no pass ran).
#include <hip/hip_runtime.h>

#include "drsf_kernels.h"

namespace drsf {
namespace {

constexpr int SORT_ITEMS = 16;                    // keys per thread in a tile
constexpr int SORT_TILE = BLOCK * SORT_ITEMS;     // 4096
constexpr int WAVE_RUN = SORT_TILE / (BLOCK / WAVE);  // keys of one wave in a tile
constexpr int RADIX = 256;
constexpr int PASSES = 8;
static_assert(BLOCK == RADIX, "one thread per digit in the histogram and prefix steps");

// Scratch layout (each part 256-byte aligned): alternate keys [count],
// alternate values [count] (pairs only), per (digit, tile) counts and their
// exclusive prefix [RADIX * tiles + 1], scan partials, then the control
// words: OR and AND of all keys and the scan's total, and per pass the
// buffer holding the keys before it (-1 the input, 0 the output, 1 the
// alternate buffer).
struct SortScratch {
    uint64_t *kalt, *valt;
    uint32_t *cnt, *pre;
    void *scan_tmp;
    unsigned long long *orand;  // [3]: OR, AND, scan total
    int32_t *cur;               // [PASSES + 1]
};

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t tiles_of(int64_t count) { return (count + SORT_TILE - 1) / SORT_TILE; }

size_t layout(int64_t count, bool pairs, void *tmp, SortScratch *o) {
    const int64_t T = tiles_of(count);
    const size_t sz[7] = {sizeof(uint64_t) * (size_t)count,
                          pairs ? sizeof(uint64_t) * (size_t)count : 0,
                          sizeof(uint32_t) * (size_t)(RADIX * T),
                          sizeof(uint32_t) * (size_t)(RADIX * T + 1),
                          scan_tmp_bytes(RADIX * T) + 64,
                          3 * sizeof(unsigned long long),
                          sizeof(int32_t) * (PASSES + 1)};
    size_t off[7], total = 0;
    for (int k = 0; k < 7; k++) {
        off[k] = total;
        total += al256(sz[k]);
    }
    if (o) {
        char *b = static_cast<char *>(tmp);
        o->kalt = reinterpret_cast<uint64_t *>(b + off[0]);
        o->valt = pairs ? reinterpret_cast<uint64_t *>(b + off[1]) : nullptr;
        o->cnt = reinterpret_cast<uint32_t *>(b + off[2]);
        o->pre = reinterpret_cast<uint32_t *>(b + off[3]);
        o->scan_tmp = b + off[4];
        o->orand = reinterpret_cast<unsigned long long *>(b + off[5]);
        o->cur = reinterpret_cast<int32_t *>(b + off[6]);
    }
    return total;
}

__global__ __launch_bounds__(BLOCK) void k_sort_init(unsigned long long *orand, int32_t *cur) {
    if (threadIdx.x == 0) {
        orand[0] = 0;
        orand[1] = ~0ull;
    }
    if (threadIdx.x <= PASSES) cur[threadIdx.x] = -1;
}

// OR and AND of every key: the bits that differ are OR ^ AND
__global__ __launch_bounds__(BLOCK) void k_sort_bits(const uint64_t *in, int64_t count, unsigned long long *orand) {
    unsigned long long o = 0, a = ~0ull;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < count; i += stride) {
        const uint64_t k = in[i];
        o |= k;
        a &= k;
    }
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        o |= __shfl_xor(o, off);
        a &= __shfl_xor(a, off);
    }
    __shared__ unsigned long long so[BLOCK / WAVE], sa[BLOCK / WAVE];
    const int w = threadIdx.x / WAVE;
    if (lane_id() == 0) {
        so[w] = o;
        sa[w] = a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < BLOCK / WAVE; k++) {
            o |= so[k];
            a &= sa[k];
        }
        atomicOr(&orand[0], o);
        atomicAnd(&orand[1], a);
    }
}

__device__ __forceinline__ bool pass_skipped(const unsigned long long *orand, int shift) {
    return (((orand[0] ^ orand[1]) >> shift) & (RADIX - 1)) == 0;
}

// Histogram of the pass's digit per tile; the first workgroup also records
// where the keys will be after the pass.
__global__ __launch_bounds__(BLOCK) void k_sort_hist(const uint64_t *in, const uint64_t *out, const uint64_t *kalt,
                                                     int64_t count, int pass, const unsigned long long *orand,
                                                     int32_t *cur, uint32_t *cnt) {
    const int shift = 8 * pass;
    const bool skip = pass_skipped(orand, shift);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int32_t c = cur[pass];
        cur[pass + 1] = skip ? c : (c == 0 ? 1 : 0);
    }
    if (skip) return;
    const int32_t c = cur[pass];
    const uint64_t *src = c < 0 ? in : c == 0 ? out : kalt;
    __shared__ uint32_t h[RADIX];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    for (int i = 0; i < SORT_ITEMS; i++) {
        const int64_t k = base + (int64_t)i * BLOCK + threadIdx.x;
        if (k < count) atomicAdd(&h[(src[k] >> shift) & (RADIX - 1)], 1u);
    }
    __syncthreads();
    cnt[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile (see the file comment).
template <bool PAIRS>
__global__ __launch_bounds__(BLOCK) void k_sort_scatter(const uint64_t *kin, uint64_t *kout, uint64_t *kalt,
                                                        const uint64_t *vin, uint64_t *vout, uint64_t *valt,
                                                        int64_t count, int pass, const unsigned long long *orand,
                                                        const int32_t *cur, const uint32_t *pre) {
    const int shift = 8 * pass;
    if (pass_skipped(orand, shift)) return;
    const int32_t cs = cur[pass], cd = cur[pass + 1];
    const uint64_t *ks = cs < 0 ? kin : cs == 0 ? kout : kalt;
    uint64_t *kd = cd == 0 ? kout : kalt;
    const uint64_t *vs = PAIRS ? (cs < 0 ? vin : cs == 0 ? vout : valt) : nullptr;
    uint64_t *vd = PAIRS ? (cd == 0 ? vout : valt) : nullptr;
    __shared__ uint32_t wcnt[BLOCK / WAVE][RADIX];  // per wave: keys of each digit seen so far
    const int w = threadIdx.x / WAVE, lane = lane_id();
    for (int k = threadIdx.x; k < (BLOCK / WAVE) * RADIX; k += BLOCK) (&wcnt[0][0])[k] = 0;
    __syncthreads();
    const int64_t run = (int64_t)blockIdx.x * SORT_TILE + (int64_t)w * WAVE_RUN;
    uint64_t key[SORT_ITEMS], val[SORT_ITEMS];
    uint32_t dr[SORT_ITEMS];  // digit << 16 | rank within the wave's run
    const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; r++) {
        const int64_t i = run + (int64_t)r * WAVE + lane;
        const bool valid = i < count;
        key[r] = valid ? ks[i] : 0;
        if (PAIRS) val[r] = valid ? vs[i] : 0;
        const uint32_t d = (uint32_t)(key[r] >> shift) & (RADIX - 1);
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const uint64_t bal = __ballot((d >> b) & 1u);
            same &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t before = wcnt[w][d];  // every lane reads before the group's leader writes
        const uint32_t rank = before + (uint32_t)__popcll(same & lt);
        if (valid && (same & lt) == 0) wcnt[w][d] = before + (uint32_t)__popcll(same);
        dr[r] = valid ? (d << 16) | rank : 0xffffffffu;
    }
    __syncthreads();
    {  // digit d: tile offset plus the keys of d in earlier waves
        const int d = threadIdx.x;
        uint32_t acc = pre[(int64_t)d * gridDim.x + blockIdx.x];
        for (int k = 0; k < BLOCK / WAVE; k++) {
            const uint32_t c = wcnt[k][d];
            wcnt[k][d] = acc;
            acc += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; r++) {
        if (dr[r] == 0xffffffffu) continue;
        const uint32_t d = dr[r] >> 16;
        const int64_t pos = (int64_t)wcnt[w][d] + (dr[r] & 0xffffu);
        kd[pos] = key[r];
        if (PAIRS) vd[pos] = val[r];
    }
}

// Moves the result into the output buffers unless the last pass that ran
// wrote it there.
__global__ __launch_bounds__(BLOCK) void k_sort_final(const uint64_t *kin, uint64_t *kout, const uint64_t *kalt,
                                                      const uint64_t *vin, uint64_t *vout, const uint64_t *valt,
                                                      int64_t count, const int32_t *cur) {
    const int32_t c = cur[PASSES];
    if (c == 0) return;
    const uint64_t *ks = c < 0 ? kin : kalt;
    const uint64_t *vs = c < 0 ? vin : valt;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < count; i += stride) {
        kout[i] = ks[i];
        if (vout) vout[i] = vs[i];
    }
}

int sort_impl(const uint64_t *kin, uint64_t *kout, const uint64_t *vin, uint64_t *vout, int64_t count, void *tmp,
              size_t tmp_bytes, hipStream_t s) {
    if (count <= 0) return 0;
    if (count >= ((int64_t)1 << 31) || kin == kout || (vout && vin == vout)) return -1;
    const bool pairs = vout != nullptr;
    SortScratch w;
    if (!tmp || layout(count, pairs, tmp, &w) > tmp_bytes) return -1;
    const int64_t T = tiles_of(count);
    const unsigned long long *orand = w.orand;
    hipLaunchKernelGGL(k_sort_init, dim3(1), dim3(BLOCK), 0, s, w.orand, w.cur);
    hipLaunchKernelGGL(k_sort_bits, dim3(grid_for(count, BLOCK * 4)), dim3(BLOCK), 0, s, kin, count, w.orand);
    for (int p = 0; p < PASSES; p++) {
        hipLaunchKernelGGL(k_sort_hist, dim3((unsigned)T), dim3(BLOCK), 0, s, kin, (const uint64_t *)kout,
                           (const uint64_t *)w.kalt, count, p, orand, w.cur, w.cnt);
        launch_scan_u32(w.cnt, w.pre, w.orand + 2, RADIX * T, w.scan_tmp, s);
        if (pairs)
            hipLaunchKernelGGL(k_sort_scatter<true>, dim3((unsigned)T), dim3(BLOCK), 0, s, kin, kout, w.kalt, vin,
                               vout, w.valt, count, p, orand, (const int32_t *)w.cur, (const uint32_t *)w.pre);
        else
            hipLaunchKernelGGL(k_sort_scatter<false>, dim3((unsigned)T), dim3(BLOCK), 0, s, kin, kout, w.kalt,
                               (const uint64_t *)nullptr, (uint64_t *)nullptr, (uint64_t *)nullptr, count, p,
                               orand, (const int32_t *)w.cur, (const uint32_t *)w.pre);
    }
    hipLaunchKernelGGL(k_sort_final, dim3(grid_for(count, BLOCK)), dim3(BLOCK), 0, s, kin, kout,
                       (const uint64_t *)w.kalt, vin, vout, (const uint64_t *)w.valt, count, (const int32_t *)w.cur);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

size_t sort_u64_tmp_bytes(int64_t count) { return layout(count > 0 ? count : 1, false, nullptr, nullptr); }

int launch_sort_u64(const uint64_t *in, uint64_t *out, int64_t count, void *tmp, size_t tmp_bytes, hipStream_t s) {
    return sort_impl(in, out, nullptr, nullptr, count, tmp, tmp_bytes, s);
}

size_t sort_pairs_u64_tmp_bytes(int64_t count) { return layout(count > 0 ? count : 1, true, nullptr, nullptr); }

int launch_sort_pairs_u64(const uint64_t *kin, uint64_t *kout, const uint64_t *vin, uint64_t *vout, int64_t count,
                          void *tmp, size_t tmp_bytes, hipStream_t s) {
    if (!vin || !vout) return -1;
    return sort_impl(kin, kout, vin, vout, count, tmp, tmp_bytes, s);
}

}  // namespace drsf
