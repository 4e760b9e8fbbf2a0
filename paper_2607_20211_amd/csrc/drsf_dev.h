// Device-side constants and helpers shared by the D-RSF kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace drsf {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;                 // 4 waves per workgroup
constexpr int32_t TOMB = (int32_t)0x80000000;  // high bit of a stored column: edge deleted
constexpr int32_t COLMASK = 0x7fffffff;
constexpr uint64_t KEY_INF = ~0ull;
constexpr uint64_t KEY_DEAD = ~0ull;       // deleted entry of the inserted-edge list
constexpr uint64_t HASH_EMPTY = ~0ull;
constexpr uint64_t HASH_TOMB_BIT = 1ull << 63;
constexpr int32_t NONE = -1;
constexpr int32_t CLAIMING = -2;

// Sweep tile: every thread of a 256-thread workgroup takes EPT consecutive
// stored edges, so one workgroup covers TILE edges.
constexpr int EPT = 16;
constexpr int TILE = BLOCK * EPT;

// status word bits (first failure wins nothing: bits accumulate)
enum : int32_t {
    ST_BAD_PAIR = 1,      // self-loop or id out of range
    ST_DUPLICATE = 2,     // edge repeated inside the batch
    ST_EXISTS = 4,        // insert of an existing edge
    ST_MISSING = 8,       // delete of a missing edge
    ST_WALK_BOUND = 16,   // a pointer chase exceeded n steps (corrupt forest)
    ST_ROUND_BOUND = 32,  // an iterative phase did not finish within its bound
    ST_CAPACITY = 64,     // an internal list overflowed its capacity
    ST_BATCH_MASK = 15,
};

// counters block (device int64 array) indices
enum : int {
    C_NP = 0,        // dense pieces registered
    C_NX0 = 1,       // cross-edge list length, buffer 0
    C_NX1 = 2,       // cross-edge list length, buffer 1
    C_NER = 3,       // replacement edges found
    C_NR = 4,        // paths to reverse
    C_NCROSS = 5,    // cross edges found by the key-edge scan (statistic)
    C_DONE_BOR = 6,  // replacement-edge rounds finished
    C_DONE_LR = 7,   // list ranking finished
    C_LR_ACTIVE0 = 8,
    C_LR_ACTIVE1 = 9,
    C_NDELTA = 10,   // inserted-edge list length (persistent)
    C_NLIVE_DELTA = 11,
    C_COUNT = 16,
};

struct Cross {      // one cross edge between pieces (dense piece ids)
    uint64_t key;   // (min << 32) | max of the graph edge
    int32_t pa, pb;
};

struct PathReq {    // reverse the path start -> ... -> stop, then parent[start] = newpar
    int32_t start, newpar, stop, pad;
};

__device__ __forceinline__ uint64_t mkkey(uint32_t a, uint32_t b) {
    return a < b ? ((uint64_t)a << 32) | b : ((uint64_t)b << 32) | a;
}
__device__ __forceinline__ int32_t key_lo(uint64_t k) { return (int32_t)(k >> 32); }
__device__ __forceinline__ int32_t key_hi(uint64_t k) { return (int32_t)(uint32_t)k; }

__device__ __forceinline__ uint64_t hmix(uint64_t k) {
    k ^= k >> 33; k *= 0xff51afd7ed558ccdull; k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull; k ^= k >> 33; return k;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// number of set lanes below this lane in a 64-bit wave mask
__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

// Wave-aggregated append: every lane with pred reserves one slot of *counter;
// returns the slot (or -1 when !pred).  One atomic per wave.
__device__ __forceinline__ int64_t wave_append(bool pred, unsigned long long *counter) {
    uint64_t mask = __ballot(pred);
    if (mask == 0) return -1;
    int leader = __ffsll((unsigned long long)mask) - 1;
    unsigned long long base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, (unsigned long long)__popcll(mask));
    base = __shfl(base, leader);
    return pred ? (int64_t)(base + lanes_below(mask)) : -1;
}

// atomicMin on a 64-bit key, skipped when the current value is already lower
__device__ __forceinline__ void min_key(uint64_t *addr, uint64_t k) {
    if (__atomic_load_n(addr, __ATOMIC_RELAXED) > k)
        atomicMin((unsigned long long *)addr, (unsigned long long)k);
}
__device__ __forceinline__ void min_i32(int32_t *addr, int32_t v) {
    if (__atomic_load_n(addr, __ATOMIC_RELAXED) > v) atomicMin(addr, v);
}

__device__ __forceinline__ int32_t ld_relaxed(const int32_t *p) {
    return __atomic_load_n(p, __ATOMIC_RELAXED);
}

}  // namespace drsf
