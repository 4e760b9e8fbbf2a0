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
constexpr uint64_t HOOK_NONE = ~0ull;  // a component that has not hooked (largest round tag)

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
    C_ORIENTED = 8,  // orientation done: the rest of the update may run
    C_OMODE = 9,     // delete sweep restricted to the orphans' adjacency
    C_NDELTA = 10,   // inserted-edge list length (persistent)
    C_OVOL = 11,     // adjacency slots of the listed orphan vertices
    C_NORPH = 13,    // listed orphan vertices (orphans with at least one slot)
    C_ARRIVE = 14,   // workgroups of the running kernel that have finished (zero between kernels)
    C_LR_FINAL = 12, // buffer holding the final list ranks
    C_NLONG = 15,    // paths longer than the walk limit, left to the host's doubling pass
    C_COUNT = 16,
};

struct Cross {      // one cross edge between pieces (dense piece ids)
    uint64_t key;   // (min << 32) | max of the graph edge
    int32_t pa, pb;
};

struct PathReq {    // reverse the path start -> ... -> stop, then parent[start] = newpar
    int32_t start, newpar, stop, pad;
};

// One orphan vertex (a vertex cut off from its old root) with adjacency to
// scan: slots [pre, pre + du + dl) of the concatenated orphan adjacency are
// its du upper-store entries from ustart, then its dl lower-store entries
// from lstart (followed by padding slots that hold no work).
struct OrphEnt {
    int64_t pre;
    uint32_t ustart, lstart;
    int32_t v, du, dl;
    int32_t pu;     // dense id of the vertex's piece
    int32_t ru;     // root of that piece (rep of the vertex)
    int32_t pk;     // dense id of the piece holding the vertex's old root
};

__device__ __forceinline__ uint64_t mkkey(uint32_t a, uint32_t b) {
    return a < b ? ((uint64_t)a << 32) | b : ((uint64_t)b << 32) | a;
}
__device__ __forceinline__ int32_t key_lo(uint64_t k) { return (int32_t)(k >> 32); }
__device__ __forceinline__ int32_t key_hi(uint64_t k) { return (int32_t)(uint32_t)k; }

// 64-bit finalizer of MurmurHash3 (Austin Appleby's published mixing
// function): spreads keys over the open-addressing tables
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

// atomicMin on a 64-bit key, skipped when a plain (possibly stale) read of
// the current value is already lower: values only decrease, so a stale read
// can cost an extra atomic but never skips a needed one.
__device__ __forceinline__ void min_key(uint64_t *addr, uint64_t k) {
    if (*addr > k) atomicMin((unsigned long long *)addr, (unsigned long long)k);
}
__device__ __forceinline__ void min_i32(int32_t *addr, int32_t v) {
    if (*addr > v) atomicMin(addr, v);
}

// Hot-address atomics.  On this part an atomic request to one address is
// serialised at the memory side (about 12 ns per request, where a request is
// one wave instruction), so lanes of a wave that target the same address are
// merged first: up to GROUP_ROUNDS times the lowest pending lane's target is
// taken, every lane with that target joins the group, and the group issues a
// single request.  Lanes left over issue their own.
constexpr int GROUP_ROUNDS = 4;

__device__ __forceinline__ void group_min_u64(bool active, int32_t target, uint64_t val,
                                              uint64_t *arr) {
    uint64_t rem = __ballot(active);
    for (int round = 0; round < GROUP_ROUNDS && rem; round++) {
        const int leader = __ffsll((unsigned long long)rem) - 1;
        const int32_t t0 = __shfl(target, leader);
        const bool in = active && target == t0;
        const uint64_t gm = __ballot(in);
        uint64_t v = in ? val : ~0ull;
        for (int o = WAVE / 2; o > 0; o >>= 1) {
            uint64_t w = __shfl_xor(v, o);
            v = w < v ? w : v;
        }
        if (lane_id() == leader && arr[t0] > v)
            atomicMin((unsigned long long *)&arr[t0], (unsigned long long)v);
        rem &= ~gm;
        if (in) active = false;
    }
    if (active && arr[target] > val) atomicMin((unsigned long long *)&arr[target], (unsigned long long)val);
}

// Push `item` onto the singly linked list headed by head[target]
// (nxt[item] = previous head).  Grouped lanes are chained among themselves
// and spliced in with one exchange.
__device__ __forceinline__ void group_push(bool active, int32_t target, int32_t item,
                                           int32_t *head, int32_t *nxt) {
    uint64_t rem = __ballot(active);
    const int lane = lane_id();
    for (int round = 0; round < GROUP_ROUNDS && rem; round++) {
        const int leader = __ffsll((unsigned long long)rem) - 1;
        const int32_t t0 = __shfl(target, leader);
        const bool in = active && target == t0;
        const uint64_t gm = __ballot(in);
        // next group lane above this one (or -1)
        const uint64_t above = lane == 63 ? 0ull : (gm & ~((2ull << lane) - 1ull));
        const int nl = above ? __ffsll((unsigned long long)above) - 1 : lane;
        const int32_t next_item = __shfl(item, nl);
        const int last = 63 - __clzll((long long)gm);
        const int32_t first_item = __shfl(item, leader);
        if (in) {
            if (lane == last) nxt[item] = atomicExch(&head[t0], first_item);
            else nxt[item] = next_item;
        }
        rem &= ~gm;
        if (in) active = false;
    }
    if (active) nxt[item] = atomicExch(&head[target], item);
}

// Plain load used by the monotone pointer chases: the value read may be
// stale (another workgroup's write not yet visible), which only means an
// ancestor closer to the starting vertex.  System-scope atomic loads would
// bypass the caches on every step.
__device__ __forceinline__ int32_t ld_relaxed(const int32_t *p) { return *p; }

}  // namespace drsf
