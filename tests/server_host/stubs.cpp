// Host-only stand-ins for the library and HIP calls the serving scheduler
// makes (test infrastructure only): a "context" holds its sizes and a
// simulated device deadline, an apply sets the deadline of the context's
// stream (100 us + 15 ns per edge, about the measured service time of the
// served workload), a stream query reports it, a wait spins until it.  Every
// stream, allocation and context is tracked: a double or unknown free
// aborts.  With these the real scheduler runs under the sanitizers.
#include <hip/hip_runtime.h>
#include "drsf.h"
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <set>
static uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
struct StubStream { std::atomic<uint64_t> ready{0}; };
static std::mutex g_mu;
static std::set<void *> g_live;
static void track(void *p) { std::lock_guard<std::mutex> g(g_mu); if (!g_live.insert(p).second) abort(); }
static void untrack(void *p) { if (!p) return; std::lock_guard<std::mutex> g(g_mu); if (!g_live.erase(p)) { fprintf(stderr, "bad free %p\n", p); abort(); } }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = new StubStream(); track(*s); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { untrack(s); delete s; return hipSuccess; }
hipError_t hipStreamQuery(hipStream_t s) { return now_ns() >= s->ready.load() ? hipSuccess : hipErrorNotReady; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipMalloc(void **p, size_t n) { *p = malloc(n); track(*p); return hipSuccess; }
hipError_t hipFree(void *p) { untrack(p); free(p); return hipSuccess; }
hipError_t hipHostMalloc(void **p, size_t n, unsigned) { *p = malloc(n); track(*p); return hipSuccess; }
hipError_t hipHostFree(void *p) { untrack(p); free(p); return hipSuccess; }
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t) { memmove(d, s, n); return hipSuccess; }
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
namespace drsf {
void launch_digest(int32_t, const int32_t *, const int32_t *, unsigned long long *out, hipStream_t) { out[0] = 1; out[1] = 2; }
}
struct drsf_ctx { int32_t n; int64_t nnz; hipStream_t s; int32_t *parent, *label; bool pending = false; uint64_t done = 0; std::string err; int64_t m; };
static thread_local std::string g_err;
extern "C" {
void drsf_default_opts(drsf_opts *o) { memset(o, 0, sizeof *o); o->validate_forest = 1; o->validate_batches = 1; o->max_batch = 1 << 20; }
int64_t drsf_footprint(int32_t n, int64_t nnz, const drsf_opts *) { return 64 * (int64_t)n + 12 * nnz + (1 << 20); }
int drsf_create(int32_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *parent, const drsf_opts *o, drsf_ctx **out) {
    if (n < 1 || !row_ptr || !parent) return DRSF_E_ARG;
    drsf_ctx *c = new drsf_ctx();
    track(c);
    c->n = n; c->nnz = row_ptr[n]; c->s = (hipStream_t)o->stream; c->m = c->nnz / 2;
    // touch the inputs as create would
    volatile int64_t acc = 0;
    for (int32_t v = 0; v < n; v += 97) acc += parent[v] + (col && c->nnz ? col[(row_ptr[v]) % (c->nnz ? c->nnz : 1)] : 0);
    c->parent = (int32_t *)calloc(n, 4); c->label = (int32_t *)calloc(n, 4);
    std::this_thread::sleep_for(std::chrono::microseconds(200 + c->nnz / 20000));  // create time
    *out = c;
    return DRSF_OK;
}
void drsf_destroy(drsf_ctx *c) { if (!c) return; untrack(c); free(c->parent); free(c->label); delete c; }
const char *drsf_last_error(const drsf_ctx *c) { return c ? c->err.c_str() : g_err.c_str(); }
int64_t drsf_device_bytes(const drsf_ctx *c) { return drsf_footprint(c->n, c->nnz, nullptr); }
int drsf_apply_async(drsf_ctx *c, const int32_t *edges, int64_t b, int op) {
    if (!c || (b > 0 && !edges)) return DRSF_E_ARG;
    if (b > 100000) return DRSF_E_CAPACITY;
    volatile int64_t acc = 0;
    for (int64_t i = 0; i < 2 * b; i += 7) acc += edges[i];  // the host copy reads every edge
    if (b > 0 && (edges[2 * b - 1] < 0 || edges[0] < 0)) acc++;
    const uint64_t t = now_ns() + 100000 + (uint64_t)b * 15;  // simulated device time
    c->s->ready.store(t);
    c->done = t;
    c->pending = true;
    c->m += op == DRSF_INSERT ? b : -b;
    return DRSF_OK;
}
int drsf_wait(drsf_ctx *c, drsf_view *out) {
    if (!c) return DRSF_E_ARG;
    while (now_ns() < c->done) {}
    c->pending = false;
    if (out) { memset(out, 0, sizeof *out); out->parent = c->parent; out->label = c->label; out->n = c->n; out->num_edges = c->m; }
    return DRSF_OK;
}
int drsf_get_view(drsf_ctx *c, drsf_view *out) { return drsf_wait(c, out); }
int drsf_copy_out(drsf_ctx *c, int32_t *p, int32_t *l) { if (p) memcpy(p, c->parent, 4 * c->n); if (l) memcpy(l, c->label, 4 * c->n); return DRSF_OK; }
}
