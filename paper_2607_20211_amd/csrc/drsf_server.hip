// Serving layer of libdrsf.so (declared in include/drsf.h): several graphs
// ("tenants") resident on one GPU, each with its own context and stream,
// updated by a stream of requests.
//
// A scheduler thread runs in ticks.  Each tick it (1) moves requests and
// tenants whose arrival time has come into the tenants' FIFOs and the
// admission queue, (2) admits waiting tenants in arrival order while their
// estimated footprint fits the memory budget, (3) starts the head request of
// every live tenant that has nothing in flight (each on its tenant's stream,
// so updates of different graphs overlap on the device), (4) completes
// requests whose stream has drained, and (5) destroys released tenants once
// their FIFO is empty, which frees memory for the admission queue.  Requests
// of one tenant are applied in arrival order.  By default each is its own
// batch, so every request's result equals applying the same requests one at
// a time.  In coalescing mode the requests of the same op waiting at the head
// of an idle tenant's FIFO go out as one batch (up to max_batch edges); a
// merged batch that is rejected leaves the graph unchanged and its requests
// are retried one at a time; each request records the batch that carried it.
// In serial mode at most one request is in flight over all tenants, in
// global arrival order: the plain one-batch-at-a-time path, for comparison.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/drsf.h"
#include "drsf_kernels.h"

namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Req {
    int64_t id = 0;
    int32_t tenant = 0;
    int op = 0;
    std::vector<int32_t> edges;
    uint64_t t_arrive = 0, t_start = 0, t_done = 0;  // ns since the server's start
    int32_t status = DRSF_OK;
    uint64_t digest[2] = {0, 0};
    int64_t batch = -1;  // the first request of the batch that carried it
    bool done = false;
};

enum TState { T_WAITING, T_QUEUED, T_LIVE, T_GONE, T_FAILED };

struct Tenant {
    int32_t id = 0;
    TState state = T_WAITING;
    uint64_t t_arrive = 0;
    uint64_t t_live = 0;  // admitted (context created)
    // host copy of the graph until admission
    int32_t n = 0;
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col, parent;
    int64_t estimate = 0;
    drsf_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    int64_t bytes = 0;
    std::deque<int64_t> fifo;
    int64_t inflight = -1;
    std::vector<int64_t> group;   // the requests of the batch in flight
    std::vector<int32_t> merged;  // their edges, when there are several
    int64_t solo = 0;             // requests to apply alone (after a rejected merge)
    int phase = 0;  // 1 update queued, 2 digest queued
    bool release = false;
    unsigned long long *d_dig = nullptr, *h_dig = nullptr;
    std::string error;
};

}  // namespace

struct drsf_server {
    int64_t budget = 0, used = 0, peak_used = 0;
    drsf_opts opts{};
    int flags = 0;
    int dev = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Tenant> tenants;  // stable references while the lock is dropped
    std::map<int64_t, Req> reqs;
    std::multimap<uint64_t, int64_t> future_reqs;    // arrival -> request
    std::multimap<uint64_t, int32_t> future_admits;  // arrival -> tenant
    std::deque<int32_t> admit_queue;
    int64_t next_req = 0;
    int64_t outstanding = 0;
    uint64_t t0 = 0;
    bool started = false, stop = false;
    std::thread th;
    std::string err;
    // statistics of completed requests: latency from arrival, and from the
    // later of arrival and the tenant's admission (service latency)
    std::vector<double> lat_ms, svc_ms;
    int64_t updates = 0;
    uint64_t first_arrive = ~0ull, last_done = 0;
};

namespace {

int sfail(drsf_server *s, int code, const std::string &m) {
    s->err = m;
    return code;
}

void complete(drsf_server *s, Req &r, int status, uint64_t t) {
    r.status = status;
    r.t_done = t;
    r.done = true;
    s->outstanding--;
    s->lat_ms.push_back((double)(r.t_done - r.t_arrive) * 1e-6);
    const uint64_t ready = std::max(r.t_arrive, s->tenants[r.tenant].t_live);
    s->svc_ms.push_back((double)(r.t_done - std::min(ready, r.t_done)) * 1e-6);
    if (status == DRSF_OK) s->updates += (int64_t)(r.edges.size() / 2);
    s->first_arrive = std::min(s->first_arrive, r.t_arrive);
    s->last_done = std::max(s->last_done, r.t_done);
    r.edges.clear();
    r.edges.shrink_to_fit();
    s->cv_done.notify_all();
}

// Moves arrived requests and tenants; caller holds the lock.
void arrivals(drsf_server *s, uint64_t t) {
    while (!s->future_admits.empty() && s->future_admits.begin()->first <= t) {
        const int32_t id = s->future_admits.begin()->second;
        s->future_admits.erase(s->future_admits.begin());
        s->tenants[id].state = T_QUEUED;
        s->admit_queue.push_back(id);
    }
    while (!s->future_reqs.empty() && s->future_reqs.begin()->first <= t) {
        const int64_t id = s->future_reqs.begin()->second;
        s->future_reqs.erase(s->future_reqs.begin());
        Req &r = s->reqs[id];
        Tenant &tn = s->tenants[r.tenant];
        if (tn.state == T_FAILED || tn.state == T_GONE) complete(s, r, DRSF_E_STATE, t);
        else tn.fifo.push_back(id);
    }
}

// Creates a tenant's context; called without the lock (create is slow).
int admit_one(drsf_server *s, Tenant &t) {
    if (hipStreamCreateWithFlags(&t.stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        return DRSF_E_DEVICE;
    }
    drsf_opts o = s->opts;
    o.stream = t.stream;
    o.inputs_on_device = 0;
    int rc = drsf_create(t.n, t.row_ptr.data(), t.col.data(), t.parent.data(), &o, &t.ctx);
    if (rc != DRSF_OK) {
        t.error = drsf_last_error(nullptr);
        (void)hipStreamDestroy(t.stream);
        t.stream = nullptr;
        return rc;
    }
    if (hipMalloc(&t.d_dig, 2 * sizeof(unsigned long long)) != hipSuccess ||
        hipHostMalloc((void **)&t.h_dig, 2 * sizeof(unsigned long long)) != hipSuccess) {
        (void)hipGetLastError();
        return DRSF_E_NOMEM;
    }
    t.bytes = drsf_device_bytes(t.ctx);
    return DRSF_OK;
}

void destroy_tenant(Tenant &t) {
    if (t.ctx) drsf_destroy(t.ctx);
    t.ctx = nullptr;
    if (t.stream) (void)hipStreamDestroy(t.stream);
    t.stream = nullptr;
    if (t.d_dig) (void)hipFree(t.d_dig);
    if (t.h_dig) (void)hipHostFree(t.h_dig);
    t.d_dig = nullptr;
    t.h_dig = nullptr;
}

void scheduler(drsf_server *s) {
    (void)hipSetDevice(s->dev);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        const uint64_t t = now_ns() - s->t0;
        arrivals(s, t);
        // (2) admission in arrival order while the estimate fits
        while (!s->admit_queue.empty()) {
            Tenant &tn = s->tenants[s->admit_queue.front()];
            if (s->used + tn.estimate > s->budget && s->used > 0) break;
            s->admit_queue.pop_front();
            lk.unlock();
            const int rc = admit_one(s, tn);
            lk.lock();
            if (rc != DRSF_OK) {
                tn.state = T_FAILED;
                destroy_tenant(tn);
                const uint64_t tf = now_ns() - s->t0;
                for (int64_t id : tn.fifo) complete(s, s->reqs[id], rc, tf);
                tn.fifo.clear();
                continue;
            }
            tn.state = T_LIVE;
            tn.t_live = now_ns() - s->t0;
            tn.row_ptr.clear(); tn.row_ptr.shrink_to_fit();
            tn.col.clear(); tn.col.shrink_to_fit();
            tn.parent.clear(); tn.parent.shrink_to_fit();
            s->used += tn.bytes;
            s->peak_used = std::max(s->peak_used, s->used);
        }
        bool busy = false;
        // (4) completions
        for (Tenant &tn : s->tenants) {
            if (tn.state != T_LIVE || tn.inflight < 0) continue;
            busy = true;
            if (hipStreamQuery(tn.stream) != hipSuccess) {
                (void)hipGetLastError();
                continue;
            }
            if (tn.phase == 1) {
                const int rc = drsf_wait(tn.ctx, nullptr);  // may finish the update on the host
                if (rc == DRSF_E_BATCH && tn.group.size() > 1) {
                    // a merged batch was rejected (the graph is unchanged):
                    // its requests go back, to be applied one at a time
                    for (auto it = tn.group.rbegin(); it != tn.group.rend(); ++it) tn.fifo.push_front(*it);
                    tn.solo = (int64_t)tn.group.size();
                    tn.group.clear();
                    tn.inflight = -1;
                    tn.phase = 0;
                    continue;
                }
                if (rc == DRSF_OK && (s->flags & DRSF_SERVER_DIGESTS)) {
                    drsf_view v;
                    drsf_get_view(tn.ctx, &v);
                    drsf::launch_digest(v.n, v.parent, v.label, tn.d_dig, tn.stream);
                    (void)hipMemcpyAsync(tn.h_dig, tn.d_dig, 2 * sizeof(unsigned long long),
                                         hipMemcpyDeviceToHost, tn.stream);
                    tn.phase = 2;
                    continue;
                }
                const uint64_t td = now_ns() - s->t0;
                for (int64_t id : tn.group) complete(s, s->reqs[id], rc, td);
            } else {
                const uint64_t td = now_ns() - s->t0;
                for (int64_t id : tn.group) {
                    Req &r = s->reqs[id];
                    r.digest[0] = tn.h_dig[0];
                    r.digest[1] = tn.h_dig[1];
                    complete(s, r, DRSF_OK, td);
                }
            }
            tn.group.clear();
            tn.inflight = -1;
            tn.phase = 0;
        }
        // (3) starts
        int64_t inflight_all = 0;
        for (Tenant &tn : s->tenants) inflight_all += tn.inflight >= 0;
        while (true) {
            Tenant *pick = nullptr;
            for (Tenant &tn : s->tenants) {
                if (tn.state != T_LIVE || tn.inflight >= 0 || tn.fifo.empty()) continue;
                if (!(s->flags & DRSF_SERVER_SERIAL)) {
                    pick = &tn;
                    break;
                }
                if (!pick || s->reqs[tn.fifo.front()].t_arrive < s->reqs[pick->fifo.front()].t_arrive)
                    pick = &tn;
            }
            if (!pick || ((s->flags & DRSF_SERVER_SERIAL) && inflight_all > 0)) break;
            const int64_t id = pick->fifo.front();
            pick->fifo.pop_front();
            Req &r = s->reqs[id];
            pick->group.assign(1, id);
            const int32_t *edges = r.edges.data();
            int64_t b = (int64_t)(r.edges.size() / 2);
            if ((s->flags & DRSF_SERVER_COALESCE) && pick->solo == 0) {
                // the following requests of the same op, while the batch fits
                const int64_t cap = s->opts.max_batch > 0 ? s->opts.max_batch : (1 << 20);
                int64_t tot = b;
                while (!pick->fifo.empty()) {
                    const Req &q = s->reqs[pick->fifo.front()];
                    const int64_t qb = (int64_t)(q.edges.size() / 2);
                    if (q.op != r.op || tot + qb > cap) break;
                    pick->group.push_back(q.id);
                    tot += qb;
                    pick->fifo.pop_front();
                }
                if (pick->group.size() > 1) {
                    pick->merged.clear();
                    pick->merged.reserve((size_t)(2 * tot));
                    for (int64_t gid : pick->group) {
                        const std::vector<int32_t> &e = s->reqs[gid].edges;
                        pick->merged.insert(pick->merged.end(), e.begin(), e.end());
                    }
                    edges = pick->merged.data();
                    b = tot;
                }
            }
            if (pick->solo > 0) pick->solo--;
            const uint64_t ts = now_ns() - s->t0;
            for (int64_t gid : pick->group) {
                s->reqs[gid].t_start = ts;
                s->reqs[gid].batch = id;
            }
            // host edges are copied before the call returns
            const int rc = drsf_apply_async(pick->ctx, edges, b, r.op);
            if (rc != DRSF_OK) {
                const uint64_t td = now_ns() - s->t0;
                for (int64_t gid : pick->group) complete(s, s->reqs[gid], rc, td);
                pick->group.clear();
                continue;
            }
            pick->inflight = id;
            pick->phase = 1;
            inflight_all++;
            busy = true;
        }
        // (5) releases
        for (Tenant &tn : s->tenants) {
            if (tn.state == T_LIVE && tn.release && tn.fifo.empty() && tn.inflight < 0) {
                bool pending = false;
                for (auto &fr : s->future_reqs)
                    if (s->reqs[fr.second].tenant == tn.id) { pending = true; break; }
                if (pending) continue;
                destroy_tenant(tn);
                s->used -= tn.bytes;
                tn.state = T_GONE;
            }
        }
        if (s->stop && s->outstanding == 0) break;
        if (busy) {
            // something is in flight: poll again shortly
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else {
            uint64_t wake = ~0ull;
            if (!s->future_reqs.empty()) wake = std::min(wake, s->future_reqs.begin()->first);
            if (!s->future_admits.empty()) wake = std::min(wake, s->future_admits.begin()->first);
            bool ready = false;
            for (Tenant &tn : s->tenants)
                if (tn.state == T_LIVE && !tn.fifo.empty()) ready = true;
            if (ready || (!s->admit_queue.empty())) {
                if (!s->admit_queue.empty()) {
                    // waiting for memory that only a release can free
                    s->cv_work.wait_for(lk, std::chrono::microseconds(200));
                }
                continue;
            }
            if (s->stop && s->outstanding == 0) break;
            if (wake == ~0ull) {
                s->cv_work.wait(lk);
            } else {
                const uint64_t tt = now_ns() - s->t0;
                if (wake > tt) {
                    const uint64_t dt = wake - tt;
                    if (dt > 50000) s->cv_work.wait_for(lk, std::chrono::nanoseconds(dt - 20000));
                    else { lk.unlock(); std::this_thread::yield(); lk.lock(); }
                }
            }
        }
    }
}

}  // namespace

extern "C" {

int drsf_server_create(int64_t budget_bytes, const drsf_opts *opts, int flags, drsf_server **out) {
    if (!out) return DRSF_E_ARG;
    *out = nullptr;
    if (budget_bytes <= 0) return DRSF_E_ARG;
    drsf_server *s = new drsf_server();
    s->budget = budget_bytes;
    if (opts) s->opts = *opts; else drsf_default_opts(&s->opts);
    s->flags = flags;
    if (hipGetDevice(&s->dev) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return DRSF_E_DEVICE;
    }
    *out = s;
    return DRSF_OK;
}

const char *drsf_server_error(const drsf_server *s) { return s ? s->err.c_str() : ""; }

int drsf_server_admit(drsf_server *s, int32_t n, const int64_t *row_ptr, const int32_t *col,
                      const int32_t *parent, int64_t arrive_ns, int32_t *tenant) {
    if (!s || !tenant || n < 1 || !row_ptr || !parent) return DRSF_E_ARG;
    const int64_t nnz = row_ptr[n];
    if (nnz < 0 || (nnz > 0 && !col)) return sfail(s, DRSF_E_ARG, "bad CSR");
    Tenant t;
    t.n = n;
    t.row_ptr.assign(row_ptr, row_ptr + n + 1);
    t.col.assign(col, col + nnz);
    t.parent.assign(parent, parent + n);
    drsf_opts o = s->opts;
    o.inputs_on_device = 0;
    t.estimate = drsf_footprint(n, nnz, &o);
    std::lock_guard<std::mutex> g(s->mu);
    if (t.estimate > s->budget) return sfail(s, DRSF_E_BUDGET, "graph larger than the whole budget");
    t.id = (int32_t)s->tenants.size();
    const uint64_t at = arrive_ns >= 0 ? (uint64_t)arrive_ns : (s->started ? now_ns() - s->t0 : 0);
    t.t_arrive = at;
    s->tenants.push_back(std::move(t));
    s->future_admits.emplace(at, s->tenants.back().id);
    *tenant = s->tenants.back().id;
    s->cv_work.notify_all();
    return DRSF_OK;
}

int drsf_server_submit(drsf_server *s, int32_t tenant, const int32_t *edges, int64_t b, int op,
                       int64_t arrive_ns, int64_t *req) {
    if (!s || !req || b < 0 || (b > 0 && !edges)) return DRSF_E_ARG;
    if (op != DRSF_INSERT && op != DRSF_DELETE) return DRSF_E_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    if (tenant < 0 || tenant >= (int32_t)s->tenants.size() || s->tenants[tenant].release)
        return sfail(s, DRSF_E_ARG, "unknown or released tenant");
    Req r;
    r.id = s->next_req++;
    r.tenant = tenant;
    r.op = op;
    r.edges.assign(edges, edges + 2 * b);
    r.t_arrive = arrive_ns >= 0 ? (uint64_t)arrive_ns : (s->started ? now_ns() - s->t0 : 0);
    r.t_arrive = std::max(r.t_arrive, s->tenants[tenant].t_arrive);
    s->future_reqs.emplace(r.t_arrive, r.id);
    *req = r.id;
    s->reqs.emplace(r.id, std::move(r));
    s->outstanding++;
    s->cv_work.notify_all();
    return DRSF_OK;
}

int drsf_server_release(drsf_server *s, int32_t tenant) {
    if (!s) return DRSF_E_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    if (tenant < 0 || tenant >= (int32_t)s->tenants.size()) return DRSF_E_ARG;
    s->tenants[tenant].release = true;
    s->cv_work.notify_all();
    return DRSF_OK;
}

int drsf_server_start(drsf_server *s) {
    if (!s) return DRSF_E_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    if (s->started) return sfail(s, DRSF_E_STATE, "already started");
    // graphs present from the start are made resident before the clock runs
    for (Tenant &tn : s->tenants) {
        if (tn.t_arrive != 0 || tn.state != T_WAITING) continue;
        if (s->used + tn.estimate > s->budget && s->used > 0) break;
        const int rc = admit_one(s, tn);
        if (rc != DRSF_OK) {
            destroy_tenant(tn);
            tn.state = T_FAILED;
        } else {
            tn.state = T_LIVE;
            tn.row_ptr.clear(); tn.row_ptr.shrink_to_fit();
            tn.col.clear(); tn.col.shrink_to_fit();
            tn.parent.clear(); tn.parent.shrink_to_fit();
            s->used += tn.bytes;
            s->peak_used = std::max(s->peak_used, s->used);
        }
        for (auto it = s->future_admits.begin(); it != s->future_admits.end(); ++it)
            if (it->second == tn.id) { s->future_admits.erase(it); break; }
    }
    s->t0 = now_ns();
    s->started = true;
    s->th = std::thread(scheduler, s);
    return DRSF_OK;
}

int drsf_server_wait_all(drsf_server *s) {
    if (!s) return DRSF_E_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (!s->started) return sfail(s, DRSF_E_STATE, "not started");
    s->cv_done.wait(lk, [s] { return s->outstanding == 0; });
    return DRSF_OK;
}

int drsf_server_result(drsf_server *s, int64_t req, int32_t *status, uint64_t *t_ns, uint64_t *digest) {
    if (!s) return DRSF_E_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req);
    if (it == s->reqs.end()) return sfail(s, DRSF_E_ARG, "unknown request");
    s->cv_done.wait(lk, [&] { return it->second.done; });
    const Req &r = it->second;
    if (status) *status = r.status;
    if (t_ns) {
        t_ns[0] = r.t_arrive;
        t_ns[1] = r.t_start;
        t_ns[2] = r.t_done;
    }
    if (digest) {
        digest[0] = r.digest[0];
        digest[1] = r.digest[1];
    }
    return DRSF_OK;
}

int drsf_server_batch(drsf_server *s, int64_t req, int64_t *batch) {
    if (!s || !batch) return DRSF_E_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req);
    if (it == s->reqs.end()) return sfail(s, DRSF_E_ARG, "unknown request");
    s->cv_done.wait(lk, [&] { return it->second.done; });
    *batch = it->second.batch;
    return DRSF_OK;
}

int drsf_server_stats(drsf_server *s, double *out) {
    if (!s || !out) return DRSF_E_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    std::vector<double> l = s->lat_ms;
    std::sort(l.begin(), l.end());
    auto q = [&](double p) {
        if (l.empty()) return 0.0;
        size_t k = (size_t)(p * (double)(l.size() - 1) + 0.5);
        return l[std::min(k, l.size() - 1)];
    };
    out[0] = (double)l.size();
    out[1] = q(0.5);
    out[2] = q(0.99);
    const double span = s->last_done > s->first_arrive ? (double)(s->last_done - s->first_arrive) * 1e-9 : 0.0;
    out[3] = span > 0 ? (double)s->updates / span : 0.0;
    out[4] = (double)s->peak_used;
    out[5] = (double)s->budget;
    l = s->svc_ms;
    std::sort(l.begin(), l.end());
    out[6] = q(0.5);
    out[7] = q(0.99);
    return DRSF_OK;
}

int32_t drsf_server_tenant_state(drsf_server *s, int32_t tenant) {
    if (!s) return -1;
    std::lock_guard<std::mutex> g(s->mu);
    if (tenant < 0 || tenant >= (int32_t)s->tenants.size()) return -1;
    return (int32_t)s->tenants[tenant].state;
}

int drsf_server_copy_out(drsf_server *s, int32_t tenant, int32_t *parent_host, int32_t *label_host) {
    if (!s) return DRSF_E_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (tenant < 0 || tenant >= (int32_t)s->tenants.size()) return sfail(s, DRSF_E_ARG, "unknown tenant");
    // the scheduler uses a tenant's context only while holding the lock, so
    // an idle tenant's context is free while the lock is held here
    auto idle = [&] {
        const Tenant &t = s->tenants[tenant];
        if (t.state != T_LIVE) return true;
        if (t.inflight >= 0 || !t.fifo.empty()) return false;
        for (auto &fr : s->future_reqs)
            if (s->reqs[fr.second].tenant == tenant) return false;
        return true;
    };
    if (s->started) s->cv_done.wait(lk, idle);
    Tenant &t = s->tenants[tenant];
    if (t.state != T_LIVE || !t.ctx) return sfail(s, DRSF_E_STATE, "the tenant is not live");
    const int rc = drsf_copy_out(t.ctx, parent_host, label_host);
    if (rc != DRSF_OK) return sfail(s, rc, drsf_last_error(t.ctx));
    return DRSF_OK;
}

void drsf_server_destroy(drsf_server *s) {
    if (!s) return;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->started) s->cv_done.wait(lk, [s] { return s->outstanding == 0; });
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    for (Tenant &t : s->tenants) destroy_tenant(t);
    delete s;
}

}  // extern "C"
