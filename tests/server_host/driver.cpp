// Replays the benchmark's served sequence against the real scheduler with
// stand-in device work (stubs.cpp): serial saturation, then each load in
// overlapped, serial and coalescing mode, then the verification pair, and
// checks that every request completes without failure.  Reads the workload
// from the file named by argv[1]: "G R", G lines "n nnz arrival", R lines
// "tenant edges op arrival" (arrivals in units of one request at rate 1).
// Test infrastructure only.
#include <hip/hip_runtime.h>
#include "drsf.h"
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>
struct G { int32_t n; int64_t nnz; double win; };
struct R { int g; int64_t b; int op; double t; };
int main(int argc, char **argv) {
    if (argc < 2) return 2;
    FILE *f = fopen(argv[1], "r");
    if (!f) return 2;
    int ng, nr;
    if (fscanf(f, "%d %d", &ng, &nr) != 2) return 1;
    std::vector<G> gs(ng);
    std::vector<R> rs(nr);
    for (auto &g : gs) if (fscanf(f, "%d %ld %lf", &g.n, &g.nnz, &g.win) != 3) return 1;
    for (auto &r : rs) if (fscanf(f, "%d %ld %d %lf", &r.g, &r.b, &r.op, &r.t) != 4) return 1;
    fclose(f);
    const double shrink = argc > 2 ? atof(argv[2]) : 1.0;  // graph sizes scaled down to save host memory
    std::vector<std::vector<int64_t>> rp(ng);
    std::vector<std::vector<int32_t>> col(ng), par(ng);
    for (int g = 0; g < ng; g++) {
        gs[g].n = std::max<int32_t>(2, (int32_t)(gs[g].n * shrink));
        gs[g].nnz = (int64_t)(gs[g].nnz * shrink) & ~1LL;
        rp[g].resize(gs[g].n + 1);
        for (int32_t v = 0; v <= gs[g].n; v++) rp[g][v] = (int64_t)((double)gs[g].nnz * v / gs[g].n);
        col[g].assign(gs[g].nnz, 1);
        par[g].resize(gs[g].n);
        for (int32_t v = 0; v < gs[g].n; v++) par[g][v] = v;
    }
    std::vector<int32_t> edges(200000, 3);
    drsf_opts o;
    drsf_default_opts(&o);
    o.max_batch = 100000;
    std::vector<int64_t> fps(ng);
    for (int g = 0; g < ng; g++) fps[g] = drsf_footprint(gs[g].n, gs[g].nnz, &o);
    std::vector<int64_t> rest(fps.begin() + 1, fps.end());
    std::sort(rest.begin(), rest.end());
    int64_t budget = fps[0];
    for (int k = 0; k < 3 && k < (int)rest.size(); k++) budget += rest[rest.size() - 1 - k];
    int64_t ups = 0;
    for (auto &r : rs) ups += r.b;
    auto serve = [&](bool serial, double rate, bool coalesce, bool digests) {
        drsf_server *s = nullptr;
        int flags = (digests ? DRSF_SERVER_DIGESTS : 0) | (serial ? DRSF_SERVER_SERIAL : 0) | (coalesce ? DRSF_SERVER_COALESCE : 0);
        if (drsf_server_create(budget, &o, flags, &s)) abort();
        const double scale = rate > 0 ? 1e9 / rate : 0.0;
        std::vector<int32_t> tids(ng);
        for (int g = 0; g < ng; g++) {
            const int64_t a = (g == 0 || rate <= 0) ? 0 : (int64_t)(gs[g].win * scale);
            if (drsf_server_admit(s, gs[g].n, rp[g].data(), col[g].data(), par[g].data(), a, &tids[g])) abort();
        }
        std::vector<int64_t> rids(nr);
        for (int i = 0; i < nr; i++) {
            const R &r = rs[i];
            if (drsf_server_submit(s, tids[r.g], edges.data(), r.b, r.op, rate > 0 ? (int64_t)(r.t * scale) : 0, &rids[i])) abort();
        }
        for (int g = 1; g < ng; g++) drsf_server_release(s, tids[g]);
        if (drsf_server_start(s)) abort();
        drsf_server_wait_all(s);
        double st[8];
        drsf_server_stats(s, st);
        int failed = 0;
        for (int i = 0; i < nr; i++) {
            int32_t status; uint64_t t[3], dg[2]; int64_t b;
            drsf_server_result(s, rids[i], &status, t, dg);
            drsf_server_batch(s, rids[i], &b);
            failed += status != DRSF_OK;
        }
        drsf_server_destroy(s);
        printf("serial %d rate %.1f coalesce %d: completed %.0f p50 %.3f p99 %.3f failed %d\n", serial, rate, coalesce, st[0], st[1], st[2], failed);
        fflush(stdout);
        if (failed || (int)st[0] != nr) exit(3);
        return st[0] > 0 ? st[3] : 0.0;
    };
    const double ups_s = serve(true, 0, false, false);
    const double mu = nr / (ups / ups_s);
    printf("mu %.1f req/s\n", mu);
    for (double lam : {0.5, 0.8, 0.95, 1.5}) {
        serve(false, lam * mu, false, false);
        serve(true, lam * mu, false, false);
        serve(false, lam * mu, true, false);
    }
    serve(false, 0, false, true);
    serve(true, 0, false, true);
    return 0;
}
