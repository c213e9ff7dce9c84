// Host-only test driver of the request server (admission thread, two compute lanes, pool,
// poll queue) against the stub runtime and stub count of stub_runtime.cpp.  Each scenario
// submits requests, polls every result under a watchdog and checks each result against its
// own request; prints one line per scenario and exits non-zero on the first failure (or
// when results stop arriving: a stall).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <random>
#include <thread>
#include <vector>

#include "../../include/glt.h"

extern "C" void stub_configure(int64_t fail_copy, int64_t ns_per_edge);
extern "C" int64_t stub_batches(void);
extern "C" int64_t stub_max_batch(void);

struct Graph {
    int64_t n = 0, m = 0;
    std::vector<int32_t> rp, col;
    uint64_t sum = 0;
};

static Graph make_graph(std::mt19937_64& rng, int64_t n, int64_t m, bool invalid) {
    Graph g;
    g.n = n;
    g.m = m;
    g.rp.assign(n + 1, 0);
    for (int64_t i = 0; i < 2 * m; i++) g.rp[1 + (int64_t)(rng() % (uint64_t)n)]++;
    for (int64_t i = 0; i < n; i++) g.rp[i + 1] += g.rp[i];
    g.col.resize(2 * m);
    for (auto& c : g.col) c = (int32_t)(rng() % (uint64_t)n);
    if (invalid && m > 0) g.col[0] = -7;
    for (auto c : g.col) g.sum += (uint64_t)(int64_t)c;
    return g;
}

static bool check(const glt_result& r, const Graph& g) {
    return r.X[0].lo == (uint64_t)g.m && r.X[1].lo == (uint64_t)g.n && r.X[2].lo == g.sum &&
           r.X[3].lo == (g.m > 0 ? (uint64_t)(int64_t)g.col[0] : 0);
}

// Submits the graphs (pool[idx[i]] as request i) at the given arrival offsets (seconds),
// polls until all are done; returns the number of results with an unexpected status or
// counts (expect[i] is the expected status), or -1 on a stall.
static int64_t run(glt_server_opts o, const std::vector<Graph>& pool, const std::vector<int>& idx,
                   const std::vector<double>& at, const std::vector<int>& expect, double stall_s) {
    glt_server* s = nullptr;
    if (glt_server_create(&o, &s) != GLT_OK) return -2;
    const size_t N = idx.size();
    std::vector<int> seen(N, 0);
    int64_t bad = 0, got = 0;
    const double t0 = glt_server_clock();
    size_t next = 0;
    double last_progress = t0;
    std::vector<glt_result> res(256);
    while (got < (int64_t)N) {
        const double now = glt_server_clock();
        while (next < N && now - t0 >= at[next]) {
            const Graph& g = pool[idx[next]];
            glt_csr c{g.n, g.m, g.rp.data(), g.col.data(), 0, 0};
            if (glt_server_submit(s, &c, next) != GLT_OK) { glt_server_destroy(s); return -3; }
            next++;
        }
        const int k = glt_server_poll(s, res.data(), 256, 1000);
        for (int i = 0; i < k; i++) {
            const uint64_t id = res[i].req_id;
            if (id >= N || seen[id]++) { bad++; continue; }
            got++;
            const int want = expect[id];
            if (res[i].status != want || (want == GLT_OK && !check(res[i], pool[idx[id]]))) {
                if (bad < 5)
                    fprintf(stderr, "request %llu: status %d, expected %d\n", (unsigned long long)id, res[i].status, want);
                bad++;
            }
        }
        if (k > 0 || next < N) last_progress = glt_server_clock();
        if (glt_server_clock() - last_progress > stall_s) {
            fprintf(stderr, "stall: %lld of %zu results, %lld in flight\n", (long long)got, N,
                    (long long)glt_server_inflight(s));
            glt_server_destroy(s);
            return -1;
        }
    }
    if (glt_server_inflight(s) != 0) bad++;
    glt_server_destroy(s);
    return bad;
}

static int report(const char* name, int64_t bad) {
    printf("%s: %s (%lld bad; %lld batches, largest %lld requests)\n", name, bad == 0 ? "ok" : "FAIL",
           (long long)bad, (long long)stub_batches(), (long long)stub_max_batch());
    fflush(stdout);
    return bad == 0 ? 0 : 1;
}

int main() {
    std::mt19937_64 rng(160805138);
    int fails = 0;
    {   // many requests through a pool far smaller than their total: admission waits for
        // slots, both lanes batch what is admitted; every result belongs to its request
        std::vector<Graph> pool;
        for (int i = 0; i < 300; i++) pool.push_back(make_graph(rng, 50 + rng() % 4950, rng() % 60000, false));
        for (int i = 0; i < 6; i++) pool.push_back(make_graph(rng, 200000, 2000000, false));
        std::vector<int> idx, expect;
        std::vector<double> at;
        for (int i = 0; i < 4000; i++) {
            idx.push_back(i % 50 == 7 ? 300 + (i % 6) : (int)(rng() % 300));
            at.push_back(0.0);
            expect.push_back(GLT_OK);
        }
        glt_server_opts o{};
        o.resident_bytes = (size_t)64 << 20;
        o.large_edges = 262144;
        stub_configure(-1, 2);
        fails += report("burst through a small pool", run(o, pool, idx, at, expect, 20.0));
        o.max_batch_graphs = 1;
        stub_configure(-1, 2);
        fails += report("one request per launch", run(o, pool, idx, at, expect, 20.0));
    }
    {   // a request larger than the whole pool fails alone with GLT_E_OOM; an invalid request
        // fails alone (its batch is re-run request by request); a request whose copy event
        // reports an error fails alone with GLT_E_DEVICE
        std::vector<Graph> pool;
        for (int i = 0; i < 50; i++) pool.push_back(make_graph(rng, 100 + rng() % 900, rng() % 5000, false));
        pool.push_back(make_graph(rng, 1000, 3000000, false));   // 24 MB: above a 16 MiB pool
        pool.push_back(make_graph(rng, 500, 2000, true));        // invalid
        std::vector<int> idx, expect;
        std::vector<double> at;
        for (int i = 0; i < 600; i++) {
            int k = (int)(rng() % 50);
            int want = GLT_OK;
            if (i == 101) { k = 50; want = GLT_E_OOM; }
            if (i % 97 == 3) { k = 51; want = GLT_E_NOT_SYMMETRIC; }
            idx.push_back(k);
            at.push_back(i * 1e-4);
            expect.push_back(want);
        }
        // the 251st copy reports an error: request 251 (admission is in request order, and the
        // oversized request 101 is never copied)
        expect[251] = GLT_E_DEVICE;
        glt_server_opts o{};
        o.resident_bytes = (size_t)16 << 20;
        stub_configure(250, 2);
        fails += report("failing requests fail alone", run(o, pool, idx, at, expect, 20.0));
    }
    {   // the served mix: Poisson arrivals at 2000 requests/s for 3 s, 99 % graphs of the batch
        // mix and 1 % graphs of 2,000,000 edges, a stub count time of 2 ns per edge
        std::vector<Graph> pool;
        std::uniform_real_distribution<double> U(0, 1);
        for (int i = 0; i < 400; i++) {
            const int64_t n = 50 + rng() % 4951;
            const double d = 4 + 60 * U(rng);
            pool.push_back(make_graph(rng, n, (int64_t)(n * d / 2), false));
        }
        for (int i = 0; i < 4; i++) pool.push_back(make_graph(rng, 200000, 2000000, false));
        std::vector<int> idx, expect;
        std::vector<double> at;
        std::exponential_distribution<double> gap(2000.0);
        double t = 0;
        while ((t += gap(rng)) < 3.0) {
            idx.push_back(U(rng) < 0.01 ? 400 + (int)(rng() % 4) : (int)(rng() % 400));
            at.push_back(t);
            expect.push_back(GLT_OK);
        }
        glt_server_opts o{};
        stub_configure(-1, 2);
        fails += report("served mix", run(o, pool, idx, at, expect, 20.0));
    }
    return fails ? 1 : 0;
}
