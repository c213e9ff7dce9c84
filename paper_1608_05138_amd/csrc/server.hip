// server.hip -- a request loop with continuous batching for graph-count requests.
//
// Requests (host CSR graphs) are queued on submit.  An admission thread moves them, in
// arrival order, into a device-resident pool when the pool's budget has room, copying them
// on a copy stream.  Two compute lanes (each a thread with its own handle, workspace and
// stream) repeatedly take every admitted request of their size class whose copy has
// finished (up to an edge budget per launch) and count the group with one batched call;
// requests that arrive while a batch runs are admitted and copied meanwhile and join the
// next batch of their lane.  Large requests (more than large_edges edges) have a lane of
// their own, so their launches overlap on the device with the small-request batches
// instead of delaying them.  Each request's result (17 global counts) is queued with its
// timestamps for poll().  A request whose graph is invalid fails alone: when a batch
// reports a validation error, its requests are re-run one by one.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/glt.h"

glt_status glt_run_batch_ptrs(glt_ctx* ctx, int64_t B, const int64_t* vb, const int64_t* sb,
                              const int* const* rp_ptrs, const int* const* col_ptrs, glt_u128* out,
                              hipStream_t st);

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t id = 0;
    int n = 0, m = 0;
    std::vector<int> buf;          // row offsets (n+1, int32) followed by columns (2m)
    double t_submit = 0, t_admit = 0;
    size_t off = 0, bytes = 0;     // slot in the device pool
    hipEvent_t ev = nullptr;       // completion of the slot's host-to-device copy
};

// First-fit allocator over [0, cap) with coalescing of freed ranges.
struct Pool {
    size_t cap = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    void init(size_t c) { cap = c; free_.clear(); free_[0] = c; }
    bool alloc(size_t len, size_t& off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= len) {
                off = it->first;
                const size_t rest = it->second - len;
                free_.erase(it);
                if (rest) free_[off + len] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t len) {
        auto it = free_.emplace(off, len).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

constexpr size_t kSlotAlign = 256;

}  // namespace

struct glt_server;

// One compute lane: a handle (workspace), a stream, a thread and its admitted queue.
struct Lane {
    glt_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    std::deque<Request*> admitted;
    std::condition_variable cv;
    std::thread thr;
};

struct glt_server {
    glt_server_opts opts{};
    int nlanes = 2;
    Lane lanes[2];
    hipStream_t copy_stream = nullptr;
    char* pool_base = nullptr;
    Pool pool;
    std::mutex mu;
    std::condition_variable cv_admit, cv_done;
    std::deque<Request*> pending;
    std::deque<glt_result> done;
    std::vector<hipEvent_t> spare_events;
    bool stop = false;
    int64_t inflight = 0;           // submitted and not yet completed
    std::thread admit_thr;

    int lane_of(const Request* r) const {
        return (nlanes > 1 && (int64_t)r->m > (int64_t)opts.large_edges) ? 1 : 0;
    }

    hipEvent_t get_event() {
        if (!spare_events.empty()) {
            hipEvent_t e = spare_events.back();
            spare_events.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }

    void finish(Request* r, int status, const glt_u128* X, double t_start, double t_done, int batch) {
        glt_result res;
        memset(&res, 0, sizeof(res));
        res.req_id = r->id;
        res.status = status;
        res.batch_graphs = batch;
        if (X) memcpy(res.X, X, sizeof(res.X));
        res.t_submit = r->t_submit;
        res.t_admit = r->t_admit;
        res.t_start = t_start;
        res.t_done = t_done;
        done.push_back(res);
        inflight--;
    }

    void admit_loop() {
        (void)hipSetDevice(opts.device);
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            cv_admit.wait(lk, [&] { return stop || !pending.empty(); });
            if (stop) return;
            Request* r = pending.front();
            if (r->bytes > pool.cap) {      // can never fit: fail it alone
                pending.pop_front();
                finish(r, GLT_E_OOM, nullptr, now_s(), now_s(), 0);
                delete r;
                cv_done.notify_all();
                continue;
            }
            size_t off = 0;
            if (!pool.alloc(r->bytes, off)) {
                cv_admit.wait(lk);           // woken when the compute thread frees slots
                continue;
            }
            pending.pop_front();
            r->off = off;
            r->ev = get_event();
            lk.unlock();
            bool ok = r->ev != nullptr &&
                      hipMemcpyAsync(pool_base + off, r->buf.data(), r->buf.size() * sizeof(int),
                                     hipMemcpyHostToDevice, copy_stream) == hipSuccess &&
                      hipEventRecord(r->ev, copy_stream) == hipSuccess;
            r->t_admit = now_s();
            lk.lock();
            if (!ok) {
                pool.release(r->off, r->bytes);
                finish(r, GLT_E_DEVICE, nullptr, r->t_admit, now_s(), 0);
                if (r->ev) spare_events.push_back(r->ev);
                delete r;
                cv_done.notify_all();
                continue;
            }
            Lane& ln = lanes[lane_of(r)];
            ln.admitted.push_back(r);
            ln.cv.notify_one();
        }
    }

    // A request whose copy to the device reported an error (its event's query or wait did not
    // return success) fails alone with GLT_E_DEVICE; its slot is released and its event, in
    // an unknown state, destroyed.  Called with the lock held.
    void fail_copy(Request* r) {
        const double t = now_s();
        finish(r, GLT_E_DEVICE, nullptr, t, t, 0);
        pool.release(r->off, r->bytes);
        (void)hipEventDestroy(r->ev);
        delete r;
        cv_admit.notify_all();
        cv_done.notify_all();
    }

    // Runs one group; on a validation error, re-runs its requests one by one so that only
    // the invalid ones fail.
    void run_group(Lane& ln, std::vector<Request*>& grp, std::vector<int>& status, std::vector<glt_u128>& X) {
        const int64_t B = (int64_t)grp.size();
        std::vector<int64_t> vb(B + 1), sb(B + 1);
        std::vector<const int*> rps(B), cols(B);
        vb[0] = sb[0] = 0;
        for (int64_t g = 0; g < B; g++) {
            Request* r = grp[g];
            vb[g + 1] = vb[g] + r->n;
            sb[g + 1] = sb[g] + 2 * (int64_t)r->m;
            rps[g] = (const int*)(pool_base + r->off);
            cols[g] = rps[g] + (r->n + 1);
        }
        X.assign((size_t)B * 17, glt_u128{0, 0});
        status.assign(B, GLT_OK);
        glt_status rc = glt_run_batch_ptrs(ln.ctx, B, vb.data(), sb.data(), rps.data(), cols.data(), X.data(),
                                           ln.stream);
        if (rc == GLT_OK) return;
        const bool input_error = rc == GLT_E_INVALID_ARG || rc == GLT_E_NOT_SIMPLE || rc == GLT_E_NOT_SYMMETRIC ||
                                 rc == GLT_E_UNSUPPORTED;
        if (!input_error || B == 1) {
            for (auto& st : status) st = rc;
            return;
        }
        for (int64_t g = 0; g < B; g++) {
            int64_t v1[2] = {0, grp[g]->n}, s1[2] = {0, 2 * (int64_t)grp[g]->m};
            status[g] = glt_run_batch_ptrs(ln.ctx, 1, v1, s1, &rps[g], &cols[g], &X[(size_t)g * 17], ln.stream);
        }
    }

    void compute_loop(int li) {
        (void)hipSetDevice(opts.device);
        Lane& ln = lanes[li];
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            ln.cv.wait(lk, [&] { return stop || !ln.admitted.empty(); });
            if (stop) return;
            // the oldest admitted request of the lane goes first; wait for its copy if needed
            // (only this thread removes entries of ln.admitted, so it stays at the front)
            Request* head = ln.admitted.front();
            hipError_t q = hipEventQuery(head->ev);
            if (q == hipErrorNotReady) {
                lk.unlock();
                q = hipEventSynchronize(head->ev);
                lk.lock();
            }
            if (q != hipSuccess) {
                ln.admitted.pop_front();
                fail_copy(head);
                continue;
            }
            std::vector<Request*> grp;
            int64_t edges = 0;
            const int64_t maxg = opts.max_batch_graphs > 0 ? opts.max_batch_graphs : INT64_MAX;
            while (!ln.admitted.empty() && (int64_t)grp.size() < maxg) {
                Request* r = ln.admitted.front();
                if (!grp.empty() && edges + r->m > opts.max_batch_edges) break;
                const hipError_t qr = hipEventQuery(r->ev);
                if (qr == hipErrorNotReady) break;
                ln.admitted.pop_front();
                if (qr != hipSuccess) {   // its copy failed: it fails alone
                    fail_copy(r);
                    continue;
                }
                grp.push_back(r);
                edges += r->m;
            }
            if (grp.empty()) continue;
            lk.unlock();
            const double t_start = now_s();
            std::vector<int> status;
            std::vector<glt_u128> X;
            run_group(ln, grp, status, X);
            const double t_done = now_s();
            lk.lock();
            for (size_t g = 0; g < grp.size(); g++) {
                Request* r = grp[g];
                finish(r, status[g], status[g] == GLT_OK ? &X[g * 17] : nullptr, t_start, t_done, (int)grp.size());
                pool.release(r->off, r->bytes);
                spare_events.push_back(r->ev);
                delete r;
            }
            cv_admit.notify_all();
            cv_done.notify_all();
        }
    }
};

extern "C" {

double glt_server_clock(void) { return now_s(); }

glt_status glt_server_create(const glt_server_opts* opts, glt_server** out) {
    if (!out) return GLT_E_INVALID_ARG;
    *out = nullptr;
    glt_server* s = new (std::nothrow) glt_server();
    if (!s) return GLT_E_OOM;
    if (opts) s->opts = *opts;
    if (s->opts.max_batch_edges <= 0) s->opts.max_batch_edges = 8 << 20;
    if (s->opts.resident_bytes == 0) s->opts.resident_bytes = (size_t)4 << 30;
    if (s->opts.max_pending <= 0) s->opts.max_pending = 1 << 20;
    if (s->opts.large_edges == 0) s->opts.large_edges = 1 << 18;
    s->nlanes = s->opts.large_edges < 0 ? 1 : 2;
    for (int i = 0; i < s->nlanes; i++) {
        glt_status rc = glt_create(s->opts.device, s->opts.workspace_bytes, &s->lanes[i].ctx);
        if (rc != GLT_OK) { glt_server_destroy(s); return rc; }
    }
    if (hipSetDevice(s->opts.device) != hipSuccess ||
        hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) != hipSuccess) {
        glt_server_destroy(s);
        return GLT_E_DEVICE;
    }
    for (int i = 0; i < s->nlanes; i++)
        if (hipStreamCreateWithFlags(&s->lanes[i].stream, hipStreamNonBlocking) != hipSuccess) {
            glt_server_destroy(s);
            return GLT_E_DEVICE;
        }
    if (hipMalloc((void**)&s->pool_base, s->opts.resident_bytes) != hipSuccess) {
        (void)hipGetLastError();
        s->pool_base = nullptr;
        glt_server_destroy(s);
        return GLT_E_OOM;
    }
    s->pool.init(s->opts.resident_bytes);
    s->admit_thr = std::thread([s] { s->admit_loop(); });
    for (int i = 0; i < s->nlanes; i++) s->lanes[i].thr = std::thread([s, i] { s->compute_loop(i); });
    *out = s;
    return GLT_OK;
}

glt_status glt_server_submit(glt_server* s, const glt_csr* g, uint64_t req_id) {
    if (!s || !g) return GLT_E_INVALID_ARG;
    if (g->on_device) return GLT_E_INVALID_ARG;
    if (g->n < 0 || g->m < 0 || !g->row_ptr || (g->m > 0 && !g->col)) return GLT_E_INVALID_ARG;
    if (g->n >= ((int64_t)1 << 30) || 2 * g->m >= ((int64_t)1 << 30)) return GLT_E_UNSUPPORTED;
    Request* r = new (std::nothrow) Request();
    if (!r) return GLT_E_OOM;
    r->id = req_id;
    r->n = (int)g->n;
    r->m = (int)g->m;
    r->t_submit = now_s();
    const int64_t S = 2 * g->m;
    r->buf.resize((size_t)(g->n + 1 + S));
    if (g->offsets_are_64bit) {
        const int64_t* rp = (const int64_t*)g->row_ptr;
        for (int64_t i = 0; i <= g->n; i++) {
            const int64_t v = rp[i];
            r->buf[i] = (v < INT32_MIN || v > INT32_MAX) ? -1 : (int)v;   // out of range: rejected later
        }
    } else {
        memcpy(r->buf.data(), g->row_ptr, (size_t)(g->n + 1) * 4);
    }
    if (S > 0) memcpy(r->buf.data() + g->n + 1, g->col, (size_t)S * 4);
    r->bytes = (r->buf.size() * sizeof(int) + kSlotAlign - 1) / kSlotAlign * kSlotAlign;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if ((int64_t)s->pending.size() >= s->opts.max_pending) {
            delete r;
            return GLT_E_BUSY;
        }
        s->pending.push_back(r);
        s->inflight++;
    }
    s->cv_admit.notify_one();
    return GLT_OK;
}

int glt_server_poll(glt_server* s, glt_result* out, int max, int timeout_us) {
    if (!s || !out || max <= 0) return 0;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && timeout_us > 0)
        s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return !s->done.empty(); });
    int k = 0;
    while (k < max && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    return k;
}

int64_t glt_server_inflight(glt_server* s) {
    if (!s) return 0;
    std::lock_guard<std::mutex> lk(s->mu);
    return s->inflight;
}

void glt_server_destroy(glt_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_admit.notify_all();
    for (Lane& ln : s->lanes) ln.cv.notify_all();
    s->cv_done.notify_all();
    if (s->admit_thr.joinable()) s->admit_thr.join();
    for (Lane& ln : s->lanes)
        if (ln.thr.joinable()) ln.thr.join();
    (void)hipSetDevice(s->opts.device);
    if (s->copy_stream) (void)hipStreamSynchronize(s->copy_stream);
    for (Lane& ln : s->lanes)
        if (ln.stream) (void)hipStreamSynchronize(ln.stream);
    for (Request* r : s->pending) delete r;
    for (Lane& ln : s->lanes)
        for (Request* r : ln.admitted) {
            if (r->ev) s->spare_events.push_back(r->ev);
            delete r;
        }
    for (hipEvent_t e : s->spare_events) (void)hipEventDestroy(e);
    if (s->pool_base) (void)hipFree(s->pool_base);
    if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
    for (Lane& ln : s->lanes) {
        if (ln.stream) (void)hipStreamDestroy(ln.stream);
        glt_destroy(ln.ctx);
    }
    delete s;
}

}  // extern "C"
