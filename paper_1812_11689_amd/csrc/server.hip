// Serving loop over a resident forest: continuous batching of kNN query requests.
//
// Requests (a block of m query rows and K, Alg. 3 search) are queued by rpf_server_submit
// and served by `slots` worker threads, each with its own HIP stream.  A free slot takes
// the oldest waiting request together with every later waiting request of the same K, up
// to max_batch_rows rows, and runs them as one batch through the query path (routing,
// grouping by leaf, MFMA tiles, merge, re-rank); the outputs of the batch are contiguous
// per request and are copied back to each request's own arrays.  Requests that arrive
// while batches run wait for the next free slot, and a batch is admitted only while the
// workspace bytes of the batches in flight stay within the memory budget, so work of
// several batches overlaps on the device without over-committing memory.
//
// The result of a request does not depend on its batch: the query path returns the exact
// top-K of the request's leaf union under the binary64 ranking.
//
// Latency of a request = time from its submit call to the completion of its batch, seen by
// the slot thread after a stream synchronisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rpf_internal.h"

namespace rpf {
namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    const float *Q = nullptr;
    int64_t m = 0;
    int32_t K = 0;
    int32_t *out_idx = nullptr;
    float *out_dist = nullptr;
    hipEvent_t ready = nullptr;  // recorded on the submitter's stream: Q holds its values
    Clock::time_point t_submit, t_done;
    int state = 0;               // 0 waiting, 1 running, 2 done
    rpf_status status = RPF_OK;
    std::string err;
};

}  // namespace
}  // namespace rpf

struct rpf_server {
    const rpf_forest *f = nullptr;
    int device = 0;
    rpf_server_config cfg{};
    std::mutex mu;
    std::condition_variable cv_work;  // slots wait for requests / memory
    std::condition_variable cv_done;  // waiters wait for completions
    std::deque<rpf::Request *> waiting;
    std::unordered_map<uint64_t, rpf::Request *> live;  // submitted, not yet collected
    std::vector<std::thread> threads;
    std::vector<hipStream_t> streams;
    uint64_t next_ticket = 1;
    uint64_t inflight_bytes = 0;
    int running_batches = 0;
    bool stop = false;
    // statistics since creation or the last reset
    std::vector<double> lat;
    int64_t rows_done = 0, requests_done = 0, batches = 0, batch_rows = 0, failed = 0;
    // device-side span of every batch (HIP events on the slot's stream, in ms after `ref`,
    // an event completed at creation), the last kLogCap batches
    hipEvent_t ref = nullptr;
    std::vector<rpf_server_batch> log;
    rpf::Clock::time_point t_first, t_last;
    bool have_first = false;
};

namespace rpf {
namespace {

constexpr size_t kLogCap = 1 << 16;

// The requests of a batch, up to kGroup at a time, as kernel arguments: their query rows are
// gathered into the batch's contiguous block, and the batch's outputs scattered back to each
// request's own arrays, by one launch each (rather than three copies per request).
constexpr int kGroup = 48;
struct GroupTable {
    const float *q[kGroup];
    int32_t *oi[kGroup];
    float *od[kGroup];
    int64_t row0[kGroup + 1];  // first row of each request in the batch block; row0[count] = end
    int count;
};

__global__ __launch_bounds__(256) void k_gather_rows(GroupTable g, float *__restrict__ dst, int d) {
    const int64_t total = (g.row0[g.count] - g.row0[0]) * d;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = g.row0[0] + i / d;
        int k = 0;
        while (row >= g.row0[k + 1]) k++;
        dst[g.row0[0] * d + i] = g.q[k][(row - g.row0[k]) * d + i % d];
    }
}

__global__ __launch_bounds__(256) void k_scatter_rows(GroupTable g, const int32_t *__restrict__ si,
                                                      const float *__restrict__ sd, int K) {
    const int64_t total = (g.row0[g.count] - g.row0[0]) * K;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = g.row0[0] + i / K;
        int k = 0;
        while (row >= g.row0[k + 1]) k++;
        const int64_t at = (row - g.row0[k]) * K + i % K;
        g.oi[k][at] = si[g.row0[0] * K + i];
        g.od[k][at] = sd[g.row0[0] * K + i];
    }
}

void finish(rpf_server *sv, std::vector<Request *> &batch, rpf_status st, const std::string &err, uint64_t bytes,
            const rpf_server_batch &span) {
    const auto now = Clock::now();
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->log.size() < kLogCap) sv->log.push_back(span);
    sv->inflight_bytes -= bytes;
    sv->running_batches--;
    int64_t rows = 0;
    for (Request *r : batch) {
        r->t_done = now;
        r->status = st;
        r->err = err;
        r->state = 2;
        rows += r->m;
        if (st == RPF_OK) {
            sv->lat.push_back(std::chrono::duration<double>(now - r->t_submit).count());
            sv->rows_done += r->m;
            sv->requests_done++;
        } else {
            sv->failed++;
        }
    }
    sv->batches++;
    sv->batch_rows += rows;
    sv->t_last = now;
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();
}

void slot_main(rpf_server *sv, int slot) {
    hipSetDevice(sv->device);
    hipStream_t s = sv->streams[slot];
    const int d = forest_dim(sv->f);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // batch start / end on this slot's stream
    hipEventCreate(&ev0);
    hipEventCreate(&ev1);
    struct Drop {
        hipEvent_t a, b;
        ~Drop() {
            hipEventDestroy(a);
            hipEventDestroy(b);
        }
    } drop{ev0, ev1};
    for (;;) {
        std::vector<Request *> batch;
        uint64_t bytes = 0;
        int64_t rows = 0;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            for (;;) {
                if (sv->stop && sv->waiting.empty()) return;
                if (!sv->waiting.empty()) {
                    // the oldest request and every later one of the same K, up to the row cap
                    Request *head = sv->waiting.front();
                    const int K = head->K;
                    int64_t r = 0;
                    std::vector<size_t> pick;
                    for (size_t i = 0; i < sv->waiting.size(); i++) {
                        Request *q = sv->waiting[i];
                        if (q->K != K) continue;
                        if (!pick.empty() && r + q->m > sv->cfg.max_batch_rows) break;
                        pick.push_back(i);
                        r += q->m;
                    }
                    const uint64_t need = query_workspace_bytes(sv->f, r, K) +
                                          (pick.size() > 1 ? (uint64_t)r * ((uint64_t)d * 4 + (uint64_t)K * 8) : 0);
                    if (sv->running_batches == 0 || sv->inflight_bytes + need <= sv->cfg.mem_budget_bytes) {
                        for (size_t k = pick.size(); k-- > 0;) {
                            batch.push_back(sv->waiting[pick[k]]);
                            sv->waiting.erase(sv->waiting.begin() + (long)pick[k]);
                        }
                        std::reverse(batch.begin(), batch.end());
                        for (Request *q : batch) q->state = 1;
                        sv->inflight_bytes += need;
                        sv->running_batches++;
                        bytes = need;
                        rows = r;
                        break;
                    }
                }
                sv->cv_work.wait(lk);
            }
        }
        // run the batch on this slot's stream
        for (Request *q : batch) hipStreamWaitEvent(s, q->ready, 0);
        hipEventRecord(ev0, s);
        rpf_status st = RPF_OK;
        std::string err;
        const int K = batch[0]->K;
        if (batch.size() == 1) {
            Request *q = batch[0];
            st = knn_query(sv->f, q->Q, q->m, K, q->out_idx, q->out_dist, s);
        } else {
            float *Qb = static_cast<float *>(cache_alloc((size_t)rows * d * 4, s));
            int32_t *ib = static_cast<int32_t *>(cache_alloc((size_t)rows * K * 4, s));
            float *db = static_cast<float *>(cache_alloc((size_t)rows * K * 4, s));
            if (!Qb || !ib || !db) {
                st = fail(RPF_ENOMEM, "rpf_server: batch staging allocation failed");
            } else {
                // the batch's requests in groups of kGroup: one gather launch per group
                std::vector<GroupTable> groups;
                int64_t off = 0;
                for (size_t b = 0; b < batch.size(); b += kGroup) {
                    GroupTable g{};
                    g.count = (int)std::min<size_t>(kGroup, batch.size() - b);
                    for (int k = 0; k < g.count; k++) {
                        Request *q = batch[b + k];
                        g.q[k] = q->Q;
                        g.oi[k] = q->out_idx;
                        g.od[k] = q->out_dist;
                        g.row0[k] = off;
                        off += q->m;
                    }
                    g.row0[g.count] = off;
                    groups.push_back(g);
                }
                auto blocks = [](int64_t elems) {
                    return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((elems + 255) / 256, 4096)));
                };
                for (const GroupTable &g : groups)
                    hipLaunchKernelGGL(k_gather_rows, blocks((g.row0[g.count] - g.row0[0]) * d), dim3(256), 0, s, g,
                                       Qb, d);
                launch_check(s, "k_gather_rows");
                st = knn_query(sv->f, Qb, rows, K, ib, db, s);
                if (st == RPF_OK) {
                    for (const GroupTable &g : groups)
                        hipLaunchKernelGGL(k_scatter_rows, blocks((g.row0[g.count] - g.row0[0]) * K), dim3(256), 0, s,
                                           g, ib, db, K);
                    launch_check(s, "k_scatter_rows");
                    const std::string le = take_launch_error();
                    if (!le.empty()) st = fail(RPF_EDEVICE, "rpf_server: " + le);
                }
            }
            cache_free(Qb, s);
            cache_free(ib, s);
            cache_free(db, s);
        }
        if (st != RPF_OK) err = rpf_last_error();
        forest_fault_mirror(sv->f, s);
        hipEventRecord(ev1, s);
        const rpf_status sync = check_hip(hipStreamSynchronize(s), "rpf_server batch");
        rpf_server_batch span{};
        span.slot = slot;
        span.requests = (int32_t)batch.size();
        span.rows = rows;
        float t0 = -1.f, t1 = -1.f;
        if (sync == RPF_OK && hipEventElapsedTime(&t0, sv->ref, ev0) == hipSuccess &&
            hipEventElapsedTime(&t1, sv->ref, ev1) == hipSuccess) {
            span.start_ms = t0;
            span.end_ms = t1;
        } else {
            span.start_ms = span.end_ms = -1.0;
        }
        if (st == RPF_OK && sync != RPF_OK) {
            st = sync;
            err = rpf_last_error();
        }
        // an out-of-range candidate index met by this batch or an earlier one fails the batch
        if (st == RPF_OK && forest_fault_seen(sv->f)) {
            st = fault_error(sv->f, "rpf_server batch");
            err = rpf_last_error();
        }
        finish(sv, batch, st, err, bytes, span);
    }
}

}  // namespace
}  // namespace rpf

using namespace rpf;

extern "C" {

rpf_status rpf_server_create(const rpf_forest *f, const rpf_server_config *cfg, rpf_server **out) {
    if (out) *out = nullptr;
    if (!f || !cfg || !out) return fail(RPF_EINVAL, "rpf_server_create: NULL pointer");
    if (cfg->slots < 1 || cfg->slots > 16) return fail(RPF_EINVAL, "rpf_server_create: slots must be in [1, 16]");
    if (cfg->max_batch_rows < 1) return fail(RPF_EINVAL, "rpf_server_create: max_batch_rows must be >= 1");
    if (cfg->max_queue < 1) return fail(RPF_EINVAL, "rpf_server_create: max_queue must be >= 1");
    if (forest_uniform(f)) return fail(RPF_EINVAL, "rpf_server_create: queries need a median-rule forest");
    rpf_server *sv = new rpf_server();
    sv->f = f;
    sv->cfg = *cfg;
    if (sv->cfg.mem_budget_bytes == 0) sv->cfg.mem_budget_bytes = UINT64_MAX;
    hipGetDevice(&sv->device);
    for (int i = 0; i < cfg->slots; i++) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t t : sv->streams) hipStreamDestroy(t);
            delete sv;
            return fail(RPF_EDEVICE, "rpf_server_create: stream creation failed");
        }
        sv->streams.push_back(s);
    }
    // the forest's query copies are made now, on the first slot's stream, not by the first batch
    rpf_status st = ensure_leaf_copies(f, sv->streams[0]);
    if (st == RPF_OK) st = check_hip(hipEventCreate(&sv->ref), "rpf_server_create event");
    if (st == RPF_OK) st = check_hip(hipEventRecord(sv->ref, sv->streams[0]), "rpf_server_create event");
    if (st == RPF_OK) st = check_hip(hipStreamSynchronize(sv->streams[0]), "rpf_server_create");
    if (st != RPF_OK) {
        for (hipStream_t t : sv->streams) hipStreamDestroy(t);
        if (sv->ref) hipEventDestroy(sv->ref);
        delete sv;
        return st;
    }
    for (int i = 0; i < cfg->slots; i++) sv->threads.emplace_back(slot_main, sv, i);
    *out = sv;
    return RPF_OK;
}

rpf_status rpf_server_submit(rpf_server *sv, const float *Q, int64_t m, int32_t K, int32_t *out_idx,
                             float *out_dist, void *stream, uint64_t *ticket) {
    if (ticket) *ticket = 0;
    if (!sv || !ticket) return fail(RPF_EINVAL, "rpf_server_submit: NULL pointer");
    if (m < 1) return fail(RPF_EINVAL, "rpf_server_submit: m must be >= 1");
    if (!Q || !out_idx || !out_dist) return fail(RPF_EINVAL, "rpf_server_submit: NULL array");
    if (K < 1 || K > forest_points(sv->f) || K > 256)
        return fail(RPF_EINVAL, "rpf_server_submit: K must be in [1, min(n, 256)]");
    if (forest_fault_seen(sv->f)) return fault_error(sv->f, "rpf_server_submit");
    Request *r = new Request();
    if (hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(r->ready, (hipStream_t)stream) != hipSuccess) {
        if (r->ready) hipEventDestroy(r->ready);
        delete r;
        return fail(RPF_EDEVICE, "rpf_server_submit: event on the submitting stream failed");
    }
    r->Q = Q;
    r->m = m;
    r->K = K;
    r->out_idx = out_idx;
    r->out_dist = out_dist;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stop) {
            hipEventDestroy(r->ready);
            delete r;
            return fail(RPF_EINVAL, "rpf_server_submit: server is shutting down");
        }
        if ((int64_t)sv->waiting.size() >= sv->cfg.max_queue) {
            hipEventDestroy(r->ready);
            delete r;
            return fail(RPF_EBUSY, "rpf_server_submit: queue full");
        }
        r->ticket = sv->next_ticket++;
        if (!sv->have_first) {
            sv->t_first = r->t_submit;
            sv->have_first = true;
        }
        sv->waiting.push_back(r);
        sv->live[r->ticket] = r;
    }
    sv->cv_work.notify_one();
    *ticket = r->ticket;
    return RPF_OK;
}

static rpf_status collect(rpf_server *sv, std::unique_lock<std::mutex> &lk, uint64_t ticket, double *latency) {
    auto it = sv->live.find(ticket);
    Request *r = it->second;
    sv->live.erase(it);
    lk.unlock();
    const rpf_status st = r->status;
    if (latency) *latency = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    if (st != RPF_OK) fail(st, r->err);
    hipEventDestroy(r->ready);
    delete r;
    return st;
}

rpf_status rpf_server_poll(rpf_server *sv, uint64_t ticket, int32_t *done, double *latency) {
    if (done) *done = 0;
    if (!sv || !done) return fail(RPF_EINVAL, "rpf_server_poll: NULL pointer");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->live.find(ticket);
    if (it == sv->live.end()) return fail(RPF_EINVAL, "rpf_server_poll: unknown ticket");
    if (it->second->state != 2) return RPF_ENOTREADY;
    *done = 1;
    return collect(sv, lk, ticket, latency);
}

rpf_status rpf_server_wait(rpf_server *sv, uint64_t ticket, double *latency) {
    if (!sv) return fail(RPF_EINVAL, "rpf_server_wait: NULL pointer");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->live.find(ticket);
    if (it == sv->live.end()) return fail(RPF_EINVAL, "rpf_server_wait: unknown ticket");
    Request *r = it->second;
    sv->cv_done.wait(lk, [&] { return r->state == 2; });
    return collect(sv, lk, ticket, latency);
}

rpf_status rpf_server_stats(rpf_server *sv, rpf_server_report *out) {
    if (!sv || !out) return fail(RPF_EINVAL, "rpf_server_stats: NULL pointer");
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = rpf_server_report{};
    out->requests = sv->requests_done;
    out->rows = sv->rows_done;
    out->batches = sv->batches;
    out->mean_batch_rows = sv->batches ? (double)sv->batch_rows / (double)sv->batches : 0.0;
    out->failed_requests = sv->failed;
    out->bad_index_rows = (int64_t)forest_fault_seen(sv->f);
    if (!sv->lat.empty()) {
        std::vector<double> v = sv->lat;
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            const size_t i = (size_t)std::min<double>((double)v.size() - 1, std::ceil(p * (double)v.size()) - 1);
            return v[i];
        };
        out->p50_s = pct(0.50);
        out->p99_s = pct(0.99);
        out->max_s = v.back();
    }
    if (sv->have_first && sv->rows_done > 0) {
        const double span = std::chrono::duration<double>(sv->t_last - sv->t_first).count();
        out->rows_per_s = span > 0 ? (double)sv->rows_done / span : 0.0;
    }
    return RPF_OK;
}

rpf_status rpf_server_batch_log(rpf_server *sv, rpf_server_batch *out, int32_t cap, int32_t *count) {
    if (!sv || !count || (cap > 0 && !out)) return fail(RPF_EINVAL, "rpf_server_batch_log: NULL pointer");
    std::lock_guard<std::mutex> lk(sv->mu);
    const int32_t k = (int32_t)sv->log.size();
    for (int32_t i = 0; i < std::min(k, cap); i++) out[i] = sv->log[i];
    *count = k;
    return RPF_OK;
}

rpf_status rpf_server_reset_stats(rpf_server *sv) {
    if (!sv) return fail(RPF_EINVAL, "rpf_server_reset_stats: NULL pointer");
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->lat.clear();
    sv->log.clear();
    sv->rows_done = sv->requests_done = sv->batches = sv->batch_rows = sv->failed = 0;
    sv->have_first = false;
    return RPF_OK;
}

rpf_status rpf_server_destroy(rpf_server *sv) {
    if (!sv) return RPF_OK;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    for (auto &t : sv->threads) t.join();  // the slots drain every waiting request first
    for (hipStream_t s : sv->streams) hipStreamDestroy(s);
    if (sv->ref) hipEventDestroy(sv->ref);
    for (auto &kv : sv->live) {
        hipEventDestroy(kv.second->ready);
        delete kv.second;
    }
    delete sv;
    return RPF_OK;
}

}  // extern "C"
