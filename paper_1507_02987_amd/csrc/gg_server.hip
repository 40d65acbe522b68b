// Served form of the search: a request loop with continuous batching under a
// device hit-buffer budget.
//
// gg_serve_submit queues a request.  A counting thread takes every newly queued
// request, counts its index hits exactly with the search's own encode and count
// kernels (a batched call on its own stream), and moves it to the admission
// queue.  Worker threads, each running its batches on its own stream and
// workspace, admit from that queue in arrival order whatever fits the free
// in-flight slots and the free part of the hit budget (16 bytes of hit keys per
// hit), run it as one batch, and release its slots and bytes the moment the
// batch's results are in host memory, so requests that arrive while others are
// on the GPU start on the next free worker and their work overlaps on the device.
//
// Admission rules, in queue order:
// * A heavy request (more than kHeavyHits hits) runs alone in its batch, so the
//   light requests admitted around it do not wait for it.
// * Light requests share a batch up to kBatchHits hits and kBatchQueries queries.
// * A request that does not fit now keeps its bytes reserved: requests behind it
//   are admitted only into the budget left beyond the reservation, so it is not
//   overtaken for ever.  A request whose hits alone exceed the budget reserves the
//   whole budget, runs when nothing else is in flight, and is searched in ranges
//   of data-bank sequences that each fit the budget.
// A query's hits do not depend on the batch it lands in: every stage keeps the
// queries of a batch apart.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gg.h"
#include "gg_internal.h"

namespace gg {
gg_status search_batch_budget(const gg_index *ix, const char *qbuf, const int64_t *qoff,
                              int64_t n_q, const gg_params *params, gg_hit *out, int32_t cap,
                              int32_t *n_out, gg_stats *stats, uint64_t budget, bool device);
gg_status count_hits(const gg_index *ix, const char *qbuf, const int64_t *qoff, int64_t n_q,
                     uint64_t *hits);
uint64_t index_budget(const gg_index *ix);
}  // namespace gg

namespace {

constexpr int kWorkers = 4;                    // concurrent batches (one stream each)
constexpr uint64_t kHeavyHits = 1ull << 24;    // a request above this runs alone
constexpr uint64_t kBatchHits = 1ull << 26;    // hits of one batch of light requests
constexpr int32_t kBatchQueries = 512;         // requests of one batch
constexpr size_t kCountBatch = 4096;           // requests counted per counting call
constexpr size_t kScanAhead = 8192;            // queued requests one admission pass looks at
constexpr uint64_t kBytesPerHit = 16;          // two 8-byte hit keys (sort input and output)

bool valid_base(char c)
{
    switch (c) {
    case 'A': case 'C': case 'G': case 'T': case 'U':
    case 'a': case 'c': case 'g': case 't': case 'u':
        return true;
    default:
        return false;
    }
}

struct Request {
    std::string query;
    uint64_t hits = 0;     // exact index hits of the query
    uint64_t bytes = 0;    // hit-key bytes it holds while in flight (at most the budget)
    bool done = false;
    gg_status status = GG_OK;
    std::vector<gg_hit> out;
};

}  // namespace

struct gg_server {
    const gg_index *ix = nullptr;
    gg_params params{};
    uint64_t budget = 0;
    int32_t max_slots = 1;
    std::mutex mu;
    std::condition_variable cv_count, cv_admit, cv_done;
    std::deque<uint64_t> uncounted;  // tickets waiting for their hit count
    std::deque<uint64_t> ready;      // counted tickets, in arrival order
    std::unordered_map<uint64_t, Request *> reqs;
    uint64_t inflight_bytes = 0;
    int32_t inflight_slots = 0;
    gg_server_stats stats{};  // totals and peaks since creation
    std::atomic<int32_t> active{0};  // submit and poll calls inside the library
    bool stop = false;
    uint64_t next_ticket = 1;
    std::thread counter;
    std::vector<std::thread> workers;
};

namespace {

void counter_loop(gg_server *sv)
{
    std::vector<uint64_t> take;
    std::vector<Request *> reqs;
    std::vector<char> buf;
    std::vector<int64_t> off;
    std::vector<uint64_t> hits;
    for (;;) {
        take.clear();
        reqs.clear();
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_count.wait(lk, [&] { return sv->stop || !sv->uncounted.empty(); });
            if (sv->stop) return;
            while (!sv->uncounted.empty() && take.size() < kCountBatch) {
                const uint64_t t = sv->uncounted.front();
                sv->uncounted.pop_front();
                take.push_back(t);
                reqs.push_back(sv->reqs.at(t));
            }
        }
        // the requests are not visible to any other thread until they are queued
        // for admission below, so their queries are read without the lock
        const size_t n = reqs.size();
        off.assign(n + 1, 0);
        for (size_t i = 0; i < n; ++i) off[i + 1] = off[i] + (int64_t)reqs[i]->query.size();
        buf.resize((size_t)off[n] + 1);
        for (size_t i = 0; i < n; ++i)
            std::copy(reqs[i]->query.begin(), reqs[i]->query.end(), buf.begin() + off[i]);
        hits.assign(n, 0);
        gg_status st = gg::count_hits(sv->ix, buf.data(), off.data(), (int64_t)n, hits.data());
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            for (size_t i = 0; i < n; ++i) {
                Request *r = reqs[i];
                if (st != GG_OK) {
                    // the request fails at once; its poll reports the status
                    r->status = st;
                    r->done = true;
                    continue;
                }
                r->hits = hits[i];
                r->bytes = std::min<uint64_t>(hits[i] * kBytesPerHit, sv->budget);
                sv->ready.push_back(take[i]);
            }
        }
        sv->cv_admit.notify_all();
        if (st != GG_OK) sv->cv_done.notify_all();
    }
}

// Admission: pick the next batch from the ready queue under the lock (see the
// rules at the top of this file).  Returns false when nothing can start now.
bool admit(gg_server *sv, std::vector<uint64_t> &take, std::vector<Request *> &batch,
           uint64_t &batch_bytes)
{
    take.clear();
    batch.clear();
    batch_bytes = 0;
    uint64_t batch_hits = 0, reserved = 0;
    bool heavy_batch = false;
    size_t looked = 0;
    for (auto it = sv->ready.begin(); it != sv->ready.end() && looked < kScanAhead;) {
        ++looked;
        Request *r = sv->reqs.at(*it);
        const bool heavy = r->hits > kHeavyHits;
        const bool slot = sv->inflight_slots + (int32_t)batch.size() < sv->max_slots;
        const bool fits = sv->inflight_bytes + batch_bytes + reserved + r->bytes <= sv->budget;
        const bool joins = batch.empty() || (!heavy && !heavy_batch &&
                                             batch_hits + r->hits <= kBatchHits &&
                                             (int32_t)batch.size() < kBatchQueries);
        if (slot && fits && joins) {
            take.push_back(*it);
            batch.push_back(r);
            batch_bytes += r->bytes;
            batch_hits += r->hits;
            heavy_batch = heavy;
            it = sv->ready.erase(it);
            if (heavy_batch) break;
            continue;
        }
        if (!slot) break;
        if (!fits) reserved += r->bytes;  // it waits; later requests may not take its bytes
        ++it;
    }
    if (batch.empty()) return false;
    sv->inflight_bytes += batch_bytes;
    sv->inflight_slots += (int32_t)batch.size();
    gg_server_stats &t = sv->stats;
    t.batches += 1;
    t.peak_inflight_bytes = std::max(t.peak_inflight_bytes, sv->inflight_bytes);
    t.peak_inflight_slots = std::max<int64_t>(t.peak_inflight_slots, sv->inflight_slots);
    t.peak_batch_queries = std::max<int64_t>(t.peak_batch_queries, (int64_t)batch.size());
    if (batch.size() == 1 && batch[0]->hits * kBytesPerHit > sv->budget) t.over_budget += 1;
    return true;
}

void worker_loop(gg_server *sv)
{
    const int32_t cap0 = sv->params.max_hits > 0 ? sv->params.max_hits : 4096;
    std::vector<uint64_t> take;
    std::vector<Request *> batch;
    std::vector<char> buf;
    std::vector<int64_t> off;
    std::vector<gg_hit> out;
    std::vector<int32_t> nout;
    for (;;) {
        uint64_t batch_bytes = 0;
        {
            // admit() takes a batch only when it returns true, and then stop was
            // false: a stopping worker holds no batch
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_admit.wait(lk, [&] { return sv->stop || admit(sv, take, batch, batch_bytes); });
            if (sv->stop) return;
        }
        const size_t n = batch.size();
        off.assign(n + 1, 0);
        for (size_t i = 0; i < n; ++i) off[i + 1] = off[i] + (int64_t)batch[i]->query.size();
        buf.resize((size_t)off[n] + 1);
        for (size_t i = 0; i < n; ++i)
            std::copy(batch[i]->query.begin(), batch[i]->query.end(), buf.begin() + off[i]);
        out.resize(n * (size_t)cap0);
        nout.assign(n, 0);
        // the batch's own bytes bound its waves: its hit keys never exceed them
        const uint64_t call_budget = std::max<uint64_t>(batch_bytes, kBytesPerHit);
        gg_status st = gg::search_batch_budget(sv->ix, buf.data(), off.data(), (int64_t)n,
                                               &sv->params, out.data(), cap0, nout.data(), nullptr,
                                               call_budget, false);
        std::vector<gg_status> each(n, st);
        if (st == GG_EBUDGET || st == GG_EINVAL) {
            // one bad or oversized query must not fail its batch-mates: run each alone
            for (size_t i = 0; i < n; ++i) {
                const int64_t o2[2] = {0, off[i + 1] - off[i]};
                each[i] = gg::search_batch_budget(sv->ix, buf.data() + off[i], o2, 1, &sv->params,
                                                  out.data() + i * cap0, cap0, &nout[i], nullptr,
                                                  std::max<uint64_t>(batch[i]->bytes, kBytesPerHit),
                                                  false);
            }
        }
        for (size_t i = 0; i < n; ++i) {
            Request *r = batch[i];
            if (each[i] == GG_OK || each[i] == GG_ETRUNC) {
                if (nout[i] > cap0) {
                    // more alignments than the default room: rerun this query with room for all
                    std::vector<gg_hit> big((size_t)nout[i]);
                    int32_t n2 = 0;
                    const int64_t o2[2] = {0, off[i + 1] - off[i]};
                    r->status = gg::search_batch_budget(
                        sv->ix, buf.data() + off[i], o2, 1, &sv->params, big.data(), nout[i], &n2,
                        nullptr, std::max<uint64_t>(r->bytes, kBytesPerHit), false);
                    big.resize((size_t)std::min(n2, nout[i]));
                    r->out.swap(big);
                } else {
                    r->status = GG_OK;
                    r->out.assign(out.begin() + i * cap0, out.begin() + i * cap0 + nout[i]);
                }
            } else {
                r->status = each[i];
            }
        }
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            for (Request *r : batch) r->done = true;
            sv->stats.completed += (int64_t)n;
            sv->inflight_bytes -= batch_bytes;
            sv->inflight_slots -= (int32_t)n;
        }
        sv->cv_done.notify_all();
        sv->cv_admit.notify_all();
    }
}

void stop_threads(gg_server *sv)
{
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_count.notify_all();
    sv->cv_admit.notify_all();
    sv->cv_done.notify_all();
    if (sv->counter.joinable()) sv->counter.join();
    for (auto &t : sv->workers)
        if (t.joinable()) t.join();
}

}  // namespace

extern "C" {

gg_status gg_server_create(const gg_index *ix, const gg_params *params, uint64_t hit_budget_bytes,
                           int32_t max_slots, gg_server **out)
{
    if (!out) return GG_EINVAL;
    *out = nullptr;
    if (!ix || !params || max_slots < 1) return GG_EINVAL;
    auto *sv = new (std::nothrow) gg_server();
    if (!sv) return GG_ENOMEM;
    sv->ix = ix;
    sv->params = *params;
    sv->budget = std::max<uint64_t>(hit_budget_bytes ? hit_budget_bytes : gg::index_budget(ix),
                                    kBytesPerHit);
    sv->max_slots = max_slots;
    // validate the parameters once, with an empty batch
    int32_t dummy = 0;
    const int64_t off0[1] = {0};
    gg_status s = gg::search_batch_budget(ix, "", off0, 0, params, nullptr, 0, &dummy, nullptr,
                                          sv->budget, false);
    if (s != GG_OK) {
        delete sv;
        return s;
    }
    try {
        sv->counter = std::thread(counter_loop, sv);
        for (int w = 0; w < kWorkers; ++w) sv->workers.emplace_back(worker_loop, sv);
    } catch (...) {
        stop_threads(sv);
        delete sv;
        return GG_ENOMEM;
    }
    *out = sv;
    return GG_OK;
}

// Counts a submit or poll call as inside the library until it returns, so that
// gg_server_destroy can wait for it.
struct Active {
    gg_server *sv;
    explicit Active(gg_server *s) : sv(s) { sv->active.fetch_add(1); }
    ~Active() { sv->active.fetch_sub(1); }
};

gg_status gg_serve_submit(gg_server *sv, const char *query, int64_t qlen, uint64_t *ticket)
{
    if (!sv) return GG_EINVAL;
    Active in(sv);
    if (!ticket || qlen < 0 || (qlen > 0 && !query) || qlen > (int64_t)INT32_MAX / 2)
        return GG_EINVAL;
    for (int64_t i = 0; i < qlen; ++i)
        if (!valid_base(query[i])) return GG_EINVAL;
    auto *r = new (std::nothrow) Request();
    if (!r) return GG_ENOMEM;
    try {
        r->query.assign(query ? query : "", (size_t)qlen);
    } catch (...) {
        delete r;
        return GG_ENOMEM;
    }
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stop) {
            delete r;
            return GG_EINVAL;
        }
        const uint64_t t = sv->next_ticket++;
        sv->reqs[t] = r;
        sv->uncounted.push_back(t);
        sv->stats.submitted += 1;
        *ticket = t;
    }
    sv->cv_count.notify_one();
    return GG_OK;
}

gg_status gg_serve_poll(gg_server *sv, uint64_t ticket, gg_hit *out, int32_t cap, int32_t *n_out,
                        int32_t timeout_us)
{
    if (!sv) return GG_EINVAL;
    Active in(sv);  // declared before the lock: released after it
    if (!n_out || cap < 0 || (cap > 0 && !out)) return GG_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    // every look at the request goes through the map: another poll of the same
    // ticket may collect and free it while this one waits
    auto finished = [&] {
        auto f = sv->reqs.find(ticket);
        return sv->stop || f == sv->reqs.end() || f->second->done;
    };
    if (sv->reqs.find(ticket) == sv->reqs.end()) return GG_ENOTFOUND;
    if (!finished()) {
        if (timeout_us == 0) return GG_EAGAIN;
        if (timeout_us < 0) sv->cv_done.wait(lk, finished);
        else sv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), finished);
    }
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return GG_ENOTFOUND;  // collected by another poll
    Request *r = it->second;
    if (!r->done) return sv->stop ? GG_ENOTFOUND : GG_EAGAIN;  // cancelled, or still running
    sv->reqs.erase(it);
    lk.unlock();
    gg_status s = r->status;
    const int32_t n = (int32_t)r->out.size();
    *n_out = n;
    if (s == GG_OK) {
        std::copy(r->out.begin(), r->out.begin() + std::min(n, cap), out);
        if (n > cap) s = GG_ETRUNC;
    }
    delete r;
    return s;
}

gg_status gg_server_info(gg_server *sv, gg_server_stats *out)
{
    if (!sv || !out) return GG_EINVAL;
    Active in(sv);
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->stats;
    out->budget_bytes = sv->budget;
    out->inflight_bytes = sv->inflight_bytes;
    out->inflight_slots = sv->inflight_slots;
    out->calls_inside = sv->active.load() - 1;  // not counting this call
    return GG_OK;
}

void gg_server_destroy(gg_server *sv)
{
    if (!sv) return;
    stop_threads(sv);
    // submit and poll calls already inside the library return (a waiting poll
    // wakes on the stop and reports its ticket cancelled) before the server goes
    // away; a call made after destroy has begun is the caller's error
    while (sv->active.load() != 0) std::this_thread::sleep_for(std::chrono::microseconds(50));
    for (auto &kv : sv->reqs) delete kv.second;
    sv->reqs.clear();
    delete sv;
}

}  // extern "C"
