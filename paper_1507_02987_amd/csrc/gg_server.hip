// Served form of the search: a request loop with continuous batching.
//
// Requests are queued by gg_serve_submit.  Worker threads, each with its own
// stream and workspace, take whatever is queued (up to their share of the
// in-flight slots) as one batch and run every GPU stage on it, bounded by their
// share of the hit-buffer budget; a request that arrives while a batch is on the
// GPU is taken by the next free worker, so batches overlap on the device.  A
// query's hits do not depend on the batch it lands in: every stage keeps the
// queries of a batch apart.
#include <algorithm>
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
uint64_t index_budget(const gg_index *ix);
}  // namespace gg

namespace {

struct Request {
    std::string query;
    bool done = false;
    gg_status status = GG_OK;
    std::vector<gg_hit> hits;
};

constexpr int kWorkers = 2;

}  // namespace

struct gg_server {
    const gg_index *ix = nullptr;
    gg_params params{};
    uint64_t budget = 0;
    int32_t slots_per_worker = 1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Request *> reqs;
    std::vector<std::thread> workers;
    bool stop = false;
    uint64_t next_ticket = 1;
};

namespace {

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
        take.clear();
        batch.clear();
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_work.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
            if (sv->stop) return;
            while (!sv->queue.empty() && (int32_t)take.size() < sv->slots_per_worker) {
                const uint64_t t = sv->queue.front();
                sv->queue.pop_front();
                auto it = sv->reqs.find(t);
                if (it == sv->reqs.end()) continue;
                take.push_back(t);
                batch.push_back(it->second);
            }
        }
        if (batch.empty()) continue;
        const size_t n = batch.size();
        off.assign(n + 1, 0);
        for (size_t i = 0; i < n; ++i) off[i + 1] = off[i] + (int64_t)batch[i]->query.size();
        buf.resize((size_t)off[n] + 1);
        for (size_t i = 0; i < n; ++i)
            std::copy(batch[i]->query.begin(), batch[i]->query.end(), buf.begin() + off[i]);
        out.resize(n * (size_t)cap0);
        nout.assign(n, 0);
        gg_status st = gg::search_batch_budget(sv->ix, buf.data(), off.data(), (int64_t)n,
                                               &sv->params, out.data(), cap0, nout.data(), nullptr,
                                               sv->budget, false);
        std::vector<gg_status> each(n, st);
        if (st == GG_EBUDGET || st == GG_EINVAL) {
            // one bad or oversized query must not fail its batch-mates: run each alone
            for (size_t i = 0; i < n; ++i) {
                const int64_t o2[2] = {0, off[i + 1] - off[i]};
                each[i] = gg::search_batch_budget(sv->ix, buf.data() + off[i], o2, 1, &sv->params,
                                                  out.data() + i * cap0, cap0, &nout[i], nullptr,
                                                  sv->budget, false);
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
                    r->status = gg::search_batch_budget(sv->ix, buf.data() + off[i], o2, 1,
                                                        &sv->params, big.data(), nout[i], &n2,
                                                        nullptr, sv->budget, false);
                    big.resize((size_t)std::min(n2, nout[i]));
                    r->hits.swap(big);
                } else {
                    r->status = GG_OK;
                    r->hits.assign(out.begin() + i * cap0, out.begin() + i * cap0 + nout[i]);
                }
            } else {
                r->status = each[i];
            }
        }
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            for (Request *r : batch) r->done = true;
        }
        sv->cv_done.notify_all();
    }
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
    const uint64_t total = hit_budget_bytes ? hit_budget_bytes : gg::index_budget(ix);
    sv->budget = std::max<uint64_t>(total / kWorkers, 16);
    sv->slots_per_worker = std::max<int32_t>(1, (max_slots + kWorkers - 1) / kWorkers);
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
        for (int w = 0; w < kWorkers; ++w) sv->workers.emplace_back(worker_loop, sv);
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stop = true;
        }
        sv->cv_work.notify_all();
        for (auto &t : sv->workers) t.join();
        delete sv;
        return GG_ENOMEM;
    }
    *out = sv;
    return GG_OK;
}

gg_status gg_serve_submit(gg_server *sv, const char *query, int64_t qlen, uint64_t *ticket)
{
    if (!sv || !ticket || qlen < 0 || (qlen > 0 && !query)) return GG_EINVAL;
    auto *r = new (std::nothrow) Request();
    if (!r) return GG_ENOMEM;
    r->query.assign(query ? query : "", (size_t)qlen);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stop) {
            delete r;
            return GG_EINVAL;
        }
        const uint64_t t = sv->next_ticket++;
        sv->reqs[t] = r;
        sv->queue.push_back(t);
        *ticket = t;
    }
    sv->cv_work.notify_one();
    return GG_OK;
}

gg_status gg_serve_poll(gg_server *sv, uint64_t ticket, gg_hit *out, int32_t cap, int32_t *n_out,
                        int32_t timeout_us)
{
    if (!sv || !n_out || cap < 0 || (cap > 0 && !out)) return GG_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return GG_ENOTFOUND;
    Request *r = it->second;
    if (!r->done) {
        if (timeout_us == 0) return GG_EAGAIN;
        auto ready = [&] { return r->done || sv->stop; };
        if (timeout_us < 0) sv->cv_done.wait(lk, ready);
        else sv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
        if (!r->done) return GG_EAGAIN;
    }
    sv->reqs.erase(it);
    lk.unlock();
    gg_status s = r->status;
    const int32_t n = (int32_t)r->hits.size();
    *n_out = n;
    if (s == GG_OK) {
        std::copy(r->hits.begin(), r->hits.begin() + std::min(n, cap), out);
        if (n > cap) s = GG_ETRUNC;
    }
    delete r;
    return s;
}

void gg_server_destroy(gg_server *sv)
{
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    sv->cv_done.notify_all();
    for (auto &t : sv->workers) t.join();
    for (auto &kv : sv->reqs) delete kv.second;
    delete sv;
}

}  // extern "C"
