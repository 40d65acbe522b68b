// Host runtime and C ABI of the MI355X indexed similar-sequence search.
//
// Owns the device-resident index, per-call workspaces (stream + growable device
// buffers), the batch orchestration of the GPU stages, per-stage timing and the
// continuous-batching server.  Every stage of a search is a kernel in
// gg_kernels.hip; this file only sizes buffers, launches, and copies results.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <string>
#include <unordered_map>
#include <vector>

#include "gg.h"
#include "gg_internal.h"

using namespace gg;

namespace {

int bits_for(uint64_t x)  // bits to hold every value in [0, x)
{
    int b = 0;
    while (b < 64 && (x > (1ull << b))) ++b;
    return b;
}

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

struct Err {
    gg_status st = GG_OK;
};

#define HIPCHK(expr)                                  \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) {                       \
            if (e_ == hipErrorOutOfMemory) return GG_ENOMEM; \
            return GG_EDEVICE;                        \
        }                                             \
    } while (0)

// Wait for the stream; a kernel that could not be launched (its error is kept
// until read) fails the call instead of leaving its outputs unwritten.
#define SYNC(stream)                                          \
    do {                                                      \
        HIPCHK(hipStreamSynchronize(stream));                 \
        if (hipGetLastError() != hipSuccess) return GG_EDEVICE; \
    } while (0)

#define TRY(expr)                     \
    do {                              \
        gg_status s_ = (expr);        \
        if (s_ != GG_OK) return s_;   \
    } while (0)

gg_status ensure(DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 1;
    if (bytes <= b.cap) return GG_OK;
    if (b.p) {
        (void)hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
    }
    size_t want = bytes + bytes / 4 + 256;
    if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        if (hipMalloc(&b.p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            b.p = nullptr;
            return GG_ENOMEM;
        }
        want = bytes;
    }
    b.cap = want;
    return GG_OK;
}

template <typename T>
T *as(DevBuf &b) { return reinterpret_cast<T *>(b.p); }

struct StageTime {
    double ms = 0;
    int64_t launches = 0;
    int64_t units = 0;
};

struct Workspace {
    int device = 0;
    hipStream_t st = nullptr;
    DevBuf ascii, qoff, qcode, qpack, kcode, cnt, lhead, qid, hoff, partials, qtot, err;
    DevBuf hrel, pbase, akey, keys, keys_alt, hist, rs_partials;
    DevBuf cands, ccount, cand_q, cand_off, boxes, boxes2, boxes3, wkeys, wkeys_alt, perm, perm_alt;
    DevBuf qstart, qend, nsel, sel_off, rstart, rend, aligns, aligns2, cells_q;
    DevBuf bplan, bcount, boff, bcands, btmp, bcoff, ctmp, cursor, qcur, bound_q, bound_off,
        btmp_b, bounds, blist, pcnt, cells_box, rbounds, rbelow, os_scratch, xqueue, gout, gn,
        gctl, gplan, gcursor, gqflag, stiles, gtiles;
    DevBuf tb_hits, tb_q, tb_dir, tb_dir_off, tb_ops_off, tb_ops, tb_len, tb_status;  // traceback
    DevBuf lhist, lthr, lvalid, ltile, lbinq;  // selection prefilter
    DevBuf fkept, fkoff, fflag, ford;   // lone-diagonal filter (ford: largest query first)
    DevBuf tpos;                        // the position where each gather tile starts
    DevBuf mbig, mranges;               // merge groups that may outgrow an LDS window
    DevBuf selbox;                      // the box index of each selection (replayed waves)
    DevBuf bsw_order;                   // the aligner's class counts and box order
    DevBuf bq;                          // the query of each encode block's first base
    // small pinned staging: [0] a wave's counts, [1] a batch's query offsets and hit
    // totals, [2] the replayed waves' plan, overflow flags and result counts
    void *pinned[3] = {nullptr, nullptr, nullptr};
    size_t pinned_cap[3] = {0, 0, 0};
    // the captured wave graph and what it was captured for (every argument baked
    // into its nodes: capacities, parameters, buffer addresses)
    hipGraphExec_t gexec = nullptr;
    std::vector<uint64_t> gkey;
    std::vector<hipEvent_t> events;
    size_t ev_used = 0;
    struct Mark {
        std::string name;
        int e0, e1;
        int64_t units;
    };
    std::vector<Mark> marks;

    ~Workspace()
    {
        if (st) (void)hipSetDevice(device);
        if (gexec) (void)hipGraphExecDestroy(gexec);
        DevBuf *all[] = {&ascii, &qoff, &qcode, &qpack, &kcode, &cnt, &lhead, &qid, &hoff, &partials, &qtot, &err,
                         &hrel, &pbase, &akey, &keys, &keys_alt, &hist, &rs_partials, &cands,
                         &ccount, &cand_q, &cand_off, &boxes, &boxes2, &boxes3, &wkeys, &wkeys_alt, &perm,
                         &perm_alt, &qstart, &qend, &nsel, &sel_off, &rstart, &rend, &aligns, &aligns2,
                         &cells_q, &bplan, &bcount, &boff, &bcands, &btmp, &bcoff, &ctmp, &cursor, &qcur,
                         &bound_q, &bound_off, &btmp_b, &bounds, &blist, &pcnt, &cells_box,
                         &rbounds, &rbelow, &os_scratch, &xqueue, &gout, &gn, &gctl, &gplan,
                         &gcursor, &gqflag, &stiles, &gtiles, &tb_hits, &tb_q, &tb_dir,
                         &tb_dir_off, &tb_ops_off, &tb_ops, &tb_len, &tb_status, &lhist, &lthr,
                         &lvalid, &ltile, &lbinq, &fkept, &fkoff, &fflag, &ford, &tpos, &selbox, &bq,
                         &mbig, &mranges, &bsw_order};
        for (DevBuf *b : all)
            if (b->p) (void)hipFree(b->p);
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (void *pn : pinned)
            if (pn) (void)hipHostFree(pn);
        if (st) (void)hipStreamDestroy(st);
    }
};

}  // namespace

struct gg_index {
    int device = 0;
    int32_t k = 0;       // bases in a window's code (the mask's weight)
    int32_t span = 0;    // bases a window covers (the mask's length; k without a mask)
    uint32_t mask = 0;   // bit t set: base t of a window is coded
    int32_t strands = 1; // 2: sequences n/2 .. n-1 are the reverse complements of the first half
    int64_t n_seqs = 0, n_bases = 0;
    uint64_t n_post = 0;
    int64_t max_seq_len = 0;
    uint32_t *d_list_off = nullptr;
    int2 *d_post = nullptr;
    uint32_t *d_dbw = nullptr;
    int64_t *d_seq_start = nullptr;
    uint64_t hit_budget = 0;
    uint64_t default_budget = 0;
    uint32_t bucket_cap = 0;  // keys of one bucket one wave sorts in LDS
    uint32_t bucket_big = 0;  // keys of one bucket one block sorts in LDS
    mutable std::mutex ws_mu;
    mutable std::vector<Workspace *> ws_free;
    std::atomic<int> prof_on{0};
    // tuned launch choices (gg_index_autotune / gg_index_set_tuning)
    std::atomic<int32_t> tune_grouping{2};
    std::atomic<int32_t> tune_lane_steps{256};
    std::atomic<int32_t> tune_wave_log2{0};  // hits of one graph wave: 2^this (0: 2^25)
    std::atomic<int32_t> tune_graph{1};      // 0: batches never replay the wave graph
    std::atomic<int32_t> tune_graph_qlog2{0};  // queries over 2^this hits skip the graph (0: none)
    mutable std::mutex prof_mu;
    mutable std::map<std::string, StageTime> prof;
};

namespace {

gg_status get_ws(const gg_index *ix, Workspace **out)
{
    {
        std::lock_guard<std::mutex> g(ix->ws_mu);
        if (!ix->ws_free.empty()) {
            *out = ix->ws_free.back();
            ix->ws_free.pop_back();
            return GG_OK;
        }
    }
    auto *ws = new (std::nothrow) Workspace();
    if (!ws) return GG_ENOMEM;
    ws->device = ix->device;
    if (hipStreamCreateWithFlags(&ws->st, hipStreamNonBlocking) != hipSuccess) {
        delete ws;
        return GG_EDEVICE;
    }
    *out = ws;
    return GG_OK;
}

void put_ws(const gg_index *ix, Workspace *ws)
{
    std::lock_guard<std::mutex> g(ix->ws_mu);
    ix->ws_free.push_back(ws);
}

gg_status pinned(Workspace *ws, size_t bytes, void **p, int slot = 0)
{
    if (bytes > ws->pinned_cap[slot]) {
        if (ws->pinned[slot]) (void)hipHostFree(ws->pinned[slot]);
        ws->pinned[slot] = nullptr;
        ws->pinned_cap[slot] = 0;
        size_t want = std::max<size_t>(bytes, 1 << 16);
        HIPCHK(hipHostMalloc(&ws->pinned[slot], want, hipHostMallocDefault));
        ws->pinned_cap[slot] = want;
    }
    *p = ws->pinned[slot];
    return GG_OK;
}

// ---- per-stage timing with events on the workspace's own stream
struct Prof {
    const gg_index *ix;
    Workspace *ws;
    bool on;
    int open = -1;
    std::string name;
    Prof(const gg_index *i, Workspace *w) : ix(i), ws(w), on(i->prof_on.load() != 0)
    {
        ws->marks.clear();
        ws->ev_used = 0;
    }
    int ev()
    {
        if (ws->ev_used == ws->events.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return -1;
            ws->events.push_back(e);
        }
        return (int)ws->ev_used++;
    }
    void begin(const char *n)
    {
        if (!on) return;
        open = ev();
        name = n;
        if (open >= 0) (void)hipEventRecord(ws->events[open], ws->st);
    }
    void end(int64_t units)
    {
        if (!on || open < 0) return;
        int e1 = ev();
        if (e1 < 0) return;
        (void)hipEventRecord(ws->events[e1], ws->st);
        ws->marks.push_back({name, open, e1, units});
        open = -1;
    }
    void collect()  // after the stream has been synchronised
    {
        if (!on || ws->marks.empty()) return;
        std::lock_guard<std::mutex> g(ix->prof_mu);
        for (auto &m : ws->marks) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, ws->events[m.e0], ws->events[m.e1]) == hipSuccess) {
                auto &s = ix->prof[m.name];
                s.ms += ms;
                s.launches += 1;
                s.units += m.units;
            }
        }
        ws->marks.clear();
        ws->ev_used = 0;
    }
};

// ---- multi-word record keys: fields packed most-significant first, never split
struct FieldSpec {
    int32_t field;
    int bits;
    int32_t desc_max;
};

gg_status make_words(const std::vector<FieldSpec> &fields, std::vector<KeyWord> &words)
{
    words.clear();
    KeyWord cur{};
    std::vector<FieldSpec> pend;
    auto flush = [&]() {
        KeyWord w{};
        int sh = 0;
        for (int i = (int)pend.size() - 1; i >= 0; --i) {
            w.field[w.n] = pend[i].field;
            w.shift[w.n] = sh;
            w.desc_max[w.n] = pend[i].desc_max;
            w.n++;
            sh += pend[i].bits;
        }
        w.bits = sh;
        words.push_back(w);
        pend.clear();
    };
    int used = 0;
    for (const auto &f : fields) {
        if (f.bits > 64) return GG_EINVAL;
        if (used + f.bits > 64 || (int)pend.size() == 8) {
            flush();
            used = 0;
        }
        pend.push_back(f);
        used += f.bits;
    }
    if (!pend.empty()) flush();
    (void)cur;
    return GG_OK;
}

// Sort n records by a multi-word key; returns the device permutation (sorted
// position -> record index) in ws->perm.
template <typename KeyFn>
gg_status sort_records(Workspace *ws, uint32_t n, const std::vector<KeyWord> &words, KeyFn keyfn,
                       uint32_t **perm_out)
{
    TRY(ensure(ws->perm, sizeof(uint32_t) * n));
    TRY(ensure(ws->perm_alt, sizeof(uint32_t) * n));
    TRY(ensure(ws->wkeys, sizeof(uint64_t) * n));
    TRY(ensure(ws->wkeys_alt, sizeof(uint64_t) * n));
    TRY(ensure(ws->hist, sizeof(uint32_t) * radix_hist_needed(n)));
    TRY(ensure(ws->rs_partials, sizeof(uint32_t) * scan_partials_needed(radix_hist_needed(n))));
    uint32_t *perm = as<uint32_t>(ws->perm), *perm_alt = as<uint32_t>(ws->perm_alt);
    launch_iota(perm, n, ws->st);
    bool first = true;
    for (int w = (int)words.size() - 1; w >= 0; --w) {
        keyfn(words[w], first ? nullptr : perm, as<uint64_t>(ws->wkeys));
        first = false;
        if (words[w].bits == 0) continue;
        int where = radix_sort(as<uint64_t>(ws->wkeys), as<uint64_t>(ws->wkeys_alt), perm, perm_alt,
                               n, 0, words[w].bits, as<uint32_t>(ws->hist),
                               as<uint32_t>(ws->rs_partials), ws->st);
        if (where) std::swap(perm, perm_alt);
    }
    *perm_out = perm;
    return GG_OK;
}

gg_status check_params(const gg_params *p)
{
    if (!p) return GG_EINVAL;
    if (p->match <= 0 || p->mismatch < 0 || p->gap_open < 0 || p->gap_extend < 0) return GG_EINVAL;
    if (p->band < 0 || p->band > kMaxBand || p->xdrop < 0 || p->max_gap < 0 ||
        p->min_hsp_len < 0)
        return GG_EINVAL;
    if ((int64_t)p->gap_open + p->gap_extend > (1 << 20) || p->match > (1 << 20) ||
        p->mismatch > (1 << 20) || p->xdrop > (1 << 28))
        return GG_EINVAL;
    return GG_OK;
}

struct BatchOut {
    gg_hit *out;        // host results (host form) or device results (device form)
    int32_t cap;
    int32_t *n_out;     // host counts (host form) or device counts (device form)
    gg_stats *stats;    // host, or NULL
    bool device = false;
    bool truncated = false;
};

// Radix tiles of hits sorted within query segments: the hits of the wave's query
// ql are the next counts[ql] keys in gather order; each query gets whole tiles.
void seg_tiles(const uint64_t *counts, int32_t nq, std::vector<SortTile> &out)
{
    out.clear();
    uint64_t start = 0;
    for (int32_t q = 0; q < nq; ++q) {
        const uint32_t c = (uint32_t)counts[q];
        const uint32_t nt = (c + kSortTile - 1) / kSortTile;
        const uint32_t hbase = (uint32_t)out.size() * kRadix;
        for (uint32_t t = 0; t < nt; ++t)
            out.push_back(SortTile{(uint32_t)start + t * kSortTile,
                                   std::min<uint32_t>(kSortTile, c - t * kSortTile), hbase, nt, t});
        start += c;
    }
}

// One query's search restricted to data-bank sequences [s_lo, s_hi) (used when
// the query's hits overflow the per-call budget).  run_wave leaves the piece's
// selected boxes, aligned and in selection order, with their in-band cell counts.
struct Piece {
    int32_t s_lo = 0, s_hi = 0;
    uint64_t hits = 0;
    uint32_t n_cands = 0, n_merged = 0;
    std::vector<Align> sel;
    std::vector<unsigned long long> cells;
};

// Run every GPU stage for queries [qa, qb) of the batch (one wave).
// How index hits become runs (Section 2.2 phase 2): kProbe tests the windows next
// to each hit and stores no hit; kBucket and kSort store every hit as a 64-bit key
// (q, s, diag, qpos) and sort them, by slices in LDS or by global radix passes.
enum Grouping { kProbe = 0, kBucket = 1, kSort = 2 };

// How the stored hit keys are sorted: a digit histogram and scan per pass
// (default), or one-sweep passes with look-back tile offsets (GG_SORT=onesweep).
// Look-back reads go to device-coherent memory across the chip's separate L2
// caches, so a tile's walk over still-running predecessors is slow here: on
// 13 M keys a one-sweep pass takes about 2.5x the time of the three kernels.
enum SortKind { kClassic = 0, kOneSweep = 1 };

SortKind sort_kind_from_env()
{
    const char *g = getenv("GG_SORT");
    return (g && !strcmp(g, "onesweep")) ? kOneSweep : kClassic;
}

// Hits alone on their (s, diag) group are dropped before grouping when no run of
// one hit can be kept (M > span) and the wave's queries average at most
// kFiltMean hits, the load at which the per-query LDS tables still drop most lone
// hits; GG_FILTER=0 turns the filter off.
constexpr uint64_t kFiltMean = 1u << 17;

// The filter's block order: a wave's nqw queries by decreasing hit count, to the
// power of two (a counting sort on the count's bit length; the order within a
// length is the query order).  Only rough order matters: the largest start first.
void filter_order(const uint64_t *qtot, int32_t nqw, int32_t *order)
{
    // key 64 - bit length: the largest counts first; start[k] = first slot of key k
    auto key = [&](int32_t x) { return qtot[x] ? __builtin_clzll(qtot[x]) : 64; };
    uint32_t start[66] = {0};
    for (int32_t x = 0; x < nqw; ++x) ++start[key(x) + 1];
    for (int k = 1; k < 66; ++k) start[k] += start[k - 1];
    for (int32_t x = 0; x < nqw; ++x) order[start[key(x)]++] = x;
}

// The merge of large waves orders and sweeps each (query, sequence) group in LDS
// windows (k_merge_tiles), whose sweep runs in parallel over a window's boxes;
// GG_MERGE=serial sweeps each group in one thread instead, and GG_MERGE=global
// sends every box through the global record sort.
bool merge_windows_enabled()
{
    const char *e = std::getenv("GG_MERGE");
    return !(e && std::strcmp(e, "global") == 0);
}

int merge_sweep_rounds()
{
    const char *e = std::getenv("GG_MERGE");
    return e && std::strcmp(e, "serial") == 0 ? 0 : kMergeRounds;
}

// The filter runs after the gather (k_gather writes every key, k_hit_filter reads
// them) unless GG_FUSE=1, which builds the keys inside the filter from the postings
// (k_gather_filter: no key stored before the filter, a quarter of the HBM traffic,
// but one block per query with block-wide steps between its batches, which on the
// mid-size bank takes longer than the two kernels apart).
bool fused_filter_enabled()
{
    const char *e = std::getenv("GG_FUSE");
    return e && std::strcmp(e, "1") == 0;
}

bool filter_for(const gg_index *ix, const gg_params *p, uint64_t hits, int64_t nq)
{
    const char *g = getenv("GG_FILTER");
    if (g && !strcmp(g, "0")) return false;
    return p->min_hsp_len > ix->span && hits <= (uint64_t)std::max<int64_t>(nq, 0) * kFiltMean;
}

// GG_GROUPING (probe, bucket or sort) pins the strategy; otherwise the index's
// tuned choice is used (sort until tuned).
Grouping grouping_for(const gg_index *ix)
{
    const char *g = getenv("GG_GROUPING");
    if (g && !strcmp(g, "probe")) return kProbe;
    if (g && !strcmp(g, "bucket")) return kBucket;
    if (g && !strcmp(g, "sort")) return kSort;
    const int32_t t = ix->tune_grouping.load();
    return t == 0 ? kProbe : t == 1 ? kBucket : kSort;
}

gg_status run_wave(const gg_index *ix, Workspace *ws, Prof &prof, const gg_params *p,
                   const std::vector<int64_t> &qoff_h, const std::vector<uint64_t> &qtot,
                   int32_t qa, int32_t qb, BatchOut &bo, Grouping grouping,
                   Piece *piece = nullptr)
{
    hipStream_t st = ws->st;
    const int32_t nqw = qb - qa;
    const int64_t g0 = qoff_h[qa], g1 = qoff_h[qb];
    uint64_t H64 = 0;
    int64_t maxL = 0;
    for (int32_t q = qa; q < qb; ++q) {
        H64 += qtot[q];
        maxL = std::max<int64_t>(maxL, qoff_h[q + 1] - qoff_h[q]);
    }
    if (piece) H64 = piece->hits;  // a piece is one query (qb == qa + 1)
    for (int32_t q = qa; q < qb && !piece; ++q) {
        const int64_t L = qoff_h[q + 1] - qoff_h[q];
        if (bo.stats) {
            gg_stats &s = bo.stats[q];
            s = gg_stats{};
            s.n_kmers = L >= ix->span ? L - ix->span + 1 : 0;
            s.n_hits = (int64_t)qtot[q];
        }
        if (!bo.device) bo.n_out[q] = 0;
    }
    if (bo.device && !piece) HIPCHK(hipMemsetAsync(bo.n_out + qa, 0, sizeof(int32_t) * nqw, st));
    if (H64 == 0) return GG_OK;
    const uint32_t H = (uint32_t)H64;

    HitKeyLayout lay;
    lay.bp = bits_for((uint64_t)maxL);
    lay.bias = (int32_t)maxL;
    lay.bd = bits_for((uint64_t)ix->max_seq_len + (uint64_t)maxL);
    lay.bs = bits_for((uint64_t)ix->n_seqs);
    lay.bq = bits_for((uint64_t)nqw);
    if (grouping != kProbe && lay.bp + lay.bd + lay.bs + lay.bq > 64) return GG_EINVAL;
    if ((uint64_t)maxL * (uint64_t)p->match >= (1ull << 30)) return GG_EINVAL;  // int32 scores

    // ---- S3 gather
    const int64_t np = g1 - g0;
    TRY(ensure(ws->hrel, sizeof(uint32_t) * (np + 1)));
    TRY(ensure(ws->pbase, sizeof(uint32_t) * (np + 1)));
    TRY(ensure(ws->akey, sizeof(uint64_t) * (np + 1)));
    prof.begin("gather_prep");
    if (piece) {
        TRY(ensure(ws->pcnt, sizeof(uint32_t) * (np + 1)));
        launch_piece_prep(as<uint32_t>(ws->kcode) + g0, as<uint32_t>(ws->cnt) + g0, np,
                          ix->d_list_off, ix->d_post, piece->s_lo, piece->s_hi, lay,
                          as<uint32_t>(ws->pcnt), as<uint32_t>(ws->pbase), as<uint64_t>(ws->akey),
                          st);
        launch_scan_u32(as<uint32_t>(ws->pcnt), as<uint32_t>(ws->hrel), np,
                        as<uint32_t>(ws->partials), st);
    } else {
        TRY(ensure(ws->tpos, sizeof(uint32_t) * ((size_t)H / kTile + 2)));
        launch_wave_prep(as<uint64_t>(ws->hoff), as<int64_t>(ws->qoff), as<uint32_t>(ws->lhead),
                         as<int32_t>(ws->qid), qa, g0, g1, lay, as<uint32_t>(ws->hrel),
                         as<uint32_t>(ws->pbase), as<uint64_t>(ws->akey), as<uint32_t>(ws->tpos),
                         st);
    }
    prof.end(np);

    // pinned staging: run and bound counts[2] | runs per query[nqw] | sel_off[nqw+1] | sel start[nqw] |
    // sel end[nqw] | report start[nqw] | report end[nqw] | (8-aligned) cells per query[nqw]
    void *pin;
    const size_t n1 = (size_t)nqw + 1;
    const size_t u32s = 2 + (size_t)nqw + n1 + 4 * (size_t)nqw;
    const size_t cells_at = ((u32s * 4 + 7) / 8) * 8;
    TRY(pinned(ws, cells_at + 12 * (size_t)nqw + 64, &pin));  // + the filter's order [nqw]
    uint32_t *h_nc = reinterpret_cast<uint32_t *>(pin);
    uint32_t *h_cq = h_nc + 2;
    uint32_t *h_sel_off = h_cq + nqw;
    uint32_t *h_ss = h_sel_off + n1, *h_se = h_ss + nqw, *h_rs = h_se + nqw, *h_re = h_rs + nqw;
    unsigned long long *h_cells =
        reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(pin) + cells_at);
    TRY(ensure(ws->cand_q, sizeof(uint32_t) * (nqw + 1)));
    TRY(ensure(ws->cand_off, sizeof(uint32_t) * (nqw + 1)));
    HIPCHK(hipMemsetAsync(ws->cand_q.p, 0, sizeof(uint32_t) * nqw, st));
    uint32_t nc = 0;

    // ---- S3 + S4 + S5, bucketed: a query's hits are cut into slices of its
    // sequence-id range of about bucket_cap / 4 hits; each slice is sorted and
    // chained in LDS.  A slice over bucket_cap hits sends the wave to the global path.
    const uint32_t target = std::max<uint32_t>(ix->bucket_cap / 4, 1);
    std::vector<uint32_t> plan(2 * (size_t)nqw);  // bucket base | bucket count per query
    uint64_t nbk64 = 0;
    for (int32_t ql = 0; ql < nqw; ++ql) {
        const uint64_t nb = std::max<uint64_t>(1, (qtot[qa + ql] + target - 1) / target);
        plan[ql] = (uint32_t)nbk64;
        plan[nqw + ql] = (uint32_t)nb;
        nbk64 += nb;
    }
    if (grouping == kProbe && p->max_gap / ix->span + 1 > kMaxProbe) grouping = kBucket;
    if (grouping == kProbe) {
        // ---- S3 + S4 + S5 by probing: single-hit runs and run bounds, no stored hit
        uint32_t ccap = (uint32_t)std::max<uint64_t>(1u << 16, H / 64);
        uint32_t bcap = (uint32_t)std::max<uint64_t>(1u << 16, H / 32);
        TRY(ensure(ws->cursor, sizeof(uint32_t) * 4));
        TRY(ensure(ws->bound_q, sizeof(uint32_t) * (nqw + 1)));
        TRY(ensure(ws->bound_off, sizeof(uint32_t) * (nqw + 1)));
        TRY(ensure(ws->qcur, sizeof(uint32_t) * (nqw + 1)));
        TRY(ensure(ws->partials, sizeof(uint64_t) * scan_partials_needed((int64_t)nqw + 1)));
        uint32_t *h_cur = h_nc;  // [0] runs, [1] bounds
        uint32_t nb = 0;
        std::vector<uint32_t> bq(nqw);
        for (int attempt = 0; attempt < 2; ++attempt) {
            TRY(ensure(ws->ctmp, sizeof(Cand) * ccap));
            TRY(ensure(ws->btmp_b, sizeof(Bound) * bcap));
            HIPCHK(hipMemsetAsync(ws->cursor.p, 0, sizeof(uint32_t) * 2, st));
            HIPCHK(hipMemsetAsync(ws->cand_q.p, 0, sizeof(uint32_t) * nqw, st));
            HIPCHK(hipMemsetAsync(ws->bound_q.p, 0, sizeof(uint32_t) * nqw, st));
            prof.begin("probe");
            launch_probe(as<uint32_t>(ws->hrel), as<uint32_t>(ws->pbase), np, ix->d_post, H, g0,
                         as<int32_t>(ws->qid), as<int64_t>(ws->qoff), qa, as<uint32_t>(ws->kcode),
                         as<uint32_t>(ws->cnt), ix->d_dbw, ix->d_seq_start, ix->span, ix->mask,
                         p->max_gap,
                         p->min_hsp_len,
                         as<Cand>(ws->ctmp), ccap, as<uint32_t>(ws->cursor),
                         as<uint32_t>(ws->cand_q), as<Bound>(ws->btmp_b), bcap,
                         as<uint32_t>(ws->cursor) + 1, as<uint32_t>(ws->bound_q), st);
            prof.end(H);
            HIPCHK(hipMemcpyAsync(h_cur, ws->cursor.p, sizeof(uint32_t) * 2, hipMemcpyDeviceToHost,
                                  st));
            HIPCHK(hipMemcpyAsync(bq.data(), ws->bound_q.p, sizeof(uint32_t) * nqw,
                                  hipMemcpyDeviceToHost, st));
            SYNC(st);
            nc = h_cur[0];
            nb = h_cur[1];
            if (nc <= ccap && nb <= bcap) break;
            ccap = std::max(ccap, nc);
            bcap = std::max(bcap, nb);
        }
        const uint32_t maxb = nqw ? *std::max_element(bq.begin(), bq.end()) : 0;
        if (maxb > (uint32_t)kBoundCap) {
            grouping = kBucket;  // a query with too many runs to pair in LDS
            nc = 0;
            HIPCHK(hipMemsetAsync(ws->cand_q.p, 0, sizeof(uint32_t) * nqw, st));
        } else {
            if (nb > 0) {
                // room for every pair after the single-hit runs
                const uint32_t need = nc + nb / 2;
                if (need > ccap) {
                    DevBuf bigger;
                    TRY(ensure(bigger, sizeof(Cand) * need));
                    HIPCHK(hipMemcpyAsync(bigger.p, ws->ctmp.p, sizeof(Cand) * nc,
                                          hipMemcpyDeviceToDevice, st));
                    SYNC(st);
                    (void)hipFree(ws->ctmp.p);
                    ws->ctmp = bigger;
                    ccap = need;
                }
                TRY(ensure(ws->bounds, sizeof(Bound) * nb));
                prof.begin("pair");
                launch_scan_u32(as<uint32_t>(ws->bound_q), as<uint32_t>(ws->bound_off), nqw,
                                as<uint32_t>(ws->partials), st);
                HIPCHK(hipMemsetAsync(ws->qcur.p, 0, sizeof(uint32_t) * nqw, st));
                launch_bounds_by_query(as<Bound>(ws->btmp_b), nb, as<uint32_t>(ws->bound_off),
                                       as<uint32_t>(ws->qcur), as<Bound>(ws->bounds), st);
                launch_pair_bounds(as<Bound>(ws->bounds), as<uint32_t>(ws->bound_off), nqw, ix->span,
                                   p->min_hsp_len, as<Cand>(ws->ctmp), ccap,
                                   as<uint32_t>(ws->cursor), as<uint32_t>(ws->cand_q), st);
                prof.end(nb);
                HIPCHK(hipMemcpyAsync(h_cur, ws->cursor.p, sizeof(uint32_t), hipMemcpyDeviceToHost,
                                      st));
                SYNC(st);
                nc = h_cur[0];
            }
            if (nc > 0) {
                TRY(ensure(ws->cands, sizeof(Cand) * nc));
                launch_scan_u32(as<uint32_t>(ws->cand_q), as<uint32_t>(ws->cand_off), nqw,
                                as<uint32_t>(ws->partials), st);
                HIPCHK(hipMemsetAsync(ws->qcur.p, 0, sizeof(uint32_t) * nqw, st));
                launch_group_by_query(as<Cand>(ws->ctmp), nc, as<uint32_t>(ws->cand_off),
                                      as<uint32_t>(ws->qcur), as<Cand>(ws->cands), st);
            }
        }
        if (grouping != kProbe && lay.bp + lay.bd + lay.bs + lay.bq > 64) return GG_EINVAL;
    }
    bool bucketed = grouping == kBucket && nbk64 < (1ull << 30);
    if (grouping != kProbe) TRY(ensure(ws->keys, sizeof(uint64_t) * H));
    if (bucketed) {
        const uint32_t nbk = (uint32_t)nbk64;
        TRY(ensure(ws->bplan, sizeof(uint32_t) * 2 * nqw));
        TRY(ensure(ws->bcount, sizeof(uint32_t) * (nbk + 1)));
        TRY(ensure(ws->boff, sizeof(uint32_t) * (nbk + 1)));
        TRY(ensure(ws->bcands, sizeof(uint32_t) * (nbk + 1)));
        TRY(ensure(ws->btmp, sizeof(uint32_t) * (nbk + 1)));
        TRY(ensure(ws->bcoff, sizeof(uint32_t) * (nbk + 1)));
        TRY(ensure(ws->cursor, sizeof(uint32_t) * 4));
        TRY(ensure(ws->partials, sizeof(uint64_t) * scan_partials_needed((int64_t)nbk + 1)));
        const uint32_t *bb = as<uint32_t>(ws->bplan), *nbq = bb + nqw;
        HIPCHK(hipMemcpyAsync(ws->bplan.p, plan.data(), sizeof(uint32_t) * 2 * nqw,
                              hipMemcpyHostToDevice, st));
        HIPCHK(hipMemsetAsync(ws->bcount.p, 0, sizeof(uint32_t) * nbk, st));
        prof.begin("gather_count");
        launch_gather_bucket(1, as<uint32_t>(ws->hrel), as<uint32_t>(ws->pbase),
                             as<uint64_t>(ws->akey), np, ix->d_post, H, lay, bb, nbq,
                             as<uint32_t>(ws->bcount), nullptr, nullptr, st);
        prof.end(H);
        launch_scan_u32(as<uint32_t>(ws->bcount), as<uint32_t>(ws->boff), nbk,
                        as<uint32_t>(ws->partials), st);
        std::vector<uint32_t> cnt(nbk);
        HIPCHK(hipMemcpyAsync(cnt.data(), ws->bcount.p, sizeof(uint32_t) * nbk,
                              hipMemcpyDeviceToHost, st));
        SYNC(st);
        const uint32_t maxb = *std::max_element(cnt.begin(), cnt.end());
        bucketed = maxb <= ix->bucket_big;
        std::vector<uint32_t> big;  // buckets over one wave's LDS slice
        for (uint32_t b = 0; bucketed && b < nbk; ++b)
            if (cnt[b] > ix->bucket_cap) big.push_back(b);
        if (bucketed) {
            TRY(ensure(ws->blist, sizeof(uint32_t) * (big.size() + 1)));
            if (!big.empty())
                HIPCHK(hipMemcpyAsync(ws->blist.p, big.data(), sizeof(uint32_t) * big.size(),
                                      hipMemcpyHostToDevice, st));
            HIPCHK(hipMemsetAsync(ws->bcount.p, 0, sizeof(uint32_t) * nbk, st));
            prof.begin("gather");
            launch_gather_bucket(2, as<uint32_t>(ws->hrel), as<uint32_t>(ws->pbase),
                                 as<uint64_t>(ws->akey), np, ix->d_post, H, lay, bb, nbq,
                                 as<uint32_t>(ws->bcount), as<uint32_t>(ws->boff),
                                 as<uint64_t>(ws->keys), st);
            prof.end(H);
            uint32_t ccap = (uint32_t)std::max<uint64_t>(1u << 16, H / 16);
            for (int attempt = 0; attempt < 2; ++attempt) {
                TRY(ensure(ws->ctmp, sizeof(Cand) * ccap));
                HIPCHK(hipMemsetAsync(ws->cursor.p, 0, sizeof(uint32_t), st));
                if (attempt) HIPCHK(hipMemsetAsync(ws->cand_q.p, 0, sizeof(uint32_t) * nqw, st));
                prof.begin("group");
                launch_bucket_sort_chain(as<uint64_t>(ws->keys), as<uint32_t>(ws->boff), nbk, maxb,
                                         lay, ix->span, p->max_gap, p->min_hsp_len,
                                         as<Cand>(ws->ctmp), ccap, as<uint32_t>(ws->cursor),
                                         as<uint32_t>(ws->btmp), as<uint32_t>(ws->bcands),
                                         as<uint32_t>(ws->cand_q), st);
                launch_bucket_sort_chain_big(as<uint64_t>(ws->keys), as<uint32_t>(ws->boff),
                                             as<uint32_t>(ws->blist), (uint32_t)big.size(), maxb,
                                             lay, ix->span, p->max_gap, p->min_hsp_len,
                                             as<Cand>(ws->ctmp), ccap, as<uint32_t>(ws->cursor),
                                             as<uint32_t>(ws->btmp), as<uint32_t>(ws->bcands),
                                             as<uint32_t>(ws->cand_q), st);
                prof.end(H);
                HIPCHK(hipMemcpyAsync(h_nc, ws->cursor.p, sizeof(uint32_t), hipMemcpyDeviceToHost,
                                      st));
                SYNC(st);
                nc = *h_nc;
                if (nc <= ccap) break;
                ccap = nc;
            }
            if (nc > 0) {
                TRY(ensure(ws->cands, sizeof(Cand) * nc));
                launch_scan_u32(as<uint32_t>(ws->bcands), as<uint32_t>(ws->bcoff), nbk,
                                as<uint32_t>(ws->partials), st);
                launch_compact_cands(as<Cand>(ws->ctmp), as<uint32_t>(ws->btmp),
                                     as<uint32_t>(ws->bcands), as<uint32_t>(ws->bcoff), nbk,
                                     as<Cand>(ws->cands), st);
                launch_scan_u32(as<uint32_t>(ws->cand_q), as<uint32_t>(ws->cand_off), nqw,
                                as<uint32_t>(ws->partials), st);
            }
        }
    }
    if (grouping != kProbe && !bucketed) {
        // ---- global path: gather in place, lone-diagonal filter with per-query LDS
        // sorts, or a stable LSD radix sort within query segments; chain
        TRY(ensure(ws->keys_alt, sizeof(uint64_t) * H));
        const int sort_lo = lay.bp, sort_hi = lay.bp + lay.bd + lay.bs + lay.bq;
        const int seg_hi = lay.bp + lay.bd + lay.bs;
        const uint64_t *sorted = nullptr;
        uint32_t Hs = H;  // keys left to chain
        const uint32_t ntile = chain_tiles(H);
        TRY(ensure(ws->ccount, sizeof(uint32_t) * (ntile + 1)));
        TRY(ensure(ws->partials,
                   sizeof(uint64_t) * scan_partials_needed(std::max<int64_t>(ntile, nqw) + 1)));
        const bool lookback = sort_kind_from_env() == kOneSweep;
        const bool filt = !lookback && !piece && filter_for(ix, p, H, nqw);
        const bool fused = fused_filter_enabled();
        if (lookback) TRY(ensure(ws->os_scratch, onesweep_scratch_bytes(H)));
        if (filt) {
            TRY(ensure(ws->fkept, sizeof(uint32_t) * (nqw + 1)));
            TRY(ensure(ws->fkoff, sizeof(uint32_t) * (nqw + 1)));
            TRY(ensure(ws->fflag, sizeof(uint32_t)));
            TRY(ensure(ws->ford, sizeof(int32_t) * nqw));
            int32_t *h_ord = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(h_cells) +
                                                         8 * (size_t)nqw);
            filter_order(qtot.data() + qa, nqw, h_ord);
            HIPCHK(hipMemcpyAsync(ws->ford.p, h_ord, sizeof(int32_t) * nqw, hipMemcpyHostToDevice,
                                  st));
        }
        // segmented radix passes over n keys in kin, counts[ql] keys per query in
        // query order; returns the buffer holding the sorted keys
        auto radix_passes = [&](uint64_t *kin, uint64_t *kout, const std::vector<uint64_t> &counts,
                                uint32_t n) -> gg_status {
            // tiles within query segments: the passes skip the query bits of the keys
            std::vector<SortTile> tiles;
            seg_tiles(counts.data(), nqw, tiles);
            const uint32_t nst = (uint32_t)tiles.size();
            TRY(ensure(ws->stiles, sizeof(SortTile) * std::max<uint32_t>(nst, 1)));
            if (nst)
                HIPCHK(hipMemcpyAsync(ws->stiles.p, tiles.data(), sizeof(SortTile) * nst,
                                      hipMemcpyHostToDevice, st));
            const size_t nhist = std::max<size_t>(radix_hist_needed(n), (size_t)nst * kRadix + 1);
            TRY(ensure(ws->hist, sizeof(uint32_t) * nhist));
            TRY(ensure(ws->rs_partials, sizeof(uint32_t) * scan_partials_needed((int64_t)nhist)));
            sorted = kin;
            if (n <= 1) return GG_OK;
            for (int shift = sort_lo; shift < seg_hi; shift += kRadixBits) {
                prof.begin("sort_hist");
                launch_rs_hist_seg(kin, nst, shift, as<SortTile>(ws->stiles),
                                   as<uint32_t>(ws->hist), st);
                prof.end(n);
                prof.begin("sort_scan");
                launch_rs_scan_seg(as<uint32_t>(ws->hist), nst, as<uint32_t>(ws->rs_partials), st);
                prof.end(n);
                prof.begin("sort_scatter");
                launch_rs_scatter_seg(kin, kout, nst, shift, as<SortTile>(ws->stiles),
                                      as<uint32_t>(ws->hist), st);
                prof.end(n);
                std::swap(kin, kout);
            }
            sorted = kin;
            return GG_OK;
        };
        std::vector<uint64_t> qcounts((size_t)nqw);
        for (int32_t ql = 0; ql < nqw; ++ql) qcounts[(size_t)ql] = piece ? piece->hits : qtot[qa + ql];
        for (int attempt = 0; attempt < 2; ++attempt) {
            // with one-sweep passes, a look-back wait that ran out sends the wave
            // back to the gather and the per-pass histogram sort
            const bool os = lookback && attempt == 0;
            uint64_t *kcur = as<uint64_t>(ws->keys), *knext = as<uint64_t>(ws->keys_alt);
            if (!(filt && fused)) {
                prof.begin("gather");
                launch_gather(as<uint32_t>(ws->hrel), as<uint32_t>(ws->pbase),
                              as<uint64_t>(ws->akey), np, ix->d_post, H, lay, kcur,
                              piece ? nullptr : as<uint32_t>(ws->tpos), st);
                prof.end(H);
            }
            if (filt) {
                HIPCHK(hipMemsetAsync(ws->fflag.p, 0, sizeof(uint32_t), st));
                if (fused) {
                    prof.begin("gather_filter");
                    launch_gather_filter(as<uint32_t>(ws->hrel), as<uint32_t>(ws->pbase),
                                         ix->d_post,
                                         as<int64_t>(ws->qoff), qa, g0, nqw, lay,
                                         as<int32_t>(ws->ford), kcur, as<uint32_t>(ws->fkept),
                                         as<uint32_t>(ws->fflag), st);
                } else {
                    prof.begin("filter");
                    launch_hit_filter(kcur, as<uint32_t>(ws->hrel), as<int64_t>(ws->qoff), qa,
                                      g0, nqw, lay.bp, as<int32_t>(ws->ford),
                                      as<uint32_t>(ws->fkept), as<uint32_t>(ws->fflag), st);
                }
                prof.end(H);
                prof.begin("filter_compact");
                launch_hit_compact(kcur, as<uint32_t>(ws->hrel), as<int64_t>(ws->qoff), qa, g0,
                                   nqw, as<uint32_t>(ws->fkept), as<uint32_t>(ws->fkoff),
                                   as<uint32_t>(ws->partials), knext, st);
                prof.end(H);
                HIPCHK(hipMemcpyAsync(h_nc, as<uint32_t>(ws->fkoff) + nqw, sizeof(uint32_t),
                                      hipMemcpyDeviceToHost, st));
                HIPCHK(hipMemcpyAsync(h_nc + 1, ws->fflag.p, sizeof(uint32_t),
                                      hipMemcpyDeviceToHost, st));
                SYNC(st);
                Hs = h_nc[0];
                sorted = knext;
                if (h_nc[1]) {
                    // a query kept more hits than its LDS sort holds: radix passes
                    // over the compacted keys, each query in qpos order
                    std::vector<uint32_t> kept((size_t)nqw);
                    HIPCHK(hipMemcpyAsync(kept.data(), ws->fkept.p, sizeof(uint32_t) * nqw,
                                          hipMemcpyDeviceToHost, st));
                    SYNC(st);
                    for (int32_t ql = 0; ql < nqw; ++ql) qcounts[(size_t)ql] = kept[(size_t)ql];
                    TRY(radix_passes(knext, kcur, qcounts, Hs));
                }
            } else if (H > 1 && os) {
                prof.begin("sort_hist");
                onesweep_prepare(kcur, H, sort_lo, sort_hi, ws->os_scratch.p, st);
                prof.end(H);
                for (int pass = 0; sort_lo + kRadixBits * pass < sort_hi; ++pass) {
                    prof.begin("sort_scatter");
                    onesweep_pass(kcur, knext, H, sort_lo, pass, ws->os_scratch.p, st);
                    prof.end(H);
                    std::swap(kcur, knext);
                }
                sorted = kcur;
            } else {
                TRY(radix_passes(kcur, knext, qcounts, H));
            }
            h_nc[0] = h_nc[1] = 0;
            prof.begin("chain");
            if (Hs > 0) {
                launch_chain_count(sorted, Hs, lay, ix->span, p->max_gap, p->min_hsp_len,
                                   as<uint32_t>(ws->ccount), st);
                launch_scan_u32(as<uint32_t>(ws->ccount), as<uint32_t>(ws->ccount),
                                chain_tiles(Hs), as<uint32_t>(ws->partials), st);
                HIPCHK(hipMemcpyAsync(h_nc, as<uint32_t>(ws->ccount) + chain_tiles(Hs),
                                      sizeof(uint32_t), hipMemcpyDeviceToHost, st));
            }
            if (os && H > 1)
                HIPCHK(hipMemcpyAsync(h_nc + 1, onesweep_fail_flag(ws->os_scratch.p),
                                      sizeof(uint32_t), hipMemcpyDeviceToHost, st));
            prof.end(Hs);
            SYNC(st);
            if (!(os && h_nc[1])) break;
        }
        nc = *h_nc;
        if (nc > 0) {
            TRY(ensure(ws->cands, sizeof(Cand) * nc));
            TRY(ensure(ws->qstart, sizeof(uint32_t) * (nqw + 1)));
            TRY(ensure(ws->qend, sizeof(uint32_t) * (nqw + 1)));
            prof.begin("chain_write");
            launch_chain_write(sorted, Hs, lay, ix->span, p->max_gap, p->min_hsp_len,
                               as<uint32_t>(ws->ccount), as<Cand>(ws->cands), st);
            launch_cand_segments(as<Cand>(ws->cands), nc, nqw, as<uint32_t>(ws->qstart),
                                 as<uint32_t>(ws->qend), st);
            launch_select_counts(as<uint32_t>(ws->qstart), as<uint32_t>(ws->qend), nqw, 0,
                                 as<uint32_t>(ws->cand_q), st);
            launch_scan_u32(as<uint32_t>(ws->cand_q), as<uint32_t>(ws->cand_off), nqw,
                            as<uint32_t>(ws->partials), st);
            prof.end(H);
        }
    }
    if (nc == 0) return GG_OK;
    HIPCHK(hipMemcpyAsync(h_cq, ws->cand_q.p, sizeof(uint32_t) * nqw, hipMemcpyDeviceToHost, st));

    // ---- S6 extend (one lane per run, long walks resumed by a wave)
    TRY(ensure(ws->boxes, sizeof(Box) * nc));
    TRY(ensure(ws->boxes2, sizeof(Box) * nc));
    TRY(ensure(ws->boxes3, sizeof(Box) * nc));
    TRY(ensure(ws->xqueue, extend_queue_bytes(nc)));
    prof.begin("extend");
    launch_extend(as<Cand>(ws->cands), nc, as<uint8_t>(ws->qcode), as<uint32_t>(ws->qpack),
                  as<int64_t>(ws->qoff), qa,
                  ix->d_dbw, ix->d_seq_start, p->match, p->mismatch, p->xdrop, as<Box>(ws->boxes),
                  ws->xqueue.p, ix->tune_lane_steps.load(), st);
    prof.end(nc);
    SYNC(st);  // h_cq ready
    uint32_t max_seg = 0;
    for (int32_t ql = 0; ql < nqw; ++ql) max_seg = std::max(max_seg, h_cq[ql]);
    const bool seg_path = max_seg <= (uint32_t)kSegCap;

    const int bq = bits_for((uint64_t)nqw + 1);  // room for the "empty" query value nqw
    const int bs = lay.bs;
    const int bl = bits_for((uint64_t)maxL + 1);
    const int bsl = bits_for((uint64_t)ix->max_seq_len + 1);
    std::vector<KeyWord> words;
    uint32_t *perm = nullptr;

    // ---- S7 merge: order each query's boxes by (s, qs, ds, qe, de), sweep each (q, s)
    prof.begin("merge");
    Box *boxes = as<Box>(ws->boxes);
    const int bdm = bits_for((uint64_t)ix->max_seq_len + (uint64_t)maxL + 1);
    // windows need each (query, sequence) group contiguous, as the sorted hits
    // leave the runs; probing writes runs in no such order
    const bool windows = !seg_path && grouping == kSort && merge_windows_enabled() &&
                         12 + 2 * bl + bdm <= 64;
    // global record sort of n boxes by merge order, then the sweep: src -> dst (with
    // goffs, the boxes are ngroup whole groups starting at goffs[0 .. ngroup] on the
    // device, each swept in parallel by a block)
    auto global_merge = [&](Box *src, uint32_t n, Box *tmp, Box *dst,
                            const uint32_t *goffs = nullptr, uint32_t ngroup = 0) -> gg_status {
        TRY(make_words({{F_Q, bq, 0}, {F_S, bs, 0}, {F_QS, bl, 0}, {F_DS, bsl, 0}, {F_QE, bl, 0},
                        {F_DE, bsl, 0}},
                       words));
        TRY(sort_records(ws, n, words,
                         [&](const KeyWord &w, const uint32_t *pm, uint64_t *out) {
                             launch_box_keys(src, n, w, nqw, out, pm, st);
                         },
                         &perm));
        launch_gather_boxes(src, perm, n, tmp, st);
        if (goffs) launch_merge_groups(tmp, goffs, ngroup, dst, merge_sweep_rounds(), st);
        else launch_merge_sweep(tmp, n, dst, st);
        return GG_OK;
    };
    // the selection prefilter's length records (one per box slot, the query in
    // 22 bits), written where the boxes are merged; the per-query segment path
    // selects in LDS and needs none
    LenSel ls;
    if (!seg_path && p->max_hits > 0 && nc > 0 && nqw < (1 << 22)) {
        TRY(ensure(ws->lbinq, sizeof(uint32_t) * (size_t)nc));
        ls = LenSel{as<uint32_t>(ws->lbinq), std::max(0, bits_for((uint64_t)maxL + 1) - 10)};
    }
    if (seg_path) {
        launch_seg_sort_box(0, boxes, as<Box>(ws->boxes2), as<uint32_t>(ws->cand_off), nqw, st);
        prof.end(nc);
        prof.begin("merge_sweep");
        launch_merge_sweep(as<Box>(ws->boxes2), nc, as<Box>(ws->boxes3), st);
        prof.end(nc);
    } else if (windows) {
        // groups in LDS windows; the few that may outgrow a window by the global sort
        constexpr uint32_t kBigCap = 1u << 16;
        TRY(ensure(ws->mbig, sizeof(uint32_t) * (1 + 2 * (size_t)kBigCap)));
        launch_merge_tiles(boxes, nc, bl, bdm, (int32_t)maxL, as<Box>(ws->boxes3),
                           as<uint32_t>(ws->mbig), kBigCap, merge_sweep_rounds(), ls, st);
        uint32_t nbig = 0;
        HIPCHK(hipMemcpyAsync(h_nc, ws->mbig.p, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        SYNC(st);
        nbig = h_nc[0];
        if (nbig > kBigCap) {
            TRY(global_merge(boxes, nc, as<Box>(ws->boxes2), as<Box>(ws->boxes3)));
            if (ls.binq) launch_len_records(as<Box>(ws->boxes3), nc, ls, st);  // all anew
        } else if (nbig > 0) {
            std::vector<uint32_t> ranges(2 * (size_t)nbig), offs((size_t)nbig + 1, 0);
            HIPCHK(hipMemcpyAsync(ranges.data(), as<uint32_t>(ws->mbig) + 1,
                                  sizeof(uint32_t) * 2 * nbig, hipMemcpyDeviceToHost, st));
            SYNC(st);
            // packed in position order, so the global sort keeps the groups' order
            std::vector<uint32_t> order((size_t)nbig);
            for (uint32_t r = 0; r < nbig; ++r) order[r] = r;
            std::sort(order.begin(), order.end(),
                      [&](uint32_t a, uint32_t b) { return ranges[2 * a] < ranges[2 * b]; });
            std::vector<uint32_t> sr(2 * (size_t)nbig);
            for (uint32_t r = 0; r < nbig; ++r) {
                sr[2 * r] = ranges[2 * order[r]];
                sr[2 * r + 1] = ranges[2 * order[r] + 1];
                offs[r + 1] = offs[r] + (sr[2 * r + 1] - sr[2 * r]);
            }
            const uint32_t B = offs[nbig];
            TRY(ensure(ws->mranges, sizeof(uint32_t) * (3 * (size_t)nbig + 1)));
            uint32_t *d_ranges = as<uint32_t>(ws->mranges), *d_offs = d_ranges + 2 * nbig;
            HIPCHK(hipMemcpyAsync(d_ranges, sr.data(), sizeof(uint32_t) * 2 * nbig,
                                  hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(d_offs, offs.data(), sizeof(uint32_t) * (nbig + 1),
                                  hipMemcpyHostToDevice, st));
            // pack the big groups (boxes2), sort and sweep them (via boxes, no longer
            // needed), and put them back in their places
            launch_copy_ranges(boxes, as<Box>(ws->boxes2), d_ranges, d_offs, nbig, true, st);
            TRY(global_merge(as<Box>(ws->boxes2), B, boxes, as<Box>(ws->boxes2) + 0, d_offs, nbig));
            launch_copy_ranges(as<Box>(ws->boxes2), as<Box>(ws->boxes3), d_ranges, d_offs, nbig,
                               false, st);
            if (ls.binq) launch_len_records_ranges(as<Box>(ws->boxes3), d_ranges, nbig, ls, st);
            SYNC(st);  // the host vectors above go out of scope
        }
        prof.end(nc);
    } else {
        TRY(global_merge(boxes, nc, as<Box>(ws->boxes2), as<Box>(ws->boxes3)));
        if (ls.binq) launch_len_records(as<Box>(ws->boxes3), nc, ls, st);
        prof.end(nc);
    }

    // ---- S8 select by length: (kept first, len desc, s, qs, ds, qe, de), first N per query
    prof.begin("select");
    Box *merged = as<Box>(ws->boxes3);
    uint32_t nbox = nc;                // boxes in the selection order
    std::vector<uint32_t> nvalid_h;    // merged boxes per query, when prefiltered
    if (seg_path) {
        launch_seg_sort_box(1, merged, as<Box>(ws->boxes2), as<uint32_t>(ws->cand_off), nqw, st);
    } else {
        if (ls.binq) {
            // only boxes at least as long as a query's N-th longest can be selected
            const uint32_t tiles = (nc + kTile - 1) / kTile;
            TRY(ensure(ws->lhist, sizeof(uint32_t) * (size_t)nqw * kLenBins));
            TRY(ensure(ws->lthr, sizeof(uint32_t) * nqw));
            TRY(ensure(ws->lvalid, sizeof(uint32_t) * nqw));
            TRY(ensure(ws->ltile, sizeof(uint32_t) * (tiles + 1)));
            TRY(ensure(ws->partials, sizeof(uint64_t) * scan_partials_needed(tiles + 1)));
            launch_len_prefilter(ls.binq, nc, nqw, p->max_hits, as<uint32_t>(ws->lhist),
                                 as<uint32_t>(ws->lthr),
                                 as<uint32_t>(ws->lvalid), as<uint32_t>(ws->ltile),
                                 as<uint32_t>(ws->partials), st);
            launch_len_compact(merged, ls.binq, nc, as<uint32_t>(ws->lthr),
                               as<uint32_t>(ws->ltile), as<Box>(ws->boxes), st);
            nvalid_h.resize((size_t)nqw);
            HIPCHK(hipMemcpyAsync(&nbox, as<uint32_t>(ws->ltile) + tiles, sizeof(uint32_t),
                                  hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(nvalid_h.data(), ws->lvalid.p, sizeof(uint32_t) * nqw,
                                  hipMemcpyDeviceToHost, st));
            SYNC(st);
            merged = as<Box>(ws->boxes);
        }
        TRY(make_words({{F_Q, bq, 0}, {F_LEN_DESC, bl, (int32_t)maxL}, {F_S, bs, 0},
                        {F_QS, bl, 0}, {F_DS, bsl, 0}, {F_QE, bl, 0}, {F_DE, bsl, 0}},
                       words));
        TRY(sort_records(ws, nbox, words,
                         [&](const KeyWord &w, const uint32_t *pm, uint64_t *out) {
                             launch_box_keys(merged, nbox, w, nqw, out, pm, st);
                         },
                         &perm));
        launch_gather_boxes(merged, perm, nbox, as<Box>(ws->boxes2), st);
    }
    TRY(ensure(ws->qstart, sizeof(uint32_t) * (nqw + 1)));
    TRY(ensure(ws->qend, sizeof(uint32_t) * (nqw + 1)));
    TRY(ensure(ws->nsel, sizeof(uint32_t) * (nqw + 1)));
    TRY(ensure(ws->sel_off, sizeof(uint32_t) * (nqw + 1)));
    HIPCHK(hipMemsetAsync(ws->qstart.p, 0, sizeof(uint32_t) * nqw, st));
    HIPCHK(hipMemsetAsync(ws->qend.p, 0, sizeof(uint32_t) * nqw, st));
    launch_segments_box(as<Box>(ws->boxes2), nbox, nqw, as<uint32_t>(ws->qstart),
                        as<uint32_t>(ws->qend), st);
    launch_select_counts(as<uint32_t>(ws->qstart), as<uint32_t>(ws->qend), nqw, p->max_hits,
                         as<uint32_t>(ws->nsel), st);
    launch_scan_u32(as<uint32_t>(ws->nsel), as<uint32_t>(ws->sel_off), nqw,
                    as<uint32_t>(ws->partials), st);
    prof.end(nc);
    HIPCHK(hipMemcpyAsync(h_sel_off, ws->sel_off.p, sizeof(uint32_t) * n1, hipMemcpyDeviceToHost, st));
    if (bo.stats || piece) {
        HIPCHK(hipMemcpyAsync(h_ss, ws->qstart.p, sizeof(uint32_t) * nqw, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(h_se, ws->qend.p, sizeof(uint32_t) * nqw, hipMemcpyDeviceToHost, st));
    }
    SYNC(st);
    const uint32_t nsel = h_sel_off[nqw];
    auto merged_of = [&](int32_t ql) -> int64_t {
        return nvalid_h.empty() ? (int64_t)(h_se[ql] - h_ss[ql]) : (int64_t)nvalid_h[(size_t)ql];
    };
    if (piece) {
        piece->n_cands = h_cq[0];
        piece->n_merged = merged_of(0);
    } else if (bo.stats) {
        for (int32_t ql = 0; ql < nqw; ++ql) {
            bo.stats[qa + ql].n_cands = h_cq[ql];
            bo.stats[qa + ql].n_merged = merged_of(ql);
        }
    }
    if (nsel == 0) return GG_OK;

    // ---- S9 banded Smith-Waterman
    TRY(ensure(ws->aligns, sizeof(Align) * nsel));
    TRY(ensure(ws->aligns2, sizeof(Align) * nsel));
    TRY(ensure(ws->cells_q, sizeof(unsigned long long) * nqw));
    HIPCHK(hipMemsetAsync(ws->cells_q.p, 0, sizeof(unsigned long long) * nqw, st));
    if (piece) TRY(ensure(ws->cells_box, sizeof(unsigned long long) * nsel));
    TRY(ensure(ws->bsw_order, sizeof(uint32_t) * ((size_t)nsel + 64)));
    prof.begin("align");
    launch_bsw(as<Box>(ws->boxes2), as<uint32_t>(ws->qstart), as<uint32_t>(ws->sel_off), nqw, nsel,
               as<uint8_t>(ws->qcode), as<int64_t>(ws->qoff), qa, ix->d_dbw, ix->d_seq_start,
               p->match, p->mismatch, p->gap_open, p->gap_extend, p->band, as<Align>(ws->aligns),
               as<unsigned long long>(ws->cells_q),
               piece ? as<unsigned long long>(ws->cells_box) : nullptr, st, nullptr, nullptr,
               as<uint32_t>(ws->bsw_order));
    prof.end(nsel);
    if (piece) {  // the piece's selection, in selection order, is its whole result
        piece->sel.resize(nsel);
        piece->cells.resize(nsel);
        HIPCHK(hipMemcpyAsync(piece->sel.data(), ws->aligns.p, sizeof(Align) * nsel,
                              hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(piece->cells.data(), ws->cells_box.p,
                              sizeof(unsigned long long) * nsel, hipMemcpyDeviceToHost, st));
        SYNC(st);
        return GG_OK;
    }

    // ---- S10 report: score > 0 first, score desc, coordinates; per-query ranges
    uint32_t max_sel = 0;
    for (int32_t ql = 0; ql < nqw; ++ql) max_sel = std::max(max_sel, h_sel_off[ql + 1] - h_sel_off[ql]);
    TRY(ensure(ws->rstart, sizeof(uint32_t) * (nqw + 1)));
    TRY(ensure(ws->rend, sizeof(uint32_t) * (nqw + 1)));
    prof.begin("report");
    Align *al = as<Align>(ws->aligns);
    bool written = false;
    if (max_sel <= (uint32_t)kSegCap) {
        launch_report_seg(al, as<Align>(ws->aligns2), as<uint32_t>(ws->sel_off), nqw,
                          as<uint32_t>(ws->rstart), as<uint32_t>(ws->rend), qa, bo.cap,
                          bo.device ? reinterpret_cast<int32_t *>(bo.out) : nullptr,
                          bo.device ? bo.n_out : nullptr, st);
        written = bo.device;
    } else {
        const int bsc = bits_for((uint64_t)maxL * (uint64_t)p->match + 1);
        TRY(make_words({{A_Q, bq, 0}, {A_SCORE_DESC, bsc, (int32_t)(maxL * p->match)},
                        {A_SEQ, bs, 0}, {A_QS, bl, 0}, {A_DS, bsl, 0}, {A_QE, bl, 0},
                        {A_DE, bsl, 0}, {A_BQS, bl, 0}, {A_BDS, bsl, 0}, {A_BQE, bl, 0},
                        {A_BDE, bsl, 0},
                        {A_D0, bits_for((uint64_t)ix->max_seq_len + (uint64_t)maxL + 1),
                         (int32_t)maxL}},
                       words));
        TRY(sort_records(ws, nsel, words,
                         [&](const KeyWord &w, const uint32_t *pm, uint64_t *out) {
                             launch_align_keys(al, nsel, w, nqw, out, pm, st);
                         },
                         &perm));
        launch_gather_aligns(al, perm, nsel, as<Align>(ws->aligns2), st);
        HIPCHK(hipMemsetAsync(ws->rstart.p, 0, sizeof(uint32_t) * nqw, st));
        HIPCHK(hipMemsetAsync(ws->rend.p, 0, sizeof(uint32_t) * nqw, st));
        launch_segments_align(as<Align>(ws->aligns2), nsel, nqw, as<uint32_t>(ws->rstart),
                              as<uint32_t>(ws->rend), st);
    }
    prof.end(nsel);

    // ---- results: ordered alignments and per-query ranges
    std::vector<Align> res;
    if (bo.device) {
        if (!written)
            launch_write_out(as<Align>(ws->aligns2), as<uint32_t>(ws->rstart),
                             as<uint32_t>(ws->rend), nqw, qa, bo.cap,
                             reinterpret_cast<int32_t *>(bo.out), bo.n_out, st);
    } else {
        res.resize(nsel);
        HIPCHK(hipMemcpyAsync(res.data(), ws->aligns2.p, sizeof(Align) * nsel,
                              hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipMemcpyAsync(h_rs, ws->rstart.p, sizeof(uint32_t) * nqw, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h_re, ws->rend.p, sizeof(uint32_t) * nqw, hipMemcpyDeviceToHost, st));
    if (bo.stats)
        HIPCHK(hipMemcpyAsync(h_cells, ws->cells_q.p, sizeof(unsigned long long) * nqw,
                              hipMemcpyDeviceToHost, st));
    SYNC(st);
    for (int32_t ql = 0; ql < nqw; ++ql) {
        const int32_t q = qa + ql;
        const uint32_t n = h_re[ql] - h_rs[ql];
        if (n > (uint32_t)bo.cap) bo.truncated = true;
        if (!bo.device) {
            bo.n_out[q] = (int32_t)n;
            const uint32_t m = std::min<uint32_t>(n, (uint32_t)bo.cap);
            gg_hit *dst = bo.out + (size_t)q * bo.cap;
            for (uint32_t r = 0; r < m; ++r) {
                const Align &a = res[h_rs[ql] + r];
                dst[r] = gg_hit{a.seq_id,      a.score,     a.q_start,     a.q_end,
                                a.d_start,     a.d_end,     a.box_q_start, a.box_q_end,
                                a.box_d_start, a.box_d_end, a.box_len,     a.band_d0};
            }
        }
        if (bo.stats) {
            gg_stats &s = bo.stats[q];
            s.n_selected = h_sel_off[ql + 1] - h_sel_off[ql];
            s.n_cells = (int64_t)h_cells[ql];
            s.n_out = n;
        }
    }
    return GG_OK;
}

// Cut sequence ids [s_lo, s_hi) into ranges whose hits for query positions
// [g0, g0 + np) stay within max_hits: hits below 256 evenly spaced ids are
// counted on the GPU, ranges are grown greedily, and a span that is too big on
// its own is cut again.  A single sequence over the budget cannot be cut.
gg_status plan_pieces(const gg_index *ix, Workspace *ws, int64_t g0, int64_t np, int32_t s_lo,
                      int32_t s_hi, uint64_t max_hits, std::vector<Piece> &out)
{
    constexpr int kBounds = 256;
    hipStream_t st = ws->st;
    std::vector<int32_t> b;
    for (int i = 0; i <= kBounds; ++i) {
        const int32_t v = s_lo + (int32_t)((int64_t)(s_hi - s_lo) * i / kBounds);
        if (b.empty() || v != b.back()) b.push_back(v);
    }
    const int32_t nb = (int32_t)b.size();
    TRY(ensure(ws->rbounds, sizeof(int32_t) * nb));
    TRY(ensure(ws->rbelow, sizeof(unsigned long long) * nb));
    std::vector<unsigned long long> below(nb);
    HIPCHK(hipMemcpyAsync(ws->rbounds.p, b.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(ws->rbelow.p, 0, sizeof(unsigned long long) * nb, st));
    launch_range_counts(as<uint32_t>(ws->kcode) + g0, as<uint32_t>(ws->cnt) + g0, np,
                        ix->d_list_off, ix->d_post, as<int32_t>(ws->rbounds), nb,
                        as<unsigned long long>(ws->rbelow), st);
    HIPCHK(hipMemcpyAsync(below.data(), ws->rbelow.p, sizeof(unsigned long long) * nb,
                          hipMemcpyDeviceToHost, st));
    SYNC(st);
    auto emit = [&](int32_t lo, int32_t hi, uint64_t h) {
        if (h == 0) return;
        Piece pc;
        pc.s_lo = lo;
        pc.s_hi = hi;
        pc.hits = h;
        out.push_back(std::move(pc));
    };
    int32_t a = 0;  // the open range starts at b[a]
    for (int32_t i = 1; i < nb; ++i) {
        if (below[i] - below[a] <= max_hits) continue;
        if (i - 1 > a) {  // close the range before b[i] and test b[i] again
            emit(b[a], b[i - 1], below[i - 1] - below[a]);
            a = i - 1;
            --i;
            continue;
        }
        if (b[i] - b[a] == 1) return GG_EBUDGET;
        TRY(plan_pieces(ix, ws, g0, np, b[a], b[i], max_hits, out));
        a = i;
    }
    if (a < nb - 1) emit(b[a], b[nb - 1], below[nb - 1] - below[a]);
    return GG_OK;
}

// Query q searched piece by piece.  Section 2.2's selection keeps the longest N
// boxes of the query; the N longest overall are among the N longest of each
// piece, so the pieces' selections are merged by the selection order, cut to N,
// and then ordered for the report like any other query's alignments.
gg_status search_pieces(const gg_index *ix, Workspace *ws, Prof &prof, const gg_params *p,
                        const std::vector<int64_t> &qoff_h, const std::vector<uint64_t> &qtot,
                        int32_t q, uint64_t max_hits, BatchOut &bo, Grouping grouping)
{
    const int64_t g0 = qoff_h[q], L = qoff_h[q + 1] - g0;
    std::vector<Piece> pieces;
    TRY(plan_pieces(ix, ws, g0, L, 0, (int32_t)ix->n_seqs, max_hits, pieces));
    std::vector<std::pair<Align, unsigned long long>> all;
    int64_t n_cands = 0, n_merged = 0;
    for (Piece &pc : pieces) {
        TRY(run_wave(ix, ws, prof, p, qoff_h, qtot, q, q + 1, bo, grouping, &pc));
        prof.collect();
        n_cands += pc.n_cands;
        n_merged += pc.n_merged;
        for (size_t i = 0; i < pc.sel.size(); ++i) all.emplace_back(pc.sel[i], pc.cells[i]);
    }
    auto sel_key = [](const Align &a) {
        return std::make_tuple(-a.box_len, a.seq_id, a.box_q_start, a.box_d_start, a.box_q_end,
                               a.box_d_end);
    };
    std::sort(all.begin(), all.end(),
              [&](const auto &x, const auto &y) { return sel_key(x.first) < sel_key(y.first); });
    if (p->max_hits > 0 && all.size() > (size_t)p->max_hits) all.resize((size_t)p->max_hits);
    unsigned long long cells = 0;
    std::vector<Align> rep;
    for (const auto &x : all) {
        cells += x.second;
        if (x.first.score > 0) rep.push_back(x.first);
    }
    auto rep_key = [](const Align &a) {
        return std::make_tuple(-a.score, a.seq_id, a.q_start, a.d_start, a.q_end, a.d_end,
                               a.box_q_start, a.box_d_start, a.box_q_end, a.box_d_end,
                               a.band_d0);
    };
    std::sort(rep.begin(), rep.end(),
              [&](const Align &x, const Align &y) { return rep_key(x) < rep_key(y); });
    const int32_t n = (int32_t)rep.size();
    const int32_t m = std::min(n, bo.cap);
    if (n > bo.cap) bo.truncated = true;
    std::vector<gg_hit> hits((size_t)std::max(m, 1));
    for (int32_t r = 0; r < m; ++r) {
        const Align &a = rep[(size_t)r];
        hits[(size_t)r] = gg_hit{a.seq_id,      a.score,     a.q_start,     a.q_end,
                                 a.d_start,     a.d_end,     a.box_q_start, a.box_q_end,
                                 a.box_d_start, a.box_d_end, a.box_len,     a.band_d0};
    }
    if (bo.device) {
        if (m > 0)
            HIPCHK(hipMemcpyAsync(bo.out + (size_t)q * bo.cap, hits.data(), sizeof(gg_hit) * m,
                                  hipMemcpyHostToDevice, ws->st));
        HIPCHK(hipMemcpyAsync(bo.n_out + q, &n, sizeof(int32_t), hipMemcpyHostToDevice, ws->st));
        SYNC(ws->st);
    } else {
        std::copy(hits.begin(), hits.begin() + m, bo.out + (size_t)q * bo.cap);
        bo.n_out[q] = n;
    }
    if (bo.stats) {
        gg_stats &s = bo.stats[q];
        s.n_kmers = L >= ix->span ? L - ix->span + 1 : 0;
        s.n_hits = (int64_t)qtot[q];
        s.n_cands = n_cands;
        s.n_merged = n_merged;
        s.n_selected = (int64_t)all.size();
        s.n_cells = (int64_t)cells;
        s.n_out = n;
    }
    return GG_OK;
}

// The regular path over ranges [qa, qb) of the batch's queries: consecutive
// queries whose stored hit keys fit the budget and the key bits form a wave
// (probing stores no hit: its waves are bounded only by 32-bit hit counts); a
// query over the budget alone is searched in ranges of sequences.
gg_status run_ranges(const gg_index *ix, Workspace *ws, Prof &prof, const gg_params *p,
                     const std::vector<int64_t> &qoff_h, const std::vector<uint64_t> &qtot,
                     const std::vector<std::pair<int32_t, int32_t>> &ranges, BatchOut &bo,
                     uint64_t budget_bytes, Grouping grouping)
{
    const uint64_t max_hits = grouping == kProbe
                                  ? (uint64_t)INT32_MAX
                                  : std::min<uint64_t>(budget_bytes / 16, (uint64_t)INT32_MAX);
    const int bs = bits_for((uint64_t)ix->n_seqs);
    for (const auto &r : ranges) {
        int32_t qa = r.first;
        const int32_t qend = r.second;
        while (qa < qend) {
            if (qtot[qa] > max_hits) {  // searched alone, by ranges of sequences
                TRY(search_pieces(ix, ws, prof, p, qoff_h, qtot, qa, max_hits, bo, grouping));
                ++qa;
                continue;
            }
            uint64_t h = 0;
            int64_t maxL = 0;
            int32_t qb = qa;
            while (qb < qend && qtot[qb] <= max_hits) {
                const uint64_t h2 = h + qtot[qb];
                const int64_t L2 = std::max<int64_t>(maxL, qoff_h[qb + 1] - qoff_h[qb]);
                const int bits = bits_for((uint64_t)L2) +
                                 bits_for((uint64_t)ix->max_seq_len + L2) + bs +
                                 bits_for((uint64_t)(qb - qa + 1));
                const int wbits = bits_for((uint64_t)(qb - qa + 2));  // record keys hold q up to nqw
                const bool too_wide = grouping != kProbe && bits > 64;
                if (qb > qa && (h2 > max_hits || too_wide || wbits > 31)) break;
                if (too_wide) return GG_EINVAL;
                h = h2;
                maxL = L2;
                ++qb;
            }
            TRY(run_wave(ix, ws, prof, p, qoff_h, qtot, qa, qb, bo, grouping));
            prof.collect();
            qa = qb;
        }
    }
    return GG_OK;
}

// ---- graph-replayed batches
// Waves of a batch are replayed from one captured HIP graph: every kernel reads
// the wave's sizes from a device WaveCtl (see k_wave_begin), so after the single
// synchronisation that gives the per-query hit counts, all waves run without
// further host round trips, and the graph is reused by later calls of the same
// shape.  It covers the radix-sort grouping with per-query LDS sorts: a wave in
// which some query has more than kSegCap runs or selections is flagged and run
// again by run_wave.  GG_GRAPH=0 turns the form off.
constexpr uint64_t kGraphHits = 1ull << 25;  // hits of one graph wave at most, by default

uint64_t graph_wave_hits(const gg_index *ix)
{
    const int32_t lg = ix->tune_wave_log2.load();
    return lg > 0 ? (1ull << lg) : kGraphHits;
}

uint64_t pow2_at_least(uint64_t v)
{
    uint64_t r = 1;
    while (r < v) r <<= 1;
    return r;
}

bool graph_enabled()
{
    const char *g = getenv("GG_GRAPH");
    return !(g && !strcmp(g, "0"));
}

gg_status run_batch(const gg_index *ix, Workspace *ws, const char *qbuf, const int64_t *qoff,
                    int64_t nq, const gg_params *p, BatchOut &bo, uint64_t budget_bytes,
                    bool allow_graph = true);

// Queries idx of a host batch packed into one sub-batch, searched by run_batch
// (with or without graph waves), and their results put back in their places.
gg_status run_packed(const gg_index *ix, Workspace *ws, const gg_params *p, const char *qbuf,
                     const std::vector<int64_t> &qoff_h, const std::vector<int32_t> &idx,
                     BatchOut &bo, uint64_t budget_bytes, bool allow_graph)
{
    if (idx.empty()) return GG_OK;
    const int32_t cap = bo.cap;
    std::vector<char> sub;
    std::vector<int64_t> soff(1, 0);
    for (int32_t q : idx) {
        sub.insert(sub.end(), qbuf + qoff_h[q], qbuf + qoff_h[q + 1]);
        soff.push_back((int64_t)sub.size());
    }
    const size_t nr = idx.size();
    std::vector<gg_hit> sout(nr * (size_t)std::max(cap, 1));
    std::vector<int32_t> sn(nr, 0);
    BatchOut sb{sout.data(), cap, sn.data(), nullptr};
    TRY(run_batch(ix, ws, sub.empty() ? nullptr : sub.data(), soff.data(), (int64_t)nr, p, sb,
                  budget_bytes, allow_graph));
    for (size_t r = 0; r < nr; ++r) {
        const int32_t q = idx[r];
        bo.n_out[q] = sn[r];
        const int32_t m = std::min(sn[r], cap);
        std::copy(sout.begin() + r * cap, sout.begin() + r * cap + m, bo.out + (size_t)q * cap);
        if (sn[r] > cap) bo.truncated = true;
    }
    return GG_OK;
}

gg_status run_graph_waves(const gg_index *ix, Workspace *ws, Prof &prof, const gg_params *p,
                          const char *qbuf, const std::vector<int64_t> &qoff_h,
                          const std::vector<uint64_t> &qtot, int64_t nq, BatchOut &bo,
                          uint64_t budget_bytes, bool *used)
{
    *used = false;
    hipStream_t st = ws->st;
    const uint64_t wave_hits = std::min<uint64_t>(graph_wave_hits(ix), budget_bytes / 16);
    // queries over a wave, or over the per-query limit (queries that heavy mostly
    // outgrow the per-query LDS sorts and would be run twice), take the regular
    // path after the replays; the others form the waves
    const int32_t qlg = ix->tune_graph_qlog2.load();
    const uint64_t graph_q = qlg > 0 ? std::min<uint64_t>(wave_hits, 1ull << qlg) : wave_hits;
    int64_t maxL = 0, n_graph = 0, stretches = 0;
    for (int64_t q = 0; q < nq; ++q) {
        if (qtot[q] > graph_q) continue;
        maxL = std::max<int64_t>(maxL, qoff_h[q + 1] - qoff_h[q]);
        ++n_graph;
        if (q == 0 || qtot[q - 1] > graph_q) ++stretches;
    }
    if (n_graph == 0) return GG_OK;
    if (stretches > 1 && !bo.device) {
        // scattered among heavier ones: the graph queries and the others, each
        // packed into a sub-batch of their own, so the graph waves come out full and
        // the heavy queries share the regular path's large waves
        std::vector<int32_t> light, heavy;
        for (int32_t q = 0; q < (int32_t)nq; ++q) (qtot[q] > graph_q ? heavy : light).push_back(q);
        TRY(run_packed(ix, ws, p, qbuf, qoff_h, light, bo, budget_bytes, true));
        TRY(run_packed(ix, ws, p, qbuf, qoff_h, heavy, bo, budget_bytes, false));
        *used = true;
        return GG_OK;
    }
    // waves by hits, each a stretch of consecutive graph queries; one key layout
    std::vector<WaveCtl> plan;
    uint64_t hmax = 0;
    int64_t npmax = 0;
    int32_t nqmax = 0;
    for (int64_t qa = 0; qa < nq;) {
        if (qtot[qa] > graph_q) {
            ++qa;
            continue;
        }
        uint64_t h = 0;
        int64_t qb = qa;
        while (qb < nq && qtot[qb] <= graph_q && (qb == qa || h + qtot[qb] <= wave_hits) &&
               qb - qa < (1 << 20))
            h += qtot[qb++];
        WaveCtl w{};
        w.qa = (int32_t)qa;
        w.nqw = (int32_t)(qb - qa);
        w.g0 = qoff_h[qa];
        w.np = qoff_h[qb] - qoff_h[qa];
        w.H = (uint32_t)h;
        plan.push_back(w);
        hmax = std::max(hmax, h);
        npmax = std::max(npmax, w.np);
        nqmax = std::max(nqmax, w.nqw);
        qa = qb;
    }
    const uint32_t hits_cap = (uint32_t)pow2_at_least(std::max<uint64_t>(hmax, kTile));
    const int64_t np_cap = (int64_t)pow2_at_least((uint64_t)std::max<int64_t>(npmax, 1));
    const int32_t nq_cap = (int32_t)pow2_at_least((uint64_t)nqmax);
    HitKeyLayout lay;
    lay.bp = bits_for((uint64_t)maxL);
    lay.bias = (int32_t)maxL;
    lay.bd = bits_for((uint64_t)ix->max_seq_len + (uint64_t)maxL);
    lay.bs = bits_for((uint64_t)ix->n_seqs);
    lay.bq = bits_for((uint64_t)nq_cap);
    if (lay.bp + lay.bd + lay.bs + lay.bq > 64) return GG_OK;
    if ((uint64_t)maxL * (uint64_t)p->match >= (1ull << 30)) return GG_EINVAL;
    uint64_t hsum = 0;
    for (const WaveCtl &w : plan) hsum += w.H;
    const bool filt = filter_for(ix, p, hsum, nq);
    const bool fused = fused_filter_enabled();
    // radix tiles within query segments, all waves in one table (none when the
    // lone-diagonal filter and the per-query LDS sorts replace the radix passes)
    std::vector<SortTile> tiles, wt;
    std::vector<uint64_t> qc;
    uint32_t ntile_max = 1;
    for (WaveCtl &w : plan) {
        w.lay = lay;
        if (filt) {
            w.tile0 = w.ntile = 0;
            continue;
        }
        qc.assign(qtot.begin() + w.qa, qtot.begin() + w.qa + w.nqw);
        seg_tiles(qc.data(), w.nqw, wt);
        w.tile0 = (uint32_t)tiles.size();
        w.ntile = (uint32_t)wt.size();
        ntile_max = std::max(ntile_max, w.ntile);
        tiles.insert(tiles.end(), wt.begin(), wt.end());
    }
    const uint32_t ntile_cap = (uint32_t)pow2_at_least(ntile_max);
    const size_t tiles_cap = (size_t)pow2_at_least(std::max<uint64_t>(tiles.size(), 1));
    const int passes = (lay.bd + lay.bs + kRadixBits - 1) / kRadixBits;
    const int32_t N = p->max_hits, cap = bo.cap;
    const uint32_t sel_cap = (uint32_t)N * (uint32_t)nq_cap;
    const uint32_t ntile = (hits_cap + kTile - 1) / kTile;
    const size_t nq_out = (size_t)pow2_at_least((uint64_t)nq);
    const size_t nwave_cap = (size_t)pow2_at_least(std::max<uint64_t>(plan.size(), 64));

    // buffers for the largest wave (they only grow, so a cached graph stays valid
    // while its key matches)
    TRY(ensure(ws->hrel, sizeof(uint32_t) * (np_cap + 1)));
    TRY(ensure(ws->pbase, sizeof(uint32_t) * (np_cap + 1)));
    TRY(ensure(ws->akey, sizeof(uint64_t) * (np_cap + 1)));
    TRY(ensure(ws->keys, sizeof(uint64_t) * hits_cap));
    TRY(ensure(ws->keys_alt, sizeof(uint64_t) * hits_cap));
    TRY(ensure(ws->hist, sizeof(uint32_t) * ((size_t)ntile_cap * kRadix + 1)));
    TRY(ensure(ws->rs_partials,
               sizeof(uint32_t) * scan_partials_needed((int64_t)ntile_cap * kRadix + 1)));
    TRY(ensure(ws->gtiles, sizeof(SortTile) * tiles_cap));
    TRY(ensure(ws->tpos, sizeof(uint32_t) * ((size_t)hits_cap / kTile + 2)));
    TRY(ensure(ws->ccount, sizeof(uint32_t) * (ntile + 1)));
    TRY(ensure(ws->partials,
               sizeof(uint64_t) * scan_partials_needed(std::max<int64_t>(ntile, nq_cap) + 1)));
    TRY(ensure(ws->cands, sizeof(Cand) * hits_cap));
    TRY(ensure(ws->boxes, sizeof(Box) * hits_cap));
    TRY(ensure(ws->boxes2, sizeof(Box) * hits_cap));
    TRY(ensure(ws->boxes3, sizeof(Box) * hits_cap));
    TRY(ensure(ws->xqueue, extend_queue_bytes(hits_cap)));
    for (DevBuf *b : {&ws->qstart, &ws->qend, &ws->cand_q, &ws->cand_off, &ws->nsel, &ws->sel_off,
                      &ws->rstart, &ws->rend})
        TRY(ensure(*b, sizeof(uint32_t) * (nq_cap + 1)));
    TRY(ensure(ws->aligns, sizeof(Align) * std::max<uint32_t>(sel_cap, 1)));
    TRY(ensure(ws->aligns2, sizeof(Align) * std::max<uint32_t>(sel_cap, 1)));
    TRY(ensure(ws->selbox, sizeof(uint32_t) * std::max<uint32_t>(sel_cap, 1)));
    TRY(ensure(ws->bsw_order, sizeof(uint32_t) * ((size_t)sel_cap + 64)));
    TRY(ensure(ws->gout, sizeof(gg_hit) * nq_out * std::max(cap, 1)));
    TRY(ensure(ws->gn, sizeof(int32_t) * nq_out));
    TRY(ensure(ws->gctl, sizeof(WaveCtl)));
    TRY(ensure(ws->gplan, sizeof(WaveCtl) * nwave_cap));
    TRY(ensure(ws->gcursor, sizeof(uint32_t) * 4));
    TRY(ensure(ws->gqflag, sizeof(uint32_t) * nq_out));

    WaveCtl *ctl = as<WaveCtl>(ws->gctl);
    uint32_t *cursor = as<uint32_t>(ws->gcursor);
    if (filt) {
        TRY(ensure(ws->fkept, sizeof(uint32_t) * (nq_cap + 1)));
        TRY(ensure(ws->fkoff, sizeof(uint32_t) * (nq_cap + 1)));
        TRY(ensure(ws->ford, sizeof(int32_t) * nq_out));
    }
    const uint64_t *sorted = (filt || (passes & 1)) ? as<uint64_t>(ws->keys_alt)
                                                    : as<uint64_t>(ws->keys);
    const int32_t steps = ix->tune_lane_steps.load();
    std::vector<uint64_t> key = {hits_cap, (uint64_t)np_cap, (uint64_t)nq_cap, (uint64_t)passes,
                                 (uint64_t)ntile_cap,
                                 (uint64_t)lay.bp, (uint64_t)lay.bd, (uint64_t)lay.bs,
                                 (uint64_t)lay.bq, (uint64_t)(uint32_t)lay.bias, (uint64_t)cap,
                                 (uint64_t)(uint32_t)steps, (uint64_t)ix->span,
                                 (uint64_t)ix->mask,
                                 (uint64_t)(uintptr_t)ix->d_post, (uint64_t)filt,
                                 (uint64_t)fused};
    for (int32_t v : {p->match, p->mismatch, p->gap_open, p->gap_extend, p->band, p->xdrop,
                      p->max_gap, p->min_hsp_len, p->max_hits})
        key.push_back((uint64_t)(uint32_t)v);
    // device-form results go straight to the caller's buffers
    const bool direct = bo.device && cap > 0;
    int32_t *gout = direct ? reinterpret_cast<int32_t *>(bo.out) : as<int32_t>(ws->gout);
    int32_t *gn = bo.device ? bo.n_out : as<int32_t>(ws->gn);
    key.push_back((uint64_t)(uintptr_t)gout);
    key.push_back((uint64_t)(uintptr_t)gn);
    for (const DevBuf *b : {&ws->hoff, &ws->qoff, &ws->kcode, &ws->qid, &ws->qcode, &ws->qpack,
                            &ws->hrel,
                            &ws->pbase, &ws->akey, &ws->keys, &ws->keys_alt, &ws->hist,
                            &ws->rs_partials, &ws->ccount, &ws->partials, &ws->cands, &ws->boxes,
                            &ws->boxes2, &ws->boxes3, &ws->xqueue, &ws->qstart, &ws->qend,
                            &ws->cand_q, &ws->cand_off, &ws->nsel, &ws->sel_off, &ws->rstart,
                            &ws->rend, &ws->aligns, &ws->aligns2, &ws->gout, &ws->gn, &ws->gctl,
                            &ws->gplan, &ws->gcursor, &ws->gqflag, &ws->gtiles, &ws->fkept,
                            &ws->fkoff, &ws->ford, &ws->tpos, &ws->selbox, &ws->bsw_order})
        key.push_back((uint64_t)(uintptr_t)b->p);

    if (!ws->gexec || ws->gkey != key) {
        if (ws->gexec) {
            (void)hipGraphExecDestroy(ws->gexec);
            ws->gexec = nullptr;
        }
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        launch_wave_prep_ctl(as<uint64_t>(ws->hoff), as<int64_t>(ws->qoff), as<uint32_t>(ws->lhead),
                             as<int32_t>(ws->qid), np_cap, as<uint32_t>(ws->hrel),
                             as<uint32_t>(ws->pbase), as<uint64_t>(ws->akey),
                             as<WaveCtl>(ws->gplan), cursor, ctl, as<uint32_t>(ws->tpos), st);
        if (!(filt && fused))
            launch_gather_ctl(as<uint32_t>(ws->hrel), as<uint32_t>(ws->pbase),
                              as<uint64_t>(ws->akey), ix->d_post, hits_cap,
                              as<uint64_t>(ws->keys), ctl, as<uint32_t>(ws->tpos), st);
        if (filt) {
            if (fused)
                launch_gather_filter(as<uint32_t>(ws->hrel), as<uint32_t>(ws->pbase),
                                     ix->d_post, as<int64_t>(ws->qoff), 0,
                                     0, 0, HitKeyLayout{}, as<int32_t>(ws->ford),
                                     as<uint64_t>(ws->keys), as<uint32_t>(ws->fkept), nullptr, st,
                                     ctl, nq_cap);
            else
                launch_hit_filter(as<uint64_t>(ws->keys), as<uint32_t>(ws->hrel),
                                  as<int64_t>(ws->qoff), 0, 0, 0, 0, as<int32_t>(ws->ford),
                                  as<uint32_t>(ws->fkept), nullptr, st, ctl, nq_cap);
            launch_hit_compact(as<uint64_t>(ws->keys), as<uint32_t>(ws->hrel),
                               as<int64_t>(ws->qoff), 0, 0, 0, as<uint32_t>(ws->fkept),
                               as<uint32_t>(ws->fkoff), as<uint32_t>(ws->partials),
                               as<uint64_t>(ws->keys_alt), st, ctl, nq_cap);
        }
        for (int pass = 0; pass < passes && !filt; ++pass) {
            const bool odd = pass & 1;
            launch_rs_pass_ctl(odd ? as<uint64_t>(ws->keys_alt) : as<uint64_t>(ws->keys),
                               odd ? as<uint64_t>(ws->keys) : as<uint64_t>(ws->keys_alt), ntile_cap,
                               pass, as<SortTile>(ws->gtiles), as<uint32_t>(ws->hist),
                               as<uint32_t>(ws->rs_partials), ctl, st);
        }
        launch_chain_ctl(sorted, hits_cap, ix->span, p->max_gap, p->min_hsp_len,
                         as<uint32_t>(ws->ccount), as<uint32_t>(ws->partials), as<Cand>(ws->cands),
                         ctl, st, filt);
        launch_cand_ranges_ctl(as<Cand>(ws->cands), nq_cap, as<uint32_t>(ws->qstart),
                               as<uint32_t>(ws->qend), as<uint32_t>(ws->cand_q),
                               as<uint32_t>(ws->cand_off), static_cast<uint32_t *>(ws->xqueue.p),
                               ctl, st);
        launch_extend(as<Cand>(ws->cands), 0, as<uint8_t>(ws->qcode), as<uint32_t>(ws->qpack),
                      as<int64_t>(ws->qoff), 0,
                      ix->d_dbw, ix->d_seq_start, p->match, p->mismatch, p->xdrop,
                      as<Box>(ws->boxes), ws->xqueue.p, steps, st, ctl, hits_cap,
                      /*count_cleared=*/true);
        launch_merge_select_seg(as<Box>(ws->boxes), as<Box>(ws->boxes2),
                                as<uint32_t>(ws->cand_off), nq_cap, ctl, st);
        if (nq_cap <= 4096) {  // ranges and their scan in one launch
            launch_box_ranges_scan_ctl(as<Box>(ws->boxes2), as<uint32_t>(ws->cand_off), nq_cap, N,
                                       as<uint32_t>(ws->qstart), as<uint32_t>(ws->qend),
                                       as<uint32_t>(ws->sel_off), as<uint32_t>(ws->selbox), ctl,
                                       st);
        } else {
            launch_box_ranges_ctl(as<Box>(ws->boxes2), as<uint32_t>(ws->cand_off), nq_cap, N,
                                  as<uint32_t>(ws->qstart), as<uint32_t>(ws->qend),
                                  as<uint32_t>(ws->nsel), ctl, st);
            launch_scan_u32(as<uint32_t>(ws->nsel), as<uint32_t>(ws->sel_off), nq_cap,
                            as<uint32_t>(ws->partials), st);
        }
        launch_bsw(as<Box>(ws->boxes2), as<uint32_t>(ws->qstart), as<uint32_t>(ws->sel_off), 0, 0,
                   as<uint8_t>(ws->qcode), as<int64_t>(ws->qoff), 0, ix->d_dbw, ix->d_seq_start,
                   p->match, p->mismatch, p->gap_open, p->gap_extend, p->band,
                   as<Align>(ws->aligns), nullptr, nullptr, st, ctl,
                   nq_cap <= 4096 ? as<uint32_t>(ws->selbox) : nullptr,
                   as<uint32_t>(ws->bsw_order));
        launch_report_seg(as<Align>(ws->aligns), as<Align>(ws->aligns2), as<uint32_t>(ws->sel_off),
                          nq_cap, as<uint32_t>(ws->rstart), as<uint32_t>(ws->rend), 0, cap,
                          gout, gn, st, ctl);
        launch_wave_end(cursor, st);
        const hipError_t ec = hipStreamEndCapture(st, &g);
        if (ec != hipSuccess) {
            (void)hipGetLastError();
            return GG_EDEVICE;
        }
        const hipError_t ei = hipGraphInstantiate(&ws->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            ws->gexec = nullptr;
            (void)hipGetLastError();
            return GG_EDEVICE;
        }
        ws->gkey = key;
    }

    // replay it once per wave
    const size_t W = plan.size();
    // staging: plan [W] | query flags [nq] | result counts [nq] | filter order [nq]
    void *pin;
    TRY(pinned(ws, sizeof(WaveCtl) * W + 3 * sizeof(int32_t) * nq + 64, &pin, 2));
    WaveCtl *h_plan = static_cast<WaveCtl *>(pin);
    uint32_t *qflags = reinterpret_cast<uint32_t *>(h_plan + W);
    int32_t *nout = reinterpret_cast<int32_t *>(qflags + nq);
    for (WaveCtl &w : plan) w.qflag = as<uint32_t>(ws->gqflag);
    std::copy(plan.begin(), plan.end(), h_plan);
    HIPCHK(hipMemcpyAsync(ws->gplan.p, h_plan, sizeof(WaveCtl) * W, hipMemcpyHostToDevice, st));
    if (filt) {  // each wave's queries, largest first, at the wave's own positions
        int32_t *h_ord = nout + nq;
        for (const WaveCtl &w : plan) {
            filter_order(qtot.data() + w.qa, w.nqw, h_ord + w.qa);
        }
        HIPCHK(hipMemcpyAsync(ws->ford.p, h_ord, sizeof(int32_t) * nq, hipMemcpyHostToDevice, st));
    }
    if (!tiles.empty() && !filt)
        HIPCHK(hipMemcpyAsync(ws->gtiles.p, tiles.data(), sizeof(SortTile) * tiles.size(),
                              hipMemcpyHostToDevice, st));
    launch_fill2_u32(cursor, 1, reinterpret_cast<uint32_t *>(gn), (size_t)nq, 0u, st);
    launch_fill_u32(as<uint32_t>(ws->gqflag), (size_t)nq, 0u, st);
    prof.begin("graph");
    for (size_t w = 0; w < W; ++w) HIPCHK(hipGraphLaunch(ws->gexec, st));
    prof.end((int64_t)W);
    HIPCHK(hipMemcpyAsync(qflags, ws->gqflag.p, sizeof(uint32_t) * nq, hipMemcpyDeviceToHost,
                          st));
    HIPCHK(hipMemcpyAsync(nout, gn, sizeof(int32_t) * nq, hipMemcpyDeviceToHost, st));
    if (cap > 0 && !direct)
        HIPCHK(hipMemcpyAsync(bo.out, ws->gout.p, sizeof(gg_hit) * (size_t)nq * cap,
                              hipMemcpyDeviceToHost, st));
    SYNC(st);
    prof.collect();
    *used = true;
    if (!bo.device) std::copy(nout, nout + nq, bo.n_out);
    for (int64_t q = 0; q < nq; ++q)
        if (nout[(size_t)q] > cap) bo.truncated = true;
    // the regular path for the queries over a wave and those whose kept hits, runs
    // or selections outgrew a per-query LDS sort
    std::vector<std::pair<int32_t, int32_t>> rest;
    std::vector<int32_t> idx;
    for (int32_t q = 0; q < (int32_t)nq; ++q) {
        if (qtot[q] <= graph_q && !qflags[q]) continue;
        idx.push_back(q);
        if (!rest.empty() && rest.back().second == q) rest.back().second = q + 1;
        else rest.emplace_back(q, q + 1);
    }
    if (rest.size() <= 1 || bo.device) {
        // few stretches (or queries in device memory): each stretch as its own waves
        TRY(run_ranges(ix, ws, prof, p, qoff_h, qtot, rest, bo, budget_bytes, kSort));
        return GG_OK;
    }
    // scattered queries: packed into one host sub-batch, searched without the graph
    // in waves as large as the budget allows, results put back in their places
    return run_packed(ix, ws, p, qbuf, qoff_h, idx, bo, budget_bytes, false);
}

gg_status run_batch(const gg_index *ix, Workspace *ws, const char *qbuf, const int64_t *qoff,
                    int64_t nq, const gg_params *p, BatchOut &bo, uint64_t budget_bytes,
                    bool allow_graph)
{
    hipStream_t st = ws->st;
    if (nq == 0) return GG_OK;
    std::vector<int64_t> qoff_h(nq + 1);
    for (int64_t q = 0; q <= nq; ++q) qoff_h[q] = qoff[q] - qoff[0];
    for (int64_t q = 0; q < nq; ++q)
        if (qoff_h[q + 1] < qoff_h[q] || qoff_h[q + 1] - qoff_h[q] > (int64_t)INT32_MAX / 2)
            return GG_EINVAL;
    const int64_t T = qoff_h[nq];
    if (T > (int64_t)INT32_MAX) return GG_EINVAL;
    if (T > 0 && !qbuf) return GG_EINVAL;
    Prof prof(ix, ws);

    const uint8_t *ascii = nullptr;
    if (bo.device) {
        ascii = reinterpret_cast<const uint8_t *>(qbuf) + qoff[0];
    } else {
        TRY(ensure(ws->ascii, T));
        ascii = as<uint8_t>(ws->ascii);
    }
    TRY(ensure(ws->qoff, sizeof(int64_t) * (nq + 1)));
    TRY(ensure(ws->qcode, T));
    TRY(ensure(ws->kcode, sizeof(uint32_t) * T));
    TRY(ensure(ws->cnt, sizeof(uint32_t) * T));
    TRY(ensure(ws->lhead, sizeof(uint32_t) * T));
    TRY(ensure(ws->qid, sizeof(int32_t) * T));
    TRY(ensure(ws->hoff, sizeof(uint64_t) * (T + 1)));
    TRY(ensure(ws->partials, sizeof(uint64_t) * scan_partials_needed(std::max<int64_t>(T, nq + 1))));
    TRY(ensure(ws->qtot, sizeof(uint64_t) * nq));
    TRY(ensure(ws->err, sizeof(int32_t) * 4));
    TRY(ensure(ws->bq, sizeof(int32_t) * ((size_t)(T + kBlock - 1) / kBlock + 1)));
    if (T > 0 && !bo.device)
        HIPCHK(hipMemcpyAsync(ws->ascii.p, qbuf + qoff[0], T, hipMemcpyHostToDevice, st));
    // staging: query offsets [nq + 1] | hit totals [nq] | error flag
    void *pin;
    TRY(pinned(ws, sizeof(int64_t) * (2 * (size_t)nq + 2), &pin, 1));
    int64_t *h_qoff = static_cast<int64_t *>(pin);
    uint64_t *h_qtot = reinterpret_cast<uint64_t *>(h_qoff + nq + 1);
    int32_t *h_err = reinterpret_cast<int32_t *>(h_qtot + nq);
    std::copy(qoff_h.begin(), qoff_h.end(), h_qoff);
    HIPCHK(hipMemcpyAsync(ws->qoff.p, h_qoff, sizeof(int64_t) * (nq + 1), hipMemcpyHostToDevice,
                          st));
    HIPCHK(hipMemsetAsync(ws->err.p, 0, sizeof(int32_t), st));

    // ---- S1 encode + S2 count and scan
    prof.begin("encode");
    launch_encode_kmers(ascii, as<int64_t>(ws->qoff), (int32_t)nq, T, ix->span, ix->mask,
                        ix->d_list_off, as<uint8_t>(ws->qcode), as<uint32_t>(ws->kcode),
                        as<uint32_t>(ws->cnt), as<uint32_t>(ws->lhead), as<int32_t>(ws->qid),
                        as<int32_t>(ws->err), as<int32_t>(ws->bq), st);
    prof.end(T);
    prof.begin("scan");
    launch_scan_u32_to_u64(as<uint32_t>(ws->cnt), as<uint64_t>(ws->hoff), T,
                           as<uint64_t>(ws->partials), st);
    launch_query_totals(as<uint64_t>(ws->hoff), as<int64_t>(ws->qoff), (int32_t)nq,
                        as<uint64_t>(ws->qtot), st);
    prof.end(T);
    TRY(ensure(ws->qpack, sizeof(uint32_t) * ((size_t)(T + 15) / 16 + 2)));
    launch_pack_query(as<uint8_t>(ws->qcode), T, as<uint32_t>(ws->qpack), st);
    HIPCHK(hipMemcpyAsync(h_qtot, ws->qtot.p, sizeof(uint64_t) * nq, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h_err, ws->err.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SYNC(st);
    if (*h_err) return GG_EINVAL;
    const std::vector<uint64_t> qtot(h_qtot, h_qtot + nq);

    // ---- waves: consecutive queries whose stored hit keys fit the budget and the key
    // bits (probing stores no hit: its waves are bounded only by 32-bit hit counts)
    const Grouping grouping = grouping_for(ix);
    if (allow_graph && ix->tune_graph.load() && graph_enabled() && grouping == kSort &&
        !bo.stats && p->max_hits >= 1 &&
        p->max_hits <= kSegCap) {
        bool used = false;
        TRY(run_graph_waves(ix, ws, prof, p, bo.device ? nullptr : qbuf + qoff[0], qoff_h, qtot,
                            nq, bo, budget_bytes, &used));
        if (used) return GG_OK;
    }
    const std::vector<std::pair<int32_t, int32_t>> all{{0, (int32_t)nq}};
    TRY(run_ranges(ix, ws, prof, p, qoff_h, qtot, all, bo, budget_bytes, grouping));
    prof.collect();
    return GG_OK;
}

uint64_t budget_of(const gg_index *ix) { return ix->hit_budget ? ix->hit_budget : ix->default_budget; }

}  // namespace

namespace gg {

uint64_t index_budget(const gg_index *ix) { return budget_of(ix); }

// Index hits of each of n_q host queries (Section 2.2: the postings of every
// query window), counted by the search's own encode and count kernels; the served
// form admits queries on these exact counts.  GG_EINVAL for a byte outside the
// alphabet anywhere in the batch.
gg_status count_hits(const gg_index *ix, const char *qbuf, const int64_t *qoff, int64_t n_q,
                     uint64_t *hits)
{
    if (!ix || n_q < 0 || (n_q > 0 && (!qoff || !hits))) return GG_EINVAL;
    if (n_q == 0) return GG_OK;
    const int64_t T = qoff[n_q] - qoff[0];
    for (int64_t q = 0; q < n_q; ++q)
        if (qoff[q + 1] < qoff[q]) return GG_EINVAL;
    if (T > (int64_t)INT32_MAX || (T > 0 && !qbuf)) return GG_EINVAL;
    if (hipSetDevice(ix->device) != hipSuccess) return GG_EDEVICE;
    Workspace *ws = nullptr;
    TRY(get_ws(ix, &ws));
    auto run = [&]() -> gg_status {
        hipStream_t st = ws->st;
        TRY(ensure(ws->ascii, T));
        TRY(ensure(ws->qoff, sizeof(int64_t) * (n_q + 1)));
        TRY(ensure(ws->qcode, T));
        TRY(ensure(ws->kcode, sizeof(uint32_t) * T));
        TRY(ensure(ws->cnt, sizeof(uint32_t) * T));
        TRY(ensure(ws->lhead, sizeof(uint32_t) * T));
        TRY(ensure(ws->qid, sizeof(int32_t) * T));
        TRY(ensure(ws->hoff, sizeof(uint64_t) * (T + 1)));
        TRY(ensure(ws->partials,
                   sizeof(uint64_t) * scan_partials_needed(std::max<int64_t>(T, n_q + 1))));
        TRY(ensure(ws->qtot, sizeof(uint64_t) * n_q));
        TRY(ensure(ws->err, sizeof(int32_t) * 4));
        TRY(ensure(ws->bq, sizeof(int32_t) * ((size_t)(T + kBlock - 1) / kBlock + 1)));
        void *pin;
        TRY(pinned(ws, sizeof(int64_t) * (2 * (size_t)n_q + 2), &pin, 1));
        int64_t *h_qoff = static_cast<int64_t *>(pin);
        uint64_t *h_qtot = reinterpret_cast<uint64_t *>(h_qoff + n_q + 1);
        int32_t *h_err = reinterpret_cast<int32_t *>(h_qtot + n_q);
        for (int64_t q = 0; q <= n_q; ++q) h_qoff[q] = qoff[q] - qoff[0];
        if (T > 0)
            HIPCHK(hipMemcpyAsync(ws->ascii.p, qbuf + qoff[0], T, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(ws->qoff.p, h_qoff, sizeof(int64_t) * (n_q + 1),
                              hipMemcpyHostToDevice, st));
        launch_fill_u32(as<uint32_t>(ws->err), 1, 0u, st);
        launch_encode_kmers(as<uint8_t>(ws->ascii), as<int64_t>(ws->qoff), (int32_t)n_q, T,
                            ix->span, ix->mask, ix->d_list_off, as<uint8_t>(ws->qcode),
                            as<uint32_t>(ws->kcode), as<uint32_t>(ws->cnt),
                            as<uint32_t>(ws->lhead), as<int32_t>(ws->qid), as<int32_t>(ws->err),
                            as<int32_t>(ws->bq), st);
        launch_scan_u32_to_u64(as<uint32_t>(ws->cnt), as<uint64_t>(ws->hoff), T,
                               as<uint64_t>(ws->partials), st);
        launch_query_totals(as<uint64_t>(ws->hoff), as<int64_t>(ws->qoff), (int32_t)n_q,
                            as<uint64_t>(ws->qtot), st);
        HIPCHK(hipMemcpyAsync(h_qtot, ws->qtot.p, sizeof(uint64_t) * n_q, hipMemcpyDeviceToHost,
                              st));
        HIPCHK(hipMemcpyAsync(h_err, ws->err.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        SYNC(st);
        if (*h_err) return GG_EINVAL;
        std::copy(h_qtot, h_qtot + n_q, hits);
        return GG_OK;
    };
    gg_status s = run();
    if (s != GG_OK) {
        (void)hipStreamSynchronize(ws->st);
        (void)hipGetLastError();
    }
    put_ws(ix, ws);
    return s;
}

gg_status search_batch_budget(const gg_index *ix, const char *qbuf, const int64_t *qoff,
                              int64_t n_q, const gg_params *params, gg_hit *out, int32_t cap,
                              int32_t *n_out, gg_stats *stats, uint64_t budget, bool device)
{
    if (!ix || n_q < 0 || n_q > (1 << 30) || cap < 0 || (n_q > 0 && (!qoff || !n_out)) ||
        (cap > 0 && n_q > 0 && !out))
        return GG_EINVAL;
    TRY(check_params(params));
    if (n_q == 0) return GG_OK;
    if (hipSetDevice(ix->device) != hipSuccess) return GG_EDEVICE;
    Workspace *ws = nullptr;
    TRY(get_ws(ix, &ws));
    BatchOut bo{out, cap, n_out, stats};
    bo.device = device;
    gg_status s = run_batch(ix, ws, qbuf, qoff, n_q, params, bo, budget);
    if (s != GG_OK) {
        (void)hipStreamSynchronize(ws->st);
        (void)hipGetLastError();
    }
    put_ws(ix, ws);
    if (s == GG_OK && bo.truncated) s = GG_ETRUNC;
    return s;
}

}  // namespace gg

// ==================================================================== C ABI

extern "C" {

const char *gg_strerror(gg_status s)
{
    switch (s) {
    case GG_OK: return "ok";
    case GG_EINVAL: return "invalid argument";
    case GG_ENOMEM: return "out of memory";
    case GG_EDEVICE: return "GPU error";
    case GG_EAGAIN: return "not finished";
    case GG_ETRUNC: return "output truncated";
    case GG_ENOTFOUND: return "unknown ticket";
    case GG_EBUDGET: return "query exceeds the hit-buffer budget";
    case GG_EIO: return "index file cannot be read or written, or is damaged";
    case GG_ESCRATCH: return "call needs more than the allocation-free scratch";
    default: return "unknown status";
    }
}

void gg_index_free(gg_index *ix)
{
    if (!ix) return;
    (void)hipSetDevice(ix->device);
    for (Workspace *ws : ix->ws_free) delete ws;
    ix->ws_free.clear();
    if (ix->d_list_off) (void)hipFree(ix->d_list_off);
    if (ix->d_post) (void)hipFree(ix->d_post);
    if (ix->d_dbw) (void)hipFree(ix->d_dbw);
    if (ix->d_seq_start) (void)hipFree(ix->d_seq_start);
    delete ix;
}

// Formatting and index construction (Sections 2, 2.1), on the GPU: the bases are
// uploaded once, packed and windowed by kernels; the lists are a stable sort of
// the windows by code, so each list keeps (sequence, position) order.
namespace {

// Device-dependent settings of a built or loaded index: the default hit budget
// and the LDS bucket sizes.
gg_status index_finish(gg_index *ix)
{
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return GG_EDEVICE;
    ix->default_budget = std::min<uint64_t>((uint64_t)16 << 30, free_b / 4);
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, ix->device) !=
        hipSuccess)
        return GG_EDEVICE;
    if ((size_t)lds < (size_t)kBucketCapMax * 8 * (kBlock / 64) + 1024) return GG_EDEVICE;
    ix->bucket_cap = kBucketCapMax;
    ix->bucket_big = (size_t)lds >= (size_t)kBucketBig * 8 + 1024 && setup_kernels() == hipSuccess
                         ? kBucketBig
                         : kBucketCapMax;
    (void)hipGetLastError();
    return GG_OK;
}

// Windows of `span` bases coded on the bases of `mask` (k of them); the plain
// index is span = k with every base coded.
gg_status index_build(const char *seqs, const int64_t *seq_off, int64_t n_in, int32_t span,
                      uint32_t mask, int32_t k, int32_t strands, int64_t max_posting,
                      int32_t device, gg_index **out)
{
    if (!out) return GG_EINVAL;
    *out = nullptr;
    if (k < 1 || k > 16 || span < k || span > 32 || n_in < 0 || (strands != 1 && strands != 2) ||
        max_posting < 0 || n_in * strands > INT32_MAX)
        return GG_EINVAL;
    // with both strands, sequence n_in + s is the reverse complement of sequence s
    const int64_t n_seqs = n_in * strands;
    if (n_in > 0 && (!seq_off || !seqs)) return GG_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return GG_EDEVICE;
    const int64_t base0 = n_in > 0 ? seq_off[0] : 0;
    int64_t maxlen = 0;
    for (int64_t s = 0; s < n_in; ++s) {
        const int64_t n = seq_off[s + 1] - seq_off[s];
        if (n < 0 || n > INT32_MAX) return GG_EINVAL;
        maxlen = std::max(maxlen, n);
    }
    const int64_t total_in = n_in > 0 ? seq_off[n_in] - base0 : 0;
    const int64_t total = total_in * strands;
    // windows before each sequence (sequence lengths only; the bases go to the GPU)
    std::vector<uint32_t> woff((size_t)n_seqs + 1, 0u);
    std::vector<int64_t> seq_start((size_t)n_seqs + 1, 0);
    uint64_t n_post = 0;
    for (int64_t s = 0; s < n_seqs; ++s) {
        const int64_t f = s % (n_in > 0 ? n_in : 1);  // the forward sequence of s
        woff[(size_t)s] = (uint32_t)std::min<uint64_t>(n_post, 0xffffffffull);
        n_post += (uint64_t)((seq_off[f + 1] - seq_off[f]) / span);
        seq_start[(size_t)s] = seq_off[f] - base0 + (s >= n_in ? total_in : 0);
    }
    if (n_post >= 0xffffffffull) return GG_EINVAL;
    woff[(size_t)n_seqs] = (uint32_t)n_post;
    seq_start[(size_t)n_seqs] = total;
    const int64_t nwords = (total + 15) / 16 + 1;  // one spare word for window reads
    const uint64_t ncode = (uint64_t)1 << (2 * k);

    auto *ix = new (std::nothrow) gg_index();
    if (!ix) return GG_ENOMEM;
    ix->device = device;
    ix->k = k;
    ix->span = span;
    ix->mask = mask;
    ix->strands = strands;
    ix->n_seqs = n_seqs;
    ix->n_bases = total;
    ix->n_post = n_post;
    ix->max_seq_len = maxlen;
    auto fail = [&](gg_status s) {
        gg_index_free(ix);
        return s;
    };
    if (hipSetDevice(device) != hipSuccess) return fail(GG_EDEVICE);
    auto alloc = [](void **dst, size_t bytes) -> gg_status {
        if (hipMalloc(dst, std::max<size_t>(bytes, 16)) != hipSuccess) {
            (void)hipGetLastError();
            *dst = nullptr;
            return GG_ENOMEM;
        }
        return GG_OK;
    };
    gg_status s;
    // with a repeat cutoff the postings are allocated once the kept count is known
    const bool cut = max_posting > 0 && (uint64_t)max_posting < n_post;
    if ((s = alloc((void **)&ix->d_list_off, sizeof(uint32_t) * (ncode + 1))) != GG_OK ||
        (!cut && (s = alloc((void **)&ix->d_post, sizeof(int2) * n_post)) != GG_OK) ||
        (s = alloc((void **)&ix->d_dbw, sizeof(uint32_t) * nwords)) != GG_OK ||
        (s = alloc((void **)&ix->d_seq_start, sizeof(int64_t) * (n_seqs + 1))) != GG_OK)
        return fail(s);

    // Sections 2, 2.1 on the GPU: pack the bases, code every window, sort the
    // windows stably by code (they start in (seq, pos) order, so every list stays
    // in that order), list heads = exclusive scan of the per-code counts.
    {
        struct Tmp {
            std::vector<void *> p;
            ~Tmp()
            {
                for (void *x : p) (void)hipFree(x);
            }
            void *get(size_t bytes)
            {
                void *x = nullptr;
                if (hipMalloc(&x, std::max<size_t>(bytes, 16)) != hipSuccess) {
                    (void)hipGetLastError();
                    return nullptr;
                }
                p.push_back(x);
                return x;
            }
        } tmp;
        hipStream_t bst = nullptr;
        if (hipStreamCreateWithFlags(&bst, hipStreamNonBlocking) != hipSuccess) return fail(GG_EDEVICE);
        struct StreamGuard {
            hipStream_t s;
            ~StreamGuard() { (void)hipStreamDestroy(s); }
        } sg{bst};
        const uint32_t nw = (uint32_t)n_post;
        auto *d_ascii = static_cast<uint8_t *>(tmp.get((size_t)total));
        auto *d_woff = static_cast<uint32_t *>(tmp.get(sizeof(uint32_t) * (n_seqs + 1)));
        auto *d_err = static_cast<int32_t *>(tmp.get(sizeof(int32_t) * 4));
        auto *d_keys = static_cast<uint64_t *>(tmp.get(sizeof(uint64_t) * nw));
        auto *d_keys2 = static_cast<uint64_t *>(tmp.get(sizeof(uint64_t) * nw));
        auto *d_vals = static_cast<uint32_t *>(tmp.get(sizeof(uint32_t) * nw));
        auto *d_vals2 = static_cast<uint32_t *>(tmp.get(sizeof(uint32_t) * nw));
        auto *d_hist = static_cast<uint32_t *>(tmp.get(sizeof(uint32_t) * radix_hist_needed(nw)));
        const size_t parts = std::max<size_t>(scan_partials_needed(radix_hist_needed(nw)),
                                              scan_partials_needed((int64_t)ncode + 1));
        auto *d_parts = static_cast<uint32_t *>(tmp.get(sizeof(uint32_t) * parts));
        auto *d_kept = cut ? static_cast<uint32_t *>(tmp.get(sizeof(uint32_t) * (ncode + 1)))
                           : nullptr;
        if (!d_ascii || !d_woff || !d_err || !d_keys || !d_keys2 || !d_vals || !d_vals2 ||
            !d_hist || !d_parts || (cut && !d_kept))
            return fail(GG_ENOMEM);
        int32_t err = 0;
        if (total_in > 0 && hipMemcpyAsync(d_ascii, seqs + base0, (size_t)total_in,
                                           hipMemcpyHostToDevice, bst) != hipSuccess)
            return fail(GG_EDEVICE);
        if (hipMemcpyAsync(d_woff, woff.data(), sizeof(uint32_t) * (n_seqs + 1),
                           hipMemcpyHostToDevice, bst) != hipSuccess ||
            hipMemcpyAsync(ix->d_seq_start, seq_start.data(), sizeof(int64_t) * (n_seqs + 1),
                           hipMemcpyHostToDevice, bst) != hipSuccess ||
            hipMemsetAsync(d_err, 0, sizeof(int32_t), bst) != hipSuccess ||
            hipMemsetAsync(ix->d_list_off, 0, sizeof(uint32_t) * (ncode + 1), bst) != hipSuccess)
            return fail(GG_EDEVICE);
        if (strands == 2)  // the first n_in + 1 starts are the forward sequences'
            launch_reverse_strand(d_ascii, ix->d_seq_start, (int32_t)n_in, d_ascii + total_in, bst);
        launch_pack_bases(d_ascii, total, ix->d_dbw, nwords, d_err, bst);
        launch_window_keys(ix->d_dbw, ix->d_seq_start, d_woff, (int32_t)n_seqs, nw, span, mask,
                           d_keys, d_vals, ix->d_list_off, bst);
        launch_scan_u32(ix->d_list_off, ix->d_list_off, (int64_t)ncode, d_parts, bst);
        const int cur = radix_sort(d_keys, d_keys2, d_vals, d_vals2, nw, 0, 2 * k, d_hist, d_parts,
                                   bst);
        if (!cut) {
            launch_postings(cur ? d_vals2 : d_vals, nw, d_woff, (int32_t)n_seqs, span, ix->d_post,
                            bst);
        } else {  // drop the lists longer than max_posting, then place the others
            const uint32_t mp = (uint32_t)max_posting;
            uint32_t kept = 0;
            launch_cut_counts(ix->d_list_off, (uint32_t)ncode, mp, d_kept, bst);
            launch_scan_u32(d_kept, d_kept, (int64_t)ncode, d_parts, bst);
            if (hipMemcpyAsync(&kept, d_kept + ncode, sizeof(uint32_t), hipMemcpyDeviceToHost,
                               bst) != hipSuccess ||
                hipStreamSynchronize(bst) != hipSuccess)
                return fail(GG_EDEVICE);
            if ((s = alloc((void **)&ix->d_post, sizeof(int2) * kept)) != GG_OK) return fail(s);
            ix->n_post = kept;
            launch_postings_cut(cur ? d_vals2 : d_vals, cur ? d_keys2 : d_keys, nw, d_woff,
                                (int32_t)n_seqs, span, ix->d_list_off, d_kept, mp, ix->d_post, bst);
            if (hipMemcpyAsync(ix->d_list_off, d_kept, sizeof(uint32_t) * (ncode + 1),
                               hipMemcpyDeviceToDevice, bst) != hipSuccess)
                return fail(GG_EDEVICE);
        }
        if (hipMemcpyAsync(&err, d_err, sizeof(int32_t), hipMemcpyDeviceToHost, bst) != hipSuccess ||
            hipStreamSynchronize(bst) != hipSuccess || hipGetLastError() != hipSuccess)
            return fail(GG_EDEVICE);
        if (err) return fail(GG_EINVAL);
    }

    if ((s = index_finish(ix)) != GG_OK) return fail(s);
    *out = ix;
    return GG_OK;
}

}  // namespace

gg_status gg_index_build(const char *seqs, const int64_t *seq_off, int64_t n_seqs, int32_t k,
                         int32_t device, gg_index **out)
{
    if (k < 1 || k > 16) {
        if (out) *out = nullptr;
        return GG_EINVAL;
    }
    return index_build(seqs, seq_off, n_seqs, k, (1u << k) - 1u, k, 1, 0, device, out);
}

gg_status gg_index_build_masked(const char *seqs, const int64_t *seq_off, int64_t n_seqs,
                                const char *mask, int32_t device, gg_index **out)
{
    gg_index_options opt{0, mask, 1, 0};
    return gg_index_build_ex(seqs, seq_off, n_seqs, &opt, device, out);
}

gg_status gg_index_build_ex(const char *seqs, const int64_t *seq_off, int64_t n_seqs,
                            const gg_index_options *opt, int32_t device, gg_index **out)
{
    if (out) *out = nullptr;
    if (!opt) return GG_EINVAL;
    if (!opt->mask) {
        if (opt->k < 1 || opt->k > 16) return GG_EINVAL;
        return index_build(seqs, seq_off, n_seqs, opt->k, (1u << opt->k) - 1u, opt->k,
                           opt->strands, opt->max_posting, device, out);
    }
    const char *mask = opt->mask;
    int32_t span = 0, weight = 0;
    uint32_t bits = 0;
    for (; mask[span]; ++span) {
        if (span >= 32) return GG_EINVAL;
        if (mask[span] == '1') {
            bits |= 1u << span;
            ++weight;
        } else if (mask[span] != '0') {
            return GG_EINVAL;
        }
    }
    if (weight < 1 || weight > 16) return GG_EINVAL;
    return index_build(seqs, seq_off, n_seqs, span, bits, weight, opt->strands, opt->max_posting,
                       device, out);
}

gg_status gg_index_info(const gg_index *ix, int64_t *n_postings, int64_t *n_bases, int64_t *n_seqs,
                        int32_t *k)
{
    if (!ix) return GG_EINVAL;
    if (n_postings) *n_postings = (int64_t)ix->n_post;
    if (n_bases) *n_bases = ix->n_bases;
    if (n_seqs) *n_seqs = ix->n_seqs;
    if (k) *k = ix->k;
    return GG_OK;
}

gg_status gg_index_export(const gg_index *ix, uint32_t *list_off, int32_t *postings,
                          int64_t cap_postings)
{
    if (!ix) return GG_EINVAL;
    if (postings && cap_postings < (int64_t)ix->n_post) return GG_ETRUNC;
    if (hipSetDevice(ix->device) != hipSuccess) return GG_EDEVICE;
    const size_t nheads = ((size_t)1 << (2 * ix->k)) + 1;
    if (list_off && hipMemcpy(list_off, ix->d_list_off, sizeof(uint32_t) * nheads,
                              hipMemcpyDeviceToHost) != hipSuccess)
        return GG_EDEVICE;
    if (postings && ix->n_post > 0 &&
        hipMemcpy(postings, ix->d_post, sizeof(int2) * ix->n_post, hipMemcpyDeviceToHost) !=
            hipSuccess)
        return GG_EDEVICE;
    return GG_OK;
}

namespace {

// Hash of an index file's bytes after the magic: 64-bit words (the last one
// zero-padded), each xored in and mixed by a multiply and a shift.
struct FileHash {
    uint64_t h = 0x9e3779b97f4a7c15ull;
    uint8_t part[8];
    size_t np = 0;
    void word(uint64_t w)
    {
        h ^= w;
        h *= 0xff51afd7ed558ccdull;
        h ^= h >> 33;
    }
    void add(const void *data, size_t n)
    {
        const uint8_t *b = static_cast<const uint8_t *>(data);
        while (n && np) {
            part[np++] = *b++;
            --n;
            if (np == 8) {
                uint64_t w;
                memcpy(&w, part, 8);
                word(w);
                np = 0;
            }
        }
        for (; n >= 8; n -= 8, b += 8) {
            uint64_t w;
            memcpy(&w, b, 8);
            word(w);
        }
        while (n--) part[np++] = *b++;
    }
    uint64_t done()
    {
        if (np) {
            memset(part + np, 0, 8 - np);
            uint64_t w;
            memcpy(&w, part, 8);
            word(w);
            np = 0;
        }
        return h;
    }
};

struct FileHeader {
    char magic[8];
    uint32_t version;
    int32_t k, span, strands;
    uint32_t mask, zero;
    int64_t n_seqs, n_bases, n_post, max_seq_len, n_words;
};
static_assert(sizeof(FileHeader) == 72, "index file header layout");
constexpr char kFileMagic[8] = {'G', 'G', 'I', 'N', 'D', 'E', 'X', '1'};

struct File {
    FILE *f = nullptr;
    ~File()
    {
        if (f) fclose(f);
    }
};

bool write_all(FILE *f, FileHash &hash, const void *data, size_t n)
{
    hash.add(data, n);
    return n == 0 || fwrite(data, 1, n, f) == n;
}

bool read_all(FILE *f, FileHash &hash, void *data, size_t n)
{
    if (n && fread(data, 1, n, f) != n) return false;
    hash.add(data, n);
    return true;
}

}  // namespace

gg_status gg_index_save(const gg_index *ix, const char *path)
{
    if (!ix || !path) return GG_EINVAL;
    if (hipSetDevice(ix->device) != hipSuccess) return GG_EDEVICE;
    const size_t nheads = ((size_t)1 << (2 * ix->k)) + 1;
    const int64_t nwords = (ix->n_bases + 15) / 16 + 1;
    std::vector<int64_t> seq_start((size_t)ix->n_seqs + 1);
    std::vector<uint32_t> heads(nheads);
    std::vector<int2> post((size_t)ix->n_post);
    std::vector<uint32_t> bank((size_t)nwords);
    if (hipMemcpy(seq_start.data(), ix->d_seq_start, sizeof(int64_t) * seq_start.size(),
                  hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(heads.data(), ix->d_list_off, sizeof(uint32_t) * nheads,
                  hipMemcpyDeviceToHost) != hipSuccess ||
        (ix->n_post && hipMemcpy(post.data(), ix->d_post, sizeof(int2) * post.size(),
                                 hipMemcpyDeviceToHost) != hipSuccess) ||
        hipMemcpy(bank.data(), ix->d_dbw, sizeof(uint32_t) * bank.size(), hipMemcpyDeviceToHost) !=
            hipSuccess)
        return GG_EDEVICE;
    FileHeader hd{};
    memcpy(hd.magic, kFileMagic, 8);
    hd.version = 1;
    hd.k = ix->k;
    hd.span = ix->span;
    hd.strands = ix->strands;
    hd.mask = ix->mask;
    hd.n_seqs = ix->n_seqs;
    hd.n_bases = ix->n_bases;
    hd.n_post = (int64_t)ix->n_post;
    hd.max_seq_len = ix->max_seq_len;
    hd.n_words = nwords;
    File fl;
    fl.f = fopen(path, "wb");
    if (!fl.f) return GG_EIO;
    FileHash hash;
    if (fwrite(hd.magic, 1, 8, fl.f) != 8 ||
        !write_all(fl.f, hash, reinterpret_cast<const char *>(&hd) + 8, sizeof(hd) - 8) ||
        !write_all(fl.f, hash, seq_start.data(), sizeof(int64_t) * seq_start.size()) ||
        !write_all(fl.f, hash, heads.data(), sizeof(uint32_t) * heads.size()) ||
        !write_all(fl.f, hash, post.data(), sizeof(int2) * post.size()) ||
        !write_all(fl.f, hash, bank.data(), sizeof(uint32_t) * bank.size()))
        return GG_EIO;
    const uint64_t check = hash.done();
    if (fwrite(&check, 1, 8, fl.f) != 8) return GG_EIO;
    const int rc = fclose(fl.f);
    fl.f = nullptr;
    return rc == 0 ? GG_OK : GG_EIO;
}

gg_status gg_index_load(const char *path, int32_t device, gg_index **out)
{
    if (!out || !path) return GG_EINVAL;
    *out = nullptr;
    File fl;
    fl.f = fopen(path, "rb");
    if (!fl.f) return GG_EIO;
    FileHeader hd{};
    FileHash hash;
    if (fread(hd.magic, 1, 8, fl.f) != 8 || memcmp(hd.magic, kFileMagic, 8) != 0 ||
        !read_all(fl.f, hash, reinterpret_cast<char *>(&hd) + 8, sizeof(hd) - 8) || hd.version != 1)
        return GG_EIO;
    // header consistency (before any size is trusted)
    if (hd.k < 1 || hd.k > 16 || hd.span < hd.k || hd.span > 32 || (hd.strands != 1 && hd.strands != 2) ||
        hd.zero != 0 || __builtin_popcount(hd.mask) != hd.k ||
        (hd.span < 32 && (hd.mask >> hd.span) != 0) || hd.n_seqs < 0 || hd.n_seqs > INT32_MAX ||
        hd.n_bases < 0 || hd.n_post < 0 || hd.n_post >= (int64_t)0xffffffffll ||
        hd.max_seq_len < 0 || hd.max_seq_len > INT32_MAX || hd.n_words != (hd.n_bases + 15) / 16 + 1)
        return GG_EINVAL;
    const uint64_t nheads = ((uint64_t)1 << (2 * hd.k)) + 1;
    const uint64_t want = 8 + sizeof(FileHeader) - 8 + 8 * ((uint64_t)hd.n_seqs + 1) + 4 * nheads +
                          8 * (uint64_t)hd.n_post + 4 * (uint64_t)hd.n_words + 8;
    if (fseeko(fl.f, 0, SEEK_END) != 0 || (uint64_t)ftello(fl.f) != want ||
        fseeko(fl.f, (off_t)sizeof(FileHeader), SEEK_SET) != 0)
        return GG_EIO;
    std::vector<int64_t> seq_start((size_t)hd.n_seqs + 1);
    std::vector<uint32_t> heads((size_t)nheads);
    std::vector<int2> post((size_t)hd.n_post);
    std::vector<uint32_t> bank((size_t)hd.n_words);
    uint64_t check = 0;
    if (!read_all(fl.f, hash, seq_start.data(), sizeof(int64_t) * seq_start.size()) ||
        !read_all(fl.f, hash, heads.data(), sizeof(uint32_t) * heads.size()) ||
        !read_all(fl.f, hash, post.data(), sizeof(int2) * post.size()) ||
        !read_all(fl.f, hash, bank.data(), sizeof(uint32_t) * bank.size()) ||
        fread(&check, 1, 8, fl.f) != 8 || check != hash.done())
        return GG_EIO;
    // contents: every later kernel indexes through these, so each is checked
    int64_t maxlen = 0;
    if (seq_start[0] != 0 || seq_start[(size_t)hd.n_seqs] != hd.n_bases) return GG_EINVAL;
    for (int64_t s = 0; s < hd.n_seqs; ++s) {
        const int64_t n = seq_start[(size_t)s + 1] - seq_start[(size_t)s];
        if (n < 0 || n > INT32_MAX) return GG_EINVAL;
        maxlen = std::max(maxlen, n);
    }
    if (maxlen != hd.max_seq_len || heads[0] != 0 || heads[(size_t)nheads - 1] != (uint64_t)hd.n_post)
        return GG_EINVAL;
    for (uint64_t c = 0; c + 1 < nheads; ++c)
        if (heads[c + 1] < heads[c]) return GG_EINVAL;
    for (const int2 &e : post) {
        if (e.x < 0 || e.x >= hd.n_seqs || e.y < 0 || e.y % hd.span != 0) return GG_EINVAL;
        if ((int64_t)e.y + hd.span > seq_start[(size_t)e.x + 1] - seq_start[(size_t)e.x])
            return GG_EINVAL;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return GG_EDEVICE;
    auto *ix = new (std::nothrow) gg_index();
    if (!ix) return GG_ENOMEM;
    ix->device = device;
    ix->k = hd.k;
    ix->span = hd.span;
    ix->mask = hd.mask;
    ix->strands = hd.strands;
    ix->n_seqs = hd.n_seqs;
    ix->n_bases = hd.n_bases;
    ix->n_post = (uint64_t)hd.n_post;
    ix->max_seq_len = hd.max_seq_len;
    auto fail = [&](gg_status st) {
        gg_index_free(ix);
        return st;
    };
    if (hipSetDevice(device) != hipSuccess) return fail(GG_EDEVICE);
    auto up = [](void **dst, const void *src, size_t bytes) -> gg_status {
        if (hipMalloc(dst, std::max<size_t>(bytes, 16)) != hipSuccess) {
            (void)hipGetLastError();
            *dst = nullptr;
            return GG_ENOMEM;
        }
        if (bytes && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess)
            return GG_EDEVICE;
        return GG_OK;
    };
    gg_status st;
    if ((st = up((void **)&ix->d_seq_start, seq_start.data(), sizeof(int64_t) * seq_start.size())) !=
            GG_OK ||
        (st = up((void **)&ix->d_list_off, heads.data(), sizeof(uint32_t) * heads.size())) != GG_OK ||
        (st = up((void **)&ix->d_post, post.data(), sizeof(int2) * post.size())) != GG_OK ||
        (st = up((void **)&ix->d_dbw, bank.data(), sizeof(uint32_t) * bank.size())) != GG_OK)
        return fail(st);
    if ((st = index_finish(ix)) != GG_OK) return fail(st);
    *out = ix;
    return GG_OK;
}

gg_status gg_index_set_hit_budget(gg_index *ix, uint64_t bytes)
{
    if (!ix) return GG_EINVAL;
    ix->hit_budget = bytes;
    return GG_OK;
}

gg_status gg_index_get_tuning(const gg_index *ix, gg_tuning *out)
{
    if (!ix || !out) return GG_EINVAL;
    out->grouping = ix->tune_grouping.load();
    out->lane_steps = ix->tune_lane_steps.load();
    out->ms = 0.0;
    const int32_t lg = ix->tune_wave_log2.load();
    out->wave_log2 = lg > 0 ? lg : 25;
    out->graph = ix->tune_graph.load();
    out->graph_query_log2 = ix->tune_graph_qlog2.load();
    return GG_OK;
}

gg_status gg_index_set_tuning(gg_index *ix, const gg_tuning *t)
{
    if (!ix || !t || t->grouping < 0 || t->grouping > 2 || t->lane_steps < 0 ||
        t->lane_steps > 4096 || (t->wave_log2 != 0 && (t->wave_log2 < 10 || t->wave_log2 > 30)) ||
        t->graph < 0 || t->graph > 1 || t->graph_query_log2 < 0 || t->graph_query_log2 > 30)
        return GG_EINVAL;
    ix->tune_grouping = t->grouping;
    ix->tune_lane_steps = t->lane_steps;
    ix->tune_wave_log2 = t->wave_log2;
    ix->tune_graph = t->graph;
    ix->tune_graph_qlog2 = t->graph_query_log2;
    return GG_OK;
}

gg_status gg_index_autotune(gg_index *ix, const char *qbuf, const int64_t *qoff, int64_t n_q,
                            const gg_params *params, gg_tuning *chosen)
{
    if (!ix || n_q < 1 || !qoff || !params) return GG_EINVAL;
    const int64_t T = qoff[n_q] - qoff[0];
    if (T < 0 || (T > 0 && !qbuf)) return GG_EINVAL;
    const int32_t cap = params->max_hits > 0 ? params->max_hits : 256;
    gg_tuning keep;
    TRY(gg_index_get_tuning(ix, &keep));
    if (hipSetDevice(ix->device) != hipSuccess) return GG_EDEVICE;
    // the sample is timed in the device-resident form (queries and hits in GPU
    // memory), so transfers do not blur the comparison
    struct Dev {
        void *q = nullptr, *out = nullptr, *n = nullptr;
        ~Dev()
        {
            for (void *x : {q, out, n})
                if (x) (void)hipFree(x);
        }
    } dev;
    const size_t out_bytes = sizeof(gg_hit) * (size_t)n_q * cap;
    if (hipMalloc(&dev.q, (size_t)std::max<int64_t>(T, 1)) != hipSuccess ||
        hipMalloc(&dev.out, out_bytes) != hipSuccess ||
        hipMalloc(&dev.n, sizeof(int32_t) * n_q) != hipSuccess) {
        (void)hipGetLastError();
        return GG_ENOMEM;
    }
    if (T > 0 && hipMemcpy(dev.q, qbuf + qoff[0], (size_t)T, hipMemcpyHostToDevice) != hipSuccess)
        return GG_EDEVICE;
    std::vector<int64_t> off((size_t)n_q + 1);
    for (int64_t q = 0; q <= n_q; ++q) off[(size_t)q] = qoff[q] - qoff[0];
    std::vector<gg_hit> ref, out((size_t)n_q * cap);
    std::vector<int32_t> ref_n, n_out((size_t)n_q);
    gg_tuning best = keep;
    best.ms = -1.0;
    // one candidate: timed (best of three runs after one untimed), and its hits
    // must equal the first candidate's
    auto trial = [&](const gg_tuning &t) -> gg_status {
        TRY(gg_index_set_tuning(ix, &t));
        double ms = -1.0;
        for (int rep = -1; rep < 3; ++rep) {  // rep -1 warms up (graph capture, buffers)
            const auto t0 = std::chrono::steady_clock::now();
            gg_status s = gg::search_batch_budget(
                ix, static_cast<const char *>(dev.q), off.data(), n_q, params,
                static_cast<gg_hit *>(dev.out), cap, static_cast<int32_t *>(dev.n), nullptr,
                gg::index_budget(ix), true);
            const double dt = std::chrono::duration<double, std::milli>(
                                  std::chrono::steady_clock::now() - t0)
                                  .count();
            if (s != GG_OK && s != GG_ETRUNC) return s;
            if (rep < 0) continue;
            ms = ms < 0 ? dt : std::min(ms, dt);
            if (best.ms >= 0 && ms > 2.0 * best.ms) break;  // clearly slower: one run is enough
        }
        if (hipMemcpy(out.data(), dev.out, out_bytes, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(n_out.data(), dev.n, sizeof(int32_t) * n_q, hipMemcpyDeviceToHost) !=
                hipSuccess)
            return GG_EDEVICE;
        if (ref.empty()) {
            ref = out;
            ref_n = n_out;
        } else {
            bool same = ref_n == n_out;
            for (int64_t q = 0; same && q < n_q; ++q) {
                const size_t m = (size_t)std::min(n_out[(size_t)q], cap);
                same = memcmp(&ref[(size_t)q * cap], &out[(size_t)q * cap],
                              sizeof(gg_hit) * m) == 0;
            }
            if (!same) return GG_EDEVICE;
        }
        if (best.ms < 0 || ms < best.ms) {
            best = t;
            best.ms = ms;
        }
        return GG_OK;
    };
    gg_status s = GG_OK;
    // how hits become runs and the extension's lane-step cap, then (for the
    // radix-sort grouping, whose batches replay a captured graph per wave) the
    // hits of one graph wave
    for (int32_t grouping = 0; grouping <= 2 && s == GG_OK; ++grouping)
        for (int32_t steps : {0, 64, 256, 4096})
            if (s == GG_OK)
                s = trial(gg_tuning{grouping, steps, 0.0, keep.wave_log2, keep.graph,
                                    keep.graph_query_log2});
    if (s == GG_OK && best.grouping == 2) {
        const gg_tuning base = best;
        auto with = [&](int32_t wave, int32_t graph, int32_t qlg) {
            return gg_tuning{base.grouping, base.lane_steps, 0.0, wave, graph, qlg};
        };
        for (int32_t lg : {23, 27})
            if (s == GG_OK && lg != base.wave_log2) s = trial(with(lg, base.graph, base.graph_query_log2));
        const gg_tuning b2 = best;
        for (int32_t qlg : {14, 18})
            if (s == GG_OK) s = trial(gg_tuning{b2.grouping, b2.lane_steps, 0.0, b2.wave_log2, 1, qlg});
        if (s == GG_OK) s = trial(gg_tuning{b2.grouping, b2.lane_steps, 0.0, b2.wave_log2, 0, 0});
    }
    if (s != GG_OK) {
        (void)gg_index_set_tuning(ix, &keep);
        return s;
    }
    TRY(gg_index_set_tuning(ix, &best));
    if (chosen) *chosen = best;
    return GG_OK;
}

gg_status gg_search_batch(const gg_index *ix, const char *qbuf, const int64_t *qoff, int64_t n_q,
                          const gg_params *params, gg_hit *out, int32_t cap, int32_t *n_out,
                          gg_stats *stats)
{
    if (!ix) return GG_EINVAL;
    return gg::search_batch_budget(ix, qbuf, qoff, n_q, params, out, cap, n_out, stats,
                                   budget_of(ix), false);
}

gg_status gg_search_batch_device(const gg_index *ix, const char *d_qbuf, const int64_t *qoff,
                                 int64_t n_q, const gg_params *params, gg_hit *d_out, int32_t cap,
                                 int32_t *d_n_out, gg_stats *stats)
{
    if (!ix) return GG_EINVAL;
    if (n_q > 0 && !d_n_out) return GG_EINVAL;
    return gg::search_batch_budget(ix, d_qbuf, qoff, n_q, params, d_out, cap, d_n_out, stats,
                                   budget_of(ix), true);
}

gg_status gg_device_alloc(int32_t device, uint64_t bytes, void **ptr)
{
    if (!ptr) return GG_EINVAL;
    *ptr = nullptr;
    if (hipSetDevice(device) != hipSuccess) return GG_EDEVICE;
    if (hipMalloc(ptr, std::max<uint64_t>(bytes, 1)) != hipSuccess) {
        (void)hipGetLastError();
        *ptr = nullptr;
        return GG_ENOMEM;
    }
    return GG_OK;
}

gg_status gg_device_free(int32_t device, void *ptr)
{
    if (!ptr) return GG_OK;
    if (hipSetDevice(device) != hipSuccess) return GG_EDEVICE;
    return hipFree(ptr) == hipSuccess ? GG_OK : GG_EDEVICE;
}

gg_status gg_memcpy_to_device(void *dst, const void *src, uint64_t bytes)
{
    if (bytes == 0) return GG_OK;
    if (!dst || !src) return GG_EINVAL;
    return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess ? GG_OK : GG_EDEVICE;
}

gg_status gg_device_copy(void *dst, const void *src, uint64_t bytes)
{
    if (bytes == 0) return GG_OK;
    if (!dst || !src) return GG_EINVAL;
    if (hipMemcpy(dst, src, bytes, hipMemcpyDeviceToDevice) != hipSuccess) return GG_EDEVICE;
    return hipDeviceSynchronize() == hipSuccess ? GG_OK : GG_EDEVICE;
}

gg_status gg_device_read(const void *src, uint64_t bytes, uint64_t *sum)
{
    if (!src || !sum || bytes % 16 != 0) return GG_EINVAL;
    void *d = nullptr;
    if (hipMalloc(&d, sizeof(unsigned long long)) != hipSuccess) return GG_ENOMEM;
    gg_status s = GG_OK;
    if (hipMemset(d, 0, sizeof(unsigned long long)) != hipSuccess) s = GG_EDEVICE;
    if (s == GG_OK) {
        gg::launch_stream_read(src, bytes, static_cast<unsigned long long *>(d), nullptr);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpy(sum, d, sizeof(uint64_t), hipMemcpyDeviceToHost) != hipSuccess)
            s = GG_EDEVICE;
    }
    (void)hipFree(d);
    return s;
}

gg_status gg_memcpy_to_host(void *dst, const void *src, uint64_t bytes)
{
    if (bytes == 0) return GG_OK;
    if (!dst || !src) return GG_EINVAL;
    return hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost) == hipSuccess ? GG_OK : GG_EDEVICE;
}

gg_status gg_search(const gg_index *ix, const char *query, int64_t qlen, const gg_params *params,
                    gg_hit *out, int32_t cap, int32_t *n_out)
{
    if (qlen < 0 || (qlen > 0 && !query) || !n_out) return GG_EINVAL;
    const int64_t off[2] = {0, qlen};
    return gg_search_batch(ix, query, off, 1, params, out, cap, n_out, nullptr);
}

gg_status gg_traceback(const gg_index *ix, const char *query, int64_t qlen, const gg_params *params,
                       const gg_hit *hits, int32_t n, char *ops, int64_t ops_cap, int64_t *ops_off,
                       int32_t *ops_len)
{
    if (!ix || qlen < 0 || qlen > INT32_MAX || (qlen > 0 && !query) || n < 0 ||
        (n > 0 && (!hits || !ops_off || !ops_len)))
        return GG_EINVAL;
    TRY(check_params(params));
    // slots: each hit's operations fit in (query span + bank span) bytes
    std::vector<int64_t> dir_off((size_t)n + 1, 0);
    ops_off[0] = 0;
    for (int32_t h = 0; h < n; ++h) {
        const gg_hit &x = hits[h];
        if (x.seq_id < 0 || x.seq_id >= ix->n_seqs || x.q_start < 0 || x.q_end <= x.q_start ||
            x.q_end > qlen || x.d_start < 0 || x.d_end <= x.d_start || x.score <= 0)
            return GG_EINVAL;
        const int64_t R = x.q_end - x.q_start, C = x.d_end - x.d_start;
        ops_off[h + 1] = ops_off[h] + R + C;
        dir_off[(size_t)h + 1] = dir_off[(size_t)h] + 64 * R;
    }
    if (n == 0) return GG_OK;
    if (ops_cap < ops_off[n] || !ops) return GG_ETRUNC;
    if (hipSetDevice(ix->device) != hipSuccess) return GG_EDEVICE;
    Workspace *ws = nullptr;
    TRY(get_ws(ix, &ws));
    std::vector<char> slots((size_t)ops_off[n]);
    std::vector<int32_t> len((size_t)n), status((size_t)n);
    auto run = [&]() -> gg_status {
        hipStream_t st = ws->st;
        TRY(ensure(ws->tb_hits, sizeof(gg_hit) * (size_t)n));
        TRY(ensure(ws->tb_q, (size_t)qlen));
        TRY(ensure(ws->tb_dir, (size_t)dir_off[(size_t)n]));
        TRY(ensure(ws->tb_dir_off, sizeof(int64_t) * (size_t)(n + 1)));
        TRY(ensure(ws->tb_ops_off, sizeof(int64_t) * (size_t)(n + 1)));
        TRY(ensure(ws->tb_ops, (size_t)ops_off[n]));
        TRY(ensure(ws->tb_len, sizeof(int32_t) * (size_t)n));
        TRY(ensure(ws->tb_status, sizeof(int32_t) * (size_t)n));
        HIPCHK(hipMemcpyAsync(ws->tb_hits.p, hits, sizeof(gg_hit) * (size_t)n,
                              hipMemcpyHostToDevice, st));
        if (qlen > 0)
            HIPCHK(hipMemcpyAsync(ws->tb_q.p, query, (size_t)qlen, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(ws->tb_dir_off.p, dir_off.data(), sizeof(int64_t) * (size_t)(n + 1),
                              hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(ws->tb_ops_off.p, ops_off, sizeof(int64_t) * (size_t)(n + 1),
                              hipMemcpyHostToDevice, st));
        launch_traceback(as<int32_t>(ws->tb_hits), n, as<uint8_t>(ws->tb_q), qlen, ix->d_dbw,
                         ix->d_seq_start, (int32_t)ix->n_seqs, params->match, params->mismatch,
                         params->gap_open, params->gap_extend, params->band,
                         as<int64_t>(ws->tb_dir_off), as<uint8_t>(ws->tb_dir),
                         as<int64_t>(ws->tb_ops_off), as<char>(ws->tb_ops), as<int32_t>(ws->tb_len),
                         as<int32_t>(ws->tb_status), st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(slots.data(), ws->tb_ops.p, slots.size(), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(len.data(), ws->tb_len.p, sizeof(int32_t) * (size_t)n,
                              hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(status.data(), ws->tb_status.p, sizeof(int32_t) * (size_t)n,
                              hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return GG_OK;
    };
    gg_status s = run();
    if (s != GG_OK) {
        (void)hipStreamSynchronize(ws->st);
        (void)hipGetLastError();
    }
    put_ws(ix, ws);
    if (s != GG_OK) return s;
    // the kernel wrote each path right-aligned in its slot; hand it over left-aligned
    bool all_ok = true;
    for (int32_t h = 0; h < n; ++h) {
        const int64_t slot = ops_off[h + 1] - ops_off[h];
        ops_len[h] = status[(size_t)h] == 0 ? len[(size_t)h] : 0;
        all_ok = all_ok && status[(size_t)h] == 0;
        memcpy(ops + ops_off[h], slots.data() + ops_off[h] + slot - ops_len[h], (size_t)ops_len[h]);
    }
    return all_ok ? GG_OK : GG_EINVAL;
}

}  // extern "C"

// ---- allocation-free traceback
// Device scratch of gg_traceback_noalloc: one file-scope array per GPU, held until
// the process ends.  Host code never passes the array's name to a kernel or a copy
// (on the host it is only a stand-in for the symbol): it looks up each device's
// own address once, with that device current, and uses that address.
namespace {

static __device__ __align__(256) uint8_t scratch[GG_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices] = {};

gg_status scratch_of(int device, uint8_t **out)
{
    if (device < 0 || device >= kMaxDevices) return GG_EDEVICE;
    std::lock_guard<std::mutex> g(scratch_mu);
    if (!scratch_ptr[device]) {
        void *p = nullptr;
        if (hipSetDevice(device) != hipSuccess ||
            hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return GG_EDEVICE;
        }
        scratch_ptr[device] = p;
    }
    *out = static_cast<uint8_t *>(scratch_ptr[device]);
    return GG_OK;
}

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

gg_status gg_traceback_noalloc(const gg_index *ix, const char *query, int64_t qlen,
                               const gg_params *params, const gg_hit *hits, int32_t n, char *ops,
                               int64_t ops_cap, int64_t *ops_off, int32_t *ops_len)
{
    if (!ix || qlen < 0 || qlen > INT32_MAX || (qlen > 0 && !query) || n < 0 ||
        (n > 0 && (!hits || !ops_off || !ops_len)))
        return GG_EINVAL;
    TRY(check_params(params));
    ops_off[0] = 0;
    int64_t rows = 0;
    for (int32_t h = 0; h < n; ++h) {
        const gg_hit &x = hits[h];
        if (x.seq_id < 0 || x.seq_id >= ix->n_seqs || x.q_start < 0 || x.q_end <= x.q_start ||
            x.q_end > qlen || x.d_start < 0 || x.d_end <= x.d_start || x.score <= 0)
            return GG_EINVAL;
        const int64_t R = x.q_end - x.q_start, C = x.d_end - x.d_start;
        ops_off[h + 1] = ops_off[h] + R + C;
        rows += R;
    }
    if (n == 0) return GG_OK;
    if (ops_cap < ops_off[n] || !ops) return GG_ETRUNC;
    // scratch layout: hits | query | direction offsets | operation offsets |
    // lengths | statuses | operations | direction rows
    const size_t o_hits = 0;
    const size_t o_q = o_hits + up256(sizeof(gg_hit) * (size_t)n);
    const size_t o_doff = o_q + up256((size_t)qlen);
    const size_t o_ooff = o_doff + up256(sizeof(int64_t) * ((size_t)n + 1));
    const size_t o_len = o_ooff + up256(sizeof(int64_t) * ((size_t)n + 1));
    const size_t o_st = o_len + up256(sizeof(int32_t) * (size_t)n);
    const size_t o_ops = o_st + up256(sizeof(int32_t) * (size_t)n);
    const size_t o_dir = o_ops + up256((size_t)ops_off[n]);
    const size_t need = o_dir + 64 * (size_t)rows;
    if (need > (size_t)GG_NOALLOC_SCRATCH_BYTES) return GG_ESCRATCH;
    uint8_t *sp = nullptr;
    TRY(scratch_of(ix->device, &sp));
    if (hipSetDevice(ix->device) != hipSuccess) return GG_EDEVICE;
    // every scratch byte a kernel reads is written earlier in this call, so what a
    // previous call left there does not matter
    hipStream_t st = nullptr;
    HIPCHK(hipMemcpy(sp + o_hits, hits, sizeof(gg_hit) * (size_t)n, hipMemcpyHostToDevice));
    if (qlen > 0) HIPCHK(hipMemcpy(sp + o_q, query, (size_t)qlen, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(sp + o_ooff, ops_off, sizeof(int64_t) * ((size_t)n + 1),
                     hipMemcpyHostToDevice));
    int32_t *d_len = reinterpret_cast<int32_t *>(sp + o_len);
    launch_dir_offsets(reinterpret_cast<const int32_t *>(sp + o_hits), n,
                       reinterpret_cast<int64_t *>(sp + o_doff), st);
    launch_traceback(reinterpret_cast<const int32_t *>(sp + o_hits), n, sp + o_q, qlen, ix->d_dbw,
                     ix->d_seq_start, (int32_t)ix->n_seqs, params->match, params->mismatch,
                     params->gap_open, params->gap_extend, params->band,
                     reinterpret_cast<const int64_t *>(sp + o_doff), sp + o_dir,
                     reinterpret_cast<const int64_t *>(sp + o_ooff),
                     reinterpret_cast<char *>(sp + o_ops), d_len,
                     reinterpret_cast<int32_t *>(sp + o_st), st);
    launch_fold_status(d_len, reinterpret_cast<const int32_t *>(sp + o_st), n, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpy(ops, sp + o_ops, (size_t)ops_off[n], hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(ops_len, d_len, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost));
    // each path was written right-aligned in its slot; move it to the slot's start
    bool all_ok = true;
    for (int32_t h = 0; h < n; ++h) {
        if (ops_len[h] < 0) {
            ops_len[h] = 0;
            all_ok = false;
        }
        const int64_t slot = ops_off[h + 1] - ops_off[h];
        memmove(ops + ops_off[h], ops + ops_off[h] + slot - ops_len[h], (size_t)ops_len[h]);
    }
    return all_ok ? GG_OK : GG_EINVAL;
}

gg_status gg_profile_enable(gg_index *ix, int32_t on)
{
    if (!ix) return GG_EINVAL;
    std::lock_guard<std::mutex> g(ix->prof_mu);
    ix->prof.clear();
    ix->prof_on = on ? 1 : 0;
    return GG_OK;
}

gg_status gg_profile_read(const gg_index *ix, const char *stage, double *ms, int64_t *launches,
                          int64_t *units)
{
    if (!ix || !stage) return GG_EINVAL;
    std::lock_guard<std::mutex> g(ix->prof_mu);
    auto it = ix->prof.find(stage);
    StageTime t;
    if (it != ix->prof.end()) t = it->second;
    if (ms) *ms = t.ms;
    if (launches) *launches = t.launches;
    if (units) *units = t.units;
    return GG_OK;
}

}  // extern "C"
