/*
 * gg.h -- C ABI of the MI355X (gfx950) indexed similar-DNA-sequence search.
 *
 * The method is Genoogle's (F. F. Albrecht, arXiv 1507.02987): an inverted index
 * of a data bank's non-overlapping k-base windows (Sections 2 and 2.1) is probed
 * with every overlapping window of a query; index hits are grouped, chained into
 * HSPs, extended, merged, selected by length, aligned with a banded
 * Smith-Waterman and reported by score (Section 2.2, seven phases).
 *
 * Every stage of a search runs as a HIP kernel on the GPU.  All integers are
 * little-endian; coordinates are 0-based and intervals half-open.  The library
 * allocates its own device memory and streams; no torch type appears here.
 *
 * Ownership: the caller owns every input and output buffer and may reuse it as
 * soon as a call returns (inputs are copied before return).  Handles are owned by
 * the library until the matching _free/_destroy call.
 *
 * Thread safety: a gg_index is read-only after build and may be shared by any
 * number of threads; concurrent gg_search / gg_search_batch calls on one index
 * each take their own stream and workspace.  A gg_server may be used from many
 * threads.
 */
#ifndef GG_H
#define GG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GG_OK = 0,
    GG_EINVAL = 1,    /* bad argument, byte outside {A,C,G,T,U} (either case), k outside 1..16 */
    GG_ENOMEM = 2,    /* host or device allocation failed */
    GG_EDEVICE = 3,   /* a HIP call failed, or no usable GPU */
    GG_EAGAIN = 4,    /* served query not finished yet */
    GG_ETRUNC = 5,    /* more hits than `cap`: the first `cap` are written, *n_out is the count */
    GG_ENOTFOUND = 6, /* unknown or already collected ticket */
    GG_EBUDGET = 7,   /* one query's hits on one sequence do not fit the hit budget */
    GG_EIO = 8,       /* an index file cannot be opened, read or written, or is not one */
    GG_ESCRATCH = 9   /* the call needs more device scratch than gg_traceback_noalloc holds */
} gg_status;

typedef struct gg_index gg_index;   /* device-resident data bank and inverted index */
typedef struct gg_server gg_server; /* continuous-batching request loop */

/*
 * Run-time parameters (Section 2, last paragraph: the maximum distance between
 * index entries of one HSP, the minimum HSP size and the extension drop-off;
 * Section 2.2 phase 5: the maximum number of alignments).  Penalties are positive
 * numbers that are subtracted.  A gap of length g costs gap_open + g * gap_extend.
 */
typedef struct {
    int32_t match;       /* +1 in the paper's workloads */
    int32_t mismatch;    /* 3 */
    int32_t gap_open;    /* 5 */
    int32_t gap_extend;  /* 2 */
    int32_t band;        /* W: half-width of the Smith-Waterman band, 0..63 (32) */
    int32_t xdrop;       /* X: extension stops when the running sum is > X below its best (20) */
    int32_t max_gap;     /* G: hits chain when qpos_next - (qpos_last + k) <= G (22) */
    int32_t min_hsp_len; /* M: a chained run [qs, qe) is kept when qe - qs >= M (22) */
    int32_t max_hits;    /* N: HSPs kept by length before alignment; <= 0 keeps all */
} gg_params;

/* One reported alignment (Section 2.2 phase 7): its score, its span in the query
 * and in data-bank sequence seq_id, and the HSP box it was aligned in. */
typedef struct {
    int32_t seq_id, score, q_start, q_end, d_start, d_end;
    int32_t box_q_start, box_q_end, box_d_start, box_d_end, box_len;
    int32_t band_d0;  /* diagonal (d - q) the alignment band was centred on: floor of the
                         mean of the merged runs' extreme diagonals (gg_traceback uses it) */
} gg_hit;

/* Per-query work counts of one search. */
typedef struct {
    int64_t n_kmers;    /* query windows probed */
    int64_t n_hits;     /* index hits gathered */
    int64_t n_cands;    /* chained runs kept by the length filter */
    int64_t n_merged;   /* HSP boxes after extension and merging */
    int64_t n_selected; /* boxes aligned */
    int64_t n_cells;    /* banded Smith-Waterman cells computed */
    int64_t n_out;      /* alignments with score > 0 */
} gg_stats;

/*
 * Format a data bank and build its inverted index on GPU `device` (Sections 2,
 * 2.1): every base is coded in 2 bits; each sequence is cut into
 * non-overlapping windows of k bases (a shorter tail is not indexed); list c of
 * the 4^k-entry main vector holds every (sequence id, position) whose window has
 * code c, in ascending (sequence, position) order.
 *
 * seqs     : all sequences' ASCII bytes, concatenated (host memory)
 * seq_off  : n_seqs + 1 non-decreasing offsets into seqs; sequence s is
 *            seqs[seq_off[s] .. seq_off[s+1])
 * k        : window length, 1..16; 4^k list heads are kept on the device
 * device   : HIP device ordinal
 * Errors   : GG_EINVAL (bad byte, bad offsets, k, more than 2^31-1 sequences or a
 *            sequence longer than 2^31-1, more than 2^32-1 windows), GG_ENOMEM,
 *            GG_EDEVICE.  Nothing is left allocated on error.
 */
gg_status gg_index_build(const char *seqs, const int64_t *seq_off, int64_t n_seqs, int32_t k,
                         int32_t device, gg_index **out);
/*
 * The same index with a spaced-seed mask (Section 2.1): mask is a NUL-terminated
 * string of '1' (base kept) and '0' (base removed), of length m <= 32 and weight s
 * (number of '1's) 1..16.  The bank is cut into non-overlapping windows of m
 * bases, coded on their s kept bases (4^s lists); queries are read with an
 * overlapping window of m bases at every offset, coded the same way.  A hit
 * covers its window's m bases: runs, gaps (G) and lengths (M) are measured with
 * m.  A mask of k '1's gives exactly gg_index_build(k).  Errors as
 * gg_index_build, and GG_EINVAL for a malformed mask.
 */
gg_status gg_index_build_masked(const char *seqs, const int64_t *seq_off, int64_t n_seqs,
                                const char *mask, int32_t device, gg_index **out);
/*
 * The general builder: a k-base window (mask NULL) or a spaced-seed mask as above,
 * and two options the paper does not have.
 *
 * strands = 2 indexes both strands of the bank: after the n given sequences, the
 * index holds the reverse complement of each, as sequence n + s (sequence s read
 * from its end, A<->T, C<->G, U pairing with A), indexed like any other.  A search
 * therefore compares the query with both strands of every sequence, in one
 * selection of the N longest boxes; a hit with seq_id >= n lies on the reverse
 * strand of sequence seq_id - n, and its d_ coordinates count on that reverse
 * complement (forward position = length - 1 - reverse position).  gg_index_info
 * then reports 2n sequences and twice the bases.  strands = 1 is the paper's
 * single-strand index.
 *
 * max_posting > 0 is a repeat cutoff: every list holding more than max_posting
 * occurrences is dropped whole (its query windows give no hits), which bounds the
 * hits that low-complexity regions create; 0 keeps every occurrence, as the paper
 * does.  Other lists are unchanged.
 *
 * Errors as gg_index_build; GG_EINVAL for strands outside {1, 2}, a negative
 * max_posting, a malformed mask, or 2n above 2^31 - 1 sequences.
 */
typedef struct {
    int32_t k;            /* window length 1..16, used when mask is NULL */
    const char *mask;     /* spaced-seed mask ('1' kept, '0' removed), or NULL */
    int32_t strands;      /* 1 or 2 */
    int64_t max_posting;  /* > 0: drop lists longer than this; 0: keep all */
} gg_index_options;
gg_status gg_index_build_ex(const char *seqs, const int64_t *seq_off, int64_t n_seqs,
                            const gg_index_options *opt, int32_t device, gg_index **out);
void gg_index_free(gg_index *index);

/*
 * Copy a built index to host memory (Section 2.1's main vector and lists):
 * list_off receives the 4^k + 1 list heads (list c holds postings
 * [list_off[c], list_off[c + 1])), postings the n_postings (sequence id, position)
 * pairs as 2 x int32 each, lists in code order and each list in (sequence,
 * position) order.  Either pointer may be NULL to skip it.  The caller owns both
 * buffers; cap_postings is the pairs postings can hold: GG_ETRUNC (nothing
 * copied) when it is below n_postings.  GG_EDEVICE on a copy failure.
 */
gg_status gg_index_export(const gg_index *index, uint32_t *list_off, int32_t *postings,
                          int64_t cap_postings);

/*
 * Persistence (Section 2.1: the index and the formatted bank are kept on disk and
 * the whole index is read into memory at start).  gg_index_save writes the index
 * and its 2-bit bank to `path` (created or replaced); gg_index_load reads such a
 * file onto `device`, where it serves exactly as the index it was saved from
 * (same lists, postings, bank, window span and mask, strands).  Tuning and the hit
 * budget are not saved.
 *
 * File layout, little-endian: "GGINDEX1"; u32 version (1); i32 k, span, strands;
 * u32 mask; u32 0; i64 n_seqs, n_bases, n_postings, max_seq_len, n_words;
 * i64 seq_start[n_seqs + 1]; u32 list_off[4^k + 1]; i32 postings[2 n_postings]
 * ((sequence, position) pairs); u32 bank[n_words] (16 bases per word, first base
 * in the top bits); u64 check, a hash of every preceding byte after the magic.
 *
 * gg_index_load checks the header, the file size, the hash, and that heads and
 * sequence starts are monotone and every posting is a whole window inside its
 * sequence, so a damaged file is refused before anything reaches the GPU.
 * Errors: GG_EIO (cannot open / read / write, wrong magic, size or hash), GG_EINVAL
 * (null argument, inconsistent contents), GG_ENOMEM, GG_EDEVICE.
 */
gg_status gg_index_save(const gg_index *index, const char *path);
gg_status gg_index_load(const char *path, int32_t device, gg_index **out);

/*
 * Report fields of Section 2.2: with each alignment the search returns its score,
 * positions, e-value, normalized score and the alignment itself.
 *
 * gg_karlin_altschul: lambda, K and H (relative entropy, nats per pair) of ungapped
 * local alignment scored +match / -mismatch on uniform, independent bases
 * (Karlin-Altschul statistics; the paper does not say how its e-values are made,
 * and gapped constants would need simulation).  GG_EINVAL for a non-positive score.
 *
 * gg_hit_significance: for n hits of one query of query_len bases searched
 * against bank_bases bases (gg_index_info's n_bases: both strands when indexed),
 * bit_score[i] = (lambda S - ln K) / ln 2 and evalue[i] = K m n exp(-lambda S),
 * S = hits[i].score, in double precision on the host.  Arrays of n, caller-owned.
 *
 * gg_traceback: the path of each of n reported hits of one query (hits as the
 * search returned them for this query, index and params).  The banded DP is
 * recomputed on the GPU over the hit's rectangle [q_start, q_end) x
 * [d_start, d_end), in the band of half-width params->band centred on band_d0,
 * and walked back from the end cell with the search's own choices (diagonal first,
 * then a gap in the query, then a gap in the bank; a gap opened rather than
 * extended on ties), so it ends exactly on (q_start, d_start).  Operations, first
 * to last, one byte each: '=' a matched pair, 'X' a mismatched pair, 'I' a query
 * base against a gap, 'D' a bank base against a gap.  Hit h's operations are
 * written at ops + ops_off[h], ops_len[h] of them; ops_off (n + 1 entries) gives
 * every hit a slot of (q_end - q_start) + (d_end - d_start) bytes and is always
 * filled first.  GG_ETRUNC (nothing else written) when ops is NULL or ops_cap <
 * ops_off[n]; GG_EINVAL for bad parameters, a hit outside the query or bank, or a
 * hit that is not an alignment of this query and bank under params (its ops_len
 * is 0; the other hits are still written).  All buffers are caller-owned host
 * memory.
 */
gg_status gg_karlin_altschul(int32_t match, int32_t mismatch, double *lambda, double *K,
                             double *H);
/*
 * gg_traceback without any device allocation, for callers that cannot allocate
 * GPU memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Arguments, outputs and errors are those of gg_traceback, and
 * so are the paths, byte for byte.  Its device scratch (the hits, the query,
 * offsets, the operations and the direction rows, 64 bytes per query row of each
 * hit) lives in one static array of GG_NOALLOC_SCRATCH_BYTES per GPU, which the
 * library holds from the first call on that GPU until the process ends; it calls
 * no hipMalloc or hipFree.  A call whose scratch would exceed the array returns
 * GG_ESCRATCH with nothing computed (use gg_traceback).  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU race and must be
 * serialised by the caller.  The transfers go through the default stream.
 */
#define GG_NOALLOC_SCRATCH_BYTES (64u << 20)
gg_status gg_traceback_noalloc(const gg_index *index, const char *query, int64_t qlen,
                               const gg_params *params, const gg_hit *hits, int32_t n, char *ops,
                               int64_t ops_cap, int64_t *ops_off, int32_t *ops_len);
gg_status gg_hit_significance(const gg_hit *hits, int64_t n, int64_t query_len, int64_t bank_bases,
                              double lambda, double K, double *bit_score, double *evalue);
gg_status gg_traceback(const gg_index *index, const char *query, int64_t qlen,
                       const gg_params *params, const gg_hit *hits, int32_t n, char *ops,
                       int64_t ops_cap, int64_t *ops_off, int32_t *ops_len);

/* Sizes of a built index: windows indexed, bases, sequences, k. */
gg_status gg_index_info(const gg_index *index, int64_t *n_postings, int64_t *n_bases,
                        int64_t *n_seqs, int32_t *k);

/*
 * Device bytes the batched search may use for index hits at once (two 8-byte
 * keys per hit).  Queries are processed in waves that fit it.  A query whose
 * hits exceed it alone is searched in pieces over ranges of data-bank sequence
 * ids (every phase up to the alignment is per sequence, so the result is the
 * same); it fails with GG_EBUDGET only if one sequence's hits exceed the budget.
 * 0 restores the default, min(16 GiB, a quarter of free device memory).
 */
gg_status gg_index_set_hit_budget(gg_index *index, uint64_t bytes);

/*
 * Launch choices of an index; none changes a result, only the time to get it.
 * grouping   : how index hits become runs (Section 2.2 phase 2):
 *              0 probe the windows next to each hit (no hit stored),
 *              1 sort hits in LDS slices of each query's sequence range,
 *              2 radix-sort all hits of a wave (the default).
 * lane_steps : X-drop steps (Section 2.2 phase 3) one lane takes before a whole
 *              wave resumes the walk; 0..4096 (0: every walk by a wave), default 256.
 * ms         : gg_index_autotune only: wall time of the sample batch with this
 *              choice (best of its runs).
 * wave_log2  : hits of one wave of a graph-replayed batch, 2^wave_log2 (10..30;
 *              0 on input: the default, 25).  Queries with more hits take the
 *              regular path after the replays.
 * graph      : 1 (default): batches without statistics, with the radix-sort grouping
 *              and 1 <= max_hits <= 1024, replay one captured graph per wave;
 *              0: they never do.
 * graph_query_log2 : queries with more than 2^graph_query_log2 index hits skip the
 *              graph and take the regular path (heavy queries mostly outgrow the
 *              graph's per-query LDS sorts); 0 (default): only the wave size limits.
 * The environment variable GG_GROUPING (probe, bucket, sort) overrides grouping.
 */
typedef struct {
    int32_t grouping;
    int32_t lane_steps;
    double ms;
    int32_t wave_log2;
    int32_t graph;
    int32_t graph_query_log2;
} gg_tuning;

gg_status gg_index_get_tuning(const gg_index *index, gg_tuning *out);
gg_status gg_index_set_tuning(gg_index *index, const gg_tuning *tuning);

/*
 * Autotuner: search the sample batch (same layout as gg_search_batch; copied once
 * to GPU memory and searched in the device-resident form) under every candidate
 * choice (3 groupings x lane steps 0, 64, 256, 4096, then, when the radix-sort
 * grouping wins, graph waves of 2^23 and 2^27 hits beside the current size, a
 * per-query graph limit of 2^14 and 2^18 hits, and no graph)
 * after one untimed run, three times each (once if the first timed run takes over
 * twice the best time so far), check that all choices return identical hits, and
 * keep the fastest on the index.
 * chosen (may be NULL) receives it.  Use queries shaped like the real workload;
 * a few hundred are enough.  Errors: those of gg_search_batch, and GG_EDEVICE if
 * two choices disagree (the previous choice is then kept).
 */
gg_status gg_index_autotune(gg_index *index, const char *queries, const int64_t *query_off,
                            int64_t n_queries, const gg_params *params, gg_tuning *chosen);

/*
 * Search one ASCII query (Section 2.2, all seven phases; forward strand only).
 * out/cap  : room for `cap` hits; *n_out receives the number found.  Hits are in
 *            descending score, then ascending (seq_id, q_start, d_start, q_end,
 *            d_end, box_q_start, box_d_start, box_q_end, box_d_end).
 * A query shorter than k has no hits (GG_OK, *n_out = 0).
 * Errors   : GG_EINVAL, GG_ETRUNC (first `cap` written), GG_EBUDGET, GG_ENOMEM,
 *            GG_EDEVICE.
 */
gg_status gg_search(const gg_index *index, const char *query, int64_t qlen,
                    const gg_params *params, gg_hit *out, int32_t cap, int32_t *n_out);

/*
 * Search n_q queries in one batched pass of the same kernels: the results are
 * those of n_q separate gg_search calls.
 * qbuf/qoff: queries' ASCII bytes concatenated, n_q + 1 non-decreasing offsets
 * out      : n_q * cap hits; query q's go to out[q * cap ..]
 * n_out    : n_q counts (each may exceed cap: then that query is truncated and the
 *            call returns GG_ETRUNC after filling every query)
 * stats    : n_q work counts, or NULL
 */
gg_status gg_search_batch(const gg_index *index, const char *qbuf, const int64_t *qoff,
                          int64_t n_q, const gg_params *params, gg_hit *out, int32_t cap,
                          int32_t *n_out, gg_stats *stats);

/*
 * Device-resident form of gg_search_batch, same results: the queries' bytes
 * already sit in GPU memory of the index's device (d_qbuf, e.g. from
 * gg_device_alloc) and the hits are written to GPU memory: d_out holds n_q * cap
 * gg_hit records (query q's at d_out + q * cap) and d_n_out n_q counts.  qoff
 * (n_q + 1 offsets into d_qbuf) and stats stay in host memory.  The call returns
 * when the results are complete in device memory.  Errors as gg_search_batch.
 */
gg_status gg_search_batch_device(const gg_index *index, const char *d_qbuf, const int64_t *qoff,
                                 int64_t n_q, const gg_params *params, gg_hit *d_out,
                                 int32_t cap, int32_t *d_n_out, gg_stats *stats);

/* Plain device-memory plumbing for the device-resident form (synchronous). */
gg_status gg_device_alloc(int32_t device, uint64_t bytes, void **ptr);
gg_status gg_device_free(int32_t device, void *ptr);
gg_status gg_memcpy_to_device(void *dst, const void *src, uint64_t bytes);
gg_status gg_memcpy_to_host(void *dst, const void *src, uint64_t bytes);
/* Device-to-device copy of `bytes` (the runtime's copy kernel); a transfer of known
 * size against which memory-traffic counters are calibrated. */
gg_status gg_device_copy(void *dst, const void *src, uint64_t bytes);
/* Read `bytes` (a multiple of 16) of device memory once with a hand-written
 * streaming kernel (coalesced 16-byte loads, one 8-byte atomic per block) and
 * return the 64-bit sum of its 32-bit words in *sum (host memory): a read of known
 * size for calibrating memory-read counters.  GG_EINVAL for a null pointer or a
 * size that is not a multiple of 16; GG_ENOMEM, GG_EDEVICE. */
gg_status gg_device_read(const void *src, uint64_t bytes, uint64_t *sum);

/*
 * Per-stage GPU timing of batched searches on this index, for roofline reports.
 * Enabling (on or off) clears the totals; when on, HIP events are recorded around
 * each stage on the stream it runs on.  Names: "encode", "scan", "gather_prep",
 * "gather" (the posting-gather kernel alone), "filter" (the kernel dropping hits
 * alone on their (sequence, diagonal) when M exceeds the seed span and sorting the
 * rest of each query), "filter_compact" (the kept hits' move into one array),
 * "sort_hist", "sort_scan", "sort_scatter" (one mark per radix pass of the hit
 * sort, when it runs), "chain" (run counts),
 * "chain_write", "extend", "merge" (ordering for the sweep), "merge_sweep",
 * "select", "align" (the banded Smith-Waterman kernel alone), "report", and
 * "graph" (all replays of a batch's captured wave graph, whose kernels are not
 * timed one by one: units = waves).  ms is the summed GPU time between the marks,
 * launches the number of marks, units the work they covered (query bases for
 * encode and scan, positions for gather_prep, hits for gather, filter and the sort
 * marks, hits left after the filter for the chain marks, runs for
 * extend/merge/select, boxes for align/report).
 *
 * Batched calls without statistics, with the radix-sort grouping and 1 <= max_hits
 * <= 1024, run each wave as a replay of one captured HIP graph (all waves after a
 * single synchronisation; the graph is kept for later calls of the same shape).
 * GG_GRAPH=0 in the environment turns this off.
 */
gg_status gg_profile_enable(gg_index *index, int32_t on);
gg_status gg_profile_read(const gg_index *index, const char *stage, double *ms,
                          int64_t *launches, int64_t *units);

/*
 * Served form (the in-process counterpart of the paper's search services,
 * Section 4): a request loop with continuous batching.  Each submitted query's
 * index hits are counted exactly on the GPU; queries are then admitted in arrival
 * order as in-flight slots and hit-buffer bytes (16 per hit) free up, and run in
 * small batches on up to four streams at once, so requests arriving while others
 * are on the GPU start as soon as room frees.  A query with more than 2^24 hits
 * runs in a batch of its own; one whose hits exceed the whole budget runs when
 * nothing else is in flight, searched in ranges of sequences.  Each query's result
 * equals its gg_search result.
 * hit_budget_bytes : device bytes for hit keys of all in-flight queries
 *                    (0: the index's hit budget)
 * max_slots        : queries in flight at once (>= 1)
 */
gg_status gg_server_create(const gg_index *index, const gg_params *params,
                           uint64_t hit_budget_bytes, int32_t max_slots, gg_server **out);
/* Queue one query (copied before return); *ticket identifies it for gg_serve_poll.
 * GG_EINVAL for a byte outside {A,C,G,T,U} (either case), with nothing queued. */
gg_status gg_serve_submit(gg_server *server, const char *query, int64_t qlen, uint64_t *ticket);
/*
 * Wait up to timeout_us (0: do not wait, < 0: wait until done) for a ticket.
 * GG_EAGAIN while it is pending; otherwise its status (GG_OK, GG_ETRUNC, ...) with
 * its hits written as for gg_search, and the ticket is released.
 */
gg_status gg_serve_poll(gg_server *server, uint64_t ticket, gg_hit *out, int32_t cap,
                        int32_t *n_out, int32_t timeout_us);
/*
 * Admission record of a server since its creation: requests submitted and
 * completed, batches started, the largest number of hit-key bytes and of requests
 * in flight at once (the bytes never exceed budget_bytes), the most requests in
 * one batch, the requests searched alone in sequence ranges because their hits
 * exceed the budget, the bytes and requests in flight now, and the submit and
 * poll calls inside the library now (a poll waiting for its ticket counts).
 */
typedef struct {
    int64_t submitted, completed, batches;
    uint64_t budget_bytes, peak_inflight_bytes, inflight_bytes;
    int64_t peak_inflight_slots, inflight_slots, peak_batch_queries, over_budget;
    int64_t calls_inside;
} gg_server_stats;
gg_status gg_server_info(gg_server *server, gg_server_stats *out);
/*
 * Stop the loop: batches on the GPU finish, queued requests are cancelled, and
 * submit or poll calls already inside the library return first (a poll waiting on
 * a cancelled ticket returns GG_ENOTFOUND).  No call may use the server once
 * destroy has begun.
 */
void gg_server_destroy(gg_server *server);

const char *gg_strerror(gg_status status);

#ifdef __cplusplus
}
#endif
#endif
