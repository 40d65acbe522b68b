// Internal declarations shared by the GPU library's own sources (kernels and
// host runtime).  Nothing here is part of the public ABI in include/gg.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gg {

constexpr int32_t kNegInf = -(1 << 30);  // minus infinity of the alignment DP
constexpr int kBlock = 256;              // threads per block for the stream kernels
constexpr int kItems = 8;                // hits per thread in the gather and chain passes
constexpr int kTile = kBlock * kItems;   // hits per gather / chain tile
constexpr int kSortItems = 8;            // keys per thread in the radix passes
constexpr int kSortTile = kBlock * kSortItems;  // keys per radix tile
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kGatherCap = 4096;         // positions of one gather tile kept in LDS
constexpr int kMaxBand = 63;             // band half-width supported by one wave
constexpr int kSegCap = 1024;            // records of one query sorted in LDS
constexpr int kBswStage = 4096;          // box bases staged in LDS by the aligner
constexpr int kBinCap = 1024;            // buckets one gather tile counts in LDS
constexpr uint32_t kBucketCapMax = 512;  // most keys of one bucket (one wave sorts it in LDS)
constexpr uint32_t kBucketBig = 16384;   // most keys of one bucket sorted by a block (128 KiB)
constexpr int kMaxProbe = 4;             // neighbour windows probed per side (G / k + 1)
constexpr int kBoundCap = 2048;          // run bounds of one query paired in LDS
constexpr int kLenBins = 1024;           // box-length bins of the selection prefilter
// Blocks of a grid-stride launch: a dispatch counts its work-items in 32 bits, so
// kernels with a wave or block per record loop over records beyond this grid.
constexpr uint32_t kMaxGrid = 1u << 20;
constexpr uint32_t kStrideGrid = 2048;  // blocks of a graph's grid-stride kernels

// First or last hit of a run of several hits: query (local), sequence, diagonal, qpos.
struct Bound {
    int32_t q, s, d, qpos;
};

// A chained run of hits: query (local to the wave), sequence, diagonal, [qs, qe).
struct Cand {
    int32_t q, s, d, qs, qe;
};

// An HSP box: query-local index, sequence, query and data-bank intervals and the
// extreme diagonals of the runs merged into it.  q < 0 marks an empty slot.
struct Box {
    int32_t q, s, qs, qe, ds, de, dmin, dmax;
};

// One alignment; same layout as gg_hit, plus the query-local index in front.
struct Align {
    int32_t q;
    int32_t seq_id, score, q_start, q_end, d_start, d_end;
    int32_t box_q_start, box_q_end, box_d_start, box_d_end, box_len;
    int32_t band_d0;
};
constexpr int kAlignInts = 13;  // int32 fields of an Align
constexpr int kHitInts = 12;    // int32 fields of a gg_hit (an Align without q)

// Bit layout of the 64-bit hit key: [q | s | diag + bias | qpos], most
// significant first.  Sorting the keys orders hits by (q, s, diag, qpos).
struct HitKeyLayout {
    int bq, bs, bd, bp;  // field widths
    int32_t bias;        // added to the diagonal so that it is >= 0
};

// One wave of a graph-replayed batch, in device memory.  The host plans the waves
// (qa .. bq, and the hit-key layout); k_wave_begin copies the next plan entry
// here, and the kernels that produce the run and selection counts store them.
// Kernels given a WaveCtl read their sizes from it instead of their arguments,
// so one captured graph serves every wave.
struct WaveCtl {
    int32_t qa, nqw;  // first query of the wave, queries in it
    int64_t g0, np;   // first base of the wave in the batch, bases
    uint32_t H;       // hits
    uint32_t nc;      // runs kept (written on the device)
    HitKeyLayout lay;
    uint32_t tile0, ntile;  // the wave's radix tiles in the batch's tile table
    // per query of the batch: set to 1 when the query's kept hits, runs or
    // selections outgrew a per-query LDS sort; the wave's other queries go on, and
    // the host runs the flagged ones again
    uint32_t *qflag;
};

// A radix tile of a sort done within query segments: keys [start, start + count)
// all belong to one query, whose nt tiles (this is its tq-th) keep their digit
// counts at hist[hbase + digit * nt + tq], after all earlier queries' counts.  One
// exclusive scan over such counts then places every key inside its query's own
// range, so the passes need not sort on the query bits.
struct SortTile {
    uint32_t start, count, hbase, nt, tq;
};

// Which box field feeds a sort-key field.
enum BoxField : int32_t {
    F_Q = 0, F_S, F_QS, F_QE, F_DS, F_DE, F_LEN_DESC
};
enum AlignField : int32_t {
    A_Q = 0, A_SCORE_DESC, A_SEQ, A_QS, A_QE, A_DS, A_DE, A_BQS, A_BQE, A_BDS, A_BDE,
    A_D0  // band centre plus the bias held in desc_max
};

// Up to 8 fields packed into one 64-bit key word.
struct KeyWord {
    int32_t n;
    int32_t field[8];
    int32_t shift[8];
    int32_t bits;        // width of the whole word
    int32_t desc_max[8]; // for *_DESC fields: value stored is desc_max - v
};

// ---------------------------------------------------------------- launchers
// Every launcher only enqueues work on `st`; sizes are checked by the caller.

void launch_encode_kmers(const uint8_t *ascii, const int64_t *qoff, int32_t nq, int64_t T,
                         int32_t span, uint32_t mask, const uint32_t *list_off, uint8_t *qcode,
                         uint32_t *kcode, uint32_t *cnt, uint32_t *lhead, int32_t *qid,
                         int32_t *err, int32_t *bq, hipStream_t st);
// out[i] = sum of in[0..i) for i in [0, n]; in is u32, out u64.
void launch_scan_u32_to_u64(const uint32_t *in, uint64_t *out, int64_t n, uint64_t *partials,
                            hipStream_t st);
// in-place style exclusive scan of u32 (out may equal in), n + 1 outputs.
void launch_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *partials,
                     hipStream_t st);
size_t scan_partials_needed(int64_t n);
void launch_query_totals(const uint64_t *hoff, const int64_t *qoff, int32_t nq, uint64_t *qtot,
                         hipStream_t st);
void launch_wave_prep(const uint64_t *hoff, const int64_t *qoff, const uint32_t *lhead,
                      const int32_t *qid, int32_t qa, int64_t g0, int64_t g1, HitKeyLayout lay,
                      uint32_t *hrel, uint32_t *pbase, uint64_t *akey, uint32_t *tile_pos,
                      hipStream_t st);
// Index build (Sections 2, 2.1): pack the bank 2 bits per base; code every
// non-overlapping window (keys = code, vals = window number, counts per code);
// after a stable sort by code, window numbers become (sequence, position) postings.
void launch_pack_bases(const uint8_t *ascii, int64_t total, uint32_t *dbw, int64_t nwords,
                       int32_t *err, hipStream_t st);
void launch_window_keys(const uint32_t *dbw, const int64_t *seq_start, const uint32_t *woff,
                        int32_t n_seqs, uint32_t n_win, int32_t span, uint32_t mask,
                        uint64_t *keys, uint32_t *vals, uint32_t *counts, hipStream_t st);
void launch_postings(const uint32_t *vals, uint32_t n_win, const uint32_t *woff, int32_t n_seqs,
                     int32_t span, int2 *post, hipStream_t st);
// Traceback of n reported alignments (gg_hit records, kHitInts int32 each) of one
// query (ASCII): per-hit direction rows of 64 bytes at dirs + dir_off[h], the
// operations right-aligned in ops[ops_off[h] .. ops_off[h] + (q span + d span)),
// their count in ops_len[h] and status[h] (0 ok, 1 not an alignment).
void launch_traceback(const int32_t *hits, int32_t n, const uint8_t *qascii, int64_t qlen,
                      const uint32_t *dbw, const int64_t *seq_start, int32_t n_seqs, int32_t match,
                      int32_t mismatch, int32_t gap_open, int32_t gap_extend, int32_t band,
                      const int64_t *dir_off, uint8_t *dirs, const int64_t *ops_off, char *ops,
                      int32_t *ops_len, int32_t *status, hipStream_t st);
// Selection prefilter over n box slots in query order.  Each slot has a length
// record binq[i] = (q << 10) | length bin (kNoBin: empty slot), written where the
// boxes are merged (LenSel) or by launch_len_records[_ranges] over the slots.
// From the records alone the prefilter takes the per-query length histograms
// (hist: nq * kLenBins, cleared here), the threshold bin thr[q] and box count
// nvalid[q], and per-tile kept counts scanned in place (kept total at
// tile_counts[tiles]); launch_len_compact then writes the kept boxes, in order, to
// out.
constexpr uint32_t kNoBin = 0xFFFFFFFFu;
struct LenSel {
    uint32_t *binq = nullptr;  // per-slot records (nullptr: no prefilter)
    int shift = 0;             // length >> shift is the bin (clamped to kLenBins - 1)
};
void launch_len_records(const Box *b, uint32_t n, LenSel ls, hipStream_t st);
void launch_len_records_ranges(const Box *b, const uint32_t *ranges, uint32_t nr, LenSel ls,
                               hipStream_t st);
void launch_len_prefilter(const uint32_t *binq, uint32_t n, int32_t nq, int32_t N, uint32_t *hist,
                          uint32_t *thr, uint32_t *nvalid, uint32_t *tile_counts,
                          uint32_t *partials, hipStream_t st);
void launch_len_compact(const Box *b, const uint32_t *binq, uint32_t n, const uint32_t *thr,
                        const uint32_t *tile_off, Box *out, hipStream_t st);
// Both strands: dst holds each sequence's reverse complement at the sequence's own
// start (start: n_seqs + 1 forward starts).
void launch_reverse_strand(const uint8_t *src, const int64_t *start, int32_t n_seqs, uint8_t *dst,
                           hipStream_t st);
// Repeat cutoff: kept list lengths (0 for a list longer than max_posting), and the
// postings of kept lists placed at their kept heads.
void launch_cut_counts(const uint32_t *off, uint32_t ncode, uint32_t max_posting, uint32_t *kept,
                       hipStream_t st);
void launch_postings_cut(const uint32_t *vals, const uint64_t *keys, uint32_t n_win,
                         const uint32_t *woff, int32_t n_seqs, int32_t span, const uint32_t *off,
                         const uint32_t *kept_off, uint32_t max_posting, int2 *post, hipStream_t st);
// A query searched by pieces over ranges of sequence ids: below[y] += its hits on
// sequences < bounds[y]; per-position sub-lists of the range [s_lo, s_hi).
void launch_range_counts(const uint32_t *kcode, const uint32_t *cnt, int64_t np,
                         const uint32_t *list_off, const int2 *post, const int32_t *bounds,
                         int32_t nbounds, unsigned long long *below, hipStream_t st);
void launch_piece_prep(const uint32_t *kcode, const uint32_t *cnt, int64_t np,
                       const uint32_t *list_off, const int2 *post, int32_t s_lo, int32_t s_hi,
                       HitKeyLayout lay, uint32_t *pcnt, uint32_t *pbase, uint64_t *akey,
                       hipStream_t st);
void launch_gather(const uint32_t *hrel, const uint32_t *pbase, const uint64_t *akey,
                   int64_t npos, const int2 *post, uint32_t nhits, HitKeyLayout lay,
                   uint64_t *keys, const uint32_t *tile_pos, hipStream_t st);
// Runs found by probing the windows next to every hit (no stored hit): single-hit
// runs and the bounds of longer runs; bounds are grouped by query, then sorted
// and paired per query.  Runs in any order are finally grouped by query.
void launch_probe(const uint32_t *hrel, const uint32_t *pbase, int64_t np, const int2 *post,
                  uint32_t nhits, int64_t g0, const int32_t *qid, const int64_t *qoff, int32_t qa,
                  const uint32_t *kcode, const uint32_t *kcnt, const uint32_t *dbw,
                  const int64_t *seq_start, int32_t k,
                  uint32_t mask, int32_t max_gap, int32_t min_len, Cand *cands, uint32_t ccap,
                  uint32_t *ccount, uint32_t *cand_per_q, Bound *bounds, uint32_t bcap,
                  uint32_t *bcount, uint32_t *bound_per_q, hipStream_t st);
void launch_bounds_by_query(const Bound *in, uint32_t n, const uint32_t *qoff_b, uint32_t *cur,
                            Bound *out, hipStream_t st);
void launch_pair_bounds(const Bound *b, const uint32_t *qoff_b, int32_t nq, int32_t k,
                        int32_t min_len, Cand *cands, uint32_t ccap, uint32_t *ccount,
                        uint32_t *cand_per_q, hipStream_t st);
void launch_group_by_query(const Cand *in, uint32_t n, const uint32_t *qoff_c, uint32_t *cur,
                           Cand *out, hipStream_t st);
// Bucketed grouping (mode 1: count hits per bucket, mode 2: write keys into
// buckets), then one block per bucket sorts and chains it in LDS.
void launch_gather_bucket(int mode, const uint32_t *hrel, const uint32_t *pbase,
                          const uint64_t *akey, int64_t npos, const int2 *post, uint32_t nhits,
                          HitKeyLayout lay, const uint32_t *bb, const uint32_t *nbq,
                          uint32_t *bcount, const uint32_t *boff, uint64_t *keys, hipStream_t st);
void launch_bucket_sort_chain(const uint64_t *keys, const uint32_t *boff, uint32_t nbk,
                              uint32_t max_bucket, HitKeyLayout lay, int32_t k, int32_t max_gap,
                              int32_t min_len, Cand *tmp, uint32_t cap, uint32_t *cursor,
                              uint32_t *btmp, uint32_t *bcands, uint32_t *cand_per_q,
                              hipStream_t st);
void launch_bucket_sort_chain_big(const uint64_t *keys, const uint32_t *boff,
                                  const uint32_t *list, uint32_t nlist, uint32_t max_bucket,
                                  HitKeyLayout lay, int32_t k, int32_t max_gap, int32_t min_len,
                                  Cand *tmp, uint32_t cap, uint32_t *cursor, uint32_t *btmp,
                                  uint32_t *bcands, uint32_t *cand_per_q, hipStream_t st);
// One-time per-process kernel attributes (dynamic LDS above 64 KiB).
hipError_t setup_kernels();
void launch_compact_cands(const Cand *tmp, const uint32_t *btmp, const uint32_t *bcands,
                          const uint32_t *coff, uint32_t nbk, Cand *out, hipStream_t st);
// Stable LSD radix sort of n keys (and optional u32 values) on bits [lo, hi).
// Returns which buffer holds the result: 0 = keys/vals, 1 = keys_alt/vals_alt.
int radix_sort(uint64_t *keys, uint64_t *keys_alt, uint32_t *vals, uint32_t *vals_alt,
               uint32_t n, int lo, int hi, uint32_t *hist, uint32_t *partials, hipStream_t st);
size_t radix_hist_needed(uint32_t n);
// One-sweep LSD sort of keys on bits [lo, hi), 8-bit digits: onesweep_prepare
// counts the digits of every pass in one read, then onesweep_pass(p) scatters
// pass p with look-back tile offsets (ping-pong buffers, like the passes above).
// scratch holds onesweep_scratch_bytes(n); the failure flag (device u32) is
// non-zero if a look-back wait ran out, and the result must then be discarded.
size_t onesweep_scratch_bytes(uint32_t n);
void onesweep_prepare(const uint64_t *keys, uint32_t n, int lo, int hi, void *scratch,
                      hipStream_t st);
void onesweep_pass(const uint64_t *kin, uint64_t *kout, uint32_t n, int lo, int pass,
                   void *scratch, hipStream_t st);
const uint32_t *onesweep_fail_flag(const void *scratch);
void launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t st);
// Read `bytes` (a multiple of 16) once and add their 32-bit words into *sum
// (memory-counter calibration).
void launch_stream_read(const void *src, size_t bytes, unsigned long long *sum, hipStream_t st);
void launch_fill2_u32(uint32_t *a, size_t na, uint32_t *b, size_t nb, uint32_t v, hipStream_t st);

// ---- graph-replayed waves: the kernels below read the wave's sizes from ctl;
// grids are sized for the largest wave of the batch (hits_cap, np_cap, nq_cap).
// The first node takes the wave's plan entry plan[*cursor] into ctl; the last
// advances the cursor.
void launch_wave_end(uint32_t *cursor, hipStream_t st);
void launch_wave_prep_ctl(const uint64_t *hoff, const int64_t *qoff, const uint32_t *lhead,
                          const int32_t *qid, int64_t np_cap, uint32_t *hrel, uint32_t *pbase,
                          uint64_t *akey, const WaveCtl *plan, const uint32_t *cursor,
                          WaveCtl *ctl, uint32_t *tile_pos, hipStream_t st);
void launch_gather_ctl(const uint32_t *hrel, const uint32_t *pbase, const uint64_t *akey,
                       const int2 *post, uint32_t hits_cap, uint64_t *keys, const WaveCtl *ctl,
                       const uint32_t *tile_pos, hipStream_t st);
// Per-query filter of hits alone on their (s, diag) group and LDS sort of the
// kept keys, in place (kept counts per query in kept[]; queries too large for the
// LDS sort set *flag, or, in a replayed wave, whose grid covers nq_cap queries,
// their ctl->qflag entry, and keep no hit).  The order array, when given, names the wave-local query that
// block r filters (largest first): order[qa + r] for a replayed wave (one array for
// the batch), order[r] otherwise.  Then the kept keys' compaction in query order into
// `out` (koff[] = exclusive scan of kept[]; a replayed wave's ctl->H becomes the
// total).
void launch_hit_filter(uint64_t *keys, const uint32_t *hrel, const int64_t *qoff, int32_t qa,
                       int64_t g0, int32_t nqw, int bp, const int32_t *order, uint32_t *kept,
                       uint32_t *flag, hipStream_t st, WaveCtl *ctl = nullptr,
                       int32_t nq_cap = 0);
// The gather and the filter's first round in one kernel (no per-hit key stored):
// one block per query reads its postings twice, to mark the (s, diag) slots and
// to write the kept keys at the query's place in `keys`; then the same further
// rounds, LDS sort and flags as launch_hit_filter.
void launch_gather_filter(const uint32_t *hrel, const uint32_t *pbase, const int2 *post, const int64_t *qoff, int32_t qa, int64_t g0,
                          int32_t nqw, HitKeyLayout lay, const int32_t *order, uint64_t *keys,
                          uint32_t *kept, uint32_t *flag, hipStream_t st, WaveCtl *ctl = nullptr,
                          int32_t nq_cap = 0);
void launch_hit_compact(const uint64_t *keys, const uint32_t *hrel, const int64_t *qoff,
                        int32_t qa, int64_t g0, int32_t nqw, const uint32_t *kept, uint32_t *koff,
                        uint32_t *partials, uint64_t *out, hipStream_t st, WaveCtl *ctl = nullptr,
                        int32_t nq_cap = 0);
void launch_rs_pass_ctl(const uint64_t *kin, uint64_t *kout, uint32_t ntile_cap, int pass,
                        const SortTile *tiles, uint32_t *hist, uint32_t *partials,
                        const WaveCtl *ctl, hipStream_t st);
// One pass within query segments (tiles from the host's table, ntile of them):
// counts, scan, scatter.
void launch_rs_hist_seg(const uint64_t *kin, uint32_t ntile, int shift, const SortTile *tiles,
                        uint32_t *hist, hipStream_t st);
void launch_rs_scan_seg(uint32_t *hist, uint32_t ntile, uint32_t *partials, hipStream_t st);
void launch_rs_scatter_seg(const uint64_t *kin, uint64_t *kout, uint32_t ntile, int shift,
                           const SortTile *tiles, const uint32_t *hist, hipStream_t st);
void launch_chain_ctl(const uint64_t *keys, uint32_t hits_cap, int32_t k, int32_t max_gap,
                      int32_t min_len, uint32_t *counts, uint32_t *partials, Cand *out,
                      WaveCtl *ctl, hipStream_t st, bool few = false);
// The three kernels of one radix pass (digit histogram, its scan, stable scatter).
void launch_rs_hist(const uint64_t *keys, uint32_t n, int shift, uint32_t *hist, hipStream_t st);
void launch_rs_scan(uint32_t *hist, uint32_t n, uint32_t *partials, hipStream_t st);
void launch_rs_scatter(const uint64_t *kin, const uint32_t *vin, uint64_t *kout, uint32_t *vout,
                       uint32_t n, int shift, const uint32_t *hist, hipStream_t st);
// Runs in hit-key order: per-tile counts, then (after a scan of them) the writes.
uint32_t chain_tiles(uint32_t n);
void launch_chain_count(const uint64_t *keys, uint32_t n, HitKeyLayout lay, int32_t k,
                        int32_t max_gap, int32_t min_len, uint32_t *counts, hipStream_t st);
void launch_chain_write(const uint64_t *keys, uint32_t n, HitKeyLayout lay, int32_t k,
                        int32_t max_gap, int32_t min_len, const uint32_t *tile_off, Cand *out,
                        hipStream_t st);
// Each query's range of runs [qstart[q], qend[q]) in n runs in query order, q < nq.
void launch_cand_segments(const Cand *c, uint32_t n, int32_t nq, uint32_t *qstart, uint32_t *qend,
                          hipStream_t st);
// Per-query LDS sorts (segments of at most kSegCap records; longer ones are skipped).
// mode 0: merge order, mode 1: selection order.
void launch_seg_sort_box(int mode, const Box *in, Box *out, const uint32_t *seg_off, int32_t nq,
                         hipStream_t st);
void launch_report_seg(const Align *in, Align *out, const uint32_t *sel_off, int32_t nq,
                       uint32_t *rstart, uint32_t *rend, int32_t qa, int32_t cap, int32_t *dev_out,
                       int32_t *dev_n, hipStream_t st, WaveCtl *ctl = nullptr);
// queue_mem: extend_queue_bytes(n) bytes of device scratch.
size_t extend_queue_bytes(uint32_t n);
void launch_extend(const Cand *c, uint32_t n, const uint8_t *qcode, const uint32_t *qpack,
                   const int64_t *qoff, int32_t qa, const uint32_t *dbw, const int64_t *seq_start,
                   int32_t match, int32_t mismatch, int32_t xdrop, Box *out, void *queue_mem,
                   int32_t lane_steps, hipStream_t st, const WaveCtl *ctl = nullptr,
                   uint32_t n_cap = 0, bool count_cleared = false);
// The batch's T query codes packed 16 bases to a word ((T + 15) / 16 + 2 words).
void launch_pack_query(const uint8_t *qcode, int64_t T, uint32_t *qpack, hipStream_t st);
void launch_box_keys(const Box *b, uint32_t n, KeyWord w, int32_t q_invalid, uint64_t *out,
                     const uint32_t *perm, hipStream_t st);
void launch_align_keys(const Align *a, uint32_t n, KeyWord w, int32_t q_invalid, uint64_t *out,
                       const uint32_t *perm, hipStream_t st);
void launch_iota(uint32_t *v, uint32_t n, hipStream_t st);
void launch_gather_boxes(const Box *in, const uint32_t *perm, uint32_t n, Box *out,
                         hipStream_t st);
void launch_gather_aligns(const Align *in, const uint32_t *perm, uint32_t n, Align *out,
                          hipStream_t st);
// A replayed wave's merge (sort, sweep) and selection sort of each query's boxes
// in one launch (in -> out, per-query segments seg_off; a query over the LDS sort
// sets its ctl->qflag entry and is skipped).
void launch_merge_select_seg(const Box *in, Box *out, const uint32_t *seg_off, int32_t nq_cap,
                             WaveCtl *ctl, hipStream_t st);
void launch_merge_sweep(const Box *sorted, uint32_t n, Box *out, hipStream_t st);
// The same sweep of ngroup whole groups, boxes [offs[g], offs[g + 1]) of sorted,
// one block per group sweeping in parallel for at most `rounds` rounds per chunk
// of boxes, else one thread (groups too big for a merge window).
void launch_merge_groups(const Box *sorted, const uint32_t *offs, uint32_t ngroup, Box *out,
                         int rounds, hipStream_t st);
// Merge (order and sweep) of boxes grouped by (query, sequence), fresh from the
// extension, in windows of whole groups held in LDS; keys (group rank | qs |
// d + bias | qe) take 12 + 2 bl + bd <= 64 bits.  Groups that may outgrow a
// window are listed in big: big[0] = count, then (first, end) pairs, at most
// big_cap of them; their positions in `out` are left for the global sort.  A
// window's sweep runs in parallel over its boxes for at most `rounds` rounds of
// segmented scans; a window that has not settled by then (every window when
// rounds = 0) is swept group by group, one thread per group.  With ls.binq the
// owned groups' slots get their length records.
constexpr int kMergeRounds = 12;
void launch_merge_tiles(const Box *in, uint32_t n, int bl, int bd, int32_t bias, Box *out,
                        uint32_t *big, uint32_t big_cap, int rounds, LenSel ls, hipStream_t st);
// Boxes of ranges [ranges[2r], ranges[2r + 1]) to (to_packed) or from a packed
// array starting at offs[r].
void launch_copy_ranges(const Box *src, Box *dst, const uint32_t *ranges, const uint32_t *offs,
                        uint32_t nr, bool to_packed, hipStream_t st);
void launch_segments_box(const Box *sorted, uint32_t n, int32_t nq, uint32_t *qstart,
                         uint32_t *qend, hipStream_t st);
void launch_segments_align(const Align *sorted, uint32_t n, int32_t nq, uint32_t *qstart,
                           uint32_t *qend, hipStream_t st);
// A replayed wave's per-query run ranges, counts and offsets (off[0..nq_cap]: runs
// are in query order, so offsets are the ranges' starts), and its per-query
// selected-box ranges and counts capped at N (each query's boxes in its own
// segment, selected ones first); grids of nq_cap threads (the first also zeroes
// *clear, the extension's queue count, when given).  The _scan form also
// writes the counts' exclusive scan (sel_off[0..nq_cap]) and, for the aligner,
// the box index of every selection (sel_box[sel_off[q] + r] = qstart[q] + r),
// from one block.
void launch_cand_ranges_ctl(const Cand *c, int32_t nq_cap, uint32_t *qstart, uint32_t *qend,
                            uint32_t *counts, uint32_t *off, uint32_t *clear, const WaveCtl *ctl,
                            hipStream_t st);
void launch_box_ranges_ctl(const Box *s, const uint32_t *seg_off, int32_t nq_cap, int32_t N,
                           uint32_t *qstart, uint32_t *qend, uint32_t *counts, const WaveCtl *ctl,
                           hipStream_t st);
void launch_box_ranges_scan_ctl(const Box *s, const uint32_t *seg_off, int32_t nq_cap, int32_t N,
                                uint32_t *qstart, uint32_t *qend, uint32_t *sel_off,
                                uint32_t *sel_box, const WaveCtl *ctl, hipStream_t st);
void launch_select_counts(const uint32_t *qstart, const uint32_t *qend, int32_t nq,
                          int32_t max_hits, uint32_t *nsel, hipStream_t st);
void launch_bsw(const Box *sorted, const uint32_t *qstart, const uint32_t *sel_off, int32_t nq,
                uint32_t nsel_total, const uint8_t *qcode, const int64_t *qoff, int32_t qa,
                const uint32_t *dbw, const int64_t *seq_start, int32_t match, int32_t mismatch,
                int32_t gap_open, int32_t gap_extend, int32_t band, Align *out,
                unsigned long long *cells_per_q, unsigned long long *cells_per_box,
                hipStream_t st, const WaveCtl *ctl = nullptr, const uint32_t *sel_box = nullptr,
                uint32_t *order_buf = nullptr);
// dir_off[h] = 64 * (sum of q_end - q_start over hits before h), h in [0, n].
void launch_dir_offsets(const int32_t *hits, int32_t n, int64_t *dir_off, hipStream_t st);
// ops_len[h] = -1 where status[h] != 0.
void launch_fold_status(int32_t *ops_len, const int32_t *status, int32_t n, hipStream_t st);
// Results of queries [qa, qa + nq) as gg_hit records (11 int32) in device memory.
void launch_write_out(const Align *sorted, const uint32_t *rstart, const uint32_t *rend,
                      int32_t nq, int32_t qa, int32_t cap, int32_t *out, int32_t *n_out,
                      hipStream_t st);

}  // namespace gg
