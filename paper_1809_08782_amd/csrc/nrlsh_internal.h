// Internal declarations of libnrlsh: launch wrappers implemented in the
// kernel translation units and called by the host orchestration (api.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nrlsh {

constexpr int kWave = 64;

// Entry of the list of items whose hash needs an FP64 recompute: `mask` has
// bit r set when projection r fell inside the FP32 uncertainty band.
struct FixEntry {
    uint64_t mask;
    int32_t item;
    int32_t pad;
};

// Build-side counters kept on the device (one struct per build).
struct BuildCounters {
    uint32_t nonfinite;      // items holding NaN / Inf
    uint32_t fix_count;      // entries appended to the FixEntry list
    unsigned long long fix_bits;
    unsigned long long fix_flips;
    uint32_t lowp_items;     // items appended for the FP32 re-hash (precision form)
    uint32_t fix_prev;       // entries of the FixEntry lists of earlier hash tables
    unsigned long long lowp_bits;
    unsigned long long lowp_changed;
    unsigned long long fix_flips_tiny;  // of fix_flips, those with |a . P(x)| < 1e-6 in FP64
};

// ------------------------------------------------------------------ build
// Squared norms in FP64 (ascending coordinate order); also emits (key bits,
// index) pairs for the radix sort and flags non-finite values.
hipError_t launch_keys(const float *X, int64_t n, int d, double *key, uint64_t *sort_key,
                       int32_t *sort_val, BuildCounters *ctr, hipStream_t s);

// Stable LSD radix sort of (uint64 key, int32 value) pairs on bits
// [0, nbits).  Buffers a/b are ping-pong; returns in *result_in_b whether the
// sorted data ended in the b buffers.  `tmp` must hold
// radix_sort_tmp_bytes(n) bytes.
size_t radix_sort_tmp_bytes(int64_t n);
hipError_t radix_sort(uint64_t *ka, int32_t *va, uint64_t *kb, int32_t *vb, int64_t n, int nbits,
                      void *tmp, bool *result_in_b, hipStream_t s);

// Sub-dataset of every item from its rank (s = floor(rank m / n)) or, with
// bounds (m - 1 increasing squared boundaries), from the uniform norm ranges;
// the largest key of each sub-dataset and the end rank of its run (subend;
// entries of sub-datasets without items are left as the caller set them),
// and (sid, index) pairs for the layout sort.
hipError_t launch_assign_subsets(const uint64_t *sorted_key, const int32_t *sorted_idx, int64_t n,
                                 int m, const double *bounds, int32_t *sid, uint64_t *layout_key,
                                 int32_t *layout_val, double *keymax, int32_t *subend, hipStream_t s);

// lo = bf16(x - hi) of `count` stored values (the bf16x3 screen's lo part).
hipError_t launch_lo_rows(const float *Xl, const uint16_t *Xh, int64_t count, uint16_t *Xlo,
                          hipStream_t s);

// Stored copy of the items (row p = item perm[p], zero-padded to dp) with the
// key and sub-dataset of each stored row, plus its bfloat16 image Xh and, when
// Xlo is not NULL, the lo part bf16(x - hi); xeb (or NULL) receives for each
// stored row an upper bound of ||x - bf16(x)|| + (d + 8) 2^-23 ||x||, so that
// |q.x - q.bf16(x)| (the latter summed in FP32, any order) is at most ||q|| xeb.
hipError_t launch_layout(const float *X, int64_t n, int d, int dp, const int32_t *perm,
                         const double *key, const int32_t *sid, float *Xl, uint16_t *Xh,
                         uint16_t *Xlo, double *key_l, int32_t *sid_l, float *xeb, hipStream_t s);

// SimpleLSH transform + sign random projection on the FP32 matrix cores, over
// the stored rows (all arrays in stored order); writes the codes codes_l.
// rows != NULL: re-hash only the stored positions rows[0 .. n).
hipError_t launch_hash(const float *Xl, int64_t n, int d, int dp, const float *A, int L,
                       const double *key_l, const int32_t *sid_l, const double *keymax,
                       const double *U, const float *tau, uint32_t *codes_l, FixEntry *fix,
                       BuildCounters *ctr, const int32_t *rows, hipStream_t s);

// Independent projections per sub-dataset: sub-dataset j (stored positions
// off[j] .. off[j+1]) hashes with rows j L .. j L + L - 1 of A and their band
// factors tau[j L ..]; block b of the launch serves sub-dataset j where
// bstart[j] <= b < bstart[j+1], covering hash_items_per_block() items each.
int hash_items_per_block();
hipError_t launch_hash_per_subset(const float *Xl, int d, int dp, const float *A, int L,
                                  const double *key_l, const int32_t *sid_l, const double *keymax,
                                  const double *U, const float *tau, const int32_t *off,
                                  const int32_t *bstart, int m, int nblocks, uint32_t *codes_l,
                                  FixEntry *fix, BuildCounters *ctr, hipStream_t s);

// Precision form: quantise rows to bfloat16 (storage 1) or E4M3 with row scales
// (storage 2), then hash from the quantised copy.  Bits inside the margin
// mq_r ||x|| + tq_r U_j are settled exactly: an item with at most 8 of them
// gets a FixEntry (those bits recomputed in FP64 by launch_hash_fixup, count
// in ctr->fix_count); one with more is appended to rows for the FP32 re-hash
// (count in ctr->lowp_items).  ctr->lowp_bits counts all of them.
hipError_t launch_quant_rows(const float *src, int64_t rows, int d, int ss, int storage, void *dst,
                             int ds, float *scales, hipStream_t s);
hipError_t launch_hash_q(int storage, const void *Xq, const float *xscale, int64_t n, int d, int dp,
                         const void *Aq, const float *ascale, const float *A, int L,
                         const double *key_l, const int32_t *sid_l, const double *keymax,
                         const double *U, const float *mq, const float *tq, uint32_t *codes_l,
                         int32_t *rows, FixEntry *fix, BuildCounters *ctr, hipStream_t s);

// Before the next hash table reuses the FixEntry list: fix_prev += fix_count,
// fix_count = 0 (one thread).
hipError_t launch_roll_fix_count(BuildCounters *ctr, hipStream_t s);

// FP64 recompute of the flagged projections, exactly as the definition.
// per_subset: an item of sub-dataset s takes its rows from block s of A.
hipError_t launch_hash_fixup(const float *Xl, int d, int dp, const float *A, int L, bool per_subset,
                             const double *key_l, const int32_t *sid_l, const double *keymax,
                             const double *U, const FixEntry *fix, BuildCounters *ctr,
                             uint32_t *codes_l, int64_t max_entries, hipStream_t s);

// ------------------------------------------------------------------ query
// Row of the query-code array that holds query q's code for sub-dataset j:
// one code per query with shared projections (qsets = 1), one per
// (query, sub-dataset) with a projection block per sub-dataset (qsets = m).
__host__ __device__ inline int64_t qrow(int64_t q, int j, int qsets)
{
    return qsets > 1 ? q * qsets + j : q;
}

struct QueryShape {
    int64_t n;
    int d, dp, m, L, W;
    int64_t Tq;      // probed items per query, min(T, n)
    int k;
    int qsets = 1;   // query codes per query: 1 (shared projections) or m
};

// Query codes (FP64 exact sign of A[:, :d] q); flags non-finite queries.
// With qsets > 1 (one projection block per sub-dataset, At = qsets blocks of
// d x L) query q gets qsets codes; code (q, j) sits at row q qsets + j of
// qcodes (W words per row), the row every query kernel reads for
// sub-dataset j.
hipError_t launch_query_hash(const float *Q, int64_t nq, int d, const float *At, int L, int W,
                             int qsets, uint32_t *qcodes, uint32_t *nonfinite, hipStream_t s);

// Pass 1: per query tile and sub-dataset, histogram of Hamming distance.
hipError_t launch_scan_hist(const uint32_t *codes_l, const int32_t *off, const uint32_t *qcodes,
                            int64_t nq, const QueryShape &sh, uint32_t *ghist, hipStream_t s);

// Threshold bucket, tie cut and per-sub-dataset emission bounds and offsets
// (bounds = false: gtie only; gbase and ghthr are left as they are; offsets =
// false: gbase is left as it is).
hipError_t launch_threshold(const uint32_t *ghist, const int32_t *R, const int32_t *inv, int64_t nq,
                            const QueryShape &sh, int32_t *gbase, int32_t *ghthr, int32_t *gtie,
                            hipStream_t s, bool bounds = true, bool offsets = true);

// Pass 2: emit the probed items (stored positions) of every query.
hipError_t launch_scan_emit(const uint32_t *codes_l, const int32_t *off, const uint32_t *qcodes,
                            int64_t nq, const QueryShape &sh, const int32_t *gbase,
                            const int32_t *ghthr, const int32_t *gtie, int32_t *cand,
                            hipStream_t s);

// Exact FP64 re-rank of the probed items and top-k selection.  Each query's
// probed list is cut into nsplit slices (rerank_splits); with nsplit > 1 the
// partial lists go to part_v / part_i (nq x nsplit x k) and are merged.
// With counts != NULL, query q's list holds min(counts[q], Tq) entries (stride Tq).
int rerank_splits(int64_t nq, int64_t Tq);
// gtheta (nq words, zeroed by the caller; may be NULL) lets the slices of a
// query share the best k-th value reached so far.
hipError_t launch_rerank(const float *Xl, const int32_t *perm, const float *Q, int64_t nq,
                         const QueryShape &sh, const int32_t *cand, const int32_t *counts,
                         int nsplit, double *part_v, int32_t *part_i, int64_t *out_ids,
                         float *out_ips, hipStream_t s, unsigned long long *gtheta = nullptr);

// Precision form of the re-rank: bounds from the bfloat16 copy Xh, appends to
// lists (nq x lcap, lcount set by the caller: zero, or the entries already
// there) every probed item of cand (nq x Tq; counts[q] entries, or Tq when
// counts is NULL) that may still belong to the exact top-k.  gtheta: nq
// words set by the caller (0, or the order key of a value that k probed
// items reach), the k-th lower bound shared by the slices of each query.
hipError_t launch_rerank_lp(const uint16_t *Xh, const float *xeb, const float *Q, int64_t nq,
                            const QueryShape &sh, const int32_t *cand,
                            const int32_t *counts, int nsplit, int lcap, int32_t *lcount, int32_t *lists,
                            unsigned long long *gtheta, hipStream_t s);
// gtheta[q] = the order key of theta[q] (0 where theta is -inf): seeds the
// bfloat16 re-rank with the screen's lower bound of the k-th best.
hipError_t launch_theta_seed(const float *theta, int64_t nq, unsigned long long *gtheta, hipStream_t s);

// Chunked passes for small query batches: one wave per (64-query tile,
// sub-dataset, chunk of `chunk` stored items), nch chunks per sub-dataset.
// Pass 1 adds into ghist (zeroed by the caller); pass 2 appends each query's
// probed items to its list (counts zeroed by the caller; order unspecified),
// cutting the threshold bucket at gpstar (launch_tie_locate).
hipError_t launch_scan_hist_c(const uint32_t *codes_l, const int32_t *off, const uint32_t *qcodes,
                              int64_t nq, const QueryShape &sh, int chunk, int nch, uint32_t *ghist,
                              hipStream_t s);
hipError_t launch_scan_emit_c(const uint32_t *codes_l, const int32_t *off, const uint32_t *qcodes,
                              int64_t nq, const QueryShape &sh, int chunk, int nch,
                              const int32_t *ghthr, const int32_t *gtie, const int32_t *gpstar,
                              int32_t *counts, int32_t *cand, hipStream_t s);

// Sets `words` 32-bit words at p to v (a fill kernel, capturable in a graph).
hipError_t launch_fill32(void *p, int64_t words, uint32_t v, hipStream_t s);

// Staged pass 1 (exact early exit in descending norm order): one block per
// (64-query tile, chunk) over the chunks (sub-dataset, first, end) of one
// stage, adding into ghist (zeroed by the caller); tiles with need[tile] = 0
// are skipped (need may be NULL: every tile).  launch_stage_check then clears
// need[tile] once every query of the tile has Tq items in buckets ranked
// before `cut`.  npairs (or NULL) accumulates the (query, item) pairs scanned.
// gstride > 1 counts a sample instead: every gstride-th 16-item group of each
// chunk (no partial group).
hipError_t launch_scan_hist_stage(const uint32_t *codes_l, const uint32_t *qcodes, int64_t nq,
                                  const QueryShape &sh, const int32_t *chunks, int nchunks,
                                  const int32_t *need, uint32_t *ghist, unsigned long long *npairs,
                                  hipStream_t s, int gstride = 1);
// Collecting scan (matrix cores, chunks of at most 2^16 items): every item
// whose bucket ranks before grho[q] is counted in ghist (zeroed by the
// caller) and, unless its sub-dataset lies in [jh0, jh1), appended to query
// q's keys (nq x cap, rank << 32 | stored position; counts zeroed by the
// caller, may exceed cap).
hipError_t launch_scan_collect(const uint32_t *codes_l, const uint32_t *qcodes, int64_t nq, const QueryShape &sh,
                               const int32_t *chunks, int nchunks, const int32_t *R, const int32_t *grho,
                               int64_t cap, int32_t *counts, uint64_t *keys, uint32_t *ghist,
                               unsigned long long *npairs, hipStream_t s, int jh0 = 0, int jh1 = 0);
// The probed list (nq x Tq) of each query from its collected keys and the
// threshold (gtie) and tie position (gpstar); lcount[q] = its length; *fail
// is set when a query's collection was incomplete (its threshold bucket not
// before the guessed cut grho, or more keys than cap).
hipError_t launch_collect_filter(const uint64_t *keys, const int32_t *counts, int64_t cap, int64_t nq,
                                 const int32_t *gtie, const int32_t *gpstar, const int32_t *grho, int64_t Tq,
                                 int32_t *cand, int32_t *lcount, uint32_t *fail, hipStream_t s);
// rho[q] = (threshold bucket of gtie) + 1, at most P: the guessed cut.
hipError_t launch_rho_from_tie(const int32_t *gtie, int64_t nq, int32_t P, int32_t *rho, hipStream_t s);
// stats[0] += sum lcount, stats[1] = max(stats[1], max lcount), stats[2] +=
// sum gcount (gdef per query when gcount is NULL); *fail |= 2 when some
// lcount exceeds lcap.
hipError_t launch_list_check(const int32_t *lcount, const int32_t *gcount, int64_t nb, int lcap, int64_t gdef,
                             unsigned long long *stats, uint32_t *fail, hipStream_t s);
// Witnesses of the dense head: per sub-dataset j the stored positions, in
// stored order, of its `top` largest keys and of every `stride`-th item
// (wpos[j W ..], wcnt[j] of them; W >= top + ceil(n_j / stride)), and compact
// copies of their bfloat16 rows (xw, m W x dp), codes (cwo, m W x cw words)
// and keys (kw).
hipError_t launch_wit_build(const uint16_t *Xh, const uint32_t *codes_l, const double *key_l, const int32_t *off,
                            int m, int dp, int cw, int top, int stride, int W, int32_t *wpos, int32_t *wcnt,
                            uint16_t *xw, uint32_t *cwo, double *kw, hipStream_t s);
// pw[q] = gpstar[q] in the witnesses' slot numbering (gtie names the tie
// bucket's sub-dataset).
hipError_t launch_wit_pstar(const int32_t *gtie, const int32_t *gpstar, const int32_t *wpos, const int32_t *wcnt,
                            int W, int64_t nq, int32_t *pw, hipStream_t s);
// Permutation of a batch by its guessed cuts rho (ascending; keys of nbits
// bits), through a radix sort in the given buffers (nq each; tmp:
// radix_sort_tmp_bytes(nq)); *order points into va or vb.
hipError_t launch_rho_order(const int32_t *rho, int64_t nq, int nbits, uint64_t *ka, int32_t *va, uint64_t *kb,
                            int32_t *vb, void *tmp, int32_t **order, hipStream_t s);
// Qp / qcp / rhop row i = Q (d floats) / qc (cw words) / rho row order[i].
hipError_t launch_permute_batch(const float *Q, const uint32_t *qc, const int32_t *rho, const int32_t *order,
                                int64_t nq, int d, int cw, float *Qp, uint32_t *qcp, int32_t *rhop, hipStream_t s);
// ids / ips row order[i] = tids / tips row i (k entries each).
hipError_t launch_unpermute_results(const int32_t *order, int64_t nq, int k, const int64_t *tids, const float *tips,
                                    int64_t *ids, float *ips, hipStream_t s);
// out[j][s] (m x sub_hits_slices(nq) words) = the sample-pass items of
// sub-dataset j (ghist of a sampled pass) that rank before grho[q], summed
// over the queries of slice s.
int sub_hits_slices(int64_t nq);
hipError_t launch_sub_hits(const uint32_t *ghist, const int32_t *R, const int32_t *grho, int64_t nq, int m, int L,
                           unsigned long long *out, hipStream_t s);
// Pass 2 over the same chunks: appends each query's probed items to its list
// (counts zeroed by the caller; order unspecified), cutting the threshold
// bucket at gpstar (launch_tie_locate).
hipError_t launch_scan_emit_stage(const uint32_t *codes_l, const uint32_t *qcodes, int64_t nq,
                                  const QueryShape &sh, const int32_t *chunks, int nchunks,
                                  const int32_t *ghthr, const int32_t *gtie, const int32_t *gpstar,
                                  int32_t *counts, int32_t *cand, hipStream_t s);
hipError_t launch_stage_check(const uint32_t *ghist, const int32_t *inv, int64_t nq, const QueryShape &sh,
                              int cut, int32_t *need, hipStream_t s);

// ------------------------------------------------------------------ single probe
// Multi-table single probe (k_single.hip): t <= MT_MAX_TABLES tables; codes_l
// holds t x n x W words (table-major), qcodes the query codes table-major
// (table tau's code for sub-dataset j of query q at row tau qstride +
// qrow(q, j, P), P = qsets of one table).  Pass 1 adds per (tile, sub-dataset) the count of items by
// f = the first table whose bucket holds them into ghist (tiles x m x t x 64,
// zeroed by the caller); launch_threshold with L = t - 1 and the (f asc, j
// desc) rank table gives the bounds and the cut bin; launch_mt_tie the
// stored position of its r*-th item; launch_mt_emit appends the probed items
// (counts zeroed by the caller; fewer than Tq when the buckets hold fewer).
constexpr int MT_MAX_TABLES = 8;
hipError_t launch_mt_hist(const uint32_t *codes_l, int64_t n, const uint32_t *qcodes, int64_t qstride, int64_t nq,
                          int m, int t, int P, int W, const int32_t *chunks, int nchunks, uint32_t *ghist,
                          hipStream_t s);
hipError_t launch_mt_tie(const uint32_t *codes_l, int64_t n, const int32_t *off, const uint32_t *qcodes,
                         int64_t qstride, int64_t nq, int t, int P, int W, const int32_t *gtie, int32_t *gpstar,
                         hipStream_t s);
hipError_t launch_mt_emit(const uint32_t *codes_l, int64_t n, const uint32_t *qcodes, int64_t qstride, int64_t nq,
                          int m, int t, int P, int W, int64_t Tq, const int32_t *chunks, int nchunks,
                          const int32_t *ghthr, const int32_t *gtie, const int32_t *gpstar, int32_t *counts,
                          int32_t *cand, hipStream_t s);

// Stored position of the r*-th item of each query's threshold bucket (-1 if none).
// ghist (or NULL): the tile histograms of the threshold pass, whose bucket
// counts let a cut past the bucket's middle be found from its last item.
hipError_t launch_tie_locate(const uint32_t *codes_l, const int32_t *off, const uint32_t *qcodes,
                             int64_t nq, int W, int qsets, const int32_t *gtie, int32_t *gpstar,
                             hipStream_t s, const uint32_t *ghist = nullptr, int m = 0, int L = 0);

// Query-tiled FP32-MFMA screen of the probed set.  Chunks / cells are
// (sub-dataset, first, end) triples of stored items.
//   launch_screen_max: per (query, 32-item group of a cell) the largest lower
//     bound over the group's probed items (cmax: nq x ncells x groups), then
//     theta[q] = the k-th largest of them (lowered for rounding; -inf if fewer
//     than k groups hold probed items).  With Q.U, the first ncells_top cells
//     go first and give a theta that lets the other cells skip the tiles whose
//     queries their items cannot lift above it (the result is the same).
//   launch_screen: appends every probed pair whose FP32 upper bound reaches
//     theta[q] to lists (nq x cap) and counts all of them (counts zeroed by
//     the caller; counts[q] > cap means the list overflowed).
// Xh and Xlo != NULL select the bf16x3 matrix-core screen (x = hi + lo
// split, products hi.hi + hi.lo + lo.hi), Xh alone the single-product bf16
// screen (q and x rounded to bfloat16), neither the FP32 matrix-core screen.
enum ScreenKind { SCREEN_FP32 = 0, SCREEN_BF16 = 1, SCREEN_BF16X3 = 2 };
// A query batch as the screens read it: the FP32 rows Q (nq x d) and, for
// the bfloat16 screens, their bfloat16 image Qh (and its lo part Ql for
// bf16x3), nq x dp, with an upper bound qn on each row's 2-norm.
struct ScreenQueries {
    const float *Q;
    const uint16_t *Qh, *Ql;
    const float *qn;
    // U_j of each sub-dataset (FP64), or NULL: with it the bfloat16 screens'
    // pass B skips a chunk when no query of the tile can keep any of its items
    // (theta_q above the Cauchy-Schwarz bound ||q|| U_j plus the error bounds)
    const double *U = nullptr;
    // pass B adds the (query, item) pairs of every chunk it does not skip
    // (valid queries of the tile x items of the chunk), or NULL
    unsigned long long *pairs = nullptr;
    // pass B's query order (a permutation of the batch), or NULL for the
    // batch order
    const int32_t *order = nullptr;
};
// Permutation of a batch's queries by theta_q / ||q|| descending (queries
// without a theta last), through a radix sort in the given buffers (nq each;
// tmp: radix_sort_tmp_bytes(nq)); *order points into va or vb.
// rec[0..4] = largest and total counts[0..nb), queries with theta = -inf
// (theta != NULL), *npairs and *flag (0 where NULL); one block
hipError_t launch_list_stats(const int32_t *counts, const float *theta, int64_t nb,
                             const unsigned long long *npairs, const uint32_t *flag, long long *rec,
                             hipStream_t s);
hipError_t launch_query_order(const float *theta, const float *qn, int64_t nq, uint64_t *ka, int32_t *va,
                              uint64_t *kb, int32_t *vb, void *tmp, int32_t **order, hipStream_t s);
hipError_t launch_query_bf16(const float *Q, int64_t nq, int d, int dp, uint16_t *Qh, uint16_t *Ql,
                             float *qn, hipStream_t s, uint32_t *nonfinite = nullptr);
// Bounds for a budget that covers every item (T >= n): ghthr = 64 (at least
// L and any distance) for every query and sub-dataset, no threshold bucket
// (the layout launch_threshold writes), gpstar = -1.
hipError_t launch_probe_all(int64_t nq, const QueryShape &sh, int32_t *ghthr, int32_t *gtie,
                            int32_t *gpstar, hipStream_t s);
int screen_chunk_items();
int screen_cell_items();
int screen_cell_groups();  // lower-bound maxima kept per cell and query
size_t screen_lds_bytes(int dp, int kind);
hipError_t launch_screen_max(const float *Xl, const uint16_t *Xh, const uint16_t *Xlo,
                             const double *key_l, const uint32_t *codes_l,
                             const ScreenQueries &Q, int64_t nq, const QueryShape &sh, const int32_t *cells,
                             int ncells, int ncells_top, const uint32_t *qcodes, const int32_t *ghthr,
                             const int32_t *gtie, const int32_t *gpstar, float *cmax, float *theta,
                             hipStream_t s);
hipError_t launch_screen(const float *Xl, const uint16_t *Xh, const uint16_t *Xlo,
                         const double *key_l, const uint32_t *codes_l,
                         const ScreenQueries &Q, int64_t nq, const QueryShape &sh, const int32_t *chunks,
                         int nchunks, const uint32_t *qcodes, const int32_t *ghthr,
                         const int32_t *gtie, const int32_t *gpstar, const float *theta, int cap,
                         int32_t *counts, int32_t *lists, hipStream_t s);

// ------------------------------------------------------------------ bucket tables
// Read-only bucket table of an index (k_table.hip): titem = stored positions
// sorted by (sub-dataset, code, position); ucode / ustart = the distinct
// codes of each sub-dataset (ascending inside it) and the start of each one's
// run in titem (ustart[U] = n); uoff[j] = first distinct code of
// sub-dataset j (uoff[m] = U); binom = C(n, k) for n, k <= 64 (65 x 65).
struct TableView {
    const uint64_t *ucode;
    const int32_t *ustart, *uoff, *titem;
    const uint64_t *binom;
};
size_t table_binom_words();
void table_binom(uint64_t *out);
size_t table_scan_words(int64_t n);
size_t table_counter_bytes();  // device counters of the table probe (3 x uint64)
// Sorts (sub-dataset, code, position), compacts the distinct codes.  Writes
// titem, ucode, ustart[0 .. U), and uoff[j] for non-empty sub-datasets; U goes
// to *total.  ka / va / kb / vb: n-entry sort buffers; bsum: table_scan_words(n).
hipError_t launch_table_build(const uint32_t *codes_l, const int32_t *sid_l, int64_t n, int m, int L,
                              uint64_t *ka, int32_t *va, uint64_t *kb, int32_t *vb, void *sort_tmp,
                              int32_t *bsum, int32_t *total, int32_t *titem, uint64_t *ucode,
                              int32_t *ustart, int32_t *uoff, hipStream_t s);
// Probe count: one wave per query walks the buckets in probing order until
// Tq items; writes ghthr / gtie like launch_threshold.  qstate (nq x m,
// zeroed by the caller) and qhist (nq x m x (L+1)) are per-query scratch;
// counters (zeroed by the caller) gather lookup statistics.
hipError_t launch_table_count(const TableView &T, const int32_t *R, const int32_t *inv,
                              const uint32_t *qcodes, int64_t nq, const QueryShape &sh, int32_t *qstate,
                              int32_t *qhist, int32_t *ghthr, int32_t *gtie, void *counters,
                              hipStream_t s);
// Emission of exactly Tq stored positions per query (order unspecified).
hipError_t launch_table_emit(const TableView &T, const uint32_t *qcodes, int64_t nq, const QueryShape &sh,
                             const int32_t *qstate, const int32_t *ghthr, const int32_t *gtie,
                             const int32_t *gpstar, int32_t *cand, hipStream_t s);

// ------------------------------------------------------------------ batching form
// One (index, query batch) pair of a multi-index launch.  Index arrays are
// read-only during the launch; the workspace arrays belong to this pair.
struct MultiDesc {
    // index
    const float *Xl;
    const int32_t *perm;
    const uint32_t *codes_l;
    const int32_t *off;   // m + 1 stored-position bounds of the sub-datasets
    const int32_t *R;     // rank table, m x (L+1)
    const int32_t *inv;   // histogram index of each probing rank
    const float *At;      // A[:, :d] transposed (d x L)
    int64_t n;
    int32_t d, dp, m, L, W;
    int32_t tile_base;    // first per-tile counter of this pair
    // queries and results
    const float *Q;       // nq x d
    int64_t nq;
    int64_t Tq;           // min(T, n)
    int64_t q_base;       // first per-query counter of this pair
    int64_t *out_ids;     // nq x k
    float *out_ips;       // nq x k
    // workspace
    uint32_t *qcodes;     // nq x W
    uint32_t *ghist;      // tiles x m x (L+1) x 64, zero between launches
    int32_t *ghthr;       // tiles x m x 64
    int32_t *gtie;        // tiles x 4 x 64
    int32_t *gpstar;      // nq
    int32_t *cand;        // nq x Tq
    double *part_v;       // nq x nsplit x k (nsplit > 1)
    int32_t *part_i;
    unsigned long long *gtheta;  // nq (nsplit > 1): best k-th value of the query's slices,
                                 // order-preserving encoding, zeroed by the query-hash phase
    // tile shape
    int32_t chunk;        // stored items per scan work item
    int32_t nch;          // scan work items per sub-dataset
    int32_t slice;        // candidates per re-rank work item
    int32_t nsplit;       // re-rank work items per query
};

// Written by the last work-group of a multi-index launch.
struct MultiResult {
    int32_t done;       // 1 once the launch has drained
    int32_t error;      // MULTI_ERR_* bits
    int32_t nonfinite;  // queries held NaN / Inf
    int32_t pad;
};

constexpr int MULTI_PHASES = 7;        // QH HIST THR TIE EMIT RR MERGE
constexpr int MULTI_CTR_TILES = 16;    // first per-tile counter
constexpr int MULTI_TILE_CTRS = 5;     // per tile: QH HIST THR TIE EMIT done
constexpr int MULTI_ERR_TIMEOUT = 1;   // a wait exceeded its wall-clock limit
constexpr int MULTI_ERR_COUNT = 2;     // a probed list did not hold min(T, n) items

// Counter words of a launch with `tiles` query tiles and `nq` queries in all.
__host__ __device__ inline int64_t multi_ctr_words(int64_t tiles, int64_t nq)
{
    return MULTI_CTR_TILES + MULTI_TILE_CTRS * tiles + 2 * nq;
}

// The persistent kernel over descs[0 .. nb) with phase-major item numbering
// seg[ph * nb + b] (prefix sums, seg[7 nb] = item count).  descs, seg and
// result live in one device block uploaded before the launch.
size_t multi_lds_bytes(int maxL);
hipError_t multi_occupancy(int k, size_t lds, int *blocks_per_cu);
// Phase-per-launch form: one launch per phase with items[ph] work-groups
// (phases without items are skipped); ctr_q: 2 nq_total words, the first
// nq_total of which the threshold phase resets.  Errors and non-finite
// queries are or-ed into *result (zeroed by the caller before the launches).
hipError_t launch_multi_phases(const MultiDesc *descs, int nb, const int64_t *seg,
                               const int64_t *items, MultiResult *result, int32_t *ctr_q,
                               int64_t nq_total, int k, size_t lds, hipStream_t s);

// Persistent form (one launch for all phases, items wait on counters).
// ctr: multi_ctr_words(ntiles, nq_total) words, zero before the first
// launch (each launch leaves them zero unless it reports an error).
// limit_ticks bounds every wait of the launch, in wall_clock64 ticks.
hipError_t launch_multi(const MultiDesc *descs, int nb, const int64_t *seg, MultiResult *result,
                        int32_t *ctr, int64_t ntiles, int64_t nq_total, int k,
                        int64_t limit_ticks, int grid, size_t lds, hipStream_t s);

}  // namespace nrlsh
