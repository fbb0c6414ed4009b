/*
 * nrlsh.h -- C ABI of libnrlsh, norm-ranging LSH for maximum inner product
 * search (Yan, Li, Dai, Chen, Cheng, "Norm-Ranging LSH for Maximum Inner
 * Product Search", NeurIPS 2018) on AMD Instinct MI355X (gfx950).
 *
 * Problem (Section 1, Eq. 1): given n items x in R^d and a query q, return the
 * k items with the largest inner products q^T x, approximately.
 *
 * Index (Algorithm 1): items are ranked by 2-norm and cut into m sub-datasets
 * of (almost) equal size by norm percentile; sub-dataset j is normalised by
 * its own maximum norm U_j, transformed with SimpleLSH (Eq. 8,
 * P(x) = [x; sqrt(1 - ||x||^2)]) and hashed with L sign random projections
 * (Eq. 4) into an L-bit code.  One projection matrix serves all sub-datasets.
 *
 * Query (Algorithm 2 realised as the single-table multi-probe of
 * Section 3.3): the query code is P(q) = [q; 0] hashed with the same
 * projections; each item scores l = number of bits identical to the query
 * code, buckets (j, l) are probed in descending order of the similarity
 * metric s_hat = U_j cos[pi (1 - l/L)] (Eq. 12, via the sorted (U_j, l)
 * structure built with the index), the first T probed items are re-ranked by
 * their exact inner product and the best k are returned.
 *
 * Conventions shared by every call
 *   - Matrices are row-major and dense: items n x d, queries nq x d (float32).
 *   - Item / query / output pointers are HOST pointers unless an _ex call is
 *     given opts->device_ptrs = 1, in which case they are device pointers on
 *     the current HIP device (e.g. a torch tensor's data_ptr()).
 *   - When a call returns, its outputs are written and the caller may reuse
 *     or free its inputs (nrlsh_query_noalloc excepted: it queues its work on
 *     the caller's stream and returns).  nrlsh_build copies the items and returns once the
 *     last read of them is done; the rest of the index's device work (the
 *     hash and its FP64 fix-up) may still be queued on the library's stream,
 *     and every later call on the index is ordered after it (queries wait
 *     on the index's ready event on their stream, inspection calls and
 *     nrlsh_free on the host).  The index owns all of its device memory
 *     until nrlsh_free.
 *   - Ids are 0-based original item indices.  Results are ordered by
 *     (inner product descending, id ascending).  When fewer than k items are
 *     probed (min(T, n) < k) the tail is padded with id -1 and ip -INFINITY.
 *   - The index is immutable after build; concurrent nrlsh_query calls on one
 *     index are safe (each call allocates its own scratch).
 *   - Errors: a non-OK status is returned and nrlsh_last_error() gives a
 *     thread-local message.  No C++ exception crosses this ABI.  Arguments
 *     are validated on the host before any device work.
 */
#ifndef NRLSH_H
#define NRLSH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nrlsh_index nrlsh_index; /* opaque */

typedef enum nrlsh_status {
    NRLSH_OK = 0,
    NRLSH_E_INVALID_ARG = 1,   /* an argument is out of range or a pointer is NULL */
    NRLSH_E_NOT_FINITE = 2,    /* an item or query holds NaN or +-Inf */
    NRLSH_E_OUT_OF_MEMORY = 3, /* a device or host allocation failed */
    NRLSH_E_DEVICE = 4,        /* a HIP runtime call failed */
    NRLSH_E_INTERNAL = 5       /* an internal invariant failed */
} nrlsh_status;

/* Limits enforced by validation. */
#define NRLSH_MAX_L 64         /* code bits per item (1 <= L <= 64) */
#define NRLSH_MAX_K 1024       /* results per query */
#define NRLSH_MAX_N 2147483647 /* items per index (positions are int32) */

/* ---------------------------------------------------------------- build --
 * nrlsh_build: Algorithm 1 plus the sorted (U_j, l) structure of Section 3.3.
 *   items  n x d float32 (host pointer), finite.
 *   n      1 <= n <= NRLSH_MAX_N;  d >= 1;  1 <= m <= n;  1 <= L <= 64.
 *   seed   seeds the projection matrix A (L x (d+1), i.i.d. N(0,1) per Eq. 4):
 *          entry (r, c) is the Box-Muller transform of SplitMix64 outputs
 *          2t and 2t+1, t = r (d+1) + c, rounded to float32.
 *   out    receives the new index (caller frees with nrlsh_free).
 * Sub-dataset j (0-based) holds the items of norm rank [ceil(j n/m),
 * ceil((j+1) n/m)) in ascending (squared norm, index) order; the squared norm
 * is summed in FP64 in ascending coordinate order.  Hash bit r of an item is
 * [A_r . P(x/U_j) > 0] with the sign decided exactly as in FP64 (projections
 * too close to zero for the FP32 matrix-core pass are recomputed in FP64). */
nrlsh_status nrlsh_build(const float *items, int64_t n, int32_t d, int32_t m, int32_t L,
                         uint64_t seed, nrlsh_index **out);

/* Precision form of the hash GEMM.  The items are also kept in FP32 (for the
 * recompute and the re-rank); the hash reads a copy in this storage:
 *   FP32:     the FP32 copy on the FP32 matrix cores (default).
 *   BF16:     bfloat16 (round to nearest even) items and projections on the
 *             bf16 matrix cores, FP32 accumulate.
 *   FP8_E4M3: OCP E4M3 (round to nearest even, saturating, subnormals kept)
 *             with one FP32 scale per item row (max |x| / 448) and per
 *             projection row, on the fp8 matrix cores, FP32 accumulate.
 * In the BF16 / FP8 forms an item whose low-precision projection p~ of some
 * bit has |p~| <= margin is re-hashed from its FP32 copy (and then, like
 * every FP32 hash, in FP64 near zero):
 *   RIGOROUS: margin = a worst-case bound of |p~ - p| from the rounding of
 *             both operands and of the accumulation: every sign equals the
 *             FP64 definition (the default).
 *   SCALED:   margin = margin_param * ||x|| on the scaled projection
 *             U_j a.P(x/U_j) (e.g. 1e-3); signs outside it may differ from
 *             FP64 where the quantisation error exceeds the margin. */
typedef enum { NRLSH_STORAGE_FP32 = 0, NRLSH_STORAGE_BF16 = 1, NRLSH_STORAGE_FP8_E4M3 = 2 } nrlsh_storage;
typedef enum { NRLSH_MARGIN_RIGOROUS = 0, NRLSH_MARGIN_SCALED = 1 } nrlsh_margin_mode;

/* How items are cut into the m sub-datasets.
 *   PERCENTILE: by norm rank, sizes floor or ceil of n/m (Algorithm 1; default).
 *   UNIFORM:    the alternative of Section 5: the 2-norm domain [nmin, nmax]
 *               of the items is cut into m ranges of equal width; boundary j
 *               (1 <= j < m) is b_j = nmin + j (nmax - nmin) / m (FP64, in this
 *               order) and an item joins range #{j : key >= b_j * b_j}, where
 *               key is its FP64 squared norm.  Ranges may be empty (U_j = 0). */
typedef enum { NRLSH_PARTITION_PERCENTILE = 0, NRLSH_PARTITION_UNIFORM = 1 } nrlsh_partition;

/* Which hash functions the sub-datasets use (Algorithm 1 and Section 3.2
 * build one SimpleLSH index per sub-dataset, independently of the others).
 *   SHARED:     every sub-dataset hashes with the same L x (d+1) matrix A, so
 *               a query has one code (default).
 *   PER_SUBSET: sub-dataset j hashes with its own rows j L .. j L + L - 1 of
 *               an (m L) x (d+1) matrix drawn exactly as A above (entry (r, c)
 *               from counter t = r (d+1) + c), so rows 0 .. L-1 equal the
 *               shared A; a query has m codes, and its code for sub-dataset j
 *               decides the number of same bits l of j's items.  Only with
 *               hash_storage FP32; not accepted by the batching form. */
typedef enum { NRLSH_PROJECTIONS_SHARED = 0, NRLSH_PROJECTIONS_PER_SUBSET = 1 } nrlsh_projections;

typedef struct nrlsh_build_opts {
    int32_t struct_size;  /* sizeof(nrlsh_build_opts) */
    int32_t device_ptrs;  /* 1: items is a device pointer, aligned to 16 bytes
                             when d % 4 == 0, to 8 bytes when d is even, else
                             to 4 (any row of an aligned allocation is);
                             otherwise NRLSH_E_INVALID_ARG */
    void *stream;         /* hipStream_t to run on, or NULL for the library's stream */
    double eps;           /* adjusted metric s_hat = U_j cos[pi (1-eps)(1 - l/L)]
                             (Section 3.3), 0 <= eps < 1; 0 = Eq. 12 */
    int32_t hash_storage; /* nrlsh_storage (read when struct_size covers it) */
    int32_t margin_mode;  /* nrlsh_margin_mode */
    double margin_param;  /* SCALED: relative margin (>= 0) */
    int32_t partition;    /* nrlsh_partition (read when struct_size covers it) */
    int32_t projections;  /* nrlsh_projections (read when struct_size covers it) */
    int32_t bucket_tables; /* 1: also build the bucket tables that NRLSH_PROBE_TABLE
                              queries read (about 16 n bytes more; read when
                              struct_size covers it) */
    int32_t hash_tables;  /* independent hash tables t, 1 <= t <= 8 (0 = 1): table tau
                             hashes with its own projection block(s), rows
                             (tau P + b) L .. + L - 1 of one (t P L) x (d+1) matrix
                             drawn by the counter rule above (P = 1, or m with
                             per-subset projections); table 0 is the index the
                             multi-probe query reads, NRLSH_PROBE_SINGLE reads all
                             (FP32 hash only; 4 n W t bytes of codes) */
} nrlsh_build_opts;

nrlsh_status nrlsh_build_ex(const float *items, int64_t n, int32_t d, int32_t m, int32_t L,
                            uint64_t seed, const nrlsh_build_opts *opts, nrlsh_index **out);

/* Releases every resource of the index.  NULL is a no-op. */
void nrlsh_free(nrlsh_index *ix);

/* ---------------------------------------------------------------- query --
 * nrlsh_query: multi-probe MIPS (Section 3.3) with exact re-rank (Algorithm 2).
 *   queries       nq x d float32 (host), finite; nq >= 0 (0 is a no-op).
 *   k             1 <= k <= NRLSH_MAX_K.
 *   probe_budget  T >= 1 items to probe per query; clamped to n.
 *   out_ids       nq x k int64 (host): original item ids.
 *   out_ips       nq x k float32 (host): q^T x computed in FP64 (ascending
 *                 coordinate order) and rounded to float32.
 * The probed set is exactly the first min(T, n) items in the order
 * (bucket rank of (j, l) ascending, id ascending): the bucket where the budget
 * runs out is cut by id.  The result is the top-k of that set by
 * (FP64 inner product desc, id asc). */
nrlsh_status nrlsh_query(const nrlsh_index *ix, const float *queries, int64_t nq, int32_t k,
                         int64_t probe_budget, int64_t *out_ids, float *out_ips);

/* How the probed items are re-ranked; every mode returns the same result.
 *   GATHER:        each query's probed list is materialised and its rows gathered.
 *   SCREEN:        queries are tiled 64 at a time against chunks of stored rows on
 *                  the bf16 matrix cores with q and x rounded to bfloat16 (one
 *                  product per pair); pairs that are probed and whose inner
 *                  product (with a rigorous bound of the rounding of both
 *                  operands and the FP32 sum, (2^-7 + 2^-16 + 2.1 gamma_d)
 *                  ||q|| ||x||) can still reach a lower bound of the k-th
 *                  best are re-ranked exactly in FP64.
 *   SCREEN_FP32:   the same screen with FP32 matrix-core products.
 *   SCREEN_BF16X3: the same screen with a bfloat16 hi/lo split (three bf16
 *                  products per pair; tighter bounds, three times the work).
 *   AUTO:          SCREEN for large budgets (T >= n/128, T >= 2048, >= 64
 *                  queries), else GATHER. */
typedef enum {
    NRLSH_RERANK_AUTO = 0,
    NRLSH_RERANK_GATHER = 1,
    NRLSH_RERANK_SCREEN = 2,
    NRLSH_RERANK_SCREEN_FP32 = 3,
    NRLSH_RERANK_SCREEN_BF16X3 = 4
} nrlsh_rerank_mode;

/* How a query finds its probed items (SCAN and TABLE give the same probed set).
 *   SCAN:  every item code of the index is compared with the query code (two
 *          linear passes: per-bucket counts, then emission).  The first pass
 *          visits the sub-datasets in descending U_j and stops for a 64-query
 *          tile once every query's threshold bucket is known (no bucket of a
 *          sub-dataset not yet visited can rank before the first bucket
 *          (j, L) of the next one).
 *   TABLE: the "standard hash lookup" of Section 3.3: buckets (j, l) are taken
 *          in probing order from a table of each sub-dataset's distinct codes
 *          (the index must be built with bucket_tables = 1).  The codes at
 *          Hamming distance L - l from the query code are enumerated and looked
 *          up, until the lookups spent on sub-dataset j would exceed its number
 *          of distinct codes; then j's distinct codes are counted by distance
 *          once.  Work grows with the buckets probed, not with n; it pays
 *          where few buckets hold the budget (short codes, small T).  Goes with
 *          the GATHER re-rank (AUTO selects it; a SCREEN mode is rejected).
 *   SINGLE: multi-table single probe, the alternative to the single-table
 *          multi-probe that Section 4 names: in each of the index's
 *          hash_tables tables only the bucket of the query's own code is
 *          probed, in every sub-dataset (l = L).  With f(i) the first table
 *          whose probed bucket holds item i, the probed set is the first
 *          min(T, |C|) items of C = {i : f(i) exists} in the order (f asc,
 *          sub-dataset desc, id asc): tables are probed in order until the
 *          budget, the table where it runs out taken higher-norm sub-datasets
 *          first.  It may hold fewer than min(T, n) items (then the result
 *          is padded as usual).  Goes with the GATHER re-rank and FP32 rows. */
typedef enum { NRLSH_PROBE_SCAN = 0, NRLSH_PROBE_TABLE = 1, NRLSH_PROBE_SINGLE = 2 } nrlsh_probe_mode;

typedef struct nrlsh_query_opts {
    int32_t struct_size; /* sizeof(nrlsh_query_opts) */
    int32_t device_ptrs; /* 1: queries, out_ids, out_ips are device pointers */
    void *stream;        /* hipStream_t to run on, or NULL for the library's stream */
    int32_t rerank_mode; /* nrlsh_rerank_mode (read when struct_size covers it) */
    int32_t rerank_storage; /* GATHER re-rank rows: NRLSH_STORAGE_FP32 (default) or
                               NRLSH_STORAGE_BF16: inner products from the bfloat16
                               copy (FP32 sums) bound each item within ||q||
                               (||x - bf16(x)|| + (d + 8) 2^-23 ||x||) (the row's own
                               rounding error, kept with the index); items that may
                               still reach the top-k are re-ranked exactly from the
                               FP32 rows (same result, fewer bytes) */
    int32_t probe_mode;  /* nrlsh_probe_mode (read when struct_size covers it) */
    int32_t scan_guess;  /* SCAN probe, how the probed sets are found (same result
                            either way): 0 = default (budgets T >= 6400 below 2n/3
                            take one collecting scan behind a sampled guess of each
                            query's cut; others, and batches whose guess missed,
                            take the two exact passes); -1 = the two passes only;
                            g in 1..4096 = the collecting scan for every budget below
                            2n/3, guessing g/16 T items (small or large g make the
                            guess miss: for tests of the fallback) */
    int32_t dense_head;  /* BF16 re-rank storage with the collecting scan (same result
                            either way): 0 = default, the contiguous range of
                            sub-datasets around the one with the largest probed
                            fraction, while that fraction is at least 3/128, is
                            screened whole on the matrix cores (bfloat16 query
                            tiles x all its items, the SCREEN path's two passes and
                            probe test) instead of gathering its probed rows; the
                            other sub-datasets' probed items are gathered as usual;
                            -1 = no dense head; g in 1..256 = fraction at least
                            g/256.  The fractions are estimated from the sample pass
                            of the call's first batch (one host round trip). */
} nrlsh_query_opts;

nrlsh_status nrlsh_query_ex(const nrlsh_index *ix, const float *queries, int64_t nq, int32_t k,
                            int64_t probe_budget, const nrlsh_query_opts *opts,
                            int64_t *out_ids, float *out_ips);

/* ------------------------------------------------------ query, no allocation --
 * nrlsh_query_noalloc: for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the query of nrlsh_query_ex with device pointers, the linear
 * scan probe and the FP32 gather re-rank, with every temporary buffer taken
 * from a device scratch array of 64 MiB that the library holds on each device
 * it runs on until the process ends.  It calls no allocation routine, copies
 * nothing between host and device and does not synchronise: it queues kernels
 * on `stream` (a hipStream_t; NULL is the default stream) and returns.
 *   queries    nq x d float32, device pointer, finite (else *nonfinite != 0)
 *   out_ids    nq x k int64, out_ips nq x k float32, device pointers
 *   nonfinite  one device word, set to 0 and then to nonzero when a query
 *              holds NaN or Inf (the results of such a call are unspecified)
 * Queries are processed in batches of the largest multiple of 64 whose
 * buffers fit the scratch; NRLSH_E_INVALID_ARG (before any device work) when
 * even 64 queries do not fit, i.e. when 64 probed lists of min(T, n) entries
 * plus 64 histograms of m (L + 1) bins exceed it (roughly T > 2e5 at
 * m = 128, L = 64, k = 100).  All calls on one device share its scratch: calls that
 * overlap on one device (different streams, or host threads) race and must
 * be ordered by the caller.  Results equal those of nrlsh_query_ex. */
nrlsh_status nrlsh_query_noalloc(const nrlsh_index *ix, const float *queries, int64_t nq, int32_t k,
                                 int64_t probe_budget, void *stream, int64_t *out_ids, float *out_ips,
                                 uint32_t *nonfinite);

/* ------------------------------------------------------- batching form --
 * Many indexes (uneven n, d, L, m), each with its own query batch (uneven nq)
 * and probe budget, served together.  Each (index, batch) pair gets exactly
 * what nrlsh_query gives it (Section 3.3 multi-probe, Algorithm 2 exact
 * re-rank, same tie rules): the batching form changes how the work is
 * scheduled, not what is computed.
 *
 * The work of all pairs is cut into items -- query hash (16 queries), scan
 * pass 1 and scan pass 2 (one chunk of stored items of one sub-dataset for a
 * tile of 64 queries), threshold (a tile), tie location (a query), re-rank
 * (one slice of a query's probed list) and merge (a query) -- and each phase
 * is ONE launch over the items of every pair (one wave per item); the seven
 * launches of a run are captured once in a hipGraph and replayed.
 *
 * A plan fixes the set's shape (the indexes, each nq and probe budget, k) and
 * owns the workspace, the captured graph and the tile shape of each pair:
 * stored items per scan item ("chunk") and candidates per re-rank item
 * ("slice").  Tile shapes come from a process-wide table keyed by (d rounded
 * up to a power of two, L, batch class: nq <= 16, <= 256, > 256), filled by
 * the autotuner, which times candidate shapes on the plan's own pairs
 * (grouped by class) while the plan is created.
 *
 * A single persistent launch for all phases (items ordered by a work queue
 * and waiting on per-tile counters) is implemented but disabled: requesting
 * it (opts->persistent = 1) returns NRLSH_E_INVALID_ARG, because launches of
 * it did not complete in testing. */
typedef struct nrlsh_query_desc {
    const nrlsh_index *index;
    const float *queries; /* nq x d of that index (host, or device with device_ptrs) */
    int64_t nq;           /* >= 0 (0: the pair is skipped) */
    int64_t probe_budget; /* T >= 1, clamped to the index's n */
    int64_t *out_ids;     /* nq x k */
    float *out_ips;       /* nq x k */
} nrlsh_query_desc;

typedef enum {
    NRLSH_TUNE_TABLE = 0,  /* shapes from the table; defaults for classes not in it */
    NRLSH_TUNE_MISSING = 1,/* tune the classes of this set that are not in the table */
    NRLSH_TUNE_ALL = 2,    /* re-tune every class of this set */
    NRLSH_TUNE_DEFAULT = 3 /* fixed default shapes, table ignored */
} nrlsh_tune_mode;

typedef struct nrlsh_multi_opts {
    int32_t struct_size; /* sizeof(nrlsh_multi_opts) */
    int32_t device_ptrs; /* 1: queries / out_ids / out_ips are device pointers */
    void *stream;        /* hipStream_t to run on, or NULL for the library's stream */
    int32_t use_graph;   /* 1: replay a captured hipGraph (default); 0: launch directly */
    int32_t tune;        /* nrlsh_tune_mode */
    int32_t chunk;       /* > 0: force this chunk for every pair (multiple of 64) */
    int32_t slice;       /* > 0: force this slice for every pair (multiple of 64) */
    int32_t persistent;  /* 1: the single persistent launch (disabled, see above) */
} nrlsh_multi_opts;

typedef struct nrlsh_multi_plan nrlsh_multi_plan; /* opaque */

/* Creates a plan for descs[0 .. count) (1 <= count <= 4096) at top-k k.  All
 * indexes must live on one device.  Pointers in descs are only checked here;
 * nrlsh_multi_run takes the pointers of its own descs.  With autotuning the
 * plan runs the launch several times on these descs (their outputs are then
 * overwritten by nrlsh_multi_run).  Limits: the probed lists of all pairs hold
 * at most 2^31 entries in all. */
nrlsh_status nrlsh_multi_plan_create(const nrlsh_query_desc *descs, int32_t count, int32_t k,
                                     const nrlsh_multi_opts *opts, nrlsh_multi_plan **out);

/* Runs the plan on descs of the same shape (same count, index, nq and probe
 * budget per entry; query and output pointers may differ from call to call).
 * Synchronous.  NRLSH_E_NOT_FINITE if a query holds NaN / Inf. */
nrlsh_status nrlsh_multi_run(nrlsh_multi_plan *plan, const nrlsh_query_desc *descs, int32_t count);

/* Releases the plan.  NULL is a no-op. */
void nrlsh_multi_plan_free(nrlsh_multi_plan *plan);

/* create + run + free. */
nrlsh_status nrlsh_query_multi(const nrlsh_query_desc *descs, int32_t count, int32_t k,
                               const nrlsh_multi_opts *opts);

typedef struct nrlsh_multi_info {
    int32_t grid;          /* work-groups (one wave each) of the largest launch */
    int32_t graph;         /* 1: runs replay a captured hipGraph */
    int64_t items[7];      /* work items per phase: QH HIST THR TIE EMIT RR MERGE */
    int32_t tuned_classes; /* classes the autotuner timed while creating the plan */
    int32_t pad;
    double tune_ms;        /* wall-clock time spent tuning */
} nrlsh_multi_info;

/* Plan summary; chunk / slice (may be NULL) receive count tile shapes. */
nrlsh_status nrlsh_multi_plan_info(const nrlsh_multi_plan *plan, nrlsh_multi_info *info,
                                   int32_t *chunk, int32_t *slice);

/* Drops every entry of the autotuner's table. */
void nrlsh_tune_clear(void);

/* Table entry of class (d, L, nq): 1 and the shape if present, else 0. */
int32_t nrlsh_tune_lookup(int32_t d, int32_t L, int64_t nq, int32_t *chunk, int32_t *slice);

/* Thread-local message for the last non-OK status of this thread. */
const char *nrlsh_last_error(void);

/* ----------------------------------------------------------- inspection --
 * Copies of index internals to HOST buffers, for parity tests and reports.
 * All are synchronous and return NRLSH_E_INVALID_ARG on NULL arguments. */

/* n, d, m, L and the padded row stride dp (floats) of the stored item copy. */
nrlsh_status nrlsh_index_info(const nrlsh_index *ix, int64_t *n, int32_t *d, int32_t *m,
                              int32_t *L, int32_t *dp);

/* sets: number of L-row projection blocks of one hash table, 1 (SHARED) or
 * m (PER_SUBSET). */
nrlsh_status nrlsh_get_projection_sets(const nrlsh_index *ix, int32_t *sets);

/* A: (tables sets L) x (d+1) float32, row r = hash function r (Eq. 4); block
 * tau sets + j (rows (tau sets + j) L .. + L - 1) belongs to hash table tau
 * and, when sets = m, to sub-dataset j. */
nrlsh_status nrlsh_get_projection(const nrlsh_index *ix, float *A);

/* key: n float64 squared 2-norms in original order (Algorithm 1 ranking key). */
nrlsh_status nrlsh_get_keys(const nrlsh_index *ix, double *key);

/* sid: n int32 sub-dataset of each original item; keymax: m float64 largest
 * squared norm of each sub-dataset; U: m float64 = sqrt(keymax). */
nrlsh_status nrlsh_get_partition(const nrlsh_index *ix, int32_t *sid, double *keymax, double *U);

/* perm: n int32, original id at each stored position (sub-dataset major,
 * ascending id inside a sub-dataset); off: m+1 int64 sub-dataset offsets. */
nrlsh_status nrlsh_get_layout(const nrlsh_index *ix, int32_t *perm, int64_t *off);

/* codes: n uint64 item codes in original order; bit r = hash r, bits >= L zero. */
nrlsh_status nrlsh_get_codes(const nrlsh_index *ix, uint64_t *codes);

/* R: m x (L+1) int32 probing rank of bucket (j, l) (0 = probed first). */
nrlsh_status nrlsh_get_rank_table(const nrlsh_index *ix, int32_t *R);

typedef struct nrlsh_build_stats {
    int64_t recomputed_items; /* items with at least one bit recomputed in FP64 */
    int64_t recomputed_bits;  /* (item, bit) projections recomputed in FP64 */
    int64_t recompute_flips;  /* of those, bits whose FP32 sign differed from FP64 */
    int64_t lowp_items;       /* BF16 / FP8: items with more than 8 bits inside the
                                 margin, re-hashed whole from the FP32 copy (the
                                 in-margin bits of the others are recomputed in FP64
                                 and counted in recomputed_items / recomputed_bits) */
    int64_t lowp_bits;        /* BF16 / FP8: (item, bit) projections inside the margin */
    int64_t lowp_changed;     /* BF16 / FP8: bits the FP32 re-hash changed */
    int64_t recompute_flips_tiny; /* of recompute_flips, those whose exact projection
                              a . P(x) (P(x) of unit norm, Eq. 8) is below 1e-6 in
                              magnitude; recompute_flips - recompute_flips_tiny flipped
                              at 1e-6 or more.  Every flip is corrected: the codes are
                              the FP64 definition's either way */
} nrlsh_build_stats;

nrlsh_status nrlsh_get_build_stats(const nrlsh_index *ix, nrlsh_build_stats *st);

/* The hash storage copy in stored order (see nrlsh_get_layout): FP32 -> n x dp
 * float; BF16 -> n x dp uint16; FP8_E4M3 -> n x dp uint8 plus n float row
 * scales (scales may be NULL otherwise).  *storage receives the kind. */
nrlsh_status nrlsh_get_hash_copy(const nrlsh_index *ix, void *data, float *scales,
                                 int32_t *storage);

/* Bucket table of an index built with bucket_tables = 1 (else
 * NRLSH_E_INVALID_ARG).  *nunique = U, the number of distinct (sub-dataset,
 * code) pairs; when ucode is not NULL also copies ucode: U uint64 codes,
 * sub-dataset by sub-dataset and ascending inside each; ustart: U + 1 int64,
 * run starts in titem (ustart[U] = n); uoff: m + 1 int64, first distinct code
 * of each sub-dataset (uoff[m] = U); titem: n int32 stored positions sorted by
 * (sub-dataset, code, position). */
nrlsh_status nrlsh_get_bucket_table(const nrlsh_index *ix, int64_t *nunique, uint64_t *ucode,
                                    int64_t *ustart, int64_t *uoff, int32_t *titem);

/* Query codes: nq x sets uint64 (host in, host out), bit r of code (q, j) =
 * [A_{j L + r}[:d] . q > 0] (sets: nrlsh_get_projection_sets). */
nrlsh_status nrlsh_query_codes(const nrlsh_index *ix, const float *queries, int64_t nq,
                               uint64_t *codes);

/* Probed set of each query: cand is nq x min(T, n) int64 original ids (host),
 * in no particular order (the set is the definition's). */
nrlsh_status nrlsh_query_candidates(const nrlsh_index *ix, const float *queries, int64_t nq,
                                    int64_t probe_budget, int64_t *cand);

/* The probed set with each item's level (Section 3.3: the probed buckets are
 * (sub-dataset, l) pairs, l = the number of the item's L code bits equal to
 * the query's, L minus their Hamming distance).  cand as nrlsh_query_candidates
 * (host, nq x min(T, n) int64 original ids, in no particular order); levels
 * (host, same shape, int32) receives l of each entry.  NRLSH_E_INVALID_ARG
 * for a NULL levels with nq > 0, otherwise as nrlsh_query_candidates.  The
 * levels are formed on the host from copies of the codes (n x ceil(L/32)
 * words): a checking aid, not a fast path. */
nrlsh_status nrlsh_query_candidates_levels(const nrlsh_index *ix, const float *queries, int64_t nq,
                                           int64_t probe_budget, int64_t *cand, int32_t *levels);

/* The same under a probe mode (SCAN or SINGLE): counts (host, nq int64)
 * receives the number of probed items of each query; entries of cand past it
 * are -1. */
nrlsh_status nrlsh_query_candidates_ex(const nrlsh_index *ix, const float *queries, int64_t nq,
                                       int64_t probe_budget, int32_t probe_mode, int64_t *cand,
                                       int64_t *counts);

/* Number of hash tables of the index (build option hash_tables). */
nrlsh_status nrlsh_get_hash_tables(const nrlsh_index *ix, int32_t *tables);

/* Item codes of hash table `table` (0 <= table < hash tables), n uint64 per
 * original item as nrlsh_get_codes (which gives table 0). */
nrlsh_status nrlsh_get_codes_table(const nrlsh_index *ix, int32_t table, uint64_t *codes);

/* Re-rank statistics of this thread's last nrlsh_query / nrlsh_query_ex. */
typedef struct nrlsh_query_stats {
    int32_t mode;          /* nrlsh_rerank_mode actually used (GATHER or a SCREEN mode) */
    int32_t screen_passes; /* screen launches (more than one per batch = a list overflowed) */
    int64_t kept_total;    /* SCREEN: pairs kept for the exact re-rank, all queries */
    int64_t kept_max;      /* SCREEN: largest kept list of one query */
    int64_t theta_unset;   /* SCREEN: queries whose lower bound theta stayed -inf */
    int64_t lp_kept_total; /* BF16 re-rank: items re-ranked exactly, all queries */
    int64_t lp_kept_max;   /* BF16 re-rank: largest exact list of one query */
    int32_t lp_fallbacks;  /* BF16 re-rank: batches that overflowed into the FP32 re-rank;
                              after one, later batches of the call, and later calls on
                              the index with at least that k and budget, use the FP32
                              rows directly */
    int32_t probe_mode;    /* nrlsh_probe_mode used */
    int64_t table_lookups; /* TABLE: codes searched in the tables, all queries */
    int64_t table_walked;  /* TABLE: distinct codes counted by whole-sub-dataset passes */
    int64_t table_passes;  /* TABLE: whole-sub-dataset passes */
    int64_t screen_pairs;  /* SCREEN: (query, item) pairs evaluated by the keep pass,
                              summed over its launches (a chunk none of whose items
                              any query of the tile can keep, by the norm bound U_j,
                              is skipped) */
    int64_t scan_pairs;    /* SCAN: (query, item) pairs the first scan pass counted; the
                              sub-datasets are scanned in descending U_j and a 64-query
                              tile stops once all its queries' threshold buckets are
                              known, so this is at most nq x n.  With the collecting
                              scan (budgets of 6400 and more, below 2n/3): the pairs of
                              that scan, whose blocks skip sub-datasets no query of
                              the tile reaches before its guessed cut */
    int64_t collect_fallbacks; /* SCAN: batches whose collecting scan missed some query's
                              budget (its guessed cut too tight, or more items than
                              the key room) and that were probed again by the two
                              exact passes; results never depend on it */
    int64_t dense_head_items; /* BF16 re-rank: items of the sub-datasets screened whole
                              (dense_head) in the call's last batch that used it, else 0 */
    int64_t lp_gathered_total; /* BF16 re-rank: probed items whose bfloat16 rows were
                              gathered (all of them, less those of a dense head), all
                              queries */
    int64_t dense_head_pairs; /* BF16 re-rank: (query, item) pairs the dense head's keep
                              pass evaluated (64-query tiles skip the chunks of a
                              sub-dataset none of their queries probes), all queries */
} nrlsh_query_stats;

nrlsh_status nrlsh_get_query_stats(nrlsh_query_stats *st);

/* ------------------------------------------------------------ profiling --
 * Optional per-kernel timing with HIP events recorded on the stream each
 * kernel is launched on.  Off by default; enabling adds one event pair per
 * timed launch.  Names: "keys", "sort", "layout", "hash", "hash_fixup",
 * "qhash", "scan_hist", "threshold", "scan_emit", "rerank", "tie_locate",
 * "screen_max", "screen", "rerank_exact", and "multi" (one persistent
 * batching-form launch). */
void nrlsh_profile_enable(int32_t on);
void nrlsh_profile_reset(void);
/* Total milliseconds and launch count of kernel `name` since the last reset. */
nrlsh_status nrlsh_profile_get(const char *name, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* NRLSH_H */
