/*
 * nrlsh_oracle.c -- plain, slow, obviously-correct CPU reference for
 * norm-ranging LSH (Yan, Li, Dai, Chen, Cheng; NeurIPS 2018).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
 * CPU-baseline leg may load this library.  It shares no code with the GPU
 * library: no headers, no helpers, no tables.
 *
 * Everything is FP64 and evaluated in the order written (built with
 * -ffp-contract=off, no fast-math), with plain loops and a library sort
 * (qsort) as the only primitive.  Each function names the passage of the
 * paper it follows.  Readings of passages that are silent or ambiguous:
 *
 *   - ranking direction: ascending 2-norm, 0-based half-open ranges,
 *     subset s = floor(rank * m / n)                     (Algorithm 1)
 *   - ties in the ranking broken by original index        (Section 3.2)
 *   - the ranking key is the FP64 sum of squares, ascending coordinate order
 *   - sign(0) is bit 0                                    (Eq. 4)
 *   - one projection matrix shared by all sub-datasets    (Section 3.3,
 *     single-table multi-probe); as an option each sub-dataset draws its own
 *     L projections (rows j L .. j L + L - 1 of one m L x (d+1) matrix from
 *     the same generator) and the query is hashed once per sub-dataset
 *     (Section 1, "independently")
 *   - U_j = 0: the transformed item is [0; 1]             (Eq. 8)
 *   - probing order is descending s_hat (best first); cos(pi/2) is taken
 *     as exactly 0 and the table is antisymmetric about l = L/2; ties are
 *     ordered by subset descending, then l descending     (Eq. 12)
 *   - the probe budget T is a number of items; the bucket where the budget
 *     runs out is cut by original index                   (Section 3.3)
 *   - the query is not normalised (bits and argmax are scale invariant)
 *   - multi-table single probe (Section 4 names it as the alternative to
 *     single-table multi-probe; its description is in the absent supplement):
 *     t tables over the same partition, table tau hashing with its own
 *     projection rows (block tau P + b of one (t P L) x (d+1) matrix from the
 *     same generator, P = 1 shared or P = m per sub-dataset, b = 0 or the
 *     item's sub-dataset); a query probes in each table only the bucket of
 *     its own code in every sub-dataset (l = L).  f(i) = the first table whose
 *     probed bucket holds item i.  Tables are probed in order until T items:
 *     the probed items are taken in (f asc, sub-dataset desc, index asc)
 *     order, so the budget is cut inside the table where it runs out with the
 *     higher-norm sub-datasets first and by index inside a sub-dataset
 *   - uniform partitioning (Section 5, the alternative scheme): the 2-norm
 *     domain [min, max] of the items is cut into m ranges of equal width;
 *     boundary j (1 <= j < m) is b_j = nmin + j * w, w = (nmax - nmin) / m,
 *     and an item joins the range of the boundaries its key reaches:
 *     s = #{j : key >= b_j * b_j}; ranges may be empty
 *
 * Parity pins: every function here is checked by the CPU test-suite against
 * closed forms, invariants, brute force and published generator vectors.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Step 1 (Algorithm 1, "rank the items according to their 2-norms"):
 * key_i = sum_t x_it^2 in FP64, ascending t.  norm_i = sqrt(key_i).        */
void orc_keys(const float *X, int64_t n, int32_t d, double *key)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t t = 0; t < d; ++t) {
            double v = (double)X[i * (int64_t)d + t];
            s = s + v * v;
        }
        key[i] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* Step 2 (Algorithm 1): order items by (key ascending, index ascending).
 * rank[i] = position of item i in that order.                             */
typedef struct { double key; int64_t idx; } orc_kv;

static int orc_cmp_kv(const void *a, const void *b)
{
    const orc_kv *x = (const orc_kv *)a, *y = (const orc_kv *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    if (x->idx < y->idx) return -1;
    if (x->idx > y->idx) return 1;
    return 0;
}

int orc_rank(const double *key, int64_t n, int64_t *rank)
{
    orc_kv *kv = (orc_kv *)malloc(sizeof(orc_kv) * (size_t)(n > 0 ? n : 1));
    if (!kv) return -1;
    for (int64_t i = 0; i < n; ++i) { kv[i].key = key[i]; kv[i].idx = i; }
    qsort(kv, (size_t)n, sizeof(orc_kv), orc_cmp_kv);
    for (int64_t r = 0; r < n; ++r) rank[kv[r].idx] = r;
    free(kv);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Projection matrix for sign random projection (Eq. 4: entries i.i.d.
 * N(0,1)).  A is L x (d+1), row r is hash function r.  Entry (r, c) uses the
 * counter t = r*(d+1) + c and two outputs of the SplitMix64 generator
 * (Steele, Lea, Flood, OOPSLA 2014) at stream positions 2t and 2t+1; the
 * k-th output (0-based) of SplitMix64 seeded with s is mix(s + (k+1)*gamma).
 * The two uniforms go through the Box-Muller transform (1958):
 *   u1 = ((h1 >> 11) + 1) * 2^-53 in (0, 1],  u2 = (h2 >> 11) * 2^-53 in [0, 1)
 *   g  = sqrt(-2 ln u1) * cos(2 pi u2),   A_rc = (float) g  (round to nearest) */
uint64_t orc_splitmix64_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double orc_box_muller(uint64_t h1, uint64_t h2)
{
    double u1 = (double)((h1 >> 11) + 1u) * (1.0 / 9007199254740992.0);
    double u2 = (double)(h2 >> 11) * (1.0 / 9007199254740992.0);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

void orc_projection(uint64_t seed, int32_t L, int32_t d, float *A)
{
    for (int32_t r = 0; r < L; ++r)
        for (int32_t c = 0; c <= d; ++c) {
            uint64_t t = (uint64_t)r * (uint64_t)(d + 1) + (uint64_t)c;
            uint64_t h1 = orc_splitmix64_at(seed, 2u * t);
            uint64_t h2 = orc_splitmix64_at(seed, 2u * t + 1u);
            A[(int64_t)r * (d + 1) + c] = (float)orc_box_muller(h1, h2);
        }
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 partition: S_j holds ranks [ceil(j n/m), ceil((j+1) n/m)),
 * i.e. s_i = floor(rank_i * m / n); keymax_j = max key in S_j;
 * U_j = sqrt(keymax_j) = max 2-norm in S_j.                                */
void orc_partition(const double *key, const int64_t *rank, int64_t n, int32_t m,
                   int32_t *sid, double *keymax, double *U)
{
    for (int32_t j = 0; j < m; ++j) keymax[j] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t s = (int32_t)((rank[i] * (int64_t)m) / n);
        sid[i] = s;
        if (key[i] > keymax[s]) keymax[s] = key[i];
    }
    for (int32_t j = 0; j < m; ++j) U[j] = sqrt(keymax[j]);
}

/* Alternative partition of Section 5: uniformly spaced ranges of the 2-norm
 * domain [nmin, nmax] (nmin, nmax = sqrt of the smallest / largest key).
 * Boundary j = 1 .. m-1 is b_j = nmin + j w with w = (nmax - nmin) / m; the
 * item goes to the number of boundaries whose square its key reaches, so the
 * comparison is made on exact keys.  keymax_j = 0 for an empty range.        */
void orc_partition_uniform(const double *key, int64_t n, int32_t m, int32_t *sid,
                           double *keymax, double *U)
{
    double kmin = key[0], kmax = key[0];
    for (int64_t i = 1; i < n; ++i) {
        if (key[i] < kmin) kmin = key[i];
        if (key[i] > kmax) kmax = key[i];
    }
    const double nmin = sqrt(kmin), nmax = sqrt(kmax);
    const double w = (nmax - nmin) / (double)m;
    double *B = (double *)malloc(sizeof(double) * (size_t)(m > 1 ? m - 1 : 1));
    for (int32_t j = 1; j < m; ++j) {
        const double b = nmin + (double)j * w;
        B[j - 1] = b * b;
    }
    for (int32_t j = 0; j < m; ++j) keymax[j] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t s = 0;
        for (int32_t j = 1; j < m; ++j)
            if (key[i] >= B[j - 1]) s = j;
        sid[i] = s;
        if (key[i] > keymax[s]) keymax[s] = key[i];
    }
    for (int32_t j = 0; j < m; ++j) U[j] = sqrt(keymax[j]);
    free(B);
}

/* ------------------------------------------------------------------------ */
/* SimpleLSH transform (Eq. 8) of item i of sub-dataset j after normalising
 * by U_j (Algorithm 1):  v = [x / U_j ; sqrt(max(0, 1 - key_i / keymax_j))],
 * and v = [0 ; 1] when U_j = 0.  v has d+1 entries.                        */
void orc_transform(const float *x, int32_t d, double key, double keymax, double Uj, double *v)
{
    if (Uj == 0.0) {
        for (int32_t c = 0; c < d; ++c) v[c] = 0.0;
        v[d] = 1.0;
        return;
    }
    for (int32_t c = 0; c < d; ++c) v[c] = (double)x[c] / Uj;
    double t = 1.0 - key / keymax;
    if (t < 0.0) t = 0.0;
    v[d] = sqrt(t);
}

/* Sign random projection of a (d+1)-vector (Eq. 4): bit r = [A_r . v > 0],
 * FP64, ascending coordinate order.  code = sum_r bit_r * 2^r.            */
uint64_t orc_hash_vec(const float *A, int32_t L, int32_t d, const double *v)
{
    uint64_t code = 0;
    for (int32_t r = 0; r < L; ++r) {
        double s = 0.0;
        for (int32_t c = 0; c <= d; ++c) s = s + (double)A[(int64_t)r * (d + 1) + c] * v[c];
        if (s > 0.0) code |= (uint64_t)1 << r;
    }
    return code;
}

/* Item codes for items [i0, i1): transform then hash (Algorithm 1, the
 * SimpleLSH index of each sub-dataset).                                    */
/* Codes of items i0 .. i1-1; per_subset: item of sub-dataset s hashes with
 * rows s L .. s L + L - 1 of A (independent projections per sub-dataset). */
void orc_item_codes2(const float *X, int64_t i0, int64_t i1, int32_t d, int32_t L,
                     const float *A, int32_t per_subset, const double *key, const int32_t *sid,
                     const double *keymax, const double *U, uint64_t *codes)
{
    double *v = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    for (int64_t i = i0; i < i1; ++i) {
        int32_t s = sid[i];
        const float *As = per_subset ? A + (int64_t)s * L * (d + 1) : A;
        orc_transform(X + i * (int64_t)d, d, key[i], keymax[s], U[s], v);
        codes[i] = orc_hash_vec(As, L, d, v);
    }
    free(v);
}

void orc_item_codes(const float *X, int64_t i0, int64_t i1, int32_t d, int32_t L,
                    const float *A, const double *key, const int32_t *sid,
                    const double *keymax, const double *U, uint64_t *codes)
{
    orc_item_codes2(X, i0, i1, d, L, A, 0, key, sid, keymax, U, codes);
}

/* Query code (Eq. 8: P(q) = [q; 0]): bit r = [sum_{t<d} A_rt q_t > 0].     */
uint64_t orc_query_code(const float *A, int32_t L, int32_t d, const float *q)
{
    uint64_t code = 0;
    for (int32_t r = 0; r < L; ++r) {
        double s = 0.0;
        for (int32_t t = 0; t < d; ++t)
            s = s + (double)A[(int64_t)r * (d + 1) + t] * (double)q[t];
        if (s > 0.0) code |= (uint64_t)1 << r;
    }
    return code;
}

/* Number of identical bits between two L-bit codes (Section 3.3).         */
int32_t orc_same_bits(uint64_t a, uint64_t b, int32_t L)
{
    int32_t same = 0;
    for (int32_t r = 0; r < L; ++r)
        if (((a >> r) & 1u) == ((b >> r) & 1u)) ++same;
    return same;
}

/* ------------------------------------------------------------------------ */
/* Similarity metric (Eq. 12) and its sorted structure (Section 3.3):
 *   s_hat(j, l) = U_j * cos[pi (1 - eps) (1 - l/L)].
 * eps = 0: c(l) = cos(pi (L-l)/L) for 2l > L, c(L/2) = 0 exactly, and
 * c(l) = -c(L-l) for 2l < L.  eps > 0: c(l) = cos(pi (1-eps) (L-l)/L).
 * All m(L+1) pairs are sorted by (s_hat desc, j desc, l desc);
 * R[j*(L+1)+l] = position (0 is probed first).  shat[] receives the values. */
typedef struct { double s; int32_t j, l; } orc_pair;

static int orc_cmp_pair(const void *a, const void *b)
{
    const orc_pair *x = (const orc_pair *)a, *y = (const orc_pair *)b;
    if (x->s > y->s) return -1;
    if (x->s < y->s) return 1;
    if (x->j > y->j) return -1;
    if (x->j < y->j) return 1;
    if (x->l > y->l) return -1;
    if (x->l < y->l) return 1;
    return 0;
}

double orc_cos_level(int32_t l, int32_t L, double eps)
{
    if (eps != 0.0) return cos(M_PI * (1.0 - eps) * (double)(L - l) / (double)L);
    if (2 * l == L) return 0.0;
    if (2 * l > L) return cos(M_PI * (double)(L - l) / (double)L);
    return -cos(M_PI * (double)l / (double)L);
}

int orc_rank_table(const double *U, int32_t m, int32_t L, double eps, int32_t *R, double *shat)
{
    int64_t P = (int64_t)m * (L + 1);
    orc_pair *p = (orc_pair *)malloc(sizeof(orc_pair) * (size_t)P);
    if (!p) return -1;
    for (int32_t j = 0; j < m; ++j)
        for (int32_t l = 0; l <= L; ++l) {
            orc_pair *e = &p[(int64_t)j * (L + 1) + l];
            e->s = U[j] * orc_cos_level(l, L, eps);
            e->j = j;
            e->l = l;
            if (shat) shat[(int64_t)j * (L + 1) + l] = e->s;
        }
    qsort(p, (size_t)P, sizeof(orc_pair), orc_cmp_pair);
    for (int64_t b = 0; b < P; ++b) R[(int64_t)p[b].j * (L + 1) + p[b].l] = (int32_t)b;
    free(p);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Candidates of one query (Section 3.3 multi-probe, probed items of Section 4):
 * the first min(T, n) items in the order (R[s_i][l_i] asc, i asc).  Written
 * to cand[] in that order; l_out[] (optional) gets each candidate's l.      */
typedef struct { int64_t key; int64_t idx; } orc_ii;

static int orc_cmp_ii(const void *a, const void *b)
{
    const orc_ii *x = (const orc_ii *)a, *y = (const orc_ii *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    if (x->idx < y->idx) return -1;
    if (x->idx > y->idx) return 1;
    return 0;
}

/* qcodes: the query code for each sub-dataset (per_subset) or one code. */
int64_t orc_candidates2(const uint64_t *codes, const int32_t *sid, int64_t n, int32_t L,
                        const int32_t *R, const uint64_t *qcodes, int32_t per_subset, int64_t T,
                        int64_t *cand, int32_t *l_out)
{
    orc_ii *e = (orc_ii *)malloc(sizeof(orc_ii) * (size_t)(n > 0 ? n : 1));
    if (!e) return -1;
    for (int64_t i = 0; i < n; ++i) {
        const uint64_t qcode = qcodes[per_subset ? sid[i] : 0];
        int32_t l = orc_same_bits(codes[i], qcode, L);
        e[i].key = R[(int64_t)sid[i] * (L + 1) + l];
        e[i].idx = i;
    }
    qsort(e, (size_t)n, sizeof(orc_ii), orc_cmp_ii);
    int64_t Tq = T < n ? T : n;
    for (int64_t c = 0; c < Tq; ++c) {
        cand[c] = e[c].idx;
        if (l_out) l_out[c] = orc_same_bits(codes[e[c].idx], qcodes[per_subset ? sid[e[c].idx] : 0], L);
    }
    free(e);
    return Tq;
}

int64_t orc_candidates(const uint64_t *codes, const int32_t *sid, int64_t n, int32_t L,
                       const int32_t *R, uint64_t qcode, int64_t T, int64_t *cand,
                       int32_t *l_out)
{
    return orc_candidates2(codes, sid, n, L, R, &qcode, 0, T, cand, l_out);
}

/* Candidates of one query under multi-table single probe (see the header):
 * codes: tables x n; qcodes: tables x P query codes (P = m with per_subset,
 * else 1), code (tau, b) at qcodes[tau P + b].  f(i) = the first table tau
 * with codes[tau][i] == qcodes[tau][b(i)]; items without one are not probed.
 * The probed items in (f asc, sub-dataset desc, index asc) order, the first
 * min(T, |C|) of them, go to cand[]; returns their number.                 */
int64_t orc_candidates_mt(const uint64_t *codes, const int32_t *sid, int64_t n, int32_t m,
                          int32_t tables, const uint64_t *qcodes, int32_t per_subset, int64_t T,
                          int64_t *cand)
{
    orc_ii *e = (orc_ii *)malloc(sizeof(orc_ii) * (size_t)(n > 0 ? n : 1));
    if (!e) return -1;
    const int32_t P = per_subset ? m : 1;
    int64_t nc = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t f = -1;
        for (int32_t tb = 0; tb < tables && f < 0; ++tb) {
            const uint64_t qc = qcodes[(int64_t)tb * P + (per_subset ? sid[i] : 0)];
            if (codes[(int64_t)tb * n + i] == qc) f = tb;
        }
        if (f < 0) continue;
        e[nc].key = (int64_t)f * m + (m - 1 - sid[i]);
        e[nc].idx = i;
        ++nc;
    }
    qsort(e, (size_t)nc, sizeof(orc_ii), orc_cmp_ii);
    const int64_t Tq = T < nc ? T : nc;
    for (int64_t c = 0; c < Tq; ++c) cand[c] = e[c].idx;
    free(e);
    return Tq;
}

/* ------------------------------------------------------------------------ */
/* Exact inner product (Eq. 1) in FP64, ascending t.                        */
double orc_ip(const float *q, const float *x, int32_t d)
{
    double s = 0.0;
    for (int32_t t = 0; t < d; ++t) s = s + (double)q[t] * (double)x[t];
    return s;
}

/* Top-k of a candidate list by (ip desc, index asc) (Algorithm 2: keep the
 * item with the largest inner product; top-k MIPS, Section 1).  Short lists
 * are padded with id -1 and ip -inf.                                       */
typedef struct { double ip; int64_t idx; } orc_di;

static int orc_cmp_di(const void *a, const void *b)
{
    const orc_di *x = (const orc_di *)a, *y = (const orc_di *)b;
    if (x->ip > y->ip) return -1;
    if (x->ip < y->ip) return 1;
    if (x->idx < y->idx) return -1;
    if (x->idx > y->idx) return 1;
    return 0;
}

int orc_topk(const float *X, int32_t d, const float *q, const int64_t *cand, int64_t nc,
             int32_t k, int64_t *ids, double *ips)
{
    orc_di *e = (orc_di *)malloc(sizeof(orc_di) * (size_t)(nc > 0 ? nc : 1));
    if (!e) return -1;
    for (int64_t c = 0; c < nc; ++c) {
        e[c].idx = cand[c];
        e[c].ip = orc_ip(q, X + cand[c] * (int64_t)d, d);
    }
    qsort(e, (size_t)nc, sizeof(orc_di), orc_cmp_di);
    for (int32_t r = 0; r < k; ++r) {
        if (r < nc) { ids[r] = e[r].idx; ips[r] = e[r].ip; }
        else { ids[r] = -1; ips[r] = -INFINITY; }
    }
    free(e);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Whole-method drivers (Algorithm 1 then Algorithm 2 realised as the global
 * multi-probe of Section 3.3), with an optional thread count so that the
 * baseline can use the host's cores.  Threads split items (build) or
 * queries (query); each thread runs the plain per-item / per-query loop.  */
typedef struct {
    int64_t n; int32_t d, m, L;
    int32_t per_subset; /* 1: sub-dataset j hashes with rows j L .. j L + L - 1 of A */
    int32_t tables;    /* independent hash tables (single probe); 1 = the index itself */
    float *A;          /* tables x (L or m L) x (d+1): block tau P + b, P = 1 or m */
    double *key;       /* n */
    int64_t *rank;     /* n */
    int32_t *sid;      /* n */
    double *keymax;    /* m */
    double *U;         /* m */
    uint64_t *codes;   /* tables x n: table 0 first */
    int32_t *R;        /* m x (L+1) */
    const float *X;    /* borrowed, n x d */
} orc_index;

typedef struct {
    const orc_index *ix; int64_t i0, i1;
} orc_build_job;

static void *orc_build_worker(void *arg)
{
    orc_build_job *jb = (orc_build_job *)arg;
    const orc_index *ix = jb->ix;
    const int64_t blk = (int64_t)(ix->per_subset ? ix->m : 1) * ix->L * (ix->d + 1);
    for (int32_t tb = 0; tb < ix->tables; ++tb)
        orc_item_codes2(ix->X, jb->i0, jb->i1, ix->d, ix->L, ix->A + tb * blk, ix->per_subset, ix->key,
                        ix->sid, ix->keymax, ix->U, ix->codes + (int64_t)tb * ix->n);
    return NULL;
}

typedef struct {
    const float *X; int64_t i0, i1; int32_t d; double *key;
} orc_key_job;

static void *orc_key_worker(void *arg)
{
    orc_key_job *jb = (orc_key_job *)arg;
    orc_keys(jb->X + jb->i0 * (int64_t)jb->d, jb->i1 - jb->i0, jb->d, jb->key + jb->i0);
    return NULL;
}

void orc_free(orc_index *ix)
{
    if (!ix) return;
    free(ix->A); free(ix->key); free(ix->rank); free(ix->sid);
    free(ix->keymax); free(ix->U); free(ix->codes); free(ix->R);
    free(ix);
}

/* partition: 0 = norm percentiles (Algorithm 1), 1 = uniform ranges (Section 5);
 * per_subset: 1 = independent projections per sub-dataset */
orc_index *orc_build4(const float *X, int64_t n, int32_t d, int32_t m, int32_t L,
                      uint64_t seed, double eps, int32_t partition, int32_t per_subset,
                      int32_t tables, int32_t nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (tables < 1) return NULL;
    orc_index *ix = (orc_index *)calloc(1, sizeof(orc_index));
    if (!ix) return NULL;
    ix->n = n; ix->d = d; ix->m = m; ix->L = L; ix->X = X;
    ix->per_subset = per_subset ? 1 : 0;
    ix->tables = tables;
    const int32_t rows = (per_subset ? m * L : L) * tables;
    ix->A = (float *)malloc(sizeof(float) * (size_t)rows * (size_t)(d + 1));
    ix->key = (double *)malloc(sizeof(double) * (size_t)n);
    ix->rank = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    ix->sid = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    ix->keymax = (double *)malloc(sizeof(double) * (size_t)m);
    ix->U = (double *)malloc(sizeof(double) * (size_t)m);
    ix->codes = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n * (size_t)tables);
    ix->R = (int32_t *)malloc(sizeof(int32_t) * (size_t)m * (size_t)(L + 1));
    if (!ix->A || !ix->key || !ix->rank || !ix->sid || !ix->keymax || !ix->U ||
        !ix->codes || !ix->R) { orc_free(ix); return NULL; }

    orc_projection(seed, rows, d, ix->A);

    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    orc_key_job *kj = (orc_key_job *)malloc(sizeof(orc_key_job) * (size_t)nthreads);
    orc_build_job *bj = (orc_build_job *)malloc(sizeof(orc_build_job) * (size_t)nthreads);
    for (int32_t t = 0; t < nthreads; ++t) {
        kj[t].X = X; kj[t].d = d; kj[t].key = ix->key;
        kj[t].i0 = n * t / nthreads; kj[t].i1 = n * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, orc_key_worker, &kj[t]);
    }
    for (int32_t t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);

    orc_rank(ix->key, n, ix->rank);
    if (partition == 1)
        orc_partition_uniform(ix->key, n, m, ix->sid, ix->keymax, ix->U);
    else
        orc_partition(ix->key, ix->rank, n, m, ix->sid, ix->keymax, ix->U);

    for (int32_t t = 0; t < nthreads; ++t) {
        bj[t].ix = ix; bj[t].i0 = n * t / nthreads; bj[t].i1 = n * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, orc_build_worker, &bj[t]);
    }
    for (int32_t t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th); free(kj); free(bj);

    orc_rank_table(ix->U, m, L, eps, ix->R, NULL);
    return ix;
}

orc_index *orc_build3(const float *X, int64_t n, int32_t d, int32_t m, int32_t L,
                      uint64_t seed, double eps, int32_t partition, int32_t per_subset,
                      int32_t nthreads)
{
    return orc_build4(X, n, d, m, L, seed, eps, partition, per_subset, 1, nthreads);
}

orc_index *orc_build2(const float *X, int64_t n, int32_t d, int32_t m, int32_t L,
                      uint64_t seed, double eps, int32_t partition, int32_t nthreads)
{
    return orc_build3(X, n, d, m, L, seed, eps, partition, 0, nthreads);
}

orc_index *orc_build(const float *X, int64_t n, int32_t d, int32_t m, int32_t L,
                     uint64_t seed, double eps, int32_t nthreads)
{
    return orc_build3(X, n, d, m, L, seed, eps, 0, 0, nthreads);
}

/* Accessors for the Python wrapper. */
void orc_index_arrays(const orc_index *ix, float **A, double **key, int64_t **rank,
                      int32_t **sid, double **keymax, double **U, uint64_t **codes, int32_t **R)
{
    *A = ix->A; *key = ix->key; *rank = ix->rank; *sid = ix->sid;
    *keymax = ix->keymax; *U = ix->U; *codes = ix->codes; *R = ix->R;
}

typedef struct {
    const orc_index *ix; const float *Q; int64_t q0, q1; int32_t k; int64_t T;
    int32_t single_probe;  /* 1: multi-table single probe over every table */
    int64_t *ids; double *ips; int rc;
} orc_query_job;

static void *orc_query_worker(void *arg)
{
    orc_query_job *jb = (orc_query_job *)arg;
    const orc_index *ix = jb->ix;
    int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ix->n > 0 ? ix->n : 1));
    const int32_t ncodes = (ix->per_subset ? ix->m : 1) * (jb->single_probe ? ix->tables : 1);
    uint64_t *qc = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)ncodes);
    if (!cand || !qc) { free(cand); free(qc); jb->rc = -1; return NULL; }
    for (int64_t q = jb->q0; q < jb->q1; ++q) {
        const float *qv = jb->Q + q * (int64_t)ix->d;
        for (int32_t j = 0; j < ncodes; ++j)
            qc[j] = orc_query_code(ix->A + (int64_t)j * ix->L * (ix->d + 1), ix->L, ix->d, qv);
        int64_t nc = jb->single_probe
                         ? orc_candidates_mt(ix->codes, ix->sid, ix->n, ix->m, ix->tables, qc,
                                             ix->per_subset, jb->T, cand)
                         : orc_candidates2(ix->codes, ix->sid, ix->n, ix->L, ix->R, qc, ix->per_subset,
                                           jb->T, cand, NULL);
        if (nc < 0) { jb->rc = -1; break; }
        orc_topk(ix->X, ix->d, qv, cand, nc, jb->k, jb->ids + q * jb->k, jb->ips + q * jb->k);
    }
    free(cand);
    free(qc);
    return NULL;
}

int orc_query2(const orc_index *ix, const float *Q, int64_t nq, int32_t k, int64_t T,
               int32_t single_probe, int32_t nthreads, int64_t *ids, double *ips)
{
    if (nthreads < 1) nthreads = 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    orc_query_job *jb = (orc_query_job *)malloc(sizeof(orc_query_job) * (size_t)nthreads);
    for (int32_t t = 0; t < nthreads; ++t) {
        jb[t].ix = ix; jb[t].Q = Q; jb[t].k = k; jb[t].T = T; jb[t].ids = ids; jb[t].ips = ips;
        jb[t].single_probe = single_probe ? 1 : 0;
        jb[t].q0 = nq * t / nthreads; jb[t].q1 = nq * (t + 1) / nthreads; jb[t].rc = 0;
        pthread_create(&th[t], NULL, orc_query_worker, &jb[t]);
    }
    int rc = 0;
    for (int32_t t = 0; t < nthreads; ++t) { pthread_join(th[t], NULL); if (jb[t].rc) rc = -1; }
    free(th); free(jb);
    return rc;
}

int orc_query(const orc_index *ix, const float *Q, int64_t nq, int32_t k, int64_t T,
              int32_t nthreads, int64_t *ids, double *ips)
{
    return orc_query2(ix, Q, nq, k, T, 0, nthreads, ids, ips);
}

/* Brute-force exact top-k MIPS over all items (Eq. 1), ground truth for recall. */
typedef struct {
    const float *X; int64_t n; int32_t d; const float *Q; int64_t q0, q1; int32_t k;
    int64_t *ids; double *ips; int rc;
} orc_bf_job;

static void *orc_bf_worker(void *arg)
{
    orc_bf_job *jb = (orc_bf_job *)arg;
    int64_t *all = (int64_t *)malloc(sizeof(int64_t) * (size_t)(jb->n > 0 ? jb->n : 1));
    if (!all) { jb->rc = -1; return NULL; }
    for (int64_t i = 0; i < jb->n; ++i) all[i] = i;
    for (int64_t q = jb->q0; q < jb->q1; ++q)
        orc_topk(jb->X, jb->d, jb->Q + q * (int64_t)jb->d, all, jb->n, jb->k,
                 jb->ids + q * jb->k, jb->ips + q * jb->k);
    free(all);
    return NULL;
}

int orc_bruteforce(const float *X, int64_t n, int32_t d, const float *Q, int64_t nq, int32_t k,
                   int32_t nthreads, int64_t *ids, double *ips)
{
    if (nthreads < 1) nthreads = 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    orc_bf_job *jb = (orc_bf_job *)malloc(sizeof(orc_bf_job) * (size_t)nthreads);
    for (int32_t t = 0; t < nthreads; ++t) {
        jb[t].X = X; jb[t].n = n; jb[t].d = d; jb[t].Q = Q; jb[t].k = k;
        jb[t].ids = ids; jb[t].ips = ips; jb[t].rc = 0;
        jb[t].q0 = nq * t / nthreads; jb[t].q1 = nq * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, orc_bf_worker, &jb[t]);
    }
    int rc = 0;
    for (int32_t t = 0; t < nthreads; ++t) { pthread_join(th[t], NULL); if (jb[t].rc) rc = -1; }
    free(th); free(jb);
    return rc;
}
