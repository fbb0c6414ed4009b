// Batching form of the query: many indexes of uneven n and d, each with its
// own query batch, served by ONE persistent launch (Section 3.3 multi-probe
// and Algorithm 2 re-rank, the same arithmetic as k_query.hip).
//
// The launch walks a work queue.  Items are numbered phase-major -- every
// item of phase p of every index comes before any item of phase p + 1:
//   QH     codes of 16 queries (FP64 exact signs of A[:, :d] q)
//   HIST   pass 1: Hamming-distance histogram of one chunk of stored items of
//          one sub-dataset for a tile of 64 queries (lane = query), added to
//          the tile's histogram
//   THR    threshold walk of a tile over the sorted (U_j, l) structure
//          (Eq. 12): per sub-dataset emission bound and the threshold bucket
//          with the number r* of its items still probed; then clears the
//          tile's histogram for the next launch
//   TIE    stored position P* of the r*-th item of one query's threshold
//          bucket; with it, "probed" is a per-pair predicate:
//          h <= hthr[q][j]  or  (j = j*, h = h*, p <= P*)
//   EMIT   pass 2: appends the probed items of one chunk to the query lists
//   RR     FP64 re-rank of one slice of one query's probed list, top-k
//   MERGE  merge of a query's slice top-k lists
// A work-group (one wave) takes the next number from an atomic counter.  An
// item waits only on counters of items of earlier phases of the same tile or
// query; since every item numbered below it has already been taken by a
// running work-group, the smallest unfinished item never waits and the queue
// always drains, with no assumption about how many work-groups are resident.
// Each wait is also bounded by a wall-clock limit and by a shared error word:
// a wait that gives up records the error, every later wait returns at once,
// and the launch still drains.  The last work-group out clears the counters
// for the next launch (unless an error left them in use) and writes the
// result word.
#include <climits>
#include <cmath>

#include "dev_rerank.h"
#include "nrlsh_internal.h"

namespace nrlsh {
namespace {

using dev::WaveTopK;

enum { PH_QH = 0, PH_HIST, PH_THR, PH_TIE, PH_EMIT, PH_RR, PH_MERGE };
enum { CTR_HEAD = 0, CTR_EXITED = 1, CTR_ERROR = 2, CTR_NONFINITE = 3 };

// Index data (codes, sub-dataset bounds) is constant for the whole launch:
// reading it through the constant address space lets wave-uniform loads go
// through the scalar cache, as in the per-index scan kernels.
typedef const __attribute__((address_space(4))) uint32_t cu32;

// Values written during the launch by other work-groups are read with
// device-coherent loads only (never through the scalar cache).
__device__ __forceinline__ int32_t ld_coh(const int32_t *p)
{
    return __hip_atomic_load(const_cast<int32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_coh(const uint32_t *p)
{
    return __hip_atomic_load(const_cast<uint32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until *c >= need.  false: the launch has failed (error recorded).
// The poll is a relaxed device-coherent load with a growing sleep between
// polls; only once the count is reached does the wave acquire (one cache
// invalidation), so that many waiting waves do not keep invalidating the
// caches the working waves read through.  Bounded by the wall clock (limit
// ticks) and, independently of the clock, by a poll count.
__device__ bool wait_for(int32_t *c, int32_t need, int32_t *err, int64_t limit)
{
    if (ld_coh(c) < need) {
        const int64_t t0 = wall_clock64();
        for (uint32_t it = 0;; ++it) {
            if (it < 8) __builtin_amdgcn_s_sleep(2);
            else __builtin_amdgcn_s_sleep(64);
            if (ld_coh(c) >= need) break;
            if (ld_coh(err) != 0) return false;
            if (wall_clock64() - t0 > limit || it > (1u << 26)) {
                if (threadIdx.x == 0)
                    __hip_atomic_fetch_or(err, MULTI_ERR_TIMEOUT, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

// Publishes every write of this wave, then counts the item done.
__device__ __forceinline__ void signal(int32_t *c)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (threadIdx.x == 0) __hip_atomic_fetch_add(c, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct Ctx {
    int32_t *ctr;        // all counters (persistent form)
    int32_t *ctr_q;      // per-query counters: [0, nq_total) list lengths, then re-rank slices done
    int32_t *err;        // MULTI_ERR_* bits
    int32_t *nonfinite;  // set when a query holds NaN / Inf
    int64_t nq_total;
    int64_t limit;
    int k;
};

__device__ __forceinline__ int32_t *tile_ctr(const Ctx &C, const MultiDesc &D, int64_t tile, int ph)
{
    return C.ctr + MULTI_CTR_TILES + (int64_t)(D.tile_base + tile) * MULTI_TILE_CTRS + ph;
}

__device__ __forceinline__ int64_t tile_queries(const MultiDesc &D, int64_t tile)
{
    return min((int64_t)64, D.nq - tile * 64);
}

// ---------------------------------------------------------------- QH
template <bool SYNC>
__device__ void item_qhash(const Ctx &C, const MultiDesc &D, int64_t u)
{
    const int lane = threadIdx.x;
    const int64_t q0 = u * 16, q1 = min(D.nq, q0 + 16);
    const bool act = lane < D.L;
    bool bad = false;
    for (int64_t q = q0; q < q1; ++q) {
        const float *qv = D.Q + q * D.d;
        double s = 0.0;
        for (int t = 0; t < D.d; ++t) {
            const float qt = qv[t];
            bad |= !__builtin_isfinite(qt);
            const float a = act ? D.At[(int64_t)t * D.L + lane] : 0.f;
            s = s + (double)a * (double)qt;
        }
        const uint64_t code = __ballot(act && s > 0.0);
        if (lane == 0) {
            D.qcodes[q * D.W] = (uint32_t)code;
            if (D.W == 2) D.qcodes[q * D.W + 1] = (uint32_t)(code >> 32);
        }
    }
    if (bad && lane == 0)
        __hip_atomic_fetch_or(C.nonfinite, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // the re-rank slices of these queries start from no shared bound
    if (D.gtheta && q0 + lane < q1) D.gtheta[q0 + lane] = 0ull;
    if (SYNC) signal(tile_ctr(C, D, q0 >> 6, PH_QH));
}

// ---------------------------------------------------------------- HIST
template <int W>
__device__ void hist_chunk(const MultiDesc &D, int64_t tile, int j, int64_t p0, int64_t p1,
                           uint32_t *hist)
{
    const int lane = threadIdx.x;
    const int64_t q = tile * 64 + lane;
    uint32_t q0 = 0, q1 = 0;
    if (q < D.nq) {
        q0 = D.qcodes[q * W];
        if (W == 2) q1 = D.qcodes[q * W + 1];
    }
    for (int h = 0; h <= D.L; ++h) hist[h * 64 + lane] = 0u;
    cu32 *codes = (cu32 *)D.codes_l;
    int64_t p = p0;
    for (; p + 16 <= p1; p += 16) {
        uint32_t c[16 * W];
#pragma unroll
        for (int u = 0; u < 16 * W; ++u) c[u] = codes[p * W + u];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            uint32_t h = (uint32_t)__popc(c[u * W] ^ q0);
            if (W == 2) h += (uint32_t)__popc(c[u * W + 1] ^ q1);
            __hip_atomic_fetch_add(&hist[h * 64 + lane], 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    for (; p < p1; ++p) {
        uint32_t h = (uint32_t)__popc(codes[p * W] ^ q0);
        if (W == 2) h += (uint32_t)__popc(codes[p * W + 1] ^ q1);
        __hip_atomic_fetch_add(&hist[h * 64 + lane], 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    uint32_t *out = D.ghist + ((tile * D.m + j) * (int64_t)(D.L + 1)) * 64;
    for (int h = 0; h <= D.L; ++h) {
        const uint32_t v = hist[h * 64 + lane];
        if (v) __hip_atomic_fetch_add(&out[h * 64 + lane], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <bool SYNC>
__device__ void item_hist(const Ctx &C, const MultiDesc &D, int64_t u, uint32_t *hist)
{
    const int64_t per_tile = (int64_t)D.m * D.nch;
    const int64_t tile = u / per_tile;
    const int64_t r = u - tile * per_tile;
    const int j = (int)(r / D.nch), c = (int)(r - (int64_t)j * D.nch);
    const int64_t need = (tile_queries(D, tile) + 15) / 16;
    if (SYNC && !wait_for(tile_ctr(C, D, tile, PH_QH), (int32_t)need, C.err, C.limit)) return;
    cu32 *off = (cu32 *)D.off;
    const int64_t pj1 = (int32_t)off[j + 1];
    const int64_t p0 = (int64_t)(int32_t)off[j] + (int64_t)c * D.chunk;
    const int64_t p1 = min(pj1, p0 + D.chunk);
    if (p0 < p1) {
        if (D.W == 1) hist_chunk<1>(D, tile, j, p0, p1, hist);
        else hist_chunk<2>(D, tile, j, p0, p1, hist);
    }
    if (SYNC) signal(tile_ctr(C, D, tile, PH_HIST));
}

// ---------------------------------------------------------------- THR
template <bool SYNC>
__device__ void item_threshold(const Ctx &C, const MultiDesc &D, int64_t tile)
{
    const int lane = threadIdx.x;
    if (SYNC && !wait_for(tile_ctr(C, D, tile, PH_HIST), D.m * D.nch, C.err, C.limit)) return;
    const int64_t q = tile * 64 + lane;
    const bool valid = q < D.nq;
    const int L = D.L, L1 = L + 1, m = D.m;
    const int64_t P = (int64_t)m * L1;
    uint32_t *H = D.ghist + tile * P * 64;
    const int32_t *inv = D.inv;
    const int32_t *R = D.R;

    int64_t cum = 0;
    int32_t bstar = -1, rstar = 0, jstar = -1, hstar = -1;
    bool rfull = false;  // the budget ends exactly at the end of bucket b*
    bool done = !valid;
    for (int64_t b = 0; b < P; b += 16) {
        if (__ballot(!done) == 0ull) break;
        int32_t io[16];
        uint32_t c[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            io[u] = (b + u < P) ? inv[b + u] : 0;
            c[u] = (b + u < P) ? H[(int64_t)io[u] * 64 + lane] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            if (!done && b + u < P) {
                if (cum + (int64_t)c[u] >= D.Tq) {
                    bstar = (int32_t)(b + u);
                    rstar = (int32_t)(D.Tq - cum);
                    rfull = cum + (int64_t)c[u] == D.Tq;
                    jstar = io[u] / L1;
                    hstar = io[u] - jstar * L1;
                    done = true;
                } else {
                    cum += c[u];
                }
            }
        }
    }
    for (int j = 0; j < m; ++j) {
        int hthr = -1;
        if (valid) {
            int nl = 0;
            for (int l = 0; l <= L; ++l) nl += (R[(int64_t)j * L1 + l] < bstar) ? 1 : 0;
            hthr = nl - 1;
        }
        D.ghthr[(tile * m + j) * 64 + lane] = hthr;
    }
    int32_t *tie = D.gtie + tile * 4 * 64;
    tie[0 * 64 + lane] = valid ? jstar : -1;
    tie[1 * 64 + lane] = hstar;
    tie[2 * 64 + lane] = rfull ? INT_MAX : rstar;  // INT_MAX: every item of the bucket
    tie[3 * 64 + lane] = bstar;
    // the tile's histogram is consumed: leave it zero for the next launch;
    // the phase-per-launch form also starts the tile's list lengths at zero
    for (int64_t i = 0; i < P; ++i) H[i * 64 + lane] = 0u;
    if (!SYNC && valid) C.ctr_q[D.q_base + q] = 0;
    if (SYNC) signal(tile_ctr(C, D, tile, PH_THR));
}

// ---------------------------------------------------------------- TIE
template <int W>
__device__ int32_t tie_walk(const MultiDesc &D, int64_t q, int jstar, int hstar, int rstar)
{
    const int lane = threadIdx.x;
    const uint32_t q0 = ld_coh(D.qcodes + q * W), q1 = W == 2 ? ld_coh(D.qcodes + q * W + 1) : 0u;
    cu32 *off = (cu32 *)D.off;
    const int64_t pe = (int32_t)off[jstar + 1];
    int cnt = 0;
    for (int64_t p0 = (int32_t)off[jstar]; p0 < pe; p0 += 64) {
        const int64_t p = p0 + lane;
        bool match = false;
        if (p < pe) {
            int h = __popc(D.codes_l[p * W] ^ q0);
            if (W == 2) h += __popc(D.codes_l[p * W + 1] ^ q1);
            match = h == hstar;
        }
        const uint64_t bal = __ballot(match);
        const int c = __popcll(bal);
        if (cnt + c >= rstar) {
            const int need = rstar - cnt;  // 1-based rank inside this group
            const int rank = __popcll(bal & ((1ull << lane) - 1ull));
            const uint64_t sel = __ballot(match && rank == need - 1);
            return (int32_t)(p0 + __ffsll((long long)sel) - 1);
        }
        cnt += c;
    }
    return -1;
}

template <bool SYNC>
__device__ void item_tie(const Ctx &C, const MultiDesc &D, int64_t q)
{
    const int64_t tile = q >> 6;
    const int ql = (int)(q & 63);
    if (SYNC && !wait_for(tile_ctr(C, D, tile, PH_THR), 1, C.err, C.limit)) return;
    const int32_t *tie = D.gtie + tile * 4 * 64;
    const int jstar = ld_coh(tie + ql), hstar = ld_coh(tie + 64 + ql), rstar = ld_coh(tie + 128 + ql);
    int32_t P = -1;
    if (jstar >= 0 && rstar == INT_MAX) P = INT_MAX;
    else if (jstar >= 0) P = D.W == 1 ? tie_walk<1>(D, q, jstar, hstar, rstar)
                                      : tie_walk<2>(D, q, jstar, hstar, rstar);
    if (threadIdx.x == 0) D.gpstar[q] = P;
    if (SYNC) signal(tile_ctr(C, D, tile, PH_TIE));
}

// ---------------------------------------------------------------- EMIT
template <int W>
__device__ void emit_chunk(const Ctx &C, const MultiDesc &D, int64_t tile, int j, int64_t p0,
                           int64_t p1)
{
    const int lane = threadIdx.x;
    const int64_t q = tile * 64 + lane;
    const bool valid = q < D.nq;
    int hthr = -1, htie = -1;
    int32_t pstar = -1;
    uint32_t q0 = 0, q1 = 0;
    if (valid) {
        const int32_t *tie = D.gtie + tile * 4 * 64;
        hthr = D.ghthr[(tile * D.m + j) * 64 + lane];
        if (tie[lane] == j) {
            htie = tie[64 + lane];
            pstar = D.gpstar[q];
        }
        q0 = D.qcodes[q * W];
        if (W == 2) q1 = D.qcodes[q * W + 1];
    }
    if (__ballot(hthr >= 0 || htie >= 0) == 0ull) return;
    cu32 *codes = (cu32 *)D.codes_l;
    // pass a: how many this lane emits; pass b: write them after one append
    int32_t cnt = 0;
    int64_t p = p0;
    for (; p + 16 <= p1; p += 16) {
        uint32_t c[16 * W];
#pragma unroll
        for (int u = 0; u < 16 * W; ++u) c[u] = codes[p * W + u];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            int h = __popc(c[u * W] ^ q0);
            if (W == 2) h += __popc(c[u * W + 1] ^ q1);
            cnt += (h <= hthr || (h == htie && p + u <= pstar)) ? 1 : 0;
        }
    }
    for (; p < p1; ++p) {
        int h = __popc(codes[p * W] ^ q0);
        if (W == 2) h += __popc(codes[p * W + 1] ^ q1);
        cnt += (h <= hthr || (h == htie && p <= pstar)) ? 1 : 0;
    }
    if (__ballot(cnt > 0) == 0ull) return;
    int64_t base = 0;
    if (cnt > 0)
        base = __hip_atomic_fetch_add(C.ctr_q + D.q_base + q, cnt, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
    const int64_t cap = cnt > 0 ? min((int64_t)cnt, D.Tq - base) : 0;  // never past the list
    int32_t *out = D.cand + (valid ? q * D.Tq + base : 0);
    int64_t w = 0;
    for (p = p0; p + 16 <= p1; p += 16) {
        uint32_t c[16 * W];
#pragma unroll
        for (int u = 0; u < 16 * W; ++u) c[u] = codes[p * W + u];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            int h = __popc(c[u * W] ^ q0);
            if (W == 2) h += __popc(c[u * W + 1] ^ q1);
            const bool e = h <= hthr || (h == htie && p + u <= pstar);
            if (e && w < cap) out[w] = (int32_t)(p + u);
            w += e ? 1 : 0;
        }
    }
    for (; p < p1; ++p) {
        int h = __popc(codes[p * W] ^ q0);
        if (W == 2) h += __popc(codes[p * W + 1] ^ q1);
        const bool e = h <= hthr || (h == htie && p <= pstar);
        if (e && w < cap) out[w] = (int32_t)p;
        w += e ? 1 : 0;
    }
}

template <bool SYNC>
__device__ void item_emit(const Ctx &C, const MultiDesc &D, int64_t u)
{
    const int64_t per_tile = (int64_t)D.m * D.nch;
    const int64_t tile = u / per_tile;
    const int64_t r = u - tile * per_tile;
    const int j = (int)(r / D.nch), c = (int)(r - (int64_t)j * D.nch);
    if (SYNC && !wait_for(tile_ctr(C, D, tile, PH_TIE), (int32_t)tile_queries(D, tile), C.err,
                          C.limit))
        return;
    cu32 *off = (cu32 *)D.off;
    const int64_t pj1 = (int32_t)off[j + 1];
    const int64_t p0 = (int64_t)(int32_t)off[j] + (int64_t)c * D.chunk;
    const int64_t p1 = min(pj1, p0 + D.chunk);
    if (p0 < p1) {
        if (D.W == 1) emit_chunk<1>(C, D, tile, j, p0, p1);
        else emit_chunk<2>(C, D, tile, j, p0, p1);
    }
    if (SYNC) signal(tile_ctr(C, D, tile, PH_EMIT));
}

// ---------------------------------------------------------------- RR / MERGE
template <int S>
__device__ void write_topk(const MultiDesc &D, int64_t q, int k, const WaveTopK<S> &top)
{
    const int lane = threadIdx.x;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int e = s * 64 + lane;
        if (e < k) {
            D.out_ids[q * k + e] = top.ti[s] == INT_MAX ? -1 : (int64_t)top.ti[s];
            D.out_ips[q * k + e] = (float)top.tv[s];
        }
    }
}

template <int S, bool SYNC>
__device__ void item_rerank(const Ctx &C, const MultiDesc &D, int64_t u, float *tile_lds)
{
    const int lane = threadIdx.x;
    const int64_t q = u / D.nsplit;
    const int split = (int)(u - q * D.nsplit);
    if (SYNC && !wait_for(tile_ctr(C, D, q >> 6, PH_EMIT), D.m * D.nch, C.err, C.limit)) return;
    int64_t len = ld_coh(C.ctr_q + D.q_base + q);
    if (len != D.Tq && split == 0 && lane == 0)
        __hip_atomic_fetch_or(C.err, MULTI_ERR_COUNT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    len = min(len, D.Tq);
    const int64_t cbeg = (int64_t)split * D.slice;
    const int64_t cend = min(len, cbeg + D.slice);
    const float *qv = D.Q + q * D.d;
    const int32_t *cq = D.cand + q * D.Tq;
    WaveTopK<S> top;
    top.init(C.k);
    for (int64_t c0 = cbeg; c0 < cend; c0 += 64) {
        bool valid = c0 + lane < cend;
        int32_t id = 0, p = 0;
        if (valid) {
            p = cq[c0 + lane];
            valid = p >= 0 && (int64_t)p < D.n;  // positions come from the scan; never trust blindly
            if (valid) id = D.perm[p];
        }
        const double acc = dev::ip64_rows_fp32(D.Xl, D.d, D.dp, qv, p, valid, lane, tile_lds);
        // values below the best k-th value any slice of this query has
        // reached cannot enter its top-k
        double floor = -INFINITY;
        if (D.gtheta) {
            const unsigned long long ge =
                __hip_atomic_load(&D.gtheta[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (ge != 0ull) floor = dev::order_value(ge);
        }
        top.offer(acc, id, valid, lane, floor);
        if (D.gtheta && top.th_v > -INFINITY && top.th_v > floor && lane == 0)
            atomicMax(&D.gtheta[q], (unsigned long long)dev::order_key(top.th_v));
    }
    if (D.nsplit == 1) {
        write_topk<S>(D, q, C.k, top);
        return;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int e = s * 64 + lane;
        if (e < C.k) {
            const int64_t o = (q * D.nsplit + split) * C.k + e;
            D.part_v[o] = top.tv[s];
            D.part_i[o] = top.ti[s];
        }
    }
    if (SYNC) signal(C.ctr_q + C.nq_total + D.q_base + q);
}

template <int S, bool SYNC>
__device__ void item_merge(const Ctx &C, const MultiDesc &D, int64_t q)
{
    const int lane = threadIdx.x;
    if (SYNC && !wait_for(C.ctr_q + C.nq_total + D.q_base + q, D.nsplit, C.err, C.limit)) return;
    WaveTopK<S> top;
    top.init(C.k);
    const int64_t total = (int64_t)D.nsplit * C.k;
    const double *pv = D.part_v + q * total;
    const int32_t *pi = D.part_i + q * total;
    for (int64_t e0 = 0; e0 < total; e0 += 64) {
        const bool in = e0 + lane < total;
        const int32_t id = in ? pi[e0 + lane] : INT_MAX;
        const bool ok = in && id != INT_MAX;
        const double v = ok ? pv[e0 + lane] : -INFINITY;
        top.offer(v, ok ? id : INT_MAX, ok, lane);
    }
    write_topk<S>(D, q, C.k, top);
}

// ---------------------------------------------------------------- the launch
template <int S>
__global__ __launch_bounds__(64) void k_multi(const MultiDesc *__restrict__ descs, int nb,
                                              const int64_t *__restrict__ seg,
                                              MultiResult *result, int32_t *ctr, int64_t ntiles,
                                              int64_t nq_total, int k, int64_t limit)
{
    extern __shared__ float lds[];  // pass-1 histogram or re-rank tile
    const int lane = threadIdx.x;
    Ctx C;
    C.ctr = ctr;
    C.ctr_q = ctr + MULTI_CTR_TILES + MULTI_TILE_CTRS * ntiles;
    C.err = ctr + CTR_ERROR;
    C.nonfinite = ctr + CTR_NONFINITE;
    C.nq_total = nq_total;
    C.limit = limit;
    C.k = k;
    const int nseg = MULTI_PHASES * nb;
    const int64_t total = seg[nseg];
    for (;;) {
        int32_t w32 = 0;
        if (lane == 0) w32 = __hip_atomic_fetch_add(ctr + CTR_HEAD, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // wave-uniform from here on: descriptor fields and index data go
        // through scalar loads
        const int64_t w = __builtin_amdgcn_readfirstlane(w32);
        if (w >= total) break;
        int lo = 0, hi = nseg;  // seg[lo] <= w < seg[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (seg[mid] <= w) lo = mid;
            else hi = mid;
        }
        const int ph = lo / nb, b = lo - ph * nb;
        const int64_t u = w - seg[lo];
        const MultiDesc &D = descs[b];
        switch (ph) {
        case PH_QH: item_qhash<true>(C, D, u); break;
        case PH_HIST: item_hist<true>(C, D, u, reinterpret_cast<uint32_t *>(lds)); break;
        case PH_THR: item_threshold<true>(C, D, u); break;
        case PH_TIE: item_tie<true>(C, D, u); break;
        case PH_EMIT: item_emit<true>(C, D, u); break;
        case PH_RR: item_rerank<S, true>(C, D, u, lds); break;
        default: item_merge<S, true>(C, D, u); break;
        }
    }
    // the last work-group out publishes the result and resets the counters
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    int32_t prev = 0;
    if (lane == 0) prev = __hip_atomic_fetch_add(ctr + CTR_EXITED, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    prev = __builtin_amdgcn_readfirstlane(prev);
    if (prev != (int32_t)gridDim.x - 1) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int32_t err = ld_coh(ctr + CTR_ERROR), nonfinite = ld_coh(ctr + CTR_NONFINITE);
    if (err == 0) {
        const int64_t words = multi_ctr_words(ntiles, nq_total);
        for (int64_t i = lane; i < words; i += 64) ctr[i] = 0;
    }
    if (lane == 0) {
        result->error = err;
        result->nonfinite = nonfinite;
        result->done = 1;
    }
}

// Phase-per-launch form: one launch per phase, one work-group per item of
// that phase over all pairs; kernel boundaries order the phases, so no item
// waits on another.  seg: the item numbering of all phases (as above).
template <int PH, int S>
__global__ __launch_bounds__(64) void k_multi_phase(const MultiDesc *__restrict__ descs, int nb,
                                                    const int64_t *__restrict__ seg,
                                                    MultiResult *result, int32_t *ctr_q,
                                                    int64_t nq_total, int k)
{
    extern __shared__ float lds[];
    Ctx C;
    C.ctr = nullptr;
    C.ctr_q = ctr_q;
    C.err = &result->error;
    C.nonfinite = &result->nonfinite;
    C.nq_total = nq_total;
    C.limit = 0;
    C.k = k;
    const int64_t w = seg[PH * nb] + blockIdx.x;
    int lo = PH * nb, hi = PH * nb + nb;  // seg[lo] <= w < seg[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg[mid] <= w) lo = mid;
        else hi = mid;
    }
    const int b = lo - PH * nb;
    const int64_t u = w - seg[lo];
    const MultiDesc &D = descs[b];
    if (PH == PH_QH) item_qhash<false>(C, D, u);
    else if (PH == PH_HIST) item_hist<false>(C, D, u, reinterpret_cast<uint32_t *>(lds));
    else if (PH == PH_THR) item_threshold<false>(C, D, u);
    else if (PH == PH_TIE) item_tie<false>(C, D, u);
    else if (PH == PH_EMIT) item_emit<false>(C, D, u);
    else if (PH == PH_RR) item_rerank<S, false>(C, D, u, lds);
    else item_merge<S, false>(C, D, u);
}

}  // namespace

size_t multi_lds_bytes(int maxL)
{
    const size_t hist = (size_t)(maxL + 1) * 64 * sizeof(uint32_t);
    const size_t tile = (size_t)dev::RR_TILE_FLOATS * sizeof(float);
    return hist > tile ? hist : tile;
}

static const void *multi_fn(int k)
{
    const int S = (k + 63) / 64;
    if (S <= 1) return (const void *)k_multi<1>;
    if (S <= 2) return (const void *)k_multi<2>;
    if (S <= 4) return (const void *)k_multi<4>;
    if (S <= 8) return (const void *)k_multi<8>;
    return (const void *)k_multi<16>;
}

hipError_t multi_occupancy(int k, size_t lds, int *blocks_per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, multi_fn(k), 64, lds);
}

hipError_t launch_multi(const MultiDesc *descs, int nb, const int64_t *seg, MultiResult *result,
                        int32_t *ctr, int64_t ntiles, int64_t nq_total, int k, int64_t limit_ticks,
                        int grid, size_t lds, hipStream_t s)
{
    const int S = (k + 63) / 64;
#define NRLSH_MULTI(SS)                                                                     \
    hipLaunchKernelGGL(k_multi<SS>, dim3((unsigned)grid), dim3(64), lds, s, descs, nb, seg, \
                       result, ctr, ntiles, nq_total, k, limit_ticks)
    if (S <= 1) NRLSH_MULTI(1);
    else if (S <= 2) NRLSH_MULTI(2);
    else if (S <= 4) NRLSH_MULTI(4);
    else if (S <= 8) NRLSH_MULTI(8);
    else NRLSH_MULTI(16);
#undef NRLSH_MULTI
    return hipGetLastError();
}

template <int S>
static hipError_t launch_phases_s(const MultiDesc *descs, int nb, const int64_t *seg,
                                  const int64_t *items, MultiResult *result, int32_t *ctr_q,
                                  int64_t nq_total, int k, size_t lds, hipStream_t s)
{
    const dim3 block(64);
#define NRLSH_PHASE(PH, SH)                                                                    \
    if (items[PH] > 0) {                                                                       \
        hipLaunchKernelGGL((k_multi_phase<PH, S>), dim3((unsigned)items[PH]), block, SH, s,   \
                           descs, nb, seg, result, ctr_q, nq_total, k);                        \
        hipError_t e = hipGetLastError();                                                      \
        if (e != hipSuccess) return e;                                                         \
    }
    NRLSH_PHASE(PH_QH, 0)
    NRLSH_PHASE(PH_HIST, lds)
    NRLSH_PHASE(PH_THR, 0)
    NRLSH_PHASE(PH_TIE, 0)
    NRLSH_PHASE(PH_EMIT, 0)
    NRLSH_PHASE(PH_RR, lds)
    NRLSH_PHASE(PH_MERGE, 0)
#undef NRLSH_PHASE
    return hipSuccess;
}

hipError_t launch_multi_phases(const MultiDesc *descs, int nb, const int64_t *seg,
                               const int64_t *items, MultiResult *result, int32_t *ctr_q,
                               int64_t nq_total, int k, size_t lds, hipStream_t s)
{
    const int S = (k + 63) / 64;
    if (S <= 1) return launch_phases_s<1>(descs, nb, seg, items, result, ctr_q, nq_total, k, lds, s);
    if (S <= 2) return launch_phases_s<2>(descs, nb, seg, items, result, ctr_q, nq_total, k, lds, s);
    if (S <= 4) return launch_phases_s<4>(descs, nb, seg, items, result, ctr_q, nq_total, k, lds, s);
    if (S <= 8) return launch_phases_s<8>(descs, nb, seg, items, result, ctr_q, nq_total, k, lds, s);
    return launch_phases_s<16>(descs, nb, seg, items, result, ctr_q, nq_total, k, lds, s);
}

}  // namespace nrlsh
