// Multi-table single probe, the alternative to the single-table multi-probe
// that Section 4 names (its description is in the paper's absent supplement):
// t hash tables over one partition, table tau hashing every sub-dataset with
// its own projection rows; a query probes, in every table, only the bucket of
// its own code in each sub-dataset (l = L).  f(q, i) = the first table whose
// probed bucket holds item i.  Tables are probed in order until the budget:
// the probed items are taken in (f asc, sub-dataset desc, stored order)
// order, stored order being ascending original index inside a sub-dataset.
//
// The passes reuse the multi-probe machinery with the bins (j, h = f) in
// place of (j, h = L - l): pass 1 counts f per (query tile, sub-dataset),
// the threshold walk of k_query.hip finds the bin (j*, f*) where the budget
// runs out and its cut r* (with a rank table over (f asc, j desc)), the tie
// location finds the stored position P* of the r*-th item of that bin, and
// pass 2 appends every item with f <= fthr[q][j] or in the cut bin up to P*.
// Codes of table tau are codes_l[tau n W + p W ..]; the query codes are
// table-major: the code of table tau for sub-dataset j is row
// tau qstride + qrow(q, j, P) (qstride = rows per table, nq P).
#include <climits>

#include "nrlsh_internal.h"

namespace nrlsh {
namespace {

constexpr int MT_WAVES = 4;   // waves per pass block
constexpr int MT_TL = 16;     // waves per tie-location block
constexpr int MT_SB = 16;     // staged appends per lane in pass 2

// Query codes of one lane for every table (zero past t or for a lane past nq).
template <int W>
struct QCodes {
    uint32_t w[MT_MAX_TABLES][W];
};

template <int W>
__device__ __forceinline__ QCodes<W> load_qcodes(const uint32_t *__restrict__ qcodes, int64_t qstride, int64_t q,
                                                 int64_t nq, int j, int t, int P)
{
    QCodes<W> c;
#pragma unroll
    for (int tb = 0; tb < MT_MAX_TABLES; ++tb) {
        const bool ok = tb < t && q < nq;
        const int64_t r = ok ? tb * qstride + qrow(q, j, P) : 0;
#pragma unroll
        for (int w = 0; w < W; ++w) c.w[tb][w] = ok ? qcodes[r * W + w] : 0u;
    }
    return c;
}

// f of stored item p for one lane's query (t when no table's bucket holds it).
template <int W>
__device__ __forceinline__ int first_table(const uint32_t *__restrict__ codes_l, int64_t n, int64_t p, int t,
                                           const QCodes<W> &qc)
{
    int f = t;
#pragma unroll
    for (int tb = MT_MAX_TABLES - 1; tb >= 0; --tb) {
        if (tb >= t) continue;
        bool eq = codes_l[(tb * n + p) * W] == qc.w[tb][0];
        if (W == 2) eq = eq && codes_l[(tb * n + p) * W + 1] == qc.w[tb][W - 1];
        f = eq ? tb : f;
    }
    return f;
}

// Pass 1: per (64-query tile, chunk of one sub-dataset) the count of items
// by f, added into ghist[tile][j][f][lane] (zeroed by the caller).
template <int W>
__global__ __launch_bounds__(MT_WAVES * 64) void k_mt_hist(const uint32_t *__restrict__ codes_l, int64_t n,
                                                           const uint32_t *__restrict__ qcodes, int64_t qstride,
                                                           int64_t nq, int m, int t, int P,
                                                           const int32_t *__restrict__ chunks,
                                                           uint32_t *__restrict__ ghist)
{
    __shared__ uint32_t hist[MT_MAX_TABLES * 64];
    const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int64_t tile = blockIdx.x;
    const int j = chunks[3 * blockIdx.y];
    const int64_t p0 = chunks[3 * blockIdx.y + 1], p1 = chunks[3 * blockIdx.y + 2];
    const int64_t q = tile * 64 + lane;
    const QCodes<W> qc = load_qcodes<W>(qcodes, qstride, q, nq, j, t, P);
    for (int e = tid; e < t * 64; e += MT_WAVES * 64) hist[e] = 0u;
    __syncthreads();
    for (int64_t p = p0 + wave; p < p1; p += MT_WAVES) {
        const int f = first_table<W>(codes_l, n, p, t, qc);
        if (f < t) __hip_atomic_fetch_add(&hist[f * 64 + lane], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    uint32_t *out = ghist + (tile * m + j) * (int64_t)t * 64;
    for (int e = tid; e < t * 64; e += MT_WAVES * 64) {
        const uint32_t v = hist[e];
        if (v) atomicAdd(&out[e], v);
    }
}

// Stored position of the r*-th item with f = f* of sub-dataset j* for each
// query (the bin where the budget runs out); -1 with no cut bin, INT_MAX when
// the bin is probed whole.  One block per query, the waves sharing
// sub-dataset j* in contiguous pieces (lane = item).
template <int W>
__global__ __launch_bounds__(MT_TL * 64) void k_mt_tie(const uint32_t *__restrict__ codes_l, int64_t n,
                                                       const int32_t *__restrict__ off,
                                                       const uint32_t *__restrict__ qcodes, int64_t qstride,
                                                       int64_t nq, int t, int P, const int32_t *__restrict__ gtie,
                                                       int32_t *__restrict__ gpstar)
{
    __shared__ int32_t cnt_s[MT_TL];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t q = blockIdx.x;
    const int64_t tile = q >> 6;
    const int ql = (int)(q & 63);
    const int32_t *tie = gtie + tile * 4 * 64;
    const int jstar = tie[ql], fstar = tie[64 + ql], rstar = tie[128 + ql];
    if (jstar < 0 || rstar == INT_MAX) {  // the same for the whole block
        if (threadIdx.x == 0) gpstar[q] = jstar < 0 ? -1 : INT_MAX;
        return;
    }
    uint32_t qw[W];
    {
        const int64_t r = fstar * qstride + qrow(q, jstar, P);
#pragma unroll
        for (int w = 0; w < W; ++w) qw[w] = qcodes[r * W + w];
    }
    // f(p) = f* <=> table f*'s bucket holds p and no earlier table's does
    QCodes<W> qc;
#pragma unroll
    for (int tb = 0; tb < MT_MAX_TABLES; ++tb) {
        const bool ok = tb < fstar;
        const int64_t r = ok ? tb * qstride + qrow(q, jstar, P) : 0;
#pragma unroll
        for (int w = 0; w < W; ++w) qc.w[tb][w] = ok ? qcodes[r * W + w] : 0u;
    }
    const int64_t ps = off[jstar], pe = off[jstar + 1];
    auto match = [&](int64_t p) {
        if (p >= pe) return false;
        bool eq = codes_l[((int64_t)fstar * n + p) * W] == qw[0];
        if (W == 2) eq = eq && codes_l[((int64_t)fstar * n + p) * W + 1] == qw[W - 1];
        return eq && first_table<W>(codes_l, n, p, fstar, qc) == fstar;
    };
    const int64_t ng = (pe - ps + 63) / 64;
    const int64_t g0 = ng * wave / MT_TL, g1 = ng * (wave + 1) / MT_TL;
    int cnt = 0;
    for (int64_t g = g0; g < g1; ++g) cnt += __popcll(__ballot(match(ps + g * 64 + lane)));
    if (lane == 0) cnt_s[wave] = cnt;
    if (threadIdx.x == 0) gpstar[q] = -1;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += cnt_s[w];
    if (before < rstar && before + cnt >= rstar) {  // wave-uniform
        int c = before;
        for (int64_t g = g0; g < g1; ++g) {
            const int64_t pg = ps + g * 64;
            const uint64_t bal = __ballot(match(pg + lane));
            const int k = __popcll(bal);
            if (c + k >= rstar) {
                const int need = rstar - c;
                const int rank = __popcll(bal & ((1ull << lane) - 1ull));
                const uint64_t sel = __ballot(((bal >> lane) & 1ull) && rank == need - 1);
                if (lane == 0) gpstar[q] = (int32_t)(pg + __ffsll((long long)sel) - 1);
                break;
            }
            c += k;
        }
    }
}

// Pass 2: every probed item (f <= fthr[q][j], or f = f* in sub-dataset j* up
// to P*) appended to its query's list through a per-lane LDS stage.
__device__ __forceinline__ void mt_flush(const int32_t *__restrict__ stage, int lane, int cnt,
                                         int32_t *__restrict__ counts, int32_t *__restrict__ cand, int64_t q,
                                         int64_t Tq)
{
    const int64_t base = atomicAdd(&counts[q], cnt);
    const int64_t lim = min((int64_t)cnt, Tq - base);
    int32_t *out = cand + q * Tq + base;
    for (int i = 0; i < lim; ++i) out[i] = stage[i * 64 + lane];
}

template <int W>
__global__ __launch_bounds__(MT_WAVES * 64) void k_mt_emit(const uint32_t *__restrict__ codes_l, int64_t n,
                                                           const uint32_t *__restrict__ qcodes, int64_t qstride,
                                                           int64_t nq, int m, int t, int P, int64_t Tq,
                                                           const int32_t *__restrict__ chunks,
                                                           const int32_t *__restrict__ ghthr,
                                                           const int32_t *__restrict__ gtie,
                                                           const int32_t *__restrict__ gpstar,
                                                           int32_t *__restrict__ counts, int32_t *__restrict__ cand)
{
    __shared__ int32_t stage_s[MT_WAVES][MT_SB * 64];
    const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int64_t tile = blockIdx.x;
    const int j = chunks[3 * blockIdx.y];
    const int64_t p0 = chunks[3 * blockIdx.y + 1], p1 = chunks[3 * blockIdx.y + 2];
    const int64_t q = tile * 64 + lane;
    const bool valid = q < nq;
    int fthr = -1, ftie = -1;
    int64_t pstar = -1;
    if (valid) {
        const int32_t *tie = gtie + tile * 4 * 64;
        fthr = ghthr[(tile * m + j) * 64 + lane];
        if (tie[lane] == j) {
            ftie = tie[64 + lane];
            pstar = gpstar[q];
        }
    }
    if (__ballot(fthr >= 0 || ftie >= 0) == 0ull) return;  // the same for every wave of the block
    const QCodes<W> qc = load_qcodes<W>(qcodes, qstride, q, nq, j, t, P);
    int32_t *stage = stage_s[wave];
    int cnt = 0;
    for (int64_t p = p0 + wave; p < p1; p += MT_WAVES) {
        const int f = first_table<W>(codes_l, n, p, t, qc);
        if (f < t && (f <= fthr || (f == ftie && p <= pstar))) {
            stage[cnt * 64 + lane] = (int32_t)p;
            if (++cnt == MT_SB) {
                mt_flush(stage, lane, cnt, counts, cand, q, Tq);
                cnt = 0;
            }
        }
    }
    if (cnt > 0) mt_flush(stage, lane, cnt, counts, cand, q, Tq);
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

hipError_t launch_mt_hist(const uint32_t *codes_l, int64_t n, const uint32_t *qcodes, int64_t qstride, int64_t nq,
                          int m, int t, int P, int W, const int32_t *chunks, int nchunks, uint32_t *ghist,
                          hipStream_t s)
{
    if (nq < 1 || nchunks < 1) return hipSuccess;
    const dim3 grid(cdiv(nq, 64), (unsigned)nchunks);
    if (W == 1)
        hipLaunchKernelGGL(k_mt_hist<1>, grid, dim3(MT_WAVES * 64), 0, s, codes_l, n, qcodes, qstride, nq, m, t, P,
                           chunks, ghist);
    else
        hipLaunchKernelGGL(k_mt_hist<2>, grid, dim3(MT_WAVES * 64), 0, s, codes_l, n, qcodes, qstride, nq, m, t, P,
                           chunks, ghist);
    return hipGetLastError();
}

hipError_t launch_mt_tie(const uint32_t *codes_l, int64_t n, const int32_t *off, const uint32_t *qcodes,
                         int64_t qstride, int64_t nq, int t, int P, int W, const int32_t *gtie, int32_t *gpstar,
                         hipStream_t s)
{
    if (nq < 1) return hipSuccess;
    if (W == 1)
        hipLaunchKernelGGL(k_mt_tie<1>, dim3((unsigned)nq), dim3(MT_TL * 64), 0, s, codes_l, n, off, qcodes, qstride,
                           nq, t, P, gtie, gpstar);
    else
        hipLaunchKernelGGL(k_mt_tie<2>, dim3((unsigned)nq), dim3(MT_TL * 64), 0, s, codes_l, n, off, qcodes, qstride,
                           nq, t, P, gtie, gpstar);
    return hipGetLastError();
}

hipError_t launch_mt_emit(const uint32_t *codes_l, int64_t n, const uint32_t *qcodes, int64_t qstride, int64_t nq,
                          int m, int t, int P, int W, int64_t Tq, const int32_t *chunks, int nchunks,
                          const int32_t *ghthr, const int32_t *gtie, const int32_t *gpstar, int32_t *counts,
                          int32_t *cand, hipStream_t s)
{
    if (nq < 1 || nchunks < 1) return hipSuccess;
    const dim3 grid(cdiv(nq, 64), (unsigned)nchunks);
    if (W == 1)
        hipLaunchKernelGGL(k_mt_emit<1>, grid, dim3(MT_WAVES * 64), 0, s, codes_l, n, qcodes, qstride, nq, m, t, P,
                           Tq, chunks, ghthr, gtie, gpstar, counts, cand);
    else
        hipLaunchKernelGGL(k_mt_emit<2>, grid, dim3(MT_WAVES * 64), 0, s, codes_l, n, qcodes, qstride, nq, m, t, P,
                           Tq, chunks, ghthr, gtie, gpstar, counts, cand);
    return hipGetLastError();
}

}  // namespace nrlsh
