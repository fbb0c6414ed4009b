// Query kernels of norm-ranging LSH for gfx950 (Section 3.3 multi-probe,
// Algorithm 2 re-rank).
//
//   query_hash  code of P(q) = [q; 0] (Eq. 4, 8): one code under the shared
//               projections, or one per sub-dataset under its own block
//   scan_hist   pass 1: per (query tile, sub-dataset) histogram of the number
//               of differing bits, h = popcount(c_i ^ c_q) = L - l
//   threshold   walk the sorted (U_j, l) structure (Eq. 12) best-first until
//               the budget T is reached: threshold bucket b*, the number r* of
//               its items still probed, per-sub-dataset bounds and offsets
//   scan_emit   pass 2: write the probed items of every query, the threshold
//               bucket cut by index (stored order inside a sub-dataset)
//   rerank      exact inner products in FP64 (ascending coordinates) of the
//               probed items, top-k by (ip desc, id asc)
//
// In both scan passes a wave holds 64 queries (lane = query) and walks the
// codes of one sub-dataset; the codes are wave-uniform and come through the
// scalar cache, so each (query, item) pair costs one XOR, one popcount and,
// in pass 1, one conflict-free LDS increment of the lane's own histogram
// column.
#include <algorithm>
#include <climits>
#include <cmath>

#include "dev_rerank.h"
#include "nrlsh_internal.h"

namespace nrlsh {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------- query_hash
// Bit r of code (q, j) is the sign of sum_t A[jL + r][t] q_t, summed in FP64
// in ascending t (products of two floats are exact in FP64).  At is
// A[:, :d] transposed, d rows of qsets L floats, so that consecutive lanes
// read consecutive words.  One wave per (QH_Q queries, group of cpw = 64 / L
// codes, at least one): lane c L + r computes bit r of the group's code c for
// all QH_Q queries at once (staged through LDS in tiles of QH_TD
// coordinates), so each projection word read serves QH_Q queries.
constexpr int QH_Q = 8;
constexpr int QH_TD = 256;

__global__ __launch_bounds__(64) void k_query_hash(const float *__restrict__ Q, int64_t nq, int d,
                                                   const float *__restrict__ At, int L, int W,
                                                   int qsets, uint32_t *__restrict__ qcodes,
                                                   uint32_t *__restrict__ nonfinite)
{
    __shared__ float qs[QH_Q][QH_TD];
    const int lane = threadIdx.x;
    const int64_t q0 = (int64_t)blockIdx.x * QH_Q;
    const int cpw = L <= 32 ? 64 / L : 1;
    const int j0 = blockIdx.y * cpw;           // first code of this wave
    const int c = lane / L, r = lane - c * L;  // code within the group, bit
    const int j = j0 + c;
    const bool act = c < cpw && j < qsets;
    const int64_t R = (int64_t)qsets * L;
    const int64_t col = (int64_t)j * L + r;
    double acc[QH_Q];
#pragma unroll
    for (int i = 0; i < QH_Q; ++i) acc[i] = 0.0;
    bool bad = false;
    for (int t0 = 0; t0 < d; t0 += QH_TD) {
        const int tn = min(QH_TD, d - t0);
        __syncthreads();
        for (int e = lane; e < QH_Q * QH_TD; e += 64) {
            const int i = e / QH_TD, t = e - i * QH_TD;
            float v = 0.f;
            if (t < tn && q0 + i < nq) {
                v = Q[(q0 + i) * d + t0 + t];
                bad |= !__builtin_isfinite(v);
            }
            qs[i][t] = v;
        }
        __syncthreads();
        for (int t = 0; t < tn; ++t) {
            const double a = act ? (double)At[(int64_t)(t0 + t) * R + col] : 0.0;
#pragma unroll
            for (int i = 0; i < QH_Q; ++i) acc[i] = acc[i] + a * (double)qs[i][t];
        }
    }
    if (bad && blockIdx.y == 0) atomicOr(nonfinite, 1u);
#pragma unroll
    for (int i = 0; i < QH_Q; ++i) {
        const uint64_t bits = __ballot(act && acc[i] > 0.0);
        const int64_t q = q0 + i;
        if (q < nq && lane < cpw && j0 + lane < qsets) {
            // code `lane` of the group: bits lane L .. lane L + L - 1 of the ballot
            const uint64_t code = L == 64 ? bits : (bits >> (lane * L)) & ((1ull << L) - 1ull);
            const int64_t row = qrow(q, j0 + lane, qsets);
            qcodes[row * W] = (uint32_t)code;
            if (W == 2) qcodes[row * W + 1] = (uint32_t)(code >> 32);
        }
    }
}

// ---------------------------------------------------------------- scan pass 1
template <int W>
__global__ __launch_bounds__(64) void k_scan_hist(const uint32_t *__restrict__ codes_l,
                                                  const int32_t *__restrict__ off,
                                                  const uint32_t *__restrict__ qcodes, int64_t nq,
                                                  int m, int L, int qsets, uint32_t *__restrict__ ghist)
{
    extern __shared__ uint32_t hist[];  // (L+1) x 64, column = lane
    const int lane = threadIdx.x;
    const int tile = blockIdx.x, j = blockIdx.y;
    const int64_t q = (int64_t)tile * 64 + lane;
    uint32_t q0 = 0, q1 = 0;
    if (q < nq) {
        const int64_t r = qrow(q, j, qsets);
        q0 = qcodes[r * W];
        if (W == 2) q1 = qcodes[r * W + 1];
    }
    for (int h = 0; h <= L; ++h) hist[h * 64 + lane] = 0u;
    const int64_t p0 = off[j], p1 = off[j + 1];
    int64_t p = p0;
    for (; p + 16 <= p1; p += 16) {
        uint32_t c[16 * W];
#pragma unroll
        for (int u = 0; u < 16 * W; ++u) c[u] = codes_l[p * W + u];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            uint32_t h = (uint32_t)__popc(c[u * W] ^ q0);
            if (W == 2) h += (uint32_t)__popc(c[u * W + 1] ^ q1);
            __hip_atomic_fetch_add(&hist[h * 64 + lane], 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    for (; p < p1; ++p) {
        uint32_t h = (uint32_t)__popc(codes_l[p * W] ^ q0);
        if (W == 2) h += (uint32_t)__popc(codes_l[p * W + 1] ^ q1);
        __hip_atomic_fetch_add(&hist[h * 64 + lane], 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    uint32_t *out = ghist + ((int64_t)tile * m + j) * (int64_t)(L + 1) * 64;
    for (int h = 0; h <= L; ++h) out[h * 64 + lane] = hist[h * 64 + lane];
}

// ---------------------------------------------------------------- threshold
// One block of TH_WAVES waves per 64-query tile (lane = query).  inv[b] is
// the histogram index j (L+1) + h of the bucket with probing rank b.
//   1. Wave w sums the bucket counts of its contiguous share of the probing
//      order; the wave whose share holds a lane's crossing of Tq walks that
//      share again to find the threshold bucket b*, the items r* still
//      probed in it and its (j*, h*).
//   2. The sub-datasets are shared out among the waves: for each j,
//      hthr = #{h : rank(j, h) < b*} - 1 by binary search (ranks grow with h
//      inside a sub-dataset), the items probed in j, and their exclusive
//      prefix over j (the emission offsets gbase).
constexpr int TH_WAVES = 16;

__device__ __forceinline__ int wave_max_int(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// MODE 0: the threshold bucket and its cut only; 1: also the per-sub-dataset
// level bounds ghthr; 2: also the emission offsets gbase (the two-pass scan).
// INV_LDS: the probing order (m (L + 1) bucket numbers) is copied into LDS
// first; read from memory in the walks, each step's bucket numbers were a
// scalar load that the step's histogram loads had to wait for (0.21 -> 0.12
// ms per 4096-query call on the large workload).
constexpr int TH_INV_LDS_MAX = 12288;  // buckets staged in LDS (48 KiB)
template <int MODE, bool INV_LDS>
__global__ __launch_bounds__(TH_WAVES * 64) void k_threshold(const uint32_t *__restrict__ ghist,
                                                             const int32_t *__restrict__ R,
                                                             const int32_t *__restrict__ inv, int64_t nq,
                                                             int m, int L, int64_t Tq,
                                                             int32_t *__restrict__ gbase,
                                                             int32_t *__restrict__ ghthr,
                                                             int32_t *__restrict__ gtie)
{
    __shared__ int64_t seg_s[TH_WAVES][64];
    __shared__ int32_t res_s[5][64];  // b*, r*, j*, h*, whole
    extern __shared__ int32_t inv_s[];  // INV_LDS: the probing order
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, tile = blockIdx.x;
    const int64_t q = (int64_t)tile * 64 + lane;
    const bool valid = q < nq;
    const int L1 = L + 1;
    const int64_t P = (int64_t)m * L1;
    const uint32_t *H = ghist + (int64_t)tile * P * 64;
    if (INV_LDS) {
        for (int e = threadIdx.x; e < (int)P; e += TH_WAVES * 64) inv_s[e] = inv[e];
        __syncthreads();
    }
    const int32_t *io_src = INV_LDS ? inv_s : inv;

    // 1a. sum of this wave's share of the probing order
    const int64_t b0 = P * wave / TH_WAVES, b1 = P * (wave + 1) / TH_WAVES;
    int64_t sum = 0;
    int64_t b = b0;
    for (; b + 16 <= b1; b += 16) {
        uint32_t c[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) c[u] = H[(int64_t)io_src[b + u] * 64 + lane];
#pragma unroll
        for (int u = 0; u < 16; ++u) sum += c[u];
    }
    for (; b < b1; ++b) sum += H[(int64_t)io_src[b] * 64 + lane];
    seg_s[wave][lane] = sum;
    if (wave == 0) {
        res_s[0][lane] = -1;
        res_s[1][lane] = 0;
        res_s[2][lane] = -1;
        res_s[3][lane] = -1;
        res_s[4][lane] = 0;
    }
    __syncthreads();
    int64_t cum = 0;
    for (int w = 0; w < wave; ++w) cum += seg_s[w][lane];

    // 1b. the wave holding the crossing finds b*
    bool done = !(valid && cum < Tq && cum + sum >= Tq);
    for (b = b0; b < b1 && __ballot(!done) != 0ull; b += 16) {
        int32_t io[16];
        uint32_t c[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            io[u] = (b + u < b1) ? io_src[b + u] : 0;
            c[u] = (b + u < b1) ? H[(int64_t)io[u] * 64 + lane] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            if (!done && b + u < b1) {
                if (cum + (int64_t)c[u] >= Tq) {
                    const int jj = io[u] / L1;
                    res_s[0][lane] = (int32_t)(b + u);
                    res_s[1][lane] = (int32_t)(Tq - cum);
                    res_s[2][lane] = jj;
                    res_s[3][lane] = io[u] - jj * L1;
                    res_s[4][lane] = cum + (int64_t)c[u] == Tq;  // the budget ends with the bucket
                    done = true;
                } else {
                    cum += c[u];
                }
            }
        }
    }
    __syncthreads();
    int32_t bstar = res_s[0][lane];
    const int32_t rstar = res_s[1][lane], jstar = res_s[2][lane];
    // all buckets together hold fewer than Tq items (only possible when some
    // items belong to no bucket, as under single probe): every bucket is
    // probed whole
    if (valid && bstar < 0) bstar = (int32_t)P;
    if (MODE == 0) {  // the threshold bucket and its cut only
        if (wave == 0) {
            int32_t *tie = gtie + (int64_t)tile * 4 * 64;
            tie[0 * 64 + lane] = valid ? jstar : -1;
            tie[1 * 64 + lane] = res_s[3][lane];
            tie[2 * 64 + lane] = res_s[4][lane] ? INT_MAX : rstar;
            tie[3 * 64 + lane] = bstar;
        }
        return;
    }

    // 2. per-sub-dataset bounds and emission offsets
    const int ja = (int)((int64_t)m * wave / TH_WAVES), jb = (int)((int64_t)m * (wave + 1) / TH_WAVES);
    int64_t run = 0;
    for (int j = ja; j < jb; ++j) {
        int lo = 0, hi = valid ? L1 : 0;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (R[(int64_t)j * L1 + (L - mid)] < bstar) lo = mid + 1;
            else hi = mid;
        }
        const int hthr = lo - 1;
        ghthr[((int64_t)tile * m + j) * 64 + lane] = hthr;
        if (MODE < 2) continue;
        const int hmax = wave_max_int(hthr);
        const uint32_t *Hj = H + (int64_t)j * L1 * 64;
        int64_t cnt = 0;
        for (int h = 0; h <= hmax; ++h) {
            const uint32_t v = Hj[h * 64 + lane];
            if (h <= hthr) cnt += v;
        }
        if (j == jstar) cnt += rstar;
        gbase[((int64_t)tile * (m + 1) + j) * 64 + lane] = (int32_t)run;  // offset inside this wave's range
        run += cnt;
    }
    if (MODE == 2) {
        __syncthreads();  // every wave is done with seg_s
        seg_s[wave][lane] = run;
        __syncthreads();
        int64_t offs = 0;
        for (int w = 0; w < wave; ++w) offs += seg_s[w][lane];
        for (int j = ja; j < jb; ++j) {
            int32_t *g = gbase + ((int64_t)tile * (m + 1) + j) * 64 + lane;
            *g = (int32_t)(*g + offs);  // this lane wrote *g above
        }
        if (wave == TH_WAVES - 1) gbase[((int64_t)tile * (m + 1) + m) * 64 + lane] = (int32_t)(offs + run);
    }
    if (wave == 0) {
        int32_t *tie = gtie + (int64_t)tile * 4 * 64;
        tie[0 * 64 + lane] = valid ? jstar : -1;
        tie[1 * 64 + lane] = res_s[3][lane];
        tie[2 * 64 + lane] = res_s[4][lane] ? INT_MAX : rstar;  // INT_MAX: every item of the bucket
        tie[3 * 64 + lane] = bstar;
    }
}

// ---------------------------------------------------------------- scan pass 2
template <int W>
__global__ __launch_bounds__(64) void k_scan_emit(const uint32_t *__restrict__ codes_l,
                                                  const int32_t *__restrict__ off,
                                                  const uint32_t *__restrict__ qcodes, int64_t nq,
                                                  int m, int L, int64_t Tq, int qsets,
                                                  const int32_t *__restrict__ gbase,
                                                  const int32_t *__restrict__ ghthr,
                                                  const int32_t *__restrict__ gtie,
                                                  int32_t *__restrict__ cand)
{
    const int lane = threadIdx.x, tile = blockIdx.x, j = blockIdx.y;
    const int64_t q = (int64_t)tile * 64 + lane;
    const bool valid = q < nq;
    int hthr = -1, htie = -1, rstar = 0;
    int64_t base = 0;
    int32_t cap = 0;  // items this (query, sub-dataset) emits; bounds every write
    uint32_t q0 = 0, q1 = 0;
    if (valid) {
        const int32_t *tie = gtie + (int64_t)tile * 4 * 64;
        hthr = ghthr[((int64_t)tile * m + j) * 64 + lane];
        if (tie[lane] == j) {
            htie = tie[64 + lane];
            rstar = tie[128 + lane];
        }
        base = gbase[((int64_t)tile * (m + 1) + j) * 64 + lane];
        cap = gbase[((int64_t)tile * (m + 1) + j + 1) * 64 + lane] - (int32_t)base;
        const int64_t r = qrow(q, j, qsets);
        q0 = qcodes[r * W];
        if (W == 2) q1 = qcodes[r * W + 1];
    }
    if (__ballot(hthr >= 0 || htie >= 0) == 0ull) return;
    int32_t *out = cand + (valid ? q * Tq + base : 0);
    int32_t w = 0, tiecnt = 0;
    const int64_t p0 = off[j], p1 = off[j + 1];
    int64_t p = p0;
    for (; p + 16 <= p1; p += 16) {
        uint32_t c[16 * W];
#pragma unroll
        for (int u = 0; u < 16 * W; ++u) c[u] = codes_l[p * W + u];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            int h = __popc(c[u * W] ^ q0);
            if (W == 2) h += __popc(c[u * W + 1] ^ q1);
            const bool tie = h == htie;
            const bool emit = (h <= hthr) || (tie && tiecnt < rstar);
            tiecnt += tie ? 1 : 0;
            if (emit && w < cap) out[w++] = (int32_t)(p + u);
        }
    }
    for (; p < p1; ++p) {
        int h = __popc(codes_l[p * W] ^ q0);
        if (W == 2) h += __popc(codes_l[p * W + 1] ^ q1);
        const bool tie = h == htie;
        const bool emit = (h <= hthr) || (tie && tiecnt < rstar);
        tiecnt += tie ? 1 : 0;
        if (emit && w < cap) out[w++] = (int32_t)p;
    }
}

// ---------------------------------------------------------------- chunked scans
// Variants of the two passes for small query batches, where (query tiles) x
// (sub-datasets) waves cannot fill the machine: a sub-dataset's stored items
// are cut into chunks of `chunk` items, one wave per (tile, sub-dataset,
// chunk) -- block b = (tile m + j) nch + c.  Pass 1 adds the chunk's
// histogram into ghist (zeroed by the caller) with device atomics.  Pass 2
// counts each query's probed items of the chunk, reserves room with one
// atomic on the query's list length (counts, zeroed by the caller) and writes
// them; the threshold bucket is cut at the stored position P* of its r*-th
// item (k_tie_locate), so the probed set does not depend on the order of the
// appends.
template <int W>
__global__ __launch_bounds__(64) void k_scan_hist_c(const uint32_t *__restrict__ codes_l,
                                                    const int32_t *__restrict__ off,
                                                    const uint32_t *__restrict__ qcodes, int64_t nq,
                                                    int m, int L, int qsets, int chunk, int nch,
                                                    uint32_t *__restrict__ ghist)
{
    extern __shared__ uint32_t hist[];  // (L+1) x 64, column = lane
    const int lane = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int c = (int)(b % nch);
    const int j = (int)((b / nch) % m);
    const int64_t tile = b / ((int64_t)nch * m);
    const int64_t p0 = (int64_t)off[j] + (int64_t)c * chunk;
    const int64_t p1 = min((int64_t)off[j + 1], p0 + chunk);
    if (p0 >= p1) return;
    const int64_t q = tile * 64 + lane;
    uint32_t q0 = 0, q1 = 0;
    if (q < nq) {
        const int64_t r = qrow(q, j, qsets);
        q0 = qcodes[r * W];
        if (W == 2) q1 = qcodes[r * W + 1];
    }
    for (int h = 0; h <= L; ++h) hist[h * 64 + lane] = 0u;
    int64_t p = p0;
    for (; p + 16 <= p1; p += 16) {
        uint32_t cc[16 * W];
#pragma unroll
        for (int u = 0; u < 16 * W; ++u) cc[u] = codes_l[p * W + u];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            uint32_t h = (uint32_t)__popc(cc[u * W] ^ q0);
            if (W == 2) h += (uint32_t)__popc(cc[u * W + 1] ^ q1);
            __hip_atomic_fetch_add(&hist[h * 64 + lane], 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    for (; p < p1; ++p) {
        uint32_t h = (uint32_t)__popc(codes_l[p * W] ^ q0);
        if (W == 2) h += (uint32_t)__popc(codes_l[p * W + 1] ^ q1);
        __hip_atomic_fetch_add(&hist[h * 64 + lane], 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    uint32_t *out = ghist + ((tile * m + j) * (int64_t)(L + 1)) * 64;
    for (int h = 0; h <= L; ++h) {
        const uint32_t v = hist[h * 64 + lane];
        if (v) atomicAdd(&out[h * 64 + lane], v);
    }
}

template <int W>
__global__ __launch_bounds__(64) void k_scan_emit_c(const uint32_t *__restrict__ codes_l,
                                                    const int32_t *__restrict__ off,
                                                    const uint32_t *__restrict__ qcodes, int64_t nq,
                                                    int m, int64_t Tq, int qsets, int chunk, int nch,
                                                    const int32_t *__restrict__ ghthr,
                                                    const int32_t *__restrict__ gtie,
                                                    const int32_t *__restrict__ gpstar,
                                                    int32_t *__restrict__ counts,
                                                    int32_t *__restrict__ cand)
{
    const int lane = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int c = (int)(b % nch);
    const int j = (int)((b / nch) % m);
    const int64_t tile = b / ((int64_t)nch * m);
    const int64_t p0 = (int64_t)off[j] + (int64_t)c * chunk;
    const int64_t p1 = min((int64_t)off[j + 1], p0 + chunk);
    if (p0 >= p1) return;
    const int64_t q = tile * 64 + lane;
    const bool valid = q < nq;
    int hthr = -1, htie = -1;
    int32_t pstar = -1;
    uint32_t q0 = 0, q1 = 0;
    if (valid) {
        const int32_t *tie = gtie + tile * 4 * 64;
        hthr = ghthr[(tile * m + j) * 64 + lane];
        if (tie[lane] == j) {
            htie = tie[64 + lane];
            pstar = gpstar[q];
        }
        const int64_t r = qrow(q, j, qsets);
        q0 = qcodes[r * W];
        if (W == 2) q1 = qcodes[r * W + 1];
    }
    if (__ballot(hthr >= 0 || htie >= 0) == 0ull) return;
    int32_t cnt = 0;
    int64_t p = p0;
    for (; p + 16 <= p1; p += 16) {
        uint32_t cc[16 * W];
#pragma unroll
        for (int u = 0; u < 16 * W; ++u) cc[u] = codes_l[p * W + u];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            int h = __popc(cc[u * W] ^ q0);
            if (W == 2) h += __popc(cc[u * W + 1] ^ q1);
            cnt += (h <= hthr || (h == htie && p + u <= pstar)) ? 1 : 0;
        }
    }
    for (; p < p1; ++p) {
        int h = __popc(codes_l[p * W] ^ q0);
        if (W == 2) h += __popc(codes_l[p * W + 1] ^ q1);
        cnt += (h <= hthr || (h == htie && p <= pstar)) ? 1 : 0;
    }
    if (__ballot(cnt > 0) == 0ull) return;
    int64_t base = 0;
    if (cnt > 0) base = atomicAdd(&counts[q], cnt);
    const int64_t cap = cnt > 0 ? min((int64_t)cnt, Tq - base) : 0;  // never past the list
    int32_t *out = cand + (valid ? q * Tq + base : 0);
    int64_t w = 0;
    for (p = p0; p + 16 <= p1; p += 16) {
        uint32_t cc[16 * W];
#pragma unroll
        for (int u = 0; u < 16 * W; ++u) cc[u] = codes_l[p * W + u];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            int h = __popc(cc[u * W] ^ q0);
            if (W == 2) h += __popc(cc[u * W + 1] ^ q1);
            const bool e = h <= hthr || (h == htie && p + u <= pstar);
            if (e && w < cap) out[w] = (int32_t)(p + u);
            w += e ? 1 : 0;
        }
    }
    for (; p < p1; ++p) {
        int h = __popc(codes_l[p * W] ^ q0);
        if (W == 2) h += __popc(codes_l[p * W + 1] ^ q1);
        const bool e = h <= hthr || (h == htie && p <= pstar);
        if (e && w < cap) out[w] = (int32_t)p;
        w += e ? 1 : 0;
    }
}

// ---------------------------------------------------------------- fill
// words 32-bit words of p set to v (a kernel rather than a memset, so that a
// caller may capture the launches in a graph).
__global__ __launch_bounds__(256) void k_fill32(uint32_t *__restrict__ p, int64_t words, uint32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (int64_t)gridDim.x * 256)
        p[i] = v;
}

// ---------------------------------------------------------------- staged pass 1
// Pass 1 with an exact early exit in descending norm order (the norm ranging
// of Section 3.2 applied to the multi-probe of Section 3.3).  The largest
// similarity any bucket of sub-dataset j can reach is U_j cos(0) = U_j, so
// with the sub-datasets ordered by (U_j desc, j desc) -- jord -- every bucket
// of the sub-datasets not yet scanned ranks after bucket (jord[S], L), whose
// rank R[jord[S]][L] is the cut.  Once a query's buckets ranked before the cut
// hold Tq items, its threshold bucket lies among them and the rest of its
// histogram is never read; a tile skips the later stages once all its queries
// are there (need[tile] = 0), leaving those histogram entries zero.
//
// One block of SH_WAVES waves per (64-query tile, chunk of one sub-dataset):
// the waves share the tile's LDS histogram (lane = query column) and take the
// chunk's 16-item groups in turn; the block adds its nonzero counts into
// ghist (zeroed by the caller).  chunks: (sub-dataset, first, end) triples.
constexpr int SH_WAVES = 4;

template <int W>
__device__ __forceinline__ void load_group16(const uint32_t *__restrict__ codes_l, int64_t p,
                                             uint32_t (&c)[16 * W])
{
#pragma unroll
    for (int u = 0; u < 16 * W; ++u) c[u] = codes_l[p * W + u];
}

template <int W>
__device__ __forceinline__ void hist_group16(const uint32_t (&c)[16 * W], uint32_t q0, uint32_t q1,
                                             uint32_t *hist, int lane)
{
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        uint32_t h = (uint32_t)__popc(c[u * W] ^ q0);
        if (W == 2) h += (uint32_t)__popc(c[u * W + 1] ^ q1);
        __hip_atomic_fetch_add(&hist[h * 64 + lane], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

template <int W>
__global__ __launch_bounds__(SH_WAVES * 64) void k_scan_hist_s(const uint32_t *__restrict__ codes_l,
                                                               const uint32_t *__restrict__ qcodes,
                                                               int64_t nq, int m, int L, int qsets,
                                                               const int32_t *__restrict__ chunks,
                                                               const int32_t *__restrict__ need,
                                                               uint32_t *__restrict__ ghist,
                                                               unsigned long long *__restrict__ npairs,
                                                               int gstride)
{
    extern __shared__ uint32_t hist[];  // (L+1) x 64, column = lane
    // the wave number is wave-uniform: read it as such so that the item codes
    // come through the scalar cache
    const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int64_t tile = blockIdx.x;
    if (need && need[tile] == 0) return;  // every query of the tile is settled
    const int j = chunks[3 * blockIdx.y];
    const int64_t p0 = chunks[3 * blockIdx.y + 1], p1 = chunks[3 * blockIdx.y + 2];
    if (npairs && tid == 0)
        atomicAdd(npairs, (unsigned long long)(min((int64_t)64, nq - tile * 64) * (p1 - p0)));
    const int64_t q = tile * 64 + lane;
    uint32_t q0 = 0, q1 = 0;
    if (q < nq) {
        const int64_t r = qrow(q, j, qsets);
        q0 = qcodes[r * W];
        if (W == 2) q1 = qcodes[r * W + 1];
    }
    const int nh = (L + 1) * 64;
    for (int e = tid; e < nh; e += SH_WAVES * 64) hist[e] = 0u;
    __syncthreads();
    const int64_t ng = (p1 - p0) >> 4;  // whole 16-item groups
    // gstride > 1: a sample, every gstride-th group (no partial group)
    const int64_t g0 = (int64_t)wave * gstride, gs = (int64_t)SH_WAVES * gstride;
    // the codes of the wave's next group are loaded while this one is counted
    uint32_t c[16 * W], cn[16 * W];
    if (g0 < ng) load_group16<W>(codes_l, p0 + g0 * 16, c);
    // wait for the first group here (lgkmcnt(0)), so that the loop body only
    // waits for its prefetch after counting, not at its top
    __builtin_amdgcn_s_waitcnt(0xC07F);
    for (int64_t g = g0; g < ng; g += gs) {
        if (g + gs < ng) load_group16<W>(codes_l, p0 + (g + gs) * 16, cn);
        hist_group16<W>(c, q0, q1, hist, lane);
#pragma unroll
        for (int u = 0; u < 16 * W; ++u) c[u] = cn[u];
    }
    if (gstride == 1 && wave == SH_WAVES - 1) {
        for (int64_t p = p0 + ng * 16; p < p1; ++p) {
            uint32_t h = (uint32_t)__popc(codes_l[p * W] ^ q0);
            if (W == 2) h += (uint32_t)__popc(codes_l[p * W + 1] ^ q1);
            __hip_atomic_fetch_add(&hist[h * 64 + lane], 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __syncthreads();
    uint32_t *out = ghist + ((tile * m + j) * (int64_t)(L + 1)) * 64;
    for (int e = tid; e < nh; e += SH_WAVES * 64) {
        const uint32_t v = hist[e];
        if (v) atomicAdd(&out[e], v);
    }
}

// need[tile] = 0 once every query of the tile has at least Tq items in the
// buckets ranked before `cut` (walked in probing order through inv).
__global__ __launch_bounds__(64) void k_stage_check(const uint32_t *__restrict__ ghist,
                                                    const int32_t *__restrict__ inv, int64_t nq, int m,
                                                    int L, int64_t Tq, int cut, int32_t *__restrict__ need)
{
    const int lane = threadIdx.x;
    const int64_t tile = blockIdx.x;
    if (need[tile] == 0) return;
    const int64_t q = tile * 64 + lane;
    const int64_t P = (int64_t)m * (L + 1);
    const uint32_t *H = ghist + tile * P * 64;
    int64_t sum = 0;
    bool ok = q >= nq;
    for (int b = 0; b < cut; b += 16) {
        if (__ballot(!ok) == 0ull) break;
        uint32_t c[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) c[u] = (b + u < cut) ? H[(int64_t)inv[b + u] * 64 + lane] : 0u;
#pragma unroll
        for (int u = 0; u < 16; ++u) sum += c[u];
        ok = ok || sum >= Tq;
    }
    const uint64_t open = __ballot(!ok);
    if (lane == 0) need[tile] = open != 0ull ? 1 : 0;
}

// ---------------------------------------------------------------- chunked pass 2
// Pass 2 over the same (sub-dataset, first, end) chunks as the staged pass 1:
// one block of SH_WAVES waves per (64-query tile, chunk), the waves taking the
// chunk's 16-item groups in turn.  A lane (query) keeps its probed items --
// h <= hthr, or h = h* of the threshold bucket at a stored position up to
// P* (k_tie_locate) -- in its own LDS column of EM_SB entries and, when the
// column is full and at the end, reserves room in the query's list with one
// atomic on counts[q] (zeroed by the caller) and writes them there.  The
// probed set does not depend on the order of the appends (the list order
// does; the re-rank's tie rule makes the top-k independent of it).
constexpr int EM_SB = 16;

__device__ __forceinline__ void emit_flush(int32_t *__restrict__ stage, int lane, int cnt,
                                           int32_t *__restrict__ counts, int32_t *__restrict__ cand,
                                           int64_t q, int64_t Tq)
{
    const int64_t base = atomicAdd(&counts[q], cnt);
    const int64_t lim = min((int64_t)cnt, Tq - base);  // never past the list
    int32_t *out = cand + q * Tq + base;
    for (int i = 0; i < lim; ++i) out[i] = stage[i * 64 + lane];
}

template <int W>
__global__ __launch_bounds__(SH_WAVES * 64) void k_scan_emit_s(const uint32_t *__restrict__ codes_l,
                                                               const uint32_t *__restrict__ qcodes,
                                                               int64_t nq, int m, int64_t Tq, int qsets,
                                                               const int32_t *__restrict__ chunks,
                                                               const int32_t *__restrict__ ghthr,
                                                               const int32_t *__restrict__ gtie,
                                                               const int32_t *__restrict__ gpstar,
                                                               int32_t *__restrict__ counts,
                                                               int32_t *__restrict__ cand)
{
    __shared__ int32_t stage_s[SH_WAVES][EM_SB * 64];
    const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int64_t tile = blockIdx.x;
    const int j = chunks[3 * blockIdx.y];
    const int64_t p0 = chunks[3 * blockIdx.y + 1], p1 = chunks[3 * blockIdx.y + 2];
    const int64_t q = tile * 64 + lane;
    const bool valid = q < nq;
    int hthr = -1, htie = -1;
    int64_t pstar = -1;
    uint32_t q0 = 0, q1 = 0;
    if (valid) {
        const int32_t *tie = gtie + tile * 4 * 64;
        hthr = ghthr[(tile * m + j) * 64 + lane];
        if (tie[lane] == j) {
            htie = tie[64 + lane];
            pstar = gpstar[q];
        }
        const int64_t r = qrow(q, j, qsets);
        q0 = qcodes[r * W];
        if (W == 2) q1 = qcodes[r * W + 1];
    }
    if (__ballot(hthr >= 0 || htie >= 0) == 0ull) return;  // the same for every wave of the block
    int32_t *stage = stage_s[wave];
    int cnt = 0;
    // h <= hthr  <=>  h - (hthr + 1) < 0: the popcounts accumulate onto
    // -(hthr + 1) and the sign bit is the probe decision
    const uint32_t negt = (uint32_t)(-(hthr + 1));
    const bool anytie = __ballot(htie >= 0) != 0ull;  // the threshold bucket of some query is here
    const int64_t ng = (p1 - p0) >> 4;
    uint32_t c[16 * W], cn[16 * W];
    if (wave < ng) load_group16<W>(codes_l, p0 + (int64_t)wave * 16, c);
    for (int64_t g = wave; g < ng; g += SH_WAVES) {
        const int64_t p = p0 + g * 16;
        if (g + SH_WAVES < ng) load_group16<W>(codes_l, p + SH_WAVES * 16, cn);
        uint32_t mask = 0;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            uint32_t hd = (uint32_t)__popc(c[u * W] ^ q0) + negt;
            if (W == 2) hd += (uint32_t)__popc(c[u * W + 1] ^ q1);
            mask |= (hd >> 31) << u;
        }
        if (anytie) {
            // h = h* at a stored position up to P*: items u <= P* - p of the group
            const int64_t ul = pstar - p;
            const uint32_t tmask = ul < 0 ? 0u : (ul >= 15 ? 0xFFFFu : ((2u << ul) - 1u));
            uint32_t mt = 0;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                int h = __popc(c[u * W] ^ q0);
                if (W == 2) h += __popc(c[u * W + 1] ^ q1);
                mt |= (uint32_t)(h == htie) << u;
            }
            mask |= mt & tmask;
        }
        while (mask != 0u) {  // rare: a few per cent of the items are probed
            const int u = __builtin_ctz(mask);
            mask &= mask - 1u;
            stage[cnt * 64 + lane] = (int32_t)(p + u);
            if (++cnt == EM_SB) {
                emit_flush(stage, lane, cnt, counts, cand, q, Tq);
                cnt = 0;
            }
        }
#pragma unroll
        for (int u = 0; u < 16 * W; ++u) c[u] = cn[u];
    }
    if (wave == SH_WAVES - 1) {
        for (int64_t p = p0 + ng * 16; p < p1; ++p) {
            int h = __popc(codes_l[p * W] ^ q0);
            if (W == 2) h += __popc(codes_l[p * W + 1] ^ q1);
            if (h <= hthr || (h == htie && p <= pstar)) {
                stage[cnt * 64 + lane] = (int32_t)p;
                if (++cnt == EM_SB) {
                    emit_flush(stage, lane, cnt, counts, cand, q, Tq);
                    cnt = 0;
                }
            }
        }
    }
    if (cnt > 0) emit_flush(stage, lane, cnt, counts, cand, q, Tq);
}

// ---------------------------------------------------------------- collecting scan
// One scan in place of the two passes when each query has a guessed cut
// rho_q (a bucket rank, from a sample): every item whose bucket (j, h) ranks
// before rho_q -- h <= hcut(q, j), the sub-dataset's deepest such level,
// since ranks grow with h inside a sub-dataset -- is appended to the query's
// list of keys rank << 32 | stored position and counted in ghist, the
// per-query bucket histogram of the collected items (zeroed by the caller).
// When a query collects at least Tq items, its first Tq items in probing
// order (bucket rank, then stored position) are all among them, and the
// threshold pass over ghist plus a filter of the keys give exactly its
// probed set; otherwise (or past `cap` keys) the caller probes it again
// with the two passes.  Blocks: (64-query tile, chunk) as in k_scan_emit_s.
// The sub-datasets j in [jh0, jh1) -- those the re-rank screens whole on the
// matrix cores -- are only counted: their hits enter the histogram (the
// threshold needs them) but not the keys.
// The scan runs on the matrix cores.  With a_k in {0, 1} the bits of
// an item's code and t_k = 1 - 2 q_k the query's bits as +-1, the integer dot
// product sum_k a_k t_k = popc(c) - 2 popc(c & q) = h - popc(q), so one
// v_mfma_i32_32x32x32_i8 per 32 code bits gives the Hamming distances of 32
// items x 32 queries; the accumulators start at popc(q) - hcut - 1, so that
// an item is collected exactly when its accumulator ends negative (h <= hcut),
// and its level is h = acc + hcut + 1.  A wave takes 32 items at a time
// against both 32-query halves of the tile (lane l: query 32 c + (l & 31) of
// half c; rows 8 (r / 4) + 4 (l / 32) + r % 4 of accumulator r); the sign
// bits become a per-lane row mask with one funnel shift each and the low
// bytes of the accumulators are packed four to a word, from which a hit's
// level is read back.  Hits are staged in LDS as 16-bit offsets in the chunk
// (chunks hold fewer than 2^16 items) plus their level, and counted per
// (query, level) in 16-bit halves of the block's histogram words.
typedef int int32x4_t __attribute__((ext_vector_type(4)));
typedef int int32x16_t __attribute__((ext_vector_type(16)));
constexpr int MX_SB = 24;  // staged hits per (lane, query half)

// byte s of the result = bit s of the low 16 bits of v (0 or 1)
__device__ __forceinline__ int32x4_t bits16_to_bytes(uint32_t v)
{
    int32x4_t r;
#pragma unroll
    for (int n = 0; n < 4; ++n) r[n] = (int)((((v >> (4 * n)) & 0xFu) * 0x00204081u) & 0x01010101u);
    return r;
}

// Every lane empties its staged hits of one query half into the query's keys:
// the reservation (one atomic for the two lanes of a query) is issued first,
// the keys are formed (levels counted in the LDS histogram, ranks read from
// the R row) while it is in flight, then stored.  Called by the whole wave.
__device__ __forceinline__ void collect_flush_mx(const uint16_t *__restrict__ so, const uint8_t *__restrict__ sh,
                                                 int lane, int cnt, int L, const int32_t *__restrict__ Rrow,
                                                 uint32_t *hist, int col, int32_t *__restrict__ counts,
                                                 uint64_t *__restrict__ keys, int64_t q, int64_t cap, int64_t p0)
{
    // lanes l and l + 32 hold the same query: one reservation for both
    const int other = __shfl_xor(cnt, 32, 64);
    int b = 0;
    if (lane < 32 && cnt + other > 0) b = atomicAdd(&counts[q], cnt + other);
    b = __shfl(b, lane & 31, 64);
    const int64_t base = lane < 32 ? b : b + other;
    int top = cnt;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) top = max(top, __shfl_xor(top, o, 64));
    const uint32_t inc = 1u << (16 * (col & 1)), hc = (uint32_t)(col >> 1);
    for (int i0 = 0; i0 < top; i0 += 8) {
        uint64_t kv[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            kv[v] = ~0ull;
            if (i0 + v < cnt) {
                const int e = (i0 + v) * 64 + lane;
                const int h = min((int)sh[e], L);  // a hit's level is at most its query's cut, <= L
                __hip_atomic_fetch_add(&hist[h * 32 + hc], inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                kv[v] = ((uint64_t)(uint32_t)Rrow[L - h] << 32) | (uint32_t)(p0 + so[e]);
            }
        }
#pragma unroll
        for (int v = 0; v < 8; ++v)
            if (i0 + v < cnt && base + i0 + v < cap) keys[q * cap + base + i0 + v] = kv[v];
    }
}

template <int W>
__global__ __launch_bounds__(SH_WAVES * 64) void k_scan_collect_mx(const uint32_t *__restrict__ codes_l,
                                                                   const uint32_t *__restrict__ qcodes,
                                                                   int64_t nq, int m, int L, int qsets,
                                                                   const int32_t *__restrict__ chunks,
                                                                   const int32_t *__restrict__ R,
                                                                   const int32_t *__restrict__ grho,
                                                                   int64_t cap, int32_t *__restrict__ counts,
                                                                   uint64_t *__restrict__ keys,
                                                                   uint32_t *__restrict__ ghist,
                                                                   unsigned long long *__restrict__ npairs,
                                                                   int jh0, int jh1)
{
    // hist (L+1) x 32 words (queries 2 w, 2 w + 1 in the low / high halves) |
    // staged offsets SH_WAVES x 2 x MX_SB x 64 (u16) | staged levels (u8) | R row
    extern __shared__ uint32_t lds[];
    uint32_t *hist = lds;
    uint16_t *stage_o = reinterpret_cast<uint16_t *>(lds + (L + 1) * 32);
    uint8_t *stage_h = reinterpret_cast<uint8_t *>(stage_o + SH_WAVES * 2 * MX_SB * 64);
    int32_t *Rrow = reinterpret_cast<int32_t *>(stage_h + SH_WAVES * 2 * MX_SB * 64);
    const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int64_t tile = blockIdx.x;
    const int j = chunks[3 * blockIdx.y];
    const int64_t p0 = chunks[3 * blockIdx.y + 1], p1 = chunks[3 * blockIdx.y + 2];
    const bool count_only = j >= jh0 && j < jh1;
    for (int e = tid; e <= L; e += SH_WAVES * 64) Rrow[e] = R[(int64_t)j * (L + 1) + e];
    __syncthreads();
    // per query of the tile (lane = query): its cut level and code
    int hq = -1;
    uint32_t w0 = 0, w1 = 0;
    {
        const int64_t q = tile * 64 + lane;
        if (q < nq) {
            const int32_t rho = grho[q];
            int lo = 0, hi = L + 1;  // #{h : rank(j, h) < rho}
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (Rrow[L - mid] < rho) lo = mid + 1;
                else hi = mid;
            }
            hq = lo - 1;
            const int64_t r = qrow(q, j, qsets);
            w0 = qcodes[r * W];
            if (W == 2) w1 = qcodes[r * W + 1];
        }
    }
    if (__ballot(hq >= 0) == 0ull) return;  // the same for every wave of the block
    if (npairs && tid == 0)
        atomicAdd(npairs, (unsigned long long)(min((int64_t)64, nq - tile * 64) * (p1 - p0)));
    for (int e = tid; e < (L + 1) * 32; e += SH_WAVES * 64) hist[e] = 0u;
    __syncthreads();

    const int hb = lane >> 5, col0 = lane & 31;
    int32x4_t bq[2][W];
    int init[2], hcut[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int src = 32 * c + col0;
        hcut[c] = __shfl(hq, src, 64);
        const uint32_t qa = __shfl(w0, src, 64);
        const uint32_t qb = W == 2 ? __shfl(w1, src, 64) : 0u;
        init[c] = __popc(qa) + __popc(qb) - hcut[c] - 1;
#pragma unroll
        for (int mm = 0; mm < W; ++mm) {
            const int32x4_t y = bits16_to_bytes(((mm == 0 ? qa : qb) >> (16 * hb)) & 0xFFFFu);
#pragma unroll
            for (int n = 0; n < 4; ++n) bq[c][mm][n] = (int)(0x01010101u + (uint32_t)y[n] * 0xFEu);  // +-1 bytes
        }
    }
    int32x16_t ini[2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) ini[c][r] = init[c];
    const int so0 = (wave * 2 + 0) * MX_SB * 64, so1 = (wave * 2 + 1) * MX_SB * 64;
    int cnt0 = 0, cnt1 = 0;
    const int64_t ng = (p1 - p0 + 31) >> 5;  // 32-item groups, the last one partial
    // codes of item min(p + col0, p1 - 1) of a group: loads stay inside the
    // chunk (rows past its end are masked out below)
    uint32_t a0, a1 = 0;
    {
        const int64_t pi = min(p0 + (int64_t)wave * 32 + col0, p1 - 1);
        a0 = codes_l[pi * W];
        if (W == 2) a1 = codes_l[pi * W + 1];
    }
    // vmcnt(0): the first group is in before the loop, whose body then waits
    // for its prefetch only at its end
    __builtin_amdgcn_s_waitcnt(0x0F70);
    for (int64_t g = wave; g < ng; g += SH_WAVES) {
        const int64_t p = p0 + g * 32;
        int32x4_t aa[W];
        aa[0] = bits16_to_bytes((a0 >> (16 * hb)) & 0xFFFFu);
        if (W == 2) aa[W - 1] = bits16_to_bytes((a1 >> (16 * hb)) & 0xFFFFu);
        // the next group's codes load while this one is matched
        {
            const int64_t pi = min(p + SH_WAVES * 32 + col0, p1 - 1);
            a0 = codes_l[pi * W];
            if (W == 2) a1 = codes_l[pi * W + 1];
        }
        // rows past the chunk's end (last group only) are never collected
        uint32_t vmask = 0xFFFFu;
        if (p + 32 > p1) {
            vmask = 0u;
#pragma unroll
            for (int r = 0; r < 16; ++r) vmask |= (uint32_t)(p + 8 * (r >> 2) + 4 * hb + (r & 3) < p1) << r;
        }
        const int gofs = (int)(p - p0) + 4 * hb;  // chunk offset of row 0 of this lane
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            int32x16_t acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(aa[0], bq[c][0], ini[c], 0, 0, 0);
#pragma unroll
            for (int mm = 1; mm < W; ++mm) acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(aa[mm], bq[c][mm], acc, 0, 0, 0);
            uint32_t mask = 0u;
#pragma unroll
            for (int r = 15; r >= 0; --r) mask = __builtin_amdgcn_alignbit(mask, (uint32_t)acc[r], 31);
            mask &= vmask;
            if (count_only) {
                // level h = acc + hcut + 1 of each hit counted straight into
                // the histogram word of (h, query 32 c + col0); the other rows
                // add 0 to a word of their own level (h <= L), so no branches
                const uint32_t inc = 1u << (16 * (col0 & 1));
                const int hw = (hcut[c] + 1) * 32 + 16 * c + (col0 >> 1);
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    __hip_atomic_fetch_add(&hist[acc[r] * 32 + hw], ((mask >> r) & 1u) * inc, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                continue;
            }
            // low bytes of the accumulators, four to a word (byte r & 3 of word r >> 2)
            uint32_t pk[4];
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const uint32_t lo = __builtin_amdgcn_perm((uint32_t)acc[4 * w + 1], (uint32_t)acc[4 * w], 0x0C0C0400u);
                const uint32_t hi = __builtin_amdgcn_perm((uint32_t)acc[4 * w + 3], (uint32_t)acc[4 * w + 2], 0x0C0C0400u);
                pk[w] = __builtin_amdgcn_perm(hi, lo, 0x05040100u);
            }
            const int sbase = c == 0 ? so0 : so1;
            int cnt = c == 0 ? cnt0 : cnt1;
            while (mask != 0u) {
                const int r = __builtin_ctz(mask);
                mask &= mask - 1u;
                const uint32_t wsel = (r & 8) ? ((r & 4) ? pk[3] : pk[2]) : ((r & 4) ? pk[1] : pk[0]);
                const int acc_lo = (int)((wsel >> (8 * (r & 3))) & 0xFFu);  // acc + 256 (acc in [-256, -1])
                const int e = sbase + cnt * 64 + lane;
                stage_o[e] = (uint16_t)(gofs + 8 * (r >> 2) + (r & 3));
                stage_h[e] = (uint8_t)(acc_lo - 256 + hcut[c] + 1);
                ++cnt;
            }
            if (c == 0) cnt0 = cnt;
            else cnt1 = cnt;
        }
        // at most 16 more per half and group: room is left while every count is <= MX_SB - 16
        if (__ballot(cnt0 > MX_SB - 16 || cnt1 > MX_SB - 16) != 0ull) {
            collect_flush_mx(stage_o + so0, stage_h + so0, lane, cnt0, L, Rrow, hist, col0, counts, keys,
                             tile * 64 + col0, cap, p0);
            collect_flush_mx(stage_o + so1, stage_h + so1, lane, cnt1, L, Rrow, hist, 32 + col0, counts, keys,
                             tile * 64 + 32 + col0, cap, p0);
            cnt0 = cnt1 = 0;
        }
    }
    if (__ballot(cnt0 > 0 || cnt1 > 0) != 0ull) {
        collect_flush_mx(stage_o + so0, stage_h + so0, lane, cnt0, L, Rrow, hist, col0, counts, keys,
                         tile * 64 + col0, cap, p0);
        collect_flush_mx(stage_o + so1, stage_h + so1, lane, cnt1, L, Rrow, hist, 32 + col0, counts, keys,
                         tile * 64 + 32 + col0, cap, p0);
    }
    __syncthreads();
    uint32_t *out = ghist + ((tile * m + j) * (int64_t)(L + 1)) * 64;
    for (int e = tid; e < (L + 1) * 32; e += SH_WAVES * 64) {
        const uint32_t v = hist[e];
        if (v == 0u) continue;
        const int h = e >> 5, qq = 2 * (e & 31);
        if (v & 0xFFFFu) atomicAdd(&out[h * 64 + qq], v & 0xFFFFu);
        if (v >> 16) atomicAdd(&out[h * 64 + qq + 1], v >> 16);
    }
}

// The probed list of each query from its collected keys: rank < b*, or
// rank = b* and stored position <= P* (k_threshold, k_tie_locate).  One
// block per query; the list order is that of arrival (the re-rank's tie rule
// makes the top-k independent of it).  lcount[q] receives the list length
// (Tq when the query's collection was complete and no sub-dataset was only
// counted); `fail` (one word per call batch) is set when a query's threshold
// bucket does not rank before its guessed cut rho (the items ranked before
// rho number fewer than Tq: the histogram of the collected items then never
// reaches the budget) or it collected more keys than cap.
__global__ __launch_bounds__(256) void k_collect_filter(const uint64_t *__restrict__ keys,
                                                        const int32_t *__restrict__ counts, int64_t cap,
                                                        const int32_t *__restrict__ gtie,
                                                        const int32_t *__restrict__ gpstar,
                                                        const int32_t *__restrict__ grho, int64_t Tq,
                                                        int32_t *__restrict__ cand,
                                                        int32_t *__restrict__ lcount,
                                                        uint32_t *__restrict__ fail)
{
    __shared__ int32_t total;
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t q = blockIdx.x;
    const int32_t *tie = gtie + (q >> 6) * 4 * 64;
    const uint32_t bstar = (uint32_t)tie[3 * 64 + (q & 63)];
    const uint32_t pstar = (uint32_t)gpstar[q];  // INT_MAX: the whole bucket
    const int64_t C = counts[q];
    const int64_t E = min(C, cap);
    if (tid == 0) {
        total = 0;
        if ((int64_t)bstar >= (int64_t)grho[q] || C > cap) atomicOr(fail, 1u);
    }
    __syncthreads();
    const uint64_t *kq = keys + q * cap;
    for (int64_t e0 = 0; e0 < E; e0 += 256) {
        const int64_t e = e0 + tid;
        bool keep = false;
        uint32_t pos = 0;
        if (e < E) {
            const uint64_t key = kq[e];
            const uint32_t rank = (uint32_t)(key >> 32);
            pos = (uint32_t)key;
            keep = rank < bstar || (rank == bstar && pos <= pstar);
        }
        const uint64_t kb = __ballot(keep);
        if (kb != 0ull) {
            const int leader = __ffsll((long long)kb) - 1;
            int base = 0;
            if (lane == leader) base = atomicAdd(&total, __popcll(kb));
            base = __shfl(base, leader, 64);
            const int64_t slot = base + __popcll(kb & ((1ull << lane) - 1ull));
            if (keep && slot < Tq) cand[q * Tq + slot] = (int32_t)pos;
        }
    }
    __syncthreads();
    if (tid == 0) lcount[q] = total;
}

// ---------------------------------------------------------------- rerank
// One wave per (query, slice of its probed list); the rows of 64 candidates
// at a time are summed in FP64 (dev::ip64_rows_fp32), the running top-k kept by
// dev::WaveTopK.  With several slices per query, each slice writes a partial
// list and k_topk_merge combines them.
using dev::RR_STRIDE;
using dev::WaveTopK;

// The slices of a query share the largest k-th value any of them has reached
// (gtheta, order-preserving encoding, 0 = none yet): the k items behind it
// have inner products at least that large, so it bounds the query's k-th best.
using dev::order_key;
using dev::order_value;

template <int S>
__global__ __launch_bounds__(64) void k_rerank(const float *__restrict__ Xl,
                                               const int32_t *__restrict__ perm,
                                               const float *__restrict__ Q, int64_t n, int d,
                                               int dp, int64_t Tq, int k,
                                               const int32_t *__restrict__ cand,
                                               const int32_t *__restrict__ counts, int nsplit,
                                               int64_t slice, int64_t *__restrict__ out_ids,
                                               float *__restrict__ out_ips,
                                               double *__restrict__ part_v,
                                               int32_t *__restrict__ part_i,
                                               unsigned long long *__restrict__ gtheta)
{
    __shared__ float tile[64 * RR_STRIDE];
    const int lane = threadIdx.x;
    const int64_t q = blockIdx.x;
    const int split = blockIdx.y;
    const float *qv = Q + q * d;
    const int32_t *cq = cand + q * Tq;
    // lists with their own lengths are cut into nsplit equal slices each
    const int64_t len = counts ? min((int64_t)counts[q], Tq) : Tq;
    const int64_t sl = counts ? ((len + nsplit - 1) / nsplit + 63) / 64 * 64 : slice;
    const int64_t cbeg = (int64_t)split * sl;
    const int64_t cend = min(len, cbeg + sl);
    WaveTopK<S> top;
    top.init(k);

    // the positions of the next 64 candidates are loaded one batch ahead
    int32_t pn = (cbeg + lane < cend) ? cq[cbeg + lane] : -1;
    for (int64_t c0 = cbeg; c0 < cend; c0 += 64) {
        int32_t p = pn;
        pn = (c0 + 64 + lane < cend) ? cq[c0 + 64 + lane] : -1;
        bool valid = c0 + lane < cend;
        int32_t id = 0;
        valid = valid && p >= 0 && (int64_t)p < n;  // positions come from the scan; never trust blindly
        if (valid) id = perm[p];
        else p = 0;
        const double acc = dev::ip64_rows_fp32(Xl, d, dp, qv, p, valid, lane, tile);
        // values below the best k-th value any slice of the query has reached
        // cannot enter the query's top-k
        double floor = -INFINITY;
        if (gtheta) {
            const unsigned long long ge =
                __hip_atomic_load(&gtheta[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (ge != 0ull) floor = order_value(ge);
        }
        top.offer(acc, id, valid, lane, floor);
        if (gtheta && top.th_v > -INFINITY && top.th_v > floor && lane == 0)
            atomicMax(&gtheta[q], (unsigned long long)order_key(top.th_v));
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int e = s * 64 + lane;
        if (e < k) {
            if (nsplit == 1) {
                out_ids[q * k + e] = top.ti[s] == INT_MAX ? -1 : (int64_t)top.ti[s];
                out_ips[q * k + e] = (float)top.tv[s];
            } else {
                const int64_t o = (q * nsplit + split) * k + e;
                part_v[o] = top.tv[s];
                part_i[o] = top.ti[s];
            }
        }
    }
}

// Merge the nsplit partial top-k lists of each query (one wave per query).
// First pass of the gather re-rank over the bfloat16 rows Xh (the precision
// form's re-rank copy): one wave per (query, slice of its probed list).  The
// order of the sum does not matter here -- only a rigorous bound is needed --
// so 16 lanes share a row, 8 coordinates each per 128-coordinate segment (a
// load instruction brings four rows x 256 contiguous bytes), and the FP32
// partial sums are reduced across the 16 lanes by shuffles (no LDS tile).
// ip~ (FP32 products of q and bf16(x), FP32 sums in any order) satisfies
// |ip~ - q.x| <= ||q|| (||x - bf16(x)|| + (d + 8) 2^-23 ||x||) <= ||q|| xeb;
// with e = ||q|| xeb (1 + 2^-20) the wave keeps a top-k of the lower bounds
// ip~ - e and appends every candidate whose upper bound ip~ + e reaches the
// k-th lower bound (the largest any slice of the query has published in
// gtheta) to the query's list (lists: nq x lcap, lcount per query, may
// exceed lcap): a superset of the exact top-k, re-ranked afterwards from the
// FP32 rows.
// One step of the transposing butterfly: H = half the number of live sums;
// the lane whose bit H is set keeps sums [H, 2H), the other [0, H).
template <int H>
__device__ __forceinline__ void reduce_half(float (&a)[16], int upper)
{
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const float keep = upper ? a[i + H] : a[i];
        const float send = upper ? a[i] : a[i + H];
        a[i] = keep + __shfl_xor(send, H, 64);
    }
}

template <int S>
__global__ __launch_bounds__(64, S <= 2 ? 4 : 1) void k_rerank_bf16(const uint16_t *__restrict__ Xh,
                                                    const float *__restrict__ xeb,
                                                    const float *__restrict__ Q, int64_t n, int d, int dp,
                                                    int64_t Tq, int k, const int32_t *__restrict__ cand,
                                                    const int32_t *__restrict__ counts,
                                                    int64_t slice, int lcap, int32_t *__restrict__ lcount,
                                                    int32_t *__restrict__ lists,
                                                    unsigned long long *__restrict__ gtheta)
{
    extern __shared__ float qs[];  // q, zero past d up to a multiple of 128
    const int lane = threadIdx.x;
    const int64_t q = blockIdx.x;
    const int split = blockIdx.y;
    const float *qv = Q + q * d;
    const int32_t *cq = cand + q * Tq;
    // lists with their own lengths (counts) are cut into gridDim.y equal slices each
    const int64_t len = counts ? min((int64_t)counts[q], Tq) : Tq;
    const int64_t ns = gridDim.y;
    const int64_t qsl = counts ? ((len + ns - 1) / ns + 63) / 64 * 64 : slice;
    const int64_t cbeg = (int64_t)split * qsl;
    const int64_t cend = min(len, cbeg + qsl);
    if (cbeg >= cend) return;
    double qn = 0.0;  // ||q|| (exact squares, FP64 sum, rounded up)
    const int dq = (dp + 127) / 128 * 128;
    for (int t = lane; t < dq; t += 64) {
        const float v = t < d ? qv[t] : 0.f;
        qs[t] = v;
        qn += (double)v * (double)v;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) qn += __shfl_xor(qn, o, 64);
    qn = __builtin_sqrt(qn) * (1.0 + 0x1p-40);
    __syncthreads();
    WaveTopK<S> top;
    top.init(k);
    const int grp = lane >> 4, sl = lane & 15;
    int32_t pn = (cbeg + lane < cend) ? cq[cbeg + lane] : -1;
    for (int64_t c0 = cbeg; c0 < cend; c0 += 64) {
        // the largest k-th lower bound published for the query so far (by
        // another slice, or the seed of a dense screen): values below it can
        // neither raise it nor enter the top-k that matters
        const unsigned long long ge = __hip_atomic_load(&gtheta[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int32_t p = pn;
        pn = (c0 + 64 + lane < cend) ? cq[c0 + 64 + lane] : -1;
        bool valid = c0 + lane < cend;
        valid = valid && p >= 0 && (int64_t)p < n;  // positions come from the scan; never trust blindly
        if (!valid) p = 0;
        const int32_t pv = valid ? p : -1;
        float part[16];
#pragma unroll
        for (int g = 0; g < 16; ++g) part[g] = 0.f;
        for (int s0 = 0; s0 < dp; s0 += 128) {
            const int c = s0 + 8 * sl;
            u16x8 v[16];
#pragma unroll
            for (int g = 0; g < 16; ++g) {
                const int32_t pr = __shfl(pv, 4 * g + grp, 64);
                v[g] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
                if (pr >= 0 && c < dp) v[g] = *reinterpret_cast<const u16x8 *>(Xh + (int64_t)pr * dp + c);
            }
            const floatx4 qa = *reinterpret_cast<const floatx4 *>(&qs[c]);
            const floatx4 qb = *reinterpret_cast<const floatx4 *>(&qs[c + 4]);
#pragma unroll
            for (int g = 0; g < 16; ++g) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    part[g] = __builtin_fmaf(qa[e], __uint_as_float((uint32_t)v[g][e] << 16), part[g]);
                    part[g] = __builtin_fmaf(qb[e], __uint_as_float((uint32_t)v[g][4 + e] << 16), part[g]);
                }
            }
        }
        // transposing butterfly over the 16 lanes of a row group: at each step
        // a lane keeps half of its partial sums (the half its lane bit names)
        // and adds the partner's copy of that half, so that lane sl ends with
        // the full sum of row 4 sl + grp (15 exchanges instead of 60)
        reduce_half<8>(part, sl & 8);
        reduce_half<4>(part, sl & 4);
        reduce_half<2>(part, sl & 2);
        reduce_half<1>(part, sl & 1);
        // row c sits in lane 16 (c & 3) + (c >> 2)
        const double acc = (double)__shfl(part[0], 16 * (lane & 3) + (lane >> 2), 64);
        const double e = qn * (double)(valid ? xeb[p] : 0.f) * (1.0 + 0x1p-20);
        const double floor = ge != 0ull ? order_value(ge) : -INFINITY;
        // only the k-th value matters here, not which items hold it: the
        // stored position stands in for the id (no read of perm)
        top.offer(acc - e, p, valid, lane, floor);
        if (top.th_v > floor && lane == 0) atomicMax(&gtheta[q], (unsigned long long)order_key(top.th_v));
        const double th = fmax(top.th_v, floor);
        const bool keep = valid && !(acc + e < th);
        const uint64_t kb = __ballot(keep);
        if (kb != 0ull) {
            const int leader = __ffsll((long long)kb) - 1;
            int base = 0;
            if (lane == leader) base = atomicAdd(&lcount[q], __popcll(kb));
            base = __shfl(base, leader, 64);
            const int slot = base + __popcll(kb & ((1ull << lane) - 1ull));
            if (keep && slot < lcap) lists[q * lcap + slot] = p;
        }
    }
}

template <int S>
__global__ __launch_bounds__(64) void k_topk_merge(const double *__restrict__ part_v,
                                                   const int32_t *__restrict__ part_i, int nsplit,
                                                   int k, int64_t *__restrict__ out_ids,
                                                   float *__restrict__ out_ips)
{
    const int lane = threadIdx.x;
    const int64_t q = blockIdx.x;
    WaveTopK<S> top;
    top.init(k);
    const int64_t total = (int64_t)nsplit * k;
    const double *pv = part_v + q * total;
    const int32_t *pi = part_i + q * total;
    for (int64_t e0 = 0; e0 < total; e0 += 64) {
        const bool ok = e0 + lane < total && pi[min(e0 + lane, total - 1)] != INT_MAX;
        const double v = ok ? pv[e0 + lane] : -INFINITY;
        const int32_t id = ok ? pi[e0 + lane] : INT_MAX;
        top.offer(v, id, ok, lane);
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int e = s * 64 + lane;
        if (e < k) {
            out_ids[q * k + e] = top.ti[s] == INT_MAX ? -1 : (int64_t)top.ti[s];
            out_ips[q * k + e] = (float)top.tv[s];
        }
    }
}

// ---------------------------------------------------------------- tie locate
// Stored position of the r*-th item of the threshold bucket (j*, h*) of each
// query: with it the probed set becomes a per-pair predicate,
//   p in C_T  <=>  h <= hthr[q][j]  or  (j = j*, h = h*, p <= P*).
// One block per query walks sub-dataset j* from its first stored item in
// rounds of TL_WAVES x TL_GROUPS 64-item groups (each wave a contiguous 256
// items, its match masks kept in registers); the block adds up the round's
// matches and stops in the round that holds the r*-th one, whose wave reads
// the position off its masks.  The walk ends where r* falls instead of
// counting all of it first.  Given the tile histograms (ghist: the bucket's
// exact item count N* at [tile][j*][h*][query]), a cut past the middle,
// r* > N* / 2, is found from the other end, as the (N* - r* + 1)-th match
// counted from the last stored item, so that no walk covers more than about
// half of the sub-dataset.  A bucket that is probed whole (r* = INT_MAX)
// needs no walk.
constexpr int TL_WAVES = 16;
constexpr int TL_GROUPS = 4;

template <int W>
__global__ __launch_bounds__(TL_WAVES * 64) void k_tie_locate(const uint32_t *__restrict__ codes_l,
                                                              const int32_t *__restrict__ off,
                                                              const uint32_t *__restrict__ qcodes,
                                                              int64_t nq, int qsets,
                                                              const int32_t *__restrict__ gtie,
                                                              int32_t *__restrict__ gpstar,
                                                              const uint32_t *__restrict__ ghist, int m, int L)
{
    __shared__ int32_t cnt_s[2][TL_WAVES];  // per round (two buffers: one barrier per round)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t q = blockIdx.x;
    const int tile = (int)(q >> 6), ql = (int)(q & 63);
    const int32_t *tie = gtie + (int64_t)tile * 4 * 64;
    const int jstar = tie[ql], hstar = tie[64 + ql], rstar = tie[128 + ql];
    if (jstar < 0 || rstar == INT_MAX) {  // the same for the whole block: no barrier is skipped
        if (threadIdx.x == 0) gpstar[q] = jstar < 0 ? -1 : INT_MAX;
        return;
    }
    const int64_t r = qrow(q, jstar, qsets);
    const uint32_t q0 = qcodes[r * W], q1 = W == 2 ? qcodes[r * W + 1] : 0u;
    const int64_t ps = off[jstar], pe = off[jstar + 1];
    auto match = [&](int64_t p) {
        if (p >= pe) return false;
        int h = __popc(codes_l[p * W] ^ q0);
        if (W == 2) h += __popc(codes_l[p * W + 1] ^ q1);
        return h == hstar;
    };
    if (threadIdx.x == 0) gpstar[q] = -1;  // replaced below if the bucket holds r* items
    // from the back: the target is the rk-th match in descending stored order
    int rk = rstar;
    bool back = false;
    if (ghist) {
        const int L1 = L + 1;
        const int64_t nstar = ghist[(((int64_t)tile * m + jstar) * L1 + hstar) * 64 + ql];
        if (2 * (int64_t)rstar > nstar && rstar <= nstar) {
            back = true;
            rk = (int)(nstar - rstar + 1);
        }
    }
    constexpr int64_t RW = TL_WAVES * TL_GROUPS * 64;  // items per round
    int c = 0;  // matches before this round (in the walk's direction)
    const int64_t nrounds = (pe - ps + RW - 1) / RW;
    for (int64_t rd = 0; rd < nrounds; ++rd) {
        // round rd covers [p0, p0 + RW); walking back, the rounds are taken
        // from the last one down and, inside a round, the waves (and each
        // wave's groups and lanes) in descending order
        const int64_t p0 = back ? ps + (nrounds - 1 - rd) * RW : ps + rd * RW;
        const int wv = back ? TL_WAVES - 1 - wave : wave;  // this wave's place in the walk
        const int64_t pw = p0 + (int64_t)wave * TL_GROUPS * 64;
        uint64_t bal[TL_GROUPS];
        bool mt[TL_GROUPS];
#pragma unroll
        for (int u = 0; u < TL_GROUPS; ++u) mt[u] = match(pw + u * 64 + lane);
        int cw = 0;
#pragma unroll
        for (int u = 0; u < TL_GROUPS; ++u) {
            bal[u] = __ballot(mt[u]);
            cw += __popcll(bal[u]);
        }
        int32_t *cs = cnt_s[rd & 1];
        if (lane == 0) cs[wave] = cw;
        __syncthreads();
        int before = 0, tot = 0;
        for (int w = 0; w < TL_WAVES; ++w) {
            const int v = cs[w];
            const int place = back ? TL_WAVES - 1 - w : w;
            before += place < wv ? v : 0;
            tot += v;
        }
        if (c + tot >= rk) {  // the same for the whole block: the target match is in this round
            if (c + before < rk && c + before + cw >= rk) {
                int need = rk - c - before;  // 1-based rank inside this wave's matches, walk order
#pragma unroll
                for (int uu = 0; uu < TL_GROUPS; ++uu) {
                    const int u = back ? TL_GROUPS - 1 - uu : uu;
                    const int k = __popcll(bal[u]);
                    if (need > 0 && need <= k) {
                        // the need-th set bit from the low end, or from the high end walking back
                        const int below = __popcll(bal[u] & ((1ull << lane) - 1ull));
                        const int rank = back ? k - 1 - below : below;
                        const uint64_t sel = __ballot(((bal[u] >> lane) & 1ull) && rank == need - 1);
                        if (lane == 0) gpstar[q] = (int32_t)(pw + u * 64 + __ffsll((long long)sel) - 1);
                    }
                    need -= k;
                }
            }
            return;
        }
        c += tot;
    }
}

// ---------------------------------------------------------------- screen
// Query-tiled screen of the probed set on the FP32 matrix cores.  A block
// holds 64 queries (staged in LDS) and one chunk of stored items of a single
// sub-dataset; each wave computes 64 queries x 32 items per iteration with
// v_mfma_f32_16x16x4_f32 (queries = M, items = N).  With e = g ||q|| ||x||
// + 2^-100, g = 2 gamma_d (a bound on the rounding error of any summation
// order), every probed pair satisfies ip32 - e <= ip <= ip32 + e.
//   MAXMODE = true : writes, per (query, 32-item group of a cell), the
//                    largest lower bound ip32 - e over the group's probed items
//                    (-inf if none).  The k-th largest of these over distinct
//                    groups is a lower bound theta_q of the k-th best exact
//                    inner product.
//   MAXMODE = false: keeps every probed pair with not (ip32 + e < theta_q)
//                    and appends its stored position to the query's list
//                    (capacity cap; counts may exceed cap, which the host
//                    detects).  The exact top-k of the probed set lies in it.
// maximum over the 16 lanes of a DPP row (lanes 16 r .. 16 r + 15), in every
// lane of the row: two quad swaps, then the half-row and row mirrors, each
// a data-parallel move into v_max (no LDS crossbar traffic)
// LDS written by some lanes of a wave and read by others: the stores are
// complete (and not moved past this point) before the wave goes on
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float row16_max(float v)
{
    v = fmaxf(v, dpp_move<0xB1>(v));   // quad_perm [1, 0, 3, 2]
    v = fmaxf(v, dpp_move<0x4E>(v));   // quad_perm [2, 3, 0, 1]
    v = fmaxf(v, dpp_move<0x141>(v));  // row_half_mirror
    return fmaxf(v, dpp_move<0x140>(v));  // row_mirror
}

constexpr int SC_CHUNK = 4096;
constexpr int SC_CELL = 1024;
constexpr int SC_GROUPS = SC_CELL / 32;  // 32-item groups per cell (MAXMODE outputs)

template <int W, bool MAXMODE>
__global__ __launch_bounds__(256) void k_screen(
    const float *__restrict__ Xl, int d, int dp, const uint32_t *__restrict__ codes_l,
    const double *__restrict__ key_l, const float *__restrict__ Q, int64_t nq,
    const int32_t *__restrict__ chunks, int m, const uint32_t *__restrict__ qcodes,
    const int32_t *__restrict__ ghthr, const int32_t *__restrict__ gtie,
    const int32_t *__restrict__ gpstar, const float *__restrict__ theta, float gam, int cap,
    int32_t *__restrict__ counts, int32_t *__restrict__ lists, float *__restrict__ cmax,
    int ncol, int L, int qsets)
{
    extern __shared__ __align__(16) float qs[];  // 64 x qstride
    __shared__ float th_s[64], qn_s[64];
    __shared__ int32_t hthr_s[64], htie_s[64], pstar_s[64];
    __shared__ uint32_t qc_s[64 * W];
    __shared__ int any_s, all_s;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int tile = blockIdx.x;
    const int j = chunks[3 * blockIdx.y], pbeg = chunks[3 * blockIdx.y + 1],
              pend = chunks[3 * blockIdx.y + 2];
    const int qstride = dp + 4;
    const int64_t q0 = (int64_t)tile * 64;

    if (tid < 64) {
        const int64_t q = q0 + tid;
        int hthr = -1, htie = -1, pstar = -1;
        float th = -INFINITY;
        if (q < nq) {
            hthr = ghthr[((int64_t)tile * m + j) * 64 + tid];
            const int32_t *tie = gtie + (int64_t)tile * 4 * 64;
            if (tie[tid] == j) {
                htie = tie[64 + tid];
                pstar = gpstar[q];
            }
            if (!MAXMODE) th = theta[q];
#pragma unroll
            for (int w = 0; w < W; ++w) qc_s[tid * W + w] = qcodes[qrow(q, j, qsets) * W + w];
        }
        hthr_s[tid] = hthr;
        htie_s[tid] = htie;
        pstar_s[tid] = pstar;
        th_s[tid] = th;
        const uint64_t b = __ballot(hthr >= 0 || htie >= 0);
        const uint64_t a = __ballot(hthr >= L);  // every possible h passes
        if (tid == 0) {
            any_s = b != 0ull;
            all_s = a == ~0ull;
        }
    }
    __syncthreads();
    if (MAXMODE && tid < 64 && q0 + tid < nq) {  // groups this block never reaches stay -inf
        for (int gi = any_s ? (pend - pbeg + 31) / 32 : 0; gi < SC_GROUPS; ++gi)
            cmax[(q0 + tid) * ncol + blockIdx.y * SC_GROUPS + gi] = -INFINITY;
    }
    if (!any_s) return;  // no query of this tile probes this chunk

    // stage the query tile, zero-padded to dp columns
    for (int r = wave; r < 64; r += 4) {
        const int64_t q = q0 + r;
        for (int c = lane; c < dp; c += 64) qs[r * qstride + c] = (q < nq && c < d) ? Q[q * d + c] : 0.f;
    }
    __syncthreads();
    if (tid < 64) {  // an upper bound on ||q||: exact squares, FP64 sum, rounded up
        double s2 = 0.0;
        for (int c = 0; c < d; ++c) s2 += (double)qs[tid * qstride + c] * (double)qs[tid * qstride + c];
        qn_s[tid] = (float)__builtin_sqrt(s2) * (1.0f + 0x1p-18f);
    }
    __syncthreads();

    const int r16 = lane & 15, g = lane >> 4;
    const bool all = all_s != 0;
    for (int p0 = pbeg + wave * 32; p0 < pend; p0 += 128) {
        // this lane's two items (column blocks ib = 0, 1)
        int32_t pit[2];
        uint32_t cw[2][W];
        float xn[2];
        bool iv[2];
#pragma unroll
        for (int ib = 0; ib < 2; ++ib) {
            pit[ib] = p0 + 16 * ib + r16;
            iv[ib] = pit[ib] < pend;
            const int64_t pp = iv[ib] ? pit[ib] : pbeg;
#pragma unroll
            for (int w = 0; w < W; ++w) cw[ib][w] = codes_l[pp * W + w];
            xn[ib] = sqrtf((float)key_l[pp]) * (1.0f + 0x1p-18f);
        }
        floatx4 acc[4][2];
#pragma unroll
        for (int qb = 0; qb < 4; ++qb)
#pragma unroll
            for (int ib = 0; ib < 2; ++ib) acc[qb][ib] = floatx4{0.f, 0.f, 0.f, 0.f};
        for (int kk = 0; kk < dp; kk += 16) {
            const int kc = kk + 4 * g;
            floatx4 bx[2];
#pragma unroll
            for (int ib = 0; ib < 2; ++ib)
                bx[ib] = (iv[ib] && kc < dp)
                             ? *reinterpret_cast<const floatx4 *>(Xl + (int64_t)pit[ib] * dp + kc)
                             : floatx4{0.f, 0.f, 0.f, 0.f};
            floatx4 aq[4];
#pragma unroll
            for (int qb = 0; qb < 4; ++qb)
                aq[qb] = kc < dp ? *reinterpret_cast<const floatx4 *>(&qs[(16 * qb + r16) * qstride + kc])
                                 : floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                for (int qb = 0; qb < 4; ++qb)
#pragma unroll
                    for (int ib = 0; ib < 2; ++ib)
                        acc[qb][ib] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[qb][jj], bx[ib][jj],
                                                                           acc[qb][ib], 0, 0, 0);
        }
        // epilogue: lane holds C[q = 16 qb + 4 g + v][item = 16 ib + r16]
#pragma unroll
        for (int qb = 0; qb < 4; ++qb) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ql = 16 * qb + 4 * g + v;
                const int hthr = hthr_s[ql], htie = htie_s[ql];
                const float th = th_s[ql], qn = qn_s[ql];
                float gmax = -INFINITY;  // MAXMODE: this lane's two items for query ql
#pragma unroll
                for (int ib = 0; ib < 2; ++ib) {
                    bool probed = iv[ib];
                    if (!all) {
                        int h = __popc(cw[ib][0] ^ qc_s[ql * W]);
                        if (W == 2) h += __popc(cw[ib][1] ^ qc_s[ql * W + 1]);
                        probed = probed && (h <= hthr || (h == htie && pit[ib] <= pstar_s[ql]));
                    }
                    const float ip = acc[qb][ib][v];
                    const float e = gam * qn * xn[ib] + 0x1p-100f;
                    if (MAXMODE) {
                        if (probed) gmax = fmaxf(gmax, ip - e);
                    } else if (probed && !(ip + e < th)) {
                        const int64_t q = q0 + ql;
                        const int slot = atomicAdd(&counts[q], 1);
                        if (slot < cap) lists[q * cap + slot] = pit[ib];
                    }
                }
                if (MAXMODE) {
                    // largest lower bound of this iteration's 32 items for query ql
                    gmax = row16_max(gmax);
                    if (r16 == 0 && q0 + ql < nq && p0 < pend)
                        cmax[(q0 + ql) * ncol + blockIdx.y * SC_GROUPS + (p0 - pbeg) / 32] = gmax;
                }
            }
        }
    }
}

// bfloat16 variants of k_screen on v_mfma_f32_16x16x32_bf16 (products of
// bfloat16 pairs are exact in FP32).  In MFMA j of a 32-coordinate step, lane
// group g carries coordinates 32 kk + 8 g .. + 7 of both operands.
//   X3 = false: q and x rounded to bfloat16 (RNE, unit roundoff u = 2^-8),
//       one product per pair.  q~_t x~_t = q_t x_t (1 + a)(1 + b) with
//       |a|, |b| <= u, so |q.x - q~.x~| <= (2u + u^2) sum |q_t x_t| =
//       (2^-7 + 2^-16) sum |q_t x_t|, and FP32 accumulation of the d exact
//       products adds at most gamma_d (1.01 sum |q_t x_t|).
//   X3 = true:  q and x split x = hi + lo (+ a residual of at most
//       2^-16 |x|), each inner product hi.hi + hi.lo + lo.hi; the dropped
//       terms are at most 3.1 * 2^-16 |q_t x_t| per coordinate, and FP32
//       accumulation of the 3d products adds at most gamma_{3d} (1.02 sum).
// The caller's g covers either with the same factor-2 margin as the FP32
// screen.  When every query of the tile probes every level of the chunk's
// sub-dataset (h <= hthr for all h, as at T = n), the probe test is skipped.
__device__ __forceinline__ uint16_t q_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 as_bf16x8(u16x8 v) { return __builtin_bit_cast(bf16x8, v); }

// 16 bytes at voffset + soffset of a raw buffer (0 past its size)
__device__ __forceinline__ u16x8 buf_load16(__amdgpu_buffer_rsrc_t r, uint32_t voffset, int soffset)
{
    return __builtin_bit_cast(u16x8, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voffset, soffset, 0));
}

// bfloat16 image of a query batch for the screen: hi = RNE(q), lo =
// RNE(q - hi) (when Ql != NULL), rows zero-padded to dp columns, and qn = an
// upper bound on ||q|| (exact squares, FP64 sum, rounded up).  One wave per
// query.
__global__ __launch_bounds__(256) void k_query_bf16(const float *__restrict__ Q, int64_t nq, int d,
                                                    int dp, uint16_t *__restrict__ Qh,
                                                    uint16_t *__restrict__ Ql,
                                                    float *__restrict__ qn,
                                                    uint32_t *__restrict__ nonfinite)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * 4 + wave;
    if (q >= nq) return;
    double s2 = 0.0;
    bool bad = false;
    for (int c = lane; c < dp; c += 64) {
        const float f = c < d ? Q[q * d + c] : 0.f;
        bad |= !__builtin_isfinite(f);
        const uint16_t hi = q_bf16_rne(f);
        Qh[q * dp + c] = hi;
        if (Ql) Ql[q * dp + c] = q_bf16_rne(f - __uint_as_float((uint32_t)hi << 16));
        s2 += (double)f * (double)f;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o, 64);
    if (lane == 0) qn[q] = (float)__builtin_sqrt(s2) * (1.0f + 0x1p-18f);
    if (nonfinite && __ballot(bad) != 0ull && lane == 0) atomicOr(nonfinite, 1u);
}

// Sort keys of the keep pass's query order: theta / ||q|| descending (as an
// order-preserving 32-bit word, complemented), queries without a theta last.
__global__ __launch_bounds__(256) void k_query_order(const float *__restrict__ theta,
                                                     const float *__restrict__ qn, int64_t nq,
                                                     uint64_t *__restrict__ key, int32_t *__restrict__ val)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= nq) return;
    const float r = qn[q] > 0.f ? theta[q] / qn[q] : -INFINITY;
    uint32_t u = __float_as_uint(r == r ? r : -INFINITY);
    u = (u >> 31) ? ~u : (u | 0x80000000u);  // larger r, larger word
    key[q] = (uint64_t)(~u);
    val[q] = (int32_t)q;
}

// Probe bounds when the budget covers every item (T >= n): every bucket of
// every sub-dataset is probed whole and there is no threshold bucket to cut;
// rows past nq get hthr = -1 as the threshold pass leaves them.  The bound
// is 64, above any distance the screens can compute: the query codes are not
// computed on this path, so a tile with rows past nq (which falls back to
// the per-pair test) compares against whatever the code buffer holds.
__global__ __launch_bounds__(256) void k_probe_all(int64_t nq, int64_t tiles, int m,
                                                   int32_t *__restrict__ ghthr, int32_t *__restrict__ gtie,
                                                   int32_t *__restrict__ gpstar)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < tiles * m * 64) {
        const int64_t q = (e / ((int64_t)m * 64)) * 64 + (e & 63);
        ghthr[e] = q < nq ? 64 : -1;
    }
    if (e < tiles * 4 * 64) gtie[e] = (e / 64) % 4 == 2 ? INT_MAX : -1;
    if (e < nq) gpstar[e] = -1;
}

// A block holds 64 queries (their bfloat16 rows staged in LDS) and one chunk
// of stored items of a single sub-dataset; each wave takes 64 items at a time
// (4 column blocks of 16) against the 64 queries (4 row blocks of 16), and
// fetches the item rows of the next 32-coordinate step while the matrix cores
// work on the current one.
#define NRLSH_SCREEN_PARAMS                                                                    \
    const uint16_t *__restrict__ Xh, const uint16_t *__restrict__ Xlo, int dp,                  \
        const uint32_t *__restrict__ codes_l, const double *__restrict__ key_l,                 \
        const uint16_t *__restrict__ Qh, const uint16_t *__restrict__ Ql,                       \
        const float *__restrict__ qnorm, int64_t nq, const int32_t *__restrict__ chunks, int m, \
        const uint32_t *__restrict__ qcodes, const int32_t *__restrict__ ghthr,                 \
        const int32_t *__restrict__ gtie, const int32_t *__restrict__ gpstar,                   \
        const float *__restrict__ theta, float gam, int cap, int32_t *__restrict__ counts,      \
        int32_t *__restrict__ lists, float *__restrict__ cmax, int ncol, int qsb, int L, int qsets, \
        const double *__restrict__ Usub, unsigned long long *__restrict__ npairs,                \
        const int32_t *__restrict__ qidx
#define NRLSH_SCREEN_ARGS                                                                      \
    Xh, Xlo, dp, codes_l, key_l, Qh, Ql, qnorm, nq, chunks, m, qcodes, ghthr, gtie, gpstar, theta, \
        gam, cap, counts, lists, cmax, ncol, qsb, L, qsets, Usub, npairs, qidx

// W = 0: every level of every sub-dataset is probed (a budget covering all
// items), so no code is read and no probe test is made.
template <int W, bool MAXMODE, bool X3>
__device__ __forceinline__ void screen_bf16(NRLSH_SCREEN_PARAMS)
{
    constexpr int WC = W > 0 ? W : 1;  // code words kept per item (storage)
    extern __shared__ __align__(16) uint16_t qsh[];  // hi: 64 x qsb, then (X3) lo: 64 x qsb
    uint16_t *qsl = qsh + 64 * qsb;
    __shared__ float th_s[64], qn_s[64];
    __shared__ int32_t hthr_s[64], htie_s[64], pstar_s[64];
    __shared__ uint32_t qc_s[64 * WC];
    __shared__ int any_s, all_s;
    // pass B with the probe test: kept items of each query row, staged in LDS
    // and appended to the query's list with one reservation at the block's end
    // (a returning global atomic per kept pair would leave its latency
    // exposed); rows whose room fills take that atomic for the rest.  With
    // every item probed (W = 0) few pairs are kept and each takes its own.
    constexpr bool STAGE = !MAXMODE && W > 0;
    constexpr int KS = STAGE ? 24 : 1;
    __shared__ int32_t kc_s[64], kl_s[64 * KS];
    // pass B: per wave, a queue of the pairs that reach theta (see below)
    constexpr int WQ = MAXMODE ? 1 : 512;
    __shared__ uint16_t wq_s[4 * WQ];
    __shared__ int wqn_s[4];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int tile = blockIdx.x;
    const int j = chunks[3 * blockIdx.y], pbeg = chunks[3 * blockIdx.y + 1],
              pend = chunks[3 * blockIdx.y + 2];
    const int64_t q0 = (int64_t)tile * 64;
    // row r of the tile is query qmap(q0 + r): the batch order, or (pass B)
    // the order of qidx, which groups queries of similar theta / ||q|| so that
    // whole tiles skip the chunks none of them can keep
    auto qmap = [&](int64_t r) -> int64_t { return (qidx && r < nq) ? (int64_t)qidx[r] : r; };

    if (tid < 64) {
        const int64_t q = qmap(q0 + tid);
        kc_s[tid] = 0;
        int hthr = -1, htie = -1, pstar = -1;
        float th = -INFINITY, qn = 0.f;
        if (q < nq) {
            const int64_t qt = q >> 6;
            const int ql0 = (int)(q & 63);
            hthr = ghthr[(qt * m + j) * 64 + ql0];
            const int32_t *tie = gtie + qt * 4 * 64;
            if (tie[ql0] == j) {
                htie = tie[64 + ql0];
                pstar = gpstar[q];
            }
            if (!MAXMODE || Usub) th = theta[q];  // pass A reads it only to skip chunks
            qn = qnorm[q];
#pragma unroll
            for (int w = 0; w < W; ++w) qc_s[tid * W + w] = qcodes[qrow(q, j, qsets) * W + w];
        }
        hthr_s[tid] = hthr;
        htie_s[tid] = htie;
        pstar_s[tid] = pstar;
        // rows past the batch keep nothing (pass B): theta +inf makes every
        // pair fall below it, whether or not a probe test runs (W = 0 and
        // all-probed tiles skip it)
        th_s[tid] = (!MAXMODE && q >= nq) ? INFINITY : th;
        qn_s[tid] = qn;
        // no item of sub-dataset j (norms <= U_j) can be kept (pass B), or raise
        // a group maximum to theta (pass A), for a query whose theta exceeds
        // qn U_j (1 + 2 gam + 2^-15): ip32 + e is at most ||q|| ||x|| + 2 e
        // (Cauchy-Schwarz); a chunk that no query of the tile reaches is skipped
        const bool reach = !Usub || q >= nq ||
                           !((double)th > (double)qn * Usub[j] * (1.0 + 2.0 * (double)gam + 0x1p-15) + 0x1p-80);
        const uint64_t b = __ballot((hthr >= 0 || htie >= 0) && reach);
        const uint64_t a = __ballot(hthr >= L);  // every possible h passes
        if (tid == 0) {
            any_s = b != 0ull;
            all_s = a == ~0ull;
        }
    }
    __syncthreads();
    // groups this block never reaches stay -inf (the loop below writes every
    // group of the chunk's items for every query row of the tile)
    if (MAXMODE && tid < 64 && q0 + tid < nq) {
        for (int gi = any_s ? (pend - pbeg + 31) / 32 : 0; gi < SC_GROUPS; ++gi)
            cmax[(q0 + tid) * ncol + blockIdx.y * SC_GROUPS + gi] = -INFINITY;
    }
    if (!any_s) return;  // no query of this tile probes (or, pass B, can keep) an item of this chunk
    if (npairs && tid == 0)
        atomicAdd(npairs, (unsigned long long)(min((int64_t)64, nq - q0) * (int64_t)(pend - pbeg)));

    // stage the query tile (rows beyond nq and columns beyond dp, up to a
    // multiple of 32, are zero)
    // (four threads per row, 8 columns each per round; the loads of SQ_U
    // rounds are issued before their LDS stores, so a tile costs one or two
    // round trips to memory rather than one per round)
    const u16x8 z8 = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
    {
        constexpr int SQ_U = 8;
        const int r = tid >> 2, cq = 8 * (tid & 3);
        const bool rok = q0 + r < nq;
        const int64_t qr = rok ? qmap(q0 + r) : 0;
        const int nu = (dp + 31) / 32;  // 32-column rounds
        for (int u0 = 0; u0 < nu; u0 += SQ_U) {
            u16x8 th[SQ_U], tl[SQ_U];
#pragma unroll
            for (int u = 0; u < SQ_U; ++u) {
                const int c = 32 * (u0 + u) + cq;
                const bool ok = rok && u0 + u < nu && c < dp;
                th[u] = ok ? *reinterpret_cast<const u16x8 *>(Qh + qr * dp + c) : z8;
                tl[u] = (X3 && ok) ? *reinterpret_cast<const u16x8 *>(Ql + qr * dp + c) : z8;
            }
#pragma unroll
            for (int u = 0; u < SQ_U; ++u) {
                if (u0 + u >= nu) break;
                const int c = 32 * (u0 + u) + cq;
                *reinterpret_cast<u16x8 *>(&qsh[r * qsb + c]) = th[u];
                if (X3) *reinterpret_cast<u16x8 *>(&qsl[r * qsb + c]) = tl[u];
            }
        }
    }
    __syncthreads();

    // NB column blocks of 16 items per wave iteration (bf16x3 keeps 2: its
    // hi and lo operands double the registers)
    constexpr int NB = X3 ? 2 : 4, IW = 16 * NB;
    const int r16 = lane & 15, g = lane >> 4;
    const bool all = W == 0 || all_s != 0;
    // stored rows of this chunk through buffer descriptors: 32-bit offsets
    // from the chunk's first row, and reads past the chunk's rows return 0
    // (finite values that meet the zero columns of the query tile, or rows
    // whose results are never used)
    const uint32_t rbytes = (uint32_t)(pend - pbeg) * (uint32_t)dp * 2u;
    const __amdgpu_buffer_rsrc_t bx =
        __builtin_amdgcn_make_buffer_rsrc((void *)(Xh + (int64_t)pbeg * dp), 0, (int)rbytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t bxl =
        __builtin_amdgcn_make_buffer_rsrc((void *)(X3 ? Xlo + (int64_t)pbeg * dp : Xh), 0, X3 ? (int)rbytes : 0,
                                          0x00020000);
    if (!MAXMODE && lane == 0) wqn_s[wave] = 0;
    wave_sync();
    for (int p0 = pbeg + wave * IW; p0 < pend; p0 += 4 * IW) {
        uint32_t cw[NB][WC];
        float xn[NB];
        uint32_t ro[NB];  // byte offset of this lane's 8 coordinates of row 16 ib + r16
#pragma unroll
        for (int ib = 0; ib < NB; ++ib) {
            const int pi = p0 + 16 * ib + r16;
            const int64_t pp = pi < pend ? pi : pbeg;
#pragma unroll
            // (pass B reads the codes of its candidates only)
            for (int w = 0; w < W; ++w) cw[ib][w] = (all || !MAXMODE) ? 0u : codes_l[pp * W + w];
            xn[ib] = sqrtf((float)key_l[pp]) * (1.0f + 0x1p-18f);
            ro[ib] = (uint32_t)(pi - pbeg) * (uint32_t)dp * 2u + 16u * g;
        }
        floatx4 acc[4][NB];
#pragma unroll
        for (int qb = 0; qb < 4; ++qb)
#pragma unroll
            for (int ib = 0; ib < NB; ++ib) acc[qb][ib] = floatx4{0.f, 0.f, 0.f, 0.f};
        // item operands of step kk: 8 coordinates of one row per lane
        u16x8 bh[NB], bl[NB];
#pragma unroll
        for (int ib = 0; ib < NB; ++ib) {
            bh[ib] = buf_load16(bx, ro[ib], 0);
            bl[ib] = X3 ? buf_load16(bxl, ro[ib], 0) : z8;
        }
        for (int kk = 0; kk < dp; kk += 32) {
            u16x8 ch[NB], cl[NB];
#pragma unroll
            for (int ib = 0; ib < NB; ++ib) {
                ch[ib] = bh[ib];
                cl[ib] = bl[ib];
            }
            if (kk + 32 < dp) {  // prefetch the next step
#pragma unroll
                for (int ib = 0; ib < NB; ++ib) {
                    bh[ib] = buf_load16(bx, ro[ib], 2 * (kk + 32));
                    if (X3) bl[ib] = buf_load16(bxl, ro[ib], 2 * (kk + 32));
                }
            }
            const int kc = kk + 8 * g;
            u16x8 ah[4], al[4];
#pragma unroll
            for (int qb = 0; qb < 4; ++qb) {
                const int o = (16 * qb + r16) * qsb + kc;
                ah[qb] = *reinterpret_cast<const u16x8 *>(&qsh[o]);
                al[qb] = X3 ? *reinterpret_cast<const u16x8 *>(&qsl[o]) : z8;
            }
#pragma unroll
            for (int qb = 0; qb < 4; ++qb)
#pragma unroll
                for (int ib = 0; ib < NB; ++ib) {
                    acc[qb][ib] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        as_bf16x8(ah[qb]), as_bf16x8(ch[ib]), acc[qb][ib], 0, 0, 0);
                    if (X3) {
                        acc[qb][ib] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            as_bf16x8(ah[qb]), as_bf16x8(cl[ib]), acc[qb][ib], 0, 0, 0);
                        acc[qb][ib] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            as_bf16x8(al[qb]), as_bf16x8(ch[ib]), acc[qb][ib], 0, 0, 0);
                    }
                }
        }
        if (!MAXMODE) {
            // pass B in two steps.  A pair whose upper bound ip32 + e reaches
            // theta is a candidate: one bound for the lane's NB items first (e
            // grows with ||x|| and float rounding is monotone, so a pair whose
            // ip + emax stays below theta is dropped with one add and one
            // compare), then each item's own bound.  Candidates, about one
            // pair in a hundred, go to the wave's queue in LDS, and only they
            // take the probe test and the list append: evaluated in place,
            // the probe test ran for nearly every pair, since almost every
            // (query row, 64 items) step of the wave holds some candidate.
            float xmax = xn[0];
#pragma unroll
            for (int ib = 1; ib < NB; ++ib) xmax = fmaxf(xmax, xn[ib]);
            uint16_t *wq = wq_s + wave * WQ;
            // the whole wave (every lane active) empties its queue: entry
            // (row ql << 6 | item offset in this iteration), one per lane
            auto drain = [&]() {
                wave_sync();
                const int nw = __builtin_amdgcn_readfirstlane(min(wqn_s[wave], WQ));
                for (int i = lane; i < nw; i += 64) {
                    const uint32_t e = wq[i];
                    const int ql = (int)(e >> 6), pi = p0 + (int)(e & 63u);
                    bool probed = pi < pend;
                    if (!all && probed) {
                        int h = __popc(codes_l[(int64_t)pi * W] ^ qc_s[ql * W]);
                        if (W == 2) h += __popc(codes_l[(int64_t)pi * W + 1] ^ qc_s[ql * W + 1]);
                        probed = h <= hthr_s[ql] || (h == htie_s[ql] && pi <= pstar_s[ql]);
                    }
                    if (probed) {
                        const int ls = STAGE ? atomicAdd(&kc_s[ql], 1) : KS;
                        if (ls < KS) {
                            kl_s[ql * KS + ls] = pi;
                        } else {
                            const int64_t q = qmap(q0 + ql);
                            const int slot = atomicAdd(&counts[q], 1);
                            if (slot < cap) lists[q * cap + slot] = pi;
                        }
                    }
                }
                wave_sync();
                if (lane == 0) wqn_s[wave] = 0;
                wave_sync();
            };
#pragma unroll
            for (int qb = 0; qb < 4; ++qb) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    // room for this step's entries (at most 64 NB), made here
                    // where every lane is active (each takes a share of the queue)
                    if (__builtin_amdgcn_readfirstlane(wqn_s[wave]) > WQ - 64 * NB) drain();
                    const int ql = 16 * qb + 4 * g + v;
                    const float th = th_s[ql], qn = qn_s[ql];
                    const float emax = gam * qn * xmax + 0x1p-90f;
                    bool near = false;
#pragma unroll
                    for (int ib = 0; ib < NB; ++ib) near |= !(acc[qb][ib][v] + emax < th);
                    if (!near) continue;
                    uint32_t cm = 0u;
#pragma unroll
                    for (int ib = 0; ib < NB; ++ib) {
                        const float e = gam * qn * xn[ib] + 0x1p-90f;
                        cm |= (uint32_t)!(acc[qb][ib][v] + e < th) << ib;
                    }
                    if (cm != 0u) {
                        int o = atomicAdd(&wqn_s[wave], __popc(cm));
#pragma unroll
                        for (int ib = 0; ib < NB; ++ib)
                            if ((cm >> ib) & 1u) wq[o++] = (uint16_t)((ql << 6) | (16 * ib + r16));
                    }
                }
            }
            drain();
        } else {
            // pass A: the largest lower bound ip32 - e over the probed items of
            // each 32-item group, per query row
#pragma unroll
            for (int qb = 0; qb < 4; ++qb) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int ql = 16 * qb + 4 * g + v;
                    const int hthr = hthr_s[ql], htie = htie_s[ql];
                    const float qn = qn_s[ql];
                    float gmax[NB / 2];
#pragma unroll
                    for (int hg = 0; hg < NB / 2; ++hg) gmax[hg] = -INFINITY;
#pragma unroll
                    for (int ib = 0; ib < NB; ++ib) {
                        const int pi = p0 + 16 * ib + r16;
                        bool probed = pi < pend;
                        if (!all) {
                            int h = __popc(cw[ib][0] ^ qc_s[ql * W]);
                            if (W == 2) h += __popc(cw[ib][1] ^ qc_s[ql * W + 1]);
                            probed = probed && (h <= hthr || (h == htie && pi <= pstar_s[ql]));
                        }
                        const float e = gam * qn * xn[ib] + 0x1p-90f;
                        if (probed) gmax[ib >> 1] = fmaxf(gmax[ib >> 1], acc[qb][ib][v] - e);
                    }
#pragma unroll
                    for (int hg = 0; hg < NB / 2; ++hg) {
                        gmax[hg] = row16_max(gmax[hg]);
                        if (r16 == 0 && q0 + ql < nq && p0 + 32 * hg < pend)
                            cmax[(q0 + ql) * ncol + blockIdx.y * SC_GROUPS + (p0 - pbeg) / 32 + hg] = gmax[hg];
                    }
                }
            }
        }
    }
    if (STAGE) {
        __syncthreads();
        if (tid < 64 && q0 + tid < nq) {
            const int n = min(kc_s[tid], KS);
            if (n > 0) {
                const int64_t q = qmap(q0 + tid);
                const int base = atomicAdd(&counts[q], n);
                for (int i = 0; i < n; ++i)
                    if (base + i < cap) lists[q * cap + base + i] = kl_s[tid * KS + i];
            }
        }
    }
}

template <int W, bool MAXMODE, bool X3>
__global__ __launch_bounds__(256) void k_screen3(NRLSH_SCREEN_PARAMS)
{
    screen_bf16<W, MAXMODE, X3>(NRLSH_SCREEN_ARGS);
}

// Pass A of the single-product screen when every item is probed: no codes,
// so a register budget for three waves per SIMD fits without spilling much.
__global__ __launch_bounds__(256, 3) void k_screen_a0(NRLSH_SCREEN_PARAMS)
{
    screen_bf16<0, true, false>(NRLSH_SCREEN_ARGS);
}

// Pass B of the single-product screen when every item is probed, on tiles of
// 128 queries: eight waves share the tile's bfloat16 image in LDS and each
// multiplies it with its own 64 items per iteration, so every item row read
// from memory serves 128 queries (the 64-query kernel reads it for 64).  The
// keep rule, the norm-bound skip of a chunk and the query order are those of
// screen_bf16; rows past the batch get theta = +inf and keep nothing.
__global__ __launch_bounds__(512) void k_screen_b128(
    const uint16_t *__restrict__ Xh, int dp, const double *__restrict__ key_l,
    const uint16_t *__restrict__ Qh, const float *__restrict__ qnorm, int64_t nq,
    const int32_t *__restrict__ chunks, const float *__restrict__ theta, float gam, int cap,
    int32_t *__restrict__ counts, int32_t *__restrict__ lists, int qsb,
    const double *__restrict__ Usub, unsigned long long *__restrict__ npairs,
    const int32_t *__restrict__ qidx)
{
    extern __shared__ __align__(16) uint16_t qsh[];  // 128 x qsb
    __shared__ float th_s[128], qn_s[128];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int j = chunks[3 * blockIdx.y], pbeg = chunks[3 * blockIdx.y + 1], pend = chunks[3 * blockIdx.y + 2];
    const int64_t q0 = (int64_t)blockIdx.x * 128;
    auto qmap = [&](int64_t r) -> int64_t { return (qidx && r < nq) ? (int64_t)qidx[r] : r; };
    bool reach = false;
    if (tid < 128) {
        const int64_t q = qmap(q0 + tid);
        float th = INFINITY, qn = 0.f;
        if (q < nq) {
            th = theta[q];
            qn = qnorm[q];
            reach = !Usub ||
                    !((double)th > (double)qn * Usub[j] * (1.0 + 2.0 * (double)gam + 0x1p-15) + 0x1p-80);
        }
        th_s[tid] = th;
        qn_s[tid] = qn;
    }
    if (!__syncthreads_or(reach)) return;  // no query of the tile can keep an item of the chunk
    if (npairs && tid == 0)
        atomicAdd(npairs, (unsigned long long)(min((int64_t)128, nq - q0) * (int64_t)(pend - pbeg)));

    // stage the query tile: four threads per row, 8 columns each per round
    const u16x8 z8 = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
    {
        constexpr int SQ_U = 8;
        const int r = tid >> 2, cq = 8 * (tid & 3);
        const bool rok = q0 + r < nq;
        const int64_t qr = rok ? qmap(q0 + r) : 0;
        const int nu = (dp + 31) / 32;
        for (int u0 = 0; u0 < nu; u0 += SQ_U) {
            u16x8 th8[SQ_U];
#pragma unroll
            for (int u = 0; u < SQ_U; ++u) {
                const int c = 32 * (u0 + u) + cq;
                th8[u] = (rok && u0 + u < nu && c < dp) ? *reinterpret_cast<const u16x8 *>(Qh + qr * dp + c) : z8;
            }
#pragma unroll
            for (int u = 0; u < SQ_U; ++u) {
                if (u0 + u >= nu) break;
                *reinterpret_cast<u16x8 *>(&qsh[r * qsb + 32 * (u0 + u) + cq]) = th8[u];
            }
        }
    }
    __syncthreads();

    const int r16 = lane & 15, g = lane >> 4;
    const uint32_t rbytes = (uint32_t)(pend - pbeg) * (uint32_t)dp * 2u;
    const __amdgpu_buffer_rsrc_t bx =
        __builtin_amdgcn_make_buffer_rsrc((void *)(Xh + (int64_t)pbeg * dp), 0, (int)rbytes, 0x00020000);
    for (int p0 = pbeg + wave * 64; p0 < pend; p0 += 8 * 64) {
        float xn[4];
        uint32_t ro[4];
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
            const int pi = p0 + 16 * ib + r16;
            const int64_t pp = pi < pend ? pi : pbeg;
            xn[ib] = sqrtf((float)key_l[pp]) * (1.0f + 0x1p-18f);
            ro[ib] = (uint32_t)(pi - pbeg) * (uint32_t)dp * 2u + 16u * g;
        }
        floatx4 acc[8][4];
#pragma unroll
        for (int qb = 0; qb < 8; ++qb)
#pragma unroll
            for (int ib = 0; ib < 4; ++ib) acc[qb][ib] = floatx4{0.f, 0.f, 0.f, 0.f};
        u16x8 bh[4];
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) bh[ib] = buf_load16(bx, ro[ib], 0);
        for (int kk = 0; kk < dp; kk += 32) {
            u16x8 ch[4];
#pragma unroll
            for (int ib = 0; ib < 4; ++ib) ch[ib] = bh[ib];
            if (kk + 32 < dp) {
#pragma unroll
                for (int ib = 0; ib < 4; ++ib) bh[ib] = buf_load16(bx, ro[ib], 2 * (kk + 32));
            }
            const int kc = kk + 8 * g;
#pragma unroll
            for (int qb = 0; qb < 8; ++qb) {
                const u16x8 ah = *reinterpret_cast<const u16x8 *>(&qsh[(16 * qb + r16) * qsb + kc]);
#pragma unroll
                for (int ib = 0; ib < 4; ++ib)
                    acc[qb][ib] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah), as_bf16x8(ch[ib]),
                                                                          acc[qb][ib], 0, 0, 0);
            }
        }
        float xmax = fmaxf(fmaxf(xn[0], xn[1]), fmaxf(xn[2], xn[3]));
#pragma unroll
        for (int qb = 0; qb < 8; ++qb) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ql = 16 * qb + 4 * g + v;
                const float th = th_s[ql], qn = qn_s[ql];
                const float emax = gam * qn * xmax + 0x1p-90f;
                bool near = false;
#pragma unroll
                for (int ib = 0; ib < 4; ++ib) near |= !(acc[qb][ib][v] + emax < th);
                if (!near) continue;
#pragma unroll
                for (int ib = 0; ib < 4; ++ib) {
                    const int pi = p0 + 16 * ib + r16;
                    const float e = gam * qn * xn[ib] + 0x1p-90f;
                    if (pi < pend && !(acc[qb][ib][v] + e < th)) {
                        const int64_t q = qmap(q0 + ql);
                        const int slot = atomicAdd(&counts[q], 1);
                        if (slot < cap) lists[q * cap + slot] = pi;
                    }
                }
            }
        }
    }
}

// Pass B of the single-product screen, the one that runs over every probed
// pair.  It holds no item codes (its candidates read theirs from the queue),
// so a register budget for three waves per SIMD fits without spills.
template <int W>
__global__ __launch_bounds__(256, 3) void k_screen1(NRLSH_SCREEN_PARAMS)
{
    screen_bf16<W, false, false>(NRLSH_SCREEN_ARGS);
}

// theta_q = the k-th largest group maximum (a lower bound of the k-th best
// exact inner product: k distinct items reach it), lowered by 2^-22 relative
// to cover float rounding; -inf when fewer than k groups hold probed items.
// One wave per query.
// Order-preserving 32-bit key of a float group maximum; 0 for -inf and NaN
// (no probed item), below every finite value's key.
__device__ __forceinline__ uint32_t theta_key(float v)
{
    const uint32_t u = __float_as_uint(v);
    return v > -INFINITY ? ((u & 0x80000000u) ? ~u : (u | 0x80000000u)) : 0u;
}
__device__ __forceinline__ float theta_value(uint32_t key)
{
    return __uint_as_float((key & 0x80000000u) ? (key & 0x7FFFFFFFu) : ~key);
}
// theta_q: the k-th largest of a query's ncol group maxima (each the largest
// lower bound among a group's probed items, so that k distinct items reach
// the k-th largest), lowered for rounding.  A radix selection
// on the order-preserving keys (-inf and NaN as 0, so that fewer than k
// finite maxima give -inf): four 8-bit passes, each counting the keys that
// share the digits found so far in a 256-bin LDS histogram and keeping the
// bin where the count from the top reaches k.  One wave per query.
__global__ __launch_bounds__(64) void k_theta(const float *__restrict__ cmax, int stride, int ncol, int k,
                                              float *__restrict__ theta)
{
    __shared__ uint32_t hist[256];
    const int lane = threadIdx.x;
    const int64_t q = blockIdx.x;
    const float *row = cmax + q * stride;
    uint32_t prefix = 0u, mask = 0u;
    uint32_t need = (uint32_t)k;
    bool found = true;
    for (int shift = 24; shift >= 0 && found; shift -= 8) {
        for (int b = lane; b < 256; b += 64) hist[b] = 0u;
        __syncthreads();
        for (int c = lane; c < ncol; c += 64) {
            const uint32_t key = theta_key(row[c]);
            if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        // lane l holds bins 4 l .. 4 l + 3; `above` = keys in the bins above them
        uint32_t h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) h[i] = hist[4 * lane + i];
        const uint32_t part = h[0] + h[1] + h[2] + h[3];
        uint32_t incl = part;  // parts of lanes >= this one
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_down(incl, o, 64);
            if (lane + o < 64) incl += y;
        }
        const uint32_t above = incl - part;
        int sel = -1;
        uint32_t rest = 0u;
        if (above < need && need <= above + part) {
            uint32_t c = above;
            for (int i = 3; i >= 0; --i) {
                if (c + h[i] >= need) {
                    sel = 4 * lane + i;
                    rest = need - c;
                    break;
                }
                c += h[i];
            }
        }
        const uint64_t who = __ballot(sel >= 0);
        found = who != 0ull;
        if (found) {
            const int src = __ffsll((long long)who) - 1;
            sel = __shfl(sel, src, 64);
            need = __shfl(rest, src, 64);
            prefix |= (uint32_t)sel << shift;
            mask |= 0xFFu << shift;
        }
        __syncthreads();
    }
    if (lane == 0) {
        const float f = theta_value(prefix);
        theta[q] = (!found || prefix == 0u) ? -INFINITY : f - fabsf(f) * 0x1p-22f - 0x1p-126f;
    }
}

// One record per screened batch for the host: the largest and the total
// kept-list length, the queries left without theta (theta != NULL), and the
// call's evaluated-pair count and non-finite flag as they stand.  One block.
__global__ __launch_bounds__(1024) void k_list_stats(const int32_t *__restrict__ counts,
                                                     const float *__restrict__ theta, int64_t nb,
                                                     const unsigned long long *__restrict__ npairs,
                                                     const uint32_t *__restrict__ flag,
                                                     long long *__restrict__ rec)
{
    __shared__ long long s_mx[16], s_sum[16], s_un[16];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    long long mx = 0, sum = 0, un = 0;
    for (int64_t i = tid; i < nb; i += 1024) {
        const long long c = counts[i];
        mx = c > mx ? c : mx;
        sum += c;
        if (theta && theta[i] == -INFINITY) ++un;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const long long m2 = __shfl_xor(mx, o, 64);
        mx = m2 > mx ? m2 : mx;
        sum += __shfl_xor(sum, o, 64);
        un += __shfl_xor(un, o, 64);
    }
    if (lane == 0) {
        s_mx[wave] = mx;
        s_sum[wave] = sum;
        s_un[wave] = un;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < 16; ++w) {
            mx = s_mx[w] > mx ? s_mx[w] : mx;
            sum += s_sum[w];
            un += s_un[w];
        }
        rec[0] = mx;
        rec[1] = sum;
        rec[2] = un;
        rec[3] = npairs ? (long long)*npairs : 0;
        rec[4] = flag ? (long long)*flag : 0;
    }
}

inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

hipError_t launch_query_hash(const float *Q, int64_t nq, int d, const float *At, int L, int W,
                             int qsets, uint32_t *qcodes, uint32_t *nonfinite, hipStream_t s)
{
    if (nq < 1) return hipSuccess;
    const int cpw = L <= 32 ? 64 / L : 1;
    const dim3 grid(ceil_div(nq, QH_Q), ceil_div(qsets, cpw));
    hipLaunchKernelGGL(k_query_hash, grid, dim3(64), 0, s, Q, nq, d, At, L, W, qsets, qcodes,
                       nonfinite);
    return hipGetLastError();
}

hipError_t launch_scan_hist(const uint32_t *codes_l, const int32_t *off, const uint32_t *qcodes,
                            int64_t nq, const QueryShape &sh, uint32_t *ghist, hipStream_t s)
{
    const dim3 grid(ceil_div(nq, 64), (unsigned)sh.m);
    const size_t lds = (size_t)(sh.L + 1) * 64 * sizeof(uint32_t);
    if (sh.W == 1)
        hipLaunchKernelGGL(k_scan_hist<1>, grid, dim3(64), lds, s, codes_l, off, qcodes, nq, sh.m,
                           sh.L, sh.qsets, ghist);
    else
        hipLaunchKernelGGL(k_scan_hist<2>, grid, dim3(64), lds, s, codes_l, off, qcodes, nq, sh.m,
                           sh.L, sh.qsets, ghist);
    return hipGetLastError();
}

hipError_t launch_threshold(const uint32_t *ghist, const int32_t *R, const int32_t *inv, int64_t nq,
                            const QueryShape &sh, int32_t *gbase, int32_t *ghthr, int32_t *gtie,
                            hipStream_t s, bool bounds, bool offsets)
{
    const int64_t P = (int64_t)sh.m * (sh.L + 1);
    const bool lds = P <= TH_INV_LDS_MAX;
    const size_t bytes = lds ? (size_t)P * sizeof(int32_t) : 0;
    const dim3 grid(ceil_div(nq, 64)), block(TH_WAVES * 64);
#define NRLSH_THRESHOLD_LAUNCH(MODE)                                                                       \
    if (lds)                                                                                               \
        hipLaunchKernelGGL((k_threshold<MODE, true>), grid, block, bytes, s, ghist, R, inv, nq, sh.m, sh.L, \
                           sh.Tq, gbase, ghthr, gtie);                                                     \
    else                                                                                                   \
        hipLaunchKernelGGL((k_threshold<MODE, false>), grid, block, 0, s, ghist, R, inv, nq, sh.m, sh.L,   \
                           sh.Tq, gbase, ghthr, gtie);
    if (bounds && offsets) {
        NRLSH_THRESHOLD_LAUNCH(2)
    } else if (bounds) {
        NRLSH_THRESHOLD_LAUNCH(1)
    } else {
        NRLSH_THRESHOLD_LAUNCH(0)
    }
#undef NRLSH_THRESHOLD_LAUNCH
    return hipGetLastError();
}

hipError_t launch_scan_emit(const uint32_t *codes_l, const int32_t *off, const uint32_t *qcodes,
                            int64_t nq, const QueryShape &sh, const int32_t *gbase,
                            const int32_t *ghthr, const int32_t *gtie, int32_t *cand,
                            hipStream_t s)
{
    const dim3 grid(ceil_div(nq, 64), (unsigned)sh.m);
    if (sh.W == 1)
        hipLaunchKernelGGL(k_scan_emit<1>, grid, dim3(64), 0, s, codes_l, off, qcodes, nq, sh.m,
                           sh.L, sh.Tq, sh.qsets, gbase, ghthr, gtie, cand);
    else
        hipLaunchKernelGGL(k_scan_emit<2>, grid, dim3(64), 0, s, codes_l, off, qcodes, nq, sh.m,
                           sh.L, sh.Tq, sh.qsets, gbase, ghthr, gtie, cand);
    return hipGetLastError();
}

hipError_t launch_scan_hist_c(const uint32_t *codes_l, const int32_t *off, const uint32_t *qcodes,
                              int64_t nq, const QueryShape &sh, int chunk, int nch, uint32_t *ghist,
                              hipStream_t s)
{
    const int64_t blocks = (int64_t)ceil_div(nq, 64) * sh.m * nch;
    const size_t lds = (size_t)(sh.L + 1) * 64 * sizeof(uint32_t);
    if (sh.W == 1)
        hipLaunchKernelGGL(k_scan_hist_c<1>, dim3((unsigned)blocks), dim3(64), lds, s, codes_l, off,
                           qcodes, nq, sh.m, sh.L, sh.qsets, chunk, nch, ghist);
    else
        hipLaunchKernelGGL(k_scan_hist_c<2>, dim3((unsigned)blocks), dim3(64), lds, s, codes_l, off,
                           qcodes, nq, sh.m, sh.L, sh.qsets, chunk, nch, ghist);
    return hipGetLastError();
}

hipError_t launch_scan_emit_c(const uint32_t *codes_l, const int32_t *off, const uint32_t *qcodes,
                              int64_t nq, const QueryShape &sh, int chunk, int nch,
                              const int32_t *ghthr, const int32_t *gtie, const int32_t *gpstar,
                              int32_t *counts, int32_t *cand, hipStream_t s)
{
    const int64_t blocks = (int64_t)ceil_div(nq, 64) * sh.m * nch;
    if (sh.W == 1)
        hipLaunchKernelGGL(k_scan_emit_c<1>, dim3((unsigned)blocks), dim3(64), 0, s, codes_l, off,
                           qcodes, nq, sh.m, sh.Tq, sh.qsets, chunk, nch, ghthr, gtie, gpstar, counts,
                           cand);
    else
        hipLaunchKernelGGL(k_scan_emit_c<2>, dim3((unsigned)blocks), dim3(64), 0, s, codes_l, off,
                           qcodes, nq, sh.m, sh.Tq, sh.qsets, chunk, nch, ghthr, gtie, gpstar, counts,
                           cand);
    return hipGetLastError();
}

hipError_t launch_fill32(void *p, int64_t words, uint32_t v, hipStream_t s)
{
    if (words < 1) return hipSuccess;
    int64_t blocks = (words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill32, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<uint32_t *>(p), words, v);
    return hipGetLastError();
}

hipError_t launch_scan_hist_stage(const uint32_t *codes_l, const uint32_t *qcodes, int64_t nq,
                                  const QueryShape &sh, const int32_t *chunks, int nchunks,
                                  const int32_t *need, uint32_t *ghist, unsigned long long *npairs,
                                  hipStream_t s, int gstride)
{
    if (nq < 1 || nchunks < 1) return hipSuccess;
    if (gstride < 1) return hipErrorInvalidValue;
    const dim3 grid(ceil_div(nq, 64), (unsigned)nchunks);
    const size_t lds = (size_t)(sh.L + 1) * 64 * sizeof(uint32_t);
    if (sh.W == 1)
        hipLaunchKernelGGL(k_scan_hist_s<1>, grid, dim3(SH_WAVES * 64), lds, s, codes_l, qcodes, nq,
                           sh.m, sh.L, sh.qsets, chunks, need, ghist, npairs, gstride);
    else
        hipLaunchKernelGGL(k_scan_hist_s<2>, grid, dim3(SH_WAVES * 64), lds, s, codes_l, qcodes, nq,
                           sh.m, sh.L, sh.qsets, chunks, need, ghist, npairs, gstride);
    return hipGetLastError();
}

hipError_t launch_scan_collect(const uint32_t *codes_l, const uint32_t *qcodes, int64_t nq, const QueryShape &sh,
                               const int32_t *chunks, int nchunks, const int32_t *R, const int32_t *grho,
                               int64_t cap, int32_t *counts, uint64_t *keys, uint32_t *ghist,
                               unsigned long long *npairs, hipStream_t s, int jh0, int jh1)
{
    if (nq < 1 || nchunks < 1) return hipSuccess;
    const dim3 grid(ceil_div(nq, 64), (unsigned)nchunks);
    const size_t lds = (size_t)(sh.L + 1) * 32 * sizeof(uint32_t) +
                       (size_t)SH_WAVES * 2 * MX_SB * 64 * (sizeof(uint16_t) + sizeof(uint8_t)) +
                       (size_t)(sh.L + 1) * sizeof(int32_t);
    if (sh.W == 1)
        hipLaunchKernelGGL(k_scan_collect_mx<1>, grid, dim3(SH_WAVES * 64), lds, s, codes_l, qcodes, nq, sh.m,
                           sh.L, sh.qsets, chunks, R, grho, cap, counts, keys, ghist, npairs, jh0, jh1);
    else
        hipLaunchKernelGGL(k_scan_collect_mx<2>, grid, dim3(SH_WAVES * 64), lds, s, codes_l, qcodes, nq, sh.m,
                           sh.L, sh.qsets, chunks, R, grho, cap, counts, keys, ghist, npairs, jh0, jh1);
    return hipGetLastError();
}

hipError_t launch_collect_filter(const uint64_t *keys, const int32_t *counts, int64_t cap, int64_t nq,
                                 const int32_t *gtie, const int32_t *gpstar, const int32_t *grho, int64_t Tq,
                                 int32_t *cand, int32_t *lcount, uint32_t *fail, hipStream_t s)
{
    if (nq < 1) return hipSuccess;
    hipLaunchKernelGGL(k_collect_filter, dim3((unsigned)nq), dim3(256), 0, s, keys, counts, cap, gtie, gpstar, grho,
                       Tq, cand, lcount, fail);
    return hipGetLastError();
}

// rho[q] = b*' + 1 of a threshold pass (gtie's b* row), capped at P buckets.
__global__ __launch_bounds__(64) void k_rho_from_tie(const int32_t *__restrict__ gtie, int64_t nq, int32_t P,
                                                     int32_t *__restrict__ rho)
{
    const int64_t q = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (q >= nq) return;
    const int32_t b = gtie[(q >> 6) * 4 * 64 + 3 * 64 + (q & 63)];
    rho[q] = b < 0 || b >= P ? P : b + 1;
}

// Per sub-dataset j: the sampled items (histogram of the sample pass) that
// rank before each query's guessed cut rho, summed over a slice of the batch
// -- the slice's probed items of j in sample units.  Ranks grow with h inside
// a sub-dataset, so each query's walk stops at its first bucket not before
// rho.  Blocks: (sub-dataset, slice of SUB_HITS_Q queries); out[j][slice].
constexpr int SUB_HITS_Q = 256;
__global__ __launch_bounds__(SUB_HITS_Q) void k_sub_hits(const uint32_t *__restrict__ ghist,
                                                         const int32_t *__restrict__ R,
                                                         const int32_t *__restrict__ grho, int64_t nq, int m,
                                                         int L, unsigned long long *__restrict__ out)
{
    __shared__ unsigned long long part[SUB_HITS_Q / 64];
    const int j = blockIdx.x, tid = threadIdx.x, L1 = L + 1;
    const int32_t *Rj = R + (int64_t)j * L1;
    const int64_t q = (int64_t)blockIdx.y * SUB_HITS_Q + tid;
    unsigned long long acc = 0;
    if (q < nq) {
        const int32_t rho = grho[q];
        const uint32_t *H = ghist + (((q >> 6) * m + j) * (int64_t)L1) * 64 + (q & 63);
        for (int h = 0; h <= L && Rj[L - h] < rho; ++h) acc += H[(int64_t)h * 64];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((tid & 63) == 0) part[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < SUB_HITS_Q / 64; ++w) t += part[w];
        out[(int64_t)j * gridDim.y + blockIdx.y] = t;
    }
}

int sub_hits_slices(int64_t nq) { return (int)std::max<int64_t>(1, (nq + SUB_HITS_Q - 1) / SUB_HITS_Q); }

hipError_t launch_sub_hits(const uint32_t *ghist, const int32_t *R, const int32_t *grho, int64_t nq, int m, int L,
                           unsigned long long *out, hipStream_t s)
{
    if (m < 1) return hipSuccess;
    hipLaunchKernelGGL(k_sub_hits, dim3((unsigned)m, (unsigned)sub_hits_slices(nq)), dim3(SUB_HITS_Q), 0, s, ghist,
                       R, grho, nq, m, L, out);
    return hipGetLastError();
}

hipError_t launch_rho_from_tie(const int32_t *gtie, int64_t nq, int32_t P, int32_t *rho, hipStream_t s)
{
    if (nq < 1) return hipSuccess;
    hipLaunchKernelGGL(k_rho_from_tie, dim3(ceil_div(nq, 64)), dim3(64), 0, s, gtie, nq, P, rho);
    return hipGetLastError();
}

hipError_t launch_scan_emit_stage(const uint32_t *codes_l, const uint32_t *qcodes, int64_t nq,
                                  const QueryShape &sh, const int32_t *chunks, int nchunks,
                                  const int32_t *ghthr, const int32_t *gtie, const int32_t *gpstar,
                                  int32_t *counts, int32_t *cand, hipStream_t s)
{
    if (nq < 1 || nchunks < 1) return hipSuccess;
    const dim3 grid(ceil_div(nq, 64), (unsigned)nchunks);
    if (sh.W == 1)
        hipLaunchKernelGGL(k_scan_emit_s<1>, grid, dim3(SH_WAVES * 64), 0, s, codes_l, qcodes, nq, sh.m,
                           sh.Tq, sh.qsets, chunks, ghthr, gtie, gpstar, counts, cand);
    else
        hipLaunchKernelGGL(k_scan_emit_s<2>, grid, dim3(SH_WAVES * 64), 0, s, codes_l, qcodes, nq, sh.m,
                           sh.Tq, sh.qsets, chunks, ghthr, gtie, gpstar, counts, cand);
    return hipGetLastError();
}

hipError_t launch_stage_check(const uint32_t *ghist, const int32_t *inv, int64_t nq, const QueryShape &sh,
                              int cut, int32_t *need, hipStream_t s)
{
    if (nq < 1) return hipSuccess;
    hipLaunchKernelGGL(k_stage_check, dim3(ceil_div(nq, 64)), dim3(64), 0, s, ghist, inv, nq, sh.m, sh.L,
                       sh.Tq, cut, need);
    return hipGetLastError();
}

hipError_t launch_tie_locate(const uint32_t *codes_l, const int32_t *off, const uint32_t *qcodes,
                             int64_t nq, int W, int qsets, const int32_t *gtie, int32_t *gpstar,
                             hipStream_t s, const uint32_t *ghist, int m, int L)
{
    if (W == 1)
        hipLaunchKernelGGL(k_tie_locate<1>, dim3((unsigned)nq), dim3(TL_WAVES * 64), 0, s, codes_l, off,
                           qcodes, nq, qsets, gtie, gpstar, ghist, m, L);
    else
        hipLaunchKernelGGL(k_tie_locate<2>, dim3((unsigned)nq), dim3(TL_WAVES * 64), 0, s, codes_l, off,
                           qcodes, nq, qsets, gtie, gpstar, ghist, m, L);
    return hipGetLastError();
}

hipError_t launch_query_order(const float *theta, const float *qn, int64_t nq, uint64_t *ka, int32_t *va,
                              uint64_t *kb, int32_t *vb, void *tmp, int32_t **order, hipStream_t s)
{
    hipLaunchKernelGGL(k_query_order, dim3(ceil_div(nq, 256)), dim3(256), 0, s, theta, qn, nq, ka, va);
    bool in_b = false;
    hipError_t e = radix_sort(ka, va, kb, vb, nq, 32, tmp, &in_b, s);
    *order = in_b ? vb : va;
    return e;
}

// A batch's queries in order of their guessed cut rho: a 64-query tile scans
// (and the dense head screens) every chunk of a sub-dataset whose first
// bucket ranks before the largest cut among its queries, so tiles of alike
// cuts touch fewer chunks.  Keys rho, values the batch index.
__global__ __launch_bounds__(256) void k_rho_keys(const int32_t *__restrict__ rho, int64_t nq,
                                                  uint64_t *__restrict__ ka, int32_t *__restrict__ va)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= nq) return;
    ka[q] = (uint64_t)(uint32_t)max(rho[q], 0);
    va[q] = (int32_t)q;
}

hipError_t launch_rho_order(const int32_t *rho, int64_t nq, int nbits, uint64_t *ka, int32_t *va, uint64_t *kb,
                            int32_t *vb, void *tmp, int32_t **order, hipStream_t s)
{
    hipLaunchKernelGGL(k_rho_keys, dim3(ceil_div(nq, 256)), dim3(256), 0, s, rho, nq, ka, va);
    bool in_b = false;
    hipError_t e = radix_sort(ka, va, kb, vb, nq, nbits, tmp, &in_b, s);
    *order = in_b ? vb : va;
    return e;
}

// Row i of the permuted batch is row order[i] of the batch: its query (d
// floats), its codes (cw words) and its guessed cut.  One wave per row.
__global__ __launch_bounds__(256) void k_permute_batch(const float *__restrict__ Q, const uint32_t *__restrict__ qc,
                                                       const int32_t *__restrict__ rho,
                                                       const int32_t *__restrict__ order, int64_t nq, int d, int cw,
                                                       float *__restrict__ Qp, uint32_t *__restrict__ qcp,
                                                       int32_t *__restrict__ rhop)
{
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= nq) return;
    const int64_t src = order[i];
    for (int t = lane; t < d; t += 64) Qp[i * d + t] = Q[src * d + t];
    for (int t = lane; t < cw; t += 64) qcp[i * cw + t] = qc[src * cw + t];
    if (lane == 0) rhop[i] = rho[src];
}

// The results of permuted row i go to row order[i] of the batch's outputs.
__global__ __launch_bounds__(256) void k_unpermute_results(const int32_t *__restrict__ order, int64_t nq, int k,
                                                           const int64_t *__restrict__ tids,
                                                           const float *__restrict__ tips,
                                                           int64_t *__restrict__ ids, float *__restrict__ ips)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= nq * k) return;
    const int64_t i = e / k, c = e - i * k;
    const int64_t dst = (int64_t)order[i] * k + c;
    ids[dst] = tids[e];
    ips[dst] = tips[e];
}

hipError_t launch_permute_batch(const float *Q, const uint32_t *qc, const int32_t *rho, const int32_t *order,
                                int64_t nq, int d, int cw, float *Qp, uint32_t *qcp, int32_t *rhop, hipStream_t s)
{
    if (nq < 1) return hipSuccess;
    hipLaunchKernelGGL(k_permute_batch, dim3(ceil_div(nq, 4)), dim3(256), 0, s, Q, qc, rho, order, nq, d, cw, Qp,
                       qcp, rhop);
    return hipGetLastError();
}

hipError_t launch_unpermute_results(const int32_t *order, int64_t nq, int k, const int64_t *tids, const float *tips,
                                    int64_t *ids, float *ips, hipStream_t s)
{
    if (nq < 1 || k < 1) return hipSuccess;
    hipLaunchKernelGGL(k_unpermute_results, dim3(ceil_div(nq * k, 256)), dim3(256), 0, s, order, nq, k, tids, tips,
                       ids, ips);
    return hipGetLastError();
}

// ---------------------------------------------------------------- witnesses
// The witnesses of each sub-dataset, in stored order: its `top` largest-norm
// items (ties by stored position) -- the k-th best lower bound of a query's
// probed items is mostly set by high-norm ones -- and every `stride`-th item
// of its stored range (so that a query whose probed items are low-norm ones
// still finds k witnesses among them).  One block per sub-dataset: radix
// selection of the top-th largest key (keys are non-negative doubles, ordered
// as their bit patterns), then an ordered compaction.  wpos: m x W stored
// positions (W >= top + ceil(n_j / stride)), wcnt[j] their number.
constexpr int WIT_THREADS = 1024;
__global__ __launch_bounds__(WIT_THREADS) void k_wit_select(const double *__restrict__ key_l,
                                                            const int32_t *__restrict__ off, int top, int stride,
                                                            int W, int32_t *__restrict__ wpos,
                                                            int32_t *__restrict__ wcnt)
{
    constexpr int NW = WIT_THREADS / 64;
    __shared__ uint32_t hist[256];
    __shared__ unsigned long long s_prefix;
    __shared__ int s_need, s_base, s_tbase;
    __shared__ int wsum[2 * NW];
    const int j = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t p0 = off[j], p1 = off[j + 1], nj = p1 - p0;
    const int want = (int)min<int64_t>(nj, (int64_t)top);
    int32_t *out = wpos + (int64_t)j * W;
    if (want == nj || nj <= W && stride == 1) {  // every item of the sub-dataset
        for (int64_t i = tid; i < nj; i += WIT_THREADS) out[i] = (int32_t)(p0 + i);
        if (tid == 0) wcnt[j] = want;
        return;
    }
    unsigned long long prefix = 0, mask = 0;
    int need = want;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int b = tid; b < 256; b += WIT_THREADS) hist[b] = 0u;
        __syncthreads();
        for (int64_t p = p0 + tid; p < p1; p += WIT_THREADS) {
            const unsigned long long u = (unsigned long long)__double_as_longlong(key_l[p]);
            if ((u & mask) == prefix) atomicAdd(&hist[(u >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            int cum = 0, sel = 0;
            for (int b = 255; b >= 0; --b) {
                if (cum + (int)hist[b] >= need) {
                    sel = b;
                    break;
                }
                cum += (int)hist[b];
            }
            s_need = need - cum;
            s_prefix = prefix | ((unsigned long long)sel << shift);
        }
        __syncthreads();
        need = s_need;
        prefix = s_prefix;
        mask |= 0xFFull << shift;
        __syncthreads();
    }
    // prefix: the bits of the want-th largest key t; need: how many keys equal
    // to t to take (the first ones in stored order), after every key above t
    if (tid == 0) {
        s_base = 0;
        s_tbase = 0;
    }
    __syncthreads();
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int64_t c0 = p0; c0 < p1; c0 += WIT_THREADS) {
        const int64_t p = c0 + tid;
        bool gt = false, eq = false;
        if (p < p1) {
            const unsigned long long u = (unsigned long long)__double_as_longlong(key_l[p]);
            gt = u > prefix;
            eq = u == prefix;
        }
        const unsigned long long be = __ballot(eq);
        if (lane == 0) wsum[wv] = __popcll(be);
        __syncthreads();
        int eoff = 0;
        for (int w = 0; w < wv; ++w) eoff += wsum[w];
        const bool keep = gt || (eq && s_tbase + eoff + __popcll(be & below) < need) ||
                          (p < p1 && (p - p0) % stride == 0);
        const unsigned long long bk = __ballot(keep);
        if (lane == 0) wsum[NW + wv] = __popcll(bk);
        __syncthreads();
        int koff = 0;
        for (int w = 0; w < wv; ++w) koff += wsum[NW + w];
        if (keep) out[s_base + koff + __popcll(bk & below)] = (int32_t)p;
        __syncthreads();
        if (tid == 0) {
            int te = 0, tk = 0;
            for (int w = 0; w < NW; ++w) {
                te += wsum[w];
                tk += wsum[NW + w];
            }
            s_tbase += te;
            s_base += tk;
        }
        __syncthreads();
    }
    if (tid == 0) wcnt[j] = s_base;
}

// Compact copies of the witnesses: slot j W + i holds item wpos[j W + i] (i <
// wcnt[j]): its bfloat16 row (dp values), codes (cw words) and key.  One wave
// per slot.
__global__ __launch_bounds__(256) void k_wit_gather(const uint16_t *__restrict__ Xh,
                                                    const uint32_t *__restrict__ codes_l,
                                                    const double *__restrict__ key_l, int dp, int cw,
                                                    const int32_t *__restrict__ wpos,
                                                    const int32_t *__restrict__ wcnt, int W, int64_t slots,
                                                    uint16_t *__restrict__ xw, uint32_t *__restrict__ cwo,
                                                    double *__restrict__ kw)
{
    const int64_t slot = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (slot >= slots) return;
    const int64_t j = slot / W, i = slot - j * W;
    if (i >= wcnt[j]) return;
    const int64_t pos = wpos[slot];
    for (int t = lane; t < dp; t += 64) xw[slot * dp + t] = Xh[pos * dp + t];
    if (lane < cw) cwo[slot * cw + lane] = codes_l[pos * cw + lane];
    if (lane == 0) kw[slot] = key_l[pos];
}

// P* of each query in the witnesses' numbering: the tie bucket's sub-dataset
// j* keeps its witnesses in stored order, so "stored position <= P*" becomes
// "slot <= j* W + (witnesses of j* at or before P*) - 1" (INT_MAX, the whole
// bucket, stays).
__global__ __launch_bounds__(256) void k_wit_pstar(const int32_t *__restrict__ gtie,
                                                   const int32_t *__restrict__ gpstar,
                                                   const int32_t *__restrict__ wpos,
                                                   const int32_t *__restrict__ wcnt, int W, int64_t nq,
                                                   int32_t *__restrict__ pw)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= nq) return;
    const int32_t js = gtie[(q >> 6) * 4 * 64 + (q & 63)];
    const int32_t ps = gpstar[q];
    if (js < 0 || ps == INT_MAX) {
        pw[q] = ps;
        return;
    }
    const int32_t *w = wpos + (int64_t)js * W;
    int lo = 0, hi = wcnt[js];  // first witness after P*
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (w[mid] <= ps) lo = mid + 1;
        else hi = mid;
    }
    pw[q] = js * W + lo - 1;
}

hipError_t launch_wit_build(const uint16_t *Xh, const uint32_t *codes_l, const double *key_l, const int32_t *off,
                            int m, int dp, int cw, int top, int stride, int W, int32_t *wpos, int32_t *wcnt,
                            uint16_t *xw, uint32_t *cwo, double *kw, hipStream_t s)
{
    if (m < 1) return hipSuccess;
    hipLaunchKernelGGL(k_wit_select, dim3((unsigned)m), dim3(WIT_THREADS), 0, s, key_l, off, top, stride, W, wpos,
                       wcnt);
    const int64_t slots = (int64_t)m * W;
    hipLaunchKernelGGL(k_wit_gather, dim3(ceil_div(slots, 4)), dim3(256), 0, s, Xh, codes_l, key_l, dp, cw, wpos,
                       wcnt, W, slots, xw, cwo, kw);
    return hipGetLastError();
}

hipError_t launch_wit_pstar(const int32_t *gtie, const int32_t *gpstar, const int32_t *wpos, const int32_t *wcnt,
                            int W, int64_t nq, int32_t *pw, hipStream_t s)
{
    if (nq < 1) return hipSuccess;
    hipLaunchKernelGGL(k_wit_pstar, dim3(ceil_div(nq, 256)), dim3(256), 0, s, gtie, gpstar, wpos, wcnt, W, nq, pw);
    return hipGetLastError();
}

// A batch's kept lists against their room, on the device: the total and the
// largest of lcount and the total of the gathered counts (gcount, or gdef
// per query without it) are added to stats[0..2] (stats[1] by maximum), and
// bit 2 of *fail is set when a list outgrew lcap (the call then runs the
// batch again without the lists).  One block.
__global__ __launch_bounds__(1024) void k_list_check(const int32_t *__restrict__ lcount,
                                                     const int32_t *__restrict__ gcount, int64_t nb, int lcap,
                                                     int64_t gdef, unsigned long long *__restrict__ stats,
                                                     uint32_t *__restrict__ fail)
{
    __shared__ unsigned long long s_tot[16], s_mx[16], s_g[16];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    unsigned long long tot = 0, mx = 0, g = 0;
    for (int64_t q = tid; q < nb; q += 1024) {
        const unsigned long long c = (unsigned long long)max(lcount[q], 0);
        tot += c;
        mx = c > mx ? c : mx;
        g += gcount ? (unsigned long long)max(gcount[q], 0) : (unsigned long long)gdef;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        tot += __shfl_xor(tot, o, 64);
        const unsigned long long om = __shfl_xor(mx, o, 64);
        mx = om > mx ? om : mx;
        g += __shfl_xor(g, o, 64);
    }
    if (lane == 0) {
        s_tot[wv] = tot;
        s_mx[wv] = mx;
        s_g[wv] = g;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < 16; ++w) {
            tot += s_tot[w];
            mx = s_mx[w] > mx ? s_mx[w] : mx;
            g += s_g[w];
        }
        atomicAdd(&stats[0], tot);
        atomicMax(&stats[1], mx);
        atomicAdd(&stats[2], g);
        if (mx > (unsigned long long)lcap) atomicOr(fail, 2u);
    }
}

hipError_t launch_list_check(const int32_t *lcount, const int32_t *gcount, int64_t nb, int lcap, int64_t gdef,
                             unsigned long long *stats, uint32_t *fail, hipStream_t s)
{
    if (nb < 1) return hipSuccess;
    hipLaunchKernelGGL(k_list_check, dim3(1), dim3(1024), 0, s, lcount, gcount, nb, lcap, gdef, stats, fail);
    return hipGetLastError();
}

hipError_t launch_probe_all(int64_t nq, const QueryShape &sh, int32_t *ghthr, int32_t *gtie,
                            int32_t *gpstar, hipStream_t s)
{
    const int64_t tiles = (nq + 63) / 64;
    const int64_t cnt = std::max<int64_t>(std::max<int64_t>(tiles * sh.m * 64, tiles * 4 * 64), nq);
    hipLaunchKernelGGL(k_probe_all, dim3(ceil_div(cnt, 256)), dim3(256), 0, s, nq, tiles, sh.m, ghthr, gtie,
                       gpstar);
    return hipGetLastError();
}

hipError_t launch_query_bf16(const float *Q, int64_t nq, int d, int dp, uint16_t *Qh, uint16_t *Ql,
                             float *qn, hipStream_t s, uint32_t *nonfinite)
{
    hipLaunchKernelGGL(k_query_bf16, dim3(ceil_div(nq, 4)), dim3(256), 0, s, Q, nq, d, dp, Qh, Ql, qn,
                       nonfinite);
    return hipGetLastError();
}

hipError_t launch_list_stats(const int32_t *counts, const float *theta, int64_t nb,
                             const unsigned long long *npairs, const uint32_t *flag, long long *rec,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_list_stats, dim3(1), dim3(1024), 0, s, counts, theta, nb, npairs, flag, rec);
    return hipGetLastError();
}

int screen_chunk_items() { return SC_CHUNK; }
int screen_cell_items() { return SC_CELL; }
int screen_cell_groups() { return SC_GROUPS; }

// bf16 row stride of the staged query tile: dp + 8 or dp + 16 so that the
// row stride in dwords is an odd multiple of 4 (16 lanes reading 16 bytes of
// 16 rows hit 16 distinct 4-bank groups)
// rows padded with zeros to a multiple of 32 coordinates (so that every
// 32-coordinate step reads real columns), plus 8 so that the row stride in
// dwords is an odd multiple of 4 (16 lanes reading 16 bytes of 16 rows hit 16
// distinct 4-bank groups)
static int screen_qsb(int dp) { return (dp + 31) / 32 * 32 + 8; }

size_t screen_lds_bytes(int dp, int kind)
{
    if (kind == SCREEN_BF16X3) return (size_t)2 * 64 * screen_qsb(dp) * sizeof(uint16_t);
    if (kind == SCREEN_BF16) return (size_t)64 * screen_qsb(dp) * sizeof(uint16_t);
    return (size_t)64 * (dp + 4) * sizeof(float);
}

template <int W, bool MAXMODE, bool X3>
static hipError_t launch_screen_bf16(const uint16_t *Xh, const uint16_t *Xlo, const double *key_l,
                                     const uint32_t *codes_l, const ScreenQueries &Q, int64_t nq,
                                     const QueryShape &sh, const int32_t *chunks, int nchunks,
                                     const uint32_t *qcodes, const int32_t *ghthr,
                                     const int32_t *gtie, const int32_t *gpstar,
                                     const float *theta, float gam, int cap, int32_t *counts,
                                     int32_t *lists, float *cmax, int ncol, hipStream_t s)
{
    const size_t lds = screen_lds_bytes(sh.dp, X3 ? SCREEN_BF16X3 : SCREEN_BF16);
    const bool one = !MAXMODE && !X3;
    const bool a0 = W == 0 && MAXMODE && !X3;
    const void *fn = one  ? (const void *)k_screen1<W>
                     : a0 ? (const void *)k_screen_a0
                          : (const void *)k_screen3<W, MAXMODE, X3>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (W == 0 && one && sh.dp >= 256) {
        // 128-query tiles when their image fits the work-group's LDS (rows of
        // at least 256 coordinates: shorter ones gain less from the halved
        // item reads than the coarser tiles lose in skipped chunks)
        const size_t lds2 = (size_t)128 * screen_qsb(sh.dp) * sizeof(uint16_t);
        int dev = 0, lim = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            lds2 + 2048 <= (size_t)lim &&
            hipFuncSetAttribute((const void *)k_screen_b128, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds2) == hipSuccess) {
            const dim3 grid2(ceil_div(nq, 128), (unsigned)nchunks);
            hipLaunchKernelGGL(k_screen_b128, grid2, dim3(512), lds2, s, Xh, sh.dp, key_l, Q.Qh, Q.qn, nq, chunks,
                               theta, gam, cap, counts, lists, screen_qsb(sh.dp), Q.U, Q.pairs, Q.order);
            return hipGetLastError();
        }
    }
    const dim3 grid(ceil_div(nq, 64), (unsigned)nchunks);
    if (a0)
        hipLaunchKernelGGL(k_screen_a0, grid, dim3(256), lds, s, Xh, Xlo, sh.dp, codes_l, key_l, Q.Qh, Q.Ql,
                           Q.qn, nq, chunks, sh.m, qcodes, ghthr, gtie, gpstar, theta, gam, cap, counts,
                           lists, cmax, ncol, screen_qsb(sh.dp), sh.L, sh.qsets, Q.U, nullptr, nullptr);
    else if (one)
        hipLaunchKernelGGL((k_screen1<W>), grid, dim3(256), lds, s, Xh, Xlo, sh.dp, codes_l, key_l,
                           Q.Qh, Q.Ql, Q.qn, nq, chunks, sh.m, qcodes, ghthr, gtie, gpstar, theta, gam,
                           cap, counts, lists, cmax, ncol, screen_qsb(sh.dp), sh.L, sh.qsets,
                           Q.U, MAXMODE ? nullptr : Q.pairs, MAXMODE ? nullptr : Q.order);
    else
        hipLaunchKernelGGL((k_screen3<W, MAXMODE, X3>), grid, dim3(256), lds, s, Xh, Xlo, sh.dp,
                           codes_l, key_l, Q.Qh, Q.Ql, Q.qn, nq, chunks, sh.m, qcodes, ghthr, gtie,
                           gpstar, theta, gam, cap, counts, lists, cmax, ncol, screen_qsb(sh.dp), sh.L,
                           sh.qsets, Q.U, MAXMODE ? nullptr : Q.pairs, MAXMODE ? nullptr : Q.order);
    return hipGetLastError();
}

template <bool MAXMODE>
static hipError_t launch_screen_t(const float *Xl, const uint16_t *Xh, const uint16_t *Xlo,
                                  const double *key_l, const uint32_t *codes_l, const ScreenQueries &Q,
                                  int64_t nq, const QueryShape &sh, const int32_t *chunks,
                                  int nchunks, const uint32_t *qcodes, const int32_t *ghthr,
                                  const int32_t *gtie, const int32_t *gpstar, const float *theta,
                                  int cap, int32_t *counts, int32_t *lists, float *cmax,
                                  hipStream_t s, int stride = 0)
{
    // MAXMODE: row stride of cmax (stride, or this launch's own columns)
    const int ncol = MAXMODE ? (stride ? stride : nchunks * SC_GROUPS) : 0;
    if (Xh && Xlo) {
        // per coordinate 3.1 * 2^-16 |q x| dropped by the split, plus FP32
        // accumulation of 3d exact products: 2 * 1.02 * gamma_{3d}
        const double u3 = 3.0 * sh.d * 0x1p-24;
        const float gam = (float)((3.2 * 0x1p-16 + 2.1 * u3 / (1.0 - u3)) * (1.0 + 0x1p-16));
        return sh.Tq >= sh.n
                   ? launch_screen_bf16<0, MAXMODE, true>(Xh, Xlo, key_l, codes_l, Q, nq, sh, chunks,
                                                          nchunks, qcodes, ghthr, gtie, gpstar, theta,
                                                          gam, cap, counts, lists, cmax, ncol, s)
               : sh.W == 1
                   ? launch_screen_bf16<1, MAXMODE, true>(Xh, Xlo, key_l, codes_l, Q, nq, sh, chunks,
                                                          nchunks, qcodes, ghthr, gtie, gpstar, theta,
                                                          gam, cap, counts, lists, cmax, ncol, s)
                   : launch_screen_bf16<2, MAXMODE, true>(Xh, Xlo, key_l, codes_l, Q, nq, sh, chunks,
                                                          nchunks, qcodes, ghthr, gtie, gpstar, theta,
                                                          gam, cap, counts, lists, cmax, ncol, s);
    }
    if (Xh) {
        // rounding of both operands to bfloat16: (2u + u^2) |q x| per
        // coordinate with u = 2^-8, plus FP32 accumulation of d exact
        // products: 2 * 1.01 * gamma_d
        const double ud = sh.d * 0x1p-24;
        const float gam = (float)((0x1p-7 + 0x1p-16 + 2.1 * ud / (1.0 - ud)) * (1.0 + 0x1p-16));
        // a budget covering every item probes every level: the variant that
        // reads no codes
        return sh.Tq >= sh.n
                   ? launch_screen_bf16<0, MAXMODE, false>(Xh, nullptr, key_l, codes_l, Q, nq, sh,
                                                           chunks, nchunks, qcodes, ghthr, gtie, gpstar,
                                                           theta, gam, cap, counts, lists, cmax, ncol, s)
               : sh.W == 1
                   ? launch_screen_bf16<1, MAXMODE, false>(Xh, nullptr, key_l, codes_l, Q, nq, sh,
                                                           chunks, nchunks, qcodes, ghthr, gtie, gpstar,
                                                           theta, gam, cap, counts, lists, cmax, ncol, s)
                   : launch_screen_bf16<2, MAXMODE, false>(Xh, nullptr, key_l, codes_l, Q, nq, sh,
                                                           chunks, nchunks, qcodes, ghthr, gtie, gpstar,
                                                           theta, gam, cap, counts, lists, cmax, ncol, s);
    }
    const size_t lds = screen_lds_bytes(sh.dp, SCREEN_FP32);
    const dim3 grid(ceil_div(nq, 64), (unsigned)nchunks);
    const double ud = (double)sh.d * 0x1p-24;
    const float gam = (float)(2.0 * ud / (1.0 - ud) * (1.0 + 0x1p-16));
    const void *fn = sh.W == 1 ? (const void *)k_screen<1, MAXMODE> : (const void *)k_screen<2, MAXMODE>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (sh.W == 1)
        hipLaunchKernelGGL((k_screen<1, MAXMODE>), grid, dim3(256), lds, s, Xl, sh.d, sh.dp, codes_l,
                           key_l, Q.Q, nq, chunks, sh.m, qcodes, ghthr, gtie, gpstar, theta, gam, cap,
                           counts, lists, cmax, ncol, sh.L, sh.qsets);
    else
        hipLaunchKernelGGL((k_screen<2, MAXMODE>), grid, dim3(256), lds, s, Xl, sh.d, sh.dp, codes_l,
                           key_l, Q.Q, nq, chunks, sh.m, qcodes, ghthr, gtie, gpstar, theta, gam, cap,
                           counts, lists, cmax, ncol, sh.L, sh.qsets);
    return hipGetLastError();
}

static void launch_theta(const float *cmax, int stride, int ncol, int64_t nq, int k, float *theta,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_theta, dim3((unsigned)nq), dim3(64), 0, s, cmax, stride, ncol, k, theta);
}

hipError_t launch_screen_max(const float *Xl, const uint16_t *Xh, const uint16_t *Xlo,
                             const double *key_l, const uint32_t *codes_l,
                             const ScreenQueries &Q, int64_t nq, const QueryShape &sh, const int32_t *cells,
                             int ncells, int ncells_top, const uint32_t *qcodes, const int32_t *ghthr,
                             const int32_t *gtie, const int32_t *gpstar, float *cmax, float *theta,
                             hipStream_t s)
{
    const int ncol = ncells * SC_GROUPS;
    if (Q.U && ncells_top > 0 && ncells_top < ncells) {
        // theta from the top sub-datasets' cells first; the other cells skip
        // every tile whose queries their items cannot lift above it (their
        // groups stay -inf, and groups below it cannot change the k-th largest)
        ScreenQueries q1 = Q;
        q1.U = nullptr;
        hipError_t e = launch_screen_t<true>(Xl, Xh, Xlo, key_l, codes_l, q1, nq, sh, cells, ncells_top,
                                             qcodes, ghthr, gtie, gpstar, nullptr, 0, nullptr, nullptr,
                                             cmax, s, ncol);
        if (e != hipSuccess) return e;
        launch_theta(cmax, ncol, ncells_top * SC_GROUPS, nq, sh.k, theta, s);
        e = launch_screen_t<true>(Xl, Xh, Xlo, key_l, codes_l, Q, nq, sh, cells + 3 * ncells_top,
                                  ncells - ncells_top, qcodes, ghthr, gtie, gpstar, theta, 0, nullptr,
                                  nullptr, cmax + ncells_top * SC_GROUPS, s, ncol);
        if (e != hipSuccess) return e;
    } else {
        ScreenQueries q1 = Q;
        q1.U = nullptr;
        hipError_t e = launch_screen_t<true>(Xl, Xh, Xlo, key_l, codes_l, q1, nq, sh, cells, ncells,
                                             qcodes, ghthr, gtie, gpstar, nullptr, 0, nullptr, nullptr,
                                             cmax, s, ncol);
        if (e != hipSuccess) return e;
    }
    launch_theta(cmax, ncol, ncol, nq, sh.k, theta, s);
    return hipGetLastError();
}

hipError_t launch_screen(const float *Xl, const uint16_t *Xh, const uint16_t *Xlo,
                         const double *key_l, const uint32_t *codes_l,
                         const ScreenQueries &Q, int64_t nq, const QueryShape &sh, const int32_t *chunks,
                         int nchunks, const uint32_t *qcodes, const int32_t *ghthr,
                         const int32_t *gtie, const int32_t *gpstar, const float *theta, int cap,
                         int32_t *counts, int32_t *lists, hipStream_t s)
{
    return launch_screen_t<false>(Xl, Xh, Xlo, key_l, codes_l, Q, nq, sh, chunks, nchunks, qcodes,
                                  ghthr, gtie, gpstar, theta, cap, counts, lists, nullptr, s);
}

int rerank_splits(int64_t nq, int64_t Tq)
{
    // enough waves to cover the machine (256 CUs x 32 waves) without slices
    // shorter than 16 candidate batches
    int64_t want = (8192 + nq - 1) / nq;
    const int64_t cap = (Tq + 1023) / 1024;
    if (want > cap) want = cap;
    if (want < 1) want = 1;
    if (want > 64) want = 64;
    return (int)want;
}

hipError_t launch_rerank(const float *Xl, const int32_t *perm, const float *Q, int64_t nq,
                         const QueryShape &sh, const int32_t *cand, const int32_t *counts,
                         int nsplit, double *part_v, int32_t *part_i, int64_t *out_ids,
                         float *out_ips, hipStream_t s, unsigned long long *gtheta)
{
    if (nsplit < 2) gtheta = nullptr;  // one slice per query: nothing to share
    const int S = (sh.k + 63) / 64;
    int64_t slice = (sh.Tq + nsplit - 1) / nsplit;
    slice = (slice + 63) / 64 * 64;
    const dim3 grid((unsigned)nq, (unsigned)nsplit), block(64);
#define NRLSH_RERANK(SS)                                                                         \
    do {                                                                                         \
        hipLaunchKernelGGL((k_rerank<SS>), grid, block, 0, s, Xl, perm, Q, sh.n, sh.d, sh.dp,    \
                           sh.Tq, sh.k, cand, counts, nsplit, slice, out_ids, out_ips, part_v,   \
                           part_i, gtheta);                                                      \
        if (nsplit > 1)                                                                          \
            hipLaunchKernelGGL(k_topk_merge<SS>, dim3((unsigned)nq), block, 0, s, part_v, part_i, \
                               nsplit, sh.k, out_ids, out_ips);                                  \
    } while (0)
    if (S <= 1) NRLSH_RERANK(1);
    else if (S <= 2) NRLSH_RERANK(2);
    else if (S <= 4) NRLSH_RERANK(4);
    else if (S <= 8) NRLSH_RERANK(8);
    else NRLSH_RERANK(16);
#undef NRLSH_RERANK
    return hipGetLastError();
}

// The screen's theta (k distinct probed items reach it) as the order key the
// bfloat16 re-rank shares between slices (0 = none).
__global__ __launch_bounds__(256) void k_theta_seed(const float *__restrict__ theta, int64_t nq,
                                                    unsigned long long *__restrict__ gtheta)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= nq) return;
    const float t = theta[q];
    gtheta[q] = t > -INFINITY ? (unsigned long long)order_key((double)t) : 0ull;
}

hipError_t launch_theta_seed(const float *theta, int64_t nq, unsigned long long *gtheta, hipStream_t s)
{
    if (nq < 1) return hipSuccess;
    hipLaunchKernelGGL(k_theta_seed, dim3(ceil_div(nq, 256)), dim3(256), 0, s, theta, nq, gtheta);
    return hipGetLastError();
}

hipError_t launch_rerank_lp(const uint16_t *Xh, const float *xeb, const float *Q, int64_t nq,
                            const QueryShape &sh, const int32_t *cand,
                            const int32_t *counts, int nsplit, int lcap, int32_t *lcount, int32_t *lists,
                            unsigned long long *gtheta, hipStream_t s)
{
    const int S = (sh.k + 63) / 64;
    int64_t slice = (sh.Tq + nsplit - 1) / nsplit;
    slice = (slice + 63) / 64 * 64;
    const dim3 grid((unsigned)nq, (unsigned)nsplit), block(64);
    const size_t lds = (size_t)(sh.dp + 127) / 128 * 128 * sizeof(float);
#define NRLSH_RERANK_LP(SS)                                                                         \
    hipLaunchKernelGGL((k_rerank_bf16<SS>), grid, block, lds, s, Xh, xeb, Q, sh.n, sh.d, sh.dp, \
                       sh.Tq, sh.k, cand, counts, slice, lcap, lcount, lists, gtheta)
    if (S <= 1) NRLSH_RERANK_LP(1);
    else if (S <= 2) NRLSH_RERANK_LP(2);
    else if (S <= 4) NRLSH_RERANK_LP(4);
    else if (S <= 8) NRLSH_RERANK_LP(8);
    else NRLSH_RERANK_LP(16);
#undef NRLSH_RERANK_LP
    return hipGetLastError();
}

}  // namespace nrlsh
