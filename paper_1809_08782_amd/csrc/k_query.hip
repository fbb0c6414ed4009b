// Query kernels of norm-ranging LSH for gfx950 (Section 3.3 multi-probe,
// Algorithm 2 re-rank).
//
//   query_hash  code of P(q) = [q; 0] under the shared projections (Eq. 4, 8)
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
#include <climits>
#include <cmath>

#include "nrlsh_internal.h"

namespace nrlsh {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- query_hash
// One wave per query, lane r computes bit r: sum_t A[r][t] q_t in FP64 in
// ascending t (products of two floats are exact in FP64).  At is A[:, :d]
// transposed (d x L) so that the lanes read consecutive words.
__global__ __launch_bounds__(256) void k_query_hash(const float *__restrict__ Q, int64_t nq, int d,
                                                    const float *__restrict__ At, int L, int W,
                                                    uint32_t *__restrict__ qcodes,
                                                    uint32_t *__restrict__ nonfinite)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * 4 + wave;
    if (q >= nq) return;
    const float *qv = Q + q * d;
    const bool act = lane < L;
    double s = 0.0;
    bool bad = false;
    for (int t = 0; t < d; ++t) {
        const float qt = qv[t];
        bad |= !__builtin_isfinite(qt);
        const float a = act ? At[(int64_t)t * L + lane] : 0.f;
        s = s + (double)a * (double)qt;
    }
    const uint64_t code = __ballot(act && s > 0.0);
    if (lane == 0) {
        qcodes[q * W] = (uint32_t)code;
        if (W == 2) qcodes[q * W + 1] = (uint32_t)(code >> 32);
        if (bad) atomicOr(nonfinite, 1u);
    }
}

// ---------------------------------------------------------------- scan pass 1
template <int W>
__global__ __launch_bounds__(64) void k_scan_hist(const uint32_t *__restrict__ codes_l,
                                                  const int32_t *__restrict__ off,
                                                  const uint32_t *__restrict__ qcodes, int64_t nq,
                                                  int m, int L, uint32_t *__restrict__ ghist)
{
    extern __shared__ uint32_t hist[];  // (L+1) x 64, column = lane
    const int lane = threadIdx.x;
    const int tile = blockIdx.x, j = blockIdx.y;
    const int64_t q = (int64_t)tile * 64 + lane;
    uint32_t q0 = 0, q1 = 0;
    if (q < nq) {
        q0 = qcodes[q * W];
        if (W == 2) q1 = qcodes[q * W + 1];
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
// One wave per query tile (lane = query).  inv[b] is the histogram index
// j*(L+1) + h of the bucket with probing rank b.
__global__ __launch_bounds__(64) void k_threshold(const uint32_t *__restrict__ ghist,
                                                  const int32_t *__restrict__ R,
                                                  const int32_t *__restrict__ inv, int64_t nq,
                                                  int m, int L, int64_t Tq,
                                                  int32_t *__restrict__ gbase,
                                                  int32_t *__restrict__ ghthr,
                                                  int32_t *__restrict__ gtie)
{
    const int lane = threadIdx.x, tile = blockIdx.x;
    const int64_t q = (int64_t)tile * 64 + lane;
    const bool valid = q < nq;
    const int L1 = L + 1;
    const int64_t P = (int64_t)m * L1;
    const uint32_t *H = ghist + (int64_t)tile * P * 64;

    int64_t cum = 0;
    int32_t bstar = -1, rstar = 0, jstar = -1, hstar = -1;
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
                if (cum + (int64_t)c[u] >= Tq) {
                    bstar = (int32_t)(b + u);
                    rstar = (int32_t)(Tq - cum);
                    jstar = io[u] / L1;
                    hstar = io[u] - jstar * L1;
                    done = true;
                } else {
                    cum += c[u];
                }
            }
        }
    }

    int32_t run = 0;
    for (int j = 0; j < m; ++j) {
        int hthr = -1;
        int32_t cnt = 0;
        if (valid) {
            int nl = 0;
            for (int l = 0; l <= L; ++l) nl += (R[(int64_t)j * L1 + l] < bstar) ? 1 : 0;
            hthr = nl - 1;
            const uint32_t *Hj = H + (int64_t)j * L1 * 64;
            for (int h = 0; h <= hthr; ++h) cnt += (int32_t)Hj[h * 64 + lane];
            if (j == jstar) cnt += rstar;
        }
        gbase[((int64_t)tile * (m + 1) + j) * 64 + lane] = run;
        ghthr[((int64_t)tile * m + j) * 64 + lane] = hthr;
        run += cnt;
    }
    gbase[((int64_t)tile * (m + 1) + m) * 64 + lane] = run;
    int32_t *tie = gtie + (int64_t)tile * 4 * 64;
    tie[0 * 64 + lane] = valid ? jstar : -1;
    tie[1 * 64 + lane] = hstar;
    tie[2 * 64 + lane] = rstar;
    tie[3 * 64 + lane] = bstar;
}

// ---------------------------------------------------------------- scan pass 2
template <int W>
__global__ __launch_bounds__(64) void k_scan_emit(const uint32_t *__restrict__ codes_l,
                                                  const int32_t *__restrict__ off,
                                                  const uint32_t *__restrict__ qcodes, int64_t nq,
                                                  int m, int L, int64_t Tq,
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
        q0 = qcodes[q * W];
        if (W == 2) q1 = qcodes[q * W + 1];
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

// ---------------------------------------------------------------- rerank
// One wave per (query, slice of its probed list).  Candidates are taken 64
// at a time (lane = candidate); their rows are streamed in 32-float chunks:
// each load instruction brings 8 rows x 128 contiguous bytes, the chunk is
// transposed through LDS and lane c adds q_t x_ct in FP64 in ascending t.
// The running top-k (sorted by (ip desc, id asc)) lives in registers, S
// entries per lane.  With several slices per query, each slice writes a
// partial list and k_topk_merge combines them.
constexpr int RR_STRIDE = 36;  // floats per LDS row (16-byte aligned, conflict-free b128)

__device__ __forceinline__ bool better(double a, int32_t ia, double b, int32_t ib)
{
    return a > b || (a == b && ia < ib);
}

// Sorted top-k list held by one wave: entry e = s*64 + lane.
template <int S>
struct WaveTopK {
    double tv[S];
    int32_t ti[S];
    double th_v;
    int32_t th_i;
    int ks, kl;

    __device__ void init(int k)
    {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            tv[s] = -INFINITY;
            ti[s] = INT_MAX;
        }
        th_v = -INFINITY;
        th_i = INT_MAX;
        ks = (k - 1) >> 6;
        kl = (k - 1) & 63;
    }

    // Offer one value per lane (ok = lane has a real candidate).
    __device__ void offer(double v, int32_t id, bool ok, int lane)
    {
        uint64_t mask = __ballot(ok && better(v, id, th_v, th_i));
        while (mask != 0ull) {
            const int src = __ffsll((long long)mask) - 1;
            mask &= mask - 1ull;
            const double nv = __shfl(v, src, 64);
            const int32_t ni = __shfl(id, src, 64);
            if (!better(nv, ni, th_v, th_i)) continue;
            int pos = 0;
#pragma unroll
            for (int s = 0; s < S; ++s) pos += __popcll(__ballot(better(tv[s], ti[s], nv, ni)));
            double nvv[S];
            int32_t nii[S];
#pragma unroll
            for (int s = 0; s < S; ++s) {
                double up_v = __shfl_up(tv[s], 1, 64);
                int32_t up_i = __shfl_up(ti[s], 1, 64);
                const double carry_v = s > 0 ? __shfl(tv[s > 0 ? s - 1 : 0], 63, 64) : -INFINITY;
                const int32_t carry_i = s > 0 ? __shfl(ti[s > 0 ? s - 1 : 0], 63, 64) : INT_MAX;
                if (lane == 0) {
                    up_v = carry_v;
                    up_i = carry_i;
                }
                const int e = s * 64 + lane;
                nvv[s] = e > pos ? up_v : (e == pos ? nv : tv[s]);
                nii[s] = e > pos ? up_i : (e == pos ? ni : ti[s]);
            }
#pragma unroll
            for (int s = 0; s < S; ++s) {
                tv[s] = nvv[s];
                ti[s] = nii[s];
            }
            th_v = __shfl(tv[ks], kl, 64);
            th_i = __shfl(ti[ks], kl, 64);
        }
    }
};

template <int S>
__global__ __launch_bounds__(64) void k_rerank(const float *__restrict__ Xp,
                                               const int32_t *__restrict__ perm,
                                               const float *__restrict__ Q, int64_t n, int d,
                                               int dp, int64_t Tq, int k,
                                               const int32_t *__restrict__ cand, int nsplit,
                                               int64_t slice, int64_t *__restrict__ out_ids,
                                               float *__restrict__ out_ips,
                                               double *__restrict__ part_v,
                                               int32_t *__restrict__ part_i)
{
    __shared__ float tile[64 * RR_STRIDE];
    const int lane = threadIdx.x;
    const int64_t q = blockIdx.x;
    const int split = blockIdx.y;
    const float *qv = Q + q * d;
    const int32_t *cq = cand + q * Tq;
    const int64_t cbeg = (int64_t)split * slice;
    const int64_t cend = min(Tq, cbeg + slice);
    WaveTopK<S> top;
    top.init(k);
    const int sub = lane >> 3, seg = 4 * (lane & 7);

    for (int64_t c0 = cbeg; c0 < cend; c0 += 64) {
        bool valid = c0 + lane < cend;
        int32_t id = 0;
        if (valid) {
            const int32_t p = cq[c0 + lane];
            valid = p >= 0 && (int64_t)p < n;  // positions come from scan_emit; never trust blindly
            if (valid) id = perm[p];
        }
        int64_t roff[8];
        bool rval[8];
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int rr = 8 * it + sub;
            roff[it] = (int64_t)__shfl(id, rr, 64) * dp;
            rval[it] = __shfl((int)valid, rr, 64) != 0;
        }
        double acc = 0.0;
        for (int k0 = 0; k0 < dp; k0 += 32) {
            const int col = k0 + seg;
#pragma unroll
            for (int it = 0; it < 8; ++it) {
                floatx4 v = floatx4{0.f, 0.f, 0.f, 0.f};
                if (rval[it] && col < dp) v = *reinterpret_cast<const floatx4 *>(Xp + roff[it] + col);
                *reinterpret_cast<floatx4 *>(&tile[(8 * it + sub) * RR_STRIDE + seg]) = v;
            }
            __syncthreads();
            const floatx4 *row = reinterpret_cast<const floatx4 *>(&tile[lane * RR_STRIDE]);
#pragma unroll
            for (int tt = 0; tt < 8; ++tt) {
                const floatx4 x4 = row[tt];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int t = k0 + 4 * tt + u;
                    const float qt = t < d ? qv[t] : 0.f;
                    acc = acc + (double)qt * (double)x4[u];
                }
            }
            __syncthreads();
        }
        top.offer(acc, id, valid, lane);
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

inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

hipError_t launch_query_hash(const float *Q, int64_t nq, int d, const float *At, int L, int W,
                             uint32_t *qcodes, uint32_t *nonfinite, hipStream_t s)
{
    hipLaunchKernelGGL(k_query_hash, dim3(ceil_div(nq, 4)), dim3(256), 0, s, Q, nq, d, At, L, W,
                       qcodes, nonfinite);
    return hipGetLastError();
}

hipError_t launch_scan_hist(const uint32_t *codes_l, const int32_t *off, const uint32_t *qcodes,
                            int64_t nq, const QueryShape &sh, uint32_t *ghist, hipStream_t s)
{
    const dim3 grid(ceil_div(nq, 64), (unsigned)sh.m);
    const size_t lds = (size_t)(sh.L + 1) * 64 * sizeof(uint32_t);
    if (sh.W == 1)
        hipLaunchKernelGGL(k_scan_hist<1>, grid, dim3(64), lds, s, codes_l, off, qcodes, nq, sh.m,
                           sh.L, ghist);
    else
        hipLaunchKernelGGL(k_scan_hist<2>, grid, dim3(64), lds, s, codes_l, off, qcodes, nq, sh.m,
                           sh.L, ghist);
    return hipGetLastError();
}

hipError_t launch_threshold(const uint32_t *ghist, const int32_t *R, const int32_t *inv, int64_t nq,
                            const QueryShape &sh, int32_t *gbase, int32_t *ghthr, int32_t *gtie,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_threshold, dim3(ceil_div(nq, 64)), dim3(64), 0, s, ghist, R, inv, nq, sh.m,
                       sh.L, sh.Tq, gbase, ghthr, gtie);
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
                           sh.L, sh.Tq, gbase, ghthr, gtie, cand);
    else
        hipLaunchKernelGGL(k_scan_emit<2>, grid, dim3(64), 0, s, codes_l, off, qcodes, nq, sh.m,
                           sh.L, sh.Tq, gbase, ghthr, gtie, cand);
    return hipGetLastError();
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

hipError_t launch_rerank(const float *Xp, const int32_t *perm, const float *Q, int64_t nq,
                         const QueryShape &sh, const int32_t *cand, int nsplit, double *part_v,
                         int32_t *part_i, int64_t *out_ids, float *out_ips, hipStream_t s)
{
    const int S = (sh.k + 63) / 64;
    int64_t slice = (sh.Tq + nsplit - 1) / nsplit;
    slice = (slice + 63) / 64 * 64;
    const dim3 grid((unsigned)nq, (unsigned)nsplit), block(64);
#define NRLSH_RERANK(SS)                                                                         \
    do {                                                                                         \
        hipLaunchKernelGGL(k_rerank<SS>, grid, block, 0, s, Xp, perm, Q, sh.n, sh.d, sh.dp,      \
                           sh.Tq, sh.k, cand, nsplit, slice, out_ids, out_ips, part_v, part_i);  \
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

}  // namespace nrlsh
