// Bucket tables: the probe of Section 3.3 through a hash lookup of the
// buckets of each sub-dataset instead of a linear scan of every code.
//
// Table of an index (built once, read-only afterwards):
//   titem   stored positions sorted by (sub-dataset, code, position)
//   ucode   the distinct codes of each sub-dataset, ascending inside it
//   ustart  start of each distinct code's run in titem (ustart[U] = n)
//   uoff    first distinct code of each sub-dataset (uoff[m] = U)
// A bucket (j, l) of the paper is the set of items of sub-dataset j whose
// code agrees with the query's in l bits, i.e. differs in h = L - l bits.
//
// Query, one wave per query, walking the buckets in probing order (the
// sorted (U_j, l) structure) until T items are reached:
//   - ball lookup: the C(L, h) codes at Hamming distance h from the query
//     code are enumerated (colex order, Gosper's successor) and looked up
//     by binary search in sub-dataset j's distinct codes;
//   - once the lookups spent on sub-dataset j would exceed the number of its
//     distinct codes, the wave instead counts every distinct code of j by
//     distance once (a histogram of j's L + 1 buckets) and reads later
//     buckets of j from it.
// The threshold bucket and per-sub-dataset bounds come out in the layout
// of the scan path, so the tie cut (k_tie_locate) and the re-rank are shared;
// the emission visits the same buckets again and copies their items.
#include <climits>

#include "nrlsh_internal.h"

namespace nrlsh {
namespace {

constexpr int TB_BLOCK = 1024;  // elements per block of the build-side scan
constexpr int BINOM_N = 65;     // C(n, k) for 0 <= n, k <= 64

__device__ __forceinline__ uint64_t load_code(const uint32_t *__restrict__ words, int64_t row, int W)
{
    uint64_t c = words[row * W];
    if (W == 2) c |= (uint64_t)words[row * W + 1] << 32;
    return c;
}

// Exclusive prefix sum over the 64 lanes of a wave; *total = the wave's sum.
__device__ __forceinline__ int64_t wave_excl_scan(int64_t v, int64_t *total)
{
    const int lane = threadIdx.x & 63;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    *total = __shfl(x, 63, 64);
    return x - v;
}

__device__ __forceinline__ int64_t wave_sum(int64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Combination of rank r (colex order) of h bits among L: bit p is set when
// r >= C(p, k) for the k bits still to place, scanning p downwards.
__device__ __forceinline__ uint64_t unrank(uint64_t r, int L, int h, const uint64_t *__restrict__ binom)
{
    uint64_t mask = 0;
    int k = h;
    for (int p = L - 1; p >= 0 && k > 0; --p) {
        const uint64_t c = binom[p * BINOM_N + k];
        if (r >= c) {
            mask |= 1ull << p;
            r -= c;
            --k;
        }
    }
    return mask;
}

// Next combination with the same number of bits (Gosper's successor).
__device__ __forceinline__ uint64_t next_comb(uint64_t x)
{
    const uint64_t c = x & (~x + 1ull);
    const uint64_t r = x + c;
    return (((r ^ x) >> 2) >> __builtin_ctzll(x)) | r;
}

// Index of `code` among ucode[u0, u1) (ascending), or -1.
__device__ __forceinline__ int64_t find_code(const uint64_t *__restrict__ ucode, int64_t u0, int64_t u1,
                                             uint64_t code)
{
    int64_t lo = u0, hi = u1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (ucode[mid] < code) lo = mid + 1;
        else hi = mid;
    }
    return (lo < u1 && ucode[lo] == code) ? lo : -1;
}

int bits_for(int64_t v)
{
    int b = 0;
    while ((int64_t(1) << b) <= v && b < 63) ++b;
    return b;
}

// ------------------------------------------------------------------ build
__global__ __launch_bounds__(256) void k_tab_keys(const uint32_t *__restrict__ codes_l, int64_t n, int W,
                                                  uint64_t *__restrict__ key, int32_t *__restrict__ val)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    key[p] = load_code(codes_l, p, W);
    val[p] = (int32_t)p;
}

__global__ __launch_bounds__(256) void k_tab_sidkeys(const int32_t *__restrict__ sid_l,
                                                     const int32_t *__restrict__ val, int64_t n,
                                                     uint64_t *__restrict__ key)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    key[i] = (uint64_t)(uint32_t)sid_l[val[i]];
}

// Element i of the sorted order starts a distinct (sub-dataset, code).
__device__ __forceinline__ bool starts_run(const uint32_t *__restrict__ codes_l, const int32_t *__restrict__ sid_l,
                                           const int32_t *__restrict__ val, int64_t i, int W)
{
    if (i == 0) return true;
    const int32_t a = val[i - 1], b = val[i];
    return sid_l[a] != sid_l[b] || load_code(codes_l, a, W) != load_code(codes_l, b, W);
}

// Pass 1 of the compaction: number of run starts in each block of TB_BLOCK.
__global__ __launch_bounds__(256) void k_tab_count_starts(const uint32_t *__restrict__ codes_l,
                                                          const int32_t *__restrict__ sid_l,
                                                          const int32_t *__restrict__ val, int64_t n,
                                                          int W, int32_t *__restrict__ bsum)
{
    __shared__ int32_t ws[4];
    const int64_t base = (int64_t)blockIdx.x * TB_BLOCK;
    int32_t c = 0;
    for (int e = threadIdx.x; e < TB_BLOCK; e += 256) {
        const int64_t i = base + e;
        if (i < n && starts_run(codes_l, sid_l, val, i, W)) ++c;
    }
    const int64_t t = wave_sum(c);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = (int32_t)t;
    __syncthreads();
    if (threadIdx.x == 0) bsum[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Pass 2: exclusive scan of the block counts (one block); total -> *total.
__global__ __launch_bounds__(256) void k_tab_scan_blocks(int32_t *__restrict__ bsum, int64_t nb,
                                                         int32_t *__restrict__ total)
{
    __shared__ int64_t ws[4];
    __shared__ int64_t carry_s;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += 256) {
        const int64_t b = b0 + threadIdx.x;
        const int64_t v = b < nb ? bsum[b] : 0;
        int64_t wt;
        const int64_t ex = wave_excl_scan(v, &wt);
        if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = wt;
        __syncthreads();
        int64_t before = carry_s;
        for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) before += ws[w];
        if (b < nb) bsum[b] = (int32_t)(before + ex);
        __syncthreads();
        if (threadIdx.x == 0) carry_s += ws[0] + ws[1] + ws[2] + ws[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = (int32_t)carry_s;
}

// Pass 3: write titem, and ucode / ustart at each run start; uoff[j] is set
// at the first run of each non-empty sub-dataset.
__global__ __launch_bounds__(256) void k_tab_scatter(const uint32_t *__restrict__ codes_l,
                                                     const int32_t *__restrict__ sid_l,
                                                     const int32_t *__restrict__ val, int64_t n, int W,
                                                     const int32_t *__restrict__ bbase,
                                                     int32_t *__restrict__ titem,
                                                     uint64_t *__restrict__ ucode,
                                                     int32_t *__restrict__ ustart,
                                                     int32_t *__restrict__ uoff)
{
    __shared__ int64_t ws[4];
    const int64_t base = (int64_t)blockIdx.x * TB_BLOCK;
    // thread t owns elements base + 4t .. base + 4t + 3 (in order)
    bool f[4];
    int32_t c = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t i = base + 4 * threadIdx.x + e;
        f[e] = i < n && starts_run(codes_l, sid_l, val, i, W);
        c += f[e] ? 1 : 0;
    }
    int64_t wt;
    const int64_t ex = wave_excl_scan(c, &wt);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = wt;
    __syncthreads();
    int64_t u = bbase[blockIdx.x] + ex;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) u += ws[w];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t i = base + 4 * threadIdx.x + e;
        if (i >= n) break;
        const int32_t v = val[i];
        titem[i] = v;
        if (f[e]) {
            ucode[u] = load_code(codes_l, v, W);
            ustart[u] = (int32_t)i;
            const int32_t sj = sid_l[v];
            if (i == 0 || sid_l[val[i - 1]] != sj) uoff[sj] = (int32_t)u;
            ++u;
        }
    }
}

// ------------------------------------------------------------------ query
struct TabCounters {
    unsigned long long lookups;  // ball lookups (codes searched)
    unsigned long long walked;   // distinct codes counted by whole-sub-dataset passes
    unsigned long long passes;   // whole-sub-dataset passes
};

// Ball count / emission of bucket (j, h): every code at distance h from qc
// is searched among ucode[u0, u1).  With emit, found runs are appended.
template <bool EMIT>
__device__ __forceinline__ int64_t ball(const uint64_t *__restrict__ ucode, const int32_t *__restrict__ ustart,
                                        const int32_t *__restrict__ titem, const uint64_t *__restrict__ binom,
                                        int64_t u0, int64_t u1, uint64_t qc, int L, int h, bool whole,
                                        int32_t pstar, int32_t *__restrict__ out, int64_t cap, int64_t w0)
{
    const int lane = threadIdx.x & 63;
    const uint64_t tot = binom[L * BINOM_N + h];
    const uint64_t per = (tot + 63) / 64;
    const uint64_t r0 = per * (uint64_t)lane;
    const uint64_t r1 = r0 + per < tot ? r0 + per : tot;
    int64_t w = w0, found = 0;
    uint64_t mask = r0 < r1 ? unrank(r0, L, h, binom) : 0;
    // lanes run the same number of steps so that the emission scans stay converged
    for (uint64_t k = 0; k < per; ++k) {
        const uint64_t r = r0 + k;
        int64_t s = 0, cnt = 0;
        if (r < r1) {
            const int64_t u = find_code(ucode, u0, u1, qc ^ mask);
            if (u >= 0) {
                s = ustart[u];
                const int64_t e = ustart[u + 1];
                if (whole) {
                    cnt = e - s;
                } else {  // threshold bucket: stored positions <= P* only (ascending in a run)
                    while (s + cnt < e && titem[s + cnt] <= pstar) ++cnt;
                }
            }
            if (r + 1 < r1 && h > 0) mask = next_comb(mask);
        }
        found += cnt;
        if (EMIT) {
            int64_t wt;
            const int64_t ex = wave_excl_scan(cnt, &wt);
            for (int64_t t = 0; t < cnt; ++t)
                if (w + ex + t < cap) out[w + ex + t] = titem[s + t];
            w += wt;
        }
    }
    return EMIT ? w - w0 : wave_sum(found);
}

// Pass over every distinct code of sub-dataset j: per-bucket counts into
// lh (L + 1 words of this wave's LDS), or, with EMIT, append the runs of
// buckets h <= hthr and, for h == htie, their positions <= P*.
template <bool EMIT>
__device__ __forceinline__ int64_t walk(const uint64_t *__restrict__ ucode, const int32_t *__restrict__ ustart,
                                        const int32_t *__restrict__ titem, int64_t u0, int64_t u1,
                                        uint64_t qc, uint32_t *lh, int hthr, int htie, int32_t pstar,
                                        int32_t *__restrict__ out, int64_t cap, int64_t w0)
{
    const int lane = threadIdx.x & 63;
    int64_t w = w0;
    for (int64_t b = u0; b < u1; b += 64) {
        const int64_t u = b + lane;
        int64_t s = 0, cnt = 0;
        if (u < u1) {
            const int h = __popcll(ucode[u] ^ qc);
            s = ustart[u];
            const int64_t e = ustart[u + 1];
            if (!EMIT) {
                atomicAdd(&lh[h], (uint32_t)(e - s));
            } else if (h <= hthr) {
                cnt = e - s;
            } else if (h == htie) {
                while (s + cnt < e && titem[s + cnt] <= pstar) ++cnt;
            }
        }
        if (EMIT) {
            int64_t wt;
            const int64_t ex = wave_excl_scan(cnt, &wt);
            for (int64_t t = 0; t < cnt; ++t)
                if (w + ex + t < cap) out[w + ex + t] = titem[s + t];
            w += wt;
        }
    }
    return w - w0;
}

// One wave per query: walk the buckets in probing order until Tq items.
// qstate[q][j]: lookups spent on j so far (>= 0) or -1 once j's histogram
// qhist[q][j][0..L] has been taken.  Writes ghthr / gtie as the scan path's
// threshold does (tile layout) and, for each query, its rank b* in gtie.
template <int W>
__global__ __launch_bounds__(256) void k_tab_count(
    const uint64_t *__restrict__ ucode, const int32_t *__restrict__ ustart,
    const int32_t *__restrict__ uoff, const int32_t *__restrict__ titem,
    const uint64_t *__restrict__ binom, const int32_t *__restrict__ R, const int32_t *__restrict__ inv,
    const uint32_t *__restrict__ qcodes, int qsets, int64_t nq, int m, int L, int64_t Tq,
    int32_t *__restrict__ qstate, int32_t *__restrict__ qhist, int32_t *__restrict__ ghthr,
    int32_t *__restrict__ gtie, TabCounters *__restrict__ ctr)
{
    __shared__ uint32_t lh_s[4][68];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * 4 + wave;
    if (q >= nq) return;  // no block-wide barrier below
    uint32_t *lh = lh_s[wave];
    const int L1 = L + 1;
    for (int h = lane; h < L1; h += 64) lh[h] = 0u;
    const int64_t P = (int64_t)m * L1;
    int64_t cum = 0;
    int32_t bstar = -1, jstar = -1, hstar = -1, rstar = 0;
    bool rfull = false;
    unsigned long long lookups = 0, walked = 0, passes = 0;
    for (int64_t b = 0; b < P; ++b) {
        const int idx = inv[b];
        const int j = idx / L1, h = idx - j * L1;
        const int64_t u0 = uoff[j], u1 = uoff[j + 1];
        if (u1 == u0) continue;
        const uint64_t qc = load_code(qcodes, qrow(q, j, qsets), W);
        int32_t *st = qstate + q * m + j;
        int32_t *hj = qhist + (q * m + j) * L1;
        const int32_t spent = *st;
        int64_t c;
        if (spent < 0) {
            c = hj[h];
        } else {
            const int64_t nu = u1 - u0;
            const uint64_t tot = binom[L * BINOM_N + h];
            const int64_t steps = 64 - __builtin_clzll((unsigned long long)nu);  // search depth
            const bool use_ball = tot <= (uint64_t)nu && (int64_t)spent + (int64_t)tot * steps <= nu;
            if (use_ball) {
                c = ball<false>(ucode, ustart, titem, binom, u0, u1, qc, L, h, true, 0, nullptr, 0, 0);
                lookups += tot;
                if (lane == 0) *st = spent + (int32_t)(tot * steps);
            } else {
                walk<false>(ucode, ustart, titem, u0, u1, qc, lh, 0, 0, 0, nullptr, 0, 0);
                walked += (unsigned long long)nu;
                ++passes;
                __builtin_amdgcn_wave_barrier();
                c = lh[h];
                for (int t = lane; t < L1; t += 64) {
                    hj[t] = (int32_t)lh[t];
                    lh[t] = 0u;
                }
                if (lane == 0) *st = -1;
                // later reads of hj / st by this wave see these writes
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (cum + c >= Tq) {
            bstar = (int32_t)b;
            rstar = (int32_t)(Tq - cum);
            rfull = cum + c == Tq;
            jstar = j;
            hstar = h;
            break;
        }
        cum += c;
    }
    const int tile = (int)(q >> 6), ql = (int)(q & 63);
    for (int j = lane; j < m; j += 64) {
        int nl = 0;
        for (int l = 0; l <= L; ++l) nl += (R[(int64_t)j * L1 + l] < bstar) ? 1 : 0;
        ghthr[((int64_t)tile * m + j) * 64 + ql] = nl - 1;
    }
    if (lane == 0) {
        int32_t *tie = gtie + (int64_t)tile * 4 * 64;
        tie[ql] = jstar;
        tie[64 + ql] = hstar;
        tie[128 + ql] = rfull ? INT_MAX : rstar;
        tie[192 + ql] = bstar;
        atomicAdd(&ctr->lookups, lookups);
        atomicAdd(&ctr->walked, walked);
        atomicAdd(&ctr->passes, passes);
    }
}

// One wave per query: copy the probed items (stored positions) into the
// query's list, sub-dataset by sub-dataset, in the mode the count pass used.
template <int W>
__global__ __launch_bounds__(256) void k_tab_emit(
    const uint64_t *__restrict__ ucode, const int32_t *__restrict__ ustart,
    const int32_t *__restrict__ uoff, const int32_t *__restrict__ titem,
    const uint64_t *__restrict__ binom, const uint32_t *__restrict__ qcodes, int qsets, int64_t nq,
    int m, int L, int64_t Tq, const int32_t *__restrict__ qstate, const int32_t *__restrict__ ghthr,
    const int32_t *__restrict__ gtie, const int32_t *__restrict__ gpstar, int32_t *__restrict__ cand)
{
    const int wave = threadIdx.x >> 6;
    const int64_t q = (int64_t)blockIdx.x * 4 + wave;
    if (q >= nq) return;
    const int tile = (int)(q >> 6), ql = (int)(q & 63);
    const int32_t *tie = gtie + (int64_t)tile * 4 * 64;
    const int jstar = tie[ql], hstar = tie[64 + ql];
    const int32_t pstar = jstar >= 0 ? gpstar[q] : -1;
    int32_t *out = cand + q * Tq;
    int64_t w = 0;
    for (int j = 0; j < m; ++j) {
        const int hthr = ghthr[((int64_t)tile * m + j) * 64 + ql];
        const int htie = j == jstar ? hstar : -1;
        if (hthr < 0 && htie < 0) continue;
        const int64_t u0 = uoff[j], u1 = uoff[j + 1];
        if (u1 == u0) continue;
        const uint64_t qc = load_code(qcodes, qrow(q, j, qsets), W);
        if (qstate[q * m + j] < 0) {
            w += walk<true>(ucode, ustart, titem, u0, u1, qc, nullptr, hthr, htie, pstar, out, Tq, w);
        } else {
            const int hmax = hthr > htie ? hthr : htie;
            for (int h = 0; h <= hmax; ++h) {
                const bool whole = h <= hthr;
                if (!whole && h != htie) continue;
                w += ball<true>(ucode, ustart, titem, binom, u0, u1, qc, L, h, whole, pstar, out, Tq, w);
            }
        }
    }
}

inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

// ------------------------------------------------------------------ launchers
size_t table_binom_words() { return (size_t)BINOM_N * BINOM_N; }

void table_binom(uint64_t *out)
{
    for (int n = 0; n < BINOM_N; ++n)
        for (int k = 0; k < BINOM_N; ++k) {
            uint64_t v;
            if (k > n) v = 0;
            else if (k == 0 || k == n) v = 1;
            else v = out[(n - 1) * BINOM_N + k - 1] + out[(n - 1) * BINOM_N + k];
            out[n * BINOM_N + k] = v;
        }
}

size_t table_scan_words(int64_t n) { return (size_t)((n + TB_BLOCK - 1) / TB_BLOCK) + 1; }

hipError_t launch_table_build(const uint32_t *codes_l, const int32_t *sid_l, int64_t n, int m, int L,
                              uint64_t *ka, int32_t *va, uint64_t *kb, int32_t *vb, void *sort_tmp,
                              int32_t *bsum, int32_t *total, int32_t *titem, uint64_t *ucode,
                              int32_t *ustart, int32_t *uoff, hipStream_t s)
{
    const int W = L > 32 ? 2 : 1;
    hipLaunchKernelGGL(k_tab_keys, dim3(ceil_div(n, 256)), dim3(256), 0, s, codes_l, n, W, ka, va);
    bool in_b = false;
    hipError_t e = radix_sort(ka, va, kb, vb, n, (L + 7) / 8 * 8, sort_tmp, &in_b, s);
    if (e != hipSuccess) return e;
    uint64_t *k1 = in_b ? kb : ka, *k2 = in_b ? ka : kb;
    int32_t *v1 = in_b ? vb : va, *v2 = in_b ? va : vb;
    const int sbits = (bits_for(m - 1) + 7) / 8 * 8;
    if (sbits > 0) {
        hipLaunchKernelGGL(k_tab_sidkeys, dim3(ceil_div(n, 256)), dim3(256), 0, s, sid_l, v1, n, k1);
        bool b2 = false;
        e = radix_sort(k1, v1, k2, v2, n, sbits, sort_tmp, &b2, s);
        if (e != hipSuccess) return e;
        if (b2) v1 = v2;
    }
    const int64_t nb = (n + TB_BLOCK - 1) / TB_BLOCK;
    hipLaunchKernelGGL(k_tab_count_starts, dim3((unsigned)nb), dim3(256), 0, s, codes_l, sid_l, v1, n, W,
                       bsum);
    hipLaunchKernelGGL(k_tab_scan_blocks, dim3(1), dim3(256), 0, s, bsum, nb, total);
    hipLaunchKernelGGL(k_tab_scatter, dim3((unsigned)nb), dim3(256), 0, s, codes_l, sid_l, v1, n, W,
                       bsum, titem, ucode, ustart, uoff);
    return hipGetLastError();
}

hipError_t launch_table_count(const TableView &T, const int32_t *R, const int32_t *inv,
                              const uint32_t *qcodes, int64_t nq, const QueryShape &sh, int32_t *qstate,
                              int32_t *qhist, int32_t *ghthr, int32_t *gtie, void *counters,
                              hipStream_t s)
{
    TabCounters *c = static_cast<TabCounters *>(counters);
    if (sh.W == 1)
        hipLaunchKernelGGL(k_tab_count<1>, dim3(ceil_div(nq, 4)), dim3(256), 0, s, T.ucode, T.ustart,
                           T.uoff, T.titem, T.binom, R, inv, qcodes, sh.qsets, nq, sh.m, sh.L, sh.Tq,
                           qstate, qhist, ghthr, gtie, c);
    else
        hipLaunchKernelGGL(k_tab_count<2>, dim3(ceil_div(nq, 4)), dim3(256), 0, s, T.ucode, T.ustart,
                           T.uoff, T.titem, T.binom, R, inv, qcodes, sh.qsets, nq, sh.m, sh.L, sh.Tq,
                           qstate, qhist, ghthr, gtie, c);
    return hipGetLastError();
}

hipError_t launch_table_emit(const TableView &T, const uint32_t *qcodes, int64_t nq, const QueryShape &sh,
                             const int32_t *qstate, const int32_t *ghthr, const int32_t *gtie,
                             const int32_t *gpstar, int32_t *cand, hipStream_t s)
{
    if (sh.W == 1)
        hipLaunchKernelGGL(k_tab_emit<1>, dim3(ceil_div(nq, 4)), dim3(256), 0, s, T.ucode, T.ustart,
                           T.uoff, T.titem, T.binom, qcodes, sh.qsets, nq, sh.m, sh.L, sh.Tq, qstate,
                           ghthr, gtie, gpstar, cand);
    else
        hipLaunchKernelGGL(k_tab_emit<2>, dim3(ceil_div(nq, 4)), dim3(256), 0, s, T.ucode, T.ustart,
                           T.uoff, T.titem, T.binom, qcodes, sh.qsets, nq, sh.m, sh.L, sh.Tq, qstate,
                           ghthr, gtie, gpstar, cand);
    return hipGetLastError();
}

size_t table_counter_bytes() { return sizeof(TabCounters); }

}  // namespace nrlsh
