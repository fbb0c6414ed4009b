// Index-build kernels of norm-ranging LSH (Algorithm 1) for gfx950.
//
//   keys        squared 2-norms (FP64, ascending coordinate order)
//                                                          [Algorithm 1, ranking]
//   radix sort  stable LSD sort of (key bits, index)      [Algorithm 1, ranking]
//   assign      sub-dataset by norm percentile, U_j        [Algorithm 1, partition]
//   layout      zero-padded item copy in stored order (sub-dataset major)
//   hash        SimpleLSH transform (Eq. 8) + sign random projection (Eq. 4)
//               on the FP32 matrix cores, sign packing, uncertainty band
//   hash_fixup  FP64 recompute of in-band projections as the definition
#include "nrlsh_internal.h"

namespace nrlsh {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint64_t lanemask_lt(int lane) { return (1ull << lane) - 1ull; }

// ---------------------------------------------------------------- keys
// One wave owns 64 consecutive rows.  Columns are streamed 32 at a time:
// each load instruction brings up to 16 bytes per lane, 8 rows x 128 contiguous
// bytes, and the next chunk's loads are in flight while the current chunk is
// transposed through LDS and summed: lane r adds the squares of row r in
// ascending column order.  Squares of FP32 values are exact in FP64, so the
// sum is bit-identical to a sequential FP64 loop.
constexpr int KC_ROWS = 64;

template <int VW>
__global__ __launch_bounds__(256) void k_keys(const float *__restrict__ X, int64_t n, int d,
                                              double *__restrict__ key,
                                              uint64_t *__restrict__ skey,
                                              int32_t *__restrict__ sval,
                                              BuildCounters *__restrict__ ctr)
{
    __shared__ float tile[4][KC_ROWS][33];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * KC_ROWS;
    const int sub = lane >> 3, seg = 4 * (lane & 7);  // row 8 it + sub, columns seg .. seg + 3
    // Loads are issued from addresses clamped into the matrix and the values
    // are masked only where the chunk is written to LDS, one chunk later,
    // so the next chunk's loads stay in flight while this one is summed.
    // VW: floats per load, the widest that d % VW == 0 keeps aligned.
    auto load = [&](floatx4 (&v)[8], int c0) {
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int64_t row = row0 + 8 * it + sub;
            const float *p = X + (row < n ? row : 0) * (int64_t)d;
            const int c = c0 + seg;
            // a column past d reads the row's last VW floats instead, which
            // the same or the previous chunk has just brought into the caches
            if constexpr (VW == 4) {
                v[it] = *reinterpret_cast<const floatx4 *>(p + min(c, d - 4));
            } else if constexpr (VW == 2) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const floatx2 t = *reinterpret_cast<const floatx2 *>(p + min(c + 2 * h, d - 2));
                    v[it][2 * h] = t[0];
                    v[it][2 * h + 1] = t[1];
                }
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) v[it][u] = p[min(c + u, d - 1)];
            }
        }
    };
    // tile[wave] is written and read by its own wave only: LDS operations of
    // one wave complete in issue order, so a wave-level barrier that keeps the
    // compiler from moving them across suffices.
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    double acc = 0.0;
    bool bad = false;
    auto consume = [&](const floatx4 (&v)[8], int c0) {
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const bool rok = row0 + 8 * it + sub < n;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float x = rok && c0 + seg + u < d ? v[it][u] : 0.f;
                bad |= !__builtin_isfinite(x);
                tile[wave][8 * it + sub][seg + u] = x;
            }
        }
        wave_sync();
        // columns past d hold zeros, and adding +0 leaves a non-negative sum unchanged
#pragma unroll
        for (int t = 0; t < 32; ++t) {
            const double x = (double)tile[wave][lane][t];
            acc = acc + x * x;
        }
        wave_sync();
    };
    // Two register buffers taken in turn, with no copy between them and no
    // branch around a load or between a load and the chunk before it: either
    // lets the compiler wait for the loads in flight.  Chunks go in pairs; a
    // chunk past d rereads cached columns (clamped) and adds only zeros.
    floatx4 va[8], vb[8];
    load(va, 0);
    for (int c0 = 0; c0 < d; c0 += 64) {
        load(vb, c0 + 32);
        consume(va, c0);
        load(va, c0 + 64);
        consume(vb, c0 + 32);
    }
    const int64_t myrow = row0 + lane;
    if (myrow < n) {
        key[myrow] = acc;
        skey[myrow] = (uint64_t)__double_as_longlong(acc);
        sval[myrow] = (int32_t)myrow;
    }
    if (__ballot(bad) != 0ull && lane == 0) atomicOr(&ctr->nonfinite, 1u);
}

// ---------------------------------------------------------------- radix sort
constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint64_t *__restrict__ keys,
                                                        int64_t n, int shift,
                                                        uint32_t *__restrict__ bhist, int nblocks)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll 4
    for (int it = 0; it < RS_ITEMS; ++it) {
        const int64_t e = base + it * RS_THREADS + threadIdx.x;
        if (e < n) atomicAdd(&h[(keys[e] >> shift) & 255u], 1u);
    }
    __syncthreads();
    bhist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__device__ __forceinline__ uint32_t block_incl_scan_256(uint32_t v, uint32_t *s)
{
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t t = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0u;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    return s[threadIdx.x];
}

// One block per digit: exclusive scan of that digit's per-block counts.
__global__ __launch_bounds__(256) void k_rs_scan(uint32_t *__restrict__ bhist, int nblocks,
                                                 uint32_t *__restrict__ totals)
{
    __shared__ uint32_t s[256];
    uint32_t *row = bhist + (int64_t)blockIdx.x * nblocks;
    uint32_t carry = 0;
    for (int c0 = 0; c0 < nblocks; c0 += 256) {
        const int i = c0 + threadIdx.x;
        const uint32_t v = i < nblocks ? row[i] : 0u;
        const uint32_t incl = block_incl_scan_256(v, s);  // s[] still holds the scan
        if (i < nblocks) row[i] = carry + incl - v;
        carry += s[255];  // total of this chunk
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// Stable scatter of one 8-bit digit.  Each block walks its tile in order,
// 256 keys per round; ranks inside a wave come from ballot matching, ranks
// across the 4 waves from per-wave digit counts in LDS.
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(
    const uint64_t *__restrict__ kin, const int32_t *__restrict__ vin, int64_t n, int shift,
    const uint32_t *__restrict__ bhist, int nblocks, const uint32_t *__restrict__ totals,
    uint64_t *__restrict__ kout, int32_t *__restrict__ vout)
{
    __shared__ uint32_t sbuf[256];
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint32_t woff[4][256];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const uint32_t tot = totals[t];
    const uint32_t incl = block_incl_scan_256(tot, sbuf);
    base[t] = incl - tot + bhist[(int64_t)t * nblocks + blockIdx.x];
#pragma unroll
    for (int w = 0; w < 4; ++w) wcnt[w][t] = 0u;
    __syncthreads();
    const int64_t tile = (int64_t)blockIdx.x * RS_TILE;
    for (int it = 0; it < RS_ITEMS; ++it) {
        const int64_t e = tile + it * RS_THREADS + t;
        const bool valid = e < n;
        uint64_t k = 0;
        int32_t v = 0;
        if (valid) {
            k = kin[e];
            v = vin[e];
        }
        const uint32_t dg = (uint32_t)(k >> shift) & 255u;
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bal = __ballot((dg >> b) & 1u);
            match &= ((dg >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(match & lanemask_lt(lane));
        const bool last = valid && ((match >> lane) >> 1) == 0ull;
        if (last) wcnt[wave][dg] = (uint32_t)__popcll(match);
        __syncthreads();
        {
            uint32_t run = base[t];
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                woff[w][t] = run;
                run += wcnt[w][t];
                wcnt[w][t] = 0u;
            }
            base[t] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = woff[wave][dg] + rank;
            kout[pos] = k;
            vout[pos] = v;
        }
    }
}

// ---------------------------------------------------------------- partition
// Sub-dataset of the item at sorted rank r: by percentile, floor(r m / n)
// (Algorithm 1); with `bounds` (m - 1 increasing squared boundaries, the
// uniform ranges of Section 5), the number of boundaries its key reaches.
// Both are nondecreasing in r, so every sub-dataset is a run of ranks; the
// last rank of a run writes the run's largest key and its end (subend,
// sub-datasets without items keep what the caller set).
__device__ __forceinline__ int64_t range_of(const double *__restrict__ bounds, int nb, double key)
{
    int lo = 0, hi = nb;  // number of bounds <= key
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (bounds[mid] <= key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_assign(const uint64_t *__restrict__ skey,
                                                const int32_t *__restrict__ sidx, int64_t n, int m,
                                                const double *__restrict__ bounds,
                                                int32_t *__restrict__ sid,
                                                uint64_t *__restrict__ lkey,
                                                int32_t *__restrict__ lval,
                                                double *__restrict__ keymax,
                                                int32_t *__restrict__ subend)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int32_t i = sidx[r];
    const double key = __longlong_as_double((long long)skey[r]);
    const int64_t s = bounds ? range_of(bounds, m - 1, key) : (r * (int64_t)m) / n;
    sid[i] = (int32_t)s;
    lkey[i] = (uint64_t)s;
    lval[r] = (int32_t)r;
    bool last = r == n - 1;
    if (!last) {
        const double kn = __longlong_as_double((long long)skey[r + 1]);
        last = (bounds ? range_of(bounds, m - 1, kn) : ((r + 1) * (int64_t)m) / n) != s;
    }
    if (last) {
        keymax[s] = key;
        subend[s] = (int32_t)(r + 1);
    }
}

// Stored copy: row p of Xl is item perm[p], zero-padded to dp floats; the
// key and sub-dataset of each stored row come along.  The same rows are also
// rounded to bfloat16 (hi = bf16(x), round to nearest even) for the
// query-tiled screen and, when Xlo is given, split further into lo =
// bf16(x - hi) (|x - hi - lo| <= 2^-16 |x|).
// A wave copies LY_ROWS consecutive stored rows: their source indices are
// read once, then the rows are treated as one run of 4-float groups, each
// read in VW-float pieces (VW = the widest of 4, 2, 1 dividing d, so no
// piece crosses an item's row end), of which each lane keeps LY_B groups in
// flight before storing them whole.
constexpr int LY_ROWS = 16;
constexpr int LY_B = 8;

__device__ __forceinline__ uint16_t bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <int VW>
struct LyVec;
template <>
struct LyVec<4> {
    using F = floatx4;
    using H = ushort4;
};
template <>
struct LyVec<2> {
    using F = floatx2;
    using H = ushort2;
};
template <>
struct LyVec<1> {
    using F = float;
    using H = uint16_t;
};

template <int VW>
__global__ __launch_bounds__(256) void k_layout(const float *__restrict__ X, int64_t n, int d,
                                                int dp, const int32_t *__restrict__ perm,
                                                const double *__restrict__ key,
                                                const int32_t *__restrict__ sid,
                                                float *__restrict__ Xl, uint16_t *__restrict__ Xh,
                                                uint16_t *__restrict__ Xlo,
                                                double *__restrict__ key_l,
                                                int32_t *__restrict__ sid_l,
                                                float *__restrict__ xeb)
{
    using F = typename LyVec<VW>::F;
    __shared__ float dsq_s[4][LY_ROWS];  // per stored row: sum of (x - bf16(x))^2
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t p0 = ((int64_t)blockIdx.x * 4 + wave) * LY_ROWS;
    const bool mine = lane < LY_ROWS && p0 + lane < n;
    const int32_t src_row = mine ? perm[p0 + lane] : 0;
    if (mine) {
        key_l[p0 + lane] = key[src_row];
        sid_l[p0 + lane] = sid[src_row];
    }
    if (lane < LY_ROWS) dsq_s[wave][lane] = 0.f;
    // each lane element is a group of 4 stored floats (dp is a multiple of
    // 8, so groups never cross a stored row and their stores are 16- and
    // 8-byte aligned), loaded as 4 / VW pieces that lie wholly inside or
    // wholly past the item's d values
    const int nv = dp / 4;  // groups per stored row
    const int total = LY_ROWS * nv;
    for (int e0 = 0; e0 < total; e0 += 64 * LY_B) {
        float v[LY_B][4];
        int64_t dst[LY_B];  // first stored element of the group, -1 = none
        int rr[LY_B];       // its row within the wave's rows
#pragma unroll
        for (int b = 0; b < LY_B; ++b) {
            const int e = e0 + 64 * b + lane;
            const int r = e / nv, c = (e - r * nv) * 4;
            rr[b] = r;
            const int64_t i = __shfl(src_row, r & (LY_ROWS - 1), 64);
            const bool ok = e < total && p0 + r < n;
            dst[b] = ok ? (p0 + r) * dp + c : -1;
#pragma unroll
            for (int q = 0; q < 4 / VW; ++q) {
                const int cc = c + q * VW;
                F t = F{};
                if (ok && cc < d) t = *reinterpret_cast<const F *>(X + i * d + cc);
#pragma unroll
                for (int u = 0; u < VW; ++u) v[b][q * VW + u] = reinterpret_cast<const float *>(&t)[u];
            }
        }
#pragma unroll
        for (int b = 0; b < LY_B; ++b) {
            if (dst[b] < 0) continue;
            floatx4 t;
            ushort4 h, l;
            float sq = 0.f;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint16_t hu = bf16_rne(v[b][u]);
                // x - bf16(x) is exact in FP32 (the two share their leading bits)
                const float dl = v[b][u] - __uint_as_float((uint32_t)hu << 16);
                t[u] = v[b][u];
                reinterpret_cast<uint16_t *>(&h)[u] = hu;
                reinterpret_cast<uint16_t *>(&l)[u] = bf16_rne(dl);
                sq += dl * dl;
            }
            *reinterpret_cast<floatx4 *>(Xl + dst[b]) = t;
            *reinterpret_cast<ushort4 *>(Xh + dst[b]) = h;
            if (Xlo) *reinterpret_cast<ushort4 *>(Xlo + dst[b]) = l;
            if (xeb) atomicAdd(&dsq_s[wave][rr[b]], sq);
        }
    }
    // error bound of the bfloat16 image of each row: ||x - bf16(x)|| (an FP32
    // sum of d rounded squares is at most (1 + (d + 2) 2^-23) below the exact
    // one; squares under the FP32 range add at most 2^-50 once rooted), plus
    // (d + 8) 2^-23 ||x|| for an FP32 sum, in any order and with fused
    // multiply-adds, of the dp <= d + 7 products of q with bf16(x) (at most
    // gamma_dp (1 + 2^-8) ||q|| ||x|| off), rounded up to FP32
    if (xeb && mine) {
        const double s2 = (double)dsq_s[wave][lane] * (1.0 + (double)(d + 2) * 0x1p-23);
        const double b = __builtin_sqrt(s2) * (1.0 + 0x1p-40) + 0x1p-50 +
                         (double)(d + 8) * 0x1p-23 * __builtin_sqrt(key[src_row]) * (1.0 + 0x1p-40);
        xeb[p0 + lane] = (float)(b * (1.0 + 0x1p-22));
    }
}

// lo = bf16(x - hi) of every stored value, from the FP32 copy and its hi part.
__global__ __launch_bounds__(256) void k_lo_rows(const float *__restrict__ Xl, const uint16_t *__restrict__ Xh,
                                                 int64_t count, uint16_t *__restrict__ Xlo)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256)
        Xlo[e] = bf16_rne(Xl[e] - __uint_as_float((uint32_t)Xh[e] << 16));
}

// ---------------------------------------------------------------- hash
// Items are the rows (M), hash bits the columns (N), coordinates the
// reduction (K) of v_mfma_f32_16x16x4_f32.  Each wave owns 64 items (4 row
// blocks of 16) and all L bits (CB column blocks of 16).  Per 16 coordinates
// a lane loads one float4 of a row (4 lanes cover 64 contiguous bytes of a
// row) and one float4 of a projection row from LDS, and issues 4 MFMAs per
// (row block, column block): in MFMA j, lane group g contributes coordinate
// 16 kk + 4 g + j for both operands, which is a permutation of the reduction
// and leaves the product unchanged.
//
// Epilogue (scaled SimpleLSH transform, Eq. 8): with s_i = sqrt(keymax_j -
// key_i), U_j a^T P(x_i / U_j) = a[:d]^T x_i + a_d s_i, whose sign is the
// hash bit (U_j > 0).  The FP32 result is trusted only outside the band
// |p| <= tau_r U_j, tau_r = 2 gamma_{d+3} ||a_r||, which bounds the rounding
// error of any summation order; in-band bits and sub-datasets with U_j
// outside [2^-60, 2^60] are recomputed in FP64 by k_hash_fixup.
constexpr int H_WAVES = 8;
constexpr int H_KC = 128;
constexpr int H_KS = H_KC + 4;

// With `rows` != NULL the kernel re-hashes the items rows[0 .. n) (a list of
// stored positions, n = its length) and counts the bits it changes.  With
// `bstart` != NULL every sub-dataset has its own projection block: block b
// hashes stored positions of sub-dataset j (bstart[j] <= b < bstart[j+1],
// found by binary search) with rows j L .. j L + L - 1 of A and tau; the
// n argument is unused and the items end at off[j+1].
template <int CB>
__global__ __launch_bounds__(H_WAVES * 64) void k_hash(
    const float *__restrict__ Xl, int64_t n, int d, int dp, const float *__restrict__ A_all, int L,
    const double *__restrict__ key_l, const int32_t *__restrict__ sid_l,
    const double *__restrict__ keymax, const double *__restrict__ U,
    const float *__restrict__ tau_all, uint32_t *__restrict__ codes_l, FixEntry *__restrict__ fix,
    BuildCounters *__restrict__ ctr, const int32_t *__restrict__ rows,
    const int32_t *__restrict__ off, const int32_t *__restrict__ bstart, int m)
{
    constexpr int NB = 16 * CB;
    __shared__ float As[NB * H_KS];
    __shared__ float sq_s[H_WAVES][64];
    __shared__ float uf_s[H_WAVES][64];
    __shared__ int sp_s[H_WAVES][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int64_t i0 = ((int64_t)blockIdx.x * H_WAVES + wave) * 64;
    const float *A = A_all;
    const float *tau = tau_all;
    if (bstart) {
        // largest j with bstart[j] <= b; an empty sub-dataset owns no block,
        // so ties resolve to the last of equal starts, the one holding b
        int lo = 0, hi = m;  // bstart[lo] <= b < bstart[hi]
        const int b = (int)blockIdx.x;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (bstart[mid] <= b) lo = mid;
            else hi = mid;
        }
        i0 = (int64_t)off[lo] + ((int64_t)(b - bstart[lo]) * H_WAVES + wave) * 64;
        n = off[lo + 1];
        A = A_all + (int64_t)lo * L * (d + 1);
        tau = tau_all + (int64_t)lo * L;
    }
    {
        const int64_t i = i0 + lane;
        float sq = 0.f, uf = 0.f;
        int sp = 1;
        if (i < n) {
            const int s = sid_l[rows ? rows[i] : i];
            const double km = keymax[s], u = U[s];
            sq = sqrtf((float)(km - key_l[rows ? rows[i] : i]));
            uf = (float)u;
            sp = !(u >= 0x1p-60 && u <= 0x1p60);
        }
        sq_s[wave][lane] = sq;
        uf_s[wave][lane] = uf;
        sp_s[wave][lane] = sp;
    }
    // stored positions of this lane's four row-block rows (identity without a
    // list); a row past n reads row n - 1 instead: an MFMA output row depends
    // only on its own input row, and rows past n are never stored
    int64_t rowpos[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        const int64_t row = min(i0 + 16 * rb + (lane & 15), n - 1);
        rowpos[rb] = rows ? (int64_t)rows[row] : row;
    }
    floatx4 acc[4][CB];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = floatx4{0.f, 0.f, 0.f, 0.f};

    const int r16 = lane & 15, g = lane >> 4;
    for (int kc0 = 0; kc0 < dp; kc0 += H_KC) {
        // the chunk's loads are issued SB at a time before their LDS stores,
        // so the block waits for one round trip per SB elements per thread
        constexpr int PER = NB * H_KC / (H_WAVES * 64);
        constexpr int SB = PER <= 16 ? PER : (PER % 16 == 0 ? 16 : 8);
        static_assert(NB * H_KC % (H_WAVES * 64) == 0 && PER % SB == 0, "whole staging rounds");
        float av[SB];
        auto stage_load = [&](int u0) {
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int e = threadIdx.x + (u0 + u) * H_WAVES * 64;
                const int r = e / H_KC, k = kc0 + (e % H_KC);
                av[u] = (r < L && k < d) ? A[(int64_t)r * (d + 1) + k] : 0.f;
            }
        };
        auto stage_store = [&](int u0) {
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int e = threadIdx.x + (u0 + u) * H_WAVES * 64;
                As[(e / H_KC) * H_KS + (e % H_KC)] = av[u];
            }
        };
        stage_load(0);
        __syncthreads();  // the previous chunk's operands have been read
        stage_store(0);
        for (int u0 = SB; u0 < PER; u0 += SB) {
            stage_load(u0);
            stage_store(u0);
        }
        __syncthreads();
        const int kend = min(H_KC, dp - kc0);
        // Row loads run one step ahead in two register sets taken in turn;
        // a step's columns past dp read columns dp - 4 .. dp - 1 instead and
        // are masked to zero where they enter the matrix cores.
        auto load_x = [&](floatx4 (&x)[4], int kk) {
            const int k = min(kc0 + kk + 4 * g, dp - 4);
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
                x[rb] = *reinterpret_cast<const floatx4 *>(Xl + rowpos[rb] * dp + k);
        };
        auto step = [&](const floatx4 (&x)[4], int kk) {
            const bool kin = kc0 + kk + 4 * g < dp;
            floatx4 bq[CB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
                bq[cb] = *reinterpret_cast<const floatx4 *>(&As[(16 * cb + r16) * H_KS + kk + 4 * g]);
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(kin ? x[rb][j] : 0.f, bq[cb][j],
                                                                           acc[rb][cb], 0, 0, 0);
        };
        // Steps go in pairs with no branch between them (a branch would let
        // the compiler sink the loads to their use), and a scheduling barrier
        // after each set of loads keeps them ahead of the previous set's
        // matrix-core work.  An odd step count ends with a step wholly past
        // dp, which reads staged zeros and in-bounds LDS (kk <= 112) and adds
        // +0 to every sum.
        floatx4 xa[4], xb[4];
        load_x(xa, 0);
        for (int kk = 0; kk < kend; kk += 32) {
            load_x(xb, kk + 16);
            __builtin_amdgcn_sched_barrier(0);
            step(xa, kk);
            load_x(xa, kk + 32);
            __builtin_amdgcn_sched_barrier(0);
            step(xb, kk + 16);
        }
    }

    // lane l assembles the code of item i0 + l (row l = 16 rb + 4 g + v)
    const int my_rb = lane >> 4, my_g = (lane >> 2) & 3, my_v = lane & 3;
    uint64_t mycode = 0, myfix = 0;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const int r = 16 * cb + r16;
        const float alast = (r < L) ? A[(int64_t)r * (d + 1) + d] : 0.f;
        const float tr = (r < L) ? tau[r] : 0.f;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * rb + 4 * g + v;
                const float p = acc[rb][cb][v] + alast * sq_s[wave][row];
                const bool inb = (r < L) && (i0 + row < n);
                const bool flag = inb && (sp_s[wave][row] != 0 || fabsf(p) <= tr * uf_s[wave][row]);
                const bool bit = inb && (p > 0.f);
                const uint64_t bb = __ballot(bit);
                const uint64_t fb = __ballot(flag);
                if (rb == my_rb && v == my_v) {
                    mycode |= ((bb >> (16 * my_g)) & 0xFFFFull) << (16 * cb);
                    myfix |= ((fb >> (16 * my_g)) & 0xFFFFull) << (16 * cb);
                }
            }
        }
    }
    const bool valid = i0 + lane < n;
    const int64_t i = valid && rows ? (int64_t)rows[i0 + lane] : i0 + lane;
    if (valid) {
        if (rows) {  // bits the FP32 re-hash changes in the low-precision code
            uint64_t old = codes_l[(CB <= 2 ? 1 : 2) * i];
            if (CB > 2) old |= (uint64_t)codes_l[2 * i + 1] << 32;
            const unsigned long long ch = (unsigned long long)__popcll(old ^ mycode);
            if (ch) atomicAdd(&ctr->lowp_changed, ch);
        }
        if (CB <= 2) {
            codes_l[i] = (uint32_t)mycode;
        } else {
            codes_l[2 * i] = (uint32_t)mycode;
            codes_l[2 * i + 1] = (uint32_t)(mycode >> 32);
        }
    }
    const bool has = valid && myfix != 0ull;
    const uint64_t hb = __ballot(has);
    if (hb != 0ull) {
        const int leader = __ffsll((long long)hb) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&ctr->fix_count, (uint32_t)__popcll(hb));
        base = __shfl(base, leader, 64);
        if (has) {
            const uint32_t slot = base + (uint32_t)__popcll(hb & lanemask_lt(lane));
            FixEntry fe;
            fe.mask = myfix;
            fe.item = (int32_t)i;
            fe.pad = 0;
            fix[slot] = fe;
        }
    }
}

// ---------------------------------------------------------------- precision form
// OCP E4M3: 1 sign, 4 exponent (bias 7), 3 mantissa bits; largest finite
// 448 (0x7E), 0x7F is NaN, subnormals m * 2^-9.  Round to nearest even,
// saturating at +-448.
__device__ __forceinline__ uint8_t f32_to_e4m3(float f)
{
    const uint8_t sign = (__float_as_uint(f) >> 24) & 0x80u;
    const float a = fabsf(f);
    if (!(a < 448.0f)) return sign | 0x7Eu;
    if (a < 0x1p-6f) {  // subnormal: a = m 2^-9, m in [0, 8]; m = 8 is the smallest normal
        const int m = (int)__builtin_rintf(a * 512.0f);
        return sign | (uint8_t)m;
    }
    int e;
    const float fr = frexpf(a, &e);  // a = fr 2^e, fr in [0.5, 1)
    int E = e - 1;                   // a = (2 fr) 2^E, 2 fr in [1, 2)
    int m = (int)__builtin_rintf((2.0f * fr - 1.0f) * 8.0f);
    if (m == 8) {
        m = 0;
        ++E;
    }
    const int code = ((E + 7) << 3) | m;
    return sign | (uint8_t)(code > 0x7E ? 0x7E : code);
}

// Quantise `rows` rows of `d` floats (source stride `ss`) into bfloat16 (ST = 1)
// or E4M3 with a per-row scale max|x| / 448 (ST = 2; 1 for an all-zero row),
// zero-padded to dst stride `ds`.  One wave per row.
template <int ST>
__global__ __launch_bounds__(256) void k_quant_rows(const float *__restrict__ src, int64_t rows,
                                                    int d, int ss, void *__restrict__ dst, int ds,
                                                    float *__restrict__ scales)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + wave;
    if (r >= rows) return;
    const float *x = src + r * ss;
    if (ST == 1) {
        uint16_t *o = static_cast<uint16_t *>(dst) + r * ds;
        for (int c = lane; c < ds; c += 64) o[c] = c < d ? bf16_rne(x[c]) : (uint16_t)0;
        return;
    }
    float mx = 0.f;
    for (int c = lane; c < d; c += 64) mx = fmaxf(mx, fabsf(x[c]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    const float sc = mx > 0.f ? mx / 448.0f : 1.0f;
    uint8_t *o = static_cast<uint8_t *>(dst) + r * ds;
    for (int c = lane; c < ds; c += 64) o[c] = c < d ? f32_to_e4m3(x[c] / sc) : (uint8_t)0;
    if (lane == 0) scales[r] = sc;
}

// Low-precision hash (ST = 1 bfloat16, ST = 2 E4M3 with row scales) on the
// bf16 / fp8 matrix cores (16x16x32, FP32 accumulate): items = M, hash bits =
// N; in an MFMA lane group g carries coordinates kk + 8 g .. + 7 of both
// operands.  p~ = (scales) acc + a_d sqrt(keymax_j - key_i).  Every bit gets
// sign(p~); an item with |p~| <= mq_r ||x_i|| + tq_r U_j for some bit (or with
// U_j outside [2^-60, 2^60]) is appended to `rows` for the FP32 re-hash.
constexpr int HQ_FEW = 8;

template <int CB, int ST>
__global__ __launch_bounds__(H_WAVES * 64) void k_hash_q(
    const void *__restrict__ Xq, const float *__restrict__ xscale, int64_t n, int d, int dp,
    const void *__restrict__ Aq, const float *__restrict__ ascale, const float *__restrict__ A,
    int L, const double *__restrict__ key_l, const int32_t *__restrict__ sid_l,
    const double *__restrict__ keymax, const double *__restrict__ U, const float *__restrict__ mq,
    const float *__restrict__ tq, uint32_t *__restrict__ codes_l, int32_t *__restrict__ rows,
    FixEntry *__restrict__ fix, BuildCounters *__restrict__ ctr)
{
    constexpr int NB = 16 * CB;
    constexpr int ES = ST == 1 ? 2 : 1;       // bytes per element
    constexpr int KCQ = 128;                  // coordinates staged per chunk
    constexpr int RB = KCQ * ES + (ST == 1 ? 16 : 8);  // LDS row stride in bytes
    __shared__ __align__(16) uint8_t As[NB * RB];
    __shared__ float sq_s[H_WAVES][64], uf_s[H_WAVES][64], xn_s[H_WAVES][64], xs_s[H_WAVES][64];
    __shared__ int sp_s[H_WAVES][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i0 = ((int64_t)blockIdx.x * H_WAVES + wave) * 64;
    {
        const int64_t i = i0 + lane;
        float sq = 0.f, uf = 0.f, xn = 0.f, xs = 1.f;
        int sp = 1;
        if (i < n) {
            const int s = sid_l[i];
            const double km = keymax[s], u = U[s];
            sq = sqrtf((float)(km - key_l[i]));
            uf = (float)u;
            xn = sqrtf((float)key_l[i]) * (1.0f + 0x1p-18f);
            sp = !(u >= 0x1p-60 && u <= 0x1p60);
            if (ST == 2) xs = xscale[i];
        }
        sq_s[wave][lane] = sq;
        uf_s[wave][lane] = uf;
        xn_s[wave][lane] = xn;
        xs_s[wave][lane] = xs;
        sp_s[wave][lane] = sp;
    }
    floatx4 acc[4][CB];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = floatx4{0.f, 0.f, 0.f, 0.f};

    const int r16 = lane & 15, g = lane >> 4;
    const uint8_t *X8 = static_cast<const uint8_t *>(Xq);
    const uint8_t *A8 = static_cast<const uint8_t *>(Aq);
    for (int kc0 = 0; kc0 < dp; kc0 += KCQ) {
        // loads issued SB at a time before their LDS stores (one round trip
        // per SB elements per thread)
        constexpr int PER = NB * KCQ / (H_WAVES * 64);
        constexpr int SB = PER <= 16 ? PER : (PER % 16 == 0 ? 16 : 8);
        static_assert(NB * KCQ % (H_WAVES * 64) == 0 && PER % SB == 0, "whole staging rounds");
        uint16_t av[SB];
        auto stage_load = [&](int u0) {
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int e = threadIdx.x + (u0 + u) * H_WAVES * 64;
                const int r = e / KCQ, k = kc0 + (e % KCQ);
                if (ST == 1)
                    av[u] = (r < L && k < dp) ? reinterpret_cast<const uint16_t *>(A8)[(int64_t)r * dp + k]
                                              : (uint16_t)0;
                else
                    av[u] = (r < L && k < dp) ? A8[(int64_t)r * dp + k] : (uint8_t)0;
            }
        };
        auto stage_store = [&](int u0) {
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int e = threadIdx.x + (u0 + u) * H_WAVES * 64;
                const int r = e / KCQ, c = e % KCQ;
                if (ST == 1) reinterpret_cast<uint16_t *>(As + r * RB)[c] = av[u];
                else As[r * RB + c] = (uint8_t)av[u];
            }
        };
        stage_load(0);
        __syncthreads();  // the previous chunk's operands have been read
        stage_store(0);
        for (int u0 = SB; u0 < PER; u0 += SB) {
            stage_load(u0);
            stage_store(u0);
        }
        __syncthreads();
        const int kend = min(KCQ, dp - kc0);
        for (int kk = 0; kk < kend; kk += 32) {
            const int k = kc0 + kk + 8 * g;
            const bool kin = kk + 8 * g < kend;
            if (ST == 1) {
                bf16x8 xa[4], bq[CB];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    const int64_t row = i0 + 16 * rb + r16;
                    u16x8 v = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
                    if (row < n && kin) v = *reinterpret_cast<const u16x8 *>(X8 + (row * dp + k) * 2);
                    xa[rb] = __builtin_bit_cast(bf16x8, v);
                }
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    u16x8 v = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
                    if (kin) v = *reinterpret_cast<const u16x8 *>(As + (16 * cb + r16) * RB + (kk + 8 * g) * 2);
                    bq[cb] = __builtin_bit_cast(bf16x8, v);
                }
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[rb], bq[cb], acc[rb][cb], 0, 0, 0);
            } else {
                long xa[4], bq[CB];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    const int64_t row = i0 + 16 * rb + r16;
                    xa[rb] = (row < n && kin) ? *reinterpret_cast<const long *>(X8 + row * dp + k) : 0l;
                }
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    bq[cb] = kin ? *reinterpret_cast<const long *>(As + (16 * cb + r16) * RB + kk + 8 * g) : 0l;
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(xa[rb], bq[cb], acc[rb][cb], 0, 0, 0);
            }
        }
    }

    const int my_rb = lane >> 4, my_g = (lane >> 2) & 3, my_v = lane & 3;
    uint64_t mycode = 0, myflag = 0;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const int r = 16 * cb + r16;
        const float alast = (r < L) ? A[(int64_t)r * (d + 1) + d] : 0.f;
        const float m1 = (r < L) ? mq[r] : 0.f, m2 = (r < L) ? tq[r] : 0.f;
        const float as = (ST == 2 && r < L) ? ascale[r] : 1.f;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * rb + 4 * g + v;
                float p = acc[rb][cb][v];
                if (ST == 2) p = p * (xs_s[wave][row] * as);
                p = p + alast * sq_s[wave][row];
                const bool inb = (r < L) && (i0 + row < n);
                const float mg = m1 * xn_s[wave][row] + m2 * uf_s[wave][row];
                const bool flag = inb && (sp_s[wave][row] != 0 || !(fabsf(p) > mg));
                const bool bit = inb && (p > 0.f);
                const uint64_t bb = __ballot(bit);
                const uint64_t fb = __ballot(flag);
                if (rb == my_rb && v == my_v) {
                    mycode |= ((bb >> (16 * my_g)) & 0xFFFFull) << (16 * cb);
                    myflag |= ((fb >> (16 * my_g)) & 0xFFFFull) << (16 * cb);
                }
            }
        }
    }
    const int64_t i = i0 + lane;
    const bool valid = i < n;
    if (valid) {
        if (CB <= 2) {
            codes_l[i] = (uint32_t)mycode;
        } else {
            codes_l[2 * i] = (uint32_t)mycode;
            codes_l[2 * i + 1] = (uint32_t)(mycode >> 32);
        }
    }
    // an item with at most HQ_FEW bits inside the margin has just those bits
    // recomputed in FP64 (k_hash_fixup); one with more is re-hashed whole from
    // the FP32 rows (then its own FP32 band goes through the fix-up)
    const int nflag = __popcll(valid ? myflag : 0ull);
    const bool few = valid && nflag > 0 && nflag <= HQ_FEW;
    const bool many = valid && nflag > HQ_FEW;
    const uint64_t fb = __ballot(few), hb = __ballot(many);
    unsigned long long wbits = (unsigned long long)nflag;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wbits += __shfl_xor(wbits, o, 64);
    if (lane == 0 && wbits) atomicAdd(&ctr->lowp_bits, wbits);
    if (fb != 0ull) {
        const int leader = __ffsll((long long)fb) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&ctr->fix_count, (uint32_t)__popcll(fb));
        base = __shfl(base, leader, 64);
        if (few) {
            FixEntry fe;
            fe.mask = myflag;
            fe.item = (int32_t)i;
            fe.pad = 0;
            fix[base + (uint32_t)__popcll(fb & lanemask_lt(lane))] = fe;
        }
    }
    if (hb != 0ull) {
        const int leader = __ffsll((long long)hb) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&ctr->lowp_items, (uint32_t)__popcll(hb));
        base = __shfl(base, leader, 64);
        if (many) rows[base + (uint32_t)__popcll(hb & lanemask_lt(lane))] = (int32_t)i;
    }
}

// The same hash with one shared projection, persistent: each block stages
// the whole L x d_p projection in LDS once (row stride d_p + 4) and then
// walks tiles of 256 stored rows (one 64-row tile per wave), loading the rows
// of step kk + 16 while the matrix cores work on step kk.  Products, bounds,
// codes and fix-up entries are those of k_hash.
constexpr int HP_WAVES = 4;

template <int CB>
__global__ __launch_bounds__(HP_WAVES * 64) void k_hash_p(
    const float *__restrict__ Xl, int64_t n, int d, int dp, const float *__restrict__ A, int L,
    const double *__restrict__ key_l, const int32_t *__restrict__ sid_l,
    const double *__restrict__ keymax, const double *__restrict__ U,
    const float *__restrict__ tau, uint32_t *__restrict__ codes_l, FixEntry *__restrict__ fix,
    BuildCounters *__restrict__ ctr, const int32_t *__restrict__ rows, int64_t ntiles)
{
    constexpr int NB = 16 * CB;
    extern __shared__ __align__(16) float As[];  // NB x (dp + 4)
    __shared__ float sq_s[HP_WAVES][64];
    __shared__ float uf_s[HP_WAVES][64];
    __shared__ int sp_s[HP_WAVES][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ks = dp + 4;
    {
        // projection rows r < L, columns < d (zero elsewhere), 16 loads per
        // thread in flight before their stores
        const int total = NB * dp;
        for (int e0 = 0; e0 < total; e0 += 16 * HP_WAVES * 64) {
            float av[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = e0 + u * HP_WAVES * 64 + (int)threadIdx.x;
                const int r = e / dp, c = e - (e / dp) * dp;
                av[u] = (e < total && r < L && c < d) ? A[(int64_t)r * (d + 1) + c] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = e0 + u * HP_WAVES * 64 + (int)threadIdx.x;
                if (e < total) As[(e / dp) * ks + (e - (e / dp) * dp)] = av[u];
            }
        }
    }
    __syncthreads();
    const int r16 = lane & 15, g = lane >> 4;
    const int my_rb = lane >> 4, my_g = (lane >> 2) & 3, my_v = lane & 3;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t i0 = (tile * HP_WAVES + wave) * 64;
        {
            const int64_t i = i0 + lane;
            float sq = 0.f, uf = 0.f;
            int sp = 1;
            if (i < n) {
                const int64_t ii = rows ? rows[i] : i;
                const int s = sid_l[ii];
                const double km = keymax[s], u = U[s];
                sq = sqrtf((float)(km - key_l[ii]));
                uf = (float)u;
                sp = !(u >= 0x1p-60 && u <= 0x1p60);
            }
            sq_s[wave][lane] = sq;
            uf_s[wave][lane] = uf;
            sp_s[wave][lane] = sp;
        }
        // a row past n reads row n - 1 (an MFMA output row depends only on its
        // own input row, and rows past n are never stored) and a column past
        // dp reads columns dp - 4 .. dp - 1, masked to zero where it is used:
        // the loads need no branch, which would make the compiler wait for
        // the loads in flight
        int64_t rowpos[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            const int64_t row = min(i0 + 16 * rb + r16, n - 1);
            rowpos[rb] = rows ? (int64_t)rows[row] : row;
        }
        auto load_rows = [&](floatx4 (&xa)[4], int k) {
            const int kc = min(k, dp - 4);
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
                xa[rb] = *reinterpret_cast<const floatx4 *>(Xl + rowpos[rb] * dp + kc);
        };
        floatx4 acc[4][CB];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
        // rows two steps ahead
        floatx4 xn[4], xn2[4];
        load_rows(xn, 4 * g);
        load_rows(xn2, 16 + 4 * g);
        for (int kk = 0; kk < dp; kk += 16) {
            const bool kin = kk + 4 * g < dp;
            floatx4 xa[4];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                xa[rb] = kin ? xn[rb] : floatx4{0.f, 0.f, 0.f, 0.f};
                xn[rb] = xn2[rb];
            }
            load_rows(xn2, kk + 32 + 4 * g);
            floatx4 bq[CB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const int k = kk + 4 * g;
                bq[cb] = k < dp ? *reinterpret_cast<const floatx4 *>(&As[(16 * cb + r16) * ks + k])
                                : floatx4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[rb][j], bq[cb][j], acc[rb][cb], 0, 0, 0);
        }
        __syncthreads();  // the wave's row parameters are in LDS

        uint64_t mycode = 0, myfix = 0;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int r = 16 * cb + r16;
            const float alast = (r < L) ? A[(int64_t)r * (d + 1) + d] : 0.f;
            const float tr = (r < L) ? tau[r] : 0.f;
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * rb + 4 * g + v;
                    const float p = acc[rb][cb][v] + alast * sq_s[wave][row];
                    const bool inb = (r < L) && (i0 + row < n);
                    const bool flag = inb && (sp_s[wave][row] != 0 || fabsf(p) <= tr * uf_s[wave][row]);
                    const bool bit = inb && (p > 0.f);
                    const uint64_t bb = __ballot(bit);
                    const uint64_t fb = __ballot(flag);
                    if (rb == my_rb && v == my_v) {
                        mycode |= ((bb >> (16 * my_g)) & 0xFFFFull) << (16 * cb);
                        myfix |= ((fb >> (16 * my_g)) & 0xFFFFull) << (16 * cb);
                    }
                }
            }
        }
        const bool valid = i0 + lane < n;
        const int64_t i = valid && rows ? (int64_t)rows[i0 + lane] : i0 + lane;
        if (valid) {
            if (rows) {  // bits the FP32 re-hash changes in the low-precision code
                uint64_t old = codes_l[(CB <= 2 ? 1 : 2) * i];
                if (CB > 2) old |= (uint64_t)codes_l[2 * i + 1] << 32;
                const unsigned long long ch = (unsigned long long)__popcll(old ^ mycode);
                if (ch) atomicAdd(&ctr->lowp_changed, ch);
            }
            if (CB <= 2) {
                codes_l[i] = (uint32_t)mycode;
            } else {
                codes_l[2 * i] = (uint32_t)mycode;
                codes_l[2 * i + 1] = (uint32_t)(mycode >> 32);
            }
        }
        const bool has = valid && myfix != 0ull;
        const uint64_t hb = __ballot(has);
        if (hb != 0ull) {
            const int leader = __ffsll((long long)hb) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(&ctr->fix_count, (uint32_t)__popcll(hb));
            base = __shfl(base, leader, 64);
            if (has) {
                const uint32_t slot = base + (uint32_t)__popcll(hb & lanemask_lt(lane));
                FixEntry fe;
                fe.mask = myfix;
                fe.item = (int32_t)i;
                fe.pad = 0;
                fix[slot] = fe;
            }
        }
        __syncthreads();  // row parameters of the next tile overwrite these
    }
}

// One thread per list entry: recompute every flagged bit in FP64 exactly as
// the definition (v = [x / U_j ; sqrt(max(0, 1 - key/keymax))], or [0; 1]
// when U_j = 0; sum over coordinates in ascending order, no contraction).
// The flagged bits are taken FX_B at a time: each coordinate's quotient
// x_c / U_j is formed once for the group and its product with each bit's
// projection entry added to that bit's own sum, in ascending c.
constexpr int FX_B = 8;

__global__ __launch_bounds__(256) void k_hash_fixup(
    const float *__restrict__ Xl, int d, int dp, const float *__restrict__ A, int L, int per_subset,
    const double *__restrict__ key_l, const int32_t *__restrict__ sid_l,
    const double *__restrict__ keymax, const double *__restrict__ U,
    const FixEntry *__restrict__ fix, BuildCounters *__restrict__ ctr,
    uint32_t *__restrict__ codes_l, int W)
{
    const uint32_t cnt = ctr->fix_count;
    unsigned long long nbits = 0, nflip = 0, ntiny = 0;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += gridDim.x * blockDim.x) {
        const FixEntry fe = fix[e];
        const int64_t i = fe.item;
        const int s = sid_l[i];
        const double u = U[s], km = keymax[s], kk = key_l[i];
        uint64_t code = codes_l[W * i];
        if (W == 2) code |= (uint64_t)codes_l[W * i + 1] << 32;
        double vd = 1.0;
        if (u != 0.0) {
            double t = 1.0 - kk / km;
            if (t < 0.0) t = 0.0;
            vd = __builtin_sqrt(t);
        }
        const float *x = Xl + i * dp;
        const double uu = u == 0.0 ? 1.0 : u;
        const float *Ab = A + (per_subset ? (int64_t)s * L : 0) * (int64_t)(d + 1);
        uint64_t mask = fe.mask;
        while (mask != 0ull) {
            int rr[FX_B];
            int nb = 0;
#pragma unroll
            for (int b = 0; b < FX_B; ++b) {
                rr[b] = 0;
                if (mask != 0ull) {
                    rr[b] = __ffsll((long long)mask) - 1;
                    mask &= mask - 1ull;
                    nb = b + 1;
                }
            }
            double sacc[FX_B];
#pragma unroll
            for (int b = 0; b < FX_B; ++b) sacc[b] = 0.0;
            for (int c = 0; c < d; ++c) {
                const double q = (double)x[c] / uu;  // formed even when U_j = 0, then replaced by 0
                const double vq = u == 0.0 ? 0.0 : q;
#pragma unroll
                for (int b = 0; b < FX_B; ++b) {
                    const double t = (double)Ab[(int64_t)rr[b] * (d + 1) + c] * vq;
                    sacc[b] = b < nb ? sacc[b] + t : sacc[b];
                }
            }
#pragma unroll
            for (int b = 0; b < FX_B; ++b) {
                if (b >= nb) break;
                const int r = rr[b];
                const double sum = sacc[b] + (double)Ab[(int64_t)r * (d + 1) + d] * vd;
                const uint64_t bit = sum > 0.0 ? 1ull : 0ull;
                // flips counted in two bands of the exact projection a . P(x)
                // (P(x) has unit norm): below 1e-6 in magnitude, and the rest
                const bool flip = ((code >> r) & 1ull) != bit;
                nflip += flip;
                ntiny += flip && __builtin_fabs(sum) < 1e-6;
                ++nbits;
                code = (code & ~(1ull << r)) | (bit << r);
            }
        }
        codes_l[W * i] = (uint32_t)code;
        if (W == 2) codes_l[W * i + 1] = (uint32_t)(code >> 32);
    }
    if (nbits) {
        atomicAdd(&ctr->fix_bits, nbits);
        atomicAdd(&ctr->fix_flips, nflip);
        if (ntiny) atomicAdd(&ctr->fix_flips_tiny, ntiny);
    }
}

__global__ void k_roll_fix_count(BuildCounters *ctr)
{
    ctr->fix_prev += ctr->fix_count;
    ctr->fix_count = 0;
}

inline unsigned grid_for(int64_t n, int per_block)
{
    return (unsigned)((n + per_block - 1) / per_block);
}

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_keys(const float *X, int64_t n, int d, double *key, uint64_t *sort_key,
                       int32_t *sort_val, BuildCounters *ctr, hipStream_t s)
{
    const dim3 grid(grid_for(n, 4 * KC_ROWS)), block(256);
    if (d % 4 == 0)
        hipLaunchKernelGGL(k_keys<4>, grid, block, 0, s, X, n, d, key, sort_key, sort_val, ctr);
    else if (d % 2 == 0)
        hipLaunchKernelGGL(k_keys<2>, grid, block, 0, s, X, n, d, key, sort_key, sort_val, ctr);
    else
        hipLaunchKernelGGL(k_keys<1>, grid, block, 0, s, X, n, d, key, sort_key, sort_val, ctr);
    return hipGetLastError();
}

size_t radix_sort_tmp_bytes(int64_t n)
{
    const int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    return (size_t)(256 * nb + 256) * sizeof(uint32_t);
}

hipError_t radix_sort(uint64_t *ka, int32_t *va, uint64_t *kb, int32_t *vb, int64_t n, int nbits,
                      void *tmp, bool *result_in_b, hipStream_t s)
{
    const int nb = (int)((n + RS_TILE - 1) / RS_TILE);
    uint32_t *bhist = static_cast<uint32_t *>(tmp);
    uint32_t *totals = bhist + (int64_t)256 * nb;
    bool in_b = false;
    for (int shift = 0; shift < nbits; shift += 8) {
        const uint64_t *ki = in_b ? kb : ka;
        const int32_t *vi = in_b ? vb : va;
        uint64_t *ko = in_b ? ka : kb;
        int32_t *vo = in_b ? va : vb;
        hipLaunchKernelGGL(k_rs_hist, dim3(nb), dim3(RS_THREADS), 0, s, ki, n, shift, bhist, nb);
        hipLaunchKernelGGL(k_rs_scan, dim3(256), dim3(256), 0, s, bhist, nb, totals);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(RS_THREADS), 0, s, ki, vi, n, shift, bhist,
                           nb, totals, ko, vo);
        in_b = !in_b;
    }
    *result_in_b = in_b;
    return hipGetLastError();
}

hipError_t launch_assign_subsets(const uint64_t *sorted_key, const int32_t *sorted_idx, int64_t n,
                                 int m, const double *bounds, int32_t *sid, uint64_t *layout_key,
                                 int32_t *layout_val, double *keymax, int32_t *subend, hipStream_t s)
{
    hipLaunchKernelGGL(k_assign, dim3(grid_for(n, 256)), dim3(256), 0, s, sorted_key, sorted_idx,
                       n, m, bounds, sid, layout_key, layout_val, keymax, subend);
    return hipGetLastError();
}

hipError_t launch_layout(const float *X, int64_t n, int d, int dp, const int32_t *perm,
                         const double *key, const int32_t *sid, float *Xl, uint16_t *Xh,
                         uint16_t *Xlo, double *key_l, int32_t *sid_l, float *xeb, hipStream_t s)
{
    const dim3 grid(grid_for(n, 4 * LY_ROWS)), block(256);
    if (d % 4 == 0)
        hipLaunchKernelGGL(k_layout<4>, grid, block, 0, s, X, n, d, dp, perm, key, sid, Xl, Xh, Xlo, key_l,
                           sid_l, xeb);
    else if (d % 2 == 0)
        hipLaunchKernelGGL(k_layout<2>, grid, block, 0, s, X, n, d, dp, perm, key, sid, Xl, Xh, Xlo, key_l,
                           sid_l, xeb);
    else
        hipLaunchKernelGGL(k_layout<1>, grid, block, 0, s, X, n, d, dp, perm, key, sid, Xl, Xh, Xlo, key_l,
                           sid_l, xeb);
    return hipGetLastError();
}

hipError_t launch_lo_rows(const float *Xl, const uint16_t *Xh, int64_t count, uint16_t *Xlo, hipStream_t s)
{
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_lo_rows, dim3((unsigned)blocks), dim3(256), 0, s, Xl, Xh, count, Xlo);
    return hipGetLastError();
}

hipError_t launch_quant_rows(const float *src, int64_t rows, int d, int ss, int storage, void *dst,
                             int ds, float *scales, hipStream_t s)
{
    const dim3 grid(grid_for(rows, 4)), block(256);
    if (storage == 1)
        hipLaunchKernelGGL(k_quant_rows<1>, grid, block, 0, s, src, rows, d, ss, dst, ds, scales);
    else
        hipLaunchKernelGGL(k_quant_rows<2>, grid, block, 0, s, src, rows, d, ss, dst, ds, scales);
    return hipGetLastError();
}

hipError_t launch_hash_q(int storage, const void *Xq, const float *xscale, int64_t n, int d, int dp,
                         const void *Aq, const float *ascale, const float *A, int L,
                         const double *key_l, const int32_t *sid_l, const double *keymax,
                         const double *U, const float *mq, const float *tq, uint32_t *codes_l,
                         int32_t *rows, FixEntry *fix, BuildCounters *ctr, hipStream_t s)
{
    const dim3 grid(grid_for(n, H_WAVES * 64)), block(H_WAVES * 64);
    const int cb = (L + 15) / 16;
#define NRLSH_HQ(CB, ST)                                                                          \
    hipLaunchKernelGGL((k_hash_q<CB, ST>), grid, block, 0, s, Xq, xscale, n, d, dp, Aq, ascale, A, L, \
                       key_l, sid_l, keymax, U, mq, tq, codes_l, rows, fix, ctr)
    if (storage == 1) {
        if (cb == 1) NRLSH_HQ(1, 1);
        else if (cb == 2) NRLSH_HQ(2, 1);
        else if (cb == 3) NRLSH_HQ(3, 1);
        else NRLSH_HQ(4, 1);
    } else {
        if (cb == 1) NRLSH_HQ(1, 2);
        else if (cb == 2) NRLSH_HQ(2, 2);
        else if (cb == 3) NRLSH_HQ(3, 2);
        else NRLSH_HQ(4, 2);
    }
#undef NRLSH_HQ
    return hipGetLastError();
}

// Persistent form when the projection fits the work-group's LDS: as many
// blocks as stay resident, each walking tiles of 256 rows.
template <int CB>
static bool launch_hash_p(const float *Xl, int64_t n, int d, int dp, const float *A, int L,
                          const double *key_l, const int32_t *sid_l, const double *keymax,
                          const double *U, const float *tau, uint32_t *codes_l, FixEntry *fix,
                          BuildCounters *ctr, const int32_t *rows, hipStream_t s)
{
    const size_t lds = (size_t)16 * CB * (dp + 4) * sizeof(float);
    int dev = 0, lim = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return false;
    if (lds + 4096 > (size_t)lim) return false;
    if (hipFuncSetAttribute((const void *)k_hash_p<CB>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
            hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_hash_p<CB>, HP_WAVES * 64, lds) != hipSuccess ||
        per_cu < 1)
        return false;
    const int64_t ntiles = (n + HP_WAVES * 64 - 1) / (HP_WAVES * 64);
    const int64_t blocks = std::min<int64_t>(ntiles, (int64_t)per_cu * cus);
    hipLaunchKernelGGL(k_hash_p<CB>, dim3((unsigned)blocks), dim3(HP_WAVES * 64), lds, s, Xl, n, d, dp, A, L,
                       key_l, sid_l, keymax, U, tau, codes_l, fix, ctr, rows, ntiles);
    return true;
}

hipError_t launch_hash(const float *Xl, int64_t n, int d, int dp, const float *A, int L,
                       const double *key_l, const int32_t *sid_l, const double *keymax,
                       const double *U, const float *tau, uint32_t *codes_l, FixEntry *fix,
                       BuildCounters *ctr, const int32_t *rows, hipStream_t s)
{
    if (n < 1) return hipSuccess;
    // more than 32 bits: the persistent form (at 32 or fewer the 8-wave
    // blocks below keep one more wave per SIMD resident and measure faster)
    bool done = false;
    switch ((L + 15) / 16) {
    case 1:
    case 2: break;
    case 3: done = launch_hash_p<3>(Xl, n, d, dp, A, L, key_l, sid_l, keymax, U, tau, codes_l, fix, ctr, rows, s); break;
    default: done = launch_hash_p<4>(Xl, n, d, dp, A, L, key_l, sid_l, keymax, U, tau, codes_l, fix, ctr, rows, s); break;
    }
    if (done) return hipGetLastError();
    const dim3 grid(grid_for(n, H_WAVES * 64)), block(H_WAVES * 64);
    switch ((L + 15) / 16) {
    case 1:
        hipLaunchKernelGGL(k_hash<1>, grid, block, 0, s, Xl, n, d, dp, A, L, key_l, sid_l, keymax, U,
                           tau, codes_l, fix, ctr, rows, nullptr, nullptr, 0);
        break;
    case 2:
        hipLaunchKernelGGL(k_hash<2>, grid, block, 0, s, Xl, n, d, dp, A, L, key_l, sid_l, keymax, U,
                           tau, codes_l, fix, ctr, rows, nullptr, nullptr, 0);
        break;
    case 3:
        hipLaunchKernelGGL(k_hash<3>, grid, block, 0, s, Xl, n, d, dp, A, L, key_l, sid_l, keymax, U,
                           tau, codes_l, fix, ctr, rows, nullptr, nullptr, 0);
        break;
    default:
        hipLaunchKernelGGL(k_hash<4>, grid, block, 0, s, Xl, n, d, dp, A, L, key_l, sid_l, keymax, U,
                           tau, codes_l, fix, ctr, rows, nullptr, nullptr, 0);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_roll_fix_count(BuildCounters *ctr, hipStream_t s)
{
    hipLaunchKernelGGL(k_roll_fix_count, dim3(1), dim3(1), 0, s, ctr);
    return hipGetLastError();
}

hipError_t launch_hash_fixup(const float *Xl, int d, int dp, const float *A, int L, bool per_subset,
                             const double *key_l, const int32_t *sid_l, const double *keymax,
                             const double *U, const FixEntry *fix, BuildCounters *ctr,
                             uint32_t *codes_l, int64_t max_entries, hipStream_t s)
{
    const int W = L > 32 ? 2 : 1;
    // one wave per block: the few hundred waves a typical list needs spread
    // over every compute unit instead of a quarter of them
    int64_t blocks = (max_entries + 63) / 64;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_hash_fixup, dim3((unsigned)blocks), dim3(64), 0, s, Xl, d, dp, A, L,
                       per_subset ? 1 : 0, key_l, sid_l, keymax, U, fix, ctr, codes_l, W);
    return hipGetLastError();
}

int hash_items_per_block() { return H_WAVES * 64; }

hipError_t launch_hash_per_subset(const float *Xl, int d, int dp, const float *A, int L,
                                  const double *key_l, const int32_t *sid_l, const double *keymax,
                                  const double *U, const float *tau, const int32_t *off,
                                  const int32_t *bstart, int m, int nblocks, uint32_t *codes_l,
                                  FixEntry *fix, BuildCounters *ctr, hipStream_t s)
{
    if (nblocks < 1) return hipSuccess;
    const dim3 grid((unsigned)nblocks), block(H_WAVES * 64);
#define NRLSH_HPS(CB)                                                                           \
    hipLaunchKernelGGL(k_hash<CB>, grid, block, 0, s, Xl, (int64_t)0, d, dp, A, L, key_l, sid_l, \
                       keymax, U, tau, codes_l, fix, ctr, nullptr, off, bstart, m)
    switch ((L + 15) / 16) {
    case 1: NRLSH_HPS(1); break;
    case 2: NRLSH_HPS(2); break;
    case 3: NRLSH_HPS(3); break;
    default: NRLSH_HPS(4); break;
    }
#undef NRLSH_HPS
    return hipGetLastError();
}

}  // namespace nrlsh
