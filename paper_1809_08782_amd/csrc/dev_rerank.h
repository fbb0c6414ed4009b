// Device helpers of the exact re-rank (Algorithm 2: the item with the largest
// inner product), shared by the per-index query kernels and the multi-index
// persistent kernel.
//
// A wave takes 64 candidates at a time (lane = candidate).  Their rows are
// streamed in 32-float chunks: each load instruction brings 8 rows x 128
// contiguous bytes, the chunk is transposed through LDS and lane c adds
// q_t x_ct in FP64 in ascending t (products of two floats are exact in FP64,
// so the sum is the definition's, bit for bit).  The running top-k, sorted by
// (ip desc, id asc), lives in registers, S entries per lane.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>

namespace nrlsh {
namespace dev {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int RR_STRIDE = 36;  // floats per LDS row (16-byte aligned, conflict-free b128)
constexpr int RR_TILE_FLOATS = 64 * RR_STRIDE;

// Order-preserving encoding of a double as an unsigned word (a larger
// double gives a larger word; 0 is below every encoded value), so that
// slices of one query can publish their k-th best value with atomicMax.
__device__ __forceinline__ uint64_t order_key(double x)
{
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double order_value(uint64_t e)
{
    return __longlong_as_double((long long)((e >> 63) ? (e & 0x7FFFFFFFFFFFFFFFull) : ~e));
}

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

    // Offer one value per lane (ok = lane has a real candidate).  Values
    // below `floor` (a known lower bound of the k-th best) are not kept.
    __device__ void offer(double v, int32_t id, bool ok, int lane, double floor = -INFINITY)
    {
        uint64_t mask = __ballot(ok && !(v < floor) && better(v, id, th_v, th_i));
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
            refresh();
        }
    }

    // (th_v, th_i) = entry k - 1.  The register arrays are read with static
    // indexes only (a runtime index would move them to scratch memory).
    __device__ void refresh()
    {
        double v = tv[0];
        int32_t i = ti[0];
#pragma unroll
        for (int s = 1; s < S; ++s) {
            if (s == ks) {
                v = tv[s];
                i = ti[s];
            }
        }
        th_v = __shfl(v, kl, 64);
        th_i = __shfl(i, kl, 64);
    }
};

// sum_t q_t x_pt in FP64, ascending t, for the stored row p of each lane
// (valid lanes only; 0 otherwise).  Xl rows are dp floats, zero past d.
// The 32-float chunks are double-buffered: the loads of chunk c + 1 are in
// flight while chunk c is summed from LDS.
__device__ __forceinline__ double ip64_rows_fp32(const float *__restrict__ Xl, int d, int dp,
                                                 const float *__restrict__ qv, int32_t p, bool valid,
                                                 int lane, float *tile)
{
    const int sub = lane >> 3, seg = 4 * (lane & 7);
    int64_t roff[8];
    bool rval[8];
#pragma unroll
    for (int it = 0; it < 8; ++it) {
        const int rr = 8 * it + sub;
        roff[it] = (int64_t)__shfl(valid ? p : 0, rr, 64) * dp;
        rval[it] = __shfl((int)valid, rr, 64) != 0;
    }
    floatx4 buf[8];
#pragma unroll
    for (int it = 0; it < 8; ++it) {
        buf[it] = floatx4{0.f, 0.f, 0.f, 0.f};
        if (rval[it] && seg < dp) buf[it] = *reinterpret_cast<const floatx4 *>(Xl + roff[it] + seg);
    }
    double acc = 0.0;
    for (int k0 = 0; k0 < dp; k0 += 32) {
#pragma unroll
        for (int it = 0; it < 8; ++it)
            *reinterpret_cast<floatx4 *>(&tile[(8 * it + sub) * RR_STRIDE + seg]) = buf[it];
        const int col = k0 + 32 + seg;
        if (k0 + 32 < dp) {
#pragma unroll
            for (int it = 0; it < 8; ++it) {
                buf[it] = floatx4{0.f, 0.f, 0.f, 0.f};
                if (rval[it] && col < dp) buf[it] = *reinterpret_cast<const floatx4 *>(Xl + roff[it] + col);
            }
        }
        __syncthreads();
        const floatx4 *row = reinterpret_cast<const floatx4 *>(&tile[lane * RR_STRIDE]);
        // the sum is one dependent chain: reading the tile two pieces at a
        // time keeps registers (and so resident waves) free
#pragma unroll 2
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
    return acc;
}

}  // namespace dev
}  // namespace nrlsh
