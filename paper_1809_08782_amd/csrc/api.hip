// Host side of libnrlsh: argument validation, device memory, the projection
// matrix generator, the sorted (U_j, l) structure and the launch sequence of
// index build (Algorithm 1) and query (Section 3.3 multi-probe + Algorithm 2
// re-rank).  Every data-parallel step runs in the kernels of k_build.hip and
// k_query.hip; the host only computes O(L d) and O(m L log(m L)) set-up
// tables.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "host_common.h"
#include "nrlsh.h"
#include "nrlsh_internal.h"

using namespace nrlsh;
using namespace nrlsh::host;

namespace {

thread_local std::string g_err;
thread_local nrlsh_query_stats g_qstats;
// scan_guess of the calling nrlsh_query_ex (0 outside it): how the scan probe
// finds the probed sets (nrlsh_query_opts)
thread_local int32_t g_scan_guess = 0;
// dense_head of the calling nrlsh_query_ex (0 outside it): which sub-datasets
// the bfloat16 re-rank screens whole instead of gathering their probed rows
thread_local int32_t g_dense_head = 0;

struct ProfEntry {
    double ms = 0.0;
    int64_t launches = 0;
};

std::atomic<int> g_prof_on{0};
std::mutex g_prof_mu;
std::map<std::string, ProfEntry> g_prof;

std::mutex g_dev_mu;
std::map<int, hipStream_t> g_streams;
std::map<int, bool> g_pool_ready;

}  // namespace

// ================================================================= plumbing
namespace nrlsh {
namespace host {

nrlsh_status fail(nrlsh_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

[[noreturn]] void throw_hip(hipError_t e, const char *what)
{
    if (e == hipErrorOutOfMemory)
        throw Failure{NRLSH_E_OUT_OF_MEMORY, std::string(what) + ": out of device memory"};
    throw Failure{NRLSH_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

bool prof_enabled() { return g_prof_on.load() != 0; }

void prof_record(const char *name, float ms)
{
    std::lock_guard<std::mutex> g(g_prof_mu);
    ProfEntry &e = g_prof[name];
    e.ms += ms;
    e.launches += 1;
}

hipStream_t library_stream(int dev)
{
    std::lock_guard<std::mutex> g(g_dev_mu);
    auto it = g_streams.find(dev);
    if (it != g_streams.end()) return it->second;
    hipStream_t s;
    HIPX(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    g_streams[dev] = s;
    return s;
}

void prepare_pool(int dev)
{
    std::lock_guard<std::mutex> g(g_dev_mu);
    if (g_pool_ready[dev]) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    g_pool_ready[dev] = true;
}

int current_device()
{
    int dev = 0;
    HIPX(hipGetDevice(&dev));
    return dev;
}

namespace {
struct CacheEntry {
    void *p;
    size_t bytes;
    hipStream_t s;  // stream of the release
    hipEvent_t ev;  // recorded on s at the release
    int dev;
};
constexpr size_t kCacheBytes = size_t(8) << 30;  // held at most, all devices
std::mutex g_cache_mu;
// never destroyed: blocks still cached when the process ends go with it
std::vector<CacheEntry> &g_cache = *new std::vector<CacheEntry>();
// idle events, per device (an event is recorded on streams of its own device)
std::map<int, std::vector<hipEvent_t>> &g_events = *new std::map<int, std::vector<hipEvent_t>>();
size_t g_cache_held = 0;

void drop_entry(const CacheEntry &e)
{
    // the block's last use is finished once its event is: free it on the
    // library stream of its device (the stream of the release may be gone)
    (void)hipEventSynchronize(e.ev);
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != e.dev) (void)hipSetDevice(e.dev);
    (void)hipFreeAsync(e.p, library_stream(e.dev));
    if (cur != e.dev) (void)hipSetDevice(cur);
    g_events[e.dev].push_back(e.ev);
}
}  // namespace

void *cached_alloc(size_t bytes, hipStream_t s, int *dev_out)
{
    const int dev = current_device();
    *dev_out = dev;
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        int best = -1;
        for (int i = 0; i < (int)g_cache.size(); ++i) {
            const CacheEntry &e = g_cache[(size_t)i];
            if (e.dev != dev || e.bytes < bytes || e.bytes > bytes + bytes / 2 + (size_t(1) << 20)) continue;
            if (best >= 0 && e.bytes >= g_cache[(size_t)best].bytes) continue;
            if (e.s == s || hipEventQuery(e.ev) == hipSuccess) best = i;
        }
        if (best >= 0) {
            const CacheEntry e = g_cache[(size_t)best];
            g_cache.erase(g_cache.begin() + best);
            g_cache_held -= e.bytes;
            g_events[e.dev].push_back(e.ev);
            return e.p;
        }
    }
    void *v = nullptr;
    hipError_t e = hipMallocAsync(&v, bytes, s);
    if (e != hipSuccess) {
        // give the cached blocks back to the pool and try once more
        {
            std::lock_guard<std::mutex> g(g_cache_mu);
            for (const CacheEntry &c : g_cache) drop_entry(c);
            g_cache.clear();
            g_cache_held = 0;
        }
        e = hipMallocAsync(&v, bytes, s);
    }
    if (e != hipSuccess) throw_hip(e, "hipMallocAsync");
    return v;
}

hipEvent_t event_take(int dev)
{
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        std::vector<hipEvent_t> &pool = g_events[dev];
        if (!pool.empty()) {
            hipEvent_t ev = pool.back();
            pool.pop_back();
            return ev;
        }
    }
    int cur = 0;
    HIPX(hipGetDevice(&cur));
    if (cur != dev) HIPX(hipSetDevice(dev));
    hipEvent_t ev = nullptr;
    const hipError_t ce = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (cur != dev) (void)hipSetDevice(cur);
    if (ce != hipSuccess) throw_hip(ce, "hipEventCreateWithFlags");
    return ev;
}

void event_give(hipEvent_t ev, int dev)
{
    if (!ev) return;
    std::lock_guard<std::mutex> g(g_cache_mu);
    g_events[dev].push_back(ev);
}

namespace {
struct PinnedEntry {
    void *p;
    size_t bytes;
    hipEvent_t ev;  // NULL: free now
    int dev;
};
std::vector<PinnedEntry> &g_pinned = *new std::vector<PinnedEntry>();
}  // namespace

void *pinned_take(size_t bytes, size_t *got)
{
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        for (size_t i = 0; i < g_pinned.size(); ++i) {
            const PinnedEntry e = g_pinned[i];
            if (e.bytes < bytes || (e.ev && hipEventQuery(e.ev) != hipSuccess)) continue;
            g_pinned.erase(g_pinned.begin() + (ptrdiff_t)i);
            if (e.ev) g_events[e.dev].push_back(e.ev);
            *got = e.bytes;
            return e.p;
        }
    }
    const size_t want = std::max<size_t>(bytes, size_t(64) << 10);
    void *p = nullptr;
    const hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
    if (e != hipSuccess) throw_hip(e, "hipHostMalloc");
    *got = want;
    return p;
}

void pinned_give(void *p, size_t bytes, hipStream_t s, int dev)
{
    if (!p) return;
    hipEvent_t ev = nullptr;
    if (s) {
        try {
            ev = event_take(dev);
        } catch (...) {
            ev = nullptr;
        }
        if (ev && hipEventRecord(ev, s) != hipSuccess) {
            event_give(ev, dev);
            (void)hipStreamSynchronize(s);
            ev = nullptr;
        } else if (!ev) {
            (void)hipStreamSynchronize(s);
        }
    }
    std::lock_guard<std::mutex> g(g_cache_mu);
    g_pinned.push_back(PinnedEntry{p, bytes, ev, dev});
}

void cached_free(void *p, size_t bytes, hipStream_t s, int dev)
{
    if (!p) return;
    std::lock_guard<std::mutex> g(g_cache_mu);
    std::vector<hipEvent_t> &pool = g_events[dev];
    hipEvent_t ev = nullptr;
    if (!pool.empty()) {
        ev = pool.back();
        pool.pop_back();
    } else {
        int cur = 0;
        (void)hipGetDevice(&cur);
        if (cur != dev) (void)hipSetDevice(dev);
        const hipError_t ce = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (cur != dev) (void)hipSetDevice(cur);
        if (ce != hipSuccess) {
            (void)hipFreeAsync(p, s);
            return;
        }
    }
    if (hipEventRecord(ev, s) != hipSuccess) {
        pool.push_back(ev);
        (void)hipFreeAsync(p, s);
        return;
    }
    g_cache.push_back(CacheEntry{p, bytes, s, ev, dev});
    g_cache_held += bytes;
    while (g_cache_held > kCacheBytes && !g_cache.empty()) {  // oldest first
        drop_entry(g_cache.front());
        g_cache_held -= g_cache.front().bytes;
        g_cache.erase(g_cache.begin());
    }
}

}  // namespace host
}  // namespace nrlsh

namespace {

// ================================================================= projection
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) addressed by position: output
// k of the generator seeded with `seed` is mix(seed + (k+1) * gamma).
uint64_t splitmix64_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Gaussian entries of the projection matrix (Eq. 4: i.i.d. N(0,1)).  Entry
// (r, c) takes outputs 2t and 2t+1, t = r (d+1) + c, through Box-Muller with
// u1 in (0, 1] and u2 in [0, 1), and is rounded to float32.
void make_projection(uint64_t seed, int L, int d, std::vector<float> &A)
{
    A.resize((size_t)L * (d + 1));
    auto rows = [&](int r0, int r1) {
        for (int r = r0; r < r1; ++r)
            for (int c = 0; c <= d; ++c) {
                const uint64_t t = (uint64_t)r * (uint64_t)(d + 1) + (uint64_t)c;
                const uint64_t h1 = splitmix64_at(seed, 2u * t);
                const uint64_t h2 = splitmix64_at(seed, 2u * t + 1u);
                const double u1 = (double)((h1 >> 11) + 1u) * (1.0 / 9007199254740992.0);
                const double u2 = (double)(h2 >> 11) * (1.0 / 9007199254740992.0);
                const double g = std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
                A[(size_t)r * (d + 1) + c] = (float)g;
            }
    };
    // entries are independent (counter-based), so large matrices (one block
    // per sub-dataset) are drawn by several host threads with the same result
    const int64_t work = (int64_t)L * (d + 1);
    const int nt = work < (1 << 16) ? 1 : (int)std::min<unsigned>(8u, std::max(1u, std::thread::hardware_concurrency()));
    if (nt == 1) {
        rows(0, L);
        return;
    }
    std::vector<std::thread> th;
    for (int i = 0; i < nt; ++i) th.emplace_back(rows, (int)((int64_t)L * i / nt), (int)((int64_t)L * (i + 1) / nt));
    for (auto &t : th) t.join();
}

// ================================================================= rank table
// Level factor of the similarity metric s_hat = U_j cos[pi (1-eps)(1 - l/L)]
// (Eq. 12 and its adjusted form).  For eps = 0 the zero at l = L/2 is exact
// and the factor is antisymmetric about it, so that sub-datasets tie exactly
// there instead of through the rounding of cos(pi/2).
double level_factor(int l, int L, double eps)
{
    if (eps != 0.0) return std::cos(M_PI * (1.0 - eps) * (double)(L - l) / (double)L);
    if (2 * l == L) return 0.0;
    if (2 * l > L) return std::cos(M_PI * (double)(L - l) / (double)L);
    return -std::cos(M_PI * (double)l / (double)L);
}

// R[j][l] = probing position of bucket (j, l), ordered by (s_hat desc,
// j desc, l desc) -- the sorted structure of Section 3.3.  inv[b] is the
// histogram index j*(L+1) + (L - l) of the bucket at position b.
void make_rank_table(const std::vector<double> &U, int L, double eps, std::vector<int32_t> &R,
                     std::vector<int32_t> &inv)
{
    const int m = (int)U.size(), L1 = L + 1;
    struct E {
        double s;
        int j, l;
    };
    std::vector<E> e((size_t)m * L1);
    for (int j = 0; j < m; ++j)
        for (int l = 0; l <= L; ++l) e[(size_t)j * L1 + l] = E{U[j] * level_factor(l, L, eps), j, l};
    std::sort(e.begin(), e.end(), [](const E &a, const E &b) {
        if (a.s != b.s) return a.s > b.s;
        if (a.j != b.j) return a.j > b.j;
        return a.l > b.l;
    });
    R.assign((size_t)m * L1, 0);
    inv.assign((size_t)m * L1, 0);
    for (size_t b = 0; b < e.size(); ++b) {
        R[(size_t)e[b].j * L1 + e[b].l] = (int32_t)b;
        inv[b] = e[b].j * L1 + (L - e[b].l);
    }
}

bool all_finite(const float *p, int64_t count)
{
    for (int64_t i = 0; i < count; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace

namespace {

hipStream_t pick_stream(void *user, int dev)
{
    return user ? static_cast<hipStream_t>(user) : library_stream(dev);
}

// Precision form of the hash: quantised copies of the items and projections,
// the low-precision matrix-core hash with its margin; the bits inside the
// margin of an item with few of them are recomputed in FP64 by the fix-up,
// an item with many is re-hashed whole from the FP32 rows (with its own FP64
// band).
void hash_low_precision(nrlsh_index *ix, const std::vector<float> &tau_h, const float *tau_d,
                        FixEntry *fix, BuildCounters *ctr, hipStream_t s, Timer &tm)
{
    const int64_t n = ix->n;
    const int d = ix->d, dp = ix->dp, L = ix->L;
    const bool fp8 = ix->storage == NRLSH_STORAGE_FP8_E4M3;
    const size_t es = fp8 ? 1 : 2;
    // margins: RIGOROUS bounds |p~ - p| by qrel ||a_r[:d]|| ||x|| (rounding of
    // both operands, exact low-precision products, FP32 accumulation) plus the
    // FP32 band tau_r U_j; SCALED uses margin_param ||x||
    const double gd = d * 0x1p-24 / (1.0 - d * 0x1p-24);
    const double qrel = fp8 ? (0x1p-3 + 0x1p-8 + 0x1p-20 + 0x1p-21 + 0x1p-10 * 2.2 * std::sqrt((double)d) / 448.0 +
                               0x1p-20 * d / (448.0 * 448.0) + 2.2 * gd)
                            : (0x1p-7 + 0x1p-16 + 0x1p-21 + 2.2 * gd);
    std::vector<float> mq_h(L), tq_h(L);
    for (int r = 0; r < L; ++r) {
        double a2 = 0.0;
        for (int c = 0; c < d; ++c) a2 += (double)ix->A_h[(size_t)r * (d + 1) + c] * ix->A_h[(size_t)r * (d + 1) + c];
        if (ix->margin_mode == NRLSH_MARGIN_RIGOROUS) {
            mq_h[r] = std::nextafter((float)(qrel * (1.0 + 0x1p-10) * std::sqrt(a2)), INFINITY);
            tq_h[r] = tau_h[r];
        } else {
            mq_h[r] = (float)ix->margin_param;
            tq_h[r] = 0.f;
        }
    }
    DBuf<float> mq(L, s), tq(L, s), ascale(L, s);
    DBuf<uint8_t> Aq((size_t)L * dp * es, s);
    DBuf<int32_t> rows((size_t)n, s);
    HIPX(hipMemcpyAsync(mq.get(), mq_h.data(), L * sizeof(float), hipMemcpyHostToDevice, s));
    HIPX(hipMemcpyAsync(tq.get(), tq_h.data(), L * sizeof(float), hipMemcpyHostToDevice, s));
    const int st = fp8 ? 2 : 1;
    HIPX(launch_quant_rows(ix->A.get(), L, d, d + 1, st, Aq.get(), dp, ascale.get(), s));
    const void *Xq = ix->Xh.get();
    if (fp8) {
        ix->Xf8 = DBuf<uint8_t>((size_t)n * dp, s);
        ix->xscale = DBuf<float>((size_t)n, s);
        tm.begin("quant");
        HIPX(launch_quant_rows(ix->Xl.get(), n, d, dp, 2, ix->Xf8.get(), dp, ix->xscale.get(), s));
        tm.end();
        Xq = ix->Xf8.get();
    }
    tm.begin("hash");
    HIPX(launch_hash_q(st, Xq, fp8 ? ix->xscale.get() : nullptr, n, d, dp, Aq.get(), ascale.get(),
                       ix->A.get(), L, ix->key_l.get(), ix->sid_l.get(), ix->keymax.get(),
                       ix->U.get(), mq.get(), tq.get(), ix->codes_l.get(), rows.get(), fix, ctr, s));
    tm.end();
    BuildCounters hc{};
    HIPX(hipMemcpyAsync(&hc, ctr, sizeof hc, hipMemcpyDeviceToHost, s));
    HIPX(hipStreamSynchronize(s));
    if (hc.lowp_items > 0) {
        tm.begin("hash_rehash");
        HIPX(launch_hash(ix->Xl.get(), hc.lowp_items, d, dp, ix->A.get(), L, ix->key_l.get(),
                         ix->sid_l.get(), ix->keymax.get(), ix->U.get(), tau_d, ix->codes_l.get(),
                         fix, ctr, rows.get(), s));
        tm.end();
    }
}

// Stages of the staged pass 1: the sub-datasets in jord_h order, cut at
// positions e_1 = ceil(m / 16), e_{i+1} = max(e_i + 1, ceil(1.5 e_i)), ..., m;
// each stage's sub-datasets cut into chunks sized so that a stage gives the
// launch about 2048 (tile, chunk) blocks.  cut[s]: rank of the first bucket
// of the first sub-dataset after stage s (the bound k_stage_check uses).
struct ScanStages {
    std::vector<int32_t> chunks;  // (sub-dataset, first, end) triples, stage by stage
    std::vector<int> cbeg;        // first triple of each stage, then the total
    std::vector<int> cut;         // per stage but the last
};

ScanStages scan_stages(const nrlsh_index *ix, int64_t tiles)
{
    ScanStages st;
    const int m = ix->m, L1 = ix->L + 1;
    std::vector<int> ends;
    int e = std::max(1, (m + 15) / 16);
    for (;;) {
        e = std::min(e, m);
        ends.push_back(e);
        if (e == m) break;
        e = std::max(e + 1, (e * 3 + 1) / 2);
    }
    int b = 0;
    for (size_t s = 0; s < ends.size(); ++s) {
        st.cbeg.push_back((int)(st.chunks.size() / 3));
        int64_t items = 0;
        for (int i = b; i < ends[s]; ++i) {
            const int j = ix->jord_h[i];
            items += ix->off_h[j + 1] - ix->off_h[j];
        }
        int64_t chunk = (items * std::max<int64_t>(tiles, 1) + 2047) / 2048;
        // fewer than 2^16 items: the collecting scan stages 16-bit offsets and
        // counts a chunk's items per (query, level) in 16-bit halves
        chunk = std::min<int64_t>(65472, std::max<int64_t>(2048, (chunk + 63) / 64 * 64));
        for (int i = b; i < ends[s]; ++i) {
            const int j = ix->jord_h[i];
            for (int64_t p = ix->off_h[j]; p < ix->off_h[j + 1]; p += chunk) {
                st.chunks.push_back(j);
                st.chunks.push_back((int32_t)p);
                st.chunks.push_back((int32_t)std::min<int64_t>(p + chunk, ix->off_h[j + 1]));
            }
        }
        if (ends[s] < m) st.cut.push_back(ix->R_h[(size_t)ix->jord_h[ends[s]] * L1 + ix->L]);
        b = ends[s];
    }
    st.cbeg.push_back((int)(st.chunks.size() / 3));
    return st;
}

void build_index(nrlsh_index *ix, const float *items, bool on_device, hipStream_t s, Timer &tm)
{
    const int64_t n = ix->n;
    const int d = ix->d, dp = ix->dp, m = ix->m, L = ix->L, W = ix->W;

    // projection matrix: one L-row block, or one per sub-dataset, for each
    // hash table (drawn on the host once the first kernels are queued)
    const int tables = ix->tables;
    const int trows = ix->qsets * L;  // rows of one table
    const int rows = tables * trows;
    const size_t a_elems = (size_t)rows * (d + 1), at_elems = (size_t)rows * d;

    Block &B = ix->mem;
    // the bfloat16 copies carry a zeroed tail pad of 32 values: the screen
    // reads whole 32-coordinate steps past the last row's dp values
    const size_t oXl = B.reserve<float>((size_t)n * dp),
                 oXh = B.reserve<uint16_t>((size_t)n * dp + 32),
                 oA = B.reserve<float>(a_elems),
                 oAt = B.reserve<float>(at_elems), okey = B.reserve<double>(n),
                 okeyl = B.reserve<double>(n), okm = B.reserve<double>(m), oU = B.reserve<double>(m),
                 osid = B.reserve<int32_t>(n), osidl = B.reserve<int32_t>(n),
                 operm = B.reserve<int32_t>(n), ooff = B.reserve<int32_t>(m + 1),
                 oR = B.reserve<int32_t>((size_t)m * (L + 1)),
                 oinv = B.reserve<int32_t>((size_t)m * (L + 1)),
                 ocodes = B.reserve<uint32_t>((size_t)n * W * tables), oxeb = B.reserve<float>(n),
                 oRs = B.reserve<int32_t>((size_t)m * tables), oinvs = B.reserve<int32_t>((size_t)m * tables),
                 ost1 = B.reserve<int32_t>(3 * ((size_t)n / 2048 + 2 * (size_t)m + 8));
    // bucket tables: room for n distinct codes (the actual count is known after the build)
    const bool tab = ix->has_table;
    const size_t otc = B.reserve<uint64_t>(tab ? (size_t)n : 1),
                 ots = B.reserve<int32_t>(tab ? (size_t)n + 1 : 1),
                 oto = B.reserve<int32_t>(tab ? (size_t)m + 1 : 1),
                 oti = B.reserve<int32_t>(tab ? (size_t)n : 1),
                 otb = B.reserve<uint64_t>(tab ? table_binom_words() : 1);
    B.allocate(s);
    ix->Xl = B.view<float>(oXl);
    ix->Xh = B.view<uint16_t>(oXh);
    ix->A = B.view<float>(oA);
    ix->At = B.view<float>(oAt);
    ix->key = B.view<double>(okey);
    ix->key_l = B.view<double>(okeyl);
    ix->keymax = B.view<double>(okm);
    ix->U = B.view<double>(oU);
    ix->sid = B.view<int32_t>(osid);
    ix->sid_l = B.view<int32_t>(osidl);
    ix->perm = B.view<int32_t>(operm);
    ix->off = B.view<int32_t>(ooff);
    ix->R = B.view<int32_t>(oR);
    ix->inv = B.view<int32_t>(oinv);
    ix->codes_l = B.view<uint32_t>(ocodes);
    ix->xeb = B.view<float>(oxeb);
    ix->Rs = B.view<int32_t>(oRs);
    ix->invs = B.view<int32_t>(oinvs);
    ix->st1_chunks_d = B.view<int32_t>(ost1);
    if (tab) {
        ix->ucode = B.view<uint64_t>(otc);
        ix->ustart = B.view<int32_t>(ots);
        ix->uoff = B.view<int32_t>(oto);
        ix->titem = B.view<int32_t>(oti);
        ix->binom = B.view<uint64_t>(otb);
    }

    // build-time scratch, one block
    Block T;
    const size_t otau = T.reserve<float>(rows), oka = T.reserve<uint64_t>(n), okb = T.reserve<uint64_t>(n),
                 ova = T.reserve<int32_t>(n), ovb = T.reserve<int32_t>(n),
                 ortmp = T.reserve<uint8_t>(radix_sort_tmp_bytes(n)), ofix = T.reserve<FixEntry>(n),
                 octr = T.reserve<BuildCounters>(1),
                 ostg = T.reserve<float>(on_device ? 1 : (size_t)n * d),
                 obnd = T.reserve<double>(m), osub = T.reserve<int32_t>(m),
                 obst = T.reserve<int32_t>((size_t)m + 1),
                 otbs = T.reserve<int32_t>(tab ? table_scan_words(n) + 1 : 1);
    T.allocate(s);
    DBuf<float> tau = T.view<float>(otau);
    DBuf<uint64_t> ka = T.view<uint64_t>(oka), kb = T.view<uint64_t>(okb);
    DBuf<int32_t> va = T.view<int32_t>(ova), vb = T.view<int32_t>(ovb);
    DBuf<uint8_t> rtmp = T.view<uint8_t>(ortmp);
    DBuf<FixEntry> fix = T.view<FixEntry>(ofix);
    DBuf<BuildCounters> ctr = T.view<BuildCounters>(octr);
    DBuf<float> staging = T.view<float>(ostg);
    DBuf<double> bounds = T.view<double>(obnd);
    DBuf<int32_t> subend = T.view<int32_t>(osub);
    DBuf<int32_t> bstart = T.view<int32_t>(obst);
    const float *X = items;
    if (!on_device) {
        HIPX(hipMemcpyAsync(staging.get(), items, (size_t)n * d * sizeof(float),
                            hipMemcpyHostToDevice, s));
        X = staging.get();
    }
    HIPX(hipMemsetAsync(ctr.get(), 0, sizeof(BuildCounters), s));

    // Algorithm 1: rank by 2-norm, cut into m percentile ranges
    tm.begin("keys");
    HIPX(launch_keys(X, n, d, ix->key.get(), ka.get(), va.get(), ctr.get(), s));
    tm.end();
    bool in_b = false;
    tm.begin("sort");
    HIPX(radix_sort(ka.get(), va.get(), kb.get(), vb.get(), n, 64, rtmp.get(), &in_b, s));
    tm.end();

    // while the device ranks the items: the projection, the transpose of each
    // block and the FP32 uncertainty band factors (first read by the hash)
    make_projection(ix->seed, rows, d, ix->A_h);
    // A[:, :d] transposed table by table: table tau's block is d x trows
    std::vector<float> At_h(at_elems), tau_h(rows);
    for (int r = 0; r < rows; ++r) {
        const int tb = r / trows, rr = r - tb * trows;
        double nrm2 = 0.0;
        for (int c = 0; c <= d; ++c) {
            const double a = ix->A_h[(size_t)r * (d + 1) + c];
            nrm2 += a * a;
            if (c < d) At_h[(size_t)tb * d * trows + (size_t)c * trows + rr] = (float)a;
        }
        // tau_r = 2 gamma_{d+3} ||a_r||, gamma_k = k u / (1 - k u), u = 2^-24,
        // rounded up so that the band is never narrower than the bound.
        const double ku = (double)(d + 3) * 0x1p-24;
        const double tau = 2.0 * (ku / (1.0 - ku)) * std::sqrt(nrm2) * (1.0 + 0x1p-20);
        tau_h[r] = std::nextafter((float)tau, INFINITY);
    }
    HIPX(hipMemcpyAsync(ix->A.get(), ix->A_h.data(), ix->A_h.size() * sizeof(float),
                        hipMemcpyHostToDevice, s));
    HIPX(hipMemcpyAsync(ix->At.get(), At_h.data(), At_h.size() * sizeof(float),
                        hipMemcpyHostToDevice, s));
    HIPX(hipMemcpyAsync(tau.get(), tau_h.data(), tau_h.size() * sizeof(float),
                        hipMemcpyHostToDevice, s));
    uint64_t *sk = in_b ? kb.get() : ka.get();
    int32_t *sv = in_b ? vb.get() : va.get();
    uint64_t *lk = in_b ? ka.get() : kb.get();
    int32_t *lv = in_b ? va.get() : vb.get();
    // uniform ranges (Section 5): boundaries from the smallest and largest
    // key, b_j = nmin + j w, compared with the keys as b_j^2
    const bool uniform = ix->partition == NRLSH_PARTITION_UNIFORM && m > 1;
    std::vector<double> bnd_h;  // outlives its copy (the stream is synchronised below)
    if (uniform) {
        double kext[2];
        HIPX(hipMemcpyAsync(&kext[0], sk, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPX(hipMemcpyAsync(&kext[1], sk + n - 1, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPX(hipStreamSynchronize(s));
        const double nmin = std::sqrt(kext[0]), nmax = std::sqrt(kext[1]);
        const double w = (nmax - nmin) / (double)m;
        bnd_h.resize((size_t)m - 1);
        for (int j = 1; j < m; ++j) {
            const double b = nmin + (double)j * w;
            bnd_h[(size_t)j - 1] = b * b;
        }
        HIPX(hipMemcpyAsync(bounds.get(), bnd_h.data(), bnd_h.size() * sizeof(double),
                            hipMemcpyHostToDevice, s));
    }
    HIPX(hipMemsetAsync(ix->keymax.get(), 0, m * sizeof(double), s));
    HIPX(hipMemsetAsync(subend.get(), 0xFF, m * sizeof(int32_t), s));
    HIPX(launch_assign_subsets(sk, sv, n, m, uniform ? bounds.get() : nullptr, ix->sid.get(), lk, lv,
                               ix->keymax.get(), subend.get(), s));

    // The host needs the counters, U_j and the sub-dataset ends for the rank
    // table; they come back through pinned memory while the device already
    // puts the items in stored order, which needs nothing from the host.
    const size_t rank_n = (size_t)m * (L + 1);
    const size_t p_hc = 0, p_km = 64, p_se = p_km + (size_t)m * 8, p_U = (p_se + (size_t)m * 4 + 15) / 16 * 16,
                 p_R = p_U + (size_t)m * 8, p_inv = p_R + rank_n * 4, p_off = p_inv + rank_n * 4,
                 p_end = p_off + ((size_t)m + 1) * 4;
    static_assert(sizeof(BuildCounters) <= 64, "counters fit their slot");
    size_t pin_bytes = 0;
    uint8_t *pin = static_cast<uint8_t *>(pinned_take(p_end, &pin_bytes));
    struct PinRelease {  // after every copy from or into it has been queued
        void *p;
        size_t b;
        hipStream_t s;
        int dev;
        ~PinRelease() { pinned_give(p, b, s, dev); }
    } pin_release{pin, pin_bytes, s, ix->device};
    HIPX(hipMemcpyAsync(pin + p_hc, ctr.get(), sizeof(BuildCounters), hipMemcpyDeviceToHost, s));
    HIPX(hipMemcpyAsync(pin + p_km, ix->keymax.get(), m * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPX(hipMemcpyAsync(pin + p_se, subend.get(), m * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    hipEvent_t ev_back = event_take(ix->device);
    struct EvRelease {
        hipEvent_t e;
        int dev;
        ~EvRelease() { event_give(e, dev); }
    } ev_back_release{ev_back, ix->device};
    HIPX(hipEventRecord(ev_back, s));

    // stored order: sub-dataset major, ascending original index inside
    int bits = 0;
    while ((1ll << bits) < (int64_t)m) ++bits;
    bits = (bits + 7) / 8 * 8;
    const int32_t *perm_src = lv;
    if (bits > 0) {
        bool lb = false;
        HIPX(radix_sort(lk, lv, sk, sv, n, bits, rtmp.get(), &lb, s));
        perm_src = lb ? sv : lv;
    }
    HIPX(hipMemcpyAsync(ix->perm.get(), perm_src, (size_t)n * sizeof(int32_t),
                        hipMemcpyDeviceToDevice, s));
    tm.begin("layout");
    HIPX(launch_layout(X, n, d, dp, ix->perm.get(), ix->key.get(), ix->sid.get(), ix->Xl.get(),
                       ix->Xh.get(), nullptr, ix->key_l.get(), ix->sid_l.get(), ix->xeb.get(), s));
    tm.end();
    HIPX(hipMemsetAsync(ix->Xh.get() + (size_t)n * dp, 0, 32 * sizeof(uint16_t), s));
    // the layout is the last reader of the caller's items
    hipEvent_t ev_items = event_take(ix->device);
    EvRelease ev_items_release{ev_items, ix->device};
    HIPX(hipEventRecord(ev_items, s));

    HIPX(hipEventSynchronize(ev_back));
    BuildCounters hc;
    std::memcpy(&hc, pin + p_hc, sizeof hc);
    if (hc.nonfinite) throw Failure{NRLSH_E_NOT_FINITE, "items hold NaN or Inf"};
    ix->keymax_h.resize(m);
    std::vector<int32_t> subend_h((size_t)m);
    std::memcpy(ix->keymax_h.data(), pin + p_km, m * sizeof(double));
    std::memcpy(subend_h.data(), pin + p_se, m * sizeof(int32_t));

    // U_j and the sorted (U_j, l) structure (host, FP64)
    ix->U_h.resize(m);
    for (int j = 0; j < m; ++j) ix->U_h[j] = std::sqrt(ix->keymax_h[j]);
    std::vector<int32_t> inv_h;
    make_rank_table(ix->U_h, L, ix->eps, ix->R_h, inv_h);
    ix->jord_h.resize(m);
    for (int j = 0; j < m; ++j) ix->jord_h[j] = j;
    std::sort(ix->jord_h.begin(), ix->jord_h.end(), [&](int32_t a, int32_t b) {
        return ix->U_h[a] != ix->U_h[b] ? ix->U_h[a] > ix->U_h[b] : a > b;
    });
    // sub-dataset j occupies sorted ranks [off_j, off_{j+1}); an empty one
    // (no end rank written) starts and ends where the previous one ended
    ix->off_h.assign(m + 1, 0);
    std::vector<int32_t> off32(m + 1, 0);
    for (int j = 0; j < m; ++j) {
        ix->off_h[j + 1] = subend_h[j] >= 0 ? subend_h[j] : ix->off_h[j];
        off32[j + 1] = (int32_t)ix->off_h[j + 1];
    }
    if (ix->off_h[m] != n) throw Failure{NRLSH_E_INTERNAL, "sub-dataset runs do not cover the items"};
    // the staged-scan plan of a single 64-query tile, kept with the index for
    // the query entry point that allocates nothing
    {
        ScanStages p1 = scan_stages(ix, 1);
        if (p1.chunks.size() > 3 * ((size_t)n / 2048 + 2 * (size_t)m + 8))
            throw Failure{NRLSH_E_INTERNAL, "scan plan exceeds its reserved room"};
        ix->st1_chunks = std::move(p1.chunks);
        ix->st1_cbeg = std::move(p1.cbeg);
        ix->st1_cut = std::move(p1.cut);
        HIPX(hipMemcpyAsync(ix->st1_chunks_d.get(), ix->st1_chunks.data(), ix->st1_chunks.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, s));
    }
    std::memcpy(pin + p_U, ix->U_h.data(), m * sizeof(double));
    std::memcpy(pin + p_R, ix->R_h.data(), rank_n * sizeof(int32_t));
    std::memcpy(pin + p_inv, inv_h.data(), rank_n * sizeof(int32_t));
    std::memcpy(pin + p_off, off32.data(), off32.size() * sizeof(int32_t));
    HIPX(hipMemcpyAsync(ix->U.get(), pin + p_U, m * sizeof(double), hipMemcpyHostToDevice, s));
    HIPX(hipMemcpyAsync(ix->R.get(), pin + p_R, rank_n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPX(hipMemcpyAsync(ix->inv.get(), pin + p_inv, rank_n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPX(hipMemcpyAsync(ix->off.get(), pin + p_off, off32.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));

    // the (f, j) rank table of the multi-table single probe: bins ordered by
    // the first table whose bucket holds the item (ascending), then
    // sub-dataset descending; bin (j, f) sits where the multi-probe table
    // keeps level l = t - 1 - f
    ix->Rs_h.assign((size_t)m * tables, 0);
    std::vector<int32_t> invs_h((size_t)m * tables);  // outlives its copy (synchronised below)
    for (int f = 0; f < tables; ++f)
        for (int j = 0; j < m; ++j) {
            const int32_t rank = f * m + (m - 1 - j);
            ix->Rs_h[(size_t)j * tables + (tables - 1 - f)] = rank;
            invs_h[(size_t)rank] = j * tables + f;
        }
    HIPX(hipMemcpyAsync(ix->Rs.get(), ix->Rs_h.data(), ix->Rs_h.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPX(hipMemcpyAsync(ix->invs.get(), invs_h.data(), invs_h.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));

    // SimpleLSH transform + sign random projection, then the FP64 fix-up,
    // table by table (table tau: projection rows tau trows .., codes tau n W ..)
    std::vector<int32_t> bstart_h((size_t)m + 1, 0);  // outlives its copy
    if (ix->qsets > 1) {
        // one projection block per sub-dataset: the launch's blocks are dealt
        // out sub-dataset by sub-dataset (first block of j = bstart[j])
        const int per_block = hash_items_per_block();
        for (int j = 0; j < m; ++j) {
            const int64_t nj = ix->off_h[j + 1] - ix->off_h[j];
            bstart_h[j + 1] = bstart_h[j] + (int32_t)((nj + per_block - 1) / per_block);
        }
        HIPX(hipMemcpyAsync(bstart.get(), bstart_h.data(), bstart_h.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, s));
    }
    for (int tb = 0; tb < tables; ++tb) {
        const float *At_b = ix->A.get() + (size_t)tb * trows * (d + 1);
        const float *tau_b = tau.get() + (size_t)tb * trows;
        uint32_t *codes_b = ix->codes_l.get() + (size_t)tb * n * W;
        if (tb > 0) HIPX(launch_roll_fix_count(ctr.get(), s));  // the fix list starts over
        if (ix->storage == NRLSH_STORAGE_FP32 && ix->qsets > 1) {
            tm.begin("hash");
            HIPX(launch_hash_per_subset(ix->Xl.get(), d, dp, At_b, L, ix->key_l.get(), ix->sid_l.get(),
                                        ix->keymax.get(), ix->U.get(), tau_b, ix->off.get(), bstart.get(), m,
                                        bstart_h[m], codes_b, fix.get(), ctr.get(), s));
            tm.end();
        } else if (ix->storage == NRLSH_STORAGE_FP32) {
            tm.begin("hash");
            HIPX(launch_hash(ix->Xl.get(), n, d, dp, At_b, L, ix->key_l.get(), ix->sid_l.get(), ix->keymax.get(),
                             ix->U.get(), tau_b, codes_b, fix.get(), ctr.get(), nullptr, s));
            tm.end();
        } else {
            hash_low_precision(ix, tau_h, tau.get(), fix.get(), ctr.get(), s, tm);
        }
        tm.begin("hash_fixup");
        HIPX(launch_hash_fixup(ix->Xl.get(), d, dp, At_b, L, ix->qsets > 1, ix->key_l.get(), ix->sid_l.get(),
                               ix->keymax.get(), ix->U.get(), fix.get(), ctr.get(), codes_b, n, s));
        tm.end();
    }

    // host sources of the copies below outlive them (synchronised at the end)
    std::vector<uint64_t> bh;
    std::vector<int32_t> uo;
    int32_t nn = (int32_t)n;
    if (tab) {
        // bucket tables over the final codes (the sort buffers are free again)
        DBuf<int32_t> tbs = T.view<int32_t>(otbs);
        int32_t *total_d = tbs.get() + table_scan_words(n);
        tm.begin("table");
        HIPX(launch_table_build(ix->codes_l.get(), ix->sid_l.get(), n, m, L, ka.get(), va.get(), kb.get(),
                                vb.get(), rtmp.get(), tbs.get(), total_d, ix->titem.get(),
                                ix->ucode.get(), ix->ustart.get(), ix->uoff.get(), s));
        tm.end();
        bh.resize(table_binom_words());
        table_binom(bh.data());
        HIPX(hipMemcpyAsync(ix->binom.get(), bh.data(), bh.size() * sizeof(uint64_t),
                            hipMemcpyHostToDevice, s));
        int32_t U = 0;
        uo.resize((size_t)m + 1);
        HIPX(hipMemcpyAsync(&U, total_d, sizeof U, hipMemcpyDeviceToHost, s));
        HIPX(hipMemcpyAsync(uo.data(), ix->uoff.get(), (size_t)m * sizeof(int32_t),
                            hipMemcpyDeviceToHost, s));
        HIPX(hipStreamSynchronize(s));
        // empty sub-datasets (no run written) start where the next one starts
        uo[m] = U;
        for (int j = m - 1; j >= 0; --j)
            if (ix->off_h[j + 1] == ix->off_h[j]) uo[j] = uo[j + 1];
        ix->nunique = U;
        ix->uoff_h.assign(uo.begin(), uo.end());
        HIPX(hipMemcpyAsync(ix->uoff.get(), uo.data(), uo.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, s));
        HIPX(hipMemcpyAsync(ix->ustart.get() + U, &nn, sizeof nn, hipMemcpyHostToDevice, s));
    }

    // the final counters arrive behind the last kernel; `ready` marks the
    // end of the build's device work, which later calls wait for (queries on
    // their stream, everything else on the host)
    ix->counters_h = pinned_take(sizeof(BuildCounters), &ix->counters_bytes);
    HIPX(hipMemcpyAsync(ix->counters_h, ctr.get(), sizeof(BuildCounters), hipMemcpyDeviceToHost, s));
    ix->ready = event_take(ix->device);
    HIPX(hipEventRecord(ix->ready, s));
    // long-lived buffers are released on the library stream by nrlsh_free
    ix->mem.mem.s = ix->home;
    ix->Xf8.s = ix->home;
    ix->xscale.s = ix->home;
    // the caller may reuse its items once this returns
    HIPX(hipEventSynchronize(ev_items));
}

}  // namespace

// The build returns with its last kernels still queued.  Queries wait for
// them on their own stream; every other use of the index waits on the host,
// which also takes the build counters in.
void index_wait(const nrlsh_index *ix, hipStream_t s)
{
    if (ix->ready && !ix->settled.load(std::memory_order_acquire)) HIPX(hipStreamWaitEvent(s, ix->ready, 0));
}

void index_settle(const nrlsh_index *ix)
{
    if (ix->settled.load(std::memory_order_acquire)) return;
    std::lock_guard<std::mutex> g(ix->ready_mu);
    if (ix->settled.load(std::memory_order_relaxed)) return;
    if (ix->ready) HIPX(hipEventSynchronize(ix->ready));
    if (ix->counters_h) {
        BuildCounters hc;
        std::memcpy(&hc, ix->counters_h, sizeof hc);
        ix->stats.lowp_items = hc.lowp_items;
        ix->stats.lowp_bits = (int64_t)hc.lowp_bits;
        ix->stats.lowp_changed = (int64_t)hc.lowp_changed;
        ix->stats.recomputed_items = (int64_t)hc.fix_count + hc.fix_prev;
        ix->stats.recomputed_bits = (int64_t)hc.fix_bits;
        ix->stats.recompute_flips = (int64_t)hc.fix_flips;
        ix->stats.recompute_flips_tiny = (int64_t)hc.fix_flips_tiny;
    }
    ix->settled.store(true, std::memory_order_release);
}

namespace {

nrlsh_status validate_build(const float *items, int64_t n, int32_t d, int32_t m, int32_t L,
                            double eps, nrlsh_index **out)
{
    if (!out) return fail(NRLSH_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!items) return fail(NRLSH_E_INVALID_ARG, "items is NULL");
    if (n < 1 || n > NRLSH_MAX_N) return fail(NRLSH_E_INVALID_ARG, "n = %lld out of [1, %d]", (long long)n, NRLSH_MAX_N);
    if (d < 1 || d > (1 << 24)) return fail(NRLSH_E_INVALID_ARG, "d = %d out of [1, 2^24]", d);
    if (m < 1 || (int64_t)m > n) return fail(NRLSH_E_INVALID_ARG, "m = %d out of [1, n]", m);
    if (L < 1 || L > NRLSH_MAX_L) return fail(NRLSH_E_INVALID_ARG, "L = %d out of [1, 64]", L);
    if ((int64_t)m * (L + 1) > INT32_MAX) return fail(NRLSH_E_INVALID_ARG, "m (L+1) too large");
    if (!(eps >= 0.0 && eps < 1.0)) return fail(NRLSH_E_INVALID_ARG, "eps out of [0, 1)");
    return NRLSH_OK;
}

nrlsh_status validate_query(const nrlsh_index *ix, const float *queries, int64_t nq, int32_t k,
                            int64_t T, const void *ids, const void *ips)
{
    if (!ix) return fail(NRLSH_E_INVALID_ARG, "index is NULL");
    if (nq < 0) return fail(NRLSH_E_INVALID_ARG, "nq < 0");
    if (k < 1 || k > NRLSH_MAX_K) return fail(NRLSH_E_INVALID_ARG, "k = %d out of [1, %d]", k, NRLSH_MAX_K);
    if (T < 1) return fail(NRLSH_E_INVALID_ARG, "probe_budget < 1");
    if (nq > 0 && (!queries || !ids || !ips)) return fail(NRLSH_E_INVALID_ARG, "NULL query or output pointer");
    if (nq > (int64_t)INT32_MAX) return fail(NRLSH_E_INVALID_ARG, "nq too large");
    return NRLSH_OK;
}

QueryShape make_shape(const nrlsh_index *ix, int64_t T, int32_t k)
{
    QueryShape sh;
    sh.n = ix->n;
    sh.d = ix->d;
    sh.dp = ix->dp;
    sh.m = ix->m;
    sh.L = ix->L;
    sh.W = ix->W;
    sh.Tq = std::min<int64_t>(T, ix->n);
    sh.k = k;
    sh.qsets = ix->qsets;
    return sh;
}

// Staged pass 1 of a batch: clears the histograms, scans stage by stage and
// stops each tile once all its queries are settled (k_stage_check).
void run_scan_hist_staged(const nrlsh_index *ix, const QueryShape &sh, const uint32_t *qc, int64_t nb,
                          const std::vector<int> &cbeg, const std::vector<int> &cut, const int32_t *chunks_d,
                          int32_t *need, uint32_t *ghist, unsigned long long *npairs, hipStream_t s)
{
    const int64_t tb = (nb + 63) / 64;
    HIPX(launch_fill32(ghist, tb * sh.m * (sh.L + 1) * 64, 0u, s));
    HIPX(launch_fill32(need, tb, 1u, s));
    if (cbeg.empty()) throw Failure{NRLSH_E_INTERNAL, "scan stages were not planned"};
    const int S = (int)cbeg.size() - 1;
    for (int k = 0; k < S; ++k) {
        HIPX(launch_scan_hist_stage(ix->codes_l.get(), qc, nb, sh, chunks_d + 3 * (size_t)cbeg[k],
                                    cbeg[k + 1] - cbeg[k], k == 0 ? nullptr : need, ghist, npairs, s));
        if (k + 1 < S) HIPX(launch_stage_check(ghist, ix->inv.get(), nb, sh, cut[k], need, s));
    }
}

bool screen_fits(const nrlsh_index *ix, int kind);

// Witnesses of the dense head, made once per index (see nrlsh_index): the
// kWitnessTop largest-norm items of each sub-dataset and every
// kWitnessStride-th one.
constexpr int kWitnessTop = 4096, kWitnessStride = 32;
void witness_rows(const nrlsh_index *ix, hipStream_t s)
{
    if (ix->wit_ready.load(std::memory_order_acquire)) return;
    std::lock_guard<std::mutex> g(ix->wit_mu);
    if (ix->wit_ready.load(std::memory_order_relaxed)) return;
    int64_t nmax = 0;
    for (int j = 0; j < ix->m; ++j) nmax = std::max<int64_t>(nmax, ix->off_h[(size_t)j + 1] - ix->off_h[(size_t)j]);
    const int W = (int)std::min<int64_t>(nmax, kWitnessTop + (nmax + kWitnessStride - 1) / kWitnessStride);
    const int m = ix->m, dp = ix->dp, cw = ix->W;
    const size_t slots = (size_t)m * W;
    DBuf<int32_t> pos(slots, s), cnt((size_t)m, s);
    DBuf<uint16_t> xw(slots * dp + 32, s);  // zeroed 32-value tail pad, as the row copies
    DBuf<uint32_t> cwo(slots * cw, s);
    DBuf<double> kw(slots, s);
    HIPX(hipMemsetAsync(xw.get() + slots * dp, 0, 32 * sizeof(uint16_t), s));
    HIPX(launch_wit_build(ix->Xh.get(), ix->codes_l.get(), ix->key_l.get(), ix->off.get(), m, dp, cw, kWitnessTop,
                          kWitnessStride, std::max(1, W), pos.get(), cnt.get(), xw.get(), cwo.get(), kw.get(), s));
    std::vector<int32_t> ch((size_t)m);
    HIPX(hipMemcpyAsync(ch.data(), cnt.get(), (size_t)m * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPX(hipStreamSynchronize(s));
    for (DBuf<int32_t> *b : {&pos, &cnt}) b->s = ix->home;  // released with the index, on the library stream
    xw.s = ix->home;
    cwo.s = ix->home;
    kw.s = ix->home;
    ix->wit_pos = std::move(pos);
    ix->wit_cnt = std::move(cnt);
    ix->wit_xh = std::move(xw);
    ix->wit_codes = std::move(cwo);
    ix->wit_key = std::move(kw);
    ix->wit_cnt_h = std::move(ch);
    ix->wit_per_sub = W;
    ix->wit_ready.store(true, std::memory_order_release);
}

// Sub-datasets that the bfloat16 re-rank screens whole (64-query tiles
// against all their items on the matrix cores, the screen path's two passes)
// instead of gathering the rows of their probed items: the contiguous range
// [jh0, jh1) around the sub-dataset with the largest probed fraction frac_j,
// extended while frac_j >= frac ({0, 0}: none).  frac_j is estimated from
// the sample pass (hits[j] sampled items of j rank before the batch's guessed
// cuts, one item in `stride` sampled).  Only the speed depends on the choice:
// the screen applies the same probe predicate, so both forms re-rank exactly
// the probed set.
std::pair<int, int> dense_head_range(const nrlsh_index *ix, const unsigned long long *hits, int64_t nb, int stride,
                                     double frac)
{
    const int m = ix->m;
    std::vector<double> f((size_t)m, 0.0);
    int jb = 0;
    for (int j = 0; j < m; ++j) {
        const double nj = (double)(ix->off_h[(size_t)j + 1] - ix->off_h[(size_t)j]);
        f[(size_t)j] = nj > 0.0 ? (double)hits[j] * stride / ((double)nb * nj) : 0.0;
        if (f[(size_t)j] > f[(size_t)jb]) jb = j;
    }
    if (!(f[(size_t)jb] >= frac)) return {0, 0};
    int j0 = jb, j1 = jb + 1;
    while (j0 > 0 && f[(size_t)j0 - 1] >= frac) --j0;
    while (j1 < m && f[(size_t)j1] >= frac) ++j1;
    return {j0, j1};
}

// (sub-dataset, first, end) triples of at most `items` stored items covering
// the sub-datasets js.
std::vector<int32_t> subset_chunks(const nrlsh_index *ix, int items, const std::vector<int> &js)
{
    std::vector<int32_t> ch;
    for (const int j : js)
        for (int64_t p = ix->off_h[(size_t)j]; p < ix->off_h[(size_t)j + 1]; p += items) {
            ch.push_back(j);
            ch.push_back((int32_t)p);
            ch.push_back((int32_t)std::min<int64_t>(p + items, ix->off_h[(size_t)j + 1]));
        }
    return ch;
}

// Gather path: materialise each query's probed list, then re-rank it.  When
// cand_out_d is given, the probed stored positions are copied there (nq x Tq)
// and the re-rank is skipped.  With `table` the probed lists come from the
// bucket tables instead of the scans.
void run_query_gather(const nrlsh_index *ix, const float *Qd, int64_t nq, int32_t k, int64_t T,
                      int64_t *ids_d, float *ips_d, int32_t *cand_out_d, uint32_t *qcodes_out_d,
                      hipStream_t s, Timer &tm, uint32_t *nonfinite_d, bool bf16_rows = false,
                      bool table = false, unsigned long long *scan_pairs_d = nullptr)
{
    const QueryShape sh = make_shape(ix, T, k);
    // queries per batch: a multiple of 64 keeping the candidate buffer <= 2^29 entries
    int64_t B = (int64_t(1) << 29) / sh.Tq;
    B = std::max<int64_t>(64, B / 64 * 64);
    B = std::min<int64_t>(B, (nq + 63) / 64 * 64);
    if (table) B = std::min<int64_t>(B, 16384);  // bounds the per-query bucket scratch
    // Large budgets take the collecting scan: a sample pass (every gstride-th
    // 16-item group) guesses each query's cut rho_q so that about 1.125 Tq
    // items rank before it, one scan collects those items, and the threshold
    // pass plus a filter of the collected keys give the probed set; a batch
    // in which some query collected fewer than Tq (or more than kcap) items
    // is probed again with the two exact passes.
    const int32_t sguess = g_scan_guess;
    const int gstride = (int)std::max<int64_t>(1, std::min<int64_t>(64, sh.Tq / 1600));
    const bool collect = !table && sguess >= 0 && (sguess > 0 || gstride >= 4) && sh.Tq * 3 < ix->n * 2;
    const int64_t guess16 = sguess > 0 ? sguess : 18;  // guessed items, in sixteenths of Tq
    const int64_t kcap = collect ? 2 * sh.Tq + 16384 : 0;
    if (collect) B = std::min<int64_t>(B, std::max<int64_t>(64, (int64_t(1) << 32) / (kcap * 8) / 64 * 64));
    const int64_t tiles = B / 64;
    const int L1 = sh.L + 1;
    const int nsplit = rerank_splits(B, sh.Tq);
    // with the collecting scan each batch is processed in order of its
    // queries' guessed cuts (tiles of alike cuts scan and screen fewer
    // chunks); the results go back to the batch's rows at the end
    const bool sortq = collect && !cand_out_d;
    int sort_bits = 1;
    while ((int64_t(1) << sort_bits) <= (int64_t)sh.m * L1) ++sort_bits;
    // dense head of the bfloat16 re-rank (collecting scan only; not when the
    // probed lists themselves are the output): dense_head -1 = none, 0 = the
    // sub-datasets with at least 3/128 of their items probed, g = at least
    // g / 256; chosen on the call's first batch
    const int32_t dh = g_dense_head;
    const bool head_ok = collect && bf16_rows && !cand_out_d && dh >= 0 && screen_fits(ix, SCREEN_BF16);
    const double head_frac = (dh > 0 ? dh : 6) / 256.0;
    bool head_decided = false, head_any = false;
    int head_lp_split = 1;  // slices per query of the gather beside the head
    std::pair<int, int> hr{0, 0};
    int nhcells = 0, nhchunks = 0;
    Block hblk;
    // the screen's kept pairs join the gather's in the exact re-rank's lists
    const int64_t lcap = std::min<int64_t>(sh.Tq, head_ok ? 8192 : 4096);
    const int lsplit = rerank_splits(B, lcap);
    const int64_t nbatches = (nq + B - 1) / B;
    // both scan passes walk the chunks of the staged pass 1; the sample pass
    // one chunk per sub-dataset (appended after them)
    ScanStages st = table ? ScanStages{} : scan_stages(ix, tiles);
    const int nstage_chunks = table ? 0 : st.cbeg.back();
    if (collect)
        for (int j = 0; j < sh.m; ++j) {
            st.chunks.push_back(j);
            st.chunks.push_back((int32_t)ix->off_h[j]);
            st.chunks.push_back((int32_t)ix->off_h[j + 1]);
        }
    Block blk;
    const size_t o_qc = blk.reserve<uint32_t>(qcodes_out_d ? 1 : (size_t)B * sh.qsets * sh.W),
                 o_gh = blk.reserve<uint32_t>(table ? 1 : (size_t)tiles * sh.m * L1 * 64),
                 o_sc = blk.reserve<int32_t>(std::max<size_t>(1, st.chunks.size())),
                 o_ne = blk.reserve<int32_t>((size_t)tiles),
                 o_gb = blk.reserve<int32_t>((size_t)tiles * (sh.m + 1) * 64),
                 o_th = blk.reserve<int32_t>((size_t)tiles * sh.m * 64),
                 o_ti = blk.reserve<int32_t>((size_t)tiles * 4 * 64),
                 o_ca = blk.reserve<int32_t>(cand_out_d ? 1 : (size_t)B * sh.Tq),
                 o_qs = blk.reserve<int32_t>(table ? (size_t)B * sh.m : 1),
                 o_qhi = blk.reserve<int32_t>(table ? (size_t)B * sh.m * L1 : 1),
                 o_tc = blk.reserve<uint8_t>(table ? table_counter_bytes() : 1),
                 o_pv = blk.reserve<double>(nsplit > 1 && !cand_out_d ? (size_t)B * nsplit * k : 1),
                 o_pi = blk.reserve<int32_t>(nsplit > 1 && !cand_out_d ? (size_t)B * nsplit * k : 1),
                 o_lc = blk.reserve<int32_t>(bf16_rows ? (size_t)B : 1),
                 o_gt = blk.reserve<unsigned long long>((size_t)B),
                 o_ps = blk.reserve<int32_t>((size_t)B),
                 o_ct = blk.reserve<int32_t>(table ? 1 : (size_t)B),
                 o_li = blk.reserve<int32_t>(bf16_rows ? (size_t)B * lcap : 1),
                 o_lv = blk.reserve<double>(bf16_rows && lsplit > 1 ? (size_t)B * lsplit * k : 1),
                 o_lp = blk.reserve<int32_t>(bf16_rows && lsplit > 1 ? (size_t)B * lsplit * k : 1),
                 o_ky = blk.reserve<uint64_t>(collect ? (size_t)B * kcap : 1),
                 o_kc = blk.reserve<int32_t>(collect ? (size_t)B : 1),
                 o_rh = blk.reserve<int32_t>(collect ? (size_t)B : 1),
                 o_tg = blk.reserve<int32_t>(collect ? (size_t)tiles * 4 * 64 : 1),
                 o_fl = blk.reserve<uint32_t>(collect ? (size_t)nbatches : 1),
                 o_sh = blk.reserve<unsigned long long>(head_ok ? (size_t)sh.m * sub_hits_slices(B) : 1),
                 o_ska = blk.reserve<uint64_t>(sortq ? (size_t)B : 1), o_skb = blk.reserve<uint64_t>(sortq ? (size_t)B : 1),
                 o_sva = blk.reserve<int32_t>(sortq ? (size_t)B : 1), o_svb = blk.reserve<int32_t>(sortq ? (size_t)B : 1),
                 o_stm = blk.reserve<uint8_t>(sortq ? radix_sort_tmp_bytes(B) : 1),
                 o_sqp = blk.reserve<float>(sortq ? (size_t)B * sh.d : 1),
                 o_sqc = blk.reserve<uint32_t>(sortq ? (size_t)B * sh.qsets * sh.W : 1),
                 o_srh = blk.reserve<int32_t>(sortq ? (size_t)B : 1),
                 o_sid = blk.reserve<int64_t>(sortq ? (size_t)B * k : 1),
                 o_sip = blk.reserve<float>(sortq ? (size_t)B * k : 1),
                 o_lst = blk.reserve<unsigned long long>(4);
    blk.allocate(s);
    DBuf<uint64_t> keys = blk.view<uint64_t>(o_ky);
    DBuf<int32_t> kcount = blk.view<int32_t>(o_kc), grho = blk.view<int32_t>(o_rh), gtie_g = blk.view<int32_t>(o_tg);
    DBuf<uint32_t> gfail = blk.view<uint32_t>(o_fl);
    if (collect) HIPX(launch_fill32(gfail.get(), nbatches, 0u, s));
    DBuf<unsigned long long> subhits = blk.view<unsigned long long>(o_sh);
    DBuf<uint64_t> ska = blk.view<uint64_t>(o_ska), skb = blk.view<uint64_t>(o_skb);
    DBuf<int32_t> sva = blk.view<int32_t>(o_sva), svb = blk.view<int32_t>(o_svb), srho = blk.view<int32_t>(o_srh);
    DBuf<uint8_t> stmp = blk.view<uint8_t>(o_stm);
    DBuf<float> sQ = blk.view<float>(o_sqp), sips = blk.view<float>(o_sip);
    DBuf<uint32_t> sqc = blk.view<uint32_t>(o_sqc);
    DBuf<int64_t> sids = blk.view<int64_t>(o_sid);
    // kept-list totals of the batches whose check is left to the device
    DBuf<unsigned long long> lstats = blk.view<unsigned long long>(o_lst);
    // (word 3: the (query, item) pairs the dense head's keep pass evaluates)
    if (collect && bf16_rows) HIPX(hipMemsetAsync(lstats.get(), 0, 4 * sizeof(unsigned long long), s));
    DBuf<uint32_t> qcodes = blk.view<uint32_t>(o_qc), ghist = blk.view<uint32_t>(o_gh);
    DBuf<int32_t> gbase = blk.view<int32_t>(o_gb), ghthr = blk.view<int32_t>(o_th),
                  gtie = blk.view<int32_t>(o_ti), cand = blk.view<int32_t>(o_ca);
    DBuf<double> part_v = blk.view<double>(o_pv);
    DBuf<int32_t> part_i = blk.view<int32_t>(o_pi);
    DBuf<int32_t> lcount = blk.view<int32_t>(o_lc), lists = blk.view<int32_t>(o_li);
    DBuf<unsigned long long> gtheta = blk.view<unsigned long long>(o_gt);
    DBuf<int32_t> gpstar = blk.view<int32_t>(o_ps), ccount = blk.view<int32_t>(o_ct);
    DBuf<double> lpart_v = blk.view<double>(o_lv);
    DBuf<int32_t> lpart_i = blk.view<int32_t>(o_lp);
    DBuf<int32_t> qstate = blk.view<int32_t>(o_qs), qhist = blk.view<int32_t>(o_qhi);
    DBuf<uint8_t> tctr = blk.view<uint8_t>(o_tc);
    DBuf<int32_t> schunks = blk.view<int32_t>(o_sc), need = blk.view<int32_t>(o_ne);
    if (!table)
        HIPX(hipMemcpyAsync(schunks.get(), st.chunks.data(), st.chunks.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, s));
    const TableView tv{ix->ucode.get(), ix->ustart.get(), ix->uoff.get(), ix->titem.get(), ix->binom.get()};
    if (table) HIPX(hipMemsetAsync(tctr.get(), 0, table_counter_bytes(), s));
    std::vector<int32_t> hl(bf16_rows ? (size_t)B : 0), hg(head_ok ? (size_t)B : 0);
    // once a batch's bfloat16 lists overflow (the bound keeps too many items
    // for this data and k), later batches of the call go straight to the
    // FP32 rows instead of paying for both passes
    bool lp_on = bf16_rows;
    const uint64_t ovf = ix->lp_overflow.load(std::memory_order_relaxed);
    if (ovf != 0 && (uint64_t)k >= (ovf >> 32) && (uint64_t)sh.Tq >= (ovf & 0xFFFFFFFFull)) lp_on = false;
    DBuf<uint16_t> hqh;
    DBuf<float> hqn, htheta, hcmax;
    DBuf<int32_t> hcells, hchunks, hpw;
    // Chooses the head from the sample pass of the batch just guessed (one
    // host round trip per call) and sets up its buffers.
    auto decide_head = [&](int64_t nb) {
        head_decided = true;
        bool cached = false;
        {
            std::lock_guard<std::mutex> g(ix->head_mu);
            if (ix->head_hint_valid && ix->head_hint_k == k && ix->head_hint_T == sh.Tq &&
                ix->head_hint_frac == head_frac) {
                hr = {ix->head_hint_j0, ix->head_hint_j1};
                head_lp_split = ix->head_hint_split;
                cached = true;
            }
        }
        if (!cached) {
            HIPX(launch_sub_hits(ghist.get(), ix->R.get(), grho.get(), nb, sh.m, sh.L, subhits.get(), s));
            const int ns = sub_hits_slices(nb);
            const size_t words = (size_t)sh.m * ns;
            size_t pb = 0;
            auto *part = static_cast<unsigned long long *>(pinned_take(words * sizeof(unsigned long long), &pb));
            HIPX(hipMemcpyAsync(part, subhits.get(), words * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
            HIPX(hipStreamSynchronize(s));
            std::vector<unsigned long long> hits((size_t)sh.m, 0ull);
            for (int j = 0; j < sh.m; ++j)
                for (int t = 0; t < ns; ++t) hits[(size_t)j] += part[(size_t)j * ns + t];
            pinned_give(part, pb, s, ix->device);
            hr = dense_head_range(ix, hits.data(), nb, gstride, head_frac);
            if (hr.second > hr.first) {
                // the probed items left to the gather, per query (the sample
                // counts items ranked before the guess, guess16 / 16 Tq of them):
                // slices of about 320 items keep the machine busy on these short
                // lists (large workload, 4,984 items per query: 1.05 ms per call
                // in 2 slices, 0.71 in 16)
                double rest = 0.0;
                for (int j = 0; j < sh.m; ++j)
                    if (j < hr.first || j >= hr.second) rest += (double)hits[(size_t)j];
                rest *= (double)gstride / (double)nb * 16.0 / (double)guess16;
                head_lp_split = (int)std::min<double>(16.0, std::max<double>(1.0, std::ceil(rest / 320.0)));
            }
            std::lock_guard<std::mutex> g(ix->head_mu);
            ix->head_hint_valid = true;
            ix->head_hint_k = k;
            ix->head_hint_T = sh.Tq;
            ix->head_hint_frac = head_frac;
            ix->head_hint_j0 = hr.first;
            ix->head_hint_j1 = hr.second;
            ix->head_hint_split = head_lp_split;
        }
        head_any = hr.second > hr.first;
        if (!head_any) return;
        // theta_q comes from witnesses in every sub-dataset of the head (a
        // sub-dataset normalised by an outlying U_j hashes almost all of its
        // items alike, so that a query probes nearly all of them or nearly
        // none, and no single sub-dataset holds k probed items for every
        // query): each one's largest-norm items, which set the k-th best
        // lower bound, screened from their compact copy.  (The screen path's
        // norm bound skips nothing here: theta_q stays far below ||q|| U_j.)
        witness_rows(ix, s);
        std::vector<int> hjs;
        for (int j = hr.second - 1; j >= hr.first; --j) hjs.push_back(j);
        std::vector<int32_t> hce;
        const int Wp = ix->wit_per_sub;
        for (const int j : hjs)
            for (int c0 = 0; c0 < ix->wit_cnt_h[(size_t)j]; c0 += screen_cell_items()) {
                hce.push_back(j);
                hce.push_back(j * Wp + c0);
                hce.push_back(j * Wp + std::min(c0 + screen_cell_items(), ix->wit_cnt_h[(size_t)j]));
            }
        const std::vector<int32_t> hch = subset_chunks(ix, screen_chunk_items(), hjs);
        nhcells = (int)(hce.size() / 3);
        nhchunks = (int)(hch.size() / 3);
        const size_t o_hq = hblk.reserve<uint16_t>((size_t)B * sh.dp), o_hn = hblk.reserve<float>((size_t)B),
                     o_ht = hblk.reserve<float>((size_t)B),
                     o_hm = hblk.reserve<float>((size_t)B * nhcells * screen_cell_groups()),
                     o_hc = hblk.reserve<int32_t>(std::max<size_t>(1, hce.size())),
                     o_hk = hblk.reserve<int32_t>(hch.size()), o_hp = hblk.reserve<int32_t>((size_t)B);
        hblk.allocate(s);
        hpw = hblk.view<int32_t>(o_hp);
        hqh = hblk.view<uint16_t>(o_hq);
        hqn = hblk.view<float>(o_hn);
        htheta = hblk.view<float>(o_ht);
        hcmax = hblk.view<float>(o_hm);
        hcells = hblk.view<int32_t>(o_hc);
        hchunks = hblk.view<int32_t>(o_hk);
        HIPX(hipMemcpyAsync(hcells.get(), hce.data(), hce.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIPX(hipMemcpyAsync(hchunks.get(), hch.data(), hch.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    };
    // one batch; returns false when it has to run again without the dense
    // head (its lists overflowed)
    // defer: the collecting path's batches leave the kept lists' overflow
    // check to the device (a failure bit read once at the end of the call)
    auto run_batch = [&](int64_t b0, int64_t bi, bool staged, bool head, bool defer) -> bool {
        bool hd = head && head_ok && !staged && lp_on;
        int jh0 = 0, jh1 = 0;
        const int64_t nb = std::min<int64_t>(B, nq - b0);
        const float *Qb = Qd + b0 * sh.d;
        uint32_t *qc = qcodes_out_d ? qcodes_out_d + b0 * sh.qsets * sh.W : qcodes.get();
        int32_t *cb = cand_out_d ? cand_out_d + b0 * sh.Tq : cand.get();
        // the batch as the steps after the guess take it: its own order, or
        // sorted by guessed cut (qord: sorted row -> batch row)
        const float *Qx = Qb;
        uint32_t *qx = qc;
        int32_t *rx = grho.get(), *qord = nullptr;
        int64_t *ox_ids = ids_d + b0 * k;
        float *ox_ips = ips_d + b0 * k;
        tm.begin("qhash");
        HIPX(launch_query_hash(Qb, nb, sh.d, ix->At.get(), sh.L, sh.W, sh.qsets, qc, nonfinite_d, s));
        tm.end();
        if (table) {
            HIPX(hipMemsetAsync(qstate.get(), 0, (size_t)nb * sh.m * sizeof(int32_t), s));
            tm.begin("table_count");
            HIPX(launch_table_count(tv, ix->R.get(), ix->inv.get(), qc, nb, sh, qstate.get(), qhist.get(),
                                    ghthr.get(), gtie.get(), tctr.get(), s));
            tm.end();
            tm.begin("tie_locate");
            HIPX(launch_tie_locate(ix->codes_l.get(), ix->off.get(), qc, nb, sh.W, sh.qsets, gtie.get(),
                                   gpstar.get(), s));
            tm.end();
            tm.begin("table_emit");
            HIPX(launch_table_emit(tv, qc, nb, sh, qstate.get(), ghthr.get(), gtie.get(), gpstar.get(),
                                   cb, s));
            tm.end();
        }
        if (!table && collect && !staged) {
            const int64_t tb = (nb + 63) / 64;
            const int32_t P = sh.m * L1;
            QueryShape shg = sh;  // the guess (1.125 Tq items by default), in sample units
            shg.Tq = std::max<int64_t>(1, (sh.Tq * guess16 / 16 + gstride - 1) / gstride);
            HIPX(launch_fill32(ghist.get(), tb * sh.m * L1 * 64, 0u, s));
            tm.begin("scan_sample");
            HIPX(launch_scan_hist_stage(ix->codes_l.get(), qc, nb, sh, schunks.get() + 3 * (size_t)nstage_chunks, sh.m,
                                        nullptr, ghist.get(), nullptr, s, gstride));
            tm.end();
            tm.begin("guess");
            HIPX(launch_threshold(ghist.get(), ix->R.get(), ix->inv.get(), nb, shg, gbase.get(), ghthr.get(),
                                  gtie_g.get(), s, false));
            HIPX(launch_rho_from_tie(gtie_g.get(), nb, P, grho.get(), s));
            tm.end();
            if (hd && !head_decided) decide_head(nb);
            hd = hd && head_any;
            if (hd) {
                jh0 = hr.first;
                jh1 = hr.second;
            }
            if (sortq) {
                tm.begin("order");
                HIPX(launch_rho_order(grho.get(), nb, sort_bits, ska.get(), sva.get(), skb.get(), svb.get(),
                                      stmp.get(), &qord, s));
                HIPX(launch_permute_batch(Qb, qc, grho.get(), qord, nb, sh.d, sh.qsets * sh.W, sQ.get(), sqc.get(),
                                          srho.get(), s));
                tm.end();
                Qx = sQ.get();
                qx = sqc.get();
                rx = srho.get();
                ox_ids = sids.get();
                ox_ips = sips.get();
            }
            HIPX(launch_fill32(ghist.get(), tb * sh.m * L1 * 64, 0u, s));
            HIPX(launch_fill32(kcount.get(), nb, 0u, s));
            tm.begin("scan_collect");
            HIPX(launch_scan_collect(ix->codes_l.get(), qx, nb, sh, schunks.get(), nstage_chunks, ix->R.get(),
                                     rx, kcap, kcount.get(), keys.get(), ghist.get(), scan_pairs_d, s, jh0, jh1));
            tm.end();
            // (the dense head's screen reads every sub-dataset's level bound)
            tm.begin("threshold");
            HIPX(launch_threshold(ghist.get(), ix->R.get(), ix->inv.get(), nb, sh, gbase.get(), ghthr.get(),
                                  gtie.get(), s, hd, false));
            tm.end();
            tm.begin("tie_locate");
            HIPX(launch_tie_locate(ix->codes_l.get(), ix->off.get(), qx, nb, sh.W, sh.qsets, gtie.get(),
                                   gpstar.get(), s, ghist.get(), sh.m, sh.L));
            tm.end();
            tm.begin("filter");
            HIPX(launch_collect_filter(keys.get(), kcount.get(), kcap, nb, gtie.get(), gpstar.get(), rx, sh.Tq, cb,
                                       ccount.get(), gfail.get() + bi, s));
            tm.end();
        } else if (!table) {
            tm.begin("scan_hist");
            run_scan_hist_staged(ix, sh, qc, nb, st.cbeg, st.cut, schunks.get(), need.get(), ghist.get(),
                                 scan_pairs_d, s);
            tm.end();
            tm.begin("threshold");
            HIPX(launch_threshold(ghist.get(), ix->R.get(), ix->inv.get(), nb, sh, gbase.get(),
                                  ghthr.get(), gtie.get(), s));
            tm.end();
            tm.begin("tie_locate");
            HIPX(launch_tie_locate(ix->codes_l.get(), ix->off.get(), qc, nb, sh.W, sh.qsets, gtie.get(),
                                   gpstar.get(), s));
            tm.end();
            HIPX(hipMemsetAsync(ccount.get(), 0, (size_t)nb * sizeof(int32_t), s));
            tm.begin("scan_emit");
            HIPX(launch_scan_emit_stage(ix->codes_l.get(), qc, nb, sh, schunks.get(), nstage_chunks,
                                        ghthr.get(), gtie.get(), gpstar.get(), ccount.get(), cb, s));
            tm.end();
        }
        if (cand_out_d) return true;
        if (lp_on) {
            HIPX(hipMemsetAsync(lcount.get(), 0, (size_t)nb * sizeof(int32_t), s));
            if (hd) {
                // the head sub-datasets: theta_q from the largest lower bounds of
                // their 32-item groups, then every probed pair of them that may
                // reach it into the lists; theta_q seeds the gather below, which
                // takes the other sub-datasets' probed items (the filter left the
                // head's out)
                ScreenQueries sq{Qx, hqh.get(), nullptr, hqn.get(), nullptr, nullptr};
                tm.begin("head_theta");
                HIPX(launch_query_bf16(Qx, nb, sh.d, sh.dp, hqh.get(), nullptr, hqn.get(), s, nonfinite_d));
                HIPX(launch_wit_pstar(gtie.get(), gpstar.get(), ix->wit_pos.get(), ix->wit_cnt.get(),
                                      ix->wit_per_sub, nb, hpw.get(), s));
                HIPX(launch_screen_max(ix->Xl.get(), ix->wit_xh.get(), nullptr, ix->wit_key.get(),
                                       ix->wit_codes.get(), sq, nb, sh, hcells.get(), nhcells, nhcells, qx,
                                       ghthr.get(), gtie.get(), hpw.get(), hcmax.get(), htheta.get(), s));
                tm.end();
                sq.pairs = lstats.get() + 3;
                tm.begin("head_screen");
                HIPX(launch_screen(ix->Xl.get(), ix->Xh.get(), nullptr, ix->key_l.get(), ix->codes_l.get(), sq, nb,
                                   sh, hchunks.get(), nhchunks, qx, ghthr.get(), gtie.get(), gpstar.get(),
                                   htheta.get(), (int)lcap, lcount.get(), lists.get(), s));
                tm.end();
                HIPX(launch_theta_seed(htheta.get(), nb, gtheta.get(), s));
            } else {
                HIPX(hipMemsetAsync(gtheta.get(), 0, (size_t)nb * sizeof(unsigned long long), s));
            }
            tm.begin("rerank_lp");
            HIPX(launch_rerank_lp(ix->Xh.get(), ix->xeb.get(), Qx, nb, sh, cb,
                                  hd ? ccount.get() : nullptr, hd ? head_lp_split : nsplit, (int)lcap,
                                  lcount.get(), lists.get(),
                                  gtheta.get(), s));
            tm.end();
            if (defer && collect && !staged) {
                // the exact re-rank reads at most lcap entries per list; a batch
                // with a longer list is run again at the end of the call
                HIPX(launch_list_check(lcount.get(), hd ? ccount.get() : nullptr, nb, (int)lcap, sh.Tq, lstats.get(),
                                       gfail.get() + bi, s));
                QueryShape shl = sh;
                shl.Tq = lcap;  // list stride; lengths come from lcount
                // kept lists are short (hundreds of items): with 2048 queries or
                // more one wave per query fills the machine, and no merge runs
                const int ns = nb >= 2048 ? 1 : std::min(rerank_splits(nb, lcap), lsplit);
                tm.begin("rerank_exact");
                HIPX(launch_rerank(ix->Xl.get(), ix->perm.get(), Qx, nb, shl, lists.get(), lcount.get(), ns,
                                   lpart_v.get(), lpart_i.get(), ox_ids, ox_ips, s));
                tm.end();
                if (qord)
                    HIPX(launch_unpermute_results(qord, nb, k, ox_ids, ox_ips, ids_d + b0 * k, ips_d + b0 * k, s));
                if (hd) g_qstats.dense_head_items = ix->off_h[(size_t)jh1] - ix->off_h[(size_t)jh0];
                return true;
            }
            HIPX(hipMemcpyAsync(hl.data(), lcount.get(), (size_t)nb * sizeof(int32_t),
                                hipMemcpyDeviceToHost, s));
            if (hd)
                HIPX(hipMemcpyAsync(hg.data(), ccount.get(), (size_t)nb * sizeof(int32_t), hipMemcpyDeviceToHost,
                                    s));
            HIPX(hipStreamSynchronize(s));
            int64_t mx = 0, tot = 0, gathered = hd ? 0 : nb * sh.Tq;
            for (int64_t i = 0; i < nb; ++i) {
                mx = std::max<int64_t>(mx, hl[i]);
                tot += hl[i];
                if (hd) gathered += hg[i];
            }
            if (mx <= lcap) {
                g_qstats.lp_kept_total += tot;
                g_qstats.lp_gathered_total += gathered;
                g_qstats.lp_kept_max = std::max<int64_t>(g_qstats.lp_kept_max, mx);
                QueryShape shl = sh;
                shl.Tq = lcap;  // list stride; lengths come from lcount
                const int ns = nb >= 2048 ? 1 : std::min(rerank_splits(nb, lcap), lsplit);
                tm.begin("rerank_exact");
                HIPX(launch_rerank(ix->Xl.get(), ix->perm.get(), Qx, nb, shl, lists.get(),
                                   lcount.get(), ns, lpart_v.get(), lpart_i.get(), ox_ids, ox_ips, s));
                tm.end();
                if (qord)
                    HIPX(launch_unpermute_results(qord, nb, k, ox_ids, ox_ips, ids_d + b0 * k, ips_d + b0 * k, s));
                if (hd) g_qstats.dense_head_items = ix->off_h[(size_t)jh1] - ix->off_h[(size_t)jh0];
                return true;
            }
            g_qstats.lp_fallbacks += 1;  // a list overflowed: re-rank this batch from FP32 rows
            lp_on = false;
            ix->lp_overflow.store(((uint64_t)k << 32) | (uint64_t)sh.Tq, std::memory_order_relaxed);
            // without the head's items in the probed lists the batch runs again
            if (hd) return false;
        }
        if (nsplit > 1) HIPX(hipMemsetAsync(gtheta.get(), 0, (size_t)nb * sizeof(unsigned long long), s));
        tm.begin("rerank");
        HIPX(launch_rerank(ix->Xl.get(), ix->perm.get(), Qx, nb, sh, cb, nullptr, nsplit, part_v.get(),
                           part_i.get(), ox_ids, ox_ips, s, gtheta.get()));
        tm.end();
        if (qord) HIPX(launch_unpermute_results(qord, nb, k, ox_ids, ox_ips, ids_d + b0 * k, ips_d + b0 * k, s));
        return true;
    };
    for (int64_t b0 = 0, bi = 0; b0 < nq; b0 += B, ++bi)
        if (!run_batch(b0, bi, false, true, true)) run_batch(b0, bi, false, false, false);
    if (collect) {
        // batches whose collection was incomplete (bit 1) are probed again with
        // the two passes; batches whose kept lists overflowed (bit 2) run
        // again without them, from the FP32 rows
        std::vector<uint32_t> fl((size_t)nbatches);
        unsigned long long ls[4] = {0, 0, 0, 0};
        HIPX(hipMemcpyAsync(fl.data(), gfail.get(), fl.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        if (bf16_rows) HIPX(hipMemcpyAsync(ls, lstats.get(), sizeof ls, hipMemcpyDeviceToHost, s));
        HIPX(hipStreamSynchronize(s));
        g_qstats.lp_kept_total += (int64_t)ls[0];
        g_qstats.lp_kept_max = std::max<int64_t>(g_qstats.lp_kept_max, (int64_t)ls[1]);
        g_qstats.lp_gathered_total += (int64_t)ls[2];
        g_qstats.dense_head_pairs += (int64_t)ls[3];
        for (int64_t bi = 0; bi < nbatches; ++bi) {
            const uint32_t f = fl[(size_t)bi];
            if (f & 1u) {
                g_qstats.collect_fallbacks += 1;
                run_batch(bi * B, bi, true, false, false);
            } else if (f & 2u) {
                g_qstats.lp_fallbacks += 1;
                lp_on = false;
                ix->lp_overflow.store(((uint64_t)k << 32) | (uint64_t)sh.Tq, std::memory_order_relaxed);
                run_batch(bi * B, bi, false, false, false);
            }
        }
    }
    if (table) {
        unsigned long long c[3] = {0, 0, 0};
        HIPX(hipMemcpyAsync(c, tctr.get(), sizeof c, hipMemcpyDeviceToHost, s));
        HIPX(hipStreamSynchronize(s));
        g_qstats.table_lookups = (int64_t)c[0];
        g_qstats.table_walked = (int64_t)c[1];
        g_qstats.table_passes = (int64_t)c[2];
    }
}

// Multi-table single probe: every table's bucket of the query's own code in
// each sub-dataset, tables in order until the budget (the passes of
// k_single.hip around the threshold walk of the multi-probe path, on the
// (sub-dataset, first table) bins), then the exact re-rank of the probed
// lists, which may be shorter than min(T, n).  When cand_out_d is given the
// probed stored positions go there (nq x Tq, count_out_d per query) and the
// re-rank is skipped.
void run_query_single(const nrlsh_index *ix, const float *Qd, int64_t nq, int32_t k, int64_t T, int64_t *ids_d,
                      float *ips_d, int32_t *cand_out_d, int32_t *count_out_d, hipStream_t s, Timer &tm,
                      uint32_t *nonfinite_d)
{
    const QueryShape sh = make_shape(ix, T, k);
    const int t = ix->tables, P = ix->qsets, L1 = t;
    QueryShape shs = sh;  // the bins' shape: levels f = 0 .. t - 1
    shs.L = t - 1;
    int64_t B = (int64_t(1) << 29) / sh.Tq;
    B = std::max<int64_t>(64, B / 64 * 64);
    B = std::min<int64_t>(B, (nq + 63) / 64 * 64);
    const int64_t tiles = B / 64;
    const int nsplit = rerank_splits(B, sh.Tq);
    const ScanStages st = scan_stages(ix, tiles);
    const int nchunks = st.cbeg.back();
    Block blk;
    const size_t o_qc = blk.reserve<uint32_t>((size_t)t * B * P * sh.W),
                 o_gh = blk.reserve<uint32_t>((size_t)tiles * sh.m * L1 * 64),
                 o_sc = blk.reserve<int32_t>(std::max<size_t>(1, st.chunks.size())),
                 o_gb = blk.reserve<int32_t>((size_t)tiles * (sh.m + 1) * 64),
                 o_th = blk.reserve<int32_t>((size_t)tiles * sh.m * 64),
                 o_ti = blk.reserve<int32_t>((size_t)tiles * 4 * 64),
                 o_ps = blk.reserve<int32_t>((size_t)B), o_ct = blk.reserve<int32_t>((size_t)B),
                 o_ca = blk.reserve<int32_t>(cand_out_d ? 1 : (size_t)B * sh.Tq),
                 o_pv = blk.reserve<double>(nsplit > 1 && !cand_out_d ? (size_t)B * nsplit * k : 1),
                 o_pi = blk.reserve<int32_t>(nsplit > 1 && !cand_out_d ? (size_t)B * nsplit * k : 1),
                 o_gt = blk.reserve<unsigned long long>((size_t)B);
    blk.allocate(s);
    uint32_t *qc = blk.view<uint32_t>(o_qc).get(), *ghist = blk.view<uint32_t>(o_gh).get();
    int32_t *chunks = blk.view<int32_t>(o_sc).get(), *gbase = blk.view<int32_t>(o_gb).get(),
            *ghthr = blk.view<int32_t>(o_th).get(), *gtie = blk.view<int32_t>(o_ti).get(),
            *gpstar = blk.view<int32_t>(o_ps).get(), *ccount = blk.view<int32_t>(o_ct).get(),
            *cand = blk.view<int32_t>(o_ca).get(), *part_i = blk.view<int32_t>(o_pi).get();
    double *part_v = blk.view<double>(o_pv).get();
    unsigned long long *gtheta = blk.view<unsigned long long>(o_gt).get();
    HIPX(hipMemcpyAsync(chunks, st.chunks.data(), st.chunks.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    const int64_t tstride_at = (int64_t)ix->d * P * sh.L;  // floats of one table's transposed block
    for (int64_t b0 = 0; b0 < nq; b0 += B) {
        const int64_t nb = std::min<int64_t>(B, nq - b0);
        const float *Qb = Qd + b0 * sh.d;
        const int64_t qstride = nb * P;  // query-code rows of one table
        int32_t *cb = cand_out_d ? cand_out_d + b0 * sh.Tq : cand;
        int32_t *cnt = count_out_d ? count_out_d + b0 : ccount;
        tm.begin("qhash");
        for (int tb = 0; tb < t; ++tb)
            HIPX(launch_query_hash(Qb, nb, sh.d, ix->At.get() + tb * tstride_at, sh.L, sh.W, P,
                                   qc + (size_t)tb * qstride * sh.W, nonfinite_d, s));
        tm.end();
        tm.begin("scan_hist");
        HIPX(launch_fill32(ghist, ((nb + 63) / 64) * sh.m * L1 * 64, 0u, s));
        HIPX(launch_mt_hist(ix->codes_l.get(), sh.n, qc, qstride, nb, sh.m, t, P, sh.W, chunks, nchunks, ghist, s));
        tm.end();
        tm.begin("threshold");
        HIPX(launch_threshold(ghist, ix->Rs.get(), ix->invs.get(), nb, shs, gbase, ghthr, gtie, s));
        tm.end();
        tm.begin("tie_locate");
        HIPX(launch_mt_tie(ix->codes_l.get(), sh.n, ix->off.get(), qc, qstride, nb, t, P, sh.W, gtie, gpstar, s));
        tm.end();
        HIPX(launch_fill32(cnt, nb, 0u, s));
        tm.begin("scan_emit");
        HIPX(launch_mt_emit(ix->codes_l.get(), sh.n, qc, qstride, nb, sh.m, t, P, sh.W, sh.Tq, chunks, nchunks, ghthr,
                            gtie, gpstar, cnt, cb, s));
        tm.end();
        if (cand_out_d) continue;
        if (nsplit > 1) HIPX(launch_fill32(gtheta, 2 * nb, 0u, s));
        tm.begin("rerank");
        HIPX(launch_rerank(ix->Xl.get(), ix->perm.get(), Qb, nb, sh, cb, cnt, nsplit, part_v, part_i, ids_d + b0 * k,
                           ips_d + b0 * k, s, gtheta));
        tm.end();
    }
}

// The bfloat16 lo part of the stored rows (x - bf16(x), rounded to
// bfloat16), needed by the bf16x3 screen only: made on the first such query
// (under the index's lock, finished before anyone uses it) and kept.
const uint16_t *lo_rows(const nrlsh_index *ix, hipStream_t s)
{
    if (ix->lo_ready.load(std::memory_order_acquire)) return ix->Xlo.get();
    std::lock_guard<std::mutex> g(ix->lo_mu);
    if (!ix->lo_ready.load(std::memory_order_relaxed)) {
        const size_t count = (size_t)ix->n * ix->dp + 32;  // zeroed 32-value tail pad
        DBuf<uint16_t> lo(count, s);
        HIPX(launch_lo_rows(ix->Xl.get(), ix->Xh.get(), (int64_t)ix->n * ix->dp, lo.get(), s));
        HIPX(hipMemsetAsync(lo.get() + (size_t)ix->n * ix->dp, 0, 32 * sizeof(uint16_t), s));
        HIPX(hipStreamSynchronize(s));
        lo.s = ix->home;  // released with the index, on the library stream
        ix->Xlo = std::move(lo);
        ix->lo_ready.store(true, std::memory_order_release);
    }
    return ix->Xlo.get();
}

bool screen_fits(const nrlsh_index *ix, int kind)
{
    int lim = 0;
    if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, ix->device) != hipSuccess)
        return false;
    return screen_lds_bytes(ix->dp, kind) + 4096 <= (size_t)lim;
}

// Screen path: (1) theta_q from the largest FP32 lower bounds of small cells
// of the highest-norm sub-datasets, (2) query-tiled MFMA screen of the whole
// probed set against theta_q, (3) exact FP64 re-rank of the kept pairs.
// (sub-dataset, first, end) triples of <= `items` stored items covering
// sub-datasets j >= j_lo entirely and, below j_lo, every `stride`-th cell
// (stride 0: none).
std::vector<int32_t> chunk_table(const nrlsh_index *ix, int items, int j_lo, int stride = 0)
{
    std::vector<int32_t> ch;
    for (int j = ix->m - 1; j >= 0; --j) {
        if (j < j_lo && stride == 0) break;
        int64_t c = 0;
        for (int64_t p = ix->off_h[j]; p < ix->off_h[j + 1]; p += items, ++c) {
            if (j < j_lo && (c + j) % stride != 0) continue;
            ch.push_back(j);
            ch.push_back((int32_t)p);
            ch.push_back((int32_t)std::min<int64_t>(p + items, ix->off_h[j + 1]));
        }
    }
    return ch;
}

// Returns the non-finite flag as read with the last batch's record.
uint32_t run_query_screen(const nrlsh_index *ix, const float *Qd, int64_t nq, int32_t k, int64_t T,
                          int kind, int64_t *ids_d, float *ips_d, hipStream_t s, Timer &tm,
                          uint32_t *nonfinite_d, unsigned long long *scan_pairs_d)
{
    const uint16_t *Xh = kind != SCREEN_FP32 ? ix->Xh.get() : nullptr;
    const uint16_t *Xlo = kind == SCREEN_BF16X3 ? lo_rows(ix, s) : nullptr;
    const QueryShape sh = make_shape(ix, T, k);
    int64_t B = std::min<int64_t>((nq + 63) / 64 * 64, 16384);
    const int64_t tiles = B / 64;
    const int L1 = sh.L + 1;
    // kept-list room per query: the k best plus the items within the bounds'
    // reach of the k-th, which grows with k (about 26 k were kept at k = 100 on
    // the large workload); an overflow re-screens the batch with longer lists
    int64_t cap = std::min<int64_t>(sh.Tq, std::max<int64_t>(1024, 32 * (int64_t)k));

    // pass-1 cells: the top sub-datasets whole (at least 16 k lower-bound
    // groups) plus, when the budget leaves items unprobed, every 16th cell of
    // the others, so that the witnesses of theta sit wherever a query's
    // probed items are (a sub-dataset normalised by an outlying U_j can hash
    // almost all of its items alike and be probed late).  When every item is
    // probed the top sub-datasets alone give every query k witnesses, and
    // the highest-norm items are the ones that set theta; pass-2 chunks:
    // every sub-dataset
    const int64_t want = std::max<int64_t>(2, 16 * (int64_t)k / screen_cell_groups());
    int j_lo = ix->m - 1;
    while (j_lo > 0 && (ix->off_h[ix->m] - ix->off_h[j_lo]) / screen_cell_items() < want) --j_lo;
    std::vector<int32_t> ce = chunk_table(ix, screen_cell_items(), j_lo, sh.Tq >= sh.n ? 0 : 16);
    std::vector<int32_t> ch = chunk_table(ix, screen_chunk_items(), 0);
    // (the FP32 screen runs the scan at every budget; the bfloat16 ones skip it
    // when every item is probed)
    const ScanStages st = sh.Tq >= sh.n && kind != SCREEN_FP32 ? ScanStages{} : scan_stages(ix, tiles);
    const int ncells = (int)(ce.size() / 3), nchunks = (int)(ch.size() / 3);
    int ncells_top = 0;  // cells of the whole top sub-datasets come first
    while (ncells_top < ncells && ce[3 * (size_t)ncells_top] >= j_lo) ++ncells_top;
    Block blk;
    const size_t o_ce = blk.reserve<int32_t>(ce.size()), o_ch = blk.reserve<int32_t>(ch.size()),
                 o_qc = blk.reserve<uint32_t>((size_t)B * sh.qsets * sh.W),
                 o_gh = blk.reserve<uint32_t>((size_t)tiles * sh.m * L1 * 64),
                 o_gb = blk.reserve<int32_t>((size_t)tiles * (sh.m + 1) * 64),
                 o_th = blk.reserve<int32_t>((size_t)tiles * sh.m * 64),
                 o_ti = blk.reserve<int32_t>((size_t)tiles * 4 * 64),
                 o_ps = blk.reserve<int32_t>((size_t)B),
                 o_cm = blk.reserve<float>((size_t)B * ncells * screen_cell_groups()),
                 o_qh = blk.reserve<uint16_t>(kind != SCREEN_FP32 ? (size_t)B * sh.dp : 1),
                 o_ql = blk.reserve<uint16_t>(kind == SCREEN_BF16X3 ? (size_t)B * sh.dp : 1),
                 o_qn = blk.reserve<float>(kind != SCREEN_FP32 ? (size_t)B : 1),
                 o_ta = blk.reserve<float>((size_t)B), o_co = blk.reserve<int32_t>((size_t)B),
                 o_li = blk.reserve<int32_t>((size_t)B * cap),
                 o_np = blk.reserve<unsigned long long>(1), o_rec = blk.reserve<long long>(5),
                 o_sc = blk.reserve<int32_t>(std::max<size_t>(1, st.chunks.size())),
                 o_ne = blk.reserve<int32_t>((size_t)tiles),
                 o_oka = blk.reserve<uint64_t>((size_t)B), o_okb = blk.reserve<uint64_t>((size_t)B),
                 o_ova = blk.reserve<int32_t>((size_t)B), o_ovb = blk.reserve<int32_t>((size_t)B),
                 o_otmp = blk.reserve<uint8_t>(radix_sort_tmp_bytes(B));
    blk.allocate(s);
    DBuf<int32_t> cells = blk.view<int32_t>(o_ce), chunks = blk.view<int32_t>(o_ch);
    DBuf<unsigned long long> npairs = blk.view<unsigned long long>(o_np);
    DBuf<long long> rec = blk.view<long long>(o_rec);
    // the per-batch record comes back through pinned memory
    size_t rec_bytes = 0;
    long long *rec_h = static_cast<long long *>(pinned_take(5 * sizeof(long long), &rec_bytes));
    struct RecRelease {
        void *p;
        size_t b;
        hipStream_t s;
        int dev;
        ~RecRelease() { pinned_give(p, b, s, dev); }
    } rec_release{rec_h, rec_bytes, s, ix->device};
    uint32_t bad = 0;
    DBuf<uint64_t> oka = blk.view<uint64_t>(o_oka), okb = blk.view<uint64_t>(o_okb);
    DBuf<int32_t> ova = blk.view<int32_t>(o_ova), ovb = blk.view<int32_t>(o_ovb);
    DBuf<uint8_t> otmp = blk.view<uint8_t>(o_otmp);
    HIPX(hipMemsetAsync(npairs.get(), 0, sizeof(unsigned long long), s));
    HIPX(hipMemcpyAsync(cells.get(), ce.data(), ce.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPX(hipMemcpyAsync(chunks.get(), ch.data(), ch.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    DBuf<int32_t> schunks = blk.view<int32_t>(o_sc), need = blk.view<int32_t>(o_ne);
    if (!st.chunks.empty())
        HIPX(hipMemcpyAsync(schunks.get(), st.chunks.data(), st.chunks.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, s));

    DBuf<uint32_t> qcodes = blk.view<uint32_t>(o_qc), ghist = blk.view<uint32_t>(o_gh);
    DBuf<int32_t> gbase = blk.view<int32_t>(o_gb), ghthr = blk.view<int32_t>(o_th),
                  gtie = blk.view<int32_t>(o_ti), gpstar = blk.view<int32_t>(o_ps);
    DBuf<float> cmax = blk.view<float>(o_cm);
    DBuf<uint16_t> qh = blk.view<uint16_t>(o_qh), ql = blk.view<uint16_t>(o_ql);
    DBuf<float> qn = blk.view<float>(o_qn), theta = blk.view<float>(o_ta);
    DBuf<int32_t> counts = blk.view<int32_t>(o_co), lists = blk.view<int32_t>(o_li);
    for (int64_t b0 = 0; b0 < nq; b0 += B) {
        const int64_t nb = std::min<int64_t>(B, nq - b0);
        const float *Qb = Qd + b0 * sh.d;
        // a budget covering every item probes every bucket whole: no codes,
        // counts or threshold are needed (the bfloat16 image checks finiteness)
        const bool everything = sh.Tq >= sh.n && kind != SCREEN_FP32;
        if (!everything) {
            tm.begin("qhash");
            HIPX(launch_query_hash(Qb, nb, sh.d, ix->At.get(), sh.L, sh.W, sh.qsets, qcodes.get(),
                                   nonfinite_d, s));
            tm.end();
        }
        ScreenQueries sq{Qb, nullptr, nullptr, nullptr, ix->U.get(), npairs.get()};
        if (kind != SCREEN_FP32) {
            sq.Qh = qh.get();
            sq.Ql = kind == SCREEN_BF16X3 ? ql.get() : nullptr;
            sq.qn = qn.get();
            HIPX(launch_query_bf16(Qb, nb, sh.d, sh.dp, qh.get(), kind == SCREEN_BF16X3 ? ql.get() : nullptr,
                                   qn.get(), s, nonfinite_d));
        }
        if (everything) {
            HIPX(launch_probe_all(nb, sh, ghthr.get(), gtie.get(), gpstar.get(), s));
        } else {
            tm.begin("scan_hist");
            run_scan_hist_staged(ix, sh, qcodes.get(), nb, st.cbeg, st.cut, schunks.get(), need.get(),
                                 ghist.get(), scan_pairs_d, s);
            tm.end();
            tm.begin("threshold");
            HIPX(launch_threshold(ghist.get(), ix->R.get(), ix->inv.get(), nb, sh, gbase.get(),
                                  ghthr.get(), gtie.get(), s));
            tm.end();
            tm.begin("tie_locate");
            HIPX(launch_tie_locate(ix->codes_l.get(), ix->off.get(), qcodes.get(), nb, sh.W, sh.qsets,
                                   gtie.get(), gpstar.get(), s));
            tm.end();
        }
        tm.begin("screen_max");
        HIPX(launch_screen_max(ix->Xl.get(), Xh, Xlo, ix->key_l.get(), ix->codes_l.get(), sq, nb, sh,
                               cells.get(), ncells, ncells_top, qcodes.get(), ghthr.get(), gtie.get(),
                               gpstar.get(), cmax.get(), theta.get(), s));
        tm.end();
        if (kind != SCREEN_FP32) {
            // pass B takes the queries in order of theta / ||q||: tiles of
            // alike queries skip more chunks by the norm bound
            int32_t *order = nullptr;
            HIPX(launch_query_order(theta.get(), qn.get(), nb, oka.get(), ova.get(), okb.get(), ovb.get(),
                                    otmp.get(), &order, s));
            sq.order = order;
        }
        // screen, then the exact re-rank of the kept lists right behind it; the
        // host checks afterwards whether a list overflowed (then the batch is
        // screened again with longer lists, which overwrites the results)
        for (bool first = true;; first = false) {
            HIPX(hipMemsetAsync(counts.get(), 0, (size_t)nb * sizeof(int32_t), s));
            tm.begin("screen");
            HIPX(launch_screen(ix->Xl.get(), Xh, Xlo, ix->key_l.get(), ix->codes_l.get(), sq, nb, sh,
                               chunks.get(), nchunks, qcodes.get(), ghthr.get(), gtie.get(),
                               gpstar.get(), theta.get(), (int)cap, counts.get(), lists.get(), s));
            tm.end();
            QueryShape shl = sh;
            shl.Tq = cap;  // list stride; lengths come from counts
            const int nsplit = rerank_splits(nb, cap);
            Block pb;
            const size_t o_pv = pb.reserve<double>(nsplit > 1 ? (size_t)nb * nsplit * k : 1),
                         o_pi = pb.reserve<int32_t>(nsplit > 1 ? (size_t)nb * nsplit * k : 1);
            pb.allocate(s);
            DBuf<double> pv = pb.view<double>(o_pv);
            DBuf<int32_t> pi = pb.view<int32_t>(o_pi);
            tm.begin("rerank_exact");
            HIPX(launch_rerank(ix->Xl.get(), ix->perm.get(), Qb, nb, shl, lists.get(), counts.get(),
                               nsplit, pv.get(), pi.get(), ids_d + b0 * k, ips_d + b0 * k, s));
            tm.end();
            HIPX(launch_list_stats(counts.get(), first ? theta.get() : nullptr, nb, npairs.get(), nonfinite_d,
                                   rec.get(), s));
            HIPX(hipMemcpyAsync(rec_h, rec.get(), 5 * sizeof(long long), hipMemcpyDeviceToHost, s));
            HIPX(hipStreamSynchronize(s));
            const int64_t mx = rec_h[0], tot = rec_h[1];
            if (first) g_qstats.theta_unset += rec_h[2];
            g_qstats.screen_pairs = rec_h[3];
            bad = rec_h[4] != 0;
            g_qstats.screen_passes += 1;
            if (mx <= cap) {
                g_qstats.kept_total += tot;
                g_qstats.kept_max = std::max<int64_t>(g_qstats.kept_max, mx);
                break;
            }
            // a list overflowed: grow the lists and screen this batch again
            cap = std::min<int64_t>(sh.Tq, std::max<int64_t>(mx, 2 * cap));
            lists = DBuf<int32_t>((size_t)B * cap, s);
        }
    }
    return bad;
}

// Returns the non-finite flag when the path has already read it back after
// its last device work (the screen), else kFlagUnread.
constexpr uint32_t kFlagUnread = 0xFFFFFFFFu;
uint32_t run_query(const nrlsh_index *ix, const float *Qd, int64_t nq, int32_t k, int64_t T, int mode,
                   bool bf16_rows, int probe, int64_t *ids_d, float *ips_d, hipStream_t s, Timer &tm,
                   uint32_t *nonfinite_d, unsigned long long *scan_pairs_d)
{
    const int64_t Tq = std::min<int64_t>(T, ix->n);
    const bool table = probe == NRLSH_PROBE_TABLE;
    g_qstats.probe_mode = probe;
    if (probe == NRLSH_PROBE_SINGLE) {
        g_qstats.mode = NRLSH_RERANK_GATHER;
        run_query_single(ix, Qd, nq, k, T, ids_d, ips_d, nullptr, nullptr, s, tm, nonfinite_d);
        return kFlagUnread;
    }
    bool screen = !table && (mode == NRLSH_RERANK_SCREEN || mode == NRLSH_RERANK_SCREEN_FP32 ||
                             mode == NRLSH_RERANK_SCREEN_BF16X3 ||
                             (mode == NRLSH_RERANK_AUTO && Tq * 128 >= ix->n && nq >= 64 && Tq >= 2048));
    const int kind = mode == NRLSH_RERANK_SCREEN_FP32     ? SCREEN_FP32
                     : mode == NRLSH_RERANK_SCREEN_BF16X3 ? SCREEN_BF16X3
                                                          : SCREEN_BF16;
    if (screen && !screen_fits(ix, kind)) screen = false;
    g_qstats.mode = !screen                ? NRLSH_RERANK_GATHER
                    : kind == SCREEN_FP32   ? NRLSH_RERANK_SCREEN_FP32
                    : kind == SCREEN_BF16X3 ? NRLSH_RERANK_SCREEN_BF16X3
                                            : NRLSH_RERANK_SCREEN;
    if (screen) return run_query_screen(ix, Qd, nq, k, T, kind, ids_d, ips_d, s, tm, nonfinite_d, scan_pairs_d);
    run_query_gather(ix, Qd, nq, k, T, ids_d, ips_d, nullptr, nullptr, s, tm, nonfinite_d, bf16_rows, table,
                     scan_pairs_d);
    return kFlagUnread;
}

// ================================================================= query without allocation
// Device scratch of nrlsh_query_noalloc: a file-scope array that the code
// object holds on every device it is loaded on, until the process ends.
// Host code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address): hipGetSymbolAddress gives each device its
// own copy's address once, with that device current, and only that address
// is used.  Every call on one device shares that device's copy, so calls
// that overlap on one device race; what must start at zero is cleared by a
// fill kernel at the start of each batch.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[kScratchDevices] = {};

// The calling thread's current device must be `dev`.
uint8_t *scratch_base(int dev)
{
    if (dev < 0 || dev >= kScratchDevices) throw Failure{NRLSH_E_INVALID_ARG, "device id out of range"};
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPX(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Failure{NRLSH_E_DEVICE, "no address for the device scratch"};
        g_scratch_ptr[dev] = static_cast<uint8_t *>(p);
    }
    return g_scratch_ptr[dev];
}

// Buffers of one batch of B queries of the gather path, laid out in order.
struct NoAllocLayout {
    Block blk;
    size_t qc, gh, ne, gb, th, ti, ca, pv, pi, gt, ps, ct;
};

void layout_noalloc(NoAllocLayout &a, const QueryShape &sh, int64_t B, int nsplit)
{
    const int64_t tiles = B / 64;
    const int L1 = sh.L + 1;
    Block &b = a.blk;
    a.qc = b.reserve<uint32_t>((size_t)B * sh.qsets * sh.W);
    a.gh = b.reserve<uint32_t>((size_t)tiles * sh.m * L1 * 64);
    a.ne = b.reserve<int32_t>((size_t)tiles);
    a.gb = b.reserve<int32_t>((size_t)tiles * (sh.m + 1) * 64);
    a.th = b.reserve<int32_t>((size_t)tiles * sh.m * 64);
    a.ti = b.reserve<int32_t>((size_t)tiles * 4 * 64);
    a.ca = b.reserve<int32_t>((size_t)B * sh.Tq);
    a.pv = b.reserve<double>(nsplit > 1 ? (size_t)B * nsplit * sh.k : 1);
    a.pi = b.reserve<int32_t>(nsplit > 1 ? (size_t)B * nsplit * sh.k : 1);
    a.gt = b.reserve<unsigned long long>((size_t)B);
    a.ps = b.reserve<int32_t>((size_t)B);
    a.ct = b.reserve<int32_t>((size_t)B);
}

// Scratch bytes of a batch of B queries.
size_t noalloc_bytes(const QueryShape &sh, int64_t B)
{
    NoAllocLayout a;
    layout_noalloc(a, sh, B, rerank_splits(B, sh.Tq));
    return a.blk.size();
}

// The gather path (staged scan, threshold, tie location, emission, FP64
// re-rank) with every buffer carved from the device scratch, in batches of
// the largest multiple of 64 queries that fits (the caller has checked that
// 64 do).  Only kernels are queued: no allocation, copy or synchronisation.
void run_query_noalloc(const nrlsh_index *ix, const float *Qd, int64_t nq, int32_t k, int64_t T,
                       int64_t *ids_d, float *ips_d, uint32_t *nonfinite_d, hipStream_t s)
{
    const QueryShape sh = make_shape(ix, T, k);
    uint8_t *base = scratch_base(ix->device);
    int64_t B = std::min<int64_t>(std::max<int64_t>(64, ((int64_t(1) << 29) / sh.Tq) / 64 * 64),
                                  (nq + 63) / 64 * 64);
    while (B > 64 && noalloc_bytes(sh, B) > kScratchBytes) B = std::max<int64_t>(64, B / 2 / 64 * 64);
    const int nsplit = rerank_splits(B, sh.Tq);
    NoAllocLayout a;
    layout_noalloc(a, sh, B, nsplit);
    if (!a.blk.place(base, kScratchBytes))
        throw Failure{NRLSH_E_INVALID_ARG, "batch does not fit the device scratch"};
    const Block &b = a.blk;
    uint32_t *qc = b.view<uint32_t>(a.qc).get(), *ghist = b.view<uint32_t>(a.gh).get();
    int32_t *need = b.view<int32_t>(a.ne).get(), *gbase = b.view<int32_t>(a.gb).get(),
            *ghthr = b.view<int32_t>(a.th).get(), *gtie = b.view<int32_t>(a.ti).get(),
            *cand = b.view<int32_t>(a.ca).get(), *part_i = b.view<int32_t>(a.pi).get(),
            *gpstar = b.view<int32_t>(a.ps).get(), *ccount = b.view<int32_t>(a.ct).get();
    double *part_v = b.view<double>(a.pv).get();
    unsigned long long *gtheta = b.view<unsigned long long>(a.gt).get();
    const int nchunks = ix->st1_cbeg.back();
    for (int64_t b0 = 0; b0 < nq; b0 += B) {
        const int64_t nb = std::min<int64_t>(B, nq - b0);
        const float *Qb = Qd + b0 * sh.d;
        HIPX(launch_query_hash(Qb, nb, sh.d, ix->At.get(), sh.L, sh.W, sh.qsets, qc, nonfinite_d, s));
        run_scan_hist_staged(ix, sh, qc, nb, ix->st1_cbeg, ix->st1_cut, ix->st1_chunks_d.get(), need, ghist,
                             nullptr, s);
        HIPX(launch_threshold(ghist, ix->R.get(), ix->inv.get(), nb, sh, gbase, ghthr, gtie, s));
        HIPX(launch_tie_locate(ix->codes_l.get(), ix->off.get(), qc, nb, sh.W, sh.qsets, gtie, gpstar, s));
        HIPX(launch_fill32(ccount, nb, 0u, s));
        HIPX(launch_scan_emit_stage(ix->codes_l.get(), qc, nb, sh, ix->st1_chunks_d.get(), nchunks, ghthr, gtie,
                                    gpstar, ccount, cand, s));
        if (nsplit > 1) HIPX(launch_fill32(gtheta, 2 * nb, 0u, s));
        HIPX(launch_rerank(ix->Xl.get(), ix->perm.get(), Qb, nb, sh, cand, nullptr, nsplit, part_v, part_i,
                           ids_d + b0 * k, ips_d + b0 * k, s, gtheta));
    }
}

}  // namespace

// ================================================================= C ABI
extern "C" {

nrlsh_status nrlsh_build_ex(const float *items, int64_t n, int32_t d, int32_t m, int32_t L,
                            uint64_t seed, const nrlsh_build_opts *opts, nrlsh_index **out)
{
    const double eps = opts ? opts->eps : 0.0;
    nrlsh_status st = validate_build(items, n, d, m, L, eps, out);
    if (st != NRLSH_OK) return st;
    int32_t storage = NRLSH_STORAGE_FP32, margin_mode = NRLSH_MARGIN_RIGOROUS;
    double margin_param = 0.0;
    if (opts && opts->struct_size >= (int32_t)(offsetof(nrlsh_build_opts, margin_param) + sizeof(double))) {
        storage = opts->hash_storage;
        margin_mode = opts->margin_mode;
        margin_param = opts->margin_param;
    }
    if (storage < NRLSH_STORAGE_FP32 || storage > NRLSH_STORAGE_FP8_E4M3)
        return fail(NRLSH_E_INVALID_ARG, "hash_storage %d unknown", storage);
    if (margin_mode != NRLSH_MARGIN_RIGOROUS && margin_mode != NRLSH_MARGIN_SCALED)
        return fail(NRLSH_E_INVALID_ARG, "margin_mode %d unknown", margin_mode);
    if (!(margin_param >= 0.0 && margin_param < 1e30))
        return fail(NRLSH_E_INVALID_ARG, "margin_param must be finite and >= 0");
    int32_t partition = NRLSH_PARTITION_PERCENTILE;
    if (opts && opts->struct_size >= (int32_t)(offsetof(nrlsh_build_opts, partition) + sizeof(int32_t)))
        partition = opts->partition;
    if (partition != NRLSH_PARTITION_PERCENTILE && partition != NRLSH_PARTITION_UNIFORM)
        return fail(NRLSH_E_INVALID_ARG, "partition %d unknown", partition);
    int32_t projections = NRLSH_PROJECTIONS_SHARED;
    if (opts && opts->struct_size >= (int32_t)(offsetof(nrlsh_build_opts, projections) + sizeof(int32_t)))
        projections = opts->projections;
    if (projections != NRLSH_PROJECTIONS_SHARED && projections != NRLSH_PROJECTIONS_PER_SUBSET)
        return fail(NRLSH_E_INVALID_ARG, "projections %d unknown", projections);
    if (projections == NRLSH_PROJECTIONS_PER_SUBSET && storage != NRLSH_STORAGE_FP32)
        return fail(NRLSH_E_INVALID_ARG, "per-subset projections need hash_storage FP32");
    if (projections == NRLSH_PROJECTIONS_PER_SUBSET && ((int64_t)m * L > INT32_MAX / (d + 1) || m > 65535))
        return fail(NRLSH_E_INVALID_ARG, "per-subset projections need m <= 65535 and m L (d+1) < 2^31");
    int32_t tables = 0;
    if (opts && opts->struct_size >= (int32_t)(offsetof(nrlsh_build_opts, bucket_tables) + sizeof(int32_t)))
        tables = opts->bucket_tables;
    if (tables != 0 && tables != 1) return fail(NRLSH_E_INVALID_ARG, "bucket_tables must be 0 or 1");
    int32_t htables = 1;
    if (opts && opts->struct_size >= (int32_t)(offsetof(nrlsh_build_opts, hash_tables) + sizeof(int32_t)))
        htables = opts->hash_tables == 0 ? 1 : opts->hash_tables;
    if (htables < 1 || htables > MT_MAX_TABLES)
        return fail(NRLSH_E_INVALID_ARG, "hash_tables %d out of [1, %d]", htables, MT_MAX_TABLES);
    if (htables > 1 && storage != NRLSH_STORAGE_FP32)
        return fail(NRLSH_E_INVALID_ARG, "several hash tables need hash_storage FP32");
    if ((int64_t)htables * (projections == NRLSH_PROJECTIONS_PER_SUBSET ? m : 1) * L > INT32_MAX / (d + 1) ||
        (int64_t)htables * n * (L > 32 ? 2 : 1) > ((int64_t)1 << 40))
        return fail(NRLSH_E_INVALID_ARG, "hash_tables: projection or code arrays too large");
    const bool on_device = opts && opts->device_ptrs;
    // device rows are read in vectors of the widest of 4, 2, 1 floats that
    // divides d, so the first row must start on such a vector
    const int vw = d % 4 == 0 ? 4 : (d % 2 == 0 ? 2 : 1);
    if (on_device && reinterpret_cast<uintptr_t>(items) % (uintptr_t)(4 * vw) != 0)
        return fail(NRLSH_E_INVALID_ARG, "device items must be aligned to 16 bytes (d % 4 == 0), 8 bytes (d even) "
                                         "or 4 bytes");
    return guarded([&]() -> nrlsh_status {
        const int dev = current_device();
        prepare_pool(dev);
        hipStream_t s = pick_stream(opts ? opts->stream : nullptr, dev);
        nrlsh_index *ix = new nrlsh_index();
        ix->device = dev;
        ix->n = n;
        ix->d = d;
        ix->dp = (d + 7) / 8 * 8;
        ix->m = m;
        ix->L = L;
        ix->W = L > 32 ? 2 : 1;
        ix->seed = seed;
        ix->eps = eps;
        ix->storage = storage;
        ix->margin_mode = margin_mode;
        ix->margin_param = margin_param;
        ix->partition = partition;
        ix->qsets = projections == NRLSH_PROJECTIONS_PER_SUBSET ? m : 1;
        ix->has_table = tables == 1;
        ix->tables = htables;
        ix->home = library_stream(dev);
        Timer tm(s);
        try {
            build_index(ix, items, on_device, s, tm);
            tm.settle();
        } catch (...) {
            (void)hipStreamSynchronize(s);
            pinned_give(ix->counters_h, ix->counters_bytes, nullptr, dev);
            event_give(ix->ready, dev);
            delete ix;
            throw;
        }
        *out = ix;
        return NRLSH_OK;
    });
}

nrlsh_status nrlsh_build(const float *items, int64_t n, int32_t d, int32_t m, int32_t L,
                         uint64_t seed, nrlsh_index **out)
{
    return nrlsh_build_ex(items, n, d, m, L, seed, nullptr, out);
}

void nrlsh_free(nrlsh_index *ix)
{
    if (!ix) return;
    hipStream_t s = ix->home;
    // the build's device work ends before its buffers go back
    if (ix->ready) (void)hipEventSynchronize(ix->ready);
    pinned_give(ix->counters_h, ix->counters_bytes, nullptr, ix->device);
    event_give(ix->ready, ix->device);
    ix->counters_h = nullptr;
    ix->ready = nullptr;
    delete ix;  // buffers are released on their home stream
    (void)hipStreamSynchronize(s);
}

nrlsh_status nrlsh_query_ex(const nrlsh_index *ix, const float *queries, int64_t nq, int32_t k,
                            int64_t probe_budget, const nrlsh_query_opts *opts, int64_t *out_ids,
                            float *out_ips)
{
    nrlsh_status st = validate_query(ix, queries, nq, k, probe_budget, out_ids, out_ips);
    if (st != NRLSH_OK) return st;
    g_qstats = nrlsh_query_stats{};
    if (opts && opts->struct_size >= (int32_t)(offsetof(nrlsh_query_opts, rerank_mode) + sizeof(int32_t)) &&
        (opts->rerank_mode < NRLSH_RERANK_AUTO || opts->rerank_mode > NRLSH_RERANK_SCREEN_BF16X3))
        return fail(NRLSH_E_INVALID_ARG, "rerank_mode %d unknown", opts->rerank_mode);
    if (opts && opts->struct_size >= (int32_t)(offsetof(nrlsh_query_opts, rerank_storage) + sizeof(int32_t)) &&
        opts->rerank_storage != NRLSH_STORAGE_FP32 && opts->rerank_storage != NRLSH_STORAGE_BF16)
        return fail(NRLSH_E_INVALID_ARG, "rerank_storage %d unsupported", opts->rerank_storage);
    int probe = NRLSH_PROBE_SCAN;
    if (opts && opts->struct_size >= (int32_t)(offsetof(nrlsh_query_opts, probe_mode) + sizeof(int32_t))) {
        if (opts->probe_mode != NRLSH_PROBE_SCAN && opts->probe_mode != NRLSH_PROBE_TABLE &&
            opts->probe_mode != NRLSH_PROBE_SINGLE)
            return fail(NRLSH_E_INVALID_ARG, "probe_mode %d unknown", opts->probe_mode);
        probe = opts->probe_mode;
    }
    const bool table = probe == NRLSH_PROBE_TABLE;
    if (table && !ix->has_table)
        return fail(NRLSH_E_INVALID_ARG, "probe_mode TABLE needs an index built with bucket_tables = 1");
    if (probe != NRLSH_PROBE_SCAN && opts->rerank_mode != NRLSH_RERANK_AUTO &&
        opts->rerank_mode != NRLSH_RERANK_GATHER)
        return fail(NRLSH_E_INVALID_ARG, "probe_mode TABLE / SINGLE go with the GATHER re-rank");
    if (probe == NRLSH_PROBE_SINGLE && opts->struct_size >= (int32_t)(offsetof(nrlsh_query_opts, rerank_storage) +
                                                                     sizeof(int32_t)) &&
        opts->rerank_storage != NRLSH_STORAGE_FP32)
        return fail(NRLSH_E_INVALID_ARG, "probe_mode SINGLE re-ranks from the FP32 rows");
    int32_t sguess = 0;
    if (opts && opts->struct_size >= (int32_t)(offsetof(nrlsh_query_opts, scan_guess) + sizeof(int32_t))) {
        if (opts->scan_guess < -1 || opts->scan_guess > 4096)
            return fail(NRLSH_E_INVALID_ARG, "scan_guess %d out of [-1, 4096]", opts->scan_guess);
        sguess = opts->scan_guess;
    }
    int32_t dhead = 0;
    if (opts && opts->struct_size >= (int32_t)(offsetof(nrlsh_query_opts, dense_head) + sizeof(int32_t))) {
        if (opts->dense_head < -1 || opts->dense_head > 256)
            return fail(NRLSH_E_INVALID_ARG, "dense_head %d out of [-1, 256]", opts->dense_head);
        dhead = opts->dense_head;
    }
    if (nq == 0) return st;
    const bool on_device = opts && opts->device_ptrs;
    struct OptScope {  // the options last for this call only
        OptScope(int32_t g, int32_t h)
        {
            g_scan_guess = g;
            g_dense_head = h;
        }
        ~OptScope()
        {
            g_scan_guess = 0;
            g_dense_head = 0;
        }
    } opt_scope(sguess, dhead);
    return guarded([&]() -> nrlsh_status {
        HIPX(hipSetDevice(ix->device));
        hipStream_t s = pick_stream(opts ? opts->stream : nullptr, ix->device);
        index_wait(ix, s);
        Timer tm(s);
        Block blk;
        const size_t o_fl = blk.reserve<uint32_t>(1), o_sp = blk.reserve<unsigned long long>(1),
                     o_q = blk.reserve<float>(on_device ? 1 : (size_t)nq * ix->d),
                     o_i = blk.reserve<int64_t>(on_device ? 1 : (size_t)nq * k),
                     o_p = blk.reserve<float>(on_device ? 1 : (size_t)nq * k);
        blk.allocate(s);
        DBuf<uint32_t> flag = blk.view<uint32_t>(o_fl);
        DBuf<unsigned long long> spairs = blk.view<unsigned long long>(o_sp);
        HIPX(hipMemsetAsync(flag.get(), 0, sizeof(uint32_t), s));
        HIPX(hipMemsetAsync(spairs.get(), 0, sizeof(unsigned long long), s));
        int mode = NRLSH_RERANK_AUTO;
        if (opts && opts->struct_size >= (int32_t)(offsetof(nrlsh_query_opts, rerank_mode) + sizeof(int32_t)))
            mode = opts->rerank_mode;
        bool bf16_rows = false;
        if (opts && opts->struct_size >= (int32_t)(offsetof(nrlsh_query_opts, rerank_storage) + sizeof(int32_t)))
            bf16_rows = opts->rerank_storage == NRLSH_STORAGE_BF16;
        uint32_t bad = kFlagUnread;
        if (on_device) {
            bad = run_query(ix, queries, nq, k, probe_budget, mode, bf16_rows, probe, out_ids, out_ips, s, tm,
                            flag.get(), spairs.get());
        } else {
            DBuf<float> Qd = blk.view<float>(o_q);
            DBuf<int64_t> ids = blk.view<int64_t>(o_i);
            DBuf<float> ips = blk.view<float>(o_p);
            HIPX(hipMemcpyAsync(Qd.get(), queries, (size_t)nq * ix->d * sizeof(float),
                                hipMemcpyHostToDevice, s));
            (void)run_query(ix, Qd.get(), nq, k, probe_budget, mode, bf16_rows, probe, ids.get(), ips.get(), s,
                            tm, flag.get(), spairs.get());
            HIPX(hipMemcpyAsync(out_ids, ids.get(), (size_t)nq * k * sizeof(int64_t),
                                hipMemcpyDeviceToHost, s));
            HIPX(hipMemcpyAsync(out_ips, ips.get(), (size_t)nq * k * sizeof(float),
                                hipMemcpyDeviceToHost, s));
        }
        // the pairs of the staged scan come back with the flag (host outputs:
        // the copies above are waited for here)
        unsigned long long sp = 0;
        const bool read_flag = bad == kFlagUnread;
        if (read_flag) bad = 0;
        if (read_flag) HIPX(hipMemcpyAsync(&bad, flag.get(), sizeof bad, hipMemcpyDeviceToHost, s));
        HIPX(hipMemcpyAsync(&sp, spairs.get(), sizeof sp, hipMemcpyDeviceToHost, s));
        HIPX(hipStreamSynchronize(s));
        g_qstats.scan_pairs = (int64_t)sp;
        tm.settle();
        if (bad) return fail(NRLSH_E_NOT_FINITE, "queries hold NaN or Inf");
        return NRLSH_OK;
    });
}

nrlsh_status nrlsh_query(const nrlsh_index *ix, const float *queries, int64_t nq, int32_t k,
                         int64_t probe_budget, int64_t *out_ids, float *out_ips)
{
    return nrlsh_query_ex(ix, queries, nq, k, probe_budget, nullptr, out_ids, out_ips);
}

nrlsh_status nrlsh_query_noalloc(const nrlsh_index *ix, const float *queries, int64_t nq, int32_t k,
                                 int64_t probe_budget, void *stream, int64_t *out_ids, float *out_ips,
                                 uint32_t *nonfinite)
{
    nrlsh_status st = validate_query(ix, queries, nq, k, probe_budget, out_ids, out_ips);
    if (st != NRLSH_OK) return st;
    if (!nonfinite) return fail(NRLSH_E_INVALID_ARG, "nonfinite is NULL");
    const QueryShape sh = make_shape(ix, probe_budget, k);
    const size_t need64 = noalloc_bytes(sh, 64);
    if (need64 > kScratchBytes)
        return fail(NRLSH_E_INVALID_ARG,
                    "a 64-query batch at this budget needs %zu bytes of scratch; the entry point that "
                    "allocates nothing holds %zu (use nrlsh_query_ex)",
                    need64, kScratchBytes);
    g_qstats = nrlsh_query_stats{};
    g_qstats.mode = NRLSH_RERANK_GATHER;
    g_qstats.probe_mode = NRLSH_PROBE_SCAN;
    return guarded([&]() -> nrlsh_status {
        HIPX(hipSetDevice(ix->device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        index_wait(ix, s);
        HIPX(launch_fill32(nonfinite, 1, 0u, s));
        if (nq > 0) run_query_noalloc(ix, queries, nq, k, probe_budget, out_ids, out_ips, nonfinite, s);
        return NRLSH_OK;
    });
}

const char *nrlsh_last_error(void) { return g_err.c_str(); }

nrlsh_status nrlsh_index_info(const nrlsh_index *ix, int64_t *n, int32_t *d, int32_t *m,
                              int32_t *L, int32_t *dp)
{
    if (!ix || !n || !d || !m || !L || !dp) return fail(NRLSH_E_INVALID_ARG, "NULL argument");
    *n = ix->n;
    *d = ix->d;
    *m = ix->m;
    *L = ix->L;
    *dp = ix->dp;
    return NRLSH_OK;
}

nrlsh_status nrlsh_get_bucket_table(const nrlsh_index *ix, int64_t *nunique, uint64_t *ucode,
                                    int64_t *ustart, int64_t *uoff, int32_t *titem)
{
    if (!ix || !nunique) return fail(NRLSH_E_INVALID_ARG, "NULL argument");
    if (!ix->has_table) return fail(NRLSH_E_INVALID_ARG, "index built without bucket tables");
    *nunique = ix->nunique;
    if (!ucode) return NRLSH_OK;
    if (!ustart || !uoff || !titem) return fail(NRLSH_E_INVALID_ARG, "NULL argument");
    return guarded([&]() -> nrlsh_status {
        HIPX(hipSetDevice(ix->device));
        index_settle(ix);
        const int64_t U = ix->nunique;
        std::vector<int32_t> us((size_t)U + 1);
        HIPX(hipMemcpy(ucode, ix->ucode.get(), (size_t)U * sizeof(uint64_t), hipMemcpyDeviceToHost));
        HIPX(hipMemcpy(us.data(), ix->ustart.get(), us.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIPX(hipMemcpy(titem, ix->titem.get(), (size_t)ix->n * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int64_t u = 0; u <= U; ++u) ustart[u] = us[(size_t)u];
        for (int j = 0; j <= ix->m; ++j) uoff[j] = ix->uoff_h[(size_t)j];
        return NRLSH_OK;
    });
}

nrlsh_status nrlsh_get_projection_sets(const nrlsh_index *ix, int32_t *sets)
{
    if (!ix || !sets) return fail(NRLSH_E_INVALID_ARG, "NULL argument");
    *sets = ix->qsets;
    return NRLSH_OK;
}

nrlsh_status nrlsh_get_hash_tables(const nrlsh_index *ix, int32_t *tables)
{
    if (!ix || !tables) return fail(NRLSH_E_INVALID_ARG, "NULL argument");
    *tables = ix->tables;
    return NRLSH_OK;
}
nrlsh_status nrlsh_get_projection(const nrlsh_index *ix, float *A)
{
    if (!ix || !A) return fail(NRLSH_E_INVALID_ARG, "NULL argument");
    std::memcpy(A, ix->A_h.data(), ix->A_h.size() * sizeof(float));
    return NRLSH_OK;
}

nrlsh_status nrlsh_get_keys(const nrlsh_index *ix, double *key)
{
    if (!ix || !key) return fail(NRLSH_E_INVALID_ARG, "NULL argument");
    return guarded([&]() -> nrlsh_status {
        HIPX(hipSetDevice(ix->device));
        index_settle(ix);
        HIPX(hipMemcpy(key, ix->key.get(), (size_t)ix->n * sizeof(double), hipMemcpyDeviceToHost));
        return NRLSH_OK;
    });
}

nrlsh_status nrlsh_get_partition(const nrlsh_index *ix, int32_t *sid, double *keymax, double *U)
{
    if (!ix || !sid || !keymax || !U) return fail(NRLSH_E_INVALID_ARG, "NULL argument");
    return guarded([&]() -> nrlsh_status {
        HIPX(hipSetDevice(ix->device));
        index_settle(ix);
        HIPX(hipMemcpy(sid, ix->sid.get(), (size_t)ix->n * sizeof(int32_t), hipMemcpyDeviceToHost));
        std::memcpy(keymax, ix->keymax_h.data(), ix->m * sizeof(double));
        std::memcpy(U, ix->U_h.data(), ix->m * sizeof(double));
        return NRLSH_OK;
    });
}

nrlsh_status nrlsh_get_layout(const nrlsh_index *ix, int32_t *perm, int64_t *off)
{
    if (!ix || !perm || !off) return fail(NRLSH_E_INVALID_ARG, "NULL argument");
    return guarded([&]() -> nrlsh_status {
        HIPX(hipSetDevice(ix->device));
        index_settle(ix);
        HIPX(hipMemcpy(perm, ix->perm.get(), (size_t)ix->n * sizeof(int32_t), hipMemcpyDeviceToHost));
        std::memcpy(off, ix->off_h.data(), (ix->m + 1) * sizeof(int64_t));
        return NRLSH_OK;
    });
}

nrlsh_status nrlsh_get_codes(const nrlsh_index *ix, uint64_t *codes)
{
    return nrlsh_get_codes_table(ix, 0, codes);
}
nrlsh_status nrlsh_get_codes_table(const nrlsh_index *ix, int32_t table, uint64_t *codes)
{
    if (!ix || !codes) return fail(NRLSH_E_INVALID_ARG, "NULL argument");
    if (table < 0 || table >= ix->tables) return fail(NRLSH_E_INVALID_ARG, "table %d out of range", table);
    return guarded([&]() -> nrlsh_status {
        HIPX(hipSetDevice(ix->device));
        index_settle(ix);
        std::vector<uint32_t> w((size_t)ix->n * ix->W);
        std::vector<int32_t> perm(ix->n);
        HIPX(hipMemcpy(w.data(), ix->codes_l.get() + (size_t)table * ix->n * ix->W, w.size() * sizeof(uint32_t),
                       hipMemcpyDeviceToHost));
        HIPX(hipMemcpy(perm.data(), ix->perm.get(), perm.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int64_t p = 0; p < ix->n; ++p) {
            uint64_t c = w[(size_t)p * ix->W];
            if (ix->W == 2) c |= (uint64_t)w[(size_t)p * 2 + 1] << 32;
            codes[perm[p]] = c;
        }
        return NRLSH_OK;
    });
}

nrlsh_status nrlsh_get_hash_copy(const nrlsh_index *ix, void *data, float *scales, int32_t *storage)
{
    if (!ix || !data || !storage) return fail(NRLSH_E_INVALID_ARG, "NULL argument");
    return guarded([&]() -> nrlsh_status {
        HIPX(hipSetDevice(ix->device));
        index_settle(ix);
        const size_t cnt = (size_t)ix->n * ix->dp;
        *storage = ix->storage;
        if (ix->storage == NRLSH_STORAGE_FP32) {
            HIPX(hipMemcpy(data, ix->Xl.get(), cnt * sizeof(float), hipMemcpyDeviceToHost));
        } else if (ix->storage == NRLSH_STORAGE_BF16) {
            HIPX(hipMemcpy(data, ix->Xh.get(), cnt * sizeof(uint16_t), hipMemcpyDeviceToHost));
        } else {
            if (!scales) return fail(NRLSH_E_INVALID_ARG, "scales is NULL");
            HIPX(hipMemcpy(data, ix->Xf8.get(), cnt, hipMemcpyDeviceToHost));
            HIPX(hipMemcpy(scales, ix->xscale.get(), (size_t)ix->n * sizeof(float), hipMemcpyDeviceToHost));
        }
        return NRLSH_OK;
    });
}

nrlsh_status nrlsh_get_rank_table(const nrlsh_index *ix, int32_t *R)
{
    if (!ix || !R) return fail(NRLSH_E_INVALID_ARG, "NULL argument");
    std::memcpy(R, ix->R_h.data(), ix->R_h.size() * sizeof(int32_t));
    return NRLSH_OK;
}

nrlsh_status nrlsh_get_build_stats(const nrlsh_index *ix, nrlsh_build_stats *st)
{
    if (!ix || !st) return fail(NRLSH_E_INVALID_ARG, "NULL argument");
    return guarded([&]() -> nrlsh_status {
        HIPX(hipSetDevice(ix->device));
        index_settle(ix);
        *st = ix->stats;
        return NRLSH_OK;
    });
}

nrlsh_status nrlsh_query_codes(const nrlsh_index *ix, const float *queries, int64_t nq,
                               uint64_t *codes)
{
    if (!ix || (nq > 0 && (!queries || !codes)) || nq < 0)
        return fail(NRLSH_E_INVALID_ARG, "bad argument");
    if (nq == 0) return NRLSH_OK;
    if (!all_finite(queries, nq * (int64_t)ix->d)) return fail(NRLSH_E_NOT_FINITE, "queries hold NaN or Inf");
    return guarded([&]() -> nrlsh_status {
        HIPX(hipSetDevice(ix->device));
        index_settle(ix);
        hipStream_t s = library_stream(ix->device);
        DBuf<float> Qd((size_t)nq * ix->d, s);
        const int64_t rows = nq * ix->qsets;
        DBuf<uint32_t> qc((size_t)rows * ix->W, s);
        DBuf<uint32_t> flag(1, s);
        HIPX(hipMemsetAsync(flag.get(), 0, sizeof(uint32_t), s));
        HIPX(hipMemcpyAsync(Qd.get(), queries, (size_t)nq * ix->d * sizeof(float), hipMemcpyHostToDevice, s));
        HIPX(launch_query_hash(Qd.get(), nq, ix->d, ix->At.get(), ix->L, ix->W, ix->qsets, qc.get(),
                               flag.get(), s));
        std::vector<uint32_t> w((size_t)rows * ix->W);
        HIPX(hipMemcpyAsync(w.data(), qc.get(), w.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIPX(hipStreamSynchronize(s));
        for (int64_t i = 0; i < rows; ++i) {
            uint64_t c = w[(size_t)i * ix->W];
            if (ix->W == 2) c |= (uint64_t)w[(size_t)i * 2 + 1] << 32;
            codes[i] = c;
        }
        return NRLSH_OK;
    });
}

nrlsh_status nrlsh_query_candidates_ex(const nrlsh_index *ix, const float *queries, int64_t nq,
                                       int64_t probe_budget, int32_t probe_mode, int64_t *cand,
                                       int64_t *counts)
{
    if (probe_mode == NRLSH_PROBE_SCAN) {
        const nrlsh_status st = nrlsh_query_candidates(ix, queries, nq, probe_budget, cand);
        if (st == NRLSH_OK && counts)
            for (int64_t q = 0; q < nq; ++q) counts[q] = std::min<int64_t>(probe_budget, ix->n);
        return st;
    }
    if (probe_mode != NRLSH_PROBE_SINGLE) return fail(NRLSH_E_INVALID_ARG, "probe_mode %d not supported here", probe_mode);
    if (!ix || nq < 0 || (nq > 0 && (!queries || !cand || !counts)) || probe_budget < 1)
        return fail(NRLSH_E_INVALID_ARG, "bad argument");
    if (nq == 0) return NRLSH_OK;
    if (!all_finite(queries, nq * (int64_t)ix->d)) return fail(NRLSH_E_NOT_FINITE, "queries hold NaN or Inf");
    return guarded([&]() -> nrlsh_status {
        HIPX(hipSetDevice(ix->device));
        index_settle(ix);
        hipStream_t s = library_stream(ix->device);
        const int64_t Tq = std::min<int64_t>(probe_budget, ix->n);
        Timer tm(s);
        DBuf<float> Qd((size_t)nq * ix->d, s);
        DBuf<int32_t> cd((size_t)nq * Tq, s), cn((size_t)nq, s);
        DBuf<uint32_t> flag(1, s);
        HIPX(hipMemsetAsync(flag.get(), 0, sizeof(uint32_t), s));
        HIPX(hipMemcpyAsync(Qd.get(), queries, (size_t)nq * ix->d * sizeof(float), hipMemcpyHostToDevice, s));
        run_query_single(ix, Qd.get(), nq, 1, probe_budget, nullptr, nullptr, cd.get(), cn.get(), s, tm, flag.get());
        std::vector<int32_t> pos((size_t)nq * Tq), perm(ix->n), cnt((size_t)nq);
        HIPX(hipMemcpyAsync(pos.data(), cd.get(), pos.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPX(hipMemcpyAsync(cnt.data(), cn.get(), cnt.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPX(hipMemcpyAsync(perm.data(), ix->perm.get(), perm.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPX(hipStreamSynchronize(s));
        for (int64_t q = 0; q < nq; ++q) {
            const int64_t c = std::min<int64_t>(cnt[(size_t)q], Tq);
            counts[q] = c;
            for (int64_t e = 0; e < Tq; ++e) {
                const int32_t p = pos[(size_t)(q * Tq + e)];
                if (e >= c) {
                    cand[q * Tq + e] = -1;
                    continue;
                }
                if (p < 0 || p >= ix->n) throw Failure{NRLSH_E_INTERNAL, "probed position out of range"};
                cand[q * Tq + e] = perm[p];
            }
        }
        return NRLSH_OK;
    });
}

namespace {
// The probed set of each query (original ids) and, when levels is not NULL,
// each probed item's number of bits equal to its query's code, l = L - h.
nrlsh_status query_candidates(const nrlsh_index *ix, const float *queries, int64_t nq, int64_t probe_budget,
                              int64_t *cand, int32_t *levels)
{
    if (!ix || nq < 0 || (nq > 0 && (!queries || !cand)) || probe_budget < 1)
        return fail(NRLSH_E_INVALID_ARG, "bad argument");
    if (nq == 0) return NRLSH_OK;
    if (!all_finite(queries, nq * (int64_t)ix->d)) return fail(NRLSH_E_NOT_FINITE, "queries hold NaN or Inf");
    return guarded([&]() -> nrlsh_status {
        HIPX(hipSetDevice(ix->device));
        index_settle(ix);
        hipStream_t s = library_stream(ix->device);
        const int64_t Tq = std::min<int64_t>(probe_budget, ix->n);
        Timer tm(s);
        DBuf<float> Qd((size_t)nq * ix->d, s);
        DBuf<int32_t> cd((size_t)nq * Tq, s);
        DBuf<uint32_t> qc((size_t)nq * ix->qsets * ix->W, s);
        DBuf<uint32_t> flag(1, s);
        HIPX(hipMemsetAsync(flag.get(), 0, sizeof(uint32_t), s));
        HIPX(hipMemcpyAsync(Qd.get(), queries, (size_t)nq * ix->d * sizeof(float), hipMemcpyHostToDevice, s));
        run_query_gather(ix, Qd.get(), nq, 1, probe_budget, nullptr, nullptr, cd.get(), qc.get(), s, tm,
                         flag.get());
        std::vector<int32_t> pos((size_t)nq * Tq), perm(ix->n);
        HIPX(hipMemcpyAsync(pos.data(), cd.get(), pos.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPX(hipMemcpyAsync(perm.data(), ix->perm.get(), perm.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPX(hipStreamSynchronize(s));
        for (size_t e = 0; e < pos.size(); ++e) {
            if (pos[e] < 0 || pos[e] >= ix->n) throw Failure{NRLSH_E_INTERNAL, "probed position out of range"};
            cand[e] = perm[pos[e]];
        }
        if (levels) {
            // codes in stored order and the query codes, then l per entry (the
            // sub-dataset of a stored position from the offsets)
            const int W = ix->W;
            std::vector<uint32_t> codes((size_t)ix->n * W), qch((size_t)nq * ix->qsets * W);
            HIPX(hipMemcpyAsync(codes.data(), ix->codes_l.get(), codes.size() * sizeof(uint32_t),
                                hipMemcpyDeviceToHost, s));
            HIPX(hipMemcpyAsync(qch.data(), qc.get(), qch.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            HIPX(hipStreamSynchronize(s));
            const std::vector<int64_t> &off = ix->off_h;
            for (int64_t q = 0; q < nq; ++q)
                for (int64_t e = 0; e < Tq; ++e) {
                    const int64_t p = pos[(size_t)(q * Tq + e)];
                    const int j = (int)(std::upper_bound(off.begin(), off.end(), p) - off.begin()) - 1;
                    const int64_t r = qrow(q, j, ix->qsets);
                    int h = 0;
                    for (int w = 0; w < W; ++w)
                        h += __builtin_popcount(codes[(size_t)(p * W + w)] ^ qch[(size_t)(r * W + w)]);
                    levels[q * Tq + e] = ix->L - h;
                }
        }
        return NRLSH_OK;
    });
}
}  // namespace

nrlsh_status nrlsh_query_candidates(const nrlsh_index *ix, const float *queries, int64_t nq,
                                    int64_t probe_budget, int64_t *cand)
{
    return query_candidates(ix, queries, nq, probe_budget, cand, nullptr);
}

nrlsh_status nrlsh_query_candidates_levels(const nrlsh_index *ix, const float *queries, int64_t nq,
                                           int64_t probe_budget, int64_t *cand, int32_t *levels)
{
    if (nq > 0 && !levels) return fail(NRLSH_E_INVALID_ARG, "NULL levels");
    return query_candidates(ix, queries, nq, probe_budget, cand, levels);
}

nrlsh_status nrlsh_get_query_stats(nrlsh_query_stats *st)
{
    if (!st) return fail(NRLSH_E_INVALID_ARG, "NULL argument");
    *st = g_qstats;
    return NRLSH_OK;
}

void nrlsh_profile_enable(int32_t on) { g_prof_on.store(on ? 1 : 0); }

void nrlsh_profile_reset(void)
{
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof.clear();
}

nrlsh_status nrlsh_profile_get(const char *name, double *total_ms, int64_t *launches)
{
    if (!name || !total_ms || !launches) return fail(NRLSH_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(g_prof_mu);
    auto it = g_prof.find(name);
    *total_ms = it == g_prof.end() ? 0.0 : it->second.ms;
    *launches = it == g_prof.end() ? 0 : it->second.launches;
    return NRLSH_OK;
}

}  // extern "C"
