// Host side of the batching form (many indexes, one persistent launch):
// plans -- the shape of a set of (index, query batch) pairs, its workspace,
// work-queue numbering and captured hipGraph -- and the table of tile shapes
// with its autotuner.  The work itself is k_multi (k_multi.hip).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "host_common.h"
#include "nrlsh.h"
#include "nrlsh_internal.h"

using namespace nrlsh;
using namespace nrlsh::host;

namespace {

constexpr int32_t kDefaultChunk = 16384;  // stored items per scan item
constexpr int32_t kDefaultSlice = 1024;   // candidates per re-rank item
constexpr int64_t kMaxSplit = 256;        // re-rank items per query
constexpr double kWaitLimitSeconds = 10.0;
constexpr int32_t kMaxPairs = 4096;

struct TileShape {
    int32_t chunk, slice;
};

// ---------------------------------------------------------------- shape table
struct ClassKey {
    int32_t d2, L, batch;
    bool operator<(const ClassKey &o) const
    {
        return std::tie(d2, L, batch) < std::tie(o.d2, o.L, o.batch);
    }
};

ClassKey class_of(int32_t d, int32_t L, int64_t nq)
{
    int32_t d2 = 1;
    while (d2 < d) d2 <<= 1;
    return ClassKey{d2, L, nq <= 16 ? 0 : (nq <= 256 ? 1 : 2)};
}

std::mutex g_tune_mu;
std::map<ClassKey, TileShape> g_tune;

bool table_get(const ClassKey &c, TileShape *t)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(c);
    if (it == g_tune.end()) return false;
    *t = it->second;
    return true;
}

void table_put(const ClassKey &c, TileShape t)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[c] = t;
}

struct PairShape {
    const nrlsh_index *ix;
    int64_t nq, T;
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

// ================================================================= the plan
struct nrlsh_multi_plan {
    int device = 0;
    hipStream_t stream = nullptr;   // runs
    hipStream_t capture = nullptr;  // private stream the graph is captured on
    bool device_ptrs = false, use_graph = true, persistent = false;
    int32_t k = 0, count = 0;
    std::vector<PairShape> shape;    // per pair, as given
    std::vector<TileShape> tile;     // per pair
    std::vector<int> active;         // pair of each descriptor (pairs with nq > 0)
    std::vector<MultiDesc> desc;     // per active pair
    std::vector<int64_t> seg;        // MULTI_PHASES x nb + 1 item numbers
    int64_t ntiles = 0, nq_total = 0;
    int64_t items[MULTI_PHASES] = {};
    int grid = 0;
    size_t lds = 0;
    int64_t limit = 0;
    DBuf<uint8_t> ws;                // per-pair workspace, then the counters
    size_t ws_bytes = 0;
    int32_t *ctr = nullptr;
    DBuf<uint8_t> blk;               // run block: result | descriptors | item numbers
    size_t blk_bytes = 0, desc_off = 0, seg_off = 0;
    uint8_t *blk_h = nullptr;        // pinned staging of the run block
    MultiResult *res_h = nullptr;    // pinned copy of the result word
    std::vector<DBuf<float>> q_stage;
    std::vector<DBuf<int64_t>> id_stage;
    std::vector<DBuf<float>> ip_stage;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool dirty = true;               // workspace must be cleared before the next launch
    int32_t tuned_classes = 0;
    double tune_ms = 0.0;

    ~nrlsh_multi_plan()
    {
        if (stream) (void)hipStreamSynchronize(stream);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        q_stage.clear();
        id_stage.clear();
        ip_stage.clear();
        ws.reset();
        blk.reset();
        if (stream) (void)hipStreamSynchronize(stream);
        if (blk_h) (void)hipHostFree(blk_h);
        if (res_h) (void)hipHostFree(res_h);
        if (capture) (void)hipStreamDestroy(capture);
    }
};

namespace {

struct PlanOpts {
    bool device_ptrs = false, use_graph = true;
    void *stream = nullptr;
    int32_t tune = NRLSH_TUNE_TABLE;
    int32_t chunk = 0, slice = 0;
    bool persistent = false;
};

nrlsh_status read_opts(const nrlsh_multi_opts *o, PlanOpts *p)
{
    if (!o) return NRLSH_OK;
    if (o->struct_size < (int32_t)(offsetof(nrlsh_multi_opts, stream) + sizeof(void *)))
        return fail(NRLSH_E_INVALID_ARG, "nrlsh_multi_opts.struct_size %d too small", o->struct_size);
    p->device_ptrs = o->device_ptrs != 0;
    p->stream = o->stream;
    auto has = [&](size_t off) { return (size_t)o->struct_size >= off + sizeof(int32_t); };
    if (has(offsetof(nrlsh_multi_opts, use_graph))) p->use_graph = o->use_graph != 0;
    if (has(offsetof(nrlsh_multi_opts, tune))) p->tune = o->tune;
    if (has(offsetof(nrlsh_multi_opts, chunk))) p->chunk = o->chunk;
    if (has(offsetof(nrlsh_multi_opts, slice))) p->slice = o->slice;
    if (has(offsetof(nrlsh_multi_opts, persistent))) p->persistent = o->persistent != 0;
    if (p->persistent)
        return fail(NRLSH_E_INVALID_ARG,
                    "the single persistent launch is disabled (its launches did not complete in "
                    "testing); the phase-per-launch form gives the same result");
    if (p->tune < NRLSH_TUNE_TABLE || p->tune > NRLSH_TUNE_DEFAULT)
        return fail(NRLSH_E_INVALID_ARG, "tune mode %d unknown", p->tune);
    for (int32_t v : {p->chunk, p->slice})
        if (v < 0 || v % 64 != 0 || v > (1 << 24))
            return fail(NRLSH_E_INVALID_ARG, "chunk / slice %d: want 0 or a multiple of 64 up to 2^24", v);
    return NRLSH_OK;
}

nrlsh_status validate_descs(const nrlsh_query_desc *descs, int32_t count, int32_t k)
{
    if (!descs) return fail(NRLSH_E_INVALID_ARG, "descs is NULL");
    if (count < 1 || count > kMaxPairs)
        return fail(NRLSH_E_INVALID_ARG, "count %d out of range [1, %d]", count, kMaxPairs);
    if (k < 1 || k > NRLSH_MAX_K) return fail(NRLSH_E_INVALID_ARG, "k %d out of range", k);
    for (int32_t i = 0; i < count; ++i) {
        const nrlsh_query_desc &q = descs[i];
        if (!q.index) return fail(NRLSH_E_INVALID_ARG, "descs[%d].index is NULL", i);
        if (q.nq < 0 || q.nq > INT32_MAX) return fail(NRLSH_E_INVALID_ARG, "descs[%d].nq out of range", i);
        if (q.probe_budget < 1) return fail(NRLSH_E_INVALID_ARG, "descs[%d].probe_budget < 1", i);
        if (q.nq > 0 && (!q.queries || !q.out_ids || !q.out_ips))
            return fail(NRLSH_E_INVALID_ARG, "descs[%d] has a NULL query or output pointer", i);
    }
    // index fields are read only once every scalar argument has passed
    for (int32_t i = 0; i < count; ++i) {
        if (descs[i].index->device != descs[0].index->device)
            return fail(NRLSH_E_INVALID_ARG, "descs[%d].index lives on another device", i);
        if (descs[i].index->qsets != 1)
            return fail(NRLSH_E_INVALID_ARG,
                        "descs[%d].index uses per-subset projections, which the batching form does not take", i);
    }
    return NRLSH_OK;
}

// Workspace layout, item numbering and launch shape of the plan.
void lay_out(nrlsh_multi_plan *P)
{
    const int nb = (int)P->active.size();
    P->desc.assign(nb, MultiDesc{});
    size_t off = 0;
    std::vector<size_t> o_qc(nb), o_gh(nb), o_th(nb), o_ti(nb), o_ps(nb), o_ca(nb), o_pv(nb), o_pi(nb),
        o_gt(nb);
    int64_t tiles_before = 0, q_before = 0, cand_total = 0;
    int maxL = 1;
    for (int b = 0; b < nb; ++b) {
        const int i = P->active[b];
        const nrlsh_index *ix = P->shape[i].ix;
        MultiDesc &D = P->desc[b];
        D.Xl = ix->Xl.get();
        D.perm = ix->perm.get();
        D.codes_l = ix->codes_l.get();
        D.off = ix->off.get();
        D.R = ix->R.get();
        D.inv = ix->inv.get();
        D.At = ix->At.get();
        D.n = ix->n;
        D.d = ix->d;
        D.dp = ix->dp;
        D.m = ix->m;
        D.L = ix->L;
        D.W = ix->W;
        D.nq = P->shape[i].nq;
        D.Tq = std::min<int64_t>(P->shape[i].T, ix->n);
        const int64_t tiles = cdiv(D.nq, 64);
        D.tile_base = (int32_t)tiles_before;
        D.q_base = q_before;
        tiles_before += tiles;
        q_before += D.nq;
        cand_total += D.nq * D.Tq;
        maxL = std::max(maxL, D.L);
        int64_t maxsub = 0;
        for (int j = 0; j < ix->m; ++j) maxsub = std::max(maxsub, ix->off_h[j + 1] - ix->off_h[j]);
        D.chunk = P->tile[i].chunk;
        D.nch = (int32_t)std::max<int64_t>(1, cdiv(maxsub, D.chunk));
        int64_t slice = P->tile[i].slice;
        if (cdiv(D.Tq, slice) > kMaxSplit) slice = align_up((size_t)cdiv(D.Tq, kMaxSplit), 64);
        D.slice = (int32_t)slice;
        D.nsplit = (int32_t)cdiv(D.Tq, slice);
        auto take = [&](size_t bytes) {
            const size_t at = off;
            off = align_up(off + std::max<size_t>(bytes, 4), 256);
            return at;
        };
        o_qc[b] = take((size_t)D.nq * D.W * 4);
        o_gh[b] = take((size_t)tiles * D.m * (D.L + 1) * 64 * 4);
        o_th[b] = take((size_t)tiles * D.m * 64 * 4);
        o_ti[b] = take((size_t)tiles * 4 * 64 * 4);
        o_ps[b] = take((size_t)D.nq * 4);
        o_ca[b] = take((size_t)D.nq * D.Tq * 4);
        const size_t parts = D.nsplit > 1 ? (size_t)D.nq * D.nsplit * P->k : 0;
        o_pv[b] = take(parts * 8);
        o_pi[b] = take(parts * 4);
        o_gt[b] = take(D.nsplit > 1 ? (size_t)D.nq * 8 : 0);
    }
    if (cand_total > INT32_MAX)
        throw Failure{NRLSH_E_INVALID_ARG, "the probed lists of the set exceed 2^31 entries; split the set"};
    P->ntiles = tiles_before;
    P->nq_total = q_before;
    const size_t ctr_off = off;
    off = align_up(off + (size_t)multi_ctr_words(P->ntiles, P->nq_total) * 4, 256);
    P->ws_bytes = off;
    P->ws = DBuf<uint8_t>(P->ws_bytes, P->stream);
    uint8_t *base = P->ws.get();
    for (int b = 0; b < nb; ++b) {
        MultiDesc &D = P->desc[b];
        D.qcodes = reinterpret_cast<uint32_t *>(base + o_qc[b]);
        D.ghist = reinterpret_cast<uint32_t *>(base + o_gh[b]);
        D.ghthr = reinterpret_cast<int32_t *>(base + o_th[b]);
        D.gtie = reinterpret_cast<int32_t *>(base + o_ti[b]);
        D.gpstar = reinterpret_cast<int32_t *>(base + o_ps[b]);
        D.cand = reinterpret_cast<int32_t *>(base + o_ca[b]);
        D.part_v = reinterpret_cast<double *>(base + o_pv[b]);
        D.part_i = reinterpret_cast<int32_t *>(base + o_pi[b]);
        D.gtheta = D.nsplit > 1 ? reinterpret_cast<unsigned long long *>(base + o_gt[b]) : nullptr;
    }
    P->ctr = reinterpret_cast<int32_t *>(base + ctr_off);

    // phase-major item numbering
    P->seg.assign((size_t)MULTI_PHASES * nb + 1, 0);
    std::fill(P->items, P->items + MULTI_PHASES, 0);
    int64_t run = 0;
    for (int ph = 0; ph < MULTI_PHASES; ++ph)
        for (int b = 0; b < nb; ++b) {
            const MultiDesc &D = P->desc[b];
            const int64_t tiles = cdiv(D.nq, 64);
            int64_t c = 0;
            switch (ph) {
            case 0: c = cdiv(D.nq, 16); break;
            case 1: c = tiles * D.m * D.nch; break;
            case 2: c = tiles; break;
            case 3: c = D.nq; break;
            case 4: c = tiles * D.m * D.nch; break;
            case 5: c = D.nq * D.nsplit; break;
            default: c = D.nsplit > 1 ? D.nq : 0; break;
            }
            P->seg[(size_t)ph * nb + b] = run;
            P->items[ph] += c;
            run += c;
        }
    P->seg[(size_t)MULTI_PHASES * nb] = run;

    P->lds = multi_lds_bytes(maxL);
    int per_cu = 0, cus = 0, rate_khz = 0;
    HIPX(multi_occupancy(P->k, P->lds, &per_cu));
    HIPX(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P->device));
    HIPX(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, P->device));
    const int64_t resident = (int64_t)std::max(1, per_cu) * std::max(1, cus);
    P->grid = (int)std::max<int64_t>(1, std::min<int64_t>(run, resident));
    if (!P->persistent) P->grid = (int)*std::max_element(P->items, P->items + MULTI_PHASES);
    if (run + P->grid >= INT32_MAX)
        throw Failure{NRLSH_E_INVALID_ARG, "too many work items in one launch; split the set"};
    if (rate_khz <= 0) rate_khz = 100000;  // the 100 MHz constant clock of gfx9 parts
    P->limit = (int64_t)(kWaitLimitSeconds * (double)rate_khz * 1000.0);

    // run block
    P->desc_off = align_up(sizeof(MultiResult), 64);
    P->seg_off = align_up(P->desc_off + (size_t)nb * sizeof(MultiDesc), 64);
    P->blk_bytes = P->seg_off + P->seg.size() * sizeof(int64_t);
    P->blk = DBuf<uint8_t>(P->blk_bytes, P->stream);
    void *h = nullptr;
    HIPX(hipHostMalloc(&h, P->blk_bytes, hipHostMallocDefault));
    P->blk_h = static_cast<uint8_t *>(h);
    HIPX(hipHostMalloc(&h, sizeof(MultiResult), hipHostMallocDefault));
    P->res_h = static_cast<MultiResult *>(h);

    if (!P->device_ptrs)
        for (int b = 0; b < nb; ++b) {
            const MultiDesc &D = P->desc[b];
            P->q_stage.emplace_back((size_t)D.nq * D.d, P->stream);
            P->id_stage.emplace_back((size_t)D.nq * P->k, P->stream);
            P->ip_stage.emplace_back((size_t)D.nq * P->k, P->stream);
        }
}

// Upload of the run block, the launches, download of the result word.
void enqueue(nrlsh_multi_plan *P, hipStream_t s)
{
    uint8_t *blk = P->blk.get();
    HIPX(hipMemcpyAsync(blk, P->blk_h, P->blk_bytes, hipMemcpyHostToDevice, s));
    const MultiDesc *descs = reinterpret_cast<const MultiDesc *>(blk + P->desc_off);
    const int64_t *seg = reinterpret_cast<const int64_t *>(blk + P->seg_off);
    MultiResult *result = reinterpret_cast<MultiResult *>(blk);
    if (P->persistent)
        HIPX(launch_multi(descs, (int)P->desc.size(), seg, result, P->ctr, P->ntiles, P->nq_total,
                          P->k, P->limit, P->grid, P->lds, s));
    else
        HIPX(launch_multi_phases(descs, (int)P->desc.size(), seg, P->items, result,
                                 P->ctr + MULTI_CTR_TILES + MULTI_TILE_CTRS * P->ntiles,
                                 P->nq_total, P->k, P->lds, s));
    HIPX(hipMemcpyAsync(P->res_h, blk, sizeof(MultiResult), hipMemcpyDeviceToHost, s));
}

void capture_graph(nrlsh_multi_plan *P)
{
    HIPX(hipStreamCreateWithFlags(&P->capture, hipStreamNonBlocking));
    HIPX(hipStreamBeginCapture(P->capture, hipStreamCaptureModeThreadLocal));
    try {
        enqueue(P, P->capture);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(P->capture, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    HIPX(hipStreamEndCapture(P->capture, &P->graph));
    HIPX(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
}

// One run.  launch_ms != NULL: HIP-event time of the launch itself.
nrlsh_status run_plan(nrlsh_multi_plan *P, const nrlsh_query_desc *descs, float *launch_ms)
{
    HIPX(hipSetDevice(P->device));
    hipStream_t s = P->stream;
    const int nb = (int)P->desc.size();
    if (nb == 0) return NRLSH_OK;
    for (int b = 0; b < nb; ++b) {
        const nrlsh_query_desc &q = descs[P->active[b]];
        MultiDesc &D = P->desc[b];
        if (P->device_ptrs) {
            D.Q = q.queries;
            D.out_ids = q.out_ids;
            D.out_ips = q.out_ips;
        } else {
            HIPX(hipMemcpyAsync(P->q_stage[b].get(), q.queries, (size_t)D.nq * D.d * sizeof(float),
                                hipMemcpyHostToDevice, s));
            D.Q = P->q_stage[b].get();
            D.out_ids = P->id_stage[b].get();
            D.out_ips = P->ip_stage[b].get();
        }
    }
    // runs are synchronous: the previous run no longer reads the staging block
    std::memset(P->blk_h, 0, P->blk_bytes);
    std::memcpy(P->blk_h + P->desc_off, P->desc.data(), P->desc.size() * sizeof(MultiDesc));
    std::memcpy(P->blk_h + P->seg_off, P->seg.data(), P->seg.size() * sizeof(int64_t));
    std::memset(P->res_h, 0, sizeof(MultiResult));
    if (P->dirty) {
        HIPX(hipMemsetAsync(P->ws.get(), 0, P->ws_bytes, s));
        P->dirty = false;
    }
    Timer tm(s);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (launch_ms) {
        HIPX(hipEventCreate(&e0));
        HIPX(hipEventCreate(&e1));
        HIPX(hipEventRecord(e0, s));
    }
    tm.begin("multi");
    if (P->exec) HIPX(hipGraphLaunch(P->exec, s));
    else enqueue(P, s);
    tm.end();
    if (launch_ms) HIPX(hipEventRecord(e1, s));
    if (!P->device_ptrs)
        for (int b = 0; b < nb; ++b) {
            const nrlsh_query_desc &q = descs[P->active[b]];
            const MultiDesc &D = P->desc[b];
            HIPX(hipMemcpyAsync(q.out_ids, D.out_ids, (size_t)D.nq * P->k * sizeof(int64_t),
                                hipMemcpyDeviceToHost, s));
            HIPX(hipMemcpyAsync(q.out_ips, D.out_ips, (size_t)D.nq * P->k * sizeof(float),
                                hipMemcpyDeviceToHost, s));
        }
    HIPX(hipStreamSynchronize(s));
    tm.settle();
    if (launch_ms) {
        HIPX(hipEventElapsedTime(launch_ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    MultiResult r = *P->res_h;
    if (!P->persistent) r.done = 1;  // stream order: every phase has run
    if (!r.done || r.error) {
        P->dirty = true;  // counters may be left in use: clear before the next launch
        if (!r.done) return fail(NRLSH_E_DEVICE, "batching launch did not report completion");
        if (r.error & MULTI_ERR_TIMEOUT)
            return fail(NRLSH_E_DEVICE, "batching launch: a wait exceeded %.0f s", kWaitLimitSeconds);
        return fail(NRLSH_E_INTERNAL, "batching launch: a probed list did not hold min(T, n) items");
    }
    if (r.nonfinite) return fail(NRLSH_E_NOT_FINITE, "queries hold NaN or Inf");
    return NRLSH_OK;
}

nrlsh_multi_plan *create_plan(const nrlsh_query_desc *descs, int32_t count, int32_t k,
                              const PlanOpts &po, const std::vector<TileShape> &tiles)
{
    auto P = new nrlsh_multi_plan();
    try {
        P->device = descs[0].index->device;
        HIPX(hipSetDevice(P->device));
        prepare_pool(P->device);
        P->stream = po.stream ? static_cast<hipStream_t>(po.stream) : library_stream(P->device);
        P->device_ptrs = po.device_ptrs;
        P->use_graph = po.use_graph;
        P->persistent = po.persistent;
        P->k = k;
        P->count = count;
        for (int32_t i = 0; i < count; ++i) {
            P->shape.push_back(PairShape{descs[i].index, descs[i].nq, descs[i].probe_budget});
            if (descs[i].nq > 0) P->active.push_back(i);
        }
        P->tile = tiles;
        lay_out(P);
        if (P->use_graph && !P->active.empty()) capture_graph(P);
    } catch (...) {
        delete P;
        throw;
    }
    return P;
}

// Tile shape of every pair: forced by the options, from the table, or timed.
std::vector<TileShape> choose_tiles(const nrlsh_query_desc *descs, int32_t count, int32_t k,
                                    const PlanOpts &po, int32_t *tuned, double *tune_ms)
{
    std::vector<TileShape> t((size_t)count, TileShape{kDefaultChunk, kDefaultSlice});
    *tuned = 0;
    *tune_ms = 0.0;
    if (po.chunk > 0 || po.slice > 0 || po.tune == NRLSH_TUNE_DEFAULT) {
        for (auto &x : t) {
            if (po.chunk > 0) x.chunk = po.chunk;
            if (po.slice > 0) x.slice = po.slice;
        }
        return t;
    }
    std::map<ClassKey, std::vector<int32_t>> classes;
    for (int32_t i = 0; i < count; ++i)
        if (descs[i].nq > 0)
            classes[class_of(descs[i].index->d, descs[i].index->L, descs[i].nq)].push_back(i);
    const auto t0 = std::chrono::steady_clock::now();
    for (auto &kv : classes) {
        TileShape best{kDefaultChunk, kDefaultSlice};
        const bool have = table_get(kv.first, &best);
        const bool tune = po.tune == NRLSH_TUNE_ALL || (po.tune == NRLSH_TUNE_MISSING && !have);
        if (tune) {
            // the class's own pairs, timed with each candidate shape: first
            // the scan chunk at the default slice, then the slice
            std::vector<nrlsh_query_desc> sub;
            for (int32_t i : kv.second) sub.push_back(descs[i]);
            PlanOpts so = po;
            so.use_graph = false;
            so.tune = NRLSH_TUNE_DEFAULT;
            auto time_shape = [&](TileShape sh) {
                std::vector<TileShape> st(sub.size(), sh);
                nrlsh_multi_plan *P = create_plan(sub.data(), (int32_t)sub.size(), k, so, st);
                float best_ms = 1e30f;
                nrlsh_status rs = NRLSH_OK;
                for (int rep = 0; rep < 3 && rs == NRLSH_OK; ++rep) {
                    float ms = 0.f;
                    rs = run_plan(P, sub.data(), &ms);
                    if (rep > 0) best_ms = std::min(best_ms, ms);
                }
                delete P;
                if (rs != NRLSH_OK) throw Failure{rs, "autotuner run failed"};
                return best_ms;
            };
            best = TileShape{kDefaultChunk, kDefaultSlice};
            float best_ms = time_shape(best);
            for (int32_t c : {4096, 65536}) {
                const float ms = time_shape(TileShape{c, kDefaultSlice});
                if (ms < best_ms) {
                    best_ms = ms;
                    best.chunk = c;
                }
            }
            for (int32_t sl : {512, 2048, 4096}) {
                const float ms = time_shape(TileShape{best.chunk, sl});
                if (ms < best_ms) {
                    best_ms = ms;
                    best.slice = sl;
                }
            }
            table_put(kv.first, best);
            *tuned += 1;
        }
        for (int32_t i : kv.second) t[i] = best;
    }
    *tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return t;
}

bool same_shape(const nrlsh_multi_plan *P, const nrlsh_query_desc *descs, int32_t count)
{
    if (count != P->count) return false;
    for (int32_t i = 0; i < count; ++i)
        if (descs[i].index != P->shape[i].ix || descs[i].nq != P->shape[i].nq ||
            descs[i].probe_budget != P->shape[i].T)
            return false;
    return true;
}

}  // namespace

// ================================================================= C ABI
extern "C" {

nrlsh_status nrlsh_multi_plan_create(const nrlsh_query_desc *descs, int32_t count, int32_t k,
                                     const nrlsh_multi_opts *opts, nrlsh_multi_plan **out)
{
    if (!out) return fail(NRLSH_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    PlanOpts po;
    nrlsh_status st = read_opts(opts, &po);
    if (st != NRLSH_OK) return st;
    st = validate_descs(descs, count, k);
    if (st != NRLSH_OK) return st;
    return guarded([&]() -> nrlsh_status {
        HIPX(hipSetDevice(descs[0].index->device));
        for (int32_t i = 0; i < count; ++i) index_settle(descs[i].index);
        int32_t tuned = 0;
        double tune_ms = 0.0;
        const std::vector<TileShape> tiles = choose_tiles(descs, count, k, po, &tuned, &tune_ms);
        nrlsh_multi_plan *P = create_plan(descs, count, k, po, tiles);
        P->tuned_classes = tuned;
        P->tune_ms = tune_ms;
        *out = P;
        return NRLSH_OK;
    });
}

nrlsh_status nrlsh_multi_run(nrlsh_multi_plan *plan, const nrlsh_query_desc *descs, int32_t count)
{
    if (!plan) return fail(NRLSH_E_INVALID_ARG, "plan is NULL");
    nrlsh_status st = validate_descs(descs, count, plan->k);
    if (st != NRLSH_OK) return st;
    if (!same_shape(plan, descs, count))
        return fail(NRLSH_E_INVALID_ARG, "descs do not match the plan's shape (index, nq, probe budget)");
    return guarded([&]() -> nrlsh_status {
        for (int32_t i = 0; i < count; ++i) index_settle(descs[i].index);
        return run_plan(plan, descs, nullptr);
    });
}

void nrlsh_multi_plan_free(nrlsh_multi_plan *plan)
{
    if (!plan) return;
    (void)hipSetDevice(plan->device);
    delete plan;
}

nrlsh_status nrlsh_query_multi(const nrlsh_query_desc *descs, int32_t count, int32_t k,
                               const nrlsh_multi_opts *opts)
{
    nrlsh_multi_plan *P = nullptr;
    nrlsh_status st = nrlsh_multi_plan_create(descs, count, k, opts, &P);
    if (st != NRLSH_OK) return st;
    st = nrlsh_multi_run(P, descs, count);
    nrlsh_multi_plan_free(P);
    return st;
}

nrlsh_status nrlsh_multi_plan_info(const nrlsh_multi_plan *plan, nrlsh_multi_info *info,
                                   int32_t *chunk, int32_t *slice)
{
    if (!plan || !info) return fail(NRLSH_E_INVALID_ARG, "NULL argument");
    *info = nrlsh_multi_info{};
    info->grid = plan->grid;
    info->graph = plan->exec != nullptr;
    for (int ph = 0; ph < MULTI_PHASES; ++ph) info->items[ph] = plan->items[ph];
    info->tuned_classes = plan->tuned_classes;
    info->tune_ms = plan->tune_ms;
    for (int32_t i = 0; i < plan->count; ++i) {
        if (chunk) chunk[i] = plan->tile[i].chunk;
        if (slice) slice[i] = plan->tile[i].slice;
    }
    return NRLSH_OK;
}

void nrlsh_tune_clear(void)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune.clear();
}

int32_t nrlsh_tune_lookup(int32_t d, int32_t L, int64_t nq, int32_t *chunk, int32_t *slice)
{
    TileShape t;
    if (!table_get(class_of(d, L, nq), &t)) return 0;
    if (chunk) *chunk = t.chunk;
    if (slice) *slice = t.slice;
    return 1;
}

}  // extern "C"
