// Host-side plumbing shared by the translation units of libnrlsh: errors,
// per-launch timing, the library stream and stream-ordered device buffers,
// and the index object itself.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <new>
#include <string>
#include <atomic>
#include <vector>

#include "nrlsh.h"

namespace nrlsh {
namespace host {

// ================================================================= errors
// Records the thread's error text and returns st.
nrlsh_status fail(nrlsh_status st, const char *fmt, ...);

struct Failure {
    nrlsh_status st;
    std::string msg;
};

[[noreturn]] void throw_hip(hipError_t e, const char *what);

#define HIPX(call)                                      \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) throw_hip(e_, #call);     \
    } while (0)

// Runs f, turning exceptions into a status and the thread's error text.
template <typename F>
nrlsh_status guarded(F &&f)
{
    try {
        return f();
    } catch (const Failure &e) {
        return fail(e.st, "%s", e.msg.c_str());
    } catch (const std::bad_alloc &) {
        return fail(NRLSH_E_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return fail(NRLSH_E_INTERNAL, "unexpected exception");
    }
}


// ================================================================= profiling
bool prof_enabled();
void prof_record(const char *name, float ms);

// Records an event pair around each timed launch; settle() must run after the
// stream has been synchronised.
class Timer {
  public:
    explicit Timer(hipStream_t s, bool allow = true) : s_(s), on_(allow && prof_enabled()) {}
    ~Timer()
    {
        for (auto &p : pending_) {
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
    }
    void begin(const char *name)
    {
        if (!on_) return;
        Pending p;
        p.name = name;
        HIPX(hipEventCreate(&p.a));
        HIPX(hipEventCreate(&p.b));
        HIPX(hipEventRecord(p.a, s_));
        pending_.push_back(p);
    }
    void end()
    {
        if (!on_) return;
        HIPX(hipEventRecord(pending_.back().b, s_));
    }
    void settle()
    {
        if (!on_) return;
        if (!pending_.empty()) HIPX(hipEventSynchronize(pending_.back().b));
        for (auto &p : pending_) {
            float ms = 0.f;
            HIPX(hipEventElapsedTime(&ms, p.a, p.b));
            prof_record(p.name, ms);
        }
    }

  private:
    struct Pending {
        const char *name;
        hipEvent_t a, b;
    };
    hipStream_t s_;
    bool on_;
    std::vector<Pending> pending_;
};

// ================================================================= device memory
// The library's own non-blocking stream on device dev (default priority).
hipStream_t library_stream(int dev);
// Keeps freed stream-ordered memory in the device pool.
void prepare_pool(int dev);
int current_device();
// Device memory with a small cache in front of the stream-ordered allocator
// (whose calls cost tens of microseconds each): a released block is kept and
// handed out again for a request of about its size on the same stream, or on
// any stream once the work queued before its release has finished.
void *cached_alloc(size_t bytes, hipStream_t s, int *dev);
void cached_free(void *p, size_t bytes, hipStream_t s, int dev);
// Pinned host staging for small copies: a block is handed out again once an
// event recorded on the stream of its release has completed (or at once when
// released with no stream).  Blocks are kept until the process ends.
void *pinned_take(size_t bytes, size_t *got);
void pinned_give(void *p, size_t bytes, hipStream_t s, int dev);
// An idle event of device dev (timing disabled), and its return.
hipEvent_t event_take(int dev);
void event_give(hipEvent_t ev, int dev);

// Stream-ordered device buffer; freed on the stream it was allocated on.  A
// view (DBuf::view) points into memory owned elsewhere and frees nothing.
template <typename T>
struct DBuf {
    T *p = nullptr;
    hipStream_t s = nullptr;
    bool own = true;
    size_t bytes = 0;
    int dev = 0;
    DBuf() = default;
    DBuf(size_t count, hipStream_t st) : s(st)
    {
        if (count == 0) count = 1;
        bytes = count * sizeof(T);
        p = static_cast<T *>(cached_alloc(bytes, st, &dev));
    }
    static DBuf view(T *ptr)
    {
        DBuf b;
        b.p = ptr;
        b.own = false;
        return b;
    }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), s(o.s), own(o.own), bytes(o.bytes), dev(o.dev) { o.p = nullptr; }
    DBuf &operator=(DBuf &&o) noexcept
    {
        reset();
        p = o.p;
        s = o.s;
        own = o.own;
        bytes = o.bytes;
        dev = o.dev;
        o.p = nullptr;
        return *this;
    }
    ~DBuf() { reset(); }
    void reset()
    {
        if (p && own) cached_free(p, bytes, s, dev);
        p = nullptr;
    }
    T *get() const { return p; }
};

// Several buffers carved from one stream-ordered allocation: each
// stream-ordered allocation and release costs tens of microseconds of host
// time, so a call reserves all of its buffers, allocates once and takes
// views (valid while the Block lives).
class Block {
  public:
    template <typename T>
    size_t reserve(size_t count)
    {
        const size_t off = (size_ + 255) / 256 * 256;
        size_ = off + (count ? count : 1) * sizeof(T);
        return off;
    }
    void allocate(hipStream_t s) { mem = DBuf<uint8_t>(size_ ? size_ : 1, s); }
    // Carves the reserved buffers out of caller-owned memory of `cap` bytes
    // (256-byte aligned) instead of allocating; false if they do not fit.
    bool place(uint8_t *base, size_t cap)
    {
        if (size_ > cap) return false;
        mem = DBuf<uint8_t>::view(base);
        return true;
    }
    size_t size() const { return size_; }
    template <typename T>
    DBuf<T> view(size_t off) const
    {
        return DBuf<T>::view(reinterpret_cast<T *>(mem.get() + off));
    }
    DBuf<uint8_t> mem;

  private:
    size_t size_ = 0;
};

}  // namespace host
}  // namespace nrlsh

// ================================================================= the index
struct nrlsh_index {
    int device = 0;
    int64_t n = 0;
    int32_t d = 0, dp = 0, m = 0, L = 0, W = 1;
    uint64_t seed = 0;
    double eps = 0.0;
    int32_t storage = NRLSH_STORAGE_FP32, margin_mode = NRLSH_MARGIN_RIGOROUS;
    double margin_param = 0.0;
    int32_t partition = NRLSH_PARTITION_PERCENTILE;
    int32_t qsets = 1;  // projection blocks of L rows per table: 1 (shared) or m (one per sub-dataset)
    int32_t tables = 1; // independent hash tables (codes_l holds tables x n x W words)
    std::vector<float> A_h;
    std::vector<double> keymax_h, U_h;
    std::vector<int64_t> off_h;
    std::vector<int32_t> R_h;
    // sub-datasets by (U_j desc, j desc): the order in which the staged scan
    // visits them (every bucket of a later one ranks after the first bucket
    // (jord_h[i], L) of the earlier ones not yet visited)
    std::vector<int32_t> jord_h;
    // the build's last device work (queued, not waited for, when nrlsh_build
    // returns): later calls wait for `ready` on their stream or on the host;
    // the build counters arrive in pinned host memory behind it
    mutable hipEvent_t ready = nullptr;
    mutable std::mutex ready_mu;
    mutable std::atomic<bool> settled{false};
    void *counters_h = nullptr;  // pinned BuildCounters
    size_t counters_bytes = 0;
    mutable nrlsh_build_stats stats{};
    hipStream_t home = nullptr;  // library stream that releases the device buffers
    nrlsh::host::Block mem;      // the long-lived buffers below are views into it
    nrlsh::host::DBuf<float> Xl, A, At;               // Xl: stored-order padded item copy
    nrlsh::host::DBuf<uint16_t> Xh;                   // its bfloat16 image (hi part)
    // lo part x - hi (bfloat16), made on the first query that needs it
    mutable nrlsh::host::DBuf<uint16_t> Xlo;
    mutable std::mutex lo_mu;
    mutable std::atomic<bool> lo_ready{false};
    // witnesses of the dense head (made on the first query that screens one):
    // per sub-dataset its wit_per_sub largest-norm items, positions in stored
    // order and compact copies of their bfloat16 rows, codes and keys
    mutable std::mutex wit_mu;
    mutable std::atomic<bool> wit_ready{false};
    mutable int32_t wit_per_sub = 0;
    mutable std::vector<int32_t> wit_cnt_h;
    mutable nrlsh::host::DBuf<int32_t> wit_pos, wit_cnt;
    mutable nrlsh::host::DBuf<uint16_t> wit_xh;
    mutable nrlsh::host::DBuf<uint32_t> wit_codes;
    mutable nrlsh::host::DBuf<double> wit_key;
    // the dense head chosen from the sample of the last call that measured
    // one, reused by later calls with the same k, budget and fraction (a speed
    // hint only; results never depend on it)
    mutable std::mutex head_mu;
    mutable bool head_hint_valid = false;
    mutable int32_t head_hint_k = 0, head_hint_j0 = 0, head_hint_j1 = 0, head_hint_split = 1;
    mutable int64_t head_hint_T = 0;
    mutable double head_hint_frac = 0.0;
    nrlsh::host::DBuf<uint8_t> Xf8;                   // FP8 E4M3 hash copy (precision form)
    nrlsh::host::DBuf<float> xscale;                  // its row scales
    nrlsh::host::DBuf<double> key, key_l, keymax, U;  // key: original order; key_l: stored order
    nrlsh::host::DBuf<int32_t> sid, sid_l, perm, off, R, inv;
    nrlsh::host::DBuf<uint32_t> codes_l;              // stored order
    nrlsh::host::DBuf<float> xeb;  // per stored row: bound on ||x - bf16(x)|| (+ FP64 sum term)
    // rank table of the (sub-dataset, first-table) bins of the multi-table
    // single probe, m x tables (level index tables - 1 - f), and its inverse
    std::vector<int32_t> Rs_h;
    nrlsh::host::DBuf<int32_t> Rs, invs;
    // staged-scan plan of one 64-query tile (chunk triples, stage starts, cut
    // ranks), read by the query entry point that allocates nothing
    std::vector<int32_t> st1_chunks;
    std::vector<int> st1_cbeg, st1_cut;
    nrlsh::host::DBuf<int32_t> st1_chunks_d;
    // (k, Tq) of the last call whose bfloat16 re-rank lists overflowed, packed
    // k << 32 | Tq (0: none): calls with at least that k and budget skip the
    // bfloat16 pass (a speed hint only; results never depend on it)
    mutable std::atomic<uint64_t> lp_overflow{0};
    // bucket tables (built on request): distinct codes of each sub-dataset
    bool has_table = false;
    int64_t nunique = 0;
    std::vector<int64_t> uoff_h;
    nrlsh::host::DBuf<uint64_t> ucode, binom;
    nrlsh::host::DBuf<int32_t> ustart, uoff, titem;
};

// The build returns with its last kernels still queued: index_wait makes
// stream s wait for them, index_settle waits on the host (and takes the
// build counters in).
void index_wait(const nrlsh_index *ix, hipStream_t s);
void index_settle(const nrlsh_index *ix);

