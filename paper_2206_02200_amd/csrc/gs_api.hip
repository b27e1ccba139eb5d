// Host side of the GridShift library: context, buffers, the fit pipelines and
// the C ABI declared in include/gridshift.h.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gridshift.h"
#include "gs_kernels.inl"

namespace {

thread_local std::string g_last_error;

gs_status fail(gs_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

#define GS_HIP(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(GS_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));        \
    } while (0)

struct DBuf {
    void* p = nullptr;
    size_t cap = 0;
    const gs_allocator* al = nullptr;  // the caller's allocator that gave p (null: hipMalloc)
    void* st = nullptr;                // and the stream it was given for
    bool arena = false;                // carved from an arena chunk (given back with the arena)
};

// Device memory of a result: a few large chunks from the caller's allocator,
// each new one at least as large as all before it, carved in order; nothing
// is given back before the result is released (then every chunk at once).
struct Arena {
    struct Chunk {
        char* p;
        size_t cap, used;
        void* stream;  // the stream it was allocated for
    };
    std::vector<Chunk> chunks;
    size_t total = 0;
};

// Device memory of a call on a context with a caller allocator comes from
// that allocator: the entry point opens an AllocScope, and every buffer grown
// during the call records where its memory came from.
thread_local const gs_allocator* t_alloc = nullptr;
thread_local void* t_alloc_stream = nullptr;
thread_local Arena* t_arena = nullptr;

constexpr size_t kArenaMinChunk = size_t(32) << 20;

void* arena_get(Arena& a, size_t bytes) {
    const size_t need = (bytes + 255) & ~size_t(255);
    if (!a.chunks.empty()) {
        Arena::Chunk& c = a.chunks.back();
        if (c.cap - c.used >= need) {
            void* p = c.p + c.used;
            c.used += need;
            return p;
        }
    }
    const size_t want = std::max(need, std::max(kArenaMinChunk, a.total));
    void* p = t_alloc->alloc(t_alloc->ctx, want, t_alloc_stream);
    if (!p) return nullptr;
    a.chunks.push_back({static_cast<char*>(p), want, need, t_alloc_stream});
    a.total += want;
    return p;
}

void dbuf_release(DBuf& b) {
    if (b.p && !b.arena) {
        if (b.al)
            b.al->free(b.al->ctx, b.p, b.st);
        else
            (void)hipFree(b.p);
    }
    b.p = nullptr;
    b.cap = 0;
    b.al = nullptr;
    b.st = nullptr;
    b.arena = false;
}

gs_status dbuf_get(DBuf& b, size_t want) {
    void* p = nullptr;
    if (t_alloc && t_arena) {
        p = arena_get(*t_arena, want);
        if (!p)
            return fail(GS_ERR_ALLOC, "the caller's allocator returned NULL (" + std::to_string(want) +
                                          " more bytes of device memory wanted)");
        b.p = p;
        b.cap = want;
        b.al = nullptr;
        b.st = nullptr;
        b.arena = true;
        return GS_OK;
    }
    if (t_alloc) {
        p = t_alloc->alloc(t_alloc->ctx, want, t_alloc_stream);
        if (!p) return fail(GS_ERR_ALLOC, "the caller's allocator returned NULL for " + std::to_string(want) + " bytes");
    } else if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GS_ERR_ALLOC, "hipMalloc of " + std::to_string(want) + " bytes failed");
    }
    b.p = p;
    b.cap = want;
    b.al = t_alloc;
    b.st = t_alloc_stream;
    return GS_OK;
}

// Optional per-kernel timing with HIP events on the launch stream.  Only
// kernels whose name starts with `filter` are timed.
struct Profiler {
    bool on = false;
    std::string filter;
    std::vector<hipEvent_t> ev;
    size_t next = 0;
    struct Rec {
        int id;
        size_t e0, e1;
        double bytes;
    };
    std::vector<Rec> recs;
    std::vector<std::string> names;
    std::vector<double> ms, bytes;
    std::vector<int64_t> launches;
};

}  // namespace

// Launch choices; every choice runs the same binary64 operations in the same
// order, so results never depend on them (only the speed does).
struct gs_config {
    int merge_small = 1;  // merge rounds of at most kMergeMax cells in one workgroup
    int tile_chunks = 4;  // staged chunks of point rows per point tile
    int dense_table = 1;  // neighbour lookups through a dense key table when the key range allows
    int sort_digit10 = 0;  // radix sorts use 10-bit digits where that saves a pass (else 8-bit)
    int sort_tile = 8192;  // keys per radix-sort pass tile (8192 or 4096)
};

struct gs_context {
    int device = 0;
    int rule = GS_UPDATE_PARALLEL;  // update rule of the shift (gs_context_set_update)
    gs_allocator alloc{};           // the caller's device allocator (has_alloc), else hipMalloc
    bool has_alloc = false;
    bool use_arena = false;         // with has_alloc: buffers carved from `arena` (results)
    Arena arena;
    bool stage_pooled = false;      // the host staging below returns to the per-device pool
    void* own_stream = nullptr;     // with has_alloc: allocate for this stream whatever the call's stream
    bool has_own_stream = false;
    int tail_tok = -1;              // profiling record of the last tail launch
    DBuf seq_moved, seq_waiting;    // sequential form: step stamps per cell, waiting flags per step
    uint32_t seq_epoch = 0;
    // point level
    DBuf kA, kB, vA, vB, cell0;
    DBuf kpt;  // keys in point order, kept through the sort when the cells of the points are looked up
    int fit_sets = 1;  // point sets (instances) of the fit in progress
    // cell tables (ping-pong) and per-round scratch
    DBuf tkey[2], tcnt[2], tsum[2], tinst[2], tstart[2], tlen[2], tfirst[2], tnch[2], tchoff[2];
    DBuf kappa, pbuf, gmap, cur, tmap, part, partc, hk, hv, ckA, ckB, cvA, cvB;
    // instances
    // Control block: one allocation holding, in this order, the boxes, the
    // counters, the instance states, the cluster row offsets, the row
    // offsets, the bandwidths, the row tiles and the packing parameters; the
    // views below point into it.  Its
    // part before the parameters is uploaded in one copy at the start of a
    // fit, and boxes + counters and counters + states are read back in one
    // copy each.
    DBuf ctl;
    DBuf param, state, koff, rowoff, hs, bbox, counters, tiles;  // views into ctl (never allocated or freed)
    std::vector<char> ctl_img;                             // host image of the uploaded part
    bool hist_dirty = true;                                // sort histograms may hold stale counts
    int64_t ntiles = 0;
    // scans and sorts
    DBuf look, tilectr, shist, sctr, slook;
    gs::SortScratch sort;
    uint32_t scan_epoch = 0;
    uint64_t tile_base = 0;  // value of the scan tile counter before the next scan
    gs_config cfg;           // launch choices (results do not depend on them)
    DBuf tune_labels;        // labels of the autotuner's timed fits
    DBuf tune_ref, tune_tab; // the first candidate's labels; cluster tables compared across candidates
    bool tune_hit = false;   // the last gs_autotune took its choice from the cache
    DBuf dk;                 // dense key -> cell table of the device-wide rounds
    uint32_t dk_epoch = 0;
    int64_t key_span = 0;    // packed key range of the current fit
    bool wide_crd = false;   // some key-box extent is 2^31 or more: the tail keeps 64-bit coordinates
    // pinned staging: downloads (every one waits for its stream) and a bump
    // area for uploads, reused only once a wait on up_stream has drained them
    void* pinned = nullptr;
    size_t pinned_cap = 0;
    char* up = nullptr;
    size_t up_cap = 0, up_used = 0;
    hipStream_t up_stream = nullptr;
    // result of the last fit
    bool has_result = false;
    int B = 0, d = 0, cur_tab = 0;
    int64_t capM = 0;
    std::vector<gs::InstState> st;
    std::vector<gs::InstParam> prm;
    Profiler prof;
    // differentiable form: trajectory tape of the last fit
    bool tape_on = false, tape_valid = false;
    int ckpt_every = 0;  // 0 or 1: every tail round recorded; k > 1: tail checkpoints every k rounds
    int ckpt_used = 0;   // the setting the last fit was recorded with
    DBuf ck_key, ck_cnt, ck_sum, ck_m;
    int ck_nslots = 0;
    DBuf sums0, inst0, wt_key, wt_cnt, wt_inst, wt_W, wt_g, wt_app;
    int64_t sweep_n = 0;  // during a bandwidth sweep: the instances share the first n rows of the points
    DBuf trk_win, trk_lab, trk_cnt, trk_sel, trk_out, trk_rect, trk_init;  // tracking buffers
    DBuf tt_key, tt_cnt, tt_W, tt_g, tt_m;
    // backward with checkpoints: a second stream recomputes the next (earlier)
    // tape segment while the current one is reversed (two tape buffers)
    hipStream_t aux = nullptr;
    // host memory mapped for the device: [counters 8][states B], written by
    // the kernel that ends a step the host waits for (no copy back)
    int64_t* hmap = nullptr;      // host view
    int64_t* hmap_dev = nullptr;  // device view
    size_t hmap_cap = 0;
    // a context over fixed memory (gs_fit_noalloc): the staging areas and the
    // published block are never reallocated, and the published block is
    // device memory that the host copies back after each wait
    bool fixed_host = false;
    bool hmap_on_device = false;
    hipEvent_t ev_start = nullptr, ev_rep[2] = {nullptr, nullptr}, ev_adj[2] = {nullptr, nullptr};
    DBuf sbA, sbB, qbuf, gmodes, modes_i, counts_i, frows, lossc, ltab;
    DBuf xkA, xkB, xvA, xvB;
    std::vector<int64_t> w_off, w_M;
    int64_t wt_used = 0;
    int tail_rounds = 0, wide_rounds = 0, dtype = 0, sort_bits = 0;
    int64_t N = 0, ld = 0, m0 = 0;
};

// The caller allocator of a context, for the duration of one entry point.
struct AllocScope {
    const gs_allocator* pa;
    void* ps;
    Arena* pr;
    AllocScope(gs_context* c, void* stream) : pa(t_alloc), ps(t_alloc_stream), pr(t_arena) {
        t_alloc = c && c->has_alloc ? &c->alloc : nullptr;
        t_alloc_stream = c && c->has_alloc ? (c->has_own_stream ? c->own_stream : stream) : nullptr;
        t_arena = c && c->has_alloc && c->use_arena ? &c->arena : nullptr;
    }
    ~AllocScope() {
        t_alloc = pa;
        t_alloc_stream = ps;
        t_arena = pr;
    }
};

namespace {

gs_status ensure(DBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (b.cap >= bytes) return GS_OK;
    dbuf_release(b);
    return dbuf_get(b, bytes + bytes / 8);
}

// Grow a buffer keeping its first `used` bytes (stream-ordered copy).
gs_status ensure_keep(DBuf& b, size_t bytes, size_t used, hipStream_t s) {
    if (b.cap >= bytes) return GS_OK;
    const size_t want = bytes + bytes / 2;
    DBuf nb;
    if (const gs_status e = dbuf_get(nb, want); e != GS_OK) return e;
    if (b.p && used) {
        if (hipMemcpyAsync(nb.p, b.p, used, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            dbuf_release(nb);
            return fail(GS_ERR_DEVICE, "tape copy failed");
        }
    }
    dbuf_release(b);
    b = nb;
    b.cap = want;
    return GS_OK;
}

#define GS_TRY(expr)                  \
    do {                              \
        gs_status s_ = (expr);        \
        if (s_ != GS_OK) return s_;   \
    } while (0)

template <typename T>
T* P(DBuf& b) {
    return static_cast<T*>(b.p);
}

// Grid size for n items (at least one block, so that empty launches are valid).
inline unsigned blocks_for(int64_t n, int threads) {
    return n <= 0 ? 1u : unsigned((n + threads - 1) / threads);
}

int prof_begin(gs_context* c, hipStream_t s, const char* name) {
    Profiler& p = c->prof;
    if (!p.on || std::strncmp(name, p.filter.c_str(), p.filter.size()) != 0) return -1;
    int id = -1;
    for (size_t i = 0; i < p.names.size(); ++i)
        if (p.names[i] == name) id = int(i);
    if (id < 0) {
        id = int(p.names.size());
        p.names.emplace_back(name);
        p.ms.push_back(0.0);
        p.bytes.push_back(0.0);
        p.launches.push_back(0);
    }
    while (p.ev.size() < p.next + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        p.ev.push_back(e);
    }
    const size_t e0 = p.next++, e1 = p.next++;
    if (hipEventRecord(p.ev[e0], s) != hipSuccess) return -1;
    p.recs.push_back({id, e0, e1, 0.0});
    return int(p.recs.size() - 1);
}

void prof_end(gs_context* c, hipStream_t s, int tok, double bytes) {
    if (tok < 0) return;
    Profiler& p = c->prof;
    (void)hipEventRecord(p.ev[p.recs[tok].e1], s);
    p.recs[tok].bytes = bytes;
}

// Algorithmic bytes of a recorded launch, once the host knows them.
void prof_set_bytes(gs_context* c, int tok, double bytes) {
    if (tok >= 0 && size_t(tok) < c->prof.recs.size()) c->prof.recs[tok].bytes = bytes;
}

// Accumulate the recorded intervals (waiting for the last of them first).
void prof_flush(gs_context* c, bool keep) {
    Profiler& p = c->prof;
    if (keep && !p.recs.empty()) (void)hipEventSynchronize(p.ev[p.recs.back().e1]);
    if (keep) {
        for (const Profiler::Rec& r : p.recs) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, p.ev[r.e0], p.ev[r.e1]) == hipSuccess) {
                p.ms[r.id] += ms;
                p.bytes[r.id] += r.bytes;
                p.launches[r.id] += 1;
            }
        }
    }
    p.recs.clear();
    p.next = 0;
}

int sort_prof_begin(void* ctx, hipStream_t s, const char* name) {
    return prof_begin(static_cast<gs_context*>(ctx), s, name);
}
void sort_prof_end(void* ctx, hipStream_t s, int tok, double bytes) {
    prof_end(static_cast<gs_context*>(ctx), s, tok, bytes);
}

#define PROF_LAUNCH(name, nbytes, ...)                 \
    do {                                              \
        const int tk_ = prof_begin(c, s, name);       \
        __VA_ARGS__;                                  \
        prof_end(c, s, tk_, double(nbytes));          \
    } while (0)

gs_status pinned_ensure(gs_context* c, size_t bytes) {
    if (c->pinned_cap >= bytes) return GS_OK;
    if (c->fixed_host)
        return fail(GS_ERR_INVALID_ARG, "a download of " + std::to_string(bytes) + " bytes exceeds the fixed staging");
    if (c->pinned) (void)hipHostFree(c->pinned);
    c->pinned = nullptr;
    c->pinned_cap = 0;
    if (hipHostMalloc(&c->pinned, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GS_ERR_ALLOC, "hipHostMalloc failed");
    }
    c->pinned_cap = bytes;
    return GS_OK;
}

// Wait for stream s; uploads staged on it are then complete.
gs_status stream_wait(gs_context* c, hipStream_t s) {
    GS_HIP(hipStreamSynchronize(s));
    if (c->up_stream == s) c->up_used = 0;
    return GS_OK;
}

// Copy device -> host through pinned memory and wait for the stream.
gs_status d2h(gs_context* c, void* dst, const void* src, size_t bytes, hipStream_t s) {
    GS_TRY(pinned_ensure(c, bytes));
    GS_HIP(hipMemcpyAsync(c->pinned, src, bytes, hipMemcpyDeviceToHost, s));
    GS_TRY(stream_wait(c, s));
    std::memcpy(dst, c->pinned, bytes);
    return GS_OK;
}

// Host -> device copy staged in the upload area; returns without waiting
// (the staged bytes stay untouched until a wait has drained the copy).
gs_status h2d(gs_context* c, void* dst, const void* src, size_t bytes, hipStream_t s) {
    const size_t need = (bytes + 255) & ~size_t(255);
    if (c->up_used > 0 && c->up_stream != s) {
        GS_HIP(hipStreamSynchronize(c->up_stream));
        c->up_used = 0;
    }
    if (c->up_used + need > c->up_cap) {
        if (c->up_used > 0) GS_TRY(stream_wait(c, s));
        c->up_used = 0;
        if (need > c->up_cap) {
            if (c->fixed_host)
                return fail(GS_ERR_INVALID_ARG,
                            "an upload of " + std::to_string(bytes) + " bytes exceeds the fixed staging");
            if (c->up) (void)hipHostFree(c->up);
            c->up = nullptr;
            c->up_cap = 0;
            const size_t want = std::max<size_t>(need, size_t(1) << 16);
            void* p = nullptr;
            if (hipHostMalloc(&p, want) != hipSuccess) {
                (void)hipGetLastError();
                return fail(GS_ERR_ALLOC, "hipHostMalloc failed");
            }
            c->up = static_cast<char*>(p);
            c->up_cap = want;
        }
    }
    char* stage = c->up + c->up_used;
    std::memcpy(stage, src, bytes);
    GS_HIP(hipMemcpyAsync(dst, stage, bytes, hipMemcpyHostToDevice, s));
    c->up_used += need;
    c->up_stream = s;
    return GS_OK;
}

struct Xfer {
    void* dev;
    const void* host;
    size_t bytes;
};

// Several host -> device copies, none waited for.
gs_status h2d_batch(gs_context* c, const std::vector<Xfer>& xs, hipStream_t s) {
    for (const Xfer& x : xs) GS_TRY(h2d(c, x.dev, x.host, x.bytes, s));
    return GS_OK;
}

// Host memory mapped for the device, for `B` published states.
gs_status hmap_ensure(gs_context* c, int B) {
    const size_t bytes = 8 * sizeof(int64_t) + sizeof(gs::InstState) * size_t(B);
    if (c->hmap_cap >= bytes) return GS_OK;
    if (c->fixed_host) return fail(GS_ERR_INVALID_ARG, "the fixed published block is too small for the instances");
    if (c->hmap) (void)hipHostFree(c->hmap);
    c->hmap = nullptr;
    c->hmap_dev = nullptr;
    c->hmap_cap = 0;
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocMapped) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GS_ERR_ALLOC, "hipHostMalloc (mapped) failed");
    }
    void* dp = nullptr;
    if (hipHostGetDevicePointer(&dp, p, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(p);
        return fail(GS_ERR_ALLOC, "hipHostGetDevicePointer failed");
    }
    c->hmap = static_cast<int64_t*>(p);
    c->hmap_dev = static_cast<int64_t*>(dp);
    c->hmap_cap = bytes;
    return GS_OK;
}

// Wait for the stream; afterwards the first `bytes` of the published block
// are readable at c->hmap (copied back when the block is device memory).
gs_status published_pull(gs_context* c, size_t bytes, hipStream_t s) {
    if (c->hmap_on_device) GS_HIP(hipMemcpyAsync(c->hmap, c->hmap_dev, bytes, hipMemcpyDeviceToHost, s));
    return stream_wait(c, s);
}

// Wait for the stream, then read the counters and states a kernel published
// into the mapped host memory.
gs_status read_published(gs_context* c, int64_t* ctrs, hipStream_t s) {
    GS_TRY(published_pull(c, 8 * sizeof(int64_t) + c->state.cap, s));
    std::memcpy(ctrs, c->hmap, 8 * sizeof(int64_t));
    std::memcpy(c->st.data(), c->hmap + 8, c->state.cap);
    return GS_OK;
}

// Several device -> host copies with one wait.
gs_status d2h_batch(gs_context* c, const std::vector<Xfer>& xs, hipStream_t s) {
    size_t total = 0;
    for (const Xfer& x : xs) total += (x.bytes + 255) & ~size_t(255);
    GS_TRY(pinned_ensure(c, total));
    size_t off = 0;
    for (const Xfer& x : xs) {
        GS_HIP(hipMemcpyAsync(static_cast<char*>(c->pinned) + off, x.host, x.bytes, hipMemcpyDeviceToHost, s));
        off += (x.bytes + 255) & ~size_t(255);
    }
    GS_TRY(stream_wait(c, s));
    off = 0;
    for (const Xfer& x : xs) {
        std::memcpy(x.dev, static_cast<char*>(c->pinned) + off, x.bytes);
        off += (x.bytes + 255) & ~size_t(255);
    }
    return GS_OK;
}

__global__ void k_fill_u64(uint64_t* __restrict__ p, int64_t n, uint64_t v) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_set_i64(int64_t* __restrict__ p, int64_t v) { *p = v; }
// Count of positions where two word arrays differ (added to *diff).
__global__ void k_count_diff_u32(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b, int64_t n,
                                 int64_t* __restrict__ diff) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool ne = i < n && a[i] != b[i];
    if (__ballot(ne) && gs::lane_id() == 0) atomicAdd(reinterpret_cast<unsigned long long*>(diff), 1ull);
}

__global__ void k_iota32(uint32_t* __restrict__ p, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = uint32_t(i);
}

// Look-back storage of the tile scans: tiles status words, cleared on growth.
// Tiles take their index from a counter that is never reset per scan: every
// block of a scan increments it once, so the host knows its value before the
// next scan (tile_base) and clears it only when it nears overflow.
gs_status scan_prepare(gs_context* c, int64_t n_bound, hipStream_t s, uint32_t* epoch_out) {
    const int64_t tiles = std::max<int64_t>(1, (n_bound + gs::kScanTile - 1) / gs::kScanTile);
    if (c->look.cap < size_t(tiles) * 8) {
        GS_TRY(ensure(c->look, size_t(tiles) * 8));
        k_fill_u64<<<blocks_for(c->look.cap / 8, 256), 256, 0, s>>>(P<uint64_t>(c->look), c->look.cap / 8, 0);
        c->scan_epoch = 0;
    }
    if (c->tilectr.cap == 0 || c->tile_base + uint64_t(tiles) >= 0x7fffffffull) {
        GS_TRY(ensure(c->tilectr, 64));
        k_fill_u32<<<1, 64, 0, s>>>(P<uint32_t>(c->tilectr), 16, 0);
        c->tile_base = 0;
    }
    if (c->scan_epoch >= 0xffffu) {
        k_fill_u64<<<blocks_for(c->look.cap / 8, 256), 256, 0, s>>>(P<uint64_t>(c->look), c->look.cap / 8, 0);
        c->scan_epoch = 0;
    }
    *epoch_out = ++c->scan_epoch;
    return GS_OK;
}

// n_dev: the length on the device, or nullptr when it is n_bound itself.
template <class Op>
gs_status run_scan(gs_context* c, Op op, const int64_t* n_dev, int64_t n_bound, int64_t* total_dev, hipStream_t s,
                   const char* name, double nbytes, int64_t* total_host = nullptr) {
    uint32_t epoch = 0;
    GS_TRY(scan_prepare(c, n_bound, s, &epoch));
    const int64_t tiles = std::max<int64_t>(1, (n_bound + gs::kScanTile - 1) / gs::kScanTile);
    const uint32_t base = uint32_t(c->tile_base);
    c->tile_base += uint64_t(tiles);
    PROF_LAUNCH(name, nbytes,
                gs::k_scan<Op><<<unsigned(tiles), gs::kScanThreads, 0, s>>>(op, n_dev, n_bound, P<uint64_t>(c->look),
                                                                            P<uint32_t>(c->tilectr), base, epoch,
                                                                            total_dev, total_host));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        c->tile_base = 0x7fffffffull;  // the counter is unknown now: clear it before the next scan
        return fail(GS_ERR_DEVICE, std::string("scan launch failed: ") + hipGetErrorString(e));
    }
    return GS_OK;
}

gs::CellTable table(gs_context* c, int i) {
    gs::CellTable t;
    t.key = P<uint64_t>(c->tkey[i]);
    t.cnt = P<int64_t>(c->tcnt[i]);
    t.sum = P<double>(c->tsum[i]);
    t.inst = P<int32_t>(c->tinst[i]);
    t.start = P<uint32_t>(c->tstart[i]);
    t.len = P<uint32_t>(c->tlen[i]);
    t.first = P<uint32_t>(c->tfirst[i]);
    t.nch = P<uint32_t>(c->tnch[i]);
    t.choff = P<uint32_t>(c->tchoff[i]);
    t.cap = c->capM;
    return t;
}

// Canonical sums R of every cell's members (cells [0, m) of t, m on device).
// With have_choff the chunk offsets and the task count (counters[1]) are
// already on the device.
template <int D, class Src>
gs_status segsum_d(gs_context* c, Src src, gs::CellTable t, int64_t m_bound, int64_t npos, hipStream_t s,
                   double member_bytes, bool have_choff, bool bin) {
    // several point sets: each XCD sums a contiguous range of chunk tasks, so
    // that the members of one set are gathered through one L2 (measured on
    // the 256-image batch: binning sums 1.655 -> 1.526 ms; a single set of
    // points in random order was slower this way, so one set keeps the
    // round-robin order)
    const int xcd = c->fit_sets > 1 ? 1 : 0;
    int64_t* ctr = P<int64_t>(c->counters);
    if (!have_choff)
        GS_TRY(run_scan(c, gs::ExclOp{t.nch, t.choff}, ctr + 0, m_bound, ctr + 1, s,
                        bin ? "bin_scan_chunks" : "scan_chunks", 8.0 * m_bound));
    const int64_t tasks_bound = npos / gs::kChunk + m_bound + 1;
    GS_TRY(ensure(c->part, size_t(tasks_bound) * D * sizeof(double)));
    GS_TRY(ensure(c->partc, size_t(tasks_bound) * sizeof(int64_t)));
    // members are read once (index + value); every cell row is written once
    PROF_LAUNCH(bin ? "bin_segsum_chunks" : "segsum_chunks", npos * member_bytes + m_bound * (8.0 * D + 8.0),
                gs::k_segsum_chunks<D, Src><<<blocks_for(tasks_bound * gs::kWave, gs::kSegThreads), gs::kSegThreads,
                                              0, s>>>(src, t, ctr + 0, ctr + 1, P<double>(c->part),
                                                      P<int64_t>(c->partc), tasks_bound, xcd));
    PROF_LAUNCH(bin ? "bin_segsum_levels" : "segsum_levels", 0.0,
                gs::k_segsum_levels<D><<<blocks_for(m_bound * gs::kWave, gs::kSegThreads), gs::kSegThreads, 0, s>>>(
                    t, ctr + 0, P<double>(c->part), P<int64_t>(c->partc), tasks_bound));
    GS_HIP(hipGetLastError());
    return GS_OK;
}

template <class Src>
gs_status segsum(gs_context* c, int d, Src src, gs::CellTable t, int64_t m_bound, int64_t npos, hipStream_t s,
                 double member_bytes, bool have_choff = false, bool bin = false) {
    switch (d) {
        case 1: return segsum_d<1>(c, src, t, m_bound, npos, s, member_bytes, have_choff, bin);
        case 2: return segsum_d<2>(c, src, t, m_bound, npos, s, member_bytes, have_choff, bin);
        case 3: return segsum_d<3>(c, src, t, m_bound, npos, s, member_bytes, have_choff, bin);
        case 4: return segsum_d<4>(c, src, t, m_bound, npos, s, member_bytes, have_choff, bin);
        case 5: return segsum_d<5>(c, src, t, m_bound, npos, s, member_bytes, have_choff, bin);
        case 6: return segsum_d<6>(c, src, t, m_bound, npos, s, member_bytes, have_choff, bin);
    }
    return fail(GS_ERR_UNSUPPORTED, "d must be in 1..6");
}

// Point gradients: Sbar of the initial cell, plus (x != nullptr: the loss's
// gradient) the direct term of the point-to-mode loss.
template <typename T>
gs_status launch_adj_points(gs_context* c, int d, const double* sb0, double* grad, const T* x,
                            const int32_t* labels, const double* gloss, hipStream_t s) {
    const unsigned g = blocks_for(c->N, 256);
    const double* modes = x ? P<double>(c->modes_i) : nullptr;
    const int64_t* row_off = x ? P<int64_t>(c->rowoff) : nullptr;
    const int64_t* koff = x ? P<int64_t>(c->koff) : nullptr;
    const uint32_t* cell0 = P<uint32_t>(c->cell0);
#define GS_AP(DD)                                                                                             \
    case DD:                                                                                                   \
        gs::k_adj_points<T, DD><<<g, 256, 0, s>>>(cell0, sb0, c->capM, c->N, grad, x, c->ld, labels, modes,   \
                                                 row_off, koff, c->B, gloss);                                \
        break;
    switch (d) {
        GS_AP(1) GS_AP(2) GS_AP(3) GS_AP(4) GS_AP(5) GS_AP(6)
        default: return fail(GS_ERR_UNSUPPORTED, "d must be in 1..6");
    }
#undef GS_AP
    GS_HIP(hipGetLastError());
    return GS_OK;
}

// Look-back storage of the radix sort for n keys of `bits` bits (grown and
// cleared when too small).
gs_status sort_look_ensure(gs_context* c, int64_t n, int bits, hipStream_t s) {
    const int64_t words = gs::sort_look_words(n, bits);
    if (c->slook.cap < size_t(words) * 8) {
        GS_TRY(ensure(c->slook, size_t(words) * 8));
        k_fill_u64<<<blocks_for(c->slook.cap / 8, 256), 256, 0, s>>>(P<uint64_t>(c->slook), c->slook.cap / 8, 0);
        GS_HIP(hipGetLastError());
        c->sort.epoch = 0;
    }
    c->sort.look = P<uint64_t>(c->slook);
    c->sort.look_words = int64_t(c->slook.cap / 8);
    return GS_OK;
}

// Ready the dense key table for one more table (allocated and cleared on
// first use or growth, cleared again before the epochs wrap) and hand out a
// new epoch for its entries (c->dk_epoch is the last one handed out, so an
// epoch reserved for a table that never got its round is never reused).
// Stream-ordered: a clear here comes after every lookup of the rounds before.
gs_status dense_reserve(gs_context* c, hipStream_t s, uint32_t* next) {
    if (c->dk.cap < size_t(c->key_span) * 8) {
        GS_TRY(ensure(c->dk, size_t(c->key_span) * 8));
        k_fill_u64<<<blocks_for(c->dk.cap / 8, 256), 256, 0, s>>>(P<uint64_t>(c->dk), c->dk.cap / 8, 0);
        c->dk_epoch = 0;
    }
    if (c->dk_epoch == 0xffffffffu) {
        k_fill_u64<<<blocks_for(c->dk.cap / 8, 256), 256, 0, s>>>(P<uint64_t>(c->dk), c->dk.cap / 8, 0);
        c->dk_epoch = 0;
    }
    *next = ++c->dk_epoch;
    GS_HIP(hipGetLastError());
    return GS_OK;
}

template <class Lookup>
gs_status launch_shift(gs_context* c, int d, gs::CellTable t, int64_t m, const gs::InstParam* prm, gs::InstState* st,
                       Lookup lk, double* pbuf, uint64_t* kappa, int32_t* Wout, hipStream_t s) {
    const unsigned g = blocks_for(m, gs::kShiftWaves);  // one wave per cell
    // the parallel form in one launch; the sequential form in up to 2^d steps
    // (a cell moves in the step after its lower-colour neighbours; steps after
    // the last waiting cell return at once)
    gs::SeqStep seq{nullptr, nullptr, 0, 0};
    const int ncol = c->rule == GS_UPDATE_SEQUENTIAL ? 1 << d : 1;
    if (c->rule == GS_UPDATE_SEQUENTIAL) {
        if (c->seq_moved.cap < size_t(c->capM) * 4 || c->seq_epoch >= (1u << 24) - 1) {
            // new storage, or the epochs wrapped: start from cleared stamps
            GS_TRY(ensure(c->seq_moved, size_t(c->capM) * 4));
            GS_TRY(ensure(c->seq_waiting, 64 * 4));
            k_fill_u32<<<blocks_for(c->seq_moved.cap / 4, 256), 256, 0, s>>>(P<uint32_t>(c->seq_moved),
                                                                            c->seq_moved.cap / 4, 0u);
            k_fill_u32<<<1, 64, 0, s>>>(P<uint32_t>(c->seq_waiting), 64, 0u);
            GS_HIP(hipGetLastError());
            c->seq_epoch = 0;
        }
        seq = {P<uint32_t>(c->seq_moved), P<uint32_t>(c->seq_waiting), ++c->seq_epoch, 0};
    }
    for (int col = 0; col < ncol; ++col) {
        seq.step = col;
        // reads every cell row once, writes p and the landing key
        const int tk = prof_begin(c, s, "shift");
        switch (d) {
#define GS_SH(D)                                                                                                  \
    case D: gs::k_shift<D, Lookup><<<g, 256, 0, s>>>(t, m, prm, st, lk, pbuf, kappa, Wout, seq, c->fit_sets > 1); break;
            GS_SH(1) GS_SH(2) GS_SH(3) GS_SH(4) GS_SH(5) GS_SH(6)
#undef GS_SH
            default: return fail(GS_ERR_UNSUPPORTED, "d must be in 1..6");
        }
        prof_end(c, s, tk, (double(m) * (8.0 + 8.0 + 4.0 + 8.0 * d) + double(m) * (8.0 * d + 8.0)) / ncol);
        GS_HIP(hipGetLastError());
    }
    return GS_OK;
}

gs_status launch_tail(gs_context* c, int d, int B, gs::CellTable t, const gs::InstParam* prm, gs::InstState* st, uint32_t* tmap,
                      int max_iter, const gs::TailTape& tape, const gs::TailCkpt& ck, int replay_r0, hipStream_t s,
                      double nbytes, const int64_t* gate = nullptr) {
    const int tk = prof_begin(c, s, replay_r0 >= 0 ? "tail_replay" : "tail");
    c->tail_tok = tk;
    switch (d) {
#define GS_TL2(D, CT)                                                                                             \
    if (c->rule == GS_UPDATE_SEQUENTIAL)                                                                          \
        gs::k_tail<D, true, CT><<<B, gs::kTailThreads, 0, s>>>(t, prm, st, tmap, max_iter, tape, ck, replay_r0,   \
                                                               gate);                                             \
    else                                                                                                          \
        gs::k_tail<D, false, CT><<<B, gs::kTailThreads, 0, s>>>(t, prm, st, tmap, max_iter, tape, ck, replay_r0,  \
                                                                gate);
#define GS_TL(D)                                                                                                  \
    case D:                                                                                                       \
        if (c->wide_crd) {                                                                                        \
            GS_TL2(D, int64_t)                                                                                    \
        } else {                                                                                                  \
            GS_TL2(D, int32_t)                                                                                    \
        }                                                                                                         \
        break;
        GS_TL(1) GS_TL(2) GS_TL(3) GS_TL(4) GS_TL(5) GS_TL(6)
#undef GS_TL
#undef GS_TL2
        default: return fail(GS_ERR_UNSUPPORTED, "d must be in 1..6");
    }
    prof_end(c, s, tk, nbytes);
    GS_HIP(hipGetLastError());
    return GS_OK;
}

// Host computation of the per-instance key packing from the device boxes.
gs_status build_params(gs_context* c, int B, int d, const int64_t* offsets, const double* h,
                       const std::vector<int64_t>& box, int* bits_out) {
    c->prm.assign(B, gs::InstParam{});
    const uint64_t kLimit = 1ull << 62;
    uint64_t total = 0;
    c->wide_crd = false;
    for (int b = 0; b < B; ++b) {
        gs::InstParam& p = c->prm[b];
        p.h = h[b];
        p.row0 = offsets[b];
        p.row1 = offsets[b + 1];
        p.base = total;
        for (int k = 0; k < gs::kMaxDim; ++k) {
            p.lo[k] = 0;
            p.E[k] = 1;
            p.stride[k] = 1;
        }
        if (p.row1 == p.row0) {
            p.span = 0;
            continue;
        }
        long double span = 1.0L;
        for (int k = 0; k < d; ++k) {
            const int64_t mn = box[(int64_t(b) * gs::kMaxDim + k) * 2 + 0];
            const int64_t mx = box[(int64_t(b) * gs::kMaxDim + k) * 2 + 1];
            p.lo[k] = mn - 1;
            p.E[k] = mx - mn + 3;
            if (p.E[k] >= (int64_t(1) << 31)) c->wide_crd = true;
            span *= (long double)p.E[k];
        }
        if (span >= (long double)kLimit)
            return fail(GS_ERR_KEY_RANGE, "the key box of instance " + std::to_string(b) + " exceeds 2^62 cells");
        p.stride[d - 1] = 1;
        for (int k = d - 2; k >= 0; --k) p.stride[k] = p.stride[k + 1] * uint64_t(p.E[k + 1]);
        p.span = p.stride[0] * uint64_t(p.E[0]);
        total += p.span;
        if (total >= kLimit) return fail(GS_ERR_KEY_RANGE, "the instances' key boxes exceed 2^62 cells in total");
    }
    *bits_out = total <= 1 ? 0 : 64 - __builtin_clzll(total - 1);
    c->key_span = int64_t(total);
    return GS_OK;
}

// Device view of the per-round tail tape, `rounds` rounds per instance.
gs_status tail_tape(gs_context* c, int rounds, int B, gs::TailTape* tape) {
    const size_t per = size_t(rounds) * gs::kTailCells;
    GS_TRY(ensure(c->tt_key, per * B * 8));
    GS_TRY(ensure(c->tt_cnt, per * B * 4));
    GS_TRY(ensure(c->tt_W, per * B * 4));
    GS_TRY(ensure(c->tt_g, per * B * 4));
    GS_TRY(ensure(c->tt_m, size_t(rounds) * B * 4));
    tape->key = P<uint64_t>(c->tt_key);
    tape->cnt = P<int32_t>(c->tt_cnt);
    tape->W = P<int32_t>(c->tt_W);
    tape->g = P<uint32_t>(c->tt_g);
    tape->m = P<int32_t>(c->tt_m);
    tape->stride = int64_t(per);
    tape->max_rounds = rounds;
    return GS_OK;
}

// Two device tapes of `rounds` rounds per instance (one allocation each
// buffer, the second half for tp[1]).
gs_status tail_tape_pair(gs_context* c, int rounds, int B, gs::TailTape* tp) {
    const size_t per = size_t(rounds) * gs::kTailCells, half = per * B;
    GS_TRY(ensure(c->tt_key, 2 * half * 8));
    GS_TRY(ensure(c->tt_cnt, 2 * half * 4));
    GS_TRY(ensure(c->tt_W, 2 * half * 4));
    GS_TRY(ensure(c->tt_g, 2 * half * 4));
    GS_TRY(ensure(c->tt_m, 2 * size_t(rounds) * B * 4));
    for (int q = 0; q < 2; ++q) {
        tp[q].key = P<uint64_t>(c->tt_key) + q * half;
        tp[q].cnt = P<int32_t>(c->tt_cnt) + q * half;
        tp[q].W = P<int32_t>(c->tt_W) + q * half;
        tp[q].g = P<uint32_t>(c->tt_g) + q * half;
        tp[q].m = P<int32_t>(c->tt_m) + q * size_t(rounds) * B;
        tp[q].stride = int64_t(per);
        tp[q].max_rounds = rounds;
    }
    return GS_OK;
}

// The context's second stream and its events (created on first use, default
// priority, non-blocking).
gs_status aux_stream(gs_context* c) {
    if (c->aux) return GS_OK;
    GS_HIP(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
    hipEvent_t* evs[] = {&c->ev_start, &c->ev_rep[0], &c->ev_rep[1], &c->ev_adj[0], &c->ev_adj[1]};
    for (hipEvent_t* e : evs) GS_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
    return GS_OK;
}

// Device view of the tail checkpoints (ns slots per instance).
gs::TailCkpt ckpt_view(gs_context* c, int ns, int B, int every) {
    gs::TailCkpt ck;
    ck.key = P<uint64_t>(c->ck_key);
    ck.cnt = P<int32_t>(c->ck_cnt);
    ck.sum = P<double>(c->ck_sum);
    ck.m = P<int32_t>(c->ck_m);
    ck.stride = int64_t(ns) * gs::kTailCells;
    ck.total = ck.stride * B;
    ck.nslots = ns;
    ck.every = every;
    c->ck_nslots = ns;
    return ck;
}

// Algorithmic bytes of a tail launch (known once its states are back): every
// shift+merge round reads and writes its cell table (key, count and d sums:
// 16 + 8d bytes a cell), the exit test reads the final table once more, and
// the map of the M entering cells is written once.
double tail_alg_bytes(const gs_context* c, int B, int d, int64_t M) {
    double cells = 0.0;
    for (int b = 0; b < B; ++b) cells += 2.0 * double(c->st[b].tail_cells) + double(c->st[b].K);
    return cells * (16.0 + 8.0 * d) + 4.0 * double(M);
}

template <typename T, typename K>
gs_status fit_typed(gs_context* c, const T* x, int d, int64_t ld, int B, const int64_t* offsets, int max_iter,
                    int bits, int32_t* labels, hipStream_t s) {
    const int64_t N = offsets[B];
    c->fit_sets = B;
    int64_t* ctr = P<int64_t>(c->counters);
    gs::InstParam* prm = P<gs::InstParam>(c->param);
    gs::InstState* st = P<gs::InstState>(c->state);
    const int64_t* row_off = P<int64_t>(c->rowoff);

    // ---- keys and the stable sort of (key, point)
    // With a dense key table and many points, each point's initial cell is
    // looked up from its key after the cell setup (coalesced, in point order)
    // instead of being scattered by member index from the heads scan: the
    // keys in point order then stay in a buffer of their own through the
    // sort.  (Measured: the 256-image batch 9.77 -> 9.08 ms, 1e7-point
    // mixtures -75 / -55 us at d = 3 / 5; on 2M image points the scatter
    // costs less than the extra pass, so smaller inputs keep it.)
    const bool dense = c->cfg.dense_table && c->key_span <= gs::kDenseMax;
    const bool map_lookup = dense && N >= (int64_t(1) << 23);
    GS_TRY(ensure(c->kA, size_t(N) * sizeof(K)));
    GS_TRY(ensure(c->kB, size_t(N) * sizeof(K)));
    GS_TRY(ensure(c->vA, size_t(N) * 4));
    GS_TRY(ensure(c->vB, size_t(N) * 4));
    GS_TRY(ensure(c->cell0, size_t(N) * 4));
    if (map_lookup) GS_TRY(ensure(c->kpt, size_t(N) * sizeof(K)));
    // the key producer's output (taken after the buffers above are in place)
    K* const kkeys = P<K>(map_lookup ? c->kpt : c->kA);
    {
        void* old = c->sctr.p;
        GS_TRY(ensure(c->sctr, 64));
        if (c->sctr.p != old) c->sort.tile_base = 0x7fffffffull;  // new counter: cleared before its first use
    }
    GS_TRY(sort_look_ensure(c, N, bits, s));
    c->sort.hist = P<uint32_t>(c->shist);
    c->sort.ctr = P<uint32_t>(c->sctr);
    c->sort.prof_ctx = c;
    c->sort.prof_begin = sort_prof_begin;
    c->sort.prof_end = sort_prof_end;

    c->sort.allow10 = c->cfg.sort_digit10 != 0;
    c->sort.tile_keys = c->cfg.sort_tile;
    const gs::SortPlan plan = gs::sort_plan(bits, c->sort.allow10);
    const int np = plan.passes;
    if (c->ntiles > 0) {  // the current histogram buffer is zero (cleared by the previous sort)
        const unsigned g = unsigned(c->ntiles);
        // the key producer stages half-size chunks: with few tiles (under
        // eight per compute unit) its workgroups take a share of a tile each
        // (at most four of its chunks), so that more of them run at once
        // (measured: 1080p keys 27.0 -> 23.1 us; the 256-image batch, with
        // ~23K tiles, was slower split)
        const unsigned ksplit = g < 2048 ? unsigned(std::max(1, c->cfg.tile_chunks / 2)) : 1u;
        const gs::RowTile* tl = P<gs::RowTile>(c->tiles);
        const int tk = prof_begin(c, s, "make_keys");
        // the LDS digit histograms of the key producers: only the passes and
        // digits of this sort (more workgroups per compute unit than a
        // histogram sized for the widest sort)
        const size_t hist_lds = size_t(np << plan.digit) * sizeof(uint32_t);
        // a sweep's instances in groups over a second grid dimension, so that
        // the launch holds about 2048 workgroups
        const unsigned sweep_groups =
            c->sweep_n > 0 ? unsigned(std::min<int64_t>(B, std::max<int64_t>(1, (2048 + int64_t(g) - 1) / int64_t(g))))
                           : 1u;
        switch (d) {
#define GS_MK(D) \
    case D:                                                                                                    \
        if (c->sweep_n > 0)                                                                                    \
            gs::k_make_keys_sweep<T, K, D><<<dim3(g, sweep_groups), gs::kBoxThreads, hist_lds, s>>>(           \
                x, ld, tl, prm, B, c->sweep_n, kkeys, np, plan.digit, c->sort.cur_hist());                    \
        else                                                                                                   \
            gs::k_make_keys<T, K, D><<<g * ksplit, gs::kBoxThreads, hist_lds, s>>>(                             \
                x, ld, tl, prm, kkeys, np, plan.digit, c->sort.cur_hist(), ksplit);                           \
        break;
            GS_MK(1) GS_MK(2) GS_MK(3) GS_MK(4) GS_MK(5) GS_MK(6)
#undef GS_MK
            default: return fail(GS_ERR_UNSUPPORTED, "d must be in 1..6");
        }
        // points read once (once in all for a sweep), a key written per position
        prof_end(c, s, tk, (c->sweep_n > 0 ? double(c->sweep_n) : double(N)) * d * sizeof(T) + N * double(sizeof(K)));
        GS_HIP(hipGetLastError());
    }
    K* skeys = nullptr;
    uint32_t* perm = nullptr;
    GS_HIP(gs::radix_sort<K>(P<K>(c->kA), P<K>(c->kB), P<uint32_t>(c->vA), P<uint32_t>(c->vB), N, bits, true,
                             c->sort, s, &skeys, &perm, map_lookup ? kkeys : nullptr));

    // ---- run heads -> cell ids (table 0 key/start/first have capacity N)
    GS_TRY(ensure(c->tkey[0], size_t(N) * 8));
    GS_TRY(ensure(c->tstart[0], size_t(N) * 4));
    GS_TRY(ensure(c->tfirst[0], size_t(N) * 4));
    {
        gs::HeadsOp<K> op{skeys, perm, P<uint64_t>(c->tkey[0]), P<uint32_t>(c->tstart[0]), P<uint32_t>(c->tfirst[0]),
                          map_lookup ? nullptr : P<uint32_t>(c->cell0)};
        GS_TRY(run_scan(c, op, nullptr, N, ctr + 0, s, "scan_heads", N * (sizeof(K) + (map_lookup ? 0.0 : 8.0)),
                        c->hmap_dev));
    }
    GS_TRY(published_pull(c, sizeof(int64_t), s));
    const int64_t m0 = c->hmap[0];  // the cell count, published by the scan's last tile

    // ---- cell tables with capacity m0
    c->capM = std::max<int64_t>(m0, 1);
    for (int i = 0; i < 2; ++i) {
        if (i == 1) {
            GS_TRY(ensure(c->tkey[1], size_t(c->capM) * 8));
            GS_TRY(ensure(c->tstart[1], size_t(c->capM) * 4));
            GS_TRY(ensure(c->tfirst[1], size_t(c->capM) * 4));
        }
        GS_TRY(ensure(c->tcnt[i], size_t(c->capM) * 8));
        GS_TRY(ensure(c->tsum[i], size_t(c->capM) * d * 8));
        GS_TRY(ensure(c->tinst[i], size_t(c->capM) * 4));
        GS_TRY(ensure(c->tlen[i], size_t(c->capM) * 4));
        GS_TRY(ensure(c->tnch[i], size_t(c->capM) * 4));
        GS_TRY(ensure(c->tchoff[i], size_t(c->capM) * 4));
    }
    gs::CellTable T0 = table(c, 0);
    // cell rows; when a device-wide round follows (some instance may hold
    // more cells than a tail workgroup), the same pass starts the map initial
    // cell -> current cell and fills the dense key table for it
    const bool wide_next = m0 > gs::kTailCells;
    bool dk_pre = false;  // the next round's table is already in the dense table, under epoch dk_pre_epoch
    uint32_t dk_pre_epoch = 0;
    {
        uint32_t* cur0 = nullptr;
        uint64_t* dk0 = nullptr;
        if (wide_next) {
            GS_TRY(ensure(c->cur, size_t(c->capM) * 4));
            cur0 = P<uint32_t>(c->cur);
            if (dense) {
                GS_TRY(dense_reserve(c, s, &dk_pre_epoch));
                dk0 = P<uint64_t>(c->dk);
                dk_pre = true;
            }
        }
        PROF_LAUNCH("bin_cell_setup", m0 * (20.0 + (wide_next ? 12.0 : 0.0)),
                    gs::k_cell_setup<<<blocks_for(c->capM, 256), 256, 0, s>>>(ctr + 0, N, T0, 0, row_off, B,
                                                                               nullptr, st, true, cur0, dk0,
                                                                               dk_pre_epoch));
        GS_HIP(hipGetLastError());
    }
    if (map_lookup && N > 0) {  // the initial cell of every point, from its key
        const unsigned g = unsigned((N + 256 * gs::kCellOfPerThread - 1) / (256 * gs::kCellOfPerThread));
        if (dk_pre) {  // the dense table holds table 0 (entered by the cell setup above)
            PROF_LAUNCH("cell_of_points", N * (sizeof(K) + 4.0),
                        gs::k_cell_of_points_dense<K><<<g, 256, 0, s>>>(kkeys, N, P<uint64_t>(c->dk),
                                                                        P<uint32_t>(c->cell0)));
        } else {  // m0 <= kTailCells: no device-wide round follows
            PROF_LAUNCH("cell_of_points", N * (sizeof(K) + 4.0),
                        gs::k_cell_of_points_search<K><<<g, 256, 0, s>>>(kkeys, N, T0.key, int(m0),
                                                                         P<uint32_t>(c->cell0)));
        }
        GS_HIP(hipGetLastError());
    }
    GS_TRY(segsum(c, d, gs::SrcPoints<T>{x, ld, perm, uint32_t(c->sweep_n)}, T0, m0, N, s,
                  4.0 + double(d) * sizeof(T), false, true));
    if (c->tape_on && m0 > 0) {  // the initial cells, for the adjoint and the loss
        GS_TRY(ensure(c->sums0, size_t(m0) * d * 8));
        GS_TRY(ensure(c->inst0, size_t(m0) * 4));
        GS_HIP(hipMemcpyAsync(c->sums0.p, T0.sum, size_t(m0) * d * 8, hipMemcpyDeviceToDevice, s));
        GS_HIP(hipMemcpyAsync(c->inst0.p, T0.inst, size_t(m0) * 4, hipMemcpyDeviceToDevice, s));
    }
    c->w_off.clear();
    c->w_M.clear();
    c->wt_used = 0;

    c->st.assign(B, gs::InstState{});
    if (B == 1) {  // one instance: it holds all m0 cells and is active unless empty
        c->st[0].active = N > 0;
        c->st[0].cs = 0;
        c->st[0].ce = m0;
    } else {
        GS_TRY(d2h(c, c->st.data(), st, sizeof(gs::InstState) * B, s));
    }
    std::vector<int64_t> m0_of(B);
    for (int b = 0; b < B; ++b) m0_of[b] = c->st[b].ce - c->st[b].cs;

    // ---- remaining rounds: one LDS-resident workgroup per instance, then labels
    auto tail_and_labels = [&](int cur_tab, int nwide, int64_t Mnow, const int64_t* gate) -> gs_status {
        gs::CellTable TC = table(c, cur_tab);
        gs::TailTape tape;
        gs::TailCkpt ck;
        c->ckpt_used = c->ckpt_every;
        if (c->tape_on && max_iter > 0 && c->ckpt_every > 1) {
            // checkpoints only: the table every ckpt_every rounds
            const int ns = max_iter / c->ckpt_every + 1;
            const size_t per = size_t(ns) * gs::kTailCells;
            GS_TRY(ensure(c->ck_key, per * B * 8));
            GS_TRY(ensure(c->ck_cnt, per * B * 4));
            GS_TRY(ensure(c->ck_sum, per * B * d * 8));
            GS_TRY(ensure(c->ck_m, size_t(ns) * B * 4));
            ck = ckpt_view(c, ns, B, c->ckpt_every);
        } else if (c->tape_on && max_iter > 0) {
            GS_TRY(tail_tape(c, max_iter, B, &tape));
        }
        // (bytes: an upper bound, replaced once the host knows the cell counts)
        GS_TRY(launch_tail(c, d, B, TC, prm, st, P<uint32_t>(c->tmap), max_iter, tape, ck, -1, s,
                           2.0 * Mnow * (16.0 + 8.0 * d), gate));
        if (N > 0) {
            PROF_LAUNCH("labels", N * 8.0,
                        gs::k_labels<<<unsigned(std::min<int64_t>(gs::kLabelBlocks, blocks_for(N, 256))), 256, 0, s>>>(
                            P<uint32_t>(c->cell0), nwide ? P<uint32_t>(c->cur) : nullptr, P<uint32_t>(c->tmap), labels, N,
                            gate, st, B, P<int64_t>(c->koff), ctr, c->hmap_dev));
            GS_HIP(hipGetLastError());
        }
        return GS_OK;
    };

    // ---- wide rounds while some active instance has more cells than a tail holds
    GS_TRY(ensure(c->tmap, size_t(c->capM) * 4));
    int cur = 0;
    int64_t M = m0;
    int wide = 0;
    bool tail_done = false;
    for (;;) {
        bool need = false;
        for (int b = 0; b < B; ++b)
            if (c->st[b].active && c->st[b].ce - c->st[b].cs > gs::kTailCells) need = true;
        if (!need) break;
        if (wide == 0) {
            GS_TRY(ensure(c->cur, size_t(c->capM) * 4));
            if (!wide_next) k_iota32<<<blocks_for(m0, 256), 256, 0, s>>>(P<uint32_t>(c->cur), m0);
            GS_TRY(ensure(c->kappa, size_t(c->capM) * 8));
            GS_TRY(ensure(c->pbuf, size_t(c->capM) * d * 8));
            GS_TRY(ensure(c->gmap, size_t(c->capM) * 4));
            GS_TRY(ensure(c->ckA, size_t(c->capM) * sizeof(K)));
            GS_TRY(ensure(c->ckB, size_t(c->capM) * sizeof(K)));
            GS_TRY(ensure(c->cvA, size_t(c->capM) * 4));
            GS_TRY(ensure(c->cvB, size_t(c->capM) * 4));
        }
        ++wide;
        gs::CellTable TT = table(c, cur), U = table(c, 1 - cur);
        // neighbour lookup structure of the round's table (the first round's
        // dense entries were written with the cell rows)
        int logcap = 1;
        uint32_t tab_epoch = 0;  // epoch of this round's table in the dense table
        if (dense) {
            if (dk_pre) {
                tab_epoch = dk_pre_epoch;
            } else {
                GS_TRY(dense_reserve(c, s, &tab_epoch));
                PROF_LAUNCH("dense_insert", M * 16.0,
                            gs::k_dense_insert<<<blocks_for(M, 256), 256, 0, s>>>(TT.key, M, P<uint64_t>(c->dk),
                                                                                   tab_epoch));
            }
            dk_pre = false;
        } else {
            while ((int64_t(1) << logcap) < 2 * M) ++logcap;
            const int64_t hcap = int64_t(1) << logcap;
            GS_TRY(ensure(c->hk, size_t(hcap) * 8));
            GS_TRY(ensure(c->hv, size_t(hcap) * 4));
            PROF_LAUNCH("hash_clear", hcap * 8.0,
                        gs::k_hash_clear<<<blocks_for(hcap, 256), 256, 0, s>>>(P<uint64_t>(c->hk), hcap));
            PROF_LAUNCH("hash_insert", M * 20.0,
                        gs::k_hash_insert<<<blocks_for(M, 256), 256, 0, s>>>(TT.key, M, P<uint64_t>(c->hk),
                                                                              P<uint32_t>(c->hv), logcap));
        }
        GS_HIP(hipGetLastError());
        int32_t* Wrec = nullptr;
        int32_t* apprec = nullptr;
        const int64_t woff = c->wt_used;
        if (c->tape_on) {  // the round's starting table, weights, merge map and applying instances
            const size_t used = size_t(woff), need = size_t(woff + M);
            GS_TRY(ensure_keep(c->wt_key, need * 8, used * 8, s));
            GS_TRY(ensure_keep(c->wt_cnt, need * 8, used * 8, s));
            GS_TRY(ensure_keep(c->wt_inst, need * 4, used * 4, s));
            GS_TRY(ensure_keep(c->wt_W, need * 4, used * 4, s));
            GS_TRY(ensure_keep(c->wt_g, need * 4, used * 4, s));
            const size_t r = c->w_off.size();
            GS_TRY(ensure_keep(c->wt_app, (r + 1) * B * 4, r * B * 4, s));
            GS_HIP(hipMemcpyAsync(P<uint64_t>(c->wt_key) + woff, TT.key, M * 8, hipMemcpyDeviceToDevice, s));
            GS_HIP(hipMemcpyAsync(P<int64_t>(c->wt_cnt) + woff, TT.cnt, M * 8, hipMemcpyDeviceToDevice, s));
            GS_HIP(hipMemcpyAsync(P<int32_t>(c->wt_inst) + woff, TT.inst, M * 4, hipMemcpyDeviceToDevice, s));
            Wrec = P<int32_t>(c->wt_W) + woff;
            apprec = P<int32_t>(c->wt_app) + r * B;
            c->w_off.push_back(woff);
            c->w_M.push_back(M);
            c->wt_used = woff + M;
        }
        if (dense)
            GS_TRY(launch_shift(c, d, TT, M, prm, st, gs::DenseLookup{P<uint64_t>(c->dk), tab_epoch},
                                P<double>(c->pbuf), P<uint64_t>(c->kappa), Wrec, s));
        else
            GS_TRY(launch_shift(c, d, TT, M, prm, st,
                                gs::HashLookup{P<uint64_t>(c->hk), P<uint32_t>(c->hv), logcap}, P<double>(c->pbuf),
                                P<uint64_t>(c->kappa), Wrec, s));
        bool gated = false;  // the round's last kernel already wrote the tail gate
        uint64_t* dk_next = nullptr;  // the merge also enters the new table in the dense table
        if (dense) {
            GS_TRY(dense_reserve(c, s, &dk_pre_epoch));
            dk_next = P<uint64_t>(c->dk);
            dk_pre = true;
        }
        if (sizeof(K) == 4 && M <= gs::kMergeMax && B <= gs::kMergeMaxInst && c->cfg.merge_small) {
            // the round's decisions, the whole merge and its bookkeeping in one workgroup
            uint32_t* gt = c->tape_on ? P<uint32_t>(c->wt_g) + woff : nullptr;
            const int tk = prof_begin(c, s, "merge_small");
            switch (d) {
#define GS_MS(D)                                                                                                   \
    case D:                                                                                                        \
        gs::k_merge_small<D><<<1, gs::kMergeThreads, 0, s>>>(TT, M, U, st, B, P<double>(c->pbuf),                  \
                                                             P<uint64_t>(c->kappa), (bits + 7) / 8, bits,          \
                                                             P<uint32_t>(c->gmap),                                 \
                                                             P<uint32_t>(c->cvA), P<uint32_t>(c->cur), m0, gt,     \
                                                             ctr, max_iter, dk_next, dk_pre_epoch);                \
        break;
                GS_MS(1) GS_MS(2) GS_MS(3) GS_MS(4) GS_MS(5) GS_MS(6)
#undef GS_MS
                default: return fail(GS_ERR_UNSUPPORTED, "d must be in 1..6");
            }
            prof_end(c, s, tk, M * (8.0 * 3 + 16.0 * d + 8.0) + m0 * 8.0);
            GS_HIP(hipGetLastError());
            gs::SrcMerge src{P<double>(c->pbuf), TT.sum, TT.cnt, TT.inst, st, P<uint32_t>(c->cvA), c->capM};
            GS_TRY(segsum(c, d, src, U, M, M, s, 4.0 + 4.0 + 8.0 + 8.0 * d, true));
            gated = B <= 256;  // one block: it also writes the tail gate
            PROF_LAUNCH("round_end", B * 48.0,
                        gs::k_round_end<<<blocks_for(B, 256), 256, 0, s>>>(P<uint32_t>(c->cur), 0,
                                                                            P<uint32_t>(c->gmap), st, B, apprec,
                                                                            gated ? ctr + 4 : nullptr, ctr,
                                                                            c->hmap_dev));
            GS_HIP(hipGetLastError());
        } else {
        gs::k_decide<<<blocks_for(B, 256), 256, 0, s>>>(st, B, max_iter);
        PROF_LAUNCH("merge_prep", M * (8.0 * 3 + 16.0 * d + sizeof(K)),
                    gs::k_merge_prep<K><<<blocks_for(M, 256), 256, 0, s>>>(TT, M, st, st, P<double>(c->pbuf),
                                                                            P<uint64_t>(c->kappa), P<K>(c->ckA), d,
                                                                            np, plan.digit, c->sort.cur_hist()));
        GS_HIP(hipGetLastError());
        K* mk = nullptr;
        uint32_t* mperm = nullptr;
        GS_HIP(gs::radix_sort<K>(P<K>(c->ckA), P<K>(c->ckB), P<uint32_t>(c->cvA), P<uint32_t>(c->cvB), M, bits,
                                 true, c->sort, s, &mk, &mperm));
        gs::HeadsOp<K> op{mk, mperm, U.key, U.start, U.first, P<uint32_t>(c->gmap)};
        GS_TRY(run_scan(c, op, nullptr, M, ctr + 0, s, "scan_heads", M * (sizeof(K) + 8.0)));
        if (c->tape_on)
            GS_HIP(hipMemcpyAsync(P<uint32_t>(c->wt_g) + woff, c->gmap.p, M * 4, hipMemcpyDeviceToDevice, s));
        PROF_LAUNCH("cell_setup", M * 24.0,
                    gs::k_cell_setup<<<blocks_for(M, 256), 256, 0, s>>>(ctr + 0, M, U, 1, row_off, B, TT.inst, st,
                                                                         true, nullptr, dk_next, dk_pre_epoch));
        GS_HIP(hipGetLastError());
        gs::SrcMerge src{P<double>(c->pbuf), TT.sum, TT.cnt, TT.inst, st, mperm, c->capM};
        GS_TRY(segsum(c, d, src, U, M, M, s, 4.0 + 4.0 + 8.0 + 8.0 * d));
        PROF_LAUNCH("round_end", m0 * 12.0,
                    gs::k_round_end<<<blocks_for(std::max<int64_t>(m0, B), 256), 256, 0, s>>>(
                        P<uint32_t>(c->cur), m0, P<uint32_t>(c->gmap), st, B, apprec, nullptr, nullptr, nullptr));
        GS_HIP(hipGetLastError());
        }
        cur = 1 - cur;
        // the tail and the labels right away, unless some instance still needs
        // a device-wide round (then the tail changes nothing and the loop goes on)
        if (!gated) {
            gs::k_tail_gate<<<1, 256, 0, s>>>(st, B, ctr + 4, ctr, c->hmap_dev);
            GS_HIP(hipGetLastError());
        }
        GS_TRY(tail_and_labels(cur, wide, M, ctr + 4));
        // the gate's kernel published the round's counters and states; the
        // labels kernel, when the tail ran, the tail's
        int64_t ctrs[8];
        GS_TRY(read_published(c, ctrs, s));
        M = ctrs[0];
        const int64_t gate = ctrs[4];
        for (int b = 0; b < B; ++b)
            if (c->st[b].err) return fail(GS_ERR_KEY_RANGE, "a moved cell left its instance's key box");
        if (!gate) {
            prof_set_bytes(c, c->tail_tok, tail_alg_bytes(c, B, d, M));
            tail_done = true;
            break;
        }
    }

    if (!tail_done) {
        GS_TRY(tail_and_labels(cur, wide, M, nullptr));
        if (N > 0) {  // published by the labels kernel
            int64_t ctrs[8];
            GS_TRY(read_published(c, ctrs, s));
        } else {
            GS_TRY(d2h(c, c->st.data(), st, sizeof(gs::InstState) * B, s));
        }
        prof_set_bytes(c, c->tail_tok, tail_alg_bytes(c, B, d, M));
    }
    for (int b = 0; b < B; ++b) {
        if (c->st[b].err) return fail(GS_ERR_KEY_RANGE, "a moved cell left its instance's key box");
        c->st[b].m0 = m0_of[b];
    }
    c->cur_tab = cur;
    c->tail_rounds = max_iter;
    c->wide_rounds = wide;
    c->sort_bits = bits;
    c->m0 = m0;
    return GS_OK;
}

// ---------------------------------------------------------------------------
// differentiable form
// ---------------------------------------------------------------------------
// Host copy of the cluster row offsets (the fit left the same values in
// c->koff on the device).
gs_status host_koff(gs_context* c, hipStream_t, std::vector<int64_t>& koff) {
    koff.assign(c->B + 1, 0);
    for (int b = 0; b < c->B; ++b) koff[b + 1] = koff[b] + c->st[b].K;
    return GS_OK;
}

gs_status launch_tail_adj(gs_context* c, int d, const gs::TailTape& tape, const gs::TailCkpt& ck, int seg_r0,
                          double* sbar, hipStream_t s) {
    const gs::InstParam* prm = P<gs::InstParam>(c->param);
    const gs::InstState* st = P<gs::InstState>(c->state);
    const int B = c->B;
    const int64_t cap = c->capM;
    const int tk = prof_begin(c, s, "tail_adj");
    switch (d) {
#define GS_TA(D)                                                                                                  \
    case D:                                                                                                       \
        if (c->wide_crd)                                                                                          \
            gs::k_tail_adj<D, int64_t><<<B, gs::kTailThreads, 0, s>>>(prm, st, tape, sbar, cap, ck, seg_r0);      \
        else                                                                                                      \
            gs::k_tail_adj<D, int32_t><<<B, gs::kTailThreads, 0, s>>>(prm, st, tape, sbar, cap, ck, seg_r0);      \
        break;
        GS_TA(1) GS_TA(2) GS_TA(3) GS_TA(4) GS_TA(5) GS_TA(6)
#undef GS_TA
        default: return fail(GS_ERR_UNSUPPORTED, "d must be in 1..6");
    }
    prof_end(c, s, tk, 0.0);
    GS_HIP(hipGetLastError());
    return GS_OK;
}

template <class Lookup>
gs_status launch_adj_stencil(gs_context* c, int d, const uint64_t* key, const int32_t* inst, const int32_t* applied,
                             int64_t m, Lookup lk, const double* q, double* out, hipStream_t s) {
    const gs::InstParam* prm = P<gs::InstParam>(c->param);
    const unsigned g = blocks_for(m, gs::kShiftWaves);
    const int64_t cap = c->capM;
    const int tk = prof_begin(c, s, "adj_stencil");
    switch (d) {
#define GS_AS(D)                                                                                                \
    case D: gs::k_adj_stencil<D, Lookup><<<g, 256, 0, s>>>(key, inst, applied, m, prm, lk, q, out, cap, c->B > 1); break;
        GS_AS(1) GS_AS(2) GS_AS(3) GS_AS(4) GS_AS(5) GS_AS(6)
#undef GS_AS
        default: return fail(GS_ERR_UNSUPPORTED, "d must be in 1..6");
    }
    prof_end(c, s, tk, double(m) * (8.0 + 8.0 * d) * 2);
    GS_HIP(hipGetLastError());
    return GS_OK;
}

// Reverse of every round: mode cotangents gm [sum K][d] -> Sbar of the
// initial cells (returned pointer, [d][capM]).
gs_status adjoint_core(gs_context* c, const double* gm, hipStream_t s, double** sbar0_out) {
    const int d = c->d, B = c->B;
    std::vector<int64_t> koff;
    GS_TRY(host_koff(c, s, koff));
    const int64_t rows = koff[B];
    const size_t cellbytes = size_t(c->capM) * d * 8;
    GS_TRY(ensure(c->sbA, cellbytes));
    GS_TRY(ensure(c->sbB, cellbytes));
    GS_TRY(ensure(c->qbuf, cellbytes));
    double* sa = P<double>(c->sbA);
    double* sb = P<double>(c->sbB);
    gs::CellTable TC = table(c, c->cur_tab);
    if (rows > 0)
        PROF_LAUNCH("adj_final", rows * (16.0 * d + 8.0),
                    gs::k_adj_final<<<blocks_for(rows, 256), 256, 0, s>>>(TC, P<gs::InstState>(c->state),
                                                                          P<int64_t>(c->koff), B, rows, d, gm, sa));
    gs::TailTape tape;
    if (c->tail_rounds > 0 && c->ckpt_used > 1) {
        // segments of ckpt_used tail rounds, last first: recompute the
        // segment's tape from its checkpoint, then reverse its rounds
        int most = 0;
        for (int b = 0; b < B; ++b) most = std::max(most, c->st[b].t - c->st[b].t_tail0);
        // Segment i is recomputed on the second stream into tape buffer i % 2
        // while segment i - 1 is reversed on s; a buffer is refilled only
        // after the reversal that read it.
        const int k = c->ckpt_used;
        gs::TailTape tp[2];
        GS_TRY(tail_tape_pair(c, k, B, tp));
        GS_TRY(aux_stream(c));
        const gs::TailCkpt ck = ckpt_view(c, c->ck_nslots, B, k);
        hipStream_t s2 = c->aux;
        GS_HIP(hipEventRecord(c->ev_start, s));
        GS_HIP(hipStreamWaitEvent(s2, c->ev_start, 0));
        int i = 0;
        for (int r0 = most > 0 ? ((most - 1) / k) * k : -1; r0 >= 0; r0 -= k, ++i) {
            const int q = i & 1;
            if (i >= 2) GS_HIP(hipStreamWaitEvent(s2, c->ev_adj[q], 0));
            GS_TRY(launch_tail(c, d, B, TC, P<gs::InstParam>(c->param), P<gs::InstState>(c->state), nullptr,
                               c->tail_rounds, tp[q], ck, r0, s2, 0.0));
            GS_HIP(hipEventRecord(c->ev_rep[q], s2));
            GS_HIP(hipStreamWaitEvent(s, c->ev_rep[q], 0));
            GS_TRY(launch_tail_adj(c, d, tp[q], ck, r0, sa, s));
            GS_HIP(hipEventRecord(c->ev_adj[q], s));
        }
    } else if (c->tail_rounds > 0) {
        tape.key = P<uint64_t>(c->tt_key);
        tape.cnt = P<int32_t>(c->tt_cnt);
        tape.W = P<int32_t>(c->tt_W);
        tape.g = P<uint32_t>(c->tt_g);
        tape.m = P<int32_t>(c->tt_m);
        tape.stride = int64_t(c->tail_rounds) * gs::kTailCells;
        tape.max_rounds = c->tail_rounds;
        GS_TRY(launch_tail_adj(c, d, tape, gs::TailCkpt{}, 0, sa, s));
    }
    for (int r = int(c->w_off.size()) - 1; r >= 0; --r) {
        const int64_t off = c->w_off[r], M = c->w_M[r];
        const int32_t* applied = P<int32_t>(c->wt_app) + int64_t(r) * B;
        PROF_LAUNCH("adj_q", M * (24.0 + 16.0 * d),
                    gs::k_adj_q<<<blocks_for(M, 256), 256, 0, s>>>(
                        P<int32_t>(c->wt_inst) + off, P<int64_t>(c->wt_cnt) + off, P<int32_t>(c->wt_W) + off,
                        P<uint32_t>(c->wt_g) + off, applied, M, d, sa, P<double>(c->qbuf), c->capM));
        const uint64_t* rkey = P<uint64_t>(c->wt_key) + off;
        if (c->cfg.dense_table && c->key_span <= gs::kDenseMax) {  // the round's table in the dense key table
            uint32_t ep = 0;
            GS_TRY(dense_reserve(c, s, &ep));
            gs::k_dense_insert<<<blocks_for(M, 256), 256, 0, s>>>(rkey, M, P<uint64_t>(c->dk), ep);
            GS_HIP(hipGetLastError());
            GS_TRY(launch_adj_stencil(c, d, rkey, P<int32_t>(c->wt_inst) + off, applied, M,
                                      gs::DenseLookup{P<uint64_t>(c->dk), ep}, P<double>(c->qbuf), sb, s));
        } else {
            int logcap = 1;
            while ((int64_t(1) << logcap) < 2 * M) ++logcap;
            const int64_t hcap = int64_t(1) << logcap;
            GS_TRY(ensure(c->hk, size_t(hcap) * 8));
            GS_TRY(ensure(c->hv, size_t(hcap) * 4));
            gs::k_hash_clear<<<blocks_for(hcap, 256), 256, 0, s>>>(P<uint64_t>(c->hk), hcap);
            gs::k_hash_insert<<<blocks_for(M, 256), 256, 0, s>>>(rkey, M, P<uint64_t>(c->hk), P<uint32_t>(c->hv),
                                                                  logcap);
            GS_HIP(hipGetLastError());
            GS_TRY(launch_adj_stencil(c, d, rkey, P<int32_t>(c->wt_inst) + off, applied, M,
                                      gs::HashLookup{P<uint64_t>(c->hk), P<uint32_t>(c->hv), logcap},
                                      P<double>(c->qbuf), sb, s));
        }
        std::swap(sa, sb);
    }
    *sbar0_out = sa;
    return GS_OK;
}

gs_status check_tape(gs_context* c) {
    if (!c) return fail(GS_ERR_INVALID_ARG, "null context");
    if (!c->has_result || !c->tape_valid)
        return fail(GS_ERR_STATE, "the context holds no fit recorded with gs_context_set_tape(ctx, 1)");
    return GS_OK;
}

// Modes and counts of every cluster row into the context's buffers.
gs_status cluster_modes(gs_context* c, hipStream_t s, int64_t rows) {
    GS_TRY(ensure(c->modes_i, size_t(std::max<int64_t>(rows, 1)) * c->d * 8));
    GS_TRY(ensure(c->counts_i, size_t(std::max<int64_t>(rows, 1)) * 8));
    if (rows > 0)
        gs::k_copy_modes<<<blocks_for(rows, 256), 256, 0, s>>>(table(c, c->cur_tab), P<gs::InstState>(c->state),
                                                               P<int64_t>(c->koff), c->B, rows, c->d,
                                                               P<double>(c->modes_i), P<int64_t>(c->counts_i), nullptr);
    GS_HIP(hipGetLastError());
    return GS_OK;
}

gs_status fit_impl(gs_context* c, const void* points, gs_dtype dtype, int d, int64_t ld, int B,
                   const int64_t* offsets, const double* h, int max_iter, int32_t* labels, gs_info* info,
                   hipStream_t s) {
    if (!c) return fail(GS_ERR_INVALID_ARG, "null context");
    c->has_result = false;
    c->tape_valid = false;
    if (d < 1 || d > gs::kMaxDim) return fail(GS_ERR_UNSUPPORTED, "d must be in 1..6");
    if (B < 1 || !offsets || !h || !info) return fail(GS_ERR_INVALID_ARG, "B >= 1, offsets, h and info are required");
    if (dtype != GS_F32 && dtype != GS_F64) return fail(GS_ERR_INVALID_ARG, "dtype must be GS_F32 or GS_F64");
    if (ld < d) return fail(GS_ERR_INVALID_ARG, "ld must be >= d");
    if (max_iter < 0) return fail(GS_ERR_INVALID_ARG, "max_iter must be >= 0");
    if (c->tape_on && c->rule != GS_UPDATE_PARALLEL)
        return fail(GS_ERR_UNSUPPORTED, "the trajectory is recorded for the parallel update only");
    if (offsets[0] != 0) return fail(GS_ERR_INVALID_ARG, "offsets[0] must be 0");
    for (int b = 0; b < B; ++b) {
        if (offsets[b + 1] < offsets[b]) return fail(GS_ERR_INVALID_ARG, "offsets must be non-decreasing");
        if (!(h[b] > 0.0) || !std::isfinite(h[b])) return fail(GS_ERR_INVALID_ARG, "h must be finite and > 0");
    }
    const int64_t N = offsets[B];
    if (N >= (int64_t(1) << 31)) return fail(GS_ERR_INVALID_ARG, "at most 2^31 - 1 points");
    if (N > 0 && (!points || !labels)) return fail(GS_ERR_INVALID_ARG, "points and labels are required");
    GS_HIP(hipSetDevice(c->device));
    prof_flush(c, true);  // records of the calls since the last fit (backward, loss)

    // row tiles of tile_chunks staged chunks of rows, each inside one instance
    const int trows = c->cfg.tile_chunks * gs::chunk_rows(d, dtype == GS_F32 ? 4 : 8);
    // (a bandwidth sweep tiles its shared rows once, as instance 0)
    std::vector<gs::RowTile> tiles;
    for (int b = 0; b < (c->sweep_n > 0 ? 1 : B); ++b) {
        for (int64_t r = offsets[b]; r < offsets[b + 1]; r += trows)
            tiles.push_back({r, std::min<int64_t>(r + trows, offsets[b + 1]), b, 0});
    }
    c->ntiles = int64_t(tiles.size());
    // control block layout (256-byte aligned parts)
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    const int nbc = B >= 64 ? 1 : 16;  // box copies per instance (fewer atomics per address)
    const size_t box_bytes = sizeof(int64_t) * size_t(B) * nbc * gs::kMaxDim * 2;
    const size_t o_ctr = al(box_bytes);
    const size_t o_state = al(o_ctr + 8 * sizeof(int64_t));
    const size_t o_koff = al(o_state + sizeof(gs::InstState) * B);
    const size_t o_rowoff = al(o_koff + sizeof(int64_t) * (B + 1));
    const size_t o_hs = al(o_rowoff + sizeof(int64_t) * (B + 1));
    const size_t o_tiles = al(o_hs + sizeof(double) * B);
    const size_t up_end = o_tiles + sizeof(gs::RowTile) * tiles.size();
    const size_t o_param = al(up_end);
    GS_TRY(ensure(c->ctl, o_param + sizeof(gs::InstParam) * B));
    char* base = static_cast<char*>(c->ctl.p);
    c->bbox = DBuf{base, box_bytes};
    c->counters = DBuf{base + o_ctr, 8 * sizeof(int64_t)};
    c->state = DBuf{base + o_state, sizeof(gs::InstState) * B};
    c->koff = DBuf{base + o_koff, sizeof(int64_t) * (B + 1)};  // written by the labels kernel (zero if no points)
    c->rowoff = DBuf{base + o_rowoff, sizeof(int64_t) * (B + 1)};
    c->hs = DBuf{base + o_hs, sizeof(double) * B};
    c->tiles = DBuf{base + o_tiles, sizeof(gs::RowTile) * tiles.size()};
    c->param = DBuf{base + o_param, sizeof(gs::InstParam) * B};
    // initial boxes (empty), counters (zero) and states (active), offsets,
    // bandwidths and tiles: one upload
    std::vector<char>& img = c->ctl_img;
    img.assign(up_end, 0);
    {
        uint64_t* bx = reinterpret_cast<uint64_t*>(img.data());
        for (size_t i = 0; i < box_bytes / 8; i += 2) {
            bx[i] = ~0ull;  // min image (the largest)
            bx[i + 1] = 0;  // max image (the smallest)
        }
        gs::InstState z{};
        z.active = 1;
        for (int b = 0; b < B; ++b) std::memcpy(img.data() + o_state + sizeof(z) * b, &z, sizeof(z));
        std::memcpy(img.data() + o_rowoff, offsets, sizeof(int64_t) * (B + 1));
        std::memcpy(img.data() + o_hs, h, sizeof(double) * B);
        if (!tiles.empty()) std::memcpy(img.data() + o_tiles, tiles.data(), sizeof(gs::RowTile) * tiles.size());
    }
    GS_TRY(h2d(c, base, img.data(), up_end, s));
    GS_TRY(hmap_ensure(c, B));
    {
        void* old = c->shist.p;
        GS_TRY(ensure(c->shist, gs::kHistEntries * 4));
        if (c->shist.p != old) c->hist_dirty = true;
    }
    if (c->hist_dirty) {  // each sort clears the buffer the next producer uses; only a new or failed use needs this
        k_fill_u32<<<blocks_for(gs::kHistEntries, 256), 256, 0, s>>>(
            P<uint32_t>(c->shist), gs::kHistEntries, 0u);
        GS_HIP(hipGetLastError());
        c->hist_dirty = false;
    }

    std::vector<int64_t> box(size_t(B) * gs::kMaxDim * 2, 0);
    if (N > 0) {
        const unsigned g = unsigned(tiles.size());
        const unsigned bsplit = 1;
        const double xb = double(N) * d * (dtype == GS_F32 ? 4.0 : 8.0);
        const gs::RowTile* tl = P<gs::RowTile>(c->tiles);
        uint64_t* bp = P<uint64_t>(c->bbox);
        int64_t* cn = P<int64_t>(c->counters);
        const float* xf = static_cast<const float*>(points);
        const double* xd = static_cast<const double*>(points);
        const int tk = prof_begin(c, s, "bbox");
        switch (d * 2 + (dtype == GS_F32 ? 0 : 1)) {
#define GS_BB(D)                                                                                               \
    case 2 * D:                                                                                                \
        gs::k_bbox_tiles<float, D><<<g * bsplit, gs::kBoxThreads, 0, s>>>(xf, ld, tl, bp, nbc, cn, bsplit);       \
        break;                                                                                                 \
    case 2 * D + 1:                                                                                            \
        gs::k_bbox_tiles<double, D><<<g * bsplit, gs::kBoxThreads, 0, s>>>(xd, ld, tl, bp, nbc, cn, bsplit);      \
        break;
            GS_BB(1) GS_BB(2) GS_BB(3) GS_BB(4) GS_BB(5) GS_BB(6)
#undef GS_BB
            default: return fail(GS_ERR_UNSUPPORTED, "d must be in 1..6");
        }
        prof_end(c, s, tk, xb);
        GS_HIP(hipGetLastError());
        // boxes and counters in one copy (counter 2 holds the error bits)
        std::vector<char> rb(o_ctr + 3 * sizeof(int64_t));
        GS_TRY(d2h(c, rb.data(), base, rb.size(), s));
        int64_t errbits = 0;
        std::memcpy(&errbits, rb.data() + o_ctr + 2 * sizeof(int64_t), sizeof(int64_t));
        if (errbits & 1) return fail(GS_ERR_NONFINITE, "a coordinate is NaN or infinite");
        // extremes of the coordinates (order-preserving images, combined over
        // the copies) -> cell coordinates floor(fl(v / h)) of the extremes,
        // which bound every point's by monotonicity
        const uint64_t* bc = reinterpret_cast<const uint64_t*>(rb.data());
        auto decode = [](uint64_t u) {
            const uint64_t bits = (u >> 63) ? (u & ~(1ull << 63)) : ~u;
            double v;
            std::memcpy(&v, &bits, sizeof(v));
            return v;
        };
        for (int b = 0; b < B; ++b) {
            if (offsets[b + 1] == offsets[b]) continue;  // empty instance: no box
            const int64_t ib = c->sweep_n > 0 ? 0 : b;  // a sweep's instances share instance 0's coordinates
            for (int k = 0; k < d; ++k) {
                uint64_t mn = ~0ull, mx = 0;
                for (int q = 0; q < nbc; ++q) {
                    const uint64_t* e = bc + ((ib * nbc + q) * gs::kMaxDim + k) * 2;
                    mn = std::min(mn, e[0]);
                    mx = std::max(mx, e[1]);
                }
                const double qlo = std::floor(decode(mn) / h[b]);
                const double qhi = std::floor(decode(mx) / h[b]);
                const double lim = 4503599627370496.0;  // 2^52
                if (!(qlo > -lim && qlo < lim && qhi > -lim && qhi < lim))
                    return fail(GS_ERR_KEY_RANGE, "|floor(x/h)| >= 2^52");
                box[(int64_t(b) * gs::kMaxDim + k) * 2 + 0] = int64_t(qlo);
                box[(int64_t(b) * gs::kMaxDim + k) * 2 + 1] = int64_t(qhi);
            }
        }
    }
    int bits = 0;
    GS_TRY(build_params(c, B, d, offsets, h, box, &bits));
    GS_TRY(h2d(c, c->param.p, c->prm.data(), sizeof(gs::InstParam) * B, s));

    gs_status rc;
    if (bits <= 32) {
        rc = dtype == GS_F32 ? fit_typed<float, uint32_t>(c, static_cast<const float*>(points), d, ld, B, offsets,
                                                          max_iter, bits, labels, s)
                             : fit_typed<double, uint32_t>(c, static_cast<const double*>(points), d, ld, B, offsets,
                                                           max_iter, bits, labels, s);
    } else {
        rc = dtype == GS_F32 ? fit_typed<float, uint64_t>(c, static_cast<const float*>(points), d, ld, B, offsets,
                                                          max_iter, bits, labels, s)
                             : fit_typed<double, uint64_t>(c, static_cast<const double*>(points), d, ld, B, offsets,
                                                           max_iter, bits, labels, s);
    }
    if (rc != GS_OK) {
        (void)hipStreamSynchronize(s);
        c->hist_dirty = true;
        prof_flush(c, false);
        return rc;
    }
    prof_flush(c, true);
    for (int b = 0; b < B; ++b) {
        info[b].n_points = offsets[b + 1] - offsets[b];
        info[b].n_cells0 = c->st[b].m0;
        info[b].n_clusters = c->st[b].K;
        info[b].n_iter = c->st[b].t;
        info[b].flags = c->st[b].flags;
    }
    c->B = B;
    c->d = d;
    c->dtype = int(dtype);
    c->N = N;
    c->ld = ld;
    c->has_result = true;
    c->tape_valid = c->tape_on;
    return GS_OK;
}

}  // namespace

namespace {

template <typename T>
static gs_status loss_fwd(gs_context* c, const T* x, const int32_t* labels, double* loss, hipStream_t s) {
    const int B = c->B;
    std::vector<int64_t> koff;
    GS_TRY(host_koff(c, s, koff));
    GS_TRY(cluster_modes(c, s, koff[B]));
    // one "cell" per instance, whose members are its points in index order
    std::vector<uint32_t> host(4 * size_t(B));
    for (int b = 0; b < B; ++b) {
        const int64_t n0 = c->prm[b].row0, n1 = c->prm[b].row1;
        host[b] = uint32_t(n0);
        host[B + b] = uint32_t(n1 - n0);
        host[2 * B + b] = uint32_t((n1 - n0 + gs::kChunk - 1) / gs::kChunk);
        host[3 * B + b] = 0;
    }
    GS_TRY(ensure(c->ltab, host.size() * 4));
    GS_TRY(ensure(c->lossc, size_t(B) * 8));
    GS_TRY(h2d(c, c->ltab.p, host.data(), host.size() * 4, s));
    gs::CellTable t;
    t.start = P<uint32_t>(c->ltab);
    t.len = t.start + B;
    t.nch = t.start + 2 * B;
    t.choff = t.start + 3 * B;
    t.sum = loss;
    t.cnt = P<int64_t>(c->lossc);
    t.cap = B;
    int64_t* ctr = P<int64_t>(c->counters);
    k_set_i64<<<1, 1, 0, s>>>(ctr + 0, B);
    gs::SrcLoss<T> src{x, c->ld, labels, P<double>(c->modes_i), P<int64_t>(c->koff), c->d};
    return segsum_d<1>(c, src, t, B, c->N, s, 4.0 + 4.0 + c->d * double(sizeof(T)), false, false);
}

template <typename T>
static gs_status loss_bwd(gs_context* c, const T* x, const int32_t* labels, const double* gloss, double* grad,
                          hipStream_t s) {
    const int B = c->B, d = c->d;
    std::vector<int64_t> koff;
    GS_TRY(host_koff(c, s, koff));
    const int64_t rows = koff[B];
    GS_TRY(cluster_modes(c, s, rows));
    const int64_t m0 = c->m0;
    // point sums of every cluster: R over its initial cells in ascending order
    GS_TRY(ensure(c->frows, size_t(std::max<int64_t>(m0, 1)) * 4));
    GS_TRY(ensure(c->xkA, size_t(std::max<int64_t>(m0, 1)) * 4));
    GS_TRY(ensure(c->xkB, size_t(std::max<int64_t>(m0, 1)) * 4));
    GS_TRY(ensure(c->xvA, size_t(std::max<int64_t>(m0, 1)) * 4));
    GS_TRY(ensure(c->xvB, size_t(std::max<int64_t>(m0, 1)) * 4));
    gs::k_final_rows<<<blocks_for(m0, 256), 256, 0, s>>>(P<int32_t>(c->inst0),
                                                          c->wide_rounds ? P<uint32_t>(c->cur) : nullptr,
                                                          P<uint32_t>(c->tmap), P<int64_t>(c->koff), m0,
                                                          P<uint32_t>(c->xkA));
    GS_HIP(hipGetLastError());
    int bits = 0;
    while ((int64_t(1) << bits) < rows) ++bits;
    GS_TRY(sort_look_ensure(c, m0, bits, s));
    uint32_t* sk = nullptr;
    uint32_t* sperm = nullptr;
    GS_HIP(gs::radix_sort<uint32_t>(P<uint32_t>(c->xkA), P<uint32_t>(c->xkB), P<uint32_t>(c->xvA),
                                    P<uint32_t>(c->xvB), m0, bits, false, c->sort, s, &sk, &sperm));
    gs::CellTable X = table(c, 1 - c->cur_tab);  // the idle ping-pong table holds the groups
    int64_t* ctr = P<int64_t>(c->counters);
    gs::HeadsOp<uint32_t> op{sk, sperm, X.key, X.start, X.first, P<uint32_t>(c->frows)};
    GS_TRY(run_scan(c, op, nullptr, m0, ctr + 0, s, "scan_heads", m0 * 12.0));
    gs::k_cell_setup<<<blocks_for(rows, 256), 256, 0, s>>>(ctr + 0, m0, X, 0, P<int64_t>(c->rowoff), B, nullptr,
                                                           P<gs::InstState>(c->state), false, nullptr, nullptr, 0);
    GS_HIP(hipGetLastError());
    GS_TRY(segsum(c, d, gs::SrcInit{P<double>(c->sums0), sperm, m0}, X, rows, m0, s, 4.0 + 8.0 * d));
    GS_TRY(ensure(c->gmodes, size_t(std::max<int64_t>(rows, 1)) * d * 8));
    if (rows > 0)
        gs::k_loss_mubar<<<blocks_for(rows, 256), 256, 0, s>>>(X.sum, X.cap, P<int64_t>(c->counts_i),
                                                               P<double>(c->modes_i), P<int64_t>(c->koff), B, rows,
                                                               d, gloss, P<double>(c->gmodes));
    GS_HIP(hipGetLastError());
    double* sb0 = nullptr;
    GS_TRY(adjoint_core(c, P<double>(c->gmodes), s, &sb0));
    gs_status ap = GS_OK;
    PROF_LAUNCH("adj_points", c->N * (4.0 + 8.0 * d + d * double(sizeof(T)) + 4.0),
                ap = launch_adj_points<T>(c, d, sb0, grad, x, labels, gloss, s));
    GS_TRY(ap);
    return GS_OK;
}

}  // namespace

namespace {

// ---- autotuner: candidates, and the choices kept per input shape
constexpr int kTuneCandidates = 64;

gs_config tune_candidate(int cand) {
    const int tcs[4] = {1, 2, 4, 8};
    gs_config c;
    c.merge_small = 1 - ((cand >> 3) & 1);
    c.dense_table = 1 - ((cand >> 2) & 1);
    c.tile_chunks = tcs[cand & 3];
    c.sort_digit10 = (cand >> 4) & 1;
    c.sort_tile = (cand >> 5) & 1 ? 4096 : 8192;
    return c;
}

// A shape: device, d, dtype, and the instance and point counts rounded down
// to powers of two.
struct TuneKey {
    int device, d, dtype, logB, logN;
    bool operator==(const TuneKey& o) const {
        return device == o.device && d == o.d && dtype == o.dtype && logB == o.logB && logN == o.logN;
    }
};

int floor_log2(int64_t v) { return v <= 1 ? 0 : 63 - __builtin_clzll(uint64_t(v)); }

TuneKey tune_key(int device, int d, int dtype, int B, int64_t N) {
    return TuneKey{device, d, dtype, floor_log2(B), floor_log2(N)};
}

std::mutex g_tune_mu;
std::vector<std::pair<TuneKey, gs_config>> g_tune;
bool g_tune_loaded = false;

// The cache file (environment GRIDSHIFT_TUNE_CACHE): one line per shape,
// "device d dtype logB logN merge_small dense_table tile_chunks sort_digit10 sort_tile ms".
void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("GRIDSHIFT_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof(line), f)) {
        TuneKey k{};
        gs_config c;
        double ms = 0.0;
        if (std::sscanf(line, "%d %d %d %d %d %d %d %d %d %d %lf", &k.device, &k.d, &k.dtype, &k.logB, &k.logN,
                        &c.merge_small, &c.dense_table, &c.tile_chunks, &c.sort_digit10, &c.sort_tile, &ms) != 11)
            continue;
        if ((c.merge_small | c.dense_table | c.sort_digit10) & ~1 || c.tile_chunks < 1 || c.tile_chunks > 64 ||
            (c.sort_tile != 8192 && c.sort_tile != 4096))
            continue;
        bool have = false;
        for (auto& e : g_tune)
            if (e.first == k) {
                e.second = c;
                have = true;
            }
        if (!have) g_tune.emplace_back(k, c);
    }
    std::fclose(f);
}

bool tune_lookup(const TuneKey& k, gs_config* out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    for (const auto& e : g_tune)
        if (e.first == k) {
            *out = e.second;
            return true;
        }
    return false;
}

void tune_store(const TuneKey& k, const gs_config& c, double ms) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    g_tune.emplace_back(k, c);
    const char* path = std::getenv("GRIDSHIFT_TUNE_CACHE");
    if (!path || !*path) return;
    if (FILE* f = std::fopen(path, "a")) {
        std::fprintf(f, "%d %d %d %d %d %d %d %d %d %d %.4f\n", k.device, k.d, k.dtype, k.logB, k.logN,
                     c.merge_small, c.dense_table, c.tile_chunks, c.sort_digit10, c.sort_tile, ms);
        std::fclose(f);
    }
}

// Host staging of results (pinned download and upload areas, the mapped
// block kernels publish into), kept per device across results: a result takes
// a set when it is created and gives it back when it is released, behind an
// event on the stream of its last upload (its staged bytes stay untouched
// until that copy has run).
struct HostStage {
    int device;
    void* pinned;
    size_t pinned_cap;
    char* up;
    size_t up_cap;
    int64_t* hmap;
    int64_t* hmap_dev;
    size_t hmap_cap;
    hipEvent_t done;  // recorded on release when an upload may still be in flight (else null)
};
std::mutex g_stage_mu;
std::vector<HostStage> g_stage_pool;
constexpr size_t kStagePoolMax = 16;

void stage_acquire(gs_context* c) {
    HostStage h{};
    bool found = false;
    {
        std::lock_guard<std::mutex> lk(g_stage_mu);
        for (size_t i = g_stage_pool.size(); i-- > 0;) {
            if (g_stage_pool[i].device == c->device) {
                h = g_stage_pool[i];
                g_stage_pool.erase(g_stage_pool.begin() + i);
                found = true;
                break;
            }
        }
    }
    c->stage_pooled = true;
    if (!found) return;  // the context allocates its staging on first use
    if (h.done) {
        (void)hipEventSynchronize(h.done);
        (void)hipEventDestroy(h.done);
    }
    c->pinned = h.pinned;
    c->pinned_cap = h.pinned_cap;
    c->up = h.up;
    c->up_cap = h.up_cap;
    c->hmap = h.hmap;
    c->hmap_dev = h.hmap_dev;
    c->hmap_cap = h.hmap_cap;
}

void stage_release(gs_context* c) {
    HostStage h{c->device, c->pinned, c->pinned_cap, c->up, c->up_cap, c->hmap, c->hmap_dev, c->hmap_cap, nullptr};
    if (c->up_used > 0 && hipEventCreateWithFlags(&h.done, hipEventDisableTiming) == hipSuccess &&
        hipEventRecord(h.done, c->up_stream) != hipSuccess) {
        (void)hipEventDestroy(h.done);
        h.done = nullptr;
        (void)hipStreamSynchronize(c->up_stream);
    }
    c->pinned = nullptr;
    c->up = nullptr;
    c->hmap = nullptr;
    c->hmap_dev = nullptr;
    c->pinned_cap = c->up_cap = c->hmap_cap = c->up_used = 0;
    if (!h.pinned && !h.up && !h.hmap) return;
    {
        std::lock_guard<std::mutex> lk(g_stage_mu);
        if (g_stage_pool.size() < kStagePoolMax) {
            g_stage_pool.push_back(h);
            return;
        }
    }
    if (h.done) {
        (void)hipEventSynchronize(h.done);
        (void)hipEventDestroy(h.done);
    }
    if (h.pinned) (void)hipHostFree(h.pinned);
    if (h.up) (void)hipHostFree(h.up);
    if (h.hmap) (void)hipHostFree(h.hmap);
}

}  // namespace

extern "C" {

int32_t gs_abi_version(void) { return GS_ABI_VERSION; }

const char* gs_last_error(void) { return g_last_error.c_str(); }

gs_status gs_context_create(gs_context** out) {
    if (!out) return fail(GS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int dev = 0;
    GS_HIP(hipGetDevice(&dev));
    gs_context* c = new (std::nothrow) gs_context();
    if (!c) return fail(GS_ERR_ALLOC, "out of host memory");
    c->device = dev;
    *out = c;
    return GS_OK;
}

void gs_context_destroy(gs_context* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->aux) {  // the second stream's work (checkpoint replays) ends first
        (void)hipStreamSynchronize(c->aux);
        (void)hipStreamDestroy(c->aux);
        hipEvent_t evs[] = {c->ev_start, c->ev_rep[0], c->ev_rep[1], c->ev_adj[0], c->ev_adj[1]};
        for (hipEvent_t e : evs)
            if (e) (void)hipEventDestroy(e);
    }
    DBuf* all[] = {&c->kA, &c->kB, &c->vA, &c->vB, &c->cell0, &c->kpt, &c->kappa, &c->pbuf, &c->gmap, &c->cur, &c->tmap,
                   &c->part, &c->partc, &c->hk, &c->hv, &c->ckA, &c->ckB, &c->cvA, &c->cvB, &c->ctl,
                   &c->look, &c->tilectr, &c->shist,
                   &c->sctr, &c->slook};
    for (DBuf* b : all) dbuf_release(*b);
    for (int i = 0; i < 2; ++i) {
        DBuf* tb[] = {&c->tkey[i], &c->tcnt[i], &c->tsum[i], &c->tinst[i], &c->tstart[i],
                      &c->tlen[i], &c->tfirst[i], &c->tnch[i], &c->tchoff[i]};
        for (DBuf* b : tb) dbuf_release(*b);
    }
    DBuf* tb2[] = {&c->sums0, &c->inst0, &c->wt_key, &c->wt_cnt, &c->wt_inst, &c->wt_W, &c->wt_g, &c->wt_app,
                   &c->tt_key, &c->tt_cnt, &c->tt_W, &c->tt_g, &c->tt_m, &c->sbA, &c->sbB, &c->qbuf, &c->gmodes,
                   &c->modes_i, &c->counts_i, &c->frows, &c->lossc, &c->ltab, &c->xkA, &c->xkB, &c->xvA, &c->xvB,
                   &c->ck_key, &c->ck_cnt, &c->ck_sum, &c->ck_m, &c->tune_labels, &c->tune_ref, &c->tune_tab, &c->dk,
                   &c->trk_win, &c->trk_lab, &c->trk_cnt, &c->trk_sel, &c->trk_out, &c->trk_rect, &c->trk_init,
                   &c->seq_moved, &c->seq_waiting};
    for (DBuf* b : tb2) dbuf_release(*b);
    // arena chunks go back on the stream each was allocated for
    for (const Arena::Chunk& ch : c->arena.chunks) c->alloc.free(c->alloc.ctx, ch.p, ch.stream);
    c->arena.chunks.clear();
    if (c->stage_pooled) {
        stage_release(c);
    } else {
        if (c->up_used > 0) (void)hipStreamSynchronize(c->up_stream);
        if (c->pinned) (void)hipHostFree(c->pinned);
        if (c->up) (void)hipHostFree(c->up);
        if (c->hmap) (void)hipHostFree(c->hmap);
    }
    for (hipEvent_t e : c->prof.ev) (void)hipEventDestroy(e);
    delete c;
}

gs_status gs_ctx_fit(gs_context* ctx, const void* points, gs_dtype dtype, int64_t n, int32_t d, int64_t ld, double h,
                 int32_t max_iter, int32_t* labels, gs_info* info, void* stream) {
    AllocScope as_(ctx, stream);
    if (n < 0) return fail(GS_ERR_INVALID_ARG, "n must be >= 0");
    const int64_t offsets[2] = {0, n};
    return fit_impl(ctx, points, dtype, d, ld, 1, offsets, &h, max_iter, labels, info,
                    static_cast<hipStream_t>(stream));
}

gs_status gs_ctx_fit_batched(gs_context* ctx, const void* points, gs_dtype dtype, int32_t d, int64_t ld, int32_t B,
                         const int64_t* offsets, const double* h, int32_t max_iter, int32_t* labels, gs_info* info,
                         void* stream) {
    AllocScope as_(ctx, stream);
    return fit_impl(ctx, points, dtype, d, ld, B, offsets, h, max_iter, labels, info,
                    static_cast<hipStream_t>(stream));
}

gs_status gs_fit_hsweep(gs_context* ctx, const void* points, gs_dtype dtype, int64_t n, int32_t d, int64_t ld,
                        int32_t H, const double* hs, int32_t max_iter, int32_t* labels, gs_info* info, void* stream) {
    AllocScope as_(ctx, stream);
    if (!ctx) return fail(GS_ERR_INVALID_ARG, "null context");
    if (n < 0 || H < 1 || !hs || !info) return fail(GS_ERR_INVALID_ARG, "n >= 0, H >= 1, hs and info are required");
    if (d < 1 || d > gs::kMaxDim) return fail(GS_ERR_UNSUPPORTED, "d must be in 1..6");
    if (dtype != GS_F32 && dtype != GS_F64) return fail(GS_ERR_INVALID_ARG, "dtype must be GS_F32 or GS_F64");
    if (ld < d) return fail(GS_ERR_INVALID_ARG, "ld must be >= d");
    if (n > 0 && int64_t(H) * n >= (int64_t(1) << 31))
        return fail(GS_ERR_INVALID_ARG, "H * n must stay below 2^31 points");
    if (n > 0 && (!points || !labels)) return fail(GS_ERR_INVALID_ARG, "points and labels are required");
    for (int j = 0; j < H; ++j)
        if (!(hs[j] > 0.0) || !std::isfinite(hs[j])) return fail(GS_ERR_INVALID_ARG, "h must be finite and > 0");
    if (ctx->tape_on) return fail(GS_ERR_UNSUPPORTED, "a bandwidth sweep records no trajectory");
    gs_context* c = ctx;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GS_HIP(hipSetDevice(c->device));
    std::vector<int64_t> off(size_t(H) + 1);
    for (int j = 0; j <= H; ++j) off[j] = int64_t(j) * n;
    // every instance reads the caller's n rows: position j * n + i is row i
    c->sweep_n = n;
    const gs_status rc = fit_impl(c, points, dtype, d, ld, H, off.data(), hs, max_iter, labels, info, s);
    c->sweep_n = 0;
    return rc;
}

gs_status gs_track_batched(gs_context* ctx, const void* frames, gs_dtype dtype, int32_t T, int32_t H, int32_t W,
                           int32_t dc, int32_t ntracks, const double* o0, const double* l0, const double* w0, double f,
                           double h, double eta, int32_t max_inner, int32_t n_select, int32_t max_iter,
                           double* windows, void* stream) {
    AllocScope as_(ctx, stream);
    if (!ctx) return fail(GS_ERR_INVALID_ARG, "null context");
    if (T < 1 || H < 1 || W < 1 || int64_t(H) * W >= (int64_t(1) << 31) || !frames || !o0 || !l0 || !w0 ||
        !windows || ntracks < 1)
        return fail(GS_ERR_INVALID_ARG, "T, H, W, ntracks >= 1, H * W < 2^31, frames, o0, l0, w0, windows required");
    if (dc < 1 || dc > gs::kTrackMaxChannels) return fail(GS_ERR_UNSUPPORTED, "dc must be in 1..4");
    if (dtype != GS_F32 && dtype != GS_F64) return fail(GS_ERR_INVALID_ARG, "dtype must be GS_F32 or GS_F64");
    auto pos_finite = [](double v) { return v > 0.0 && std::isfinite(v); };
    if (!pos_finite(f) || !pos_finite(h) || !pos_finite(eta))
        return fail(GS_ERR_INVALID_ARG, "f, h and eta must be finite and > 0");
    for (int t = 0; t < ntracks; ++t)
        if (!pos_finite(l0[t]) || !pos_finite(w0[t]) || !std::isfinite(o0[2 * t]) || !std::isfinite(o0[2 * t + 1]))
            return fail(GS_ERR_INVALID_ARG, "l0, w0 must be finite and > 0, o0 finite");
    if (max_inner < 1 || n_select < 1 || max_iter < 0)
        return fail(GS_ERR_INVALID_ARG, "max_inner >= 1, n_select >= 1, max_iter >= 0");
    gs_context* c = ctx;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GS_HIP(hipSetDevice(c->device));
    const size_t es = dtype == GS_F32 ? 4 : 8;
    // the initial windows of frame 0: an interval of columns and one of rows
    // each (the membership test |p - o| <= extent / 2 separates)
    auto span = [](int n, double o, double ext, int* a, int* b) {
        *a = n;
        *b = -1;
        for (int p = 0; p < n; ++p)
            if (std::fabs(double(p) - o) <= 0.5 * ext) {
                *a = std::min(*a, p);
                *b = std::max(*b, p);
            }
    };
    std::vector<gs::TrackRect> rects(static_cast<size_t>(ntracks));
    std::vector<int64_t> woff(size_t(ntracks) + 1, 0);
    for (int t = 0; t < ntracks; ++t) {
        int cx0, cx1, ry0, ry1;
        span(W, o0[2 * t], l0[t], &cx0, &cx1);
        span(H, o0[2 * t + 1], w0[t], &ry0, &ry1);
        const int ncols = cx1 >= cx0 ? cx1 - cx0 + 1 : 0, nrows = ry1 >= ry0 ? ry1 - ry0 + 1 : 0;
        rects[t] = {std::max(cx0, 0), std::max(ry0, 0), ncols, nrows, woff[t]};
        woff[t + 1] = woff[t] + int64_t(ncols) * nrows;
    }
    const int64_t ntot = woff[ntracks];
    if (ntot >= (int64_t(1) << 31)) return fail(GS_ERR_INVALID_ARG, "the initial windows hold 2^31 pixels or more");
    std::vector<gs_info> infos(static_cast<size_t>(ntracks));
    std::vector<int64_t> koff(size_t(ntracks) + 1, 0);
    if (ntot > 0) {
        GS_TRY(ensure(c->trk_win, size_t(ntot) * dc * es));
        GS_TRY(ensure(c->trk_lab, size_t(ntot) * 4));
        GS_TRY(ensure(c->trk_rect, sizeof(gs::TrackRect) * ntracks));
        GS_TRY(h2d(c, c->trk_rect.p, rects.data(), sizeof(gs::TrackRect) * ntracks, s));
        if (dtype == GS_F32)
            gs::k_track_windows<float><<<ntracks, 256, 0, s>>>(static_cast<const float*>(frames), W, dc,
                                                              P<gs::TrackRect>(c->trk_rect), P<float>(c->trk_win));
        else
            gs::k_track_windows<double><<<ntracks, 256, 0, s>>>(static_cast<const double*>(frames), W, dc,
                                                               P<gs::TrackRect>(c->trk_rect), P<double>(c->trk_win));
        GS_HIP(hipGetLastError());
        // GridShift on every window's colours (Algorithm 2, initialisation), one batched pass
        std::vector<double> hs(static_cast<size_t>(ntracks), h);
        GS_TRY(fit_impl(c, c->trk_win.p, dtype, dc, dc, ntracks, woff.data(), hs.data(), max_iter,
                        P<int32_t>(c->trk_lab), infos.data(), s));
    }
    for (int t = 0; t < ntracks; ++t) koff[t + 1] = koff[t] + infos[t].n_clusters;
    const int64_t ktot = koff[ntracks];
    // per track, the n_select largest clusters (count descending, then cluster id)
    std::vector<int32_t> sel(size_t(std::max<int64_t>(ktot, 1)), 0);
    if (ktot > 0) {
        GS_TRY(ensure(c->trk_cnt, size_t(ktot) * 8));
        GS_TRY(gs_copy_modes(c, nullptr, P<int64_t>(c->trk_cnt), nullptr, s));
        std::vector<int64_t> cnt(static_cast<size_t>(ktot));
        GS_TRY(d2h(c, cnt.data(), c->trk_cnt.p, size_t(ktot) * 8, s));
        for (int t = 0; t < ntracks; ++t) {
            const int64_t k0 = koff[t], K = koff[t + 1] - k0;
            std::vector<int32_t> order(static_cast<size_t>(K));
            for (int32_t i = 0; i < K; ++i) order[i] = i;
            std::stable_sort(order.begin(), order.end(),
                             [&](int32_t a, int32_t b) { return cnt[k0 + a] > cnt[k0 + b]; });
            for (int32_t i = 0; i < std::min<int64_t>(n_select, K); ++i) sel[k0 + order[i]] = 1;
        }
    }
    std::vector<gs::TrackInit> init(static_cast<size_t>(ntracks));
    for (int t = 0; t < ntracks; ++t) init[t] = {o0[2 * t], o0[2 * t + 1], l0[t], w0[t], woff[t], woff[t + 1], koff[t]};
    GS_TRY(ensure(c->trk_sel, sel.size() * 4));
    GS_TRY(h2d(c, c->trk_sel.p, sel.data(), sel.size() * 4, s));
    GS_TRY(ensure(c->trk_init, sizeof(gs::TrackInit) * ntracks));
    GS_TRY(h2d(c, c->trk_init.p, init.data(), sizeof(gs::TrackInit) * ntracks, s));
    const size_t wbytes = size_t(ntracks) * T * 4 * 8;
    GS_TRY(ensure(c->trk_out, wbytes + size_t(ntracks) * 4 + 256));
    int32_t* derr = reinterpret_cast<int32_t*>(static_cast<char*>(c->trk_out.p) + wbytes);
    const int tk = prof_begin(c, s, "track");
    if (dtype == GS_F32)
        gs::k_track<float><<<ntracks, gs::kTrackThreads, 0, s>>>(
            static_cast<const float*>(frames), T, H, W, dc, P<float>(c->trk_win), P<int32_t>(c->trk_lab),
            P<gs::TrackInit>(c->trk_init), P<int32_t>(c->trk_sel), f, h, eta, max_inner, P<double>(c->trk_out), derr);
    else
        gs::k_track<double><<<ntracks, gs::kTrackThreads, 0, s>>>(
            static_cast<const double*>(frames), T, H, W, dc, P<double>(c->trk_win), P<int32_t>(c->trk_lab),
            P<gs::TrackInit>(c->trk_init), P<int32_t>(c->trk_sel), f, h, eta, max_inner, P<double>(c->trk_out), derr);
    prof_end(c, s, tk, double(wbytes));
    GS_HIP(hipGetLastError());
    std::vector<char> back(wbytes + size_t(ntracks) * 4);
    GS_TRY(d2h(c, back.data(), c->trk_out.p, back.size(), s));
    for (int t = 0; t < ntracks; ++t) {
        int32_t e = 0;
        std::memcpy(&e, back.data() + wbytes + size_t(t) * 4, 4);
        if (e & 1) return fail(GS_ERR_KEY_RANGE, "a selected colour cell index is outside [-32768, 32767)");
        if (e & 2) return fail(GS_ERR_UNSUPPORTED, "the selected clusters span more than 2048 colour cells");
    }
    std::memcpy(windows, back.data(), wbytes);
    return GS_OK;
}

gs_status gs_track(gs_context* ctx, const void* frames, gs_dtype dtype, int32_t T, int32_t H, int32_t W, int32_t dc,
                   const double* o0, double l0, double w0, double f, double h, double eta, int32_t max_inner,
                   int32_t n_select, int32_t max_iter, double* windows, void* stream) {
    return gs_track_batched(ctx, frames, dtype, T, H, W, dc, 1, o0, &l0, &w0, f, h, eta, max_inner, n_select,
                            max_iter, windows, stream);
}

gs_status gs_context_set_config(gs_context* ctx, int32_t key, int32_t value) {
    if (!ctx) return fail(GS_ERR_INVALID_ARG, "null context");
    switch (key) {
        case GS_CFG_MERGE_SMALL:
            if (value != 0 && value != 1) return fail(GS_ERR_INVALID_ARG, "GS_CFG_MERGE_SMALL takes 0 or 1");
            ctx->cfg.merge_small = value;
            return GS_OK;
        case GS_CFG_TILE_CHUNKS:
            if (value < 1 || value > 64) return fail(GS_ERR_INVALID_ARG, "GS_CFG_TILE_CHUNKS takes 1..64");
            ctx->cfg.tile_chunks = value;
            return GS_OK;
        case GS_CFG_DENSE_TABLE:
            if (value != 0 && value != 1) return fail(GS_ERR_INVALID_ARG, "GS_CFG_DENSE_TABLE takes 0 or 1");
            ctx->cfg.dense_table = value;
            return GS_OK;
        case GS_CFG_SORT_DIGIT10:
            if (value != 0 && value != 1) return fail(GS_ERR_INVALID_ARG, "GS_CFG_SORT_DIGIT10 takes 0 or 1");
            ctx->cfg.sort_digit10 = value;
            return GS_OK;
        case GS_CFG_SORT_TILE:
            if (value != 8192 && value != 4096) return fail(GS_ERR_INVALID_ARG, "GS_CFG_SORT_TILE takes 8192 or 4096");
            ctx->cfg.sort_tile = value;
            return GS_OK;
    }
    return fail(GS_ERR_INVALID_ARG, "unknown configuration key");
}

gs_status gs_context_get_config(const gs_context* ctx, int32_t key, int32_t* value) {
    if (!ctx || !value) return fail(GS_ERR_INVALID_ARG, "null argument");
    switch (key) {
        case GS_CFG_MERGE_SMALL: *value = ctx->cfg.merge_small; return GS_OK;
        case GS_CFG_TILE_CHUNKS: *value = ctx->cfg.tile_chunks; return GS_OK;
        case GS_CFG_DENSE_TABLE: *value = ctx->cfg.dense_table; return GS_OK;
        case GS_CFG_SORT_DIGIT10: *value = ctx->cfg.sort_digit10; return GS_OK;
        case GS_CFG_SORT_TILE: *value = ctx->cfg.sort_tile; return GS_OK;
    }
    return fail(GS_ERR_INVALID_ARG, "unknown configuration key");
}

gs_status gs_autotune(gs_context* ctx, const void* points, gs_dtype dtype, int32_t d, int64_t ld, int32_t B,
                      const int64_t* offsets, const double* h, int32_t max_iter, int32_t reps, void* stream) {
    AllocScope as_(ctx, stream);
    if (!ctx) return fail(GS_ERR_INVALID_ARG, "null context");
    if (B < 1 || !offsets || !h || reps < 1) return fail(GS_ERR_INVALID_ARG, "B, offsets, h and reps are required");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t N = offsets[B];
    if (N < 0) return fail(GS_ERR_INVALID_ARG, "offsets must be non-decreasing from 0");
    GS_HIP(hipSetDevice(ctx->device));
    const TuneKey key = tune_key(ctx->device, d, dtype, B, N);
    gs_config cached;
    if (tune_lookup(key, &cached)) {
        ctx->cfg = cached;
        ctx->tune_hit = true;
        return GS_OK;
    }
    ctx->tune_hit = false;
    GS_TRY(ensure(ctx->tune_labels, size_t(std::max<int64_t>(N, 1)) * 4));
    GS_TRY(ensure(ctx->tune_ref, size_t(std::max<int64_t>(N, 1)) * 4));
    std::vector<gs_info> info(B), info0(B);
    const bool prof = ctx->prof.on;
    ctx->prof.on = false;
    const gs_config keep = ctx->cfg;
    gs_config best = keep;
    double best_ms = 0.0;
    bool first = true;
    gs_status rc = GS_OK;
    int64_t rows0 = 0;
    int64_t* ctr = nullptr;
    for (int cand = 0; cand < kTuneCandidates && rc == GS_OK; ++cand) {
        ctx->cfg = tune_candidate(cand);
        double t_min = 0.0;
        for (int r = 0; r <= reps; ++r) {  // the first run is a warm-up
            const auto t0 = std::chrono::steady_clock::now();
            rc = fit_impl(ctx, points, dtype, d, ld, B, offsets, h, max_iter, P<int32_t>(ctx->tune_labels),
                          info.data(), s);
            const auto t1 = std::chrono::steady_clock::now();
            if (rc != GS_OK) break;
            const double t = std::chrono::duration<double, std::milli>(t1 - t0).count();
            if (r == 1 || (r > 1 && t < t_min)) t_min = t;
        }
        if (rc != GS_OK) break;
        // every candidate runs the same binary64 operations in the same
        // order: its labels, counts and sums must equal the first's bit for bit
        int64_t rows = 0;
        for (int b = 0; b < B; ++b) rows += info[b].n_clusters;
        const size_t tab = size_t(std::max<int64_t>(rows, 1)) * (size_t(d) + 1) * 8;
        if (cand == 0) {
            info0 = info;
            rows0 = rows;
            GS_TRY(ensure(ctx->tune_tab, 2 * tab + 64));
            ctr = reinterpret_cast<int64_t*>(static_cast<char*>(ctx->tune_tab.p) + 2 * tab);
            if (N > 0)
                GS_HIP(hipMemcpyAsync(ctx->tune_ref.p, ctx->tune_labels.p, size_t(N) * 4, hipMemcpyDeviceToDevice, s));
        }
        bool same = rows == rows0;
        for (int b = 0; b < B && same; ++b)
            same = info[b].n_clusters == info0[b].n_clusters && info[b].n_iter == info0[b].n_iter &&
                   info[b].flags == info0[b].flags && info[b].n_cells0 == info0[b].n_cells0;
        if (same && rows > 0) {
            // the cluster table, dense: sums then counts (cand 0 into the first half)
            char* dst = static_cast<char*>(ctx->tune_tab.p) + (cand == 0 ? 0 : tab);
            gs::k_copy_modes<<<blocks_for(rows, 256), 256, 0, s>>>(
                table(ctx, ctx->cur_tab), P<gs::InstState>(ctx->state), P<int64_t>(ctx->koff), B, rows, d, nullptr,
                reinterpret_cast<int64_t*>(dst + size_t(rows) * d * 8), reinterpret_cast<double*>(dst));
            GS_HIP(hipGetLastError());
        }
        if (same && cand > 0) {
            k_fill_u64<<<1, 64, 0, s>>>(reinterpret_cast<uint64_t*>(ctr), 1, 0);
            if (N > 0)
                k_count_diff_u32<<<blocks_for(N, 256), 256, 0, s>>>(P<uint32_t>(ctx->tune_labels),
                                                                    P<uint32_t>(ctx->tune_ref), N, ctr);
            if (rows > 0)
                k_count_diff_u32<<<blocks_for(int64_t(tab / 4), 256), 256, 0, s>>>(
                    reinterpret_cast<const uint32_t*>(static_cast<char*>(ctx->tune_tab.p) + tab),
                    reinterpret_cast<const uint32_t*>(ctx->tune_tab.p), int64_t(tab / 4), ctr);
            GS_HIP(hipGetLastError());
            int64_t diff = 0;
            GS_TRY(d2h(ctx, &diff, ctr, sizeof(diff), s));
            same = diff == 0;
        }
        if (!same) {
            rc = fail(GS_ERR_DEVICE, "autotune: launch configuration " + std::to_string(cand) +
                                         " gave results that differ from configuration 0");
            break;
        }
        if (first || t_min < best_ms) {
            best_ms = t_min;
            best = ctx->cfg;
            first = false;
        }
    }
    ctx->prof.on = prof;
    ctx->cfg = rc == GS_OK ? best : keep;
    if (rc == GS_OK) tune_store(key, best, best_ms);
    return rc;
}

gs_status gs_profile_enable(gs_context* ctx, const char* prefix) {
    if (!ctx) return fail(GS_ERR_INVALID_ARG, "null context");
    ctx->prof.on = prefix != nullptr;
    ctx->prof.filter = prefix ? prefix : "";
    return GS_OK;
}

gs_status gs_profile_reset(gs_context* ctx) {
    if (!ctx) return fail(GS_ERR_INVALID_ARG, "null context");
    prof_flush(ctx, false);  // launches recorded before the reset are not counted
    ctx->prof.names.clear();
    ctx->prof.ms.clear();
    ctx->prof.bytes.clear();
    ctx->prof.launches.clear();
    return GS_OK;
}

int32_t gs_profile_count(const gs_context* ctx) {
    if (!ctx) return 0;
    // launches since the last fit (backward, loss) are accumulated first
    prof_flush(const_cast<gs_context*>(ctx), true);
    return int32_t(ctx->prof.names.size());
}

gs_status gs_profile_entry(const gs_context* ctx, int32_t i, const char** name, double* total_ms, int64_t* launches,
                           double* bytes) {
    if (!ctx || i < 0 || i >= int32_t(ctx->prof.names.size())) return fail(GS_ERR_INVALID_ARG, "bad profile index");
    if (name) *name = ctx->prof.names[i].c_str();
    if (total_ms) *total_ms = ctx->prof.ms[i];
    if (launches) *launches = ctx->prof.launches[i];
    if (bytes) *bytes = ctx->prof.bytes[i];
    return GS_OK;
}

gs_status gs_context_set_update(gs_context* ctx, int32_t rule) {
    if (!ctx) return fail(GS_ERR_INVALID_ARG, "null context");
    if (rule != GS_UPDATE_PARALLEL && rule != GS_UPDATE_SEQUENTIAL)
        return fail(GS_ERR_INVALID_ARG, "rule must be GS_UPDATE_PARALLEL or GS_UPDATE_SEQUENTIAL");
    ctx->rule = rule;
    return GS_OK;
}

gs_status gs_context_get_update(const gs_context* ctx, int32_t* rule) {
    if (!ctx || !rule) return fail(GS_ERR_INVALID_ARG, "null context or output");
    *rule = ctx->rule;
    return GS_OK;
}

gs_status gs_context_set_tape(gs_context* ctx, int32_t ckpt_every) {
    if (!ctx) return fail(GS_ERR_INVALID_ARG, "null context");
    if (ckpt_every < 0) return fail(GS_ERR_INVALID_ARG, "the checkpoint interval must be >= 0");
    ctx->tape_on = ckpt_every != 0;
    ctx->ckpt_every = ckpt_every;
    return GS_OK;
}

gs_status gs_ctx_backward(gs_context* ctx, const double* grad_modes, double* grad_points, void* stream) {
    AllocScope as_(ctx, stream);
    GS_TRY(check_tape(ctx));
    gs_context* c = ctx;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GS_HIP(hipSetDevice(c->device));
    if (c->N == 0) return GS_OK;
    if (!grad_points) return fail(GS_ERR_INVALID_ARG, "grad_points is NULL");
    double* sb0 = nullptr;
    GS_TRY(adjoint_core(c, grad_modes, s, &sb0));
    gs_status ap = GS_OK;
    PROF_LAUNCH("adj_points", c->N * (4.0 + 8.0 * c->d),
                ap = launch_adj_points<float>(c, c->d, sb0, grad_points, nullptr, nullptr, nullptr, s));
    GS_TRY(ap);
    return GS_OK;
}

gs_status gs_ctx_point_mode_loss(gs_context* ctx, const void* points, const int32_t* labels, double* loss, void* stream) {
    AllocScope as_(ctx, stream);
    GS_TRY(check_tape(ctx));
    gs_context* c = ctx;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GS_HIP(hipSetDevice(c->device));
    if (!loss) return fail(GS_ERR_INVALID_ARG, "loss is NULL");
    if (c->N > 0 && (!points || !labels)) return fail(GS_ERR_INVALID_ARG, "points and labels are required");
    if (c->dtype == GS_F32) return loss_fwd(c, static_cast<const float*>(points), labels, loss, s);
    return loss_fwd(c, static_cast<const double*>(points), labels, loss, s);
}

gs_status gs_ctx_point_mode_loss_backward(gs_context* ctx, const void* points, const int32_t* labels,
                                      const double* grad_loss, double* grad_points, void* stream) {
    AllocScope as_(ctx, stream);
    GS_TRY(check_tape(ctx));
    gs_context* c = ctx;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GS_HIP(hipSetDevice(c->device));
    if (c->N == 0) return GS_OK;
    if (!points || !labels || !grad_loss || !grad_points)
        return fail(GS_ERR_INVALID_ARG, "points, labels, grad_loss and grad_points are required");
    if (c->dtype == GS_F32)
        return loss_bwd(c, static_cast<const float*>(points), labels, grad_loss, grad_points, s);
    return loss_bwd(c, static_cast<const double*>(points), labels, grad_loss, grad_points, s);
}

static gs_status prepare_copy(gs_context* c, hipStream_t s, int64_t* rows) {
    if (!c) return fail(GS_ERR_INVALID_ARG, "null context");
    if (!c->has_result) return fail(GS_ERR_STATE, "the context holds no fit result");
    GS_HIP(hipSetDevice(c->device));
    int64_t rows_total = 0;  // the cluster row offsets are on the device since the fit
    for (int b = 0; b < c->B; ++b) rows_total += c->st[b].K;
    (void)s;
    *rows = rows_total;
    return GS_OK;
}

gs_status gs_copy_modes(gs_context* ctx, double* modes, int64_t* counts, double* sums, void* stream) {
    AllocScope as_(ctx, stream);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int64_t rows = 0;
    GS_TRY(prepare_copy(ctx, s, &rows));
    if (rows == 0) return GS_OK;
    gs::CellTable t = table(ctx, ctx->cur_tab);
    gs::k_copy_modes<<<blocks_for(rows, 256), 256, 0, s>>>(t, P<gs::InstState>(ctx->state), P<int64_t>(ctx->koff),
                                                           ctx->B, rows, ctx->d, modes, counts, sums);
    GS_HIP(hipGetLastError());
    return GS_OK;
}

gs_status gs_copy_keys(gs_context* ctx, int64_t* keys, void* stream) {
    AllocScope as_(ctx, stream);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int64_t rows = 0;
    GS_TRY(prepare_copy(ctx, s, &rows));
    if (rows == 0) return GS_OK;
    if (!keys) return fail(GS_ERR_INVALID_ARG, "keys is NULL");
    gs::CellTable t = table(ctx, ctx->cur_tab);
    gs::k_copy_keys<<<blocks_for(rows, 256), 256, 0, s>>>(t, P<gs::InstState>(ctx->state), P<gs::InstParam>(ctx->param),
                                                          P<int64_t>(ctx->koff), ctx->B, rows, ctx->d, keys);
    GS_HIP(hipGetLastError());
    return GS_OK;
}

// ---------------------------------------------------------------------------
// per-fit results (each owns a context whose device memory comes from the
// caller's allocator when one is given)
// ---------------------------------------------------------------------------
}  // extern "C"

struct gs_result {
    gs_context* ctx = nullptr;
    void* stream = nullptr;
    const int32_t* labels = nullptr;  // the caller's labels of the fit (for the loss)
    std::vector<gs_info> info;
    std::vector<int64_t> koff;
    // Calls on another stream than the fit's: that stream first waits for the
    // fit stream (memory the result allocates is handed out for the fit
    // stream), and an event recorded after the call lets the release wait
    // for it.
    mutable hipEvent_t fit_ev = nullptr;
    mutable std::vector<std::pair<void*, hipEvent_t>> side;
};

namespace {

gs_status side_begin(const gs_result* r, void* stream) {
    if (stream == r->stream) return GS_OK;
    GS_HIP(hipSetDevice(r->ctx->device));
    if (!r->fit_ev) GS_HIP(hipEventCreateWithFlags(&r->fit_ev, hipEventDisableTiming));
    GS_HIP(hipEventRecord(r->fit_ev, static_cast<hipStream_t>(r->stream)));
    GS_HIP(hipStreamWaitEvent(static_cast<hipStream_t>(stream), r->fit_ev, 0));
    return GS_OK;
}

// After a call on `stream` (whatever its status: kernels may have been queued).
gs_status side_end(const gs_result* r, void* stream, gs_status rc) {
    if (stream == r->stream) return rc;
    hipEvent_t ev = nullptr;
    for (auto& pr : r->side)
        if (pr.first == stream) ev = pr.second;
    if (!ev) {
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
            return rc;
        }
        r->side.emplace_back(stream, ev);
    }
    if (hipEventRecord(ev, static_cast<hipStream_t>(stream)) != hipSuccess)
        (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
    return rc;
}

gs_status result_fit(const void* points, gs_dtype dtype, int32_t d, int64_t ld, int32_t B, const int64_t* offsets,
                     const double* h, int32_t max_iter, int32_t ckpt_every, const gs_allocator* a, void* stream,
                     int32_t* labels, gs_result** out) {
    if (!out) return fail(GS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (a && (!a->alloc || !a->free)) return fail(GS_ERR_INVALID_ARG, "the allocator needs alloc and free");
    if (B < 1) return fail(GS_ERR_INVALID_ARG, "B must be >= 1");
    gs_context* c = nullptr;
    GS_TRY(gs_context_create(&c));
    if (a) {
        c->alloc = *a;
        c->has_alloc = true;
        c->use_arena = true;
        c->own_stream = stream;
        c->has_own_stream = true;
    }
    stage_acquire(c);
    gs_result* r = new (std::nothrow) gs_result();
    if (!r) {
        gs_context_destroy(c);
        return fail(GS_ERR_ALLOC, "out of host memory");
    }
    r->ctx = c;
    r->stream = stream;
    r->labels = labels;
    r->info.assign(size_t(B), gs_info{});
    gs_status rc = gs_context_set_tape(c, ckpt_every);
    if (rc == GS_OK)
        rc = gs_ctx_fit_batched(c, points, dtype, d, ld, B, offsets, h, max_iter, labels, r->info.data(), stream);
    if (rc != GS_OK) {
        const std::string msg = gs_last_error();
        gs_result_free(r);
        g_last_error = msg;
        return rc;
    }
    r->koff.assign(size_t(B) + 1, 0);
    for (int32_t b = 0; b < B; ++b) r->koff[b + 1] = r->koff[b] + r->info[b].n_clusters;
    *out = r;
    return GS_OK;
}

}  // namespace

extern "C" {

gs_status gs_fit(const gs_problem* p, const gs_allocator* a, void* stream, int32_t* labels, gs_result** out) {
    if (!p) return fail(GS_ERR_INVALID_ARG, "problem is NULL");
    if (p->n < 0) return fail(GS_ERR_INVALID_ARG, "n must be >= 0");
    const int64_t offsets[2] = {0, p->n};
    return result_fit(p->points, p->dtype, p->d, p->ld, 1, offsets, &p->h, p->max_iter, p->ckpt_every, a, stream,
                      labels, out);
}

gs_status gs_fit_batched(const void* points, gs_dtype dtype, int32_t d, int32_t B, const int64_t* offsets,
                         const double* h, int32_t max_iter, int32_t ckpt_every, const gs_allocator* a, void* stream,
                         int32_t* labels, gs_result** out) {
    return result_fit(points, dtype, d, d, B, offsets, h, max_iter, ckpt_every, a, stream, labels, out);
}

gs_status gs_result_info(const gs_result* r, int32_t instance, gs_info* out) {
    if (!r || !out) return fail(GS_ERR_INVALID_ARG, "null result or output");
    if (instance < 0 || size_t(instance) >= r->info.size()) return fail(GS_ERR_INVALID_ARG, "no such instance");
    *out = r->info[size_t(instance)];
    return GS_OK;
}

gs_status gs_result_offsets(const gs_result* r, int64_t* k_offsets) {
    if (!r || !k_offsets) return fail(GS_ERR_INVALID_ARG, "null result or output");
    std::memcpy(k_offsets, r->koff.data(), r->koff.size() * sizeof(int64_t));
    return GS_OK;
}

gs_status gs_result_copy(const gs_result* r, double* modes, int64_t* counts, void* stream) {
    if (!r) return fail(GS_ERR_INVALID_ARG, "null result");
    GS_TRY(side_begin(r, stream));
    return side_end(r, stream, gs_copy_modes(r->ctx, modes, counts, nullptr, stream));
}

gs_status gs_backward(const gs_result* r, const double* grad_modes, double* grad_points, void* stream) {
    if (!r) return fail(GS_ERR_INVALID_ARG, "null result");
    GS_TRY(side_begin(r, stream));
    return side_end(r, stream, gs_ctx_backward(r->ctx, grad_modes, grad_points, stream));
}

gs_status gs_point_mode_loss(const gs_result* r, const void* points, double* loss, void* stream) {
    if (!r) return fail(GS_ERR_INVALID_ARG, "null result");
    GS_TRY(side_begin(r, stream));
    return side_end(r, stream, gs_ctx_point_mode_loss(r->ctx, points, r->labels, loss, stream));
}

gs_status gs_point_mode_loss_backward(const gs_result* r, const void* points, const double* grad_loss,
                                      double* grad_points, void* stream) {
    if (!r) return fail(GS_ERR_INVALID_ARG, "null result");
    GS_TRY(side_begin(r, stream));
    return side_end(r, stream,
                    gs_ctx_point_mode_loss_backward(r->ctx, points, r->labels, grad_loss, grad_points, stream));
}

void gs_result_free(gs_result* r) {
    if (!r) return;
    if (r->ctx) {
        // Stream-ordered, without waiting on the host: the fit stream waits
        // for every other stream a result call used, then the memory goes
        // back to the caller's allocator for the fit stream (a caching
        // allocator hands it out again only to work ordered after that), and
        // the host staging to the per-device pool behind an event.  Memory
        // from hipMalloc (no allocator) is given back with hipFree, which
        // waits for the device.
        hipStream_t s = static_cast<hipStream_t>(r->stream);
        (void)hipSetDevice(r->ctx->device);
        for (auto& pr : r->side) (void)hipStreamWaitEvent(s, pr.second, 0);
        gs_context_destroy(r->ctx);
        for (auto& pr : r->side) (void)hipEventDestroy(pr.second);
        if (r->fit_ev) (void)hipEventDestroy(r->fit_ev);
    }
    delete r;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// plain fit without allocation: every device buffer of the fit is carved out
// of one fixed array of device memory
// ---------------------------------------------------------------------------
// The fixed array.  Host code never uses its name as an address: each device
// has its own copy, whose address hipGetSymbolAddress gives (fixed_setup).
static __device__ __align__(256) unsigned char scratch[GS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kFixedPublished = 4096;  // head of the array: counters and states the kernels publish
constexpr size_t kFixedStage = 16384;     // host staging per device and direction
constexpr int kFixedDevices = 16;

struct FixedDevice {
    bool ready = false;
    void* scratch = nullptr;  // this device's copy of `scratch`
    alignas(256) char down[kFixedStage];
    alignas(256) char up[kFixedStage];
    alignas(256) int64_t published[kFixedPublished / sizeof(int64_t)];
};
FixedDevice g_fixed[kFixedDevices];
std::mutex g_fixed_mu;

// Once per device, with that device current: the device address of its copy
// of the array.
gs_status fixed_setup(int dev, FixedDevice** out) {
    if (dev < 0 || dev >= kFixedDevices)
        return fail(GS_ERR_UNSUPPORTED, "gs_fit_noalloc supports devices 0.." + std::to_string(kFixedDevices - 1));
    std::lock_guard<std::mutex> lk(g_fixed_mu);
    FixedDevice& fd = g_fixed[dev];
    if (!fd.ready) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(GS_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        fd.scratch = ptr;
        fd.ready = true;
    }
    *out = &fd;
    return GS_OK;
}

// Bump allocation over the array (after its published head); nothing is
// given back before the call ends, and the next call starts again at 0.
struct Bump {
    char* base;
    size_t cap, used, failed;
};
void* bump_alloc(void* ctx, size_t bytes, void*) {
    Bump* b = static_cast<Bump*>(ctx);
    const size_t need = (bytes + 255) & ~size_t(255);
    if (need > b->cap - b->used) {
        b->failed = bytes;
        return nullptr;
    }
    void* p = b->base + b->used;
    b->used += need;
    return p;
}
void bump_free(void*, void*, void*) {}

}  // namespace

extern "C" {

gs_status gs_fit_noalloc(const gs_problem* p, void* stream, int32_t* labels, double* modes, int64_t* counts,
                         int64_t max_clusters, gs_info* info) {
    if (!p || !info) return fail(GS_ERR_INVALID_ARG, "problem and info are required");
    if (p->n < 0) return fail(GS_ERR_INVALID_ARG, "n must be >= 0");
    if (p->n > GS_NOALLOC_MAX_POINTS)
        return fail(GS_ERR_INVALID_ARG, "gs_fit_noalloc takes at most " + std::to_string(GS_NOALLOC_MAX_POINTS) +
                                            " points (its fixed scratch is " +
                                            std::to_string(GS_NOALLOC_SCRATCH_BYTES >> 20) + " MiB); got " +
                                            std::to_string(p->n));
    if (p->ckpt_every != 0) return fail(GS_ERR_UNSUPPORTED, "gs_fit_noalloc records no trajectory (ckpt_every 0)");
    if (max_clusters < 0) return fail(GS_ERR_INVALID_ARG, "max_clusters must be >= 0");
    int dev = 0;
    GS_HIP(hipGetDevice(&dev));
    FixedDevice* fd = nullptr;
    GS_TRY(fixed_setup(dev, &fd));
    hipStream_t s = static_cast<hipStream_t>(stream);

    // a fresh context each call (epochs, tickets and look-back storage start
    // cleared, as in a new context), its device memory from the array
    Bump bump{static_cast<char*>(fd->scratch) + kFixedPublished, size_t(GS_NOALLOC_SCRATCH_BYTES) - kFixedPublished,
              0, 0};
    gs_context c;
    c.device = dev;
    c.alloc = gs_allocator{bump_alloc, bump_free, &bump};
    c.has_alloc = true;
    c.cfg.dense_table = 0;  // neighbour lookups through the per-round hash (the dense table can reach 1 GiB)
    c.fixed_host = true;
    c.pinned = fd->down;
    c.pinned_cap = sizeof(fd->down);
    c.up = fd->up;
    c.up_cap = sizeof(fd->up);
    c.hmap = fd->published;
    c.hmap_dev = static_cast<int64_t*>(fd->scratch);
    c.hmap_cap = kFixedPublished;
    c.hmap_on_device = true;
    AllocScope as_(&c, stream);
    const int64_t offsets[2] = {0, p->n};
    gs_status rc = fit_impl(&c, p->points, p->dtype, p->d, p->ld, 1, offsets, &p->h, p->max_iter, labels, info, s);
    if (rc == GS_ERR_ALLOC)
        return fail(GS_ERR_ALLOC, "gs_fit_noalloc: the fit needs more than the fixed " +
                                      std::to_string(GS_NOALLOC_SCRATCH_BYTES >> 20) + " MiB of scratch (" +
                                      std::to_string(bump.used) + " bytes in use, " + std::to_string(bump.failed) +
                                      " more asked for)");
    if (rc != GS_OK) return rc;
    const int64_t K = info->n_clusters;
    if (K > max_clusters)
        return fail(GS_ERR_INVALID_ARG, "the fit found " + std::to_string(K) + " clusters; modes and counts hold " +
                                            std::to_string(max_clusters));
    if (K > 0) {
        if (!modes && !counts) return GS_OK;
        gs::k_copy_modes<<<blocks_for(K, 256), 256, 0, s>>>(table(&c, c.cur_tab), P<gs::InstState>(c.state),
                                                            P<int64_t>(c.koff), 1, K, c.d, modes, counts, nullptr);
        GS_HIP(hipGetLastError());
    }
    // the next call reuses the array: this call's work ends first
    GS_HIP(hipStreamSynchronize(s));
    return GS_OK;
}

}  // extern "C"
