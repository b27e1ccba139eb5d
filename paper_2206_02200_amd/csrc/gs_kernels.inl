// GridShift pipeline kernels for gfx950 (included by gs_api.hip: one translation unit).
//
// Binning (Section 2.1 (i), Algorithm 1 initialisation):
//   k_bbox        per-instance box of the integer keys floor(fl(x/h)), plus the
//                 non-finite and key-range checks
//   k_make_keys   packed 32/64-bit key per point (instance = top digit) and the
//                 digit histograms of every radix pass
//   (radix sort)  stable sort of (key, point index), gs_sort.hip
//   k_scan        one-pass look-back scans: run heads -> cell ids, chunk offsets
//   k_cell_setup  run lengths, chunk counts, instance of every cell
//   k_segsum_*    canonical pairwise sums R over every cell's members (one wave
//                 per aligned 256-member chunk, then the chunk subtrees)
// Rounds while some instance still has many cells (Section 2.1 (ii)-(v)):
//   k_hash_*      open-addressing table packed key -> cell index
//   k_shift       3^d neighbour fold in ascending key, p = N / W, landing key
//   k_decide      per-instance stop test (no neighbour / max_iter)
//   k_merge_prep  landing keys of applying instances, stationarity check
//   (radix sort + k_scan + k_cell_setup + k_segsum) the merge of Eq. 3-4
//   k_compose     initial cell -> current cell maps
// Remaining rounds: k_tail, one 1024-thread workgroup per instance with its
// whole cell table in LDS, looping on the device until it stops.
// Outputs: k_labels, k_copy_modes, k_copy_keys.
//
// All floating point is binary64 without contraction (-ffp-contract=off).
#include <math.h>

#include "gs_device.hpp"
#include "gs_pipeline.hpp"

namespace gs {

// ===========================================================================
// small helpers
// ===========================================================================
template <typename T>
__device__ __forceinline__ double load_coord(const T* __restrict__ x, int64_t row, int64_t ld, int k) {
    return double(x[row * ld + k]);
}

__device__ __forceinline__ uint64_t dbits(double v) { return __double_as_longlong(v); }

// floor(fl(v / h)) as a double.
__device__ __forceinline__ double cell_floor(double v, double h) { return floor(v / h); }

// ===========================================================================
// point-tile staging
// ===========================================================================
// Rows are cut into tiles that never straddle two instances.  A block walks
// its tile in chunks of at most kStageBytes of coordinates: it copies a chunk
// into LDS with consecutive lanes reading consecutive dwords (whole cache
// lines per wave instruction), issues the next chunk's loads, and meanwhile
// each thread reads whole rows of the current chunk back from LDS.
constexpr int kBoxThreads = 256;
constexpr int kStageBytes = 24576;
constexpr int kMaxChunkRows = 2048;

// Rows per chunk for d coordinates of `elem` bytes: a multiple of the block
// size, at most kMaxChunkRows, with rows * d * elem <= bytes.
__host__ __device__ constexpr int chunk_rows(int d, int elem, int bytes = kStageBytes) {
    return (bytes / (d * elem)) / kBoxThreads * kBoxThreads > kMaxChunkRows
               ? kMaxChunkRows
               : (bytes / (d * elem)) / kBoxThreads * kBoxThreads;
}
// The key producers stage half as much per chunk: fewer registers hold the
// next chunk's loads and less LDS, so more workgroups share a compute unit
// (their tiles, sized for the box kernel, take twice as many chunks).
constexpr int kKeyStageBytes = kStageBytes / 2;

struct RowTile {
    int64_t r0, r1;  // rows [r0, r1) of one instance
    int32_t inst;
    int32_t pad;
};

// Rows of part `blockIdx.x % split` of tile `blockIdx.x / split`: the tile's
// chunks of R rows shared out evenly over `split` workgroups.
__device__ inline RowTile tile_part(const RowTile* __restrict__ tiles, int split, int R) {
    RowTile tl = tiles[blockIdx.x / split];
    if (split > 1) {
        const int part = int(blockIdx.x % split);
        const int64_t nc = (tl.r1 - tl.r0 + R - 1) / R;
        const int64_t c0 = nc * part / split, c1 = nc * (part + 1) / split;
        const int64_t r1 = tl.r0 + c1 * R;
        tl.r0 += c0 * R;
        tl.r1 = r1 < tl.r1 ? r1 : tl.r1;
        if (tl.r0 > tl.r1) tl.r0 = tl.r1;
    }
    return tl;
}

template <typename T, int D, int BYTES = kStageBytes>
struct Stager {
    static constexpr int R = chunk_rows(D, int(sizeof(T)), BYTES);
    static constexpr int DW = R * D * int(sizeof(T)) / 4;           // dwords of a full chunk
    static constexpr int PER = (DW + kBoxThreads - 1) / kBoxThreads;  // dwords per thread
    uint32_t v[PER];
    // Issue the loads of rows [r0, r0 + rows) (contiguous rows only).
    __device__ __forceinline__ void load(const T* __restrict__ x, int64_t ld, int64_t r0, int rows) {
        if (ld != D) return;
        const uint32_t* src = reinterpret_cast<const uint32_t*>(x + r0 * D);
        const int ndw = rows * D * int(sizeof(T)) / 4;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = int(threadIdx.x) + i * kBoxThreads;
            v[i] = e < ndw ? src[e] : 0u;
        }
    }
    // Rows [r0, r0 + rows) into lds as rows * D consecutive elements.
    __device__ __forceinline__ void store(const T* __restrict__ x, int64_t ld, int64_t r0, int rows, T* lds) {
        if (ld == D) {
            uint32_t* dst = reinterpret_cast<uint32_t*>(lds);
            const int ndw = rows * D * int(sizeof(T)) / 4;
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int e = int(threadIdx.x) + i * kBoxThreads;
                if (e < ndw) dst[e] = v[i];
            }
        } else {
            for (int e = int(threadIdx.x); e < rows * D; e += kBoxThreads) {
                const int r = e / D, k = e - r * D;
                lds[e] = x[(r0 + r) * ld + k];
            }
        }
    }
};

// ===========================================================================
// bbox: per instance and dimension, min/max of the coordinates
// ===========================================================================
// floor(fl(v / h)) is non-decreasing in v (h > 0; division and floor are
// monotone), so the box of the cell coordinates is [floor(fl(min/h)),
// floor(fl(max/h))]: the device reduces the raw coordinates only, the host
// divides the two extremes.  Each block reduces one tile and merges the
// result into one of `ncopies` copies of its instance's box,
// [B][ncopies][kMaxDim][2], as order-preserving 64-bit images of the
// binary64 values (initialised to all ones / zero) with atomic min/max;
// spreading the blocks over copies keeps atomics on one address few (the
// host combines the copies).  Non-finite coordinates set bit 0 of
// counters[2] and are left out of the box.
__device__ __forceinline__ uint64_t ordered_bits(double v) {
    const uint64_t u = uint64_t(__double_as_longlong(v));
    return (u >> 63) ? ~u : (u | (1ull << 63));
}

template <typename T, int D>
__global__ __launch_bounds__(kBoxThreads) void k_bbox_tiles(const T* __restrict__ x, int64_t ld,
                                                            const RowTile* __restrict__ tiles,
                                                            uint64_t* __restrict__ bbox, int ncopies,
                                                            int64_t* __restrict__ counters, int split) {
    using S = Stager<T, D>;
    constexpr int R = S::R;
    constexpr int RPT = R / kBoxThreads;
    __shared__ T stage[R * D];
    __shared__ uint64_t red[kBoxThreads / kWave][2 * D];
    const RowTile tl = tile_part(tiles, split, R);
    if (tl.r0 >= tl.r1) return;
    const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
    T mn[D], mx[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        mn[k] = T(INFINITY);
        mx[k] = T(-INFINITY);
    }
    int err = 0;
    S sg;
    int64_t c0 = tl.r0;
    int crows = int(tl.r1 - c0 < R ? tl.r1 - c0 : R);
    sg.load(x, ld, c0, crows);
    while (crows > 0) {
        sg.store(x, ld, c0, crows, stage);
        __syncthreads();
        const int64_t n0 = c0 + crows;
        const int nrows = int(tl.r1 - n0 < R ? tl.r1 - n0 : R);
        if (nrows > 0) sg.load(x, ld, n0, nrows);  // in flight while this chunk is reduced
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int r = tid + i * kBoxThreads;
            if (r >= crows) continue;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const T v = stage[r * D + k];
                if (!isfinite(v)) {
                    err = 1;
                    continue;
                }
                mn[k] = fmin(mn[k], v);
                mx[k] = fmax(mx[k], v);
            }
        }
        __syncthreads();  // every row read before the next chunk is stored
        c0 = n0;
        crows = nrows;
    }
    uint64_t kmn[D], kmx[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        kmn[k] = ordered_bits(double(mn[k]));
        kmx[k] = ordered_bits(double(mx[k]));
        for (int off = 32; off >= 1; off >>= 1) {
            const uint64_t a = __shfl_xor((unsigned long long)kmn[k], off, kWave);
            const uint64_t c = __shfl_xor((unsigned long long)kmx[k], off, kWave);
            kmn[k] = a < kmn[k] ? a : kmn[k];
            kmx[k] = c > kmx[k] ? c : kmx[k];
        }
        if (lane == 0) {
            red[w][2 * k] = kmn[k];
            red[w][2 * k + 1] = kmx[k];
        }
    }
    if (__ballot(err != 0) && lane == 0) atomicOr((unsigned long long*)&counters[2], 1ull);
    __syncthreads();
    if (tid < 2 * D) {
        const bool isMin = (tid & 1) == 0;
        uint64_t a = isMin ? ~0ull : 0ull;
        for (int ww = 0; ww < kBoxThreads / kWave; ++ww) {
            const uint64_t c = red[ww][tid];
            a = isMin ? (c < a ? c : a) : (c > a ? c : a);
        }
        uint64_t* dst = bbox + (int64_t(tl.inst) * ncopies + int(blockIdx.x) % ncopies) * 2 * kMaxDim + tid;
        if (isMin) __hip_atomic_fetch_min(dst, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else __hip_atomic_fetch_max(dst, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ===========================================================================
// packed keys + radix digit histograms
// ===========================================================================
// Adds one key per valid lane to the LDS digit histograms of `npasses`
// passes.  Neighbouring points usually share a cell, so lanes are grouped in
// runs of consecutive lanes with the same digit: the first lane of a run adds
// the run's length (one LDS atomic per run instead of one per lane).
template <typename K>
__device__ __forceinline__ void wave_digit_hist(uint32_t* hl, K key, bool valid, int npasses, int digit) {
    const uint64_t act = __ballot(valid);
    if (!act) return;
    const int lane = lane_id();
    const uint32_t dmask = (1u << digit) - 1u;
    K prev;
    if constexpr (sizeof(K) == 4) {
        prev = K(__shfl_up(uint32_t(key), 1, kWave));
    } else {
        const uint32_t lo = __shfl_up(uint32_t(key), 1, kWave), hi = __shfl_up(uint32_t(key >> 32), 1, kWave);
        prev = K((uint64_t(hi) << 32) | lo);
    }
    const bool prev_valid = lane > 0 && ((act >> (lane - 1)) & 1ull);
    const uint64_t above = ~((2ull << lane) - 1ull);  // lanes after this one (none for lane 63)
    for (int p = 0; p < npasses; ++p) {
        const uint32_t dgt = uint32_t(key >> (digit * p)) & dmask;
        const bool head = valid && (!prev_valid || (uint32_t(prev >> (digit * p)) & dmask) != dgt);
        const uint64_t brk = __ballot(head || !valid) & above;  // a run ends where another starts
        if (head) {
            const int end = brk ? __ffsll((unsigned long long)brk) - 1 : kWave;
            atomicAdd(&hl[(p << digit) + dgt], uint32_t(end - lane));
        }
    }
}

template <typename T, typename K, int D>
__global__ __launch_bounds__(kBoxThreads) void k_make_keys(const T* __restrict__ x, int64_t ld,
                                                           const RowTile* __restrict__ tiles,
                                                           const InstParam* __restrict__ param,
                                                           K* __restrict__ keys, int npasses, int digit,
                                                           uint32_t* __restrict__ hist, int split) {
    using S = Stager<T, D, kKeyStageBytes>;
    constexpr int R = S::R;
    constexpr int RPT = R / kBoxThreads;
    __shared__ T stage[R * D];
    extern __shared__ uint32_t hl[];  // pass p, digit v at (p << digit) + v (npasses << digit words, sized at launch)
    __shared__ InstParam sp;
    const RowTile tl = tile_part(tiles, split, R);
    if (tl.r0 >= tl.r1) return;
    const int tid = threadIdx.x;
    const int nh = npasses << digit;
    for (int i = tid; i < nh; i += kBoxThreads) hl[i] = 0;
    if (tid == 0) sp = param[tl.inst];
    S sg;
    int64_t c0 = tl.r0;
    int crows = int(tl.r1 - c0 < R ? tl.r1 - c0 : R);
    sg.load(x, ld, c0, crows);
    while (crows > 0) {
        sg.store(x, ld, c0, crows, stage);
        __syncthreads();
        const int64_t n0 = c0 + crows;
        const int nrows = int(tl.r1 - n0 < R ? tl.r1 - n0 : R);
        if (nrows > 0) sg.load(x, ld, n0, nrows);  // in flight while this chunk is keyed
        const double hh = sp.h;
        K kv[RPT];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int r = tid + i * kBoxThreads;
            if constexpr (sizeof(K) == 4) {
                // the whole key is below 2^32, so is every term: 32-bit
                // arithmetic, with q - lo exact in binary64 and below 2^32
                uint32_t key = uint32_t(sp.base);
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const double q = cell_floor(double(stage[(r < crows ? r : 0) * D + k]), hh);
                    key += uint32_t(q - double(sp.lo[k])) * uint32_t(sp.stride[k]);
                }
                kv[i] = K(key);
            } else {
                uint64_t key = sp.base;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const double q = cell_floor(double(stage[(r < crows ? r : 0) * D + k]), hh);
                    key += uint64_t(int64_t(q) - sp.lo[k]) * sp.stride[k];
                }
                kv[i] = K(key);
            }
            if (r < crows) keys[c0 + r] = kv[i];
        }
#pragma unroll
        for (int i = 0; i < RPT; ++i) wave_digit_hist(hl, kv[i], tid + i * kBoxThreads < crows, npasses, digit);
        __syncthreads();  // every row read before the next chunk is stored
        c0 = n0;
        crows = nrows;
    }
    uint32_t* hc = hist + (blockIdx.x % kHistCopies) * kHistStride;
    for (int i = tid; i < nh; i += kBoxThreads)
        if (hl[i]) atomicAdd(&hc[hist_index(i, digit)], hl[i]);
}

// Keys of a bandwidth sweep: H instances that share one point set of n rows
// (instance j owns positions j * n .. j * n + n - 1, its keys with bandwidth
// param[j].h).  The tiles cover the n source rows once; workgroup (t, g)
// keys the staged rows of tile t for the g-th group of ceil(H / gridDim.y)
// consecutive instances, so the points are read once per group (from L2
// after the first) and the instances spread over many workgroups.
template <typename T, typename K, int D>
__global__ __launch_bounds__(kBoxThreads) void k_make_keys_sweep(const T* __restrict__ x, int64_t ld,
                                                                 const RowTile* __restrict__ tiles,
                                                                 const InstParam* __restrict__ param, int H,
                                                                 int64_t n, K* __restrict__ keys, int npasses,
                                                                 int digit, uint32_t* __restrict__ hist) {
    using S = Stager<T, D, kKeyStageBytes>;
    constexpr int R = S::R;
    constexpr int RPT = R / kBoxThreads;
    __shared__ T stage[R * D];
    extern __shared__ uint32_t hl[];  // pass p, digit v at (p << digit) + v (npasses << digit words, sized at launch)
    const RowTile tl = tiles[blockIdx.x];
    if (tl.r0 >= tl.r1) return;
    const int tid = threadIdx.x;
    const int nh = npasses << digit;
    for (int i = tid; i < nh; i += kBoxThreads) hl[i] = 0;
    S sg;
    int64_t c0 = tl.r0;
    int crows = int(tl.r1 - c0 < R ? tl.r1 - c0 : R);
    sg.load(x, ld, c0, crows);
    while (crows > 0) {
        sg.store(x, ld, c0, crows, stage);
        __syncthreads();
        const int64_t n0 = c0 + crows;
        const int nrows = int(tl.r1 - n0 < R ? tl.r1 - n0 : R);
        if (nrows > 0) sg.load(x, ld, n0, nrows);  // in flight while this chunk is keyed
        const int hg = (H + int(gridDim.y) - 1) / int(gridDim.y);
        const int j0 = int(blockIdx.y) * hg, j1 = j0 + hg < H ? j0 + hg : H;
        for (int j = j0; j < j1; ++j) {
            const InstParam& sp = param[j];
            const double hh = sp.h;
            K kv[RPT];
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int r = tid + i * kBoxThreads;
                if constexpr (sizeof(K) == 4) {
                    uint32_t key = uint32_t(sp.base);
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        const double q = cell_floor(double(stage[(r < crows ? r : 0) * D + k]), hh);
                        key += uint32_t(q - double(sp.lo[k])) * uint32_t(sp.stride[k]);
                    }
                    kv[i] = K(key);
                } else {
                    uint64_t key = sp.base;
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        const double q = cell_floor(double(stage[(r < crows ? r : 0) * D + k]), hh);
                        key += uint64_t(int64_t(q) - sp.lo[k]) * sp.stride[k];
                    }
                    kv[i] = K(key);
                }
                if (r < crows) keys[int64_t(j) * n + c0 + r] = kv[i];
            }
#pragma unroll
            for (int i = 0; i < RPT; ++i) wave_digit_hist(hl, kv[i], tid + i * kBoxThreads < crows, npasses, digit);
        }
        __syncthreads();  // every row read before the next chunk is stored
        c0 = n0;
        crows = nrows;
    }
    uint32_t* hc = hist + (blockIdx.x % kHistCopies) * kHistStride;
    for (int i = tid; i < nh; i += kBoxThreads)
        if (hl[i]) atomicAdd(&hc[hist_index(i, digit)], hl[i]);
}

// ===========================================================================
// one-pass look-back scan over positions (tile = 8192, wave-striped slots)
// ===========================================================================
constexpr int kScanThreads = 512;
constexpr int kScanItems = kScanTile / kScanThreads;  // 16

// Scan operations: load(p) reads everything position p needs (the kernel
// issues every load of a thread before any store), value() is its value
// (< 2^32, and a tile's sum stays below 2^32), emit() writes its results.

// Run heads of a sorted key array: emits the cell table rows and, when
// member_cell is given, the map member -> cell (a scatter by member index;
// without it the permutation is read at heads only).
template <typename K>
struct HeadsOp {
    const K* key;            // sorted keys [n]
    const uint32_t* perm;    // sorted position -> member index
    uint64_t* cell_key;      // [m] packed key of every cell
    uint32_t* cell_start;    // [m]
    uint32_t* cell_first;    // [m] member at the start of the run
    uint32_t* member_cell;   // [n] member index -> cell id, or nullptr
    static constexpr bool kBinary = true;  // values are 0 or 1
    // the key itself is not kept between load and emit (fewer registers per
    // item, so more workgroups per compute unit): a head reads it again
    struct Item {
        uint32_t mem;
        uint32_t head;
    };
    __device__ Item load(int64_t p) const {
        Item it;
        const K k = key[p];
        it.head = (p == 0 || k != key[p - 1]) ? 1u : 0u;
        it.mem = (member_cell || it.head) ? perm[p] : 0u;
        return it;
    }
    __device__ static uint32_t value(const Item& it) { return it.head; }
    __device__ void emit(int64_t p, uint64_t excl, const Item& it) const {
        const uint64_t cid = excl + it.head - 1;
        if (it.head) {
            cell_key[cid] = uint64_t(key[p]);
            cell_start[cid] = uint32_t(p);
            cell_first[cid] = it.mem;
        }
        if (member_cell) member_cell[it.mem] = uint32_t(cid);
    }
};

// Cell of every point from its key, the keys in point order (the map a
// heads scan would scatter, written in point order instead): through the
// dense key table, which holds the cells of the table under the current
// epoch ...
constexpr int kCellOfPerThread = 4;
template <typename K>
__global__ __launch_bounds__(256) void k_cell_of_points_dense(const K* __restrict__ key, int64_t n,
                                                              const uint64_t* __restrict__ dk,
                                                              uint32_t* __restrict__ cell) {
    const int64_t i0 = int64_t(blockIdx.x) * (256 * kCellOfPerThread) + threadIdx.x;
    K k[kCellOfPerThread];
#pragma unroll
    for (int u = 0; u < kCellOfPerThread; ++u) {
        const int64_t i = i0 + u * 256;
        k[u] = i < n ? key[i] : K(0);
    }
    uint64_t e[kCellOfPerThread];
#pragma unroll
    for (int u = 0; u < kCellOfPerThread; ++u) e[u] = i0 + u * 256 < n ? dk[uint64_t(k[u])] : 0ull;
#pragma unroll
    for (int u = 0; u < kCellOfPerThread; ++u)
        if (i0 + u * 256 < n) cell[i0 + u * 256] = uint32_t(e[u]);
}

// ... or by binary search over the m <= kTailCells sorted cell keys, staged
// in LDS by every workgroup.
template <typename K>
__global__ __launch_bounds__(256) void k_cell_of_points_search(const K* __restrict__ key, int64_t n,
                                                               const uint64_t* __restrict__ cell_key, int m,
                                                               uint32_t* __restrict__ cell) {
    __shared__ uint64_t ck[kTailCells];
    for (int j = threadIdx.x; j < m; j += 256) ck[j] = cell_key[j];
    __syncthreads();
    const int64_t i0 = int64_t(blockIdx.x) * (256 * kCellOfPerThread) + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kCellOfPerThread; ++u) {
        const int64_t i = i0 + u * 256;
        if (i >= n) break;
        const uint64_t k = uint64_t(key[i]);
        int lo = 0, hi = m - 1;  // the cell with key k exists: the first index whose key is >= k
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (ck[mid] < k) lo = mid + 1; else hi = mid;
        }
        cell[i] = uint32_t(lo);
    }
}

// Exclusive scan of a u32 array.
struct ExclOp {
    const uint32_t* in;
    uint32_t* out;
    static constexpr bool kBinary = false;
    struct Item {
        uint32_t v;
    };
    __device__ Item load(int64_t p) const { return Item{in[p]}; }
    __device__ static uint32_t value(const Item& it) { return it.v; }
    __device__ void emit(int64_t p, uint64_t excl, const Item&) const { out[p] = uint32_t(excl); }
};

// n_ptr: device count of positions (read once per block); total: device
// result (sum of all values).  Tiles take their index from tile_ctr.
template <class Op>
__global__ __launch_bounds__(kScanThreads) void k_scan(Op op, const int64_t* __restrict__ n_ptr, int64_t n_val,
                                                       uint64_t* __restrict__ look, uint32_t* __restrict__ tile_ctr,
                                                       uint32_t tile_base, uint32_t epoch,
                                                       int64_t* __restrict__ total, int64_t* __restrict__ total_host) {
    constexpr int W = kScanThreads / kWave;
    __shared__ int64_t s_tile;
    __shared__ uint32_t wtot[W];
    __shared__ uint64_t s_excl;
    const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
    if (tid == 0) s_tile = atomicAdd(tile_ctr, 1u) - tile_base;
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t n = n_ptr ? *n_ptr : n_val;
    const int64_t t0 = tile * kScanTile;
    if (t0 >= n && tile > 0) return;

    typename Op::Item it[kScanItems];
    uint32_t v[kScanItems];
    uint32_t incl[kScanItems];  // tile-local inclusive sums
    uint32_t run = 0;
    // all loads first, so that their latency overlaps
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t p = t0 + int64_t(w) * (kWave * kScanItems) + i * kWave + lane;
        if (p < n) it[i] = op.load(p);
    }
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t p = t0 + int64_t(w) * (kWave * kScanItems) + i * kWave + lane;
        v[i] = p < n ? Op::value(it[i]) : 0u;
    }
    if constexpr (Op::kBinary) {  // 0/1 values: prefix counts from ballots
        const uint64_t le = lanemask_lt() | (1ull << lane);
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const uint64_t bal = __ballot(v[i] != 0);
            incl[i] = run + uint32_t(__popcll(bal & le));
            run += uint32_t(__popcll(bal));
        }
    } else {
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const uint32_t xs = wave_incl_scan_u32(v[i]);
            incl[i] = run + xs;
            run += uint32_t(__builtin_amdgcn_readlane(int(xs), kWave - 1));
        }
    }
    if (lane == 0) wtot[w] = run;
    __syncthreads();
    if (w == 0) {  // wave 0 publishes the tile total and looks back
        uint64_t tot = 0;
        for (int ww = 0; ww < W; ++ww) tot += wtot[ww];
        uint64_t excl = 0;
        if (tile == 0) {
            if (lane == 0) lb_store(look, lb_pack(epoch, kFlagPrefix, tot));
        } else {
            if (lane == 0) lb_store(look + tile, lb_pack(epoch, kFlagAgg, tot));
            excl = lb_exclusive_wave(look, tile, epoch);
            if (lane == 0) lb_store(look + tile, lb_pack(epoch, kFlagPrefix, excl + tot));
        }
        if (lane == 0) {
            s_excl = excl;
            if (t0 + kScanTile >= n) {
                *total = int64_t(excl + tot);
                if (total_host) *total_host = int64_t(excl + tot);
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t acc = 0;
        for (int ww = 0; ww < W; ++ww) {
            const uint32_t c = wtot[ww];
            wtot[ww] = acc;
            acc += c;
        }
    }
    __syncthreads();
    const uint64_t base = s_excl + wtot[w];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t p = t0 + int64_t(w) * (kWave * kScanItems) + i * kWave + lane;
        if (p < n) op.emit(p, base + incl[i] - v[i], it[i]);
    }
}

// ===========================================================================
// cell setup after a heads scan
// ===========================================================================
// mode 0 (binning): instance from the member's row; mode 1 (merge): from the
// member cell's instance, and flag instances whose round merged cells.
// With `ranges` it also records each instance's row range [cs, ce) of the
// new table (the ranges of instances without cells were cleared beforehand).
// With `cur` / `dk` (a device-wide round follows the binning) it also starts
// the map initial cell -> current cell (identity) and enters the cells in
// the dense key table under `epoch`.
__global__ void k_cell_setup(const int64_t* __restrict__ m_ptr, int64_t npos, CellTable t, int mode,
                             const int64_t* __restrict__ row_off, int B, const int32_t* __restrict__ old_inst,
                             InstState* __restrict__ st, bool ranges, uint32_t* __restrict__ cur,
                             uint64_t* __restrict__ dk, uint32_t epoch) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t m = *m_ptr;
    bool merged = false;
    int b = 0;
    if (c < m) {
        const uint32_t s0 = t.start[c];
        const uint32_t s1 = (c + 1 < m) ? t.start[c + 1] : uint32_t(npos);
        const uint32_t len = s1 - s0;
        t.len[c] = len;
        t.nch[c] = (len + kChunk - 1) / kChunk;
        int bp = -1;  // instance of the previous cell
        if (mode == 0) {
            b = inst_of_row(row_off, B, int64_t(t.first[c]));
            if (c > 0) bp = inst_of_row(row_off, B, int64_t(t.first[c - 1]));
        } else {
            b = old_inst[t.first[c]];
            if (c > 0) bp = old_inst[t.first[c - 1]];
            merged = len > 1 && st[b].apply;
        }
        t.inst[c] = b;
        if (cur) cur[c] = uint32_t(c);
        if (dk) dk[t.key[c]] = (uint64_t(epoch) << 32) | uint64_t(c);
        if (ranges) {
            if (bp != b) {
                st[b].cs = c;
                if (bp >= 0) st[bp].ce = c;
            }
            if (c == m - 1) st[b].ce = m;
        }
    }
    if (mode == 1) wave_flag_or(&st[b].changed, merged);
}

// ===========================================================================
// canonical segmented sums
// ===========================================================================
// Point members: value = (double)x[row][k], count 1.
template <typename T>
struct SrcPoints {
    const T* x;
    int64_t ld;
    const uint32_t* perm;
    uint32_t src_n = 0;  // > 0: positions are instances of n shared rows (a bandwidth sweep): row = position mod n
    __device__ int64_t load(int64_t p, double* v, int d, int64_t) const {
        const int64_t r = src_n ? int64_t(perm[p] % src_n) : int64_t(perm[p]);
        for (int k = 0; k < d; ++k) v[k] = load_coord(x, r, ld, k);
        return 1;
    }
};

// Merge members (old cells): value fl(C_j * p_j) if the instance applies the
// round, else the unchanged sum S_j; count C_j.
struct SrcMerge {
    const double* pbuf;   // [d][cap] shifted positions
    const double* sum;    // [d][cap] old sums
    const int64_t* cnt;   // old counts
    const int32_t* inst;  // old instance ids
    const InstState* st;
    const uint32_t* perm;
    int64_t cap;
    __device__ int64_t load(int64_t p, double* v, int d, int64_t) const {
        const int64_t j = perm[p];
        const int64_t C = cnt[j];
        if (st[inst[j]].apply) {
            for (int k = 0; k < d; ++k) v[k] = double(C) * pbuf[k * cap + j];
        } else {
            for (int k = 0; k < d; ++k) v[k] = sum[k * cap + j];
        }
        return C;
    }
};

constexpr int kSegThreads = 256;

// One wave per chunk task: the R subtree of 256 members aligned at the
// cell's first member.  Lane l holds members l, 64 + l, 128 + l and 192 + l
// of the chunk (consecutive lanes read consecutive members); the subtree is
// the four 64-leaf trees over the lanes, combined as (t0 + t1) + (t2 + t3).
// Workgroup b's place in a grid of G when workgroups go round-robin to the
// chip's 8 XCDs (b % 8) and each XCD is to take one contiguous share.
__device__ __forceinline__ int64_t xcd_contiguous(int64_t b, int64_t G) {
    constexpr int X = 8;
    const int64_t x = b % X, k = b / X, q = G / X, r = G % X;
    return x * q + (x < r ? x : r) + k;
}

// With xcd != 0 the workgroups that hold tasks are remapped so that each XCD
// sums one contiguous range of chunk tasks: the rows the chunks gather then
// stay within one XCD's L2 (the point sets of a batch are contiguous in the
// task order).
template <int D, class Src>
__global__ __launch_bounds__(kSegThreads) void k_segsum_chunks(Src src, CellTable t, const int64_t* __restrict__ m_ptr,
                                                               const int64_t* __restrict__ tasks_ptr,
                                                               double* __restrict__ part,
                                                               int64_t* __restrict__ partc, int64_t pcap, int xcd) {
    constexpr int TPB = kSegThreads / kWave;  // tasks per workgroup
    const int64_t ntask = *tasks_ptr;
    const int64_t G = (ntask + TPB - 1) / TPB;  // workgroups that hold tasks (the grid is sized for a bound)
    if (int64_t(blockIdx.x) >= G) return;
    const int64_t blk = xcd ? xcd_contiguous(blockIdx.x, G) : int64_t(blockIdx.x);
    const int64_t task = (blk * kSegThreads + threadIdx.x) / kWave;
    const int lane = lane_id();
    if (task >= ntask) return;
    const int64_t m = *m_ptr;
    // last cell with choff <= task, by a 65-way search: the lanes test 64
    // increasing positions strictly inside (lo, hi) at once, and the bracket
    // shrinks to the two positions around the last one that passes
    // (choff[lo] <= task < choff[hi], choff[m] read as infinite)
    int64_t lo = 0, hi = m;
    while (hi - lo > 1) {
        const int64_t span = hi - lo;
        const int64_t pos = span <= kWave ? lo + 1 + lane : lo + (int64_t(lane + 1) * span) / (kWave + 1);
        const bool ok = pos < hi && t.choff[pos] <= uint32_t(task);
        const uint64_t pass = __ballot(ok), fail = __ballot(pos < hi && !ok);
        const int64_t new_lo = pass ? int64_t(__shfl((long long)pos, 63 - __clzll(pass), kWave)) : lo;
        const int64_t new_hi = fail ? int64_t(__shfl((long long)pos, __ffsll((unsigned long long)fail) - 1, kWave)) : hi;
        lo = new_lo;
        hi = new_hi;
        if (span <= kWave) break;  // every position in (lo, hi) was tested
    }
    const int64_t c = lo;
    const int64_t ch = task - t.choff[c];
    const int64_t len = t.len[c];
    const int64_t p0 = int64_t(t.start[c]) + ch * kChunk;
    const int64_t cnt = (len - ch * kChunk) < kChunk ? (len - ch * kChunk) : kChunk;
    double acc[D];
    int64_t cacc = 0;
    {
        double a[4][D];
        int64_t ca[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t r = i * kWave + lane;
            if (r < cnt) {
                ca[i] = src.load(p0 + r, a[i], D, c);
            } else {
                ca[i] = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) a[i][k] = -0.0;
            }
        }
        double sl[4][D];
        int64_t cs[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (i * kWave < cnt) {
#pragma unroll
                for (int k = 0; k < D; ++k) sl[i][k] = wave_tree_sum(a[i][k]);
                cs[i] = wave_tree_sum_i64(ca[i]);
            } else {
#pragma unroll
                for (int k = 0; k < D; ++k) sl[i][k] = -0.0;
                cs[i] = 0;
            }
        }
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] = (sl[0][k] + sl[1][k]) + (sl[2][k] + sl[3][k]);
        cacc = (cs[0] + cs[1]) + (cs[2] + cs[3]);
    }
    if (lane == 0) {
        if (t.nch[c] == 1) {
#pragma unroll
            for (int k = 0; k < D; ++k) t.sum[k * t.cap + c] = acc[k];
            t.cnt[c] = cacc;
        } else {
#pragma unroll
            for (int k = 0; k < D; ++k) part[k * pcap + task] = acc[k];
            partc[task] = cacc;
        }
    }
}

__device__ __forceinline__ double ld_agent(const double* p) {
    return __longlong_as_double(
        (long long)__hip_atomic_load((uint64_t*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_agent(double* p, double v) {
    __hip_atomic_store((uint64_t*)p, (uint64_t)__double_as_longlong(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t ld_agent_i(const int64_t* p) {
    return __hip_atomic_load(const_cast<int64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent_i(int64_t* p, int64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One wave per cell with more than one chunk: combine the chunk subtrees 64
// at a time (aligned, -0 padded) until one value is left; that is R.
template <int D>
__global__ __launch_bounds__(kSegThreads) void k_segsum_levels(CellTable t, const int64_t* __restrict__ m_ptr,
                                                               double* __restrict__ part, int64_t* __restrict__ partc,
                                                               int64_t pcap) {
    const int64_t c = (int64_t(blockIdx.x) * kSegThreads + threadIdx.x) / kWave;
    const int lane = lane_id();
    if (c >= *m_ptr) return;
    int64_t len = t.nch[c];
    if (len <= 1) return;
    const int64_t base = t.choff[c];
    if (len <= kWave) {  // one level: the partials come from the previous kernel
        double v[D];
#pragma unroll
        for (int k = 0; k < D; ++k) v[k] = lane < len ? part[k * pcap + base + lane] : -0.0;
        int64_t cv = lane < len ? partc[base + lane] : 0;
#pragma unroll
        for (int k = 0; k < D; ++k) v[k] = wave_tree_sum(v[k]);
        cv = wave_tree_sum_i64(cv);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < D; ++k) t.sum[k * t.cap + c] = v[k];
            t.cnt[c] = cv;
        }
        return;
    }
    // Each level replaces every 64 partials by their R subtree (piece pc of
    // the level -> partial pc of the next).  PC pieces are loaded at a time;
    // piece pc's result is written only after every load of pieces <= pc is
    // done (pieces are read in ascending order, and piece pc is written to
    // position pc <= 64 * pc), so the level reads only its own inputs.
    constexpr int PC = 4;
    while (len > 1) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int64_t pieces = (len + kWave - 1) / kWave;
        for (int64_t pc0 = 0; pc0 < pieces; pc0 += PC) {
            double v[PC][D];
            int64_t cv[PC];
#pragma unroll
            for (int u = 0; u < PC; ++u) {
                const int64_t i = (pc0 + u) * kWave + lane;
#pragma unroll
                for (int k = 0; k < D; ++k) v[u][k] = i < len ? ld_agent(&part[k * pcap + base + i]) : -0.0;
                cv[u] = i < len ? ld_agent_i(&partc[base + i]) : 0;
            }
#pragma unroll
            for (int u = 0; u < PC; ++u) {
#pragma unroll
                for (int k = 0; k < D; ++k) v[u][k] = wave_tree_sum(v[u][k]);
                cv[u] = wave_tree_sum_i64(cv[u]);
            }
            if (lane == 0) {
#pragma unroll
                for (int u = 0; u < PC; ++u) {
                    if (pc0 + u >= pieces) break;
#pragma unroll
                    for (int k = 0; k < D; ++k) st_agent(&part[k * pcap + base + pc0 + u], v[u][k]);
                    st_agent_i(&partc[base + pc0 + u], cv[u]);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        }
        len = pieces;
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < D; ++k) t.sum[k * t.cap + c] = ld_agent(&part[k * pcap + base]);
        t.cnt[c] = ld_agent_i(&partc[base]);
    }
}

// ===========================================================================
// wide rounds
// ===========================================================================
constexpr uint64_t kEmpty = ~0ull;

__device__ __forceinline__ uint64_t hash_slot(uint64_t key, int logcap) {
    uint64_t z = key + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z >> (64 - logcap);
}

__global__ void k_hash_clear(uint64_t* __restrict__ hk, int64_t cap) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < cap) hk[i] = kEmpty;
}

__global__ void k_hash_insert(const uint64_t* __restrict__ key, int64_t m, uint64_t* __restrict__ hk,
                              uint32_t* __restrict__ hv, int logcap) {
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const uint64_t k = key[j];
    const uint64_t mask = (1ull << logcap) - 1;
    uint64_t s = hash_slot(k, logcap);
    for (;;) {
        const uint64_t prev = atomicCAS((unsigned long long*)&hk[s], (unsigned long long)kEmpty,
                                        (unsigned long long)k);
        if (prev == kEmpty || prev == k) {
            hv[s] = uint32_t(j);
            return;
        }
        s = (s + 1) & mask;
    }
}

__device__ __forceinline__ int64_t hash_find(const uint64_t* __restrict__ hk, const uint32_t* __restrict__ hv,
                                             uint64_t k, int logcap) {
    const uint64_t mask = (1ull << logcap) - 1;
    uint64_t s = hash_slot(k, logcap);
    for (;;) {
        const uint64_t e = hk[s];
        if (e == k) return hv[s];
        if (e == kEmpty) return -1;
        s = (s + 1) & mask;
    }
}

// Neighbour lookup through the open-addressing hash.  find_all looks up N
// keys of a lane together: the first slot of every key is loaded at once,
// then the keys still probing (linear probing) load their next slots
// together, and the values of the keys found are loaded at once; the chain
// of dependent loads is the longest probe sequence instead of their sum.
struct HashLookup {
    const uint64_t* hk;
    const uint32_t* hv;
    int logcap;
    __device__ __forceinline__ int64_t find(uint64_t k) const { return hash_find(hk, hv, k, logcap); }
    template <int N>
    __device__ __forceinline__ void find_all(const uint64_t* key, const bool* want, int64_t* idx) const {
        const uint64_t mask = (1ull << logcap) - 1;
        uint64_t slot[N];
        int st[N];  // 0: probing, 1: found, 2: absent or not wanted
#pragma unroll
        for (int i = 0; i < N; ++i) {
            slot[i] = hash_slot(key[i], logcap);
            st[i] = want[i] ? 0 : 2;
        }
        for (;;) {
            uint64_t e[N];
#pragma unroll
            for (int i = 0; i < N; ++i) e[i] = st[i] == 0 ? hk[slot[i]] : 0ull;
            bool probing = false;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                if (st[i] != 0) continue;
                if (e[i] == key[i]) {
                    st[i] = 1;
                } else if (e[i] == kEmpty) {
                    st[i] = 2;
                } else {
                    slot[i] = (slot[i] + 1) & mask;
                    probing = true;
                }
            }
            if (!probing) break;
        }
#pragma unroll
        for (int i = 0; i < N; ++i) idx[i] = st[i] == 1 ? int64_t(hv[slot[i]]) : -1;
    }
};

// Neighbour lookup through a dense table over the whole packed key range:
// entry k holds (epoch << 32) | cell for the keys of the current table and
// older epochs elsewhere, so it is never cleared between rounds.
struct DenseLookup {
    const uint64_t* dk;
    uint32_t epoch;
    __device__ __forceinline__ int64_t find(uint64_t k) const {
        const uint64_t e = dk[k];
        return uint32_t(e >> 32) == epoch ? int64_t(uint32_t(e)) : -1;
    }
    template <int N>
    __device__ __forceinline__ void find_all(const uint64_t* key, const bool* want, int64_t* idx) const {
        uint64_t e[N];
#pragma unroll
        for (int i = 0; i < N; ++i) e[i] = want[i] ? dk[key[i]] : 0ull;
#pragma unroll
        for (int i = 0; i < N; ++i) idx[i] = want[i] && uint32_t(e[i] >> 32) == epoch ? int64_t(uint32_t(e[i])) : -1;
    }
};

__global__ void k_dense_insert(const uint64_t* __restrict__ key, int64_t m, uint64_t* __restrict__ dk,
                               uint32_t epoch) {
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j < m) dk[key[j]] = (uint64_t(epoch) << 32) | uint64_t(j);
}

// Shift of every cell of an active instance (Eq. 1-2, parallel form Eq. 6).
// One wave per cell: the lanes probe the 3^D neighbour keys j+v in parallel,
// v enumerated lexicographically (dimension 0 most significant, which is
// ascending packed key); the cells found are compacted in that order; then
// lane k folds dimension k left to right and lane D adds the integer weight.
// p = N / W and the landing key floor(p/h) follow.
constexpr int kShiftWaves = 4;
constexpr int64_t kDenseMax = int64_t(1) << 27;  // largest key range with a dense lookup table (1 GiB)
constexpr int kSlabMax = 4096;       // most columns of a tail's column table


__host__ __device__ constexpr int pow3(int d) { return d == 0 ? 1 : 3 * pow3(d - 1); }

// One step of the sequential form's device-wide shift: moved[cell] =
// (epoch << 8) | step of the step that moved it; waiting[step] = epoch when
// some cell still waited after that step.  epoch is unique per round and
// fit (24 bits), so neither array needs clearing.  moved == nullptr: the
// parallel form.
struct SeqStep {
    uint32_t* moved;
    uint32_t* waiting;
    uint32_t epoch;
    int step;
};

template <int D, class Lookup>
__global__ __launch_bounds__(kShiftWaves * kWave) void k_shift(CellTable t, int64_t m,
                                                               const InstParam* __restrict__ param,
                                                               InstState* __restrict__ st, Lookup lk,
                                                               double* __restrict__ pbuf,
                                                               uint64_t* __restrict__ kappa,
                                                               int32_t* __restrict__ Wout, SeqStep seq, int xcd) {
    constexpr int NOFF = pow3(D);
    __shared__ uint32_t list[kShiftWaves][NOFF];
    __shared__ double gval[kShiftWaves][D][kWave];  // gathered rows of found cells
    __shared__ int64_t gcnt[kShiftWaves][kWave];
    const int w = threadIdx.x / kWave, lane = lane_id();
    // xcd != 0: each XCD takes a contiguous range of cells, whose neighbours'
    // rows (the same point set's cells) then stay in its L2
    const int64_t blk = xcd ? xcd_contiguous(blockIdx.x, gridDim.x) : int64_t(blockIdx.x);
    const int64_t j = blk * kShiftWaves + w;
    if (j >= m) return;  // wave-uniform
    const bool sequential = seq.moved != nullptr;
    if (sequential) {
        // no cell was left waiting by the previous step: nothing to do
        if (seq.step > 0 && seq.waiting[seq.step - 1] != seq.epoch) return;
        if ((seq.moved[j] >> 8) == seq.epoch) return;  // moved in an earlier step
    }
    const int b = t.inst[j];
    if (!st[b].active) return;
    const InstParam& P = param[b];
    const uint64_t key = t.key[j];
    // the cell's own count and sum, for the stationarity test at the end
    const int64_t own_cnt = t.cnt[j];
    const double own_sum = lane < D ? t.sum[int64_t(lane) * t.cap + j] : 0.0;
    const uint64_t local = key - P.base;
    int64_t crd[D];
#pragma unroll
    for (int k = 0; k < D; ++k) crd[k] = int64_t((local / P.stride[k]) % uint64_t(P.E[k]));
    // Sequential form (Eq. 5) in the colour-by-colour order (bit D-1-k of a
    // colour = parity of integer coordinate k; cells of one colour are never
    // neighbours): a cell moves in the first step (launch) after all its
    // neighbours of lower colours have moved, and reads their fl(C_k * p_k);
    // its neighbours of higher colours wait for it, so it reads their sums.
    int own_col = 0;
    if (sequential) {
#pragma unroll
        for (int k = 0; k < D; ++k) own_col = (own_col << 1) | int((crd[k] + P.lo[k]) & 1);
    }
    const uint64_t lt = lanemask_lt();
    // every probe of the cell first (independent loads, all in flight), then
    // the found cells compacted in probe order
    constexpr int NIT = (NOFF + kWave - 1) / kWave;
    int64_t idx[NIT];
    bool upd[NIT];  // the neighbour was moved earlier in this sweep
    uint64_t nks[NIT];
    bool want[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int r = it * kWave + lane;
        nks[it] = 0;
        want[it] = false;
        upd[it] = false;
        if (r < NOFF) {
            int rr = r;
            bool inside = true;
            uint64_t nk = key;
            int flip = 0;  // colour bits in which the neighbour differs
#pragma unroll
            for (int k = D - 1; k >= 0; --k) {
                const int v = rr % 3 - 1;
                rr /= 3;
                const int64_t c = crd[k] + v;
                inside = inside && c >= 0 && c < P.E[k];
                nk += uint64_t(int64_t(v)) * P.stride[k];
                flip |= (v != 0 ? 1 : 0) << (D - 1 - k);
            }
            upd[it] = sequential && (own_col ^ flip) < own_col;
            nks[it] = nk;
            want[it] = inside;
        }
    }
    lk.template find_all<NIT>(nks, want, idx);
    if (sequential) {  // wait unless every lower-colour neighbour moved in an earlier step
        bool wait = false;
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            if (idx[it] >= 0 && upd[it]) {
                const uint32_t mv = seq.moved[idx[it]];
                wait = wait || (mv >> 8) != seq.epoch || int(mv & 255u) >= seq.step;
            }
        }
        if (__ballot(wait)) {
            if (lane == 0) seq.waiting[seq.step] = seq.epoch;
            return;
        }
    }
    int nfound = 0;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const uint64_t bal = __ballot(idx[it] >= 0);
        if (idx[it] >= 0) list[w][nfound + __popcll(bal & lt)] = uint32_t(idx[it]) | (upd[it] ? 0x80000000u : 0u);
        nfound += __popcll(bal);
    }
    __builtin_amdgcn_wave_barrier();
    // The found cells' rows are gathered kWave at a time by the whole wave (a
    // cell per lane: its D values and its count) into LDS; then lane k < D
    // folds dimension k left to right over them and lane D adds the counts.
    double acc = 0.0;
    int64_t W = 0;
    for (int q0 = 0; q0 < nfound; q0 += kWave) {
        if (q0 + lane < nfound) {
            const uint32_t e = list[w][q0 + lane];
            const uint32_t k = e & 0x7fffffffu;
            const int64_t ck = t.cnt[k];
            double v[D];
#pragma unroll
            for (int dd = 0; dd < D; ++dd)
                v[dd] = (e >> 31) ? pbuf[int64_t(dd) * t.cap + k] : t.sum[int64_t(dd) * t.cap + k];
#pragma unroll
            for (int dd = 0; dd < D; ++dd) gval[w][dd][lane] = (e >> 31) ? double(ck) * v[dd] : v[dd];
            gcnt[w][lane] = ck;
        }
        __builtin_amdgcn_wave_barrier();
        const int nq = nfound - q0 < kWave ? nfound - q0 : kWave;
        if (lane < D) {
            for (int u0 = 0; u0 < nq; u0 += 16) {
                double sv[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) sv[u] = u0 + u < nq ? gval[w][lane][u0 + u] : 0.0;
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    if (u0 + u < nq) acc = (q0 + u0 + u == 0) ? sv[u] : acc + sv[u];
            }
        } else if (lane == D) {
            for (int u = 0; u < nq; ++u) W += gcnt[w][u];
        }
        __builtin_amdgcn_wave_barrier();  // read before the next rows are written
    }
    W = __shfl(W, D, kWave);
    bool bad = false, chg = false;
    uint64_t term = 0;
    if (lane < D) {
        const double p = acc / double(W);
        pbuf[int64_t(lane) * t.cap + j] = p;
        // stationarity: the cell's merge value C_j * p_j against its sum
        chg = dbits(double(own_cnt) * p) != dbits(own_sum);
        const double q = cell_floor(p, P.h);
        const double rel = q - double(P.lo[lane]);
        bad = !(rel >= 0.0 && rel < double(P.E[lane]));
        term = bad ? 0 : uint64_t(int64_t(q) - P.lo[lane]) * P.stride[lane];
    }
#pragma unroll
    for (int off = 1; off < 8; off <<= 1) term += __shfl_xor((unsigned long long)term, off, kWave);
    const bool moved = __ballot(chg) != 0 || P.base + term != key;  // wave-uniform
    if (lane == 0) {
        kappa[j] = P.base + term;
        if (sequential) seq.moved[j] = (seq.epoch << 8) | uint32_t(seq.step);
        if (Wout) Wout[j] = int32_t(W);
        // instance flags: some cell has a neighbour; the round changes the
        // table (used only if the instance applies it).  One coherent read of
        // both, and an atomic only while a flag is still clear.
        if (nfound > 1 || moved) {
            const uint64_t both = __hip_atomic_load(reinterpret_cast<uint64_t*>(&st[b].any_nb), __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
            if (nfound > 1 && uint32_t(both) == 0) atomicOr(&st[b].any_nb, 1);
            if (moved && uint32_t(both >> 32) == 0) atomicOr(&st[b].changed, 1);
        }
    }
    if (__ballot(bad) && lane == 0) atomicOr(&st[b].err, 3);  // GS_ERR_KEY_RANGE
}

// Stop test of the round (Section 2.1 (v)): decides whether each instance
// applies the shift and merge computed by k_shift.
__device__ inline int decide_state(InstState* __restrict__ sp, int max_iter) {
    InstState s = *sp;
    s.apply = 0;  // (changed was raised by this round's shift; the round end clears it)
    if (s.active) {
        if (!s.any_nb) {
            s.flags |= 1u;  // converged
            s.active = 0;
        } else if (s.t >= max_iter) {
            s.flags |= 4u;  // capped
            s.active = 0;
        } else {
            s.apply = 1;
        }
    }
    s.any_nb = 0;
    s.cs = 0;  // the merge's cell setup records the new table's ranges
    s.ce = 0;
    *sp = s;
    return s.apply;
}

__global__ void k_decide(InstState* __restrict__ st, int B, int max_iter) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) decide_state(st + b, max_iter);
}

// Landing keys for the merge sort, with their radix digit histograms;
// stationarity of applying instances.
template <typename K>
__global__ __launch_bounds__(256) void k_merge_prep(CellTable t, int64_t m, const InstState* __restrict__ stc,
                                                    InstState* __restrict__ st, const double* __restrict__ pbuf,
                                                    const uint64_t* __restrict__ kappa, K* __restrict__ skey, int d,
                                                    int npasses, int digit, uint32_t* __restrict__ hist) {
    __shared__ uint32_t hl[kHistLds];  // pass p, digit v at (p << digit) + v
    const int tid = threadIdx.x;
    const int nh = npasses << digit;
    for (int i = tid; i < nh; i += 256) hl[i] = 0;
    __syncthreads();
    const int64_t j0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool valid = j0 < m;
    const int64_t j = valid ? j0 : m - 1;  // idle lanes shadow the last cell and raise nothing
    const int b = t.inst[j];
    const uint64_t key = t.key[j];
    K out = K(key);
    if (stc[b].apply) out = K(kappa[j]);
    if (valid) skey[j] = out;
    wave_digit_hist(hl, out, valid, npasses, digit);
    __syncthreads();
    uint32_t* hc = hist + (blockIdx.x % kHistCopies) * kHistStride;
    for (int i = tid; i < nh; i += 256)
        if (hl[i]) atomicAdd(&hc[hist_index(i, digit)], hl[i]);
}

// One block copies the 8 counters and the B instance states into host
// memory mapped for the device (host [counters 8][states B]), which the host
// reads after its next wait on the stream instead of copying them back.
// Every thread of the block calls this after a barrier that orders the
// counter and state writes it publishes.
__device__ inline void publish_host(const int64_t* __restrict__ ctr, const InstState* __restrict__ st, int B,
                                    int64_t* __restrict__ host) {
    constexpr int SW = int(sizeof(InstState) / sizeof(int64_t));
    static_assert(sizeof(InstState) % sizeof(int64_t) == 0, "states are copied in 64-bit words");
    const int64_t* sw = reinterpret_cast<const int64_t*>(st);
    for (int i = threadIdx.x; i < 8 + SW * B; i += blockDim.x) host[i] = i < 8 ? ctr[i] : sw[i - 8];
}

// End of a wide round: initial cell -> current cell maps (threads < m0) and
// the per-instance round count and stationarity (threads < B).
// With `gate` (a single block holding every instance) it also writes
// whether some active instance still holds more cells than a tail workgroup.
__global__ void k_round_end(uint32_t* __restrict__ cur, int64_t m0, const uint32_t* __restrict__ g,
                            InstState* __restrict__ st, int B, int32_t* __restrict__ applied,
                            int64_t* __restrict__ gate, const int64_t* __restrict__ ctr,
                            int64_t* __restrict__ host) {
    __shared__ int any;
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gate && threadIdx.x == 0) any = 0;
    if (c < m0) cur[c] = g[cur[c]];
    const int b = int(c);
    bool big = false;
    if (c < B) {
        InstState s = st[b];
        if (applied) applied[b] = s.apply;
        if (s.apply) {
            s.t += 1;
            if (!s.changed) {
                s.flags |= 2u;  // stationary
                s.active = 0;
            }
        }
        s.apply = 0;
        s.changed = 0;
        st[b] = s;
        big = s.active && s.ce - s.cs > kTailCells;
    }
    if (!gate) return;
    __syncthreads();
    if (big) any = 1;
    __syncthreads();
    if (threadIdx.x == 0) *gate = any;
    if (host) {
        __syncthreads();
        publish_host(ctr, st, B, host);
    }
}

// ===========================================================================
// merge of a small table in one workgroup
// ===========================================================================
// For a round whose table holds at most kMergeMax cells (32-bit keys), one
// 1024-thread workgroup does what the device-wide path does with
// k_merge_prep, the radix sort, the heads scan, k_cell_setup and the
// chunk-offset scan: sort keys (landing key of cells of applying instances,
// own key otherwise), a stable LSD radix sort of (key, cell) in LDS, run heads
// -> new cells, their member ranges and chunk offsets, the merge map and its
// composition with the initial cells' map.  The canonical sums of the new
// cells are then computed by k_segsum_chunks / k_segsum_levels over the
// sorted member order it writes to `mperm`, and k_round_end (instances only)
// closes the round.
constexpr int kMergeThreads = 1024;
constexpr int kMergeMax = 8192;
constexpr int kMergeMaxInst = 8192;  // instances whose change flags it keeps in LDS
constexpr int kMergeIPT = kMergeMax / kMergeThreads;  // 8

// Exclusive block-wide scan of one value per thread (kMergeThreads threads);
// returns this thread's exclusive prefix and, through *total, the sum.
__device__ __forceinline__ uint32_t merge_block_scan(uint32_t v, uint32_t* wtot, uint32_t* total) {
    constexpr int NW = kMergeThreads / kWave;
    const int w = threadIdx.x / kWave, lane = lane_id();
    const uint32_t incl = wave_incl_scan_u32(v);
    if (lane == kWave - 1) wtot[w] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) {
        const uint32_t c = wtot[ww];
        before += ww < w ? c : 0u;
        all += c;
    }
    *total = all;
    __syncthreads();  // wtot may be reused after this
    return before + incl - v;
}

template <int D>
__global__ __launch_bounds__(kMergeThreads) void k_merge_small(CellTable t, int64_t m, CellTable u,
                                                               InstState* __restrict__ st, int B,
                                                               const double* __restrict__ pbuf,
                                                               const uint64_t* __restrict__ kappa, int npasses,
                                                               int kbits,
                                                               uint32_t* __restrict__ gmap,
                                                               uint32_t* __restrict__ mperm,
                                                               uint32_t* __restrict__ cur, int64_t m0,
                                                               uint32_t* __restrict__ gtape,
                                                               int64_t* __restrict__ counters, int max_iter,
                                                               uint64_t* __restrict__ dk, uint32_t dk_epoch) {
    constexpr int NW = kMergeThreads / kWave;
    __shared__ uint32_t kbuf[2][kMergeMax];
    __shared__ uint16_t vbuf[2][kMergeMax];
    __shared__ uint32_t wcnt[NW][256];
    __shared__ uint16_t hs[kMergeMax + 1];  // first sorted position of every new cell
    __shared__ uint16_t gm[kMergeMax];      // merge map (old cell -> new cell)
    __shared__ uint32_t wtot[NW];
    __shared__ uint32_t chmask[kMergeMaxInst / 32];  // instances whose round changed the state
    __shared__ uint32_t apmask[kMergeMaxInst / 32];  // instances that apply the round
    const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
    const uint64_t lt = lanemask_lt();
    const int mm = int(m);
    for (int i = tid; i < kMergeMaxInst / 32; i += kMergeThreads) chmask[i] = 0;
    // the cells' instances, keys and landing keys, loaded before the
    // decisions below (they do not depend on them)
    int bi[kMergeIPT];
    uint64_t key[kMergeIPT], kap[kMergeIPT];
#pragma unroll
    for (int i = 0; i < kMergeIPT; ++i) {
        const int j = min(tid + i * kMergeThreads, mm - 1);
        bi[i] = t.inst[j];
        key[i] = t.key[j];
        kap[i] = kappa[j];  // read for every cell, used for applying instances only
    }
    // the initial cells' current cells, composed with the merge map at the end
    constexpr int kCurPT = 4;  // entries per thread and step of the composition
    uint32_t cur0[kCurPT];
#pragma unroll
    for (int i = 0; i < kCurPT; ++i) {
        const int64_t c = tid + int64_t(i) * kMergeThreads;
        cur0[i] = c < m0 ? cur[c] : 0u;
    }
    // the round's decision per instance (converged, capped or applying); the
    // 64 lanes of a wave decide 64 consecutive instances and its first lane
    // writes their two words of the apply mask (every word below B / 32 is
    // written once, so the mask needs no clearing)
    for (int b0 = 0; b0 < B; b0 += kMergeThreads) {
        const int b = b0 + tid;
        const uint64_t ab = __ballot(b < B && decide_state(st + b, max_iter) != 0);
        const int bw = b0 + w * kWave;  // first instance of the wave
        if (lane == 0 && bw < B) {
            apmask[bw >> 5] = uint32_t(ab);
            if (bw + 32 < B) apmask[(bw >> 5) + 1] = uint32_t(ab >> 32);
        }
    }

    // ---- sort keys: landing key for cells of applying instances, own key
    // otherwise (the shift already flagged instances whose cells moved or
    // whose merge values differ from their sums)
    {
        __syncthreads();  // chmask cleared, apmask written
#pragma unroll
        for (int i = 0; i < kMergeIPT; ++i) {
            const int j = tid + i * kMergeThreads;
            if (j >= mm) continue;
            const bool ap = (apmask[bi[i] >> 5] >> (bi[i] & 31)) & 1u;
            kbuf[0][j] = uint32_t(ap ? kap[i] : key[i]);
            vbuf[0][j] = uint16_t(j);
        }
    }

    // ---- stable LSD radix sort of (key, cell) in LDS; wave w ranks the
    // S slots of 64 positions from w * S * 64 (S: the slots spread evenly
    // over the waves), so (wave, slot, lane) order is position order
    const int S = ((mm + kWave - 1) / kWave + NW - 1) / NW;  // <= kMergeIPT
    int src = 0;
    for (int p = 0; p < npasses; ++p) {
        const int shift = 8 * p;
        const int nbits = kbits - shift < 8 ? kbits - shift : 8;  // the last digit may be narrower
        for (int i = tid; i < NW * 256; i += kMergeThreads) (&wcnt[0][0])[i] = 0;
        __syncthreads();
        uint32_t kk[kMergeIPT];
        uint16_t vv[kMergeIPT];
        uint32_t rk[kMergeIPT];
#pragma unroll
        for (int i = 0; i < kMergeIPT; ++i) {
            const int pos = (w * S + i) * kWave + lane;
            if (i >= S || (w * S + i) * kWave >= mm) {  // no slot, or the whole slot is past the end
                kk[i] = 0u;
                vv[i] = 0;
                rk[i] = 0u;
                continue;
            }
            const bool valid = pos < mm;
            kk[i] = valid ? kbuf[src][pos] : 0u;
            vv[i] = valid ? vbuf[src][pos] : uint16_t(0);
            const uint32_t dgt = (kk[i] >> shift) & 255u;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int bb = 0; bb < 8; ++bb) {
                if (bb >= nbits) break;
                const bool bit = (dgt >> bb) & 1u;
                const uint64_t bal = __ballot(bit);
                peers &= bit ? bal : ~bal;
            }
            uint32_t prior = 0;
            if (valid) prior = wcnt[w][dgt];
            rk[i] = prior + uint32_t(__popcll(peers & lt));
            if (valid && lane == 63 - __clzll(peers)) wcnt[w][dgt] = prior + uint32_t(__popcll(peers));
        }
        __syncthreads();
        // digit d (thread d): exclusive over the waves, then over the digits
        uint32_t run = 0;
        if (tid < 256) {
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) {
                const uint32_t c = wcnt[ww][tid];
                wcnt[ww][tid] = run;
                run += c;
            }
        }
        uint32_t total = 0;
        const uint32_t base = merge_block_scan(tid < 256 ? run : 0u, wtot, &total);
        if (tid < 256) {
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) wcnt[ww][tid] += base;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kMergeIPT; ++i) {
            const int pos = (w * S + i) * kWave + lane;
            if (i < S && pos < mm) {
                const uint32_t dgt = (kk[i] >> shift) & 255u;
                const uint32_t dst = wcnt[w][dgt] + rk[i];
                kbuf[src ^ 1][dst] = kk[i];
                vbuf[src ^ 1][dst] = vv[i];
            }
        }
        __syncthreads();
        src ^= 1;
    }
    const uint32_t* sk = kbuf[src];
    const uint16_t* sv = vbuf[src];

    // ---- run heads -> new cells (the ranking's slots: consecutive lanes
    // read and write consecutive positions)
    uint64_t hb[kMergeIPT];
    int nh = 0;  // heads of the wave
#pragma unroll
    for (int i = 0; i < kMergeIPT; ++i) {
        const int p = (w * S + i) * kWave + lane;
        hb[i] = __ballot(i < S && p < mm && (p == 0 || sk[p] != sk[p - 1]));
        nh += __popcll(hb[i]);
    }
    if (lane == 0) wtot[w] = uint32_t(nh);
    __syncthreads();
    int cid_base = 0, mnew = 0;  // heads before this wave, all heads
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) {
        const int c = int(wtot[ww]);
        cid_base += ww < w ? c : 0;
        mnew += c;
    }
    const uint64_t le = lt | (1ull << lane);
#pragma unroll
    for (int i = 0; i < kMergeIPT; ++i) {
        const int p = (w * S + i) * kWave + lane;
        if (i < S && p < mm) {
            const int cid = cid_base + __popcll(hb[i] & le) - 1;  // the last head at or before p
            if ((hb[i] >> lane) & 1u) {
                hs[cid] = uint16_t(p);
                u.key[cid] = uint64_t(sk[p]);
                if (dk) dk[sk[p]] = (uint64_t(dk_epoch) << 32) | uint64_t(cid);
            }
            const int j = sv[p];
            mperm[p] = uint32_t(j);
            gm[j] = uint16_t(cid);
        }
        cid_base += __popcll(hb[i]);
    }
    if (tid == 0) hs[mnew] = uint16_t(mm);
    __syncthreads();  // hs and gm complete; wtot free again
    // the merge map in old-cell order
    for (int j = tid; j < mm; j += kMergeThreads) {
        const uint32_t g = gm[j];
        gmap[j] = g;
        if (gtape) gtape[j] = g;
    }

    // ---- new cells: members, chunks, instance ranges, merged groups (one
    // cell per thread, kMergeThreads cells at a time; chunk offsets by a
    // block scan per group of cells)
    uint32_t tasks = 0;  // chunks of the cells before the current group
    for (int c0 = 0; c0 < mnew; c0 += kMergeThreads) {
        const int c = c0 + tid;
        int p0 = 0, b = -1, bp = -1;
        uint32_t len = 0, nch = 0;
        if (c < mnew) {
            p0 = hs[c];
            len = uint32_t(hs[c + 1]) - uint32_t(p0);
            nch = (len + kChunk - 1) / kChunk;
            b = t.inst[sv[p0]];
            bp = c > 0 ? t.inst[sv[hs[c - 1]]] : -1;
        }
        uint32_t group = 0;
        const uint32_t choff = tasks + merge_block_scan(nch, wtot, &group);
        tasks += group;
        if (c < mnew) {
            u.start[c] = uint32_t(p0);
            u.len[c] = len;
            u.first[c] = uint32_t(sv[p0]);
            u.nch[c] = nch;
            u.choff[c] = choff;
            u.inst[c] = b;
            if (bp != b) {
                st[b].cs = c;
                if (bp >= 0) st[bp].ce = c;
            }
            if (c == mnew - 1) st[b].ce = mnew;
            const bool ap = (apmask[b >> 5] >> (b & 31)) & 1u;
            if (len > 1 && ap) atomicOr(&chmask[b >> 5], 1u << (b & 31));
        }
    }
    __syncthreads();
    for (int b = tid; b < B; b += kMergeThreads)
        if ((chmask[b >> 5] >> (b & 31)) & 1u) st[b].changed = 1;

    // ---- initial cell -> current cell (the per-instance round end follows
    // the sums, which still read which instances apply the round)
    for (int64_t c0 = tid; c0 < m0; c0 += kCurPT * kMergeThreads) {
        uint32_t v[kCurPT];
#pragma unroll
        for (int i = 0; i < kCurPT; ++i) {
            const int64_t c = c0 + int64_t(i) * kMergeThreads;
            v[i] = c0 == tid ? cur0[i] : (c < m0 ? cur[c] : 0u);  // the first step's entries were loaded at the start
        }
#pragma unroll
        for (int i = 0; i < kCurPT; ++i) {
            const int64_t c = c0 + int64_t(i) * kMergeThreads;
            if (c < m0) cur[c] = gm[v[i]];
        }
    }
    if (tid == 0) {
        counters[0] = mnew;   // new cells
        counters[1] = tasks;  // chunk tasks of their sums
    }
}

// ===========================================================================
// tail: one workgroup per instance, whole cell table in LDS
// ===========================================================================
// Candidate neighbours of a tail cell.  The table is sorted by key (dimension
// 0 most significant), so the cells whose first one or two coordinates are
// within +-1 of a cell's own form at most three ascending index ranges.  A
// column table in LDS gives them directly: col[v] = first cell whose column
// (c0, or c0 * E1 + c1) is >= v, for v in [0, ncol].  Without one (too many
// columns) a binary search gives the range of dimension-0 coordinates.
// Coordinates of tail cells relative to the box origin: 32-bit while every
// extent of the instances' key boxes is below 2^31, else 64-bit (the neighbour
// test |a - b| <= 1 is (a - b + 1) <= 2 in the unsigned type of the same width).
template <typename CT> struct CoordUnsigned;
template <> struct CoordUnsigned<int32_t> { using type = uint32_t; };
template <> struct CoordUnsigned<int64_t> { using type = uint64_t; };

struct TailCols {
    int mode;  // 2: columns of (c0, c1); 1: of c0; 0: no table
    int E0, E1, ncol;
    int first_test;  // first dimension the candidates still have to be tested in
};

template <int D>
__device__ inline TailCols tail_cols(int64_t E0, int64_t E1) {
    TailCols c;
    c.E0 = int(E0);
    c.E1 = D >= 2 ? int(E1) : 1;
    if (D >= 2 && E0 * E1 <= kSlabMax) {
        c.mode = 2;
        c.ncol = int(E0 * E1);
        c.first_test = 2;
    } else if (E0 <= kSlabMax) {
        c.mode = 1;
        c.ncol = int(E0);
        c.first_test = 1;
    } else {
        c.mode = 0;
        c.ncol = 0;
        c.first_test = 1;
    }
    return c;
}

template <typename CT>
__device__ inline int tail_col(const TailCols& c, const CT* crd0, const CT* crd1, int i) {
    return c.mode == 2 ? int(crd0[i]) * c.E1 + int(crd1[i]) : int(crd0[i]);
}

// Every thread of the workgroup calls this; a barrier must follow.  Entry v
// is a binary search over the m cells' columns (ascending with the cells).
template <typename CT>
__device__ inline void tail_cols_build(const TailCols& c, const CT* crd0, const CT* crd1, int m, int tid,
                                       uint16_t* col) {
    if (c.mode == 0) return;
    for (int v = tid; v <= c.ncol; v += kTailThreads) {
        int lo = 0, hi = m;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (tail_col(c, crd0, crd1, mid) < v) lo = mid + 1; else hi = mid;
        }
        col[v] = uint16_t(lo);
    }
}

struct TailWindow {
    int a[3], n[3];  // ranges [a[u], a[u] + n[u]), ascending and disjoint
};

template <typename CT>
__device__ inline TailWindow tail_window(const TailCols& c, const CT* crd0, const CT* crd1, int m, int i,
                                         const uint16_t* col) {
    TailWindow w;
    const CT c0 = crd0[i];
    if (c.mode == 2) {
        const int c1 = int(crd1[i]);
        const int lo1 = c1 - 1 < 0 ? 0 : c1 - 1;
        const int hi1 = c1 + 2 > c.E1 ? c.E1 : c1 + 2;
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int a0 = int(c0) - 1 + u;
            if (a0 < 0 || a0 >= c.E0) {
                w.a[u] = 0;
                w.n[u] = 0;
            } else {
                w.a[u] = col[a0 * c.E1 + lo1];
                w.n[u] = int(col[a0 * c.E1 + hi1]) - w.a[u];
            }
        }
        return w;
    }
    int a, z;  // cells with dimension-0 coordinate in [c0 - 1, c0 + 1]
    if (c.mode == 1) {
        const int c0i = int(c0);
        a = col[c0i - 1 < 0 ? 0 : c0i - 1];
        z = col[c0i + 2 > c.E0 ? c.E0 : c0i + 2];
    } else {
        a = 0;
        z = m;
        while (a < z) {
            const int mid = (a + z) >> 1;
            if (crd0[mid] < c0 - 1) a = mid + 1; else z = mid;
        }
        z = a;
        while (z < m && crd0[z] <= c0 + 1) ++z;
    }
    w.a[0] = a;
    w.n[0] = z - a;
    w.a[1] = w.a[2] = 0;
    w.n[1] = w.n[2] = 0;
    return w;
}

// Index of the e-th candidate of a window (e < n[0] + n[1] + n[2]).
__device__ inline int tail_cand(const TailWindow& w, int e) {
    const int n01 = w.n[0] + w.n[1];
    return e < w.n[0] ? w.a[0] + e : (e < n01 ? w.a[1] + e - w.n[0] : w.a[2] + e - n01);
}

// With ck.every > 0 the forward also saves the table at the start of every
// ck.every-th tail round.  With replay_r0 >= 0 the kernel instead recomputes
// tail rounds [replay_r0, replay_r0 + ck.every) of a finished fit from the
// checkpoint at replay_r0, writing only their tape (rounds numbered from
// replay_r0); the fit's outputs and state are left untouched.
// Whether some active instance still holds more cells than a tail workgroup
// (the tail launched right after a device-wide round checks it first).
__global__ void k_tail_gate(const InstState* __restrict__ st, int B, int64_t* __restrict__ gate,
                            const int64_t* __restrict__ ctr, int64_t* __restrict__ host) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int b = threadIdx.x; b < B; b += blockDim.x)
        if (st[b].active && st[b].ce - st[b].cs > kTailCells) any = 1;
    __syncthreads();
    if (threadIdx.x == 0) *gate = any;
    if (host) {
        __syncthreads();
        publish_host(ctr, st, B, host);
    }
}

// With `gate` set and nonzero the kernel returns at once, changing nothing.
// SEQ runs the sequential form of Eq. 5 in the colour-by-colour order (bit
// D-1-k of a cell's colour = parity of its integer coordinate k; cells of one
// colour are never neighbours): a moved cell writes fl(C_j * p_j) over its sum
// for the cells moving after it, and a round that stops puts the sums back.
// SEQ fits record no tape or checkpoints.
template <int D, bool SEQ, typename CT>
__global__ __launch_bounds__(kTailThreads) void k_tail(CellTable t, const InstParam* __restrict__ param,
                                                       InstState* __restrict__ st, uint32_t* __restrict__ tmap,
                                                       int max_iter, TailTape tape, TailCkpt ck, int replay_r0,
                                                       const int64_t* __restrict__ gate) {
    constexpr int MT = kTailCells;
    constexpr int NW = kTailThreads / kWave;
    using UCT = typename CoordUnsigned<CT>::type;
    __shared__ uint64_t lkey[MT];     // local packed key (key - base), ascending
    __shared__ CT crd[D][MT];         // unpacked coordinates relative to lo
    __shared__ int32_t cnt[MT];       // counts
    __shared__ double sm[D][MT];      // sums; reused as the sorted merge values
    __shared__ uint64_t kap[MT];      // landing keys
    __shared__ uint64_t skey[MT];     // landing keys sorted
    __shared__ int32_t scnt[MT];      // counts sorted
    __shared__ uint16_t gmap[MT];     // old cell -> new cell
    __shared__ uint16_t lmap[MT];     // entry cell -> current cell
    __shared__ uint16_t gid_of[MT];   // sorted position -> group
    __shared__ uint16_t hstart[MT + 1];
    __shared__ int32_t wsum[NW];
    __shared__ int32_t s_maxsz;
    __shared__ uint16_t col[kSlabMax + 1];  // column table of the current cells
    __shared__ uint16_t rank_of[MT];        // old cell -> sorted position
    __shared__ int32_t s_flag[2][3];         // per round parity: any neighbour, bad key, changed
    __shared__ uint8_t cstate[MT];  // sequential form: colour of each cell, bit 7 once it has moved
    __shared__ int32_t s_pend[2];   // sequential form, per step parity: some cell still waits

    if (gate && *gate) return;
    const int b = blockIdx.x;
    const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
    InstState* S = st + b;
    const bool replay = replay_r0 >= 0;
    const int64_t cs = S->cs, ce = S->ce;
    int m_entry = int(ce - cs);
    int seg_rounds = 0;  // replay: rounds of the segment this instance ran
    if (replay) {
        seg_rounds = min(ck.every, S->t - S->t_tail0 - replay_r0);
        if (seg_rounds <= 0) return;
        m_entry = ck.m[int64_t(b) * ck.nslots + replay_r0 / ck.every];
    } else if (!S->active) {
        for (int e = tid; e < m_entry; e += kTailThreads) tmap[cs + e] = uint32_t(e);
        if (tid == 0) {
            S->K = m_entry;
            S->t_tail0 = S->t;  // no tail round: the adjoint skips this instance's tail
        }
        return;
    }
    const InstParam& P = param[b];
    const double h = P.h;
    // packing of the instance's keys, read from LDS where used (kept out of
    // registers, which the rounds need)
    __shared__ int64_t s_lo[D];
    __shared__ uint64_t s_stride[D];
    __shared__ double s_lod[D], s_Ed[D];
    __shared__ int64_t s_E01[2];
    if (tid < D) {
        s_lo[tid] = P.lo[tid];
        s_stride[tid] = P.stride[tid];
        s_lod[tid] = double(P.lo[tid]);
        s_Ed[tid] = double(P.E[tid]);
        if (tid < 2) s_E01[tid] = P.E[tid < D ? tid : 0];
    }

    if (tid < m_entry) {
        uint64_t lk;
        if (replay) {
            const int64_t e = int64_t(b) * ck.stride + int64_t(replay_r0 / ck.every) * kTailCells + tid;
            lk = ck.key[e];
            cnt[tid] = ck.cnt[e];
#pragma unroll
            for (int k = 0; k < D; ++k) sm[k][tid] = ck.sum[k * ck.total + e];
        } else {
            const int64_t c = cs + tid;
            lk = t.key[c] - P.base;
            cnt[tid] = int32_t(t.cnt[c]);
#pragma unroll
            for (int k = 0; k < D; ++k) sm[k][tid] = t.sum[k * t.cap + c];
        }
        lkey[tid] = lk;
#pragma unroll
        for (int k = 0; k < D; ++k) crd[k][tid] = CT((lk / P.stride[k]) % uint64_t(P.E[k]));
        lmap[tid] = uint16_t(tid);
    }
    __syncthreads();

    int m = m_entry;
    int64_t msum = 0;  // table sizes of the rounds run here (thread 0)
    int tt = replay ? S->t_tail0 + replay_r0 : S->t;
    const int t_entry = tt;
    if (tid == 0 && !replay) S->t_tail0 = t_entry;
    uint32_t flags = S->flags;
    int err = 0;
    const uint64_t lt = lanemask_lt();
    const TailCols cols = tail_cols<D>(s_E01[0], D >= 2 ? s_E01[1] : 1);
    const bool fast_rank = P.span <= (1ull << 53);  // (key << 10 | index) fits in 63 bits
    if (tid < 6) (&s_flag[0][0])[tid] = 0;
    int lo_par = 0;  // parities of the box origin, as colour bits
    if constexpr (SEQ) {
#pragma unroll
        for (int k = 0; k < D; ++k) lo_par = (lo_par << 1) | int(P.lo[k] & 1);
    }
    for (int round = 0;; ++round) {
        if (replay && round == seg_rounds) break;
        int32_t* flg = s_flag[round & 1];
        if (!replay && ck.every > 0 && round % ck.every == 0 && tid < m) {  // checkpoint of the table
            const int slot = round / ck.every;
            const int64_t e = int64_t(b) * ck.stride + int64_t(slot) * kTailCells + tid;
            ck.key[e] = lkey[tid];
            ck.cnt[e] = cnt[tid];
#pragma unroll
            for (int k = 0; k < D; ++k) ck.sum[k * ck.total + e] = sm[k][tid];
            if (tid == 0) ck.m[int64_t(b) * ck.nslots + slot] = m;
        }
        // ---- column table of the current cells
        tail_cols_build(cols, crd[0], crd[D >= 2 ? 1 : 0], m, tid, col);
        int my_col = 0;
        if constexpr (SEQ) {
            if (tid < m) {
                int rp = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) rp = (rp << 1) | int(crd[k][tid] & 1);
                my_col = rp ^ lo_par;
                cstate[tid] = uint8_t(my_col);  // colour; bit 7 set once the cell has moved
            }
            if (tid < 2) s_pend[tid] = 0;
        }
        __syncthreads();
        // every thread has finished reading the other parity's flags
        if (tid < 3) s_flag[(round + 1) & 1][tid] = 0;
        // ---- shift (one cell per thread)
        // Sequential form: instead of one step per colour, a cell moves in the
        // first step in which all its neighbours of lower colours have moved
        // (its neighbours of higher colours wait for it in turn), so it reads
        // exactly the sums the colour-by-colour sweep gives it: C_k * p_k of
        // the lower colours, the round's sums of the higher ones.  Moves are
        // committed after a barrier; the steps number the longest chain of
        // ascending colours among neighbours, at most 2^D.
        bool nb = false, bad = false;
        bool chg = false;  // stationarity: landing key or merge value differs from the cell's own
        double p[D];
        double val[D];
        double orig[SEQ ? D : 1];  // the cell's sums before the sweep overwrote them
        CT q[D];
        uint64_t kj = 0;
        int32_t Wj = 0;
        bool pending = tid < m;
        for (int lvl = 0; lvl < (SEQ ? (1 << D) : 1); ++lvl) {
        bool ready = true;
        if (pending) {
            const TailWindow win = tail_window(cols, crd[0], crd[D >= 2 ? 1 : 0], m, tid, col);
            const int ncand = win.n[0] + win.n[1] + win.n[2];
            CT me[D];
#pragma unroll
            for (int dd = 1; dd < D; ++dd) me[dd] = crd[dd][tid];
            // Left fold over the neighbours among the candidates, in
            // ascending index, starting from -0.0 (the exact additive
            // identity); non-neighbours' rows are not read (fewer LDS bank
            // conflicts in the large rounds).
            int64_t W = 0;
#pragma unroll
            for (int dd = 0; dd < D; ++dd) p[dd] = -0.0;
            int nbs = 0;
            constexpr int U = (D >= 5 || (SEQ && D >= 4)) ? 2 : 4;  // candidates per step (register budget of 1024 threads)
            for (int k0 = 0; k0 < ncand; k0 += U) {
                int okm[U];
                int kk[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    okm[u] = (k0 + u < ncand) ? 1 : 0;
                    kk[u] = okm[u] ? tail_cand(win, k0 + u) : tid;
                }
#pragma unroll
                for (int dd = 1; dd < D; ++dd) {
                    if (dd < cols.first_test) continue;
#pragma unroll
                    for (int u = 0; u < U; ++u) okm[u] &= (UCT(crd[dd][kk[u]] - me[dd] + 1) <= UCT(2)) ? 1 : 0;
                }
                if constexpr (SEQ) {
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int k = kk[u];
                        const bool ok = okm[u] != 0;
                        // a neighbour of a lower colour that has not moved yet
                        const int cs8 = cstate[k];
                        if (ok && (cs8 & 63) < my_col && !(cs8 & 128)) ready = false;
                        if (ok) {  // only neighbours' rows are read (a non-neighbour would add -0.0)
                            W += int64_t(cnt[k]);
                            nbs += 1;
#pragma unroll
                            for (int dd = 0; dd < D; ++dd) p[dd] = p[dd] + sm[dd][k];
                        }
                    }
                } else {
                    // every candidate's count and sums loaded at once (rows of
                    // candidates outside the table are the cell's own), then
                    // added where the candidate is a neighbour: a non-neighbour
                    // adds -0.0, the exact additive identity, so the fold's
                    // bits are those of the neighbours alone
                    int32_t cv[U];
                    double sv[U][D];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        cv[u] = cnt[kk[u]];
#pragma unroll
                        for (int dd = 0; dd < D; ++dd) sv[u][dd] = sm[dd][kk[u]];
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const bool ok = okm[u] != 0;
                        W += ok ? int64_t(cv[u]) : int64_t(0);
                        nbs += ok ? 1 : 0;
#pragma unroll
                        for (int dd = 0; dd < D; ++dd) p[dd] = p[dd] + (ok ? sv[u][dd] : -0.0);
                    }
                }
            }
            if (ready) {
            nb = nbs > 1;  // the cell itself is always among the candidates
            Wj = int32_t(W);
#pragma unroll
            for (int dd = 0; dd < D; ++dd) {
                p[dd] = p[dd] / double(W);
                const double qq = cell_floor(p[dd], h);
                const double rel = qq - s_lod[dd];
                if (!(rel >= 0.0 && rel < s_Ed[dd])) bad = true;
                q[dd] = CT(int64_t(qq) - s_lo[dd]);
                kj += uint64_t(int64_t(qq) - s_lo[dd]) * s_stride[dd];
            }
            // merge values and stationarity (own cell only: nothing writes it
            // before the scatter below)
            chg = kj != lkey[tid];
#pragma unroll
            for (int dd = 0; dd < D; ++dd) {
                val[dd] = double(cnt[tid]) * p[dd];
                chg = chg || dbits(val[dd]) != dbits(sm[dd][tid]);
            }
            }
        }
        if constexpr (SEQ) {
            if (__ballot(pending && !ready) && lane == 0) atomicOr(&s_pend[lvl & 1], 1);
            __syncthreads();
            if (pending && ready) {  // commit: the cells moving later read C_j * p_j
#pragma unroll
                for (int dd = 0; dd < D; ++dd) {
                    orig[dd] = sm[dd][tid];
                    sm[dd][tid] = val[dd];
                }
                cstate[tid] = uint8_t(my_col | 128);
                pending = false;
            }
            const int more = s_pend[lvl & 1];
            if (tid == 0) s_pend[(lvl + 1) & 1] = 0;
            __syncthreads();
            if (!more) break;
        }
        }
        if (__ballot(nb) && lane == 0) atomicOr(&flg[0], 1);
        if (__ballot(bad) && lane == 0) atomicOr(&flg[1], 1);
        __syncthreads();
        if (SEQ && (!flg[0] || tt >= max_iter) && tid < m) {  // the round is not applied
#pragma unroll
            for (int dd = 0; dd < D; ++dd) sm[dd][tid] = orig[dd];
        }
        if (!flg[0]) {
            flags |= 1u;
            break;
        }
        if (tt >= max_iter) {
            flags |= 4u;
            break;
        }
        if (flg[1]) {
            err = 3;
            break;
        }
        msum += m;
        // ---- landing keys (read by the linear rank only)
        if (!fast_rank) {
            if (tid < m) kap[tid] = kj;
            __syncthreads();
        }
        // ---- stable rank by (landing key, old index)
        int rank = 0;
        if (fast_rank) {
            // (key, index) packed in one word; each wave sorts its 64 words in
            // registers (bitonic network over lanes), then the rank of a word
            // is its place in its own run plus its lower bound in every other
            // run (binary search in LDS)
            const int nruns = (m + kWave - 1) / kWave;
            uint64_t v = tid < m ? ((kj << 10) | uint64_t(tid)) : ~0ull;
            if (w < nruns) v = wave_sort_u64(v);
            if (nruns > 1) {  // other waves' runs are read below
                skey[tid] = v;
                __syncthreads();
            }
            if (w < nruns) {
                int r = lane;
                for (int rr = 0; rr < nruns; ++rr) {
                    if (rr == w) continue;
                    const uint64_t* run = skey + rr * kWave;
                    int pos = 0;
#pragma unroll
                    for (int step = 32; step >= 1; step >>= 1)
                        if (run[pos + step - 1] < v) pos += step;
                    if (pos == kWave - 1 && run[kWave - 1] < v) pos = kWave;
                    r += pos;
                }
                if (v != ~0ull) rank_of[v & 1023u] = uint16_t(r);
            }
            __syncthreads();
            if (tid < m) rank = rank_of[tid];
        } else if (tid < m) {
            int k = 0;
            for (; k + 8 <= m; k += 8) {
                uint64_t u[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) u[e] = kap[k + e];
#pragma unroll
                for (int e = 0; e < 8; ++e) rank += (u[e] < kj) || (u[e] == kj && k + e < tid);
            }
            for (; k < m; ++k) {
                const uint64_t u = kap[k];
                rank += (u < kj) || (u == kj && k < tid);
            }
        }
        if (tid < m) {
            skey[rank] = kj;
            scnt[rank] = cnt[tid];
#pragma unroll
            for (int dd = 0; dd < D; ++dd) {
                sm[dd][rank] = val[dd];
                crd[dd][rank] = q[dd];
            }
        }
        __syncthreads();
        // ---- groups of equal landing keys
        const bool head = tid < m && (tid == 0 || skey[tid] != skey[tid - 1]);
        const uint64_t hb = __ballot(head);
        if (lane == 0) wsum[w] = __popcll(hb);
        if (tid == 0) s_maxsz = 1;
        __syncthreads();
        int gex = 0, mnew = 0;
        for (int ww = 0; ww < NW; ++ww) {
            const int c = wsum[ww];
            gex += ww < w ? c : 0;
            mnew += c;
        }
        const int gid = gex + __popcll(hb & lt) + (head ? 1 : 0) - 1;
        if (tid < m) gid_of[tid] = uint16_t(gid);
        if (head) hstart[gid] = uint16_t(tid);
        if (tid == 0) hstart[mnew] = uint16_t(m);
        __syncthreads();
        if (head) {
            const int sz = int(hstart[gid + 1]) - tid;
            if (sz > 1) atomicMax(&s_maxsz, sz);
        }
        __syncthreads();
        const int maxsz = s_maxsz;
        {
            int rel = 0, sz = 0;  // place in the group, group size
            if (tid < m) {
                const int g0 = hstart[gid];
                rel = tid - g0;
                sz = int(hstart[gid + 1]) - g0;
            }
            for (int s = 1; s < maxsz; s <<= 1) {
                if (tid < m && (rel & (2 * s - 1)) == 0 && rel + s < sz) {
                    // both operands of every coordinate read before any write
                    // (the LDS reads then overlap)
                    double a[D], o[D];
#pragma unroll
                    for (int dd = 0; dd < D; ++dd) {
                        a[dd] = sm[dd][tid];
                        o[dd] = sm[dd][tid + s];
                    }
                    const int32_t ca = scnt[tid], co = scnt[tid + s];
#pragma unroll
                    for (int dd = 0; dd < D; ++dd) sm[dd][tid] = a[dd] + o[dd];
                    scnt[tid] = ca + co;
                }
                __syncthreads();
            }
        }
        // ---- new table
        uint64_t nk = 0;
        int32_t nc = 0;
        double ns[D];
        CT nq[D];
        if (head) {
            nk = skey[tid];
            nc = scnt[tid];
#pragma unroll
            for (int dd = 0; dd < D; ++dd) {
                ns[dd] = sm[dd][tid];
                nq[dd] = crd[dd][tid];
            }
        }
        if (tid < m) {
            gmap[tid] = gid_of[rank];
            if (tape.key) {  // the round's starting table, weights and merge map
                const int64_t e = int64_t(b) * tape.stride + int64_t(tt - t_entry) * kTailCells + tid;
                tape.key[e] = lkey[tid];
                tape.cnt[e] = cnt[tid];
                tape.W[e] = Wj;
                tape.g[e] = gid_of[rank];
                if (tid == 0) tape.m[int64_t(b) * tape.max_rounds + (tt - t_entry)] = m;
            }
        }
        __syncthreads();
        if (head) {
            lkey[gid] = nk;
            cnt[gid] = nc;
#pragma unroll
            for (int dd = 0; dd < D; ++dd) {
                sm[dd][gid] = ns[dd];
                crd[dd][gid] = nq[dd];
            }
        }
        __syncthreads();
        if (tid < m_entry) lmap[tid] = gmap[lmap[tid]];
        if (__ballot(chg) && lane == 0) atomicOr(&flg[2], 1);
        __syncthreads();
        const int changed = flg[2] || (mnew != m);
        m = mnew;
        ++tt;
        if (!changed) {
            flags |= 2u;
            break;
        }
    }
    __syncthreads();
    if (replay) return;
    if (err) {
        if (tid == 0) S->err = err;
        return;
    }
    if (tid < m) {
        const int64_t c = cs + tid;
        t.key[c] = lkey[tid] + P.base;
        t.cnt[c] = cnt[tid];
#pragma unroll
        for (int k = 0; k < D; ++k) t.sum[k * t.cap + c] = sm[k][tid];
    }
    if (tid < m_entry) tmap[cs + tid] = lmap[tid];
    if (tid == 0) {
        S->t = tt;
        S->flags = flags;
        S->K = m;
        S->active = 0;
        S->tail_cells = msum;
    }
}

// ===========================================================================
// adjoint along the recorded trajectory
// ===========================================================================
// Sbar of the final cells: the mode cotangent over the count.
__global__ void k_adj_final(CellTable t, const InstState* __restrict__ st, const int64_t* __restrict__ koff, int B,
                            int64_t rows, int d, const double* __restrict__ gmodes, double* __restrict__ sbar) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const int b = inst_of_row(koff, B, r);
    const int64_t c = st[b].cs + (r - koff[b]);
    const double C = double(t.cnt[c]);
    for (int k = 0; k < d; ++k) sbar[k * t.cap + c] = gmodes[r * d + k] / C;
}

// Reverse of the tail rounds of one instance per workgroup: Sbar of the final
// cells -> Sbar of the cells the tail started from.  For round t (reversed):
// q_j = (C_j * Sbar_{g(j)}) / W_j, then Sbar_k = left fold in ascending key
// of q_j over the round's cells j with Chebyshev key distance <= 1.
// With ck.every > 0 the tape holds only the segment of tail rounds
// [seg_r0, seg_r0 + ck.every) (recomputed from its checkpoint) and the kernel
// reverses just those rounds; sbar then holds, per instance, the Sbar of the
// cells at the segment's end on entry and at its start on exit.
template <int D, typename CT>
__global__ __launch_bounds__(kTailThreads) void k_tail_adj(const InstParam* __restrict__ param,
                                                           const InstState* __restrict__ st, TailTape tape,
                                                           double* __restrict__ sbar, int64_t cap, TailCkpt ck,
                                                           int seg_r0) {
    constexpr int MT = kTailCells;
    using UCT = typename CoordUnsigned<CT>::type;
    __shared__ CT crd[D][MT];
    __shared__ double A[D][MT];
    __shared__ double Q[D][MT];
    __shared__ uint16_t col[kSlabMax + 1];
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    const InstState S = st[b];
    const int all_rounds = S.t - S.t_tail0;
    int rounds = all_rounds;
    int mnext = int(S.K);
    if (ck.every > 0) {
        rounds = min(ck.every, all_rounds - seg_r0);
        if (rounds > 0 && seg_r0 + rounds < all_rounds)  // cells at the start of the next segment
            mnext = ck.m[int64_t(b) * ck.nslots + seg_r0 / ck.every + 1];
    }
    if (rounds <= 0) return;  // no tail round here: Sbar is already that of the segment's start
    const InstParam& P = param[b];
    int64_t E[D];
    uint64_t stride[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        E[k] = P.E[k];
        stride[k] = P.stride[k];
    }
    const TailCols cols = tail_cols<D>(E[0], E[D >= 2 ? 1 : 0]);
    if (tid < mnext)
#pragma unroll
        for (int k = 0; k < D; ++k) A[k][tid] = sbar[k * cap + S.cs + tid];
    int m = 0;
    for (int tl = rounds - 1; tl >= 0; --tl) {
        m = tape.m[int64_t(b) * tape.max_rounds + tl];
        const int64_t e0 = int64_t(b) * tape.stride + int64_t(tl) * kTailCells;
        __syncthreads();  // A of the later round is complete; the previous round's reads are done
        if (tid < m) {
            const uint64_t lk = tape.key[e0 + tid];
#pragma unroll
            for (int k = 0; k < D; ++k) crd[k][tid] = CT((lk / stride[k]) % uint64_t(E[k]));
            const int32_t C = tape.cnt[e0 + tid];
            const int32_t W = tape.W[e0 + tid];
            const uint32_t g = tape.g[e0 + tid];
#pragma unroll
            for (int k = 0; k < D; ++k) Q[k][tid] = (double(C) * A[k][g]) / double(W);
        }
        __syncthreads();
        tail_cols_build(cols, crd[0], crd[D >= 2 ? 1 : 0], m, tid, col);
        __syncthreads();
        if (tid < m) {
            const TailWindow win = tail_window(cols, crd[0], crd[D >= 2 ? 1 : 0], m, tid, col);
            const int ncand = win.n[0] + win.n[1] + win.n[2];
            CT me[D];
#pragma unroll
            for (int dd = 1; dd < D; ++dd) me[dd] = crd[dd][tid];
            double acc[D];
#pragma unroll
            for (int dd = 0; dd < D; ++dd) acc[dd] = -0.0;
            for (int k0 = 0; k0 < ncand; k0 += 4) {
                int okm[4], kk[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    okm[u] = (k0 + u < ncand) ? 1 : 0;
                    kk[u] = okm[u] ? tail_cand(win, k0 + u) : tid;
                }
#pragma unroll
                for (int dd = 1; dd < D; ++dd) {
                    if (dd < cols.first_test) continue;
#pragma unroll
                    for (int u = 0; u < 4; ++u) okm[u] &= (UCT(crd[dd][kk[u]] - me[dd] + 1) <= UCT(2)) ? 1 : 0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool ok = okm[u] != 0;
#pragma unroll
                    for (int dd = 0; dd < D; ++dd) acc[dd] = acc[dd] + (ok ? Q[dd][kk[u]] : -0.0);
                }
            }
#pragma unroll
            for (int dd = 0; dd < D; ++dd) A[dd][tid] = acc[dd];
        }
        mnext = m;
    }
    __syncthreads();
    if (tid < m)
#pragma unroll
        for (int k = 0; k < D; ++k) sbar[k * cap + S.cs + tid] = A[k][tid];
}

// Wide round r, reversed: q_j from the later round's Sbar (identity for
// instances that did not apply the round).
__global__ void k_adj_q(const int32_t* __restrict__ inst, const int64_t* __restrict__ cnt,
                        const int32_t* __restrict__ W, const uint32_t* __restrict__ g,
                        const int32_t* __restrict__ applied, int64_t m, int d, const double* __restrict__ sbar,
                        double* __restrict__ q, int64_t cap) {
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const uint32_t gj = g[j];
    if (applied[inst[j]]) {
        const double C = double(cnt[j]), Wd = double(W[j]);
        for (int k = 0; k < d; ++k) q[k * cap + j] = (C * sbar[k * cap + gj]) / Wd;
    } else {
        for (int k = 0; k < d; ++k) q[k * cap + j] = sbar[k * cap + gj];
    }
}

// Wide round r, reversed: Sbar_k = fold over the 3^D neighbour keys (ascending)
// of q; one wave per cell, the probes in parallel as in k_shift.
template <int D, class Lookup>
__global__ __launch_bounds__(kShiftWaves * kWave) void k_adj_stencil(const uint64_t* __restrict__ key,
                                                                     const int32_t* __restrict__ inst,
                                                                     const int32_t* __restrict__ applied, int64_t m,
                                                                     const InstParam* __restrict__ param, Lookup lk,
                                                                     const double* __restrict__ q,
                                                                     double* __restrict__ out, int64_t cap, int xcd) {
    constexpr int NOFF = pow3(D);
    __shared__ int32_t list[kShiftWaves][NOFF];
    __shared__ double gval[kShiftWaves][D][kWave];  // gathered rows of found cells
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int64_t blk = xcd ? xcd_contiguous(blockIdx.x, gridDim.x) : int64_t(blockIdx.x);  // as in k_shift
    const int64_t j = blk * kShiftWaves + w;
    if (j >= m) return;
    const int b = inst[j];
    if (!applied[b]) {
        if (lane < D) out[int64_t(lane) * cap + j] = q[int64_t(lane) * cap + j];
        return;
    }
    const InstParam& P = param[b];
    const uint64_t kj = key[j];
    const uint64_t local = kj - P.base;
    int64_t crd[D];
#pragma unroll
    for (int k = 0; k < D; ++k) crd[k] = int64_t((local / P.stride[k]) % uint64_t(P.E[k]));
    const uint64_t lt = lanemask_lt();
    // every probe first (independent loads), then the found cells compacted
    // in probe order, as in k_shift
    constexpr int NIT = (NOFF + kWave - 1) / kWave;
    int64_t idx[NIT];
    uint64_t nks[NIT];
    bool want[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int r = it * kWave + lane;
        nks[it] = 0;
        want[it] = false;
        if (r < NOFF) {
            int rr = r;
            bool inside = true;
            uint64_t nk = kj;
#pragma unroll
            for (int k = D - 1; k >= 0; --k) {
                const int v = rr % 3 - 1;
                rr /= 3;
                const int64_t c = crd[k] + v;
                inside = inside && c >= 0 && c < P.E[k];
                nk += uint64_t(int64_t(v)) * P.stride[k];
            }
            nks[it] = nk;
            want[it] = inside;
        }
    }
    lk.template find_all<NIT>(nks, want, idx);
    int nfound = 0;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const uint64_t bal = __ballot(idx[it] >= 0);
        if (idx[it] >= 0) list[w][nfound + __popcll(bal & lt)] = int32_t(idx[it]);
        nfound += __popcll(bal);
    }
    __builtin_amdgcn_wave_barrier();
    // rows of the found cells gathered kWave at a time by the whole wave into
    // LDS, then lane k < D folds dimension k left to right from -0.0
    double acc = -0.0;
    for (int q0 = 0; q0 < nfound; q0 += kWave) {
        if (q0 + lane < nfound) {
            const int64_t k = list[w][q0 + lane];
#pragma unroll
            for (int dd = 0; dd < D; ++dd) gval[w][dd][lane] = q[int64_t(dd) * cap + k];
        }
        __builtin_amdgcn_wave_barrier();
        const int nq = nfound - q0 < kWave ? nfound - q0 : kWave;
        if (lane < D) {
            for (int u0 = 0; u0 < nq; u0 += 16) {
                double sv[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) sv[u] = u0 + u < nq ? gval[w][lane][u0 + u] : -0.0;
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    if (u0 + u < nq) acc = acc + sv[u];
            }
        }
        __builtin_amdgcn_wave_barrier();  // read before the next rows are written
    }
    if (lane < D) out[int64_t(lane) * cap + j] = acc;
}

// Gradient of the points: the Sbar of their initial cell, plus (for the loss)
// the direct term gL * (2 * (x - mode)).
template <typename T, int D>
__global__ __launch_bounds__(256) void k_adj_points(const uint32_t* __restrict__ cell0,
                                                    const double* __restrict__ sbar0, int64_t cap, int64_t n,
                                                    double* __restrict__ grad, const T* __restrict__ x, int64_t ld,
                                                    const int32_t* __restrict__ labels,
                                                    const double* __restrict__ modes,
                                                    const int64_t* __restrict__ row_off,
                                                    const int64_t* __restrict__ koff, int B,
                                                    const double* __restrict__ gloss) {
    const int64_t i0 = int64_t(blockIdx.x) * blockDim.x;
    const int64_t i = i0 + threadIdx.x;
    // instance of the block's first row, searched once; a row's own instance
    // is at most a few steps further (instances without rows are stepped over)
    __shared__ int s_b0;
    if (x) {
        if (threadIdx.x == 0) s_b0 = inst_of_row(row_off, B, i0 < n ? i0 : n - 1);
        __syncthreads();
    }
    if (i >= n) return;
    const uint32_t c = cell0[i];
    double sb[D];
#pragma unroll
    for (int k = 0; k < D; ++k) sb[k] = sbar0[k * cap + c];
    if (!x) {
#pragma unroll
        for (int k = 0; k < D; ++k) grad[i * D + k] = sb[k];
        return;
    }
    int b = s_b0;
    while (b + 1 < B && row_off[b + 1] <= i) ++b;
    const int64_t r = koff[b] + labels[i];
    const double gl = gloss[b];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double direct = gl * (2.0 * (load_coord(x, i, ld, k) - modes[r * D + k]));
        grad[i * D + k] = direct + sb[k];
    }
}

// ===========================================================================
// point-to-mode loss
// ===========================================================================
// Member p of instance b's "cell" is point p: value = left fold over k of
// (x_pk - mode_k)^2 of its cluster's mode.
template <typename T>
struct SrcLoss {
    const T* x;
    int64_t ld;
    const int32_t* labels;
    const double* modes;    // [sum K][d]
    const int64_t* koff;
    int d;
    // the cells of the loss table are the instances: b = cell
    __device__ int64_t load(int64_t p, double* v, int, int64_t cell) const {
        const int b = int(cell);
        const int64_t r = koff[b] + labels[p];
        double acc = 0.0;
        for (int k = 0; k < d; ++k) {
            const double e = load_coord(x, p, ld, k) - modes[r * d + k];
            acc = k == 0 ? e * e : acc + e * e;
        }
        v[0] = acc;
        return 1;
    }
};

// Member p of a cluster group is initial cell perm[p]: its initial sums.
struct SrcInit {
    const double* sums0;  // [d][m0]
    const uint32_t* perm;
    int64_t m0;
    __device__ int64_t load(int64_t p, double* v, int d, int64_t) const {
        const int64_t c = perm[p];
        for (int k = 0; k < d; ++k) v[k] = sums0[k * m0 + c];
        return 1;
    }
};

// Final cluster row of every initial cell.
__global__ void k_final_rows(const int32_t* __restrict__ inst0, const uint32_t* __restrict__ cur,
                             const uint32_t* __restrict__ tmap, const int64_t* __restrict__ koff, int64_t m0,
                             uint32_t* __restrict__ rows) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= m0) return;
    const uint32_t cc = cur ? cur[c] : uint32_t(c);
    rows[c] = uint32_t(koff[inst0[c]] + tmap[cc]);
}

// mubar_c = gL_b * (-2 * (X_c - C_c * mode_c)) for every cluster row.
__global__ void k_loss_mubar(const double* __restrict__ X, int64_t xcap, const int64_t* __restrict__ counts,
                             const double* __restrict__ modes, const int64_t* __restrict__ koff, int B, int64_t rows,
                             int d, const double* __restrict__ gloss, double* __restrict__ mubar) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const int b = inst_of_row(koff, B, r);
    const double C = double(counts[r]);
    for (int k = 0; k < d; ++k)
        mubar[r * d + k] = gloss[b] * (-2.0 * (X[k * xcap + r] - C * modes[r * d + k]));
}

// ===========================================================================
// outputs
// ===========================================================================
// Grid-stride over the points, four per thread per step; returns at once when
// `gate` is set and nonzero (the tail did not run).
constexpr int kLabelBlocks = 2048;
__global__ __launch_bounds__(256) void k_labels(const uint32_t* __restrict__ cell0, const uint32_t* __restrict__ cur,
                                                const uint32_t* __restrict__ tmap, int32_t* __restrict__ labels,
                                                int64_t n, const int64_t* __restrict__ gate,
                                                const InstState* __restrict__ st, int B, int64_t* __restrict__ koff,
                                                const int64_t* __restrict__ ctr, int64_t* __restrict__ host) {
    if (gate && *gate) return;
    if (koff && blockIdx.x == 0) {  // first output row of every instance's clusters
        __shared__ int64_t wt[4];
        const int w = int(threadIdx.x) / kWave, lane = lane_id();
        int64_t carry = 0;
        for (int b0 = 0; b0 < B; b0 += 256) {
            const int b = b0 + int(threadIdx.x);
            int64_t x = b < B ? st[b].K : 0;
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const int64_t y = __shfl_up(x, off, kWave);
                if (lane >= off) x += y;
            }
            if (lane == kWave - 1) wt[w] = x;
            __syncthreads();
            int64_t before = carry;
            for (int ww = 0; ww < w; ++ww) before += wt[ww];
            if (b < B) koff[b + 1] = before + x;
            carry += wt[0] + wt[1] + wt[2] + wt[3];
            __syncthreads();
        }
        if (threadIdx.x == 0) koff[0] = 0;
    }
    if (host && blockIdx.x == 0) publish_host(ctr, st, B, host);  // the tail's final states
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i0 < n; i0 += 4 * stride) {
        uint32_t c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + u * stride;
            c[u] = i < n ? cell0[i] : 0u;
        }
        if (cur) {
#pragma unroll
            for (int u = 0; u < 4; ++u) c[u] = cur[c[u]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + u * stride;
            if (i < n) labels[i] = int32_t(tmap[c[u]]);
        }
    }
}

// Row r of the concatenated output belongs to instance b with
// koff[b] <= r < koff[b+1]; its cell is cs[b] + (r - koff[b]).
__global__ void k_copy_modes(CellTable t, const InstState* __restrict__ st, const int64_t* __restrict__ koff, int B,
                             int64_t rows, int d, double* __restrict__ modes, int64_t* __restrict__ counts,
                             double* __restrict__ sums) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const int b = inst_of_row(koff, B, r);
    const int64_t c = st[b].cs + (r - koff[b]);
    const int64_t C = t.cnt[c];
    if (counts) counts[r] = C;
    for (int k = 0; k < d; ++k) {
        const double s = t.sum[k * t.cap + c];
        if (modes) modes[r * d + k] = s / double(C);
        if (sums) sums[r * d + k] = s;
    }
}

__global__ void k_copy_keys(CellTable t, const InstState* __restrict__ st, const InstParam* __restrict__ param,
                            const int64_t* __restrict__ koff, int B, int64_t rows, int d, int64_t* __restrict__ out) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const int b = inst_of_row(koff, B, r);
    const int64_t c = st[b].cs + (r - koff[b]);
    const InstParam& P = param[b];
    const uint64_t local = t.key[c] - P.base;
    for (int k = 0; k < d; ++k) out[r * d + k] = int64_t((local / P.stride[k]) % uint64_t(P.E[k])) + P.lo[k];
}

// ===========================================================================
// object tracking (Algorithm 2, Section 2.3)
// ===========================================================================
constexpr int kTrackThreads = 1024;
constexpr int kTrackSlots = 4096;  // LDS hash of the colour cells B
constexpr int kTrackMaxCells = 2048;
constexpr int kTrackMaxChannels = 4;

// Colour cell floor(fl(c_k / h)) of every channel, packed 16 bits per channel
// (q + 32768); false if some channel is outside [-32768, 32767), or not finite.
template <typename T>
__device__ __forceinline__ bool track_cell(const T* __restrict__ c, int dc, double h, uint64_t* out) {
    uint64_t key = 0;
    bool ok = true;
    for (int k = 0; k < dc; ++k) {
        const double q = floor(double(c[k]) / h);
        ok = ok && q >= -32768.0 && q < 32767.0;
        key |= uint64_t(ok ? int64_t(q) + 32768 : 0) << (16 * k);
    }
    *out = key;
    return ok;
}

__device__ __forceinline__ int track_hash(uint64_t key) {
    return int((key * 0x9E3779B97F4A7C15ull) >> (64 - 12));  // 12 bits: kTrackSlots
}

// Slot of `key` in the LDS table, or -1.
__device__ __forceinline__ int track_find(const uint64_t* tab, uint64_t key) {
    int s = track_hash(key);
    for (int probe = 0; probe < kTrackSlots; ++probe) {
        const uint64_t v = tab[s];
        if (v == key) return s;
        if (v == ~0ull) return -1;
        s = (s + 1) & (kTrackSlots - 1);
    }
    return -1;
}

// Copies the initial window of every track (rows y0.., columns x0.. of frame
// 0, ncols x nrows pixels, dc values each) densely into win at row p0 of the
// track, in raster order; one workgroup per track.
struct TrackRect {
    int x0, y0, ncols, nrows;
    int64_t p0;
};
template <typename T>
__global__ void k_track_windows(const T* __restrict__ frame0, int W, int dc, const TrackRect* __restrict__ rects,
                                T* __restrict__ win) {
    const TrackRect r = rects[blockIdx.x];
    const int64_t npx = int64_t(r.ncols) * r.nrows;
    for (int64_t e = threadIdx.x; e < npx * dc; e += blockDim.x) {
        const int64_t pix = e / dc;
        const int k = int(e - pix * dc);
        const int yy = r.y0 + int(pix / r.ncols), xx = r.x0 + int(pix % r.ncols);
        win[(r.p0 + pix) * dc + k] = frame0[(int64_t(yy) * W + xx) * dc + k];
    }
}

// One workgroup tracks one object through frames 1..T-1 (frame t, pixel
// (px, py): colour at ((t * H + py) * W + px) * dc).  B starts as the colour
// cells of the window pixels (win, n0 rows of dc values, raster order) whose
// initial cluster label is selected (sel[label] != 0).  Per frame, at most
// max_inner times: the search window W(o, l/f, w/f) (|px - o_x| <= l'/2,
// |py - o_y| <= w'/2); R = its pixels whose colour cell is in B; an empty R
// widens l and w by 1.1; otherwise o moves to the mean pixel position of R
// (exact integer sums), B shrinks to the cells R hit, l and w shrink by 0.99
// when R's extent along them is below them and grow by 1.01 otherwise, and
// the loop ends once the centre moved by less than eta.  windows[t] =
// (o_x, o_y, l, w) after frame t.  err: 1 = a selected colour cell is out of
// the packable range, 2 = B exceeds kTrackMaxCells.
// Per track: the initial window (centre, extents), its pixels' rows in the
// window buffer and their labels [p0, p1), and where its clusters' selection
// flags start.
struct TrackInit {
    double ox, oy, l, w;
    int64_t p0, p1, k0;
};

template <typename T>
__global__ __launch_bounds__(kTrackThreads) void k_track(const T* __restrict__ frames, int nT, int H, int W, int dc,
                                                         const T* __restrict__ win_all,
                                                         const int32_t* __restrict__ labels_all,
                                                         const TrackInit* __restrict__ init,
                                                         const int32_t* __restrict__ sel_all, double f, double h,
                                                         double eta, int max_inner, double* __restrict__ windows_all,
                                                         int32_t* __restrict__ err_all) {
    constexpr int NW = kTrackThreads / kWave;
    // one workgroup per track
    const TrackInit ti = init[blockIdx.x];
    const T* __restrict__ win = win_all + ti.p0 * dc;
    const int32_t* __restrict__ labels = labels_all + ti.p0;
    const int32_t* __restrict__ sel = sel_all + ti.k0;
    const int64_t n0 = ti.p1 - ti.p0;
    const double ox0 = ti.ox, oy0 = ti.oy, l0 = ti.l, w0 = ti.w;
    double* __restrict__ windows = windows_all + int64_t(blockIdx.x) * nT * 4;
    int32_t* __restrict__ err = err_all + blockIdx.x;
    __shared__ uint64_t tab[kTrackSlots];
    __shared__ uint32_t hit[kTrackSlots];  // stamp of the last step whose R held the cell
    __shared__ uint8_t alive[kTrackSlots];
    __shared__ int64_t red_i[NW][3];       // count, sum px, sum py
    __shared__ int32_t red_m[NW][4];       // min px, -max px, min py, -max py
    __shared__ double st_d[4];             // o_x, o_y, l, w
    __shared__ int st_flag[2];             // done, R non-empty
    __shared__ int s_ncells, s_err;
    const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
    for (int i = tid; i < kTrackSlots; i += kTrackThreads) {
        tab[i] = ~0ull;
        hit[i] = 0;
        alive[i] = 0;
    }
    if (tid == 0) {
        s_ncells = 0;
        s_err = 0;
        st_d[0] = ox0;
        st_d[1] = oy0;
        st_d[2] = l0;
        st_d[3] = w0;
    }
    __syncthreads();
    // ---- B: colour cells of the selected initial clusters
    for (int64_t j = tid; j < n0; j += kTrackThreads) {
        if (!sel[labels[j]]) continue;
        uint64_t key;
        if (!track_cell(win + j * dc, dc, h, &key)) {
            atomicOr(&s_err, 1);
            continue;
        }
        int s = track_hash(key);
        for (int probe = 0; probe < kTrackSlots; ++probe) {
            const uint64_t prev = atomicCAS(reinterpret_cast<unsigned long long*>(&tab[s]), ~0ull, key);
            if (prev == ~0ull) {
                alive[s] = 1;
                atomicAdd(&s_ncells, 1);
                break;
            }
            if (prev == key) break;
            s = (s + 1) & (kTrackSlots - 1);
        }
    }
    __syncthreads();
    if (tid == 0 && s_ncells > kTrackMaxCells) s_err |= 2;
    __syncthreads();
    if (s_err) {
        if (tid == 0) *err = s_err;
        return;
    }
    uint32_t stamp = 0;
    for (int t = 1; t < nT; ++t) {
        const T* fr = frames + int64_t(t) * H * W * dc;
        for (int it = 0; it < max_inner; ++it) {
            ++stamp;
            const double ox = st_d[0], oy = st_d[1];
            const double hl = 0.5 * (st_d[2] / f), hw = 0.5 * (st_d[3] / f);
            // bounding rows and columns (one pixel of margin), clamped to the frame
            const int c0 = int(fmax(0.0, ceil(ox - hl) - 1.0)), c1 = int(fmin(double(W - 1), floor(ox + hl) + 1.0));
            const int r0 = int(fmax(0.0, ceil(oy - hw) - 1.0)), r1 = int(fmin(double(H - 1), floor(oy + hw) + 1.0));
            const int ncols = c1 >= c0 ? c1 - c0 + 1 : 0;
            const int npix = r1 >= r0 ? (r1 - r0 + 1) * ncols : 0;  // H * W < 2^31
            int64_t cnt = 0, sx = 0, sy = 0;
            int32_t mnx = INT32_MAX, mxx = INT32_MIN, mny = INT32_MAX, mxy = INT32_MIN;
            // TP pixels per thread per pass, every colour load issued before any is used
            constexpr int TP = 4;
            for (int e0 = 0; e0 < npix; e0 += TP * kTrackThreads) {
                T cv[TP][kTrackMaxChannels];
                int pxs[TP], pys[TP];
                bool in[TP];
#pragma unroll
                for (int u = 0; u < TP; ++u) {
                    const int e = e0 + u * kTrackThreads + tid;
                    const int rr = e / ncols;
                    pys[u] = r0 + rr;
                    pxs[u] = c0 + (e - rr * ncols);
                    in[u] = e < npix && fabs(double(pxs[u]) - ox) <= hl && fabs(double(pys[u]) - oy) <= hw;
                    const T* c = fr + (int64_t(in[u] ? pys[u] : 0) * W + (in[u] ? pxs[u] : 0)) * dc;
#pragma unroll
                    for (int k = 0; k < kTrackMaxChannels; ++k) cv[u][k] = k < dc ? c[k] : T(0);
                }
#pragma unroll
                for (int u = 0; u < TP; ++u) {
                    uint64_t key;
                    if (!in[u] || !track_cell(cv[u], dc, h, &key)) continue;
                    const int s = track_find(tab, key);
                    if (s < 0 || !alive[s]) continue;
                    const int px = pxs[u], py = pys[u];
                    hit[s] = stamp;
                    ++cnt;
                    sx += px;
                    sy += py;
                    mnx = min(mnx, px);
                    mxx = max(mxx, px);
                    mny = min(mny, py);
                    mxy = max(mxy, py);
                }
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                cnt += __shfl_xor(cnt, off, kWave);
                sx += __shfl_xor(sx, off, kWave);
                sy += __shfl_xor(sy, off, kWave);
                mnx = min(mnx, __shfl_xor(mnx, off, kWave));
                mxx = max(mxx, __shfl_xor(mxx, off, kWave));
                mny = min(mny, __shfl_xor(mny, off, kWave));
                mxy = max(mxy, __shfl_xor(mxy, off, kWave));
            }
            if (lane == 0) {
                red_i[w][0] = cnt;
                red_i[w][1] = sx;
                red_i[w][2] = sy;
                red_m[w][0] = mnx;
                red_m[w][1] = mxx;
                red_m[w][2] = mny;
                red_m[w][3] = mxy;
            }
            __syncthreads();
            if (tid == 0) {
                int64_t C = 0, SX = 0, SY = 0;
                int32_t a = INT32_MAX, bx = INT32_MIN, c = INT32_MAX, dy_ = INT32_MIN;
                for (int ww = 0; ww < NW; ++ww) {
                    C += red_i[ww][0];
                    SX += red_i[ww][1];
                    SY += red_i[ww][2];
                    a = min(a, red_m[ww][0]);
                    bx = max(bx, red_m[ww][1]);
                    c = min(c, red_m[ww][2]);
                    dy_ = max(dy_, red_m[ww][3]);
                }
                double l = st_d[2], wd = st_d[3];
                int done = 0;
                if (C == 0) {
                    l = 1.1 * l;
                    wd = 1.1 * wd;
                } else {
                    const double nx = double(SX) / double(C), ny = double(SY) / double(C);
                    l = double(bx - a) < l ? 0.99 * l : 1.01 * l;
                    wd = double(dy_ - c) < wd ? 0.99 * wd : 1.01 * wd;
                    const double ddx = nx - ox, ddy = ny - oy;
                    done = ddx * ddx + ddy * ddy < eta * eta;
                    st_d[0] = nx;
                    st_d[1] = ny;
                }
                st_d[2] = l;
                st_d[3] = wd;
                st_flag[0] = done;
                st_flag[1] = C > 0;
            }
            __syncthreads();
            if (st_flag[1]) {  // B becomes the cells R hit
                for (int i = tid; i < kTrackSlots; i += kTrackThreads)
                    if (alive[i] && hit[i] != stamp) alive[i] = 0;
            }
            const int done = st_flag[0];
            __syncthreads();
            if (done) break;
        }
        if (tid == 0) {
            windows[int64_t(t) * 4 + 0] = st_d[0];
            windows[int64_t(t) * 4 + 1] = st_d[1];
            windows[int64_t(t) * 4 + 2] = st_d[2];
            windows[int64_t(t) * 4 + 3] = st_d[3];
        }
    }
    if (tid == 0) {
        windows[0] = ox0;
        windows[1] = oy0;
        windows[2] = l0;
        windows[3] = w0;
        *err = 0;
    }
}

}  // namespace gs
