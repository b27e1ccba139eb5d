// Stable LSD radix sort of (key, index) pairs for gfx950 (host interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gs {

constexpr int kSortThreads = 256;                        // histogram kernel block
constexpr int kPassThreads = 512;                        // one sort-pass tile: 8 waves
constexpr int kSortItems = 16;                           // keys per thread
constexpr int kSortTile = kPassThreads * kSortItems;     // 8192 keys per tile
constexpr int kSortMaxPasses = 8;                        // 8-bit digits, up to 64 bits
constexpr int kRadixMax = 1024;                          // widest digit: 10 bits
constexpr int kHistCopies = 16;                          // histogram copies that producers spread atomics over
constexpr int kHistStride = kSortMaxPasses * kRadixMax;  // entries of one copy (pass p from p * kRadixMax)
constexpr int64_t kHistEntries = 2 * kHistCopies * kHistStride;  // both histogram buffers
constexpr int kHistLds = 4096;                           // LDS histogram of a producer: passes x digits

// Digits of a sort: with allow10, 10-bit digits where that saves a pass (at
// most 4 of them, e.g. 17..20-bit or 25..30-bit keys), else 8-bit digits.
struct SortPlan {
    int passes;
    int digit;  // bits per digit (8 or 10); the last digit holds the remaining bits
};
inline SortPlan sort_plan(int bits, bool allow10 = true) {
    if (bits <= 0) return {0, 8};
    const int p8 = (bits + 7) / 8, p10 = (bits + 9) / 10;
    if (allow10 && p10 < p8 && p10 <= 4) return {p10, 10};
    return {p8, 8};
}

// Optional timing hooks: begin returns a token (or -1), end closes it with the
// algorithmic bytes the launch had to move.
typedef int (*ProfBeginFn)(void* ctx, hipStream_t s, const char* name);
typedef void (*ProfEndFn)(void* ctx, hipStream_t s, int token, double bytes);

struct SortScratch {
    // [2][kHistCopies][kSortMaxPasses][256] digit histograms (summed over the
    // copies), two buffers: producers accumulate into buffer `parity`, which
    // is zero beforehand; a sort reads it and clears the other one
    uint32_t* hist = nullptr;
    int parity = 0;
    uint32_t* cur_hist() const { return hist + int64_t(parity) * kHistCopies * kHistStride; }
    uint32_t* ctr = nullptr;    // tile ticket counter
    uint64_t tile_base = 0x7fffffffull;  // its value before the next pass (>= 2^31 - 1: clear it first)
    uint64_t* look = nullptr;   // [tiles][radix] look-back status words
    int64_t look_words = 0;     // capacity of `look` in words
    uint32_t epoch = 0;         // last epoch used in `look`
    bool allow10 = true;        // sort_plan's choice of 10-bit digits
    int tile_keys = kSortTile;  // keys per pass tile: kSortTile or kSortTile / 2
    void* prof_ctx = nullptr;
    ProfBeginFn prof_begin = nullptr;
    ProfEndFn prof_end = nullptr;
};

inline int sort_passes(int bits) { return sort_plan(bits).passes; }

// Tiles of a pass over n keys (with the smaller of the two tile sizes).
inline int64_t sort_look_tiles(int64_t n) { return (n + kSortTile / 2 - 1) / (kSortTile / 2); }

// Look-back words a sort of n keys by `bits`-bit keys needs (one per tile
// and digit value).
inline int64_t sort_look_words(int64_t n, int bits) {
    return sort_look_tiles(n) * (int64_t(1) << sort_plan(bits, true).digit);  // the wider of the two plans
}

// Sort n pairs by the low `bits` bits of the key, stably.  The keys are in
// `kin` when it is given (left unchanged; kA is then a third buffer), else in
// kA; the values are implicitly 0..n-1.  kB, vA, vB are ping-pong buffers of
// n entries.  If `hist_ready`, histogram buffer sc.parity already holds the
// digit histograms of the keys for every pass (computed by the key producer).
// On return *kout/*vout point at the sorted keys and the permutation (inside
// kA/kB, vA/vB; *kout is `kin` itself when the keys have no bits to sort).
template <typename K>
hipError_t radix_sort(K* kA, K* kB, uint32_t* vA, uint32_t* vB, int64_t n, int bits, bool hist_ready,
                      SortScratch& sc, hipStream_t s, K** kout, uint32_t** vout, const K* kin = nullptr);

// Per-pass digit histogram accumulation for a key (device helper used by
// producers that compute keys and histograms in one pass); the LDS
// histogram holds pass p at p << digit.
template <typename K>
__device__ __forceinline__ void sort_hist_add(uint32_t* lds_hist, K key, int npasses, int digit) {
    const uint32_t mask = (1u << digit) - 1u;
    for (int p = 0; p < npasses; ++p) {
        const uint32_t dgt = uint32_t(key >> (digit * p)) & mask;
        atomicAdd(&lds_hist[(p << digit) + dgt], 1u);
    }
}

// Global histogram index of LDS histogram entry i (pass i >> digit).
__host__ __device__ inline int hist_index(int i, int digit) {
    return (i >> digit) * kRadixMax + (i & ((1 << digit) - 1));
}

}  // namespace gs
