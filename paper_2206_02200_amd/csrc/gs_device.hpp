// Device-side building blocks shared by the GridShift kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gs {

constexpr int kMaxDim = 6;
constexpr int kWave = 64;

// Per-instance key packing.  The cell with integer key q (d coordinates) of
// instance b has the packed key  base + sum_k (q_k - lo_k) * stride_k, with
// lo_k = min_k - 1, E_k = max_k - min_k + 3 (one empty margin cell on each
// side), stride_{d-1} = 1 and stride_k = stride_{k+1} * E_{k+1}.  Ascending
// packed order is ascending (instance, lexicographic key) order.
struct InstParam {
    double h;
    int64_t lo[kMaxDim];
    int64_t E[kMaxDim];
    uint64_t stride[kMaxDim];
    uint64_t base;   // first packed key of the instance
    uint64_t span;   // prod_k E_k (0 for an empty instance)
    int64_t row0;    // first point row
    int64_t row1;    // one past the last point row
};

// Per-instance iteration state.
struct InstState {
    int32_t t;        // rounds executed
    uint32_t flags;   // GS_CONVERGED / GS_STATIONARY / GS_CAPPED
    int32_t active;   // still iterating
    int32_t apply;    // this round shifts and merges
    int32_t any_nb;   // some cell had an active neighbour this round
    int32_t changed;  // this round changed keys, counts or sums
    int32_t err;      // error code raised on the device (GS_ERR_*)
    int32_t t_tail0;  // rounds executed before the tail workgroup took over
    int64_t cs, ce;   // cell range [cs, ce) in the current cell table
    int64_t K;        // clusters at exit
    int64_t m0;       // cells after binning
    int64_t tail_cells;  // sum over the tail's shift+merge rounds of the table size entering each
};
// the shift reads any_nb and changed with one 64-bit load
static_assert(offsetof(InstState, any_nb) % 8 == 0 && offsetof(InstState, changed) == offsetof(InstState, any_nb) + 4,
              "any_nb and changed share one aligned 64-bit word");

// ---------------------------------------------------------------------------
// wave helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Lane l + S of the same 16-lane row (DPP row_shl:S, S = 1, 2, 4 or 8) for a
// 64-bit value; lanes whose source lies past the row end keep their own.
template <int S>
__device__ __forceinline__ uint64_t row_down_u64(uint64_t x) {
    const int lo = int(uint32_t(x)), hi = int(uint32_t(x >> 32));
    const uint32_t nlo = uint32_t(__builtin_amdgcn_update_dpp(lo, lo, 0x100 + S, 0xf, 0xf, false));
    const uint32_t nhi = uint32_t(__builtin_amdgcn_update_dpp(hi, hi, 0x100 + S, 0xf, 0xf, false));
    return (uint64_t(nhi) << 32) | nlo;
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t x, int l) {
    const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(x)), l));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(x >> 32)), l));
    return (uint64_t(hi) << 32) | lo;
}

// Perfect binary tree over the 64 lane values (lane l holds leaf l), with the
// pairing of R: pairs (l, l + 1), then pairs of pairs, ... each level adding
// the left block's value to the right block's in that order (DPP row shifts
// within each 16-lane row, then the four row totals read out as
// (r0 + r1) + (r2 + r3)).  Missing leaves must hold -0.0, the exact additive
// identity.  Every lane returns the total.
__device__ __forceinline__ double wave_tree_sum(double v) {
    v = v + __longlong_as_double((long long)row_down_u64<1>(uint64_t(__double_as_longlong(v))));
    v = v + __longlong_as_double((long long)row_down_u64<2>(uint64_t(__double_as_longlong(v))));
    v = v + __longlong_as_double((long long)row_down_u64<4>(uint64_t(__double_as_longlong(v))));
    v = v + __longlong_as_double((long long)row_down_u64<8>(uint64_t(__double_as_longlong(v))));
    const uint64_t bv = uint64_t(__double_as_longlong(v));
    const double r0 = __longlong_as_double((long long)readlane_u64(bv, 0));
    const double r1 = __longlong_as_double((long long)readlane_u64(bv, 16));
    const double r2 = __longlong_as_double((long long)readlane_u64(bv, 32));
    const double r3 = __longlong_as_double((long long)readlane_u64(bv, 48));
    return (r0 + r1) + (r2 + r3);
}

__device__ __forceinline__ int64_t wave_tree_sum_i64(int64_t v) {
    v = v + int64_t(row_down_u64<1>(uint64_t(v)));
    v = v + int64_t(row_down_u64<2>(uint64_t(v)));
    v = v + int64_t(row_down_u64<4>(uint64_t(v)));
    v = v + int64_t(row_down_u64<8>(uint64_t(v)));
    return (int64_t(readlane_u64(uint64_t(v), 0)) + int64_t(readlane_u64(uint64_t(v), 16))) +
           (int64_t(readlane_u64(uint64_t(v), 32)) + int64_t(readlane_u64(uint64_t(v), 48)));
}

// ---------------------------------------------------------------------------
// look-back status words: [epoch:16][flag:2][value:46]
// ---------------------------------------------------------------------------
constexpr uint64_t kFlagAgg = 1;
constexpr uint64_t kFlagPrefix = 2;

__device__ __forceinline__ uint64_t lb_pack(uint32_t epoch, uint64_t flag, uint64_t value) {
    return (uint64_t(epoch & 0xffffu) << 48) | (flag << 46) | (value & ((1ull << 46) - 1));
}
__device__ __forceinline__ uint32_t lb_epoch(uint64_t w) { return uint32_t(w >> 48); }
__device__ __forceinline__ uint64_t lb_flag(uint64_t w) { return (w >> 46) & 3ull; }
__device__ __forceinline__ uint64_t lb_value(uint64_t w) { return w & ((1ull << 46) - 1); }

__device__ __forceinline__ void lb_store(uint64_t* p, uint64_t w) {
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t lb_load(const uint64_t* p) {
    return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix of `total` over all earlier tiles (decoupled look-back).
// The caller has already published its own aggregate.  Tile 0 returns 0.
// kWin predecessors are read per round trip; their words are consumed
// nearest first until an inclusive prefix is found.
constexpr int kLookSleep = 2;  // back-off (s_sleep units of 64 clocks) before polling an unpublished tile again

template <int kWin>
__device__ __forceinline__ uint64_t lb_exclusive(const uint64_t* status, int64_t tile, int64_t stride,
                                                 uint32_t epoch) {
    const uint32_t ep = epoch & 0xffffu;
    uint64_t excl = 0;
    int64_t p = tile - 1;
    while (p >= 0) {
        uint64_t w[kWin];
#pragma unroll
        for (int i = 0; i < kWin; ++i) w[i] = (p - i >= 0) ? lb_load(status + (p - i) * stride) : 0ull;
        int used = 0;
        bool done = false;
#pragma unroll
        for (int i = 0; i < kWin; ++i) {
            if (done || used != i) continue;
            if (p - i < 0) {
                done = true;
                continue;
            }
            if (lb_epoch(w[i]) != ep || lb_flag(w[i]) == 0) continue;  // not published yet
            excl += lb_value(w[i]);
            ++used;
            if (lb_flag(w[i]) == kFlagPrefix) done = true;
        }
        if (done) break;
        p -= used;  // unpublished predecessor: read again from there
        if (kLookSleep > 0 && used < kWin) __builtin_amdgcn_s_sleep(kLookSleep);
    }
    return excl;
}

// lb_exclusive for N adjacent status columns at once (status + j for column
// j): each column keeps its own position and stops at its own inclusive
// prefix, and every round trip reads the next kWin words of every column
// still walking.
template <int kWin, int N>
__device__ __forceinline__ void lb_exclusive_cols(const uint64_t* status, int64_t tile, int64_t stride,
                                                  uint32_t epoch, uint64_t* excl) {
    const uint32_t ep = epoch & 0xffffu;
    int64_t p[N];
    bool done[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        excl[j] = 0;
        p[j] = tile - 1;
        done[j] = p[j] < 0;
    }
    for (;;) {
        bool all = true;
#pragma unroll
        for (int j = 0; j < N; ++j) all = all && done[j];
        if (all) break;
        uint64_t w[N][kWin];
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int i = 0; i < kWin; ++i)
                w[j][i] = (!done[j] && p[j] - i >= 0) ? lb_load(status + (p[j] - i) * stride + j) : 0ull;
        bool stalled = false;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            if (done[j]) continue;
            int used = 0;
            bool fin = false;
#pragma unroll
            for (int i = 0; i < kWin; ++i) {
                if (fin || used != i) continue;
                if (p[j] - i < 0) {
                    fin = true;
                    continue;
                }
                if (lb_epoch(w[j][i]) != ep || lb_flag(w[j][i]) == 0) continue;  // not published yet
                excl[j] += lb_value(w[j][i]);
                ++used;
                if (lb_flag(w[j][i]) == kFlagPrefix) fin = true;
            }
            if (fin) {
                done[j] = true;
            } else {
                p[j] -= used;
                stalled = stalled || used < kWin;
            }
        }
        if (kLookSleep > 0 && stalled) __builtin_amdgcn_s_sleep(kLookSleep);
    }
}

// Look-back by a whole wave for one status word per tile: lane l reads
// predecessor p - l, so 64 predecessors cost one round trip.  Every lane
// returns the exclusive prefix.
__device__ __forceinline__ uint64_t lb_exclusive_wave(const uint64_t* status, int64_t tile, uint32_t epoch) {
    const uint32_t ep = epoch & 0xffffu;
    const int lane = __lane_id();
    uint64_t excl = 0;
    int64_t p = tile - 1;
    while (p >= 0) {
        const int64_t q = p - lane;
        // before tile 0 sits a virtual inclusive prefix of 0
        const uint64_t w = q >= 0 ? lb_load(status + q) : lb_pack(ep, kFlagPrefix, 0);
        const bool ready = lb_epoch(w) == ep && lb_flag(w) != 0;
        const uint64_t notready = __ballot(!ready);
        const uint64_t isprefix = __ballot(ready && lb_flag(w) == kFlagPrefix);
        const int first_nr = notready ? __ffsll((unsigned long long)notready) - 1 : 64;
        const uint64_t below = first_nr == 64 ? ~0ull : ((1ull << first_nr) - 1);
        const uint64_t pre = isprefix & below;
        const int upto = pre ? __ffsll((unsigned long long)pre) : first_nr;  // lanes consumed
        uint64_t v = lane < upto ? lb_value(w) : 0ull;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor((unsigned long long)v, off, 64);
        excl += v;
        p -= upto;
        if (pre) break;
    }
    return excl;
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP moves (row
// shifts by 1, 2, 4, 8 within each 16-lane row, then the row-15 and row-31
// broadcasts into the later rows), no LDS traffic.  Lanes whose DPP source
// lies outside the row, or whose row the mask leaves out, add 0.
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x) {
    x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x111, 0xf, 0xf, false));  // row_shr:1
    x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x112, 0xf, 0xf, false));  // row_shr:2
    x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x114, 0xf, 0xf, false));  // row_shr:4
    x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x118, 0xf, 0xf, false));  // row_shr:8
    x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x142, 0xa, 0xf, false));  // row_bcast:15 -> rows 1, 3
    x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x143, 0xc, 0xf, false));  // row_bcast:31 -> rows 2, 3
    return x;
}

// Value of lane (lane ^ S) for a compile-time S: DPP moves for S = 1, 2
// (quad permutations), 4 (row shifts left / right by 4, picked by lane bit
// 2) and 8 (row rotation by 8); a cross-lane permute otherwise.
template <int S>
__device__ __forceinline__ uint32_t lane_xor_u32(uint32_t x) {
    if constexpr (S == 1) {
        return uint32_t(__builtin_amdgcn_update_dpp(int(x), int(x), 0xB1, 0xf, 0xf, false));  // quad_perm 1,0,3,2
    } else if constexpr (S == 2) {
        return uint32_t(__builtin_amdgcn_update_dpp(int(x), int(x), 0x4E, 0xf, 0xf, false));  // quad_perm 2,3,0,1
    } else if constexpr (S == 4) {
        const uint32_t up = uint32_t(__builtin_amdgcn_update_dpp(int(x), int(x), 0x104, 0xf, 0xf, false));  // row_shl:4
        const uint32_t dn = uint32_t(__builtin_amdgcn_update_dpp(int(x), int(x), 0x114, 0xf, 0xf, false));  // row_shr:4
        return (__lane_id() & 4) ? dn : up;
    } else if constexpr (S == 8) {
        return uint32_t(__builtin_amdgcn_update_dpp(int(x), int(x), 0x128, 0xf, 0xf, false));  // row_ror:8
    } else {
        return uint32_t(__shfl_xor(int(x), S, 64));
    }
}

template <int S>
__device__ __forceinline__ uint64_t lane_xor_u64(uint64_t x) {
    const uint32_t lo = lane_xor_u32<S>(uint32_t(x));
    const uint32_t hi = lane_xor_u32<S>(uint32_t(x >> 32));
    return (uint64_t(hi) << 32) | lo;
}

// One bitonic compare-exchange step (partner lane ^ STRIDE) of the ascending
// sort of 64 values over the lanes, within blocks of SIZE.
template <int SIZE, int STRIDE>
__device__ __forceinline__ uint64_t bitonic_step_u64(uint64_t v) {
    const uint64_t o = lane_xor_u64<STRIDE>(v);
    const int lane = __lane_id();
    const bool keep_min = ((lane & STRIDE) == 0) == ((lane & SIZE) == 0);
    return keep_min ? (o < v ? o : v) : (o > v ? o : v);
}

template <int SIZE, int STRIDE>
__device__ __forceinline__ uint64_t bitonic_merge_u64(uint64_t v) {
    v = bitonic_step_u64<SIZE, STRIDE>(v);
    if constexpr (STRIDE > 1) v = bitonic_merge_u64<SIZE, STRIDE / 2>(v);
    return v;
}

// Ascending sort of one value per lane over the 64 lanes of a wave.
__device__ __forceinline__ uint64_t wave_sort_u64(uint64_t v) {
    v = bitonic_merge_u64<2, 1>(v);
    v = bitonic_merge_u64<4, 2>(v);
    v = bitonic_merge_u64<8, 4>(v);
    v = bitonic_merge_u64<16, 8>(v);
    v = bitonic_merge_u64<32, 16>(v);
    v = bitonic_merge_u64<64, 32>(v);
    return v;
}

// Raise *flag (set it to 1) for every lane with `pred`, with one atomic per
// distinct flag address in the wave (skipped when the flag is already set):
// many lanes raising one flag at once would serialise on that address.
__device__ __forceinline__ void wave_flag_or(int32_t* flag, bool pred) {
    const uint64_t bal = __ballot(pred);
    if (!bal) return;
    const int leader = __ffsll((unsigned long long)bal) - 1;
    const uint64_t lf = __shfl((unsigned long long)(uintptr_t)flag, leader, 64);
    const bool mine = (__lane_id() == leader) || (pred && (uint64_t)(uintptr_t)flag != lf);
    if (mine && __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) atomicOr(flag, 1);
}

// Instance of a row / packed key by binary search over the sorted bounds.
__device__ __forceinline__ int inst_of_row(const int64_t* __restrict__ row_off, int B, int64_t row) {
    int lo = 0, hi = B;  // row_off[lo] <= row < row_off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (row_off[mid] <= row) lo = mid; else hi = mid;
    }
    return lo;
}

}  // namespace gs
