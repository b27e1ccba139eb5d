// Stable LSD radix sort of (key, index) pairs, one read and one write of the
// pairs per digit of 8 or 10 bits (a single-pass "onesweep" scheme):
//   * all digit histograms come from one up-front pass (or from the key
//     producer, which fuses it); every tile derives its pass's digit bases
//     from them, and the first pass clears the other of two histogram
//     buffers for the next sort;
//   * every pass ranks its tile (8192 keys, or 4096) in LDS with wave64 ballots, stably
//     (positions ascend with the input order), publishes the tile's digit
//     counts and finds the counts of all earlier tiles by decoupled look-back;
//   * the tile is reordered by digit in LDS and written out in digit runs, so
//     consecutive lanes store consecutive addresses.
// Tiles take their index from an atomic counter (never reset: the host keeps
// its value before each launch), so a tile only ever waits on tiles that
// started before it: the look-back always terminates.
#include "gs_device.hpp"
#include "gs_sort.hpp"

namespace gs {

template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const K* __restrict__ keys, int64_t n, int npasses,
                                                            int digit, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[kHistLds];
    const int nh = npasses << digit;
    for (int i = threadIdx.x; i < nh; i += kSortThreads) h[i] = 0;
    __syncthreads();
    const int64_t stride = int64_t(gridDim.x) * kSortThreads;
    for (int64_t i = int64_t(blockIdx.x) * kSortThreads + threadIdx.x; i < n; i += stride)
        sort_hist_add<K>(h, keys[i], npasses, digit);
    __syncthreads();
    uint32_t* hc = hist + (blockIdx.x % kHistCopies) * kHistStride;
    for (int i = threadIdx.x; i < nh; i += kSortThreads)
        if (h[i]) atomicAdd(&hc[hist_index(i, digit)], h[i]);
}

__global__ void k_iota(uint32_t* __restrict__ v, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) v[i] = uint32_t(i);
}

__global__ void k_clear_u32(uint32_t* __restrict__ p, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_clear_u64(uint64_t* __restrict__ p, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

constexpr int kSortLookWindow = 4;

// One pass over digit (key >> shift) of DIG bits (the last pass ranks only
// its nbits significant bits).  Threads t < RADIX / DPT own digits
// t * DPT .. t * DPT + DPT - 1.
template <typename K, int DIG, int ITEMS>
__global__ __launch_bounds__(kPassThreads) void k_sort_pass(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                            K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                            int64_t n, int shift, int nbits,
                                                            const uint32_t* __restrict__ hist,
                                                            uint32_t* __restrict__ clear, int64_t ntiles,
                                                            uint64_t* __restrict__ look, uint32_t* __restrict__ ctr,
                                                            uint32_t tile_base, uint32_t epoch) {
    constexpr int W = kPassThreads / kWave;
    constexpr int TILE = kPassThreads * ITEMS;
    constexpr int RADIX = 1 << DIG;
    constexpr int DPT = RADIX > kPassThreads ? RADIX / kPassThreads : 1;  // digits per owning thread
    constexpr int OWN = RADIX / DPT;                                      // owning threads
    constexpr int OW = OWN / kWave;                                       // owning waves
    static_assert(OWN <= kPassThreads && OWN % kWave == 0, "digits are owned by whole waves");
    __shared__ uint32_t wcnt[W][RADIX];  // per-wave digit counts, then their exclusive scan over waves
    __shared__ uint32_t doff[RADIX];     // tile-local exclusive digit offsets
    __shared__ uint32_t wsum[OW];        // per-wave totals of the digit scan (owning waves)
    __shared__ uint32_t hsum[OW];        // per-wave totals of the histogram scan (owning waves)
    __shared__ uint32_t gbase[RADIX];    // global position of the tile's first key of each digit
    __shared__ K skey[TILE];
    __shared__ uint32_t sval[TILE];
    __shared__ int64_t s_tile;

    const int tid = threadIdx.x;
    const int w = tid / kWave;
    const int lane = lane_id();
    if (tid == 0) s_tile = int64_t(atomicAdd(ctr, 1u) - tile_base);
    for (int i = tid; i < W * RADIX; i += kPassThreads) (&wcnt[0][0])[i] = 0;
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t t0 = tile * TILE;
    const bool dig = tid < OWN;
    const int d0 = tid * DPT;  // first digit of this thread
    // the pass's count of each owned digit over all keys (its histogram
    // copies), loaded now and scanned over the digits after the ranking
    uint32_t dtot[DPT];
#pragma unroll
    for (int j = 0; j < DPT; ++j) dtot[j] = 0;
    if (dig) {
#pragma unroll
        for (int c = 0; c < kHistCopies; ++c)
#pragma unroll
            for (int j = 0; j < DPT; ++j) dtot[j] += hist[c * kHistStride + d0 + j];
    }
    if (clear) {  // this tile's slice of the other histogram buffer
        const int64_t total = int64_t(kHistCopies) * kHistStride;
        const int64_t per = (total + ntiles - 1) / ntiles;
        const int64_t z1 = (tile + 1) * per < total ? (tile + 1) * per : total;
        for (int64_t i = tile * per + tid; i < z1; i += kPassThreads) clear[i] = 0;
    }

    // Load: wave w owns keys [w*64*ITEMS, (w+1)*64*ITEMS) of the tile, slot i
    // covers 64 consecutive keys, so (slot, lane) order is input order.
    K key[ITEMS];
    uint32_t val[ITEMS];
    uint32_t rank[ITEMS];
    const uint64_t lt = lanemask_lt();
    const int64_t wbase = t0 + int64_t(w) * (kWave * ITEMS) + lane;
    // all loads first, so that the 16 slots' memory latency overlaps
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t pos = wbase + i * kWave;
        key[i] = pos < n ? kin[pos] : K(0);
    }
    if (vin) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int64_t pos = wbase + i * kWave;
            val[i] = pos < n ? vin[pos] : 0u;
        }
    } else {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) val[i] = uint32_t(wbase + i * kWave);
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const bool valid = wbase + i * kWave < n;
        const uint32_t dgt = uint32_t(key[i] >> shift) & uint32_t(RADIX - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < DIG; ++b) {
            if (b >= nbits) break;  // digits of the last pass may be narrower (higher bits are zero)
            const bool bit = (dgt >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        uint32_t prior = 0;
        if (valid) prior = wcnt[w][dgt];
        rank[i] = prior + uint32_t(__popcll(peers & lt));
        if (valid && lane == 63 - __clzll(peers)) wcnt[w][dgt] = prior + uint32_t(__popcll(peers));
    }
    __syncthreads();

    // Scan the per-wave counts over waves (per owned digit) and publish the
    // tile totals for the look-back at once, so that later tiles can use them.
    uint32_t run[DPT];  // this tile's count of each owned digit
    uint64_t* st = look + tile * RADIX + d0;
    if (dig) {
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            run[j] = 0;
#pragma unroll
            for (int ww = 0; ww < W; ++ww) {
                const uint32_t c = wcnt[ww][d0 + j];
                wcnt[ww][d0 + j] = run[j];
                run[j] += c;
            }
            lb_store(st + j, lb_pack(epoch, tile == 0 ? kFlagPrefix : kFlagAgg, run[j]));
        }
    } else {
#pragma unroll
        for (int j = 0; j < DPT; ++j) run[j] = 0;
    }
    // tile-local exclusive scan over the digit totals and global one over the
    // pass's digit counts: within the thread over its digits, then a DPP scan
    // over the owning waves' lanes, then across those waves' totals
    uint32_t dbase[DPT];  // keys of all smaller digits in the whole pass
    {
        uint32_t tsum = 0, hts = 0;
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            tsum += run[j];
            hts += dtot[j];
        }
        const uint32_t incl = wave_incl_scan_u32(tsum), hincl = wave_incl_scan_u32(hts);
        if (dig && lane == kWave - 1) {
            wsum[w] = incl;
            hsum[w] = hincl;
        }
        __syncthreads();
        if (dig) {
            uint32_t before = 0, hbefore = 0;
#pragma unroll
            for (int ww = 0; ww < OW; ++ww) {
                before += ww < w ? wsum[ww] : 0u;
                hbefore += ww < w ? hsum[ww] : 0u;
            }
            uint32_t a = before + incl - tsum, ha = hbefore + hincl - hts;
#pragma unroll
            for (int j = 0; j < DPT; ++j) {
                doff[d0 + j] = a;
                dbase[j] = ha;
                a += run[j];
                ha += dtot[j];
            }
        }
    }
    __syncthreads();

    // Reorder the tile by digit in LDS (local offsets only), which leaves the
    // items' registers free for a wide look-back.
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t pos = t0 + int64_t(w) * (kWave * ITEMS) + i * kWave + lane;
        if (pos < n) {
            const uint32_t dgt = uint32_t(key[i] >> shift) & uint32_t(RADIX - 1);
            const uint32_t lp = doff[dgt] + wcnt[w][dgt] + rank[i];
            skey[lp] = key[i];
            sval[lp] = val[i];
        }
    }
    // Exclusive prefix of each owned digit over all earlier tiles (decoupled
    // look-back, kSortLookWindow predecessors per round trip), then this
    // tile's prefix.
    if (dig) {
        if (tile == 0) {
#pragma unroll
            for (int j = 0; j < DPT; ++j) gbase[d0 + j] = dbase[j];
        } else {
            uint64_t excl[DPT];
            lb_exclusive_cols<kSortLookWindow, DPT>(look + d0, tile, RADIX, epoch, excl);
#pragma unroll
            for (int j = 0; j < DPT; ++j) {
                lb_store(st + j, lb_pack(epoch, kFlagPrefix, excl[j] + run[j]));
                gbase[d0 + j] = dbase[j] + uint32_t(excl[j]);
            }
        }
    }
    __syncthreads();

    // Write out: entry j of the reordered tile goes to gbase[digit] + (j - doff[digit]).
    const int64_t cnt = (n - t0) < TILE ? (n - t0) : TILE;
    for (int j = tid; j < cnt; j += kPassThreads) {
        const K k = skey[j];
        const uint32_t dgt = uint32_t(k >> shift) & uint32_t(RADIX - 1);
        const uint32_t g = gbase[dgt] + (uint32_t(j) - doff[dgt]);
        kout[g] = k;
        vout[g] = sval[j];
    }
}

template <typename K>
hipError_t radix_sort(K* kA, K* kB, uint32_t* vA, uint32_t* vB, int64_t n, int bits, bool hist_ready,
                      SortScratch& sc, hipStream_t s, K** kout, uint32_t** vout, const K* kin) {
    const SortPlan plan = sort_plan(bits, sc.allow10);
    const int np = plan.passes, dg = plan.digit;
    const K* k0 = kin ? kin : kA;  // keys read by the first pass
    *kout = const_cast<K*>(k0);
    *vout = vA;
    if (n <= 0) return hipSuccess;
    if (np == 0) {
        k_iota<<<dim3(unsigned((n + 255) / 256)), dim3(256), 0, s>>>(vA, n);
        return hipGetLastError();
    }
    const int items = sc.tile_keys == kSortTile / 2 ? kSortItems / 2 : kSortItems;
    const int64_t tiles = (n + int64_t(kPassThreads) * items - 1) / (int64_t(kPassThreads) * items);
    if (tiles * (int64_t(1) << dg) > sc.look_words) return hipErrorInvalidValue;
    uint32_t* hcur = sc.hist + int64_t(sc.parity) * kHistCopies * kHistStride;
    uint32_t* hother = sc.hist + int64_t(sc.parity ^ 1) * kHistCopies * kHistStride;
    if (!hist_ready) {
        k_clear_u32<<<dim3(unsigned((kHistCopies * kHistStride + 255) / 256)), dim3(256), 0, s>>>(
            hcur, kHistCopies * kHistStride);
        int64_t blocks = (n + kSortThreads * 16 - 1) / (kSortThreads * 16);
        if (blocks > 2048) blocks = 2048;
        const int tk = sc.prof_begin ? sc.prof_begin(sc.prof_ctx, s, "sort_hist") : -1;
        k_sort_hist<K><<<dim3(unsigned(blocks)), dim3(kSortThreads), 0, s>>>(k0, n, np, dg, hcur);
        if (sc.prof_end) sc.prof_end(sc.prof_ctx, s, tk, double(n) * sizeof(K));
    }
    const K* ki = k0;
    K* ko = kB;
    uint32_t* vi = nullptr;
    uint32_t* vo = vA;
    for (int p = 0; p < np; ++p) {
        if (sc.epoch >= 0xffffu) {  // epochs wrap: clear the status words once
            k_clear_u64<<<dim3(unsigned((sc.look_words + 255) / 256)), dim3(256), 0, s>>>(sc.look, sc.look_words);
            sc.epoch = 0;
        }
        if (sc.tile_base + uint64_t(tiles) >= 0x7fffffffull) {  // first use, or the counter nears overflow
            k_clear_u32<<<dim3(1), dim3(64), 0, s>>>(sc.ctr, 1);
            sc.tile_base = 0;
        }
        const uint32_t ep = ++sc.epoch;
        const uint32_t base = uint32_t(sc.tile_base);
        sc.tile_base += uint64_t(tiles);
        const int tk = sc.prof_begin ? sc.prof_begin(sc.prof_ctx, s, "sort_pass") : -1;
        const int nb = bits - dg * p < dg ? bits - dg * p : dg;
#define GS_PASS(DG, IT)                                                                                        \
    k_sort_pass<K, DG, IT><<<dim3(unsigned(tiles)), dim3(kPassThreads), 0, s>>>(                                \
        ki, vi, ko, vo, n, dg * p, nb, hcur + p * kRadixMax, p == 0 ? hother : nullptr, tiles, sc.look, sc.ctr, \
        base, ep)
        if (dg == 10) {
            if (items == kSortItems) GS_PASS(10, kSortItems); else GS_PASS(10, kSortItems / 2);
        } else {
            if (items == kSortItems) GS_PASS(8, kSortItems); else GS_PASS(8, kSortItems / 2);
        }
#undef GS_PASS
        // reads keys (and values after the first pass), writes keys and values
        if (sc.prof_end)
            sc.prof_end(sc.prof_ctx, s, tk, double(n) * (sizeof(K) + (p ? 4 : 0) + sizeof(K) + 4));
        // the next pass reads this one's output and writes over the buffer
        // this one read (kA when the first pass read `kin`)
        K* kt = (p == 0) ? kA : const_cast<K*>(ki);
        ki = ko;
        ko = kt;
        vi = vo;
        vo = (vo == vA) ? vB : vA;
    }
    sc.parity ^= 1;  // the next producer accumulates into the buffer cleared above
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) sc.tile_base = 0x7fffffffull;  // counter state unknown: clear it before the next use
    *kout = const_cast<K*>(ki);
    *vout = vi;
    return e;
}

template hipError_t radix_sort<uint32_t>(uint32_t*, uint32_t*, uint32_t*, uint32_t*, int64_t, int, bool,
                                         SortScratch&, hipStream_t, uint32_t**, uint32_t**, const uint32_t*);
template hipError_t radix_sort<uint64_t>(uint64_t*, uint64_t*, uint32_t*, uint32_t*, int64_t, int, bool,
                                         SortScratch&, hipStream_t, uint64_t**, uint32_t**, const uint64_t*);

}  // namespace gs
