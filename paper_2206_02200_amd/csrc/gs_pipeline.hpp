// Data structures and constants of the GridShift pipeline.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs_device.hpp"
#include "gs_sort.hpp"

namespace gs {

constexpr int kTailCells = 1024;    // cells one tail workgroup holds in LDS
constexpr int kTailThreads = 1024;  // one cell per thread
constexpr int kChunk = 256;         // leaves of one wave's sum subtree (64 lanes x 4)
constexpr int kScanTile = 8192;     // positions per look-back scan tile

// Device pointers of one cell table (struct of arrays with capacity cap).
struct CellTable {
    uint64_t* key = nullptr;    // packed key, ascending
    int64_t* cnt = nullptr;     // point count C
    double* sum = nullptr;      // coordinate sums S, [d][cap]
    int32_t* inst = nullptr;    // instance of the cell
    uint32_t* start = nullptr;  // first sorted position of the cell's members
    uint32_t* len = nullptr;    // number of members (points, or merged cells)
    uint32_t* first = nullptr;  // member index at `start`
    uint32_t* nch = nullptr;    // chunks of kChunk members
    uint32_t* choff = nullptr;  // exclusive scan of nch
    int64_t cap = 0;
};

// Per-round record of the tail rounds of every instance (for the adjoint):
// round tl of instance b occupies entries [b * stride + tl * kTailCells, ...).
struct TailTape {
    uint64_t* key = nullptr;  // local packed key of the cells the round started from
    int32_t* cnt = nullptr;   // their counts
    int32_t* W = nullptr;     // their shift weights
    uint32_t* g = nullptr;    // their merge map
    int32_t* m = nullptr;     // [B][max_rounds] cells of each round
    int64_t stride = 0;       // entries per instance
    int32_t max_rounds = 0;
};

// Checkpoints of the tail (differentiable form with recomputation): slot s of
// instance b holds the cell table at the start of tail round s * every, in
// entries [b * stride + s * kTailCells, ...); a k-round segment of the tape
// is recomputed from its slot during the backward pass.
struct TailCkpt {
    uint64_t* key = nullptr;  // local packed key
    int32_t* cnt = nullptr;   // counts
    double* sum = nullptr;    // sums, [d][total]
    int32_t* m = nullptr;     // [B][nslots] cells in each slot
    int64_t stride = 0;       // entries per instance (nslots * kTailCells)
    int64_t total = 0;        // B * stride
    int32_t nslots = 0;
    int32_t every = 0;        // 0: no checkpoints
};

}  // namespace gs
