/*
 * gridshift.h - C ABI of the MI355X (gfx950) GridShift library.
 *
 * GridShift (Kumar et al., arXiv 2206.02200) clusters points by grid-based
 * mode seeking.  Section 2.1 (i) and Algorithm 1 bin the points into cells of
 * side h; every active cell keeps a point count and a coordinate sum.  Each
 * round (Section 2.1 (ii)-(iv), Eq. 1-4, in the parallel form of Eq. 6) moves
 * every active cell to the count-weighted mean of the active cells among its
 * 3^d neighbours, re-bins the moved cells and merges the cells that land on
 * the same key (gs_context_set_update selects the sequential form of Eq. 5
 * instead).  The rounds stop when no active cell has an active neighbour
 * (Section 2.1 (v), Theorem 2), after max_iter rounds, or when a round leaves
 * the state bitwise unchanged.  Labels are then propagated back to the points.
 *
 * Arithmetic: every sum, division and floor runs in IEEE binary64 without
 * contraction, in a fixed order, so results do not depend on launch shapes:
 *   key(v)       = floor(fl(v / h)) per coordinate (Section 2.1 (i), (iii));
 *   cell sum     = R over the cell's points in ascending point index, where
 *                  R(a_0..a_{L-1}) = a_0 if L = 1, else R(first P) + R(rest),
 *                  P the largest power of two below L;
 *   3^d sum      = left fold over the active neighbours in ascending key
 *                  (lexicographic, dimension 0 most significant), integer
 *                  weight sum (Eq. 1-2);
 *   merge sum    = R over fl(C_j * p_j) for the merging cells in ascending old
 *                  key (Eq. 3); the merged cell keeps the landing key;
 *   mode         = fl(S / C).
 * Clusters are numbered per instance in ascending lexicographic key.
 *
 * Conventions:
 *   - "device" pointers are HIP device memory on the context's device;
 *     "host" pointers are ordinary host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All device work of a call is ordered on it.  gs_fit / gs_fit_batched
 *     synchronise the stream before returning, because cluster counts and
 *     flags are returned in host memory.
 *   - The caller owns every array it passes.  A result (gs_fit) or a context
 *     (gs_ctx_fit) owns its scratch device memory, taken from the caller's
 *     gs_allocator when one is given and from hipMalloc otherwise; a
 *     context's grows on demand and is reused by later calls, and its last
 *     fit's results stay in it until its next fit.
 *   - Errors are returned as gs_status codes; gs_last_error() gives text.  The
 *     library never aborts the process.  On error the context holds no result.
 *   - A context is used by one host thread at a time; different contexts may
 *     be used concurrently on different streams.
 *   - Limits: 1 <= d <= 6, 0 <= n < 2^31 points in total, h finite and > 0,
 *     |floor(x/h)| < 2^52, and the per-instance key boxes
 *     prod_k (max_k - min_k + 3) must sum to less than 2^62 (else
 *     GS_ERR_KEY_RANGE).
 */
#ifndef GRIDSHIFT_H
#define GRIDSHIFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_ABI_VERSION 1

typedef enum {
    GS_OK = 0,
    GS_ERR_INVALID_ARG = 1, /* bad sizes, pointers, h, d, max_iter */
    GS_ERR_NONFINITE = 2,   /* a NaN or infinite coordinate */
    GS_ERR_KEY_RANGE = 3,   /* cell keys do not fit the packed 62-bit key space */
    GS_ERR_ALLOC = 4,       /* device allocation failed */
    GS_ERR_DEVICE = 5,      /* a HIP runtime error */
    GS_ERR_UNSUPPORTED = 6, /* d outside 1..6; a recorded fit with the sequential update */
    GS_ERR_STATE = 7        /* no fit result in the context */
} gs_status;

typedef enum { GS_F32 = 0, GS_F64 = 1 } gs_dtype;

/* gs_info.flags bits */
#define GS_CONVERGED 1u  /* no active cell had an active neighbour */
#define GS_STATIONARY 2u /* the last round left keys, counts and sums unchanged */
#define GS_CAPPED 4u     /* stopped after max_iter rounds with neighbours left */

typedef struct {
    int64_t n_points;   /* points of the instance */
    int64_t n_cells0;   /* active cells after binning (m_0) */
    int64_t n_clusters; /* K: active cells at exit */
    int32_t n_iter;     /* shift+merge rounds executed */
    uint32_t flags;     /* GS_CONVERGED | GS_STATIONARY | GS_CAPPED */
} gs_info;

/*
 * Device memory supplied by the caller (for instance a framework's caching
 * allocator): alloc returns `bytes` of device memory usable on `stream` (NULL
 * on failure), free gives back a pointer alloc returned, ordered on the
 * stream it was allocated for.  ctx is passed back unchanged.
 */
typedef struct {
    void* (*alloc)(void* ctx, size_t bytes, void* stream);
    void (*free)(void* ctx, void* p, void* stream);
    void* ctx;
} gs_allocator;

/* One point set for gs_fit.  ckpt_every: 0 records nothing, 1 records the
 * whole trajectory for gs_backward and the loss gradient, k > 1 records it
 * with tail checkpoints every k rounds (see gs_context_set_tape). */
typedef struct {
    const void* points; /* device, n rows of ld elements of dtype (ld >= d) */
    gs_dtype dtype;
    int64_t n;
    int32_t d;
    int64_t ld;
    double h;
    int32_t max_iter;
    int32_t ckpt_every;
} gs_problem;

/* The result of one fit: its cluster tables, summaries and (when recorded)
 * trajectory, held in device memory from the fit's allocator until
 * gs_result_free. */
typedef struct gs_result gs_result;

/*
 * Plain fit of one point set (Section 2.1, Algorithm 1; the update of Eq. 6),
 * with every piece of scratch and the trajectory taken from `a` (NULL:
 * hipMalloc; with an allocator, in a few large chunks, each at least as
 * large as all before it, asked for the fit's stream).  labels device int32 [n] receives the cluster of every point
 * (0..K-1, ascending final key); *out the result, owned by the caller and
 * released with gs_result_free.  The stream is synchronised once before the
 * call returns (K and the flags are host-visible).  On error *out is NULL.
 */
gs_status gs_fit(const gs_problem* p, const gs_allocator* a, void* stream, int32_t* labels, gs_result** out);

/*
 * Batched fit of B concatenated instances (rows offsets[b]..offsets[b+1]-1
 * of points [offsets[B]][d], bandwidth h[b]; offsets, h host), bitwise B
 * plain fits; labels device int32 [offsets[B]] (ids local per instance).
 */
gs_status gs_fit_batched(const void* points, gs_dtype dtype, int32_t d, int32_t B, const int64_t* offsets,
                         const double* h, int32_t max_iter, int32_t ckpt_every, const gs_allocator* a, void* stream,
                         int32_t* labels, gs_result** out);

/* Summary of instance `instance` (0 for a plain fit) into host *out. */
gs_status gs_result_info(const gs_result* r, int32_t instance, gs_info* out);

/* Host int64 [B+1]: instance b's clusters are rows k_offsets[b] .. k_offsets[b+1]-1. */
gs_status gs_result_offsets(const gs_result* r, int64_t* k_offsets);

/* Modes fl(S/C) device double [sum K][d] and counts device int64 [sum K]
 * (either may be NULL), instances concatenated. */
gs_status gs_result_copy(const gs_result* r, double* modes, int64_t* counts, void* stream);

/* Adjoint of the modes (a recorded fit, ckpt_every >= 1; else GS_ERR_STATE):
 * grad_modes device double [sum K][d], grad_points device double [N][d]
 * (overwritten); the reverse pass is described at gs_context_set_tape. */
gs_status gs_backward(const gs_result* r, const double* grad_modes, double* grad_points, void* stream);

/* Point-to-mode loss per instance (see gs_ctx_point_mode_loss) of a recorded
 * fit, with the labels the fit wrote (they must still hold them); loss
 * device double [B]. */
gs_status gs_point_mode_loss(const gs_result* r, const void* points, double* loss, void* stream);

/* Gradient of sum_b grad_loss[b] * L_b (see gs_ctx_point_mode_loss_backward). */
gs_status gs_point_mode_loss_backward(const gs_result* r, const void* points, const double* grad_loss,
                                      double* grad_points, void* stream);

/* Release a result without waiting on the host: the stream its fit ran on
 * (which must still exist) first waits for every other stream a result call
 * used, then the result's device memory goes back to its allocator for that
 * stream (a stream-ordered caching allocator hands it out again only to work
 * queued after it; memory from hipMalloc goes back with hipFree, which waits
 * for the device).  A result call on another stream than the fit's first
 * makes that stream wait for the fit's.  NULL is a no-op. */
void gs_result_free(gs_result* r);

/*
 * Plain fit for callers that cannot allocate (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): gs_fit without a
 * result object and without any device allocation.  The fit's scratch comes
 * from a fixed array of GS_NOALLOC_SCRATCH_BYTES of device memory that the
 * library holds on every GPU it runs on until the process ends; no hipMalloc,
 * hipHostMalloc, hipFree or caller allocator is called (host bookkeeping
 * uses ordinary heap memory).
 *   p            as for gs_fit; p->n <= GS_NOALLOC_MAX_POINTS (larger sets
 *                return GS_ERR_INVALID_ARG before any device work) and
 *                p->ckpt_every must be 0 (else GS_ERR_UNSUPPORTED).
 *   labels       device int32 [n], as for gs_fit.
 *   modes        device double [max_clusters][d]: fl(S / C) of clusters 0..K-1.
 *   counts       device int64 [max_clusters]: C of clusters 0..K-1.
 *   max_clusters rows the caller gave modes and counts (K <= n always); if
 *                K exceeds it the call returns GS_ERR_INVALID_ARG with *info
 *                filled and labels written, modes and counts untouched.
 *   info         host, the summary (as gs_result_info).
 * Results are bitwise those of gs_fit.  The stream is synchronised before
 * the call returns.  Every call on one GPU uses that GPU's one scratch array
 * and overwrites what the previous call left there: calls that overlap on
 * one GPU (other host threads, or other streams whose work has not ended)
 * race, and must be serialised by the caller.  The worst case (n points,
 * every point its own cell, d = 6, binary64) fits the array for every
 * n <= GS_NOALLOC_MAX_POINTS; a fit that would still exceed it returns
 * GS_ERR_ALLOC.
 */
#define GS_NOALLOC_MAX_POINTS 131072
#define GS_NOALLOC_SCRATCH_BYTES (64u << 20)
gs_status gs_fit_noalloc(const gs_problem* p, void* stream, int32_t* labels, double* modes, int64_t* counts,
                         int64_t max_clusters, gs_info* info);

/*
 * Contexts.  A gs_context holds the scratch of repeated fits and the last
 * fit's result; the gs_ctx_* calls below do what the calls above do, on a
 * context that the caller keeps (no allocation after the first fit of a
 * given size), plus the bandwidth sweep, tracking, launch configuration,
 * autotuning and timing.
 */
typedef struct gs_context gs_context;

/* ABI version (GS_ABI_VERSION). */
int32_t gs_abi_version(void);

/* Text of the last error on the calling thread (valid until its next call). */
const char* gs_last_error(void);

/* Create a context bound to the current HIP device.  *out receives it. */
gs_status gs_context_create(gs_context** out);

/* Destroy a context and free its device memory (NULL is a no-op).  The caller
 * must make sure no work of the context is still running. */
void gs_context_destroy(gs_context* ctx);

/*
 * Plain fit of one point set (Section 2.1, Algorithm 1).
 *   points  device, n rows of `ld` elements of `dtype`; row i holds x_i in its
 *           first d elements (ld >= d).  float32 is widened exactly.
 *   h       cell side (bandwidth), finite and > 0.
 *   max_iter maximum number of rounds (>= 0; 0 = binning only).
 *   labels  device int32 [n]: cluster id of every point (0..K-1).
 *   info    host, receives the result summary.
 * The cluster table stays in the context (gs_copy_modes, gs_copy_keys).
 */
gs_status gs_ctx_fit(gs_context* ctx, const void* points, gs_dtype dtype, int64_t n, int32_t d, int64_t ld,
                     double h, int32_t max_iter, int32_t* labels, gs_info* info, void* stream);

/*
 * Batched fit: B independent instances, concatenated, each with its own h,
 * in one pass of the pipeline (keys carry the instance as top digit; the
 * per-round tail runs one workgroup per instance in a single launch).
 * Results are bitwise those of B separate gs_ctx_fit calls.
 *   points  device [offsets[B]][ld] of dtype; instance b owns rows
 *           offsets[b] .. offsets[b+1]-1.
 *   offsets host int64 [B+1], offsets[0] = 0, non-decreasing.
 *   h       host double [B].
 *   labels  device int32 [offsets[B]]: per-instance cluster ids.
 *   info    host gs_info [B].
 */
gs_status gs_ctx_fit_batched(gs_context* ctx, const void* points, gs_dtype dtype, int32_t d, int64_t ld, int32_t B,
                             const int64_t* offsets, const double* h, int32_t max_iter, int32_t* labels,
                             gs_info* info, void* stream);

/*
 * Bandwidth sweep: the same point set fitted once per bandwidth hs[0..H-1]
 * (the tuning of Section 4.1 scans h over (0,1]), all H fits in one batched
 * pass in which bandwidth j is instance j.  The points are not copied: the
 * box of the coordinates is reduced once, every staged row is keyed for all
 * H bandwidths in one read, and the cell sums read each member from the
 * shared rows.  Results per bandwidth are bitwise those of gs_fit with that h.
 *   points  device, n rows of ld elements of dtype (as gs_fit).
 *   hs      host double [H], each finite and > 0.
 *   labels  device int32 [H][n]: the labels of bandwidth j at j * n.
 *   info    host gs_info [H].
 * H * n must stay below 2^31.  A context recording the trajectory
 * (gs_context_set_tape) returns GS_ERR_UNSUPPORTED.  The cluster tables stay
 * in the context as after gs_fit_batched (gs_copy_modes: bandwidth j's
 * clusters after those of bandwidths 0..j-1).
 */
gs_status gs_fit_hsweep(gs_context* ctx, const void* points, gs_dtype dtype, int64_t n, int32_t d, int64_t ld,
                        int32_t H, const double* hs, int32_t max_iter, int32_t* labels, gs_info* info, void* stream);

/*
 * Object tracking (Algorithm 2, Section 2.3) through a sequence of frames.
 *   frames  device [T][H][W][dc] of dtype: the colour features (1 <= dc <= 4)
 *           of pixel (px, py) (column, row) of frame t at
 *           ((t * H + py) * W + px) * dc.  H * W < 2^31.
 *   o0      host double [2]: the initial centre (x, y); l0 and w0 the initial
 *           window's extents along x and y (all > 0).
 * The window W(o, l, w) holds the pixels with |px - o_x| <= l/2 and
 * |py - o_y| <= w/2 (binary64).  Initialisation: GridShift with bandwidth h
 * (max_iter rounds, the context's update rule) on the colours of
 * W(o0, l0, w0) of frame 0 in raster order; the n_select largest clusters
 * (count descending, then cluster id) give the set B of colour cells
 * floor(fl(c / h)) of their pixels.  Every later frame repeats, at most
 * max_inner times: R = the pixels of the search window W(o, l/f, w/f) whose
 * colour cell is in B; an empty R multiplies l and w by 1.1; otherwise the
 * centre moves to the mean pixel position of R (exact integer sums, one
 * division), B becomes the colour cells of R, l becomes 0.99 l if R's extent
 * max px - min px is below l and 1.01 l otherwise (w likewise along y), and
 * the loop ends once the centre moved by less than eta (dx*dx + dy*dy <
 * eta*eta).  One workgroup runs the whole sequence in one launch.
 *   windows host double [T][4]: (o_x, o_y, l, w) after every frame (frame 0:
 *           the initial window).
 * The context's last fit becomes the initial clustering.  Errors:
 * GS_ERR_KEY_RANGE if a selected colour cell index is outside
 * [-32768, 32767); GS_ERR_UNSUPPORTED if B would hold more than 2048 cells
 * or dc is outside 1..4; GS_ERR_INVALID_ARG for bad sizes or parameters.
 * Pixels whose colour cells cannot be packed are never in R (B holds none).
 */
gs_status gs_track(gs_context* ctx, const void* frames, gs_dtype dtype, int32_t T, int32_t H, int32_t W, int32_t dc,
                   const double* o0, double l0, double w0, double f, double h, double eta, int32_t max_inner,
                   int32_t n_select, int32_t max_iter, double* windows, void* stream);

/*
 * Several objects tracked through the same frames at once: gs_track for
 * each of ntracks initial windows, bitwise the same per track.  The initial
 * windows are clustered in one batched pass and each track runs in its own
 * workgroup of one launch.
 *   o0      host double [ntracks][2]; l0, w0 host double [ntracks].
 *   windows host double [ntracks][T][4].
 * The context's last fit becomes the batched initial clustering.
 */
gs_status gs_track_batched(gs_context* ctx, const void* frames, gs_dtype dtype, int32_t T, int32_t H, int32_t W,
                           int32_t dc, int32_t ntracks, const double* o0, const double* l0, const double* w0, double f,
                           double h, double eta, int32_t max_inner, int32_t n_select, int32_t max_iter,
                           double* windows, void* stream);

/*
 * Copy the cluster table of the last fit, instances concatenated in order
 * (instance b's K_b clusters start at row sum_{b'<b} K_b').
 *   modes   device double [sum K][d]: fl(S / C)           (may be NULL)
 *   counts  device int64 [sum K]: C                       (may be NULL)
 *   sums    device double [sum K][d]: S                   (may be NULL)
 */
gs_status gs_copy_modes(gs_context* ctx, double* modes, int64_t* counts, double* sums, void* stream);

/* Integer cell keys floor(.) of the last fit's clusters: device int64 [sum K][d]. */
gs_status gs_copy_keys(gs_context* ctx, int64_t* keys, void* stream);

/*
 * Update rule of the shift of every round.
 *   GS_UPDATE_PARALLEL (default): Eq. 6, every cell moves to the mean over the
 *     round's table.
 *   GS_UPDATE_SEQUENTIAL: Eq. 5 (Section 2.2; Algorithm 1 overwrites S'(j) while
 *     it loops over the cells): the cells move one after another, and a cell
 *     that has moved contributes C_k * p_k (its count times its new centroid,
 *     fl(C_k * p_k) in binary64) instead of its sum S_k to the cells that move
 *     after it; the weights stay the counts of the round's table.  The visiting
 *     order is colour by colour: the colour of a cell has bit d-1-k equal to
 *     the parity of its integer coordinate k; colours ascend, and cells of one
 *     colour (never neighbours of each other) move together, so the order
 *     among them does not matter.  Relocation, merge and stopping are those of
 *     the parallel rule.
 * The rule applies to later fits of the context.  A fit with the sequential
 * rule while a trajectory is being recorded (gs_context_set_tape) returns
 * GS_ERR_UNSUPPORTED.  Other values are GS_ERR_INVALID_ARG.
 */
enum { GS_UPDATE_PARALLEL = 0, GS_UPDATE_SEQUENTIAL = 1 };
gs_status gs_context_set_update(gs_context* ctx, int32_t rule);
gs_status gs_context_get_update(const gs_context* ctx, int32_t* rule);

/*
 * Differentiable form.  With the discrete trajectory of a fit held fixed
 * (initial cells, and every round's neighbour sets, weights W and merge
 * groups), the modes are a linear function of the points (Eq. 1-4 with
 * constant keys, counts and groups), with the same weights for every
 * coordinate.  gs_context_set_tape(ctx, 1) makes later fits record that
 * trajectory in the context (device memory: the initial cells, and per round
 * the cell keys, counts, weights and merge maps); the calls below then act on
 * the context's last fit.
 * gs_context_set_tape(ctx, k) with k > 1 records the device-wide rounds (the
 * rounds run while some instance has more than 1024 cells, a few at most) the
 * same way, but of the remaining rounds keeps only checkpoints: the cell
 * table (keys, counts, sums) at the start of every k-th of them.  The backward
 * calls then recompute the per-round record one k-round segment at a time,
 * last segment first, from its checkpoint, bitwise as the fit ran it, so the
 * gradients are identical to those of a fully recorded fit.  0 records
 * nothing; k < 0 is GS_ERR_INVALID_ARG.  Reverse mode, in binary64 in a fixed
 * order:
 *   Sbar_c = grad_mode_c / C_c for the final cells;
 *   for every round, last first:  q_j = (C_j * Sbar_{g(j)}) / W_j  and
 *   Sbar_k = left fold, over the round's active cells j with Chebyshev key
 *   distance <= 1 from k, in ascending key, of q_j;
 *   grad_point_i = Sbar_{initial cell of i}.
 */
gs_status gs_context_set_tape(gs_context* ctx, int32_t ckpt_every);

/* grad_modes device double [sum K][d] (the concatenated cluster rows of
 * gs_copy_modes); grad_points device double [N][d], overwritten.  Returns
 * GS_ERR_STATE if the last fit was not recorded. */
gs_status gs_ctx_backward(gs_context* ctx, const double* grad_modes, double* grad_points, void* stream);

/*
 * Point-to-mode loss of every instance, L_b = sum over its points of
 * ||x_i - mode(label_i)||^2, summed as R over the points in ascending index of
 * the left fold over the coordinates.  points and labels are the arrays of
 * the recorded fit (same layout); loss device double [B].
 */
gs_status gs_ctx_point_mode_loss(gs_context* ctx, const void* points, const int32_t* labels, double* loss,
                                 void* stream);

/*
 * Gradient of sum_b grad_loss[b] * L_b with respect to the points, the
 * trajectory held fixed:  grad_i = gL * 2 (x_i - mode_c) + [J^T mubar]_i with
 * mubar_c = gL * (-2 (X_c - C_c mode_c)), X_c the sum of the points of
 * cluster c (R over its initial cells' sums in ascending cell order).
 * grad_loss device double [B]; grad_points device double [N][d], overwritten.
 */
gs_status gs_ctx_point_mode_loss_backward(gs_context* ctx, const void* points, const int32_t* labels,
                                          const double* grad_loss, double* grad_points, void* stream);

/*
 * Launch configuration of a context.  Every choice runs the same binary64
 * operations in the same order, so labels, counts, sums and modes never
 * depend on it; only the speed does.
 *   GS_CFG_MERGE_SMALL  1 (default): the merge of a round run while some
 *                       instance has more than 1024 cells, when the table
 *                       holds at most 8192 cells and keys fit 32 bits, is done
 *                       by one 1024-thread workgroup; 0: by device-wide
 *                       kernels (radix sort, scans, segmented sums).
 *   GS_CFG_TILE_CHUNKS  1..64 (default 4): chunks of staged point rows (24 KiB
 *                       of coordinates each) per workgroup of the point-level
 *                       binning kernels.
 *   GS_CFG_DENSE_TABLE  1 (default): the device-wide rounds find neighbour
 *                       cells through a table over the whole packed key range
 *                       (8 bytes per key, kept in the context) when that range
 *                       is at most 2^27 keys; 0: through an open-addressing
 *                       hash rebuilt every round.
 *   GS_CFG_SORT_DIGIT10 0 (default): the radix sorts use 8-bit digits; 1:
 *                       10-bit digits where that saves a pass (measured
 *                       slower per pass than the pass it saves on the
 *                       workloads here).
 *   GS_CFG_SORT_TILE    8192 (default) or 4096: keys per workgroup tile of a
 *                       radix-sort pass.
 * Unknown keys and out-of-range values are GS_ERR_INVALID_ARG.
 */
enum {
    GS_CFG_MERGE_SMALL = 0,
    GS_CFG_TILE_CHUNKS = 1,
    GS_CFG_DENSE_TABLE = 2,
    GS_CFG_SORT_DIGIT10 = 3,
    GS_CFG_SORT_TILE = 4
};
gs_status gs_context_set_config(gs_context* ctx, int32_t key, int32_t value);
gs_status gs_context_get_config(const gs_context* ctx, int32_t key, int32_t* value);

/*
 * Autotuner: fits the given input (the arguments of gs_fit_batched; B = 1 and
 * offsets {0, n} for one point set) once per candidate configuration
 * (GS_CFG_MERGE_SMALL in {1, 0} x GS_CFG_DENSE_TABLE in {1, 0} x
 * GS_CFG_TILE_CHUNKS in {1, 2, 4, 8} x GS_CFG_SORT_DIGIT10 in {0, 1} x
 * GS_CFG_SORT_TILE in {8192, 4096}: 64 candidates), one
 * warm-up run and `reps` timed runs each (host wall time of the whole call,
 * best of the reps), and keeps the fastest configuration in the context.
 * Every candidate's labels, cluster counts and cluster sums are compared bit
 * for bit with the first candidate's on the device; a difference is
 * GS_ERR_DEVICE (it would be a defect of the library).  The choice is kept
 * per shape (device, d, dtype, and B and the point count rounded down to
 * powers of two) for the rest of the process, and appended to the file the
 * environment variable GRIDSHIFT_TUNE_CACHE names, if set, which later
 * processes read: a shape met before takes its configuration without any
 * fit.  The labels of the timed fits go to a buffer the context owns; after
 * a tuning run the context's last result is that of the last timed fit
 * (identical for every configuration), after a cache hit it is unchanged.
 * On error the previous configuration is kept.
 */
gs_status gs_autotune(gs_context* ctx, const void* points, gs_dtype dtype, int32_t d, int64_t ld, int32_t B,
                      const int64_t* offsets, const double* h, int32_t max_iter, int32_t reps, void* stream);

/*
 * Kernel timing (instrumentation, not part of the method).  When enabled,
 * every kernel launch of later fits whose name starts with `prefix` is
 * bracketed by HIP events on the launch stream; the elapsed times, launch
 * counts and the algorithmic bytes each launch had to move (its inputs read
 * once and its outputs written once) accumulate per kernel name until
 * gs_profile_reset.  prefix NULL disables timing; "" times every kernel.
 */
gs_status gs_profile_enable(gs_context* ctx, const char* prefix);
gs_status gs_profile_reset(gs_context* ctx);
/* Number of kernel names with accumulated timings (launches not yet
 * accumulated are waited for and added first). */
int32_t gs_profile_count(const gs_context* ctx);
/* Entry i: *name stays valid until gs_profile_reset / gs_context_destroy. */
gs_status gs_profile_entry(const gs_context* ctx, int32_t i, const char** name, double* total_ms, int64_t* launches,
                           double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* GRIDSHIFT_H */
