/*
 * tfdp.h - C ABI of the MI355X t-FDP layout library (libtfdp.so).
 *
 * t-FDP ("Force-directed graph layouts revisited: a new force based on the
 * t-Distribution", Zhong et al., arXiv 2303.03964) lays out an undirected
 * graph in 2D. One iteration computes, for every node i,
 *
 *   repulsion  F^r_i = sum_j (x_i - x_j) / (1 + |x_i - x_j|^2)^gamma
 *              (Sec. 3.3 Eq.5, rewritten as kernel sums in Sec. 3.4 Eq.11-15),
 *   attraction F^a_i = -alpha sum_{j in N(i)} (1 + beta/(1 + |x_i - x_j|^2)) (x_i - x_j)
 *              (Sec. 3.3 Eq.6, weighted as in Eq.7),
 *   motion     D_i = rep_weight * F^r_i + F^a_i  (Eq.7; rep_weight = 1 is the
 *              paper's model, other values give the global refinement of Sec. 5),
 *
 * then moves every node. The repulsion is evaluated either exactly (O(n^2),
 * the "exact method" of Sec. 3.4) or by the interpolation-based FFT scheme of
 * Sec. 3.4: spread the nodes onto an equispaced grid of N_int x N_int
 * intervals with k x k Lagrange nodes each, convolve with the kernel by FFT,
 * interpolate back.
 *
 * Readings of points the paper leaves open (the same in the library and in
 * its FP64 test oracle):
 *  - box: square of side W = max(x range, y range) centred on the mid-range
 *    of each axis (W = 1 if all nodes coincide); interval index and
 *    in-interval coordinate computed in float64;
 *  - interpolation nodes at (j + 1/2)/k of each interval, j = 0..k-1;
 *  - update: x_i += D_i * min(1, T_t / |D_i|), T_t = t0 * (1 - t / T)
 *    (the paper gives no rule; Sec. 3.1 only says the force moves the node);
 *  - k schedule (Sec. 3.4, "Choices of k"): k = 1 for t < floor(0.9 T),
 *    k = 2 for t < floor(0.95 T), k = 3 afterwards.
 *
 * Memory and ownership. Every pointer named d_* is device memory on the
 * current HIP device. The caller owns the CSR arrays, the positions, the
 * force outputs and the workspace; the library never allocates or frees
 * device memory and keeps the pointers given to tfdp_layout_init, so they must
 * outlive the handle. Positions are float32 [n][2] interleaved (x0 y0 x1 y1 ..).
 * The CSR is symmetric: every undirected edge {u, v} appears as u->v and
 * v->u, row_ptr int32[n+1], col_idx int32[nnz], no self-loops or duplicates.
 *
 * Streams. Work is enqueued on the caller's stream and is asynchronous;
 * functions that must read device results (init, sync_status, phase_times)
 * synchronise that stream.
 *
 * Errors. Functions return a tfdp_status; no exception crosses the ABI and
 * the library never aborts. tfdp_last_error() returns a thread-local message
 * for the last failure (or a warning after TFDP_OK). Asynchronous failures
 * (a HIP launch error, a non-finite position) are reported by the next call
 * that synchronises: tfdp_layout_sync_status.
 */
#ifndef TFDP_H
#define TFDP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tfdp_status {
    TFDP_OK = 0,
    TFDP_ERR_INVALID_ARG = -1,  /* bad parameter, pointer, size or CSR */
    TFDP_ERR_WORKSPACE = -2,    /* workspace missing or smaller than tfdp_workspace_size */
    TFDP_ERR_HIP = -3,          /* a HIP runtime call or kernel launch failed */
    TFDP_ERR_NONFINITE = -4,    /* a position became NaN or infinite */
    TFDP_ERR_UNSUPPORTED = -5   /* valid request outside the built limits (e.g. grid too large) */
} tfdp_status;

/* Model and schedule parameters. */
typedef struct tfdp_params {
    float alpha;         /* attraction weight (Eq.7), default 0.1 (Sec. 3.3) */
    float beta;          /* weight of the attractive t-force (Eq.6), default 8 */
    float gamma;         /* repulsive t-force exponent (Eq.5), default 2; must be > 1 (Eq.10) */
    float rep_weight;    /* multiplier of the repulsion, default 1 (Sec. 5, global refinement) */
    int32_t n_int;       /* intervals per box side N_int (Sec. 3.4), 1..1024; 0: automatic, chosen
                            every 10 iterations (at counters that are multiples of 10) as
                            max(50, ceil(W)) for the box side W of the current layout, the rule the
                            paper cites for t-SNE (Sec. 3.4, "Choices of k"), capped at 1024 / k_max;
                            the workspace is then sized for the cap */
    int32_t k_mode;      /* 0: exact O(n^2) repulsion; 1, 2, 3: fixed k; -1: k schedule.
                            The exact method takes each unordered pair once from 4096
                            nodes on (sums in 64-bit fixed point, order-independent);
                            below, one kernel sums every row over all nodes. */
    int32_t total_iters; /* T of the k schedule and the cooling, >= 1 */
    float t0;            /* initial step cap; <= 0 selects max(1, sqrt(n)/10) */
    float tau;           /* length scale of both t-forces, > 0, default 1: (1 + tau d^2) in
                            place of (1 + d^2) (the generalised t-force of Sec. 3.2, Eq.3; the
                            paper's model has tau = 1) */
} tfdp_params;

typedef struct tfdp_layout tfdp_layout; /* opaque handle (host memory) */

/* Fill *p with the defaults: alpha 0.1, beta 8, gamma 2 (Sec. 3.3),
 * rep_weight 1, n_int 64, k_mode -1, total_iters 300, t0 0 (automatic),
 * tau 1. */
void tfdp_params_default(tfdp_params* p);

/* Host-only check of parameters and sizes; touches no device.
 * TFDP_ERR_INVALID_ARG: p NULL, n < 1, nnz < 0, gamma <= 1 (Eq.10), alpha,
 * beta or rep_weight negative or not finite, n_int < 0, k_mode outside
 * {-1,0,1,2,3}, total_iters < 1, t0 not finite, tau not finite or <= 0.
 * TFDP_ERR_UNSUPPORTED: N_int * k_max > 1024 (FFT length above 2048), where
 * k_max is k_mode for k_mode 1 or 2 and 3 otherwise.
 * Returns TFDP_OK with a warning in tfdp_last_error() when
 * alpha (1 + beta) >= 1, which breaks the contact condition of Eq.9 (the
 * paper's guideline, not a hard limit). */
tfdp_status tfdp_params_validate(const tfdp_params* p, int32_t n, int64_t nnz);

/* Bytes of device workspace needed by a handle with these sizes and
 * parameters (host-only; 0 if tfdp_params_validate fails). The workspace
 * holds the second position buffer, the binning arrays, the grids, spectra
 * and twiddle tables, and a few counters. */
size_t tfdp_workspace_size(int32_t n, int64_t nnz, const tfdp_params* p);

/* Create a layout handle.
 *   out        receives the handle (set to NULL on failure)
 *   n, nnz     node count and number of CSR entries (2 x edges)
 *   d_row_ptr  int32[n+1], d_col_idx int32[nnz]: symmetric CSR (device)
 *   d_pos      float32[n][2] positions (device); tfdp_layout_step updates
 *              it in place
 *   d_ws       device workspace of ws_bytes >= tfdp_workspace_size(...),
 *              256-byte aligned; owned by the caller, used exclusively by
 *              this handle
 *   p          parameters (copied)
 *   stream     stream for the set-up work; init synchronises it
 * Validates p (as tfdp_params_validate), checks on the device that row_ptr
 * is monotone with row_ptr[0] = 0 and row_ptr[n] = nnz and that every column
 * index is in [0, n) and not i itself (TFDP_ERR_INVALID_ARG otherwise),
 * builds the FFT twiddle tables and sets the iteration counter to 0. */
tfdp_status tfdp_layout_init(tfdp_layout** out, int32_t n, int64_t nnz,
                             const int32_t* d_row_ptr, const int32_t* d_col_idx,
                             float* d_pos, void* d_ws, size_t ws_bytes,
                             const tfdp_params* p, hipStream_t stream);

/* Advance the layout by `iters` iterations from the handle's counter t
 * (asynchronous). Each iteration picks k from k_mode (or from the schedule
 * with T = total_iters), evaluates the forces at the current positions and
 * moves every node with the capped step T_t = t0 (1 - t/T); the counter then
 * increases by one. Iterations past T keep going with k = 3 and a negative
 * cap clamped to 0, i.e. no motion. The final positions are in d_pos when
 * the stream reaches the end of the enqueued work. iters >= 0. */
tfdp_status tfdp_layout_step(tfdp_layout* h, int32_t iters, hipStream_t stream);

/* Evaluate the forces at d_pos_in (float32 [n][2], device) without moving
 * anything and without changing the handle's state (asynchronous).
 *   k = 0      exact repulsion (Sec. 3.4, "exact method")
 *   k = 1,2,3  interpolated repulsion with k x k nodes per interval
 * d_f_rep receives F^r, d_f_att F^a and d_f_tot D = rep_weight F^r + F^a,
 * each float32 [n][2]; any of them may be NULL. d_pos_in may be the
 * handle's own d_pos. TFDP_ERR_WORKSPACE if k exceeds the k the workspace
 * was sized for. */
tfdp_status tfdp_layout_forces(tfdp_layout* h, const float* d_pos_in, int32_t k,
                               float* d_f_rep, float* d_f_att, float* d_f_tot,
                               hipStream_t stream);

/* Replace the parameters (re-tune, Sec. 5 "Global Refinement"). alpha, beta,
 * gamma, rep_weight, total_iters, t0 may change freely. n_int and k_mode may
 * change when the handle's workspace (ws_bytes at init) holds the new grid:
 * size it with tfdp_workspace_size for the largest grid planned
 * (TFDP_ERR_WORKSPACE otherwise); the grid arrays are then re-laid inside the
 * workspace, so work of the handle enqueued earlier must be ordered before
 * later work (one stream, or synchronised). Positions and the counter are
 * kept. Takes effect for work enqueued afterwards. */
tfdp_status tfdp_layout_set_params(tfdp_layout* h, const tfdp_params* p);

/* The handle's current parameters (with the automatic grid: the grid in
 * use as n_int). */
tfdp_status tfdp_layout_get_params(const tfdp_layout* h, tfdp_params* out);

/* Local refinement (Sec. 5): per-node weights that make chosen nodes pull
 * their neighbours closer and push the others away.
 *   d_rep_w  float32[n] (device) or NULL: node i's repulsion enters its
 *            motion as rep_weight * d_rep_w[i] * F^r_i
 *   d_att_w  float32[n] (device) or NULL: the attraction term of edge (i, j)
 *            is scaled by (d_att_w[i] + d_att_w[j]) / 2 (the same for both
 *            ends, so the attraction stays symmetric)
 * NULL restores weight 1. The arrays stay owned by the caller and are read
 * by every later step and forces call until replaced; values should be
 * finite and >= 0 (not checked). tfdp_layout_forces reports F^r unweighted,
 * F^a and D weighted. Takes effect for work enqueued afterwards. */
tfdp_status tfdp_layout_set_node_weights(tfdp_layout* h, const float* d_rep_w, const float* d_att_w);

/* Read / set the iteration counter t (checkpoint and resume: positions plus t
 * are the whole state). */
tfdp_status tfdp_layout_get_iter(const tfdp_layout* h, int32_t* t);
tfdp_status tfdp_layout_set_iter(tfdp_layout* h, int32_t t);

/* Synchronise `stream` and report asynchronous failures: TFDP_ERR_HIP for a
 * failed kernel, TFDP_ERR_NONFINITE if any position computed since the last
 * call was NaN or infinite (the flag is then cleared). */
tfdp_status tfdp_layout_sync_status(tfdp_layout* h, hipStream_t stream);

/* Destroy the handle (host memory only; the caller's buffers stay). */
void tfdp_layout_destroy(tfdp_layout* h);

/* Thread-local text for the last failure or warning ("" if none). */
const char* tfdp_last_error(void);

/* How the edge pass (attraction, repulsion gather and move) is scheduled:
 *   1   overlapped: the attraction sums run on a second stream of the
 *       library (created on first use, default priority) concurrently with
 *       the binning and FFT passes, as a launch of a fixed number of blocks
 *       that leaves room on every CU; a node pass then gathers the repulsion
 *       and moves every node once both are done;
 *   0   fused: one edge pass after the grid passes;
 *  -1   automatic (default): overlapped from 4,194,304 CSR entries on
 *       (below, the node pass and the waits between the streams cost more
 *       than the attraction pass hides).
 * The two schedules compute bit-identical results. The caller's stream still
 * orders everything: the second stream waits for the caller's stream at the
 * start of each iteration and the caller's stream waits for it before the
 * node pass. TFDP_ERR_UNSUPPORTED for mode 1 on a handle whose edge pass is
 * split into column slices. */
tfdp_status tfdp_layout_set_overlap(tfdp_layout* h, int32_t mode);

/* Launch groups of eight (else two) iterations of one k as captured HIP
 * graphs (default on; a graph per group size, k, parity and buffer
 * orientation is captured on first use on the step's stream and dropped by
 * tfdp_layout_set_params). Off: every kernel is launched directly.
 * Profiling (below) always launches directly. */
tfdp_status tfdp_layout_set_graphs(tfdp_layout* h, int32_t enable);

/* Per-phase timing with HIP events recorded on the launch stream around the
 * kernels of each phase. Enabling costs two event records per phase launch. */
tfdp_status tfdp_layout_set_profiling(tfdp_layout* h, int32_t enable);
/* Number of phases and their names ("bin_count", "gather_update", ...). */
int32_t tfdp_phase_count(void);
const char* tfdp_phase_name(int32_t phase);
/* Synchronise the stream of the recorded events and write, per phase, the
 * summed milliseconds and the number of timed launches since profiling was
 * enabled (arrays of at least tfdp_phase_count() entries); then reset. */
tfdp_status tfdp_layout_phase_times(tfdp_layout* h, double* total_ms, int64_t* launches,
                                    int32_t nphases);

/* ---- Layout quality (Sec. 4, "Metrics") ----
 *
 * Stress error estimated from a sample of source nodes:
 *   SE = mean over pairs (s, v), v != s, v reachable from s, of
 *        (c ||x_s - x_v|| / D(s, v) - 1)^2
 * with D the hop distance and c = sum(||x_s - x_v|| / D) / sum((||x_s - x_v|| / D)^2)
 * the optimal uniform scale of the layout. Hop distances come from one
 * multi-source BFS on the device, stored as 16-bit integers: graphs whose
 * BFS from the sources still finds new nodes at level 65534 are refused with
 * TFDP_ERR_UNSUPPORTED (every connected graph of diameter below 65534 is
 * measured exactly; nodes in other components count as unreachable).
 *   n, nnz, d_row_ptr, d_col_idx  symmetric CSR (device, as for tfdp_layout_init;
 *               checked on the device first: TFDP_ERR_INVALID_ARG if invalid)
 *   d_pos       float32[n][2] positions (device)
 *   d_sources   int32[nsrc] source nodes in [0, n) (device), 1 <= nsrc <= 64;
 *               checked on the device: TFDP_ERR_INVALID_ARG otherwise
 *   d_work      device scratch of work_bytes >= tfdp_stress_workspace_size(n, nsrc),
 *               256-byte aligned (TFDP_ERR_WORKSPACE otherwise)
 *   se          result (host); NaN when no pair is reachable
 *   levels      BFS levels run (host, may be NULL)
 * Synchronises `stream`. */
size_t tfdp_stress_workspace_size(int32_t n, int32_t nsrc);
tfdp_status tfdp_stress_sampled(int32_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col_idx,
                                const float* d_pos, const int32_t* d_sources, int32_t nsrc, void* d_work,
                                size_t work_bytes, double* se, int32_t* levels, hipStream_t stream);
/* Stress error as above plus neighbourhood preservation over the same
 * sources (Sec. 4, "Metrics"): for r = 1, 2 and each source s with a
 * non-empty graph ring N_G(s, r) = {v : 1 <= D(s, v) <= r} of k_s nodes, the
 * Jaccard index of that ring and the k_s nearest layout neighbours of s
 * (s excluded; equal distances, compared as float64 squared distances, go
 * to the lower node index); NP_r = the mean of those indices. The k_s-th
 * nearest node is found by an exact radix select on the device.
 *   np          double[2] result (host): NP_1, NP_2; NaN where no source
 *               has a non-empty ring
 * Other arguments, workspace size and errors as for tfdp_stress_sampled. */
tfdp_status tfdp_quality_sampled(int32_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col_idx,
                                 const float* d_pos, const int32_t* d_sources, int32_t nsrc, void* d_work,
                                 size_t work_bytes, double* se, double* np, int32_t* levels, hipStream_t stream);

/* tfdp_quality_sampled without a workspace, for callers that cannot allocate
 * device memory (code that must not call hipMalloc: tight serving loops,
 * harnesses that forbid allocation). The call makes no device allocation
 * (no hipMalloc or hipFree) and, on success, no host heap allocation: the
 * metric's scratch is a fixed 64 MiB array of the library, one copy per GPU,
 * resident from the first call on that GPU until the process ends. Limit: tfdp_stress_workspace_size(n, nsrc) <= 64 MiB
 * (about n * (24 + 2 nsrc) bytes; e.g. n <= 400,000 with 64 sources),
 * TFDP_ERR_UNSUPPORTED beyond it, checked before any device work.
 * The stream must belong to the current device. Every call on one GPU uses
 * that GPU's one array: calls from the threads of this process are
 * serialised by the library (each returns only after its stream has finished
 * the metric's work), but work that overlaps on one GPU by other means would
 * race on it; after a TFDP_ERR_HIP return the array may still be in use by
 * the failed stream. Arguments, results and the other errors as for
 * tfdp_quality_sampled (se and np must be set). Synchronises `stream`. */
tfdp_status tfdp_quality_sampled_noalloc(int32_t n, int64_t nnz, const int32_t* d_row_ptr,
                                         const int32_t* d_col_idx, const float* d_pos, const int32_t* d_sources,
                                         int32_t nsrc, double* se, double* np, int32_t* levels, hipStream_t stream);

/* ---- Batched stepping ----
 *
 * A batch steps many layout handles (graphs of any sizes, each with its own
 * parameters, grid and iteration counter) together: every phase of an
 * iteration is one launch per class of graphs that share the kernel shape
 * (k, FFT length, spreading block), whose blocks each work on one graph.
 * Each member's positions and counter after tfdp_batch_step(b, iters) are
 * bit-identical to those after tfdp_layout_step(h, iters) on that handle
 * alone: the blocks of a batched launch run the same kernel code on the same
 * data partition.
 *
 * The batch references the handles (it does not own them): remove a handle
 * before destroying it. A handle may be in at most one batch at a time and
 * may still be used with the plain calls between batch calls (the batch
 * picks up new parameters and counters). All calls on one batch must be
 * ordered on the device (one stream, or synchronised).
 *
 * Device memory: the batch's tables live in a caller workspace (the library
 * allocates no device memory): per member slot its kernel arguments and
 * counter, then an arena of block maps, one region per composition (the
 * members, their grids and the k of each). Compositions are kept for reuse;
 * when the arena is full it is reset after one synchronisation of the
 * stream. A composition needs at most about n/60 + nnz/200 + 4,300 map
 * entries per member (8 bytes each; the constant covers the largest grid).
 * While graphs are enabled (tfdp_batch_set_graphs), at its first step the
 * batch creates a second stream and two events on the device that was
 * current at tfdp_batch_create (no device memory): the grid passes and the
 * edge pass of the members of all but the FFT length with the most blocks,
 * and the one-launch exact kernel of the small exact members, run there,
 * between the binning and the edge pass of the other members in each
 * iteration; the call is still ordered on `stream` as a whole.
 * With graphs disabled every launch stays on `stream`. tfdp_batch_destroy
 * releases them.
 * Adding, removing or re-tuning members costs no synchronisation: the new
 * kernel arguments and counters are written by small kernels on the stream
 * at the next step. Groups of eight (else two) iterations of a composition
 * are captured as HIP graphs the second time the same group is needed. A
 * batch with a single member steps it by tfdp_layout_step (the same result,
 * with the kernel tiles of a single graph). */
typedef struct tfdp_batch tfdp_batch; /* opaque handle (host memory) */

/* Bytes of device workspace for a batch of `capacity` slots whose map arena
 * holds `map_entries` entries (at least 256 are reserved); 0 for
 * capacity < 1 or map_entries < 0. Host-only. */
size_t tfdp_batch_workspace_size(int32_t capacity, int64_t map_entries);
/* Empty batch for up to `capacity` members (>= 1) over the caller's device
 * workspace d_ws (256-byte aligned, ws_bytes >= tfdp_batch_workspace_size(
 * capacity, 0); the arena takes everything after the slot tables), owned by
 * the caller and used by this batch only until tfdp_batch_destroy. No device
 * work. TFDP_ERR_WORKSPACE for a missing, misaligned or short workspace. */
tfdp_status tfdp_batch_create(tfdp_batch** out, int32_t capacity, void* d_ws, size_t ws_bytes);
/* Add / remove a member (host bookkeeping; the device tables are rebuilt at
 * the next step). TFDP_ERR_INVALID_ARG: NULL, already a member (add) or not
 * a member (remove). TFDP_ERR_UNSUPPORTED: batch full, a handle whose edge
 * pass is split into column slices, or one with the automatic grid
 * (n_int = 0). */
tfdp_status tfdp_batch_add(tfdp_batch* b, tfdp_layout* h);
tfdp_status tfdp_batch_remove(tfdp_batch* b, tfdp_layout* h);
/* Number of members (0 for NULL). */
int32_t tfdp_batch_count(const tfdp_batch* b);
/* Advance every member by `iters` iterations (asynchronous, on `stream`),
 * each from its own counter t with its own k schedule and parameters
 * (k_mode 0 members run the exact method by the kernels of their plain
 * steps: the one-launch kernel below 4096 nodes, else the pair-symmetric
 * passes, whose map needs one entry per tile pair of 256 nodes, about
 * (n / 256)^2 / 2, beyond the bound given above).
 * TFDP_ERR_WORKSPACE if one composition needs more map entries than the
 * arena holds. Asynchronous failures are reported per member by
 * tfdp_layout_sync_status. */
tfdp_status tfdp_batch_step(tfdp_batch* b, int32_t iters, hipStream_t stream);
/* Tile schedule of the batched grid passes for one FFT length (64, 128, ...,
 * 2048): rows per block of the row FFT passes (2, 4 or 8) and column groups
 * per block of the column pass (1 or 2), selectable for lengths up to 768 (a
 * fixed tile above); 0 selects the default (8 rows up to length 256, 2
 * groups at 256, 4 rows and 1 group at 768). Tiles change only how the work is cut into blocks: every
 * tile gives bit-identical results. The project's autotuner times the
 * candidates on a batch and keeps the fastest per length. Changing a tile
 * synchronises `stream` (the batch's maps are rebuilt).
 * TFDP_ERR_INVALID_ARG for another length, TFDP_ERR_UNSUPPORTED for a tile
 * that is not available. */
tfdp_status tfdp_batch_set_tiles(tfdp_batch* b, int32_t fft_length, int32_t rows_per_block, int32_t column_groups,
                                 hipStream_t stream);
tfdp_status tfdp_batch_get_tiles(const tfdp_batch* b, int32_t fft_length, int32_t* rows_per_block,
                                 int32_t* column_groups);
/* Capture groups of iterations as HIP graphs (default on; the stream must
 * then not be the legacy default stream). Off: every kernel is launched
 * directly on the step's stream (no second stream either). */
tfdp_status tfdp_batch_set_graphs(tfdp_batch* b, int32_t enable);
/* Free the batch (host memory and captured graphs; the members and the
 * workspace stay valid). */
void tfdp_batch_destroy(tfdp_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* TFDP_H */
