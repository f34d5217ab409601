// Host-side definitions shared by the translation units of the C ABI: the
// layout handle, its workspace views and small helpers. Not part of the
// public ABI (see include/tfdp.h).
#pragma once

#include <cmath>
#include <string>
#include <vector>

#include "tfdp.h"
#include "tfdp_internal.h"

namespace tfdp {

// Thread-local text returned by tfdp_last_error().
void set_msg(const std::string& s);
const char* last_msg();
// TFDP_OK, or TFDP_ERR_HIP with the HIP error text as the message.
tfdp_status check_hip(hipError_t e, const char* what);

inline int k_workspace(const tfdp_params* p) { return (p->k_mode == 1 || p->k_mode == 2) ? p->k_mode : 3; }

// FFT length: the smallest 2^a >= max(64, 2M), or 3 * 2^(a-2) when that is
// still >= 2M and one of the radix-3 lengths 384, 768, 1536 (any L >= 2M - 1
// gives the same linear convolution; the circulant is zero in the gap).
inline Geom make_geom(int n_int, int k) {
    Geom g;
    g.k = k;
    g.m = n_int * k;
    int L = 64;
    while (L < 2 * g.m) L <<= 1;
    const int l3 = 3 * (L / 4);
    if (l3 >= 2 * g.m && (l3 == 384 || l3 == 768 || l3 == 1536)) L = l3;
    g.L = L;
    g.H = L / 2 + 1;
    g.cw = fft_task_ffts(L);  // transforms per FFT task
    return g;
}

// Bump allocator over the caller's workspace (base == nullptr: size only).
struct Carve {
    char* base;
    size_t off;
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

struct Layout {
    Bufs b;         // tw filled per k
    float2* pos_alt;
    float2* tw[4];  // per k
    int nslices;
    int* slice_rp;      // [nslices][n + 1] (nslices > 1)
    int* slice_col;     // [nnz] packed entries: column | (row index in its wave group) << 26
    float2* fpart;      // [n] attraction sums of the earlier slices, or of the overlapped pass
    int2* sched;        // [4 * edge_blocks_bound] schedules of all slices
    EdgeSlice slice[kMaxSlices];
};

}  // namespace tfdp

struct tfdp_layout {
    int n;
    int64_t nnz;
    const int* row_ptr;
    const int* col_idx;
    float* pos;
    void* ws;
    size_t ws_bytes;
    tfdp_params p;
    int k_ws;
    int t;
    tfdp::Layout lay;
    // captured groups of iterations: [group size: 2 or kGraphIters][k]
    // [parity of t at the start][orientation]
    bool graphs;
    hipGraphExec_t gexec[2][4][2][2];
    // profiling
    bool prof;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used;
    std::vector<int> ev_phase;  // phase of each recorded pair
    hipStream_t ev_stream;
    // bumped by every change a batch that holds the handle must pick up
    unsigned int version;
    long long slice_nodes;  // column-slice width fixed at init
    bool tw_pending;        // twiddle tables to (re)compute before the next launch
    const float* rep_w;     // local-refinement weights (caller's device arrays) or null
    const float* att_w;
    bool auto_grid;         // n_int chosen from the box every kAutoGridChunk iterations
    // edge pass: -1 automatic, 0 fused (one pass after the grid passes), 1
    // overlapped (attraction on a second stream beside the grid passes, then
    // a node pass)
    int overlap_mode;
    int device;             // device current at init (the second stream is created on it)
    int attract_blocks[2];  // blocks of the overlapped attraction pass at k = 1 and at k = 2, 3
    hipStream_t side;       // second stream of the overlapped attraction pass (created on first use)
    hipEvent_t ev_fork, ev_join, ev_node;  // start of a run, grid passes done, node pass done
    unsigned long long uid; // unique per handle of the process (batch compositions are keyed by it)
};

namespace tfdp {

// Twiddle tables of every k of the workspace, on stream s, if the grid
// changed since they were last computed.
void enqueue_twiddles(tfdp_layout* h, hipStream_t s);

inline ModelArgs model_args(const tfdp_layout* h) {
    ModelArgs a;
    a.alpha = h->p.alpha;
    a.beta = h->p.beta;
    a.gamma = h->p.gamma;
    a.rep_weight = h->p.rep_weight;
    a.t0 = h->p.t0 > 0.f ? h->p.t0 : std::fmax(1.0f, (float)(std::sqrt((double)h->n) / 10.0));
    a.total_iters = h->p.total_iters;
    a.tau = h->p.tau;
    a.rep_w = h->rep_w;
    a.att_w = h->att_w;
    return a;
}

inline Bufs bufs_for(const tfdp_layout* h, int k, bool batched = false) {
    Bufs b = h->lay.b;
    b.tw = h->lay.tw[k];
    // sparse rows grouped per spreading block in batched launches only:
    // there the blocks of many graphs fill the chip, while the plain pass of
    // one graph needs a block per row for its parallelism (the grouping does
    // not change the exact sums)
    b.rgroup = batched ? spread_row_group(k, b.n_int, b.n) : 1;
    // grouped rows leave about max_chunks / rgroup work chunks: launch that
    // many blocks (each loops over the chunks it is given) rather than one
    // block per possible chunk
    b.chunk_blocks = (b.max_chunks + b.rgroup - 1) / b.rgroup;
    return b;
}

// k of iteration t: k_mode, or the schedule of Sec. 3.4 ("Choices of k").
inline int k_at(const tfdp_params& p, int t) {
    if (p.k_mode >= 0) return p.k_mode;
    const int T = p.total_iters;
    if (t < (9 * T) / 10) return 1;
    if (t < (19 * T) / 20) return 2;
    return 3;
}

}  // namespace tfdp
