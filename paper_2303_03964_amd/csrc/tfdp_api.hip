// Host side of the C ABI declared in include/tfdp.h: parameter validation,
// workspace layout, the per-iteration launch sequence and profiling.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "tfdp_handle.h"

using namespace tfdp;

namespace tfdp {

namespace {
thread_local std::string g_msg;
}

void set_msg(const std::string& s) { g_msg = s; }
const char* last_msg() { return g_msg.c_str(); }

tfdp_status check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return TFDP_OK;
    set_msg(std::string(what) + ": " + hipGetErrorString(e));
    return TFDP_ERR_HIP;
}

void enqueue_twiddles(tfdp_layout* h, hipStream_t s) {
    if (!h->tw_pending) return;
    for (int k = 1; k <= h->k_ws; ++k) launch_twiddles(h->lay.tw[k], make_geom(h->p.n_int, k).L, s);
    h->tw_pending = false;
}

int sym_min_nodes() {
    const char* e = std::getenv("TFDP_SYM_MIN_NODES");
    if (e) {
        const long long v = std::atoll(e);
        if (v >= 1 && v <= 0x7fffffffLL) return (int)v;
    }
    return kSymMinNodes;
}

}  // namespace tfdp

namespace {

enum Phase {
    PH_BOX = 0,
    PH_BIN_COUNT,
    PH_BIN_SCAN,
    PH_BIN_SCATTER,
    PH_SPREAD,
    PH_ROWFFT,
    PH_COLCONV,
    PH_ROWIFFT,
    PH_GATHER,
    PH_BRUTE,
    PH_ATTRACT,
    PH_NODE,
    PH_COUNT
};

const char* kPhaseNames[PH_COUNT] = {"box",     "bin_count", "bin_scan", "bin_scatter",   "spread",
                                     "rowfft",  "colconv",   "rowifft",  "gather_update", "brute",
                                     "attract", "node_update"};

// Overlapped edge pass: used automatically from kOverlapMinEntries CSR
// entries on. It pays where the attraction pass is long enough to hide the
// grid passes: 1M-node Chung-Lu graph (10M entries) 64.6 -> 58-59 ms per 500
// iterations; the 100k-node mesh (0.4M entries) went from 20.9 to 30.4 ms,
// the node pass and the two waits between the streams costing more than the
// short attraction pass hides. Blocks of the attraction pass per compute
// unit: 3 at k = 1 and 2 at k = 2, 3 (measured at 1M: 2, 3, 4, 6 per CU gave
// 116.9, 108.9, 113.2, 119.4 us per k = 1 iteration and 154, 161, 161, 168
// us at k = 2; the longer grid passes of k = 2, 3 need more room), or the
// value of TFDP_ATTRACT_BLOCKS_PER_CU (1..32, read at init) for every k.
constexpr long long kOverlapMinEntries = 1LL << 22;

int attract_blocks_per_cu(int k) {
    const char* e = std::getenv("TFDP_ATTRACT_BLOCKS_PER_CU");
    if (e) {
        const int v = std::atoi(e);
        if (v >= 1 && v <= 32) return v;
    }
    return k <= 1 ? 3 : 2;
}

// Column-slice width of the edge pass: kSliceNodesDefault, or the value of
// the environment variable TFDP_EDGE_SLICE_NODES (>= 1024) read at each call.
// One slice is fastest on MI355X up to millions of nodes (measured); the
// sliced pass bounds the neighbour working set of one launch.
long long slice_nodes() {
    const char* e = std::getenv("TFDP_EDGE_SLICE_NODES");
    if (e) {
        const long long v = std::atoll(e);
        if (v >= 1024) return v;
    }
    return kSliceNodesDefault;
}

// Workspace layout. The arrays that do not depend on the grid (state,
// positions, edge-pass entries and schedules) come first, so that a new
// N_int or k range (tfdp_layout_set_params) re-lays only the tail.
Layout carve(void* base, int n, long long nnz, const tfdp_params* p, long long sn, size_t* bytes) {
    Layout l;
    std::memset(&l, 0, sizeof(l));
    Carve c{static_cast<char*>(base), 0};
    const int kw = k_workspace(p);
    const Geom gw = make_geom(p->n_int, kw);
    l.b.n = n;
    l.b.n_int = p->n_int;
    l.b.nblk = (n + kBinChunk - 1) / kBinChunk;
    l.b.max_chunks = (n + kSpreadChunk - 1) / kSpreadChunk + p->n_int;
    l.b.st = c.take<DevState>(1);
    l.pos_alt = c.take<float2>((size_t)n);
    l.b.spos = c.take<float2>((size_t)n);
    l.nslices = edge_slices(n, sn);
    l.slice_col = c.take<int>((size_t)nnz);
    l.fpart = c.take<float2>((size_t)n);  // attraction sums (earlier slices, or the overlapped pass)
    l.b.sym_acc = c.take<unsigned long long>((size_t)2 * n);  // exact-method sums (kept zero between passes)
    if (l.nslices > 1) l.slice_rp = c.take<int>((size_t)l.nslices * ((size_t)n + 1));
    l.sched = c.take<int2>((size_t)4 * edge_blocks_bound(n, nnz, sn));
    l.b.blkcnt = c.take<int>((size_t)p->n_int * l.b.nblk);
    l.b.bucket_cnt = c.take<int>((size_t)p->n_int);
    l.b.bucket_start = c.take<int>((size_t)p->n_int + 1);
    l.b.chunk_start = c.take<int>((size_t)p->n_int + 1);
    l.b.wchunk = c.take<int4>((size_t)l.b.max_chunks + 1);
    l.b.spart = c.take<unsigned long long>((size_t)l.b.max_chunks * kw * gw.m * 3);
    l.b.qcol = c.take<float2>((size_t)3 * gw.H * gw.m);
    l.b.kcol = c.take<float2>((size_t)gw.H * (gw.L / 2 + 1));
    l.b.pcol = c.take<float2>((size_t)3 * gw.H * gw.m);
    l.b.pot = c.take<float4>((size_t)gw.m * gw.m);
    for (int k = 1; k <= kw; ++k) l.tw[k] = c.take<float2>((size_t)make_geom(p->n_int, k).L);
    *bytes = (c.off + 255) & ~(size_t)255;
    return l;
}

bool finite_f(float v) { return std::isfinite(v); }

// Automatic grid (n_int = 0): the largest grid the workspace holds for the
// k range of the parameters, and the parameters the workspace is sized for.
int auto_grid_cap(const tfdp_params* p) { return (kMaxL / 2) / k_workspace(p); }
tfdp_params sizing_params(const tfdp_params* p) {
    tfdp_params q = *p;
    if (q.n_int == 0) q.n_int = auto_grid_cap(p);
    return q;
}

// Edge-pass schedule: rows with more than kGroupEdges entries get a block
// each (slot 0 = {row, -1}); the other rows are cut, in order, into wave
// groups of at most kGroupRows rows and kGroupEdges entries, four groups per
// block (slot = {first row, rows}; {0, 0} = idle wave). Heavy blocks first.
// local[r] receives the row's index inside its wave group (0 for heavy rows).
std::vector<int2> build_edge_schedule(const std::vector<int>& rp, int n, std::vector<int>& local) {
    std::vector<int2> heavy, groups;
    local.assign((size_t)n, 0);
    int r = 0;
    while (r < n) {
        const int d = rp[r + 1] - rp[r];
        if (d > kGroupEdges) {
            heavy.push_back(make_int2(r, -1));
            ++r;
            continue;
        }
        const int r0 = r;
        int edges = 0, cnt = 0;
        while (r < n && cnt < kGroupRows) {
            const int dd = rp[r + 1] - rp[r];
            if (dd > kGroupEdges || edges + dd > kGroupEdges) break;
            edges += dd;
            local[r] = cnt;
            ++cnt;
            ++r;
        }
        groups.push_back(make_int2(r0, cnt));
    }
    std::vector<int2> out;
    out.reserve(4 * (heavy.size() + (groups.size() + 3) / 4));
    for (const int2& hrow : heavy) {
        out.push_back(hrow);
        for (int k = 0; k < 3; ++k) out.push_back(make_int2(0, 0));
    }
    for (size_t gi = 0; gi < groups.size(); gi += 4)
        for (size_t k = 0; k < 4; ++k) out.push_back(gi + k < groups.size() ? groups[gi + k] : make_int2(0, 0));
    return out;
}

// Event bracket around the launches of one phase when profiling.
struct PhaseTimer {
    tfdp_layout* h;
    int phase;
    hipStream_t s;
    PhaseTimer(tfdp_layout* h_, int ph, hipStream_t s_) : h(h_), phase(ph), s(s_) {
        if (h->prof) record();
    }
    ~PhaseTimer() {
        if (h->prof) {
            record();
            h->ev_phase.push_back(phase);
        }
    }
    void record() {
        if (h->ev_used == h->ev_pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) {
                h->prof = false;
                return;
            }
            h->ev_pool.push_back(e);
        }
        (void)hipEventRecord(h->ev_pool[h->ev_used++], s);
        h->ev_stream = s;
    }
};


// One evaluation of the interpolated repulsion up to the grid potentials;
// the box comes from extremes slot set `set`, set ^ 1 is reset for the
// update that follows.
// Exact method at pos (k = 0): the one-launch kernel for small graphs, the
// pair-symmetric passes from sym_min_nodes() nodes on.
void enqueue_exact(tfdp_layout* h, const float2* pos, float2* pos_out, const ModelArgs& a, float2* fr, float2* fa,
                   float2* ft, hipStream_t s) {
    if (use_sym(h->n))
        launch_sym(pos, pos_out, h->row_ptr, h->col_idx, h->n, h->lay.b.sym_acc, h->lay.b.st, a, h->t, fr, fa, ft, s);
    else
        launch_brute(pos, pos_out, h->row_ptr, h->col_idx, h->n, h->lay.b.st, a, h->t, fr, fa, ft, s);
}

void enqueue_grid(tfdp_layout* h, const float2* pos, const Bufs& b, const Geom& g, int set, hipStream_t s) {
    { PhaseTimer pt(h, PH_BIN_COUNT, s); launch_bin_count(pos, b, set, s); }
    { PhaseTimer pt(h, PH_BIN_SCAN, s); launch_bin_scan(b, set ^ 1, s); }
    { PhaseTimer pt(h, PH_BIN_SCATTER, s); launch_bin_scatter(pos, b, s); }
    { PhaseTimer pt(h, PH_SPREAD, s); launch_spread(b, g, h->p.gamma, h->p.tau, s); }
    { PhaseTimer pt(h, PH_ROWFFT, s); launch_rowfft(b, g, s); }
    { PhaseTimer pt(h, PH_COLCONV, s); launch_colconv(b, g, s); }
    { PhaseTimer pt(h, PH_ROWIFFT, s); launch_rowifft(b, g, s); }
}

// Extremes of `pos` into slot set `set` (both sets reset first).
void enqueue_box(tfdp_layout* h, const float2* pos, int set, hipStream_t s) {
    PhaseTimer pt(h, PH_BOX, s);
    launch_box_begin(h->lay.b.st, h->t, s);
    launch_box_reduce(pos, h->n, h->lay.b.st, set, s);
}

// Column slices of the edge pass: for slice s (columns [s W, (s+1) W),
// W = ceil(n / nslices)) a CSR of all rows holding each row's entries of
// that column range in their original order, and its schedule. Entries are
// stored packed, column | (row index inside its wave group) << 26, so that a
// lane knows its row without searching. With one slice the caller's row_ptr
// is used as is. Built on the host from copies of the caller's CSR (init
// only).
tfdp_status build_slices(tfdp_layout* h, hipStream_t stream) {
    const int n = h->n;
    const long long nnz = h->nnz;
    Layout& l = h->lay;
    // copies ordered on the caller's stream
    std::vector<int> rp((size_t)n + 1);
    tfdp_status st = check_hip(hipMemcpyAsync(rp.data(), h->row_ptr, rp.size() * sizeof(int),
                                              hipMemcpyDeviceToHost, stream), "hipMemcpyAsync");
    if (st != TFDP_OK) return st;
    std::vector<int> ci((size_t)nnz);
    if (nnz > 0)
        st = check_hip(hipMemcpyAsync(ci.data(), h->col_idx, ci.size() * sizeof(int), hipMemcpyDeviceToHost,
                                      stream), "hipMemcpyAsync");
    if (st == TFDP_OK) st = check_hip(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (st != TFDP_OK) return st;
    const int S = l.nslices;
    const long long W = ((long long)n + S - 1) / S;
    std::vector<int> srp((size_t)S * ((size_t)n + 1), 0);
    for (int i = 0; i < n; ++i)
        for (int e = rp[i]; e < rp[i + 1]; ++e) srp[(size_t)(ci[e] / W) * (n + 1) + i + 1] += 1;
    std::vector<long long> col_off(S + 1, 0);
    for (int s = 0; s < S; ++s) {
        int* r = srp.data() + (size_t)s * (n + 1);
        for (int i = 0; i < n; ++i) r[i + 1] += r[i];
        col_off[s + 1] = col_off[s] + r[n];
    }
    std::vector<int2> all_sched;
    std::vector<int> scol((size_t)nnz);
    std::vector<int> local;
    for (int s = 0; s < S; ++s) {
        std::vector<int> r(srp.begin() + (size_t)s * (n + 1), srp.begin() + (size_t)(s + 1) * (n + 1));
        std::vector<int2> sch = build_edge_schedule(r, n, local);
        int* out = scol.data() + col_off[s];
        for (int i = 0; i < n; ++i) {
            int f = r[i];
            for (int e = rp[i]; e < rp[i + 1]; ++e)
                if (ci[e] / W == s) out[f++] = ci[e] | (local[i] << 26);
        }
        l.slice[s].rp = S == 1 ? h->row_ptr : l.slice_rp + (size_t)s * (n + 1);
        l.slice[s].col = l.slice_col + col_off[s];
        l.slice[s].sched = l.sched + all_sched.size();
        l.slice[s].blocks = (int)(sch.size() / 4);
        all_sched.insert(all_sched.end(), sch.begin(), sch.end());
    }
    if ((long long)all_sched.size() > 4 * edge_blocks_bound(n, nnz, slice_nodes())) {
        set_msg("internal: edge schedule exceeds its bound");
        return TFDP_ERR_WORKSPACE;
    }
    if (S > 1)
        st = check_hip(hipMemcpyAsync(l.slice_rp, srp.data(), srp.size() * sizeof(int), hipMemcpyHostToDevice,
                                      stream), "hipMemcpyAsync");
    if (st == TFDP_OK && nnz > 0)
        st = check_hip(hipMemcpyAsync(l.slice_col, scol.data(), scol.size() * sizeof(int), hipMemcpyHostToDevice,
                                      stream), "hipMemcpyAsync");
    if (st == TFDP_OK)
        st = check_hip(hipMemcpyAsync(l.sched, all_sched.data(), all_sched.size() * sizeof(int2),
                                      hipMemcpyHostToDevice, stream), "hipMemcpyAsync");
    if (st == TFDP_OK) st = check_hip(hipStreamSynchronize(stream), "hipStreamSynchronize");
    return st;
}

// Edge pass of one iteration: slices 0 .. S-2 accumulate attraction sums,
// the last slice finishes every node (pos_out == nullptr: force outputs).
void enqueue_edges(tfdp_layout* h, const float2* pos, float2* pos_out, const Bufs& b, const Geom& g,
                   const ModelArgs& a, int set, float2* fr, float2* fa, float2* ft, hipStream_t s) {
    const Layout& l = h->lay;
    const int S = l.nslices;
    for (int sl = 0; sl + 1 < S; ++sl)
        launch_edges(pos, nullptr, l.slice[sl], sl == 0 ? 0 : 1, 0, l.fpart, b, g, a, set, nullptr, nullptr,
                     nullptr, s);
    launch_edges(pos, pos_out, l.slice[S - 1], 2, S > 1 ? 1 : 0, l.fpart, b, g, a, set, fr, fa, ft, s);
}

// Whether the edge pass of this handle runs overlapped with the grid passes
// (single-slice handles only); creates the second stream and its events on
// first use, on the handle's device. False (fused pass) if they cannot be
// created.
bool use_overlap(tfdp_layout* h) {
    if (h->lay.nslices != 1) return false;
    if (h->overlap_mode == 0 || (h->overlap_mode < 0 && h->nnz < kOverlapMinEntries)) return false;
    if (h->side) return true;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return false;
    if (cur != h->device && hipSetDevice(h->device) != hipSuccess) return false;
    bool ok = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&h->ev_node, hipEventDisableTiming) == hipSuccess;
    if (cur != h->device) (void)hipSetDevice(cur);
    if (!ok) {
        if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
        if (h->ev_join) (void)hipEventDestroy(h->ev_join);
        if (h->ev_node) (void)hipEventDestroy(h->ev_node);
        if (h->side) (void)hipStreamDestroy(h->side);
        h->ev_fork = h->ev_join = h->ev_node = nullptr;
        h->side = nullptr;
        h->overlap_mode = 0;
        (void)hipGetLastError();
        return false;
    }
    return true;
}

// Forces at pos for one k >= 1 and, with pos_out, the move: grid passes, then
// the edge pass. `set` is the slot set of the box extremes read now (set ^ 1
// receives the extremes of pos_out). Overlapped: the attraction pass runs on
// the second stream from the start of the grid passes, the node pass joins
// both on s.
void enqueue_evaluation(tfdp_layout* h, int k, int set, const float2* pos, float2* pos_out, const ModelArgs& a,
                        float2* fr, float2* fa, float2* ft, hipStream_t s) {
    const Bufs b = bufs_for(h, k);
    const Geom g = make_geom(h->p.n_int, k);
    if (use_overlap(h)) {
        (void)hipEventRecord(h->ev_fork, s);
        (void)hipStreamWaitEvent(h->side, h->ev_fork, 0);
        {
            PhaseTimer pt(h, PH_ATTRACT, h->side);
            launch_attract(pos, h->lay.slice[0], h->lay.fpart, b, g, a, h->attract_blocks[k <= 1 ? 0 : 1], h->side);
        }
        (void)hipEventRecord(h->ev_join, h->side);
        enqueue_grid(h, pos, b, g, set, s);
        (void)hipStreamWaitEvent(s, h->ev_join, 0);
        PhaseTimer pt(h, PH_NODE, s);
        launch_node_update(pos, pos_out, h->lay.fpart, b, g, a, set ^ 1, fr, fa, ft, s);
        return;
    }
    enqueue_grid(h, pos, b, g, set, s);
    PhaseTimer pt(h, PH_GATHER, s);
    enqueue_edges(h, pos, pos_out, b, g, a, set ^ 1, fr, fa, ft, s);
}

void drop_graphs(tfdp_layout* h) {
    for (int z = 0; z < 2; ++z)
        for (int k = 0; k < 4; ++k)
            for (int p = 0; p < 2; ++p)
                for (int o = 0; o < 2; ++o)
                    if (h->gexec[z][k][p][o]) {
                        (void)hipGraphExecDestroy(h->gexec[z][k][p][o]);
                        h->gexec[z][k][p][o] = nullptr;
                    }
}

// `iters` consecutive interpolated iterations (k >= 1) from positions A
// (then alternating between B and A); `parity` = t & 1 of the first selects
// its box-extremes slot set. Overlapped schedule, pipelined over the run:
// the attraction pass and the node pass of every iteration follow each other
// on the second stream, and the grid passes of an iteration (on s) start
// when the node pass of the previous one is done:
//   side: attract(t), [wait grid(t)] node(t), attract(t + 1), [wait grid(t + 1)] node(t + 1), ...
//   s:    grid(t), [wait node(t)] grid(t + 1), [wait node(t + 1)] ...
// At k = 1 on the 1M-node graph the attraction pass is the longer branch, so
// its stream runs back to back and only the grid passes wait across
// streams. s waits for the last node pass, so the run ends ordered on s.
void enqueue_run(tfdp_layout* h, int k, int parity, float2* A, float2* B, int iters, const ModelArgs& a,
                 hipStream_t s) {
    if (!use_overlap(h)) {
        for (int i = 0; i < iters; ++i) {
            enqueue_evaluation(h, k, (parity + i) & 1, A, B, a, nullptr, nullptr, nullptr, s);
            float2* t = A;
            A = B;
            B = t;
        }
        return;
    }
    const Bufs b = bufs_for(h, k);
    const Geom g = make_geom(h->p.n_int, k);
    const int ab = h->attract_blocks[k <= 1 ? 0 : 1];
    (void)hipEventRecord(h->ev_fork, s);
    (void)hipStreamWaitEvent(h->side, h->ev_fork, 0);
    {
        PhaseTimer pt(h, PH_ATTRACT, h->side);
        launch_attract(A, h->lay.slice[0], h->lay.fpart, b, g, a, ab, h->side);
    }
    for (int i = 0; i < iters; ++i) {
        const int set = (parity + i) & 1;
        enqueue_grid(h, A, b, g, set, s);
        (void)hipEventRecord(h->ev_join, s);
        (void)hipStreamWaitEvent(h->side, h->ev_join, 0);
        {
            PhaseTimer pt(h, PH_NODE, h->side);
            launch_node_update(A, B, h->lay.fpart, b, g, a, set ^ 1, nullptr, nullptr, nullptr, h->side);
        }
        // the next grid passes wait for this node pass only, not for the
        // attraction pass queued behind it
        (void)hipEventRecord(h->ev_node, h->side);
        (void)hipStreamWaitEvent(s, h->ev_node, 0);
        if (i + 1 < iters) {
            PhaseTimer pt(h, PH_ATTRACT, h->side);
            launch_attract(B, h->lay.slice[0], h->lay.fpart, b, g, a, ab, h->side);
        }
        float2* t = A;
        A = B;
        B = t;
    }
}

// Graph of `iters` (2 or kGraphIters, even) consecutive iterations at k
// starting with slot set `parity` and positions in the caller's buffer
// (orient 0) or the second buffer (orient 1), which they end in again;
// captured on first use. Longer groups spread the cost of a graph launch
// (a gap of several microseconds on the device) over more iterations.
hipGraphExec_t group_graph(tfdp_layout* h, int iters, int k, int parity, int orient, const ModelArgs& a,
                           hipStream_t s) {
    hipGraphExec_t& ex = h->gexec[iters == 2 ? 0 : 1][k][parity][orient];
    if (ex) return ex;
    float2* A = reinterpret_cast<float2*>(h->pos);
    float2* B = h->lay.pos_alt;
    if (orient) {
        float2* t = A;
        A = B;
        B = t;
    }
    if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) return nullptr;
    enqueue_run(h, k, parity, A, B, iters, a, s);
    hipGraph_t graph = nullptr;
    if (hipStreamEndCapture(s, &graph) != hipSuccess || !graph) return nullptr;
    if (hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0) != hipSuccess) ex = nullptr;
    (void)hipGraphDestroy(graph);
    return ex;
}


// New parameters; a new grid re-lays the grid arrays inside the same
// workspace (TFDP_ERR_WORKSPACE if they do not fit).
tfdp_status relay_grid(tfdp_layout* h, const tfdp_params& q) {
    if (q.n_int != h->p.n_int || k_workspace(&q) != h->k_ws) {
        size_t need = 0;
        Layout nl = carve(h->ws, h->n, h->nnz, &q, h->slice_nodes, &need);
        if (need > h->ws_bytes) {
            set_msg("workspace too small for this n_int / k_mode: need " + std::to_string(need) + " bytes");
            return TFDP_ERR_WORKSPACE;
        }
        for (int s = 0; s < kMaxSlices; ++s) nl.slice[s] = h->lay.slice[s];
        h->lay = nl;
        h->k_ws = k_workspace(&q);
        h->tw_pending = true;
    }
    h->p = q;
    h->version += 1;
    drop_graphs(h);
    return TFDP_OK;
}

float host_dec_ord(unsigned int u) {
    const unsigned int v = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
    float f;
    std::memcpy(&f, &v, sizeof(f));
    return f;
}

// Automatic grid: intervals per side = max(kAutoGridMin, ceil(W)) for the
// box side W of the current positions (one interval per unit of layout
// length), capped by the workspace. Reads the box extremes back to the host.
tfdp_status choose_auto_grid(tfdp_layout* h, hipStream_t s) {
    DevState* st = h->lay.b.st;
    const int set = h->t & 1;
    launch_box_begin(st, h->t, s);
    launch_box_reduce(reinterpret_cast<const float2*>(h->pos), h->n, st, set, s);
    unsigned int mm[kBoxSlots][32];
    tfdp_status r = check_hip(hipMemcpyAsync(mm, st->mm[set], sizeof(mm), hipMemcpyDeviceToHost, s),
                              "hipMemcpyAsync");
    if (r == TFDP_OK) r = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (r != TFDP_OK) return r;
    unsigned int a0 = 0xffffffffu, a1 = 0xffffffffu, a2 = 0u, a3 = 0u;
    for (int i = 0; i < kBoxSlots; ++i) {
        a0 = std::min(a0, mm[i][0]);
        a1 = std::min(a1, mm[i][1]);
        a2 = std::max(a2, mm[i][2]);
        a3 = std::max(a3, mm[i][3]);
    }
    double w = 1.0;
    if (a0 != 0xffffffffu) {
        w = std::max((double)host_dec_ord(a2) - (double)host_dec_ord(a0),
                     (double)host_dec_ord(a3) - (double)host_dec_ord(a1));
        if (!(w > 0.0)) w = 1.0;
    }
    const int cap = auto_grid_cap(&h->p);
    const double want = std::max((double)kAutoGridMin, std::ceil(w));
    tfdp_params q = h->p;
    q.n_int = (int)std::min((double)cap, want);
    return relay_grid(h, q);
}

}  // namespace

extern "C" {

const char* tfdp_last_error(void) { return last_msg(); }

void tfdp_params_default(tfdp_params* p) {
    if (!p) return;
    p->alpha = 0.1f;
    p->beta = 8.0f;
    p->gamma = 2.0f;
    p->rep_weight = 1.0f;
    p->n_int = 64;
    p->k_mode = -1;
    p->total_iters = 300;
    p->t0 = 0.0f;
    p->tau = 1.0f;
}

tfdp_status tfdp_params_validate(const tfdp_params* p, int32_t n, int64_t nnz) {
    set_msg("");
    if (!p) {
        set_msg("params is NULL");
        return TFDP_ERR_INVALID_ARG;
    }
    if (n < 1) {
        set_msg("n must be >= 1");
        return TFDP_ERR_INVALID_ARG;
    }
    if (nnz < 0 || nnz > 2147483647LL) {
        set_msg("nnz must be in [0, 2^31)");
        return TFDP_ERR_INVALID_ARG;
    }
    if (!finite_f(p->gamma) || !(p->gamma > 1.0f)) {
        set_msg("gamma must be > 1 (Eq.10)");
        return TFDP_ERR_INVALID_ARG;
    }
    if (!finite_f(p->tau) || !(p->tau > 0.f)) {
        set_msg("tau must be finite and > 0 (Eq.3)");
        return TFDP_ERR_INVALID_ARG;
    }
    if (!finite_f(p->alpha) || p->alpha < 0.f || !finite_f(p->beta) || p->beta < 0.f ||
        !finite_f(p->rep_weight) || p->rep_weight < 0.f) {
        set_msg("alpha, beta and rep_weight must be finite and >= 0");
        return TFDP_ERR_INVALID_ARG;
    }
    if (p->n_int < 0 || p->n_int > kMaxNInt) {
        set_msg("n_int must be 0 (automatic) or in [1, 1024]");
        return TFDP_ERR_INVALID_ARG;
    }
    if (p->k_mode < -1 || p->k_mode > 3) {
        set_msg("k_mode must be -1, 0, 1, 2 or 3");
        return TFDP_ERR_INVALID_ARG;
    }
    if (p->total_iters < 1) {
        set_msg("total_iters must be >= 1");
        return TFDP_ERR_INVALID_ARG;
    }
    if (!finite_f(p->t0)) {
        set_msg("t0 must be finite");
        return TFDP_ERR_INVALID_ARG;
    }
    if (n > (1 << 26)) {
        set_msg("n above 2^26 is not supported (packed edge entries)");
        return TFDP_ERR_UNSUPPORTED;
    }
    if ((long long)p->n_int * k_workspace(p) > kMaxL / 2) {
        set_msg("n_int * k exceeds 1024 (FFT length above 2048)");
        return TFDP_ERR_UNSUPPORTED;
    }
    if (p->alpha * (1.0f + p->beta) >= 1.0f)
        set_msg("warning: alpha (1 + beta) >= 1 violates the contact condition of Eq.9");
    return TFDP_OK;
}

size_t tfdp_workspace_size(int32_t n, int64_t nnz, const tfdp_params* p) {
    if (tfdp_params_validate(p, n, nnz) != TFDP_OK) return 0;
    size_t bytes = 0;
    const tfdp_params q = sizing_params(p);
    carve(nullptr, n, nnz, &q, slice_nodes(), &bytes);
    return bytes;
}

tfdp_status tfdp_layout_init(tfdp_layout** out, int32_t n, int64_t nnz, const int32_t* d_row_ptr,
                             const int32_t* d_col_idx, float* d_pos, void* d_ws, size_t ws_bytes,
                             const tfdp_params* p, hipStream_t stream) {
    if (!out) {
        set_msg("out is NULL");
        return TFDP_ERR_INVALID_ARG;
    }
    *out = nullptr;
    tfdp_status st = tfdp_params_validate(p, n, nnz);
    if (st != TFDP_OK) return st;
    std::string warn = g_msg;
    if (!d_row_ptr || (!d_col_idx && nnz > 0) || !d_pos) {
        set_msg("row_ptr, col_idx and pos must be non-NULL");
        return TFDP_ERR_INVALID_ARG;
    }
    size_t need = 0;
    const long long sn = slice_nodes();
    const tfdp_params sizing = sizing_params(p);
    carve(nullptr, n, nnz, &sizing, sn, &need);
    if (!d_ws || ws_bytes < need) {
        set_msg("workspace too small: need " + std::to_string(need) + " bytes");
        return TFDP_ERR_WORKSPACE;
    }
    if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) {
        set_msg("workspace must be 256-byte aligned");
        return TFDP_ERR_WORKSPACE;
    }
    tfdp_layout* h = new (std::nothrow) tfdp_layout();
    if (!h) {
        set_msg("host allocation failed");
        return TFDP_ERR_INVALID_ARG;
    }
    h->n = n;
    h->nnz = nnz;
    h->row_ptr = d_row_ptr;
    h->col_idx = d_col_idx;
    h->pos = d_pos;
    h->ws = d_ws;
    h->ws_bytes = ws_bytes;
    h->p = *p;
    h->auto_grid = p->n_int == 0;
    if (h->auto_grid) h->p.n_int = std::min(kAutoGridMin, auto_grid_cap(p));
    h->k_ws = k_workspace(p);
    h->t = 0;
    h->prof = false;
    h->graphs = true;
    std::memset(h->gexec, 0, sizeof(h->gexec));
    h->ev_used = 0;
    h->ev_stream = nullptr;
    size_t bytes = 0;
    h->slice_nodes = sn;
    h->lay = carve(d_ws, n, nnz, &h->p, sn, &bytes);
    static std::atomic<unsigned long long> next_uid{1};
    h->uid = next_uid.fetch_add(1);
    h->overlap_mode = -1;
    h->side = nullptr;
    h->ev_fork = h->ev_join = h->ev_node = nullptr;
    h->device = 0;
    int cus = 0;
    st = check_hip(hipGetDevice(&h->device), "hipGetDevice");
    if (st == TFDP_OK)
        st = check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device),
                       "hipDeviceGetAttribute");
    if (st != TFDP_OK) {
        delete h;
        return st;
    }
    h->attract_blocks[0] = std::max(1, cus) * attract_blocks_per_cu(1);
    h->attract_blocks[1] = std::max(1, cus) * attract_blocks_per_cu(2);

    DevState* dst = h->lay.b.st;
    static const bool attrs = (init_kernel_attributes(), true);
    (void)attrs;
    st = check_hip(hipMemsetAsync(dst, 0, sizeof(DevState), stream), "hipMemsetAsync");
    if (st == TFDP_OK)
        st = check_hip(hipMemsetAsync(h->lay.b.sym_acc, 0, (size_t)2 * n * sizeof(unsigned long long), stream),
                       "hipMemsetAsync");
    if (st == TFDP_OK) {
        if (nnz > 0 || n > 0) launch_csr_check(d_row_ptr, d_col_idx, n, nnz, dst, stream);
        h->tw_pending = true;
        enqueue_twiddles(h, stream);
        st = check_hip(hipGetLastError(), "kernel launch");
    }
    DevState hs;
    if (st == TFDP_OK) st = check_hip(hipMemcpyAsync(&hs, dst, sizeof(DevState), hipMemcpyDeviceToHost, stream), "hipMemcpyAsync");
    if (st == TFDP_OK) st = check_hip(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (st == TFDP_OK && hs.csr_bad) {
        set_msg("invalid CSR: row_ptr must start at 0, be monotone and end at nnz; columns in [0, n) without self-loops");
        st = TFDP_ERR_INVALID_ARG;
    }
    if (st == TFDP_OK) st = build_slices(h, stream);
    if (st != TFDP_OK) {
        delete h;
        return st;
    }
    set_msg(warn);
    *out = h;
    return TFDP_OK;
}

static tfdp_status step_fixed_grid(tfdp_layout* h, int32_t iters, hipStream_t s);

tfdp_status tfdp_layout_step(tfdp_layout* h, int32_t iters, hipStream_t s) {
    if (!h || iters < 0) {
        set_msg("invalid handle or iteration count");
        return TFDP_ERR_INVALID_ARG;
    }
    set_msg("");
    if (iters == 0) return TFDP_OK;
    if (!h->auto_grid) return step_fixed_grid(h, iters, s);
    for (int done = 0; done < iters;) {
        const int c = std::min(kAutoGridChunk - h->t % kAutoGridChunk, iters - done);
        if (h->t % kAutoGridChunk == 0) {  // chosen at fixed counters: independent of how calls split
            tfdp_status st = choose_auto_grid(h, s);
            if (st != TFDP_OK) return st;
        }
        tfdp_status st = step_fixed_grid(h, c, s);
        if (st != TFDP_OK) return st;
        done += c;
    }
    return TFDP_OK;
}

static tfdp_status step_fixed_grid(tfdp_layout* h, int32_t iters, hipStream_t s) {
    const ModelArgs a = model_args(h);
    float2* cur = reinterpret_cast<float2*>(h->pos);
    float2* alt = h->lay.pos_alt;
    enqueue_twiddles(h, s);
    enqueue_box(h, cur, h->t & 1, s);
    const bool use_graphs = h->graphs && !h->prof;
    for (int it = 0; it < iters;) {
        const int k = k_at(h->p, h->t);
        // a captured group when the next G iterations share k (the schedule
        // never lowers k, so checking the last one suffices)
        int G = 0;
        if (use_graphs && k > 0) {
            if (it + kGraphIters <= iters && k_at(h->p, h->t + kGraphIters - 1) == k)
                G = kGraphIters;
            else if (it + 2 <= iters && k_at(h->p, h->t + 1) == k)
                G = 2;
        }
        if (G > 0) {
            const int orient = cur == reinterpret_cast<float2*>(h->pos) ? 0 : 1;
            hipGraphExec_t ex = group_graph(h, G, k, h->t & 1, orient, a, s);
            if (ex) {
                tfdp_status st = check_hip(hipGraphLaunch(ex, s), "hipGraphLaunch");
                if (st != TFDP_OK) return st;
                h->t += G;
                it += G;
                continue;  // an even number of swaps: cur and alt keep their roles
            }
            (void)hipGetLastError();
        }
        if (k == 0) {
            PhaseTimer pt(h, PH_BRUTE, s);
            enqueue_exact(h, cur, alt, a, nullptr, nullptr, nullptr, s);
        } else {
            enqueue_run(h, k, h->t & 1, cur, alt, 1, a, s);
        }
        float2* tmp = cur;
        cur = alt;
        alt = tmp;
        h->t += 1;
        ++it;
    }
    if (cur != reinterpret_cast<float2*>(h->pos)) {
        tfdp_status st = check_hip(hipMemcpyAsync(h->pos, cur, (size_t)h->n * sizeof(float2),
                                                  hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
        if (st != TFDP_OK) return st;
    }
    return check_hip(hipGetLastError(), "kernel launch");
}

tfdp_status tfdp_layout_forces(tfdp_layout* h, const float* d_pos_in, int32_t k, float* d_f_rep,
                               float* d_f_att, float* d_f_tot, hipStream_t s) {
    if (!h || !d_pos_in || k < 0 || k > 3) {
        set_msg("invalid handle, position pointer or k");
        return TFDP_ERR_INVALID_ARG;
    }
    if (k > h->k_ws) {
        set_msg("k exceeds the k the workspace was sized for");
        return TFDP_ERR_WORKSPACE;
    }
    set_msg("");
    const ModelArgs a = model_args(h);
    enqueue_twiddles(h, s);
    const float2* pos = reinterpret_cast<const float2*>(d_pos_in);
    float2* fr = reinterpret_cast<float2*>(d_f_rep);
    float2* fa = reinterpret_cast<float2*>(d_f_att);
    float2* ft = reinterpret_cast<float2*>(d_f_tot);
    if (k == 0) {
        PhaseTimer pt(h, PH_BRUTE, s);
        enqueue_exact(h, pos, nullptr, a, fr, fa, ft, s);
    } else {
        enqueue_box(h, pos, 0, s);
        enqueue_evaluation(h, k, 0, pos, nullptr, a, fr, fa, ft, s);
    }
    return check_hip(hipGetLastError(), "kernel launch");
}

tfdp_status tfdp_layout_set_params(tfdp_layout* h, const tfdp_params* p) {
    if (!h) {
        set_msg("invalid handle");
        return TFDP_ERR_INVALID_ARG;
    }
    tfdp_status st = tfdp_params_validate(p, h->n, h->nnz);
    if (st != TFDP_OK) return st;
    tfdp_params q = *p;
    const bool automatic = p->n_int == 0;
    if (automatic) {
        // the workspace must hold the largest automatic grid
        size_t need = 0;
        const tfdp_params sizing = sizing_params(p);
        carve(nullptr, h->n, h->nnz, &sizing, h->slice_nodes, &need);
        if (need > h->ws_bytes) {
            set_msg("workspace too small for the automatic grid: need " + std::to_string(need) + " bytes");
            return TFDP_ERR_WORKSPACE;
        }
        q.n_int = h->auto_grid ? std::min(h->p.n_int, auto_grid_cap(p)) : std::min(kAutoGridMin, auto_grid_cap(p));
    }
    st = relay_grid(h, q);
    if (st != TFDP_OK) return st;
    h->auto_grid = automatic;
    return TFDP_OK;
}

tfdp_status tfdp_layout_get_params(const tfdp_layout* h, tfdp_params* out) {
    if (!h || !out) {
        set_msg("invalid handle or pointer");
        return TFDP_ERR_INVALID_ARG;
    }
    *out = h->p;
    return TFDP_OK;
}

tfdp_status tfdp_layout_set_node_weights(tfdp_layout* h, const float* d_rep_w, const float* d_att_w) {
    if (!h) {
        set_msg("invalid handle");
        return TFDP_ERR_INVALID_ARG;
    }
    set_msg("");
    h->rep_w = d_rep_w;
    h->att_w = d_att_w;
    h->version += 1;
    drop_graphs(h);
    return TFDP_OK;
}

tfdp_status tfdp_layout_get_iter(const tfdp_layout* h, int32_t* t) {
    if (!h || !t) {
        set_msg("invalid handle or pointer");
        return TFDP_ERR_INVALID_ARG;
    }
    *t = h->t;
    return TFDP_OK;
}

tfdp_status tfdp_layout_set_iter(tfdp_layout* h, int32_t t) {
    if (!h || t < 0) {
        set_msg("invalid handle or iteration");
        return TFDP_ERR_INVALID_ARG;
    }
    h->t = t;
    return TFDP_OK;
}

tfdp_status tfdp_layout_sync_status(tfdp_layout* h, hipStream_t s) {
    if (!h) {
        set_msg("invalid handle");
        return TFDP_ERR_INVALID_ARG;
    }
    tfdp_status st = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (st != TFDP_OK) return st;
    st = check_hip(hipGetLastError(), "kernel");
    if (st != TFDP_OK) return st;
    int flag = 0;
    DevState* dst = h->lay.b.st;
    st = check_hip(hipMemcpyAsync(&flag, &dst->nonfinite, sizeof(int), hipMemcpyDeviceToHost, s),
                   "hipMemcpyAsync");
    if (st == TFDP_OK) st = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (st != TFDP_OK) return st;
    if (flag) {
        int zero = 0;
        (void)hipMemcpyAsync(&dst->nonfinite, &zero, sizeof(int), hipMemcpyHostToDevice, s);
        (void)hipStreamSynchronize(s);
        set_msg("a position became NaN or infinite");
        return TFDP_ERR_NONFINITE;
    }
    return TFDP_OK;
}

void tfdp_layout_destroy(tfdp_layout* h) {
    if (!h) return;
    drop_graphs(h);
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    if (h->ev_node) (void)hipEventDestroy(h->ev_node);
    if (h->side) (void)hipStreamDestroy(h->side);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    delete h;
}

tfdp_status tfdp_layout_set_profiling(tfdp_layout* h, int32_t enable) {
    if (!h) {
        set_msg("invalid handle");
        return TFDP_ERR_INVALID_ARG;
    }
    h->prof = enable != 0;
    h->ev_used = 0;
    h->ev_phase.clear();
    return TFDP_OK;
}

tfdp_status tfdp_layout_set_overlap(tfdp_layout* h, int32_t mode) {
    if (!h || mode < -1 || mode > 1) {
        set_msg("invalid handle or overlap mode (-1, 0 or 1)");
        return TFDP_ERR_INVALID_ARG;
    }
    if (mode == 1 && h->lay.nslices != 1) {
        set_msg("the overlapped edge pass needs a single column slice");
        return TFDP_ERR_UNSUPPORTED;
    }
    set_msg("");
    if (mode != h->overlap_mode) {
        h->overlap_mode = mode;
        drop_graphs(h);
    }
    return TFDP_OK;
}

tfdp_status tfdp_layout_set_graphs(tfdp_layout* h, int32_t enable) {
    if (!h) {
        set_msg("invalid handle");
        return TFDP_ERR_INVALID_ARG;
    }
    h->graphs = enable != 0;
    if (!h->graphs) drop_graphs(h);
    return TFDP_OK;
}

size_t tfdp_stress_workspace_size(int32_t n, int32_t nsrc) {
    if (n < 1 || nsrc < 1 || nsrc > 64) return 0;
    return stress_workspace_bytes(n, nsrc);
}

static tfdp_status quality_sampled(int32_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col_idx,
                                   const float* d_pos, const int32_t* d_sources, int32_t nsrc, void* d_work,
                                   size_t work_bytes, double* se, double* np, int32_t* levels, hipStream_t stream) {
    set_msg("");
    if (n < 1 || nnz < 0 || nsrc < 1 || nsrc > 64 || !d_row_ptr || (!d_col_idx && nnz > 0) || !d_pos ||
        !d_sources || !se) {
        set_msg("invalid sizes or pointers (1 <= nsrc <= 64)");
        return TFDP_ERR_INVALID_ARG;
    }
    if (!d_work || work_bytes < stress_workspace_bytes(n, nsrc) || ((uintptr_t)d_work & 255u)) {
        set_msg("metric workspace missing, misaligned or smaller than tfdp_stress_workspace_size");
        return TFDP_ERR_WORKSPACE;
    }
    int lv = 0;
    const int e = stress_sampled(n, nnz, d_row_ptr, d_col_idx, reinterpret_cast<const float2*>(d_pos), d_sources,
                                 nsrc, d_work, se, np, &lv, stream);
    if (levels) *levels = lv;
    if (e == -1) {
        set_msg("invalid CSR: row_ptr must start at 0, be monotone and end at nnz; columns in [0, n)");
        return TFDP_ERR_INVALID_ARG;
    }
    if (e == -2) {
        set_msg("a source node is outside [0, n)");
        return TFDP_ERR_INVALID_ARG;
    }
    if (e == -3) {
        set_msg("the BFS still reaches new nodes at hop distance 65534 (16-bit distances)");
        return TFDP_ERR_UNSUPPORTED;
    }
    if (e != 0) return check_hip((hipError_t)e, "metrics");
    return check_hip(hipGetLastError(), "kernel launch");
}

tfdp_status tfdp_stress_sampled(int32_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col_idx,
                                const float* d_pos, const int32_t* d_sources, int32_t nsrc, void* d_work,
                                size_t work_bytes, double* se, int32_t* levels, hipStream_t stream) {
    return quality_sampled(n, nnz, d_row_ptr, d_col_idx, d_pos, d_sources, nsrc, d_work, work_bytes, se, nullptr,
                           levels, stream);
}

tfdp_status tfdp_quality_sampled(int32_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col_idx,
                                 const float* d_pos, const int32_t* d_sources, int32_t nsrc, void* d_work,
                                 size_t work_bytes, double* se, double* np, int32_t* levels, hipStream_t stream) {
    if (!np) {
        set_msg("np must point to two doubles");
        return TFDP_ERR_INVALID_ARG;
    }
    return quality_sampled(n, nnz, d_row_ptr, d_col_idx, d_pos, d_sources, nsrc, d_work, work_bytes, se, np,
                           levels, stream);
}

int32_t tfdp_phase_count(void) { return PH_COUNT; }

const char* tfdp_phase_name(int32_t phase) {
    if (phase < 0 || phase >= PH_COUNT) return "";
    return kPhaseNames[phase];
}

tfdp_status tfdp_layout_phase_times(tfdp_layout* h, double* total_ms, int64_t* launches, int32_t nphases) {
    if (!h || !total_ms || !launches || nphases < PH_COUNT) {
        set_msg("invalid handle or arrays shorter than tfdp_phase_count()");
        return TFDP_ERR_INVALID_ARG;
    }
    for (int i = 0; i < PH_COUNT; ++i) {
        total_ms[i] = 0.0;
        launches[i] = 0;
    }
    if (h->ev_used >= 2) {
        tfdp_status st = check_hip(hipEventSynchronize(h->ev_pool[h->ev_used - 1]), "hipEventSynchronize");
        if (st != TFDP_OK) return st;
    }
    for (size_t i = 0; i < h->ev_phase.size() && 2 * i + 1 < h->ev_used; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->ev_pool[2 * i], h->ev_pool[2 * i + 1]) == hipSuccess) {
            total_ms[h->ev_phase[i]] += ms;
            launches[h->ev_phase[i]] += 1;
        }
    }
    h->ev_used = 0;
    h->ev_phase.clear();
    return TFDP_OK;
}

}  // extern "C"
