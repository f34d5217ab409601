// Host side of the C ABI declared in include/tfdp.h: parameter validation,
// workspace layout, the per-iteration launch sequence and profiling.
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "tfdp.h"
#include "tfdp_internal.h"

using namespace tfdp;

namespace {

thread_local std::string g_msg;

void set_msg(const std::string& s) { g_msg = s; }

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
    PH_COUNT
};

const char* kPhaseNames[PH_COUNT] = {"box",     "bin_count", "bin_scan", "bin_scatter",   "spread",
                                     "rowfft",  "colconv",   "rowifft",  "gather_update", "brute"};

int k_workspace(const tfdp_params* p) { return (p->k_mode == 1 || p->k_mode == 2) ? p->k_mode : 3; }

Geom make_geom(int n_int, int k) {
    Geom g;
    g.k = k;
    g.m = n_int * k;
    int L = 64, logL = 6;
    while (L < 2 * g.m) {
        L <<= 1;
        ++logL;
    }
    g.L = L;
    g.logL = logL;
    g.H = L / 2 + 1;
    g.cw = L >= 512 ? 1 : 512 / L;  // transforms per FFT task
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
};

Layout carve(void* base, int n, long long nnz, const tfdp_params* p, size_t* bytes) {
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
    l.b.blkcnt = c.take<int>((size_t)p->n_int * l.b.nblk);
    l.b.bucket_cnt = c.take<int>((size_t)p->n_int);
    l.b.bucket_start = c.take<int>((size_t)p->n_int + 1);
    l.b.chunk_start = c.take<int>((size_t)p->n_int + 1);
    l.b.chunk_row = c.take<int>((size_t)l.b.max_chunks);
    l.b.spart = c.take<float>((size_t)l.b.max_chunks * kw * gw.m * 3);
    l.b.qcol = c.take<float2>((size_t)3 * gw.H * gw.m);
    l.b.kcol = c.take<float2>((size_t)gw.H * gw.L);
    l.b.pcol = c.take<float2>((size_t)3 * gw.H * gw.m);
    l.b.pot = c.take<float4>((size_t)gw.m * gw.m);
    l.b.sched = c.take<int2>((size_t)4 * edge_blocks_bound(n, nnz));
    for (int k = 1; k <= kw; ++k) l.tw[k] = c.take<float2>((size_t)make_geom(p->n_int, k).L);
    *bytes = (c.off + 255) & ~(size_t)255;
    return l;
}

bool finite_f(float v) { return std::isfinite(v); }

// Edge-pass schedule: rows with more than kGroupEdges entries get a block
// each (slot 0 = {row, -1}); the other rows are cut, in order, into wave
// groups of at most kGroupRows rows and kGroupEdges entries, four groups per
// block (slot = {first row, rows}; {0, 0} = idle wave). Heavy blocks first.
std::vector<int2> build_edge_schedule(const std::vector<int>& rp, int n) {
    std::vector<int2> heavy, groups;
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

tfdp_status check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return TFDP_OK;
    set_msg(std::string(what) + ": " + hipGetErrorString(e));
    return TFDP_ERR_HIP;
}

}  // namespace

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
    Layout lay;
    // profiling
    bool prof;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used;
    std::vector<int> ev_phase;  // phase of each recorded pair
    hipStream_t ev_stream;
};

namespace {

ModelArgs model_args(const tfdp_layout* h) {
    ModelArgs a;
    a.alpha = h->p.alpha;
    a.beta = h->p.beta;
    a.gamma = h->p.gamma;
    a.rep_weight = h->p.rep_weight;
    a.t0 = h->p.t0 > 0.f ? h->p.t0 : std::fmax(1.0f, (float)(std::sqrt((double)h->n) / 10.0));
    a.total_iters = h->p.total_iters;
    return a;
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

Bufs bufs_for(const tfdp_layout* h, int k) {
    Bufs b = h->lay.b;
    b.tw = h->lay.tw[k];
    return b;
}

// One evaluation of the interpolated repulsion up to the grid potentials;
// the box comes from extremes slot set `set`, set ^ 1 is reset for the
// update that follows.
void enqueue_grid(tfdp_layout* h, const float2* pos, const Bufs& b, const Geom& g, int set, hipStream_t s) {
    { PhaseTimer pt(h, PH_BIN_COUNT, s); launch_bin_count(pos, b, set, s); }
    { PhaseTimer pt(h, PH_BIN_SCAN, s); launch_bin_scan(b, set ^ 1, s); }
    { PhaseTimer pt(h, PH_BIN_SCATTER, s); launch_bin_scatter(pos, b, s); }
    { PhaseTimer pt(h, PH_SPREAD, s); launch_spread(b, g, h->p.gamma, s); }
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

int k_at(const tfdp_params& p, int t) {
    if (p.k_mode >= 0) return p.k_mode;
    const int T = p.total_iters;
    if (t < (9 * T) / 10) return 1;
    if (t < (19 * T) / 20) return 2;
    return 3;
}

}  // namespace

extern "C" {

const char* tfdp_last_error(void) { return g_msg.c_str(); }

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
    if (!finite_f(p->alpha) || p->alpha < 0.f || !finite_f(p->beta) || p->beta < 0.f ||
        !finite_f(p->rep_weight) || p->rep_weight < 0.f) {
        set_msg("alpha, beta and rep_weight must be finite and >= 0");
        return TFDP_ERR_INVALID_ARG;
    }
    if (p->n_int < 1 || p->n_int > kMaxNInt) {
        set_msg("n_int must be in [1, 1024]");
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
    carve(nullptr, n, nnz, p, &bytes);
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
    carve(nullptr, n, nnz, p, &need);
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
    h->k_ws = k_workspace(p);
    h->t = 0;
    h->prof = false;
    h->ev_used = 0;
    h->ev_stream = nullptr;
    size_t bytes = 0;
    h->lay = carve(d_ws, n, nnz, p, &bytes);

    DevState* dst = h->lay.b.st;
    st = check_hip(hipMemsetAsync(dst, 0, sizeof(DevState), stream), "hipMemsetAsync");
    if (st == TFDP_OK) {
        if (nnz > 0 || n > 0) launch_csr_check(d_row_ptr, d_col_idx, n, nnz, dst, stream);
        for (int k = 1; k <= h->k_ws; ++k) launch_twiddles(h->lay.tw[k], make_geom(p->n_int, k).L, stream);
        st = check_hip(hipGetLastError(), "kernel launch");
    }
    DevState hs;
    if (st == TFDP_OK) st = check_hip(hipMemcpyAsync(&hs, dst, sizeof(DevState), hipMemcpyDeviceToHost, stream), "hipMemcpyAsync");
    if (st == TFDP_OK) st = check_hip(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (st == TFDP_OK && hs.csr_bad) {
        set_msg("invalid CSR: row_ptr must start at 0, be monotone and end at nnz; columns in [0, n) without self-loops");
        st = TFDP_ERR_INVALID_ARG;
    }
    if (st == TFDP_OK) {
        std::vector<int> rp((size_t)n + 1);
        st = check_hip(hipMemcpy(rp.data(), d_row_ptr, rp.size() * sizeof(int), hipMemcpyDeviceToHost), "hipMemcpy");
        if (st == TFDP_OK) {
            std::vector<int2> sched = build_edge_schedule(rp, n);
            h->lay.b.edge_blocks = (int)(sched.size() / 4);
            if ((long long)h->lay.b.edge_blocks > edge_blocks_bound(n, nnz)) {
                set_msg("internal: edge schedule exceeds its bound");
                st = TFDP_ERR_WORKSPACE;
            } else {
                st = check_hip(hipMemcpyAsync(const_cast<int2*>(h->lay.b.sched), sched.data(),
                                              sched.size() * sizeof(int2), hipMemcpyHostToDevice, stream),
                               "hipMemcpyAsync");
                if (st == TFDP_OK) st = check_hip(hipStreamSynchronize(stream), "hipStreamSynchronize");
            }
        }
    }
    if (st != TFDP_OK) {
        delete h;
        return st;
    }
    set_msg(warn);
    *out = h;
    return TFDP_OK;
}

tfdp_status tfdp_layout_step(tfdp_layout* h, int32_t iters, hipStream_t s) {
    if (!h || iters < 0) {
        set_msg("invalid handle or iteration count");
        return TFDP_ERR_INVALID_ARG;
    }
    set_msg("");
    if (iters == 0) return TFDP_OK;
    const ModelArgs a = model_args(h);
    float2* cur = reinterpret_cast<float2*>(h->pos);
    float2* alt = h->lay.pos_alt;
    enqueue_box(h, cur, h->t & 1, s);
    for (int it = 0; it < iters; ++it) {
        const int k = k_at(h->p, h->t);
        if (k == 0) {
            PhaseTimer pt(h, PH_BRUTE, s);
            launch_brute(cur, alt, h->row_ptr, h->col_idx, h->n, h->lay.b.st, a, h->t, nullptr, nullptr,
                         nullptr, s);
        } else {
            const Bufs b = bufs_for(h, k);
            const Geom g = make_geom(h->p.n_int, k);
            const int set = h->t & 1;
            enqueue_grid(h, cur, b, g, set, s);
            PhaseTimer pt(h, PH_GATHER, s);
            launch_gather(cur, alt, h->row_ptr, h->col_idx, b, g, a, set ^ 1, nullptr, nullptr, nullptr, s);
        }
        float2* tmp = cur;
        cur = alt;
        alt = tmp;
        h->t += 1;
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
    const float2* pos = reinterpret_cast<const float2*>(d_pos_in);
    float2* fr = reinterpret_cast<float2*>(d_f_rep);
    float2* fa = reinterpret_cast<float2*>(d_f_att);
    float2* ft = reinterpret_cast<float2*>(d_f_tot);
    if (k == 0) {
        PhaseTimer pt(h, PH_BRUTE, s);
        launch_brute(pos, nullptr, h->row_ptr, h->col_idx, h->n, h->lay.b.st, a, h->t, fr, fa, ft, s);
    } else {
        enqueue_box(h, pos, 0, s);
        const Bufs b = bufs_for(h, k);
        const Geom g = make_geom(h->p.n_int, k);
        enqueue_grid(h, pos, b, g, 0, s);
        PhaseTimer pt(h, PH_GATHER, s);
        launch_gather(pos, nullptr, h->row_ptr, h->col_idx, b, g, a, 1, fr, fa, ft, s);
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
    if (p->n_int != h->p.n_int) {
        set_msg("n_int cannot change on an existing handle");
        return TFDP_ERR_UNSUPPORTED;
    }
    if (k_workspace(p) > h->k_ws) {
        set_msg("k_mode needs a larger workspace than the handle has");
        return TFDP_ERR_WORKSPACE;
    }
    h->p = *p;
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
    st = check_hip(hipMemcpy(&flag, &dst->nonfinite, sizeof(int), hipMemcpyDeviceToHost), "hipMemcpy");
    if (st != TFDP_OK) return st;
    if (flag) {
        int zero = 0;
        (void)hipMemcpy(&dst->nonfinite, &zero, sizeof(int), hipMemcpyHostToDevice);
        set_msg("a position became NaN or infinite");
        return TFDP_ERR_NONFINITE;
    }
    return TFDP_OK;
}

void tfdp_layout_destroy(tfdp_layout* h) {
    if (!h) return;
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
