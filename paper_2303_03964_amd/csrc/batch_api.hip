// Host side of the batched C ABI (tfdp_batch_*): many layout handles stepped
// together. Every phase of an iteration is one launch per class of graphs
// (graphs in a class share the kernel template: k, FFT length and spreading
// block shape) whose blocks are listed in a device map {member entry, block};
// each block runs the plain kernel's body for that graph and block, so the
// result of every graph is bit-identical to tfdp_layout_step on it alone.
//
// Device tables live in the caller's workspace: per slot the member entries
// (one per k) and the counter at the start of a call, then an arena of block
// maps. A member keeps its slot while it is in the batch; entries and
// counters are written by small kernels whose arguments carry the values, so
// that adding, removing or re-tuning a member needs no stream
// synchronisation. A composition (the members, their grids and the k of each)
// owns a region of the arena and is kept for reuse; groups of eight (else
// two) of its iterations are captured as HIP graphs from the second time the
// same group is needed (a composition used once, as when serving changes the
// membership at every chunk, launches its kernels directly). A full arena is
// reset after one synchronisation.
#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "tfdp_handle.h"

using namespace tfdp;

namespace {

enum BPhase {
    B_BIN_COUNT, B_BIN_SCAN, B_BIN_SCATTER, B_SPREAD, B_ROWFFT, B_COLCONV, B_ROWIFFT, B_EDGES,
    B_BRUTE, B_SYM_PAIRS, B_SYM_NODE, B_TICK
};

struct BLaunch {
    int phase;
    int k, len, nw;  // row passes: nw = rows per block; column pass: nw = column groups per block
                     // (B_TICK: blocks = members, one map entry each)
    size_t off;       // first map entry (relative to the composition's region)
    int blocks;
    size_t lds;
    int lane = 0;     // 1: a grid pass of a class other than the largest (second stream)
};

// Index of an FFT length in the batch's tile table.
int len_index(int L) {
    switch (L) {
        case 64: return 0;
        case 128: return 1;
        case 256: return 2;
        case 384: return 3;
        case 512: return 4;
        case 768: return 5;
        case 1024: return 6;
        case 1536: return 7;
        default: return 8;
    }
}
constexpr int kLens[9] = {64, 128, 256, 384, 512, 768, 1024, 1536, 2048};

// One composition: the members (slot, handle, grid) with the k of each, the
// launches of an iteration and the maps of the call-level launches.
struct Comp {
    std::vector<long long> key;     // slot, handle uid, N_int, k for every member in slot order
    std::vector<BLaunch> launches;  // one iteration, in dependency order
    std::vector<int2> host_map;     // the region's contents (kept until the region is dropped)
    size_t off = 0;                 // first arena entry of the region
    int box_begin = 0, n_begin = 0, box_red = 0, n_red = 0, copy = 0, n_copy = 0;  // call-level maps
    // captured groups of 2 and kGraphIters iterations starting at an even /
    // odd j: [2 * (size == kGraphIters) + parity of j], and how often each was needed
    hipGraphExec_t gexec[4] = {nullptr, nullptr, nullptr, nullptr};
    int wanted[4] = {0, 0, 0, 0};
    unsigned long long last_use = 0;
};

constexpr int kMaxComps = 64;
constexpr int kCounterSet = 240;     // counters written per launch of kb_set_counters
constexpr size_t kMinArena = 256;    // map entries the workspace must leave at least

int entry_of(int slot, int k) { return slot * 3 + (k - 1); }

struct MemberEntries {
    Member e[3];  // k = 1, 2, 3
};
struct CounterSet {
    int count;
    int2 v[kCounterSet];  // {slot, counter}
};

__global__ void kb_set_entries(Member* dst, MemberEntries e) {
    if (threadIdx.x < 3) dst[threadIdx.x] = e.e[threadIdx.x];
}
__global__ void kb_set_counters(int* tcall, CounterSet cs) {
    const int i = threadIdx.x;
    if (i < cs.count) tcall[cs.v[i].x] = cs.v[i].y;
}
__global__ void kb_zero_counters(int* tcall, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) tcall[i] = 0;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
size_t entries_bytes(int cap) { return align256((size_t)cap * 3 * sizeof(Member)); }
size_t counters_bytes(int cap) { return align256((size_t)cap * sizeof(int)); }

}  // namespace

struct tfdp_batch {
    int cap;
    std::vector<tfdp_layout*> slot;            // [cap] member of each slot, or null
    std::vector<unsigned long long> seen_uid;  // [cap] handle whose entries the slot holds (0: none)
    std::vector<unsigned int> seen;            // [cap] that handle's version when they were written
    std::vector<int> t_dev;                    // [cap] counter the device holds for the next call
    int count;
    bool counters_ready;                       // device counters initialised
    Member* d_mem;                             // [cap][3] entries for k = 1..3 (caller's workspace)
    int* d_t;                                  // [cap] counters at the start of a call
    int2* d_arena;                             // block maps of the compositions
    size_t arena_cap, arena_used;              // in entries
    bool graphs;
    std::vector<Comp> comps;
    unsigned long long clock;
    int2 tiles[9];  // per FFT length: rows per block of the row passes, column groups of the column pass
    int device;                    // device current at creation
    hipStream_t side;              // second stream of the grid passes (created on first use)
    hipEvent_t ev_fork, ev_join;
    bool side_failed;
};

namespace {

Member make_member(const tfdp_layout* h, int slot, int k) {
    Member m;
    std::memset(&m, 0, sizeof(m));
    m.b = bufs_for(h, k, true);
    m.g = make_geom(h->p.n_int, k);
    m.a = model_args(h);
    m.es = h->lay.slice[0];
    m.pos = reinterpret_cast<float2*>(h->pos);
    m.alt = h->lay.pos_alt;
    m.slot = slot;
    spread_dims(m.b, m.g, &m.nw, &m.nkb);
    m.box_blocks = box_reduce_dims(h->n).grid;
    return m;
}

void free_comp(Comp& c) {
    for (hipGraphExec_t& g : c.gexec)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

void drop_comps(tfdp_batch* b) {
    for (Comp& c : b->comps) free_comp(c);
    b->comps.clear();
    b->arena_used = 0;
}

void drop_comp_graphs(tfdp_batch* b) {
    for (Comp& c : b->comps) free_comp(c);
}

// Work of a member in a phase, for the block order of a launch: the biggest
// graphs' blocks are dispatched first so that they do not form the tail.
long long member_work(const tfdp_layout* h) { return (long long)h->n + h->nnz; }

// Maps of composition c for the members in slots `act` with k values ks
// (the launches of one iteration, then the call-level maps).
void build_comp(tfdp_batch* b, const std::vector<int>& act, const std::vector<int>& ks, Comp& c) {
    const int nm = (int)act.size();
    auto H = [&](int i) { return b->slot[act[i]]; };
    std::vector<int> order, brute;
    for (int i = 0; i < nm; ++i) (ks[i] == 0 ? brute : order).push_back(i);
    auto bigger_first = [&](int x, int y) { return member_work(H(x)) > member_work(H(y)); };
    std::stable_sort(order.begin(), order.end(), bigger_first);
    std::stable_sort(brute.begin(), brute.end(), bigger_first);
    std::vector<int2>& map = c.host_map;
    auto emit = [&](int phase, int k, int len, int nw, size_t lds, const std::vector<int>& who,
                    const std::vector<int>& blocks) {
        BLaunch L{phase, k, len, nw, map.size(), 0, lds};
        for (size_t q = 0; q < who.size(); ++q)
            for (int j = 0; j < blocks[q]; ++j)
                map.push_back(make_int2(entry_of(act[who[q]], ks[who[q]] > 0 ? ks[who[q]] : 1), j));
        L.blocks = (int)(map.size() - L.off);
        if (L.blocks > 0) c.launches.push_back(L);
    };
    // binning (k-independent shapes): one launch each for all members
    {
        std::vector<int> bc, bs, bsc;
        size_t lds_c = 0, lds_s = 0;
        for (int i : order) {
            const Bufs bb = bufs_for(H(i), ks[i], true);
            const Dims dc = bin_count_dims(bb), ds = bin_scan_dims(bb), dsc = bin_scatter_dims(bb);
            bc.push_back(dc.grid);
            bs.push_back(ds.grid);
            bsc.push_back(dsc.grid);
            lds_c = std::max(lds_c, dc.lds);
            lds_s = std::max(lds_s, dsc.lds);
        }
        emit(B_BIN_COUNT, 0, 0, 0, lds_c, order, bc);
        emit(B_BIN_SCAN, 0, 0, 0, 0, order, bs);
        emit(B_BIN_SCATTER, 0, 0, 0, lds_s, order, bsc);
    }
    // spreading: classes (k, L, nw)
    {
        std::map<std::tuple<int, int, int>, std::vector<int>> cls;
        for (int i : order) {
            const Geom g = make_geom(H(i)->p.n_int, ks[i]);
            int nw, nkb;
            spread_dims(bufs_for(H(i), ks[i], true), g, &nw, &nkb);
            cls[std::make_tuple(ks[i], g.L, nw)].push_back(i);
        }
        for (auto& kv : cls) {
            std::vector<int> blocks;
            size_t lds = 0;
            for (int i : kv.second) {
                int nw, nkb;
                const Dims d = spread_dims(bufs_for(H(i), ks[i], true), make_geom(H(i)->p.n_int, ks[i]), &nw, &nkb);
                blocks.push_back(d.grid);
                lds = std::max(lds, d.lds);
            }
            emit(B_SPREAD, std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), lds, kv.second,
                 blocks);
        }
    }
    // row FFTs, column pass, inverse rows: classes by FFT length
    {
        std::map<int, std::vector<int>> cls;
        for (int i : order) cls[make_geom(H(i)->p.n_int, ks[i]).L].push_back(i);
        for (int phase : {B_ROWFFT, B_COLCONV, B_ROWIFFT})
            for (auto& kv : cls) {
                const int2 tile = b->tiles[len_index(kv.first)];
                const int param = phase == B_COLCONV ? tile.y : tile.x;
                std::vector<int> blocks;
                for (int i : kv.second) {
                    const Geom g = make_geom(H(i)->p.n_int, ks[i]);
                    int nb = 0;
                    if (phase == B_ROWFFT)
                        rowfft_dims(g, &nb, tile.x);
                    else if (phase == B_COLCONV)
                        nb = colconv_dims(g, tile.y).grid;
                    else
                        rowifft_dims(g, &nb, tile.x);
                    blocks.push_back(nb);
                }
                emit(phase, 0, kv.first, param, 0, kv.second, blocks);
            }
    }
    // The grid passes of different FFT lengths are independent chains: all
    // but the length with the most blocks run on the second stream, between
    // the binning and the edge pass. (The pair-symmetric exact launches stay
    // on the first stream after the edge pass: beside the FFT passes their
    // arithmetic-bound blocks slowed those latency-bound ones more than they
    // gained, size-rule grids 3.17e9 -> 2.76e9 node-it/s. The small exact
    // members' one launch, about 27 us at k = 1, does go to the second
    // stream below: 3.68e9 -> 3.77e9.)
    int main_len = 0;
    {
        std::map<int, long long> work;
        for (const BLaunch& L : c.launches)
            if (L.phase == B_SPREAD || L.phase == B_ROWFFT || L.phase == B_COLCONV || L.phase == B_ROWIFFT)
                work[L.len] += L.blocks;
        long long most = -1;
        for (auto& kv : work)
            if (kv.second > most) {
                most = kv.second;
                main_len = kv.first;
            }
        for (BLaunch& L : c.launches)
            if ((L.phase == B_SPREAD || L.phase == B_ROWFFT || L.phase == B_COLCONV || L.phase == B_ROWIFFT) &&
                L.len != main_len)
                L.lane = 1;
    }
    // exact method, split by size: the one-launch kernel for the small
    // members, the pair-symmetric passes for the others
    std::vector<int> small, big, bs, bp, bn;
    for (int i : brute) {
        if (use_sym(H(i)->n)) {
            big.push_back(i);
            bp.push_back((int)sym_pair_blocks(H(i)->n));
            bn.push_back(sym_node_blocks(H(i)->n));
        } else {
            small.push_back(i);
            bs.push_back((H(i)->n + kBruteRows - 1) / kBruteRows);
        }
    }
    // the small exact members need no grid: with a second stream in use
    // their launch runs there, after the shorter grid chains and before the
    // join, instead of on the longer chain's stream
    // (with their counters' advance behind them on the same stream)
    auto emit_tick = [&](const std::vector<int>& who, int lane) {
        if (who.empty()) return;
        BLaunch L{B_TICK, 0, 0, 0, map.size(), 0, 0};
        for (int i : who) map.push_back(make_int2(entry_of(act[i], 1), 0));
        L.blocks = (int)who.size();
        L.lane = lane;
        c.launches.push_back(L);
    };
    {
        bool side = false;
        for (const BLaunch& L : c.launches) side = side || L.lane == 1;
        const size_t at = c.launches.size();
        emit(B_BRUTE, 0, 0, 0, 0, small, bs);
        if (side && c.launches.size() > at) c.launches.back().lane = 1;
        emit_tick(small, side ? 1 : 0);
    }
    // edge pass + gather + move: classes by k, and by stream: the members of
    // the second stream's grid chains take theirs there too, before the
    // join, so that only the longer chain's members are left after it
    {
        bool side = false;
        for (const BLaunch& L : c.launches) side = side || L.lane == 1;
        std::map<std::pair<int, int>, std::vector<int>> cls;  // (lane, k): lane 1 first
        for (int i : order) {
            const int lane = side && make_geom(H(i)->p.n_int, ks[i]).L != main_len ? 1 : 0;
            cls[std::make_pair(-lane, ks[i])].push_back(i);
        }
        for (auto& kv : cls) {
            std::vector<int> blocks;
            for (int i : kv.second) blocks.push_back(H(i)->lay.slice[0].blocks);
            const size_t at = c.launches.size();
            emit(B_EDGES, kv.first.second, 0, 0, 0, kv.second, blocks);
            if (c.launches.size() > at) c.launches.back().lane = -kv.first.first;
        }
    }
    // the pair-symmetric passes, then their members' counters
    if (!big.empty()) {
        emit(B_SYM_PAIRS, 0, 0, 0, 0, big, bp);
        emit(B_SYM_NODE, 0, 0, 0, 0, big, bn);
        emit_tick(big, 0);
    }
    // call-level maps: a box-begin block per member, box-reduce blocks, copy blocks
    c.box_begin = (int)map.size();
    for (int i = 0; i < nm; ++i) map.push_back(make_int2(entry_of(act[i], 1), 0));
    c.n_begin = nm;
    c.box_red = (int)map.size();
    for (int i = 0; i < nm; ++i) {
        const int nb = box_reduce_dims(H(i)->n).grid;
        for (int j = 0; j < nb; ++j) map.push_back(make_int2(entry_of(act[i], 1), j));
    }
    c.n_red = (int)map.size() - c.box_red;
    c.copy = (int)map.size();
    for (int i = 0; i < nm; ++i) {
        const int nb = (H(i)->n + kThreads * 8 - 1) / (kThreads * 8);
        for (int j = 0; j < nb; ++j) map.push_back(make_int2(entry_of(act[i], 1), j));
    }
    c.n_copy = (int)map.size() - c.copy;
}

// The composition of the members in slots `act` at k values ks: an existing
// one, or a new one whose maps are copied into the arena (asynchronously, from
// the composition's host copy). A full arena is reset after a
// synchronisation of the stream (its regions may be read by enqueued work).
// Returns the index in b->comps or -1.
int get_comp(tfdp_batch* b, const std::vector<int>& act, const std::vector<int>& ks, hipStream_t s,
             tfdp_status* st) {
    *st = TFDP_OK;
    std::vector<long long> key;
    key.reserve(act.size() * 4);
    for (size_t i = 0; i < act.size(); ++i) {
        const tfdp_layout* h = b->slot[act[i]];
        key.push_back(act[i]);
        key.push_back((long long)h->uid);
        key.push_back(h->p.n_int);
        key.push_back(ks[i]);
    }
    for (size_t ci = 0; ci < b->comps.size(); ++ci)
        if (b->comps[ci].key == key) {
            b->comps[ci].last_use = ++b->clock;
            return (int)ci;
        }
    Comp c;
    c.key = std::move(key);
    build_comp(b, act, ks, c);
    const size_t need = c.host_map.size();
    if (need > b->arena_cap) {
        set_msg("batch workspace too small: this composition needs " + std::to_string(need) +
                " map entries, the workspace holds " + std::to_string(b->arena_cap));
        *st = TFDP_ERR_WORKSPACE;
        return -1;
    }
    if (b->arena_used + need > b->arena_cap || (int)b->comps.size() >= kMaxComps) {
        *st = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
        if (*st != TFDP_OK) return -1;
        drop_comps(b);
    }
    c.off = b->arena_used;
    b->arena_used += need;
    if (need > 0) {
        *st = check_hip(hipMemcpyAsync(b->d_arena + c.off, c.host_map.data(), need * sizeof(int2),
                                       hipMemcpyHostToDevice, s), "hipMemcpyAsync");
        if (*st != TFDP_OK) return -1;
    }
    c.last_use = ++b->clock;
    b->comps.push_back(std::move(c));
    return (int)b->comps.size() - 1;
}

// Iteration j of the call (the kernels read each member's counter at the
// start of the call from the device and add j).
// Second stream of the batch and its two events, created on first use on
// the batch's device; false (one stream) if they cannot be created.
bool use_side(tfdp_batch* b) {
    if (b->side) return true;
    if (b->side_failed) return false;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) cur = -1;
    if (cur != b->device) (void)hipSetDevice(b->device);
    bool ok = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming) == hipSuccess;
    if (cur >= 0 && cur != b->device) (void)hipSetDevice(cur);
    if (!ok) {
        if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
        if (b->ev_join) (void)hipEventDestroy(b->ev_join);
        if (b->side) (void)hipStreamDestroy(b->side);
        b->side = nullptr;
        b->ev_fork = b->ev_join = nullptr;
        b->side_failed = true;
        (void)hipGetLastError();
    }
    return ok;
}

void enqueue_iter(tfdp_batch* b, const Comp& c, int j, hipStream_t s) {
    const Member* mem = b->d_mem;
    const int2* base = b->d_arena + c.off;
    // the second stream starts after the binning (the grid passes of the
    // other lengths need it) and joins before the edge pass; only in batches
    // that capture their iterations: launched directly, every iteration pays
    // the fork and join as API calls and waits between hardware queues
    // (serving loop, where other streams also step batches: p50 / p99 at
    // 0.8x load 30 / 223 ms with one stream against 67 / 323 ms with two)
    bool side = false;
    for (const BLaunch& L : c.launches) side = side || L.lane == 1;
    side = side && b->graphs && use_side(b);
    bool forked = false;
    for (const BLaunch& L : c.launches) {
        const int2* map = base + L.off;
        const bool bin = L.phase == B_BIN_COUNT || L.phase == B_BIN_SCAN || L.phase == B_BIN_SCATTER;
        if (side && !forked && !bin && !(L.phase == B_EDGES && L.lane == 0)) {
            (void)hipEventRecord(b->ev_fork, s);
            (void)hipStreamWaitEvent(b->side, b->ev_fork, 0);
            forked = true;
        }
        if (forked && L.phase == B_EDGES && L.lane == 0) {  // the edge pass needs every grid
            (void)hipEventRecord(b->ev_join, b->side);
            (void)hipStreamWaitEvent(s, b->ev_join, 0);
            forked = false;
            side = false;
        }
        const hipStream_t ls = (forked && L.lane == 1) ? b->side : s;
        switch (L.phase) {
            case B_BIN_COUNT: launch_b_bin_count(mem, map, L.blocks, L.lds, b->d_t, j, ls); break;
            case B_BIN_SCAN: launch_b_bin_scan(mem, map, L.blocks, b->d_t, j, ls); break;
            case B_BIN_SCATTER: launch_b_bin_scatter(mem, map, L.blocks, L.lds, j, ls); break;
            case B_SPREAD: launch_b_spread(L.k, L.len, L.nw, mem, map, L.blocks, L.lds, ls); break;
            case B_ROWFFT: launch_b_rowfft(L.len, L.nw, mem, map, L.blocks, ls); break;
            case B_COLCONV: launch_b_colconv(L.len, L.nw, mem, map, L.blocks, ls); break;
            case B_ROWIFFT: launch_b_rowifft(L.len, L.nw, mem, map, L.blocks, ls); break;
            case B_EDGES: launch_b_edges(L.k, mem, map, L.blocks, b->d_t, j, ls); break;
            case B_BRUTE: launch_b_brute(mem, map, L.blocks, j, ls); break;
            case B_SYM_PAIRS: launch_b_sym_pairs(mem, map, L.blocks, j, ls); break;
            case B_SYM_NODE: launch_b_sym_node(mem, map, L.blocks, j, ls); break;
            default: launch_b_tick(mem, map, L.blocks, ls); break;
        }
    }
    if (forked) {
        (void)hipEventRecord(b->ev_join, b->side);
        (void)hipStreamWaitEvent(s, b->ev_join, 0);
    }
}

// Graph of `iters` (2 or kGraphIters) iterations of composition c starting
// at a j of parity jpar (the kernels use j only through its parity), captured
// the second time it is needed; nullptr: launch directly.
hipGraphExec_t group_graph(tfdp_batch* b, Comp& c, int iters, int jpar, hipStream_t s) {
    const int gi = 2 * (iters == 2 ? 0 : 1) + jpar;
    hipGraphExec_t& ex = c.gexec[gi];
    if (ex) return ex;
    if (++c.wanted[gi] < 2) return nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) return nullptr;
    for (int i = 0; i < iters; ++i) enqueue_iter(b, c, jpar + i, s);
    hipGraph_t graph = nullptr;
    if (hipStreamEndCapture(s, &graph) != hipSuccess || !graph) return nullptr;
    if (hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0) != hipSuccess) ex = nullptr;
    (void)hipGraphDestroy(graph);
    return ex;
}

}  // namespace

extern "C" {

size_t tfdp_batch_workspace_size(int32_t capacity, int64_t map_entries) {
    if (capacity < 1 || map_entries < 0) return 0;
    const size_t arena = std::max((size_t)map_entries, kMinArena);
    return entries_bytes(capacity) + counters_bytes(capacity) + align256(arena * sizeof(int2));
}

tfdp_status tfdp_batch_create(tfdp_batch** out, int32_t capacity, void* d_ws, size_t ws_bytes) {
    set_msg("");
    if (!out || capacity < 1) {
        set_msg("invalid output pointer or capacity");
        return TFDP_ERR_INVALID_ARG;
    }
    *out = nullptr;
    const size_t fixed = entries_bytes(capacity) + counters_bytes(capacity);
    if (!d_ws || ws_bytes < tfdp_batch_workspace_size(capacity, 0) || (reinterpret_cast<uintptr_t>(d_ws) & 255u)) {
        set_msg("batch workspace missing, not 256-byte aligned or smaller than tfdp_batch_workspace_size(capacity, 0)");
        return TFDP_ERR_WORKSPACE;
    }
    tfdp_batch* b = new (std::nothrow) tfdp_batch();
    if (!b) {
        set_msg("out of host memory");
        return TFDP_ERR_INVALID_ARG;
    }
    char* base = static_cast<char*>(d_ws);
    b->cap = capacity;
    b->slot.assign((size_t)capacity, nullptr);
    b->seen_uid.assign((size_t)capacity, 0);
    b->seen.assign((size_t)capacity, 0);
    b->t_dev.assign((size_t)capacity, 0);
    b->count = 0;
    b->counters_ready = false;
    b->d_mem = reinterpret_cast<Member*>(base);
    b->d_t = reinterpret_cast<int*>(base + entries_bytes(capacity));
    b->d_arena = reinterpret_cast<int2*>(base + fixed);
    b->arena_cap = (ws_bytes - fixed) / sizeof(int2);
    b->arena_used = 0;
    b->graphs = true;
    b->clock = 0;
    if (hipGetDevice(&b->device) != hipSuccess) b->device = 0;
    b->side = nullptr;
    b->ev_fork = b->ev_join = nullptr;
    b->side_failed = false;
    for (int i = 0; i < 9; ++i) b->tiles[i] = make_int2(batch_rows_default(kLens[i]), batch_groups_default(kLens[i]));
    *out = b;
    return TFDP_OK;
}

tfdp_status tfdp_batch_set_tiles(tfdp_batch* b, int32_t fft_length, int32_t rows_per_block, int32_t column_groups,
                                 hipStream_t stream) {
    if (!b) {
        set_msg("invalid batch handle");
        return TFDP_ERR_INVALID_ARG;
    }
    const int li = len_index(fft_length);
    if (kLens[li] != fft_length) {
        set_msg("fft_length must be one of 64, 128, 256, 384, 512, 768, 1024, 1536, 2048");
        return TFDP_ERR_INVALID_ARG;
    }
    const int rows = rows_per_block > 0 ? rows_per_block : batch_rows_default(fft_length);
    const int groups = column_groups > 0 ? column_groups : batch_groups_default(fft_length);
    if (!batch_tile_valid(fft_length, rows, groups)) {
        set_msg("tile not available for this FFT length (rows 2, 4, 8 and column groups 1, 2 up to length 768; "
                "the default tile above)");
        return TFDP_ERR_UNSUPPORTED;
    }
    set_msg("");
    if (b->tiles[li].x == rows && b->tiles[li].y == groups) return TFDP_OK;
    // the maps of every composition change: drop them once enqueued work is done
    tfdp_status st = check_hip(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (st != TFDP_OK) return st;
    drop_comps(b);
    b->tiles[li] = make_int2(rows, groups);
    return TFDP_OK;
}

tfdp_status tfdp_batch_get_tiles(const tfdp_batch* b, int32_t fft_length, int32_t* rows_per_block,
                                 int32_t* column_groups) {
    if (!b || !rows_per_block || !column_groups) {
        set_msg("invalid batch handle or pointer");
        return TFDP_ERR_INVALID_ARG;
    }
    const int li = len_index(fft_length);
    if (kLens[li] != fft_length) {
        set_msg("fft_length must be one of 64, 128, 256, 384, 512, 768, 1024, 1536, 2048");
        return TFDP_ERR_INVALID_ARG;
    }
    *rows_per_block = b->tiles[li].x;
    *column_groups = b->tiles[li].y;
    return TFDP_OK;
}

tfdp_status tfdp_batch_add(tfdp_batch* b, tfdp_layout* h) {
    set_msg("");
    if (!b || !h) {
        set_msg("invalid batch or layout handle");
        return TFDP_ERR_INVALID_ARG;
    }
    if (std::find(b->slot.begin(), b->slot.end(), h) != b->slot.end()) {
        set_msg("the layout is already a member of this batch");
        return TFDP_ERR_INVALID_ARG;
    }
    if (b->count >= b->cap) {
        set_msg("the batch is full");
        return TFDP_ERR_UNSUPPORTED;
    }
    if (h->lay.nslices != 1) {
        set_msg("batched stepping needs a single edge-pass column slice");
        return TFDP_ERR_UNSUPPORTED;
    }
    if (h->auto_grid) {
        set_msg("batched stepping needs a fixed grid (n_int > 0)");
        return TFDP_ERR_UNSUPPORTED;
    }
    const int sl = (int)(std::find(b->slot.begin(), b->slot.end(), nullptr) - b->slot.begin());
    b->slot[sl] = h;
    b->seen_uid[sl] = 0;  // entries written at the next step
    b->count += 1;
    return TFDP_OK;
}

tfdp_status tfdp_batch_remove(tfdp_batch* b, tfdp_layout* h) {
    set_msg("");
    if (!b || !h) {
        set_msg("invalid batch or layout handle");
        return TFDP_ERR_INVALID_ARG;
    }
    auto it = std::find(b->slot.begin(), b->slot.end(), h);
    if (it == b->slot.end()) {
        set_msg("the layout is not a member of this batch");
        return TFDP_ERR_INVALID_ARG;
    }
    *it = nullptr;
    b->count -= 1;
    return TFDP_OK;
}

int32_t tfdp_batch_count(const tfdp_batch* b) { return b ? (int32_t)b->count : 0; }

tfdp_status tfdp_batch_set_graphs(tfdp_batch* b, int32_t enable) {
    if (!b) {
        set_msg("invalid batch handle");
        return TFDP_ERR_INVALID_ARG;
    }
    b->graphs = enable != 0;
    if (!b->graphs) drop_comp_graphs(b);
    return TFDP_OK;
}

tfdp_status tfdp_batch_step(tfdp_batch* b, int32_t iters, hipStream_t s) {
    if (!b || iters < 0) {
        set_msg("invalid batch handle or iteration count");
        return TFDP_ERR_INVALID_ARG;
    }
    set_msg("");
    if (iters == 0 || b->count == 0) return TFDP_OK;
    std::vector<int> act;
    for (int sl = 0; sl < b->cap; ++sl)
        if (b->slot[sl]) act.push_back(sl);
    const int nm = (int)act.size();
    // a single member steps by the plain call: the same results (the batched
    // launches run the plain kernels' code), with the plain passes' tiles and
    // schedule, which suit one graph better (the batched row passes take more
    // rows per block to fill the chip with many graphs); its device counter
    // is written again by the next batched call
    if (nm == 1) return tfdp_layout_step(b->slot[act[0]], iters, s);
    if (!b->counters_ready) {
        hipLaunchKernelGGL(kb_zero_counters, dim3((b->cap + 255) / 256), dim3(256), 0, s, b->d_t, b->cap);
        std::fill(b->t_dev.begin(), b->t_dev.end(), 0);
        b->counters_ready = true;
    }
    // entries of new members and of members whose parameters changed, and
    // counters moved by the plain API, written by kernels (stream order keeps
    // them after every launch enqueued earlier)
    CounterSet cs;
    cs.count = 0;
    for (int sl : act) {
        tfdp_layout* h = b->slot[sl];
        enqueue_twiddles(h, s);
        if (b->seen_uid[sl] != h->uid || b->seen[sl] != h->version) {
            MemberEntries e;
            for (int k = 1; k <= 3; ++k) e.e[k - 1] = make_member(h, sl, k <= h->k_ws ? k : h->k_ws);
            hipLaunchKernelGGL(kb_set_entries, dim3(1), dim3(64), 0, s, b->d_mem + (size_t)sl * 3, e);
            b->seen_uid[sl] = h->uid;
            b->seen[sl] = h->version;
        }
        if (b->t_dev[sl] != h->t) {
            cs.v[cs.count++] = make_int2(sl, h->t);
            b->t_dev[sl] = h->t;
            if (cs.count == kCounterSet) {
                hipLaunchKernelGGL(kb_set_counters, dim3(1), dim3(256), 0, s, b->d_t, cs);
                cs.count = 0;
            }
        }
    }
    if (cs.count > 0) hipLaunchKernelGGL(kb_set_counters, dim3(1), dim3(256), 0, s, b->d_t, cs);
    tfdp_status st = TFDP_OK;
    std::vector<int> ks((size_t)nm);
    for (int i = 0; i < nm; ++i) ks[i] = k_at(b->slot[act[i]]->p, b->slot[act[i]]->t);
    int ci = get_comp(b, act, ks, s, &st);
    if (ci < 0) return st;
    {
        const Comp& c = b->comps[ci];
        const int2* base = b->d_arena + c.off;
        launch_b_box(b->d_mem, base + c.box_begin, c.n_begin, base + c.box_red, c.n_red, b->d_t, s);
    }
    int j = 0;
    while (j < iters) {
        for (int i = 0; i < nm; ++i) ks[i] = k_at(b->slot[act[i]]->p, b->slot[act[i]]->t + j);
        ci = get_comp(b, act, ks, s, &st);
        if (ci < 0) return st;
        // a group when every member keeps its k over the next G iterations
        // (the schedule never lowers k: the last one decides)
        auto same_k_through = [&](int last) {
            if (last >= iters) return false;
            for (int i = 0; i < nm; ++i)
                if (k_at(b->slot[act[i]]->p, b->slot[act[i]]->t + last) != ks[i]) return false;
            return true;
        };
        int G = 1;
        if (same_k_through(j + kGraphIters - 1))
            G = kGraphIters;
        else if (same_k_through(j + 1))
            G = 2;
        Comp& c = b->comps[ci];
        hipGraphExec_t ex = (b->graphs && G > 1) ? group_graph(b, c, G, j & 1, s) : nullptr;
        if (ex) {
            st = check_hip(hipGraphLaunch(ex, s), "hipGraphLaunch");
            if (st != TFDP_OK) return st;
        } else {
            (void)hipGetLastError();
            for (int i = 0; i < G; ++i) enqueue_iter(b, c, j + i, s);
        }
        j += G;
    }
    if (iters & 1) {
        const Comp& c = b->comps[ci];
        launch_b_copy(b->d_mem, b->d_arena + c.off + c.copy, c.n_copy, s);
    }
    launch_b_advance(b->d_t, b->cap, iters, s);
    for (int sl = 0; sl < b->cap; ++sl) b->t_dev[sl] += iters;
    for (int sl : act) b->slot[sl]->t += iters;
    return check_hip(hipGetLastError(), "kernel launch");
}

void tfdp_batch_destroy(tfdp_batch* b) {
    if (!b) return;
    drop_comps(b);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    if (b->side) (void)hipStreamDestroy(b->side);
    delete b;
}

}  // extern "C"
