// Host side of the batched C ABI (tfdp_batch_*): many layout handles stepped
// together. Every phase of an iteration is one launch per class of graphs
// (graphs in a class share the kernel template: k, FFT length and spreading
// block shape) whose blocks are listed in a device map {member entry, block};
// each block runs the plain kernel's body for that graph and block, so the
// result of every graph is bit-identical to tfdp_layout_step on it alone.
// Groups of eight (else two) iterations of one composition (the k of every
// member) are captured as HIP graphs.
#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "tfdp_handle.h"

using namespace tfdp;

namespace {

enum BPhase { B_BIN_COUNT, B_BIN_SCAN, B_BIN_SCATTER, B_SPREAD, B_ROWFFT, B_COLCONV, B_ROWIFFT, B_EDGES, B_BRUTE };

struct BLaunch {
    int phase;
    int k, len, nw;  // B_BRUTE: nw = offset of the tick map (one entry per member), k = members
    size_t off;       // first map entry
    int blocks;
    size_t lds;
};

// One composition: the k of every member and the launches of an iteration.
struct Comp {
    std::vector<int> ks;            // k per slot (0: exact method)
    std::vector<BLaunch> launches;  // one iteration, in dependency order
    int2* d_map = nullptr;
    // captured groups of 2 and kGraphIters iterations starting at an even /
    // odd j: [2 * (size == kGraphIters) + parity of j]
    hipGraphExec_t gexec[4] = {nullptr, nullptr, nullptr, nullptr};
    unsigned long long last_use = 0;
};

constexpr int kMaxComps = 8;

int entry_of(int slot, int k) { return slot * 3 + (k - 1); }

}  // namespace

struct tfdp_batch {
    int cap;
    std::vector<tfdp_layout*> mem;   // members in slot order
    std::vector<unsigned int> seen;  // member version when its entries were written
    std::vector<int2> geo;           // member {n_int, k range} when the maps were built
    std::vector<int> t_dev;          // counter the device holds per slot for the next call
    Member* d_mem;                   // [cap][3] entries for k = 1..3
    int* d_t;                        // [cap] counters at the start of a call
    int2* d_fixed;                   // maps of the box begin, box reduce and final copy
    size_t fixed_cap;
    int n_begin, n_red, n_copy;
    bool dirty;  // membership changed since the entries were written
    bool graphs;
    std::vector<Comp> comps;
    unsigned long long clock;
};

namespace {

tfdp_status upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return TFDP_OK;
    tfdp_status st = check_hip(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    if (st == TFDP_OK) st = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    return st;
}

Member make_member(const tfdp_layout* h, int slot, int k) {
    Member m;
    std::memset(&m, 0, sizeof(m));
    m.b = bufs_for(h, k);
    m.g = make_geom(h->p.n_int, k);
    m.a = model_args(h);
    m.es = h->lay.slice[0];
    m.pos = reinterpret_cast<float2*>(h->pos);
    m.alt = h->lay.pos_alt;
    m.slot = slot;
    spread_dims(m.b, m.g, &m.nw, &m.nkb);
    rowfft_dims(m.g, &m.nqb, true);
    rowifft_dims(m.g, &m.nrb, true);
    m.box_blocks = box_reduce_dims(h->n).grid;
    return m;
}

tfdp_status write_entries(tfdp_batch* b, int slot, hipStream_t s) {
    const tfdp_layout* h = b->mem[slot];
    Member e[3];
    for (int k = 1; k <= 3; ++k) e[k - 1] = make_member(h, slot, k <= h->k_ws ? k : h->k_ws);
    b->seen[slot] = h->version;
    b->geo[slot] = make_int2(h->p.n_int, h->k_ws);
    return upload(b->d_mem + (size_t)slot * 3, e, sizeof(e), s);
}

void free_comp(Comp& c) {
    for (hipGraphExec_t& g : c.gexec)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    if (c.d_map) (void)hipFree(c.d_map);
    c.d_map = nullptr;
}

void drop_comps(tfdp_batch* b) {
    for (Comp& c : b->comps) free_comp(c);
    b->comps.clear();
}

void drop_comp_graphs(tfdp_batch* b) {
    for (Comp& c : b->comps)
        for (hipGraphExec_t& g : c.gexec)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
}

// Entries, counters and the fixed maps after a membership change.
tfdp_status rebuild(tfdp_batch* b, hipStream_t s) {
    tfdp_status st = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (st != TFDP_OK) return st;
    drop_comps(b);
    const int nm = (int)b->mem.size();
    std::vector<Member> ent((size_t)nm * 3);
    for (int i = 0; i < nm; ++i) {
        const tfdp_layout* h = b->mem[i];
        for (int k = 1; k <= 3; ++k) ent[(size_t)i * 3 + k - 1] = make_member(h, i, k <= h->k_ws ? k : h->k_ws);
        b->seen[i] = h->version;
        b->geo[i] = make_int2(h->p.n_int, h->k_ws);
    }
    st = upload(b->d_mem, ent.data(), ent.size() * sizeof(Member), s);
    if (st != TFDP_OK) return st;
    std::vector<int> tv((size_t)nm);
    for (int i = 0; i < nm; ++i) tv[i] = b->mem[i]->t;
    st = upload(b->d_t, tv.data(), tv.size() * sizeof(int), s);
    if (st != TFDP_OK) return st;
    b->t_dev = tv;
    // fixed maps: one box-begin block per member, box-reduce blocks, copy blocks
    std::vector<int2> fm;
    for (int i = 0; i < nm; ++i) fm.push_back(make_int2(entry_of(i, 1), 0));
    b->n_begin = nm;
    for (int i = 0; i < nm; ++i) {
        const int nb = box_reduce_dims(b->mem[i]->n).grid;
        for (int j = 0; j < nb; ++j) fm.push_back(make_int2(entry_of(i, 1), j));
    }
    b->n_red = (int)fm.size() - b->n_begin;
    for (int i = 0; i < nm; ++i) {
        const int nb = (b->mem[i]->n + kThreads * 8 - 1) / (kThreads * 8);
        for (int j = 0; j < nb; ++j) fm.push_back(make_int2(entry_of(i, 1), j));
    }
    b->n_copy = (int)fm.size() - b->n_begin - b->n_red;
    if (fm.size() > b->fixed_cap) {
        if (b->d_fixed) (void)hipFree(b->d_fixed);
        b->d_fixed = nullptr;
        b->fixed_cap = 0;
        st = check_hip(hipMalloc(&b->d_fixed, fm.size() * sizeof(int2)), "hipMalloc");
        if (st != TFDP_OK) return st;
        b->fixed_cap = fm.size();
    }
    st = upload(b->d_fixed, fm.data(), fm.size() * sizeof(int2), s);
    if (st != TFDP_OK) return st;
    b->dirty = false;
    return TFDP_OK;
}

// Work of a member in a phase, for the block order of a launch: the biggest
// graphs' blocks are dispatched first so that they do not form the tail.
long long member_work(const tfdp_layout* h) { return (long long)h->n + h->nnz; }

tfdp_status build_comp(tfdp_batch* b, const std::vector<int>& ks, hipStream_t s, Comp& c) {
    c.ks = ks;
    const int nm = (int)b->mem.size();
    std::vector<int> order, brute;
    for (int i = 0; i < nm; ++i) (ks[i] == 0 ? brute : order).push_back(i);
    auto bigger_first = [&](int x, int y) { return member_work(b->mem[x]) > member_work(b->mem[y]); };
    std::stable_sort(order.begin(), order.end(), bigger_first);
    std::stable_sort(brute.begin(), brute.end(), bigger_first);
    std::vector<int2> map;
    auto emit = [&](int phase, int k, int len, int nw, size_t lds, const std::vector<int>& who,
                    const std::vector<int>& blocks) {
        BLaunch L{phase, k, len, nw, map.size(), 0, lds};
        for (size_t q = 0; q < who.size(); ++q)
            for (int j = 0; j < blocks[q]; ++j)
                map.push_back(make_int2(entry_of(who[q], ks[who[q]] > 0 ? ks[who[q]] : 1), j));
        L.blocks = (int)(map.size() - L.off);
        if (L.blocks > 0) c.launches.push_back(L);
    };
    // binning (k-independent shapes): one launch each for all members
    {
        std::vector<int> bc, bs, bsc;
        size_t lds_c = 0, lds_s = 0;
        for (int i : order) {
            const Bufs bb = bufs_for(b->mem[i], ks[i]);
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
            const tfdp_layout* h = b->mem[i];
            const Geom g = make_geom(h->p.n_int, ks[i]);
            int nw, nkb;
            spread_dims(bufs_for(h, ks[i]), g, &nw, &nkb);
            cls[std::make_tuple(ks[i], g.L, nw)].push_back(i);
        }
        for (auto& kv : cls) {
            std::vector<int> blocks;
            size_t lds = 0;
            for (int i : kv.second) {
                const tfdp_layout* h = b->mem[i];
                int nw, nkb;
                const Dims d = spread_dims(bufs_for(h, ks[i]), make_geom(h->p.n_int, ks[i]), &nw, &nkb);
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
        for (int i : order) cls[make_geom(b->mem[i]->p.n_int, ks[i]).L].push_back(i);
        for (int phase : {B_ROWFFT, B_COLCONV, B_ROWIFFT})
            for (auto& kv : cls) {
                std::vector<int> blocks;
                for (int i : kv.second) {
                    const Geom g = make_geom(b->mem[i]->p.n_int, ks[i]);
                    int nb = 0;
                    if (phase == B_ROWFFT)
                        rowfft_dims(g, &nb, true);
                    else if (phase == B_COLCONV)
                        nb = colconv_dims(g, true).grid;
                    else
                        rowifft_dims(g, &nb, true);
                    blocks.push_back(nb);
                }
                emit(phase, 0, kv.first, 0, 0, kv.second, blocks);
            }
    }
    // edge pass + gather + move: classes by k
    {
        std::map<int, std::vector<int>> cls;
        for (int i : order) cls[ks[i]].push_back(i);
        for (auto& kv : cls) {
            std::vector<int> blocks;
            for (int i : kv.second) blocks.push_back(b->mem[i]->lay.slice[0].blocks);
            emit(B_EDGES, kv.first, 0, 0, 0, kv.second, blocks);
        }
    }
    // exact method: one launch for all such members, then their counters
    if (!brute.empty()) {
        std::vector<int> blocks;
        for (int i : brute) blocks.push_back((b->mem[i]->n + kBruteRows - 1) / kBruteRows);
        const size_t tick = map.size();
        for (int i : brute) map.push_back(make_int2(entry_of(i, 1), 0));
        emit(B_BRUTE, (int)brute.size(), 0, (int)tick, 0, brute, blocks);
    }
    if (!map.empty()) {
        tfdp_status st = check_hip(hipMalloc(&c.d_map, map.size() * sizeof(int2)), "hipMalloc");
        if (st != TFDP_OK) return st;
        st = upload(c.d_map, map.data(), map.size() * sizeof(int2), s);
        if (st != TFDP_OK) return st;
    }
    return TFDP_OK;
}

Comp* get_comp(tfdp_batch* b, const std::vector<int>& ks, hipStream_t s, tfdp_status* st) {
    *st = TFDP_OK;
    for (Comp& c : b->comps)
        if (c.ks == ks) {
            c.last_use = ++b->clock;
            return &c;
        }
    if ((int)b->comps.size() >= kMaxComps) {
        *st = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
        if (*st != TFDP_OK) return nullptr;
        auto lru = std::min_element(b->comps.begin(), b->comps.end(),
                                    [](const Comp& x, const Comp& y) { return x.last_use < y.last_use; });
        free_comp(*lru);
        b->comps.erase(lru);
    }
    b->comps.emplace_back();
    Comp& c = b->comps.back();
    *st = build_comp(b, ks, s, c);
    if (*st != TFDP_OK) {
        free_comp(c);
        b->comps.pop_back();
        return nullptr;
    }
    c.last_use = ++b->clock;
    return &c;
}

// Iteration j of the call (the kernels read each member's counter at the
// start of the call from the device and add j).
void enqueue_iter(tfdp_batch* b, const Comp& c, int j, hipStream_t s) {
    const Member* mem = b->d_mem;
    for (const BLaunch& L : c.launches) {
        const int2* map = c.d_map + L.off;
        switch (L.phase) {
            case B_BIN_COUNT: launch_b_bin_count(mem, map, L.blocks, L.lds, b->d_t, j, s); break;
            case B_BIN_SCAN: launch_b_bin_scan(mem, map, L.blocks, b->d_t, j, s); break;
            case B_BIN_SCATTER: launch_b_bin_scatter(mem, map, L.blocks, L.lds, j, s); break;
            case B_SPREAD: launch_b_spread(L.k, L.len, L.nw, mem, map, L.blocks, L.lds, s); break;
            case B_ROWFFT: launch_b_rowfft(L.len, mem, map, L.blocks, s); break;
            case B_COLCONV: launch_b_colconv(L.len, mem, map, L.blocks, s); break;
            case B_ROWIFFT: launch_b_rowifft(L.len, mem, map, L.blocks, s); break;
            case B_EDGES: launch_b_edges(L.k, mem, map, L.blocks, b->d_t, j, s); break;
            default: launch_b_brute(mem, map, L.blocks, c.d_map + L.nw, L.k, j, s); break;
        }
    }
}

// Graph of `iters` (2 or kGraphIters) iterations of composition c starting
// at a j of parity jpar (the kernels use j only through its parity).
hipGraphExec_t group_graph(tfdp_batch* b, Comp& c, int iters, int jpar, hipStream_t s) {
    hipGraphExec_t& ex = c.gexec[2 * (iters == 2 ? 0 : 1) + jpar];
    if (ex) return ex;
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

tfdp_status tfdp_batch_create(tfdp_batch** out, int32_t capacity) {
    set_msg("");
    if (!out || capacity < 1) {
        set_msg("invalid output pointer or capacity");
        return TFDP_ERR_INVALID_ARG;
    }
    *out = nullptr;
    tfdp_batch* b = new (std::nothrow) tfdp_batch();
    if (!b) {
        set_msg("out of host memory");
        return TFDP_ERR_INVALID_ARG;
    }
    b->cap = capacity;
    b->d_mem = nullptr;
    b->d_t = nullptr;
    b->d_fixed = nullptr;
    b->fixed_cap = 0;
    b->n_begin = b->n_red = b->n_copy = 0;
    b->dirty = true;
    b->graphs = true;
    b->clock = 0;
    *out = b;
    return TFDP_OK;
}

tfdp_status tfdp_batch_add(tfdp_batch* b, tfdp_layout* h) {
    set_msg("");
    if (!b || !h) {
        set_msg("invalid batch or layout handle");
        return TFDP_ERR_INVALID_ARG;
    }
    if (std::find(b->mem.begin(), b->mem.end(), h) != b->mem.end()) {
        set_msg("the layout is already a member of this batch");
        return TFDP_ERR_INVALID_ARG;
    }
    if ((int)b->mem.size() >= b->cap) {
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
    b->mem.push_back(h);
    b->seen.push_back(0);
    b->geo.push_back(make_int2(0, 0));
    b->dirty = true;
    return TFDP_OK;
}

tfdp_status tfdp_batch_remove(tfdp_batch* b, tfdp_layout* h) {
    set_msg("");
    if (!b || !h) {
        set_msg("invalid batch or layout handle");
        return TFDP_ERR_INVALID_ARG;
    }
    auto it = std::find(b->mem.begin(), b->mem.end(), h);
    if (it == b->mem.end()) {
        set_msg("the layout is not a member of this batch");
        return TFDP_ERR_INVALID_ARG;
    }
    b->seen.erase(b->seen.begin() + (it - b->mem.begin()));
    b->geo.erase(b->geo.begin() + (it - b->mem.begin()));
    b->mem.erase(it);
    b->dirty = true;
    return TFDP_OK;
}

int32_t tfdp_batch_count(const tfdp_batch* b) { return b ? (int32_t)b->mem.size() : 0; }

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
    const int nm = (int)b->mem.size();
    if (iters == 0 || nm == 0) return TFDP_OK;
    tfdp_status st = TFDP_OK;
    if (!b->d_mem) {
        st = check_hip(hipMalloc(&b->d_mem, (size_t)b->cap * 3 * sizeof(Member)), "hipMalloc");
        if (st == TFDP_OK) st = check_hip(hipMalloc(&b->d_t, (size_t)b->cap * sizeof(int)), "hipMalloc");
        if (st != TFDP_OK) return st;
    }
    // a new grid of a member changes the launch shapes: rebuild everything
    for (int i = 0; i < nm && !b->dirty; ++i)
        if (b->mem[i]->p.n_int != b->geo[i].x || b->mem[i]->k_ws != b->geo[i].y) b->dirty = true;
    for (int i = 0; i < nm; ++i) enqueue_twiddles(b->mem[i], s);
    if (b->dirty) {
        st = rebuild(b, s);
        if (st != TFDP_OK) return st;
    } else {
        // parameter changes: rewrite those members' entries; counters moved
        // by the plain API: upload all counters
        bool t_moved = false;
        for (int i = 0; i < nm; ++i) {
            if (b->mem[i]->version != b->seen[i]) {
                st = write_entries(b, i, s);
                if (st != TFDP_OK) return st;
            }
            if (b->mem[i]->t != b->t_dev[i]) t_moved = true;
        }
        if (t_moved) {
            std::vector<int> tv((size_t)nm);
            for (int i = 0; i < nm; ++i) tv[i] = b->mem[i]->t;
            st = upload(b->d_t, tv.data(), tv.size() * sizeof(int), s);
            if (st != TFDP_OK) return st;
            b->t_dev = tv;
        }
    }
    launch_b_box(b->d_mem, b->d_fixed, b->n_begin, b->d_fixed + b->n_begin, b->n_red, b->d_t, s);
    std::vector<int> ks((size_t)nm), kn((size_t)nm);
    int j = 0;
    while (j < iters) {
        for (int i = 0; i < nm; ++i) ks[i] = k_at(b->mem[i]->p, b->mem[i]->t + j);
        Comp* c = get_comp(b, ks, s, &st);
        if (!c) return st;
        // a captured group when every member keeps its k over the next G
        // iterations (the schedule never lowers k: the last one decides)
        auto same_k_through = [&](int last) {
            if (last >= iters) return false;
            for (int i = 0; i < nm; ++i)
                if (k_at(b->mem[i]->p, b->mem[i]->t + last) != ks[i]) return false;
            return true;
        };
        int G = 0;
        if (b->graphs) {
            if (same_k_through(j + kGraphIters - 1))
                G = kGraphIters;
            else if (same_k_through(j + 1))
                G = 2;
        }
        if (G > 0) {
            hipGraphExec_t ex = group_graph(b, *c, G, j & 1, s);
            if (ex) {
                st = check_hip(hipGraphLaunch(ex, s), "hipGraphLaunch");
                if (st != TFDP_OK) return st;
                j += G;
                continue;
            }
            (void)hipGetLastError();
        }
        enqueue_iter(b, *c, j, s);
        ++j;
    }
    if (iters & 1) launch_b_copy(b->d_mem, b->d_fixed + b->n_begin + b->n_red, b->n_copy, s);
    launch_b_advance(b->d_t, nm, iters, s);
    for (int i = 0; i < nm; ++i) {
        b->mem[i]->t += iters;
        b->t_dev[i] = b->mem[i]->t;
    }
    return check_hip(hipGetLastError(), "kernel launch");
}

void tfdp_batch_destroy(tfdp_batch* b) {
    if (!b) return;
    drop_comps(b);
    if (b->d_fixed) (void)hipFree(b->d_fixed);
    if (b->d_t) (void)hipFree(b->d_t);
    if (b->d_mem) (void)hipFree(b->d_mem);
    delete b;
}

}  // extern "C"
