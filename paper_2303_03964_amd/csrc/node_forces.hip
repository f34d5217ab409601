// Per-node work of one iteration: back-projection of the grid potentials
// (Sec. 3.4, third step), attraction along the CSR rows (Sec. 3.3, Eq.6-7),
// the displacement D = w_r F^r + F^a and the capped move; or, for the exact
// method (Sec. 3.4), the all-pairs repulsion tiled through LDS.
//
// Edge pass schedule (built once at init for each column slice): rows are cut into
// wave groups of at most kGroupRows rows and kGroupEdges CSR entries, packed
// four per block; a row with more than kGroupEdges entries gets a block of
// its own. In a wave group, lane l walks CSR entry e0 + l (coalesced reads of
// packed entries: column plus the row's index in the group), reads its row's
// position from LDS and computes its term; a segmented wave sum adds the terms
// of each row's run into a wave-private LDS accumulator (no float LDS
// atomics, which are several times slower than the rest of the pass on
// gfx950); lane r then finishes row r0 + r. A heavy row is summed by all 256 threads and
// reduced in a fixed order. Every wave handles at most kGroupEdges entries,
// whatever the degree distribution.
#include "tfdp_internal.h"

namespace tfdp {

// Interpolated repulsion at p from the grid potentials (phi_1, G_x, G_y):
// F = sum_g w_g (delta_g phi_1(g) + G(g)) over the K x K nodes of p's interval.
template <int K>
__device__ __forceinline__ void grid_repulsion(const Bufs& b, const Geom& g, const Box& bx, float2 p,
                                               float& frx, float& fry) {
    int cx, cy;
    double tx, ty;
    bin_axis(p.x, bx.lo_x, bx.h, b.n_int, cx, tx);
    bin_axis(p.y, bx.lo_y, bx.h, b.n_int, cy, ty);
    double wx[K], wy[K], dx[K], dy[K];
    lagrange<K>(tx, wx);
    lagrange<K>(ty, wy);
    node_deltas<K>(tx, bx.h, dx);
    node_deltas<K>(ty, bx.h, dy);
    const int M = g.m;
    frx = 0.f;
    fry = 0.f;
#pragma unroll
    for (int bb = 0; bb < K; ++bb) {
        const float4* row = b.pot + (size_t)(cy * K + bb) * M + cx * K;
        const float ddy = (float)dy[bb];
#pragma unroll
        for (int aa = 0; aa < K; ++aa) {
            double wd;
            {
#pragma clang fp contract(off)
                wd = wx[aa] * wy[bb];
            }
            const float w = (float)wd;
            const float4 v = row[aa];
            frx += w * ((float)dx[aa] * v.x + v.y);
            fry += w * (ddy * v.x + v.z);
        }
    }
}

// Segmented inclusive sums of (x, y) over the lanes of a wave whose keys are
// non-decreasing with the lane index (a run of equal keys is a segment):
// afterwards the last lane of every segment holds the segment's sum. Steps of
// 1, 2, 4, 8 lanes inside each 16-lane row by DPP row shifts, then rows 1 and
// 3 take the end of rows 0 and 2, then rows 2 and 3 the end of row 1 (a fixed
// association order, so the sums are reproducible).
template <int N>
__device__ __forceinline__ void seg_step_dpp(float& x, float& y, int key) {
    const int kk = __builtin_amdgcn_update_dpp(-1, key, 0x110 | N, 0xf, 0xf, false);
    const float xx = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x110 | N, 0xf, 0xf, false));
    const float yy = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(y), 0x110 | N, 0xf, 0xf, false));
    if (kk == key) {
        x += xx;
        y += yy;
    }
}

__device__ __forceinline__ void seg_step_lane(float& x, float& y, int key, int lane, int src) {
    const int kk = __shfl(key, src);
    const float xx = __shfl(x, src);
    const float yy = __shfl(y, src);
    if (src != lane && kk == key) {
        x += xx;
        y += yy;
    }
}

__device__ __forceinline__ void wave_segmented_sum(float& x, float& y, int key, int lane) {
    seg_step_dpp<1>(x, y, key);
    seg_step_dpp<2>(x, y, key);
    seg_step_dpp<4>(x, y, key);
    seg_step_dpp<8>(x, y, key);
    seg_step_lane(x, y, key, lane, ((lane >> 4) & 1) ? (lane & ~15) - 1 : lane);
    seg_step_lane(x, y, key, lane, lane >= 32 ? 31 : lane);
}

// Attraction term of one CSR entry: (1 + beta / (1 + tau d^2)) (x_i - x_j)
// (tau = 1: Eq.6; other tau: the generalised t-force of Eq.3).
__device__ __forceinline__ void edge_term(float px, float py, float2 q, float beta, float tau, float& ax,
                                          float& ay) {
    const float dx = px - q.x;
    const float dy = py - q.y;
    const float f = 1.f + beta / (1.f + tau * (dx * dx + dy * dy));
    ax = f * dx;
    ay = f * dy;
}

// Displacement of node i from its repulsion and summed attraction terms;
// writes the force outputs (pos_out == nullptr) or the capped move and
// widens the block's box extremes.
__device__ __forceinline__ void node_output(int i, float2 p, float frx, float fry, float sax, float say,
                                            const ModelArgs& a, int t, DevState* st, float2* __restrict__ pos_out,
                                            float2* f_rep, float2* f_att, float2* f_tot, float& xmin,
                                            float& ymin, float& xmax, float& ymax) {
    const float fax = -a.alpha * sax;
    const float fay = -a.alpha * say;
    // local refinement (Sec. 5): node i's repulsion scaled by rep_w[i]
    const float wr = a.rep_w ? a.rep_weight * a.rep_w[i] : a.rep_weight;
    const float dxt = wr * frx + fax;
    const float dyt = wr * fry + fay;
    if (pos_out == nullptr) {
        if (f_rep) f_rep[i] = make_float2(frx, fry);
        if (f_att) f_att[i] = make_float2(fax, fay);
        if (f_tot) f_tot[i] = make_float2(dxt, dyt);
        return;
    }
    const double c = (double)a.t0 * (1.0 - (double)t / (double)a.total_iters);
    const float cap = c > 0.0 ? (float)c : 0.f;
    const float norm = sqrtf(dxt * dxt + dyt * dyt);
    const float scale = norm > cap ? cap / norm : 1.f;
    const float2 np = make_float2(p.x + dxt * scale, p.y + dyt * scale);
    pos_out[i] = np;
    if (isfinite(np.x) && isfinite(np.y)) {
        xmin = fminf(xmin, np.x);
        xmax = fmaxf(xmax, np.x);
        ymin = fminf(ymin, np.y);
        ymax = fmaxf(ymax, np.y);
    } else {
        st->nonfinite = 1;
    }
}

// Edge pass over one column slice. MODE 0: write the slice's attraction sums
// of every row to fpart; MODE 1: add them to fpart; MODE 2 (last slice): add
// fpart (use_part), gather the repulsion, and write the forces or the move.
// Slicing bounds the neighbour positions read by one launch to one column
// range.
template <int K, int MODE>
__device__ __forceinline__ void edges_body(const float2* __restrict__ pos, float2* __restrict__ pos_out,
                                           const EdgeSlice& es, int use_part, float2* __restrict__ fpart,
                                           const Bufs& b, const Geom& g, const ModelArgs& a, int set,
                                           float2* f_rep, float2* f_att, float2* f_tot, int bid) {
    __shared__ float accx[kThreads];
    __shared__ float accy[kThreads];
    __shared__ float hred[2][kThreads / 64];
    __shared__ float2 pown[kThreads];
    __shared__ float aown[kThreads];
    const int* __restrict__ row_ptr = es.rp;
    const int* __restrict__ col_idx = es.col;
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    accx[threadIdx.x] = 0.f;
    accy[threadIdx.x] = 0.f;
    __syncthreads();
    const int2 s0 = es.sched[4 * bid];
    float xmin = INFINITY, ymin = INFINITY, xmax = -INFINITY, ymax = -INFINITY;
    bool have = false;
    int i = 0;
    float2 p = make_float2(0.f, 0.f);
    float sax = 0.f, say = 0.f;
    if (s0.y < 0) {
        // one row with more than kGroupEdges entries, summed by the whole block;
        // four independent column/neighbour loads in flight per thread
        const int row = s0.x;
        const int e1 = row_ptr[row + 1];
        const float2 pr = pos[row];
        const float* __restrict__ aw = a.att_w;
        const float ai = aw ? aw[row] : 0.f;
        float sx = 0.f, sy = 0.f;
        for (int e = row_ptr[row] + threadIdx.x; e < e1; e += 4 * kThreads) {
            // past the row's end the row itself stands in: its term is zero
            int c[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                c[u] = e + u * kThreads < e1 ? (col_idx[e + u * kThreads] & 0x3ffffff) : row;
            float2 q[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) q[u] = pos[c[u]];
            float wgt[4] = {1.f, 1.f, 1.f, 1.f};
            if (aw) {
#pragma unroll
                for (int u = 0; u < 4; ++u) wgt[u] = 0.5f * (ai + aw[c[u]]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                float ax, ay;
                edge_term(pr.x, pr.y, q[u], a.beta, a.tau, ax, ay);
                sx += wgt[u] * ax;
                sy += wgt[u] * ay;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            sx += __shfl_xor(sx, off);
            sy += __shfl_xor(sy, off);
        }
        if (lane == 0) {
            hred[0][w] = sx;
            hred[1][w] = sy;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            sax = (hred[0][0] + hred[0][1]) + (hred[0][2] + hred[0][3]);
            say = (hred[1][0] + hred[1][1]) + (hred[1][2] + hred[1][3]);
            have = true;
            i = row;
            p = pr;
        }
    } else {
        const int2 gd = es.sched[4 * bid + w];
        const int r0 = gd.x, nr = gd.y;
        if (nr > 0) {
            // positions of the group's rows in LDS; entry e carries its row's
            // index in the group in bits 26..31
            float2* pw = reinterpret_cast<float2*>(pown) + w * 64;
            const float2 po = lane < nr ? pos[r0 + lane] : make_float2(0.f, 0.f);
            pw[lane] = po;
            const float* __restrict__ aw = a.att_w;
            float* awn = aown + w * 64;
            if (aw) awn[lane] = lane < nr ? aw[r0 + lane] : 0.f;
            const int eb = row_ptr[r0];
            const int ee = row_ptr[r0 + nr];
            float* ax_w = accx + w * 64;
            float* ay_w = accy + w * 64;
            __builtin_amdgcn_wave_barrier();
            // all entry reads of the group first, then all neighbour reads:
            // up to kGroupEdges/64 independent loads in flight per lane
            constexpr int R = kGroupEdges / 64;
            unsigned int ent[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int e = eb + r * 64 + lane;
                ent[r] = e < ee ? (unsigned int)col_idx[e] : (unsigned int)r0;
            }
            float2 q[R];
#pragma unroll
            for (int r = 0; r < R; ++r) q[r] = pos[ent[r] & 0x3ffffffu];
            // local refinement weights of the neighbours (Sec. 5), when set
            float aj[R];
            if (aw) {
#pragma unroll
                for (int r = 0; r < R; ++r) aj[r] = aw[ent[r] & 0x3ffffffu];
            }
            // per round: terms of 64 consecutive entries, summed per row by
            // a segmented wave sum; the last lane of each row's run adds the
            // run's sum to the row (one lane per row and round, so plain LDS
            // updates suffice: no float atomics)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (eb + r * 64 >= ee) break;
                const bool valid = eb + r * 64 + lane < ee;
                const int key = valid ? (int)(ent[r] >> 26) : 127;
                float ax = 0.f, ay = 0.f;
                if (valid) {
                    edge_term(pw[key].x, pw[key].y, q[r], a.beta, a.tau, ax, ay);
                    if (aw) {
                        const float wgt = 0.5f * (awn[key] + aj[r]);
                        ax *= wgt;
                        ay *= wgt;
                    }
                }
                wave_segmented_sum(ax, ay, key, lane);
                const int knext = __shfl_down(key, 1);
                if (valid && (lane == 63 || knext != key)) {
                    ax_w[key] += ax;
                    ay_w[key] += ay;
                }
            }
            if (lane < nr) {
                sax = ax_w[lane];
                say = ay_w[lane];
                have = true;
                i = r0 + lane;
                p = po;
            }
        }
    }
    if constexpr (MODE < 2) {
        if (have) {
            float2 v = make_float2(sax, say);
            if (MODE == 1) {
                const float2 old = fpart[i];
                v = make_float2(old.x + sax, old.y + say);
            }
            fpart[i] = v;
        }
    } else {
        if (have) {
            if (use_part) {
                const float2 old = fpart[i];
                sax = old.x + sax;
                say = old.y + say;
            }
            const Box bx = b.st->box;
            float frx, fry;
            grid_repulsion<K>(b, g, bx, p, frx, fry);
            node_output(i, p, frx, fry, sax, say, a, b.st->t, b.st, pos_out, f_rep, f_att, f_tot, xmin, ymin,
                        xmax, ymax);
        }
        if (pos_out != nullptr) block_minmax_commit(xmin, ymin, xmax, ymax, b.st, set, bid);
    }
}

template <int K, int MODE>
__global__ __launch_bounds__(kThreads) void k_edges(const float2* __restrict__ pos,
                                                    float2* __restrict__ pos_out, EdgeSlice es,
                                                    int use_part, float2* __restrict__ fpart, Bufs b,
                                                    Geom g, ModelArgs a, int set, float2* f_rep,
                                                    float2* f_att, float2* f_tot) {
    edges_body<K, MODE>(pos, pos_out, es, use_part, fpart, b, g, a, set, f_rep, f_att, f_tot, blockIdx.x);
}

// Attraction pass that runs beside the grid passes (on a second stream): the
// attraction sums of every row into fpart, nothing else. A fixed number of
// blocks walks the schedule (block b takes entries b, b + gridDim.x, ...), so
// that the launch holds only part of every CU and the binning and FFT
// kernels of the same iteration find room next to it. Each row's sum is
// formed exactly as in the fused pass, so the results do not depend on the
// number of blocks.
__global__ __launch_bounds__(kThreads) void k_attract(const float2* __restrict__ pos, EdgeSlice es,
                                                      float2* __restrict__ fpart, Bufs b, Geom g, ModelArgs a) {
    for (int bid = blockIdx.x; bid < es.blocks; bid += gridDim.x)
        edges_body<1, 0>(pos, nullptr, es, 0, fpart, b, g, a, 0, nullptr, nullptr, nullptr, bid);
}

void launch_attract(const float2* pos, const EdgeSlice& es, float2* fpart, const Bufs& b, const Geom& g,
                    const ModelArgs& a, int blocks, hipStream_t s) {
    const int grid = es.blocks < blocks ? es.blocks : blocks;
    if (grid <= 0) return;
    hipLaunchKernelGGL(k_attract, dim3(grid), dim3(kThreads), 0, s, pos, es, fpart, b, g, a);
}

// Node pass after the overlapped attraction pass: repulsion gathered from
// the grid potentials, displacement from fpart, then the capped move (or the
// force outputs); the same arithmetic per node as the fused pass. Each thread
// takes kNodesPerThread nodes (a stride of the block size apart) and issues
// all their loads before the first store, so that the pass is not a chain of
// one load round trip per node.
constexpr int kNodesPerThread = 4;

template <int K>
__global__ __launch_bounds__(kThreads) void k_node_update(const float2* __restrict__ pos, float2* __restrict__ pos_out,
                                                          const float2* __restrict__ fpart, Bufs b, Geom g,
                                                          ModelArgs a, int set, float2* f_rep, float2* f_att,
                                                          float2* f_tot) {
    const int base = blockIdx.x * (kThreads * kNodesPerThread) + threadIdx.x;
    float2 p[kNodesPerThread], sa[kNodesPerThread];
#pragma unroll
    for (int u = 0; u < kNodesPerThread; ++u) {
        const int i = min(base + u * kThreads, b.n - 1);
        p[u] = pos[i];
        sa[u] = fpart[i];
    }
    const Box bx = b.st->box;
    const int t = b.st->t;
    float frx[kNodesPerThread], fry[kNodesPerThread];
#pragma unroll
    for (int u = 0; u < kNodesPerThread; ++u) grid_repulsion<K>(b, g, bx, p[u], frx[u], fry[u]);
    float xmin = INFINITY, ymin = INFINITY, xmax = -INFINITY, ymax = -INFINITY;
#pragma unroll
    for (int u = 0; u < kNodesPerThread; ++u) {
        const int i = base + u * kThreads;
        if (i < b.n)
            node_output(i, p[u], frx[u], fry[u], sa[u].x, sa[u].y, a, t, b.st, pos_out, f_rep, f_att, f_tot, xmin,
                        ymin, xmax, ymax);
    }
    if (pos_out != nullptr) block_minmax_commit(xmin, ymin, xmax, ymax, b.st, set, blockIdx.x);
}

void launch_node_update(const float2* pos, float2* pos_out, const float2* fpart, const Bufs& b, const Geom& g,
                        const ModelArgs& a, int set, float2* f_rep, float2* f_att, float2* f_tot, hipStream_t s) {
    const int per = kThreads * kNodesPerThread;
    const dim3 grid((b.n + per - 1) / per), block(kThreads);
    switch (g.k) {
        case 1: hipLaunchKernelGGL(k_node_update<1>, grid, block, 0, s, pos, pos_out, fpart, b, g, a, set, f_rep, f_att, f_tot); break;
        case 2: hipLaunchKernelGGL(k_node_update<2>, grid, block, 0, s, pos, pos_out, fpart, b, g, a, set, f_rep, f_att, f_tot); break;
        default: hipLaunchKernelGGL(k_node_update<3>, grid, block, 0, s, pos, pos_out, fpart, b, g, a, set, f_rep, f_att, f_tot); break;
    }
}

// Batched edge pass of iteration j of a call (single slice, positions moved
// from the current buffer to the other one).
template <int K>
__global__ __launch_bounds__(kThreads) void kb_edges(const Member* __restrict__ mem, const int2* __restrict__ map,
                                                     const int* __restrict__ tcall, int j) {
    const int2 e = map[blockIdx.x];
    const Member& m = mem[e.x];
    const float2* cur = (j & 1) ? m.alt : m.pos;
    float2* nxt = (j & 1) ? m.pos : m.alt;
    edges_body<K, 2>(cur, nxt, m.es, 0, nullptr, m.b, m.g, m.a, batch_set(tcall, m, j) ^ 1, nullptr, nullptr,
                     nullptr, e.y);
}

void launch_b_edges(int k, const Member* mem, const int2* map, int blocks, const int* tcall, int j,
                    hipStream_t s) {
    if (blocks <= 0) return;
    const dim3 grid(blocks), block(kThreads);
    switch (k) {
        case 1: hipLaunchKernelGGL(kb_edges<1>, grid, block, 0, s, mem, map, tcall, j); break;
        case 2: hipLaunchKernelGGL(kb_edges<2>, grid, block, 0, s, mem, map, tcall, j); break;
        default: hipLaunchKernelGGL(kb_edges<3>, grid, block, 0, s, mem, map, tcall, j); break;
    }
}

template <int K>
static void launch_edges_k(const float2* pos, float2* pos_out, const EdgeSlice& es, int mode, int use_part,
                           float2* fpart, const Bufs& b, const Geom& g, const ModelArgs& a, int set,
                           float2* f_rep, float2* f_att, float2* f_tot, hipStream_t s) {
    const dim3 grid(es.blocks), block(kThreads);
    if (mode == 0)
        hipLaunchKernelGGL((k_edges<K, 0>), grid, block, 0, s, pos, pos_out, es, use_part, fpart, b, g, a, set,
                           f_rep, f_att, f_tot);
    else if (mode == 1)
        hipLaunchKernelGGL((k_edges<K, 1>), grid, block, 0, s, pos, pos_out, es, use_part, fpart, b, g, a, set,
                           f_rep, f_att, f_tot);
    else
        hipLaunchKernelGGL((k_edges<K, 2>), grid, block, 0, s, pos, pos_out, es, use_part, fpart, b, g, a, set,
                           f_rep, f_att, f_tot);
}

void launch_edges(const float2* pos, float2* pos_out, const EdgeSlice& es, int mode, int use_part,
                  float2* fpart, const Bufs& b, const Geom& g, const ModelArgs& a, int set, float2* f_rep,
                  float2* f_att, float2* f_tot, hipStream_t s) {
    // partial modes do not depend on k: one instantiation serves all
    const int k = mode < 2 ? 1 : g.k;
    switch (k) {
        case 1: launch_edges_k<1>(pos, pos_out, es, mode, use_part, fpart, b, g, a, set, f_rep, f_att, f_tot, s); break;
        case 2: launch_edges_k<2>(pos, pos_out, es, mode, use_part, fpart, b, g, a, set, f_rep, f_att, f_tot, s); break;
        default: launch_edges_k<3>(pos, pos_out, es, mode, use_part, fpart, b, g, a, set, f_rep, f_att, f_tot, s); break;
    }
}

// Exact repulsion: F_i = sum_j K_ij (x_i - x_j), K_ij = (1 + tau d_ij^2)^-gamma
// (Eq.11; the j = i term is zero), positions streamed through 256-position
// LDS tiles; attraction by a per-lane row loop (used for small graphs).
// A block holds kBruteRows = 64 rows, one per lane; its four waves sum
// interleaved quarters of every tile (8 positions per LDS batch) and wave 0
// adds the four sums in a fixed order, then finishes its rows.
// Columns are read through the 26-bit column mask, so the packed edge-pass
// entries (column | row-in-group << 26) serve as well as a plain CSR.
// 1 + tau d^2; for tau = 1 two fused multiply-adds.
template <bool T1>
__device__ __forceinline__ float one_plus_tau_d2(float dx, float dy, float tau) {
    if constexpr (T1)
        return __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, 1.f));
    else
        return 1.f + tau * (dx * dx + dy * dy);
}

template <bool G2, bool T1>
__device__ __forceinline__ void brute_term(float2 p, float2 q, float tau, float gamma, float& frx, float& fry) {
    const float dx = p.x - q.x;
    const float dy = p.y - q.y;
    const float u = one_plus_tau_d2<T1>(dx, dy, tau);
    float kk;
    if constexpr (G2) {
        const float r = __builtin_amdgcn_rcpf(u);  // u >= 1: hardware reciprocal, <= 1 ulp
        kk = r * r;
    } else {
        kk = powf(u, -gamma);
    }
    frx += kk * dx;
    fry += kk * dy;
}

template <bool G2, bool T1>
__device__ __forceinline__ void brute_tile(const float2* tile, int j0, int j1, float2 p, float tau, float gamma,
                                           float& frx, float& fry) {
    // four independent partial sums (positions jj + u, u mod 4) shorten the
    // dependent chain of adds; they are combined in a fixed order
    float sx[4] = {0.f, 0.f, 0.f, 0.f}, sy[4] = {0.f, 0.f, 0.f, 0.f};
    int jj = j0;
    for (; jj + 8 <= j1; jj += 8) {
        float2 q[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) q[u] = tile[jj + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) brute_term<G2, T1>(p, q[u], tau, gamma, sx[u & 3], sy[u & 3]);
    }
    for (; jj < j1; ++jj) brute_term<G2, T1>(p, tile[jj], tau, gamma, sx[0], sy[0]);
    frx += (sx[0] + sx[1]) + (sx[2] + sx[3]);
    fry += (sy[0] + sy[1]) + (sy[2] + sy[3]);
}

__device__ __forceinline__ void brute_body(const float2* __restrict__ pos, int n, float2* __restrict__ pos_out,
                                           const int* __restrict__ row_ptr, const int* __restrict__ col_idx,
                                           DevState* st, const ModelArgs& a, int t, float2* f_rep, float2* f_att,
                                           float2* f_tot, int bid) {
    __shared__ float2 tile[kThreads];
    __shared__ float2 part[kThreads / 64 - 1][64];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int i = bid * kBruteRows + lane;
    const bool active = i < n;
    const float2 p = active ? pos[i] : make_float2(0.f, 0.f);
    const bool g2 = a.gamma == 2.0f;
    const float tau = a.tau;
    float frx = 0.f, fry = 0.f;
    for (int base = 0; base < n; base += kThreads) {
        const int j = base + threadIdx.x;
        tile[threadIdx.x] = j < n ? pos[j] : make_float2(0.f, 0.f);
        __syncthreads();
        const int cnt = min(kThreads, n - base);
        const int j0 = w * 64;
        const int j1 = min(j0 + 64, cnt);
        if (g2)
            tau == 1.f ? brute_tile<true, true>(tile, j0, j1, p, tau, a.gamma, frx, fry)
                       : brute_tile<true, false>(tile, j0, j1, p, tau, a.gamma, frx, fry);
        else
            brute_tile<false, false>(tile, j0, j1, p, tau, a.gamma, frx, fry);
        __syncthreads();
    }
    if (w > 0) part[w - 1][lane] = make_float2(frx, fry);
    __syncthreads();
    if (w != 0 || !active) return;
    const float2 s1 = part[0][lane], s2 = part[1][lane], s3 = part[2][lane];
    frx = (frx + s1.x) + (s2.x + s3.x);
    fry = (fry + s1.y) + (s2.y + s3.y);
    float xmin = INFINITY, ymin = INFINITY, xmax = -INFINITY, ymax = -INFINITY;
    float sax = 0.f, say = 0.f;
    const int e1 = row_ptr[i + 1];
    const float* __restrict__ aw = a.att_w;
    for (int e = row_ptr[i]; e < e1; ++e) {
        const int j = col_idx[e] & 0x3ffffff;
        float ax, ay;
        edge_term(p.x, p.y, pos[j], a.beta, tau, ax, ay);
        const float wgt = aw ? 0.5f * (aw[i] + aw[j]) : 1.f;
        sax += wgt * ax;
        say += wgt * ay;
    }
    node_output(i, p, frx, fry, sax, say, a, t, st, pos_out, f_rep, f_att, f_tot, xmin, ymin, xmax, ymax);
}

__global__ __launch_bounds__(kThreads) void k_brute(const float2* __restrict__ pos, int n,
                                                    float2* __restrict__ pos_out,
                                                    const int* __restrict__ row_ptr,
                                                    const int* __restrict__ col_idx, DevState* st,
                                                    ModelArgs a, int t, float2* f_rep, float2* f_att,
                                                    float2* f_tot) {
    brute_body(pos, n, pos_out, row_ptr, col_idx, st, a, t, f_rep, f_att, f_tot, blockIdx.x);
}

// Batched exact method, iteration j of a call (j by its parity only: the
// kernels are replayed from captured graphs). The update's counter is the
// member's device counter plus one; kb_tick then advances that counter
// (the call start sets it to t0 - 1, like the binning scan of the
// interpolated path).
__global__ __launch_bounds__(kThreads) void kb_brute(const Member* __restrict__ mem, const int2* __restrict__ map,
                                                     int j) {
    const int2 e = map[blockIdx.x];
    const Member& m = mem[e.x];
    const float2* cur = (j & 1) ? m.alt : m.pos;
    float2* nxt = (j & 1) ? m.pos : m.alt;
    brute_body(cur, m.b.n, nxt, m.es.rp, m.es.col, m.b.st, m.a, m.b.st->t + 1, nullptr, nullptr, nullptr, e.y);
}

__global__ void kb_tick(const Member* __restrict__ mem, const int2* __restrict__ map, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) mem[map[i].x].b.st->t += 1;
}

void launch_b_brute(const Member* mem, const int2* map, int blocks, int j, hipStream_t s) {
    if (blocks > 0) hipLaunchKernelGGL(kb_brute, dim3(blocks), dim3(kThreads), 0, s, mem, map, j);
}

void launch_b_tick(const Member* mem, const int2* tick_map, int members, hipStream_t s) {
    if (members > 0) hipLaunchKernelGGL(kb_tick, dim3((members + 255) / 256), dim3(256), 0, s, mem, tick_map, members);
}

void launch_brute(const float2* pos, float2* pos_out, const int* row_ptr, const int* col_idx, int n,
                  DevState* st, const ModelArgs& a, int t, float2* f_rep, float2* f_att, float2* f_tot,
                  hipStream_t s) {
    const int blocks = (n + kBruteRows - 1) / kBruteRows;
    hipLaunchKernelGGL(k_brute, dim3(blocks), dim3(kThreads), 0, s, pos, n, pos_out, row_ptr, col_idx,
                       st, a, t, f_rep, f_att, f_tot);
}

// ----------------------------------------------------------------- exact method, pair-symmetric form
//
// For larger graphs the exact repulsion takes every unordered pair once
// (Newton's third law: the term of (j, i) is minus that of (i, j)). Blocks
// take tile pairs (I, J), I <= J, of kSymTile nodes. Every wave holds the
// whole row tile, lane l the rows I kSymTile + 64 r + l (r < 4), and takes
// one quarter of tile J's columns: at step s lane l meets column
// 64 w + ((l + s) mod 64) with its four rows; the column's running sum of
// minus the row terms travels with it, one lane down per step, so that after
// 64 steps lane l holds the sum of column 64 w + l over the row tile. The
// waves' row sums are combined in LDS in a fixed order. A diagonal block
// sums both orders of its pairs into the rows only. Each block adds its row
// and column sums to per-node 64-bit fixed-point accumulators with integer
// atomics, which are exact, so the totals do not depend on the order of the
// blocks; the node pass reads and clears them.

// Scale of the fixed-point sums: a pair term is below tmax = max over d of
// d (1 + tau d^2)^-gamma in magnitude (reached at d^2 = 1 / (tau (2 gamma -
// 1))), so n terms stay below 2^61 with the scale 2^(61 - e), n tmax < 2^e.
__device__ __forceinline__ double sym_scale(int n, float gamma, float tau) {
    const double g = gamma, tt = tau;
    const double d2 = 1.0 / (tt * (2.0 * g - 1.0));
    const double tmax = sqrt(d2) * pow(1.0 + tt * d2, -g);
    int e;
    (void)frexp((double)n * tmax, &e);
    return ldexp(1.0, 61 - e);
}

// Tile pair p (0 <= p < nt (nt + 1) / 2) in row order: row I starts at
// I nt - I (I - 1) / 2.
__device__ __forceinline__ void sym_tile_pair(int p, int nt, int& I, int& J) {
    const double b = (double)nt + 0.5;
    int r = (int)(b - sqrt(b * b - 2.0 * (double)p));
    if (r < 0) r = 0;
    if (r > nt - 1) r = nt - 1;
    auto start = [nt](int x) { return (long long)x * nt - (long long)x * (x - 1) / 2; };
    while (r > 0 && start(r) > p) --r;
    while (r < nt - 1 && start(r + 1) <= p) ++r;
    I = r;
    J = r + (int)(p - start(r));
}

// Repulsion term factor K(d) = (1 + tau d^2)^-gamma of one pair.
template <bool G2, bool T1>
__device__ __forceinline__ float sym_kernel(float dx, float dy, float tau, float gamma) {
    const float u = one_plus_tau_d2<T1>(dx, dy, tau);
    if constexpr (G2) {
        const float r = __builtin_amdgcn_rcpf(u);
        return r * r;
    } else {
        return powf(u, -gamma);
    }
}

// Lane l receives the value of lane (l + 1) mod 64 (DPP wavefront rotate).
__device__ __forceinline__ float lane_next(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x134, 0xf, 0xf, false));
}

__device__ __forceinline__ void sym_add(unsigned long long* acc, int node, float fx, float fy, double scale) {
    atomicAdd(acc + 2 * (size_t)node, (unsigned long long)__double2ll_rn((double)fx * scale));
    atomicAdd(acc + 2 * (size_t)node + 1, (unsigned long long)__double2ll_rn((double)fy * scale));
}

template <bool G2, bool T1>
__device__ __forceinline__ void sym_pairs_t(const float2* __restrict__ pos, int n, unsigned long long* __restrict__ acc,
                                            float gamma, float tau, int p) {
    constexpr int R = kSymTile / 64;  // rows per lane: every wave holds the whole row tile
    __shared__ float2 cols[kSymTile];
    __shared__ float2 rpart[kSymTile / 64][kSymTile];  // each wave's row sums over its column quarter
    const int nt = (n + kSymTile - 1) / kSymTile;
    int I, J;
    sym_tile_pair(p, nt, I, J);
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int jt = J * kSymTile + threadIdx.x;
    cols[threadIdx.x] = jt < n ? pos[jt] : make_float2(0.f, 0.f);
    float2 pi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = I * kSymTile + r * 64 + lane;
        pi[r] = i < n ? pos[i] : make_float2(0.f, 0.f);
    }
    const double scale = sym_scale(n, gamma, tau);
    const int cnt = min(kSymTile, n - J * kSymTile);  // columns of tile J inside the graph
    const int cbase = w * 64;                         // this wave's quarter of the columns
    __syncthreads();
    float fx[R], fy[R];
#pragma unroll
    for (int r = 0; r < R; ++r) fx[r] = fy[r] = 0.f;
    if (I == J) {
        // both orders of every pair of the tile, into the rows (the term of
        // a node with itself is zero)
        const int c1 = min(cbase + 64, cnt);
        for (int c = cbase; c < c1; ++c) {
            const float2 v = cols[c];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float dx = pi[r].x - v.x, dy = pi[r].y - v.y;
                const float kk = sym_kernel<G2, T1>(dx, dy, tau, gamma);
                fx[r] += kk * dx;
                fy[r] += kk * dy;
            }
        }
    } else {
        float gx = 0.f, gy = 0.f;
        const bool full = cnt == kSymTile;
        for (int s = 0; s < 64; ++s) {
            const int c = cbase + ((lane + s) & 63);
            const float2 v = cols[c];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float dx = pi[r].x - v.x, dy = pi[r].y - v.y;
                float kk = sym_kernel<G2, T1>(dx, dy, tau, gamma);
                if (!full && c >= cnt) kk = 0.f;
                fx[r] += kk * dx;
                fy[r] += kk * dy;
                gx -= kk * dx;
                gy -= kk * dy;
            }
            gx = lane_next(gx);
            gy = lane_next(gy);
        }
        // lane l now holds column cbase + l, summed over the whole row tile
        const int j = J * kSymTile + cbase + lane;
        if (j < n) sym_add(acc, j, gx, gy, scale);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) rpart[w][r * 64 + lane] = make_float2(fx[r], fy[r]);
    __syncthreads();
    const float2 a0 = rpart[0][threadIdx.x], a1 = rpart[1][threadIdx.x];
    const float2 a2 = rpart[2][threadIdx.x], a3 = rpart[3][threadIdx.x];
    const int i = I * kSymTile + threadIdx.x;
    if (i < n) sym_add(acc, i, (a0.x + a1.x) + (a2.x + a3.x), (a0.y + a1.y) + (a2.y + a3.y), scale);
}

__device__ __forceinline__ void sym_pairs_body(const float2* __restrict__ pos, int n,
                                               unsigned long long* __restrict__ acc, const ModelArgs& a, int p) {
    if (a.gamma == 2.0f && a.tau == 1.0f)
        sym_pairs_t<true, true>(pos, n, acc, a.gamma, a.tau, p);
    else if (a.gamma == 2.0f)
        sym_pairs_t<true, false>(pos, n, acc, a.gamma, a.tau, p);
    else
        sym_pairs_t<false, false>(pos, n, acc, a.gamma, a.tau, p);
}

// Node pass of the pair-symmetric exact method: repulsion from the
// accumulators (cleared for the next pass), attraction along the row,
// displacement and move (or the force outputs); one node per thread.
__device__ __forceinline__ void sym_node_body(const float2* __restrict__ pos, int n, float2* __restrict__ pos_out,
                                              const int* __restrict__ row_ptr, const int* __restrict__ col_idx,
                                              unsigned long long* __restrict__ acc, DevState* st,
                                              const ModelArgs& a, int t, float2* f_rep, float2* f_att,
                                              float2* f_tot, int bid) {
    const int i = bid * kThreads + threadIdx.x;
    if (i < n) {
        float xmin = INFINITY, ymin = INFINITY, xmax = -INFINITY, ymax = -INFINITY;
        const double inv = 1.0 / sym_scale(n, a.gamma, a.tau);
        const unsigned long long ux = acc[2 * (size_t)i], uy = acc[2 * (size_t)i + 1];
        acc[2 * (size_t)i] = 0ull;
        acc[2 * (size_t)i + 1] = 0ull;
        const float frx = (float)((double)(long long)ux * inv);
        const float fry = (float)((double)(long long)uy * inv);
        const float2 p = pos[i];
        float sax = 0.f, say = 0.f;
        const int e1 = row_ptr[i + 1];
        const float* __restrict__ aw = a.att_w;
        for (int e = row_ptr[i]; e < e1; ++e) {
            const int j = col_idx[e] & 0x3ffffff;
            float ax, ay;
            edge_term(p.x, p.y, pos[j], a.beta, a.tau, ax, ay);
            const float wgt = aw ? 0.5f * (aw[i] + aw[j]) : 1.f;
            sax += wgt * ax;
            say += wgt * ay;
        }
        node_output(i, p, frx, fry, sax, say, a, t, st, pos_out, f_rep, f_att, f_tot, xmin, ymin, xmax, ymax);
    }
}

__global__ __launch_bounds__(kThreads) void k_sym_pairs(const float2* __restrict__ pos, int n,
                                                        unsigned long long* __restrict__ acc, ModelArgs a) {
    sym_pairs_body(pos, n, acc, a, blockIdx.x);
}

__global__ __launch_bounds__(kThreads) void k_sym_node(const float2* __restrict__ pos, int n,
                                                       float2* __restrict__ pos_out, const int* __restrict__ row_ptr,
                                                       const int* __restrict__ col_idx,
                                                       unsigned long long* __restrict__ acc, DevState* st, ModelArgs a,
                                                       int t, float2* f_rep, float2* f_att, float2* f_tot) {
    sym_node_body(pos, n, pos_out, row_ptr, col_idx, acc, st, a, t, f_rep, f_att, f_tot, blockIdx.x);
}

long long sym_pair_blocks(int n) {
    const long long nt = (n + kSymTile - 1) / kSymTile;
    return nt * (nt + 1) / 2;
}

int sym_node_blocks(int n) { return (n + kThreads - 1) / kThreads; }

void launch_sym(const float2* pos, float2* pos_out, const int* row_ptr, const int* col_idx, int n,
                unsigned long long* acc, DevState* st, const ModelArgs& a, int t, float2* f_rep, float2* f_att,
                float2* f_tot, hipStream_t s) {
    hipLaunchKernelGGL(k_sym_pairs, dim3((unsigned)sym_pair_blocks(n)), dim3(kThreads), 0, s, pos, n, acc, a);
    hipLaunchKernelGGL(k_sym_node, dim3(sym_node_blocks(n)), dim3(kThreads), 0, s, pos, n, pos_out, row_ptr, col_idx,
                       acc, st, a, t, f_rep, f_att, f_tot);
}

// Batched pair-symmetric exact method: map entries {member, tile pair} for
// the pair pass and {member, node block} for the node pass, iteration j of
// the call by its parity (like kb_brute; kb_tick advances the counters).
__global__ __launch_bounds__(kThreads) void kb_sym_pairs(const Member* __restrict__ mem, const int2* __restrict__ map,
                                                         int j) {
    const int2 e = map[blockIdx.x];
    const Member& m = mem[e.x];
    sym_pairs_body((j & 1) ? m.alt : m.pos, m.b.n, m.b.sym_acc, m.a, e.y);
}

__global__ __launch_bounds__(kThreads) void kb_sym_node(const Member* __restrict__ mem, const int2* __restrict__ map,
                                                        int j) {
    const int2 e = map[blockIdx.x];
    const Member& m = mem[e.x];
    const float2* cur = (j & 1) ? m.alt : m.pos;
    float2* nxt = (j & 1) ? m.pos : m.alt;
    sym_node_body(cur, m.b.n, nxt, m.es.rp, m.es.col, m.b.sym_acc, m.b.st, m.a, m.b.st->t + 1, nullptr, nullptr,
                  nullptr, e.y);
}

void launch_b_sym_pairs(const Member* mem, const int2* map, int blocks, int j, hipStream_t s) {
    if (blocks > 0) hipLaunchKernelGGL(kb_sym_pairs, dim3(blocks), dim3(kThreads), 0, s, mem, map, j);
}

void launch_b_sym_node(const Member* mem, const int2* map, int blocks, int j, hipStream_t s) {
    if (blocks > 0) hipLaunchKernelGGL(kb_sym_node, dim3(blocks), dim3(kThreads), 0, s, mem, map, j);
}

// CSR sanity check: row_ptr[0] = 0, monotone, row_ptr[n] = nnz, columns in
// [0, n) and different from the row. Reads stay inside [0, nnz).
__global__ void k_csr_check(const int* __restrict__ row_ptr, const int* __restrict__ col_idx, int n,
                            long long nnz, DevState* st) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    if (i == n) {
        if ((long long)row_ptr[n] != nnz) st->csr_bad = 1;
        if (row_ptr[0] != 0) st->csr_bad = 1;
        return;
    }
    const long long e0 = row_ptr[i];
    const long long e1 = row_ptr[i + 1];
    if (e0 > e1 || e0 < 0 || e1 > nnz) {
        st->csr_bad = 1;
        return;
    }
    for (long long e = e0; e < e1; ++e) {
        const int c = col_idx[e];
        if (c < 0 || c >= n || c == i) {
            st->csr_bad = 1;
            return;
        }
    }
}

void launch_csr_check(const int* row_ptr, const int* col_idx, int n, long long nnz, DevState* st,
                      hipStream_t s) {
    const int blocks = (n + 1 + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_csr_check, dim3(blocks), dim3(kThreads), 0, s, row_ptr, col_idx, n, nnz, st);
}

}  // namespace tfdp
