// Box reduction and interval-row binning of the nodes (Sec. 3.4: the layout
// box is split into N_int x N_int intervals; each node is interpolated from
// the k x k nodes of its own interval).
//
// The nodes are bucketed by interval row with a counting sort so that
// the spreading pass can accumulate every row of the grid in LDS without
// global atomics:
//   bin_count   per block of kBinChunk nodes: LDS histogram of interval rows
//   bin_scan    exclusive scan of the per-block counts of every row
//   bin_scatter per block: slots inside the block's part of each row by
//               LDS atomics, positions written to their slot
#include "tfdp_internal.h"

namespace tfdp {

static_assert(kBoxSlots == 64, "the box finalize reduces one slot per lane of a wave");

// ----------------------------------------------------------------- box
//
// Extremes of the positions are committed with integer atomics into one of
// two slot sets: the update of iteration t fills set (t+1) & 1 while the
// binning of iteration t reads set t & 1 and its scan resets set (t+1) & 1
// for the next update. The box itself is derived by bin_count.

__device__ __forceinline__ void reset_slot(DevState* st, int set, int i) {
    st->mm[set][i][0] = 0xffffffffu;
    st->mm[set][i][1] = 0xffffffffu;
    st->mm[set][i][2] = 0u;
    st->mm[set][i][3] = 0u;
}

// Reset of both slot sets; st->t = t - 1 (the scan of each iteration
// advances it before the update reads it).
__global__ void k_box_begin(DevState* st, int t) {
    if (threadIdx.x < kBoxSlots) {
        reset_slot(st, 0, threadIdx.x);
        reset_slot(st, 1, threadIdx.x);
    }
    if (threadIdx.x == 0) st->t = t - 1;
}

__device__ __forceinline__ void box_reduce_body(const float2* __restrict__ pos, int n, DevState* st, int set,
                                                int bid, int nblocks) {
    float xmin = INFINITY, ymin = INFINITY, xmax = -INFINITY, ymax = -INFINITY;
    for (int i = bid * blockDim.x + threadIdx.x; i < n; i += nblocks * blockDim.x) {
        float2 p = pos[i];
        if (isfinite(p.x) && isfinite(p.y)) {
            xmin = fminf(xmin, p.x);
            xmax = fmaxf(xmax, p.x);
            ymin = fminf(ymin, p.y);
            ymax = fmaxf(ymax, p.y);
        }
    }
    block_minmax_commit(xmin, ymin, xmax, ymax, st, set, bid);
}

__global__ __launch_bounds__(kThreads) void k_box_reduce(const float2* __restrict__ pos, int n,
                                                         DevState* st, int set) {
    box_reduce_body(pos, n, st, set, blockIdx.x, gridDim.x);
}

void launch_box_begin(DevState* st, int t, hipStream_t s) {
    hipLaunchKernelGGL(k_box_begin, dim3(1), dim3(kBoxSlots), 0, s, st, t);
}

Dims box_reduce_dims(int n) {
    int blocks = (n + kThreads * 8 - 1) / (kThreads * 8);
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    return Dims{blocks, kThreads, 0};
}

void launch_box_reduce(const float2* pos, int n, DevState* st, int set, hipStream_t s) {
    const Dims d = box_reduce_dims(n);
    hipLaunchKernelGGL(k_box_reduce, dim3(d.grid), dim3(d.block), 0, s, pos, n, st, set);
}

// ----------------------------------------------------------------- binning

// Box of this iteration from slot set `set` (every block derives it; block 0
// publishes it for the later kernels of the iteration), then the LDS
// histogram of interval rows of this block's nodes.
__device__ __forceinline__ void bin_count_body(const float2* __restrict__ pos, const Bufs& b, int set, int bid) {
    extern __shared__ int hist[];
    __shared__ Box sbox;
    const int n_int = b.n_int;
    for (int c = threadIdx.x; c < n_int; c += blockDim.x) hist[c] = 0;
    if (threadIdx.x < 64) {
        unsigned int a0 = b.st->mm[set][threadIdx.x][0];
        unsigned int a1 = b.st->mm[set][threadIdx.x][1];
        unsigned int a2 = b.st->mm[set][threadIdx.x][2];
        unsigned int a3 = b.st->mm[set][threadIdx.x][3];
        for (int off = 32; off > 0; off >>= 1) {
            a0 = min(a0, (unsigned int)__shfl_xor((int)a0, off));
            a1 = min(a1, (unsigned int)__shfl_xor((int)a1, off));
            a2 = max(a2, (unsigned int)__shfl_xor((int)a2, off));
            a3 = max(a3, (unsigned int)__shfl_xor((int)a3, off));
        }
        if (threadIdx.x == 0) {
            sbox = box_from_extremes(a0, a1, a2, a3, n_int);
            if (bid == 0) b.st->box = sbox;
        }
    }
    __syncthreads();
    const Box bx = sbox;
    const int beg = bid * kBinChunk;
    const int end = min(beg + kBinChunk, b.n);
    for (int i0 = beg + threadIdx.x; i0 < end; i0 += 4 * blockDim.x) {
        float yv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) yv[u] = pos[min(i0 + u * (int)blockDim.x, end - 1)].y;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (i0 + u * (int)blockDim.x < end) {
                int cy;
                double ty;
                bin_axis(yv[u], bx.lo_y, bx.h, n_int, cy, ty);
                atomicAdd(&hist[cy], 1);
            }
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < n_int; c += blockDim.x)
        b.blkcnt[(size_t)c * b.nblk + bid] = hist[c];
}

__global__ __launch_bounds__(kThreads) void k_bin_count(const float2* __restrict__ pos, Bufs b, int set) {
    grid_pass_priority();
    bin_count_body(pos, b, set, blockIdx.x);
}

// Exclusive scan of kThreads values held one per thread; returns the
// thread's exclusive prefix and writes the block total.
__device__ __forceinline__ int block_exclusive_scan(int v, int* lds /* kThreads/64 + 1 */, int& total) {
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    int x = v;
    for (int off = 1; off < 64; off <<= 1) {
        int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) lds[w] = x;
    __syncthreads();
    int base = 0;
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < w; ++i) base += lds[i];
    int tot = 0;
    for (int i = 0; i < nw; ++i) tot += lds[i];
    total = tot;
    __syncthreads();
    return base + x - v;
}

// Exclusive scan of every interval row's per-block counts in place, totals
// into bucket_cnt: one block per row, or, for graphs of at most
// kSerialScanBlocks binning blocks, one block for all rows with a row per
// thread (bin_scan_dims). Block 0 also resets slot set `reset_set` for the
// coming update and advances the iteration counter.
constexpr int kSerialScanBlocks = 32;

__device__ __forceinline__ void bin_scan_body(const Bufs& b, int reset_set, int c) {
    __shared__ int lds[kThreads / 64 + 1];
    if (c == 0) {
        if (threadIdx.x < kBoxSlots) reset_slot(b.st, reset_set, threadIdx.x);
        if (threadIdx.x == 0) b.st->t += 1;
    }
    if (b.nblk <= kSerialScanBlocks) {
        for (int r = threadIdx.x; r < b.n_int; r += blockDim.x) {
            int* row = b.blkcnt + (size_t)r * b.nblk;
            int carry = 0;
            for (int i = 0; i < b.nblk; ++i) {
                const int v = row[i];
                row[i] = carry;
                carry += v;
            }
            b.bucket_cnt[r] = carry;
        }
        return;
    }
    int* row = b.blkcnt + (size_t)c * b.nblk;
    int carry = 0;
    for (int base = 0; base < b.nblk; base += blockDim.x) {
        const int i = base + threadIdx.x;
        const int v = i < b.nblk ? row[i] : 0;
        int tot;
        const int ex = block_exclusive_scan(v, lds, tot);
        if (i < b.nblk) row[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) b.bucket_cnt[c] = carry;
}

__global__ __launch_bounds__(kThreads) void k_bin_scan(Bufs b, int reset_set) {
    grid_pass_priority();
    bin_scan_body(b, reset_set, blockIdx.x);
}

// Scatter of the positions into interval-row buckets. Block 0 also
// publishes the bucket starts and the first spreading chunk of each row
// (rows split into chunks of kSpreadChunk nodes, at least one per row).
__device__ __forceinline__ void bin_scatter_body(const float2* __restrict__ pos, const Bufs& b, int bid) {
    extern __shared__ int sm[];
    const int n_int = b.n_int;
    int* base = sm;                  // [n_int] global slot of this block's first node per row
    int* run = base + n_int;         // [n_int] nodes of this block already placed per row
    int* scan_lds = run + n_int;     // [kThreads/64 + 1]
    int* gflag = scan_lds + kThreads / 64 + 1;  // [groups] (block 0) the row group is one chunk
    int* bsl = gflag + n_int;                   // [n_int + 1] (block 0) bucket starts
    const int rg = b.rgroup;
    const int ngroups = (n_int + rg - 1) / rg;
    if (bid == 0 && rg > 1) {
        // a group of rg consecutive rows holding at most 2 kSpreadChunk nodes
        // together is spread by one block
        for (int gi = threadIdx.x; gi < ngroups; gi += blockDim.x) {
            const int r0 = gi * rg, r1 = min(r0 + rg, n_int);
            int tot = 0;
            for (int c = r0; c < r1; ++c) tot += b.bucket_cnt[c];
            gflag[gi] = (r1 - r0 >= 2 && tot <= 2 * kSpreadChunk) ? 1 : 0;
        }
        __syncthreads();
    }
    // bucket starts: exclusive scan over rows (n_int <= 1024, four per
    // thread); block 0 also numbers the partial rows of the spreading pass:
    // one per row of a grouped row, else one per kSpreadChunk nodes (at
    // least one), consecutive for each row
    int carry = 0;
    int chunk_carry = 0;
    for (int c0 = 0; c0 < n_int; c0 += blockDim.x) {
        const int c = c0 + threadIdx.x;
        const int cnt = c < n_int ? b.bucket_cnt[c] : 0;
        int parts = 0;
        if (bid == 0 && c < n_int)
            parts = (rg > 1 && gflag[c / rg]) ? 1 : max(1, (cnt + kSpreadChunk - 1) / kSpreadChunk);
        int tot, tot2;
        const int ex = block_exclusive_scan(cnt, scan_lds, tot);
        const int ex2 = block_exclusive_scan(parts, scan_lds, tot2);
        if (c < n_int) {
            base[c] = carry + ex + b.blkcnt[(size_t)c * b.nblk + bid];
            run[c] = 0;
            if (bid == 0) {
                b.bucket_start[c] = carry + ex;
                b.chunk_start[c] = chunk_carry + ex2;
                bsl[c] = carry + ex;
                if (rg == 1)  // one block per row share: work chunks = partial rows
                    for (int u = 0; u < parts; ++u)
                        b.wchunk[chunk_carry + ex2 + u] = make_int4(
                            c, 1, carry + ex + u * kSpreadChunk, min(carry + ex + (u + 1) * kSpreadChunk, carry + ex + cnt));
            }
        }
        carry += tot;
        chunk_carry += tot2;
    }
    if (bid == 0 && rg == 1 && threadIdx.x == 0) {
        b.bucket_start[n_int] = carry;
        b.chunk_start[n_int] = chunk_carry;
        b.wchunk[b.max_chunks] = make_int4(chunk_carry, 0, 0, 0);
    }
    if (bid == 0 && rg > 1) {
        if (threadIdx.x == 0) {
            b.bucket_start[n_int] = carry;
            b.chunk_start[n_int] = chunk_carry;
            bsl[n_int] = carry;
        }
        __syncthreads();
        // work chunks of the spreading pass, {first row, rows, first node,
        // end}: a grouped row group, or a row's share of kSpreadChunk nodes
        int wcarry = 0;
        for (int g0 = 0; g0 < ngroups; g0 += blockDim.x) {
            const int gi = g0 + threadIdx.x;
            int nw = 0;
            const int r0 = gi * rg, r1 = min(r0 + rg, n_int);
            if (gi < ngroups) {
                if (gflag[gi]) {
                    nw = 1;
                } else {
                    for (int c = r0; c < r1; ++c) nw += max(1, (bsl[c + 1] - bsl[c] + kSpreadChunk - 1) / kSpreadChunk);
                }
            }
            int tot;
            const int ex = block_exclusive_scan(nw, scan_lds, tot);
            if (gi < ngroups) {
                int k = wcarry + ex;
                if (gflag[gi]) {
                    b.wchunk[k] = make_int4(r0, r1 - r0, bsl[r0], bsl[r1]);
                } else {
                    for (int c = r0; c < r1; ++c) {
                        const int q = max(1, (bsl[c + 1] - bsl[c] + kSpreadChunk - 1) / kSpreadChunk);
                        for (int u = 0; u < q; ++u)
                            b.wchunk[k++] = make_int4(c, 1, bsl[c] + u * kSpreadChunk,
                                                      min(bsl[c] + (u + 1) * kSpreadChunk, bsl[c + 1]));
                    }
                }
            }
            wcarry += tot;
        }
        if (threadIdx.x == 0) b.wchunk[b.max_chunks] = make_int4(wcarry, 0, 0, 0);
    }
    __syncthreads();
    // slots inside the block's range of each row by LDS atomics: the order
    // of the nodes inside a row is not fixed, which nothing depends on (the
    // spreading sums are exact integers)
    const Box bx = b.st->box;
    const int beg = bid * kBinChunk;
    const int end = min(beg + kBinChunk, b.n);
    for (int i0 = beg + threadIdx.x; i0 < end; i0 += 4 * blockDim.x) {
        float2 pp[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) pp[u] = pos[min(i0 + u * (int)blockDim.x, end - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (i0 + u * (int)blockDim.x < end) {
                int key;
                double ty;
                bin_axis(pp[u].y, bx.lo_y, bx.h, n_int, key, ty);
                const int slot = atomicAdd(&run[key], 1);
                b.spos[base[key] + slot] = pp[u];
            }
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_bin_scatter(const float2* __restrict__ pos, Bufs b) {
    grid_pass_priority();
    bin_scatter_body(pos, b, blockIdx.x);
}

Dims bin_count_dims(const Bufs& b) { return Dims{b.nblk, kThreads, (size_t)b.n_int * sizeof(int)}; }
Dims bin_scan_dims(const Bufs& b) { return Dims{b.nblk <= kSerialScanBlocks ? 1 : b.n_int, kThreads, 0}; }
Dims bin_scatter_dims(const Bufs& b) {
    return Dims{b.nblk, kThreads, (size_t)(4 * b.n_int + kThreads / 64 + 2) * sizeof(int)};
}

void launch_bin_count(const float2* pos, const Bufs& b, int set, hipStream_t s) {
    const Dims d = bin_count_dims(b);
    hipLaunchKernelGGL(k_bin_count, dim3(d.grid), dim3(d.block), d.lds, s, pos, b, set);
}

void launch_bin_scan(const Bufs& b, int reset_set, hipStream_t s) {
    const Dims d = bin_scan_dims(b);
    hipLaunchKernelGGL(k_bin_scan, dim3(d.grid), dim3(d.block), 0, s, b, reset_set);
}

void launch_bin_scatter(const float2* pos, const Bufs& b, hipStream_t s) {
    const Dims d = bin_scatter_dims(b);
    hipLaunchKernelGGL(k_bin_scatter, dim3(d.grid), dim3(d.block), d.lds, s, pos, b);
}

// ----------------------------------------------------------------- batched
//
// The same bodies over many graphs in one launch. Iteration j of a call
// reads positions from pos (j even) or alt (j odd) of each member, like the
// plain step, which swaps the two buffers after every iteration.

__device__ __forceinline__ const float2* batch_cur(const Member& m, int j) { return (j & 1) ? m.alt : m.pos; }

// Start of a call: both slot sets reset and the iteration counter set to
// t0 - 1 (one block per member), then the box extremes of the positions into
// set t0 & 1.
__global__ void kb_box_begin(const Member* __restrict__ mem, const int2* __restrict__ map,
                             const int* __restrict__ tcall) {
    const Member& m = mem[map[blockIdx.x].x];
    DevState* st = m.b.st;
    if (threadIdx.x < kBoxSlots) {
        reset_slot(st, 0, threadIdx.x);
        reset_slot(st, 1, threadIdx.x);
    }
    if (threadIdx.x == 0) st->t = tcall[m.slot] - 1;
}

__global__ __launch_bounds__(kThreads) void kb_box_reduce(const Member* __restrict__ mem,
                                                          const int2* __restrict__ map,
                                                          const int* __restrict__ tcall) {
    const int2 e = map[blockIdx.x];
    const Member& m = mem[e.x];
    box_reduce_body(m.pos, m.b.n, m.b.st, tcall[m.slot] & 1, e.y, m.box_blocks);
}

__global__ __launch_bounds__(kThreads) void kb_bin_count(const Member* __restrict__ mem,
                                                         const int2* __restrict__ map,
                                                         const int* __restrict__ tcall, int j) {
    const int2 e = map[blockIdx.x];
    const Member& m = mem[e.x];
    bin_count_body(batch_cur(m, j), m.b, batch_set(tcall, m, j), e.y);
}

__global__ __launch_bounds__(kThreads) void kb_bin_scan(const Member* __restrict__ mem,
                                                        const int2* __restrict__ map,
                                                        const int* __restrict__ tcall, int j) {
    const int2 e = map[blockIdx.x];
    const Member& m = mem[e.x];
    bin_scan_body(m.b, batch_set(tcall, m, j) ^ 1, e.y);
}

__global__ __launch_bounds__(kThreads) void kb_bin_scatter(const Member* __restrict__ mem,
                                                           const int2* __restrict__ map, int j) {
    const int2 e = map[blockIdx.x];
    const Member& m = mem[e.x];
    bin_scatter_body(batch_cur(m, j), m.b, e.y);
}

// Final copy of odd-length calls: alt -> pos, kThreads * 8 nodes per block.
__global__ __launch_bounds__(kThreads) void kb_copy(const Member* __restrict__ mem,
                                                    const int2* __restrict__ map) {
    const int2 e = map[blockIdx.x];
    const Member& m = mem[e.x];
    const int beg = e.y * kThreads * 8;
    const int end = min(beg + kThreads * 8, m.b.n);
    for (int i = beg + threadIdx.x; i < end; i += kThreads) m.pos[i] = m.alt[i];
}

void launch_b_box(const Member* mem, const int2* map_begin, int n_begin, const int2* map_red, int n_red,
                  const int* tcall, hipStream_t s) {
    if (n_begin > 0) hipLaunchKernelGGL(kb_box_begin, dim3(n_begin), dim3(kBoxSlots), 0, s, mem, map_begin, tcall);
    if (n_red > 0) hipLaunchKernelGGL(kb_box_reduce, dim3(n_red), dim3(kThreads), 0, s, mem, map_red, tcall);
}

void launch_b_bin_count(const Member* mem, const int2* map, int blocks, size_t lds, const int* tcall, int j,
                        hipStream_t s) {
    if (blocks > 0) hipLaunchKernelGGL(kb_bin_count, dim3(blocks), dim3(kThreads), lds, s, mem, map, tcall, j);
}

void launch_b_bin_scan(const Member* mem, const int2* map, int blocks, const int* tcall, int j, hipStream_t s) {
    if (blocks > 0) hipLaunchKernelGGL(kb_bin_scan, dim3(blocks), dim3(kThreads), 0, s, mem, map, tcall, j);
}

void launch_b_bin_scatter(const Member* mem, const int2* map, int blocks, size_t lds, int j, hipStream_t s) {
    if (blocks > 0) hipLaunchKernelGGL(kb_bin_scatter, dim3(blocks), dim3(kThreads), lds, s, mem, map, j);
}

// End of a call: every slot's counter advances by the call's iterations.
__global__ void kb_advance(int* tcall, int slots, int iters) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < slots) tcall[i] += iters;
}

void launch_b_advance(int* tcall, int slots, int iters, hipStream_t s) {
    if (slots > 0) hipLaunchKernelGGL(kb_advance, dim3((slots + 255) / 256), dim3(256), 0, s, tcall, slots, iters);
}

void launch_b_copy(const Member* mem, const int2* map, int blocks, hipStream_t s) {
    if (blocks > 0) hipLaunchKernelGGL(kb_copy, dim3(blocks), dim3(kThreads), 0, s, mem, map);
}

}  // namespace tfdp
