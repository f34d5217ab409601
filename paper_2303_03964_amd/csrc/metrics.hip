// Layout quality on the device (Sec. 4, "Metrics"): the stress error SE and
// the neighbourhood preservation NP_1, NP_2 estimated from a sample of
// source nodes. Hop distances from up to 64
// sources come from one multi-source BFS with a 64-bit source mask per node
// (a level per launch, pulled from the neighbours' frontier masks; 16-bit
// distances, so graphs of diameter up to kMaxLevel are measured exactly); the
// stress sums over all (source, node) pairs at finite distance are reduced
// per block in float64 and added on the host in block order.
#include <cmath>
#include <cstring>

#include "tfdp_internal.h"

namespace tfdp {

constexpr int kMetricThreads = 256;
// Hop distances are stored as uint16: levels 0 .. kMaxLevel, kUnreached for
// nodes no source reaches. A BFS still finding nodes at level kMaxLevel is
// refused (the distances of farther nodes would not fit).
typedef unsigned short hop_t;
constexpr int kUnreached = 0xffff;
constexpr int kMaxLevel = kUnreached - 1;

// Sources outside [0, n) mark the check flag (read with the CSR check).
__global__ void k_src_check(const int* __restrict__ src, int nsrc, int n, int* bad) {
    const int q = threadIdx.x;
    if (q < nsrc && (src[q] < 0 || src[q] >= n)) *bad = 2;
}

// visited = frontier = the mask of the sources at each node; distances of
// the sources to themselves 0, all others unreached.
__global__ void k_bfs_init(int n, const int* __restrict__ src, int nsrc, unsigned long long* visited,
                           unsigned long long* frontier, hop_t* dist) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    unsigned long long m = 0ull;
    for (int s = 0; s < nsrc; ++s) {
        dist[(size_t)s * n + v] = (hop_t)kUnreached;
        if (src[s] == v) m |= 1ull << s;
    }
    for (int s = 0; s < nsrc; ++s)
        if ((m >> s) & 1ull) dist[(size_t)s * n + v] = 0;
    visited[v] = m;
    frontier[v] = m;
}

// One BFS level: a node joins the frontier of every source that reached a
// neighbour in the previous level and not the node itself.
__global__ void k_bfs_level(int n, const int* __restrict__ row_ptr, const int* __restrict__ col_idx,
                            const unsigned long long* __restrict__ frontier, unsigned long long* next,
                            unsigned long long* visited, hop_t* dist, int level, int* changed) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    unsigned long long acc = 0ull;
    const int e1 = row_ptr[v + 1];
    for (int e = row_ptr[v]; e < e1; ++e) acc |= frontier[col_idx[e]];
    const unsigned long long vis = visited[v];
    const unsigned long long nb = acc & ~vis;
    next[v] = nb;
    if (nb) {
        visited[v] = vis | nb;
        unsigned long long m = nb;
        while (m) {
            const int s = __ffsll((long long)m) - 1;
            m &= m - 1;
            dist[(size_t)s * n + v] = (hop_t)level;
        }
        *changed = 1;
    }
}

// Per block: sums over (source, node) pairs at finite hop distance D >= 1 of r = d / D
// and r^2 (d = layout distance, D = hop distance) and the pair count.
__global__ __launch_bounds__(kMetricThreads) void k_stress_sums(int n, const float2* __restrict__ pos,
                                                               const int* __restrict__ src, int nsrc,
                                                               const hop_t* __restrict__ dist,
                                                               double* partial) {
    __shared__ double red[3][kMetricThreads / 64];
    double sr = 0.0, sr2 = 0.0, cnt = 0.0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const float2 p = pos[v];
        for (int s = 0; s < nsrc; ++s) {
            const int d = dist[(size_t)s * n + v];
            if (d == 0 || d == kUnreached) continue;
            const float2 q = pos[src[s]];
            const double dx = (double)p.x - (double)q.x;
            const double dy = (double)p.y - (double)q.y;
            const double r = sqrt(dx * dx + dy * dy) / (double)d;
            sr += r;
            sr2 += r * r;
            cnt += 1.0;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        sr += __shfl_xor(sr, off);
        sr2 += __shfl_xor(sr2, off);
        cnt += __shfl_xor(cnt, off);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = sr;
        red[1][w] = sr2;
        red[2][w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0, c = 0.0;
        for (int i = 0; i < kMetricThreads / 64; ++i) {
            a += red[0][i];
            b += red[1][i];
            c += red[2][i];
        }
        partial[3 * blockIdx.x + 0] = a;
        partial[3 * blockIdx.x + 1] = b;
        partial[3 * blockIdx.x + 2] = c;
    }
}

constexpr int kStressBlocks = 1024;

// neighbourhood preservation over the BFS distances (below)
int np_sampled(int n, const float2* pos, const int* src, int nsrc, const hop_t* dist, void* extra,
               double* np, hipStream_t s);
size_t np_extra_bytes(int nsrc);

size_t stress_workspace_bytes(int n, int nsrc) {
    size_t b = 0;
    auto take = [&](size_t bytes) { b = (b + 255) & ~(size_t)255; b += bytes; };
    take(sizeof(DevState));       // CSR check flag
    take((size_t)n * 8);          // visited
    take((size_t)n * 8);          // frontier
    take((size_t)n * 8);          // next
    take((size_t)nsrc * n * sizeof(hop_t));  // distances
    take(sizeof(int));            // changed flag
    take((size_t)kStressBlocks * 3 * sizeof(double));
    take(np_extra_bytes(nsrc));
    return (b + 255) & ~(size_t)255;
}

// Returns 0 on success, -1 for an invalid CSR, -2 for a source outside
// [0, n), -3 when the BFS still reaches new nodes at level kMaxLevel, else
// the HIP error; fills SE
// (NaN without pairs) and, when np is not NULL, NP_1 and NP_2.
int stress_sampled(int n, long long nnz, const int* row_ptr, const int* col_idx, const float2* pos, const int* src,
                   int nsrc, void* work, double* se, double* np, int* levels, hipStream_t s) {
    char* base = static_cast<char*>(work);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        void* p = base + off;
        off += bytes;
        return p;
    };
    // the BFS reads every column: check the CSR first (as layout_init does)
    auto* chk = static_cast<DevState*>(take(sizeof(DevState)));
    {
        hipError_t e = hipMemsetAsync(chk, 0, sizeof(DevState), s);
        if (e != hipSuccess) return (int)e;
        launch_csr_check(row_ptr, col_idx, n, nnz, chk, s);
        hipLaunchKernelGGL(k_src_check, dim3(1), dim3(64), 0, s, src, nsrc, n, &chk->pad);
        int bad[2] = {0, 0};  // csr_bad, pad (sources)
        e = hipMemcpyAsync(bad, &chk->csr_bad, 2 * sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return (int)e;
        if (bad[0]) return -1;
        if (bad[1]) return -2;
    }
    auto* visited = static_cast<unsigned long long*>(take((size_t)n * 8));
    auto* frontier = static_cast<unsigned long long*>(take((size_t)n * 8));
    auto* next = static_cast<unsigned long long*>(take((size_t)n * 8));
    auto* dist = static_cast<hop_t*>(take((size_t)nsrc * n * sizeof(hop_t)));
    auto* changed = static_cast<int*>(take(sizeof(int)));
    auto* partial = static_cast<double*>(take((size_t)kStressBlocks * 3 * sizeof(double)));
    void* np_extra = take(np_extra_bytes(nsrc));
    const int blocks = (n + kMetricThreads - 1) / kMetricThreads;
    hipLaunchKernelGGL(k_bfs_init, dim3(blocks), dim3(kMetricThreads), 0, s, n, src, nsrc, visited, frontier, dist);
    int level = 1;
    bool ended = false;
    for (; level <= kMaxLevel; ++level) {
        hipError_t e = hipMemsetAsync(changed, 0, sizeof(int), s);
        if (e != hipSuccess) return (int)e;
        hipLaunchKernelGGL(k_bfs_level, dim3(blocks), dim3(kMetricThreads), 0, s, n, row_ptr, col_idx, frontier,
                           next, visited, dist, level, changed);
        int h = 0;
        e = hipMemcpyAsync(&h, changed, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return (int)e;
        unsigned long long* t = frontier;
        frontier = next;
        next = t;
        if (!h) {
            ended = true;
            break;
        }
    }
    *levels = level;
    if (!ended) return -3;
    hipLaunchKernelGGL(k_stress_sums, dim3(kStressBlocks), dim3(kMetricThreads), 0, s, n, pos, src, nsrc, dist,
                       partial);
    double host[kStressBlocks * 3];  // fixed host buffers: the metric makes no allocation of its own
    hipError_t e = hipMemcpyAsync(host, partial, sizeof(host), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return (int)e;
    double sr = 0.0, sr2 = 0.0, cnt = 0.0;
    for (int b = 0; b < kStressBlocks; ++b) {
        sr += host[3 * b];
        sr2 += host[3 * b + 1];
        cnt += host[3 * b + 2];
    }
    // optimal scale s* = sum r / sum r^2; SE = mean (s* r - 1)^2
    if (cnt > 0.0 && sr2 > 0.0) {
        const double sc = sr / sr2;
        *se = (sc * sc * sr2 - 2.0 * sc * sr + cnt) / cnt;
    } else {
        *se = std::nan("");
    }
    if (np) return np_sampled(n, pos, src, nsrc, dist, np_extra, np, s);
    return 0;
}

}  // namespace tfdp

namespace tfdp {

// ----------------------------------------------------------------- neighbourhood preservation
//
// NP_r for sampled nodes s (Sec. 4, "Metrics"): the k_s = |N_G(s, r)| nearest
// layout neighbours of s (s excluded, distance ties to the lower index)
// against the graph ring N_G(s, r) = {v : 1 <= D(s, v) <= r} from the BFS
// distances; NP_r = mean over sampled nodes with k_s > 0 of the Jaccard
// index |A & B| / |A | B| = o / (2 k_s - o). The k_s-th smallest key
// (squared distance in float64, then the node index) is found per source by
// an exact radix select: eight 8-bit passes over the bits of the squared
// distance, then four over the index among exact ties.

constexpr int kNpBlocks = 128;

__device__ __forceinline__ unsigned long long d2_key(const float2 p, const float2 q) {
#pragma clang fp contract(off)  // the plain sum of the two rounded squares
    const double dx = (double)p.x - (double)q.x;
    const double dy = (double)p.y - (double)q.y;
    return (unsigned long long)__double_as_longlong(dx * dx + dy * dy);  // >= 0: monotone as unsigned
}

// Ring sizes: count[s] += #{v : lo <= D(s, v) <= r}.
__global__ __launch_bounds__(kMetricThreads) void k_ring_count(int n, int nsrc, const hop_t* __restrict__ dist,
                                                              int r, unsigned int* count) {
    __shared__ unsigned int c[64];
    if (threadIdx.x < 64) c[threadIdx.x] = 0;
    __syncthreads();
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        for (int s = 0; s < nsrc; ++s) {
            const int d = dist[(size_t)s * n + v];
            if (d >= 1 && d <= r) atomicAdd(&c[s], 1u);
        }
    __syncthreads();
    if (threadIdx.x < nsrc && c[threadIdx.x]) atomicAdd(&count[threadIdx.x], c[threadIdx.x]);
}

// One radix pass: per source, histogram of digit `shift` of the key among
// nodes whose key matches the source's prefix on `mask`. Phase 0 keys are
// the squared distances; phase 1 keys are node indices among nodes whose
// squared distance equals the selected value (sel[s]).
struct NpSel {
    unsigned long long prefix[64];
    unsigned long long mask[64];
    unsigned long long dsel[64];  // phase 1: the selected squared distance
    int active[64];
};

__global__ __launch_bounds__(kMetricThreads) void k_np_hist(int n, const float2* __restrict__ pos,
                                                           const int* __restrict__ src, int nsrc, NpSel sel,
                                                           int phase, int shift, unsigned int* hist) {
    extern __shared__ unsigned int h[];  // [nsrc][256]
    for (int i = threadIdx.x; i < nsrc * 256; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const float2 p = pos[v];
        for (int s = 0; s < nsrc; ++s) {
            if (!sel.active[s] || v == src[s]) continue;
            const unsigned long long d2 = d2_key(p, pos[src[s]]);
            unsigned long long key;
            if (phase == 0) {
                key = d2;
            } else {
                if (d2 != sel.dsel[s]) continue;
                key = (unsigned long long)v;
            }
            if ((key & sel.mask[s]) != sel.prefix[s]) continue;
            atomicAdd(&h[s * 256 + (int)((key >> shift) & 255ull)], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nsrc * 256; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

// Overlap per source: nodes both in the ring and among the k nearest
// (key below the selected (squared distance, index) pair).
__global__ __launch_bounds__(kMetricThreads) void k_np_overlap(int n, const float2* __restrict__ pos,
                                                              const int* __restrict__ src, int nsrc,
                                                              const hop_t* __restrict__ dist, int r,
                                                              NpSel sel, const unsigned int* __restrict__ isel,
                                                              unsigned int* overlap) {
    __shared__ unsigned int c[64];
    __shared__ float2 sp[64];
    if (threadIdx.x < 64) c[threadIdx.x] = 0;
    if (threadIdx.x < nsrc) sp[threadIdx.x] = pos[src[threadIdx.x]];
    __syncthreads();
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const float2 p = pos[v];
        for (int s = 0; s < nsrc; ++s) {
            if (!sel.active[s] || v == src[s]) continue;
            const int d = dist[(size_t)s * n + v];
            if (d < 1 || d > r) continue;
            const unsigned long long d2 = d2_key(p, sp[s]);
            if (d2 < sel.dsel[s] || (d2 == sel.dsel[s] && (unsigned int)v <= isel[s])) atomicAdd(&c[s], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < nsrc && c[threadIdx.x]) atomicAdd(&overlap[threadIdx.x], c[threadIdx.x]);
}

size_t np_extra_bytes(int) { return ((size_t)64 * 256 * 4 + 256) + ((size_t)64 * 4 + 256) * 3; }

// NP_r for r = 1 and 2 from the BFS distances in the stress workspace (the
// same sources); np[0] = NP_1, np[1] = NP_2 (NaN when no source has a
// non-empty ring).
int np_sampled(int n, const float2* pos, const int* src, int nsrc, const hop_t* dist, void* extra,
               double* np, hipStream_t s) {
    char* base = static_cast<char*>(extra);
    unsigned int* hist = reinterpret_cast<unsigned int*>(base);
    unsigned int* count = reinterpret_cast<unsigned int*>(base + 64 * 256 * 4 + 256);
    unsigned int* isel_d = count + 128;
    unsigned int* overlap = isel_d + 128;
    for (int r = 1; r <= 2; ++r) {
        hipError_t e = hipMemsetAsync(count, 0, 64 * 4, s);
        if (e != hipSuccess) return (int)e;
        hipLaunchKernelGGL(k_ring_count, dim3(kNpBlocks), dim3(kMetricThreads), 0, s, n, nsrc, dist, r, count);
        unsigned int k[64] = {0};
        e = hipMemcpyAsync(k, count, nsrc * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return (int)e;
        NpSel sel;
        std::memset(&sel, 0, sizeof(sel));
        unsigned long long rank[64];
        for (int q = 0; q < nsrc; ++q) {
            sel.active[q] = k[q] > 0 ? 1 : 0;
            rank[q] = k[q];
        }
        unsigned int isel[64] = {0};
        // phase 0: squared distance bits; phase 1: index among ties
        for (int phase = 0; phase < 2; ++phase) {
            const int top = phase == 0 ? 56 : 24;
            for (int shift = top; shift >= 0; shift -= 8) {
                e = hipMemsetAsync(hist, 0, (size_t)nsrc * 256 * 4, s);
                if (e != hipSuccess) return (int)e;
                hipLaunchKernelGGL(k_np_hist, dim3(kNpBlocks), dim3(kMetricThreads), (size_t)nsrc * 256 * 4, s, n,
                                   pos, src, nsrc, sel, phase, shift, hist);
                unsigned int hh[64 * 256];
                e = hipMemcpyAsync(hh, hist, (size_t)nsrc * 256 * 4, hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e != hipSuccess) return (int)e;
                for (int q = 0; q < nsrc; ++q) {
                    if (!sel.active[q]) continue;
                    unsigned long long acc = 0;
                    int dgt = 0;
                    for (; dgt < 256; ++dgt) {
                        const unsigned long long c = hh[(size_t)q * 256 + dgt];
                        if (acc + c >= rank[q]) break;
                        acc += c;
                    }
                    if (dgt > 255) dgt = 255;  // not reached: rank <= candidates
                    rank[q] -= acc;
                    sel.prefix[q] |= (unsigned long long)dgt << shift;
                    sel.mask[q] |= 255ull << shift;
                }
            }
            if (phase == 0) {
                for (int q = 0; q < nsrc; ++q) {
                    sel.dsel[q] = sel.prefix[q];
                    sel.prefix[q] = 0;
                    sel.mask[q] = 0;
                }
            } else {
                for (int q = 0; q < nsrc; ++q) isel[q] = (unsigned int)sel.prefix[q];
            }
        }
        e = hipMemcpyAsync(isel_d, isel, nsrc * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemsetAsync(overlap, 0, 64 * 4, s);
        if (e != hipSuccess) return (int)e;
        hipLaunchKernelGGL(k_np_overlap, dim3(kNpBlocks), dim3(kMetricThreads), 0, s, n, pos, src, nsrc, dist, r, sel,
                           isel_d, overlap);
        unsigned int o[64] = {0};
        e = hipMemcpyAsync(o, overlap, nsrc * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return (int)e;
        double sum = 0.0;
        int used = 0;
        for (int q = 0; q < nsrc; ++q) {
            if (!k[q]) continue;
            sum += (double)o[q] / (2.0 * (double)k[q] - (double)o[q]);
            ++used;
        }
        np[r - 1] = used ? sum / used : std::nan("");
    }
    return 0;
}

}  // namespace tfdp
