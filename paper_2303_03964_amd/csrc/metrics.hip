// Layout quality on the device (Sec. 4, "Metrics"): the stress error SE
// estimated from a sample of source nodes. Hop distances from up to 64
// sources come from one multi-source BFS with a 64-bit source mask per node
// (a level per launch, pulled from the neighbours' frontier masks); the
// stress sums over all (source, node) pairs at finite distance are reduced
// per block in float64 and added on the host in block order.
#include <cmath>
#include <vector>

#include "tfdp_internal.h"

namespace tfdp {

constexpr int kMetricThreads = 256;

// visited = frontier = the mask of the sources at each node; distances of
// the sources to themselves 0, all others unreached (255).
__global__ void k_bfs_init(int n, const int* __restrict__ src, int nsrc, unsigned long long* visited,
                           unsigned long long* frontier, unsigned char* dist) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    unsigned long long m = 0ull;
    for (int s = 0; s < nsrc; ++s) {
        dist[(size_t)s * n + v] = 255;
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
                            unsigned long long* visited, unsigned char* dist, int level, int* changed) {
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
            dist[(size_t)s * n + v] = (unsigned char)level;
        }
        *changed = 1;
    }
}

// Per block: sums over (source, node) pairs with 1 <= D < 255 of r = d / D
// and r^2 (d = layout distance, D = hop distance) and the pair count.
__global__ __launch_bounds__(kMetricThreads) void k_stress_sums(int n, const float2* __restrict__ pos,
                                                               const int* __restrict__ src, int nsrc,
                                                               const unsigned char* __restrict__ dist,
                                                               double* partial) {
    __shared__ double red[3][kMetricThreads / 64];
    double sr = 0.0, sr2 = 0.0, cnt = 0.0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const float2 p = pos[v];
        for (int s = 0; s < nsrc; ++s) {
            const int d = dist[(size_t)s * n + v];
            if (d == 0 || d == 255) continue;
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

size_t stress_workspace_bytes(int n, int nsrc) {
    size_t b = 0;
    auto take = [&](size_t bytes) { b = (b + 255) & ~(size_t)255; b += bytes; };
    take(sizeof(DevState));       // CSR check flag
    take((size_t)n * 8);          // visited
    take((size_t)n * 8);          // frontier
    take((size_t)n * 8);          // next
    take((size_t)nsrc * n);       // distances
    take(sizeof(int));            // changed flag
    take((size_t)kStressBlocks * 3 * sizeof(double));
    return (b + 255) & ~(size_t)255;
}

// Returns 0 on success, -1 for an invalid CSR, else the HIP error; fills SE
// (NaN without pairs).
int stress_sampled(int n, long long nnz, const int* row_ptr, const int* col_idx, const float2* pos, const int* src,
                   int nsrc, void* work, double* se, int* levels, hipStream_t s) {
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
        int bad = 0;
        e = hipMemcpyAsync(&bad, &chk->csr_bad, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return (int)e;
        if (bad) return -1;
    }
    auto* visited = static_cast<unsigned long long*>(take((size_t)n * 8));
    auto* frontier = static_cast<unsigned long long*>(take((size_t)n * 8));
    auto* next = static_cast<unsigned long long*>(take((size_t)n * 8));
    auto* dist = static_cast<unsigned char*>(take((size_t)nsrc * n));
    auto* changed = static_cast<int*>(take(sizeof(int)));
    auto* partial = static_cast<double*>(take((size_t)kStressBlocks * 3 * sizeof(double)));
    const int blocks = (n + kMetricThreads - 1) / kMetricThreads;
    hipLaunchKernelGGL(k_bfs_init, dim3(blocks), dim3(kMetricThreads), 0, s, n, src, nsrc, visited, frontier, dist);
    int level = 1;
    for (; level < 255; ++level) {
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
        if (!h) break;
    }
    *levels = level;
    hipLaunchKernelGGL(k_stress_sums, dim3(kStressBlocks), dim3(kMetricThreads), 0, s, n, pos, src, nsrc, dist,
                       partial);
    std::vector<double> host((size_t)kStressBlocks * 3);
    hipError_t e = hipMemcpyAsync(host.data(), partial, host.size() * sizeof(double), hipMemcpyDeviceToHost, s);
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
    return 0;
}

}  // namespace tfdp
