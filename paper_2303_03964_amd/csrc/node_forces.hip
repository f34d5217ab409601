// Per-node work of one iteration: back-projection of the grid potentials
// (Sec. 3.4, third step), attraction along the CSR rows (Sec. 3.3, Eq.6-7),
// the displacement D = w_r F^r + F^a and the capped move; or, for the exact
// method (Sec. 3.4), the all-pairs repulsion tiled through LDS.
#include "tfdp_internal.h"

namespace tfdp {

// Attraction, displacement and either the force outputs (pos_out == nullptr)
// or the capped move plus the block's share of the next box.
__device__ __forceinline__ void finish_node(bool active, int i, float2 p, float frx, float fry,
                                            const float2* __restrict__ pos,
                                            const int* __restrict__ row_ptr,
                                            const int* __restrict__ col_idx, const ModelArgs& a,
                                            DevState* st, float2* __restrict__ pos_out,
                                            float2* f_rep, float2* f_att, float2* f_tot) {
    float xmin = INFINITY, ymin = INFINITY, xmax = -INFINITY, ymax = -INFINITY;
    if (active) {
        float fax = 0.f, fay = 0.f;
        const int e1 = row_ptr[i + 1];
        for (int e = row_ptr[i]; e < e1; ++e) {
            const float2 q = pos[col_idx[e]];
            const float dx = p.x - q.x;
            const float dy = p.y - q.y;
            const float f = 1.f + a.beta / (1.f + (dx * dx + dy * dy));
            fax += f * dx;
            fay += f * dy;
        }
        fax *= -a.alpha;
        fay *= -a.alpha;
        const float dxt = a.rep_weight * frx + fax;
        const float dyt = a.rep_weight * fry + fay;
        if (pos_out == nullptr) {
            if (f_rep) f_rep[i] = make_float2(frx, fry);
            if (f_att) f_att[i] = make_float2(fax, fay);
            if (f_tot) f_tot[i] = make_float2(dxt, dyt);
        } else {
            const int t = st->t;
            double c = (double)a.t0 * (1.0 - (double)t / (double)a.total_iters);
            const float cap = c > 0.0 ? (float)c : 0.f;
            const float norm = sqrtf(dxt * dxt + dyt * dyt);
            const float scale = norm > cap ? cap / norm : 1.f;
            const float2 np = make_float2(p.x + dxt * scale, p.y + dyt * scale);
            pos_out[i] = np;
            if (isfinite(np.x) && isfinite(np.y)) {
                xmin = np.x;
                xmax = np.x;
                ymin = np.y;
                ymax = np.y;
            } else {
                st->nonfinite = 1;
            }
        }
    }
    if (pos_out != nullptr) block_minmax_commit(xmin, ymin, xmax, ymax, st);
}

template <int K>
__global__ __launch_bounds__(kThreads) void k_gather(const float2* __restrict__ pos,
                                                     float2* __restrict__ pos_out,
                                                     const int* __restrict__ row_ptr,
                                                     const int* __restrict__ col_idx, Bufs b, Geom g,
                                                     ModelArgs a, float2* f_rep, float2* f_att,
                                                     float2* f_tot) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < b.n;
    float2 p = make_float2(0.f, 0.f);
    float frx = 0.f, fry = 0.f;
    if (active) {
        const Box bx = b.st->box;
        p = pos[i];
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
    finish_node(active, i, p, frx, fry, pos, row_ptr, col_idx, a, b.st, pos_out, f_rep, f_att, f_tot);
}

void launch_gather(const float2* pos, float2* pos_out, const int* row_ptr, const int* col_idx,
                   const Bufs& b, const Geom& g, const ModelArgs& a, float2* f_rep, float2* f_att,
                   float2* f_tot, hipStream_t s) {
    const int blocks = (b.n + kThreads - 1) / kThreads;
    switch (g.k) {
        case 1:
            hipLaunchKernelGGL(k_gather<1>, dim3(blocks), dim3(kThreads), 0, s, pos, pos_out, row_ptr,
                               col_idx, b, g, a, f_rep, f_att, f_tot);
            break;
        case 2:
            hipLaunchKernelGGL(k_gather<2>, dim3(blocks), dim3(kThreads), 0, s, pos, pos_out, row_ptr,
                               col_idx, b, g, a, f_rep, f_att, f_tot);
            break;
        default:
            hipLaunchKernelGGL(k_gather<3>, dim3(blocks), dim3(kThreads), 0, s, pos, pos_out, row_ptr,
                               col_idx, b, g, a, f_rep, f_att, f_tot);
            break;
    }
}

// Exact repulsion: F_i = sum_j K_ij (x_i - x_j), K_ij = (1 + d_ij^2)^-gamma
// (Eq.11; the j = i term is zero), positions streamed through LDS tiles.
__global__ __launch_bounds__(kThreads) void k_brute(const float2* __restrict__ pos, int n,
                                                    float2* __restrict__ pos_out,
                                                    const int* __restrict__ row_ptr,
                                                    const int* __restrict__ col_idx, DevState* st,
                                                    ModelArgs a, float2* f_rep, float2* f_att,
                                                    float2* f_tot) {
    __shared__ float2 tile[kThreads];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < n;
    const float2 p = active ? pos[i] : make_float2(0.f, 0.f);
    const bool g2 = a.gamma == 2.0f;
    float frx = 0.f, fry = 0.f;
    for (int base = 0; base < n; base += kThreads) {
        const int j = base + threadIdx.x;
        tile[threadIdx.x] = j < n ? pos[j] : make_float2(0.f, 0.f);
        __syncthreads();
        const int cnt = min(kThreads, n - base);
        for (int jj = 0; jj < cnt; ++jj) {
            const float2 q = tile[jj];
            const float dx = p.x - q.x;
            const float dy = p.y - q.y;
            const float u = 1.f + (dx * dx + dy * dy);
            float kk;
            if (g2) {
                const float r = 1.f / u;
                kk = r * r;
            } else {
                kk = powf(u, -a.gamma);
            }
            frx += kk * dx;
            fry += kk * dy;
        }
        __syncthreads();
    }
    finish_node(active, i, p, frx, fry, pos, row_ptr, col_idx, a, st, pos_out, f_rep, f_att, f_tot);
}

void launch_brute(const float2* pos, float2* pos_out, const int* row_ptr, const int* col_idx, int n,
                  DevState* st, const ModelArgs& a, float2* f_rep, float2* f_att, float2* f_tot,
                  hipStream_t s) {
    const int blocks = (n + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_brute, dim3(blocks), dim3(kThreads), 0, s, pos, n, pos_out, row_ptr, col_idx,
                       st, a, f_rep, f_att, f_tot);
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
