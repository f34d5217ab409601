// Interpolation grid and FFT convolution of the repulsion (Sec. 3.4,
// Eq.11-15, in offset form).
//
// For grid spacing s = h/k and grid nodes y_g = lo + (g + 1/2) s the kernel
// sums psi_v (Eq.15) are evaluated through three grid charges
//   q_1(g) = sum_i w_ig,  q_dx(g) = sum_i w_ig dx_ig,  q_dy(g) = sum_i w_ig dy_ig
// (d_ig = x_i - y_g) and three grid potentials
//   phi_1 = K * q_1,  G_x = H_x * q_1 - K * q_dx,  G_y = H_y * q_1 - K * q_dy
// with K(a,b) = (1 + s^2 (a^2 + b^2))^-gamma, H_x = K s a, H_y = K s b and *
// the linear convolution over the M x M grid; F_i = sum_g w_ig (d_ig phi_1 + G).
// This is x_i psi_1 - psi_x of Eq.13-14 with every position written relative
// to its grid node, which keeps float32 away from the cancellation of two
// large terms.
//
// Pipeline (all FFTs radix-2 in LDS, length L = power of two >= 2M, the
// linear convolution embedded in an L x L circulant):
//   spread   one block per (interval row, chunk of sorted nodes): per-wave
//            LDS accumulation of the k grid rows, partial rows to HBM
//   rowfft   one block per interval row: sum of the partial rows, real FFT of
//            the k grid rows (two real rows packed per complex FFT);
//            further blocks: FFT of the L kernel rows (K + i H_x packed)
//   colconv  one block per group of spectrum columns: column FFTs of kernel
//            and charges, spectral products, inverse column FFTs
//   rowifft  one block per grid row: inverse real FFT, potentials to HBM
#include <climits>

#include "tfdp_internal.h"

namespace tfdp {

// In-place radix-2 FFTs (decimation in time) of `nfft` contiguous length-L
// complex arrays in LDS, by all threads of the block. tw[j] = exp(-2 pi i j/L),
// j < L/2; `inverse` uses the conjugate twiddles (no scaling).
__device__ void fft_batch(float2* buf, int nfft, int L, int logL, const float2* __restrict__ tw,
                          bool inverse) {
    const int total = nfft << logL;
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
        const int f = t >> logL;
        const int i = t & (L - 1);
        const int j = (int)(__brev((unsigned)i) >> (32 - logL));
        if (i < j) {
            float2* a = buf + (f << logL);
            const float2 tmp = a[i];
            a[i] = a[j];
            a[j] = tmp;
        }
    }
    __syncthreads();
    const int half_total = total >> 1;
    const int hmask = (L >> 1) - 1;
    for (int s = 1; s <= logL; ++s) {
        const int half = 1 << (s - 1);
        const int tshift = logL - s;
        for (int t = threadIdx.x; t < half_total; t += blockDim.x) {
            const int f = t >> (logL - 1);
            const int bi = t & hmask;
            const int p = bi & (half - 1);
            const int i0 = ((bi >> (s - 1)) << s) + p;
            const int i1 = i0 + half;
            float2 w = tw[p << tshift];
            if (inverse) w.y = -w.y;
            float2* a = buf + (f << logL);
            const float2 u = a[i0];
            const float2 v = a[i1];
            const float2 vw = make_float2(v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x);
            a[i0] = make_float2(u.x + vw.x, u.y + vw.y);
            a[i1] = make_float2(u.x - vw.x, u.y - vw.y);
        }
        __syncthreads();
    }
}

__global__ void k_twiddles(float2* tw, int L) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < L / 2) {
        double sn, cs;
        sincospi(-2.0 * (double)j / (double)L, &sn, &cs);
        tw[j] = make_float2((float)cs, (float)sn);
    }
}

void launch_twiddles(float2* tw, int L, hipStream_t s) {
    hipLaunchKernelGGL(k_twiddles, dim3((L / 2 + 255) / 256), dim3(256), 0, s, tw, L);
}

// ----------------------------------------------------------------- spread

template <int K>
__global__ void k_spread(Bufs b, Geom g, int nw) {
    extern __shared__ float acc[];  // [nw][K][M][3]
    const int M = g.m;
    const int per = K * M * 3;
    const int blk = blockIdx.x;
    const int n_int = b.n_int;
    if (blk >= b.chunk_start[n_int]) return;
    int lo = 0, hi = n_int;  // chunk_start[lo] <= blk < chunk_start[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (b.chunk_start[mid] <= blk) lo = mid;
        else hi = mid;
    }
    const int cy = lo;
    const int beg = b.bucket_start[cy] + (blk - b.chunk_start[cy]) * kSpreadChunk;
    const int end = min(beg + kSpreadChunk, b.bucket_start[cy + 1]);
    for (int i = threadIdx.x; i < nw * per; i += blockDim.x) acc[i] = 0.f;
    __syncthreads();
    const Box bx = b.st->box;
    float* my = acc + (threadIdx.x >> 6) * per;
    for (int j = beg + threadIdx.x; j < end; j += blockDim.x) {
        const float2 p = b.spos[j];
        int cx, cyy;
        double tx, ty;
        bin_axis(p.x, bx.lo_x, bx.h, n_int, cx, tx);
        bin_axis(p.y, bx.lo_y, bx.h, n_int, cyy, ty);
        double wx[K], wy[K], dx[K], dy[K];
        lagrange<K>(tx, wx);
        lagrange<K>(ty, wy);
        node_deltas<K>(tx, bx.h, dx);
        node_deltas<K>(ty, bx.h, dy);
#pragma unroll
        for (int bb = 0; bb < K; ++bb) {
#pragma unroll
            for (int a = 0; a < K; ++a) {
                double w;
                {
#pragma clang fp contract(off)
                    w = wx[a] * wy[bb];
                }
                float* cell = my + ((bb * M) + cx * K + a) * 3;
                atomicAdd(cell + 0, (float)w);
                atomicAdd(cell + 1, (float)(w * dx[a]));
                atomicAdd(cell + 2, (float)(w * dy[bb]));
            }
        }
    }
    __syncthreads();
    float* out = b.spart + (size_t)blk * per;
    for (int i = threadIdx.x; i < per; i += blockDim.x) {
        float v = 0.f;
        for (int w = 0; w < nw; ++w) v += acc[w * per + i];
        out[i] = v;
    }
}

static int spread_waves(const Geom& g) {
    const size_t per = (size_t)g.k * g.m * 3 * sizeof(float);
    int nw = 4;
    while (nw > 1 && nw * per > 65536) nw >>= 1;
    return nw;
}

void launch_spread(const Bufs& b, const Geom& g, hipStream_t s) {
    const int nw = spread_waves(g);
    const size_t lds = (size_t)nw * g.k * g.m * 3 * sizeof(float);
    switch (g.k) {
        case 1: hipLaunchKernelGGL(k_spread<1>, dim3(b.max_chunks), dim3(nw * 64), lds, s, b, g, nw); break;
        case 2: hipLaunchKernelGGL(k_spread<2>, dim3(b.max_chunks), dim3(nw * 64), lds, s, b, g, nw); break;
        default: hipLaunchKernelGGL(k_spread<3>, dim3(b.max_chunks), dim3(nw * 64), lds, s, b, g, nw); break;
    }
}

// ----------------------------------------------------------------- row FFTs

__device__ __forceinline__ int signed_offset(int r, int M, int L) {
    return r < M ? r : (r > L - M ? r - L : INT_MIN);
}

__global__ __launch_bounds__(kThreads) void k_rowfft(Bufs b, Geom g, float gamma) {
    extern __shared__ float2 sm2[];
    const int L = g.L, M = g.m, H = g.H, K = g.k;
    if ((int)blockIdx.x < b.n_int) {
        // charges of the K grid rows of interval row cy
        const int cy = blockIdx.x;
        const int c0 = b.chunk_start[cy], c1 = b.chunk_start[cy + 1];
        const int per = K * M * 3;
        float2* z = sm2;                     // [2][L]
        float* q = (float*)(sm2 + 2 * L);    // [M][3] of the current grid row
        for (int bb = 0; bb < K; ++bb) {
            for (int i = threadIdx.x; i < 3 * M; i += blockDim.x) {
                float v = 0.f;
                for (int c = c0; c < c1; ++c) v += b.spart[(size_t)c * per + bb * M * 3 + i];
                q[i] = v;
            }
            __syncthreads();
            for (int x = threadIdx.x; x < L; x += blockDim.x) {
                if (x < M) {
                    z[x] = make_float2(q[3 * x + 0], q[3 * x + 1]);
                    z[L + x] = make_float2(q[3 * x + 2], 0.f);
                } else {
                    z[x] = make_float2(0.f, 0.f);
                    z[L + x] = make_float2(0.f, 0.f);
                }
            }
            __syncthreads();
            fft_batch(z, 2, L, g.logL, b.tw, false);
            const int y = cy * K + bb;
            float2* q1row = b.qrow + ((size_t)0 * M + y) * H;
            float2* qxrow = b.qrow + ((size_t)1 * M + y) * H;
            float2* qyrow = b.qrow + ((size_t)2 * M + y) * H;
            for (int u = threadIdx.x; u < H; u += blockDim.x) {
                const float2 a = z[u];
                const float2 c = z[(L - u) & (L - 1)];
                // Z = FFT(q1 + i qdx): Q1 = (Z(u) + conj Z(L-u))/2, Qdx = (Z(u) - conj Z(L-u))/(2i)
                q1row[u] = make_float2(0.5f * (a.x + c.x), 0.5f * (a.y - c.y));
                qxrow[u] = make_float2(0.5f * (a.y + c.y), -0.5f * (a.x - c.x));
                qyrow[u] = z[L + u];
            }
            __syncthreads();
        }
    } else {
        // kernel row r: FFT over a of K(a, b) + i H_x(a, b); the result is real,
        // its even part is the row spectrum of K, minus its odd part the
        // (imaginary) row spectrum of H_x divided by i
        const int r = blockIdx.x - b.n_int;
        float2* z = sm2;
        float* R1 = b.krow + (size_t)r * H;
        float* R2 = b.krow + (size_t)(L + r) * H;
        const int bt = signed_offset(r, M, L);
        if (bt == INT_MIN) {
            for (int u = threadIdx.x; u < H; u += blockDim.x) {
                R1[u] = 0.f;
                R2[u] = 0.f;
            }
            return;
        }
        const Box bx = b.st->box;
        const double s = bx.h / (double)K;
        for (int a = threadIdx.x; a < L; a += blockDim.x) {
            const int at = signed_offset(a, M, L);
            float2 v = make_float2(0.f, 0.f);
            if (at != INT_MIN) {
                const double d2 = s * s * ((double)at * at + (double)bt * bt);
                const double kk = (gamma == 2.0f) ? 1.0 / ((1.0 + d2) * (1.0 + d2)) : pow(1.0 + d2, -(double)gamma);
                v = make_float2((float)kk, (float)(kk * s * (double)at));
            }
            z[a] = v;
        }
        __syncthreads();
        fft_batch(z, 1, L, g.logL, b.tw, false);
        for (int u = threadIdx.x; u < H; u += blockDim.x) {
            const float a = z[u].x;
            const float c = z[(L - u) & (L - 1)].x;
            R1[u] = 0.5f * (a + c);
            R2[u] = -0.5f * (a - c);
        }
    }
}

void launch_rowfft(const Bufs& b, const Geom& g, float gamma, hipStream_t s) {
    const size_t lds = (size_t)2 * g.L * sizeof(float2) + (size_t)3 * g.m * sizeof(float);
    hipLaunchKernelGGL(k_rowfft, dim3(b.n_int + g.L), dim3(kThreads), lds, s, b, g, gamma);
}

// ----------------------------------------------------------------- column pass

__global__ __launch_bounds__(kThreads) void k_colconv(Bufs b, Geom g) {
    extern __shared__ float2 sm2[];
    const int L = g.L, M = g.m, H = g.H, CW = g.cw, logL = g.logL;
    const int hl = L / 2 + 1;                 // stored half of the even / odd kernel spectra
    const int u0 = blockIdx.x * CW;
    const int n1 = CW * L;
    float2* cq = sm2;                         // [3][CW][L]
    float* kr = (float*)(cq + 3 * n1);        // [CW][hl]  K^ (real, even in v)
    float* hx = kr + CW * hl;                 // [CW][hl]  H_x^ / i (real, even in v)
    float* hy = hx + CW * hl;                 // [CW][hl]  H_y^ / i (real, odd in v)
    const float inv = 1.f / ((float)L * (float)L);
    const Box bx = b.st->box;
    const float s = (float)(bx.h / (double)g.k);
    const float* R1 = b.krow;
    const float* R2 = b.krow + (size_t)L * H;

    // kernel spectra: C1 = FFT_b(R1 + i R2) -> K^ = Re C1, H_x^ = i Im C1
    for (int t = threadIdx.x; t < n1; t += blockDim.x) {
        const int c = t % CW, r = t / CW;
        const int u = u0 + c;
        float2 v = make_float2(0.f, 0.f);
        if (u < H) v = make_float2(R1[(size_t)r * H + u], R2[(size_t)r * H + u]);
        cq[c * L + r] = v;
    }
    __syncthreads();
    fft_batch(cq, CW, L, logL, b.tw, false);
    for (int t = threadIdx.x; t < CW * hl; t += blockDim.x) {
        const int c = t / hl, v = t % hl;
        kr[t] = cq[c * L + v].x * inv;
        hx[t] = cq[c * L + v].y * inv;
    }
    __syncthreads();
    // C2 = FFT_b(s b R1) -> H_y^ = i Im C2
    for (int t = threadIdx.x; t < n1; t += blockDim.x) {
        const int c = t % CW, r = t / CW;
        const int u = u0 + c;
        const int bt = signed_offset(r, M, L);
        float v = 0.f;
        if (u < H && bt != INT_MIN) v = s * (float)bt * R1[(size_t)r * H + u];
        cq[c * L + r] = make_float2(v, 0.f);
    }
    __syncthreads();
    fft_batch(cq, CW, L, logL, b.tw, false);
    for (int t = threadIdx.x; t < CW * hl; t += blockDim.x) {
        const int c = t / hl, v = t % hl;
        hy[t] = cq[c * L + v].y * inv;
    }
    __syncthreads();
    // charge columns (rows y < M nonzero)
    for (int t = threadIdx.x; t < 3 * n1; t += blockDim.x) {
        const int ch = t / n1, rem = t % n1;
        const int c = rem % CW, y = rem / CW;
        const int u = u0 + c;
        float2 v = make_float2(0.f, 0.f);
        if (u < H && y < M) v = b.qrow[((size_t)ch * M + y) * H + u];
        cq[(ch * CW + c) * L + y] = v;
    }
    __syncthreads();
    fft_batch(cq, 3 * CW, L, logL, b.tw, false);
    // phi_1 = K q1; G_x = H_x q1 - K qdx; G_y = H_y q1 - K qdy
    for (int t = threadIdx.x; t < n1; t += blockDim.x) {
        const int c = t / L, v = t % L;
        const int vv = v < hl ? v : L - v;
        const float kk = kr[c * hl + vv];
        const float h1 = hx[c * hl + vv];
        const float h2 = v < hl ? hy[c * hl + vv] : -hy[c * hl + vv];
        const float2 q1 = cq[t], qx = cq[n1 + t], qy = cq[2 * n1 + t];
        cq[t] = make_float2(kk * q1.x, kk * q1.y);
        cq[n1 + t] = make_float2(-h1 * q1.y - kk * qx.x, h1 * q1.x - kk * qx.y);
        cq[2 * n1 + t] = make_float2(-h2 * q1.y - kk * qy.x, h2 * q1.x - kk * qy.y);
    }
    __syncthreads();
    fft_batch(cq, 3 * CW, L, logL, b.tw, true);
    for (int t = threadIdx.x; t < 3 * CW * M; t += blockDim.x) {
        const int ch = t / (CW * M), rem = t % (CW * M);
        const int c = rem % CW, y = rem / CW;
        const int u = u0 + c;
        if (u < H) b.qrow[((size_t)ch * M + y) * H + u] = cq[(ch * CW + c) * L + y];
    }
}

size_t colconv_lds(const Geom& g) {
    return (size_t)3 * g.cw * g.L * sizeof(float2) + (size_t)3 * g.cw * (g.L / 2 + 1) * sizeof(float);
}

void launch_colconv(const Bufs& b, const Geom& g, hipStream_t s) {
    const int blocks = (g.H + g.cw - 1) / g.cw;
    hipLaunchKernelGGL(k_colconv, dim3(blocks), dim3(kThreads), colconv_lds(g), s, b, g);
}

// ----------------------------------------------------------------- inverse rows

__global__ __launch_bounds__(kThreads) void k_rowifft(Bufs b, Geom g) {
    extern __shared__ float2 z[];  // [2][L]
    const int L = g.L, M = g.m, H = g.H;
    const int y = blockIdx.x;
    const float2* p0 = b.qrow + ((size_t)0 * M + y) * H;
    const float2* p1 = b.qrow + ((size_t)1 * M + y) * H;
    const float2* p2 = b.qrow + ((size_t)2 * M + y) * H;
    for (int u = threadIdx.x; u < L; u += blockDim.x) {
        float2 a, c, e;
        if (u < H) {
            a = p0[u];
            c = p1[u];
            e = p2[u];
        } else {  // Hermitian extension of the spectra of real rows
            const int uu = L - u;
            a = make_float2(p0[uu].x, -p0[uu].y);
            c = make_float2(p1[uu].x, -p1[uu].y);
            e = make_float2(p2[uu].x, -p2[uu].y);
        }
        z[u] = make_float2(a.x - c.y, a.y + c.x);  // phi_1 + i G_x
        z[L + u] = e;
    }
    __syncthreads();
    fft_batch(z, 2, L, g.logL, b.tw, true);
    for (int x = threadIdx.x; x < M; x += blockDim.x)
        b.pot[(size_t)y * M + x] = make_float4(z[x].x, z[x].y, z[L + x].x, 0.f);
}

void launch_rowifft(const Bufs& b, const Geom& g, hipStream_t s) {
    hipLaunchKernelGGL(k_rowifft, dim3(g.m), dim3(kThreads), (size_t)2 * g.L * sizeof(float2), s, b, g);
}

}  // namespace tfdp
