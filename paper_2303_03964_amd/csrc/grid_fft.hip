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
// The linear convolution is embedded in an L x L circulant (L = power of two
// >= 2M) and computed with 2D FFTs:
//   spread_rows  one block per interval row: the nodes of the row (sorted by
//                the binning pass) accumulate in per-wave LDS copies of the
//                row's k grid rows, which are summed in a fixed order and
//                real-FFT'd (two real rows per complex FFT); further blocks
//                FFT the kernel rows (K + i H_x packed). Spectra are stored
//                column-major for the column pass.
//   colconv      one block per group of spectrum columns: five forward
//                column FFTs (kernel pair, three charges), spectral products,
//                three inverse column FFTs; results stored row-major.
//   rowifft      inverse real FFTs of the potential rows, (phi_1, G_x, G_y)
//                written per grid node.
//
// Every FFT is a task of one wave: a Stockham autosort FFT with radix-8
// passes (and one radix-4 or radix-2 pass), each lane holding its points in
// registers between LDS exchanges. A task is one transform of length
// L >= 512 or 512/L transforms of a shorter length, so every task has 512 or
// more points and needs no block-wide barrier.
#include <climits>

#include "tfdp_internal.h"

namespace tfdp {

// ----------------------------------------------------------------- wave FFT

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiplication by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2* v) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2* v) {
    const float2 a0 = cadd(v[0], v[2]), a2 = csub(v[0], v[2]);
    const float2 a1 = cadd(v[1], v[3]), a3 = mul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(a0, a1);
    v[1] = cadd(a2, a3);
    v[2] = csub(a0, a1);
    v[3] = csub(a2, a3);
}

// 8-point DFT: three radix-2 decimation-in-frequency stages, output
// reordered from bit-reversed to natural order.
template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
    const float c = 0.70710678118654752f;
    const float2 w1 = INV ? make_float2(c, c) : make_float2(c, -c);
    const float2 w3 = INV ? make_float2(-c, c) : make_float2(-c, -c);
    float2 a[8];
    a[0] = cadd(v[0], v[4]);
    a[4] = csub(v[0], v[4]);
    a[1] = cadd(v[1], v[5]);
    a[5] = cmul(csub(v[1], v[5]), w1);
    a[2] = cadd(v[2], v[6]);
    a[6] = mul_mi<INV>(csub(v[2], v[6]));
    a[3] = cadd(v[3], v[7]);
    a[7] = cmul(csub(v[3], v[7]), w3);
    float2 b[8];
#pragma unroll
    for (int h = 0; h < 8; h += 4) {
        b[h + 0] = cadd(a[h + 0], a[h + 2]);
        b[h + 2] = csub(a[h + 0], a[h + 2]);
        b[h + 1] = cadd(a[h + 1], a[h + 3]);
        b[h + 3] = mul_mi<INV>(csub(a[h + 1], a[h + 3]));
    }
    v[0] = cadd(b[0], b[1]);
    v[4] = csub(b[0], b[1]);
    v[2] = cadd(b[2], b[3]);
    v[6] = csub(b[2], b[3]);
    v[1] = cadd(b[4], b[5]);
    v[5] = csub(b[4], b[5]);
    v[3] = cadd(b[6], b[7]);
    v[7] = csub(b[6], b[7]);
}

template <int R, bool INV>
__device__ __forceinline__ void dft_r(float2* v) {
    if constexpr (R == 8) dft8<INV>(v);
    else if constexpr (R == 4) dft4<INV>(v);
    else dft2<INV>(v);
}

// One Stockham pass of radix 2^LOGR over a task of F transforms of length
// L = 2^LOGL (F L >= 512, contiguous in LDS). 2^LOGNS: length of the
// sub-transforms already combined. Every lane owns NITEMS/64 butterflies;
// all reads of the wave precede its writes (LDS executes a wave's
// operations in order), so the pass is in place.
template <int LOGL, int LOGR, int LOGNS, bool INV>
__device__ __forceinline__ void wave_pass(float2* buf, const float2* __restrict__ tw, int lane) {
    constexpr int L = 1 << LOGL;
    constexpr int R = 1 << LOGR;
    constexpr int F = L < 512 ? 512 / L : 1;
    constexpr int LOGLR = LOGL - LOGR;
    constexpr int NITEMS = F * L / R;
    constexpr int IPL = NITEMS / 64;
    constexpr int TSHIFT = LOGL - LOGNS - LOGR;  // twiddle index = k r 2^TSHIFT
    static_assert(NITEMS % 64 == 0, "task size");
    float2 v[IPL][R];
#pragma unroll
    for (int it = 0; it < IPL; ++it) {
        const int item = lane + it * 64;
        const int f = item >> LOGLR;
        const int j = item & ((1 << LOGLR) - 1);
        const int k = j & ((1 << LOGNS) - 1);
        const float2* src = buf + (f << LOGL) + j;
#pragma unroll
        for (int r = 0; r < R; ++r) v[it][r] = src[r << LOGLR];
        if (LOGNS > 0) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 w = tw[(k * r) << TSHIFT];
                if (INV) w.y = -w.y;
                v[it][r] = cmul(v[it][r], w);
            }
        }
        dft_r<R, INV>(v[it]);
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int it = 0; it < IPL; ++it) {
        const int item = lane + it * 64;
        const int f = item >> LOGLR;
        const int j = item & ((1 << LOGLR) - 1);
        const int k = j & ((1 << LOGNS) - 1);
        float2* dst = buf + (f << LOGL) + ((j >> LOGNS) << (LOGNS + LOGR)) + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[r << LOGNS] = v[it][r];
    }
    __builtin_amdgcn_wave_barrier();
}

template <int LOGL, bool INV, int LOGNS = 0>
__device__ __forceinline__ void wave_fft_passes(float2* buf, const float2* __restrict__ tw, int lane) {
    constexpr int REM = LOGL - LOGNS;
    if constexpr (REM >= 3) {
        wave_pass<LOGL, 3, LOGNS, INV>(buf, tw, lane);
        wave_fft_passes<LOGL, INV, LOGNS + 3>(buf, tw, lane);
    } else if constexpr (REM == 2) {
        wave_pass<LOGL, 2, LOGNS, INV>(buf, tw, lane);
    } else if constexpr (REM == 1) {
        wave_pass<LOGL, 1, LOGNS, INV>(buf, tw, lane);
    }
}

// FFT task of one wave: F = max(1, 512/L) contiguous transforms of length
// L = 2^LOGL; tw[j] = exp(-2 pi i j / L), j < L. Unnormalised; INV uses the
// conjugate roots.
template <int LOGL, bool INV>
__device__ __forceinline__ void wave_fft(float2* buf, const float2* __restrict__ tw, int lane) {
    wave_fft_passes<LOGL, INV, 0>(buf, tw, lane);
}

template <int LOGL>
constexpr int task_ffts() { return (1 << LOGL) < 512 ? 512 / (1 << LOGL) : 1; }

__global__ void k_twiddles(float2* tw, int L) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < L) {
        double sn, cs;
        sincospi(-2.0 * (double)j / (double)L, &sn, &cs);
        tw[j] = make_float2((float)cs, (float)sn);
    }
}

void launch_twiddles(float2* tw, int L, hipStream_t s) {
    hipLaunchKernelGGL(k_twiddles, dim3((L + 255) / 256), dim3(256), 0, s, tw, L);
}

__device__ __forceinline__ int signed_offset(int r, int M, int L) {
    return r < M ? r : (r > L - M ? r - L : INT_MIN);
}

// ----------------------------------------------------------------- spread + row FFTs

// Block size: nw waves (host-chosen, <= 16; <= 8 for L = 2048 so that the
// 2048-point wave FFT keeps its points in registers).
template <int K, int LOGL>
__global__ __launch_bounds__(LOGL >= 11 ? 512 : 1024) void k_spread_rows(Bufs b, Geom g, float gamma, int nw) {
    extern __shared__ float4 smem4[];
    float* sm = reinterpret_cast<float*>(smem4);
    constexpr int L = 1 << LOGL;
    constexpr int logL = LOGL;
    constexpr int F = task_ffts<LOGL>();
    constexpr int TL = F * L;  // points per task
    const int M = g.m, H = g.H;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int n_int = b.n_int;
    if ((int)blockIdx.x < n_int) {
        const int cy = blockIdx.x;
        const int per = K * M * 3;
        for (int i = threadIdx.x; i < nw * per; i += blockDim.x) sm[i] = 0.f;
        __syncthreads();
        const Box bx = b.st->box;
        float* my = sm + w * per;
        const int beg = b.bucket_start[cy], end = b.bucket_start[cy + 1];
        const int stride = nw * 64;
        // wave w takes nodes beg + w*64 + lane + it*stride: a fixed subset
        // and order per wave accumulator, hence a reproducible sum
        for (int j0 = beg + threadIdx.x; j0 < end; j0 += 4 * stride) {
            float2 pp[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) pp[u] = b.spos[min(j0 + u * stride, end - 1)];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (j0 + u * stride >= end) continue;
                const float2 p = pp[u];
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
                        double wt;
                        {
#pragma clang fp contract(off)
                            wt = wx[a] * wy[bb];
                        }
                        float* cell = my + ((bb * M) + cx * K + a) * 3;
                        atomicAdd(cell + 0, (float)wt);
                        atomicAdd(cell + 1, (float)(wt * dx[a]));
                        atomicAdd(cell + 2, (float)(wt * dy[bb]));
                    }
                }
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < per; i += blockDim.x) {
            float v = sm[i];
            for (int ww = 1; ww < nw; ++ww) v += sm[ww * per + i];
            sm[i] = v;
        }
        __syncthreads();
        // 2K real rows packed into K complex pairs: Z = q1 + i qdx, Z' = qdy
        const int nfft = 2 * K;
        const int ntask = (nfft + F - 1) / F;
        float2* z = reinterpret_cast<float2*>(sm + ((per + 3) & ~3));
        for (int i = threadIdx.x; i < ntask * TL; i += blockDim.x) {
            const int f = i >> logL, x = i & (L - 1);
            float2 v = make_float2(0.f, 0.f);
            if (f < nfft && x < M) {
                const float* e = sm + ((f >> 1) * M + x) * 3;
                v = (f & 1) ? make_float2(e[2], 0.f) : make_float2(e[0], e[1]);
            }
            z[i] = v;
        }
        __syncthreads();
        for (int tk = w; tk < ntask; tk += nw) wave_fft<LOGL, false>(z + tk * TL, b.tw, lane);
        __syncthreads();
        for (int i = threadIdx.x; i < K * H; i += blockDim.x) {
            const int bb = i / H, u = i % H;
            const float2* z1 = z + (2 * bb) * L;
            const float2* z2 = z1 + L;
            const float2 a = z1[u];
            const float2 c = z1[(L - u) & (L - 1)];
            const int y = cy * K + bb;
            // Z = FFT(q1 + i qdx): Q1 = (Z(u) + conj Z(L-u))/2, Qdx = (Z(u) - conj Z(L-u))/(2i)
            b.qcol[((size_t)0 * H + u) * M + y] = make_float2(0.5f * (a.x + c.x), 0.5f * (a.y - c.y));
            b.qcol[((size_t)1 * H + u) * M + y] = make_float2(0.5f * (a.y + c.y), -0.5f * (a.x - c.x));
            b.qcol[((size_t)2 * H + u) * M + y] = z2[u];
        }
    } else {
        // kernel rows r: FFT over a of K(a, b) + i H_x(a, b); the result is
        // real, its even part is the row spectrum of K, minus its odd part
        // the row spectrum of H_x divided by i
        const int tk = (blockIdx.x - n_int) * nw + w;
        const int r0 = tk * F;
        if (r0 >= L) return;  // whole wave idle (uniform per wave)
        float2* z = reinterpret_cast<float2*>(sm) + w * TL;
        const Box bx = b.st->box;
        const double s = bx.h / (double)K;
        for (int i = lane; i < TL; i += 64) {
            const int r = r0 + (i >> logL), a = i & (L - 1);
            const int bt = signed_offset(r, M, L), at = signed_offset(a, M, L);
            float2 v = make_float2(0.f, 0.f);
            if (bt != INT_MIN && at != INT_MIN) {
                const double d2 = s * s * ((double)at * at + (double)bt * bt);
                const double kk = (gamma == 2.0f) ? 1.0 / ((1.0 + d2) * (1.0 + d2)) : pow(1.0 + d2, -(double)gamma);
                v = make_float2((float)kk, (float)(kk * s * (double)at));
            }
            z[i] = v;
        }
        __builtin_amdgcn_wave_barrier();
        wave_fft<LOGL, false>(z, b.tw, lane);
        for (int i = lane; i < F * H; i += 64) {
            const int rr = i / H, u = i % H;
            const float2* zr = z + rr * L;
            const float a = zr[u].x;
            const float c = zr[(L - u) & (L - 1)].x;
            const int r = r0 + rr;
            b.kcol[((size_t)0 * H + u) * L + r] = 0.5f * (a + c);
            b.kcol[((size_t)1 * H + u) * L + r] = -0.5f * (a - c);
        }
    }
}

static size_t spread_need(const Geom& g, int nw) {
    const size_t per = (size_t)g.k * g.m * 3 * sizeof(float);
    const int L = g.L;
    const int F = L < 512 ? 512 / L : 1;
    const size_t TL = (size_t)F * L * sizeof(float2);
    const int ntask = (2 * g.k + F - 1) / F;
    size_t need = (size_t)nw * per;
    const size_t fft = ((per + 15) & ~(size_t)15) + ntask * TL;
    if (fft > need) need = fft;
    const size_t krow = (size_t)nw * TL;
    if (krow > need) need = krow;
    return need;
}

static int spread_waves(const Geom& g) {
    int nw = g.L >= 2048 ? 8 : 16;
    while (nw > 4 && spread_need(g, nw) > 150 * 1024) nw >>= 1;
    return nw;
}

// Allow dynamic LDS beyond 64 KB (gfx950 has 160 KB per workgroup); once per kernel.
template <class Kern>
static void allow_big_lds(Kern k) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
}

template <int K, int LOGL>
static void launch_spread_rows_t(const Bufs& b, const Geom& g, float gamma, hipStream_t s) {
    static const bool once = (allow_big_lds(k_spread_rows<K, LOGL>), true);
    (void)once;
    const int nw = spread_waves(g);
    const size_t lds = spread_need(g, nw);
    constexpr int F = task_ffts<LOGL>();
    const int ktasks = g.L / F;
    const int blocks = b.n_int + (ktasks + nw - 1) / nw;
    hipLaunchKernelGGL((k_spread_rows<K, LOGL>), dim3(blocks), dim3(nw * 64), lds, s, b, g, gamma, nw);
}

template <int K>
static void launch_spread_rows_k(const Bufs& b, const Geom& g, float gamma, hipStream_t s) {
    switch (g.logL) {
        case 6: launch_spread_rows_t<K, 6>(b, g, gamma, s); break;
        case 7: launch_spread_rows_t<K, 7>(b, g, gamma, s); break;
        case 8: launch_spread_rows_t<K, 8>(b, g, gamma, s); break;
        case 9: launch_spread_rows_t<K, 9>(b, g, gamma, s); break;
        case 10: launch_spread_rows_t<K, 10>(b, g, gamma, s); break;
        default: launch_spread_rows_t<K, 11>(b, g, gamma, s); break;
    }
}

void launch_spread_rows(const Bufs& b, const Geom& g, float gamma, hipStream_t s) {
    switch (g.k) {
        case 1: launch_spread_rows_k<1>(b, g, gamma, s); break;
        case 2: launch_spread_rows_k<2>(b, g, gamma, s); break;
        default: launch_spread_rows_k<3>(b, g, gamma, s); break;
    }
}

// ----------------------------------------------------------------- column pass

// Columns u0 .. u0+F-1 (F = transforms per task). Forward column FFTs of
//   C1 = FFT_b(R1 + i R2)   -> K^ = Re C1, H_x^ = i Im C1   (both real-even rows)
//   C2 = FFT_b(s b R1)      -> H_y^ = i Im C2                (real-odd rows)
//   Q1, Qdx, Qdy            (charge row spectra, rows y < M)
// then phi_1 = K^ Q1, G_x = H_x^ Q1 - K^ Qdx, G_y = H_y^ Q1 - K^ Qdy (scaled by
// 1/L^2) and three inverse column FFTs; rows y < M stored row-major.
template <int LOGL>
__global__ __launch_bounds__(512) void k_colconv(Bufs b, Geom g) {
    extern __shared__ float2 sm2[];
    constexpr int L = 1 << LOGL;
    constexpr int logL = LOGL;
    constexpr int F = task_ffts<LOGL>();
    constexpr int TL = F * L;
    const int M = g.m, H = g.H;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int u0 = blockIdx.x * F;
    const Box bx = b.st->box;
    const float s = (float)(bx.h / (double)g.k);
    const float inv = 1.f / ((float)L * (float)L);
    const float* R1 = b.kcol;
    const float* R2 = b.kcol + (size_t)H * L;
    // task c (0..4) of transform f covers column u0 + f
    for (int i = threadIdx.x; i < TL; i += blockDim.x) {
        const int f = i >> logL, r = i & (L - 1);
        const int u = u0 + f;
        float r1 = 0.f, r2 = 0.f;
        if (u < H) {
            r1 = R1[(size_t)u * L + r];
            r2 = R2[(size_t)u * L + r];
        }
        const int bt = signed_offset(r, M, L);
        sm2[i] = make_float2(r1, r2);
        sm2[TL + i] = make_float2(bt != INT_MIN ? s * (float)bt * r1 : 0.f, 0.f);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float2 v = make_float2(0.f, 0.f);
            if (u < H && r < M) v = b.qcol[((size_t)ch * H + u) * M + r];
            sm2[(2 + ch) * TL + i] = v;
        }
    }
    __syncthreads();
    if (w < 5) wave_fft<LOGL, false>(sm2 + w * TL, b.tw, lane);
    __syncthreads();
    for (int i = threadIdx.x; i < TL; i += blockDim.x) {
        const float kk = sm2[i].x * inv;
        const float h1 = sm2[i].y * inv;
        const float h2 = sm2[TL + i].y * inv;
        const float2 q1 = sm2[2 * TL + i], qx = sm2[3 * TL + i], qy = sm2[4 * TL + i];
        sm2[2 * TL + i] = make_float2(kk * q1.x, kk * q1.y);
        sm2[3 * TL + i] = make_float2(-h1 * q1.y - kk * qx.x, h1 * q1.x - kk * qx.y);
        sm2[4 * TL + i] = make_float2(-h2 * q1.y - kk * qy.x, h2 * q1.x - kk * qy.y);
    }
    __syncthreads();
    if (w < 3) wave_fft<LOGL, true>(sm2 + (2 + w) * TL, b.tw, lane);
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * F * M; i += blockDim.x) {
        const int ch = i / (F * M), rem = i % (F * M);
        const int f = rem % F, y = rem / F;
        const int u = u0 + f;
        if (u < H) b.prow[((size_t)ch * M + y) * H + u] = sm2[(2 + ch) * TL + f * L + y];
    }
}

template <int LOGL>
static void launch_colconv_t(const Bufs& b, const Geom& g, hipStream_t s) {
    static const bool once = (allow_big_lds(k_colconv<LOGL>), true);
    (void)once;
    constexpr int F = task_ffts<LOGL>();
    const int blocks = (g.H + F - 1) / F;
    const size_t lds = (size_t)5 * F * g.L * sizeof(float2);
    hipLaunchKernelGGL(k_colconv<LOGL>, dim3(blocks), dim3(512), lds, s, b, g);
}

void launch_colconv(const Bufs& b, const Geom& g, hipStream_t s) {
    switch (g.logL) {
        case 6: launch_colconv_t<6>(b, g, s); break;
        case 7: launch_colconv_t<7>(b, g, s); break;
        case 8: launch_colconv_t<8>(b, g, s); break;
        case 9: launch_colconv_t<9>(b, g, s); break;
        case 10: launch_colconv_t<10>(b, g, s); break;
        default: launch_colconv_t<11>(b, g, s); break;
    }
}

// ----------------------------------------------------------------- inverse rows

// Grid rows y0 .. y0+2F-1: four tasks of F transforms, the first two hold
// phi_1 + i G_x of F rows each, the last two G_y.
template <int LOGL>
__global__ __launch_bounds__(kThreads) void k_rowifft(Bufs b, Geom g) {
    extern __shared__ float2 z[];
    constexpr int L = 1 << LOGL;
    constexpr int logL = LOGL;
    constexpr int F = task_ffts<LOGL>();
    constexpr int TL = F * L;
    const int M = g.m, H = g.H;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int RB = 2 * F;
    const int y0 = blockIdx.x * RB;
    for (int i = threadIdx.x; i < RB * L; i += blockDim.x) {
        const int rr = i >> logL, u = i & (L - 1);
        const int y = y0 + rr;
        float2 a = make_float2(0.f, 0.f), c = a, e = a;
        if (y < M) {
            const float2* p0 = b.prow + ((size_t)0 * M + y) * H;
            const float2* p1 = b.prow + ((size_t)1 * M + y) * H;
            const float2* p2 = b.prow + ((size_t)2 * M + y) * H;
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
        }
        z[i] = make_float2(a.x - c.y, a.y + c.x);  // phi_1 + i G_x
        z[2 * TL + i] = e;
    }
    __syncthreads();
    wave_fft<LOGL, true>(z + w * TL, b.tw, lane);
    __syncthreads();
    for (int i = threadIdx.x; i < RB * M; i += blockDim.x) {
        const int rr = i / M, x = i % M;
        const int y = y0 + rr;
        if (y < M) {
            const float2 v = z[rr * L + x];
            b.pot[(size_t)y * M + x] = make_float4(v.x, v.y, z[2 * TL + rr * L + x].x, 0.f);
        }
    }
}

template <int LOGL>
static void launch_rowifft_t(const Bufs& b, const Geom& g, hipStream_t s) {
    constexpr int F = task_ffts<LOGL>();
    const int blocks = (g.m + 2 * F - 1) / (2 * F);
    hipLaunchKernelGGL(k_rowifft<LOGL>, dim3(blocks), dim3(kThreads), (size_t)4 * F * g.L * sizeof(float2), s, b, g);
}

void launch_rowifft(const Bufs& b, const Geom& g, hipStream_t s) {
    switch (g.logL) {
        case 6: launch_rowifft_t<6>(b, g, s); break;
        case 7: launch_rowifft_t<7>(b, g, s); break;
        case 8: launch_rowifft_t<8>(b, g, s); break;
        case 9: launch_rowifft_t<9>(b, g, s); break;
        case 10: launch_rowifft_t<10>(b, g, s); break;
        default: launch_rowifft_t<11>(b, g, s); break;
    }
}

}  // namespace tfdp
