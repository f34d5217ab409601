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
// The linear convolution is embedded in an L x L circulant (L = the smallest
// 2^a or 3 * 2^a >= 2M, see make_geom) and computed with 2D FFTs:
//   spread   one block per chunk of an interval row's nodes (sorted by the
//            binning pass): per-wave LDS copies of the row's k grid rows,
//            summed in a fixed order, written as one partial row set
//   rowfft   RB grid rows per block: partial rows summed straight into the
//            FFT inputs (q1 + i qdx per row, qdy of two rows in one complex
//            transform), row spectra stored column-major in tiles of RB
//            consecutive rows (one cache line per column); further blocks do
//            the same for the kernel rows (K + i H_x packed)
//   colconv  one block per one or two groups of spectrum columns: four
//            forward column FFTs per group (kernel spectra, three charges),
//            spectral products, three inverse column FFTs; contiguous column
//            reads and writes
//   rowifft  RB potential rows per block from column tiles: inverse real
//            FFTs, (phi_1, G_x, G_y) written per grid node.
//
// Every FFT is a task of one wave: a Stockham autosort FFT with a radix-3
// pass when 3 divides L, then radix-8 passes (and one radix-4 or radix-2
// pass), each lane holding its points in registers between LDS exchanges. A
// task is F transforms (FftLen<L>::F: 512 or more points for L = 2^a, 1536
// for L = 3 * 2^a, so that every pass gives each lane whole butterflies) and
// needs no block-wide barrier.
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

// 3-point DFT: X1,2 = v0 - (v1 + v2)/2 -/+ i sin(2 pi/3) (v1 - v2) (forward;
// the signs of the i terms swap for the inverse).
template <bool INV>
__device__ __forceinline__ void dft3(float2* v) {
    const float c = 0.86602540378443865f;
    const float2 t1 = cadd(v[1], v[2]);
    const float2 t2 = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
    const float2 d = csub(v[1], v[2]);
    const float2 t3 = INV ? make_float2(-c * d.y, c * d.x) : make_float2(c * d.y, -c * d.x);
    v[0] = cadd(v[0], t1);
    v[1] = cadd(t2, t3);
    v[2] = csub(t2, t3);
}

template <int R, bool INV>
__device__ __forceinline__ void dft_r(float2* v) {
    if constexpr (R == 8) dft8<INV>(v);
    else if constexpr (R == 4) dft4<INV>(v);
    else if constexpr (R == 3) dft3<INV>(v);
    else dft2<INV>(v);
}

// Transforms per wave task for length L.
template <int L>
struct FftLen {
    static constexpr bool R3 = (L % 3) == 0;
    static constexpr int F = fft_task_ffts(L);
    static_assert(F >= 1 && (R3 ? 1536 % L == 0 : (L & (L - 1)) == 0), "FFT length");
};

// FFT buffers of power-of-two lengths are padded in LDS by one element per
// 32 (element i at zp<L>(i)): the passes' writes, strided by R or NS R
// elements, then spread over the LDS banks instead of falling on a few
// (batched column pass at L = 256: 5.6 -> 1.2 conflict cycles per LDS
// instruction, 22 % fewer wave cycles). Lengths and task sizes are multiples
// of 32, so a task starting at zp(t) holds its element i at zp(t) + zp(i).
// Radix-3 lengths, whose strides conflict little, stay unpadded: the index
// arithmetic doubled their registers.
__host__ __device__ constexpr int zp_len(int L, int i) { return L % 3 == 0 ? i : i + (i >> 5); }
template <int L>
__device__ __forceinline__ constexpr int zp(int i) { return zp_len(L, i); }

// One Stockham pass of radix R over a task of F transforms of length L
// (contiguous in LDS); NS: length of the sub-transforms already combined.
// Every lane owns F L / (64 R) butterflies; all reads of the wave precede its
// writes (LDS executes a wave's operations in order), so the pass is in
// place.
template <int L, int R, int NS, bool INV>
__device__ __forceinline__ void wave_pass(float2* buf, const float2* __restrict__ tw, int lane) {
    constexpr int F = FftLen<L>::F;
    constexpr int N = L / R;             // butterflies per transform
    constexpr int NITEMS = F * N;
    constexpr int IPL = NITEMS / 64;
    constexpr int TSTEP = L / (NS * R);  // twiddle index = k r TSTEP
    static_assert(NITEMS % 64 == 0 && L % (NS * R) == 0, "task size");
    float2 v[IPL][R];
#pragma unroll
    for (int it = 0; it < IPL; ++it) {
        const int item = lane + it * 64;
        const int f = item / N;
        const int j = item % N;
        const int k = j % NS;
#pragma unroll
        for (int r = 0; r < R; ++r) v[it][r] = buf[zp<L>(f * L + j + r * N)];
        if (NS > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 w = tw[k * r * TSTEP];
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
        const int f = item / N;
        const int j = item % N;
        const int k = j % NS;
        const int d0 = f * L + (j / NS) * (NS * R) + k;
#pragma unroll
        for (int r = 0; r < R; ++r) buf[zp<L>(d0 + r * NS)] = v[it][r];
    }
    __builtin_amdgcn_wave_barrier();
}

template <int L, bool INV, int NS = 1>
__device__ __forceinline__ void wave_fft_passes(float2* buf, const float2* __restrict__ tw, int lane) {
    if constexpr (NS == 1 && FftLen<L>::R3) {
        wave_pass<L, 3, 1, INV>(buf, tw, lane);
        wave_fft_passes<L, INV, 3>(buf, tw, lane);
    } else {
        constexpr int REM = L / NS;  // a power of two
        if constexpr (REM >= 8) {
            wave_pass<L, 8, NS, INV>(buf, tw, lane);
            wave_fft_passes<L, INV, NS * 8>(buf, tw, lane);
        } else if constexpr (REM == 4) {
            wave_pass<L, 4, NS, INV>(buf, tw, lane);
        } else if constexpr (REM == 2) {
            wave_pass<L, 2, NS, INV>(buf, tw, lane);
        }
    }
}

// FFT task of one wave: F contiguous transforms of length L (element i at
// buf[zp<L>(i)]); tw[j] = exp(-2 pi i j / L), j < L. Unnormalised; INV uses the
// conjugate roots.
template <int L, bool INV>
__device__ __forceinline__ void wave_fft(float2* buf, const float2* __restrict__ tw, int lane) {
    wave_fft_passes<L, INV, 1>(buf, tw, lane);
}

template <int L>
constexpr int task_ffts() { return FftLen<L>::F; }

// The block's copy of the twiddle table in LDS (after its transform area):
// the passes then read their twiddles at LDS latency instead of from L2.
// The caller synchronises the block before the first transform.
template <int L>
__device__ __forceinline__ const float2* stage_twiddles(float2* lds, const float2* __restrict__ tw) {
    for (int i = threadIdx.x; i < L; i += blockDim.x) lds[i] = tw[i];
    return lds;
}

// Every FFT length make_geom can choose: 2^a (64 .. 2048) and 3 * 2^a
// (384, 768, 1536).
#define TFDP_L_SWITCH(len, CALL)        \
    switch (len) {                      \
        case 64: CALL(64); break;       \
        case 128: CALL(128); break;     \
        case 256: CALL(256); break;     \
        case 384: CALL(384); break;     \
        case 512: CALL(512); break;     \
        case 768: CALL(768); break;     \
        case 1024: CALL(1024); break;   \
        case 1536: CALL(1536); break;   \
        default: CALL(2048); break;     \
    }

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

// Rows per block of the row passes: RB grid rows make 1.5 RB transforms;
// RBK kernel rows make RBK transforms. Column tiles of RB (RBK) consecutive
// rows are stored with one RB * 8-byte write per column; pairs of logical
// blocks share an XCD so that a line is filled from fewer L2s.
// Longest FFT length whose batched tiles the autotuner may choose (rows per
// block 2, 4, 8; column groups 1, 2); longer lengths keep RowTile<L>::RBB
// and col_groups(L, true).
constexpr int kMaxTunedL = 768;

// Kernel rows per block of the spreading launch. Four rows from L = 768 on
// (less LDS per block, so more spreading blocks per CU) measured: 1M nodes
// k = 3 spread 54.5 -> 52.8 us, the 512-graph batch's k = 3 spread at
// L = 768 1014 -> 1094 us (twice the kernel-row blocks); kept at eight.
__host__ __device__ constexpr int kernel_row_tile(int) { return 8; }

template <int L>
struct RowTile {
    // few rows per block at small L so that a 256 x 256 grid still makes
    // 128 blocks (measured: RB 8 -> 2 took the k = 1 row passes at N_int 256
    // from 17.5 + 11.2 us to 10.3 + 8.5 us)
    static constexpr int RB = L <= 512 ? 2 : 4;
    // batched launches have blocks of many graphs to fill the chip: more
    // rows per block at short lengths (512-graph workload: 2.49e9 ->
    // 2.73e9 node-it/s with 8 rows at L <= 256; 4 and 16 rows were slower)
    static constexpr int RBB = L <= 256 ? 8 : RB;
    static constexpr int RBK = kernel_row_tile(L);
    // a single grid at L = 512 has only M / 2 = 128 row blocks: eight waves
    // halve each thread's partial-row loads and column stores (the k = 1
    // forward row pass at N_int 256: 8.0 -> 5.7 us against four waves)
    static constexpr int THREADS = L <= 256 ? 256 : 512;
    // batched blocks at L = 768 have three transform tasks (two transforms
    // each): four waves, so that two blocks of ~170-VGPR waves share a CU
    // (a single grid of 384 rows keeps eight: its 96 blocks are too few)
    static constexpr int THREADS_B = (L <= 512 || L == 768) ? 256 : 512;
};

// Allow dynamic LDS beyond 64 KB (gfx950 has 160 KB per workgroup, static
// and dynamic together); once per kernel.
template <class Kern>
static void allow_big_lds(Kern k) {
    hipFuncAttributes fa;
    int stat = 0;
    if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(k)) == hipSuccess) stat = (int)fa.sharedSizeBytes;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024 - stat);
}

// ----------------------------------------------------------------- spread + kernel rows

// Blocks [0, chunk_blocks): the work chunks the binning pass listed, block
// bid taking chunks bid, bid + chunk_blocks, ...: up to kSpreadChunk sorted
// nodes of one interval row, or a group of sparse consecutive rows (batched
// launches), accumulated into the rows' K grid rows in LDS (exact
// fixed-point sums, hence reproducible) and written as one partial row set
// per row.
// Blocks past chunk_blocks: RBK kernel rows each, FFT over a of
// K(a, b) + i H_x(a, b); the result is real, its even part the row spectrum of
// K, minus its odd part the row spectrum of H_x divided by i.
// bid < chunk_blocks: chunk block; otherwise lb = logical kernel-row block.
template <int K, int L>
__device__ __forceinline__ void spread_body(const Bufs& b, const Geom& g, float gamma, float tau, int nw, int bid,
                                            int lb) {
    extern __shared__ float4 smem4[];
    const int M = g.m;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    if (bid < b.chunk_blocks) {
        // One block-wide copy of the interval row's K grid rows in 64-bit
        // fixed point (units of 2^-32; offsets in interval units): integer
        // LDS atomics are exact, so the sums do not depend on the order of
        // the adds, and they run several times faster than float LDS
        // atomics. A chunk holds at most kSpreadChunk nodes with Lagrange
        // weights of magnitude < 2, far from the 2^63 limit.
        unsigned long long* acc = reinterpret_cast<unsigned long long*>(smem4);  // [rows][K][M][3]
        __shared__ int slot[kSpreadGroupRows];
        const int per = K * M * 3;
        const int n_int = b.n_int;
        const int nwork = b.wchunk[b.max_chunks].x;
        // work chunks bid, bid + chunk_blocks, ... (block-uniform loop)
        for (int blk = bid; blk < nwork; blk += b.chunk_blocks) {
        const int4 wc = b.wchunk[blk];
        const int row0 = wc.x, nrows = wc.y, beg = wc.z, end = wc.w;
        // partial row of each covered row: one per row of a group, else this
        // chunk's place among its row's chunks
        if (threadIdx.x < nrows)
            slot[threadIdx.x] = nrows > 1 ? b.chunk_start[row0 + threadIdx.x]
                                          : b.chunk_start[row0] + (beg - b.bucket_start[row0]) / kSpreadChunk;
        for (int i = threadIdx.x; i < nrows * per; i += blockDim.x) acc[i] = 0ull;
        __syncthreads();
        const Box bx = b.st->box;
        constexpr double kFix = 4294967296.0;  // 2^32
        const int stride = blockDim.x;
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
                // the node's row inside the chunk (the binning pass put it in
                // row cyy by the same computation)
                unsigned long long* racc = acc + (size_t)min(max(cyy - row0, 0), nrows - 1) * per;
                double wx[K], wy[K], ux[K], uy[K];
                lagrange<K>(tx, wx);
                lagrange<K>(ty, wy);
                node_deltas<K>(tx, 1.0, ux);
                node_deltas<K>(ty, 1.0, uy);
#pragma unroll
                for (int bb = 0; bb < K; ++bb) {
#pragma unroll
                    for (int a = 0; a < K; ++a) {
                        double wt;
                        {
#pragma clang fp contract(off)
                            wt = wx[a] * wy[bb];
                        }
                        unsigned long long* cell = racc + ((bb * M) + cx * K + a) * 3;
                        atomicAdd(cell + 0, (unsigned long long)__double2ll_rn(wt * kFix));
                        atomicAdd(cell + 1, (unsigned long long)__double2ll_rn(wt * ux[a] * kFix));
                        atomicAdd(cell + 2, (unsigned long long)__double2ll_rn(wt * uy[bb] * kFix));
                    }
                }
            }
        }
        __syncthreads();
        // partial rows stay in fixed point: the row pass sums the chunks of a
        // row exactly, so no result depends on how a row is cut into chunks
        for (int i = threadIdx.x; i < nrows * per; i += blockDim.x) {
            const int q = i / per;
            b.spart[(size_t)slot[q] * per + (i - q * per)] = acc[i];
        }
        __syncthreads();  // acc and slot are reused by the next work chunk
        }
        return;
    }
    constexpr int F = task_ffts<L>();
    constexpr int TL = F * L;
    constexpr int RBK = RowTile<L>::RBK;
    constexpr int NKT = (RBK + F - 1) / F;
    float2* z = reinterpret_cast<float2*>(smem4);
    const int H = g.H;
    const int r0 = lb * RBK;
    const Box bx = b.st->box;
    const double s = bx.h / (double)K;
    for (int i = threadIdx.x; i < NKT * TL; i += blockDim.x) {
        const int f = i / L, a = i % L;
        const int r = r0 + f;
        float2 v = make_float2(0.f, 0.f);
        if (f < RBK && r <= L / 2) {
            const int bt = signed_offset(r, M, L), at = signed_offset(a, M, L);
            if (bt != INT_MIN && at != INT_MIN) {
                const double d2 = (double)tau * (s * s * ((double)at * at + (double)bt * bt));
                const double kk = (gamma == 2.0f) ? 1.0 / ((1.0 + d2) * (1.0 + d2)) : pow(1.0 + d2, -(double)gamma);
                v = make_float2((float)kk, (float)(kk * s * (double)at));
            }
        }
        z[zp<L>(i)] = v;
    }
    const float2* tws = stage_twiddles<L>(z + zp<L>(NKT * TL), b.tw);
    __syncthreads();
    for (int tk = w; tk < NKT; tk += nw) wave_fft<L, false>(z + zp<L>(tk * TL), tws, lane);
    __syncthreads();
    // K and H_x are even in the row offset, so rows r and L - r of the
    // table are equal: rows 0 .. L/2 are transformed and stored once (the
    // column pass reads row L - r for r > L/2)
    constexpr int KH = L / 2 + 1;
    for (int i = threadIdx.x; i < H * RBK; i += blockDim.x) {
        const int f = i % RBK, u = i / RBK;
        const int r = r0 + f;
        if (r > L / 2) continue;
        const float a = z[zp<L>(f * L + u)].x;
        const float c = z[zp<L>(f * L + (u == 0 ? 0 : L - u))].x;
        b.kcol[(size_t)u * KH + r] = make_float2(0.5f * (a + c), -0.5f * (a - c));
    }
}

template <int K, int L>
__global__ __launch_bounds__(512) void k_spread(Bufs b, Geom g, float gamma, float tau, int nw, int nkb) {
    grid_pass_priority();
    const int bid = blockIdx.x;
    int lb = -1;
    if (bid >= b.chunk_blocks) {
        lb = xcd_pair_block(bid - b.chunk_blocks, nkb);
        if (lb < 0) return;
    }
    spread_body<K, L>(b, g, gamma, tau, nw, bid, lb);
}

// Batched: map entry {member, block}; blocks past the member's chunk_blocks
// are its logical kernel-row blocks.
template <int K, int L>
__global__ __launch_bounds__(512) void kb_spread(const Member* __restrict__ mem, const int2* __restrict__ map) {
    const int2 e = map[blockIdx.x];
    const Member& m = mem[e.x];
    spread_body<K, L>(m.b, m.g, m.a.gamma, m.a.tau, m.nw, e.y, e.y - m.b.chunk_blocks);
}

Dims spread_dims(const Bufs& b, const Geom& g, int* nw_out, int* nkb_out) {
    // rgroup row copies (rgroup x per <= 48 KB, or one row of <= 74 KB at M <= 1023)
    const size_t per = (size_t)b.rgroup * g.k * g.m * 3 * sizeof(unsigned long long);
    // waves per block: graphs of a few ten thousand nodes have rows of tens
    // to hundreds of nodes, which four waves spread as fast as eight, and
    // half the threads leave room for more blocks (batched 512-graph
    // workload: 2.29e9 -> 2.50e9 node-it/s; two waves the same, one slower)
    const int nw = b.n <= 32768 ? 4 : 8;
    const int F = fft_task_ffts(g.L);
    const int RBK = kernel_row_tile(g.L);
    const size_t kern = ((size_t)zp_len(g.L, (RBK + F - 1) / F * F * g.L) + g.L) * sizeof(float2);  // + twiddles
    const size_t lds = per > kern ? per : kern;
    const int nkb = (g.L / 2 + 1 + RBK - 1) / RBK;  // rows 0 .. L/2
    *nw_out = nw;
    *nkb_out = nkb;
    return Dims{b.chunk_blocks + nkb, nw * 64, lds};
}

template <int K, int L>
static void launch_spread_t(const Bufs& b, const Geom& g, float gamma, float tau, hipStream_t s) {
    int nw, nkb;
    const Dims d = spread_dims(b, g, &nw, &nkb);
    hipLaunchKernelGGL((k_spread<K, L>), dim3(b.chunk_blocks + xcd_pair_grid(nkb)), dim3(d.block), d.lds, s, b, g,
                       gamma, tau, nw, nkb);
}

template <int K, int L>
static void launch_b_spread_t(const Member* mem, const int2* map, int blocks, int nw, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((kb_spread<K, L>), dim3(blocks), dim3(nw * 64), lds, s, mem, map);
}

template <int K>
static void launch_b_spread_k(int len, int nw, const Member* mem, const int2* map, int blocks, size_t lds,
                              hipStream_t s) {
#define TFDP_C(LL) launch_b_spread_t<K, LL>(mem, map, blocks, nw, lds, s)
    TFDP_L_SWITCH(len, TFDP_C)
#undef TFDP_C
}

void launch_b_spread(int k, int len, int nw, const Member* mem, const int2* map, int blocks, size_t lds,
                     hipStream_t s) {
    if (blocks <= 0) return;
    switch (k) {
        case 1: launch_b_spread_k<1>(len, nw, mem, map, blocks, lds, s); break;
        case 2: launch_b_spread_k<2>(len, nw, mem, map, blocks, lds, s); break;
        default: launch_b_spread_k<3>(len, nw, mem, map, blocks, lds, s); break;
    }
}

template <int K>
static void launch_spread_k(const Bufs& b, const Geom& g, float gamma, float tau, hipStream_t s) {
#define TFDP_C(LL) launch_spread_t<K, LL>(b, g, gamma, tau, s)
    TFDP_L_SWITCH(g.L, TFDP_C)
#undef TFDP_C
}

void launch_spread(const Bufs& b, const Geom& g, float gamma, float tau, hipStream_t s) {
    switch (g.k) {
        case 1: launch_spread_k<1>(b, g, gamma, tau, s); break;
        case 2: launch_spread_k<2>(b, g, gamma, tau, s); break;
        default: launch_spread_k<3>(b, g, gamma, tau, s); break;
    }
}

// ----------------------------------------------------------------- row FFTs of the charges

// RB grid rows per (logical) block. Transforms of row pair q:
// 3q = q1 + i qdx (row 2q), 3q+1 = qdy(2q) + i qdy(2q+1), 3q+2 = q1 + i qdx (row 2q+1).
template <int L, int RB>
__device__ __forceinline__ void rowfft_body(const Bufs& b, const Geom& g, int lb) {
    extern __shared__ float2 z[];
    constexpr int F = task_ffts<L>();
    constexpr int TL = F * L;
    constexpr int NQT = (3 * RB / 2 + F - 1) / F;
    const int M = g.m, H = g.H, K = g.k;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int nwav = blockDim.x >> 6;
    const int y0 = lb * RB;
    const int per = K * M * 3;
    const double u1 = 1.0 / 4294967296.0;
    const double uh = b.st->box.h / 4294967296.0;
    for (int i = threadIdx.x; i < NQT * TL; i += blockDim.x) z[zp<L>(i)] = make_float2(0.f, 0.f);
    __syncthreads();
    for (int i = threadIdx.x; i < RB * M; i += blockDim.x) {
        const int r = i / M, x = i % M;
        const int y = y0 + r;
        if (y >= M) continue;
        const int cy = y / K, bb = y % K;
        const int c0 = b.chunk_start[cy], c1 = b.chunk_start[cy + 1];
        unsigned long long a1 = 0, ax = 0, ay = 0;
        for (int c = c0; c < c1; ++c) {
            const unsigned long long* e = b.spart + (size_t)c * per + (bb * M + x) * 3;
            a1 += e[0];
            ax += e[1];
            ay += e[2];
        }
        // fixed point (2^-32 units; offsets in interval units) to layout units
        const float s1 = (float)((double)(long long)a1 * u1);
        const float sx = (float)((double)(long long)ax * uh);
        const float sy = (float)((double)(long long)ay * uh);
        const int q = r >> 1;
        z[zp<L>((3 * q + ((r & 1) ? 2 : 0)) * L + x)] = make_float2(s1, sx);
        reinterpret_cast<float*>(z + zp<L>((3 * q + 1) * L + x))[r & 1] = sy;
    }
    const float2* tws = stage_twiddles<L>(z + zp<L>(NQT * TL), b.tw);
    __syncthreads();
    for (int tk = w; tk < NQT; tk += nwav) wave_fft<L, false>(z + zp<L>(tk * TL), tws, lane);
    __syncthreads();
    // unpack with Z(u) and Z(L-u); r fastest so each column gets RB consecutive rows
    for (int i = threadIdx.x; i < 3 * H * RB; i += blockDim.x) {
        const int r = i % RB, cu = i / RB;
        const int ch = cu / H, u = cu % H;
        const int y = y0 + r;
        if (y >= M) continue;
        const int q = r >> 1, odd = r & 1;
        const int um = u == 0 ? 0 : L - u;
        float2 v;
        if (ch < 2) {
            const int zr = (3 * q + (odd ? 2 : 0)) * L;
            const float2 a = z[zp<L>(zr + u)], c = z[zp<L>(zr + um)];
            // Z = FFT(q1 + i qdx): Q1 = (Z(u) + conj Z(L-u))/2, Qdx = (Z(u) - conj Z(L-u))/(2i)
            v = ch == 0 ? make_float2(0.5f * (a.x + c.x), 0.5f * (a.y - c.y))
                        : make_float2(0.5f * (a.y + c.y), -0.5f * (a.x - c.x));
        } else {
            const int zr = (3 * q + 1) * L;
            const float2 a = z[zp<L>(zr + u)], c = z[zp<L>(zr + um)];
            v = odd ? make_float2(0.5f * (a.y + c.y), -0.5f * (a.x - c.x))
                    : make_float2(0.5f * (a.x + c.x), 0.5f * (a.y - c.y));
        }
        b.qcol[((size_t)ch * H + u) * M + y] = v;
    }
}

template <int L>
__global__ __launch_bounds__(RowTile<L>::THREADS) void k_rowfft(Bufs b, Geom g, int nqb) {
    grid_pass_priority();
    const int lb = xcd_pair_block(blockIdx.x, nqb);
    if (lb < 0) return;
    rowfft_body<L, RowTile<L>::RB>(b, g, lb);
}

// Batched row passes take RB rows per block from the batch's tile schedule
// (tfdp_batch_set_tiles, chosen by the autotuner): 2, 4 or 8 at L <= 768,
// RowTile<L>::RBB above. The transforms, their pairing of rows and every
// sum do not depend on RB, so all tiles give bit-identical results.
template <int L, int RB>
__global__ __launch_bounds__(RowTile<L>::THREADS_B) void kb_rowfft(const Member* __restrict__ mem,
                                                                     const int2* __restrict__ map) {
    const int2 e = map[blockIdx.x];
    const Member& m = mem[e.x];
    rowfft_body<L, RB>(m.b, m.g, e.y);
}

// Blocks, threads and LDS of a row pass of RB rows per block (rows = 0: the
// plain launch's RowTile<L>::RB and block size; rows > 0: a batched launch).
template <int L>
static Dims row_pass_dims_t(const Geom& g, int* nb, int rows) {
    constexpr int F = task_ffts<L>();
    constexpr int TL = F * L;
    const int RB = rows > 0 ? rows : RowTile<L>::RB;
    const int NT = (3 * RB / 2 + F - 1) / F;
    *nb = (g.m + RB - 1) / RB;
    const int T = rows > 0 ? RowTile<L>::THREADS_B : RowTile<L>::THREADS;
    return Dims{*nb, T, (size_t)(zp_len(L, NT * TL) + L) * sizeof(float2)};
}

template <int L>
static void launch_rowfft_t(const Bufs& b, const Geom& g, hipStream_t s) {
    int nqb;
    const Dims d = row_pass_dims_t<L>(g, &nqb, 0);
    hipLaunchKernelGGL(k_rowfft<L>, dim3(xcd_pair_grid(nqb)), dim3(d.block), d.lds, s, b, g, nqb);
}

void launch_rowfft(const Bufs& b, const Geom& g, hipStream_t s) {
#define TFDP_C(LL) launch_rowfft_t<LL>(b, g, s)
    TFDP_L_SWITCH(g.L, TFDP_C)
#undef TFDP_C
}

// ----------------------------------------------------------------- column pass

// Column groups per block: one for a single grid; two for the batched
// launches at L = 256, where a group's four forward transform tasks leave
// half of the eight waves idle and the blocks of many graphs fill the chip
// (at L <= 128 a graph has only 33-65 columns, and halving its few blocks
// measured slower).
constexpr int col_groups(int L, bool batched) { return batched && L == 256 ? 2 : 1; }

// Columns u0 .. u0 + G F - 1 (F = transforms per task, G column groups).
// Per group, forward column FFTs of
//   Z = FFT_b(R1 + s b R1 + i R2)  (R1 = K row spectrum and R2 = H_x row
//       spectrum / i, both real and even in b; s b R1 real and odd in b):
//       K^ = Re Z; Im Z = H_x^/i + H_y^/i, H_x^/i its even part in the
//       frequency, H_y^/i its odd part
//   Q1, Qdx, Qdy  (charge row spectra, rows y < M)
// then phi_1 = K^ Q1, G_x = H_x^ Q1 - K^ Qdx, G_y = H_y^ Q1 - K^ Qdy (scaled by
// 1/L^2) and three inverse column FFTs; rows y < M stored column-major.
template <int L, int G>
__device__ __forceinline__ void colconv_body(const Bufs& b, const Geom& g, int bid) {
    extern __shared__ float2 sm2[];
    constexpr int F = task_ffts<L>();
    constexpr int TL = F * L;
    constexpr int GT = 4 * TL;  // one group's areas: Z, Q1, Qdx, Qdy
    const int M = g.m, H = g.H;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int u0 = bid * G * F;
    const Box bx = b.st->box;
    const float s = (float)(bx.h / (double)g.k);
    const float inv = 1.f / ((float)L * (float)L);
    // transform f of group gi covers column u0 + gi F + f
    for (int i = threadIdx.x; i < G * TL; i += blockDim.x) {
        const int gi = i / TL, j = i % TL;
        const int f = j / L, r = j % L;
        const int u = u0 + gi * F + f;
        const int a = gi * GT;
        float2 kr = make_float2(0.f, 0.f);
        if (u < H) kr = b.kcol[(size_t)u * (L / 2 + 1) + (r <= L / 2 ? r : L - r)];
        const int bt = signed_offset(r, M, L);
        const float e = bt != INT_MIN ? s * (float)bt * kr.x : 0.f;
        sm2[zp<L>(a + j)] = make_float2(kr.x + e, kr.y);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float2 v = make_float2(0.f, 0.f);
            if (u < H && r < M) v = b.qcol[((size_t)ch * H + u) * M + r];
            sm2[zp<L>(a + (1 + ch) * TL + j)] = v;
        }
    }
    const float2* tws = stage_twiddles<L>(sm2 + zp<L>(G * GT), b.tw);
    __syncthreads();
    static_assert(4 * G <= 8, "one forward task per wave of the 512-thread block");
    if (w < 4 * G) wave_fft<L, false>(sm2 + zp<L>(w * TL), tws, lane);
    __syncthreads();
    for (int i = threadIdx.x; i < G * TL; i += blockDim.x) {
        const int gi = i / TL, j = i % TL;
        const int f = j / L, v = j % L;
        const int a = gi * GT;
        const float2 zj = sm2[zp<L>(a + j)];
        const float zi = zj.y, zm = sm2[zp<L>(a + f * L + (v == 0 ? 0 : L - v))].y;
        const float kk = zj.x * inv;
        const float h1 = 0.5f * (zi + zm) * inv;
        const float h2 = 0.5f * (zi - zm) * inv;
        const float2 q1 = sm2[zp<L>(a + TL + j)], qx = sm2[zp<L>(a + 2 * TL + j)], qy = sm2[zp<L>(a + 3 * TL + j)];
        sm2[zp<L>(a + TL + j)] = make_float2(kk * q1.x, kk * q1.y);
        sm2[zp<L>(a + 2 * TL + j)] = make_float2(-h1 * q1.y - kk * qx.x, h1 * q1.x - kk * qx.y);
        sm2[zp<L>(a + 3 * TL + j)] = make_float2(-h2 * q1.y - kk * qy.x, h2 * q1.x - kk * qy.y);
    }
    __syncthreads();
    if (w < 3 * G) wave_fft<L, true>(sm2 + zp<L>((w / 3) * GT + (1 + w % 3) * TL), tws, lane);
    __syncthreads();
    for (int i = threadIdx.x; i < G * 3 * F * M; i += blockDim.x) {
        const int gi = i / (3 * F * M), rem0 = i % (3 * F * M);
        const int ch = rem0 / (F * M), rem = rem0 % (F * M);
        const int f = rem / M, y = rem % M;
        const int u = u0 + gi * F + f;
        if (u < H) b.pcol[((size_t)ch * H + u) * M + y] = sm2[zp<L>(gi * GT + (1 + ch) * TL + f * L + y)];
    }
}

template <int L>
__global__ __launch_bounds__(512) void k_colconv(Bufs b, Geom g) {
    grid_pass_priority();
    colconv_body<L, col_groups(L, false)>(b, g, blockIdx.x);
}

// Batched column passes take G column groups per block from the batch's
// tile schedule (1 or 2 at L <= 768; col_groups(L, true) above); each column
// is transformed alike in either, so the results are bit-identical.
template <int L, int G>
__global__ __launch_bounds__(512) void kb_colconv(const Member* __restrict__ mem, const int2* __restrict__ map) {
    const int2 e = map[blockIdx.x];
    const Member& m = mem[e.x];
    colconv_body<L, G>(m.b, m.g, e.y);
}

Dims colconv_dims(const Geom& g, int groups) {
    const int F = fft_task_ffts(g.L);
    const int G = groups > 0 ? groups : col_groups(g.L, false);
    return Dims{(g.H + G * F - 1) / (G * F), 512, ((size_t)zp_len(g.L, 4 * G * F * g.L) + g.L) * sizeof(float2)};
}

template <int L>
static void launch_colconv_t(const Bufs& b, const Geom& g, hipStream_t s) {
    const Dims d = colconv_dims(g);
    hipLaunchKernelGGL(k_colconv<L>, dim3(d.grid), dim3(d.block), d.lds, s, b, g);
}

void launch_colconv(const Bufs& b, const Geom& g, hipStream_t s) {
#define TFDP_C(LL) launch_colconv_t<LL>(b, g, s)
    TFDP_L_SWITCH(g.L, TFDP_C)
#undef TFDP_C
}

// ----------------------------------------------------------------- inverse rows

// RB potential rows per block, read as column tiles. Transforms: row r holds
// phi_1 + i G_x (task area r), row pair q holds G_y(2q) + i G_y(2q+1)
// (area RB + q); the spectra of real rows are extended by Hermitian symmetry.
template <int L, int RB>
__device__ __forceinline__ void rowifft_body(const Bufs& b, const Geom& g, int lb) {
    extern __shared__ float2 z[];
    constexpr int F = task_ffts<L>();
    constexpr int TL = F * L;
    constexpr int NT = (3 * RB / 2 + F - 1) / F;
    const int M = g.m, H = g.H;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int nwav = blockDim.x >> 6;
    const int y0 = lb * RB;
    for (int i = threadIdx.x; i < (NT * TL - (3 * RB / 2) * L); i += blockDim.x)
        z[zp<L>((3 * RB / 2) * L + i)] = make_float2(0.f, 0.f);
    for (int i = threadIdx.x; i < L * (RB / 2); i += blockDim.x) {
        const int q = i % (RB / 2), u = i / (RB / 2);
        const bool ext = u >= H;
        const int uu = ext ? L - u : u;
        float2 p[3][2];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
#pragma unroll
            for (int o = 0; o < 2; ++o) {
                const int y = y0 + 2 * q + o;
                float2 v = make_float2(0.f, 0.f);
                if (y < M) v = b.pcol[((size_t)ch * H + uu) * M + y];
                if (ext) v.y = -v.y;
                p[ch][o] = v;
            }
        }
#pragma unroll
        for (int o = 0; o < 2; ++o)
            z[zp<L>((2 * q + o) * L + u)] = make_float2(p[0][o].x - p[1][o].y, p[0][o].y + p[1][o].x);
        z[zp<L>((RB + q) * L + u)] = make_float2(p[2][0].x - p[2][1].y, p[2][0].y + p[2][1].x);
    }
    const float2* tws = stage_twiddles<L>(z + zp<L>(NT * TL), b.tw);
    __syncthreads();
    for (int tk = w; tk < NT; tk += nwav) wave_fft<L, true>(z + zp<L>(tk * TL), tws, lane);
    __syncthreads();
    for (int i = threadIdx.x; i < RB * M; i += blockDim.x) {
        const int r = i / M, x = i % M;
        const int y = y0 + r;
        if (y < M) {
            const float2 v = z[zp<L>(r * L + x)];
            const float2 e = z[zp<L>((RB + (r >> 1)) * L + x)];
            b.pot[(size_t)y * M + x] = make_float4(v.x, v.y, (r & 1) ? e.y : e.x, 0.f);
        }
    }
}

template <int L>
__global__ __launch_bounds__(RowTile<L>::THREADS) void k_rowifft(Bufs b, Geom g, int nrb) {
    grid_pass_priority();
    const int lb = xcd_pair_block(blockIdx.x, nrb);
    if (lb < 0) return;
    rowifft_body<L, RowTile<L>::RB>(b, g, lb);
}

template <int L, int RB>
__global__ __launch_bounds__(RowTile<L>::THREADS_B) void kb_rowifft(const Member* __restrict__ mem,
                                                                      const int2* __restrict__ map) {
    const int2 e = map[blockIdx.x];
    const Member& m = mem[e.x];
    rowifft_body<L, RB>(m.b, m.g, e.y);
}

template <int L>
static void launch_rowifft_t(const Bufs& b, const Geom& g, hipStream_t s) {
    int nrb;
    const Dims d = row_pass_dims_t<L>(g, &nrb, 0);
    hipLaunchKernelGGL(k_rowifft<L>, dim3(xcd_pair_grid(nrb)), dim3(d.block), d.lds, s, b, g, nrb);
}

void launch_rowifft(const Bufs& b, const Geom& g, hipStream_t s) {
#define TFDP_C(LL) launch_rowifft_t<LL>(b, g, s)
    TFDP_L_SWITCH(g.L, TFDP_C)
#undef TFDP_C
}

Dims rowfft_dims(const Geom& g, int* nqb, int rows) {
    Dims d{};
#define TFDP_D(LG) d = row_pass_dims_t<LG>(g, nqb, rows)
    TFDP_L_SWITCH(g.L, TFDP_D)
#undef TFDP_D
    return d;
}

Dims rowifft_dims(const Geom& g, int* nrb, int rows) { return rowfft_dims(g, nrb, rows); }

int batch_rows_default(int L) {
    int r = 0;
#define TFDP_R(LG) r = RowTile<LG>::RBB
    TFDP_L_SWITCH(L, TFDP_R)
#undef TFDP_R
    return r;
}

int batch_groups_default(int L) { return col_groups(L, true); }

bool batch_tile_valid(int L, int rows, int groups) {
    if (L > kMaxTunedL) return rows == batch_rows_default(L) && groups == batch_groups_default(L);
    return (rows == 2 || rows == 4 || rows == 8) && (groups == 1 || groups == 2);
}

// Launch of a batched row pass (kernel template K) with `rows` rows per block.
#define TFDP_ROWPASS_LAUNCH(KERN, LG, rows, d, blocks, s, mem, map)                                             \
    do {                                                                                                        \
        if constexpr (LG <= kMaxTunedL) {                                                                       \
            if ((rows) == 2)                                                                                    \
                hipLaunchKernelGGL((KERN<LG, 2>), dim3(blocks), dim3((d).block), (d).lds, s, mem, map);        \
            else if ((rows) == 4)                                                                               \
                hipLaunchKernelGGL((KERN<LG, 4>), dim3(blocks), dim3((d).block), (d).lds, s, mem, map);        \
            else                                                                                                \
                hipLaunchKernelGGL((KERN<LG, 8>), dim3(blocks), dim3((d).block), (d).lds, s, mem, map);        \
        } else {                                                                                                \
            hipLaunchKernelGGL((KERN<LG, RowTile<LG>::RBB>), dim3(blocks), dim3((d).block), (d).lds, s, mem,    \
                               map);                                                                            \
        }                                                                                                       \
    } while (0)

template <int L>
static void launch_b_rowfft_t(int rows, const Member* mem, const int2* map, int blocks, hipStream_t s) {
    const Geom g{1, 1, L, L / 2 + 1, 1};
    int nqb;
    const Dims d = row_pass_dims_t<L>(g, &nqb, rows);
    TFDP_ROWPASS_LAUNCH(kb_rowfft, L, rows, d, blocks, s, mem, map);
}

template <int L>
static void launch_b_rowifft_t(int rows, const Member* mem, const int2* map, int blocks, hipStream_t s) {
    const Geom g{1, 1, L, L / 2 + 1, 1};
    int nrb;
    const Dims d = row_pass_dims_t<L>(g, &nrb, rows);
    TFDP_ROWPASS_LAUNCH(kb_rowifft, L, rows, d, blocks, s, mem, map);
}

template <int L>
static void launch_b_colconv_t(int groups, const Member* mem, const int2* map, int blocks, hipStream_t s) {
    const Geom g{1, 1, L, L / 2 + 1, 1};
    const Dims d = colconv_dims(g, groups);
    if constexpr (L <= kMaxTunedL) {
        if (groups == 2)
            hipLaunchKernelGGL((kb_colconv<L, 2>), dim3(blocks), dim3(d.block), d.lds, s, mem, map);
        else
            hipLaunchKernelGGL((kb_colconv<L, 1>), dim3(blocks), dim3(d.block), d.lds, s, mem, map);
    } else {
        hipLaunchKernelGGL((kb_colconv<L, col_groups(L, true)>), dim3(blocks), dim3(d.block), d.lds, s, mem, map);
    }
}

void launch_b_rowfft(int len, int rows, const Member* mem, const int2* map, int blocks, hipStream_t s) {
    if (blocks <= 0) return;
#define TFDP_L(LG) launch_b_rowfft_t<LG>(rows, mem, map, blocks, s)
    TFDP_L_SWITCH(len, TFDP_L)
#undef TFDP_L
}

void launch_b_colconv(int len, int groups, const Member* mem, const int2* map, int blocks, hipStream_t s) {
    if (blocks <= 0) return;
#define TFDP_L(LG) launch_b_colconv_t<LG>(groups, mem, map, blocks, s)
    TFDP_L_SWITCH(len, TFDP_L)
#undef TFDP_L
}

void launch_b_rowifft(int len, int rows, const Member* mem, const int2* map, int blocks, hipStream_t s) {
    if (blocks <= 0) return;
#define TFDP_L(LG) launch_b_rowifft_t<LG>(rows, mem, map, blocks, s)
    TFDP_L_SWITCH(len, TFDP_L)
#undef TFDP_L
}

// Large-LDS attribute for every kernel instantiation that can exceed 64 KB
// (called once at set-up, so that no attribute call happens during stream
// capture).
template <int L>
static void allow_big_lds_all_l() {
    allow_big_lds(k_spread<1, L>);
    allow_big_lds(k_spread<2, L>);
    allow_big_lds(k_spread<3, L>);
    allow_big_lds(k_rowfft<L>);
    allow_big_lds(k_colconv<L>);
    allow_big_lds(k_rowifft<L>);
    allow_big_lds(kb_spread<1, L>);
    allow_big_lds(kb_spread<2, L>);
    allow_big_lds(kb_spread<3, L>);
    if constexpr (L <= kMaxTunedL) {
        allow_big_lds(kb_rowfft<L, 2>);
        allow_big_lds(kb_rowfft<L, 4>);
        allow_big_lds(kb_rowfft<L, 8>);
        allow_big_lds(kb_rowifft<L, 2>);
        allow_big_lds(kb_rowifft<L, 4>);
        allow_big_lds(kb_rowifft<L, 8>);
        allow_big_lds(kb_colconv<L, 1>);
        allow_big_lds(kb_colconv<L, 2>);
    } else {
        allow_big_lds(kb_rowfft<L, RowTile<L>::RBB>);
        allow_big_lds(kb_rowifft<L, RowTile<L>::RBB>);
        allow_big_lds(kb_colconv<L, col_groups(L, true)>);
    }
}

void init_kernel_attributes() {
#define TFDP_A(LL) allow_big_lds_all_l<LL>()
    TFDP_A(64);
    TFDP_A(128);
    TFDP_A(256);
    TFDP_A(384);
    TFDP_A(512);
    TFDP_A(768);
    TFDP_A(1024);
    TFDP_A(1536);
    TFDP_A(2048);
#undef TFDP_A
}

}  // namespace tfdp
