// Internal definitions shared by the HIP translation units of libtfdp.so.
// Not part of the public ABI (see include/tfdp.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <cstdlib>

namespace tfdp {

constexpr int kThreads = 256;        // threads per block of the node and FFT kernels
constexpr int kBinChunk = 2048;      // nodes per block of the binning passes
constexpr int kSpreadChunk = 4096;   // sorted nodes per block of the spreading pass (one row's share)
constexpr int kSpreadGroupRows = 8;  // sparse interval rows one spreading block may take together
constexpr long long kSpreadGroupNodes = 1024;  // nodes of an average row group
constexpr int kBoxSlots = 64;        // slots of the box extremes (one 128-byte line each)
constexpr int kMaxL = 2048;          // largest FFT length per side
constexpr int kMaxNInt = 1024;       // largest number of intervals per side
constexpr int kGroupEdges = 512;     // CSR entries of one wave group of the edge pass
constexpr int kSliceNodesDefault = 1 << 24;  // column slice width of the edge pass (nodes)
constexpr int kMaxSlices = 64;
constexpr int kGraphIters = 8;             // iterations per captured graph (even; pairs for the rest)
constexpr int kGroupRows = 64;       // rows of one wave group of the edge pass
constexpr int kBruteRows = 64;       // rows per block of the exact repulsion (one per lane)
constexpr int kSymTile = 256;        // nodes per tile of the pair-symmetric exact method
constexpr int kSymMinNodes = 4096;   // graphs from this size on use it (the one-launch kernel below)
constexpr int kAutoGridMin = 50;     // automatic grid: at least this many intervals per side
constexpr int kAutoGridChunk = 10;   // automatic grid: iterations between grid choices

// Square box of the current positions, in float64 (lo, side W, interval h = W / N_int).
struct Box {
    double lo_x, lo_y, w, h;
};

// Device-resident per-handle state.
struct DevState {
    // order-preserving encodings of min x, min y, max x, max y; two sets used
    // by alternate iterations (one is read while the next is reset and
    // filled); blocks commit to slot blockIdx % kBoxSlots so that no single
    // address sees thousands of device-scope atomics per launch
    unsigned int mm[2][kBoxSlots][32];
    int t;                // iteration index used by the update (cooling)
    int nonfinite;        // set when a computed position is NaN or infinite
    int csr_bad;          // set by the CSR check at init
    int pad;
    Box box;              // box used by every kernel of the current iteration
};

// Geometry of the grid for one k.
struct Geom {
    int k;      // interpolation nodes per interval per axis
    int m;      // grid nodes per side, N_int * k
    int L;      // FFT length per side (2^a or 3 * 2^a, >= 2M, >= 64)
    int H;      // L/2 + 1 stored spectrum columns
    int cw;     // spectrum columns per block of the column pass
};

// Transforms per FFT task (one wave) of length L: 512 or more points for
// L = 2^a, 1536 for L = 3 * 2^a (every pass then gives each of the 64 lanes
// whole butterflies).
__host__ __device__ constexpr int fft_task_ffts(int L) { return L % 3 == 0 ? 1536 / L : (L < 512 ? 512 / L : 1); }

// Workspace views used by the kernels.
struct Bufs {
    int n;
    int n_int;
    int nblk;            // blocks of the binning passes
    int max_chunks;      // upper bound of spreading blocks
    float2* spos;        // positions sorted by interval row
    int* blkcnt;         // [n_int][nblk] counts, then exclusive offsets
    int* bucket_cnt;     // [n_int]
    int* bucket_start;   // [n_int + 1]
    int* chunk_start;    // [n_int + 1] first partial row of each interval row (spreading pass)
    int4* wchunk;        // [max_chunks + 1] spreading blocks {first row, rows, first node, end};
                         // entry max_chunks: {number of blocks, 0, 0, 0}
    int rgroup;          // interval rows one spreading block may take (this k's row size)
    int chunk_blocks;    // spreading blocks launched for the work chunks (each takes every
                         // chunk_blocks-th one); then the kernel-row blocks
    unsigned long long* spart;  // [max_chunks][k][M][3] partial grid rows (fixed point)
    unsigned long long* sym_acc;  // [n][2] fixed-point repulsion sums of the pair-symmetric exact method (zero between passes)
    float2* qcol;        // [3][H][M] charge row spectra, column-major
    float2* kcol;        // [H][L/2+1] kernel row spectra (K^, H_x^/i) of rows 0 .. L/2, column-major
    float2* pcol;        // [3][H][M] potential row spectra after the column pass
    float4* pot;         // [M][M] (phi_1, G_x, G_y, 0)
    const float2* tw;    // twiddles for this L: exp(-2 pi i j / L), j < L
    DevState* st;
};

// One column slice of the edge pass: the CSR entries whose column lies in one
// contiguous column range, as a CSR of all n rows, with its schedule.
struct EdgeSlice {
    const int* rp;       // [n + 1]
    const int* col;      // [entries of the slice]
    const int2* sched;   // [4 * blocks]
    int blocks;
};

struct ModelArgs {
    float alpha, beta, gamma, rep_weight;
    float t0;
    int total_iters;
    float tau;             // length scale of the t-forces (Eq.3), 1 in the paper's model
    const float* rep_w;    // per-node repulsion weights (local refinement, Sec. 5) or null
    const float* att_w;    // per-node attraction weights or null
};

// One graph of a batched launch: the arguments of its plain launches for one
// k. Batched kernels read it through a block map entry {member, block} and
// run the plain kernel's body for that block, so every graph gets exactly
// the arithmetic of its plain launch.
struct Member {
    Bufs b;             // views for this entry's k
    Geom g;
    ModelArgs a;
    EdgeSlice es;       // the single column slice of the edge pass
    float2* pos;        // caller's positions (current at even iterations of a call)
    float2* alt;        // second buffer (current at odd iterations)
    int slot;           // index of the graph's iteration counter at the start of the call
    int nw;             // waves per block of the spreading pass
    int nkb;            // logical kernel-row blocks of the spreading pass
    int box_blocks;     // blocks of the box reduction
};

// Interval rows one spreading block may hold in LDS at once for k and
// n_int: up to kSpreadGroupRows row copies of K x M x 3 64-bit sums in 48 KB,
// and about kSpreadGroupNodes nodes for the graph's average row (n / n_int):
// rows of a few tens to hundreds of nodes leave a block per row mostly idle,
// while grouping rows of thousands would only take blocks from a graph that
// has few companions in the launch.
inline int spread_row_group(int k, int n_int, long long n) {
    const long long per = (long long)k * n_int * k * 3 * 8;
    long long cap = kSpreadGroupRows;
    if (const char* e = std::getenv("TFDP_SPREAD_GROUP_ROWS")) {  // 1 .. kSpreadGroupRows
        const long long v = std::atoll(e);
        if (v >= 1 && v <= kSpreadGroupRows) cap = v;
    }
    const long long avg = n_int > 0 ? n / n_int : n;
    const long long by_nodes = kSpreadGroupNodes / (avg > 1 ? avg : 1);
    if (by_nodes < cap) cap = by_nodes;
    const long long g = per > 0 ? 49152 / per : 1;
    return (int)(g < 1 || cap < 1 ? 1 : (g > cap ? cap : g));
}

// Slot-set parity and position buffers of iteration j of a batched call for
// a graph whose counter was t0 at the start of the call.
__device__ __forceinline__ int batch_set(const int* tcall, const Member& m, int j) {
    return (tcall[m.slot] + j) & 1;
}

// ---- launchers (each defined next to its kernels) ----
void launch_box_begin(DevState* st, int t, hipStream_t s);
void launch_box_reduce(const float2* pos, int n, DevState* st, int set, hipStream_t s);
void launch_bin_count(const float2* pos, const Bufs& b, int set, hipStream_t s);
void launch_bin_scan(const Bufs& b, int reset_set, hipStream_t s);
void launch_bin_scatter(const float2* pos, const Bufs& b, hipStream_t s);
void launch_spread(const Bufs& b, const Geom& g, float gamma, float tau, hipStream_t s);
void launch_rowfft(const Bufs& b, const Geom& g, hipStream_t s);
void launch_colconv(const Bufs& b, const Geom& g, hipStream_t s);
void launch_rowifft(const Bufs& b, const Geom& g, hipStream_t s);
void launch_twiddles(float2* tw, int L, hipStream_t s);
void init_kernel_attributes();
// Edge pass of slice `es`: mode 0 writes the slice's attraction sums to
// fpart, mode 1 adds them to fpart, mode 2 (last slice) adds fpart (when
// use_part) and finishes every node: repulsion gather, displacement, output.
void launch_edges(const float2* pos, float2* pos_out, const EdgeSlice& es, int mode, int use_part,
                  float2* fpart, const Bufs& b, const Geom& g, const ModelArgs& a, int set,
                  float2* f_rep, float2* f_att, float2* f_tot, hipStream_t s);
// Overlapped form of the edge pass: launch_attract writes the attraction sums
// of every row to fpart with at most `blocks` blocks looping over the
// schedule (run concurrently with the grid passes), launch_node_update then
// gathers the repulsion and finishes every node as mode 2 does.
void launch_attract(const float2* pos, const EdgeSlice& es, float2* fpart, const Bufs& b, const Geom& g,
                    const ModelArgs& a, int blocks, hipStream_t s);
void launch_node_update(const float2* pos, float2* pos_out, const float2* fpart, const Bufs& b, const Geom& g,
                        const ModelArgs& a, int set, float2* f_rep, float2* f_att, float2* f_tot, hipStream_t s);
// Workgroups are dispatched to the 8 XCDs round robin. xcd_pair_block maps
// the physical block index so that logical blocks 2j and 2j+1 run on the
// same XCD (and so share its L2) when their stores fill one cache line
// together; returns -1 for padding blocks. nb: logical blocks; grid size
// xcd_pair_grid(nb).
__host__ __device__ __forceinline__ int xcd_pair_grid(int nb) { return ((nb + 15) / 16) * 16; }
__device__ __forceinline__ int xcd_pair_block(int phys, int nb) {
    const int per = xcd_pair_grid(nb) / 8;  // logical blocks per XCD (even)
    const int logical = (phys % 8) * per + phys / 8;
    return logical < nb ? logical : -1;
}

// Column slices for n nodes with slices of at most slice_nodes columns, and
// an upper bound of the edge-pass blocks of all slices together. Per slice:
// H heavy rows (more than kGroupEdges entries; H <= entries / 513 over all
// slices) get a block each; a wave group ends with kGroupRows rows (at most
// n / 64 such groups), at the last row (one), before a heavy row (at most
// H), or when the next row's entries do not fit, in which case the group and
// the next one hold more than kGroupEdges entries together (fewer than
// entries / 256 such groups); four groups per block.
inline int edge_slices(long long n, long long slice_nodes) {
    long long s = (n + slice_nodes - 1) / slice_nodes;
    return (int)(s < 1 ? 1 : (s > kMaxSlices ? kMaxSlices : s));
}
inline long long edge_blocks_bound(long long n, long long nnz, long long slice_nodes) {
    return (long long)edge_slices(n, slice_nodes) * ((n / kGroupRows + 2) / 4 + 3) + nnz / (2 * kGroupEdges) +
           2 * (nnz / (kGroupEdges + 1)) + 1;
}
void launch_brute(const float2* pos, float2* pos_out, const int* row_ptr, const int* col_idx,
                  int n, DevState* st, const ModelArgs& a, int t,
                  float2* f_rep, float2* f_att, float2* f_tot, hipStream_t s);
// Pair-symmetric exact method (graphs of at least kSymMinNodes nodes): the
// pair pass over tile pairs, then the node pass, which clears acc.
void launch_sym(const float2* pos, float2* pos_out, const int* row_ptr, const int* col_idx, int n,
                unsigned long long* acc, DevState* st, const ModelArgs& a, int t, float2* f_rep, float2* f_att,
                float2* f_tot, hipStream_t s);
long long sym_pair_blocks(int n);
int sym_node_blocks(int n);
// Smallest graph on the pair-symmetric exact method: kSymMinNodes, or the
// environment variable TFDP_SYM_MIN_NODES (>= 1) read at each call; graphs
// whose tile pairs would not fit one launch keep the one-launch kernel.
int sym_min_nodes();
inline bool use_sym(int n) { return n >= sym_min_nodes() && sym_pair_blocks(n) <= 0x7fffffffLL; }
void launch_csr_check(const int* row_ptr, const int* col_idx, int n, long long nnz,
                      DevState* st, hipStream_t s);

// ---- launch geometry shared by the plain and the batched launchers ----
struct Dims {
    int grid;     // blocks of the plain launch (logical blocks for the batched map)
    int block;    // threads per block
    size_t lds;   // dynamic LDS bytes
};
Dims box_reduce_dims(int n);
Dims bin_count_dims(const Bufs& b);
Dims bin_scan_dims(const Bufs& b);
Dims bin_scatter_dims(const Bufs& b);
// spreading: grid = chunk blocks + logical kernel-row blocks (nkb); nw waves
Dims spread_dims(const Bufs& b, const Geom& g, int* nw, int* nkb);
// rows / groups: 0 for the plain launches, else the batched launch's rows
// per block (row passes) or column groups per block (column pass)
Dims rowfft_dims(const Geom& g, int* nqb, int rows = 0);
Dims colconv_dims(const Geom& g, int groups = 0);
Dims rowifft_dims(const Geom& g, int* nrb, int rows = 0);
// Tile schedule of the batched grid passes per FFT length: the defaults, and
// whether (rows, groups) is one of the instantiated tiles for length L.
int batch_rows_default(int L);
int batch_groups_default(int L);
bool batch_tile_valid(int L, int rows, int groups);

// ---- batched launchers: one launch for every map entry {member, block} ----
// tcall: per-slot iteration counters at the start of the call; j: iteration
// index inside the call. Members of one launch share k, L and the spreading
// block size (the launch's template and block shape).
void launch_b_box(const Member* mem, const int2* map_begin, int n_begin, const int2* map_red, int n_red,
                  const int* tcall, hipStream_t s);
void launch_b_bin_count(const Member* mem, const int2* map, int blocks, size_t lds, const int* tcall, int j,
                        hipStream_t s);
void launch_b_bin_scan(const Member* mem, const int2* map, int blocks, const int* tcall, int j, hipStream_t s);
void launch_b_bin_scatter(const Member* mem, const int2* map, int blocks, size_t lds, int j, hipStream_t s);
void launch_b_spread(int k, int len, int nw, const Member* mem, const int2* map, int blocks, size_t lds,
                     hipStream_t s);
void launch_b_rowfft(int len, int rows, const Member* mem, const int2* map, int blocks, hipStream_t s);
void launch_b_colconv(int len, int groups, const Member* mem, const int2* map, int blocks, hipStream_t s);
void launch_b_rowifft(int len, int rows, const Member* mem, const int2* map, int blocks, hipStream_t s);
void launch_b_edges(int k, const Member* mem, const int2* map, int blocks, const int* tcall, int j,
                    hipStream_t s);
void launch_b_copy(const Member* mem, const int2* map, int blocks, hipStream_t s);
void launch_b_advance(int* tcall, int slots, int iters, hipStream_t s);
// exact method of the k = 0 members: one-launch kernel (map {member, row
// block}), pair-symmetric passes (maps {member, tile pair} and {member, node
// block}); then their counters advance (tick_map: one entry per member)
void launch_b_brute(const Member* mem, const int2* map, int blocks, int j, hipStream_t s);
void launch_b_sym_pairs(const Member* mem, const int2* map, int blocks, int j, hipStream_t s);
void launch_b_sym_node(const Member* mem, const int2* map, int blocks, int j, hipStream_t s);
void launch_b_tick(const Member* mem, const int2* tick_map, int members, hipStream_t s);

// ---- layout quality (metrics.hip) ----
size_t stress_workspace_bytes(int n, int nsrc);
// 0, -1 (invalid CSR), -2 (a source outside [0, n)) or the HIP error;
// *se = sampled stress error,
// np (NULL: skipped) = {NP_1, NP_2} over the same sources, *levels = BFS
// levels run
int stress_sampled(int n, long long nnz, const int* row_ptr, const int* col_idx, const float2* pos, const int* src,
                   int nsrc, void* work, double* se, double* np, int* levels, hipStream_t s);

// ---- device helpers used by several translation units ----

// Issue priority of the waves of the plain binning, spreading and FFT
// passes. When the attraction pass of the same iteration runs beside them on
// a second stream, its gathers fill the memory queues; the grid passes are
// short chains of dependent accesses, and a raised priority lets their few
// accesses go first (1M-node graph, k = 1: 116.9 -> 108.9 us per iteration
// with the overlapped schedule; no change when they run alone).
__device__ __forceinline__ void grid_pass_priority() { __builtin_amdgcn_s_setprio(2); }

// Order-preserving map float -> uint (min/max of floats via integer atomics).
__device__ __forceinline__ unsigned int enc_ord(float f) {
    unsigned int u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float dec_ord(unsigned int u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// Interval index and in-interval coordinate along one axis, float64 with a
// fixed operation order and no contraction (the same operations as the CPU
// oracle, so both choose the same interval for every node).
__device__ __forceinline__ void bin_axis(float x, double lo, double h, int n_int,
                                         int& c, double& t) {
#pragma clang fp contract(off)
    double r = ((double)x - lo) / h;
    double f = floor(r);
    f = fmin(fmax(f, 0.0), (double)(n_int - 1));
    c = (int)f;
    t = r - f;
}

// Lagrange basis on the K nodes (j + 1/2)/K of one interval, float64. The
// node differences (j - m)/K have compile-time reciprocals K/(j - m), so no
// division is needed (the weights only have to be accurate, unlike the
// interval index, which must match the oracle bit for bit).
template <int K>
__device__ __forceinline__ void lagrange(double t, double* w) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
        double v = 1.0;
#pragma unroll
        for (int m = 0; m < K; ++m) {
            if (m == j) continue;
            const double tm = ((double)m + 0.5) / (double)K;
            v = v * ((t - tm) * ((double)K / (double)(j - m)));
        }
        w[j] = v;
    }
}

// Square box from the encoded extremes of one slot set (same float64
// operations as the oracle): side W = max(x range, y range) centred on the
// mid-ranges, W = 1 if nothing finite was seen or all points coincide.
__device__ __forceinline__ Box box_from_extremes(unsigned int a0, unsigned int a1, unsigned int a2,
                                                 unsigned int a3, int n_int) {
#pragma clang fp contract(off)
    Box b;
    if (a0 == 0xffffffffu) {
        b.lo_x = 0.0;
        b.lo_y = 0.0;
        b.w = 1.0;
    } else {
        const double xmin = (double)dec_ord(a0);
        const double ymin = (double)dec_ord(a1);
        const double xmax = (double)dec_ord(a2);
        const double ymax = (double)dec_ord(a3);
        const double rx = xmax - xmin;
        const double ry = ymax - ymin;
        double w = rx >= ry ? rx : ry;
        if (!(w > 0.0)) w = 1.0;
        const double cx = (xmin + xmax) / 2.0;
        const double cy = (ymin + ymax) / 2.0;
        b.lo_x = cx - w / 2.0;
        b.lo_y = cy - w / 2.0;
        b.w = w;
    }
    b.h = b.w / (double)n_int;
    return b;
}

// Offsets delta_j = (t - tau_j) h of a point from the K nodes of its interval.
template <int K>
__device__ __forceinline__ void node_deltas(double t, double h, double* d) {
#pragma clang fp contract(off)
#pragma unroll
    for (int j = 0; j < K; ++j) {
        double tj = ((double)j + 0.5) / (double)K;
        d[j] = (t - tj) * h;
    }
}

// Block-wide min/max of the given extremes, committed to st->mm[set][slot]
// with one set of integer atomics per block (blockDim.x a multiple of 64,
// <= kThreads).
__device__ __forceinline__ void block_minmax_commit(float xmin, float ymin, float xmax, float ymax,
                                                    DevState* st, int set, int slot) {
    // wave reduction, then one lane per wave commits with atomics
    for (int off = 32; off > 0; off >>= 1) {
        xmin = fminf(xmin, __shfl_xor(xmin, off));
        ymin = fminf(ymin, __shfl_xor(ymin, off));
        xmax = fmaxf(xmax, __shfl_xor(xmax, off));
        ymax = fmaxf(ymax, __shfl_xor(ymax, off));
    }
    __shared__ float red[4][kThreads / 64];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = xmin;
        red[1][w] = ymin;
        red[2][w] = xmax;
        red[3][w] = ymax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
        for (int i = 1; i < nw; ++i) {
            xmin = fminf(xmin, red[0][i]);
            ymin = fminf(ymin, red[1][i]);
            xmax = fmaxf(xmax, red[2][i]);
            ymax = fmaxf(ymax, red[3][i]);
        }
        if (xmin <= xmax) {  // at least one finite position in the block
            unsigned int* mm = st->mm[set][slot % kBoxSlots];
            atomicMin(mm + 0, enc_ord(xmin));
            atomicMin(mm + 1, enc_ord(ymin));
            atomicMax(mm + 2, enc_ord(xmax));
            atomicMax(mm + 3, enc_ord(ymax));
        }
    }
}

}  // namespace tfdp
