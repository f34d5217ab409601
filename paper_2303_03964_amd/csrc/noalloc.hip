// Layout quality (Sec. 4, "Metrics") for callers that cannot allocate device
// memory: the metric's scratch lives in a fixed array of this library, one
// copy per GPU, instead of a caller workspace.
//
// The array's name is only a host-side stand-in in host code: its device
// address is resolved once per device with hipGetSymbolAddress (the device
// current at the first call) and that address is what the kernels and the
// memsets receive.
#include <mutex>

#include "tfdp_handle.h"

namespace {

constexpr size_t kStaticScratchBytes = (size_t)64 << 20;  // 64 MiB per GPU, held until the process ends
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_mu;                 // guards g_ptr and serialises the calls of this process
void* g_ptr[kMaxDevices] = {};   // device address of `scratch` per device (null until resolved)

// Address of the current device's copy of the scratch array (resolved on the
// first call on that device). Caller holds g_mu.
tfdp_status scratch_for_current_device(void** out) {
    int dev = -1;
    tfdp_status st = tfdp::check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (st != TFDP_OK) return st;
    if (dev < 0 || dev >= kMaxDevices) {
        tfdp::set_msg("device index outside the library's table of static scratch arrays");
        return TFDP_ERR_UNSUPPORTED;
    }
    if (!g_ptr[dev]) {
        void* p = nullptr;
        st = tfdp::check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
        if (st != TFDP_OK) return st;
        if (!p) {
            tfdp::set_msg("hipGetSymbolAddress returned no address for the static scratch array");
            return TFDP_ERR_HIP;
        }
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return TFDP_OK;
}

}  // namespace

extern "C" tfdp_status tfdp_quality_sampled_noalloc(int32_t n, int64_t nnz, const int32_t* d_row_ptr,
                                                    const int32_t* d_col_idx, const float* d_pos,
                                                    const int32_t* d_sources, int32_t nsrc, double* se, double* np,
                                                    int32_t* levels, hipStream_t stream) {
    tfdp::set_msg("");
    if (n < 1 || nnz < 0 || nsrc < 1 || nsrc > 64 || !d_row_ptr || (!d_col_idx && nnz > 0) || !d_pos ||
        !d_sources || !se || !np) {
        tfdp::set_msg("invalid sizes or pointers (1 <= nsrc <= 64; se and np must be set)");
        return TFDP_ERR_INVALID_ARG;
    }
    const size_t need = tfdp::stress_workspace_bytes(n, nsrc);
    if (need > kStaticScratchBytes) {
        tfdp::set_msg("metric scratch of " + std::to_string(need) + " bytes exceeds the static scratch of " +
                      std::to_string(kStaticScratchBytes) + " bytes (use tfdp_quality_sampled with a workspace)");
        return TFDP_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    void* work = nullptr;
    tfdp_status st = scratch_for_current_device(&work);
    if (st != TFDP_OK) return st;
    // every buffer the metric reads is cleared or initialised by the metric
    // itself, so the contents left by an earlier call do not matter
    int lv = 0;
    const int e = tfdp::stress_sampled(n, nnz, d_row_ptr, d_col_idx, reinterpret_cast<const float2*>(d_pos),
                                       d_sources, nsrc, work, se, np, &lv, stream);
    if (levels) *levels = lv;
    if (e == -1) {
        tfdp::set_msg("invalid CSR: row_ptr must start at 0, be monotone and end at nnz; columns in [0, n)");
        return TFDP_ERR_INVALID_ARG;
    }
    if (e == -2) {
        tfdp::set_msg("a source node is outside [0, n)");
        return TFDP_ERR_INVALID_ARG;
    }
    if (e == -3) {
        tfdp::set_msg("the BFS still reaches new nodes at hop distance 65534 (16-bit distances)");
        return TFDP_ERR_UNSUPPORTED;
    }
    if (e != 0) return tfdp::check_hip((hipError_t)e, "metrics");
    return tfdp::check_hip(hipGetLastError(), "kernel launch");
}
