// Block Gram product without device allocation: the entry point for callers
// that cannot allocate (code under HIP graph capture, serving loops, hosts
// that forbid hipMalloc).  The reduction partials live in a file-scope device
// array instead of a context's workspace.
#include <mutex>

#include "wd_internal.h"

namespace {

// Partial tiles of the two-pass Gram reduction: up to 512 workgroups, each
// writing one 16 x 16 complex tile plus 16 extra entries (as k_gram lays them
// out), 2.2 MB per GPU, held until the process ends.
constexpr size_t kScratchPairs = 512 * 272;
static __device__ __align__(256) double2 scratch[kScratchPairs];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double2* g_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of scratch, looked up once per device
// with the device current.  In host code the symbol name is only a host-side
// stand-in, so kernels receive this address instead.
int scratch_ptr(double2** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return WD_EHIP;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return WD_EHIP;
        }
        g_ptr[dev] = static_cast<double2*>(p);
    }
    *out = g_ptr[dev];
    return WD_OK;
}

}  // namespace

extern "C" {

int wd_block_gram_static(const void* P, const void* Q, long long N, int L, void* C, void* hip_stream) {
    if (!P || !Q || !C || N < 1 || L < 1 || L > WD_MAX_L) return WD_EINVAL;
    const int nb = wd::gram_blocks((size_t)N);
    if ((size_t)nb * wd::partial_stride() > kScratchPairs) return WD_EINVAL;
    double2* part = nullptr;
    int r = scratch_ptr(&part);
    if (r) return r;
    hipStream_t s = (hipStream_t)hip_stream;
    if (wd::launch_gram_partials((const double2*)P, (const double2*)Q, (size_t)N, L, part, nb, s) != hipSuccess)
        return WD_EHIP;
    if (wd::launch_reduce_gram(part, nb, L, (double2*)C, s) != hipSuccess) return WD_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return WD_EHIP;
    return WD_OK;
}

}  // extern "C"
