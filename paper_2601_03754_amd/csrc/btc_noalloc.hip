// Solve entry point for callers that cannot allocate device memory (code
// under HIP graph capture, serving loops that must not call the allocator):
// the solve workspace lives in a fixed device array of this file instead of
// memory from the allocator.
#include <hip/hip_runtime.h>

#include <mutex>

#include "btc.h"
#include "btc_handle.h"

using namespace btc_host;

namespace {

constexpr size_t kScratchBytes = (size_t)BTC_NOALLOC_MAX_BYTES;
constexpr int kMaxDevices = 64;

// One copy per GPU, held until the process ends.  In host code the name is
// only a stand-in for the symbol: kernels and copies get the address that
// hipGetSymbolAddress reports for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array (looked up once per device,
// with that device current).
int scratch_ptr(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return BTC_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return BTC_ERR_HIP;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return BTC_OK;
}

}  // namespace

extern "C" {

BTC_API int btc_solve_noalloc(btc_handle h, const double* B, double* X, int64_t nrhs, void* stream,
                              btc_solve_info* info) {
    int rc = check_solve(h, B, X, nrhs);
    if (rc != 0) return rc < 0 ? rc : BTC_OK;
    if (workspace_bytes(h->N, h->n, h->precision, nrhs) > kScratchBytes) return BTC_ERR_UNSUPPORTED;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return BTC_ERR_HIP;
    if (dev != h->device) return -1;  // the handle lives on another device
    void* base = nullptr;
    rc = scratch_ptr(dev, &base);
    if (rc != BTC_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    note_stream(h, st);
    h->stream = st;
    const Workspace w = carve_at(base, h->N, h->n, h->precision, nrhs);
    return solve_with(h, w, B, X, nrhs, st, info);
}

}  // extern "C"
