// tp_tprod_noalloc: the t-product of tp_tprod with its workspace in a
// device-resident array of this file instead of a caller-given buffer, for
// callers that cannot allocate.
#include <mutex>

#include "tp_internal.h"

// One array per GPU, allocated with the code object when the library is
// loaded on a device and held until the process ends.  Host code never uses
// the array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device (with that device current), and is
// kept in g_scratch.  Calls on one GPU share its array.
static constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
void* g_scratch[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];

int device_scratch(void** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return TP_ERR_HIP;
    std::call_once(g_scratch_once[dev], [dev]() {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_err[dev] = e;
        g_scratch[dev] = e == hipSuccess ? p : nullptr;
    });
    if (g_scratch_err[dev] != hipSuccess || !g_scratch[dev]) return TP_ERR_HIP;
    *out = g_scratch[dev];
    return TP_OK;
}

}  // namespace

extern "C" {

size_t tp_tprod_noalloc_max_bytes(void) { return kScratchBytes; }

int tp_tprod_noalloc(const float* A, const float* B, float* C, int n1, int n2, int l, int n3, int prec, void* stream)
{
    const int c = tp::check_tprod(A, B, C, n1, n2, l, n3, prec);
    if (c != TP_OK) return c;
    if (tp_tprod_workspace_size(n1, n2, l, n3, prec) > kScratchBytes) return TP_ERR_WORKSPACE;
    void* ws = nullptr;
    const int st = device_scratch(&ws);
    if (st != TP_OK) return st;
    return tp::run_tprod(A, B, C, n1, n2, l, n3, prec, ws, kScratchBytes, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
