// rplu_dense_noalloc: the dense step loop of rplu_dense on a fixed device
// array instead of context workspace, for callers that may not allocate.
//
// The array below is this library's scratch on every device it runs on. Host
// code never uses its name as an address: the first call on a device asks the
// runtime for that device's copy (hipGetSymbolAddress, with the device
// current) and keeps the pointer; kernels receive that pointer, as they
// receive the context workspace in rplu_dense. Nothing in this path calls
// hipMalloc, hipFree, graph instantiation or any other allocating routine.
// Every buffer the kernels read is written first in the same call (the step
// state by its init kernel, the masses by the initial sweep, chunk totals by
// each draw), so leftovers of an earlier call are never read. Calls that
// overlap on one device share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rplu.h"
#include "runtime.hpp"

namespace rplu {
namespace {

static __device__ __align__(256) unsigned char scratch[RPLU_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (the current device).
rplu_status scratch_ptr(int device, void** out) {
    if (device < 0 || device >= kMaxDevices)
        return fail(RPLU_E_ARG, "rplu_dense_noalloc: device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device] == nullptr) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (p == nullptr || (uintptr_t)p % 256 != 0)
            return fail(RPLU_E_HIP, "rplu_dense_noalloc: scratch address %p unusable", p);
        g_ptr[device] = p;
    }
    *out = g_ptr[device];
    return RPLU_OK;
}

}  // namespace
}  // namespace rplu

using namespace rplu;

extern "C" {

size_t rplu_dense_noalloc_bytes(int dtype, int64_t n, int64_t m, uint32_t flags, int has_U) {
    if (dtype_size(dtype) == 0 || n < 1 || m < 1) return 0;
    return dense_ws_layout(dtype, n, m, flags, has_U == 0, false).total;
}

rplu_status rplu_dense_noalloc(rplu_dtype dtype, int64_t n, int64_t m, void* A, int64_t lda,
                               const rplu_opts* opts, int32_t* piv, void* L, int64_t ldl,
                               void* U, int64_t ldu, rplu_info* info, void* hip_stream) {
    rplu_status rc = dense_check("rplu_dense_noalloc", dtype, n, m, A, lda, opts, piv, L, ldl, U,
                                 ldu, info);
    if (rc) return rc;
    if (opts->flags & RPLU_FLAG_KEEP_INPUT)
        return fail(RPLU_E_UNSUPPORTED, "rplu_dense_noalloc: RPLU_FLAG_KEEP_INPUT needs a copy of A");
    const DenseWs w = dense_ws_layout(dtype, n, m, opts->flags, U == nullptr, false);
    if (w.total > (size_t)RPLU_NOALLOC_SCRATCH_BYTES)
        return fail(RPLU_E_ARG,
                    "rplu_dense_noalloc: needs %zu bytes of scratch, the limit is %zu "
                    "(use rplu_dense)", w.total, (size_t)RPLU_NOALLOC_SCRATCH_BYTES);
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    void* ws = nullptr;
    rc = scratch_ptr(device, &ws);
    if (rc) return rc;
    return dense_run(nullptr, (char*)ws, dtype, n, m, A, lda, opts, piv, L, ldl, U, ldu, info,
                     (hipStream_t)hip_stream);
}

}  // extern "C"
