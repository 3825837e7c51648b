// The solve entry point that allocates no memory: for callers that cannot
// allocate device memory (a serving loop that must not call hipMalloc, a
// harness that forbids it).  Its workspace is `scratch`, a fixed array in
// device memory of CGS_NOALLOC_SCRATCH_BYTES: every GPU the library runs on
// holds its own copy at its own address from the time the library's code is
// loaded until the process ends.  Host code never passes the array's name to
// a kernel or a copy (on the host it only stands in for the symbol): the
// device address is looked up once per device with hipGetSymbolAddress and
// kept in g_scratch[device].
#include <hip/hip_runtime.h>

#include <mutex>

#include "engine.hpp"

namespace {

static __device__ __align__(256) unsigned char scratch[CGS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu[kMaxDevices];           // one call at a time per device
void* g_scratch[kMaxDevices] = {};      // device address of `scratch` (null: not looked up yet)

// The device address of the calling thread's current device's array.
int scratch_ptr(int dev, void** out) {
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return cgs::fail(CGS_EHIP, "hipGetSymbolAddress of the scratch array on device %d failed: %s", dev,
                             hipGetErrorString(e));
        if ((uintptr_t)p % 256)
            return cgs::fail(CGS_EHIP, "scratch array on device %d is not 256-byte aligned", dev);
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return CGS_OK;
}

}  // namespace

extern "C" int cgs_solve_noalloc(const cgs_op* op, int64_t l, const int64_t* q, int64_t nq,
                                 const cgs_settings* st, const double* b, const double* c, void* stream,
                                 double* x, double* y, double* sl, cgs_info* info) {
    if (!op || !st || !b || !c) return cgs::fail(CGS_EINVAL, "op, settings, b and c must not be null");
    CGS_TRY(cgs::validate_settings(st));
    if (st->precision == CGS_BF16) return cgs::fail(CGS_EINVAL, "the no-allocation solve takes FP64 or FP32");
    // no graph: instantiating one allocates device memory
    cgs_settings s2 = *st;
    s2.use_graph = 0;
    size_t need = 0;
    CGS_TRY(cgs_workspace_bytes(op, l, q, nq, &s2, 1, &need));
    if (need > (size_t)CGS_NOALLOC_SCRATCH_BYTES)
        return cgs::fail(CGS_ENOMEM,
                         "the problem needs %zu bytes of device workspace; the no-allocation solve has %zu "
                         "(CGS_NOALLOC_SCRATCH_BYTES): use cgs_solver_create with a workspace of that size",
                         need, (size_t)CGS_NOALLOC_SCRATCH_BYTES);
    int dev = -1;
    CGS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return cgs::fail(CGS_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_mu[dev]);
    void* ws = nullptr;
    CGS_TRY(scratch_ptr(dev, &ws));
    // Everything the solve reads is written first by the creation, the data
    // upload and the reset kernels, so the previous call's contents do not matter.
    cgs_solver* s = nullptr;
    CGS_TRY(cgs::solver_create(op, l, q, nq, &s2, 1, ws, (size_t)CGS_NOALLOC_SCRATCH_BYTES, stream, true, &s));
    int rc = cgs_solver_set_data(s, 0, b, c);
    if (rc == CGS_OK) rc = cgs_solve(s, info);
    if (rc == CGS_OK) rc = cgs_solver_get_solution(s, 0, x, y, sl);
    cgs_solver_destroy(s);   // (synchronises the stream: the array is free again)
    return rc;
}
