// Block solve (Sec. III-A, Eq. (4)) on scratch memory the library holds
// itself, for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The scratch is one file-scope device array of fixed size.  Each GPU the
// library runs on holds its own copy until the process ends; its address on
// a device comes from hipGetSymbolAddress, looked up once per device with
// that device current (the array's name in host code is only a stand-in
// for the symbol, never a device address).  The solve initialises every
// part of its workspace it reads, so the previous call's contents do not
// matter; calls that overlap on one GPU share the array and race.
#include <mutex>

#include "kernels.hpp"

namespace bko {

constexpr size_t kNoAllocScratchBytes = BKO_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up on the
// first call on that device).
bko_status scratch_address(void **out)
{
    int dev = -1;
    BKO_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d outside the %d devices the scratch table covers", dev, kMaxDevices);
        return BKO_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        BKO_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (p == nullptr || reinterpret_cast<uintptr_t>(p) % 256 != 0) {
            set_error("scratch symbol address %p is not usable", p);
            return BKO_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return BKO_OK;
}

}  // namespace
}  // namespace bko

using namespace bko;

extern "C" {

bko_status bko_block_krylov_solve_noalloc(bko_op A, int s, const double *B, int ldb, double *X, int ldx,
                                          const double *X0, int ldx0, bko_dtype compute, double tol, int max_iter,
                                          bko_solve_info *info, void *stream)
{
    try {
        size_t need = 0;
        bko_status st = bko_block_krylov_workspace_bytes(A, s, compute, &need);
        if (st != BKO_OK) return st;
        if (need > kNoAllocScratchBytes) {
            set_error("this solve needs %zu bytes of scratch; the no-allocation entry point holds %zu per device "
                      "(use bko_block_krylov_solve with a caller workspace)",
                      need, kNoAllocScratchBytes);
            return BKO_EINVAL;
        }
        void *work = nullptr;
        if ((st = scratch_address(&work)) != BKO_OK) return st;
        return bko_block_krylov_solve(A, s, B, ldb, X, ldx, X0, ldx0, compute, tol, max_iter, work,
                                      kNoAllocScratchBytes, info, stream);
    } catch (...) {
        set_error("unexpected C++ exception");
        return BKO_EINVAL;
    }
}

}  // extern "C"
