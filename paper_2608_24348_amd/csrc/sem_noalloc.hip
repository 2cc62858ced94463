// Allocation-free entry point: the Poisson solve of sem_poisson_solve for one
// context, with its Krylov workspace in a static device array instead of
// device memory the caller allocates.  For callers that cannot allocate:
// code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc.
//
// The array lives for the whole process on every device the library runs on
// (the code object's global data).  Host code never passes the array's name
// to a kernel or a copy: in host code that name is a host-side stand-in.  The
// array's device address is looked up once per device, with that device
// current, by hipGetSymbolAddress, and only that address is used.
#include <mutex>
#include <string>

#include "sem_internal.h"

#define SEM_NOALLOC_BYTES ((size_t)256 << 20)
#define SEM_NOALLOC_MAXDEV 64

static __device__ __align__(256) unsigned char scratch[SEM_NOALLOC_BYTES];

namespace {

std::mutex g_mu;
char* g_ptr[SEM_NOALLOC_MAXDEV];

// device address of `scratch` on device dev
int scratch_ptr(int dev, char** out)
{
    if (dev < 0 || dev >= SEM_NOALLOC_MAXDEV)
        return semk::set_error(SEM_EINVAL, "device index out of range for the static workspace");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) return semk::set_error(SEM_EHIP, "hipGetDevice failed");
        if (cur != dev && hipSetDevice(dev) != hipSuccess) return semk::set_error(SEM_EHIP, "hipSetDevice failed");
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev && hipSetDevice(cur) != hipSuccess) return semk::set_error(SEM_EHIP, "hipSetDevice failed");
        if (e != hipSuccess || !p)
            return semk::set_error(SEM_EHIP, (std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)).c_str());
        g_ptr[dev] = (char*)p;
    }
    *out = g_ptr[dev];
    return 0;
}

}  // namespace

extern "C" {

size_t sem_noalloc_max_bytes(void) { return SEM_NOALLOC_BYTES; }

int sem_poisson_solve_noalloc(sem_ctx* ctx, const void* rhs, void* sol, sem_solve_stats* stats)
{
    size_t need = 0;
    int dev = 0;
    int rc = semk::poisson_external_bytes(ctx, &need, &dev);
    if (rc) return rc;
    if (need > SEM_NOALLOC_BYTES)
        return semk::set_error(SEM_ENOMEM, ("the allocation-free solve needs " + std::to_string(need) +
                                            " bytes of Krylov workspace; its static array holds " +
                                            std::to_string(SEM_NOALLOC_BYTES)).c_str());
    char* base = nullptr;
    if ((rc = scratch_ptr(dev, &base))) return rc;
    return semk::poisson_solve_external(ctx, base, SEM_NOALLOC_BYTES, rhs, sol, stats);
}

}  // extern "C"
