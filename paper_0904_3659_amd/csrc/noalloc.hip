// nbody_forces_noalloc (include/nbody.h): the forward evaluation with its
// workspace in a fixed device region the library declares here, for
// callers that cannot allocate device memory.
#include "common.hpp"

#include <map>
#include <mutex>

namespace nbody {

// Device memory of nbody_forces_noalloc: partial sums in the first
// NBODY_NOALLOC_SCRATCH_BYTES - kScratchCounterBytes bytes, int counters
// (zero between calls) in the last kScratchCounterBytes.  Every device the
// library runs on holds its own copy until the process ends.  In host code
// `scratch` names a host-side stand-in, never the device memory: kernels and
// fills take the address hipGetSymbolAddress gives for the current device.
constexpr size_t kScratchCounterBytes = 4096;
static __device__ __align__(256) unsigned char scratch[NBODY_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, unsigned char *> g_scratch;  // device -> address of its scratch
}  // namespace

// The scratch region of the current device as an Arena; on the first call
// on a device, looks up its address and zeroes its counters on `stream`
// with a fill kernel (no memset, so the call may sit in a captured graph).
static nbody_status scratch_arena(const Device &dev, hipStream_t stream, Arena *out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch.find(dev.id);
    unsigned char *ptr = nullptr;
    if (it == g_scratch.end()) {
        hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        nbody_status st = fill_zero_int(
            reinterpret_cast<int *>(ptr + NBODY_NOALLOC_SCRATCH_BYTES - kScratchCounterBytes),
            kScratchCounterBytes / sizeof(int), stream);
        if (st != NBODY_OK) return st;
        g_scratch[dev.id] = ptr;
    } else {
        ptr = it->second;
    }
    out->base = ptr;
    out->cap = NBODY_NOALLOC_SCRATCH_BYTES - kScratchCounterBytes;
    out->counters = reinterpret_cast<int *>(ptr + out->cap);
    out->counter_count = kScratchCounterBytes / sizeof(int);
    return NBODY_OK;
}

}  // namespace nbody

using namespace nbody;

extern "C" {

nbody_status nbody_forces_noalloc(const float *x, const float *m, int64_t n, float eps2,
                                  float *a, float *p, void *stream)
{
    clear_error();
    if (n < 0 || n > NBODY_MAX_N)
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "n = %lld outside [0, %lld]", (long long)n,
                    (long long)NBODY_MAX_N);
    if (bad_eps2(eps2)) return fail(NBODY_ERROR_INVALID_ARGUMENT, "eps2 = %g is negative or not finite", eps2);
    if (n == 0) return NBODY_OK;
    if (!x || !m || !a) return fail(NBODY_ERROR_INVALID_ARGUMENT, "NULL x, m or a with n = %lld", (long long)n);
    const size_t v3 = 12 * (size_t)n, v1 = 4 * (size_t)n;
    if (overlaps(a, v3, x, v3) || overlaps(a, v3, m, v1) || overlaps(p, v1, x, v3) ||
        overlaps(p, v1, m, v1) || overlaps(a, v3, p, v1))
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "output arrays overlap each other or the inputs");
    Device dev;
    nbody_status st = current_device(&dev);
    if (st != NBODY_OK) return st;
    Arena arena;
    st = scratch_arena(dev, (hipStream_t)stream, &arena);
    if (st != NBODY_OK) return st;
    return forward_run(select_variant(NBODY_KIND_FORWARD, n), dev, x, m, (int)n, eps2, a, p,
                       (hipStream_t)stream, nullptr, nullptr, arena);
}

}  // extern "C"
