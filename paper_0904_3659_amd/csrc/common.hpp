// Internal declarations shared by the translation units of libnbody.so.
// Host side: status reporting, device checks, workspace cache, variant
// tables.  Device side: the softened pair interaction of Eq. (gravity).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/nbody.h"
#include "leapfrog_epi.hpp"

namespace nbody {

// ------------------------------------------------------------------ host

// Record a failure for nbody_last_error() and return `status`.
nbody_status fail(nbody_status status, const char *fmt, ...);
// Map a HIP error to a status, recording `what` and the HIP message.
nbody_status hip_fail(hipError_t err, const char *what);
// Clear the thread-local error text (called at the start of each entry).
void clear_error();

struct Device {
    int id = -1;
    int num_cu = 0;
};

// Current HIP device; UNSUPPORTED_DEVICE unless it is a gfx950.
nbody_status current_device(Device *dev);

// Grow-only device buffer private to (device, stream).  The pointer stays
// valid until the next workspace() call on the same (device, stream) that
// asks for more bytes, or nbody_release_workspace().
nbody_status workspace(const Device &dev, hipStream_t stream, size_t bytes, void **ptr);
// A second buffer of the same kind (same lifetime rules), for callers that
// keep data across calls that use workspace() (the leap-frog adjoint's
// unfused VJP results).
nbody_status workspace_aux(const Device &dev, hipStream_t stream, size_t bytes, void **ptr);

// Per-(device, stream) array of at least `count` int counters that are zero
// between calls (kernels that use them leave them at zero); zero-filled
// with a kernel when first allocated or grown.
nbody_status counters(const Device &dev, hipStream_t stream, size_t count, int **ptr);

// Where a call's library workspace comes from: the per-(device, stream)
// grow-only cache above (base == NULL), or a fixed region of `cap` bytes
// that the caller owns (the entry point that allocates nothing), with
// `counter_count` int counters at `counters` that are zero between calls.
struct Arena {
    void *base = nullptr;
    size_t cap = 0;
    int *counters = nullptr;
    size_t counter_count = 0;
    // Bytes a kernel family may plan for, given its own default limit.
    size_t budget(size_t dflt) const { return base ? (cap < dflt ? cap : dflt) : dflt; }
    // `bytes` of workspace (INVALID_ARGUMENT if a fixed region is too small).
    nbody_status get(const Device &dev, hipStream_t stream, size_t bytes, void **ptr) const;
    // `count` counters that are zero between calls.
    nbody_status get_counters(const Device &dev, hipStream_t stream, size_t count, int **ptr) const;
};

// NBODY_FAULT=<what> makes the named step report failure (tests of the
// error paths; checked on the host before anything is launched).
bool fault_injected(const char *what);

// Check that [a, a+abytes) and [b, b+bbytes) are disjoint (NULL or empty
// ranges never overlap).
bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes);

// Launch status of the last kernel launch on this thread.
nbody_status check_launch(const char *what);

// Profiling marks (no-ops unless nbody_profile_enable(1)): 0 before the
// pair kernel, 1 after it, 2 after the call's last kernel (commits).
void prof_mark(hipStream_t stream, int which);

// Variant of `kind` for size n: forced, else tuned, else the default.
int select_variant(int kind, int64_t n);
// eps2 negative, NaN or infinite (rejected by every entry point).
bool bad_eps2(float eps2);

// Forced variant (>= 0) for a kind, or -1 for automatic choice.
int forced_variant(int kind);
// Tuned variant for (kind, n) from the tuning table, or -1.
int tuned_variant(int kind, int64_t n);
void record_tuned_variant(int kind, int64_t n, int index);

// ---- forward (Eq. (gravity))
int forward_variant_count();
const char *forward_variant_name(int index);
int forward_default_variant(int64_t n);
bool forward_variant_f64sum(int variant);
int forward_default_f64sum_variant(int64_t n);
// With `epi` (mode != kLfNone) the leap-frog update follows the store of a:
// inside the final reduction kernel where the variant has one that can take
// it (*fused = true), otherwise not at all (*fused = false; the caller then
// runs lf_epilogue_run).
nbody_status forward_run(int variant, const Device &dev, const float *x, const float *m,
                         int n, float eps2, float *a, float *p, hipStream_t stream,
                         const LfEpi *epi = nullptr, bool *fused = nullptr,
                         const Arena &arena = Arena{});

// Pair-once forward kernel (forward_sym.hip) with W waves and K rows/lane.
nbody_status forward_sym_run(int W, int K, int occ, int rounds, const char *name,
                             const Device &dev, const float *x, const float *m, int n, float eps2,
                             float *a, float *p, hipStream_t stream, const LfEpi *epi, bool *fused,
                             const Arena &arena);

// Occupancy of the pair-once forward kernel with W waves and K rows/lane.
nbody_status forward_sym_occupancy(int W, int K, int *per_cu);
// Workspace bytes of a forward variant at size n on a device of num_cu CUs
// where its pair kernel fits per_cu workgroups per CU (host arithmetic
// only), or -1 for bad arguments or a size its plan cannot hold.
int64_t forward_plan_bytes(int variant, int64_t n, int num_cu, int per_cu);
// Largest n the variant timer times a forward variant at.
int64_t forward_variant_max_n(int variant);
// Workgroups per CU of a forward variant's pair kernel.
nbody_status forward_variant_occupancy(int variant, int *per_cu);

// ---- backward (vector-Jacobian product of Eq. (gravity))
int backward_variant_count();
const char *backward_variant_name(int index);
// The same with and without upstream potential weights (grad_p).
int backward_default_variant(int64_t n);
// `epi` / `fused` as for forward_run (kLfAdjoint updates; gx, gm still
// receive the result when the update is not fused).
nbody_status backward_run(int variant, const Device &dev, const float *x, const float *m,
                          int n, float eps2, const float *ga, const float *gp,
                          float *gx, float *gm, hipStream_t stream,
                          const LfEpi *epi = nullptr, bool *fused = nullptr,
                          const Arena &arena = Arena{});

// As the forward_* planning functions, for the backward variants.
int64_t backward_plan_bytes(int variant, int64_t n, int num_cu, int per_cu);
int64_t backward_variant_max_n(int variant);
nbody_status backward_variant_occupancy(int variant, int *per_cu);

// ---- batched independent systems
int batched_variant_count();
const char *batched_variant_name(int index);
int batched_default_variant(int64_t mean_n);
nbody_status batched_run(int variant, const Device &dev, const int64_t *offsets,
                         int64_t num_systems, const float *x, const float *m, float eps2,
                         float *a, float *p, hipStream_t stream);

// ---- elementwise
nbody_status axpy_run(float *y, const float *xv, int64_t len, float alpha, hipStream_t stream);
nbody_status kick_drift_run(float *x, float *v, const float *a, int64_t len, float kick, float dt,
                            hipStream_t stream);
// The update `e` for n rows whose result is in r3[n][3] (and r1[n], may be
// NULL): the unfused form of the epilogue of forward_run / backward_run.
nbody_status lf_epilogue_run(const float *r3, const float *r1, int64_t n, const LfEpi &e,
                             hipStream_t stream);
// Zero len ints with a fill kernel on `stream` (no hipMemsetAsync, so the
// work can sit in a captured graph).
nbody_status fill_zero_int(int *p, size_t len, hipStream_t stream);
// Deterministic timing inputs (unit cube, masses 1/n, weights in [-1,1));
// w and v may be NULL.
nbody_status fill_synthetic(float *x, float *m, float *w, float *v, int n, uint32_t seed,
                            hipStream_t stream);

// ---- variant timer (nbody_autotune)
// The timer times a variant only where its size band admits n and its
// workspace (-1: its plan cannot hold n) fits `cap`.
inline bool tune_admissible(int64_t n, int64_t max_n, int64_t ws_bytes, size_t cap)
{
    return ws_bytes >= 0 && n <= max_n && (size_t)ws_bytes <= cap;
}
// Workspace cap of the timer: NBODY_TUNE_WORKSPACE_CAP bytes (default 2 GiB)
// or a quarter of the device's free memory, whichever is smaller.
size_t tune_workspace_cap(size_t free_bytes);
// Bytes of the (device, stream) workspace, and shrinking it back to at
// most `bytes` (freed if 0; synchronises when it frees).
size_t workspace_size(const Device &dev, hipStream_t stream);
nbody_status workspace_trim(const Device &dev, hipStream_t stream, size_t bytes);

nbody_status autotune_run(int kind, const Device &dev, const int64_t *sizes, int64_t count,
                          hipStream_t stream);
// Times every batched variant on the caller's ensemble and records the
// fastest for the bucket of its mean system size.
nbody_status autotune_batched_run(const Device &dev, const int64_t *offsets, int64_t num_systems,
                                  const float *x, const float *m, float eps2, hipStream_t stream);

// ---- errors
const char *last_error_cstr();

// ---- workspace release hooks of the batched plan cache
void release_batched_plans();
// Until end_private_batched_plans(), batched plans built on this thread go
// to a private list (not the shared cache); the end frees them.
void begin_private_batched_plans();
void end_private_batched_plans();

}  // namespace nbody

#include "pair_term.hpp"
