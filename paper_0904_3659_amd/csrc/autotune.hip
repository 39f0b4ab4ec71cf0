// Variant timer: runs every compiled variant of a kind on synthetic inputs
// of each requested size, times it with HIP events on the caller's stream
// and records the fastest in the tuning table (bucketed by log2 of the
// size).  The paper notes that the depth of loop unrolling decides the
// speed (Sec. VII); here the choice is measured instead of fixed.
#include "common.hpp"

#include <algorithm>
#include <vector>

namespace nbody {
namespace {

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

struct DeviceBuffers {
    std::vector<void *> ptrs;
    ~DeviceBuffers()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
    nbody_status alloc(size_t bytes, float **out)
    {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(autotune inputs)");
        ptrs.push_back(p);
        *out = static_cast<float *>(p);
        return NBODY_OK;
    }
};

// Times run(v) for every v < count with timed(v), keeping the fastest in
// *best (-1 if none ran).  A variant whose run fails for lack of memory is
// skipped like one that is not timed; any other failure ends the timing.
template <class Run, class Timed>
nbody_status time_best(int count, hipStream_t stream, Run run, Timed timed, int *best)
{
    Events ev;
    hipError_t e = hipEventCreate(&ev.a);
    if (e == hipSuccess) e = hipEventCreate(&ev.b);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    float best_ms = 0.f;
    *best = -1;
    int warm = -1;  // the first variant that is timed and runs
    for (int v = 0; v < count && warm < 0; ++v) {
        if (!timed(v)) continue;
        const nbody_status st = run(v);
        if (st == NBODY_OK) warm = v;
        else if (st != NBODY_ERROR_OUT_OF_MEMORY) return st;
    }
    if (warm < 0) return NBODY_OK;
    // bring the clock up first: at least 100 ms of back-to-back runs, so the
    // first variants are not timed while the GPU leaves its idle state
    if ((e = hipEventRecord(ev.a, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    for (int k = 0; k < 1000; ++k) {
        nbody_status st = run(warm);
        if (st != NBODY_OK) return st;
        if ((e = hipEventRecord(ev.b, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        if ((e = hipEventSynchronize(ev.b)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, ev.a, ev.b)) != hipSuccess)
            return hip_fail(e, "hipEventElapsedTime");
        if (ms >= 100.f) break;
    }
    for (int v = 0; v < count; ++v) {
        if (!timed(v)) continue;
        nbody_status st = run(v);  // warm-up (also builds any plan)
        if (st == NBODY_ERROR_OUT_OF_MEMORY) {
            clear_error();  // skipped: the device cannot hold its workspace
            continue;
        }
        if (st != NBODY_OK) return st;
        float min_ms = -1.f;
        for (int rep = 0; rep < 3; ++rep) {
            if ((e = hipEventRecord(ev.a, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
            if ((st = run(v)) != NBODY_OK) return st;
            if ((e = hipEventRecord(ev.b, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
            if ((e = hipEventSynchronize(ev.b)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
            float ms = 0.f;
            if ((e = hipEventElapsedTime(&ms, ev.a, ev.b)) != hipSuccess)
                return hip_fail(e, "hipEventElapsedTime");
            if (min_ms < 0.f || ms < min_ms) min_ms = ms;
            if (ms > 200.f) break;  // long runs: one timing is enough
        }
        if (*best < 0 || min_ms < best_ms) {
            best_ms = min_ms;
            *best = v;
        }
    }
    return NBODY_OK;
}

}  // namespace

nbody_status autotune_batched_run(const Device &dev, const int64_t *offsets, int64_t num_systems,
                                  const float *x, const float *m, float eps2, hipStream_t stream)
{
    const int64_t n = offsets[num_systems];
    DeviceBuffers buf;
    float *a, *p;
    nbody_status st;
    if ((st = buf.alloc(12 * (size_t)n, &a)) || (st = buf.alloc(4 * (size_t)n, &p))) return st;
    int best = -1;
    // the timing runs' plans stay out of the shared cache; the winner's is
    // then built there by one ordinary run
    begin_private_batched_plans();
    st = time_best(batched_variant_count(), stream, [&](int v) {
        return batched_run(v, dev, offsets, num_systems, x, m, eps2, a, p, stream);
    }, [](int) { return true; }, &best);
    end_private_batched_plans();
    if (st != NBODY_OK) return st;
    if (best < 0) return fail(NBODY_ERROR_OUT_OF_MEMORY, "no batched variant fits device memory");
    record_tuned_variant(NBODY_KIND_BATCHED, num_systems > 0 ? n / num_systems : 0, best);
    return batched_run(best, dev, offsets, num_systems, x, m, eps2, a, p, stream);
}

nbody_status autotune_run(int kind, const Device &dev, const int64_t *sizes, int64_t count,
                          hipStream_t stream)
{
    for (int64_t k = 0; k < count; ++k) {
        const int64_t size = sizes[k];
        DeviceBuffers buf;
        nbody_status st;
        int best = -1;
        if (kind == NBODY_KIND_BATCHED) {
            const int64_t ns = size;
            const int64_t systems = std::max<int64_t>(1, ((int64_t)1 << 22) / ns);
            const int n = (int)(ns * systems);
            std::vector<int64_t> offsets(systems + 1);
            for (int64_t s = 0; s <= systems; ++s) offsets[s] = s * ns;
            float *x, *m, *a, *p;
            if ((st = buf.alloc(12 * (size_t)n, &x)) || (st = buf.alloc(4 * (size_t)n, &m)) ||
                (st = buf.alloc(12 * (size_t)n, &a)) || (st = buf.alloc(4 * (size_t)n, &p)))
                return st;
            if ((st = fill_synthetic(x, m, nullptr, nullptr, n, 7u, stream)) != NBODY_OK) return st;
            begin_private_batched_plans();  // plans of synthetic offsets: not kept
            st = time_best(batched_variant_count(), stream, [&](int v) {
                return batched_run(v, dev, offsets.data(), systems, x, m, 1e-4f, a, p, stream);
            }, [](int) { return true; }, &best);
            end_private_batched_plans();
            if (st != NBODY_OK) return st;
            if (best < 0) return fail(NBODY_ERROR_OUT_OF_MEMORY, "no batched variant fits device memory");
            record_tuned_variant(kind, ns, best);
            continue;
        }
        const int n = (int)size;
        // variants timed at this size: those whose size band admits n and
        // whose workspace fits the cap (a quarter of free memory, at most
        // NBODY_TUNE_WORKSPACE_CAP); the workspace the timing grows is given
        // back afterwards
        size_t free_b = 0, total_b = 0;
        hipError_t he = hipMemGetInfo(&free_b, &total_b);
        if (he != hipSuccess) return hip_fail(he, "hipMemGetInfo");
        const size_t cap = tune_workspace_cap(free_b);
        const int nv = kind == NBODY_KIND_FORWARD ? forward_variant_count() : backward_variant_count();
        std::vector<char> admit(nv, 0);
        for (int v = 0; v < nv; ++v) {
            int per_cu = 1;
            st = kind == NBODY_KIND_FORWARD ? forward_variant_occupancy(v, &per_cu)
                                            : backward_variant_occupancy(v, &per_cu);
            if (st != NBODY_OK) return st;
            const int64_t ws = kind == NBODY_KIND_FORWARD ? forward_plan_bytes(v, n, dev.num_cu, per_cu)
                                                          : backward_plan_bytes(v, n, dev.num_cu, per_cu);
            const int64_t mx = kind == NBODY_KIND_FORWARD ? forward_variant_max_n(v)
                                                          : backward_variant_max_n(v);
            admit[v] = tune_admissible(n, mx, ws, cap);
        }
        const auto timed = [&](int v) { return admit[v] != 0; };
        const size_t ws_before = workspace_size(dev, stream);
        float *x, *m, *a, *p;
        if ((st = buf.alloc(12 * (size_t)n, &x)) || (st = buf.alloc(4 * (size_t)n, &m)) ||
            (st = buf.alloc(12 * (size_t)n, &a)) || (st = buf.alloc(4 * (size_t)n, &p)))
            return st;
        if (kind == NBODY_KIND_FORWARD) {
            if ((st = fill_synthetic(x, m, nullptr, nullptr, n, 11u, stream)) != NBODY_OK) return st;
            st = time_best(forward_variant_count(), stream, [&](int v) {
                return forward_run(v, dev, x, m, n, 1e-4f, a, p, stream);
            }, timed, &best);
        } else {
            float *w, *vv, *gx, *gm;
            if ((st = buf.alloc(12 * (size_t)n, &w)) || (st = buf.alloc(4 * (size_t)n, &vv)) ||
                (st = buf.alloc(12 * (size_t)n, &gx)) || (st = buf.alloc(4 * (size_t)n, &gm)))
                return st;
            if ((st = fill_synthetic(x, m, w, vv, n, 13u, stream)) != NBODY_OK) return st;
            st = time_best(backward_variant_count(), stream, [&](int v) {
                return backward_run(v, dev, x, m, n, 1e-4f, w, vv, gx, gm, stream);
            }, timed, &best);
        }
        const nbody_status trim = workspace_trim(dev, stream, ws_before);
        if (st != NBODY_OK) return st;
        if (trim != NBODY_OK) return trim;
        if (best < 0) return fail(NBODY_ERROR_OUT_OF_MEMORY, "no variant fits at n = %d", n);
        record_tuned_variant(kind, n, best);
        // buffers are freed by hipFree (which waits for the device)
    }
    return NBODY_OK;
}

}  // namespace nbody
