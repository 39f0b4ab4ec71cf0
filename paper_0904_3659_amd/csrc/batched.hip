// Eq. (gravity) (Sec. I) on many independent systems in one persistent
// launch, float32 on gfx950.
//
// Plan (host, built once per offsets content and cached):
//   every non-empty system s is cut into i-tiles of BLOCK particles; each
//   (system, i-tile) is a work unit {i_begin, i_end, j_begin, j_end} in
//   absolute particle indices.  A unit's cost is BLOCK lanes times its
//   system's padded j count, so units are sorted by decreasing cost
//   (largest first; ties keep system order) and dealt to the resident
//   workgroups in a snake order (g, 2G-1-g, 2G+g, ...), which balances the
//   static schedule without atomics or counters.
//
// Pair-once variants (bat_sym_*, bat_symd_*): a unit is (system s, block I)
// and runs the pair-once block evaluation of pair_once.hpp on that system
// alone (one chunk per block); its partial slots live in a per-plan region of
// library workspace, and a second launch adds each particle's slots in fixed
// order.  bat_symd_* take units from a ticket counter instead of the static
// snake deal.
//
// Kernel: a grid of exactly as many workgroups as the device holds at once;
// workgroup g walks its units, staging each system's j-range through LDS
// in BLOCK-particle tiles with the same masked/unmasked split, register
// i-rows and two-level accumulation as the single-system kernel.  Systems
// never read one another's particles, so a system's result does not depend
// on the rest of the batch.
#include "common.hpp"
#include "pair_once.hpp"

#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

namespace nbody {
namespace {

struct BatArgs {
    const int4 *units;
    int num_units;
    const float *x;
    const float *m;
    float eps2;
    float *a;
    float *p;
};

template <int BLOCK, int U>
__global__ __launch_bounds__(BLOCK) void batched_kernel(BatArgs P)
{
    constexpr int TILE = BLOCK;
    __shared__ float4 tile[TILE];
    const int tid = threadIdx.x;
    const int G = gridDim.x;
    const int g = blockIdx.x;
    const float eps2 = P.eps2;

    for (int pass = 0;; ++pass) {
        const int idx = (pass & 1) ? pass * G + (G - 1 - g) : pass * G + g;
        if (idx >= P.num_units) break;
        const int4 w = P.units[idx];
        const int i0 = w.x, iend = w.y, jbeg = w.z, jend = w.w;

        const int i = i0 + tid;
        const int ic = i < iend ? i : iend - 1;
        const float xi = P.x[3 * ic], yi = P.x[3 * ic + 1], zi = P.x[3 * ic + 2];
        float ax = 0.f, ay = 0.f, az = 0.f, pp = 0.f;

        float4 next = make_float4(0.f, 0.f, 0.f, 0.f);
        if (jbeg + tid < jend) {
            const int j = jbeg + tid;
            next = make_float4(P.x[3 * j], P.x[3 * j + 1], P.x[3 * j + 2], P.m[j]);
        }
        for (int t0 = jbeg; t0 < jend; t0 += TILE) {
            __syncthreads();
            tile[tid] = next;
            __syncthreads();
            {
                const int j = t0 + TILE + tid;
                next = make_float4(0.f, 0.f, 0.f, 0.f);
                if (j < jend) next = make_float4(P.x[3 * j], P.x[3 * j + 1], P.x[3 * j + 2], P.m[j]);
            }
            float tx = 0.f, ty = 0.f, tz = 0.f, tp = 0.f;
            const int cnt = min(TILE, jend - t0);
            const bool masked = (cnt < TILE) || (t0 < i0 + BLOCK && t0 + TILE > i0);
            if (!masked) {
                for (int jj = 0; jj < TILE; jj += U) {
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        pair_term(xi, yi, zi, tile[jj + u], eps2, tx, ty, tz, tp);
                }
            } else {
                for (int jj = 0; jj < cnt; ++jj)
                    pair_term_masked(xi, yi, zi, tile[jj], eps2, t0 + jj == i, tx, ty, tz, tp);
            }
            ax += tx;
            ay += ty;
            az += tz;
            pp += tp;
        }
        if (i < iend) {
            P.a[3 * i + 0] = ax;
            P.a[3 * i + 1] = ay;
            P.a[3 * i + 2] = az;
            if (P.p) P.p[i] = pp;
        }
    }
}

// ---- pair-once units: {system base, system size, block I, partial offset}
struct BatSymArgs {
    const int4 *units;
    int num_units;
    const float *x;
    const float *m;
    float eps2;
    float4 *partial;
};

template <int W, int K>
__global__ __launch_bounds__(W * 64) void batched_sym_kernel(BatSymArgs A)
{
    constexpr int PB = W * 64 * K;
    __shared__ float4 tile[kTileLds];
    __shared__ float4 jacc[W][kSlotLds];
    const int G = gridDim.x;
    const int g = blockIdx.x;
    for (int pass = 0;; ++pass) {
        const int idx = (pass & 1) ? pass * G + (G - 1 - g) : pass * G + g;
        if (idx >= A.num_units) break;
        const int4 u = A.units[idx];
        const int ns = u.y;
        const int M = (ns + PB - 1) / PB;
        pair_once_block<W, K, true>(A.x + 3 * (size_t)u.x, A.m + u.x, ns, A.eps2, M, u.z, 0, 1,
                                    0, M / 2 + 1, A.partial + u.w, tile, jacc);
    }
}

// The same units taken dynamically: workgroups draw the next unit of the
// cost-sorted list from a ticket counter (largest first, then whoever is
// free takes the next), which balances the tail better than a static deal
// when units of equal estimated cost run at different speeds.  The last
// workgroup to finish resets the counters for the next launch on the stream.
template <int W, int K>
__global__ __launch_bounds__(W * 64) void batched_sym_dyn_kernel(BatSymArgs A, int *ctr)
{
    constexpr int PB = W * 64 * K;
    __shared__ float4 tile[kTileLds];
    __shared__ float4 jacc[W][kSlotLds];
    __shared__ int s_idx;
    for (;;) {
        __syncthreads();  // every thread has read the previous ticket
        if (threadIdx.x == 0) s_idx = atomicAdd(ctr, 1);
        __syncthreads();
        const int idx = s_idx;
        if (idx >= A.num_units) break;
        const int4 u = A.units[idx];
        const int ns = u.y;
        const int M = (ns + PB - 1) / PB;
        pair_once_block<W, K, true>(A.x + 3 * (size_t)u.x, A.m + u.x, ns, A.eps2, M, u.z, 0, 1,
                                    0, M / 2 + 1, A.partial + u.w, tile, jacc);
    }
    if (threadIdx.x == 0) {
        // Every workgroup draws tickets until it fails once and only then
        // counts itself done, so the last one to count sees no more draws.
        if (atomicAdd(ctr + 1, 1) == (int)gridDim.x - 1) {
            atomicExch(ctr, 0);
            atomicExch(ctr + 1, 0);
        }
    }
}

// a, p of block I of system s = its slots (i-side, then the ring slots the
// block received), added in slot order.  One workgroup per unit.
template <int PB>
__global__ __launch_bounds__(256) void batched_sym_reduce_kernel(const int4 *__restrict__ units,
                                                                 const float4 *__restrict__ partial,
                                                                 float *a, float *p)
{
    const int4 u = units[blockIdx.x];
    const int ns = u.y;
    const int M = (ns + PB - 1) / PB;
    const int slots = 1 + ring_in(u.z, M);
    const float4 *P = partial + u.w;
    const int lo = u.z * PB;
    const int hi = min(ns, lo + PB);
    for (int j = lo + (int)threadIdx.x; j < hi; j += 256) {
        float4 s = P[j];
        for (int k = 1; k < slots; ++k) {
            const float4 q = P[(size_t)k * ns + j];
            s.x += q.x;
            s.y += q.y;
            s.z += q.z;
            s.w += q.w;
        }
        const size_t g = (size_t)u.x + j;
        a[3 * g + 0] = s.x;
        a[3 * g + 1] = s.y;
        a[3 * g + 2] = s.z;
        if (p) p[g] = s.w;
    }
}

using KernelFn = void (*)(BatArgs);
using SymKernelFn = void (*)(BatSymArgs);
using SymReduceFn = void (*)(const int4 *, const float4 *, float *, float *);
using SymDynKernelFn = void (*)(BatSymArgs, int *);

struct Variant {
    const char *name;
    int block, unroll;
    KernelFn fn;
    int sym_pb;          // particles per block of the pair-once variant (0: gather)
    SymKernelFn sym_fn;
    SymReduceFn sym_reduce;
    int sym_threads;
    SymDynKernelFn sym_dyn;  // dynamic-ticket pair-once kernel (sym_fn unused)
};

#define BAT_VARIANT(B, U) {"bat_b" #B "_u" #U, B, U, batched_kernel<B, U>, 0, nullptr, nullptr, 0, nullptr}
#define BAT_SYM_VARIANT(W, K) \
    {"bat_sym_w" #W "_k" #K, 0, 0, nullptr, W * 64 * K, batched_sym_kernel<W, K>, \
     batched_sym_reduce_kernel<W * 64 * K>, W * 64, nullptr}
#define BAT_SYMD_VARIANT(W, K) \
    {"bat_symd_w" #W "_k" #K, 0, 0, nullptr, W * 64 * K, batched_sym_kernel<W, K>, \
     batched_sym_reduce_kernel<W * 64 * K>, W * 64, batched_sym_dyn_kernel<W, K>}

const Variant kVariants[] = {
    BAT_VARIANT(64, 8),
    BAT_VARIANT(128, 8),
    BAT_VARIANT(256, 8),
    BAT_SYM_VARIANT(1, 4),
    BAT_SYM_VARIANT(1, 2),
    BAT_SYM_VARIANT(1, 3),
    BAT_SYM_VARIANT(2, 2),
    BAT_SYM_VARIANT(1, 8),
    BAT_SYM_VARIANT(2, 4),
    BAT_SYMD_VARIANT(1, 3),
    BAT_SYMD_VARIANT(1, 4),
    BAT_SYMD_VARIANT(1, 2),
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

// ---------------------------------------------------------------- plans

struct Plan {
    int device = -1;
    int variant = -1;
    std::vector<int64_t> offsets;  // exact key
    int num_units = 0;
    int grid = 0;
    size_t partial_elems = 0;      // float4 slots (pair-once variants)
    int4 *d_units = nullptr;
    ~Plan()
    {
        if (d_units) (void)hipFree(d_units);
    }
};

std::mutex g_plan_mu;
std::vector<std::shared_ptr<Plan>> g_plans;  // most recent last
constexpr size_t kMaxPlans = 8;

// While on (the variant timer), this thread's plans go to a private list
// instead of the shared cache: timing every variant then evicts no plan
// that a caller's captured graph may still read.
thread_local bool t_private_on = false;
thread_local std::vector<std::shared_ptr<Plan>> t_private_plans;

nbody_status build_plan(int variant, const Device &dev, const int64_t *offsets,
                        int64_t num_systems, hipStream_t stream, std::shared_ptr<Plan> *out)
{
    const Variant &V = kVariants[variant];
    std::lock_guard<std::mutex> lock(g_plan_mu);
    std::vector<std::shared_ptr<Plan>> &plans = t_private_on ? t_private_plans : g_plans;
    for (size_t k = 0; k < plans.size(); ++k) {
        Plan *pl = plans[k].get();
        if (pl->device == dev.id && pl->variant == variant &&
            pl->offsets.size() == (size_t)num_systems + 1 &&
            std::memcmp(pl->offsets.data(), offsets, sizeof(int64_t) * (num_systems + 1)) == 0) {
            // move to the back (most recently used)
            std::shared_ptr<Plan> keep = plans[k];
            plans.erase(plans.begin() + k);
            plans.push_back(keep);
            *out = keep;
            return NBODY_OK;
        }
    }
    auto plan = std::make_shared<Plan>();
    plan->device = dev.id;
    plan->variant = variant;
    plan->offsets.assign(offsets, offsets + num_systems + 1);

    struct Item {
        int64_t cost;
        int4 u;
    };
    std::vector<Item> items;
    if (V.sym_pb == 0) {
        for (int64_t s = 0; s < num_systems; ++s) {
            const int64_t lo = offsets[s], hi = offsets[s + 1];
            const int64_t ns = hi - lo;
            if (ns <= 0) continue;
            const int64_t padded_j = (ns + V.block - 1) / V.block * V.block;
            for (int64_t t = lo; t < hi; t += V.block)
                items.push_back(Item{padded_j, make_int4((int)t, (int)std::min<int64_t>(hi, t + V.block),
                                                         (int)lo, (int)hi)});
        }
    } else {
        // unit (system, block I); cost = the block's 64-particle tiles
        size_t poff = 0;
        for (int64_t s = 0; s < num_systems; ++s) {
            const int64_t lo = offsets[s], ns = offsets[s + 1] - offsets[s];
            if (ns <= 0) continue;
            const int M = (int)((ns + V.sym_pb - 1) / V.sym_pb);
            for (int I = 0; I < M; ++I) {
                const int64_t tiles = (int64_t)(1 + ring_len(I, M)) * (V.sym_pb / 64);
                items.push_back(Item{tiles, make_int4((int)lo, (int)ns, I, (int)poff)});
            }
            poff += (size_t)(1 + M / 2) * (size_t)ns;
        }
        plan->partial_elems = poff;
        if (poff > (size_t)INT32_MAX)
            return fail(NBODY_ERROR_INVALID_ARGUMENT,
                        "ensemble too large for the pair-once batched variant (%zu partial slots)", poff);
    }
    // largest first; ties keep system order
    std::stable_sort(items.begin(), items.end(),
                     [](const Item &p, const Item &q) { return p.cost > q.cost; });
    std::vector<int4> host(items.size());
    for (size_t k = 0; k < items.size(); ++k) host[k] = items[k].u;
    plan->num_units = (int)host.size();

    int per_cu = 0;
    hipError_t e = V.sym_dyn
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, V.sym_dyn, V.sym_threads, 0)
        : V.sym_pb
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, V.sym_fn, V.sym_threads, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, V.fn, V.block, 0);
    if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    if (per_cu < 1) per_cu = 1;
    int64_t grid = (int64_t)per_cu * dev.num_cu;
    if (grid > plan->num_units) grid = plan->num_units;
    plan->grid = (int)std::max<int64_t>(grid, 1);

    if (plan->num_units > 0) {
        if (fault_injected("alloc")) return fail(NBODY_ERROR_OUT_OF_MEMORY, "injected allocation fault");
        e = hipMalloc(&plan->d_units, sizeof(int4) * host.size());
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(batched plan)");
        e = hipMemcpyAsync(plan->d_units, host.data(), sizeof(int4) * host.size(),
                           hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(batched plan)");
        // The host vector dies with this scope: wait for the copy.
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(batched plan)");
    }
    if (!t_private_on && plans.size() >= kMaxPlans)
        plans.erase(plans.begin());  // hipFree syncs the device
    plans.push_back(plan);
    *out = plan;
    return NBODY_OK;
}

int variant_index(const char *name)
{
    for (int v = 0; v < kNumVariants; ++v)
        if (std::strcmp(kVariants[v].name, name) == 0) return v;
    return 0;
}

}  // namespace

int batched_variant_count() { return kNumVariants; }

const char *batched_variant_name(int index)
{
    return (index >= 0 && index < kNumVariants) ? kVariants[index].name : nullptr;
}

// Measured on MI355X (4,096 Plummer systems of 8..2048 particles): the
// pair-once variant with 256-particle blocks drawn from the ticket counter
// is fastest; very small systems gain nothing from pairing and take the
// gather variant.
int batched_default_variant(int64_t mean_n)
{
    static const int pair_once = variant_index("bat_symd_w1_k4");
    static const int gather = variant_index("bat_b64_u8");
    return mean_n >= 128 ? pair_once : gather;
}

void release_batched_plans()
{
    std::lock_guard<std::mutex> lock(g_plan_mu);
    g_plans.clear();
}

void begin_private_batched_plans() { t_private_on = true; }

void end_private_batched_plans()
{
    std::lock_guard<std::mutex> lock(g_plan_mu);
    t_private_on = false;
    t_private_plans.clear();  // hipFree in each plan's destructor syncs the device
}

nbody_status batched_run(int variant, const Device &dev, const int64_t *offsets,
                         int64_t num_systems, const float *x, const float *m, float eps2,
                         float *a, float *p, hipStream_t stream)
{
    std::shared_ptr<Plan> plan;
    nbody_status st = build_plan(variant, dev, offsets, num_systems, stream, &plan);
    if (st != NBODY_OK) return st;
    if (plan->num_units == 0) return NBODY_OK;
    const Variant &V = kVariants[variant];
    if (V.sym_pb) {
        void *ws = nullptr;
        st = workspace(dev, stream, sizeof(float4) * plan->partial_elems, &ws);
        if (st != NBODY_OK) return st;
        BatSymArgs S{plan->d_units, plan->num_units, x, m, eps2, static_cast<float4 *>(ws)};
        int *ctr = nullptr;
        if (V.sym_dyn) {
            st = counters(dev, stream, 2, &ctr);
            if (st != NBODY_OK) return st;
        }
        if (fault_injected("launch")) return fail(NBODY_ERROR_LAUNCH_FAILED, "injected launch fault");
        prof_mark(stream, 0);
        if (V.sym_dyn)
            hipLaunchKernelGGL(V.sym_dyn, dim3(plan->grid), dim3(V.sym_threads), 0, stream, S, ctr);
        else
            hipLaunchKernelGGL(V.sym_fn, dim3(plan->grid), dim3(V.sym_threads), 0, stream, S);
        prof_mark(stream, 1);
        st = check_launch(V.name);
        if (st != NBODY_OK) return st;
        hipLaunchKernelGGL(V.sym_reduce, dim3(plan->num_units), dim3(256), 0, stream,
                           (const int4 *)plan->d_units, (const float4 *)S.partial, a, p);
        return check_launch("batched_sym_reduce");
    }
    BatArgs P{plan->d_units, plan->num_units, x, m, eps2, a, p};
    if (fault_injected("launch")) return fail(NBODY_ERROR_LAUNCH_FAILED, "injected launch fault");
    prof_mark(stream, 0);
    hipLaunchKernelGGL(V.fn, dim3(plan->grid), dim3(V.block), 0, stream, P);
    prof_mark(stream, 1);
    return check_launch(V.name);
}

}  // namespace nbody
