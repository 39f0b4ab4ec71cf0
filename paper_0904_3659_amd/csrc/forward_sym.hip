// Forward evaluation of Eq. (gravity) (Sec. I) with every unordered pair
// computed once (see pair_once.hpp for the block/ring decomposition, the
// LDS slot sums and the partial layout).  Grid: one workgroup per (block I,
// chunk c); a second kernel adds each particle's partial slots.
#include "pair_once.hpp"

namespace nbody {
namespace {

struct SymArgs {
    const float *x;
    const float *m;
    int n;
    float eps2;
    int M;            // blocks
    int C;            // chunks per block
    int d_lo, d_hi;   // ring deltas of this launch's group
    float4 *partial;  // [C + G][n]
};

template <int W, int K, bool POT>
__global__ __launch_bounds__(W * 64) void forward_sym_kernel(SymArgs A)
{
    __shared__ float4 tile[kTileLds];
    __shared__ float4 jacc[W][kSlotLds];
    const int I = blockIdx.x / A.C;
    const int c = blockIdx.x - I * A.C;
    pair_once_block<W, K, false, POT>(A.x, A.m, A.n, A.eps2, A.M, I, c, A.C, A.d_lo, A.d_hi,
                                      A.partial, tile, jacc);
}

// OCC divides the chunk count: 1 fills every resident workgroup slot once;
// 2 gives half as many, twice as long workgroups (fewer partial slots, less
// tail imbalance at small n, lower occupancy).  ROUNDS multiplies it: that
// many rounds of shorter workgroups (down to one tile each), which the
// hardware dispatcher hands out as slots free up, evening out the tail of
// a grid whose workgroups hold only a few tiles.
template <int W, int K, int OCC, int ROUNDS = 1>
nbody_status run_sym(const char *name, const Device &dev, const float *x, const float *m, int n,
                     float eps2, float *a, float *p, hipStream_t stream, const LfEpi *epi,
                     bool *fused, const Arena &arena)
{
    constexpr int PB = W * 64 * K;
    int per_cu = 0;
    // sized by the kernel that forms the potential, also when p is not
    // stored: the same plan keeps a bitwise the same either way
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, forward_sym_kernel<W, K, true>, W * 64, 0);
    if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    if (per_cu < 1) per_cu = 1;
    SymPlan pl;
    if (!sym_plan(n, PB, (int64_t)per_cu * dev.num_cu * ROUNDS, OCC,
                  arena.budget(sym_workspace_budget(n)), &pl))
        return fail(NBODY_ERROR_INVALID_ARGUMENT,
                    "n = %d needs more than the %zu-byte workspace limit of %s", n,
                    arena.budget(sym_workspace_budget(n)), name);
    void *ws = nullptr;
    nbody_status st = arena.get(dev, stream, pl.bytes(), &ws);
    if (st != NBODY_OK) return st;
    float4 *partial = static_cast<float4 *>(ws);
    double4 *acc = pl.acc_bytes ? reinterpret_cast<double4 *>(static_cast<char *>(ws) + pl.partial_bytes)
                                : nullptr;
    if (fault_injected("launch")) return fail(NBODY_ERROR_LAUNCH_FAILED, "injected launch fault");
    const bool lf = epi && epi->mode != kLfNone;
    for (int g = 0; g < pl.groups; ++g) {
        SymArgs A{x, m, n, eps2, pl.M, pl.C, 0, 0, partial};
        sym_group(pl, g, &A.d_lo, &A.d_hi);
        prof_mark(stream, 0);
        if (p)
            hipLaunchKernelGGL((forward_sym_kernel<W, K, true>), dim3(pl.M * pl.C), dim3(W * 64), 0,
                               stream, A);
        else
            hipLaunchKernelGGL((forward_sym_kernel<W, K, false>), dim3(pl.M * pl.C), dim3(W * 64),
                               0, stream, A);
        prof_mark(stream, 1);
        st = check_launch(name);
        if (st != NBODY_OK) return st;
        const int first = g == 0, last = g == pl.groups - 1;
        if (last && lf)
            hipLaunchKernelGGL((slot_fold_kernel<PB, true>), dim3((n + 63) / 64), dim3(256), 0,
                               stream, partial, n, pl.M, pl.C, A.d_lo, A.d_hi, first, last, acc, a,
                               p, *epi);
        else
            hipLaunchKernelGGL((slot_fold_kernel<PB>), dim3((n + 63) / 64), dim3(256), 0, stream,
                               partial, n, pl.M, pl.C, A.d_lo, A.d_hi, first, last, acc, a, p,
                               LfEpi{});
        st = check_launch("slot_fold");
        if (st != NBODY_OK) return st;
    }
    if (lf && fused) *fused = true;
    return NBODY_OK;
}

template <int W, int K>
nbody_status sym_occupancy(int *per_cu)
{
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        per_cu, forward_sym_kernel<W, K, true>, W * 64, 0);
    if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    if (*per_cu < 1) *per_cu = 1;
    return NBODY_OK;
}

}  // namespace

nbody_status forward_sym_occupancy(int W, int K, int *per_cu)
{
    if (W == 8 && K == 4) return sym_occupancy<8, 4>(per_cu);
    if (W == 4 && K == 8) return sym_occupancy<4, 8>(per_cu);
    if (W == 4 && K == 4) return sym_occupancy<4, 4>(per_cu);
    if (W == 2 && K == 8) return sym_occupancy<2, 8>(per_cu);
    if (W == 16 && K == 4) return sym_occupancy<16, 4>(per_cu);
    if (W == 2 && K == 4) return sym_occupancy<2, 4>(per_cu);
    if (W == 1 && K == 4) return sym_occupancy<1, 4>(per_cu);
    if (W == 1 && K == 2) return sym_occupancy<1, 2>(per_cu);
    if (W == 2 && K == 2) return sym_occupancy<2, 2>(per_cu);
    if (W == 4 && K == 2) return sym_occupancy<4, 2>(per_cu);
    return fail(NBODY_ERROR_INTERNAL, "no pair-once forward kernel for W=%d K=%d", W, K);
}

nbody_status forward_sym_run(int W, int K, int occ, int rounds, const char *name,
                             const Device &dev, const float *x, const float *m, int n, float eps2,
                             float *a, float *p, hipStream_t stream, const LfEpi *epi, bool *fused,
                             const Arena &arena)
{
    if (rounds == 8) {
        if (W == 1 && K == 4 && occ == 1) return run_sym<1, 4, 1, 8>(name, dev, x, m, n, eps2, a, p, stream, epi, fused, arena);
        if (W == 1 && K == 2 && occ == 1) return run_sym<1, 2, 1, 8>(name, dev, x, m, n, eps2, a, p, stream, epi, fused, arena);
        if (W == 4 && K == 4 && occ == 1) return run_sym<4, 4, 1, 8>(name, dev, x, m, n, eps2, a, p, stream, epi, fused, arena);
        if (W == 8 && K == 4 && occ == 1) return run_sym<8, 4, 1, 8>(name, dev, x, m, n, eps2, a, p, stream, epi, fused, arena);
        return fail(NBODY_ERROR_INTERNAL, "no pair-once forward kernel for W=%d K=%d occ=%d rounds=%d", W, K, occ, rounds);
    }
    if (W == 8 && K == 4 && occ == 1) return run_sym<8, 4, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused, arena);
    if (W == 8 && K == 4 && occ == 2) return run_sym<8, 4, 2>(name, dev, x, m, n, eps2, a, p, stream, epi, fused, arena);
    if (W == 4 && K == 8 && occ == 1) return run_sym<4, 8, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused, arena);
    if (W == 4 && K == 4 && occ == 1) return run_sym<4, 4, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused, arena);
    if (W == 2 && K == 8 && occ == 1) return run_sym<2, 8, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused, arena);
    if (W == 16 && K == 4 && occ == 1) return run_sym<16, 4, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused, arena);
    if (W == 2 && K == 4 && occ == 1) return run_sym<2, 4, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused, arena);
    if (W == 1 && K == 4 && occ == 1) return run_sym<1, 4, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused, arena);
    if (W == 1 && K == 2 && occ == 1) return run_sym<1, 2, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused, arena);
    if (W == 2 && K == 2 && occ == 1) return run_sym<2, 2, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused, arena);
    if (W == 4 && K == 2 && occ == 1) return run_sym<4, 2, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused, arena);
    return fail(NBODY_ERROR_INTERNAL, "no pair-once forward kernel for W=%d K=%d occ=%d", W, K, occ);
}

}  // namespace nbody
