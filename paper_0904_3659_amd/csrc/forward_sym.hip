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
    float4 *partial;  // [C + M/2][n]
};

template <int W, int K, bool POT>
__global__ __launch_bounds__(W * 64) void forward_sym_kernel(SymArgs A)
{
    __shared__ float4 tile[kTileLds];
    __shared__ float4 jacc[W][kSlotLds];
    const int I = blockIdx.x / A.C;
    const int c = blockIdx.x - I * A.C;
    pair_once_block<W, K, false, POT>(A.x, A.m, A.n, A.eps2, A.M, I, c, A.C, A.partial, tile, jacc);
}

// OCC divides the chunk count: 1 fills every resident workgroup slot once;
// 2 gives half as many, twice as long workgroups (fewer partial slots, less
// tail imbalance at small n, lower occupancy).
template <int W, int K, int OCC>
nbody_status run_sym(const char *name, const Device &dev, const float *x, const float *m, int n,
                     float eps2, float *a, float *p, hipStream_t stream, const LfEpi *epi,
                     bool *fused)
{
    constexpr int PB = W * 64 * K;
    const int M = (n + PB - 1) / PB;
    int per_cu = 0;
    // sized by the kernel that forms the potential, also when p is not
    // stored: the same chunking keeps a bitwise the same either way
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, forward_sym_kernel<W, K, true>, W * 64, 0);
    if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    if (per_cu < 1) per_cu = 1;
    const int resident = per_cu * dev.num_cu;
    // chunks: fill the device once; never more chunks than tiles to share
    int C = resident / (M * OCC);
    if (C < 1) C = 1;
    const int max_c = (M / 2 + 1) * (PB / 64);
    if (C > max_c) C = max_c;
    const int slots = C + M / 2;
    void *ws = nullptr;
    nbody_status st = workspace(dev, stream, sizeof(float4) * (size_t)slots * n, &ws);
    if (st != NBODY_OK) return st;
    SymArgs A{x, m, n, eps2, M, C, static_cast<float4 *>(ws)};
    if (fault_injected("launch")) return fail(NBODY_ERROR_LAUNCH_FAILED, "injected launch fault");
    prof_mark(stream, 0);
    if (p)
        hipLaunchKernelGGL((forward_sym_kernel<W, K, true>), dim3(M * C), dim3(W * 64), 0, stream, A);
    else
        hipLaunchKernelGGL((forward_sym_kernel<W, K, false>), dim3(M * C), dim3(W * 64), 0, stream,
                           A);
    prof_mark(stream, 1);
    st = check_launch(name);
    if (st != NBODY_OK) return st;
    if (epi && epi->mode != kLfNone) {
        hipLaunchKernelGGL((slot_reduce_kernel<PB, true>), dim3((n + 63) / 64), dim3(256), 0,
                           stream, A.partial, n, M, C, a, p, *epi);
        if (fused) *fused = true;
    } else {
        hipLaunchKernelGGL((slot_reduce_kernel<PB>), dim3((n + 63) / 64), dim3(256), 0, stream,
                           A.partial, n, M, C, a, p, LfEpi{});
    }
    return check_launch("slot_reduce");
}

}  // namespace

nbody_status forward_sym_run(int W, int K, int occ, const char *name, const Device &dev,
                             const float *x, const float *m, int n, float eps2, float *a, float *p,
                             hipStream_t stream, const LfEpi *epi, bool *fused)
{
    if (W == 8 && K == 4 && occ == 1) return run_sym<8, 4, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused);
    if (W == 8 && K == 4 && occ == 2) return run_sym<8, 4, 2>(name, dev, x, m, n, eps2, a, p, stream, epi, fused);
    if (W == 4 && K == 8 && occ == 1) return run_sym<4, 8, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused);
    if (W == 4 && K == 4 && occ == 1) return run_sym<4, 4, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused);
    if (W == 2 && K == 8 && occ == 1) return run_sym<2, 8, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused);
    if (W == 16 && K == 4 && occ == 1) return run_sym<16, 4, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused);
    if (W == 2 && K == 4 && occ == 1) return run_sym<2, 4, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused);
    if (W == 1 && K == 4 && occ == 1) return run_sym<1, 4, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused);
    if (W == 1 && K == 2 && occ == 1) return run_sym<1, 2, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused);
    if (W == 2 && K == 2 && occ == 1) return run_sym<2, 2, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused);
    if (W == 4 && K == 2 && occ == 1) return run_sym<4, 2, 1>(name, dev, x, m, n, eps2, a, p, stream, epi, fused);
    return fail(NBODY_ERROR_INTERNAL, "no pair-once forward kernel for W=%d K=%d occ=%d", W, K, occ);
}

}  // namespace nbody
