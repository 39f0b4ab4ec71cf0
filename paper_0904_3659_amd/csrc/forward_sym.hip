// Forward evaluation of Eq. (gravity) (Sec. I) with every unordered pair
// computed once: the term of pair (i, j) gives m_j d r^3 to a_i and, by the
// antisymmetry of the softened force (one eps2 for all pairs), -m_i d r^3 to
// a_j; the potential term gives m_j r to p_i and m_i r to p_j.  That shares
// the difference, distance, rsqrt and r^3 of both ordered pairs, cutting the
// VALU issue cost per ordered pair by about a third.
//
// Blocks and the ring
//   Particles are cut into M blocks of P = W*64*K.  Workgroup (I, c) keeps
//   block I in VGPRs (K rows per lane, W waves) and meets
//     - its own block (the diagonal) as ordered pairs, i-side only, j == i
//       masked by index, and
//     - the blocks J = I + delta (mod M) for delta = 1..H_I (the ring), with
//       H_I = (M-1)/2, plus delta = M/2 when M is even and I < M/2,
//   so every unordered pair of distinct blocks is met exactly once.  The
//   ring and diagonal tiles of block I are shared among C chunks.
//
// j-tiles of 64 particles are staged in LDS.  On a ring tile, lane l at
// step s (0..63) meets particle (l + s) mod 64 of the tile: each step is a
// permutation of the 64 particles over the 64 lanes, so every lane owns a
// different per-wave LDS slot at every step.  A lane reads its slot at the
// start of the step and writes it back at the end; the next step's owner of
// that slot is another lane of the same wave, and one wave's LDS accesses
// complete in issue order, so the sums are exact read-modify-writes in a
// fixed order (no atomics; LDS atomics serialise and were 4x slower).  After
// the 64 steps the W waves' slots are added in wave order and written as the
// tile's partial.
//
// Partials (float4 per particle): slots 0..C-1 hold the i-side sums of the
// C chunks; slot C+delta-1 holds what particle j in block J received from
// block J - delta.  A second kernel adds, per particle, its slots in fixed
// order.  No atomics outside LDS, no cross-workgroup races: the result is
// bitwise reproducible for a given variant, n and chunk count.
//
// Padding: rows past n take position +1e18 and mass 0, tile slots past n
// take -1e18 and mass 0, so padded terms are exactly zero for finite
// positions below 1e17 in magnitude.
#include "common.hpp"

namespace nbody {
namespace {

constexpr float kPadRow = 1e18f;
constexpr float kPadCol = -1e18f;

struct SymArgs {
    const float *x;
    const float *m;
    int n;
    float eps2;
    int M;            // blocks
    int C;            // chunks per block
    float4 *partial;  // [C + M/2][n]
};

__device__ __forceinline__ int ring_len(int I, int M)
{
    return (M - 1) / 2 + (((M & 1) == 0 && I < M / 2) ? 1 : 0);
}

template <int W, int K>
__global__ __launch_bounds__(W * 64) void forward_sym_kernel(SymArgs A)
{
    constexpr int PB = W * 64 * K;   // particles per block
    constexpr int TPB = PB / 64;     // 64-particle tiles per block
    __shared__ float4 tile[64];
    __shared__ float4 jacc[W][64];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int n = A.n;
    const int M = A.M, C = A.C;
    const int I = blockIdx.x / C;
    const int c = blockIdx.x - I * C;
    const float eps2 = A.eps2;

    // ---- own rows
    float xi[K], yi[K], zi[K], mi[K];
    int ii[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = I * PB + wv * 64 * K + k * 64 + lane;
        ii[k] = i;
        if (i < n) {
            xi[k] = A.x[3 * i];
            yi[k] = A.x[3 * i + 1];
            zi[k] = A.x[3 * i + 2];
            mi[k] = A.m[i];
        } else {
            xi[k] = yi[k] = zi[k] = kPadRow;
            mi[k] = 0.0f;
        }
    }
    float ax[K], ay[K], az[K], ap[K];
#pragma unroll
    for (int k = 0; k < K; ++k) ax[k] = ay[k] = az[k] = ap[k] = 0.0f;

    for (int t = tid; t < W * 64; t += W * 64) (&jacc[0][0])[t] = make_float4(0.f, 0.f, 0.f, 0.f);

    // ---- this chunk's tiles: diagonal tiles t = c, c + C, ...; then ring
    // tiles q in [q0, q1) of the block's ring sequence (delta-major).
    const int ndiag = (TPB - c + C - 1) / C;
    const int Q = ring_len(I, M) * TPB;
    const int q0 = (int)((long long)Q * c / C);
    const int q1 = (int)((long long)Q * (c + 1) / C);
    const int ntiles = ndiag + (q1 - q0);

    for (int it = 0; it < ntiles; ++it) {
        int jbase, delta;
        if (it < ndiag) {
            delta = 0;
            jbase = I * PB + (c + it * C) * 64;
        } else {
            const int q = q0 + (it - ndiag);
            delta = 1 + q / TPB;
            const int t = q - (delta - 1) * TPB;
            int J = I + delta;
            if (J >= M) J -= M;
            jbase = J * PB + t * 64;
        }
        if (jbase >= n) continue;  // an all-padding tile adds nothing (uniform branch)

        __syncthreads();  // previous tile and its j-slot reduction are done
        if (tid < 64) {
            const int j = jbase + tid;
            tile[tid] = (j < n) ? make_float4(A.x[3 * j], A.x[3 * j + 1], A.x[3 * j + 2], A.m[j])
                                : make_float4(kPadCol, kPadCol, kPadCol, 0.0f);
        }
        __syncthreads();

        float tx[K], ty[K], tz[K], tp[K];
#pragma unroll
        for (int k = 0; k < K; ++k) tx[k] = ty[k] = tz[k] = tp[k] = 0.0f;

        if (delta == 0) {
            // diagonal: ordered pairs, i-side only, j == i removed by index
            for (int s = 0; s < 64; ++s) {
                const float4 q = tile[s];
                const int j = jbase + s;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    pair_term_masked(xi[k], yi[k], zi[k], q, eps2, j == ii[k], tx[k], ty[k],
                                     tz[k], tp[k]);
            }
        } else {
            float4 *slot = &jacc[wv][0];
            float4 q = tile[lane];
            for (int s = 0; s < 64; ++s) {
                const int jj = (lane + s) & 63;
                // Compiler-only barrier: this step's slot read stays after the
                // previous step's slot write (another lane may have written it).
                __asm__ volatile("" ::: "memory");
                float4 acc = slot[jj];
                const float4 qn = tile[(jj + 1) & 63];  // next step's particle (read-only tile)
                float gx, gy, gz, gp;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const float dx = xi[k] - q.x;
                    const float dy = yi[k] - q.y;
                    const float dz = zi[k] - q.z;
                    float s2 = __builtin_fmaf(dx, dx, eps2);
                    s2 = __builtin_fmaf(dy, dy, s2);
                    s2 = __builtin_fmaf(dz, dz, s2);
                    const float r = __builtin_amdgcn_rsqf(s2);
                    const float r3 = r * (r * r);
                    // i-side: + m_j r^3 d, + m_j r
                    const float f = q.w * r3;
                    tp[k] = __builtin_fmaf(q.w, r, tp[k]);
                    tx[k] = __builtin_fmaf(f, dx, tx[k]);
                    ty[k] = __builtin_fmaf(f, dy, ty[k]);
                    tz[k] = __builtin_fmaf(f, dz, tz[k]);
                    // j-side: - m_i r^3 d, + m_i r
                    const float g = mi[k] * r3;
                    if (k == 0) {
                        gx = -g * dx;
                        gy = -g * dy;
                        gz = -g * dz;
                        gp = mi[k] * r;
                    } else {
                        gx = __builtin_fmaf(-g, dx, gx);
                        gy = __builtin_fmaf(-g, dy, gy);
                        gz = __builtin_fmaf(-g, dz, gz);
                        gp = __builtin_fmaf(mi[k], r, gp);
                    }
                }
                acc.x += gx;
                acc.y += gy;
                acc.z += gz;
                acc.w += gp;
                slot[jj] = acc;
                q = qn;
            }
            __asm__ volatile("" ::: "memory");
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            ax[k] += tx[k];
            ay[k] += ty[k];
            az[k] += tz[k];
            ap[k] += tp[k];
        }
        if (delta != 0) {
            __syncthreads();  // every wave's j-side slots are complete
            if (tid < 64) {
                float4 s = jacc[0][tid];
                jacc[0][tid] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                for (int w2 = 1; w2 < W; ++w2) {
                    const float4 v = jacc[w2][tid];
                    s.x += v.x;
                    s.y += v.y;
                    s.z += v.z;
                    s.w += v.w;
                    jacc[w2][tid] = make_float4(0.f, 0.f, 0.f, 0.f);
                }
                const int j = jbase + tid;
                if (j < n) A.partial[(size_t)(C + delta - 1) * n + j] = s;
            }
        }
    }

#pragma unroll
    for (int k = 0; k < K; ++k)
        if (ii[k] < n) A.partial[(size_t)c * n + ii[k]] = make_float4(ax[k], ay[k], az[k], ap[k]);
}

// a_j, p_j = i-side chunk slots + the j-side slots the particle's block
// received, added in slot order.
template <int PB>
__global__ __launch_bounds__(256) void forward_sym_reduce_kernel(const float4 *__restrict__ partial,
                                                                 int n, int M, int C, float *a,
                                                                 float *p)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const int J = j / PB;
    const int H = (M - 1) / 2 + (((M & 1) == 0 && J >= M / 2) ? 1 : 0);
    float4 s = partial[j];
    for (int k = 1; k < C + H; ++k) {
        const float4 q = partial[(size_t)k * n + j];
        s.x += q.x;
        s.y += q.y;
        s.z += q.z;
        s.w += q.w;
    }
    a[3 * j + 0] = s.x;
    a[3 * j + 1] = s.y;
    a[3 * j + 2] = s.z;
    if (p) p[j] = s.w;
}

template <int W, int K>
nbody_status run_sym(const char *name, const Device &dev, const float *x, const float *m, int n,
                     float eps2, float *a, float *p, hipStream_t stream)
{
    constexpr int PB = W * 64 * K;
    const int M = (n + PB - 1) / PB;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, forward_sym_kernel<W, K>,
                                                                W * 64, 0);
    if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    if (per_cu < 1) per_cu = 1;
    const int resident = per_cu * dev.num_cu;
    // chunks: fill the device once; never more chunks than tiles to share
    int C = resident / M;
    if (C < 1) C = 1;
    const int max_c = (M / 2 + 1) * (PB / 64);
    if (C > max_c) C = max_c;
    const int slots = C + M / 2;
    void *ws = nullptr;
    nbody_status st = workspace(dev, stream, sizeof(float4) * (size_t)slots * n, &ws);
    if (st != NBODY_OK) return st;
    SymArgs A{x, m, n, eps2, M, C, static_cast<float4 *>(ws)};
    if (fault_injected("launch")) return fail(NBODY_ERROR_LAUNCH_FAILED, "injected launch fault");
    hipLaunchKernelGGL((forward_sym_kernel<W, K>), dim3(M * C), dim3(W * 64), 0, stream, A);
    st = check_launch(name);
    if (st != NBODY_OK) return st;
    hipLaunchKernelGGL((forward_sym_reduce_kernel<PB>), dim3((n + 255) / 256), dim3(256), 0, stream,
                       A.partial, n, M, C, a, p);
    return check_launch("forward_sym_reduce");
}

}  // namespace

nbody_status forward_sym_run(int W, int K, const char *name, const Device &dev, const float *x,
                             const float *m, int n, float eps2, float *a, float *p,
                             hipStream_t stream)
{
    if (W == 4 && K == 8) return run_sym<4, 8>(name, dev, x, m, n, eps2, a, p, stream);
    if (W == 2 && K == 8) return run_sym<2, 8>(name, dev, x, m, n, eps2, a, p, stream);
    if (W == 1 && K == 8) return run_sym<1, 8>(name, dev, x, m, n, eps2, a, p, stream);
    if (W == 8 && K == 4) return run_sym<8, 4>(name, dev, x, m, n, eps2, a, p, stream);
    if (W == 2 && K == 16) return run_sym<2, 16>(name, dev, x, m, n, eps2, a, p, stream);
    return fail(NBODY_ERROR_INTERNAL, "no symmetric forward kernel for W=%d K=%d", W, K);
}

}  // namespace nbody
