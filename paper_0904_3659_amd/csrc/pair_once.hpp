// The pair-once block evaluation of Eq. (gravity) (Sec. I), shared by the
// single-system forward kernel (forward_sym.hip) and the batched ensemble
// kernel (batched.hip).
//
// Every unordered pair is computed once: the term of pair (i, j) gives
// m_j d r^3 to a_i and, by the antisymmetry of the softened force (one eps2
// for all pairs), -m_i d r^3 to a_j; the potential term gives m_j r to p_i
// and m_i r to p_j.  That shares the difference, distance, rsqrt and r^3 of
// both ordered pairs.
//
// Blocks and the ring
//   A system of n particles is cut into M blocks of P = W*64*K.  The caller
//   (one workgroup) owns block I, chunk c of C: it keeps block I in VGPRs
//   (K rows per lane, W waves) and meets
//     - its own block (the diagonal) as ordered pairs, i-side only, j == i
//       removed by index, and
//     - the blocks J = I + delta (mod M) for delta = 1..H_I (the ring), with
//       H_I = (M-1)/2, plus delta = M/2 when M is even and I < M/2,
//   so every unordered pair of distinct blocks is met exactly once.  The
//   block's tile sequence (diagonal tiles, then ring tiles delta-major) is
//   shared evenly among the C chunks.
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
// Partials (float4 per particle, [C + M/2][n]): slots 0..C-1 hold the i-side
// sums of the C chunks; slot C+delta-1 holds what particle j in block J
// received from block J - delta.  A second pass adds, per particle, its
// slots in fixed order.  No atomics, no cross-workgroup races: the result is
// bitwise reproducible for a given variant, n and chunk count.
//
// Padding: rows past n take position +1e18 and mass 0, tile slots past n
// take -1e18 and mass 0, so padded terms are exactly zero for finite
// positions below 1e17 in magnitude.
#pragma once

#include "common.hpp"

namespace nbody {

constexpr float kPadRow = 1e18f;
constexpr float kPadCol = -1e18f;

__host__ __device__ __forceinline__ int ring_len(int I, int M)
{
    return (M - 1) / 2 + (((M & 1) == 0 && I < M / 2) ? 1 : 0);
}

// Number of j-side slots block J of an M-block system receives.
__host__ __device__ __forceinline__ int ring_in(int J, int M)
{
    return (M - 1) / 2 + (((M & 1) == 0 && J >= M / 2) ? 1 : 0);
}

// One workgroup of W*64 lanes evaluates chunk c of block I.  x, m and
// partial are the system's own arrays (offsets already applied).  tile and
// jacc are the workgroup's LDS buffers.  Starts with a workgroup barrier, so
// the LDS buffers may be reused by consecutive calls.
template <int W, int K>
__device__ __forceinline__ void pair_once_block(const float *__restrict__ x,
                                                const float *__restrict__ m, int n, float eps2,
                                                int M, int I, int c, int C, float4 *partial,
                                                float4 *tile, float4 (*jacc)[64])
{
    constexpr int PB = W * 64 * K;   // particles per block
    constexpr int TPB = PB / 64;     // 64-particle tiles per block
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;

    // ---- own rows
    float xi[K], yi[K], zi[K], mi[K];
    int ii[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = I * PB + wv * 64 * K + k * 64 + lane;
        ii[k] = i;
        if (i < n) {
            xi[k] = x[3 * i];
            yi[k] = x[3 * i + 1];
            zi[k] = x[3 * i + 2];
            mi[k] = m[i];
        } else {
            xi[k] = yi[k] = zi[k] = kPadRow;
            mi[k] = 0.0f;
        }
    }
    float ax[K], ay[K], az[K], ap[K];
#pragma unroll
    for (int k = 0; k < K; ++k) ax[k] = ay[k] = az[k] = ap[k] = 0.0f;

    __syncthreads();  // LDS buffers are free (callers may loop over blocks)
    for (int t = tid; t < W * 64; t += W * 64) (&jacc[0][0])[t] = make_float4(0.f, 0.f, 0.f, 0.f);

    // ---- this chunk's tiles: the block's TPB diagonal tiles followed by its
    // ring tiles (delta-major), shared evenly among the C chunks.
    const int U = TPB + ring_len(I, M) * TPB;
    const int u0 = (int)((long long)U * c / C);
    const int u1 = (int)((long long)U * (c + 1) / C);

    for (int u = u0; u < u1; ++u) {
        int jbase, delta;
        if (u < TPB) {
            delta = 0;
            jbase = I * PB + u * 64;
        } else {
            const int q = u - TPB;
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
            tile[tid] = (j < n) ? make_float4(x[3 * j], x[3 * j + 1], x[3 * j + 2], m[j])
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
                if (j < n) partial[(size_t)(C + delta - 1) * n + j] = s;
            }
        }
    }

#pragma unroll
    for (int k = 0; k < K; ++k)
        if (ii[k] < n) partial[(size_t)c * n + ii[k]] = make_float4(ax[k], ay[k], az[k], ap[k]);
}


}  // namespace nbody
