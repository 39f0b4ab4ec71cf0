// Backward (vector-Jacobian product) of Eq. (gravity) (Sec. I), float32 on
// gfx950.  For upstream weights w = dL/da and v = dL/dp the gradient of
// L = sum_i w_i . a_i + v_i p_i, gathered per output row k over j != k with
// d = x_k - x_j, r = (|d|^2 + eps2)^(-1/2), is
//     dL/dx_k = sum_j r^3 c_kj - r^3 (3 r^2 (c_kj . d) + b_kj) d,
//     dL/dm_k = sum_j r v_j - r^3 (w_j . d),
// with c_kj = m_j w_k - m_k w_j and b_kj = m_j v_k + m_k v_j.  The first
// sum is split as
//     sum_j r^3 c_kj = w_k A_k - m_k B_k,  A_k = sum_j m_j r^3,
//                                          B_k = sum_j r^3 w_j,
// so that the per-pair work is about 30 VALU operations and one v_rsq_f32.
//
// Decomposition as in the forward kernel: K rows per lane in VGPRs, j-tiles
// of BLOCK particles staged in LDS as two float4 per particle, (x, y, z, m)
// and (w_x, w_y, w_z, v); j-splits with a fixed-order reduction when the
// row count alone cannot fill the device; per-tile partial sums folded into
// the running sums (two-level accumulation).  No atomics.
#include "common.hpp"
#include "pair_once.hpp"
#include "wave_sum.hpp"

#include <cstring>

namespace nbody {
namespace {

struct BwdArgs {
    const float *x;
    const float *m;
    const float *ga;  // [n][3] or NULL
    const float *gp;  // [n] or NULL
    int n;
    float eps2;
    int chunk;
    float4 *partial;  // [splits][n] (dL/dx, dL/dm) per split when PARTIAL
    float *gx;
    float *gm;
};

struct RowAcc {
    float A, Bx, By, Bz, Cx, Cy, Cz, G;
};

__device__ __forceinline__ void adj_term(float xk, float yk, float zk, float mk, float wkx,
                                         float wky, float wkz, float vk, float4 q, float4 wq,
                                         float eps2, bool skip, RowAcc &t)
{
    const float dx = xk - q.x;
    const float dy = yk - q.y;
    const float dz = zk - q.z;
    float s = __builtin_fmaf(dx, dx, eps2);
    s = __builtin_fmaf(dy, dy, s);
    s = __builtin_fmaf(dz, dz, s);
    const float r = skip ? 0.0f : __builtin_amdgcn_rsqf(s);
    const float r2 = r * r;
    const float r3 = r * r2;
    // A += m_j r^3 ; B += r^3 w_j
    t.A = __builtin_fmaf(q.w, r3, t.A);
    t.Bx = __builtin_fmaf(r3, wq.x, t.Bx);
    t.By = __builtin_fmaf(r3, wq.y, t.By);
    t.Bz = __builtin_fmaf(r3, wq.z, t.Bz);
    // c . d = m_j (w_k . d) - m_k (w_j . d)
    float wkd = wkx * dx;
    wkd = __builtin_fmaf(wky, dy, wkd);
    wkd = __builtin_fmaf(wkz, dz, wkd);
    float wjd = wq.x * dx;
    wjd = __builtin_fmaf(wq.y, dy, wjd);
    wjd = __builtin_fmaf(wq.z, dz, wjd);
    const float cd = __builtin_fmaf(q.w, wkd, -mk * wjd);
    // b = m_j v_k + m_k v_j
    const float b = __builtin_fmaf(mk, wq.w, q.w * vk);
    // u = r^3 (3 r^2 (c . d) + b) ; C += u d
    const float u = r3 * __builtin_fmaf(3.0f * r2, cd, b);
    t.Cx = __builtin_fmaf(u, dx, t.Cx);
    t.Cy = __builtin_fmaf(u, dy, t.Cy);
    t.Cz = __builtin_fmaf(u, dz, t.Cz);
    // dL/dm_k += r v_j - r^3 (w_j . d)
    t.G = __builtin_fmaf(r, wq.w, t.G);
    t.G = __builtin_fmaf(-r3, wjd, t.G);
}

__device__ __forceinline__ void fold(RowAcc &acc, const RowAcc &t)
{
    acc.A += t.A;
    acc.Bx += t.Bx;
    acc.By += t.By;
    acc.Bz += t.Bz;
    acc.Cx += t.Cx;
    acc.Cy += t.Cy;
    acc.Cz += t.Cz;
    acc.G += t.G;
}

__device__ __forceinline__ void zero(RowAcc &t) { t.A = t.Bx = t.By = t.Bz = t.Cx = t.Cy = t.Cz = t.G = 0.0f; }

__device__ __forceinline__ float4 load_xm(const BwdArgs &P, int j)
{
    return make_float4(P.x[3 * j], P.x[3 * j + 1], P.x[3 * j + 2], P.m[j]);
}

__device__ __forceinline__ float4 load_wv(const BwdArgs &P, int j)
{
    float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
    if (P.ga) {
        r.x = P.ga[3 * j];
        r.y = P.ga[3 * j + 1];
        r.z = P.ga[3 * j + 2];
    }
    if (P.gp) r.w = P.gp[j];
    return r;
}

template <int BLOCK, int K, int U, bool PARTIAL>
__global__ __launch_bounds__(BLOCK) void backward_kernel(BwdArgs P)
{
    constexpr int TILE = BLOCK;
    __shared__ float4 tile_xm[TILE];
    __shared__ float4 tile_wv[TILE];

    const int tid = threadIdx.x;
    const int n = P.n;
    const int i0 = blockIdx.x * (BLOCK * K);
    const int jbeg = blockIdx.y * P.chunk;
    const int jend = min(n, jbeg + P.chunk);
    const float eps2 = P.eps2;

    float4 xk[K], wk[K];
    int kk[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = i0 + k * BLOCK + tid;
        kk[k] = i;
        const int ic = i < n ? i : n - 1;
        xk[k] = load_xm(P, ic);
        wk[k] = load_wv(P, ic);
    }
    RowAcc acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) zero(acc[k]);

    float4 nxm = make_float4(0.f, 0.f, 0.f, 0.f), nwv = nxm;
    if (jbeg + tid < jend) {
        nxm = load_xm(P, jbeg + tid);
        nwv = load_wv(P, jbeg + tid);
    }

    const int iblk_end = i0 + BLOCK * K;
    for (int t0 = jbeg; t0 < jend; t0 += TILE) {
        __syncthreads();
        tile_xm[tid] = nxm;
        tile_wv[tid] = nwv;
        __syncthreads();
        {
            const int j = t0 + TILE + tid;
            nxm = make_float4(0.f, 0.f, 0.f, 0.f);
            nwv = nxm;
            if (j < jend) {
                nxm = load_xm(P, j);
                nwv = load_wv(P, j);
            }
        }
        RowAcc t[K];
#pragma unroll
        for (int k = 0; k < K; ++k) zero(t[k]);

        const int cnt = min(TILE, jend - t0);
        const bool masked = (cnt < TILE) || (t0 < iblk_end && t0 + TILE > i0);
        if (!masked) {
            for (int jj = 0; jj < TILE; jj += U) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const float4 q = tile_xm[jj + u];
                    const float4 wq = tile_wv[jj + u];
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        adj_term(xk[k].x, xk[k].y, xk[k].z, xk[k].w, wk[k].x, wk[k].y, wk[k].z,
                                 wk[k].w, q, wq, eps2, false, t[k]);
                }
            }
        } else {
            for (int jj = 0; jj < cnt; ++jj) {
                const float4 q = tile_xm[jj];
                const float4 wq = tile_wv[jj];
                const int j = t0 + jj;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    adj_term(xk[k].x, xk[k].y, xk[k].z, xk[k].w, wk[k].x, wk[k].y, wk[k].z,
                             wk[k].w, q, wq, eps2, j == kk[k], t[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) fold(acc[k], t[k]);
    }

#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = kk[k];
        if (i >= n) continue;
        // dL/dx_k = w_k A - m_k B - C
        const RowAcc &c = acc[k];
        const float gx = wk[k].x * c.A - xk[k].w * c.Bx - c.Cx;
        const float gy = wk[k].y * c.A - xk[k].w * c.By - c.Cy;
        const float gz = wk[k].z * c.A - xk[k].w * c.Bz - c.Cz;
        if (PARTIAL) {
            P.partial[(size_t)blockIdx.y * n + i] = make_float4(gx, gy, gz, c.G);
        } else {
            P.gx[3 * i + 0] = gx;
            P.gx[3 * i + 1] = gy;
            P.gx[3 * i + 2] = gz;
            if (P.gm) P.gm[i] = c.G;
        }
    }
}

// Row-per-wave adjoint for the smallest n, where launch latency and the
// longest dependent chain set the time: wave w owns rows [K w, K w + K)
// (the same for every lane), lane l gathers j = l, l + 64, ... into each
// row's sums A, B, C, G, and a fixed butterfly adds the 64 lane sums
// (bitwise reproducible).  One launch, no LDS, no partials.
template <int K>
__global__ __launch_bounds__(256) void backward_row_kernel(BwdArgs P)
{
    const int n = P.n;
    const float eps2 = P.eps2;
    const int lane = threadIdx.x & 63;
    const int i0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6))) * K;
    if (i0 >= n) return;  // the whole wave: no barrier follows
    float4 xk[K], wk[K];
    RowAcc acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int ic = min(i0 + k, n - 1);  // rows past n are computed, not stored
        xk[k] = load_xm(P, ic);
        wk[k] = load_wv(P, ic);
        zero(acc[k]);
    }
#pragma unroll 2
    for (int j = lane; j < n; j += 64) {
        const float4 q = load_xm(P, j);
        const float4 wq = load_wv(P, j);
#pragma unroll
        for (int k = 0; k < K; ++k)
            adj_term(xk[k].x, xk[k].y, xk[k].z, xk[k].w, wk[k].x, wk[k].y, wk[k].z, wk[k].w, q,
                     wq, eps2, j == i0 + k, acc[k]);
    }
    float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        RowAcc c = acc[k];
        c.A = wave_sum(c.A);
        c.Bx = wave_sum(c.Bx);
        c.By = wave_sum(c.By);
        c.Bz = wave_sum(c.Bz);
        c.Cx = wave_sum(c.Cx);
        c.Cy = wave_sum(c.Cy);
        c.Cz = wave_sum(c.Cz);
        c.G = wave_sum(c.G);
        // dL/dx_k = w_k A - m_k B - C
        const float4 g = make_float4(wk[k].x * c.A - xk[k].w * c.Bx - c.Cx,
                                     wk[k].y * c.A - xk[k].w * c.By - c.Cy,
                                     wk[k].z * c.A - xk[k].w * c.Bz - c.Cz, c.G);
        if (lane == k) out = g;  // lane k stores row i0 + k
    }
    const int i = i0 + lane;
    if (lane < K && i < n) {
        P.gx[3 * i + 0] = out.x;
        P.gx[3 * i + 1] = out.y;
        P.gx[3 * i + 2] = out.z;
        if (P.gm) P.gm[i] = out.w;
    }
}

__global__ __launch_bounds__(256) void backward_reduce_kernel(const float4 *__restrict__ partial,
                                                              int splits, int n, float *gx,
                                                              float *gm)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float4 s = partial[i];
    for (int k = 1; k < splits; ++k) {
        const float4 q = partial[(size_t)k * n + i];
        s.x += q.x;
        s.y += q.y;
        s.z += q.z;
        s.w += q.w;
    }
    gx[3 * i + 0] = s.x;
    gx[3 * i + 1] = s.y;
    gx[3 * i + 2] = s.z;
    if (gm) gm[i] = s.w;
}

// ---------------------------------------------------------------------------
// Pair-once adjoint.  With d = x_k - x_j, c_kj = m_j w_k - m_k w_j and
// b_kj = m_j v_k + m_k v_j, the x-gradient term
//     F(k, j) = r^3 c_kj - r^3 (3 r^2 (c_kj . d) + b_kj) d
// satisfies F(j, k) = -F(k, j) (c and d flip sign, b and c.d do not), so one
// evaluation serves both rows: dL/dx_k += F, dL/dx_j -= F.  The mass terms
//     dL/dm_k += r v_j - r^3 (w_j . d),   dL/dm_j += r v_k + r^3 (w_k . d)
// share r, r^3 and the two dot products.  The block/ring decomposition, LDS
// slot read-modify-writes and partial slots are those of the pair-once
// forward kernel (pair_once.hpp), diagonal tiles included; tiles hold two
// float4 per particle.

struct SymBwdArgs {
    const float *x;
    const float *m;
    const float *ga;
    const float *gp;
    int n;
    float eps2;
    int M;
    int C;
    int d_lo, d_hi;   // ring deltas of this launch's group
    float4 *partial;  // [C + G][n]: (dL/dx, dL/dm)
};

// One unordered pair: adds F and the k mass term to tk; returns the j-side
// contributions (-F, j mass term) through jx..jm.
__device__ __forceinline__ void adj_pair_once(const float4 &xk, const float4 &wk, const float4 &q,
                                              const float4 &wq, float eps2, float4 &tk, float &jx,
                                              float &jy, float &jz, float &jm)
{
    const float dx = xk.x - q.x;
    const float dy = xk.y - q.y;
    const float dz = xk.z - q.z;
    float s = __builtin_fmaf(dx, dx, eps2);
    s = __builtin_fmaf(dy, dy, s);
    s = __builtin_fmaf(dz, dz, s);
    const float r = __builtin_amdgcn_rsqf(s);
    const float r2 = r * r;
    const float r3 = r * r2;
    float wkd = wk.x * dx;
    wkd = __builtin_fmaf(wk.y, dy, wkd);
    wkd = __builtin_fmaf(wk.z, dz, wkd);
    float wjd = wq.x * dx;
    wjd = __builtin_fmaf(wq.y, dy, wjd);
    wjd = __builtin_fmaf(wq.z, dz, wjd);
    const float cd = __builtin_fmaf(q.w, wkd, -xk.w * wjd);
    const float b = __builtin_fmaf(xk.w, wq.w, q.w * wk.w);
    // F = r^3 (c - t d) with t = 3 r^2 (c . d) + b
    const float t = __builtin_fmaf(3.0f * r2, cd, b);
    const float cx = __builtin_fmaf(q.w, wk.x, -xk.w * wq.x);
    const float cy = __builtin_fmaf(q.w, wk.y, -xk.w * wq.y);
    const float cz = __builtin_fmaf(q.w, wk.z, -xk.w * wq.z);
    const float Fx = r3 * __builtin_fmaf(-t, dx, cx);
    const float Fy = r3 * __builtin_fmaf(-t, dy, cy);
    const float Fz = r3 * __builtin_fmaf(-t, dz, cz);
    tk.x += Fx;
    tk.y += Fy;
    tk.z += Fz;
    tk.w = __builtin_fmaf(r, wq.w, tk.w);
    tk.w = __builtin_fmaf(-r3, wjd, tk.w);
    jx = -Fx;
    jy = -Fy;
    jz = -Fz;
    jm = __builtin_fmaf(r3, wkd, r * wk.w);
}

// adj_pair_once for ring tiles, with the j-side added straight into the
// slot value ja: F = r^3 u with u = c - t d enters both sides as one FMA per
// component (r^3 u to tk, -r^3 u to ja), and the j mass term likewise.
template <bool HAS_V = true>
__device__ __forceinline__ void adj_pair_fold(const float4 &xk, const float4 &wk, const float4 &q,
                                              const float4 &wq, float eps2, float4 &tk, float4 &ja)
{
    const float dx = xk.x - q.x;
    const float dy = xk.y - q.y;
    const float dz = xk.z - q.z;
    float s = __builtin_fmaf(dx, dx, eps2);
    s = __builtin_fmaf(dy, dy, s);
    s = __builtin_fmaf(dz, dz, s);
    const float r = __builtin_amdgcn_rsqf(s);
    const float r2 = r * r;
    const float r3 = r * r2;
    float wkd = wk.x * dx;
    wkd = __builtin_fmaf(wk.y, dy, wkd);
    wkd = __builtin_fmaf(wk.z, dz, wkd);
    float wjd = wq.x * dx;
    wjd = __builtin_fmaf(wq.y, dy, wjd);
    wjd = __builtin_fmaf(wq.z, dz, wjd);
    const float cd = __builtin_fmaf(q.w, wkd, -xk.w * wjd);
    // without potential weights (v = 0) b vanishes and t = 3 r^2 (c . d)
    // exactly as the fused form with a zero addend
    const float t = HAS_V ? __builtin_fmaf(3.0f * r2, cd, __builtin_fmaf(xk.w, wq.w, q.w * wk.w))
                          : (3.0f * r2) * cd;
    const float ux = __builtin_fmaf(-t, dx, __builtin_fmaf(q.w, wk.x, -xk.w * wq.x));
    const float uy = __builtin_fmaf(-t, dy, __builtin_fmaf(q.w, wk.y, -xk.w * wq.y));
    const float uz = __builtin_fmaf(-t, dz, __builtin_fmaf(q.w, wk.z, -xk.w * wq.z));
    tk.x = __builtin_fmaf(r3, ux, tk.x);
    tk.y = __builtin_fmaf(r3, uy, tk.y);
    tk.z = __builtin_fmaf(r3, uz, tk.z);
    if (HAS_V) tk.w = __builtin_fmaf(r, wq.w, tk.w);
    tk.w = __builtin_fmaf(-r3, wjd, tk.w);
    ja.x = __builtin_fmaf(-r3, ux, ja.x);
    ja.y = __builtin_fmaf(-r3, uy, ja.y);
    ja.z = __builtin_fmaf(-r3, uz, ja.z);
    ja.w = __builtin_fmaf(r3, wkd, ja.w);
    if (HAS_V) ja.w = __builtin_fmaf(r, wk.w, ja.w);
}

// The k-side alone, with the pair removed when `skip` holds (diagonal tiles).
__device__ __forceinline__ void adj_row_term(const float4 &xk, const float4 &wk, const float4 &q,
                                             const float4 &wq, float eps2, bool skip, float4 &tk)
{
    const float dx = xk.x - q.x;
    const float dy = xk.y - q.y;
    const float dz = xk.z - q.z;
    float s = __builtin_fmaf(dx, dx, eps2);
    s = __builtin_fmaf(dy, dy, s);
    s = __builtin_fmaf(dz, dz, s);
    const float r = skip ? 0.0f : __builtin_amdgcn_rsqf(s);
    const float r2 = r * r;
    const float r3 = r * r2;
    float wkd = wk.x * dx;
    wkd = __builtin_fmaf(wk.y, dy, wkd);
    wkd = __builtin_fmaf(wk.z, dz, wkd);
    float wjd = wq.x * dx;
    wjd = __builtin_fmaf(wq.y, dy, wjd);
    wjd = __builtin_fmaf(wq.z, dz, wjd);
    const float cd = __builtin_fmaf(q.w, wkd, -xk.w * wjd);
    const float b = __builtin_fmaf(xk.w, wq.w, q.w * wk.w);
    const float t = __builtin_fmaf(3.0f * r2, cd, b);
    tk.x = __builtin_fmaf(r3, __builtin_fmaf(-t, dx, __builtin_fmaf(q.w, wk.x, -xk.w * wq.x)), tk.x);
    tk.y = __builtin_fmaf(r3, __builtin_fmaf(-t, dy, __builtin_fmaf(q.w, wk.y, -xk.w * wq.y)), tk.y);
    tk.z = __builtin_fmaf(r3, __builtin_fmaf(-t, dz, __builtin_fmaf(q.w, wk.z, -xk.w * wq.z)), tk.z);
    tk.w = __builtin_fmaf(r, wq.w, tk.w);
    tk.w = __builtin_fmaf(-r3, wjd, tk.w);
}

constexpr float kBwdPadRow = 1e18f;
constexpr float kBwdPadCol = -1e18f;

__device__ __forceinline__ void load_xw(const SymBwdArgs &A, int j, float4 &xm, float4 &wv)
{
    if (j < A.n) {
        xm = make_float4(A.x[3 * j], A.x[3 * j + 1], A.x[3 * j + 2], A.m[j]);
        wv = make_float4(A.ga ? A.ga[3 * j] : 0.f, A.ga ? A.ga[3 * j + 1] : 0.f,
                         A.ga ? A.ga[3 * j + 2] : 0.f, A.gp ? A.gp[j] : 0.f);
    } else {
        xm = make_float4(kBwdPadCol, kBwdPadCol, kBwdPadCol, 0.f);
        wv = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// Steps s0 .. s0 + NS - 1 of one tile for one wave (lane l meets tile
// particle (l + s) mod 64 at step s).  Ring tiles: every row tile pair-once.
// Diagonal tile t: row tile a = a0 + k pair-once if a < t, masked ordered
// pairs if a == t, nothing if a > t (met on diagonal tile a).
template <int K, bool DIAG, int NS = 64>
__device__ __forceinline__ void adj_tile_steps(const float4 (&xk)[K], const float4 (&wk)[K],
                                               const int (&kk)[K], const float4 *tile_xm,
                                               const float4 *tile_wv, float4 *slot, int lane,
                                               int a0, int t, int jbase, int s0, float eps2,
                                               float4 (&tk)[K])
{
    const bool any_once = !DIAG || a0 < t;
    float4 q = tile_xm[(lane + s0) & 63];
    float4 wq = tile_wv[(lane + s0) & 63];
    for (int s = s0; s < s0 + NS; ++s) {
        const int jj = (lane + s) & 63;
        // keep this step's slot read after the previous step's write
        __asm__ volatile("" ::: "memory");
        float4 ja = make_float4(0.f, 0.f, 0.f, 0.f);
        if (any_once) ja = slot[jj];
        const float4 qn = tile_xm[(jj + 1) & 63];
        const float4 wqn = tile_wv[(jj + 1) & 63];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!DIAG || a0 + k < t) {
                float jx, jy, jz, jm;
                adj_pair_once(xk[k], wk[k], q, wq, eps2, tk[k], jx, jy, jz, jm);
                ja.x += jx;
                ja.y += jy;
                ja.z += jz;
                ja.w += jm;
            } else if (a0 + k == t) {
                adj_row_term(xk[k], wk[k], q, wq, eps2, jbase + jj == kk[k], tk[k]);
            }
        }
        if (any_once) slot[jj] = ja;
        q = qn;
        wq = wqn;
    }
}

// Ring tiles: the tiles are staged twice (entries e and e + 64 hold
// particle e) and the wave's j-side slots number 128, so lane l at step s
// reads entry l + s and updates slot l + s with no index wrap (immediate
// LDS offsets in the unrolled loop); particle e's j-side sum is slot e plus
// slot e + 64, folded into slot e at the end.  Same scheme and ordering
// argument as the forward pair-once kernel.  The wave takes steps
// s0 .. s0 + NS - 1 (all 64 unless a tile's steps are split between waves;
// s0 + NS <= 64 keeps every entry and slot below 128).
template <int K, bool HAS_V = true, int NS = 64>
__device__ __forceinline__ void adj_ring_steps(const float4 (&xk)[K], const float4 (&wk)[K],
                                               const float4 *tile_xm, const float4 *tile_wv,
                                               float4 *slot, int lane, int s0, float eps2,
                                               float4 (&tk)[K])
{
    const float4 *txm = tile_xm + lane + s0;
    const float4 *twv = tile_wv + lane + s0;
    float4 *sl = slot + lane + s0;
    float4 q = txm[0];
    float4 wq = twv[0];
#pragma unroll 4
    for (int s = 0; s < NS; ++s) {
        // keep this step's slot read after the previous step's write
        __asm__ volatile("" ::: "memory");
        float4 ja = sl[s];
        const float4 qn = txm[s + 1];
        const float4 wqn = twv[s + 1];
#pragma unroll
        for (int k = 0; k < K; ++k) adj_pair_fold<HAS_V>(xk[k], wk[k], q, wq, eps2, tk[k], ja);
        sl[s] = ja;
        q = qn;
        wq = wqn;
    }
    __asm__ volatile("" ::: "memory");
    const float4 lo = slot[lane];
    const float4 hi = slot[lane + 64];
    slot[lane] = make_float4(lo.x + hi.x, lo.y + hi.y, lo.z + hi.z, lo.w + hi.w);
}

// HAS_V false: no potential weights (grad_p NULL); their terms are not
// formed on ring tiles (bitwise the same result as v = 0).
// S = 1: each wave owns K * 64 of the block's rows.  S = W > 1: the W waves
// share the block's K * 64 rows and each takes 64 / W of every tile's steps
// (workgroups W times shorter for the same block size, so the grid's drain
// is shorter); their row sums are added in wave order at the end.
template <int W, int K, bool HAS_V, int S = 1>
__global__ __launch_bounds__(W * 64) void backward_sym_kernel(SymBwdArgs A)
{
    static_assert(S == 1 || (S == W && K <= 2), "a step split spans all waves, two rows at most");
    constexpr int PB = (S > 1 ? 64 : W * 64) * K;
    constexpr int TPB = PB / 64;
    constexpr int NS = 64 / S;
    __shared__ float4 tile_xm[128];
    __shared__ float4 tile_wv[128];
    __shared__ float4 jacc[W][128];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int n = A.n;
    const int M = A.M, C = A.C;
    const int I = blockIdx.x / C;
    const int c = blockIdx.x - I * C;
    const float eps2 = A.eps2;
    const int wrow = S > 1 ? 0 : wv;      // this wave's row group
    const int s0 = S > 1 ? wv * NS : 0;   // and first step of each tile

    float4 xk[K], wk[K], acc[K];
    int kk[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = I * PB + wrow * 64 * K + k * 64 + lane;
        kk[k] = i;
        if (i < n) {
            load_xw(A, i, xk[k], wk[k]);
        } else {
            xk[k] = make_float4(kBwdPadRow, kBwdPadRow, kBwdPadRow, 0.f);
            wk[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        acc[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    }

    // this chunk's share of the block's tiles in the launch's ring group
    // (diagonal first, then the ring delta-major); all-padding tiles are
    // skipped (uniform)
    const int d_lo = A.d_lo;
    const int dj = group_first_delta(d_lo);
    const int U = group_tiles(I, M, d_lo, A.d_hi, TPB);
    const int u0 = (int)((long long)U * c / C);
    const int u1 = (int)((long long)U * (c + 1) / C);
    int u = u0, delta = 0, jbase = 0;
    for (; u < u1; ++u)
        if ((jbase = tile_base<PB>(u, I, M, d_lo, delta)) < n) break;
    float4 nxm = make_float4(0.f, 0.f, 0.f, 0.f), nwv = nxm;
    if (u < u1 && tid < 64) load_xw(A, jbase + tid, nxm, nwv);

    while (u < u1) {
        __syncthreads();  // the previous tile and its slot sums are done
        if (tid < 64) {
            tile_xm[tid] = nxm;
            tile_wv[tid] = nwv;
            tile_xm[tid + 64] = nxm;
            tile_wv[tid + 64] = nwv;
        }
        jacc[wv][lane] = make_float4(0.f, 0.f, 0.f, 0.f);
        jacc[wv][lane + 64] = make_float4(0.f, 0.f, 0.f, 0.f);
        __syncthreads();
        const int cur_u = u, cur_delta = delta, cur_base = jbase;
        for (++u; u < u1; ++u)
            if ((jbase = tile_base<PB>(u, I, M, d_lo, delta)) < n) break;
        if (u < u1 && tid < 64) load_xw(A, jbase + tid, nxm, nwv);

        float4 tk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) tk[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        float4 *slot = &jacc[wv][0];
        const bool diag = (cur_delta == 0);
        if (!diag)
            adj_ring_steps<K, HAS_V, NS>(xk, wk, tile_xm, tile_wv, slot, lane, s0, eps2, tk);
        else
            adj_tile_steps<K, true, NS>(xk, wk, kk, tile_xm, tile_wv, slot, lane, wrow * K,
                                        cur_u, cur_base, s0, eps2, tk);
        __asm__ volatile("" ::: "memory");
#pragma unroll
        for (int k = 0; k < K; ++k) {
            acc[k].x += tk[k].x;
            acc[k].y += tk[k].y;
            acc[k].z += tk[k].z;
            acc[k].w += tk[k].w;
        }
        __syncthreads();  // every wave's j-side slots are complete
        if (!diag) {
            if (tid < 64) {
                float4 sum = jacc[0][tid];
#pragma unroll
                for (int w2 = 1; w2 < W; ++w2) {
                    const float4 v = jacc[w2][tid];
                    sum.x += v.x;
                    sum.y += v.y;
                    sum.z += v.z;
                    sum.w += v.w;
                }
                const int j = cur_base + tid;
                if (j < n) A.partial[(size_t)(C + cur_delta - dj) * n + j] = sum;
            }
        } else if (wv == (S > 1 ? 0 : cur_u / K)) {
            // this wave holds diagonal tile cur_u's rows (lane-slot cur_u % K;
            // with a step split every wave does, and wave 0 adds); the
            // diagonal steps use slots 0..63 only
            float4 sum = jacc[0][lane];
#pragma unroll
            for (int w2 = 1; w2 < W; ++w2) {
                const float4 v = jacc[w2][lane];
                sum.x += v.x;
                sum.y += v.y;
                sum.z += v.z;
                sum.w += v.w;
            }
            const int kt = cur_u - wrow * K;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (k == kt) {
                    acc[k].x += sum.x;
                    acc[k].y += sum.y;
                    acc[k].z += sum.z;
                    acc[k].w += sum.w;
                }
        }
    }
    if (S > 1) {
        // the waves' row sums, added in wave order by wave 0 (through the
        // j-side slots, which the last tile's reads are done with)
        __syncthreads();
        if (wv > 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) jacc[wv][k * 64 + lane] = acc[k];
        }
        __syncthreads();
        if (wv > 0) return;
#pragma unroll
        for (int w2 = 1; w2 < W; ++w2)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float4 v = jacc[w2][k * 64 + lane];
                acc[k].x += v.x;
                acc[k].y += v.y;
                acc[k].z += v.z;
                acc[k].w += v.w;
            }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (kk[k] < n) A.partial[(size_t)c * n + kk[k]] = acc[k];
}

// OCC divides the chunk count and ROUNDS multiplies it (as in the
// pair-once forward kernel); S splits each tile's steps between the waves.
template <int W, int K, int OCC, int ROUNDS = 1, int S = 1>
nbody_status run_backward_sym(const char *name, const Device &dev, const float *x, const float *m,
                              int n, float eps2, const float *ga, const float *gp, float *gx,
                              float *gm, hipStream_t stream, const LfEpi *epi, bool *fused,
                              const Arena &arena)
{
    constexpr int PB = (S > 1 ? 64 : W * 64) * K;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, backward_sym_kernel<W, K, true, S>, W * 64, 0);
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
        SymBwdArgs A{x, m, ga, gp, n, eps2, pl.M, pl.C, 0, 0, partial};
        sym_group(pl, g, &A.d_lo, &A.d_hi);
        prof_mark(stream, 0);
        if (gp)
            hipLaunchKernelGGL((backward_sym_kernel<W, K, true, S>), dim3(pl.M * pl.C),
                               dim3(W * 64), 0, stream, A);
        else
            hipLaunchKernelGGL((backward_sym_kernel<W, K, false, S>), dim3(pl.M * pl.C),
                               dim3(W * 64), 0, stream, A);
        prof_mark(stream, 1);
        st = check_launch(name);
        if (st != NBODY_OK) return st;
        const int first = g == 0, last = g == pl.groups - 1;
        if (last && lf)
            hipLaunchKernelGGL((slot_fold_kernel<PB, true>), dim3((n + 63) / 64), dim3(256), 0,
                               stream, partial, n, pl.M, pl.C, A.d_lo, A.d_hi, first, last, acc, gx,
                               gm, *epi);
        else
            hipLaunchKernelGGL((slot_fold_kernel<PB>), dim3((n + 63) / 64), dim3(256), 0, stream,
                               partial, n, pl.M, pl.C, A.d_lo, A.d_hi, first, last, acc, gx, gm,
                               LfEpi{});
        st = check_launch("slot_fold");
        if (st != NBODY_OK) return st;
    }
    if (lf && fused) *fused = true;
    return NBODY_OK;
}

using KernelFn = void (*)(BwdArgs);

using SymRunFn = nbody_status (*)(const char *, const Device &, const float *, const float *,
                                  int, float, const float *, const float *, float *, float *,
                                  hipStream_t, const LfEpi *, bool *, const Arena &);

using SymKernelFn = void (*)(SymBwdArgs);

// A gather variant (rows own all j) or, with sym set, a pair-once variant
// with W waves, K rows per lane and chunk divisor O.
struct Variant {
    const char *name;
    int block, k, unroll;
    KernelFn direct, partial;
    SymRunFn sym;
    SymKernelFn sym_kernel;
    int sym_w, sym_k, sym_occ, sym_rounds;
    KernelFn row;  // row-per-wave kernel (K = row_k rows per wave)
    int row_k;
    int sym_split;  // pair-once: waves sharing a block's rows (0 or 1: none)
};

// Particles per pair-once block of a variant.
int sym_block(const Variant &V)
{
    return V.sym_w * 64 * V.sym_k / (V.sym_split > 1 ? V.sym_split : 1);
}

#define BWD_VARIANT(B, K, U) \
    {"bwd_b" #B "_k" #K "_u" #U, B, K, U, backward_kernel<B, K, U, false>, backward_kernel<B, K, U, true>, nullptr, nullptr, 0, 0, 0, 1}
#define BWD_SYM_VARIANT(W, K, O) \
    {"bwd_sym_w" #W "_k" #K "_o" #O, 0, 0, 0, nullptr, nullptr, run_backward_sym<W, K, O>, \
     backward_sym_kernel<W, K, true>, W, K, O, 1}
// Pair-once blocks in R rounds of workgroups (R times the chunks).
#define BWD_SYM_R_VARIANT(W, K, R) \
    {"bwd_sym_w" #W "_k" #K "_r" #R, 0, 0, 0, nullptr, nullptr, run_backward_sym<W, K, 1, R>, \
     backward_sym_kernel<W, K, true>, W, K, 1, R}

// Pair-once blocks of K * 64 rows whose W waves split each tile's steps, in
// R rounds of workgroups.
#define BWD_SYM_S_VARIANT(W, K, R) \
    {"bwd_sym_s" #W "_k" #K "_r" #R, 0, 0, 0, nullptr, nullptr, run_backward_sym<W, K, 1, R, W>, \
     backward_sym_kernel<W, K, true, W>, W, K, 1, R, nullptr, 0, W}

#define BWD_ROW_VARIANT(K) \
    {"bwd_row_k" #K, 64, K, 0, nullptr, nullptr, nullptr, nullptr, 0, 0, 0, 1, backward_row_kernel<K>, K}

const Variant kVariants[] = {
    BWD_VARIANT(256, 2, 4),
    BWD_VARIANT(256, 1, 8),
    BWD_VARIANT(128, 1, 8),
    BWD_VARIANT(64, 1, 4),
    BWD_VARIANT(64, 1, 8),
    BWD_VARIANT(64, 2, 4),
    BWD_SYM_VARIANT(8, 2, 1),
    BWD_SYM_VARIANT(8, 2, 2),
    BWD_SYM_VARIANT(4, 2, 1),
    BWD_SYM_VARIANT(4, 2, 2),
    BWD_SYM_VARIANT(8, 4, 1),
    BWD_SYM_VARIANT(16, 2, 1),
    BWD_SYM_VARIANT(4, 1, 1),
    BWD_SYM_VARIANT(2, 2, 1),
    BWD_SYM_VARIANT(2, 4, 1),
    BWD_SYM_VARIANT(1, 2, 1),
    BWD_SYM_VARIANT(2, 1, 1),
    BWD_SYM_VARIANT(1, 4, 1),
    BWD_SYM_R_VARIANT(1, 2, 8),
    BWD_SYM_R_VARIANT(2, 2, 8),
    BWD_SYM_R_VARIANT(2, 1, 8),
    BWD_SYM_R_VARIANT(8, 2, 8),
    BWD_SYM_R_VARIANT(4, 2, 8),
    BWD_ROW_VARIANT(1),
    BWD_ROW_VARIANT(2),
    BWD_SYM_S_VARIANT(2, 2, 8),
    BWD_SYM_S_VARIANT(2, 2, 16),
    BWD_SYM_R_VARIANT(1, 2, 16),
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

}  // namespace

int backward_variant_count() { return kNumVariants; }

const char *backward_variant_name(int index)
{
    return (index >= 0 && index < kNumVariants) ? kVariants[index].name : nullptr;
}

static int variant_index(const char *name)
{
    for (int v = 0; v < kNumVariants; ++v)
        if (std::strcmp(kVariants[v].name, name) == 0) return v;
    return 0;
}

// Measured on MI355X: the pair-once adjoint wins from about 4,000 particles
// on, one wave per row below; its workspace is bounded as the forward's (ring
// groups), and above 2^24 particles the gather kernel takes over.  The same
// choice serves calls with and without potential weights.
int backward_default_variant(int64_t n)
{
    static const int pair_once_big = variant_index("bwd_sym_w8_k2_r8");
    static const int pair_once_large = variant_index("bwd_sym_w4_k2_r8");
    static const int pair_once_r8 = variant_index("bwd_sym_w1_k2_r8");
    static const int pair_once_r16 = variant_index("bwd_sym_w1_k2_r16");
    static const int pair_once_split = variant_index("bwd_sym_s2_k2_r8");
    static const int gather = variant_index("bwd_b256_k1_u8");
    static const int row_1 = variant_index("bwd_row_k1");
    static const int row_2 = variant_index("bwd_row_k2");
    if (n > (1 << 24)) return gather;
    // Eight rounds of workgroups (each block's tiles cut into eight times as
    // many chunks as the device holds workgroups, down to one tile; the
    // dispatcher hands the short ones out as slots free up) lead from 4,000
    // bodies up in forced-variant sweeps on one box (whole calls, with and
    // without potential weights): blocks of 128 rows whose two waves split
    // each tile's steps up to 12,000 (4-6% ahead of the two-row row kernel
    // at 4,000, level with it at 3,500; 5-10% ahead of one round of two-wave
    // one-row blocks from 4,500 to 5,600; 2-7% ahead of one-wave two-row and
    // two-wave one-row blocks in eight rounds from 7,000 to 10,000, level at
    // 6,000 and 12,000), then one-wave two-row blocks (4-9% ahead of one round up to
    // 2^17), in sixteen rounds from 24,000 to 29,999 (one tile per chunk
    // where eight rounds mix chunks of one and two tiles: 4% ahead at
    // 24,576, 1% at 28,000, behind at 22,000 and 32,768), 4-wave blocks
    // from 40,000 (10-13% ahead of one round of two-wave blocks with
    // potential weights at 49,152 and 60,000, 9-11% of 8-wave ones at 2^17)
    // and 8-wave blocks from 2^18 (3-7% ahead of one round of them at 2^18
    // and 2^19).
    if (n >= (1 << 18)) return pair_once_big;
    if (n >= 40000) return pair_once_large;
    if (n >= 24000 && n < 30000) return pair_once_r16;
    if (n >= 12000) return pair_once_r8;
    if (n >= 4000) return pair_once_split;
    // one wave per row below 4,000 bodies (two rows from 3,500): 4.7 against
    // 16.1 us per call at 1,024 (split gather and its reduction), 13.3-14.4
    // against 21.5-22.0 at 1,500 (pair-once and its fold)
    return n >= 3500 ? row_2 : row_1;
}

// Geometry of the row gather: j-splits and j per split.
static void bwd_gather_geometry(const Variant &V, int n, int num_cu, int *splits_out,
                                int *chunk_out)
{
    const int iblk = V.block * V.k;
    const int iblocks = (n + iblk - 1) / iblk;
    const int target = 4 * num_cu;
    const int max_splits = (n + V.block - 1) / V.block;
    int splits = (target + iblocks - 1) / iblocks;
    splits = splits < 1 ? 1 : (splits > max_splits ? max_splits : splits);
    int chunk = (n + splits - 1) / splits;
    chunk = (chunk + V.block - 1) / V.block * V.block;
    *splits_out = (n + chunk - 1) / chunk;
    *chunk_out = chunk;
}

int64_t backward_plan_bytes(int variant, int64_t n, int num_cu, int per_cu)
{
    if (variant < 0 || variant >= kNumVariants || n < 0 || n > NBODY_MAX_N || num_cu < 1 ||
        per_cu < 1)
        return -1;
    if (n == 0) return 0;
    const Variant &V = kVariants[variant];
    if (V.row) return 0;
    if (V.sym) {
        SymPlan pl;
        if (!sym_plan(n, sym_block(V), (int64_t)per_cu * num_cu * V.sym_rounds, V.sym_occ,
                      sym_workspace_budget(n), &pl))
            return -1;
        return (int64_t)pl.bytes();
    }
    int splits = 1, chunk = 0;
    bwd_gather_geometry(V, (int)n, num_cu, &splits, &chunk);
    return splits > 1 ? (int64_t)sizeof(float4) * splits * n : 0;
}

int64_t backward_variant_max_n(int variant)
{
    if (variant < 0 || variant >= kNumVariants) return -1;
    // the row-per-wave kernels are built for launch-latency-bound sizes
    return kVariants[variant].row ? (1 << 16) : NBODY_MAX_N;
}

nbody_status backward_variant_occupancy(int variant, int *per_cu)
{
    const Variant &V = kVariants[variant];
    const hipError_t e =
        V.sym   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, V.sym_kernel, V.sym_w * 64, 0)
        : V.row ? hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, V.row, 256, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, V.partial, V.block, 0);
    if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    if (*per_cu < 1) *per_cu = 1;
    return NBODY_OK;
}

nbody_status backward_run(int variant, const Device &dev, const float *x, const float *m, int n,
                          float eps2, const float *ga, const float *gp, float *gx, float *gm,
                          hipStream_t stream, const LfEpi *epi, bool *fused, const Arena &arena)
{
    const Variant &V = kVariants[variant];
    if (fused) *fused = false;
    if (V.sym) return V.sym(V.name, dev, x, m, n, eps2, ga, gp, gx, gm, stream, epi, fused, arena);
    if (V.row) {
        const int64_t waves = ((int64_t)n + V.row_k - 1) / V.row_k;
        BwdArgs P{x, m, ga, gp, n, eps2, 0, nullptr, gx, gm};
        if (fault_injected("launch")) return fail(NBODY_ERROR_LAUNCH_FAILED, "injected launch fault");
        prof_mark(stream, 0);
        hipLaunchKernelGGL(V.row, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, stream, P);
        prof_mark(stream, 1);
        return check_launch(V.name);
    }
    const int iblk = V.block * V.k;
    const int iblocks = (n + iblk - 1) / iblk;
    int splits = 1, chunk = 0;
    bwd_gather_geometry(V, n, dev.num_cu, &splits, &chunk);

    BwdArgs P{x, m, ga, gp, n, eps2, chunk, nullptr, gx, gm};
    if (splits == 1) {
        if (fault_injected("launch")) return fail(NBODY_ERROR_LAUNCH_FAILED, "injected launch fault");
        prof_mark(stream, 0);
        hipLaunchKernelGGL(V.direct, dim3(iblocks, 1), dim3(V.block), 0, stream, P);
        prof_mark(stream, 1);
        return check_launch(V.name);
    }
    void *ws = nullptr;
    nbody_status st = arena.get(dev, stream, sizeof(float4) * (size_t)splits * n, &ws);
    if (st != NBODY_OK) return st;
    P.partial = static_cast<float4 *>(ws);
    if (fault_injected("launch")) return fail(NBODY_ERROR_LAUNCH_FAILED, "injected launch fault");
    prof_mark(stream, 0);
    hipLaunchKernelGGL(V.partial, dim3(iblocks, splits), dim3(V.block), 0, stream, P);
    prof_mark(stream, 1);
    st = check_launch(V.name);
    if (st != NBODY_OK) return st;
    hipLaunchKernelGGL(backward_reduce_kernel, dim3((n + 255) / 256), dim3(256), 0, stream,
                       P.partial, splits, n, gx, gm);
    return check_launch("backward_reduce");
}

}  // namespace nbody
