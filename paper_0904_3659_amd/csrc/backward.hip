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

using KernelFn = void (*)(BwdArgs);

struct Variant {
    const char *name;
    int block, k, unroll;
    KernelFn direct, partial;
};

#define BWD_VARIANT(B, K, U) \
    {"bwd_b" #B "_k" #K "_u" #U, B, K, U, backward_kernel<B, K, U, false>, backward_kernel<B, K, U, true>}

const Variant kVariants[] = {
    BWD_VARIANT(256, 2, 4),
    BWD_VARIANT(256, 1, 8),
    BWD_VARIANT(128, 1, 8),
    BWD_VARIANT(64, 1, 4),
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

}  // namespace

int backward_variant_count() { return kNumVariants; }

const char *backward_variant_name(int index)
{
    return (index >= 0 && index < kNumVariants) ? kVariants[index].name : nullptr;
}

int backward_default_variant(int64_t n)
{
    if (n >= (1 << 15)) return 0;
    if (n >= (1 << 12)) return 1;
    if (n >= (1 << 10)) return 2;
    return 3;
}

nbody_status backward_run(int variant, const Device &dev, const float *x, const float *m, int n,
                          float eps2, const float *ga, const float *gp, float *gx, float *gm,
                          hipStream_t stream)
{
    const Variant &V = kVariants[variant];
    const int iblk = V.block * V.k;
    const int iblocks = (n + iblk - 1) / iblk;
    const int target = 4 * dev.num_cu;
    const int max_splits = (n + V.block - 1) / V.block;
    int splits = (target + iblocks - 1) / iblocks;
    splits = splits < 1 ? 1 : (splits > max_splits ? max_splits : splits);
    int chunk = (n + splits - 1) / splits;
    chunk = (chunk + V.block - 1) / V.block * V.block;
    splits = (n + chunk - 1) / chunk;

    BwdArgs P{x, m, ga, gp, n, eps2, chunk, nullptr, gx, gm};
    if (splits == 1) {
        if (fault_injected("launch")) return fail(NBODY_ERROR_LAUNCH_FAILED, "injected launch fault");
        hipLaunchKernelGGL(V.direct, dim3(iblocks, 1), dim3(V.block), 0, stream, P);
        return check_launch(V.name);
    }
    void *ws = nullptr;
    nbody_status st = workspace(dev, stream, sizeof(float4) * (size_t)splits * n, &ws);
    if (st != NBODY_OK) return st;
    P.partial = static_cast<float4 *>(ws);
    if (fault_injected("launch")) return fail(NBODY_ERROR_LAUNCH_FAILED, "injected launch fault");
    hipLaunchKernelGGL(V.partial, dim3(iblocks, splits), dim3(V.block), 0, stream, P);
    st = check_launch(V.name);
    if (st != NBODY_OK) return st;
    hipLaunchKernelGGL(backward_reduce_kernel, dim3((n + 255) / 256), dim3(256), 0, stream,
                       P.partial, splits, n, gx, gm);
    return check_launch("backward_reduce");
}

}  // namespace nbody
