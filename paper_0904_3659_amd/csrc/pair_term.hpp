// Device form of one term of Eq. (gravity) (Sec. I), shared by the
// row-gather kernels and the masked (diagonal) tiles of the pair-once kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace nbody {

// One term of Eq. (gravity): particle i at (xi, yi, zi) against
// q = (x_j, y_j, z_j, m_j); adds m_j d r^3 to (ax, ay, az) and m_j r to pp,
// with d = x_i - x_j and r = (|d|^2 + eps2)^(-1/2).  13 VALU operations plus
// one hardware reciprocal square root (v_rsq_f32).
__device__ __forceinline__ void pair_term(float xi, float yi, float zi, float4 q, float eps2,
                                          float &ax, float &ay, float &az, float &pp)
{
    const float dx = xi - q.x;
    const float dy = yi - q.y;
    const float dz = zi - q.z;
    float s = __builtin_fmaf(dx, dx, eps2);
    s = __builtin_fmaf(dy, dy, s);
    s = __builtin_fmaf(dz, dz, s);
    const float r = __builtin_amdgcn_rsqf(s);
    const float mr = q.w * r;
    const float r2 = r * r;
    const float mr3 = mr * r2;
    pp += mr;
    ax = __builtin_fmaf(mr3, dx, ax);
    ay = __builtin_fmaf(mr3, dy, ay);
    az = __builtin_fmaf(mr3, dz, az);
}

// The same term with the pair removed when `skip` holds (j == i, or a
// padded slot): r is forced to 0 so every product vanishes exactly, also
// for eps2 == 0 where the self distance would give an infinite r.
__device__ __forceinline__ void pair_term_masked(float xi, float yi, float zi, float4 q,
                                                 float eps2, bool skip, float &ax, float &ay,
                                                 float &az, float &pp)
{
    const float dx = xi - q.x;
    const float dy = yi - q.y;
    const float dz = zi - q.z;
    float s = __builtin_fmaf(dx, dx, eps2);
    s = __builtin_fmaf(dy, dy, s);
    s = __builtin_fmaf(dz, dz, s);
    const float r = skip ? 0.0f : __builtin_amdgcn_rsqf(s);
    const float mr = q.w * r;
    const float r2 = r * r;
    const float mr3 = mr * r2;
    pp += mr;
    ax = __builtin_fmaf(mr3, dx, ax);
    ay = __builtin_fmaf(mr3, dy, ay);
    az = __builtin_fmaf(mr3, dz, az);
}

}  // namespace nbody
