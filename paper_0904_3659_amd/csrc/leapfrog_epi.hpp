// Leap-frog updates (Eqs. (1)-(3), Sec. III) folded into the final store of
// a force or force-adjoint evaluation, so a device-resident integrator needs
// no separate kick, drift or accumulate launches between force kernels.
//
// Every update is written with the same float32 FMAs, in the same order, as
// the stand-alone element-wise kernels (axpy_kernel, kick_drift_kernel): the
// fused and the unfused sequences give bitwise equal trajectories.
#pragma once

#include <hip/hip_runtime.h>

namespace nbody {

enum : int {
    kLfNone = 0,     // store the result only
    kLfKick = 1,     // forward: kick(s) of v with the new a, then an optional drift of x
    kLfAdjoint = 2,  // reverse: accumulate the weighted VJP into (lx, lm), optional lv += dt lx
};

struct LfEpi {
    int mode = kLfNone;
    // kLfKick: v += k1 a; if kicks == 2: v += k2 a; if drift: x += dt v (and
    // xh = x when xh is not NULL).  The second kick is the start kick of the
    // next step, the drift that step's drift, both at the positions the
    // force was evaluated at.
    int kicks = 1;
    int drift = 0;
    float k1 = 0.f, k2 = 0.f, dt = 0.f;
    float *v = nullptr, *x = nullptr, *xh = nullptr;
    // kLfAdjoint: lx += c gx; lm += c gm; if chain: lv += dt lx (the adjoint
    // of the drift of the step before, with the updated lx).
    int chain = 0;
    float c = 0.f;
    float *lx = nullptr, *lm = nullptr, *lv = nullptr;
};

// Finish row j with the reduced result r (xyz: a or grad_x, w: p or grad_m):
// store r into out3[j][3] / out1[j] when those are not NULL, then apply the
// update of `e`.
__device__ __forceinline__ void lf_finish(const LfEpi &e, int j, float4 r, float *out3,
                                          float *out1)
{
    const float rr[3] = {r.x, r.y, r.z};
    const size_t b = 3 * (size_t)j;
    if (e.mode == kLfAdjoint) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float lx = __builtin_fmaf(e.c, rr[k], e.lx[b + k]);
            e.lx[b + k] = lx;
            if (e.chain) e.lv[b + k] = __builtin_fmaf(e.dt, lx, e.lv[b + k]);
        }
        e.lm[j] = __builtin_fmaf(e.c, r.w, e.lm[j]);
        return;
    }
    if (out3) {
        out3[b + 0] = r.x;
        out3[b + 1] = r.y;
        out3[b + 2] = r.z;
    }
    if (out1) out1[j] = r.w;
    if (e.mode == kLfKick) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float v = __builtin_fmaf(e.k1, rr[k], e.v[b + k]);
            if (e.kicks == 2) v = __builtin_fmaf(e.k2, rr[k], v);
            e.v[b + k] = v;
            if (e.drift) {
                const float x = __builtin_fmaf(e.dt, v, e.x[b + k]);
                e.x[b + k] = x;
                if (e.xh) e.xh[b + k] = x;
            }
        }
    }
}

}  // namespace nbody
