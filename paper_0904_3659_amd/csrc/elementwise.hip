// Element-wise kernels around the force evaluation: the leap-frog kick and
// drift of Eqs. (1)-(3) (Sec. III) as one float32 axpy, and the synthetic
// particle fill used by the variant timer.
#include "common.hpp"

namespace nbody {
namespace {

// y[t] += alpha * xv[t]; grid-stride over 64-bit lengths.
__global__ __launch_bounds__(256) void axpy_kernel(float *__restrict__ y,
                                                   const float *__restrict__ xv, int64_t len,
                                                   float alpha)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < len; t += stride)
        y[t] = __builtin_fmaf(alpha, xv[t], y[t]);
}

// Kick then drift of one leap-frog step, Eqs. (1)-(2): v += kick * a, then
// x += dt * v (with the kicked v), in one pass over the particles.
__global__ __launch_bounds__(256) void kick_drift_kernel(float *__restrict__ x,
                                                         float *__restrict__ v,
                                                         const float *__restrict__ a, int64_t len,
                                                         float kick, float dt)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < len; t += stride) {
        const float vh = __builtin_fmaf(kick, a[t], v[t]);
        v[t] = vh;
        x[t] = __builtin_fmaf(dt, vh, x[t]);
    }
}

// The leap-frog update of `e` for rows whose force (or VJP) result is
// already stored in r3 / r1: the unfused form of the reduction epilogue.
__global__ __launch_bounds__(256) void lf_epilogue_kernel(const float *__restrict__ r3,
                                                          const float *__restrict__ r1, int n,
                                                          LfEpi e)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const float4 r = make_float4(r3[3 * (size_t)j + 0], r3[3 * (size_t)j + 1],
                                 r3[3 * (size_t)j + 2], r1 ? r1[j] : 0.f);
    lf_finish(e, j, r, nullptr, nullptr);
}

// 32-bit integer hash (Wang/Jenkins-style mixing) -> uniform float in [0,1).
__device__ __forceinline__ float hash_unit(uint32_t v)
{
    v = (v ^ 61u) ^ (v >> 16);
    v *= 9u;
    v ^= v >> 4;
    v *= 0x27d4eb2du;
    v ^= v >> 15;
    return (float)(v >> 8) * (1.0f / 16777216.0f);
}

// Timing inputs: positions uniform in the unit cube, masses 1/n, upstream
// weights uniform in [-1, 1).  Only used to time variants.
__global__ __launch_bounds__(256) void fill_kernel(float *x, float *m, float *w, float *v, int n,
                                                   uint32_t seed)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const uint32_t b = (uint32_t)i * 8u + seed * 0x9E3779B9u;
    x[3 * i + 0] = hash_unit(b + 0);
    x[3 * i + 1] = hash_unit(b + 1);
    x[3 * i + 2] = hash_unit(b + 2);
    m[i] = 1.0f / (float)n;
    if (w) {
        w[3 * i + 0] = 2.0f * hash_unit(b + 3) - 1.0f;
        w[3 * i + 1] = 2.0f * hash_unit(b + 4) - 1.0f;
        w[3 * i + 2] = 2.0f * hash_unit(b + 5) - 1.0f;
    }
    if (v) v[i] = 2.0f * hash_unit(b + 6) - 1.0f;
}

__global__ __launch_bounds__(256) void zero_int_kernel(int *p, int64_t len)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < len) p[i] = 0;
}

}  // namespace

nbody_status fill_zero_int(int *p, size_t len, hipStream_t stream)
{
    hipLaunchKernelGGL(zero_int_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, stream, p,
                       (int64_t)len);
    return check_launch("zero_int");
}

nbody_status axpy_run(float *y, const float *xv, int64_t len, float alpha, hipStream_t stream)
{
    int64_t blocks = (len + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (fault_injected("launch")) return fail(NBODY_ERROR_LAUNCH_FAILED, "injected launch fault");
    hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, y, xv, len, alpha);
    return check_launch("axpy");
}

nbody_status kick_drift_run(float *x, float *v, const float *a, int64_t len, float kick, float dt,
                            hipStream_t stream)
{
    int64_t blocks = (len + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (fault_injected("launch")) return fail(NBODY_ERROR_LAUNCH_FAILED, "injected launch fault");
    hipLaunchKernelGGL(kick_drift_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, x, v, a, len,
                       kick, dt);
    return check_launch("kick_drift");
}

nbody_status lf_epilogue_run(const float *r3, const float *r1, int64_t n, const LfEpi &e,
                             hipStream_t stream)
{
    if (fault_injected("launch")) return fail(NBODY_ERROR_LAUNCH_FAILED, "injected launch fault");
    hipLaunchKernelGGL(lf_epilogue_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       r3, r1, (int)n, e);
    return check_launch("lf_epilogue");
}

nbody_status fill_synthetic(float *x, float *m, float *w, float *v, int n, uint32_t seed,
                            hipStream_t stream)
{
    hipLaunchKernelGGL(fill_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, x, m, w, v, n, seed);
    return check_launch("fill_synthetic");
}

}  // namespace nbody
