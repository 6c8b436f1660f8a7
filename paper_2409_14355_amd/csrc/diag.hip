// Diagnostics for the roofline of the path search: the VALU issue rate of
// gfx950 measured with long chains of independent instructions, so that the
// counters of the detection kernels (VALU wave-instructions per launch) can be
// set against what the compute units actually issue.  Not part of the
// detection path.
#include "mpnl.h"

#include "device_common.h"

namespace mpnl {
namespace dev {
namespace {

// Eight independent accumulators per lane, `iters` rounds; every round issues
// eight VALU instructions of the chosen kind (the loop counter is scalar).
// kind 0: v_fma_f32.  kind 1: the point-choice mix of the descent (round,
// clamp, subtract, square, compare, select on pairs of values).  kind 2: DPP
// row shifts (the lane exchanges of the butterfly minimum).
__device__ __forceinline__ void diag_fma(float (&v)[8], float b, float c)
{
#pragma unroll
    for (int i = 0; i < 8; ++i)
        v[i] = fmaf(v[i], b, c);
}

__device__ __forceinline__ void diag_mix(float (&v)[8], float b, float c)
{
#pragma unroll
    for (int i = 0; i < 8; i += 2) {
        const float r = __builtin_rintf(v[i]);                         // v_rndne_f32
        const float m = __builtin_amdgcn_fmed3f(r, -3.f, 3.f);         // v_med3_f32
        const float d = v[i + 1] - m;                                   // v_sub_f32
        const float e = d * d;                                          // v_mul_f32
        v[i] = (e < b) ? e : c;                                         // v_cmp + v_cndmask
        v[i + 1] = m;
    }
}

__device__ __forceinline__ void diag_dpp(float (&v)[8])
{
#pragma unroll
    for (int i = 0; i < 8; ++i)
        v[i] = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[i]), 0x111, 0xF, 0xF, false));
}

__global__ __launch_bounds__(64) void valu_probe_kernel(float *out, int iters, int kind, float b, float c)
{
    float v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
        v[i] = (float)(threadIdx.x + i) * 1e-3f;
    if (kind == 0) {
        for (int it = 0; it < iters; ++it)
            diag_fma(v, b, c);
    } else if (kind == 1) {
        for (int it = 0; it < iters; ++it)
            diag_mix(v, b, c);
    } else {
        for (int it = 0; it < iters; ++it)
            diag_dpp(v);
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i)
        s += v[i];
    out[blockIdx.x * 64 + threadIdx.x] = s;  // keeps the chains alive
}

}  // namespace
}  // namespace dev
}  // namespace mpnl

extern "C" int mpnl_diag_valu_rate(int device, int kind, int waves, int iters, double *ms_out)
{
    if (kind < 0 || kind > 2 || waves < 1 || waves > (1 << 20) || iters < 1 || !ms_out)
        return MPNL_E_INVAL;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess)
        return MPNL_E_HIP;
    float *out = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t e = hipMalloc(&out, (size_t)waves * 64 * sizeof(float));
    if (e == hipSuccess)
        e = hipEventCreate(&t0);
    if (e == hipSuccess)
        e = hipEventCreate(&t1);
    float ms = 0.f;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first launch warms up
        e = hipEventRecord(t0, nullptr);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(mpnl::dev::valu_probe_kernel, dim3(waves), dim3(64), 0, nullptr, out, iters, kind,
                               0.5f, 0.25f);
            e = hipGetLastError();
        }
        if (e == hipSuccess)
            e = hipEventRecord(t1, nullptr);
        if (e == hipSuccess)
            e = hipEventSynchronize(t1);
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, t0, t1);
    }
    if (t0)
        (void)hipEventDestroy(t0);
    if (t1)
        (void)hipEventDestroy(t1);
    if (out)
        (void)hipFree(out);
    if (prev >= 0)
        (void)hipSetDevice(prev);
    if (e != hipSuccess)
        return MPNL_E_HIP;
    *ms_out = ms;
    return MPNL_OK;
}
