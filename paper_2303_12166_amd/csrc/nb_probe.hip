// nb_probe.hip -- issue-rate probe of the vector ALU (a measurement aid for the force kernels'
// roofline). Each lane runs PROBE_CHAINS independent dependency chains of one instruction type,
// so with several waves per SIMD the rate is bounded by instruction issue, not by latency.
// Built with the library's flags (no packed FP32), so every FP32 operation is one non-packed
// VALU instruction.
#include "nb_internal.h"

namespace nbk {

constexpr int PROBE_CHAINS = 8;

// op 0: v_fma_f32; op 1: v_rsq_f32; op 2: v_rcp_f32; op 3: three v_fma_f32 per v_rsq_f32 (the
// transcendental and FMA streams interleaved, to see whether they overlap).
template <int OP>
__global__ __launch_bounds__(256) void k_valu_probe(float *sink, int iters, float b, float c)
{
    float v[PROBE_CHAINS];
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) v[k] = 1.0f + 0.001f * (float)(threadIdx.x + k);
    float u[PROBE_CHAINS];
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) u[k] = 2.0f + 0.001f * (float)k;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < PROBE_CHAINS; ++k) {
            if constexpr (OP == 0) {
                v[k] = fmaf(v[k], b, c);
            } else if constexpr (OP == 1) {
                v[k] = __builtin_amdgcn_rsqf(v[k]);
            } else if constexpr (OP == 2) {
                v[k] = __builtin_amdgcn_rcpf(v[k]);
            } else {
                u[k] = fmaf(u[k], b, c);
                u[k] = fmaf(u[k], b, c);
                u[k] = fmaf(u[k], b, c);
                v[k] = __builtin_amdgcn_rsqf(v[k]);
            }
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) s += v[k] + u[k];
    // the chains stay finite and positive (fma with b < 1, c > 0 converges; rsq and rcp of
    // values near 1 stay near 1), so the store never happens; it keeps the chains live
    if (!(s < 1.0e30f)) sink[0] = s;
}

hipError_t launch_valu_probe(int op, float *sink, int blocks, int iters, hipStream_t s)
{
    const dim3 g(blocks), b(256);
    const float fb = 0.999999f, fc = 1.0e-6f;
    switch (op) {
    case 0: hipLaunchKernelGGL(k_valu_probe<0>, g, b, 0, s, sink, iters, fb, fc); break;
    case 1: hipLaunchKernelGGL(k_valu_probe<1>, g, b, 0, s, sink, iters, fb, fc); break;
    case 2: hipLaunchKernelGGL(k_valu_probe<2>, g, b, 0, s, sink, iters, fb, fc); break;
    case 3: hipLaunchKernelGGL(k_valu_probe<3>, g, b, 0, s, sink, iters, fb, fc); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace nbk
