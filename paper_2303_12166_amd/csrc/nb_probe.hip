// nb_probe.hip -- issue-rate probe of the vector ALU (a measurement aid for the force kernels'
// roofline). Each lane runs PROBE_CHAINS independent dependency chains of one instruction type,
// so with several waves per SIMD the rate is bounded by instruction issue, not by latency.
// Built with the library's flags (no packed FP32), so every FP32 operation is one non-packed
// VALU instruction.
#include "nb_internal.h"

namespace nbk {

constexpr int PROBE_CHAINS = 8;

// op 0: v_fma_f32 (VOP3, the addend a uniform value); op 1: v_rsq_f32; op 2: v_rcp_f32; op 3:
// three v_fma_f32 per v_rsq_f32 (the transcendental and FMA streams interleaved, to see whether
// they overlap); op 4: v_fmac_f32 (VOP2, accumulating into the chain); op 5: v_add_f32 (VOP2);
// op 6: v_mul_f32 (VOP2); op 7: v_sub_f32 with a DPP wave-rotation source (the symmetric force
// kernels' rotated j update); op 8: one v_mul_f32 and one v_add_f32 chain step in turn (whether an
// add issues beside a multiply). The force kernels' pair loops are mostly VOP2 adds, subtractions,
// multiplies and fmac.
template <int OP>
__global__ __launch_bounds__(256) void k_valu_probe(float *sink, int iters, float b, float c)
{
    // shader-clock and constant-rate counters around block 0's run (the clock the chip holds
    // under this instruction stream)
    const unsigned long long c0 = __builtin_amdgcn_s_memtime();
    const unsigned long long r0 = __builtin_amdgcn_s_memrealtime();
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
            } else if constexpr (OP == 4) {
                v[k] = fmaf(c, u[k], v[k]);
            } else if constexpr (OP == 5) {
                v[k] = v[k] + u[k];
            } else if constexpr (OP == 6) {
                v[k] = v[k] * b;
            } else if constexpr (OP == 8) {
                u[k] = u[k] * b;
                v[k] = v[k] + c;
            } else if constexpr (OP == 7) {
                // lane l takes lane l - 1's value (wave_ror:1) and subtracts u
                v[k] = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v[k]), 0x13C, 0xf,
                                                               0xf, true)) - u[k];
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
    // values near 1 stay near 1; the fmac chain grows by about 2e-6 and the add chain by about 2
    // per step, the DPP chain falls by about 2 per step, the mul chain decays slowly towards 0),
    // so the store never happens; it keeps the chains live
    if (!(s < 1.0e30f)) sink[0] = s;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const unsigned long long c1 = __builtin_amdgcn_s_memtime();
        const unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
        unsigned long long *clk = reinterpret_cast<unsigned long long *>(sink + 2);
        clk[0] = c1 - c0;
        clk[1] = r1 - r0;
    }
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
    case 4: hipLaunchKernelGGL(k_valu_probe<4>, g, b, 0, s, sink, iters, fb, fc); break;
    case 5: hipLaunchKernelGGL(k_valu_probe<5>, g, b, 0, s, sink, iters, fb, fc); break;
    case 6: hipLaunchKernelGGL(k_valu_probe<6>, g, b, 0, s, sink, iters, fb, fc); break;
    case 7: hipLaunchKernelGGL(k_valu_probe<7>, g, b, 0, s, sink, iters, fb, fc); break;
    case 8: hipLaunchKernelGGL(k_valu_probe<8>, g, b, 0, s, sink, iters, fb, fc); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace nbk
