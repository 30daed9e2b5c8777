// shg_ceiling.hip -- measured FP64 vector ceiling of the device: a kernel of
// independent FMA chains (no memory traffic in the loop), so that the
// roofline of the integral kernels can be read against what the chip
// sustains as well as against its published peak.
#include <hip/hip_runtime.h>

#include "shg_ctx.h"

using namespace shg;

namespace {

constexpr int CL_TPB = 256, CL_CHAINS = 8;

__global__ __launch_bounds__(CL_TPB) void k_fma_ceiling(int64_t iters, double y, double z, double *out)
{
    double x[CL_CHAINS];
#pragma unroll
    for (int c = 0; c < CL_CHAINS; ++c) x[c] = 1.0 + 1e-3 * (threadIdx.x + c);
    for (int64_t i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < CL_CHAINS; ++c) x[c] = fma(x[c], y, z);
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < CL_CHAINS; ++c) s += x[c];
    out[(int64_t)blockIdx.x * CL_TPB + threadIdx.x] = s;
}

}  // namespace

extern "C" int shg_fp64_ceiling(shg_ctx *c, int64_t iters, int blocks, double *out, double *flops)
{
    if (!c) return SHG_EINVAL;
    if (iters < 1 || blocks < 1 || !out || !flops)
        return set_err(c, SHG_EINVAL, "shg_fp64_ceiling: iters >= 1, blocks >= 1 and non-NULL pointers");
    // x stays bounded: the fixed point of x -> x y + z is z / (1 - y)
    hipLaunchKernelGGL(k_fma_ceiling, dim3(blocks), dim3(CL_TPB), 0, c->stream, iters, 0.999999, 1e-6, out);
    HIP_TRY(c, hipGetLastError());
    *flops = 2.0 * CL_CHAINS * (double)iters * (double)blocks * CL_TPB;
    return 0;
}
