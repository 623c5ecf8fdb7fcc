// FP64 throughput probe (diagnostic entry point mandel_fp64_probe in mandel.h):
// a pure fma chain and the bare escape-time update, timed on the device, give
// the ceiling that the render kernel's rate is compared with.
#include <hip/hip_runtime.h>

#include "mandel.h"
#include "mandel_internal.h"

#pragma clang fp contract(off)

namespace {

__global__ void __launch_bounds__(256) fma_chain_kernel(double *sink, int32_t iters, double a,
                                                        double b)
{
    double v0 = threadIdx.x * 1e-3, v1 = v0 + 1.0, v2 = v0 + 2.0, v3 = v0 + 3.0;
    for (int32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            v0 = __builtin_fma(v0, a, b);
            v1 = __builtin_fma(v1, a, b);
            v2 = __builtin_fma(v2, a, b);
            v3 = __builtin_fma(v3, a, b);
        }
    }
    sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = v0 + v1 + v2 + v3;
}

// z <- z^2 + c with c inside the main cardioid (bounded orbits, no escape).
template <int ILP>
__global__ void __launch_bounds__(256) update_loop_kernel(double *sink, int32_t iters)
{
    double x[ILP], y[ILP], cx[ILP], cy[ILP];
#pragma unroll
    for (int k = 0; k < ILP; ++k) {
        x[k] = 0.0;
        y[k] = 0.0;
        cx[k] = -0.1 - 1e-5 * (double)(threadIdx.x + k);
        cy[k] = 0.1 + 1e-6 * (double)blockIdx.x;
    }
    for (int32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
#pragma unroll
            for (int k = 0; k < ILP; ++k) {
                const double xx = x[k] * x[k];
                const double yy = y[k] * y[k];
                const double t = x[k] * y[k];
                x[k] = (xx - yy) + cx[k];
                y[k] = __builtin_fma(2.0, t, cy[k]);
            }
        }
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < ILP; ++k)
        s += x[k] + y[k];
    sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

} // namespace

using namespace mandel;

extern "C" int mandel_fp64_probe(int32_t kind, int32_t iters, int32_t blocks_per_cu, double *sink,
                                 double *flops, float *ms, void *stream)
{
    clear_error();
    if (kind < 0 || kind > 2)
        return fail(MANDEL_EINVAL, "kind=%d outside [0, 2]", kind);
    if (iters < 1 || iters > (1 << 24))
        return fail(MANDEL_EINVAL, "iters=%d outside [1, 2^24]", iters);
    if (blocks_per_cu < 1 || blocks_per_cu > 8)
        return fail(MANDEL_EINVAL, "blocks_per_cu=%d outside [1, 8]", blocks_per_cu);
    if (!sink || !flops || !ms)
        return fail(MANDEL_EINVAL, "null pointer");
    int cus = 0;
    int rc = device_cus(&cus);
    if (rc)
        return rc;
    const unsigned blocks = (unsigned)(cus * blocks_per_cu);
    const double lanes = (double)blocks * 256.0;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess)
        return hip_fail(e, "hipEventCreate");
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, s);
        if (kind == 0)
            hipLaunchKernelGGL(fma_chain_kernel, dim3(blocks), dim3(256), 0, s, sink, iters,
                               0.999, 1e-3);
        else if (kind == 1)
            hipLaunchKernelGGL(update_loop_kernel<1>, dim3(blocks), dim3(256), 0, s, sink, iters);
        else
            hipLaunchKernelGGL(update_loop_kernel<2>, dim3(blocks), dim3(256), 0, s, sink, iters);
        if (e == hipSuccess)
            e = hipGetLastError();
        if (e == hipSuccess)
            e = hipEventRecord(e1, s);
        if (e == hipSuccess)
            e = hipEventSynchronize(e1);
    }
    if (e == hipSuccess)
        e = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess)
        return hip_fail(e, "fp64 probe");
    const double per = kind == 0 ? 4.0 * 8.0 * 2.0 : (kind == 1 ? 8.0 * 7.0 : 2.0 * 8.0 * 7.0);
    *flops = lanes * (double)iters * per;
    return MANDEL_OK;
}
