// gen_device.hip -- writes the arrays of gen_common.h's recipe on the device
// (input construction for instances too large to build on the host).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gen_common.h"

namespace {

constexpr int kB = 256;

__global__ void __launch_bounds__(kB) k_col_ptr(int64_t *cp, int64_t n, int d)
{
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i <= n; i += (int64_t)gridDim.x * kB)
        cp[i] = (int64_t)d * i;
}

// dtype 0: float32, 1: bf16 bits (round to nearest even), 2: float64
__device__ inline uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += ((u >> 16) & 1u) + 0x7FFFu;
    return (uint16_t)(u >> 16);
}

__global__ void __launch_bounds__(kB) k_columns(uint64_t seed, uint64_t m, uint64_t n, int d, int32_t *rows,
                                               void *vals, int dtype)
{
    int32_t r[GEN_MAX_D];
    double v[GEN_MAX_D];
    for (uint64_t i = (uint64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kB) {
        gen_column(seed, m, n, d, i, r, v);
        const uint64_t base = (uint64_t)d * i;
        for (int t = 0; t < d; ++t) {
            rows[base + t] = r[t];
            if (dtype == 0)
                ((float *)vals)[base + t] = (float)v[t];
            else if (dtype == 1)
                ((uint16_t *)vals)[base + t] = to_bf16((float)v[t]);
            else
                ((double *)vals)[base + t] = v[t];
        }
    }
}

__global__ void __launch_bounds__(kB) k_noise(uint64_t seed, uint64_t m, double sigma, double *b)
{
    for (uint64_t j = (uint64_t)blockIdx.x * kB + threadIdx.x; j < m; j += (uint64_t)gridDim.x * kB)
        b[j] = gen_noise(seed, j, sigma);
}

// b += x*_j a_{pos_j} with the stored (rounded) values; x* written densely.
__global__ void __launch_bounds__(kB) k_plant(uint64_t seed, uint64_t m, uint64_t n, int d, uint64_t K, int dtype,
                                             double *b, double *xstar)
{
    int32_t r[GEN_MAX_D];
    double v[GEN_MAX_D];
    for (uint64_t j = (uint64_t)blockIdx.x * kB + threadIdx.x; j < K; j += (uint64_t)gridDim.x * kB) {
        uint64_t pos;
        double xv;
        gen_xstar(seed, n, j, &pos, &xv);
        xstar[pos] = xv;
        gen_column(seed, m, n, d, pos, r, v);
        for (int t = 0; t < d; ++t) {
            double s = v[t];
            if (dtype == 0)
                s = (double)(float)v[t];
            else if (dtype == 1)
                s = (double)__uint_as_float(((uint32_t)to_bf16((float)v[t])) << 16);
            unsafeAtomicAdd(b + r[t], xv * s);
        }
    }
}

int grid(uint64_t items) { return (int)(items / kB + 1 < 65536 ? items / kB + 1 : 65536); }

}  // namespace

extern "C" {

// col_ptr [n+1], rows [n*d], vals [n*d] of dtype; b [m]; xstar [n] (zeroed here).
int gen_device_instance(uint64_t seed, uint64_t m, uint64_t n, int d, uint64_t K, double sigma, int dtype,
                        int64_t *col_ptr, int32_t *rows, void *vals, double *b, double *xstar, void *stream)
{
    if (d < 1 || d > GEN_MAX_D || (uint64_t)d > m || K > n || m == 0 || n == 0)
        return -1;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_col_ptr, dim3(grid(n + 1)), dim3(kB), 0, s, col_ptr, (int64_t)n, d);
    hipLaunchKernelGGL(k_columns, dim3(grid(n)), dim3(kB), 0, s, seed, m, n, d, rows, vals, dtype);
    hipLaunchKernelGGL(k_noise, dim3(grid(m)), dim3(kB), 0, s, seed, m, sigma, b);
    if (hipMemsetAsync(xstar, 0, n * sizeof(double), s) != hipSuccess)
        return -2;
    hipLaunchKernelGGL(k_plant, dim3(grid(K)), dim3(kB), 0, s, seed, m, n, d, K, dtype, b, xstar);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // extern "C"
