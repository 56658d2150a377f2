// Memory-system calibration used by the benchmark (not part of the method).
// Random reads (the gathers of r) and random atomic adds (the scatter into r).
//
// Each of `nthreads` threads reads kReads floats of table[0, m) at positions
// drawn by a chain of MurmurHash3 fmix32 steps and writes their sum.  The
// positions do not depend on loaded data, so every read is an independent
// 4-byte load at a random line: with a table the size of the residual the
// launch measures the rate at which the chip serves random lines from L2,
// the resource the partial-derivative gathers of a coordinate step consume.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kReads = 20;
constexpr int kBlock = 256;

__device__ __forceinline__ uint32_t fmix32(uint32_t h)
{
    h = (h ^ (h >> 16)) * 0x85EBCA6Bu;
    h = (h ^ (h >> 13)) * 0xC2B2AE35u;
    return h ^ (h >> 16);
}

__global__ void __launch_bounds__(kBlock)
k_random_gather(const float *__restrict__ table, uint32_t m, int64_t nthreads, uint32_t salt,
                float *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nthreads)
        return;
    uint32_t h = fmix32((uint32_t)t ^ salt);
    float acc = 0.0f;
#pragma unroll
    for (int q = 0; q < kReads; ++q) {
        h = fmix32(h + (uint32_t)q);
        acc += table[h % m];
    }
    out[t] = acc;
}

// Each thread adds 1 to kReads entries of table[0, m) picked as above, with
// hardware float atomics (no return): the rate of random atomic updates, the
// resource the residual scatter consumes.
__global__ void __launch_bounds__(kBlock)
k_random_atomic(float *__restrict__ table, uint32_t m, int64_t nthreads, uint32_t salt)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nthreads)
        return;
    uint32_t h = fmix32((uint32_t)t ^ salt);
#pragma unroll
    for (int q = 0; q < kReads; ++q) {
        h = fmix32(h + (uint32_t)q);
        unsafeAtomicAdd(table + (h % m), 1.0f);
    }
}

}  // namespace

// table: device, m floats (0 < m < 2^32); out: device, nthreads floats
// (0 < nthreads < 2^31 * 256); stream: a hipStream_t or null.  Enqueues one
// launch that performs nthreads * 20 random 4-byte reads.  Returns 0, 1 for
// invalid sizes, or the HIP error code of the launch.
extern "C" int pcdm_calib_random_gather(const float *table, int64_t m, int64_t nthreads, uint32_t salt, float *out,
                                        void *stream)
{
    if (!table || !out || m <= 0 || m > (int64_t)UINT32_MAX || nthreads <= 0 ||
        nthreads > (int64_t)0x7FFFFFFF * kBlock)
        return 1;
    const unsigned grid = (unsigned)((nthreads + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_random_gather, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, table, (uint32_t)m,
                       nthreads, salt, out);
    return (int)hipGetLastError();
}

// table: device, m floats (0 < m < 2^32), updated in place; other arguments
// as above.  Enqueues one launch that performs nthreads * 20 random atomic
// adds of 1.0f.  Returns 0, 1 for invalid sizes, or the HIP error code.
extern "C" int pcdm_calib_random_atomic(float *table, int64_t m, int64_t nthreads, uint32_t salt, void *stream)
{
    if (!table || m <= 0 || m > (int64_t)UINT32_MAX || nthreads <= 0 || nthreads > (int64_t)0x7FFFFFFF * kBlock)
        return 1;
    const unsigned grid = (unsigned)((nthreads + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_random_atomic, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, table, (uint32_t)m,
                       nthreads, salt);
    return (int)hipGetLastError();
}

// Reads (or atomic adds) per thread of one launch.
extern "C" int pcdm_calib_reads_per_thread(void) { return kReads; }
