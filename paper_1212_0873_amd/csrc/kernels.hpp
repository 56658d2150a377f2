// kernels.hpp -- gfx950 kernels of the synchronous PCDM1 step on the LASSO.
//
// Device layout (built once by k_pack):
//   seg     : column segments.  Column i starts at entry offset pc[i] (a
//             multiple of 4) and holds dpad_i = pc[i+1] - pc[i] entries
//             (its nonzeros rounded up to a multiple of 4): first dpad_i int32
//             row indices, then dpad_i values of type V.  One sampled column
//             is therefore one contiguous byte range, read with 16-byte (8-byte
//             for bf16) vector loads.  Padding entries repeat the column's last
//             row with value 0, so they add nothing to a dot product and are
//             skipped by the scatter.
//   invL    : 1 / L_i, L_i = ||a_i||^2 summed in float64 from stored values.
//   x, r    : iterate and working residual r = A x - b in the compute type T.
//   id_slot, delta_slot : per step, slot j's coordinate and its update.
//
// One step = k_gather (sample, gather-dot, prox, write x) followed by
// k_scatter (r += delta_i a_i for delta_i != 0).  The kernel boundary between
// them is the phase barrier that makes the step synchronous: every partial
// derivative of step k reads r_k, and every scatter of step k is visible to
// step k+1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sampler.hpp"

namespace pcdm {

constexpr int kBlock = 256;

struct bf16s {
    uint16_t bits;
};

// Device control block (one per problem).
struct Ctrl {
    uint64_t k;        // steps taken: key of the next step's sample
    uint32_t err;      // validation flags written at create
    uint32_t pad0;
    double scal[8];    // reduction results
    int64_t imax;      // integer reduction result
};

enum : uint32_t {
    ERR_PTR = 1u,      // col_ptr malformed
    ERR_EMPTY = 2u,    // empty column
    ERR_ROW = 4u,      // row index out of range
    ERR_DUP = 8u,      // repeated row in a column
    ERR_NONFINITE = 16u,
    ERR_ZEROCOL = 32u  // column with L_i = 0
};

template <typename V> struct ValT;
template <> struct ValT<float> { using T = float; };
template <> struct ValT<double> { using T = double; };
template <> struct ValT<bf16s> { using T = float; };

__device__ __forceinline__ float widen(float v) { return v; }
__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ float widen(bf16s v) { return __uint_as_float(((uint32_t)v.bits) << 16); }

template <typename V> constexpr int entry_bytes() { return 4 + (int)sizeof(V); }

// Load entries e..e+3 of a column (e a multiple of 4).
template <typename V> struct Chunk4;

template <> struct Chunk4<float> {
    __device__ __forceinline__ static void load(const char *col, int64_t dpad, int64_t e, int (&rw)[4],
                                                float (&v)[4])
    {
        const int4 a = *reinterpret_cast<const int4 *>(col + 4 * e);
        const float4 b = *reinterpret_cast<const float4 *>(col + 4 * dpad + 4 * e);
        rw[0] = a.x; rw[1] = a.y; rw[2] = a.z; rw[3] = a.w;
        v[0] = b.x; v[1] = b.y; v[2] = b.z; v[3] = b.w;
    }
};

template <> struct Chunk4<double> {
    __device__ __forceinline__ static void load(const char *col, int64_t dpad, int64_t e, int (&rw)[4],
                                                double (&v)[4])
    {
        const int4 a = *reinterpret_cast<const int4 *>(col + 4 * e);
        const double2 b0 = *reinterpret_cast<const double2 *>(col + 4 * dpad + 8 * e);
        const double2 b1 = *reinterpret_cast<const double2 *>(col + 4 * dpad + 8 * e + 16);
        rw[0] = a.x; rw[1] = a.y; rw[2] = a.z; rw[3] = a.w;
        v[0] = b0.x; v[1] = b0.y; v[2] = b1.x; v[3] = b1.y;
    }
};

template <> struct Chunk4<bf16s> {
    __device__ __forceinline__ static void load(const char *col, int64_t dpad, int64_t e, int (&rw)[4],
                                                float (&v)[4])
    {
        const int2 a0 = *reinterpret_cast<const int2 *>(col + 4 * e);
        const int2 a1 = *reinterpret_cast<const int2 *>(col + 4 * e + 8);
        const uint2 b = *reinterpret_cast<const uint2 *>(col + 4 * dpad + 2 * e);
        rw[0] = a0.x; rw[1] = a0.y; rw[2] = a1.x; rw[3] = a1.y;
        v[0] = __uint_as_float(b.x << 16);
        v[1] = __uint_as_float(b.x & 0xFFFF0000u);
        v[2] = __uint_as_float(b.y << 16);
        v[3] = __uint_as_float(b.y & 0xFFFF0000u);
    }
};

template <typename T> __device__ __forceinline__ T soft_threshold(T u, T c)
{
    return u > c ? u - c : (u < -c ? u + c : T(0));
}

template <typename T> __device__ __forceinline__ void atomic_add_hw(T *p, T v)
{
    // Hardware global float atomics (global_atomic_add_f32 / _f64): the
    // buffers are ordinary device allocations, for which they are exact.
    unsafeAtomicAdd(p, v);
}

// Sum over the G lanes of a group (G a power of two, groups aligned).
template <int G, typename T> __device__ __forceinline__ T group_sum(T v)
{
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1)
        v += __shfl_xor(v, o, G);
    return v;
}

template <typename T> __device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t *lds)
{
    // wave reduce then LDS
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        lds[w] = v;
    __syncthreads();
    uint64_t s = 0;
    if (threadIdx.x == 0)
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q)
            s += lds[q];
    return s;
}

// --------------------------------------------------------------------------
// The step.
// --------------------------------------------------------------------------

// Phase 1 of step k: for each slot j < tau (G lanes per slot) take
// i = pi_k(j), g_i = a_i^T r, the damped soft-threshold update of x_i, and
// record (i, delta_i) in slot j.
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_gather(const char *__restrict__ seg, const int64_t *__restrict__ pc,
         const typename ValT<V>::T *__restrict__ r, typename ValT<V>::T *__restrict__ x,
         const typename ValT<V>::T *__restrict__ invL, int32_t *__restrict__ id_slot,
         typename ValT<V>::T *__restrict__ delta_slot, const Ctrl *__restrict__ ctrl,
         uint64_t *__restrict__ nz_part, uint64_t seed, int64_t tau, uint32_t n,
         typename ValT<V>::T inv_beta, typename ValT<V>::T lam)
{
    using T = typename ValT<V>::T;
    constexpr int EB = entry_bytes<V>();
    __shared__ uint32_t s_keys[kNiceRounds];
    __shared__ uint64_t s_red[kBlock / 64];

    const NiceKey key = nice_key_block(seed, ctrl->k, n, s_keys);
    const int lane = threadIdx.x & (G - 1);
    const int64_t groups_per_block = kBlock / G;
    const int64_t stride = (int64_t)gridDim.x * groups_per_block;
    uint64_t nz = 0;

    for (int64_t slot = (int64_t)blockIdx.x * groups_per_block + threadIdx.x / G; slot < tau;
         slot += stride) {
        const uint32_t i = nice_slot((uint32_t)slot, key);
        const int64_t p0 = pc[i];
        const int64_t dpad = pc[i + 1] - p0;
        const char *col = seg + p0 * EB;
        T acc = T(0);
        for (int64_t e = 4 * lane; e < dpad; e += 4 * G) {
            int rw[4];
            T v[4];
            Chunk4<V>::load(col, dpad, e, rw, v);
            acc += v[0] * r[rw[0]];
            acc += v[1] * r[rw[1]];
            acc += v[2] * r[rw[2]];
            acc += v[3] * r[rw[3]];
        }
        acc = group_sum<G>(acc);
        if (lane == 0) {
            const T xi = x[i];
            const T scale = invL[i] * inv_beta;  // 1 / (beta L_i)
            const T xn = soft_threshold<T>(xi - acc * scale, lam * scale);
            const T d = xn - xi;
            id_slot[slot] = (int32_t)i;
            delta_slot[slot] = d;
            if (d != T(0)) {
                x[i] = xn;
                ++nz;
            }
        }
    }
    const uint64_t tot = block_sum_u64<T>(nz, s_red);
    if (threadIdx.x == 0 && tot)
        nz_part[blockIdx.x] += tot;
}

// Phase 2 of step k: r += delta_i a_i over the slots with delta_i != 0, with
// hardware float atomics (at most min(omega, tau) columns of one step share
// a row).  Also advances the step counter for step k+1.
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_scatter(const char *__restrict__ seg, const int64_t *__restrict__ pc,
          typename ValT<V>::T *__restrict__ r, const int32_t *__restrict__ id_slot,
          const typename ValT<V>::T *__restrict__ delta_slot, Ctrl *__restrict__ ctrl, int64_t tau)
{
    using T = typename ValT<V>::T;
    constexpr int EB = entry_bytes<V>();
    if (blockIdx.x == 0 && threadIdx.x == 0)
        ctrl->k += 1;  // no block of this kernel reads k
    const int lane = threadIdx.x & (G - 1);
    const int64_t groups_per_block = kBlock / G;
    const int64_t stride = (int64_t)gridDim.x * groups_per_block;
    for (int64_t slot = (int64_t)blockIdx.x * groups_per_block + threadIdx.x / G; slot < tau;
         slot += stride) {
        const T d = delta_slot[slot];
        if (d == T(0))
            continue;
        const int32_t i = id_slot[slot];
        const int64_t p0 = pc[i];
        const int64_t dpad = pc[i + 1] - p0;
        const char *col = seg + p0 * EB;
        for (int64_t e = 4 * lane; e < dpad; e += 4 * G) {
            int rw[4];
            T v[4];
            Chunk4<V>::load(col, dpad, e, rw, v);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (v[q] != T(0))
                    atomic_add_hw<T>(r + rw[q], d * v[q]);
        }
    }
}

// The sampler alone (for tests and callers that want S_k).
__global__ void __launch_bounds__(kBlock)
k_sample(uint64_t seed, uint64_t step, int64_t tau, uint32_t n, int32_t *__restrict__ out)
{
    __shared__ uint32_t s_keys[kNiceRounds];
    const NiceKey key = nice_key_block(seed, step, n, s_keys);
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < tau; j += (int64_t)gridDim.x * kBlock)
        out[j] = (int32_t)nice_slot((uint32_t)j, key);
}

// --------------------------------------------------------------------------
// float64 residual refresh r = A x - b.
// --------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock)
k_neg_copy(const double *__restrict__ b, double *__restrict__ r64, int64_t m)
{
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < m; j += (int64_t)gridDim.x * kBlock)
        r64[j] = -b[j];
}

// r64 += x_i a_i for x_i != 0 (float64 atomics).
template <typename V>
__global__ void __launch_bounds__(kBlock)
k_refresh_cols(const char *__restrict__ seg, const int64_t *__restrict__ pc,
               const typename ValT<V>::T *__restrict__ x, double *__restrict__ r64, int64_t n)
{
    constexpr int EB = entry_bytes<V>();
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double xi = (double)x[i];
        if (xi == 0.0)
            continue;
        const int64_t p0 = pc[i];
        const int64_t dpad = pc[i + 1] - p0;
        const char *col = seg + p0 * EB;
        for (int64_t e = 0; e < dpad; e += 4) {
            int rw[4];
            typename ValT<V>::T v[4];
            Chunk4<V>::load(col, dpad, e, rw, v);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (v[q] != 0)
                    atomic_add_hw<double>(r64 + rw[q], xi * (double)v[q]);
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_narrow(const double *__restrict__ r64, T *__restrict__ r, int64_t m)
{
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < m; j += (int64_t)gridDim.x * kBlock)
        r[j] = (T)r64[j];
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_widen(const T *__restrict__ src, double *__restrict__ dst, int64_t len)
{
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < len; j += (int64_t)gridDim.x * kBlock)
        dst[j] = (double)src[j];
}

template <typename S, typename D>
__global__ void __launch_bounds__(kBlock)
k_convert(const S *__restrict__ src, D *__restrict__ dst, int64_t len)
{
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < len; j += (int64_t)gridDim.x * kBlock)
        dst[j] = (D)src[j];
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_fill(T *__restrict__ p, T v, int64_t len)
{
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < len; j += (int64_t)gridDim.x * kBlock)
        p[j] = v;
}

// --------------------------------------------------------------------------
// Deterministic float64 reductions (fixed grid, fixed order).
// --------------------------------------------------------------------------

__device__ __forceinline__ double block_sum_f64(double v, double *lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    const double out = lds[0];
    __syncthreads();
    return out;
}

__device__ __forceinline__ double block_max_f64(double v, double *lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            lds[threadIdx.x] = fmax(lds[threadIdx.x], lds[threadIdx.x + s]);
        __syncthreads();
    }
    const double out = lds[0];
    __syncthreads();
    return out;
}

// part[3*blk + {0,1,2}] = partial sums of r64^2, b.r64, |x|.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_obj_partials(const double *__restrict__ r64, const double *__restrict__ b, const T *__restrict__ x,
               int64_t m, int64_t n, double *__restrict__ part)
{
    __shared__ double lds[kBlock];
    double rr = 0.0, br = 0.0, ax = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < m; j += stride) {
        const double v = r64[j];
        rr += v * v;
        br += b[j] * v;
    }
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        ax += fabs((double)x[i]);
    rr = block_sum_f64(rr, lds);
    br = block_sum_f64(br, lds);
    ax = block_sum_f64(ax, lds);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = rr;
        part[3 * blockIdx.x + 1] = br;
        part[3 * blockIdx.x + 2] = ax;
    }
}

// out[c] = sum_b part[ncomp*b + c] (c < ncomp) or max for mode 1; one block.
__global__ void __launch_bounds__(kBlock)
k_final(const double *__restrict__ part, int nparts, int ncomp, int mode, double *__restrict__ out)
{
    __shared__ double lds[kBlock];
    for (int c = 0; c < ncomp; ++c) {
        double a = mode ? 0.0 : 0.0;
        for (int q = threadIdx.x; q < nparts; q += kBlock)
            a = mode ? fmax(a, part[ncomp * q + c]) : a + part[ncomp * q + c];
        a = mode ? block_max_f64(a, lds) : block_sum_f64(a, lds);
        if (threadIdx.x == 0)
            out[c] = a;
    }
}

// part[blk] = max over the block's columns of |a_i^T r64| (float64 sums).
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_atr_absmax(const char *__restrict__ seg, const int64_t *__restrict__ pc, const double *__restrict__ r64,
             int64_t n, double *__restrict__ part)
{
    constexpr int EB = entry_bytes<V>();
    __shared__ double lds[kBlock];
    const int lane = threadIdx.x & (G - 1);
    const int64_t groups_per_block = kBlock / G;
    const int64_t stride = (int64_t)gridDim.x * groups_per_block;
    double best = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * groups_per_block + threadIdx.x / G; i < n; i += stride) {
        const int64_t p0 = pc[i];
        const int64_t dpad = pc[i + 1] - p0;
        const char *col = seg + p0 * EB;
        double acc = 0.0;
        for (int64_t e = 4 * lane; e < dpad; e += 4 * G) {
            int rw[4];
            typename ValT<V>::T v[4];
            Chunk4<V>::load(col, dpad, e, rw, v);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc += (double)v[q] * r64[rw[q]];
        }
        acc = group_sum<G>(acc);
        best = fmax(best, fabs(acc));
    }
    best = block_max_f64(best, lds);
    if (threadIdx.x == 0)
        part[blockIdx.x] = best;
}

// --------------------------------------------------------------------------
// Set-up: validation and packing into the segment layout.
// --------------------------------------------------------------------------

// dpad[i] = nonzeros of column i rounded up to 4 (dpad[n] = 0); flags bad pointers.
__global__ void __launch_bounds__(kBlock)
k_check_ptr(const int64_t *__restrict__ col_ptr, int64_t n, int64_t nnz, int64_t *__restrict__ dpad,
            Ctrl *__restrict__ ctrl)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i <= n; i += (int64_t)gridDim.x * kBlock) {
        if (i == n) {
            dpad[n] = 0;
            if (col_ptr[n] != nnz)
                atomicOr(&ctrl->err, ERR_PTR);
            continue;
        }
        const int64_t a = col_ptr[i], b = col_ptr[i + 1];
        if (i == 0 && a != 0)
            atomicOr(&ctrl->err, ERR_PTR);
        if (b < a || a < 0 || b > nnz) {
            atomicOr(&ctrl->err, ERR_PTR);
            dpad[i] = 0;
            continue;
        }
        if (b == a)
            atomicOr(&ctrl->err, ERR_EMPTY);
        dpad[i] = ((b - a) + 3) & ~(int64_t)3;
    }
}

__device__ __forceinline__ bool finite_val(float v) { return isfinite(v); }
__device__ __forceinline__ bool finite_val(double v) { return isfinite(v); }
__device__ __forceinline__ bool finite_val(bf16s v) { return ((v.bits >> 7) & 0xFF) != 0xFF; }

// Copy column i into its segment; L_i in float64 -> invL; row histogram of nonzeros.
template <typename V>
__global__ void __launch_bounds__(kBlock)
k_pack(const int64_t *__restrict__ col_ptr, const int32_t *__restrict__ row_idx, const V *__restrict__ val,
       const int64_t *__restrict__ pc, int64_t n, int64_t m, char *__restrict__ seg,
       typename ValT<V>::T *__restrict__ invL, int32_t *__restrict__ hist, Ctrl *__restrict__ ctrl)
{
    using T = typename ValT<V>::T;
    constexpr int EB = entry_bytes<V>();
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const int64_t a = col_ptr[i], b = col_ptr[i + 1];
        const int64_t p0 = pc[i], dpad = pc[i + 1] - p0;
        int32_t *rows = reinterpret_cast<int32_t *>(seg + p0 * EB);
        V *vals = reinterpret_cast<V *>(seg + p0 * EB + 4 * dpad);
        if (b <= a || dpad < b - a)
            continue;  // flagged by k_check_ptr
        uint32_t err = 0;
        double L = 0.0;
        bool sorted = true;
        int32_t prev = -1;
        for (int64_t p = a; p < b; ++p) {
            const int32_t rw = row_idx[p];
            const V v = val[p];
            if (rw < 0 || (int64_t)rw >= m) {
                err |= ERR_ROW;
                rows[p - a] = 0;
            } else {
                rows[p - a] = rw;
            }
            if (!finite_val(v))
                err |= ERR_NONFINITE;
            vals[p - a] = v;
            const double w = (double)widen(v);
            L += w * w;
            if (rw <= prev)
                sorted = false;
            prev = rw;
            if (w != 0.0 && rw >= 0 && (int64_t)rw < m)
                atomicAdd(hist + rw, 1);
        }
        if (!sorted) {
            for (int64_t p = a; p < b && !(err & ERR_DUP); ++p)
                for (int64_t q = p + 1; q < b; ++q)
                    if (row_idx[p] == row_idx[q]) {
                        err |= ERR_DUP;
                        break;
                    }
        }
        const int32_t last = rows[b - a - 1];
        for (int64_t p = b - a; p < dpad; ++p) {
            rows[p] = last;
            V z;
            if constexpr (sizeof(V) == 2) z.bits = 0; else z = V(0);
            vals[p] = z;
        }
        if (!(L > 0.0))
            err |= ERR_ZEROCOL;
        invL[i] = (T)(L > 0.0 ? 1.0 / L : 0.0);
        if (err)
            atomicOr(&ctrl->err, err);
    }
}

__global__ void __launch_bounds__(kBlock)
k_imax_partials(const int32_t *__restrict__ h, int64_t len, int64_t *__restrict__ part)
{
    __shared__ int64_t lds[kBlock];
    int64_t best = 0;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < len; j += (int64_t)gridDim.x * kBlock)
        best = best > h[j] ? best : (int64_t)h[j];
    lds[threadIdx.x] = best;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            lds[threadIdx.x] = lds[threadIdx.x] > lds[threadIdx.x + s] ? lds[threadIdx.x] : lds[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = lds[0];
}

__global__ void __launch_bounds__(kBlock)
k_imax_final(const int64_t *__restrict__ part, int nparts, Ctrl *__restrict__ ctrl)
{
    __shared__ int64_t lds[kBlock];
    int64_t best = 0;
    for (int q = threadIdx.x; q < nparts; q += kBlock)
        best = best > part[q] ? best : part[q];
    lds[threadIdx.x] = best;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            lds[threadIdx.x] = lds[threadIdx.x] > lds[threadIdx.x + s] ? lds[threadIdx.x] : lds[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        ctrl->imax = lds[0];
}

// Per-slot sum of nz_part (counter of nonzero updates).
__global__ void __launch_bounds__(kBlock)
k_sum_u64(const uint64_t *__restrict__ part, int nparts, Ctrl *__restrict__ ctrl)
{
    __shared__ uint64_t lds[kBlock / 64];
    uint64_t s = 0;
    for (int q = threadIdx.x; q < nparts; q += kBlock)
        s += part[q];
    s = block_sum_u64<double>(s, lds);
    if (threadIdx.x == 0)
        ctrl->imax = (int64_t)s;
}

}  // namespace pcdm
