// inc_bound.hpp -- the rounding bounds of the incremental ||A^T r||_inf.
//
// One float64 evaluation keeps, per column i, an upper bound ub_i on
// |a_i^T r_old| and the float32 norm nrm_i >= ||a_i||_1.  For the next
// residual r, Hoelder's inequality gives |a_i^T (r - r_old)| <=
// ||a_i||_1 ||r - r_old||_inf, and a float64 sum of d products formed in any
// order is within gam ||a_i||_1 ||r||_inf of the exact value, gam =
// (d + 2) 2^-52.  So the computed sum moves by at most ||a_i||_1 D with
//     D = ||r - r_old||_inf + 2 gam max(||r||_inf, ||r_old||_inf),
// every column's bound moves to ub_i + nrm_i D, and the new maximum is at
// least M_old - max_i nrm_i D.  The extra relative margins below cover the
// rounding of these bound computations themselves.  The same functions
// serve the kernels and a host library that the CPU tests call, so the
// constants are checked where they are used.
#pragma once

#include <hip/hip_runtime.h>

namespace pcdm {

// gam for columns of at most dmax stored entries
__host__ __device__ inline double inc_gamma(double dmax) { return (dmax + 2.0) * 0x1p-52; }

// factor on the float64 sum of |a_ji| (at most dmax terms) so that the
// float32 value rounded up is >= ||a_i||_1
__host__ __device__ inline double inc_l1_factor(double dmax) { return 1.0 + (dmax + 8.0) * 0x1p-52; }

// D from the computed ||r - r_old||_inf (|fl(x - o)| understates |x - o| by
// at most a relative 2^-53) and the two residuals' max norms
__host__ __device__ inline double inc_shift(double dlt, double rmax, double gam)
{
    return (dlt * (1.0 + 0x1p-50) + 2.0 * gam * rmax) * (1.0 + 0x1p-40);
}

// lower bound on the new maximum from the old maximum and max_i nrm_i
__host__ __device__ inline double inc_lower(double m_old, double nrm_max, double D)
{
    return (m_old - nrm_max * D) * (1.0 - 0x1p-40) - 0x1p-1000;
}

// column bound moved by its norm times D
__host__ __device__ inline double inc_moved(double ub, double nrm, double D) { return ub * (1.0 + 0x1p-40) + nrm * D; }

}  // namespace pcdm
