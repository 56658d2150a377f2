// batch_kernels.hpp -- many independent LASSO problems advanced by one
// launch per phase.
//
// Every problem keeps its own column records, residual, x mirror, sampler
// key (seed_j, k_j), tau_j, beta_j and lambda_j (a regularisation path, or
// many right-hand sides).  The work of a launch is a list of 64-slot tiles
// (steps) or 64-column / 64-row tiles (refresh, objective) over all problems;
// tile t belongs to problem tile_inst[t].  The descriptor table and the
// active flags live in device memory, so the same launch sequence serves
// every step and can be captured once into a graph and replayed.
#pragma once

#include "kernels.hpp"

namespace pcdm {

struct BatchInst {
    Layout lay;            // pc already offset to this problem
    int64_t rec_base;      // byte offset of its records in seg
    int64_t row_base;      // element offset into r, r64, b
    int64_t col_base;      // element offset into the x mirror
    int64_t slot_base;     // element offset into id_slot / delta_slot
    int64_t step_tile0;    // first step tile of this problem
    int64_t col_tile0;     // first column tile
    int64_t row_tile0;     // first row tile
    int64_t m, n, tau, spe;  // spe = steps per epoch = refresh period
    uint64_t seed, k;
    double inv_beta, lam;
};

// Phase 1 for every active problem.
template <typename V, int G, int C>
__global__ void __launch_bounds__(kBlock)
k_batch_gather(char *__restrict__ seg, const BatchInst *__restrict__ desc, const int32_t *__restrict__ active,
               const int32_t *__restrict__ tile_inst, int64_t ntiles, const typename ValT<V>::T *__restrict__ r,
               double *__restrict__ xm, int32_t *__restrict__ id_slot, typename ValT<V>::T *__restrict__ delta_slot,
               uint64_t *__restrict__ nz_part)
{
    __shared__ uint64_t s_red[kBlock / 64];
    const TileLanes<G> tl;
    uint64_t nz = 0;
    for (int64_t t = wave_global_id(); t < ntiles; t += wave_count()) {
        const int j = tile_inst[t];
        if (!active[j])
            continue;
        const BatchInst d = desc[j];
        const NiceKey key = nice_key_wave(d.seed, d.k, (uint32_t)d.n);
        const SlotDraw sd = slot_draw_for(plan_nice(), d.seed, d.k);
        gather_tile<V, G, C>(seg + d.rec_base, d.lay, r + d.row_base, xm + d.col_base, id_slot + d.slot_base,
                             delta_slot + d.slot_base, key, sd, tl, (t - d.step_tile0) * 64, d.tau, d.inv_beta,
                             prox_lasso(d.lam), nz);
    }
    const uint64_t tot = block_sum_u64(nz, s_red);
    if (threadIdx.x == 0 && tot)
        nz_part[blockIdx.x] += tot;
}

// Phase 2 for every active problem; block 0 advances each active k_j.
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_batch_scatter(const char *__restrict__ seg, BatchInst *__restrict__ desc, const int32_t *__restrict__ active,
                int count, const int32_t *__restrict__ tile_inst, int64_t ntiles,
                typename ValT<V>::T *__restrict__ r, const int32_t *__restrict__ id_slot,
                const typename ValT<V>::T *__restrict__ delta_slot)
{
    if (blockIdx.x == 0)
        for (int j = threadIdx.x; j < count; j += kBlock)
            if (active[j])
                desc[j].k += 1;  // no block of this kernel reads k
    const TileLanes<G> tl;
    for (int64_t t = wave_global_id(); t < ntiles; t += wave_count()) {
        const int j = tile_inst[t];
        if (!active[j])
            continue;
        const BatchInst &d = desc[j];
        scatter_tile<V, G>(seg + d.rec_base, d.lay, r + d.row_base, id_slot + d.slot_base,
                           delta_slot + d.slot_base, tl, (t - d.step_tile0) * 64, d.tau);
    }
}

// Problems whose float64 refresh is due after this step (k_j a multiple of
// the epoch length), or every problem when `all` is set (objective).
__device__ __forceinline__ bool batch_due(const BatchInst &d, int act, int all)
{
    return all || (act && d.spe > 0 && d.k % (uint64_t)d.spe == 0);
}

// r64 = -b over the row tiles of due problems.
__global__ void __launch_bounds__(kBlock)
k_batch_neg_b(const BatchInst *__restrict__ desc, const int32_t *__restrict__ active,
              const int32_t *__restrict__ tile_inst, int64_t ntiles, const double *__restrict__ b,
              double *__restrict__ r64, int all)
{
    const int lane = threadIdx.x & 63;
    for (int64_t t = wave_global_id(); t < ntiles; t += wave_count()) {
        const int j = tile_inst[t];
        const BatchInst &d = desc[j];
        if (!batch_due(d, active[j], all))
            continue;
        const int64_t row = (t - d.row_tile0) * 64 + lane;
        if (row < d.m)
            r64[d.row_base + row] = -b[d.row_base + row];
    }
}

// r64 += x_i a_i over the column tiles of due problems (float64 atomics).
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_batch_refresh_cols(const char *__restrict__ seg, const BatchInst *__restrict__ desc,
                     const int32_t *__restrict__ active, const int32_t *__restrict__ tile_inst, int64_t ntiles,
                     const double *__restrict__ xm, double *__restrict__ r64, int all)
{
    using T = typename ValT<V>::T;
    const TileLanes<G> tl;
    for (int64_t t = wave_global_id(); t < ntiles; t += wave_count()) {
        const int j = tile_inst[t];
        const BatchInst &d = desc[j];
        if (!batch_due(d, active[j], all))
            continue;
        const int64_t col = (t - d.col_tile0) * 64 + tl.lane;
        const double xi = col < d.n ? xm[d.col_base + col] : 0.0;
        const bool live = xi != 0.0;
        if (!__any(live))
            continue;
        int64_t off = 0;
        int32_t dp = 0;
        if (live)
            locate<V>(d.lay, col, off, dp);
        double *rr = r64 + d.row_base;
        tile_entries<V, G>(seg + d.rec_base, tl, off, dp, xi, [&](int, double xq, int row, T val) {
            if (val != T(0))
                atomic_add_hw<double>(rr + row, xq * (double)val);
        });
    }
}

// r = (T) r64 over the row tiles of due problems.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_batch_narrow(const BatchInst *__restrict__ desc, const int32_t *__restrict__ active,
               const int32_t *__restrict__ tile_inst, int64_t ntiles, const double *__restrict__ r64,
               T *__restrict__ r)
{
    const int lane = threadIdx.x & 63;
    for (int64_t t = wave_global_id(); t < ntiles; t += wave_count()) {
        const int j = tile_inst[t];
        const BatchInst &d = desc[j];
        if (!batch_due(d, active[j], 0))
            continue;
        const int64_t row = (t - d.row_tile0) * 64 + lane;
        if (row < d.m)
            r[d.row_base + row] = (T)r64[d.row_base + row];
    }
}

// Per-problem objective pieces: acc[4j+0] += ||r64||^2, acc[4j+1] += b.r64
// (row tiles) and acc[4j+2] += ||x||_1 (column tiles, see k_batch_cols_obj).
__global__ void __launch_bounds__(kBlock)
k_batch_row_sums(const BatchInst *__restrict__ desc, const int32_t *__restrict__ tile_inst, int64_t ntiles,
                 const double *__restrict__ b, const double *__restrict__ r64, double *__restrict__ acc)
{
    const int lane = threadIdx.x & 63;
    for (int64_t t = wave_global_id(); t < ntiles; t += wave_count()) {
        const int j = tile_inst[t];
        const BatchInst &d = desc[j];
        const int64_t row = (t - d.row_tile0) * 64 + lane;
        double rr = 0.0, br = 0.0;
        if (row < d.m) {
            const double v = r64[d.row_base + row];
            rr = v * v;
            br = b[d.row_base + row] * v;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            rr += __shfl_xor(rr, o, 64);
            br += __shfl_xor(br, o, 64);
        }
        if (lane == 0) {
            atomic_add_hw<double>(acc + 4 * j + 0, rr);
            atomic_add_hw<double>(acc + 4 * j + 1, br);
        }
    }
}

// acc[4j+2] += ||x_j||_1 and acc[4j+3] = max(|a_i^T r64|) over column tiles.
// The max goes through the unsigned bit pattern (monotone for values >= 0).
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_batch_col_obj(const char *__restrict__ seg, const BatchInst *__restrict__ desc,
                const int32_t *__restrict__ tile_inst, int64_t ntiles, const double *__restrict__ xm,
                const double *__restrict__ r64, double *__restrict__ acc)
{
    using T = typename ValT<V>::T;
    const TileLanes<G> tl;
    for (int64_t t = wave_global_id(); t < ntiles; t += wave_count()) {
        const int j = tile_inst[t];
        const BatchInst &d = desc[j];
        const int64_t col = (t - d.col_tile0) * 64 + tl.lane;
        int64_t off = 0;
        int32_t dp = 0;
        double ax = 0.0;
        if (col < d.n) {
            locate<V>(d.lay, col, off, dp);
            ax = fabs(xm[d.col_base + col]);
        }
        double a[G];
#pragma unroll
        for (int q = 0; q < G; ++q)
            a[q] = 0.0;
        const double *rr = r64 + d.row_base;
        tile_entries<V, G>(seg + d.rec_base, tl, off, dp, 0, [&](int q, int, int row, T val) {
            a[q] += (double)val * rr[row];
        });
        double mine = 0.0;
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double s = group_sum<G>(a[q]);
            const double got = __shfl(s, tl.leader_of_mine(q));
            if (tl.lane / TileLanes<G>::CPR == q)
                mine = got;
        }
        double gm = col < d.n ? fabs(mine) : 0.0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            ax += __shfl_xor(ax, o, 64);
            gm = fmax(gm, __shfl_xor(gm, o, 64));
        }
        if (tl.lane == 0) {
            atomic_add_hw<double>(acc + 4 * j + 2, ax);
            atomicMax(reinterpret_cast<unsigned long long *>(acc + 4 * j + 3),
                      (unsigned long long)__double_as_longlong(gm));
        }
    }
}

}  // namespace pcdm
