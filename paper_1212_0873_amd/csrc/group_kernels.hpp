// group_kernels.hpp -- PCDM1 with blocks of several coordinates: the group
// LASSO  F(x) = 0.5||A x - b||^2 + lambda sum_i ||x^(i)||_2.
//
// Block i is the column range bp[i] .. bp[i+1]-1 (at most kGroupMax columns;
// section "Block structure, notation and assumptions" with consecutive
// blocks).  The block norms are Euclidean (B_i = I), so the block Lipschitz
// constant is L_i = lambda_max(A_i^T A_i), and the block update (eq. h(x)
// with w = L and Omega_i = lambda ||.||_2) is the block soft threshold
//     u = x^(i) - A_i^T r / (beta L_i),
//     x^(i) <- max(0, 1 - lambda / (beta L_i ||u||)) u.
// omega counts, per row, the distinct blocks with a nonzero in it.
#pragma once

#include "kernels.hpp"

namespace pcdm {

constexpr int kGroupMax = 16;

// One workgroup per block: the Gram matrix A_i^T A_i (float64, from the
// stored values) in LDS, its largest eigenvalue by cyclic Jacobi rotations
// (symmetric Schur decompositions, Golub & Van Loan), 1/L_i to invl; and the
// row histogram of distinct blocks (for omega).
template <typename V>
__global__ void __launch_bounds__(kBlock)
k_group_setup(const char *__restrict__ seg, Layout lay, const int64_t *__restrict__ bp, int64_t nb,
              double *__restrict__ invl, int32_t *__restrict__ hist, Ctrl *__restrict__ ctrl)
{
    using T = typename ValT<V>::T;
    __shared__ double Gm[kGroupMax][kGroupMax + 1];
    __shared__ int64_t s_off[kGroupMax];
    __shared__ int32_t s_dp[kGroupMax];
    for (int64_t blk = blockIdx.x; blk < nb; blk += gridDim.x) {
        const int64_t c0 = bp[blk];
        const int N = (int)(bp[blk + 1] - c0);
        if ((int)threadIdx.x < N) {
            int64_t off;
            int32_t dp;
            locate<V>(lay, c0 + threadIdx.x, off, dp);
            s_off[threadIdx.x] = off;
            s_dp[threadIdx.x] = dp;
        }
        __syncthreads();
        // Gram entries: thread t takes pairs t, t + kBlock, ... of a <= b
        const int npairs = N * (N + 1) / 2;
        for (int q = threadIdx.x; q < npairs; q += kBlock) {
            int a = 0, rem = q;
            while (rem >= N - a) {
                rem -= N - a;
                ++a;
            }
            const int b = a + rem;
            const char *ra = seg + s_off[a] + kHeader;
            const char *rb = seg + s_off[b] + kHeader;
            const int da = s_dp[a], db = s_dp[b];
            double acc = 0.0;
            for (int e = 0; e < da; e += 4) {
                int rwa[4];
                T va[4];
                Chunk4<V>::load(ra, da, e, rwa, va);
                for (int f = 0; f < db; f += 4) {
                    int rwb[4];
                    T vb[4];
                    Chunk4<V>::load(rb, db, f, rwb, vb);
#pragma unroll
                    for (int s = 0; s < 4; ++s)
#pragma unroll
                        for (int t = 0; t < 4; ++t)
                            if (rwa[s] == rwb[t])
                                acc += (double)va[s] * (double)vb[t];
                }
            }
            Gm[a][b] = acc;
            Gm[b][a] = acc;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double fro = 0.0;
            for (int a = 0; a < N; ++a)
                for (int b = 0; b < N; ++b)
                    fro += Gm[a][b] * Gm[a][b];
            for (int sweep = 0; sweep < 60; ++sweep) {
                double off = 0.0;
                for (int a = 0; a < N; ++a)
                    for (int b = a + 1; b < N; ++b)
                        off += Gm[a][b] * Gm[a][b];
                if (off <= 1e-32 * fro)
                    break;
                for (int p = 0; p < N; ++p)
                    for (int q = p + 1; q < N; ++q) {
                        const double apq = Gm[p][q];
                        if (apq == 0.0)
                            continue;
                        const double th = (Gm[q][q] - Gm[p][p]) / (2.0 * apq);
                        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        const double c = 1.0 / sqrt(t * t + 1.0);
                        const double s = t * c;
                        for (int k = 0; k < N; ++k) {  // columns p, q
                            const double gkp = Gm[k][p], gkq = Gm[k][q];
                            Gm[k][p] = c * gkp - s * gkq;
                            Gm[k][q] = s * gkp + c * gkq;
                        }
                        for (int k = 0; k < N; ++k) {  // rows p, q
                            const double gpk = Gm[p][k], gqk = Gm[q][k];
                            Gm[p][k] = c * gpk - s * gqk;
                            Gm[q][k] = s * gpk + c * gqk;
                        }
                    }
            }
            double lmax = 0.0;
            for (int a = 0; a < N; ++a)
                lmax = fmax(lmax, Gm[a][a]);
            invl[blk] = lmax > 0.0 ? 1.0 / lmax : 0.0;
            if (!(lmax > 0.0))
                atomicOr(&ctrl->err, (uint32_t)ERR_ZEROCOL);
        }
        // distinct blocks per row: count an entry if no earlier column of
        // the block has its row (rows within a column are distinct; padding
        // entries have value 0 and are skipped)
        for (int c = 0; c < N; ++c) {
            const char *rc = seg + s_off[c] + kHeader;
            for (int e = threadIdx.x; e < s_dp[c]; e += kBlock) {
                const int32_t row = reinterpret_cast<const int32_t *>(rc)[e];
                const V v = reinterpret_cast<const V *>(rc + 4 * (int64_t)s_dp[c])[e];
                if ((double)widen(v) == 0.0)
                    continue;
                bool first = true;
                for (int c2 = 0; c2 < c && first; ++c2) {
                    const char *r2 = seg + s_off[c2] + kHeader;
                    for (int f = 0; f < s_dp[c2]; ++f)
                        if (reinterpret_cast<const int32_t *>(r2)[f] == row &&
                            (double)widen(reinterpret_cast<const V *>(r2 + 4 * (int64_t)s_dp[c2])[f]) != 0.0) {
                            first = false;
                            break;
                        }
                }
                if (first)
                    atomicAdd(hist + row, 1);
            }
        }
        __syncthreads();
    }
}

// Phase 1 of a group step: a group of G lanes per sampled block (64/G blocks
// per wave).  Every lane of the group reads the block's columns with the
// same column dot as the coordinate path; the new block, x and dx (the
// change per column, read by the scatter) are written by the group's lanes;
// the slot holds the block, or its complement when nothing changed.
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_group_gather(char *__restrict__ seg, Layout lay, const typename ValT<V>::T *__restrict__ r,
               double *__restrict__ xm, const int64_t *__restrict__ bp, const double *__restrict__ invl,
               int32_t *__restrict__ id_slot, typename ValT<V>::T *__restrict__ dx, const Ctrl *__restrict__ ctrl,
               uint64_t *__restrict__ nz_part, uint64_t seed, int64_t tau, uint32_t nb, double inv_beta, double lam)
{
    using T = typename ValT<V>::T;
    __shared__ uint32_t s_keys[kNiceRounds];
    __shared__ uint64_t s_red[kBlock / 64];
    constexpr int SPW = 64 / G;
    const NiceKey key = nice_key_block(seed, ctrl->k, nb, s_keys);
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const int leader = lane & ~(G - 1);
    uint64_t nz = 0;
    for (int64_t base = wave_global_id() * SPW; base < tau; base += wave_count() * SPW) {
        const int64_t slot = base + lane / G;
        const bool act = slot < tau;  // the same for the whole group
        uint32_t i = 0;
        if (act && gl == 0)
            i = nice_slot((uint32_t)slot, key);
        i = (uint32_t)__shfl((int)i, leader);
        int64_t c0 = 0;
        int N = 0;
        double scale = 0.0;
        if (act) {
            c0 = bp[i];
            N = (int)(bp[i + 1] - c0);
            scale = invl[i] * inv_beta;  // 1 / (beta L_i)
        }
        double u[kGroupMax], xs[kGroupMax];
#pragma unroll
        for (int c = 0; c < kGroupMax; ++c) {
            u[c] = 0.0;
            xs[c] = 0.0;
        }
        double nrm2 = 0.0;
        // The block's columns in batches of CB: the record loads of a batch,
        // then its r gathers, then its reductions, so that the loads of
        // several columns are in flight together.  Each column is summed as
        // lane_dot sums it (first chunk, then the remaining ones).
        constexpr int CB = 4;
#pragma unroll
        for (int cb = 0; cb < kGroupMax; cb += CB) {
            if (!__any(cb < N))
                break;
            int64_t off[CB];
            int32_t dp[CB];
            int rw[CB][4];
            T v[CB][4];
#pragma unroll
            for (int q = 0; q < CB; ++q) {
                const int c = cb + q;
                off[q] = 0;
                dp[q] = 0;
                if (c < N) {
                    locate<V>(lay, c0 + c, off[q], dp[q]);
                    xs[c] = *reinterpret_cast<const double *>(seg + off[q]);
                }
                if (4 * gl < dp[q]) {
                    Chunk4<V>::load(seg + off[q] + kHeader, dp[q], 4 * gl, rw[q], v[q]);
                } else {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        rw[q][t] = 0;
                        v[q][t] = T(0);
                    }
                }
            }
            T acc[CB];
#pragma unroll
            for (int q = 0; q < CB; ++q) {
                acc[q] = T(0);
                if (4 * gl < dp[q]) {
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        acc[q] += v[q][t] * load_row(r, rw[q][t]);
                }
            }
#pragma unroll
            for (int q = 0; q < CB; ++q) {
                const char *rows = seg + off[q] + kHeader;
                for (int e = 4 * (gl + G); e < dp[q]; e += 4 * G) {
                    int rr[4];
                    T vv[4];
                    Chunk4<V>::load(rows, dp[q], e, rr, vv);
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        acc[q] += vv[t] * load_row(r, rr[t]);
                }
            }
#pragma unroll
            for (int q = 0; q < CB; ++q) {
                const int c = cb + q;
                if (c < N) {
                    const T g = group_sum<G>(acc[q]);
                    u[c] = xs[c] - (double)g * scale;
                    nrm2 += u[c] * u[c];
                }
            }
        }
        const double nrm = sqrt(nrm2);
        const double thr = lam * scale;
        const double fac = nrm > thr ? 1.0 - thr / nrm : 0.0;
        bool changed = false;
#pragma unroll
        for (int c = 0; c < kGroupMax; ++c) {
            if (c < N) {
                const double xn = fac * u[c];
                const double d = xn - xs[c];
                changed = changed || d != 0.0;
                if ((c & (G - 1)) == gl) {
                    int64_t off;
                    int32_t dp;
                    locate<V>(lay, c0 + c, off, dp);
                    if (d != 0.0) {
                        *reinterpret_cast<double *>(seg + off) = xn;
                        xm[c0 + c] = xn;
                    }
                    dx[c0 + c] = (T)d;
                }
            }
        }
        if (act && gl == 0) {
            id_slot[slot] = changed ? (int32_t)i : ~(int32_t)i;  // ~i: nothing to scatter
            if (changed)
                ++nz;
        }
    }
    const uint64_t tot = block_sum_u64(nz, s_red);
    if (threadIdx.x == 0 && tot)
        nz_part[blockIdx.x] += tot;
}

// Phase 2: r += A_i dx^(i) for the sampled blocks that changed (slot id >= 0;
// columns with dx != 0), hardware float atomics; advances the step counter.
// Each workgroup first packs the changed columns of kGroupScatterSpan
// consecutive slots into LDS as (column, dx) pairs, then scatters them in
// dense 64-column tiles as the coordinate scatter does: late in a run few
// blocks change, and a block's columns are no longer walked one after another.
constexpr int kGroupScatterSpan = 128;

template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_group_scatter(const char *__restrict__ seg, Layout lay, typename ValT<V>::T *__restrict__ r,
                const int64_t *__restrict__ bp, const int32_t *__restrict__ id_slot,
                const typename ValT<V>::T *__restrict__ dx, Ctrl *__restrict__ ctrl, int64_t tau)
{
    using T = typename ValT<V>::T;
    constexpr int kCap = kGroupScatterSpan * kGroupMax;
    __shared__ int32_t s_col[kCap];
    __shared__ T s_d[kCap];
    __shared__ int s_cnt;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        ctrl->k += 1;  // no block of this kernel reads k
    const TileLanes<G> tl;
    const int wave = threadIdx.x >> 6;
    for (int64_t base = (int64_t)blockIdx.x * kGroupScatterSpan; base < tau;
         base += (int64_t)gridDim.x * kGroupScatterSpan) {
        if (threadIdx.x == 0)
            s_cnt = 0;
        __syncthreads();
        if (threadIdx.x < kGroupScatterSpan) {
            const int64_t slot = base + threadIdx.x;
            const int32_t i = slot < tau ? id_slot[slot] : -1;
            if (i >= 0) {  // i < 0: block unchanged this step
                const int64_t c0 = bp[i];
                const int N = (int)(bp[i + 1] - c0);
                for (int c = 0; c < N; ++c) {
                    const T d = dx[c0 + c];
                    if (d != T(0)) {
                        const int q = atomicAdd(&s_cnt, 1);
                        s_col[q] = (int32_t)(c0 + c);
                        s_d[q] = d;
                    }
                }
            }
        }
        __syncthreads();
        const int cnt = s_cnt;
        for (int t0 = wave * 64; t0 < cnt; t0 += kBlock) {
            const int e = t0 + tl.lane;
            const bool live = e < cnt;
            const T d = live ? s_d[e] : T(0);
            int64_t off = 0;
            int32_t dp = 0;
            if (live)
                locate<V>(lay, s_col[e], off, dp);
            tile_entries<V, G>(seg, tl, off, dp, d, [&](int, T dq, int row, T val) {
                if (val != T(0))
                    atomic_add_hw<T>(r + row, dq * val);
            });
        }
        __syncthreads();
    }
}

// part[blk] = sum over this block's share of the blocks of ||x^(i)||_2.
__global__ void __launch_bounds__(kBlock)
k_group_xnorms(const int64_t *__restrict__ bp, int64_t nb, const double *__restrict__ xm, double *__restrict__ part)
{
    __shared__ double lds[kBlock];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nb; i += (int64_t)gridDim.x * kBlock) {
        double s = 0.0;
        for (int64_t c = bp[i]; c < bp[i + 1]; ++c)
            s += xm[c] * xm[c];
        acc += sqrt(s);
    }
    acc = block_sum_f64(acc, lds);
    if (threadIdx.x == 0)
        part[blockIdx.x] = acc;
}

// part[blk] = max over this block's share of the blocks of ||A_i^T r64||_2
// (float64), a group of G lanes per block.  With `ub` given, only the blocks
// with ub[i] >= *lo are evaluated (the others count as 0); each evaluated
// block's norm is summed exactly as without the filter.
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_group_atr(const char *__restrict__ seg, Layout lay, const double *__restrict__ r64, const int64_t *__restrict__ bp,
            int64_t nb, const float *__restrict__ ub, const double *__restrict__ lo, double *__restrict__ part)
{
    using T = typename ValT<V>::T;
    __shared__ double lds[kBlock];
    constexpr int SPW = 64 / G;
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const double thr = ub ? *lo : 0.0;
    double best = 0.0;
    for (int64_t base = wave_global_id() * SPW; base < nb; base += wave_count() * SPW) {
        const int64_t i = base + lane / G;
        const bool cand = i < nb && (!ub || (double)ub[i] >= thr);
        if (!__any(cand))
            continue;
        int N = 0;
        int64_t c0 = 0;
        if (cand) {
            c0 = bp[i];
            N = (int)(bp[i + 1] - c0);
        }
        double s2 = 0.0;
        for (int c = 0; c < kGroupMax; ++c) {
            if (c >= N)
                break;
            int64_t off;
            int32_t dp;
            locate<V>(lay, c0 + c, off, dp);
            const char *rows = seg + off + kHeader;
            double acc = 0.0;
            for (int e = 4 * gl; e < dp; e += 4 * G) {
                int rw[4];
                T v[4];
                Chunk4<V>::load(rows, dp, e, rw, v);
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc += (double)v[t] * r64[rw[t]];
            }
            const double g = group_sum<G>(acc);
            s2 += g * g;
        }
        best = fmax(best, sqrt(s2));
    }
    best = block_max_f64(best, lds);
    if (threadIdx.x == 0)
        part[blockIdx.x] = best;
}

// Bound pass of max_i ||A_i^T r64||_2 for values of at most float32
// precision, as for the coordinate maximum: each column's exact float64 dot
// with r64 lies within E_c of its dot v_c with t = fl32(r64) (the bound of the
// coordinate pass), so the block norm lies in
// [sqrt(sum max(0, |v_c| - E_c)^2), sqrt(sum (|v_c| + E_c)^2)], widened by
// 2^-40 relative for the rounding of the norms.  Writes the upper end to
// ub[i] (float32, rounded up) and part[blk] = the largest lower end.
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_group_atr_bound(const char *__restrict__ seg, Layout lay, const float *__restrict__ t32,
                  const int64_t *__restrict__ bp, int64_t nb, float *__restrict__ ub, double *__restrict__ part)
{
    using T = typename ValT<V>::T;
    __shared__ double lds[kBlock];
    constexpr int SPW = 64 / G;
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    double best = 0.0;
    for (int64_t base = wave_global_id() * SPW; base < nb; base += wave_count() * SPW) {
        const int64_t i = base + lane / G;
        int N = 0;
        int64_t c0 = 0;
        if (i < nb) {
            c0 = bp[i];
            N = (int)(bp[i + 1] - c0);
        }
        double hi2 = 0.0, lo2 = 0.0;
        for (int c = 0; c < kGroupMax; ++c) {
            if (c >= N)
                break;
            int64_t off;
            int32_t dp;
            locate<V>(lay, c0 + c, off, dp);
            const char *rows = seg + off + kHeader;
            double acc = 0.0, mag = 0.0, s1 = 0.0;
            for (int e = 4 * gl; e < dp; e += 4 * G) {
                int rw[4];
                T v[4];
                Chunk4<V>::load(rows, dp, e, rw, v);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const double pr = (double)v[t] * (double)t32[rw[t]];
                    acc += pr;
                    mag += fabs(pr);
                    s1 += fabs((double)v[t]);
                }
            }
            const double vv = group_sum<G>(acc), g = group_sum<G>(mag), a1 = group_sum<G>(s1);
            const double gam = (double)(dp + 2) * 0x1p-52;
            const double E = (0x1p-24 * g + 0x1p-149 * a1 + 3.0 * gam * g) * (1.0 + 4.0 * gam) + 0x1p-50 * fabs(vv);
            const double up = fabs(vv) + E, dn = fmax(0.0, fabs(vv) - E);
            hi2 += up * up;
            lo2 += dn * dn;
        }
        if (i < nb) {
            const double hi = sqrt(hi2) * (1.0 + 0x1p-40);
            float u = __builtin_inff();  // not finite (r beyond float32 range): always a candidate
            if (hi < 3.0e38) {
                u = (float)hi;
                if ((double)u < hi)
                    u = __int_as_float(__float_as_int(u) + 1);  // next float up (u >= 0, finite)
                best = fmax(best, sqrt(lo2) * (1.0 - 0x1p-40));
            }
            if (gl == 0)
                ub[i] = u;
        }
    }
    best = block_max_f64(best, lds);
    if (threadIdx.x == 0)
        part[blockIdx.x] = best;
}

}  // namespace pcdm
