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

// The problems a refresh or objective pass covers: those whose float64
// refresh is due after this step (k_j a multiple of the epoch length), or,
// with `sel` given, those with sel[j] != 0.  k_batch_list writes them once
// per pass as a list with prefix sums of their column and row tiles; the
// pass kernels then map a flat tile index onto (problem, tile) by a binary
// search of the prefix sums held in LDS, so a step in which few problems are
// due touches only their rows and columns.
struct BatchList {
    int32_t *n;       // [1] number of listed problems
    int32_t *ids;     // [count]
    int64_t *colp;    // [count + 1] prefix sums of ceil(n_j / 64)
    int64_t *rowp;    // [count + 1] prefix sums of ceil(m_j / 64)
};

// One block.  Chunks of kBlock problems: flags and tile counts, a block
// scan, then the selected problems are appended in order.  Every thread of
// the block must call it (it synchronises the block).
__device__ void batch_list_body(const BatchInst *__restrict__ desc, const int32_t *__restrict__ active, int count,
                                const int32_t *__restrict__ sel, const BatchList &out)
{
    __shared__ int32_t s_f[kBlock];
    __shared__ int64_t s_c[kBlock], s_r[kBlock];
    __shared__ int32_t s_base;
    __shared__ int64_t s_cb, s_rb;
    if (threadIdx.x == 0) {
        s_base = 0;
        s_cb = 0;
        s_rb = 0;
    }
    __syncthreads();
    for (int j0 = 0; j0 < count; j0 += kBlock) {
        const int j = j0 + (int)threadIdx.x;
        int32_t f = 0;
        int64_t c = 0, r = 0;
        if (j < count) {
            const BatchInst &d = desc[j];
            f = sel ? (sel[j] != 0) : (active[j] && d.spe > 0 && d.k % (uint64_t)d.spe == 0);
            if (f) {
                c = (d.n + 63) / 64;
                r = (d.m + 63) / 64;
            }
        }
        s_f[threadIdx.x] = f;
        s_c[threadIdx.x] = c;
        s_r[threadIdx.x] = r;
        __syncthreads();
        // inclusive scans (Hillis-Steele)
        for (int o = 1; o < kBlock; o <<= 1) {
            const int32_t fa = threadIdx.x >= (unsigned)o ? s_f[threadIdx.x - o] : 0;
            const int64_t ca = threadIdx.x >= (unsigned)o ? s_c[threadIdx.x - o] : 0;
            const int64_t ra = threadIdx.x >= (unsigned)o ? s_r[threadIdx.x - o] : 0;
            __syncthreads();
            s_f[threadIdx.x] += fa;
            s_c[threadIdx.x] += ca;
            s_r[threadIdx.x] += ra;
            __syncthreads();
        }
        if (f) {
            const int q = s_base + s_f[threadIdx.x] - 1;
            out.ids[q] = j;
            out.colp[q] = s_cb + s_c[threadIdx.x] - c;
            out.rowp[q] = s_rb + s_r[threadIdx.x] - r;
        }
        __syncthreads();
        if (threadIdx.x == kBlock - 1) {
            s_base += s_f[threadIdx.x];
            s_cb += s_c[threadIdx.x];
            s_rb += s_r[threadIdx.x];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out.n[0] = s_base;
        out.colp[s_base] = s_cb;
        out.rowp[s_base] = s_rb;
    }
}

__global__ void __launch_bounds__(kBlock)
k_batch_list(const BatchInst *__restrict__ desc, const int32_t *__restrict__ active, int count,
             const int32_t *__restrict__ sel, BatchList out)
{
    batch_list_body(desc, active, count, sel, out);
}

// Phase 2 for every active problem; block 0 also advances k_j of the active
// problems and then lists the problems whose refresh is due after this step
// (the list the refresh kernels that follow read).
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_batch_scatter(const char *__restrict__ seg, BatchInst *__restrict__ desc, const int32_t *__restrict__ active,
                int count, const int32_t *__restrict__ tile_inst, int64_t ntiles,
                typename ValT<V>::T *__restrict__ r, const int32_t *__restrict__ id_slot,
                const typename ValT<V>::T *__restrict__ delta_slot, BatchList due)
{
    if (blockIdx.x == 0) {
        for (int j = threadIdx.x; j < count; j += kBlock)
            if (active[j])
                desc[j].k += 1;  // other blocks of this kernel do not read k
        __syncthreads();
        batch_list_body(desc, active, count, nullptr, due);
    }
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

// Loads the list's count and one prefix array into LDS (kMaxListLds entries
// at most; longer lists are searched in global memory).
constexpr int kMaxListLds = 1024;

struct ListView {
    int n;
    const int64_t *p;  // LDS copy or global prefix sums [n + 1]
    const int32_t *ids;
    __device__ __forceinline__ int64_t total() const { return p[n]; }
    // index q with p[q] <= t < p[q + 1]
    __device__ __forceinline__ int find(int64_t t) const
    {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (p[mid] <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        return lo;
    }
};

__device__ __forceinline__ ListView load_list(const BatchList &L, const int64_t *pref, int64_t *lds)
{
    ListView v;
    v.n = L.n[0];
    v.ids = L.ids;
    if (v.n + 1 <= kMaxListLds) {
        for (int q = threadIdx.x; q <= v.n; q += kBlock)
            lds[q] = pref[q];
        __syncthreads();
        v.p = lds;
    } else {
        v.p = pref;
    }
    return v;
}

// r64 = -b over the rows of the listed problems.
__global__ void __launch_bounds__(kBlock)
k_batch_neg_b(const BatchInst *__restrict__ desc, BatchList L, const double *__restrict__ b,
              double *__restrict__ r64)
{
    __shared__ int64_t lds[kMaxListLds];
    const ListView v = load_list(L, L.rowp, lds);
    const int lane = threadIdx.x & 63;
    for (int64_t t = wave_global_id(); t < v.total(); t += wave_count()) {
        const int q = v.find(t);
        const BatchInst &d = desc[v.ids[q]];
        const int64_t row = (t - v.p[q]) * 64 + lane;
        if (row < d.m)
            r64[d.row_base + row] = -b[d.row_base + row];
    }
}

// r64 += x_i a_i over the columns of the listed problems (float64 atomics).
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_batch_refresh_cols(const char *__restrict__ seg, const BatchInst *__restrict__ desc, BatchList L,
                     const double *__restrict__ xm, double *__restrict__ r64)
{
    using T = typename ValT<V>::T;
    __shared__ int64_t lds[kMaxListLds];
    const ListView v = load_list(L, L.colp, lds);
    const TileLanes<G> tl;
    for (int64_t t = wave_global_id(); t < v.total(); t += wave_count()) {
        const int q = v.find(t);
        const BatchInst &d = desc[v.ids[q]];
        const int64_t col = (t - v.p[q]) * 64 + tl.lane;
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

// r = (T) r64 over the rows of the listed problems.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_batch_narrow(const BatchInst *__restrict__ desc, BatchList L, const double *__restrict__ r64, T *__restrict__ r)
{
    __shared__ int64_t lds[kMaxListLds];
    const ListView v = load_list(L, L.rowp, lds);
    const int lane = threadIdx.x & 63;
    for (int64_t t = wave_global_id(); t < v.total(); t += wave_count()) {
        const int q = v.find(t);
        const BatchInst &d = desc[v.ids[q]];
        const int64_t row = (t - v.p[q]) * 64 + lane;
        if (row < d.m)
            r[d.row_base + row] = (T)r64[d.row_base + row];
    }
}

// Per-problem objective pieces of the listed problems: acc[4j+0] +=
// ||r64||^2, acc[4j+1] += b.r64 (rows) and acc[4j+2] += ||x||_1 (columns, see
// k_batch_col_obj).  For the incremental maximum also dacc[4j+0] =
// max |r64 - rold|, dacc[4j+1] = max |rold| and dacc[4j+3] = max |r64|
// (maxima of values >= 0 through their bit patterns), after which rold = r64.
// Each wave takes a contiguous run of row tiles and keeps per-lane partial
// sums while the problem stays the same: the per-problem atomics go to a
// handful of addresses, so they are issued once per (wave, problem) rather
// than once per tile.
__global__ void __launch_bounds__(kBlock)
k_batch_row_sums(const BatchInst *__restrict__ desc, BatchList L, const double *__restrict__ b,
                 const double *__restrict__ r64, double *__restrict__ acc, double *__restrict__ rold,
                 double *__restrict__ dacc)
{
    __shared__ int64_t lds[kMaxListLds];
    const ListView v = load_list(L, L.rowp, lds);
    const int lane = threadIdx.x & 63;
    const int64_t T = v.total();
    const int64_t per = (T + wave_count() - 1) / wave_count();
    const int64_t t0 = wave_global_id() * per;
    const int64_t t1 = t0 + per < T ? t0 + per : T;
    double rr = 0.0, br = 0.0, dd = 0.0, oo = 0.0, xx = 0.0;
    int q = -1;
    int64_t qend = 0;
    auto amax = [](double *p, double v) {
        atomicMax(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v));
    };
    auto flush = [&]() {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            rr += __shfl_xor(rr, o, 64);
            br += __shfl_xor(br, o, 64);
            dd = fmax(dd, __shfl_xor(dd, o, 64));
            oo = fmax(oo, __shfl_xor(oo, o, 64));
            xx = fmax(xx, __shfl_xor(xx, o, 64));
        }
        if (lane == 0) {
            const int j = v.ids[q];
            atomic_add_hw<double>(acc + 4 * j + 0, rr);
            atomic_add_hw<double>(acc + 4 * j + 1, br);
            amax(dacc + 4 * j + 0, dd);
            amax(dacc + 4 * j + 1, oo);
            amax(dacc + 4 * j + 3, xx);
        }
        rr = br = dd = oo = xx = 0.0;
    };
    for (int64_t t = t0; t < t1; ++t) {
        if (t >= qend) {  // wave-uniform: next problem
            if (q >= 0)
                flush();
            q = v.find(t);
            qend = v.p[q + 1];
        }
        const BatchInst &d = desc[v.ids[q]];
        const int64_t row = (t - v.p[q]) * 64 + lane;
        if (row < d.m) {
            const int64_t g = d.row_base + row;
            const double x = r64[g], o = rold[g];
            rr += x * x;
            br += b[g] * x;
            dd = fmax(dd, fabs(x - o));
            oo = fmax(oo, fabs(o));
            xx = fmax(xx, fabs(x));
            rold[g] = x;
        }
    }
    if (q >= 0)
        flush();
}

// acc[4j+2] += ||x_j||_1 and acc[4j+3] = max(|a_i^T r64|) over the columns
// of the listed problems.  The max goes through the unsigned bit pattern
// (monotone for values >= 0).  Contiguous tile runs per wave, as in
// k_batch_row_sums.
//
// Incremental maximum (ist[4j] = M_old, the maximum of the last evaluation
// at rold; ist[4j+1] >= max_i ||a_i||_1; ist[4j+3] != 0 once that state
// exists; ub[i] >= |the computed sum of column i| at rold): every computed
// float64 sum moves by at most ||a_i||_1 D, D = ||r - rold||_inf + 2 gamma
// max(||r||_inf, ||rold||_inf) (Hoelder), gamma = (d + 2) 2^-52 covering the
// summation rounding at either point.  A column whose moved bound stays below
// M_old - max_i ||a_i||_1 D (a lower bound of the new maximum) cannot attain
// it and is not summed; the others are summed exactly as in the full pass,
// so the maximum is the same number.  ub is moved (non-candidates) or set
// to the computed value (candidates), rounded up; dacc[4j+2] counts the
// candidates.
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_batch_col_obj(const char *__restrict__ seg, const BatchInst *__restrict__ desc, BatchList L,
                const double *__restrict__ xm, const double *__restrict__ r64, double *__restrict__ acc,
                float *__restrict__ ub, const float *__restrict__ nrm, const double *__restrict__ ist,
                double *__restrict__ dacc, int incremental)
{
    using T = typename ValT<V>::T;
    __shared__ int64_t lds[kMaxListLds];
    const ListView v = load_list(L, L.colp, lds);
    const TileLanes<G> tl;
    const int64_t NT = v.total();
    const int64_t per = (NT + wave_count() - 1) / wave_count();
    const int64_t t0 = wave_global_id() * per;
    const int64_t t1 = t0 + per < NT ? t0 + per : NT;
    double ax = 0.0, gm = 0.0;
    int ncand = 0;
    int q = -1, j = 0;
    int64_t qend = 0;
    bool inc = false;
    double D = 0.0, lo = 0.0;
    auto flush = [&]() {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            ax += __shfl_xor(ax, o, 64);
            gm = fmax(gm, __shfl_xor(gm, o, 64));
        }
        if (tl.lane == 0) {
            atomic_add_hw<double>(acc + 4 * j + 2, ax);
            atomicMax(reinterpret_cast<unsigned long long *>(acc + 4 * j + 3),
                      (unsigned long long)__double_as_longlong(gm));
            if (ncand)
                atomic_add_hw<double>(dacc + 4 * j + 2, (double)ncand);
        }
        ax = gm = 0.0;
        ncand = 0;
    };
    for (int64_t t = t0; t < t1; ++t) {
        if (t >= qend) {  // wave-uniform: next problem
            if (q >= 0)
                flush();
            q = v.find(t);
            qend = v.p[q + 1];
            j = v.ids[q];
            const BatchInst &d = desc[j];
            inc = incremental && ist[4 * j + 3] != 0.0;
            if (inc) {
                const double dmax = d.lay.fixed_dpad ? (double)d.lay.fixed_dpad : (double)d.m;
                D = inc_shift(dacc[4 * j], fmax(dacc[4 * j + 3], dacc[4 * j + 1]), inc_gamma(dmax));
                lo = inc_lower(ist[4 * j], ist[4 * j + 1], D);
            }
        }
        const BatchInst &d = desc[j];
        const int64_t col = (t - v.p[q]) * 64 + tl.lane;
        int64_t off = 0;
        int32_t dp = 0;
        double bnd = 0.0;
        bool cand = false;
        if (col < d.n) {
            ax += fabs(xm[d.col_base + col]);
            cand = true;
            if (inc) {
                bnd = inc_moved((double)ub[d.col_base + col], (double)nrm[d.col_base + col], D);
                cand = !(bnd < lo);
            }
            if (cand)
                locate<V>(d.lay, col, off, dp);
        }
        const int nc = __popcll(__ballot(cand));
        ncand += nc;
        if (nc) {
            double a[G];
#pragma unroll
            for (int g = 0; g < G; ++g)
                a[g] = 0.0;
            const double *rr = r64 + d.row_base;
            tile_entries<V, G>(seg + d.rec_base, tl, off, dp, 0, [&](int g, int, int row, T val) {
                a[g] += (double)val * rr[row];
            });
            double mine = 0.0;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const double sq = group_sum<G>(a[g]);
                const double got = __shfl(sq, tl.leader_of_mine(g));
                if (tl.lane / TileLanes<G>::CPR == g)
                    mine = got;
            }
            if (cand) {
                gm = fmax(gm, fabs(mine));
                bnd = fabs(mine);
            }
        }
        if (col < d.n)
            ub[d.col_base + col] = round_up_f32(bnd);
    }
    if (q >= 0)
        flush();
}

// After an objective pass: the listed problems' maxima become M_old.
__global__ void k_batch_keep_max(BatchList L, const double *__restrict__ acc, double *__restrict__ ist)
{
    const int cnt = *L.n;
    for (int q = threadIdx.x; q < cnt; q += blockDim.x) {
        const int j = L.ids[q];
        ist[4 * j + 0] = acc[4 * j + 3];
        ist[4 * j + 3] = 1.0;
    }
}

}  // namespace pcdm
