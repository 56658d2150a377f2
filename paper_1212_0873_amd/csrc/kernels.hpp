// kernels.hpp -- gfx950 kernels of the synchronous PCDM1 step on the LASSO.
//
// Device layout (built once by k_pack):
//   seg  : one contiguous record per column i (coordinate i):
//            [ x_i : f64 ][ 1/L_i : f64 ][ dpad_i rows : int32 ][ dpad_i values : V ]
//          dpad_i = the column's nonzeros rounded up to a multiple of 4.
//          Padding entries repeat the column's last row with value 0: they add
//          nothing to a dot product and the scatter skips them.  A sampled
//          coordinate's whole update (x_i, 1/L_i, its rows and values) is one
//          contiguous read, so a random column costs its own bytes and no
//          separate random lines for x, 1/L or a pointer array.
//          Record offset: when every column has the same dpad (the usual
//          fixed-degree case) it is i * stride and no pointer array is read;
//          otherwise pc[i] * (4 + sizeof(V)) + 16 i, with pc the padded column
//          pointers.
//   x    : dense float64 mirror of the x_i held in the records, written with
//          them, read by the column-ordered passes (refresh, objective).
//          x is float64 on every path: a damped step (1/beta of the
//          coordinate-minimising step) below half a float32 ulp of x_i would
//          be lost, and the iteration would stall at a KKT residual near
//          beta L_i ulp(x_i).  1/L_i = 1/||a_i||^2 is summed in float64.
//   r    : working residual r = A x - b in the compute type T.
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

#include "inc_bound.hpp"
#include "sampler.hpp"

namespace pcdm {

constexpr int kBlock = 256;
constexpr int kHeader = 16;  // bytes of {x_i, 1/L_i} in front of each column

// Fixed-stride records are padded to a multiple of this many bytes: a 176-byte
// record (20 float32 entries) at 64-byte alignment spans two 128-byte lines
// instead of 2.25 on average (measured: gather 163 -> 161 us per 1e6-slot
// step on the 1e6-row instance, for 9% more record memory).
#ifndef PCDM_RECORD_ALIGN
#define PCDM_RECORD_ALIGN 64
#endif

// Column chunks (4 entries) a gather lane keeps in flight before its first
// dependent r load: more hides latency, fewer leaves registers for more waves.
#ifndef PCDM_CHUNK_BUDGET
#define PCDM_CHUNK_BUDGET 8
#endif
// Column entries are read with the non-temporal hint: each sampled record is
// used once per step, and keeping it out of the way leaves more of L2 to r
// (measured, gather per 1e6-slot step on the 1e6-row instance: float32
// 168.7 -> 163.4 us, bf16 163.8 -> 159.4 us, float64 224.9 -> 219.5 us).
#ifndef PCDM_NT_RECORDS
#define PCDM_NT_RECORDS 1
#endif
// 1: in the tiles, a lane of each column's group that holds no entries reads
// the record header {x_i, 1/L_i} in the same load instruction as the rows,
// instead of the owner lane reading it separately: one L2 request less per
// column, and the header's registers are not held across the rounds
// (measured: gather 161 -> 150 us per 1e6-slot step on the 1e6-row instance).
#ifndef PCDM_HDR_FOLD
#define PCDM_HDR_FOLD 1
#endif

typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef int v2i_t __attribute__((ext_vector_type(2)));
typedef unsigned int v2u_t __attribute__((ext_vector_type(2)));
typedef double v2d_t __attribute__((ext_vector_type(2)));

template <typename T> __device__ __forceinline__ T ld_rec(const T *p)
{
#if PCDM_NT_RECORDS
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

struct bf16s {
    uint16_t bits;
};

// Device control block (one per problem).
struct Ctrl {
    uint64_t k;           // steps taken: key of the next step's sample
    uint32_t err;         // validation flags written at create
    uint32_t nonuniform;  // set when padded column lengths differ
    double scal[8];       // reduction results
    int64_t imax;         // integer reduction result
};

enum : uint32_t {
    ERR_PTR = 1u,      // col_ptr malformed
    ERR_EMPTY = 2u,    // empty column
    ERR_ROW = 4u,      // row index out of range
    ERR_DUP = 8u,      // repeated row in a column
    ERR_NONFINITE = 16u,
    ERR_ZEROCOL = 32u,  // column with L_i = 0
    ERR_LABEL = 64u     // label other than +-1 (logistic / square hinge)
};

template <typename V> struct ValT;
template <> struct ValT<float> { using T = float; };
template <> struct ValT<double> { using T = double; };
template <> struct ValT<bf16s> { using T = float; };

__device__ __forceinline__ float widen(float v) { return v; }
__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ float widen(bf16s v) { return __uint_as_float(((uint32_t)v.bits) << 16); }

template <typename V> constexpr int entry_bytes() { return 4 + (int)sizeof(V); }

// Where column records live.
struct Layout {
    const int64_t *pc;  // padded column pointers (entries), used when fixed_dpad == 0
    int64_t fixed_dpad; // common padded length, or 0
    int64_t stride;     // record bytes when fixed_dpad != 0
};

template <typename V>
__device__ __forceinline__ void locate(const Layout &L, int64_t i, int64_t &off, int32_t &dp)
{
    if (L.fixed_dpad) {
        dp = (int32_t)L.fixed_dpad;
        off = i * L.stride;
    } else {
        const int64_t p0 = L.pc[i];
        dp = (int32_t)(L.pc[i + 1] - p0);
        off = p0 * entry_bytes<V>() + (int64_t)kHeader * i;
    }
}

// Load entries e..e+3 of a column whose rows start at `rows` (e a multiple of 4).
template <typename V> struct Chunk4;

// `bits16` reads 16 bytes (four rows, or a record header) and `vals` the
// values of entries e..e+3.
template <> struct Chunk4<float> {
    __device__ __forceinline__ static v4i_t bits16(const char *p) { return ld_rec(reinterpret_cast<const v4i_t *>(p)); }
    __device__ __forceinline__ static void vals(const char *rows, int32_t dpad, int32_t e, float (&v)[4])
    {
        const v4f_t b = ld_rec(reinterpret_cast<const v4f_t *>(rows + 4 * dpad + 4 * e));
        v[0] = b.x; v[1] = b.y; v[2] = b.z; v[3] = b.w;
    }
    __device__ __forceinline__ static void load(const char *rows, int32_t dpad, int32_t e, int (&rw)[4],
                                                float (&v)[4])
    {
        const v4i_t a = bits16(rows + 4 * e);
        vals(rows, dpad, e, v);
        rw[0] = a.x; rw[1] = a.y; rw[2] = a.z; rw[3] = a.w;
    }
};

template <> struct Chunk4<double> {
    __device__ __forceinline__ static v4i_t bits16(const char *p) { return ld_rec(reinterpret_cast<const v4i_t *>(p)); }
    __device__ __forceinline__ static void vals(const char *rows, int32_t dpad, int32_t e, double (&v)[4])
    {
        const v2d_t b0 = ld_rec(reinterpret_cast<const v2d_t *>(rows + 4 * dpad + 8 * e));
        const v2d_t b1 = ld_rec(reinterpret_cast<const v2d_t *>(rows + 4 * dpad + 8 * e + 16));
        v[0] = b0.x; v[1] = b0.y; v[2] = b1.x; v[3] = b1.y;
    }
    __device__ __forceinline__ static void load(const char *rows, int32_t dpad, int32_t e, int (&rw)[4],
                                                double (&v)[4])
    {
        const v4i_t a = bits16(rows + 4 * e);
        vals(rows, dpad, e, v);
        rw[0] = a.x; rw[1] = a.y; rw[2] = a.z; rw[3] = a.w;
    }
};

// bf16 records are only 8-byte aligned in the variable-length layout, so 16
// bytes are read as two 8-byte loads.
template <> struct Chunk4<bf16s> {
    __device__ __forceinline__ static v4i_t bits16(const char *p)
    {
        const v2i_t a0 = ld_rec(reinterpret_cast<const v2i_t *>(p));
        const v2i_t a1 = ld_rec(reinterpret_cast<const v2i_t *>(p + 8));
        return v4i_t{a0.x, a0.y, a1.x, a1.y};
    }
    __device__ __forceinline__ static void vals(const char *rows, int32_t dpad, int32_t e, float (&v)[4])
    {
        const v2u_t b = ld_rec(reinterpret_cast<const v2u_t *>(rows + 4 * dpad + 2 * e));
        v[0] = __uint_as_float(b.x << 16);
        v[1] = __uint_as_float(b.x & 0xFFFF0000u);
        v[2] = __uint_as_float(b.y << 16);
        v[3] = __uint_as_float(b.y & 0xFFFF0000u);
    }
    __device__ __forceinline__ static void load(const char *rows, int32_t dpad, int32_t e, int (&rw)[4],
                                                float (&v)[4])
    {
        const v4i_t a = bits16(rows + 4 * e);
        vals(rows, dpad, e, v);
        rw[0] = a.x; rw[1] = a.y; rw[2] = a.z; rw[3] = a.w;
    }
};

template <typename T> __device__ __forceinline__ T soft_threshold(T u, T c)
{
    return u > c ? u - c : (u < -c ? u + c : T(0));
}

// Smooth losses f = s * sum_j phi(m_j) (introduction, table of three losses).
// For the logistic and square-hinge losses the labels are folded into the
// stored values (row j times y_j), so the maintained vector holds the
// margins m_j = y_j a_j^T x and phi needs no label: logistic
// log(1 + exp(-m)), square hinge 0.5 max(0, 1 - m)^2.  The square loss keeps
// r = A x - b and phi(r) = 0.5 r^2.  dphi is d phi / d m (or d r).
enum : int { kLossSquare = 0, kLossLogistic = 1, kLossSqHinge = 2 };

template <int Loss, typename T> __device__ __forceinline__ T dphi(T m)
{
    if constexpr (Loss == kLossLogistic) {
        return T(-1) / (T(1) + exp(m));
    } else if constexpr (Loss == kLossSqHinge) {
        const T h = T(1) - m;
        return h > T(0) ? -h : T(0);
    } else {
        return m;
    }
}

template <int Loss> __device__ __forceinline__ double phi64(double m)
{
    if constexpr (Loss == kLossLogistic) {
        return m < 0.0 ? -m + log1p(exp(m)) : log1p(exp(-m));
    } else if constexpr (Loss == kLossSqHinge) {
        const double h = 1.0 - m;
        return h > 0.0 ? 0.5 * h * h : 0.0;
    } else {
        return 0.5 * m * m;
    }
}

// Separable regulariser Omega_i(t) = l1|t| + (l2/2)t^2 + c t + [lo <= t <= hi]
// and the scale s of the loss (partial derivatives are s * a_i^T phi'(.)).
struct ProxParams {
    double l1, l2, c, lo, hi, gscale;
};

__host__ __device__ inline ProxParams prox_lasso(double lam)
{
    ProxParams p;
    p.l1 = lam;
    p.l2 = 0.0;
    p.c = 0.0;
    p.lo = -HUGE_VAL;
    p.hi = HUGE_VAL;
    p.gscale = 1.0;
    return p;
}

// Block minimiser of g t + (beta L/2) t^2 + Omega(x + t), returned as the new
// x (scale = 1/(beta L)): for u = x + t the smooth part is
// ((beta L + l2)/2)(u - w)^2 + const, w = (x - (g + c) scale)/(1 + l2 scale);
// l1|u| makes it a soft threshold at l1 scale/(1 + l2 scale), and the box a
// clip (the minimiser of a convex function of one variable over an interval).
// With l2 = c = 0 this is the LASSO step soft(x - g scale, l1 scale).
__device__ __forceinline__ double model_prox(double xi, double g, double scale, const ProxParams &pp)
{
    double u;
    if (pp.l2 == 0.0 && pp.c == 0.0)
        u = soft_threshold<double>(xi - g * scale, pp.l1 * scale);
    else
        u = soft_threshold<double>(xi - (g + pp.c) * scale, pp.l1 * scale) / (1.0 + pp.l2 * scale);
    return fmin(fmax(u, pp.lo), pp.hi);
}

template <typename T> __device__ __forceinline__ void atomic_add_hw(T *p, T v)
{
    // Hardware global float atomics (global_atomic_add_f32 / _f64): the
    // buffers are ordinary device allocations, for which they are exact.
    unsafeAtomicAdd(p, v);
}

// base[row] through a 32-bit byte offset from a uniform base (the host
// checks that r spans < 4 GiB).
template <typename T> __device__ __forceinline__ T load_row(const T *__restrict__ base, int row)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + (uint32_t)row * (uint32_t)sizeof(T));
}

// Sum over the G lanes of a group (G a power of two, groups aligned).
template <int G, typename T> __device__ __forceinline__ T group_sum(T v)
{
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1)
        v += __shfl_xor(v, o, G);
    return v;
}

__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t *lds)
{
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
// Tiles.  A wave owns 64 consecutive slots (or columns).  Per-slot work
// (sampling, locating the record, x_i and 1/L_i, the update) runs one lane
// per slot; the column entries are then read in G rounds, each round giving
// 64/G columns to groups of G lanes, so a column's contiguous entries are read
// by G neighbouring lanes with 16-byte loads.  Each lane holds C chunks (4
// entries each) of its round's column in registers, with the loads of a
// batch of rounds issued before any dependent gather; longer columns finish
// in a loop.
// --------------------------------------------------------------------------

template <int G> struct TileLanes {
    static constexpr int CPR = 64 / G;  // columns per round
    int lane, gl, grp;
    __device__ __forceinline__ TileLanes()
    {
        lane = threadIdx.x & 63;
        gl = lane & (G - 1);
        grp = lane / G;
    }
    // lane owning the column handled by this lane's group in round q
    __device__ __forceinline__ int owner(int q) const { return q * CPR + grp; }
    // in round q, the group leader of column `lane` (valid when lane / CPR == q)
    __device__ __forceinline__ int leader_of_mine(int q) const { return ((lane - q * CPR) & (CPR - 1)) * G; }
};

__device__ __forceinline__ int64_t wave_global_id() { return (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); }
__device__ __forceinline__ int64_t wave_count() { return (int64_t)gridDim.x * (kBlock / 64); }

// For every live column of a tile (owner lanes give the record offset and
// length; dp = 0 means nothing to do) call f(q, wq, row, value) on each
// stored entry, where wq is the owner's scalar w broadcast to its group.
template <typename V, int G, typename W, typename F>
__device__ __forceinline__ void tile_entries(const char *__restrict__ seg, const TileLanes<G> &tl, int64_t off,
                                             int32_t dp, W w, F &&f)
{
    using T = typename ValT<V>::T;
#pragma unroll
    for (int q = 0; q < G; ++q) {
        const int64_t coff = __shfl(off, tl.owner(q));
        const int32_t cdp = __shfl(dp, tl.owner(q));
        const W wq = __shfl(w, tl.owner(q));
        const char *rows = seg + coff + kHeader;
        for (int e = 4 * tl.gl; e < cdp; e += 4 * G) {
            int rw[4];
            T v[4];
            Chunk4<V>::load(rows, cdp, e, rw, v);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                f(q, wq, rw[t], v[t]);
        }
    }
}

// --------------------------------------------------------------------------
// The step.
// --------------------------------------------------------------------------

// One tile of phase 1: slots base .. base+63 of a step with sampler key
// `key`.  Slot j takes i = pi_k(j), g_i = a_i^T r (working precision T) and
// the damped soft-threshold update of x_i in float64; records (i, delta_i) in
// slot j and writes x_i (record and mirror).  Pointers are the problem's own.
template <typename V, int G, int C, int Loss = kLossSquare>
__device__ __forceinline__ void gather_tile(char *__restrict__ seg, const Layout &lay,
                                            const typename ValT<V>::T *__restrict__ r, double *__restrict__ xm,
                                            int32_t *__restrict__ id_slot,
                                            typename ValT<V>::T *__restrict__ delta_slot, const NiceKey &key,
                                            const SlotDraw &sd, const TileLanes<G> &tl, int64_t base, int64_t tau,
                                            double inv_beta, const ProxParams &pp, uint64_t &nz)
{
    using T = typename ValT<V>::T;
    const int64_t slot = base + tl.lane;
    const bool act = slot < tau;
    bool live = false;
    uint32_t i = 0;
    int64_t off = 0;
    int32_t dp = 0;
    double xi = 0.0, il = 0.0;
    if (act)
        live = draw_slot(sd, key, (uint32_t)slot, i);
    // A column of at most 4(G-1) entries leaves its group's last lane idle:
    // that lane reads the header with the rows (PCDM_HDR_FOLD).
    constexpr bool kFold = PCDM_HDR_FOLD && G >= 2;
    if (live) {
        locate<V>(lay, i, off, dp);
        if (!kFold || dp > 4 * (G - 1)) {
            const double *hdr = reinterpret_cast<const double *>(seg + off);
            xi = hdr[0];
            il = hdr[1];
        }
    }
    // rounds in batches of RB so that at most PCDM_CHUNK_BUDGET chunks per lane are live
    constexpr int RB = (G < PCDM_CHUNK_BUDGET / C) ? G : (PCDM_CHUNK_BUDGET / C > 0 ? PCDM_CHUNK_BUDGET / C : 1);
    T mine = T(0);
    constexpr int kUnroll = (G == RB) ? 1 : 2;
#pragma unroll kUnroll
    for (int q0 = 0; q0 < G; q0 += RB) {
        int64_t qoff[RB];
        int32_t qdp[RB];
        int rw[RB][C][4];
        T v[RB][C][4];
#pragma unroll
        for (int qq = 0; qq < RB; ++qq) {
            const int q = q0 + qq;
            qoff[qq] = __shfl(off, tl.owner(q));
            qdp[qq] = __shfl(dp, tl.owner(q));
            const char *rows = seg + qoff[qq] + kHeader;
            if constexpr (kFold) {
                // chunk 0: rows of entries 4gl..4gl+3, or the header on the idle last lane
                const int e = 4 * tl.gl;
                const bool hl = tl.gl == G - 1 && qdp[qq] > 0 && qdp[qq] <= 4 * (G - 1);
                const bool ld = e < qdp[qq];
                // the header lane keeps the header's bits in rw: its entries are idle
                if (ld || hl) {
                    const v4i_t a = Chunk4<V>::bits16(ld ? rows + 4 * e : seg + qoff[qq]);
                    rw[qq][0][0] = a.x; rw[qq][0][1] = a.y; rw[qq][0][2] = a.z; rw[qq][0][3] = a.w;
                } else {
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        rw[qq][0][t] = 0;
                }
                if (ld) {
                    Chunk4<V>::vals(rows, qdp[qq], e, v[qq][0]);
                } else {
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        v[qq][0][t] = T(0);
                }
            }
#pragma unroll
            for (int c = kFold ? 1 : 0; c < C; ++c) {
                const int e = 4 * (tl.gl + G * c);
                if (e < qdp[qq]) {
                    Chunk4<V>::load(rows, qdp[qq], e, rw[qq][c], v[qq][c]);
                } else {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        rw[qq][c][t] = 0;
                        v[qq][c][t] = T(0);
                    }
                }
            }
        }
        T acc[RB];
#pragma unroll
        for (int qq = 0; qq < RB; ++qq) {
            if constexpr (kFold) {
                const int q = q0 + qq;
                const int hsrc = tl.leader_of_mine(q) + G - 1;
                const int h0 = __shfl(rw[qq][0][0], hsrc), h1 = __shfl(rw[qq][0][1], hsrc);
                const int h2 = __shfl(rw[qq][0][2], hsrc), h3 = __shfl(rw[qq][0][3], hsrc);
                if (tl.lane / TileLanes<G>::CPR == q && dp <= 4 * (G - 1)) {
                    xi = __hiloint2double(h1, h0);
                    il = __hiloint2double(h3, h2);
                }
            }
            acc[qq] = T(0);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if (4 * (tl.gl + G * c) < qdp[qq]) {
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        acc[qq] += v[qq][c][t] * dphi<Loss>(load_row(r, rw[qq][c][t]));
                }
            }
        }
#pragma unroll
        for (int qq = 0; qq < RB; ++qq) {
            const char *rows = seg + qoff[qq] + kHeader;
            for (int e = 4 * (tl.gl + G * C); e < qdp[qq]; e += 4 * G) {
                int rr[4];
                T vv[4];
                Chunk4<V>::load(rows, qdp[qq], e, rr, vv);
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc[qq] += vv[t] * dphi<Loss>(load_row(r, rr[t]));
            }
        }
#pragma unroll
        for (int qq = 0; qq < RB; ++qq) {
            const int q = q0 + qq;
            const T sum = group_sum<G>(acc[qq]);
            const T got = __shfl(sum, tl.leader_of_mine(q));
            if (tl.lane / TileLanes<G>::CPR == q)
                mine = got;
        }
    }
    if (act) {
        const double xn = model_prox(xi, (double)mine * pp.gscale, il * inv_beta, pp);  // il * inv_beta = 1/(beta L_i)
        const double d = live ? xn - xi : 0.0;
        id_slot[slot] = (int32_t)i;
        delta_slot[slot] = (T)d;
        if (d != 0.0) {
            // streaming stores: neither line is read again in this step
            __builtin_nontemporal_store(xn, reinterpret_cast<double *>(seg + off));
            __builtin_nontemporal_store(xn, xm + i);
            ++nz;
        }
    }
}

// One tile of phase 2: r += delta_i a_i for the tile's slots with delta_i != 0.
template <typename V, int G>
__device__ __forceinline__ void scatter_tile(const char *__restrict__ seg, const Layout &lay,
                                             typename ValT<V>::T *__restrict__ r,
                                             const int32_t *__restrict__ id_slot,
                                             const typename ValT<V>::T *__restrict__ delta_slot,
                                             const TileLanes<G> &tl, int64_t base, int64_t tau)
{
    using T = typename ValT<V>::T;
    const int64_t slot = base + tl.lane;
    const T d = slot < tau ? delta_slot[slot] : T(0);
    const bool live = d != T(0);
    if (!__any(live))
        return;
    int64_t off = 0;
    int32_t dp = 0;
    if (live)
        locate<V>(lay, id_slot[slot], off, dp);
    tile_entries<V, G>(seg, tl, off, dp, d, [&](int, T dq, int row, T val) {
        if (val != T(0))
            atomic_add_hw<T>(r + row, dq * val);
    });
}

// Phase 1 of step k over all tiles of one problem.
template <typename V, int G, int C, int Loss = kLossSquare>
__global__ void __launch_bounds__(kBlock)
k_gather(char *__restrict__ seg, Layout lay, const typename ValT<V>::T *__restrict__ r,
         double *__restrict__ xm, int32_t *__restrict__ id_slot, typename ValT<V>::T *__restrict__ delta_slot,
         const Ctrl *__restrict__ ctrl, uint64_t *__restrict__ nz_part, uint64_t seed, int64_t tau,
         uint32_t n, double inv_beta, ProxParams pp, SlotPlan plan)
{
    __shared__ uint32_t s_keys[kNiceRounds];
    __shared__ uint64_t s_red[kBlock / 64];
    const uint64_t k = ctrl->k;
    const NiceKey key = nice_key_block(seed, k, n, s_keys);
    const SlotDraw sd = slot_draw_for(plan, seed, k);
    const TileLanes<G> tl;
    uint64_t nz = 0;
    for (int64_t base = wave_global_id() * 64; base < tau; base += wave_count() * 64)
        gather_tile<V, G, C, Loss>(seg, lay, r, xm, id_slot, delta_slot, key, sd, tl, base, tau, inv_beta, pp, nz);
    const uint64_t tot = block_sum_u64(nz, s_red);
    if (threadIdx.x == 0 && tot)
        nz_part[blockIdx.x] += tot;
}

// Phase 2 of step k: r += delta_i a_i over the slots with delta_i != 0, with
// hardware float atomics (at most min(omega, tau) columns of one step share
// a row).  Also advances the step counter for step k+1.  Late in a run few
// updates are nonzero, scattered over the slots; so each workgroup first
// packs the nonzero (i, delta_i) of kScatterSpan consecutive slots into LDS
// and then scatters them in dense 64-column tiles.
constexpr int kScatterSpan = 1024;

template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_scatter(const char *__restrict__ seg, Layout lay, typename ValT<V>::T *__restrict__ r,
          const int32_t *__restrict__ id_slot, const typename ValT<V>::T *__restrict__ delta_slot,
          Ctrl *__restrict__ ctrl, int64_t tau)
{
    using T = typename ValT<V>::T;
    __shared__ int32_t s_id[kScatterSpan];
    __shared__ T s_d[kScatterSpan];
    __shared__ int s_cnt;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        ctrl->k += 1;  // no block of this kernel reads k
    const TileLanes<G> tl;
    const int wave = threadIdx.x >> 6;
    for (int64_t base = (int64_t)blockIdx.x * kScatterSpan; base < tau; base += (int64_t)gridDim.x * kScatterSpan) {
        if (threadIdx.x == 0)
            s_cnt = 0;
        __syncthreads();
        for (int j = threadIdx.x; j < kScatterSpan; j += kBlock) {
            const int64_t slot = base + j;
            if (slot < tau) {
                const T d = delta_slot[slot];
                if (d != T(0)) {
                    const int q = atomicAdd(&s_cnt, 1);
                    s_id[q] = id_slot[slot];
                    s_d[q] = d;
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
                locate<V>(lay, s_id[e], off, dp);
            tile_entries<V, G>(seg, tl, off, dp, d, [&](int, T dq, int row, T val) {
                if (val != T(0))
                    atomic_add_hw<T>(r + row, dq * val);
            });
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------------------
// Narrow schedule for small tau: one slot per group of G lanes (64/G slots
// per wave), so tau slots spread over tau*G/64 waves instead of tau/64 and a
// small step is not left to a handful of waves.  The group leader draws the
// slot, reads the record header and writes the result; the G lanes read the
// column's entries as in the tiles.
// --------------------------------------------------------------------------

// This lane's share of a_i^T r for a column of dp (padded) entries whose rows
// start at `rows`, read by the G lanes of a group (lane gl takes chunks gl,
// gl + G, ...; C of them loaded before any dependent gather).
// Reads of r in the asynchronous kernel: kReadCached = ordinary loads (they
// may return a line the XCD's L2 holds from before other XCDs' atomics);
// kReadAtomic = a returning atomic add of zero, performed where the
// scatter-adds are, so it sees every add that has landed.
enum : int { kReadCached = 0, kReadAcquire = 1, kReadAtomic = 2 };

template <typename T, int Mode> __device__ __forceinline__ T load_r(const T *base, int row)
{
    if constexpr (Mode == kReadAtomic)
        return unsafeAtomicAdd(const_cast<T *>(base) + (uint32_t)row, T(0));
    else
        return load_row(base, row);
}

template <typename V, int G, int C, int Fresh = kReadCached, int Loss = kLossSquare>
__device__ __forceinline__ typename ValT<V>::T lane_dot(const char *rows, int32_t dp, int gl,
                                                        const typename ValT<V>::T *r)
{
    using T = typename ValT<V>::T;
    int rw[C][4];
    T v[C][4];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int e = 4 * (gl + G * c);
        if (e < dp) {
            Chunk4<V>::load(rows, dp, e, rw[c], v[c]);
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                rw[c][t] = 0;
                v[c][t] = T(0);
            }
        }
    }
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        if (4 * (gl + G * c) < dp) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc += v[c][t] * dphi<Loss>(load_r<T, Fresh>(r, rw[c][t]));
        }
    }
    for (int e = 4 * (gl + G * C); e < dp; e += 4 * G) {
        int rr[4];
        T vv[4];
        Chunk4<V>::load(rows, dp, e, rr, vv);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc += vv[t] * dphi<Loss>(load_r<T, Fresh>(r, rr[t]));
    }
    return acc;
}

template <typename V, int G, int C, int Loss>
__device__ __forceinline__ void gather_slot_narrow(char *__restrict__ seg, const Layout &lay,
                                                   const typename ValT<V>::T *__restrict__ r, double *__restrict__ xm,
                                                   int32_t *__restrict__ id_slot,
                                                   typename ValT<V>::T *__restrict__ delta_slot, const NiceKey &key,
                                                   const SlotDraw &sd, int gl, int leader, int64_t slot,
                                                   int64_t tau, double inv_beta, const ProxParams &pp, uint64_t &nz)
{
    using T = typename ValT<V>::T;
    const bool act = slot < tau;  // the same for the whole group
    int live = 0;
    uint32_t i = 0;
    int64_t off = 0;
    int32_t dp = 0;
    double xi = 0.0, il = 0.0;
    if (act && gl == 0) {
        live = draw_slot(sd, key, (uint32_t)slot, i) ? 1 : 0;
        if (live) {
            locate<V>(lay, i, off, dp);
            const double *hdr = reinterpret_cast<const double *>(seg + off);
            xi = hdr[0];
            il = hdr[1];
        }
    }
    off = __shfl(off, leader);
    dp = __shfl(dp, leader);
    const T g = group_sum<G>(lane_dot<V, G, C, kReadCached, Loss>(seg + off + kHeader, dp, gl, r));
    if (act && gl == 0) {
        const double xn = model_prox(xi, (double)g * pp.gscale, il * inv_beta, pp);
        const double d = live ? xn - xi : 0.0;
        id_slot[slot] = (int32_t)i;
        delta_slot[slot] = (T)d;
        if (d != 0.0) {
            // streaming stores: neither line is read again in this step
            __builtin_nontemporal_store(xn, reinterpret_cast<double *>(seg + off));
            __builtin_nontemporal_store(xn, xm + i);
            ++nz;
        }
    }
}

template <typename V, int G, int C, int Loss = kLossSquare>
__global__ void __launch_bounds__(kBlock)
k_gather_narrow(char *__restrict__ seg, Layout lay, const typename ValT<V>::T *__restrict__ r,
                double *__restrict__ xm, int32_t *__restrict__ id_slot, typename ValT<V>::T *__restrict__ delta_slot,
                const Ctrl *__restrict__ ctrl, uint64_t *__restrict__ nz_part, uint64_t seed, int64_t tau,
                uint32_t n, double inv_beta, ProxParams pp, SlotPlan plan)
{
    __shared__ uint32_t s_keys[kNiceRounds];
    __shared__ uint64_t s_red[kBlock / 64];
    constexpr int SPW = 64 / G;
    const uint64_t k = ctrl->k;
    const NiceKey key = nice_key_block(seed, k, n, s_keys);
    const SlotDraw sd = slot_draw_for(plan, seed, k);
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const int leader = lane & ~(G - 1);
    uint64_t nz = 0;
    for (int64_t base = wave_global_id() * SPW; base < tau; base += wave_count() * SPW)
        gather_slot_narrow<V, G, C, Loss>(seg, lay, r, xm, id_slot, delta_slot, key, sd, gl, leader, base + lane / G,
                                          tau, inv_beta, pp, nz);
    const uint64_t tot = block_sum_u64(nz, s_red);
    if (threadIdx.x == 0 && tot)
        nz_part[blockIdx.x] += tot;
}

template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_scatter_narrow(const char *__restrict__ seg, Layout lay, typename ValT<V>::T *__restrict__ r,
                 const int32_t *__restrict__ id_slot, const typename ValT<V>::T *__restrict__ delta_slot,
                 Ctrl *__restrict__ ctrl, int64_t tau)
{
    using T = typename ValT<V>::T;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        ctrl->k += 1;  // no block of this kernel reads k
    constexpr int SPW = 64 / G;
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const int leader = lane & ~(G - 1);
    for (int64_t base = wave_global_id() * SPW; base < tau; base += wave_count() * SPW) {
        const int64_t slot = base + lane / G;
        T d = T(0);
        int32_t id = 0;
        if (slot < tau && gl == 0) {
            d = delta_slot[slot];
            id = id_slot[slot];
        }
        d = __shfl(d, leader);
        id = __shfl(id, leader);
        if (!__any(d != T(0)))
            continue;
        int64_t off = 0;
        int32_t dp = 0;
        if (d != T(0))
            locate<V>(lay, id, off, dp);
        const char *rows = seg + off + kHeader;
        for (int e = 4 * gl; e < dp; e += 4 * G) {
            int rw[4];
            T v[4];
            Chunk4<V>::load(rows, dp, e, rw, v);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (v[t] != T(0))
                    atomic_add_hw<T>(r + rw[t], d * v[t]);
        }
    }
}

// --------------------------------------------------------------------------
// Asynchronous variant (the implementation behind the paper's
// billion-variable LASSO timings): no phase boundary inside a launch.  Each
// group of G lanes is a processor that repeatedly picks a block uniformly and
// independently, reads x_i and r, and applies its update to x_i and r at
// once.  The x_i slot of the column record is also the block's lock: a
// processor takes block i by atomically swapping a reserved NaN pattern into
// it (the old value is the current x_i) and releases it by swapping in the
// new value, so acquisition, the read of x_i and its write are atomic
// operations on one address.  A processor whose pick is held by another idles
// for that pick (as when two cores pick the same block).  Only the records
// hold x during the launch: plain stores from several XCDs to one mirror
// entry could land in either order, so the host rebuilds the mirror from the
// records afterwards.
// Each XCD has its own L2, so a plain load of r can return a line cached
// before other XCDs' scatter-adds; how fresh the reads are is the Mode:
// kReadCached (plain loads; the host bounds staleness by ending the launch
// every few rounds), kReadAcquire (the swap that takes a block has acquire
// semantics, which invalidates the caches before the reads), kReadAtomic
// (r read through returning atomics).  Every processor makes a fixed number
// of picks and no lane waits on another, so every wave ends.
//   pick u of call c: i = floor(w n / 2^64), w = SplitMix64 output u of the
//   stream started at kappa_c = SplitMix64 output c of the stream started at
//   seed ^ 0x5043444D4153594E; this launch makes picks u0 .. u0+picks-1, and
//   processor p picks u0 + p, u0 + p + P, ...
// --------------------------------------------------------------------------
constexpr uint64_t kAsyncStream = 0x5043444D4153594Eull;
constexpr uint64_t kHeldBits = 0x7FF4C0DE7FF4C0DEull;  // a NaN: x values are finite

template <typename V, int G, int C, int Mode>
__global__ void __launch_bounds__(kBlock)
k_async(char *__restrict__ seg, Layout lay, typename ValT<V>::T *r, uint64_t *__restrict__ nz_part, uint64_t seed, uint64_t call, int64_t u0, int64_t picks, int64_t procs,
        uint32_t n, double inv_beta, double lam)
{
    using T = typename ValT<V>::T;
    __shared__ uint64_t s_red[kBlock / 64];
    constexpr int GPW = 64 / G;
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const int leader = lane & ~(G - 1);
    const int64_t p = wave_global_id() * GPW + lane / G;
    const uint64_t kappa = splitmix_output(seed ^ kAsyncStream, call);
    const int64_t rounds = (picks + procs - 1) / procs;
    uint64_t nz = 0;
    for (int64_t t = 0; t < rounds; ++t) {
        const int64_t u = t * procs + p;
        int got = 0;
        uint32_t i = 0;
        int64_t off = 0;
        int32_t dp = 0;
        double xi = 0.0, il = 0.0;
        if (gl == 0 && p < procs && u < picks) {
            i = (uint32_t)__umul64hi(splitmix_output(kappa, (uint64_t)(u0 + u)), (uint64_t)n);
            locate<V>(lay, i, off, dp);
            uint64_t *slot = reinterpret_cast<uint64_t *>(seg + off);
            uint64_t old;
            if constexpr (Mode == kReadAcquire)
                old = __hip_atomic_exchange(slot, kHeldBits, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            else
                old = __hip_atomic_exchange(slot, kHeldBits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            got = old != kHeldBits;
            if (got) {
                xi = __longlong_as_double((long long)old);
                il = reinterpret_cast<const double *>(seg + off)[1];
            } else {
                dp = 0;
            }
        }
        off = __shfl(off, leader);
        dp = __shfl(dp, leader);
        const T g = group_sum<G>(lane_dot<V, G, C, Mode>(seg + off + kHeader, dp, gl, r));
        double d = 0.0;
        if (got) {
            const double scale = il * inv_beta;
            const double xn = soft_threshold<double>(xi - (double)g * scale, lam * scale);
            d = xn - xi;
            uint64_t *slot = reinterpret_cast<uint64_t *>(seg + off);
            (void)__hip_atomic_exchange(slot, (uint64_t)__double_as_longlong(xn), __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
            if (d != 0.0)
                ++nz;
        }
        const T dq = (T)__shfl(d, leader);
        if (dq != T(0)) {
            const char *rows = seg + off + kHeader;
            for (int e = 4 * gl; e < dp; e += 4 * G) {
                int rw[4];
                T v[4];
                Chunk4<V>::load(rows, dp, e, rw, v);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (v[q] != T(0))
                        atomic_add_hw<T>(r + rw[q], dq * v[q]);
            }
        }
    }
    const uint64_t tot = block_sum_u64(nz, s_red);
    if (threadIdx.x == 0 && tot)
        nz_part[blockIdx.x] += tot;
}

// The sampler alone (for tests and callers that want S_k).
__global__ void __launch_bounds__(kBlock)
k_sample(uint64_t seed, uint64_t step, int64_t tau, uint32_t n, int mode, double pb, int32_t *__restrict__ out)
{
    __shared__ uint32_t s_keys[kNiceRounds];
    const NiceKey key = nice_key_block(seed, step, n, s_keys);
    SlotPlan plan = plan_nice();
    plan.mode = mode;
    plan.pb = pb;
    const SlotDraw sd = slot_draw_for(plan, seed, step);
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < tau; j += (int64_t)gridDim.x * kBlock) {
        uint32_t i = 0;
        const bool avail = slot_block(sd, key, (uint32_t)j, i);
        out[j] = avail ? (int32_t)i : -1;
    }
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

// r64 += x_i a_i for x_i != 0 (float64 atomics); tiles of 64 consecutive columns.
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_refresh_cols(const char *__restrict__ seg, Layout lay, const double *__restrict__ xm,
               double *__restrict__ r64, int64_t n)
{
    using T = typename ValT<V>::T;
    const TileLanes<G> tl;
    for (int64_t base = wave_global_id() * 64; base < n; base += wave_count() * 64) {
        const int64_t col = base + tl.lane;
        const double xi = col < n ? xm[col] : 0.0;
        const bool live = xi != 0.0;
        if (!__any(live))
            continue;
        int64_t off = 0;
        int32_t dp = 0;
        if (live)
            locate<V>(lay, col, off, dp);
        tile_entries<V, G>(seg, tl, off, dp, xi, [&](int, double xq, int row, T val) {
            if (val != T(0))
                atomic_add_hw<double>(r64 + row, xq * (double)val);
        });
    }
}

// Copy the dense x mirror into the column records (after pcdm_set_x).
template <typename V>
__global__ void __launch_bounds__(kBlock)
k_x_to_records(char *__restrict__ seg, Layout lay, const double *__restrict__ xm, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        int64_t off;
        int32_t dp;
        locate<V>(lay, i, off, dp);
        *reinterpret_cast<double *>(seg + off) = xm[i];
    }
}

// The dense x mirror from the records (after the asynchronous kernel, which
// writes x only in the records).
template <typename V>
__global__ void __launch_bounds__(kBlock)
k_records_to_x(const char *__restrict__ seg, Layout lay, double *__restrict__ xm, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        int64_t off;
        int32_t dp;
        locate<V>(lay, i, off, dp);
        xm[i] = *reinterpret_cast<const double *>(seg + off);
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
__global__ void __launch_bounds__(kBlock)
k_obj_partials(const double *__restrict__ r64, const double *__restrict__ b, const double *__restrict__ xm,
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
        ax += fabs(xm[i]);
    rr = block_sum_f64(rr, lds);
    br = block_sum_f64(br, lds);
    ax = block_sum_f64(ax, lds);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = rr;
        part[3 * blockIdx.x + 1] = br;
        part[3 * blockIdx.x + 2] = ax;
    }
}

// out[c] = sum (mode 0) or max (mode 1) over q of part[ncomp*q + c]; one block.
__global__ void __launch_bounds__(kBlock)
k_final(const double *__restrict__ part, int nparts, int ncomp, int mode, double *__restrict__ out)
{
    __shared__ double lds[kBlock];
    for (int c = 0; c < ncomp; ++c) {
        double a = 0.0;
        for (int q = threadIdx.x; q < nparts; q += kBlock)
            a = mode ? fmax(a, part[ncomp * q + c]) : a + part[ncomp * q + c];
        a = mode ? block_max_f64(a, lds) : block_sum_f64(a, lds);
        if (threadIdx.x == 0)
            out[c] = a;
    }
}

// part[2*blk + {0,1}] = partial sums of phi(r64_j) over rows and of
// Omega(x_i) over columns (outside the box: +inf).
template <int Loss>
__global__ void __launch_bounds__(kBlock)
k_model_partials(const double *__restrict__ r64, int64_t m, const double *__restrict__ xm, int64_t n,
                 ProxParams pp, double *__restrict__ part)
{
    __shared__ double lds[kBlock];
    double fl = 0.0, om = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < m; j += stride)
        fl += phi64<Loss>(r64[j]);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const double t = xm[i];
        om += (t < pp.lo || t > pp.hi) ? HUGE_VAL : pp.l1 * fabs(t) + 0.5 * pp.l2 * t * t + pp.c * t;
    }
    fl = block_sum_f64(fl, lds);
    om = block_sum_f64(om, lds);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x + 0] = fl;
        part[2 * blockIdx.x + 1] = om;
    }
}

// Fold labels into the stored values: every entry of row j (padding
// included) times y[j]; flags labels other than +-1.
template <typename V>
__global__ void __launch_bounds__(kBlock)
k_fold_labels(char *__restrict__ seg, Layout lay, int64_t n, const double *__restrict__ y, Ctrl *__restrict__ ctrl)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        int64_t off;
        int32_t dp;
        locate<V>(lay, i, off, dp);
        const int32_t *rows = reinterpret_cast<const int32_t *>(seg + off + kHeader);
        V *vals = reinterpret_cast<V *>(seg + off + kHeader + 4 * (int64_t)dp);
        for (int32_t e = 0; e < dp; ++e) {
            const double lab = y[rows[e]];
            if (lab == -1.0) {
                if constexpr (sizeof(V) == 2)
                    vals[e].bits ^= 0x8000u;
                else
                    vals[e] = -vals[e];
            } else if (lab != 1.0) {
                atomicOr(&ctrl->err, (uint32_t)ERR_LABEL);
            }
        }
    }
}

// 1/L_i in the record headers times `factor`.
template <typename V>
__global__ void __launch_bounds__(kBlock)
k_scale_invl(char *__restrict__ seg, Layout lay, int64_t n, double factor)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        int64_t off;
        int32_t dp;
        locate<V>(lay, i, off, dp);
        reinterpret_cast<double *>(seg + off)[1] *= factor;
    }
}

// part[blk] = max over the block's columns of |a_i^T r64| (float64 sums);
// tiles of 64 consecutive columns, so the records stream.
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_atr_absmax(const char *__restrict__ seg, Layout lay, const double *__restrict__ r64, int64_t n,
             double *__restrict__ part)
{
    using T = typename ValT<V>::T;
    __shared__ double lds[kBlock];
    const TileLanes<G> tl;
    double best = 0.0;
    for (int64_t base = wave_global_id() * 64; base < n; base += wave_count() * 64) {
        const int64_t col = base + tl.lane;
        int64_t off = 0;
        int32_t dp = 0;
        if (col < n)
            locate<V>(lay, col, off, dp);
        double acc[G];
#pragma unroll
        for (int q = 0; q < G; ++q)
            acc[q] = 0.0;
        tile_entries<V, G>(seg, tl, off, dp, 0, [&](int q, int, int row, T val) {
            acc[q] += (double)val * r64[row];
        });
        double mine = 0.0;
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double s = group_sum<G>(acc[q]);
            const double got = __shfl(s, tl.leader_of_mine(q));
            if (tl.lane / TileLanes<G>::CPR == q)
                mine = got;
        }
        best = fmax(best, fabs(mine));
    }
    best = block_max_f64(best, lds);
    if (threadIdx.x == 0)
        part[blockIdx.x] = best;
}

// ||A^T r||_inf exactly, in two passes, for stored values of at most float32
// precision.  Pass 1 (k_atr_bound) gathers t = fl32(r64), whose rows fit the
// L2 of one XCD where r64 does not, and computes per column v_i = a_i^T t in
// float64 with a bound E_i >= |a_i^T r64 (as the exact pass rounds it) - v_i|;
// it writes ub_i >= |v_i| + E_i (float32, rounded up) and the largest
// |v_i| - E_i.  Pass 2 (k_atr_exact) computes a_i^T r64 exactly as
// k_atr_absmax does, but only for the columns with ub_i >= that lower bound:
// every column attaining the maximum is among them, so the result is the
// same number k_atr_absmax returns.
//
// Bound: t_j = r64_j rounded to nearest, so |r64_j - t_j| <= 2^-24 |t_j| +
// 2^-150 (half an ulp, or half the least subnormal).  With g = sum |a_j t_j|,
// s1 = sum |a_j| over the column's entries and gamma = (entries + 2) 2^-52
// covering the float64 rounding of both passes' sums and of this bound's own
// terms: E = (2^-24 g + 2^-149 s1 + 3 gamma g) (1 + 4 gamma).  A column whose
// bound is not finite (NaN, or r beyond the float32 range) is always a
// candidate.
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_atr_bound(const char *__restrict__ seg, Layout lay, const float *__restrict__ t32, int64_t n,
            float *__restrict__ ub, double *__restrict__ part)
{
    using T = typename ValT<V>::T;
    __shared__ double lds[kBlock];
    const TileLanes<G> tl;
    double best = 0.0;
    for (int64_t base = wave_global_id() * 64; base < n; base += wave_count() * 64) {
        const int64_t col = base + tl.lane;
        int64_t off = 0;
        int32_t dp = 0;
        if (col < n)
            locate<V>(lay, col, off, dp);
        double acc[G], mag[G], s1[G];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            acc[q] = 0.0;
            mag[q] = 0.0;
            s1[q] = 0.0;
        }
        tile_entries<V, G>(seg, tl, off, dp, 0, [&](int q, int, int row, T val) {
            const double pr = (double)val * (double)t32[row];
            acc[q] += pr;
            mag[q] += fabs(pr);
            s1[q] += fabs((double)val);
        });
        double v = 0.0, g = 0.0, a1 = 0.0;
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double sv = group_sum<G>(acc[q]), sg = group_sum<G>(mag[q]), sa = group_sum<G>(s1[q]);
            const int src = tl.leader_of_mine(q);
            const double gv = __shfl(sv, src), gg = __shfl(sg, src), ga = __shfl(sa, src);
            if (tl.lane / TileLanes<G>::CPR == q) {
                v = gv;
                g = gg;
                a1 = ga;
            }
        }
        if (col < n) {
            const double gam = (double)(dp + 2) * 0x1p-52;
            const double E = (0x1p-24 * g + 0x1p-149 * a1 + 3.0 * gam * g) * (1.0 + 4.0 * gam);
            // 2^-50 |v| covers the rounding of these last additions
            const double hi = fabs(v) + E + 0x1p-50 * fabs(v);
            float u = __builtin_inff();  // not finite (r beyond float32 range): always a candidate
            if (hi < 3.0e38) {
                u = (float)hi;
                if ((double)u < hi)
                    u = __int_as_float(__float_as_int(u) + 1);  // next float up (u >= 0, finite)
                best = fmax(best, fabs(v) - E - 0x1p-50 * fabs(v));
            }
            ub[col] = u;
        }
    }
    best = block_max_f64(best, lds);
    if (threadIdx.x == 0)
        part[blockIdx.x] = best;
}

// Pass 2: max over the columns with ub_i >= *lo of |a_i^T r64|, each summed as
// in k_atr_absmax.
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_atr_exact(const char *__restrict__ seg, Layout lay, const double *__restrict__ r64, int64_t n,
            const float *__restrict__ ub, const double *__restrict__ lo, double *__restrict__ part)
{
    using T = typename ValT<V>::T;
    __shared__ double lds[kBlock];
    const TileLanes<G> tl;
    const double thr = *lo;
    double best = 0.0;
    for (int64_t base = wave_global_id() * 64; base < n; base += wave_count() * 64) {
        const int64_t col = base + tl.lane;
        const bool cand = col < n && (double)ub[col] >= thr;
        if (!__any(cand))
            continue;
        int64_t off = 0;
        int32_t dp = 0;
        if (cand)
            locate<V>(lay, col, off, dp);
        double acc[G];
#pragma unroll
        for (int q = 0; q < G; ++q)
            acc[q] = 0.0;
        tile_entries<V, G>(seg, tl, off, dp, 0, [&](int q, int, int row, T val) {
            acc[q] += (double)val * r64[row];
        });
        double mine = 0.0;
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double s = group_sum<G>(acc[q]);
            const double got = __shfl(s, tl.leader_of_mine(q));
            if (tl.lane / TileLanes<G>::CPR == q)
                mine = got;
        }
        if (cand)
            best = fmax(best, fabs(mine));
    }
    best = block_max_f64(best, lds);
    if (threadIdx.x == 0)
        part[blockIdx.x] = best;
}

// Incremental route between two evaluations of ||A^T r||_inf (float32 /
// bf16 values).  Kept from the last evaluation: r_old (the r64 it used),
// ub_i >= |a_i^T r_old| as the exact pass sums it, for every column, and its
// result M_old.  For the new r64, Hoelder's inequality gives
//     |a_i^T r_new| <= |a_i^T r_old| + ||a_i||_1 ||r_new - r_old||_inf,
// so with D = ||r_new - r_old||_inf + 2 gamma max(||r_old||_inf,
// ||r_new||_inf) (gamma = (d_max + 2) 2^-52 covers the rounding of both exact
// sums, each within gamma ||a_i||_1 ||r||_inf) every column's exact sum is at
// most ub_i + ||a_i||_1 D, and the new maximum is at least
// M_old - max_i ||a_i||_1 D (the old maximiser moved by at most that).  Only
// the columns whose bound reaches that lower bound are summed exactly; the
// bounds of the others grow by ||a_i||_1 D.  The result is the single pass's.
//
// inc[0] = M_old, inc[1..3] = max |r - r_old|, max |r|, max |r_old|,
// inc[4] = D, inc[5] = the lower bound.

// part[3 * blk + {0,1,2}] = the block's max |r - ro|, max |r|, max |ro|
// (r: the float64 residual now, ro: the one of the last evaluation).
__global__ void __launch_bounds__(kBlock)
k_inc_sums(const double *__restrict__ r, const double *__restrict__ ro, int64_t m, double *__restrict__ part)
{
    __shared__ double lds[kBlock];
    double dd = 0.0, rr = 0.0, oo = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < m; j += (int64_t)gridDim.x * kBlock) {
        const double a = r[j], o = ro[j];
        dd = fmax(dd, fabs(a - o));
        rr = fmax(rr, fabs(a));
        oo = fmax(oo, fabs(o));
    }
    dd = block_max_f64(dd, lds);
    rr = block_max_f64(rr, lds);
    oo = block_max_f64(oo, lds);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = dd;
        part[3 * blockIdx.x + 1] = rr;
        part[3 * blockIdx.x + 2] = oo;
    }
}

// One thread: D and the lower bound from the maxima.  The computed sum of
// column i at r is within gam ||a_i||_1 ||r||_inf of a_i^T r (float64
// summation of at most d products), and |a_i^T (r - ro)| <= ||a_i||_1
// ||r - ro||_inf (Hoelder), so the computed sums move by at most
// ||a_i||_1 D with D = ||r - ro||_inf + 2 gam max(||r||_inf, ||ro||_inf);
// |fl(a - o)| understates |a - o| by at most a relative 2^-53.
__global__ void k_inc_prepare(double *__restrict__ inc, double nrm_max, double gam)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    const double D = inc_shift(inc[1], fmax(inc[2], inc[3]), gam);
    inc[4] = D;
    inc[5] = inc_lower(inc[0], nrm_max, D);
}

__device__ __forceinline__ float round_up_f32(double v)
{
    if (!(v < 3.0e38))
        return __builtin_inff();
    float u = (float)v;
    if ((double)u < v)
        u = __int_as_float(__float_as_int(u) + 1);  // next float up (v >= 0)
    return u;
}

// *cnt += the number of columns whose bound reaches the lower bound.
__global__ void __launch_bounds__(kBlock)
k_inc_count(const float *__restrict__ ub, const float *__restrict__ nrm, int64_t n, const double *__restrict__ inc,
            unsigned long long *__restrict__ cnt)
{
    __shared__ uint64_t s_red[kBlock / 64];
    const double D = inc[4], lo = inc[5];
    uint64_t c = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        c += !(inc_moved((double)ub[i], (double)nrm[i], D) < lo);
    c = block_sum_u64(c, s_red);
    if (threadIdx.x == 0 && c)
        atomicAdd(cnt, (unsigned long long)c);
}

// The candidates' exact sums (as k_atr_absmax forms them) and their maximum;
// ub_i becomes the exact value (rounded up) for a candidate and
// ub_i + ||a_i|| D (rounded up) for the others.
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_atr_inc(const char *__restrict__ seg, Layout lay, const double *__restrict__ r64, int64_t n,
          float *__restrict__ ub, const float *__restrict__ nrm, const double *__restrict__ inc,
          double *__restrict__ part)
{
    using T = typename ValT<V>::T;
    __shared__ double lds[kBlock];
    const TileLanes<G> tl;
    const double D = inc[4], lo = inc[5];
    double best = 0.0;
    for (int64_t base = wave_global_id() * 64; base < n; base += wave_count() * 64) {
        const int64_t col = base + tl.lane;
        double bnd = 0.0;
        bool cand = false;
        if (col < n) {
            bnd = inc_moved((double)ub[col], (double)nrm[col], D);
            cand = !(bnd < lo);
        }
        if (__any(cand)) {
            int64_t off = 0;
            int32_t dp = 0;
            if (cand)
                locate<V>(lay, col, off, dp);
            double acc[G];
#pragma unroll
            for (int q = 0; q < G; ++q)
                acc[q] = 0.0;
            tile_entries<V, G>(seg, tl, off, dp, 0, [&](int q, int, int row, T val) {
                acc[q] += (double)val * r64[row];
            });
            double mine = 0.0;
#pragma unroll
            for (int q = 0; q < G; ++q) {
                const double s = group_sum<G>(acc[q]);
                const double got = __shfl(s, tl.leader_of_mine(q));
                if (tl.lane / TileLanes<G>::CPR == q)
                    mine = got;
            }
            if (cand) {
                best = fmax(best, fabs(mine));
                bnd = fabs(mine);
            }
        }
        if (col < n)
            ub[col] = round_up_f32(bnd);
    }
    best = block_max_f64(best, lds);
    if (threadIdx.x == 0)
        part[blockIdx.x] = best;
}

// nrm_i >= ||a_i||_1 (float32, rounded up; `fac` covers the float64
// summation), part[blk] = the block's max.
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_col_norms(const char *__restrict__ seg, Layout lay, int64_t n, double fac, float *__restrict__ nrm,
            double *__restrict__ part)
{
    using T = typename ValT<V>::T;
    __shared__ double lds[kBlock];
    const TileLanes<G> tl;
    double best = 0.0;
    for (int64_t base = wave_global_id() * 64; base < n; base += wave_count() * 64) {
        const int64_t col = base + tl.lane;
        int64_t off = 0;
        int32_t dp = 0;
        if (col < n)
            locate<V>(lay, col, off, dp);
        double acc[G];
#pragma unroll
        for (int q = 0; q < G; ++q)
            acc[q] = 0.0;
        tile_entries<V, G>(seg, tl, off, dp, 0, [&](int q, int, int, T val) { acc[q] += fabs((double)val); });
        double mine = 0.0;
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double s = group_sum<G>(acc[q]);
            const double got = __shfl(s, tl.leader_of_mine(q));
            if (tl.lane / TileLanes<G>::CPR == q)
                mine = got;
        }
        if (col < n) {
            const float u = round_up_f32(mine * fac);
            nrm[col] = u;
            best = fmax(best, (double)u);
        }
    }
    best = block_max_f64(best, lds);
    if (threadIdx.x == 0)
        part[blockIdx.x] = best;
}

__global__ void k_copy_f64(const double *__restrict__ src, double *__restrict__ dst, int64_t len)
{
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < len; j += (int64_t)gridDim.x * kBlock)
        dst[j] = src[j];
}

// --------------------------------------------------------------------------
// Set-up: validation and packing into the record layout.
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

// Flags columns whose padded length differs from column 0's.
__global__ void __launch_bounds__(kBlock)
k_check_uniform(const int64_t *__restrict__ dpad, int64_t n, Ctrl *__restrict__ ctrl)
{
    const int64_t d0 = dpad[0];
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        if (dpad[i] != d0)
            ctrl->nonuniform = 1u;
}

__device__ __forceinline__ bool finite_val(float v) { return isfinite(v); }
__device__ __forceinline__ bool finite_val(double v) { return isfinite(v); }
__device__ __forceinline__ bool finite_val(bf16s v) { return ((v.bits >> 7) & 0xFF) != 0xFF; }

// Copy column i into its record (x_i = 0, 1/L_i from float64 sums of the
// stored values); row histogram of the nonzeros (for omega).
template <typename V>
__global__ void __launch_bounds__(kBlock)
k_pack(const int64_t *__restrict__ col_ptr, const int32_t *__restrict__ row_idx, const V *__restrict__ val,
       Layout lay, int64_t n, int64_t m, char *__restrict__ seg, int32_t *__restrict__ hist,
       Ctrl *__restrict__ ctrl)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const int64_t a = col_ptr[i], b = col_ptr[i + 1];
        int64_t off;
        int32_t dpad;
        locate<V>(lay, i, off, dpad);
        if (b <= a || dpad < b - a)
            continue;  // flagged by k_check_ptr
        double *hdr = reinterpret_cast<double *>(seg + off);
        int32_t *rows = reinterpret_cast<int32_t *>(seg + off + kHeader);
        V *vals = reinterpret_cast<V *>(seg + off + kHeader + 4 * (int64_t)dpad);
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
            if constexpr (sizeof(V) == 2)
                z.bits = 0;
            else
                z = V(0);
            vals[p] = z;
        }
        if (!(L > 0.0))
            err |= ERR_ZEROCOL;
        hdr[0] = 0.0;
        hdr[1] = L > 0.0 ? 1.0 / L : 0.0;
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

// Sum of the per-block counters of nonzero updates.
__global__ void __launch_bounds__(kBlock)
k_sum_u64(const uint64_t *__restrict__ part, int nparts, Ctrl *__restrict__ ctrl)
{
    __shared__ uint64_t lds[kBlock / 64];
    uint64_t s = 0;
    for (int q = threadIdx.x; q < nparts; q += kBlock)
        s += part[q];
    s = block_sum_u64(s, lds);
    if (threadIdx.x == 0)
        ctrl->imax = (int64_t)s;
}

// --------------------------------------------------------------------------
// Adjoint: PCDM on q(v) = 0.5 ||A_S v||^2 - g^T v over the active set S
// (lambda = 0), with rho = A_S v kept in float64.  Coordinate c of the
// sub-problem is column S[c].  Same sampler and tile reads as the step.
// --------------------------------------------------------------------------

// flags[i] = (x_i != 0)
__global__ void __launch_bounds__(kBlock)
k_flag_nonzero(const double *__restrict__ xm, int64_t n, uint8_t *__restrict__ flags)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        flags[i] = xm[i] != 0.0;
}

// gS[c] = g[S[c]]
__global__ void __launch_bounds__(kBlock)
k_gather_g(const int32_t *__restrict__ S, const double *__restrict__ g, int64_t ns, double *__restrict__ gS)
{
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < ns; c += (int64_t)gridDim.x * kBlock)
        gS[c] = g[S[c]];
}

// Row histogram of the nonzeros of the columns in S (omega of the sub-problem).
template <typename V>
__global__ void __launch_bounds__(kBlock)
k_adj_hist(const char *__restrict__ seg, Layout lay, const int32_t *__restrict__ S, int64_t ns,
           int32_t *__restrict__ hist)
{
    using T = typename ValT<V>::T;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < ns; c += (int64_t)gridDim.x * kBlock) {
        int64_t off;
        int32_t dp;
        locate<V>(lay, S[c], off, dp);
        const char *rows = seg + off + kHeader;
        for (int e = 0; e < dp; e += 4) {
            int rw[4];
            T v[4];
            Chunk4<V>::load(rows, dp, e, rw, v);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (v[t] != T(0))
                    atomicAdd(hist + rw[t], 1);
        }
    }
}

// Phase 1 of an adjoint step: slot j takes c = pi(j) over [0, ns), column
// S[c], partial derivative h = a^T rho - g_c, and v_c -= h / (beta_S L).
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_adj_gather(const char *__restrict__ seg, Layout lay, const int32_t *__restrict__ S,
             const double *__restrict__ gS, double *__restrict__ vS, const double *__restrict__ rho,
             int32_t *__restrict__ id_slot, double *__restrict__ delta_slot, uint64_t seed, uint64_t step,
             int64_t tau, uint32_t ns, double inv_beta)
{
    using T = typename ValT<V>::T;
    __shared__ uint32_t s_keys[kNiceRounds];
    const NiceKey key = nice_key_block(seed, step, ns, s_keys);
    const TileLanes<G> tl;
    for (int64_t base = wave_global_id() * 64; base < tau; base += wave_count() * 64) {
        const int64_t slot = base + tl.lane;
        const bool act = slot < tau;
        uint32_t c = 0;
        int32_t col = 0;
        int64_t off = 0;
        int32_t dp = 0;
        double il = 0.0;
        if (act) {
            c = nice_slot((uint32_t)slot, key);
            col = S[c];
            locate<V>(lay, col, off, dp);
            il = reinterpret_cast<const double *>(seg + off)[1];
        }
        double acc[G];
#pragma unroll
        for (int q = 0; q < G; ++q)
            acc[q] = 0.0;
        tile_entries<V, G>(seg, tl, off, dp, 0, [&](int q, int, int row, T val) {
            acc[q] += (double)val * rho[row];
        });
        double mine = 0.0;
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double s = group_sum<G>(acc[q]);
            const double got = __shfl(s, tl.leader_of_mine(q));
            if (tl.lane / TileLanes<G>::CPR == q)
                mine = got;
        }
        if (act) {
            const double d = -(mine - gS[c]) * il * inv_beta;
            vS[c] += d;
            id_slot[slot] = col;
            delta_slot[slot] = d;
        }
    }
}

// Phase 2 of an adjoint step: rho += delta a_col (float64 atomics).
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_adj_scatter(const char *__restrict__ seg, Layout lay, double *__restrict__ rho,
              const int32_t *__restrict__ id_slot, const double *__restrict__ delta_slot, int64_t tau)
{
    using T = typename ValT<V>::T;
    const TileLanes<G> tl;
    for (int64_t base = wave_global_id() * 64; base < tau; base += wave_count() * 64) {
        const int64_t slot = base + tl.lane;
        const double d = slot < tau ? delta_slot[slot] : 0.0;
        const bool live = d != 0.0;
        if (!__any(live))
            continue;
        int64_t off = 0;
        int32_t dp = 0;
        if (live)
            locate<V>(lay, id_slot[slot], off, dp);
        tile_entries<V, G>(seg, tl, off, dp, d, [&](int, double dq, int row, T val) {
            if (val != T(0))
                atomic_add_hw<double>(rho + row, dq * (double)val);
        });
    }
}

// rho += v_c a_{S[c]} over all c (rho zeroed before): float64 A_S v.
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_adj_apply(const char *__restrict__ seg, Layout lay, const int32_t *__restrict__ S,
            const double *__restrict__ vS, double *__restrict__ rho, int64_t ns)
{
    using T = typename ValT<V>::T;
    const TileLanes<G> tl;
    for (int64_t base = wave_global_id() * 64; base < ns; base += wave_count() * 64) {
        const int64_t c = base + tl.lane;
        const double w = c < ns ? vS[c] : 0.0;
        const bool live = w != 0.0;
        if (!__any(live))
            continue;
        int64_t off = 0;
        int32_t dp = 0;
        if (live)
            locate<V>(lay, S[c], off, dp);
        tile_entries<V, G>(seg, tl, off, dp, w, [&](int, double wq, int row, T val) {
            if (val != T(0))
                atomic_add_hw<double>(rho + row, wq * (double)val);
        });
    }
}

// part[blk] = max_c |a_{S[c]}^T rho - g_c| (residual of A_S^T A_S v = g).
template <typename V, int G>
__global__ void __launch_bounds__(kBlock)
k_adj_resid(const char *__restrict__ seg, Layout lay, const int32_t *__restrict__ S,
            const double *__restrict__ gS, const double *__restrict__ rho, int64_t ns, double *__restrict__ part)
{
    using T = typename ValT<V>::T;
    __shared__ double lds[kBlock];
    const TileLanes<G> tl;
    double best = 0.0;
    for (int64_t base = wave_global_id() * 64; base < ns; base += wave_count() * 64) {
        const int64_t c = base + tl.lane;
        int64_t off = 0;
        int32_t dp = 0;
        if (c < ns)
            locate<V>(lay, S[c], off, dp);
        double acc[G];
#pragma unroll
        for (int q = 0; q < G; ++q)
            acc[q] = 0.0;
        tile_entries<V, G>(seg, tl, off, dp, 0, [&](int q, int, int row, T val) {
            acc[q] += (double)val * rho[row];
        });
        double mine = 0.0;
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double s = group_sum<G>(acc[q]);
            const double got = __shfl(s, tl.leader_of_mine(q));
            if (tl.lane / TileLanes<G>::CPR == q)
                mine = got;
        }
        if (c < ns)
            best = fmax(best, fabs(mine - gS[c]));
    }
    best = block_max_f64(best, lds);
    if (threadIdx.x == 0)
        part[blockIdx.x] = best;
}

// part[3*blk] = partial sum of -sign(x_{S[c]}) v_c, part[3*blk+1] = max |g_c|.
__global__ void __launch_bounds__(kBlock)
k_adj_lambda(const int32_t *__restrict__ S, const double *__restrict__ xm, const double *__restrict__ vS,
             const double *__restrict__ gS, int64_t ns, double *__restrict__ part)
{
    __shared__ double lds[kBlock];
    double s = 0.0, gm = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < ns; c += (int64_t)gridDim.x * kBlock) {
        const double xv = xm[S[c]];
        s -= (xv > 0.0 ? 1.0 : -1.0) * vS[c];
        gm = fmax(gm, fabs(gS[c]));
    }
    s = block_sum_f64(s, lds);
    gm = block_max_f64(gm, lds);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = s;
        part[3 * blockIdx.x + 1] = gm;
        part[3 * blockIdx.x + 2] = 0.0;
    }
}

}  // namespace pcdm
