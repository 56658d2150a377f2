// binned_kernels.hpp -- the partial derivatives of a step taken by rows: a
// route for residuals far larger than the caches.
//
// The plain gather reads, for every sampled coordinate i, r at the rows of
// column i.  With r of hundreds of MB and S_k drawn uniformly, those reads
// land on random 128-byte lines, each fetched from HBM for one 4-byte value,
// although a large step touches most lines of r several times.  Here the
// step's entries are first regrouped by row, so r is read window by window
// and every line serves all the entries of the step that fall in it:
//
//   k_bin      (one workgroup of 1024 threads per 1024 consecutive slots,
//              taken in two halves of 512): draws the slots'
//              coordinates (tau-nice, as the plain gather), keeps x_i and
//              1/L_i of each slot, and deals the column entries into
//              sub-bins keyed by (row range, row window), in LDS first and
//              then as contiguous runs in the workgroup's own part of `bins`;
//   k_bin_dot  (one workgroup per (row range, block of 16384 slots)): walks
//              the windows of its row range in order, reading its slots'
//              entries from the sub-bins, r at their rows, and summing
//              value * r into per-slot LDS accumulators; writes one partial
//              derivative per (row range, slot);
//   k_bin_prox (one lane per slot): adds the partials of the row ranges and
//              takes the update as the plain gather does.
//
// Row ranges are eight, one per XCD: workgroup b of k_bin_dot takes range
// b mod 8, the XCD it is dispatched to (workgroups are dealt to the XCDs in
// turn; checked on the device with the XCC id register), so the workgroups
// of one XCD share their windows through that XCD's L2 while the others read
// other rows.
// The sum g_i = a_i^T r is the same as the plain gather's up to the order of
// the float32 additions.
//
// Sub-bins have a fixed capacity (a few standard deviations above the mean
// count of a uniform matrix).  A step in which any sub-bin overflows sets a
// flag that k_bin_prox reads: it then computes that step by the plain gather
// instead, so the result never depends on the capacity.
#pragma once

#include "kernels.hpp"

namespace pcdm {

constexpr int kBinRanges = 8;
constexpr int kBinWinBits = 18;  // window = 2^18 rows (1 MB of float32 r)
constexpr uint32_t kBinWinMask = (1u << kBinWinBits) - 1u;
constexpr int kBinBlockBits = 14;  // k_bin_dot: 2^14 slots per workgroup
constexpr int kBinBlock = 1 << kBinBlockBits;
constexpr int kBinSlotsA = 1024;  // k_bin: slots per workgroup
constexpr int kBinHalf = 512;     // k_bin: slots staged at once
constexpr int kBinThreads = 1024; // k_bin: threads
constexpr int kBinColsPerWave = kBinHalf / (kBinThreads / 64);  // columns a wave reads per half
constexpr int kBinRounds = kBinColsPerWave / 8;                 // 8 columns per round
constexpr int kBinDotThreads = 512;
constexpr int kBinMaxDpad = 32;   // one 4-entry chunk per lane of an 8-lane group
constexpr int kBinMaxSub = 1024;  // sub-bins per k_bin workgroup (8 ranges x windows)
static_assert(kBinWinBits + kBinBlockBits == 32, "key = slot in block | row in window");
static_assert(kBinBlock % kBinSlotsA == 0, "a k_bin workgroup feeds one k_bin_dot block");
static_assert(kBinColsPerWave % 8 == 0 && kBinColsPerWave <= 64, "whole rounds of 8 columns, owners in one wave");

struct BinGeom {
    int64_t rx;    // rows per range, ceil(m / 8)
    int32_t nw;    // windows per range
    int32_t ns;    // sub-bins per k_bin workgroup: 8 * nw
    int32_t cap;   // entries per sub-bin
    int32_t dpad;  // entries per record (fixed-length records)
};

struct BinEntry {
    uint32_t key;  // slot within its k_bin_dot block << 18 | row within its window
    float val;
};

// Dynamic LDS of k_bin: four counters per sub-bin, then per staged entry its
// key and value (one 8-byte pair), sub-bin and a sorted-order index.
__host__ __device__ inline size_t bin_lds_bytes(int ns, int dpad)
{
    return (size_t)4 * ns * sizeof(int32_t) + (size_t)kBinHalf * dpad * (4 + 4 + 2 + 2);
}

// Exclusive prefix sum of v[0..cnt) (cnt <= 2 * blockDim.x, blockDim.x a
// multiple of 64 and at most 1024) into out[]; `wtot` holds one int per wave.
__device__ __forceinline__ void block_exclusive_scan(const int32_t *v, int32_t *out, int cnt, int32_t *wtot)
{
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int i0 = 2 * t, i1 = 2 * t + 1;
    const int32_t a = i0 < cnt ? v[i0] : 0;
    const int32_t b = i1 < cnt ? v[i1] : 0;
    int32_t s = a + b, inc = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(inc, o, 64);
        if (lane >= o)
            inc += y;
    }
    if (lane == 63)
        wtot[w] = inc;
    __syncthreads();
    int32_t before = 0;
    for (int q = 0; q < w; ++q)
        before += wtot[q];
    const int32_t ex = before + inc - s;
    if (i0 < cnt)
        out[i0] = ex;
    if (i1 < cnt)
        out[i1] = ex + a;
    __syncthreads();
}

// In-place exclusive prefix sum of v[0..cnt) for cnt <= 4 * blockDim.x
// (blockDim.x a multiple of 64, at most 1024): thread t sums a contiguous
// quarter-run of the array; returns the total.  `wtot` holds one int per wave.
__device__ __forceinline__ int32_t block_exclusive_scan4(int32_t *v, int cnt, int32_t *wtot)
{
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6, nwv = (int)(blockDim.x >> 6);
    const int per = (cnt + (int)blockDim.x - 1) / (int)blockDim.x;  // <= 4
    const int b0 = t * per;
    int32_t loc[4] = {0, 0, 0, 0};
    int32_t s = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (u < per && b0 + u < cnt) {
            loc[u] = v[b0 + u];
            s += loc[u];
        }
    int32_t inc = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(inc, o, 64);
        if (lane >= o)
            inc += y;
    }
    if (lane == 63)
        wtot[w] = inc;
    __syncthreads();
    int32_t before = 0, total = 0;
    for (int q = 0; q < nwv; ++q) {
        if (q < w)
            before += wtot[q];
        total += wtot[q];
    }
    int32_t run = before + inc - s;
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (u < per && b0 + u < cnt) {
            v[b0 + u] = run;
            run += loc[u];
        }
    __syncthreads();
    return total;
}

// Binning: workgroup a takes slots [1024 a, 1024 a + 1024) of step k in two
// halves of 512.  Writes id_slot, hdr (x_i, 1/L_i) per slot, the runs of its
// sub-bins and their counts; sets over[k & 1] if a sub-bin overflows.  The
// entries of the second half are loaded (into the registers the first half's
// entries have left) before the first half is sorted and written, so their
// HBM latency overlaps that work.
template <typename V>
__global__ void __launch_bounds__(kBinThreads)
k_bin(const char *__restrict__ seg, Layout lay, BinGeom geo, const Ctrl *__restrict__ ctrl, uint64_t seed,
      int64_t tau, uint32_t n, int32_t *__restrict__ id_slot, v2d_t *__restrict__ hdr,
      BinEntry *__restrict__ bins, int32_t *__restrict__ counts, uint32_t *__restrict__ over)
{
    using VT = typename ValT<V>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_keys[kNiceRounds];
    __shared__ int32_t s_wtot[kBinThreads / 64];
    const int ns = geo.ns, dpad = geo.dpad;
    const int nstage = kBinHalf * dpad;
    int32_t *cnt = reinterpret_cast<int32_t *>(smem);
    int32_t *offs = cnt + ns;
    int32_t *fill = offs + ns;
    int32_t *run = fill + ns;
    uint2 *stkv = reinterpret_cast<uint2 *>(run + ns);  // (key, value bits) of each staged entry
    uint16_t *stsub = reinterpret_cast<uint16_t *>(stkv + nstage);
    uint16_t *order = stsub + nstage;

    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6, gl = lane & 7, grp = lane >> 3;
    const int e = 4 * gl;  // this lane's 4-entry chunk of each column it reads
    const int64_t na = (tau + kBinSlotsA - 1) / kBinSlotsA;  // chunks of 1024 slots
    for (int q = t; q < ns; q += kBinThreads) {
        cnt[q] = 0;
        fill[q] = 0;
        run[q] = 0;
    }
    const uint64_t k = ctrl->k;
    const NiceKey key = nice_key_block(seed, k, n, s_keys);  // synchronises the block

    // entries of one half: wave w reads the columns of slots
    // [w * kBinColsPerWave, (w + 1) * kBinColsPerWave) of the half, whose
    // coordinates lanes 0..kBinColsPerWave-1 draw; in round q the 8 lanes of
    // group grp read column q * 8 + grp of the wave, one 4-entry chunk each
    // (dpad <= 32).  The loads are unconditional (an idle lane reads column
    // 0's first chunk, always present, and ignores it): loads under a branch
    // would make the compiler wait for each round's data before issuing the
    // next round.
    int rw[kBinRounds][4];
    VT v[kBinRounds][4];
    bool cact[kBinRounds];
    bool hact = false;
    int64_t hslot = 0;
    uint32_t hid = 0;
    v2d_t hv;
    auto load_half = [&](int64_t ca, int h) {
        hslot = ca * kBinSlotsA + (int64_t)h * kBinHalf + w * kBinColsPerWave + lane;
        hact = lane < kBinColsPerWave && hslot < tau;
        int64_t off = 0;
        hid = 0;
        if (hact) {
            hid = nice_slot((uint32_t)hslot, key);
            off = (int64_t)hid * lay.stride;
        }
        hv = ld_rec(reinterpret_cast<const v2d_t *>(seg + off));
        const int el = e < dpad ? e : 0;
#pragma unroll
        for (int q = 0; q < kBinRounds; ++q) {
            const int o = q * 8 + grp;
            const int64_t coff = __shfl(off, o);
            cact[q] = __shfl((int)hact, o) != 0 && e < dpad;
            Chunk4<V>::load(seg + coff + kHeader, dpad, el, rw[q], v[q]);
        }
    };
    // the slot's coordinate and record header, stored once the half's loads
    // are all in flight
    auto store_half = [&]() {
        if (hact) {
            id_slot[hslot] = (int32_t)hid;
            hdr[hslot] = hv;
        }
    };

    bool overflow = false;
    const double inv_rx = 1.0 / (double)geo.rx;
    // workgroup blockIdx.x takes chunks blockIdx.x, + gridDim.x, ... (the
    // grid is one workgroup per CU, which is all the LDS allows); the first
    // half of its next chunk is loaded while the second half of this one is
    // sorted and written
    int64_t a = blockIdx.x;
    if (a < na)
        load_half(a, 0);
    for (; a < na; a += gridDim.x) {
        // unrolled: the second half's loads land in the registers its staging
        // reads, with no copies across a loop edge that would wait for them
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            store_half();
            // stage this half's entries in LDS, keyed and counted by sub-bin
#pragma unroll
            for (int q = 0; q < kBinRounds; ++q) {
                const int sl = w * kBinColsPerWave + q * 8 + grp;  // staged column within the half
                if (e < dpad) {
                    // slot of column sl within its k_bin_dot block
                    const uint32_t sblk =
                        (uint32_t)(((a * kBinSlotsA + (int64_t)h * kBinHalf + sl)) & (int64_t)(kBinBlock - 1));
                    uint32_t kk[4];
                    float vv[4];
                    uint16_t ss[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        kk[u] = 0u;
                        vv[u] = 0.0f;
                        ss[u] = 0xFFFFu;
                        if (cact[q] && v[q][u] != VT(0)) {
                            const uint32_t row = (uint32_t)rw[q][u];
                            // row range xr = floor(row / rx): the float64 quotient is
                            // within one of it, and one comparison each way fixes it
                            uint32_t xr = (uint32_t)((double)row * inv_rx);
                            int64_t lo = (int64_t)xr * geo.rx;
                            if (lo > (int64_t)row) {
                                xr -= 1u;
                                lo -= geo.rx;
                            } else if (lo + geo.rx <= (int64_t)row) {
                                xr += 1u;
                                lo += geo.rx;
                            }
                            const uint32_t within = row - (uint32_t)lo;
                            const int sub = (int)(xr * (uint32_t)geo.nw + (within >> kBinWinBits));
                            kk[u] = (sblk << kBinWinBits) | (within & kBinWinMask);
                            vv[u] = (float)v[q][u];
                            ss[u] = (uint16_t)sub;
                            atomicAdd(&cnt[sub], 1);
                        }
                    }
                    // two 16-byte LDS stores of (key, value) pairs and one 8-byte
                    // store of sub-bins: padded column lengths are multiples of 4,
                    // so idx is too
                    const int idx = sl * dpad + e;
                    *reinterpret_cast<uint4 *>(stkv + idx) =
                        make_uint4(kk[0], __float_as_uint(vv[0]), kk[1], __float_as_uint(vv[1]));
                    *reinterpret_cast<uint4 *>(stkv + idx + 2) =
                        make_uint4(kk[2], __float_as_uint(vv[2]), kk[3], __float_as_uint(vv[3]));
                    *reinterpret_cast<ushort4 *>(stsub + idx) = make_ushort4(ss[0], ss[1], ss[2], ss[3]);
                }
            }
            if (h == 0)
                load_half(a, 1);  // in flight while this half is sorted and written
            else if (a + gridDim.x < na)
                load_half(a + gridDim.x, 0);  // the next chunk's first half, likewise
            __syncthreads();
            block_exclusive_scan(cnt, offs, ns, s_wtot);  // ends with a barrier
            const int nvalid = offs[ns - 1] + cnt[ns - 1];
            for (int idx = t; idx < nstage; idx += kBinThreads) {
                const uint16_t sub = stsub[idx];
                if (sub != 0xFFFFu)
                    order[offs[sub] + atomicAdd(&fill[sub], 1)] = (uint16_t)idx;
            }
            __syncthreads();
            // offs[q] becomes the place in the sub-bin's run of sorted position 0
            for (int q = t; q < ns; q += kBinThreads)
                offs[q] = run[q] - offs[q];
            __syncthreads();
            for (int j = t; j < nvalid; j += kBinThreads) {
                const int idx = order[j];
                const int sub = stsub[idx];
                const int pos = offs[sub] + j;
                if (pos < geo.cap) {
                    const uint2 kv = stkv[idx];
                    BinEntry be;
                    be.key = kv.x;
                    be.val = __uint_as_float(kv.y);
                    bins[((int64_t)a * ns + sub) * geo.cap + pos] = be;
                } else {
                    overflow = true;
                }
            }
            __syncthreads();
            for (int q = t; q < ns; q += kBinThreads) {
                run[q] += cnt[q];
                cnt[q] = 0;
                fill[q] = 0;
            }
            __syncthreads();
        }
        for (int q = t; q < ns; q += kBinThreads) {
            counts[a * ns + q] = run[q] < geo.cap ? run[q] : geo.cap;
            run[q] = 0;  // cnt and fill are already cleared
        }
    }
    if (overflow)
        atomicOr(over + (k & 1), 1u);
}

// Per (row range xr = blockIdx.x mod 8, slot block c = blockIdx.x / 8): the
// range's part of g for the block's slots.  The block's sub-bin runs are
// taken in window-major order (window tw, then the 16 k_bin workgroups of the
// block) as one flat list of entries, 512 at a time (one per thread): every
// block of a range then moves through the range's rows at the same pace, so
// the rows in use at any moment (about 1.3 MB for the 64 blocks of an XCD)
// stay in that XCD's L2.  (Measured on the 2e8-row instance: 1024 entries
// per block at a time, or two windows per stage taken by each wave on its
// own, let the blocks drift apart and L2 misses rose from 8.0e6 to
// 1.3e7-1.6e7 per launch.)
constexpr int kBinPerBlock = kBinBlock / kBinSlotsA;  // k_bin workgroups per block (16)
constexpr int kBinMaxRuns = (kBinMaxSub / kBinRanges) * kBinPerBlock;

// Entry j of the block's flat list (j < pre[nruns]): its bin entry and the
// first row of its window.
__device__ __forceinline__ void bin_flat_entry(const BinEntry *__restrict__ bins, const int32_t *pre, int nruns,
                                               const BinGeom &geo, int xr, int64_t a0, int32_t j, BinEntry &be,
                                               uint32_t &rowb)
{
    // the run holding j: the last q with pre[q] <= j
    int lo = 0, hi = nruns;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= j)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int tw = lo / kBinPerBlock;
    const int64_t sb = (a0 + (lo % kBinPerBlock)) * geo.ns + (int64_t)xr * geo.nw + tw;
    // entries are read once: keep them out of L2, which holds the rows of r
    const uint64_t raw =
        __builtin_nontemporal_load(reinterpret_cast<const uint64_t *>(bins + sb * geo.cap + (j - pre[lo])));
    be.key = (uint32_t)raw;
    be.val = __uint_as_float((uint32_t)(raw >> 32));
    rowb = (uint32_t)((int64_t)xr * geo.rx + ((int64_t)tw << kBinWinBits));
}

template <typename T>
__global__ void __launch_bounds__(kBinDotThreads)
k_bin_dot(const BinEntry *__restrict__ bins, const int32_t *__restrict__ counts, const T *__restrict__ r,
          BinGeom geo, int64_t tau, int64_t na, T *__restrict__ partial)
{
    __shared__ float acc[kBinBlock];
    __shared__ int32_t pre[kBinMaxRuns + 1];
    __shared__ int32_t s_wtot[kBinDotThreads / 64];
    const int t = threadIdx.x;
    const int xr = (int)(blockIdx.x % kBinRanges);
    const int64_t c = blockIdx.x / kBinRanges;
    const int64_t a0 = c * kBinPerBlock;
    const int ns = geo.ns, nw = geo.nw;
    const int nruns = nw * kBinPerBlock;
    for (int j = t; j < kBinBlock; j += kBinDotThreads)
        acc[j] = 0.0f;
    // run q = tw * 16 + u: sub-bin (workgroup a0 + u, range xr, window tw)
    for (int q = t; q < nruns; q += kBinDotThreads) {
        const int u = q / nw, tw = q % nw;  // consecutive threads: consecutive windows of one workgroup
        const int64_t a = a0 + u;
        pre[tw * kBinPerBlock + u] = a < na ? counts[a * ns + (int64_t)xr * nw + tw] : 0;
    }
    __syncthreads();
    const int32_t total = block_exclusive_scan4(pre, nruns, s_wtot);
    if (t == 0)
        pre[nruns] = total;
    __syncthreads();
    // one entry per thread at a time; the next stretch's entry is looked up
    // and loaded after r is read for the current one.  The load sits under a
    // branch, so the compiler drains it before the next read of r: each
    // stretch costs an entry load and a read of r in turn, and that common
    // pace keeps the blocks of a range on the same rows (prefetching the
    // entries two stretches ahead, branch-free, let the blocks drift apart:
    // 325 us per launch with twice the L2 misses, 1.6e7)
    BinEntry cur{0u, 0.0f};
    uint32_t rowb = 0;
    if (t < total)
        bin_flat_entry(bins, pre, nruns, geo, xr, a0, t, cur, rowb);
    for (int32_t j = t; j < total; j += kBinDotThreads) {
        const T rv = load_row(r, (int)(rowb + (cur.key & kBinWinMask)));
        BinEntry nxt{0u, 0.0f};
        uint32_t nrowb = 0;
        if (j + kBinDotThreads < total)
            bin_flat_entry(bins, pre, nruns, geo, xr, a0, j + kBinDotThreads, nxt, nrowb);
        atomicAdd(&acc[cur.key >> kBinWinBits], (float)(cur.val * rv));
        cur = nxt;
        rowb = nrowb;
    }
    __syncthreads();
    for (int j = t; j < kBinBlock; j += kBinDotThreads) {
        const int64_t s = c * kBinBlock + j;
        if (s < tau)
            partial[(int64_t)xr * tau + s] = (T)acc[j];
    }
}

// The update of every slot from the summed partials, or, when the binning of
// this step overflowed, the whole step by the plain gather.
template <typename V, int G, int C>
__global__ void __launch_bounds__(kBlock)
k_bin_prox(char *__restrict__ seg, Layout lay, const typename ValT<V>::T *__restrict__ r,
           double *__restrict__ xm, int32_t *__restrict__ id_slot, typename ValT<V>::T *__restrict__ delta_slot,
           const Ctrl *__restrict__ ctrl, uint64_t *__restrict__ nz_part, uint64_t seed, int64_t tau, uint32_t n,
           double inv_beta, ProxParams pp, const v2d_t *__restrict__ hdr,
           const typename ValT<V>::T *__restrict__ partial, uint32_t *__restrict__ over)
{
    using T = typename ValT<V>::T;
    __shared__ uint32_t s_keys[kNiceRounds];
    __shared__ uint64_t s_red[kBlock / 64];
    const uint64_t k = ctrl->k;
    const bool plain = over[k & 1] != 0;
    uint64_t nz = 0;
    if (plain) {
        const NiceKey key = nice_key_block(seed, k, n, s_keys);
        const SlotDraw sd = slot_draw_for(plan_nice(), seed, k);
        const TileLanes<G> tl;
        for (int64_t base = wave_global_id() * 64; base < tau; base += wave_count() * 64)
            gather_tile<V, G, C, kLossSquare>(seg, lay, r, xm, id_slot, delta_slot, key, sd, tl, base, tau,
                                              inv_beta, pp, nz);
    } else {
        for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < tau; s += (int64_t)gridDim.x * kBlock) {
            T g = T(0);
#pragma unroll
            for (int xr = 0; xr < kBinRanges; ++xr)
                g += partial[(int64_t)xr * tau + s];
            const v2d_t hv = hdr[s];
            const double xi = hv.x;
            const double xn = model_prox(xi, (double)g * pp.gscale, hv.y * inv_beta, pp);
            const double d = xn - xi;
            delta_slot[s] = (T)d;
            if (d != 0.0) {
                const int32_t i = id_slot[s];
                __builtin_nontemporal_store(xn, reinterpret_cast<double *>(seg + (int64_t)i * lay.stride));
                __builtin_nontemporal_store(xn, xm + i);
                ++nz;
            }
        }
    }
    const uint64_t tot = block_sum_u64(nz, s_red);
    if (threadIdx.x == 0 && tot)
        nz_part[blockIdx.x] += tot;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        over[(k + 1) & 1] = 0u;  // the next step's flag; nobody reads it during this step
}

}  // namespace pcdm

namespace pcdm {

// --------------------------------------------------------------------------
// Residual scatter by row blocks (option scatter_route = 2): r += delta_i a_i
// without global atomics.  The rows are cut into blocks of 2^12; each block
// is owned by one workgroup of k_sapply, which sums its entries in LDS and
// adds the sums to r with plain stores.
//
//   k_sbin    (one workgroup per 1024 consecutive slots, as k_scatter): packs
//             the slots with delta_i != 0; when they hold at most 2048
//             products (late in a solve, when few coordinates still move) it
//             adds them with atomics as k_scatter does; otherwise it reads
//             their columns and deals the products delta_i a_ji into runs
//             keyed by row block (LDS
//             counting sort, then contiguous runs in the workgroup's own part
//             of `bins`); a run that would pass its capacity adds the rest
//             to r with atomics at once (k_sapply reads r only after this
//             kernel has finished).  Advances the step counter.
//   k_sapply  (one workgroup per row block): the block's runs of every
//             k_sbin workgroup, summed per row in LDS, then added to r; it
//             returns at once when no k_sbin workgroup made runs.
// --------------------------------------------------------------------------

constexpr int kRowBlockBits = 12;
constexpr int kRowBlock = 1 << kRowBlockBits;
constexpr int kSbinThreads = 256;     // k_sbin: threads, and packed columns staged at once
constexpr int kSbinMaxBlocks = 1024;  // row blocks (m <= 2^22): 4 per k_sbin thread in its scan
constexpr int kSbinMaxWg = 2048;      // k_sbin workgroups (tau <= 2^21)
constexpr int kSapplyThreads = 1024;
constexpr int kSbinDirect = 2048;  // k_sbin: at most this many products go straight to atomics

struct SbinGeom {
    int32_t nrb;   // row blocks, ceil(m / 4096)
    int32_t nwg;   // k_sbin workgroups, ceil(tau / 1024)
    int32_t cap;   // entries per run
    int32_t dpad;  // entries per record (fixed-length records)
};

__host__ __device__ inline size_t sbin_lds_bytes(int nrb, int dpad)
{
    return (size_t)4 * nrb * sizeof(int32_t) + (size_t)kSbinThreads * dpad * (4 + 4 + 2 + 2);
}

template <typename V>
__global__ void __launch_bounds__(kSbinThreads)
k_sbin(const char *__restrict__ seg, Layout lay, SbinGeom geo, typename ValT<V>::T *__restrict__ r,
       const int32_t *__restrict__ id_slot, const typename ValT<V>::T *__restrict__ delta_slot,
       Ctrl *__restrict__ ctrl, int64_t tau, BinEntry *__restrict__ bins, int32_t *__restrict__ counts,
       uint32_t *__restrict__ sync)
{
    using T = typename ValT<V>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int32_t s_id[kScatterSpan];
    __shared__ T s_d[kScatterSpan];
    __shared__ int s_cnt;
    __shared__ int32_t s_wtot[kSbinThreads / 64];
    const int nrb = geo.nrb, dpad = geo.dpad;
    const int nstage = kSbinThreads * dpad;
    int32_t *cnt = reinterpret_cast<int32_t *>(smem);
    int32_t *offs = cnt + nrb;
    int32_t *fill = offs + nrb;
    int32_t *run = fill + nrb;
    uint32_t *strow = reinterpret_cast<uint32_t *>(run + nrb);
    float *stval = reinterpret_cast<float *>(strow + nstage);
    uint16_t *stblk = reinterpret_cast<uint16_t *>(stval + nstage);
    uint16_t *order = stblk + nstage;

    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6, gl = lane & 7, grp = lane >> 3;
    const int64_t wg = blockIdx.x;
    if (wg == 0 && t == 0)
        ctrl->k += 1;  // no block of this kernel reads k
    if (t == 0)
        s_cnt = 0;
    for (int q = t; q < nrb; q += kSbinThreads) {
        cnt[q] = 0;
        fill[q] = 0;
        run[q] = 0;
    }
    __syncthreads();
    for (int j = t; j < kScatterSpan; j += kSbinThreads) {
        const int64_t slot = wg * kScatterSpan + j;
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
    const int npk = s_cnt;
    if (npk * dpad <= kSbinDirect) {
        // few changed columns (late in a solve): the plain atomic scatter of
        // k_scatter costs less than binning them; the runs stay empty
        const TileLanes<8> tl;
        for (int t0 = w * 64; t0 < npk; t0 += kSbinThreads) {
            const int e = t0 + tl.lane;
            const bool live = e < npk;
            const T d = live ? s_d[e] : T(0);
            int64_t off = 0;
            int32_t dp = 0;
            if (live)
                locate<V>(lay, s_id[e], off, dp);
            tile_entries<V, 8>(seg, tl, off, dp, d, [&](int, T dq, int row, T val) {
                if (val != T(0))
                    atomic_add_hw<T>(r + row, dq * val);
            });
        }
        for (int q = t; q < nrb; q += kSbinThreads)
            counts[(int64_t)q * geo.nwg + wg] = 0;
        return;
    }
    if (t == 0)
        atomicOr(sync, 1u);  // k_sapply has runs to add this step
    for (int c0 = 0; c0 < npk; c0 += kSbinThreads) {
        // column c0 + t is packed column w * 64 + o of this chunk; its entries
        // are read by the 8 lanes of group grp in round q (o = q * 8 + grp)
        const int mine = c0 + t;
        int64_t off = 0;
        if (mine < npk)
            off = (int64_t)s_id[mine] * lay.stride;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int o = q * 8 + grp;
            const int sl = w * 64 + o;
            const bool cact = c0 + sl < npk;
            const int64_t coff = __shfl(off, o);
            const int e = 4 * gl;
            if (e < dpad) {
                int rw[4] = {0, 0, 0, 0};
                T v[4] = {T(0), T(0), T(0), T(0)};
                T dq = T(0);
                if (cact) {
                    Chunk4<V>::load(seg + coff + kHeader, dpad, e, rw, v);
                    dq = s_d[c0 + sl];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int idx = sl * dpad + e + u;
                    if (cact && v[u] != T(0)) {
                        const uint32_t row = (uint32_t)rw[u];
                        const int blk = (int)(row >> kRowBlockBits);
                        strow[idx] = row & (kRowBlock - 1);
                        stval[idx] = (float)(dq * v[u]);
                        stblk[idx] = (uint16_t)blk;
                        atomicAdd(&cnt[blk], 1);
                    } else {
                        stblk[idx] = 0xFFFFu;
                    }
                }
            }
        }
        __syncthreads();
        for (int q = t; q < nrb; q += kSbinThreads)
            offs[q] = cnt[q];
        __syncthreads();
        const int32_t nvalid = block_exclusive_scan4(offs, nrb, s_wtot);  // ends with a barrier
        for (int idx = t; idx < nstage; idx += kSbinThreads) {
            const uint16_t blk = stblk[idx];
            if (blk != 0xFFFFu)
                order[offs[blk] + atomicAdd(&fill[blk], 1)] = (uint16_t)idx;
        }
        __syncthreads();
        for (int j = t; j < nvalid; j += kSbinThreads) {
            const int idx = order[j];
            const int blk = stblk[idx];
            const int pos = run[blk] + (j - offs[blk]);
            if (pos < geo.cap) {
                BinEntry be;
                be.key = strow[idx];
                be.val = stval[idx];
                bins[((int64_t)blk * geo.nwg + wg) * geo.cap + pos] = be;
            } else {
                // past the run's capacity: straight into r (k_sapply runs later)
                atomic_add_hw<T>(r + (((uint32_t)blk << kRowBlockBits) | strow[idx]), (T)stval[idx]);
            }
        }
        __syncthreads();
        for (int q = t; q < nrb; q += kSbinThreads) {
            run[q] += cnt[q];
            cnt[q] = 0;
            fill[q] = 0;
        }
        __syncthreads();
    }
    for (int q = t; q < nrb; q += kSbinThreads)
        counts[(int64_t)q * geo.nwg + wg] = run[q] < geo.cap ? run[q] : geo.cap;
}

// Row block b = blockIdx.x: the sums of its entries over every k_sbin
// workgroup, added to r[4096 b ..].
template <typename T>
__global__ void __launch_bounds__(kSapplyThreads)
k_sapply(const BinEntry *__restrict__ bins, const int32_t *__restrict__ counts, SbinGeom geo, int64_t m,
         T *__restrict__ r, uint32_t *__restrict__ sync)
{
    __shared__ T acc[kRowBlock];
    __shared__ int32_t pre[kSbinMaxWg + 1];
    __shared__ int32_t s_wtot[kSapplyThreads / 64];
    const int t = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int nwg = geo.nwg;
    // sync[0] != 0: some k_sbin workgroup made runs this step; sync[1] counts
    // the blocks of this kernel that are done; the last one resets both for
    // the next step (every other block has read sync[0] before counting)
    const bool any = __hip_atomic_load(sync, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
    if (!any) {
        if (t == 0 && atomicAdd(sync + 1, 1u) == gridDim.x - 1) {
            sync[0] = 0u;
            sync[1] = 0u;
        }
        return;
    }
    for (int j = t; j < kRowBlock; j += kSapplyThreads)
        acc[j] = T(0);
    for (int q = t; q < nwg; q += kSapplyThreads)
        pre[q] = counts[b * nwg + q];
    __syncthreads();
    const int32_t total = block_exclusive_scan4(pre, nwg, s_wtot);
    if (t == 0)
        pre[nwg] = total;
    __syncthreads();
    for (int32_t j = t; j < total; j += kSapplyThreads) {
        int lo = 0, hi = nwg;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (pre[mid] <= j)
                lo = mid;
            else
                hi = mid - 1;
        }
        const BinEntry be = bins[(b * nwg + lo) * geo.cap + (j - pre[lo])];
        atomicAdd(&acc[be.key], (T)be.val);
    }
    __syncthreads();
    for (int j = t; j < kRowBlock; j += kSapplyThreads) {
        const int64_t row = (b << kRowBlockBits) + j;
        const T a = acc[j];
        if (row < m && a != T(0))
            r[row] += a;
    }
    if (t == 0 && atomicAdd(sync + 1, 1u) == gridDim.x - 1) {
        sync[0] = 0u;
        sync[1] = 0u;
    }
}

}  // namespace pcdm
