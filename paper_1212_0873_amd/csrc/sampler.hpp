// sampler.hpp -- the tau-nice sampler on the device.
//
// The method needs S_k drawn so that every subset of tau coordinates is
// equally likely (nice sampling, section "Block Samplings"), independently
// across steps.  Here S_k = { pi_k(j) : 0 <= j < tau } for a keyed
// pseudo-random permutation pi_k of [0, n): any thread can produce slot j's
// coordinate on its own, with no shared state, no duplicates and no
// de-duplication pass.
//
// Definition (built from published primitives):
//   * SplitMix64 (Steele, Lea & Flood, 2014): output t of the stream started
//     at state s is finalise(s + (t+1) * 0x9E3779B97F4A7C15), finalise being
//     Stafford's mix: xor-shift 30, * 0xBF58476D1CE4E5B9, xor-shift 27,
//     * 0x94D049BB133111EB, xor-shift 31.
//   * Round keys of step k: low 32 bits of outputs 10k .. 10k+9 of the stream
//     started at seed ^ 0x5043444D4E494345.
//   * Round function: MurmurHash3's 32-bit finaliser (Appleby) of
//     (right half ^ round key), truncated to the half width.
//   * A balanced ten-round Feistel network on [0, 4^h), h >= 1 the least
//     value with 4^h >= n; the input splits as (high h bits, low h bits) and
//     each round maps (hi, lo) -> (lo, hi ^ F(lo)).
//   * Cycle walking (Black & Rogaway, 2002) restricts it to [0, n): apply the
//     network again while the value is >= n.
// Ten rounds: fewer leave the subset law visibly non-uniform on the tiny
// domains of small n.
//
// Other doubly uniform samplings (section "Block Samplings"), from the same
// primitives.  Step key kappa_k = SplitMix64 output k of the stream started at
// seed ^ 0x5043444D494E4450 (independent picks) or seed ^ 0x5043444D42494E4F
// (binomial availability); draw j of step k = SplitMix64 output j of the
// stream started at kappa_k.
//   * tau-independent: processor j picks block floor(draw_j * n / 2^64)
//     (Lemire's multiply-shift reduction); a block picked by several
//     processors is updated once (the first claim at its stamp wins, the
//     others idle), so S_k is the set of distinct picks.
//   * (tau, p_b)-binomial, implicit selection: slot j keeps its tau-nice block
//     pi_k(j) and is available iff (draw_j >> 11) * 2^-53 < p_b.
// A drop mask (processors that are down) removes slot j when mask[j] == 0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcdm {

constexpr int kNiceRounds = 10;
constexpr uint64_t kNiceStream = 0x5043444D4E494345ull;

__host__ __device__ inline uint64_t splitmix_output(uint64_t state, uint64_t t)
{
    uint64_t z = state + (t + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t murmur_fmix(uint32_t v)
{
    v = (v ^ (v >> 16)) * 0x85EBCA6Bu;
    v = (v ^ (v >> 13)) * 0xC2B2AE35u;
    return v ^ (v >> 16);
}

// Width of one Feistel half for a domain of n >= 1 values.
__host__ __device__ inline uint32_t nice_half_width(uint32_t n)
{
    uint32_t h = 1;
    while (h < 16 && (1ull << (2 * h)) < (uint64_t)n)
        ++h;
    return h;
}

struct NiceKey {
    uint32_t rk[kNiceRounds];
    uint32_t half;
    uint32_t mask;
    uint32_t n;
};

__device__ __forceinline__ uint32_t nice_permute_once(uint32_t v, const NiceKey &key)
{
    uint32_t hi = v >> key.half;
    uint32_t lo = v & key.mask;
#pragma unroll
    for (int q = 0; q < kNiceRounds; ++q) {
        const uint32_t mixed = hi ^ (murmur_fmix(lo ^ key.rk[q]) & key.mask);
        hi = lo;
        lo = mixed;
    }
    return (hi << key.half) | lo;
}

// Coordinate held by slot j of the step whose key is `key` (j < n).
__device__ __forceinline__ uint32_t nice_slot(uint32_t j, const NiceKey &key)
{
    uint32_t v = nice_permute_once(j, key);
    while (v >= key.n)
        v = nice_permute_once(v, key);
    return v;
}

// Every thread of the block calls this; round keys go through LDS once.
__device__ __forceinline__ NiceKey nice_key_block(uint64_t seed, uint64_t step, uint32_t n,
                                                  uint32_t *lds_keys)
{
    if (threadIdx.x < kNiceRounds)
        lds_keys[threadIdx.x] =
            (uint32_t)splitmix_output(seed ^ kNiceStream, step * kNiceRounds + threadIdx.x);
    __syncthreads();
    NiceKey key;
#pragma unroll
    for (int q = 0; q < kNiceRounds; ++q)
        key.rk[q] = lds_keys[q];
    key.half = nice_half_width(n);
    key.mask = (1u << key.half) - 1u;
    key.n = n;
    return key;
}

// Per-wave variant (a block may serve several problems): lanes 0..9 derive
// the round keys, which are then broadcast across the wave.
__device__ __forceinline__ NiceKey nice_key_wave(uint64_t seed, uint64_t step, uint32_t n)
{
    const int lane = threadIdx.x & 63;
    uint32_t mine = 0;
    if (lane < kNiceRounds)
        mine = (uint32_t)splitmix_output(seed ^ kNiceStream, step * kNiceRounds + lane);
    NiceKey key;
#pragma unroll
    for (int q = 0; q < kNiceRounds; ++q)
        key.rk[q] = (uint32_t)__shfl((int)mine, q);
    key.half = nice_half_width(n);
    key.mask = (1u << key.half) - 1u;
    key.n = n;
    return key;
}

enum : int { kSampleNice = 0, kSampleIndependent = 1, kSampleBinomial = 2 };
constexpr uint64_t kIndepStream = 0x5043444D494E4450ull;
constexpr uint64_t kBinomStream = 0x5043444D42494E4Full;

// What the host fixes about a problem's sampling (kernel argument).
struct SlotPlan {
    int mode;                // kSample*
    double pb;               // availability of a binomial slot
    const uint8_t *mask;     // nullptr: every slot alive
    int64_t mask_len;        // slots >= mask_len are alive
    uint32_t *claim;         // [n] claim stamps (independent picks)
    uint64_t claim_base;     // step at which claim was last zeroed
};

__host__ __device__ inline SlotPlan plan_nice()
{
    SlotPlan p;
    p.mode = kSampleNice;
    p.pb = 1.0;
    p.mask = nullptr;
    p.mask_len = 0;
    p.claim = nullptr;
    p.claim_base = 0;
    return p;
}

// The plan specialised to step k.
struct SlotDraw {
    SlotPlan plan;
    uint64_t kappa;
    uint32_t stamp;  // unique per step since the last zeroing of claim, never 0
};

__device__ __forceinline__ SlotDraw slot_draw_for(const SlotPlan &p, uint64_t seed, uint64_t k)
{
    SlotDraw d;
    d.plan = p;
    d.kappa = 0;
    if (p.mode == kSampleIndependent)
        d.kappa = splitmix_output(seed ^ kIndepStream, k);
    else if (p.mode == kSampleBinomial)
        d.kappa = splitmix_output(seed ^ kBinomStream, k);
    d.stamp = (uint32_t)(k - p.claim_base) + 1u;
    return d;
}

// Slot j's block before masks and claims; false when a binomial slot is
// unavailable.
__device__ __forceinline__ bool slot_block(const SlotDraw &d, const NiceKey &key, uint32_t j, uint32_t &i)
{
    if (d.plan.mode == kSampleIndependent) {
        i = (uint32_t)__umul64hi(splitmix_output(d.kappa, j), (uint64_t)key.n);
        return true;
    }
    i = nice_slot(j, key);
    if (d.plan.mode == kSampleBinomial)
        return (double)(splitmix_output(d.kappa, j) >> 11) * 0x1.0p-53 < d.plan.pb;
    return true;
}

// Slot j's block and whether the slot updates it this step (mask, binomial
// availability, first claim of an independent pick).
__device__ __forceinline__ bool draw_slot(const SlotDraw &d, const NiceKey &key, uint32_t j, uint32_t &i)
{
    bool keep = slot_block(d, key, j, i);
    if (d.plan.mask && (int64_t)j < d.plan.mask_len && d.plan.mask[j] == 0)
        keep = false;
    if (keep && d.plan.mode == kSampleIndependent)
        keep = atomicExch(d.plan.claim + i, d.stamp) != d.stamp;
    return keep;
}

}  // namespace pcdm
