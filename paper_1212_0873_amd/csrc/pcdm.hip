// pcdm.hip -- host runtime behind the C ABI of include/pcdm.h.
//
// Owns the device copy of the problem in the segment layout of kernels.hpp,
// launches the step, refresh, objective and set-up kernels on the caller's
// stream, and turns every failure into a status code plus a thread-local
// message.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "binned_kernels.hpp"
#include "group_kernels.hpp"
#include "kernels.hpp"
#include "pcdm.h"

using namespace pcdm;

// Fixed device region for the entry points that allocate nothing
// (pcdm_grad_backward_noalloc).  Each device the library runs on holds its
// own copy until the process ends.  Host code never passes `scratch` itself
// to a kernel or a copy: that name is the host-side stand-in; the device
// address comes from hipGetSymbolAddress (scratch_base).
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string t_err;

int fail(int code, const std::string &msg)
{
    t_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? PCDM_ENOMEM : PCDM_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e__ = (expr);                        \
        if (e__ != hipSuccess)                          \
            return hip_fail(e__, #expr);                \
    } while (0)

#define PCDM_TRY(expr)           \
    do {                         \
        int s__ = (expr);        \
        if (s__ != PCDM_OK)      \
            return s__;          \
    } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

size_t value_bytes(int dtype)
{
    switch (dtype) {
    case PCDM_F32: return 4;
    case PCDM_BF16: return 2;
    case PCDM_F64: return 8;
    default: return 0;
    }
}

int grid_for(int64_t items, int64_t per_block, int cap)
{
    int64_t g = ceil_div(std::max<int64_t>(items, 1), per_block);
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

constexpr int kReduceBlocks = 1024;

// Upper bound on the workgroups of a step launch per compute unit (the
// kernels loop over their tiles, so a smaller grid only changes balance).
#ifndef PCDM_BLOCKS_PER_CU
#define PCDM_BLOCKS_PER_CU 8
#endif
constexpr int64_t kAsyncAcquireProcs = 8192;  // automatic read mode: acquire up to this many processors

// Device time of one kernel kind, from HIP events recorded around each launch.
struct KernelClock {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    int64_t launches = 0;
    double total_ms = 0.0;
};

enum { CLK_GATHER = 0, CLK_SCATTER = 1, CLK_REFRESH = 2, CLK_ASYNC = 3, CLK_COUNT = 4 };

}  // namespace

struct pcdm_problem {
    int device = 0;
    int64_t m = 0, n = 0, nnz = 0, stored_nnz = 0, tau = 0;
    int dtype = PCDM_F32;
    size_t tbytes = 4;  // compute type size
    double lambda = 0.0, beta = 1.0, atb_inf = 0.0;
    int beta_rule = 0;
    int64_t omega = 0;
    uint64_t seed = 0;
    int64_t k_host = 0;
    int64_t refresh_every = 0;
    int lanes = 8;
    int chunks = 1;
    int64_t narrow_below = 131072;  // tau below which a slot gets a lane group (not a lane)
    int lanes_auto = 1;
    int nblk_max = 2048;
    hipStream_t last_stream = nullptr;

    char *seg = nullptr;
    int64_t *pc = nullptr;
    Layout lay{nullptr, 0, 0};
    double *x = nullptr;  // dense mirror of the x_i in the column records
    void *r = nullptr;
    double *r64 = nullptr, *b64 = nullptr;
    int32_t *id_slot = nullptr;
    void *delta_slot = nullptr;
    int64_t slot_cap = 0;
    Ctrl *ctrl = nullptr;
    uint64_t *nz_part = nullptr;
    double *part = nullptr;   // kReduceBlocks * 3
    double *part2 = nullptr;  // nblk_max
    float *t32 = nullptr;     // m: fl32(r64) for the bound pass of ||A^T r||_inf (values below float64)
    float *ub = nullptr;      // n: per-column upper bounds of that pass
    int max_passes = 0;       // ||A^T r||_inf: 2 = bound + exact pass where available, 1 = one exact pass,
                              // 3 = incremental from the last evaluation where it pays, else as 2,
                              // 0 = 3 from kIncMinEntries stored entries, else 2
    // incremental route: r of the last evaluation, column l1 norms (rounded up),
    // [M_old, maxima, D, lower bound], candidate count; valid after a 2- or 3-route evaluation
    double *rold = nullptr;
    float *nrm = nullptr;
    double *inc = nullptr;
    unsigned long long *cnt = nullptr;
    double nrm_max = 0.0, gam = 0.0;
    bool inc_valid = false;
    int64_t inc_hits = 0, inc_cands = -1;

    int timing = 0;
    KernelClock clocks[CLK_COUNT];

    // sampling of S_k (kSampleNice / kSampleIndependent / kSampleBinomial)
    int sampling = kSampleNice;
    double pb = 1.0;
    uint8_t *mask = nullptr;   // device drop mask over slots, or nullptr
    int64_t mask_len = 0;
    uint32_t *claim = nullptr; // [n] claim stamps for independent picks
    int64_t claim_base = 0;    // step at which claim was last zeroed

    // model: f = lscale * sum_j phi(.), Omega_i = lambda|t| + (l2/2)t^2 + lin t + box
    int loss = kLossSquare;
    double lscale = 1.0, l2 = 0.0, lin = 0.0, lo = -HUGE_VAL, hi = HUGE_VAL;

    // blocks of several coordinates (group LASSO): block i = columns bp[i] .. bp[i+1]-1
    int group = 0;
    int64_t nb = 0;
    int64_t *bp = nullptr;    // [nb+1] device
    double *invlb = nullptr;  // [nb] 1 / lambda_max(A_i^T A_i)
    void *dx = nullptr;       // [n] per-column change of the last step (working type)

    // runs of steps captured into a graph and replayed
    int64_t graph_len = 32;  // steps per graph; 0 = launch every step directly
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<unsigned char> graph_sig;  // step-kernel arguments the graph was captured with
    int64_t graph_captured_len = 0;

    // asynchronous variant
    int cus = 0;
    int async_reads = -1;      // kReadCached / kReadAcquire / kReadAtomic, -1 = by processor count
    int64_t async_rounds = 4;  // rounds of picks per launch with cached reads (0 = the whole call)
    int64_t async_launches = 0;
    int64_t async_picks = 0;
    int64_t async_procs_opt = 0;   // 0 = min(tau, resident lane groups)
    int64_t async_procs_last = 0;

    // adjoint solve settings
    double adj_tol = 1e-6;
    int64_t adj_max_epochs = 20000;
    int64_t adj_tau = 0;  // 0 = the problem's tau
    int64_t adj_check_every = 10;
    int64_t adj_last_epochs = 0;
    double adj_last_resid = 0.0;
    std::vector<hipEvent_t> event_pool;

    // row-binned route of the partial derivatives (binned_kernels.hpp)
    int gather_route = 0;     // option: 0 automatic, 1 plain gather, 2 binned where eligible
    bool binned = false;      // route in effect
    int64_t bin_cap_opt = 0;  // option: entries per sub-bin (0 = from the expected count)
    BinGeom bgeo{};
    int64_t bin_tau = 0;      // tau the buffers were sized for
    void *bins = nullptr;     // [ceil(tau/1024) * ns * cap] BinEntry
    int32_t *bcounts = nullptr;
    void *bhdr = nullptr;     // [tau] {x_i, 1/L_i}
    void *bpart = nullptr;    // [8 * tau] working type
    uint32_t *bover = nullptr;  // [2] overflow flags by step parity

    // residual scatter by row blocks (binned_kernels.hpp)
    int scatter_route = 0;     // option: 0 automatic, 1 atomics, 2 row blocks where eligible
    bool srows = false;        // route in effect
    int64_t sbin_cap_opt = 0;  // option: entries per run (0 = from the expected count)
    SbinGeom sgeo{};
    int64_t sbin_tau = 0;
    void *sbins = nullptr;     // [nrb * ceil(tau/1024) * cap] BinEntry
    int32_t *scounts = nullptr;
    uint32_t *ssync = nullptr;  // [2] runs-made flag, k_sapply blocks done
};

namespace {
// Below this many stored entries the incremental route's fixed costs (its
// extra launches and the host read of the candidate count) exceed a bound
// pass, so the automatic choice (max_passes 0) takes the two-pass route.
constexpr int64_t kIncMinEntries = int64_t(1) << 24;
inline int passes(const pcdm_problem *P)
{
    return P->max_passes ? P->max_passes : (P->stored_nnz >= kIncMinEntries ? 3 : 2);
}
}  // namespace

namespace {

void drop_step_graph(pcdm_problem *P)
{
    if (P->graph_exec)
        (void)hipGraphExecDestroy(P->graph_exec);
    if (P->graph)
        (void)hipGraphDestroy(P->graph);
    P->graph_exec = nullptr;
    P->graph = nullptr;
    P->graph_sig.clear();
}

void free_problem(pcdm_problem *P)
{
    if (!P)
        return;
    drop_step_graph(P);
    if (P->cap_stream)
        (void)hipStreamDestroy(P->cap_stream);
    for (auto &c : P->clocks)
        for (auto &pr : c.pending) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (hipEvent_t e : P->event_pool)
        (void)hipEventDestroy(e);
    void *bufs[] = {P->seg, P->pc, P->x, P->r, P->r64, P->b64, P->id_slot,
                    P->delta_slot, P->ctrl, P->nz_part, P->part, P->part2, P->mask, P->claim, P->bp, P->invlb, P->dx,
                    P->t32, P->ub, P->rold, P->nrm, P->inc, P->cnt, P->bins, P->bcounts, P->bhdr, P->bpart,
                    P->bover, P->sbins, P->scounts, P->ssync};
    for (void *b : bufs)
        if (b)
            (void)hipFree(b);
    delete P;
}

// tau-independent picks: with p1 = P(i in S) and p2 = P(i, j in S) for i != j,
// E|S| = n p1 and E|S|^2/E|S| - 1 = (n-1) p2 / p1.  p2 = 1 - 2(1-1/n)^tau +
// (1-2/n)^tau is summed as the binomial series
//     p2 = sum_{s>=2} (-1)^s C(tau, s) (2^s - 2) / n^s,
// whose terms shrink from s = 2 on (tau <= n), so it keeps full relative
// precision where the closed form cancels (tau << n).
void independent_moments(int64_t tau, int64_t n, double &e1, double &ratio)
{
    const double nn = (double)n, t = (double)tau;
    const double p1 = -std::expm1(t * std::log1p(-1.0 / nn));
    e1 = nn * p1;
    ratio = 0.0;
    if (n < 2 || tau < 2)
        return;
    double c = 1.0, pw = 1.0, p2 = 0.0;  // c = C(tau, s) / n^s, pw = 2^s
    for (int64_t q = 1; q <= tau && q <= 4096; ++q) {
        c *= (t - (double)(q - 1)) / ((double)q * nn);
        pw *= 2.0;
        if (q < 2)
            continue;
        const double term = c * (pw - 2.0);
        p2 += (q & 1) ? -term : term;
        if (term <= 1e-18 * std::fabs(p2))
            break;
    }
    ratio = (nn - 1.0) * p2 / p1;
}

// E|S| of the sampling (before any drop mask).
double expected_set_size(const pcdm_problem *P)
{
    if (P->sampling == kSampleIndependent) {
        double e1, ratio;
        independent_moments(P->tau, P->n, e1, ratio);
        return e1;
    }
    if (P->sampling == kSampleBinomial)
        return (double)P->tau * P->pb;
    return (double)P->tau;
}

// beta_rule 0: the ESO beta of the sampling in use (Table ESO: tau-nice row;
// doubly uniform row beta = 1 + (omega-1)(E|S|^2/E|S| - 1)/max(1, n-1) for
// tau-independent picks; binomial row).  beta_rule 1: min(omega, tau).
int compute_beta(pcdm_problem *P)
{
    const double om = (double)P->omega, ta = (double)P->tau, nn = (double)(P->group ? P->nb : P->n);
    const double den = std::max(1.0, nn - 1.0);
    if (P->beta_rule == 0) {
        if (P->sampling == kSampleIndependent) {
            double e1, ratio;
            independent_moments(P->tau, P->n, e1, ratio);
            P->beta = 1.0 + (om - 1.0) * ratio / den;
        } else if (P->sampling == kSampleBinomial) {
            P->beta = 1.0 + P->pb * (om - 1.0) * (ta - 1.0) / den;
        } else {
            P->beta = 1.0 + (om - 1.0) * (ta - 1.0) / den;
        }
    } else if (P->beta_rule == 1) {
        P->beta = std::min(om, ta);
    }
    return PCDM_OK;
}

// Kernel view of the sampling.
SlotPlan slot_plan(const pcdm_problem *P)
{
    SlotPlan p = plan_nice();
    p.mode = P->sampling;
    p.pb = P->pb;
    p.mask = P->mask;
    p.mask_len = P->mask_len;
    p.claim = P->claim;
    p.claim_base = (uint64_t)P->claim_base;
    return p;
}

// The LASSO of the paper's experiments (square loss, l1 only): the paths
// that are specific to it (duality gap, adjoint, batches, asynchronous
// variant) require it.
bool is_lasso(const pcdm_problem *P)
{
    return !P->group && P->loss == kLossSquare && P->lscale == 1.0 && P->l2 == 0.0 && P->lin == 0.0 && P->lo == -HUGE_VAL &&
           P->hi == HUGE_VAL;
}

ProxParams prox_params(const pcdm_problem *P)
{
    ProxParams p = prox_lasso(P->lambda);
    p.l2 = P->l2;
    p.c = P->lin;
    p.lo = P->lo;
    p.hi = P->hi;
    p.gscale = P->lscale;
    return p;
}

// Zero the claim stamps and restart their numbering at step k (a fill
// kernel, so the call is safe inside a captured stream).
void reset_claims(pcdm_problem *P, int64_t k, hipStream_t s)
{
    if (!P->claim)
        return;
    const int g = grid_for(P->n, kBlock, P->nblk_max);
    hipLaunchKernelGGL((k_fill<uint32_t>), dim3(g), dim3(kBlock), 0, s, P->claim, 0u, P->n);
    P->claim_base = k;
}

// Tile schedule from the mean padded column length: G lanes per column with
// C chunks (of 4 entries) each, G*C >= the mean number of chunks.
void pick_schedule(pcdm_problem *P)
{
    const double chunks = (double)P->stored_nnz / (4.0 * (double)P->n);
    if (chunks <= 1.0) {
        P->lanes = 1; P->chunks = 1;
    } else if (chunks <= 2.0) {
        P->lanes = 2; P->chunks = 1;
    } else if (chunks <= 4.0) {
        P->lanes = 4; P->chunks = 1;
    } else if (chunks <= 8.0) {
        P->lanes = 8; P->chunks = 1;
    } else if (chunks <= 16.0) {
        P->lanes = 16; P->chunks = 1;
    } else if (chunks <= 32.0) {
        P->lanes = 32; P->chunks = 1;
    } else {
        P->lanes = 64; P->chunks = 1;
    }
}

bool schedule_supported(int g, int c, int loss = kLossSquare)
{
    if (loss != kLossSquare && c != 1)
        return false;  // other losses are built with one chunk per lane
    switch (g * 16 + c) {
    case 1 * 16 + 1: case 1 * 16 + 2: case 1 * 16 + 4: case 2 * 16 + 1: case 2 * 16 + 2:
    case 2 * 16 + 4: case 4 * 16 + 1: case 4 * 16 + 2: case 8 * 16 + 1: case 8 * 16 + 2:
    case 16 * 16 + 1: case 32 * 16 + 1: case 64 * 16 + 1:
        return true;
    default:
        return false;
    }
}

hipEvent_t take_event(pcdm_problem *P)
{
    hipEvent_t e = nullptr;
    if (!P->event_pool.empty()) {
        e = P->event_pool.back();
        P->event_pool.pop_back();
        return e;
    }
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

// Record a start event for a kernel kind (no-op unless timing is on).
hipEvent_t clock_start(pcdm_problem *P, hipStream_t s)
{
    if (!P->timing)
        return nullptr;
    hipEvent_t e = take_event(P);
    if (e)
        (void)hipEventRecord(e, s);
    return e;
}

void clock_stop(pcdm_problem *P, int kind, hipEvent_t start, hipStream_t s)
{
    if (!P->timing || !start)
        return;
    hipEvent_t e = take_event(P);
    if (!e)
        return;
    (void)hipEventRecord(e, s);
    P->clocks[kind].pending.emplace_back(start, e);
}

// Fold finished event pairs into the totals (synchronises on the events).
int clock_collect(pcdm_problem *P, int kind)
{
    KernelClock &c = P->clocks[kind];
    for (auto &pr : c.pending) {
        HIP_TRY(hipEventSynchronize(pr.second));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
        c.total_ms += ms;
        c.launches += 1;
        P->event_pool.push_back(pr.first);
        P->event_pool.push_back(pr.second);
    }
    c.pending.clear();
    return PCDM_OK;
}

int ensure_slots(pcdm_problem *P, int64_t tau)
{
    if (tau <= P->slot_cap)
        return PCDM_OK;
    if (P->id_slot)
        HIP_TRY(hipFree(P->id_slot));
    if (P->delta_slot)
        HIP_TRY(hipFree(P->delta_slot));
    P->id_slot = nullptr;
    P->delta_slot = nullptr;
    P->slot_cap = 0;
    HIP_TRY(hipMalloc(&P->id_slot, (size_t)tau * sizeof(int32_t)));
    HIP_TRY(hipMalloc(&P->delta_slot, (size_t)tau * P->tbytes));
    P->slot_cap = tau;
    return PCDM_OK;
}

void free_bins(pcdm_problem *P)
{
    void *b[] = {P->bins, P->bcounts, P->bhdr, P->bpart, P->bover};
    for (void *q : b)
        if (q)
            (void)hipFree(q);
    P->bins = nullptr;
    P->bcounts = nullptr;
    P->bhdr = nullptr;
    P->bpart = nullptr;
    P->bover = nullptr;
    P->bin_tau = 0;
}

// Whether the row-binned route can take this problem's steps, and why not.
const char *bin_ineligible(const pcdm_problem *P)
{
    if (P->loss != kLossSquare || P->group)
        return "the binned route is built for the LASSO over coordinates";
    if (P->dtype == PCDM_F64)
        return "the binned route takes float32 or bf16 values";
    if (P->lay.fixed_dpad < 1 || P->lay.fixed_dpad > kBinMaxDpad)
        return "the binned route needs equal column lengths of at most 32 entries";
    if (P->sampling != kSampleNice || P->mask)
        return "the binned route takes the tau-nice sampling without a drop mask";
    const int64_t rx = ceil_div(P->m, kBinRanges);
    const int64_t ns = kBinRanges * ceil_div(rx, (int64_t)1 << kBinWinBits);
    if (ns > kBinMaxSub || bin_lds_bytes((int)ns, (int)P->lay.fixed_dpad) > (size_t)160 * 1024)
        return "too many rows for the binned route";
    return nullptr;
}

// Decide the route of the partial derivatives and size its buffers
// (called from API calls only, never inside a captured step).
int route_update(pcdm_problem *P)
{
    // automatic (0) takes the binned route only where it was measured to win:
    // r larger than the 256 MB Infinity Cache, so that the plain gather's
    // random reads of r are line fills from HBM, and tau >= 2^20, so that
    // k_bin_dot has two workgroups per CU (the 1e10-entry instance at
    // tau = 2^20: 434 against 438 us per step, with 1.7 instead of 3.0 GB past
    // L2; the 1e6-row instance, r = 4 MB: 361 against 145 us)
    const bool ok = bin_ineligible(P) == nullptr;
    const bool large = P->m * (int64_t)P->tbytes >= ((int64_t)256 << 20) && P->tau >= ((int64_t)1 << 20);
    const bool want = P->gather_route == 2 || (P->gather_route == 0 && large);
    if (!(ok && want)) {
        P->binned = false;
        free_bins(P);
        return PCDM_OK;
    }
    BinGeom g;
    g.rx = ceil_div(P->m, kBinRanges);
    g.nw = (int32_t)ceil_div(g.rx, (int64_t)1 << kBinWinBits);
    g.ns = kBinRanges * g.nw;
    g.dpad = (int32_t)P->lay.fixed_dpad;
    if (P->bin_cap_opt > 0) {
        g.cap = (int32_t)P->bin_cap_opt;
    } else {
        // mean count of a sub-bin when rows are uniform, plus 7 standard deviations
        const double mu = (double)kBinSlotsA * g.dpad / g.ns;
        g.cap = (int32_t)(16 * ceil_div((int64_t)std::ceil(mu + 7.0 * std::sqrt(mu) + 16.0), 16));
    }
    if (P->bins && P->bin_tau == P->tau && P->bgeo.ns == g.ns && P->bgeo.cap == g.cap && P->bgeo.dpad == g.dpad &&
        P->bgeo.rx == g.rx) {
        P->binned = true;
        return PCDM_OK;
    }
    free_bins(P);
    P->binned = false;
    const int64_t na = ceil_div(P->tau, kBinSlotsA);
    const size_t lds = bin_lds_bytes(g.ns, g.dpad);
    hipError_t e = hipMalloc(&P->bins, (size_t)na * g.ns * g.cap * sizeof(BinEntry));
    if (e == hipSuccess)
        e = hipMalloc(&P->bcounts, (size_t)na * g.ns * sizeof(int32_t));
    if (e == hipSuccess)
        e = hipMalloc(&P->bhdr, (size_t)P->tau * 16);
    if (e == hipSuccess)
        e = hipMalloc(&P->bpart, (size_t)kBinRanges * P->tau * P->tbytes);
    if (e == hipSuccess)
        e = hipMalloc(&P->bover, 2 * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMemset(P->bover, 0, 2 * sizeof(uint32_t));
    if (e == hipSuccess)
        e = P->dtype == PCDM_BF16
                ? hipFuncSetAttribute((const void *)k_bin<bf16s>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
                : hipFuncSetAttribute((const void *)k_bin<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) {
        free_bins(P);
        (void)hipGetLastError();
        if (P->gather_route == 2)
            return hip_fail(e, "binned route set-up");
        return PCDM_OK;  // automatic choice: keep the plain gather
    }
    P->bgeo = g;
    P->bin_tau = P->tau;
    P->binned = true;
    return PCDM_OK;
}

void free_sbins(pcdm_problem *P)
{
    if (P->sbins)
        (void)hipFree(P->sbins);
    if (P->scounts)
        (void)hipFree(P->scounts);
    if (P->ssync)
        (void)hipFree(P->ssync);
    P->sbins = nullptr;
    P->scounts = nullptr;
    P->ssync = nullptr;
    P->sbin_tau = 0;
}

// Whether the row-block scatter can take this problem's steps, and why not.
const char *sbin_ineligible(const pcdm_problem *P)
{
    if (P->group)
        return "the row-block scatter is built for coordinates";
    if (P->dtype == PCDM_F64)
        return "the row-block scatter takes float32 or bf16 values";
    if (P->lay.fixed_dpad < 1 || P->lay.fixed_dpad > kBinMaxDpad)
        return "the row-block scatter needs equal column lengths of at most 32 entries";
    if (ceil_div(P->m, kRowBlock) > kSbinMaxBlocks)
        return "too many rows for the row-block scatter (at most 2^22)";
    if (ceil_div(P->tau, kScatterSpan) > kSbinMaxWg)
        return "tau too large for the row-block scatter (at most 2^21)";
    return nullptr;
}

// Decide the scatter route and size its buffers (API calls only).
int sroute_update(pcdm_problem *P)
{
    const bool ok = sbin_ineligible(P) == nullptr;
    const bool want = P->scatter_route == 2;
    if (!(ok && want)) {
        P->srows = false;
        free_sbins(P);
        return PCDM_OK;
    }
    SbinGeom g;
    g.nrb = (int32_t)ceil_div(P->m, kRowBlock);
    g.nwg = (int32_t)ceil_div(P->tau, kScatterSpan);
    g.dpad = (int32_t)P->lay.fixed_dpad;
    if (P->sbin_cap_opt > 0) {
        g.cap = (int32_t)P->sbin_cap_opt;
    } else {
        // mean count of a run when every slot changes and rows are uniform, plus 7 standard deviations
        const double mu = (double)kScatterSpan * g.dpad / g.nrb;
        g.cap = (int32_t)(16 * ceil_div((int64_t)std::ceil(mu + 7.0 * std::sqrt(mu) + 16.0), 16));
    }
    if (P->sbins && P->sbin_tau == P->tau && P->sgeo.nrb == g.nrb && P->sgeo.cap == g.cap &&
        P->sgeo.dpad == g.dpad) {
        P->srows = true;
        return PCDM_OK;
    }
    free_sbins(P);
    P->srows = false;
    const size_t lds = sbin_lds_bytes(g.nrb, g.dpad);
    hipError_t e = hipMalloc(&P->sbins, (size_t)g.nrb * g.nwg * g.cap * sizeof(BinEntry));
    if (e == hipSuccess)
        e = hipMalloc(&P->scounts, (size_t)g.nrb * g.nwg * sizeof(int32_t));
    if (e == hipSuccess)
        e = hipMalloc(&P->ssync, 2 * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMemset(P->ssync, 0, 2 * sizeof(uint32_t));
    if (e == hipSuccess)
        e = P->dtype == PCDM_BF16
                ? hipFuncSetAttribute((const void *)k_sbin<bf16s>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
                : hipFuncSetAttribute((const void *)k_sbin<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) {
        free_sbins(P);
        (void)hipGetLastError();
        return hip_fail(e, "row-block scatter set-up");
    }
    P->sgeo = g;
    P->sbin_tau = P->tau;
    P->srows = true;
    return PCDM_OK;
}

// ---------------------------------------------------------------------------
// Per value type operations.
// ---------------------------------------------------------------------------

template <typename V> struct Ops {
    using T = typename ValT<V>::T;

    // The residual scatter of a step over 64-slot tiles: hardware atomics
    // (k_scatter), or row blocks (k_sbin, k_sapply).
    template <int G> static void launch_scatter(pcdm_problem *P, hipStream_t s)
    {
        hipEvent_t t1 = clock_start(P, s);
        if constexpr (!std::is_same<V, double>::value) {
            if (P->srows && P->sbins && P->sbin_tau == P->tau) {
                const SbinGeom geo = P->sgeo;
                hipLaunchKernelGGL((k_sbin<V>), dim3((unsigned)geo.nwg), dim3(kSbinThreads),
                                   sbin_lds_bytes(geo.nrb, geo.dpad), s, (const char *)P->seg, P->lay, geo, (T *)P->r,
                                   (const int32_t *)P->id_slot, (const T *)P->delta_slot, P->ctrl, P->tau,
                                   (BinEntry *)P->sbins, P->scounts, P->ssync);
                hipLaunchKernelGGL((k_sapply<T>), dim3((unsigned)geo.nrb), dim3(kSapplyThreads), 0, s,
                                   (const BinEntry *)P->sbins, (const int32_t *)P->scounts, geo, P->m, (T *)P->r,
                                   P->ssync);
                clock_stop(P, CLK_SCATTER, t1, s);
                return;
            }
        }
        const int sgrid = grid_for(P->tau, kScatterSpan, P->nblk_max);
        hipLaunchKernelGGL((k_scatter<V, G>), dim3(sgrid), dim3(kBlock), 0, s, (const char *)P->seg, P->lay,
                           (T *)P->r, (const int32_t *)P->id_slot, (const T *)P->delta_slot, P->ctrl, P->tau);
        clock_stop(P, CLK_SCATTER, t1, s);
    }

    // Partial derivatives by rows (k_bin, k_bin_dot, k_bin_prox), then the scatter.
    template <int G, int C> static void launch_binned(pcdm_problem *P, hipStream_t s)
    {
        const BinGeom geo = P->bgeo;
        const int64_t na = ceil_div(P->tau, kBinSlotsA);
        const int64_t nb = ceil_div(P->tau, kBinBlock);
        hipEvent_t t0 = clock_start(P, s);
        hipLaunchKernelGGL((k_bin<V>), dim3((unsigned)std::min<int64_t>(na, std::max(P->cus, 1))), dim3(kBinThreads),
                           bin_lds_bytes(geo.ns, geo.dpad), s,
                           (const char *)P->seg, P->lay, geo, (const Ctrl *)P->ctrl, P->seed, P->tau, (uint32_t)P->n,
                           P->id_slot, (v2d_t *)P->bhdr, (BinEntry *)P->bins, P->bcounts, P->bover);
        hipLaunchKernelGGL((k_bin_dot<T>), dim3((unsigned)(kBinRanges * nb)), dim3(kBinDotThreads), 0, s,
                           (const BinEntry *)P->bins, (const int32_t *)P->bcounts, (const T *)P->r, geo, P->tau, na,
                           (T *)P->bpart);
        const int grid = grid_for(P->tau, kBlock, P->nblk_max);
        hipLaunchKernelGGL((k_bin_prox<V, G, C>), dim3(grid), dim3(kBlock), 0, s, P->seg, P->lay, (const T *)P->r,
                           P->x, P->id_slot, (T *)P->delta_slot, (const Ctrl *)P->ctrl, P->nz_part, P->seed, P->tau,
                           (uint32_t)P->n, 1.0 / P->beta, prox_params(P), (const v2d_t *)P->bhdr,
                           (const T *)P->bpart, P->bover);
        clock_stop(P, CLK_GATHER, t0, s);
        launch_scatter<G>(P, s);
    }

    template <int G, int C, int Loss> static void launch_step(pcdm_problem *P, hipStream_t s)
    {
        if constexpr (Loss == kLossSquare && !std::is_same<V, double>::value) {
            if (P->binned && P->bins && P->bin_tau == P->tau) {
                launch_binned<G, C>(P, s);
                return;
            }
        }
        if (P->tau < P->narrow_below) {
            // one slot per group of G lanes
            const int grid = grid_for(P->tau * G, kBlock, P->nblk_max);
            hipEvent_t t0 = clock_start(P, s);
            hipLaunchKernelGGL((k_gather_narrow<V, G, C, Loss>), dim3(grid), dim3(kBlock), 0, s, P->seg, P->lay,
                               (const T *)P->r, P->x, P->id_slot, (T *)P->delta_slot, P->ctrl, P->nz_part, P->seed,
                               P->tau, (uint32_t)P->n, 1.0 / P->beta, prox_params(P), slot_plan(P));
            clock_stop(P, CLK_GATHER, t0, s);
            if (P->srows && P->sbins && P->sbin_tau == P->tau) {
                launch_scatter<G>(P, s);
                return;
            }
            hipEvent_t t1 = clock_start(P, s);
            hipLaunchKernelGGL((k_scatter_narrow<V, G>), dim3(grid), dim3(kBlock), 0, s, (const char *)P->seg,
                               P->lay, (T *)P->r, (const int32_t *)P->id_slot, (const T *)P->delta_slot, P->ctrl,
                               P->tau);
            clock_stop(P, CLK_SCATTER, t1, s);
            return;
        }
        const int grid = grid_for(P->tau, kBlock, P->nblk_max);  // one slot per thread per tile
        hipEvent_t t0 = clock_start(P, s);
        hipLaunchKernelGGL((k_gather<V, G, C, Loss>), dim3(grid), dim3(kBlock), 0, s, P->seg, P->lay,
                           (const T *)P->r, P->x, P->id_slot, (T *)P->delta_slot, P->ctrl, P->nz_part,
                           P->seed, P->tau, (uint32_t)P->n, 1.0 / P->beta, prox_params(P), slot_plan(P));
        clock_stop(P, CLK_GATHER, t0, s);
        launch_scatter<G>(P, s);
    }

    // One call of the asynchronous variant: `picks` picks over P processors
    // (lane groups), in launches of async_rounds rounds; returns P.
    template <int G, int C> static int64_t launch_async(pcdm_problem *P, int64_t picks, hipStream_t s)
    {
        int mode = P->async_reads;
        if (mode < 0) {
            // few processors: each pick's latency chain dominates, fresh reads
            // through the acquire cost little; many: plain reads, launch
            // boundaries every few rounds
            const int64_t want = P->async_procs_opt > 0 ? P->async_procs_opt : P->tau;
            mode = want <= kAsyncAcquireProcs ? kReadAcquire : kReadCached;
        }
        switch (mode) {
        case kReadAcquire: return launch_async_as<G, C, kReadAcquire>(P, picks, s);
        case kReadAtomic: return launch_async_as<G, C, kReadAtomic>(P, picks, s);
        default: return launch_async_as<G, C, kReadCached>(P, picks, s);
        }
    }

    template <int G, int C, int Mode> static int64_t launch_async_as(pcdm_problem *P, int64_t picks, hipStream_t s)
    {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_async<V, G, C, Mode>, kBlock, 0) !=
                hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        const int64_t gpb = (kBlock / 64) * (64 / G);  // lane groups per block
        const int64_t resident = (int64_t)per_cu * std::max(P->cus, 1) * gpb;
        int64_t procs = P->async_procs_opt > 0 ? P->async_procs_opt : std::min<int64_t>(P->tau, resident);
        procs = std::max<int64_t>(1, std::min<int64_t>(procs, picks));
        const int64_t blocks = std::min<int64_t>(ceil_div(procs, gpb), P->nblk_max);
        procs = std::min<int64_t>(procs, blocks * gpb);
        const int64_t per_launch = (Mode == kReadCached && P->async_rounds > 0) ? P->async_rounds * procs : picks;
        for (int64_t u0 = 0; u0 < picks; u0 += per_launch) {
            const int64_t cnt = std::min(per_launch, picks - u0);
            hipEvent_t t0 = clock_start(P, s);
            hipLaunchKernelGGL((k_async<V, G, C, Mode>), dim3((unsigned)blocks), dim3(kBlock), 0, s, P->seg, P->lay,
                               (T *)P->r, P->nz_part, P->seed, (uint64_t)P->async_launches, u0, cnt, procs,
                               (uint32_t)P->n, 1.0 / P->beta, P->lambda);
            clock_stop(P, CLK_ASYNC, t0, s);
        }
        const int gn = grid_for(P->n, kBlock, P->nblk_max);
        hipLaunchKernelGGL((k_records_to_x<V>), dim3(gn), dim3(kBlock), 0, s, (const char *)P->seg, P->lay, P->x,
                           P->n);
        return procs;
    }

    static int async_once(pcdm_problem *P, int64_t picks, hipStream_t s, int64_t &procs)
    {
        switch (P->lanes * 16 + P->chunks) {
        case 1 * 16 + 1: procs = launch_async<1, 1>(P, picks, s); break;
        case 1 * 16 + 2: procs = launch_async<1, 2>(P, picks, s); break;
        case 1 * 16 + 4: procs = launch_async<1, 4>(P, picks, s); break;
        case 2 * 16 + 1: procs = launch_async<2, 1>(P, picks, s); break;
        case 2 * 16 + 2: procs = launch_async<2, 2>(P, picks, s); break;
        case 2 * 16 + 4: procs = launch_async<2, 4>(P, picks, s); break;
        case 4 * 16 + 1: procs = launch_async<4, 1>(P, picks, s); break;
        case 4 * 16 + 2: procs = launch_async<4, 2>(P, picks, s); break;
        case 8 * 16 + 1: procs = launch_async<8, 1>(P, picks, s); break;
        case 8 * 16 + 2: procs = launch_async<8, 2>(P, picks, s); break;
        case 16 * 16 + 1: procs = launch_async<16, 1>(P, picks, s); break;
        case 32 * 16 + 1: procs = launch_async<32, 1>(P, picks, s); break;
        case 64 * 16 + 1: procs = launch_async<64, 1>(P, picks, s); break;
        default: return fail(PCDM_EINVAL, "unsupported (lanes_per_column, chunks_per_lane) pair");
        }
        return PCDM_OK;
    }

    template <int G> static void launch_group(pcdm_problem *P, hipStream_t s)
    {
        const int grid = grid_for(P->tau * G, kBlock, P->nblk_max);
        hipEvent_t t0 = clock_start(P, s);
        hipLaunchKernelGGL((k_group_gather<V, G>), dim3(grid), dim3(kBlock), 0, s, P->seg, P->lay, (const T *)P->r,
                           P->x, (const int64_t *)P->bp, (const double *)P->invlb, P->id_slot, (T *)P->dx, P->ctrl,
                           P->nz_part, P->seed, P->tau, (uint32_t)P->nb, 1.0 / P->beta, P->lambda);
        clock_stop(P, CLK_GATHER, t0, s);
        hipEvent_t t1 = clock_start(P, s);
        const int sgrid = grid_for(P->tau, kGroupScatterSpan, P->nblk_max);
        hipLaunchKernelGGL((k_group_scatter<V, G>), dim3(sgrid), dim3(kBlock), 0, s, (const char *)P->seg, P->lay,
                           (T *)P->r, (const int64_t *)P->bp, (const int32_t *)P->id_slot, (const T *)P->dx, P->ctrl,
                           P->tau);
        clock_stop(P, CLK_SCATTER, t1, s);
    }

    static int group_once(pcdm_problem *P, hipStream_t s)
    {
        switch (P->lanes) {
        case 1: launch_group<1>(P, s); return PCDM_OK;
        case 2: launch_group<2>(P, s); return PCDM_OK;
        case 4: launch_group<4>(P, s); return PCDM_OK;
        case 8: launch_group<8>(P, s); return PCDM_OK;
        case 16: launch_group<16>(P, s); return PCDM_OK;
        case 32: launch_group<32>(P, s); return PCDM_OK;
        case 64: launch_group<64>(P, s); return PCDM_OK;
        default: return fail(PCDM_EINVAL, "unsupported lanes_per_column");
        }
    }

    // ctrl->scal[2] = sum_i ||x^(i)||, and with gap ctrl->scal[3] = max_i ||A_i^T r64||.
    static void group_sums(pcdm_problem *P, bool gap, hipStream_t s)
    {
        const int g = grid_for(P->nb, kBlock, P->nblk_max);
        hipLaunchKernelGGL(k_group_xnorms, dim3(g), dim3(kBlock), 0, s, (const int64_t *)P->bp, P->nb,
                           (const double *)P->x, P->part2);
        hipLaunchKernelGGL(k_final, dim3(1), dim3(kBlock), 0, s, (const double *)P->part2, g, 1, 0, P->ctrl->scal + 2);
        if (gap) {
            // max_i ||A_i^T r64||_2: two passes as for the coordinate maximum
            // (bound over fl32(r64), exact norms of the candidate blocks), or one
            const int ga = grid_for(P->nb * 8, kBlock, P->nblk_max);
            const bool two = !std::is_same<V, double>::value && P->t32 && P->ub && passes(P) != 1;
            if (two)
                P->inc_valid = false;  // ub will hold block bounds
            if (two) {
                const int gm = grid_for(P->m, kBlock, P->nblk_max);
                hipLaunchKernelGGL((k_narrow<float>), dim3(gm), dim3(kBlock), 0, s, (const double *)P->r64, P->t32,
                                   P->m);
                hipLaunchKernelGGL((k_group_atr_bound<V, 8>), dim3(ga), dim3(kBlock), 0, s, (const char *)P->seg,
                                   P->lay, (const float *)P->t32, (const int64_t *)P->bp, P->nb, P->ub, P->part2);
                hipLaunchKernelGGL(k_final, dim3(1), dim3(kBlock), 0, s, (const double *)P->part2, ga, 1, 1,
                                   P->ctrl->scal + 3);
            }
            hipLaunchKernelGGL((k_group_atr<V, 8>), dim3(ga), dim3(kBlock), 0, s, (const char *)P->seg, P->lay,
                               (const double *)P->r64, (const int64_t *)P->bp, P->nb,
                               two ? (const float *)P->ub : nullptr, (const double *)(P->ctrl->scal + 3), P->part2);
            hipLaunchKernelGGL(k_final, dim3(1), dim3(kBlock), 0, s, (const double *)P->part2, ga, 1, 1,
                               P->ctrl->scal + 3);
        }
    }

    static void group_setup(pcdm_problem *P, int32_t *hist, hipStream_t s)
    {
        const int g = grid_for(P->nb, 1, 4 * P->nblk_max);
        hipLaunchKernelGGL((k_group_setup<V>), dim3(g), dim3(kBlock), 0, s, (const char *)P->seg, P->lay,
                           (const int64_t *)P->bp, P->nb, P->invlb, hist, P->ctrl);
    }

    static int step_once(pcdm_problem *P, hipStream_t s)
    {
        if (P->group)
            return group_once(P, s);
        switch (P->loss) {
        case kLossLogistic: return step_loss<kLossLogistic>(P, s);
        case kLossSqHinge: return step_loss<kLossSqHinge>(P, s);
        default: return step_loss<kLossSquare>(P, s);
        }
    }

    template <int Loss> static int step_loss(pcdm_problem *P, hipStream_t s)
    {
        // the square loss has every schedule; the others one chunk per lane
        constexpr bool all = Loss == kLossSquare;
        switch (P->lanes * 16 + P->chunks) {
        case 1 * 16 + 1: launch_step<1, 1, Loss>(P, s); return PCDM_OK;
        case 2 * 16 + 1: launch_step<2, 1, Loss>(P, s); return PCDM_OK;
        case 4 * 16 + 1: launch_step<4, 1, Loss>(P, s); return PCDM_OK;
        case 8 * 16 + 1: launch_step<8, 1, Loss>(P, s); return PCDM_OK;
        case 16 * 16 + 1: launch_step<16, 1, Loss>(P, s); return PCDM_OK;
        case 32 * 16 + 1: launch_step<32, 1, Loss>(P, s); return PCDM_OK;
        case 64 * 16 + 1: launch_step<64, 1, Loss>(P, s); return PCDM_OK;
        default: break;
        }
        if constexpr (all) {
            switch (P->lanes * 16 + P->chunks) {
            case 1 * 16 + 2: launch_step<1, 2, Loss>(P, s); return PCDM_OK;
            case 1 * 16 + 4: launch_step<1, 4, Loss>(P, s); return PCDM_OK;
            case 2 * 16 + 2: launch_step<2, 2, Loss>(P, s); return PCDM_OK;
            case 2 * 16 + 4: launch_step<2, 4, Loss>(P, s); return PCDM_OK;
            case 4 * 16 + 2: launch_step<4, 2, Loss>(P, s); return PCDM_OK;
            case 8 * 16 + 2: launch_step<8, 2, Loss>(P, s); return PCDM_OK;
            default: break;
            }
        }
        return fail(PCDM_EINVAL, "unsupported (lanes_per_column, chunks_per_lane) pair");
    }

    // F = lscale * sum_j phi(r64_j) + sum_i Omega(x_i) into ctrl->scal[0..1]
    // (r64 already A x - b).
    static void model_sums(pcdm_problem *P, hipStream_t s)
    {
        const ProxParams pp = prox_params(P);
        switch (P->loss) {
        case kLossLogistic:
            hipLaunchKernelGGL(k_model_partials<kLossLogistic>, dim3(kReduceBlocks), dim3(kBlock), 0, s,
                               (const double *)P->r64, P->m, (const double *)P->x, P->n, pp, P->part);
            break;
        case kLossSqHinge:
            hipLaunchKernelGGL(k_model_partials<kLossSqHinge>, dim3(kReduceBlocks), dim3(kBlock), 0, s,
                               (const double *)P->r64, P->m, (const double *)P->x, P->n, pp, P->part);
            break;
        default:
            hipLaunchKernelGGL(k_model_partials<kLossSquare>, dim3(kReduceBlocks), dim3(kBlock), 0, s,
                               (const double *)P->r64, P->m, (const double *)P->x, P->n, pp, P->part);
            break;
        }
        hipLaunchKernelGGL(k_final, dim3(1), dim3(kBlock), 0, s, (const double *)P->part, kReduceBlocks, 2, 0,
                           P->ctrl->scal);
    }

    static void fold_and_scale(pcdm_problem *P, const double *labels, double invl_factor, hipStream_t s)
    {
        const int gn = grid_for(P->n, kBlock, P->nblk_max);
        if (labels)
            hipLaunchKernelGGL((k_fold_labels<V>), dim3(gn), dim3(kBlock), 0, s, P->seg, P->lay, P->n, labels,
                               P->ctrl);
        if (invl_factor != 1.0)
            hipLaunchKernelGGL((k_scale_invl<V>), dim3(gn), dim3(kBlock), 0, s, P->seg, P->lay, P->n, invl_factor);
    }

    // r64 = A x - b in float64.
    static void residual64(pcdm_problem *P, hipStream_t s)
    {
        const int gm = grid_for(P->m, kBlock, P->nblk_max);
        const int gn = grid_for(P->n, kBlock, P->nblk_max);
        hipLaunchKernelGGL(k_neg_copy, dim3(gm), dim3(kBlock), 0, s, (const double *)P->b64, P->r64, P->m);
        hipLaunchKernelGGL((k_refresh_cols<V, 8>), dim3(gn), dim3(kBlock), 0, s, (const char *)P->seg, P->lay,
                           (const double *)P->x, P->r64, P->n);
    }

    static void refresh(pcdm_problem *P, hipStream_t s)
    {
        residual64(P, s);
        const int gm = grid_for(P->m, kBlock, P->nblk_max);
        hipLaunchKernelGGL((k_narrow<T>), dim3(gm), dim3(kBlock), 0, s, (const double *)P->r64, (T *)P->r, P->m);
    }

    // ctrl->scal[3] = max_i |a_i^T rv| (rv: device, m doubles).  Values of at
    // most float32 precision take the two-pass route (a bound pass over
    // fl32(rv), then the exact sums for the candidate columns only); it
    // returns the same number as the single exact pass.
    static int atr_absmax(pcdm_problem *P, const double *rv, hipStream_t s)
    {
        const int grid = grid_for(P->n, kBlock, P->nblk_max);
        const int mp = passes(P);
        const bool inc_route = mp == 3 && P->rold;
        if (inc_route && P->inc_valid) {
            // bounds moved from the last evaluation; taken when few columns remain
            const int gm = grid_for(P->m, kBlock, kReduceBlocks);
            hipLaunchKernelGGL(k_inc_sums, dim3(gm), dim3(kBlock), 0, s, rv, (const double *)P->rold, P->m, P->part);
            hipLaunchKernelGGL(k_final, dim3(1), dim3(kBlock), 0, s, (const double *)P->part, gm, 3, 1, P->inc + 1);
            hipLaunchKernelGGL(k_inc_prepare, dim3(1), dim3(1), 0, s, P->inc, P->nrm_max, P->gam);
            hipLaunchKernelGGL((k_fill<unsigned long long>), dim3(1), dim3(kBlock), 0, s, P->cnt, 0ull, (int64_t)1);
            hipLaunchKernelGGL(k_inc_count, dim3(grid), dim3(kBlock), 0, s, (const float *)P->ub,
                               (const float *)P->nrm, P->n, (const double *)P->inc, P->cnt);
            unsigned long long c = 0;
            HIP_TRY(hipMemcpyAsync(&c, P->cnt, 8, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            P->inc_cands = (int64_t)c;
            if ((int64_t)c <= P->n / 8) {
                P->inc_hits++;
                hipLaunchKernelGGL((k_atr_inc<V, 8>), dim3(grid), dim3(kBlock), 0, s, (const char *)P->seg, P->lay,
                                   rv, P->n, P->ub, (const float *)P->nrm, (const double *)P->inc, P->part2);
                hipLaunchKernelGGL(k_final, dim3(1), dim3(kBlock), 0, s, (const double *)P->part2, grid, 1, 1,
                                   P->ctrl->scal + 3);
                keep_state(P, rv, s);
                return PCDM_OK;
            }
        }
        if (std::is_same<V, double>::value || !P->t32 || !P->ub || mp == 1) {
            // touches neither ub nor the kept state
            hipLaunchKernelGGL((k_atr_absmax<V, 8>), dim3(grid), dim3(kBlock), 0, s, (const char *)P->seg, P->lay,
                               rv, P->n, P->part2);
        } else {
            const int gm = grid_for(P->m, kBlock, P->nblk_max);
            hipLaunchKernelGGL((k_narrow<float>), dim3(gm), dim3(kBlock), 0, s, rv, P->t32, P->m);
            hipLaunchKernelGGL((k_atr_bound<V, 8>), dim3(grid), dim3(kBlock), 0, s, (const char *)P->seg, P->lay,
                               (const float *)P->t32, P->n, P->ub, P->part2);
            hipLaunchKernelGGL(k_final, dim3(1), dim3(kBlock), 0, s, (const double *)P->part2, grid, 1, 1,
                               P->ctrl->scal + 3);
            hipLaunchKernelGGL((k_atr_exact<V, 8>), dim3(grid), dim3(kBlock), 0, s, (const char *)P->seg, P->lay,
                               rv, P->n, (const float *)P->ub, (const double *)(P->ctrl->scal + 3), P->part2);
        }
        hipLaunchKernelGGL(k_final, dim3(1), dim3(kBlock), 0, s, (const double *)P->part2, grid, 1, 1,
                           P->ctrl->scal + 3);
        if (!std::is_same<V, double>::value && P->t32 && P->ub && mp != 1) {
            // ub now holds bounds for rv
            if (inc_route)
                keep_state(P, rv, s);
            else
                P->inc_valid = false;
        }
        return PCDM_OK;
    }

    // The incremental route's state after an evaluation at rv: r_old = rv,
    // M_old = the result.
    static void keep_state(pcdm_problem *P, const double *rv, hipStream_t s)
    {
        const int gm = grid_for(P->m, kBlock, P->nblk_max);
        hipLaunchKernelGGL(k_copy_f64, dim3(gm), dim3(kBlock), 0, s, rv, P->rold, P->m);
        hipLaunchKernelGGL(k_copy_f64, dim3(1), dim3(kBlock), 0, s, (const double *)(P->ctrl->scal + 3), P->inc,
                           (int64_t)1);
        P->inc_valid = true;
    }

    // Column l1 norms for the incremental route (rounded up) and their maximum.
    static int col_norms(pcdm_problem *P, hipStream_t s)
    {
        const int grid = grid_for(P->n, kBlock, P->nblk_max);
        const double dmax = P->lay.fixed_dpad ? (double)P->lay.fixed_dpad : (double)P->m;
        hipLaunchKernelGGL((k_col_norms<V, 8>), dim3(grid), dim3(kBlock), 0, s, (const char *)P->seg, P->lay, P->n,
                           inc_l1_factor(dmax), P->nrm, P->part2);
        hipLaunchKernelGGL(k_final, dim3(1), dim3(kBlock), 0, s, (const double *)P->part2, grid, 1, 1,
                           P->ctrl->scal + 5);
        double v = 0.0;
        HIP_TRY(hipMemcpyAsync(&v, P->ctrl->scal + 5, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        P->nrm_max = v;
        P->gam = inc_gamma(dmax);
        return PCDM_OK;
    }

    // ctrl->scal[0..2] = ||r64||^2, b.r64, ||x||_1
    static void sums(pcdm_problem *P, hipStream_t s)
    {
        hipLaunchKernelGGL(k_obj_partials, dim3(kReduceBlocks), dim3(kBlock), 0, s,
                           (const double *)P->r64, (const double *)P->b64, (const double *)P->x, P->m, P->n,
                           P->part);
        hipLaunchKernelGGL(k_final, dim3(1), dim3(kBlock), 0, s, (const double *)P->part, kReduceBlocks, 3, 0,
                           P->ctrl->scal);
    }

    static void adj_hist(pcdm_problem *P, const int32_t *S, int64_t ns, int32_t *hist, hipStream_t s)
    {
        const int g = grid_for(ns, kBlock, P->nblk_max);
        hipLaunchKernelGGL((k_adj_hist<V>), dim3(g), dim3(kBlock), 0, s, (const char *)P->seg, P->lay, S, ns, hist);
    }

    static void adj_step(pcdm_problem *P, const int32_t *S, const double *gS, double *vS, double *rho,
                         int32_t *ids, double *dels, uint64_t seed, uint64_t step, int64_t tau, int64_t ns,
                         double inv_beta, hipStream_t s)
    {
        const int g = grid_for(tau, kBlock, P->nblk_max);
        hipLaunchKernelGGL((k_adj_gather<V, 8>), dim3(g), dim3(kBlock), 0, s, (const char *)P->seg, P->lay, S, gS,
                           vS, (const double *)rho, ids, dels, seed, step, tau, (uint32_t)ns, inv_beta);
        hipLaunchKernelGGL((k_adj_scatter<V, 8>), dim3(g), dim3(kBlock), 0, s, (const char *)P->seg, P->lay, rho,
                           (const int32_t *)ids, (const double *)dels, tau);
    }

    // rho = A_S v, then ctrl->scal[4] = max_c |a_{S_c}^T rho - g_c|
    static void adj_check(pcdm_problem *P, const int32_t *S, const double *gS, const double *vS, double *rho,
                          int64_t ns, hipStream_t s)
    {
        const int gm = grid_for(P->m, kBlock, P->nblk_max);
        const int g = grid_for(ns, kBlock, P->nblk_max);
        hipLaunchKernelGGL((k_fill<double>), dim3(gm), dim3(kBlock), 0, s, rho, 0.0, P->m);
        hipLaunchKernelGGL((k_adj_apply<V, 8>), dim3(g), dim3(kBlock), 0, s, (const char *)P->seg, P->lay, S, vS,
                           rho, ns);
        hipLaunchKernelGGL((k_adj_resid<V, 8>), dim3(g), dim3(kBlock), 0, s, (const char *)P->seg, P->lay, S, gS,
                           (const double *)rho, ns, P->part2);
        hipLaunchKernelGGL(k_final, dim3(1), dim3(kBlock), 0, s, (const double *)P->part2, g, 1, 1,
                           P->ctrl->scal + 4);
    }

    static void x_to_records(pcdm_problem *P, hipStream_t s)
    {
        const int g = grid_for(P->n, kBlock, P->nblk_max);
        hipLaunchKernelGGL((k_x_to_records<V>), dim3(g), dim3(kBlock), 0, s, P->seg, P->lay, (const double *)P->x,
                           P->n);
    }

    static int pack(pcdm_problem *P, const int64_t *col_ptr, const int32_t *rows, const void *vals,
                    int32_t *hist, hipStream_t s)
    {
        const int gn = grid_for(P->n, kBlock, P->nblk_max);
        hipLaunchKernelGGL((k_pack<V>), dim3(gn), dim3(kBlock), 0, s, col_ptr, rows, (const V *)vals, P->lay,
                           P->n, P->m, P->seg, hist, P->ctrl);
        return PCDM_OK;
    }
};

template <typename F> int dispatch(int dtype, F &&f)
{
    switch (dtype) {
    case PCDM_F32: return f(Ops<float>());
    case PCDM_BF16: return f(Ops<bf16s>());
    case PCDM_F64: return f(Ops<double>());
    default: return fail(PCDM_EINVAL, "unknown dtype");
    }
}

int check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_fail(e, what);
    return PCDM_OK;
}

// Device address of `scratch` on device `dev`, looked up once per device
// (with that device current) and kept.
int scratch_base(int dev, void **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    if (dev < 0 || dev >= kMaxDevices)
        return fail(PCDM_EDEVICE, "device ordinal out of range for the fixed scratch");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        addr[dev] = p;
    }
    *out = addr[dev];
    return PCDM_OK;
}

// Device temporaries of one call, freed when it returns.
struct DevTemps {
    std::vector<void *> p;
    ~DevTemps()
    {
        for (void *q : p)
            if (q)
                (void)hipFree(q);
    }
    template <typename T> int get(T **out, size_t bytes)
    {
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, std::max<size_t>(bytes, 16));
        if (e != hipSuccess)
            return hip_fail(e, "temporary allocation");
        p.push_back(q);
        *out = (T *)q;
        return PCDM_OK;
    }
};

// Where one call's device temporaries come from: hipMalloc through a
// DevTemps (freed when the call returns), or consecutive 256-byte aligned
// pieces of a fixed device region that is never freed (no allocation at all).
struct TempSource {
    DevTemps *heap = nullptr;
    char *base = nullptr;
    size_t cap = 0, used = 0;
    const char *who = "";
    template <typename T> int get(T **out, size_t bytes)
    {
        if (heap)
            return heap->get(out, bytes);
        const size_t need = (std::max<size_t>(bytes, 16) + 255) & ~(size_t)255;
        if (used + need > cap)
            return fail(PCDM_EINVAL, std::string(who) + ": needs more than the fixed scratch of " +
                                         std::to_string(cap) + " bytes (" + std::to_string(used + need) +
                                         " bytes taken so far); call the allocating entry point instead");
        *out = (T *)(base + used);
        used += need;
        return PCDM_OK;
    }
};

int refresh_now(pcdm_problem *P, hipStream_t s)
{
    hipEvent_t t0 = clock_start(P, s);
    dispatch(P->dtype, [&](auto ops) {
        decltype(ops)::refresh(P, s);
        return PCDM_OK;
    });
    clock_stop(P, CLK_REFRESH, t0, s);
    return check_launch("refresh");
}

std::string describe_err(uint32_t e)
{
    std::string out;
    if (e & ERR_PTR) out += "col_ptr malformed (col_ptr[0] != 0, decreasing, or col_ptr[n] != nnz); ";
    if (e & ERR_EMPTY) out += "empty column (the method needs L_i > 0); ";
    if (e & ERR_ROW) out += "row index out of [0, m); ";
    if (e & ERR_DUP) out += "repeated row index within a column; ";
    if (e & ERR_NONFINITE) out += "non-finite value; ";
    if (e & ERR_ZEROCOL) out += "column with only zero values (L_i = 0); ";
    if (e & ERR_LABEL) out += "label other than +1 / -1; ";
    return out;
}

int create_impl(const pcdm_csc *A, const double *b, double lambda, int64_t tau, uint64_t seed,
                const pcdm_model *model, pcdm_problem **out)
{
    if (!out)
        return fail(PCDM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!A || !b)
        return fail(PCDM_EINVAL, "A or b is NULL");
    if (A->m < 1 || A->n < 1 || A->m > INT32_MAX || A->n > INT32_MAX - 1)
        return fail(PCDM_EINVAL, "need 1 <= m <= 2^31 - 1 and 1 <= n <= 2^31 - 2");
    if (A->nnz < A->n || A->nnz > (int64_t)1 << 40)
        return fail(PCDM_EINVAL, "nnz must be >= n (no empty column) and < 2^40");
    if (!A->col_ptr || !A->row_idx || !A->values)
        return fail(PCDM_EINVAL, "A has a NULL array");
    if (value_bytes(A->dtype) == 0)
        return fail(PCDM_EINVAL, "unknown dtype");
    if (tau < 1 || tau > A->n)
        return fail(PCDM_EINVAL, "need 1 <= tau <= n");
    if ((uint64_t)A->m * (A->dtype == PCDM_F64 ? 8u : 4u) >= (1ull << 32))
        return fail(PCDM_EINVAL, "the residual must span < 4 GiB (m < 2^30 for float32/bf16, m < 2^29 for float64)");
    if (!(lambda >= 0.0) || !std::isfinite(lambda))
        return fail(PCDM_EINVAL, "lambda must be finite and >= 0");

    pcdm_problem *P = new (std::nothrow) pcdm_problem();
    if (!P)
        return fail(PCDM_ENOMEM, "host allocation failed");
    struct Guard {
        pcdm_problem *p;
        void *tmp[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
        ~Guard()
        {
            for (void *t : tmp)
                if (t)
                    (void)hipFree(t);
            free_problem(p);
        }
    } guard{P};

    HIP_TRY(hipGetDevice(&P->device));
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P->device));
    P->nblk_max = std::max(64, cus * PCDM_BLOCKS_PER_CU);
    P->cus = cus;
    P->m = A->m;
    P->n = A->n;
    P->nnz = A->nnz;
    P->tau = tau;
    P->dtype = A->dtype;
    P->tbytes = (A->dtype == PCDM_F64) ? 8 : 4;
    P->lambda = lambda;
    P->seed = seed;
    const size_t vb = value_bytes(A->dtype);
    hipStream_t s = nullptr;

    // Inputs on the device (copied there first when given on the host).
    const int64_t *col_ptr = A->col_ptr;
    const int32_t *rows = A->row_idx;
    const void *vals = A->values;
    const double *bdev = b;
    if (!A->on_device) {
        HIP_TRY(hipMalloc(&guard.tmp[0], (size_t)(A->n + 1) * 8));
        HIP_TRY(hipMalloc(&guard.tmp[1], (size_t)A->nnz * 4));
        HIP_TRY(hipMalloc(&guard.tmp[2], (size_t)A->nnz * vb));
        HIP_TRY(hipMalloc(&guard.tmp[3], (size_t)A->m * 8));
        HIP_TRY(hipMemcpy(guard.tmp[0], A->col_ptr, (size_t)(A->n + 1) * 8, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(guard.tmp[1], A->row_idx, (size_t)A->nnz * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(guard.tmp[2], A->values, (size_t)A->nnz * vb, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(guard.tmp[3], b, (size_t)A->m * 8, hipMemcpyHostToDevice));
        col_ptr = (const int64_t *)guard.tmp[0];
        rows = (const int32_t *)guard.tmp[1];
        vals = guard.tmp[2];
        bdev = (const double *)guard.tmp[3];
    }

    HIP_TRY(hipMalloc(&P->ctrl, sizeof(Ctrl)));
    HIP_TRY(hipMemset(P->ctrl, 0, sizeof(Ctrl)));
    HIP_TRY(hipMalloc(&P->nz_part, (size_t)P->nblk_max * 8));
    HIP_TRY(hipMemset(P->nz_part, 0, (size_t)P->nblk_max * 8));
    HIP_TRY(hipMalloc(&P->part, (size_t)kReduceBlocks * 3 * 8));
    HIP_TRY(hipMalloc(&P->part2, (size_t)P->nblk_max * 8));

    // Padded column pointers.
    int64_t *dpad = nullptr;
    HIP_TRY(hipMalloc(&guard.tmp[4], (size_t)(A->n + 1) * 8));
    dpad = (int64_t *)guard.tmp[4];
    HIP_TRY(hipMalloc(&P->pc, (size_t)(A->n + 1) * 8));
    {
        const int g = grid_for(A->n + 1, kBlock, P->nblk_max);
        hipLaunchKernelGGL(k_check_ptr, dim3(g), dim3(kBlock), 0, s, col_ptr, A->n, A->nnz, dpad, P->ctrl);
        PCDM_TRY(check_launch("k_check_ptr"));
        Ctrl hc;
        HIP_TRY(hipMemcpy(&hc, P->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
        if (hc.err)
            return fail(PCDM_EINVAL, "invalid matrix: " + describe_err(hc.err));
        size_t tmp_bytes = 0;
        HIP_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, dpad, P->pc, (int)(A->n + 1), s));
        HIP_TRY(hipMalloc(&guard.tmp[5], std::max<size_t>(tmp_bytes, 16)));
        HIP_TRY(hipcub::DeviceScan::ExclusiveSum(guard.tmp[5], tmp_bytes, dpad, P->pc, (int)(A->n + 1), s));
        HIP_TRY(hipMemcpy(&P->stored_nnz, P->pc + A->n, 8, hipMemcpyDeviceToHost));
        hipLaunchKernelGGL(k_check_uniform, dim3(g), dim3(kBlock), 0, s, (const int64_t *)dpad, A->n, P->ctrl);
        PCDM_TRY(check_launch("k_check_uniform"));
        HIP_TRY(hipMemcpy(&hc, P->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
        P->lay.pc = P->pc;
        if (!hc.nonuniform) {
            HIP_TRY(hipMemcpy(&P->lay.fixed_dpad, dpad, 8, hipMemcpyDeviceToHost));
            const int64_t rec = kHeader + P->lay.fixed_dpad * (int64_t)(4 + vb);
            P->lay.stride = (rec + PCDM_RECORD_ALIGN - 1) / PCDM_RECORD_ALIGN * PCDM_RECORD_ALIGN;
        }
    }

    const size_t seg_bytes = P->lay.fixed_dpad ? (size_t)P->lay.stride * (size_t)A->n
                                               : (size_t)P->stored_nnz * (4 + vb) + (size_t)kHeader * A->n;
    HIP_TRY(hipMalloc(&P->seg, seg_bytes));
    HIP_TRY(hipMalloc(&P->x, (size_t)A->n * 8));
    HIP_TRY(hipMalloc(&P->r, (size_t)A->m * P->tbytes));
    HIP_TRY(hipMalloc(&P->r64, (size_t)A->m * 8));
    HIP_TRY(hipMalloc(&P->b64, (size_t)A->m * 8));
    if (P->dtype != PCDM_F64) {
        HIP_TRY(hipMalloc(&P->t32, (size_t)A->m * 4));
        HIP_TRY(hipMalloc(&P->ub, (size_t)A->n * 4));
        HIP_TRY(hipMalloc(&P->rold, (size_t)A->m * 8));
        HIP_TRY(hipMalloc(&P->nrm, (size_t)A->n * 4));
        HIP_TRY(hipMalloc(&P->inc, 8 * 8));
        HIP_TRY(hipMalloc(&P->cnt, 8));
    }
    HIP_TRY(hipMemset(P->x, 0, (size_t)A->n * 8));
    HIP_TRY(hipMemcpy(P->b64, bdev, (size_t)A->m * 8, hipMemcpyDeviceToDevice));
    PCDM_TRY(ensure_slots(P, tau));

    // Pack, L_i, row histogram.
    {
        int32_t *hist = nullptr;
        HIP_TRY(hipMalloc(&hist, (size_t)A->m * 4));
        hipError_t e = hipMemset(hist, 0, (size_t)A->m * 4);
        int st = PCDM_OK;
        if (e == hipSuccess)
            st = dispatch(P->dtype, [&](auto ops) { return decltype(ops)::pack(P, col_ptr, rows, vals, hist, s); });
        if (e == hipSuccess && st == PCDM_OK) {
            const int g = grid_for(A->m, kBlock, P->nblk_max);
            hipLaunchKernelGGL(k_imax_partials, dim3(g), dim3(kBlock), 0, s, (const int32_t *)hist, A->m,
                               (int64_t *)P->part2);
            hipLaunchKernelGGL(k_imax_final, dim3(1), dim3(kBlock), 0, s, (const int64_t *)P->part2, g, P->ctrl);
            e = hipDeviceSynchronize();
        }
        (void)hipFree(hist);
        if (e != hipSuccess)
            return hip_fail(e, "pack");
        PCDM_TRY(st);
        PCDM_TRY(check_launch("k_pack"));
        Ctrl hc;
        HIP_TRY(hipMemcpy(&hc, P->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
        if (hc.err)
            return fail(PCDM_EINVAL, "invalid matrix: " + describe_err(hc.err));
        P->omega = hc.imax;
    }

    if (model) {
        // labels folded into the values, L_i scaled by s * sup(phi'')
        P->loss = model->loss;
        P->lscale = model->scale;
        P->l2 = model->l2;
        P->lin = model->linear;
        P->lo = model->lower;
        P->hi = model->upper;
        const double curv = P->loss == kLossLogistic ? 0.25 : 1.0;
        const double *labels = P->loss != kLossSquare ? P->b64 : nullptr;
        PCDM_TRY(dispatch(P->dtype, [&](auto ops) {
            decltype(ops)::fold_and_scale(P, labels, 1.0 / (P->lscale * curv), s);
            return PCDM_OK;
        }));
        PCDM_TRY(check_launch("model set-up"));
        Ctrl hc;
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipMemcpy(&hc, P->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
        if (hc.err & ERR_LABEL)
            return fail(PCDM_EINVAL, "labels of the logistic / square-hinge loss must be +1 or -1");
        if (labels) {
            const int gm = grid_for(A->m, kBlock, P->nblk_max);
            hipLaunchKernelGGL((k_fill<double>), dim3(gm), dim3(kBlock), 0, s, P->b64, 0.0, P->m);
        }
    }

    pick_schedule(P);
    P->lanes_auto = 1;
    compute_beta(P);
    P->refresh_every = ceil_div(P->n, P->tau);

    if (P->nrm)
        PCDM_TRY(dispatch(P->dtype, [&](auto ops) { return decltype(ops)::col_norms(P, s); }));

    // r = -b, ||A^T b||_inf.
    {
        const int gm = grid_for(A->m, kBlock, P->nblk_max);
        hipLaunchKernelGGL(k_neg_copy, dim3(gm), dim3(kBlock), 0, s, (const double *)P->b64, P->r64, P->m);
        PCDM_TRY(dispatch(P->dtype, [&](auto ops) {
            using T = typename decltype(ops)::T;
            hipLaunchKernelGGL((k_narrow<T>), dim3(gm), dim3(kBlock), 0, s, (const double *)P->r64, (T *)P->r,
                               P->m);
            return decltype(ops)::atr_absmax(P, P->r64, s);
        }));
        PCDM_TRY(check_launch("init residual"));
        Ctrl hc;
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipMemcpy(&hc, P->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
        P->atb_inf = hc.scal[3];
    }
    PCDM_TRY(route_update(P));
    PCDM_TRY(sroute_update(P));
    guard.p = nullptr;
    *out = P;
    return PCDM_OK;
}

// Everything the step kernels take from the host, as bytes: a captured graph
// is valid only while this is unchanged (the step counter is read on the
// device, so replays advance through successive steps).
std::vector<unsigned char> step_signature(const pcdm_problem *P)
{
    std::vector<unsigned char> sig;
    auto put = [&](const auto &v) {
        const unsigned char *b = reinterpret_cast<const unsigned char *>(&v);
        sig.insert(sig.end(), b, b + sizeof(v));
    };
    put(P->tau);
    put(P->beta);
    put(P->lambda);
    put(P->lanes);
    put(P->chunks);
    put(P->narrow_below);
    put(P->loss);
    put(P->lscale);
    put(P->l2);
    put(P->lin);
    put(P->lo);
    put(P->hi);
    put(P->sampling);
    put(P->pb);
    put(P->mask);
    put(P->mask_len);
    put(P->claim);
    put(P->claim_base);
    put(P->group);
    put(P->seed);
    put(P->id_slot);
    put(P->delta_slot);
    put(P->dx);
    put(P->binned);
    put(P->bins);
    put(P->bcounts);
    put(P->bhdr);
    put(P->bpart);
    put(P->bover);
    put(P->bgeo.cap);
    put(P->bgeo.ns);
    put(P->bin_tau);
    put(P->srows);
    put(P->sbins);
    put(P->scounts);
    put(P->ssync);
    put(P->sgeo.cap);
    put(P->sbin_tau);
    return sig;
}

int ensure_step_graph(pcdm_problem *P)
{
    std::vector<unsigned char> sig = step_signature(P);
    if (P->graph_exec && P->graph_captured_len == P->graph_len && sig == P->graph_sig)
        return PCDM_OK;
    drop_step_graph(P);
    if (!P->cap_stream)
        HIP_TRY(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
    int st = PCDM_OK;
    for (int64_t q = 0; q < P->graph_len && st == PCDM_OK; ++q)
        st = dispatch(P->dtype, [&](auto ops) { return decltype(ops)::step_once(P, P->cap_stream); });
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(P->cap_stream, &g);
    if (st != PCDM_OK || e != hipSuccess) {
        if (g)
            (void)hipGraphDestroy(g);
        return st != PCDM_OK ? st : hip_fail(e, "hipStreamEndCapture");
    }
    P->graph = g;
    HIP_TRY(hipGraphInstantiate(&P->graph_exec, P->graph, nullptr, nullptr, 0));
    P->graph_sig = std::move(sig);
    P->graph_captured_len = P->graph_len;
    return PCDM_OK;
}

}  // namespace

extern "C" {

const char *pcdm_last_error(void) { return t_err.c_str(); }

int pcdm_create(const pcdm_csc *A, const double *b, double lambda, int64_t tau, uint64_t seed,
                pcdm_problem **out)
{
    t_err.clear();
    try {
        return create_impl(A, b, lambda, tau, seed, nullptr, out);
    } catch (const std::exception &e) {
        return fail(PCDM_EDEVICE, std::string("exception: ") + e.what());
    } catch (...) {
        return fail(PCDM_EDEVICE, "unknown exception");
    }
}

int pcdm_create_model(const pcdm_csc *A, const double *y, const pcdm_model *model, int64_t tau, uint64_t seed,
                      pcdm_problem **out)
{
    t_err.clear();
    if (out)
        *out = nullptr;
    if (!model)
        return fail(PCDM_EINVAL, "model is NULL");
    if (model->loss < kLossSquare || model->loss > kLossSqHinge)
        return fail(PCDM_EINVAL, "loss must be PCDM_LOSS_SQUARE, PCDM_LOSS_LOGISTIC or PCDM_LOSS_SQHINGE");
    if (!(model->scale > 0.0) || !std::isfinite(model->scale))
        return fail(PCDM_EINVAL, "scale must be finite and > 0");
    if (!(model->l1 >= 0.0) || !std::isfinite(model->l1) || !(model->l2 >= 0.0) || !std::isfinite(model->l2))
        return fail(PCDM_EINVAL, "l1 and l2 must be finite and >= 0");
    if (!std::isfinite(model->linear))
        return fail(PCDM_EINVAL, "linear must be finite");
    if (!(model->lower <= 0.0) || !(model->upper >= 0.0))
        return fail(PCDM_EINVAL, "need lower <= 0 <= upper (x starts at 0)");
    try {
        return create_impl(A, y, model->l1, tau, seed, model, out);
    } catch (const std::exception &e) {
        return fail(PCDM_EDEVICE, std::string("exception: ") + e.what());
    } catch (...) {
        return fail(PCDM_EDEVICE, "unknown exception");
    }
}

int pcdm_create_group(const pcdm_csc *A, const double *b, double lambda, const int64_t *block_ptr, int64_t nblocks,
                      int64_t tau, uint64_t seed, pcdm_problem **out)
{
    t_err.clear();
    if (out)
        *out = nullptr;
    if (!A || !block_ptr || !out)
        return fail(PCDM_EINVAL, "NULL argument");
    if (nblocks < 1 || nblocks > A->n)
        return fail(PCDM_EINVAL, "need 1 <= nblocks <= n");
    if (tau < 1 || tau > nblocks)
        return fail(PCDM_EINVAL, "need 1 <= tau <= nblocks");
    std::vector<int64_t> hbp((size_t)nblocks + 1);
    if (A->on_device) {
        HIP_TRY(hipMemcpy(hbp.data(), block_ptr, hbp.size() * 8, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(hbp.data(), block_ptr, hbp.size() * 8);
    }
    if (hbp[0] != 0 || hbp[(size_t)nblocks] != A->n)
        return fail(PCDM_EINVAL, "block_ptr must start at 0 and end at n");
    for (int64_t i = 0; i < nblocks; ++i) {
        const int64_t sz = hbp[(size_t)i + 1] - hbp[(size_t)i];
        if (sz < 1 || sz > kGroupMax)
            return fail(PCDM_EINVAL, "every block needs 1 to 16 columns (block_ptr strictly increasing)");
    }
    pcdm_problem *P = nullptr;
    try {
        PCDM_TRY(create_impl(A, b, lambda, 1, seed, nullptr, &P));
    } catch (...) {
        return fail(PCDM_EDEVICE, "exception during create");
    }
    struct Guard {
        pcdm_problem *p;
        ~Guard() { free_problem(p); }
    } guard{P};
    hipStream_t s = nullptr;
    P->group = 1;
    P->nb = nblocks;
    HIP_TRY(hipMalloc(&P->bp, hbp.size() * 8));
    HIP_TRY(hipMemcpy(P->bp, hbp.data(), hbp.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&P->invlb, (size_t)nblocks * 8));
    HIP_TRY(hipMalloc(&P->dx, (size_t)P->n * P->tbytes));
    int32_t *hist = nullptr;
    HIP_TRY(hipMalloc(&hist, (size_t)P->m * 4));
    hipError_t e = hipMemset(hist, 0, (size_t)P->m * 4);
    if (e == hipSuccess) {
        (void)dispatch(P->dtype, [&](auto ops) {
            decltype(ops)::group_setup(P, hist, s);
            return PCDM_OK;
        });
        const int g = grid_for(P->m, kBlock, P->nblk_max);
        hipLaunchKernelGGL(k_imax_partials, dim3(g), dim3(kBlock), 0, s, (const int32_t *)hist, P->m,
                           (int64_t *)P->part2);
        hipLaunchKernelGGL(k_imax_final, dim3(1), dim3(kBlock), 0, s, (const int64_t *)P->part2, g, P->ctrl);
        e = hipDeviceSynchronize();
    }
    (void)hipFree(hist);
    if (e != hipSuccess)
        return hip_fail(e, "group set-up");
    PCDM_TRY(check_launch("group set-up"));
    Ctrl hc;
    HIP_TRY(hipMemcpy(&hc, P->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    if (hc.err)
        return fail(PCDM_EINVAL, "invalid block: " + describe_err(hc.err));
    P->omega = hc.imax;
    PCDM_TRY(ensure_slots(P, tau));
    P->tau = tau;
    P->lanes = 8;
    P->chunks = 1;
    P->lanes_auto = 1;
    compute_beta(P);
    P->refresh_every = ceil_div(P->nb, P->tau);
    guard.p = nullptr;
    *out = P;
    return PCDM_OK;
}

int pcdm_destroy(pcdm_problem *h)
{
    if (!h)
        return PCDM_OK;
    hipError_t e = hipDeviceSynchronize();
    free_problem(h);
    if (e != hipSuccess)
        return hip_fail(e, "pcdm_destroy");
    return PCDM_OK;
}

int pcdm_set_option(pcdm_problem *h, const char *key, double value)
{
    if (!h || !key)
        return fail(PCDM_EINVAL, "NULL handle or key");
    const std::string k(key);
    if (!std::isfinite(value))
        return fail(PCDM_EINVAL, "option value must be finite");
    if (k == "refresh_every") {
        if (value < 0)
            return fail(PCDM_EINVAL, "refresh_every must be >= 0");
        h->refresh_every = (value == 0.0) ? 0 : (int64_t)value;
    } else if (k == "beta_rule") {
        if (value != 0.0 && value != 1.0)
            return fail(PCDM_EINVAL, "beta_rule must be 0 (nice) or 1 (uniform)");
        h->beta_rule = (int)value;
        compute_beta(h);
    } else if (k == "beta") {
        if (!(value > 0.0))
            return fail(PCDM_EINVAL, "beta must be > 0");
        h->beta_rule = 2;
        h->beta = value;
    } else if (k == "lambda") {
        if (!(value >= 0.0))
            return fail(PCDM_EINVAL, "lambda must be >= 0");
        h->lambda = value;
    } else if (k == "tau") {
        const int64_t t = (int64_t)value;
        const int64_t units = h->group ? h->nb : h->n;
        if ((double)t != value || t < 1 || t > units)
            return fail(PCDM_EINVAL, "tau must be an integer in [1, n] (n blocks for a block problem)");
        PCDM_TRY(ensure_slots(h, t));
        h->tau = t;
        compute_beta(h);
        PCDM_TRY(route_update(h));
        PCDM_TRY(sroute_update(h));
    } else if (k == "lanes_per_column" || k == "chunks_per_lane") {
        const int v = (int)value;
        if ((double)v != value || v < 0)
            return fail(PCDM_EINVAL, k + " must be a non-negative integer");
        if (v == 0) {
            pick_schedule(h);
            h->lanes_auto = 1;
        } else {
            const int g = k == "lanes_per_column" ? v : h->lanes;
            const int c = k == "chunks_per_lane" ? v : (schedule_supported(v, h->chunks, h->loss) ? h->chunks : 1);
            if (!schedule_supported(g, c, h->loss) || (h->group && c != 1))
                return fail(PCDM_EINVAL, "unsupported (lanes_per_column, chunks_per_lane) pair");
            h->lanes = g;
            h->chunks = c;
            h->lanes_auto = 0;
        }
    } else if (k == "sampling") {
        const int v = (int)value;
        if (h->group && value != 0.0)
            return fail(PCDM_EINVAL, "block problems use the tau-nice sampling");
        if ((double)v != value || v < kSampleNice || v > kSampleBinomial)
            return fail(PCDM_EINVAL, "sampling must be 0 (tau-nice), 1 (tau-independent) or 2 (binomial)");
        if (v == kSampleIndependent && !h->claim) {
            HIP_TRY(hipMalloc(&h->claim, (size_t)h->n * sizeof(uint32_t)));
            reset_claims(h, h->k_host, h->last_stream);
            PCDM_TRY(check_launch("claim reset"));
        }
        h->sampling = v;
        compute_beta(h);
        PCDM_TRY(route_update(h));
    } else if (k == "binomial_p") {
        if (!(value > 0.0 && value <= 1.0))
            return fail(PCDM_EINVAL, "binomial_p must be in (0, 1]");
        h->pb = value;
        compute_beta(h);
    } else if (k == "async_processors") {
        if (!(value >= 0.0) || value > 9.0e15)
            return fail(PCDM_EINVAL, "async_processors must be >= 0");
        h->async_procs_opt = (int64_t)value;
    } else if (k == "async_reads") {
        if (value != -1.0 && value != 0.0 && value != 1.0 && value != 2.0)
            return fail(PCDM_EINVAL, "async_reads must be -1 (automatic), 0 (cached), 1 (acquire) or 2 (atomic)");
        h->async_reads = (int)value;
    } else if (k == "async_rounds") {
        if (!(value >= 0.0) || value > 9.0e15 || value != std::floor(value))
            return fail(PCDM_EINVAL, "async_rounds must be a non-negative integer");
        h->async_rounds = (int64_t)value;
    } else if (k == "graph_steps") {
        if (!(value >= 0.0) || value > 4096.0 || value != std::floor(value))
            return fail(PCDM_EINVAL, "graph_steps must be an integer in [0, 4096]");
        h->graph_len = (int64_t)value;
    } else if (k == "max_passes") {
        if (value != 0.0 && value != 1.0 && value != 2.0 && value != 3.0)
            return fail(PCDM_EINVAL, "max_passes must be 0, 1, 2 or 3");
        h->max_passes = (int)value;
    } else if (k == "narrow_below") {
        if (!(value >= 0.0))
            return fail(PCDM_EINVAL, "narrow_below must be >= 0");
        h->narrow_below = value > 9.0e18 ? INT64_MAX : (int64_t)value;
    } else if (k == "adj_tol") {
        if (!(value > 0.0))
            return fail(PCDM_EINVAL, "adj_tol must be > 0");
        h->adj_tol = value;
    } else if (k == "adj_max_epochs") {
        if (!(value >= 1.0))
            return fail(PCDM_EINVAL, "adj_max_epochs must be >= 1");
        h->adj_max_epochs = (int64_t)value;
    } else if (k == "adj_tau") {
        if (!(value >= 0.0))
            return fail(PCDM_EINVAL, "adj_tau must be >= 0");
        h->adj_tau = (int64_t)value;
    } else if (k == "adj_check_every") {
        if (!(value >= 1.0))
            return fail(PCDM_EINVAL, "adj_check_every must be >= 1");
        h->adj_check_every = (int64_t)value;
    } else if (k == "kernel_timing") {
        for (int c = 0; c < CLK_COUNT; ++c) {
            PCDM_TRY(clock_collect(h, c));
            h->clocks[c].launches = 0;
            h->clocks[c].total_ms = 0.0;
        }
        h->timing = value != 0.0;
    } else if (k == "gather_route") {
        if (value != 0.0 && value != 1.0 && value != 2.0)
            return fail(PCDM_EINVAL, "gather_route must be 0 (automatic), 1 (plain gather) or 2 (binned)");
        if (value == 2.0) {
            const char *why = bin_ineligible(h);
            if (why)
                return fail(PCDM_EINVAL, why);
        }
        HIP_TRY(hipStreamSynchronize(h->last_stream));  // queued steps may use the buffers
        h->gather_route = (int)value;
        PCDM_TRY(route_update(h));
    } else if (k == "bin_capacity") {
        if (!(value >= 0.0) || value > 65536.0 || value != std::floor(value))
            return fail(PCDM_EINVAL, "bin_capacity must be an integer in [0, 65536]");
        HIP_TRY(hipStreamSynchronize(h->last_stream));
        h->bin_cap_opt = (int64_t)value;
        PCDM_TRY(route_update(h));
    } else if (k == "scatter_route") {
        if (value != 0.0 && value != 1.0 && value != 2.0)
            return fail(PCDM_EINVAL, "scatter_route must be 0 (automatic), 1 (atomics) or 2 (row blocks)");
        if (value == 2.0) {
            const char *why = sbin_ineligible(h);
            if (why)
                return fail(PCDM_EINVAL, why);
        }
        HIP_TRY(hipStreamSynchronize(h->last_stream));
        h->scatter_route = (int)value;
        PCDM_TRY(sroute_update(h));
    } else if (k == "scatter_capacity") {
        if (!(value >= 0.0) || value > 65536.0 || value != std::floor(value))
            return fail(PCDM_EINVAL, "scatter_capacity must be an integer in [0, 65536]");
        HIP_TRY(hipStreamSynchronize(h->last_stream));
        h->sbin_cap_opt = (int64_t)value;
        PCDM_TRY(sroute_update(h));
    } else if (k == "reset_counters") {
        hipLaunchKernelGGL((k_fill<uint64_t>), dim3(1), dim3(kBlock), 0, h->last_stream, h->nz_part,
                           (uint64_t)0, (int64_t)h->nblk_max);
        PCDM_TRY(check_launch("reset_counters"));
    } else {
        return fail(PCDM_EINVAL, "unknown option '" + k + "'");
    }
    return PCDM_OK;
}

int pcdm_get_info(pcdm_problem *h, pcdm_info *out)
{
    if (!h || !out)
        return fail(PCDM_EINVAL, "NULL argument");
    hipStream_t s = h->last_stream;
    hipLaunchKernelGGL(k_sum_u64, dim3(1), dim3(kBlock), 0, s, (const uint64_t *)h->nz_part, h->nblk_max, h->ctrl);
    PCDM_TRY(check_launch("k_sum_u64"));
    int64_t nz = 0;
    HIP_TRY(hipMemcpyAsync(&nz, &h->ctrl->imax, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::memset(out, 0, sizeof(*out));
    out->m = h->m;
    out->n = h->n;
    out->nnz = h->nnz;
    out->tau = h->tau;
    out->k = h->k_host;
    out->omega = h->omega;
    out->refresh_every = h->refresh_every;
    out->nonzero_updates = nz;
    out->stored_nnz = h->stored_nnz;
    out->beta = h->beta;
    out->lambda = h->lambda;
    out->atb_inf = h->atb_inf;
    out->dtype = h->dtype;
    out->beta_rule = h->beta_rule;
    out->lanes_per_column = h->lanes;
    out->chunks_per_lane = h->chunks;
    out->sampling = h->sampling;
    out->gather_route = h->binned ? 2 : 1;
    out->scatter_route = h->srows ? 2 : 1;
    out->binomial_p = h->pb;
    out->expected_set_size = expected_set_size(h);
    out->mask_len = h->mask_len;
    out->narrow_below = h->narrow_below;
    out->nblocks = h->group ? h->nb : 0;
    out->loss = h->loss;
    out->loss_scale = h->lscale;
    out->l2 = h->l2;
    out->linear = h->lin;
    out->lower = h->lo;
    out->upper = h->hi;
    out->async_picks = h->async_picks;
    out->async_processors = h->async_procs_last;
    out->max_incremental = h->inc_hits;
    out->max_candidates = h->inc_cands;
    return PCDM_OK;
}

int pcdm_step(pcdm_problem *h, int64_t nsteps, void *stream)
{
    if (!h)
        return fail(PCDM_EINVAL, "NULL handle");
    if (nsteps < 0)
        return fail(PCDM_EINVAL, "nsteps must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    h->last_stream = s;
    const int64_t L = h->graph_len;
    const bool graphs = L > 0 && !h->timing;  // per-launch events need direct launches
    int64_t left = nsteps;
    while (left > 0) {
        if (h->claim && h->k_host - h->claim_base >= (int64_t)0xFFFFFFFE - std::max<int64_t>(L, 1))
            reset_claims(h, h->k_host, s);  // 32-bit stamps must not repeat
        const int64_t to_refresh =
            h->refresh_every > 0 ? h->refresh_every - h->k_host % h->refresh_every : INT64_MAX;
        if (graphs && left >= L && to_refresh >= L) {
            PCDM_TRY(ensure_step_graph(h));
            HIP_TRY(hipGraphLaunch(h->graph_exec, s));
            h->k_host += L;
            left -= L;
        } else {
            PCDM_TRY(dispatch(h->dtype, [&](auto ops) { return decltype(ops)::step_once(h, s); }));
            h->k_host += 1;
            left -= 1;
        }
        if (h->refresh_every > 0 && h->k_host % h->refresh_every == 0)
            PCDM_TRY(refresh_now(h, s));
    }
    return check_launch("pcdm_step");
}

int pcdm_step_async(pcdm_problem *h, int64_t picks, void *stream)
{
    if (!h)
        return fail(PCDM_EINVAL, "NULL handle");
    if (!is_lasso(h))
        return fail(PCDM_EINVAL, "the asynchronous variant is built for the LASSO (square loss, l1 term)");
    if (picks < 0)
        return fail(PCDM_EINVAL, "picks must be >= 0");
    if (picks == 0)
        return PCDM_OK;
    hipStream_t s = (hipStream_t)stream;
    h->last_stream = s;
    int64_t procs = 0;
    PCDM_TRY(dispatch(h->dtype, [&](auto ops) { return decltype(ops)::async_once(h, picks, s, procs); }));
    PCDM_TRY(check_launch("pcdm_step_async"));
    h->async_launches += 1;
    h->async_picks += picks;
    h->async_procs_last = procs;
    if (h->refresh_every > 0)
        PCDM_TRY(refresh_now(h, s));
    return PCDM_OK;
}

int pcdm_objective(pcdm_problem *h, double *F, double *dual_gap, void *stream)
{
    if (!h || !F)
        return fail(PCDM_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    h->last_stream = s;
    if (h->group) {
        PCDM_TRY(dispatch(h->dtype, [&](auto ops) {
            decltype(ops)::residual64(h, s);
            decltype(ops)::sums(h, s);
            decltype(ops)::group_sums(h, dual_gap != nullptr, s);
            return PCDM_OK;
        }));
        PCDM_TRY(check_launch("pcdm_objective"));
        double sc[4] = {0, 0, 0, 0};
        HIP_TRY(hipMemcpyAsync(sc, h->ctrl->scal, sizeof(sc), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const double rr = sc[0], br = sc[1], gn = sc[2];
        *F = 0.5 * rr + h->lambda * gn;
        if (dual_gap) {
            const double gmax = sc[3];
            const double th = (gmax > h->lambda) ? h->lambda / gmax : 1.0;
            *dual_gap = *F - (-0.5 * th * th * rr - th * br);
        }
        return PCDM_OK;
    }
    if (!is_lasso(h)) {
        if (dual_gap)
            return fail(PCDM_EINVAL, "the duality gap is computed for the LASSO only (square loss, l1 term)");
        PCDM_TRY(dispatch(h->dtype, [&](auto ops) {
            decltype(ops)::residual64(h, s);
            decltype(ops)::model_sums(h, s);
            return PCDM_OK;
        }));
        PCDM_TRY(check_launch("pcdm_objective"));
        double sc2[2] = {0, 0};
        HIP_TRY(hipMemcpyAsync(sc2, h->ctrl->scal, sizeof(sc2), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        *F = h->lscale * sc2[0] + sc2[1];
        return PCDM_OK;
    }
    PCDM_TRY(dispatch(h->dtype, [&](auto ops) {
        decltype(ops)::residual64(h, s);
        decltype(ops)::sums(h, s);
        if (dual_gap)
            decltype(ops)::atr_absmax(h, h->r64, s);
        return PCDM_OK;
    }));
    PCDM_TRY(check_launch("pcdm_objective"));
    double sc[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(sc, h->ctrl->scal, sizeof(sc), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double rr = sc[0], br = sc[1], l1 = sc[2];
    *F = 0.5 * rr + h->lambda * l1;
    if (dual_gap) {
        const double gmax = sc[3];
        const double sc_theta = (gmax > h->lambda) ? h->lambda / gmax : 1.0;
        const double D = -0.5 * sc_theta * sc_theta * rr - sc_theta * br;
        *dual_gap = *F - D;
    }
    return PCDM_OK;
}

int pcdm_get_x(pcdm_problem *h, void *x_out, int32_t dtype, int32_t on_device, void *stream)
{
    if (!h || !x_out)
        return fail(PCDM_EINVAL, "NULL argument");
    if (dtype != PCDM_F32 && dtype != PCDM_F64)
        return fail(PCDM_EINVAL, "x dtype must be PCDM_F32 or PCDM_F64");
    hipStream_t s = (hipStream_t)stream;
    const size_t ob = dtype == PCDM_F64 ? 8 : 4;
    void *dst = x_out;
    void *tmp = nullptr;
    if (!on_device)
        HIP_TRY(hipMalloc(&tmp, (size_t)h->n * ob));
    if (tmp)
        dst = tmp;
    const int g = grid_for(h->n, kBlock, h->nblk_max);
    if (dtype == PCDM_F64)
        hipLaunchKernelGGL((k_convert<double, double>), dim3(g), dim3(kBlock), 0, s, (const double *)h->x, (double *)dst, h->n);
    else
        hipLaunchKernelGGL((k_convert<double, float>), dim3(g), dim3(kBlock), 0, s, (const double *)h->x, (float *)dst, h->n);
    int st = check_launch("pcdm_get_x");
    if (tmp) {
        if (st == PCDM_OK) {
            hipError_t e = hipMemcpyAsync(x_out, tmp, (size_t)h->n * ob, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
                e = hipStreamSynchronize(s);
            if (e != hipSuccess)
                st = hip_fail(e, "pcdm_get_x copy");
        }
        (void)hipFree(tmp);
    }
    return st;
}

int pcdm_set_x(pcdm_problem *h, const void *x, int32_t dtype, int32_t on_device, int64_t k, void *stream)
{
    if (!h || !x)
        return fail(PCDM_EINVAL, "NULL argument");
    if (dtype != PCDM_F32 && dtype != PCDM_F64)
        return fail(PCDM_EINVAL, "x dtype must be PCDM_F32 or PCDM_F64");
    if (k < 0)
        return fail(PCDM_EINVAL, "k must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    h->last_stream = s;
    const size_t ib = dtype == PCDM_F64 ? 8 : 4;
    const void *src = x;
    void *tmp = nullptr;
    if (!on_device) {
        HIP_TRY(hipMalloc(&tmp, (size_t)h->n * ib));
        hipError_t e = hipMemcpy(tmp, x, (size_t)h->n * ib, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(tmp);
            return hip_fail(e, "pcdm_set_x copy");
        }
        src = tmp;
    }
    const int g = grid_for(h->n, kBlock, h->nblk_max);
    if (dtype == PCDM_F64)
        hipLaunchKernelGGL((k_convert<double, double>), dim3(g), dim3(kBlock), 0, s, (const double *)src, (double *)h->x, h->n);
    else
        hipLaunchKernelGGL((k_convert<float, double>), dim3(g), dim3(kBlock), 0, s, (const float *)src, (double *)h->x, h->n);
    dispatch(h->dtype, [&](auto ops) {
        decltype(ops)::x_to_records(h, s);
        return PCDM_OK;
    });
    hipLaunchKernelGGL((k_fill<uint64_t>), dim3(1), dim3(kBlock), 0, s, &h->ctrl->k, (uint64_t)k, (int64_t)1);
    reset_claims(h, k, s);  // stamps of steps after k may have been used already
    int st = check_launch("pcdm_set_x");
    if (st == PCDM_OK)
        st = refresh_now(h, s);
    if (tmp) {
        hipError_t e = hipStreamSynchronize(s);
        (void)hipFree(tmp);
        if (st == PCDM_OK && e != hipSuccess)
            st = hip_fail(e, "pcdm_set_x sync");
    }
    if (st == PCDM_OK)
        h->k_host = k;
    return st;
}

int pcdm_get_residual(pcdm_problem *h, double *r_out, int32_t on_device, void *stream)
{
    if (!h || !r_out)
        return fail(PCDM_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    double *dst = r_out;
    void *tmp = nullptr;
    if (!on_device) {
        HIP_TRY(hipMalloc(&tmp, (size_t)h->m * 8));
        dst = (double *)tmp;
    }
    const int g = grid_for(h->m, kBlock, h->nblk_max);
    if (h->dtype == PCDM_F64)
        hipLaunchKernelGGL((k_widen<double>), dim3(g), dim3(kBlock), 0, s, (const double *)h->r, dst, h->m);
    else
        hipLaunchKernelGGL((k_widen<float>), dim3(g), dim3(kBlock), 0, s, (const float *)h->r, dst, h->m);
    int st = check_launch("pcdm_get_residual");
    if (tmp) {
        if (st == PCDM_OK) {
            hipError_t e = hipMemcpyAsync(r_out, tmp, (size_t)h->m * 8, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
                e = hipStreamSynchronize(s);
            if (e != hipSuccess)
                st = hip_fail(e, "pcdm_get_residual copy");
        }
        (void)hipFree(tmp);
    }
    return st;
}

// The adjoint solve of pcdm_grad_backward with its temporaries from `tmp`.
static int grad_backward_impl(pcdm_problem *h, const double *dL_dx, double *dL_db, double *dL_dlambda,
                              int32_t on_device, hipStream_t s, TempSource &tmp)
{
    if (!h || !dL_dx || !dL_db || !dL_dlambda)
        return fail(PCDM_EINVAL, "NULL argument");
    if (!is_lasso(h))
        return fail(PCDM_EINVAL, "the adjoint is built for the LASSO (square loss, l1 term)");
    h->last_stream = s;
    const int64_t n = h->n, m = h->m;
    double *g = nullptr, *gS = nullptr, *vS = nullptr, *rho = nullptr, *dels = nullptr;
    uint8_t *flags = nullptr;
    int32_t *S = nullptr, *ids = nullptr, *hist = nullptr, *nsel = nullptr;
    PCDM_TRY(tmp.get(&g, (size_t)n * 8));
    PCDM_TRY(tmp.get(&flags, (size_t)n));
    PCDM_TRY(tmp.get(&S, (size_t)n * 4));
    PCDM_TRY(tmp.get(&nsel, 16));
    PCDM_TRY(tmp.get(&rho, (size_t)m * 8));
    HIP_TRY(hipMemcpyAsync(g, dL_dx, (size_t)n * 8, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));

    // active set S = {i : x_i != 0}, ascending
    const int gn = grid_for(n, kBlock, h->nblk_max);
    hipLaunchKernelGGL(k_flag_nonzero, dim3(gn), dim3(kBlock), 0, s, (const double *)h->x, n, flags);
    size_t tb = 0;
    hipcub::CountingInputIterator<int32_t> count_it(0);
    HIP_TRY(hipcub::DeviceSelect::Flagged(nullptr, tb, count_it, flags, S, nsel, (int)n, s));
    void *tstore = nullptr;
    PCDM_TRY(tmp.get(&tstore, tb));
    HIP_TRY(hipcub::DeviceSelect::Flagged(tstore, tb, count_it, flags, S, nsel, (int)n, s));
    int32_t ns32 = 0;
    HIP_TRY(hipMemcpyAsync(&ns32, nsel, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int64_t ns = ns32;
    const int gm = grid_for(m, kBlock, h->nblk_max);
    if (ns == 0) {
        hipLaunchKernelGGL((k_fill<double>), dim3(gm), dim3(kBlock), 0, s, rho, 0.0, m);
        HIP_TRY(hipMemcpyAsync(dL_db, rho, (size_t)m * 8, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        *dL_dlambda = 0.0;
        h->adj_last_epochs = 0;
        h->adj_last_resid = 0.0;
        return PCDM_OK;
    }
    const int64_t tau_s = std::min<int64_t>(h->adj_tau > 0 ? h->adj_tau : h->tau, ns);
    PCDM_TRY(tmp.get(&gS, (size_t)ns * 8));
    PCDM_TRY(tmp.get(&vS, (size_t)ns * 8));
    PCDM_TRY(tmp.get(&hist, (size_t)m * 4));
    PCDM_TRY(tmp.get(&ids, (size_t)tau_s * 4));
    PCDM_TRY(tmp.get(&dels, (size_t)tau_s * 8));
    const int gs = grid_for(ns, kBlock, h->nblk_max);
    hipLaunchKernelGGL(k_gather_g, dim3(gs), dim3(kBlock), 0, s, (const int32_t *)S, (const double *)g, ns, gS);
    hipLaunchKernelGGL((k_fill<double>), dim3(gs), dim3(kBlock), 0, s, vS, 0.0, ns);
    hipLaunchKernelGGL((k_fill<double>), dim3(gm), dim3(kBlock), 0, s, rho, 0.0, m);
    hipLaunchKernelGGL((k_fill<int32_t>), dim3(gm), dim3(kBlock), 0, s, hist, 0, m);
    PCDM_TRY(dispatch(h->dtype, [&](auto ops) {
        decltype(ops)::adj_hist(h, S, ns, hist, s);
        return PCDM_OK;
    }));
    hipLaunchKernelGGL(k_imax_partials, dim3(gm), dim3(kBlock), 0, s, (const int32_t *)hist, m, (int64_t *)h->part2);
    hipLaunchKernelGGL(k_imax_final, dim3(1), dim3(kBlock), 0, s, (const int64_t *)h->part2, gm, h->ctrl);
    hipLaunchKernelGGL(k_adj_lambda, dim3(kReduceBlocks), dim3(kBlock), 0, s, (const int32_t *)S, (const double *)h->x,
                       (const double *)vS, (const double *)gS, ns, h->part);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kBlock), 0, s, (const double *)h->part, kReduceBlocks, 3, 1,
                       h->ctrl->scal);  // scal[1] = max |g_S|
    PCDM_TRY(check_launch("adjoint set-up"));
    Ctrl hc;
    HIP_TRY(hipMemcpyAsync(&hc, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int64_t omega_s = std::max<int64_t>(hc.imax, 1);
    const double gmax = hc.scal[1];
    const double beta_s = 1.0 + (double)(omega_s - 1) * (double)(tau_s - 1) / std::max(1.0, (double)ns - 1.0);
    const int64_t spe = ceil_div(ns, tau_s);
    const uint64_t seed_adj = h->seed ^ 0xAD101E5EEDull;
    double resid = gmax;
    bool converged = gmax == 0.0;
    int64_t epoch = 0;
    uint64_t step = 0;
    while (!converged && epoch < h->adj_max_epochs) {
        for (int64_t q = 0; q < spe; ++q, ++step)
            dispatch(h->dtype, [&](auto ops) {
                decltype(ops)::adj_step(h, S, gS, vS, rho, ids, dels, seed_adj, step, tau_s, ns, 1.0 / beta_s, s);
                return PCDM_OK;
            });
        ++epoch;
        if (epoch % h->adj_check_every == 0 || epoch == h->adj_max_epochs) {
            dispatch(h->dtype, [&](auto ops) {
                decltype(ops)::adj_check(h, S, gS, vS, rho, ns, s);
                return PCDM_OK;
            });
            PCDM_TRY(check_launch("adjoint check"));
            double r4 = 0.0;
            HIP_TRY(hipMemcpyAsync(&r4, h->ctrl->scal + 4, 8, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            resid = r4;
            converged = resid <= h->adj_tol * gmax;
        }
    }
    // the loop ends at a check (or with v = 0), so rho = A_S v is fresh
    // dL/db = A_S v (rho, fresh after the last check), dL/dlambda = -s^T v
    hipLaunchKernelGGL(k_adj_lambda, dim3(kReduceBlocks), dim3(kBlock), 0, s, (const int32_t *)S, (const double *)h->x,
                       (const double *)vS, (const double *)gS, ns, h->part);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kBlock), 0, s, (const double *)h->part, kReduceBlocks, 3, 0,
                       h->ctrl->scal);  // scal[0] = -s^T v
    PCDM_TRY(check_launch("adjoint outputs"));
    HIP_TRY(hipMemcpyAsync(dL_db, rho, (size_t)m * 8, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    double lam_grad = 0.0;
    HIP_TRY(hipMemcpyAsync(&lam_grad, h->ctrl->scal, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *dL_dlambda = lam_grad;
    h->adj_last_epochs = epoch;
    h->adj_last_resid = gmax > 0.0 ? resid / gmax : 0.0;
    if (!converged)
        return fail(PCDM_ENOTCONV, "adjoint solve stopped at relative normal-equation residual " +
                                       std::to_string(h->adj_last_resid) + " after " + std::to_string(epoch) +
                                       " epochs");
    return PCDM_OK;
}

int pcdm_grad_backward(pcdm_problem *h, const double *dL_dx, double *dL_db, double *dL_dlambda,
                       int32_t on_device, void *stream)
{
    DevTemps heap;  // freed on every exit
    TempSource tmp;
    tmp.heap = &heap;
    return grad_backward_impl(h, dL_dx, dL_db, dL_dlambda, on_device, (hipStream_t)stream, tmp);
}

int pcdm_grad_backward_noalloc(pcdm_problem *h, const double *dL_dx, double *dL_db, double *dL_dlambda,
                               void *stream)
{
    if (!h || !dL_dx || !dL_db || !dL_dlambda)
        return fail(PCDM_EINVAL, "NULL argument");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != h->device)
        return fail(PCDM_EINVAL, "pcdm_grad_backward_noalloc: the handle was created on device " +
                                     std::to_string(h->device) + " but device " + std::to_string(dev) +
                                     " is current");
    void *base = nullptr;
    PCDM_TRY(scratch_base(dev, &base));
    TempSource tmp;
    tmp.base = (char *)base;
    tmp.cap = kScratchBytes;
    tmp.who = "pcdm_grad_backward_noalloc";
    return grad_backward_impl(h, dL_dx, dL_db, dL_dlambda, 1, (hipStream_t)stream, tmp);
}

int pcdm_set_rhs(pcdm_problem *h, const double *b, int32_t on_device, void *stream)
{
    if (!h || !b)
        return fail(PCDM_EINVAL, "NULL argument");
    if (h->loss != kLossSquare)
        return fail(PCDM_EINVAL, "labels are folded into the stored values: create a new problem to change them");
    hipStream_t s = (hipStream_t)stream;
    h->last_stream = s;
    HIP_TRY(hipMemcpyAsync(h->b64, b, (size_t)h->m * 8, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    PCDM_TRY(refresh_now(h, s));
    // ||A^T b||_inf for callers that set lambda relative to it
    const int gm = grid_for(h->m, kBlock, h->nblk_max);
    hipLaunchKernelGGL(k_neg_copy, dim3(gm), dim3(kBlock), 0, s, (const double *)h->b64, h->r64, h->m);
    PCDM_TRY(dispatch(h->dtype, [&](auto ops) { return decltype(ops)::atr_absmax(h, h->r64, s); }));
    PCDM_TRY(check_launch("pcdm_set_rhs"));
    double c = 0.0;
    HIP_TRY(hipMemcpyAsync(&c, h->ctrl->scal + 3, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    h->atb_inf = c;
    return PCDM_OK;
}

int pcdm_kernel_time(pcdm_problem *h, const char *kernel, int64_t *launches, double *total_ms)
{
    if (!h || !kernel || !launches || !total_ms)
        return fail(PCDM_EINVAL, "NULL argument");
    const std::string k(kernel);
    int kind = k == "gather" ? CLK_GATHER
               : k == "scatter" ? CLK_SCATTER
               : k == "refresh" ? CLK_REFRESH
               : k == "async"   ? CLK_ASYNC
                                : -1;
    if (kind < 0)
        return fail(PCDM_EINVAL, "kernel must be \"gather\", \"scatter\", \"refresh\" or \"async\"");
    PCDM_TRY(clock_collect(h, kind));
    *launches = h->clocks[kind].launches;
    *total_ms = h->clocks[kind].total_ms;
    return PCDM_OK;
}

int pcdm_autotune(pcdm_problem *h, int64_t steps_per_candidate, void *stream)
{
    if (!h || steps_per_candidate < 1)
        return fail(PCDM_EINVAL, "NULL handle or steps_per_candidate < 1");
    hipStream_t s = (hipStream_t)stream;
    h->last_stream = s;
    static const int cand[][2] = {{1, 1}, {1, 2}, {1, 4}, {2, 1}, {2, 2}, {2, 4}, {4, 1}, {4, 2}, {8, 1}, {8, 2}, {16, 1}};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best = std::numeric_limits<float>::max();
    int bg = h->lanes, bc = h->chunks;
    int64_t bn = h->narrow_below;
    int st = PCDM_OK;
    const int keep_timing = h->timing;
    h->timing = 0;
    // each schedule with tiles of 64 slots (narrow_below = 0) and with a lane
    // group per slot (narrow_below above tau)
    const int64_t widths[2] = {0, INT64_MAX};
    for (int64_t nb : widths) {
        for (const auto &c : cand) {
            if (!schedule_supported(c[0], c[1], h->loss) || (h->group && c[1] != 1))
                continue;
            h->lanes = c[0];
            h->chunks = c[1];
            h->narrow_below = nb;
            (void)hipEventRecord(e0, s);
            st = pcdm_step(h, steps_per_candidate, stream);
            (void)hipEventRecord(e1, s);
            if (st != PCDM_OK)
                break;
            float ms = 0.f;
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                break;
            if (ms < best) {
                best = ms;
                bg = c[0];
                bc = c[1];
                bn = nb;
            }
        }
        if (st != PCDM_OK)
            break;
    }
    h->timing = keep_timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->lanes = bg;
    h->chunks = bc;
    h->narrow_below = bn;
    h->lanes_auto = 0;
    return st;
}

int pcdm_sample_draw(int32_t sampling, double binomial_p, uint64_t seed, uint64_t k, int64_t tau, int64_t n,
                     int32_t *out_device, void *stream)
{
    if (!out_device)
        return fail(PCDM_EINVAL, "NULL output");
    if (n < 1 || n > INT32_MAX || tau < 0 || tau > n)
        return fail(PCDM_EINVAL, "need 1 <= n <= 2^31-1 and 0 <= tau <= n");
    if (sampling < kSampleNice || sampling > kSampleBinomial)
        return fail(PCDM_EINVAL, "sampling must be 0, 1 or 2");
    if (sampling == kSampleBinomial && !(binomial_p > 0.0 && binomial_p <= 1.0))
        return fail(PCDM_EINVAL, "binomial_p must be in (0, 1]");
    if (tau == 0)
        return PCDM_OK;
    hipStream_t s = (hipStream_t)stream;
    const int g = grid_for(tau, kBlock, 4096);
    hipLaunchKernelGGL(k_sample, dim3(g), dim3(kBlock), 0, s, seed, k, tau, (uint32_t)n, (int)sampling,
                       binomial_p, out_device);
    return check_launch("pcdm_sample_draw");
}

int pcdm_sample(uint64_t seed, uint64_t k, int64_t tau, int64_t n, int32_t *out_device, void *stream)
{
    return pcdm_sample_draw(kSampleNice, 1.0, seed, k, tau, n, out_device, stream);
}

int pcdm_set_slot_mask(pcdm_problem *h, const uint8_t *mask, int64_t len, int32_t on_device, void *stream)
{
    if (!h)
        return fail(PCDM_EINVAL, "NULL handle");
    if (h->group)
        return fail(PCDM_EINVAL, "block problems take no slot mask");
    if (len < 0 || (len > 0 && !mask))
        return fail(PCDM_EINVAL, "need len >= 0 and a mask when len > 0");
    if (len > h->n)
        return fail(PCDM_EINVAL, "mask longer than n (tau never exceeds n)");
    hipStream_t s = (hipStream_t)stream;
    h->last_stream = s;
    HIP_TRY(hipStreamSynchronize(s));  // steps already queued may still read the old mask
    if (h->mask)
        HIP_TRY(hipFree(h->mask));
    h->mask = nullptr;
    h->mask_len = 0;
    if (len == 0)
        return route_update(h);
    HIP_TRY(hipMalloc(&h->mask, (size_t)len));
    HIP_TRY(hipMemcpyAsync(h->mask, mask, (size_t)len, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           s));
    HIP_TRY(hipStreamSynchronize(s));
    h->mask_len = len;
    return route_update(h);
}

}  // extern "C"

#include "batch_runtime.hpp"
