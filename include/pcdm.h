/*
 * pcdm.h -- C ABI of the MI355X (gfx950) library for synchronous parallel
 * coordinate descent (PCDM1) on the LASSO
 *
 *     minimise  F(x) = 0.5 * ||A x - b||_2^2 + lambda * ||x||_1 ,  x in R^n,
 *
 * the composite problem of the paper's problem statement (eq. P) with the
 * partially separable smooth part f(x) = 0.5||Ax-b||^2 and the separable
 * regulariser Omega(x) = lambda||x||_1 (Richtarik & Takac, "Parallel
 * Coordinate Descent Methods for Big Data Optimization"; the LASSO of the
 * experiments section, with lambda general).
 *
 * One step (Algorithm PCDM1):
 *   1. draw S_k, a tau-nice random set of tau distinct coordinates
 *      (section "Block Samplings", nice sampling);
 *   2. for every i in S_k, from the same residual r = A x_k - b:
 *        g_i = a_i^T r                              (partial derivative),
 *        u   = x_i - g_i / (beta L_i),
 *        x_i <- sign(u) max(|u| - lambda/(beta L_i), 0)
 *      i.e. x_i + h^(i)(x_k) with h(x) = argmin H_{beta,w}(x, .) and w = L,
 *      L_i = ||a_i||^2, beta = 1 + (omega-1)(tau-1)/max(1, n-1)
 *      (Table "ESO", tau-nice row; theorem "ESO for nice samplings");
 *   3. r <- r + sum_{i in S_k} delta_i a_i (residual kept by scatter-add).
 * omega is the largest number of nonzeros in a row of A (degree of partial
 * separability).
 *
 * Every function returns an int status: PCDM_OK (0) or a negative
 * pcdm_status; pcdm_last_error() then gives a message (thread-local, valid
 * until the next call on the same thread).  No C++ exception and no exit()
 * crosses this boundary.  A handle is not thread-safe: calls on one handle
 * must be serialised by the caller; handles are independent of each other.
 *
 * Device work is enqueued on the HIP stream passed in (void* = hipStream_t,
 * NULL = the default stream) and is asynchronous unless stated otherwise.
 */
#ifndef PCDM_H
#define PCDM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PCDM_OK = 0,
    PCDM_EINVAL = -1,   /* invalid argument or invalid matrix            */
    PCDM_ENOMEM = -2,   /* device allocation failed                      */
    PCDM_EDEVICE = -3,  /* HIP runtime error (no device, launch failure) */
    PCDM_ESTATE = -4,   /* call not valid for this handle's state        */
    PCDM_ENOTCONV = -5  /* iterative solve did not reach its tolerance   */
} pcdm_status;

/* Value types.  The dtype of A's values selects the arithmetic:
 *   PCDM_F64  : values and r in float64, float64 sums;
 *   PCDM_F32  : values and r in float32, float32 dot products;
 *   PCDM_BF16 : values stored as bfloat16 (raw uint16 bit patterns), r in
 *               float32, float32 dot products.
 * In every mode x, 1/L_i and the update of x_i are float64, and the periodic
 * residual refresh r = A x - b, the objective and the duality gap are
 * computed in float64. */
typedef enum { PCDM_F32 = 0, PCDM_BF16 = 1, PCDM_F64 = 2 } pcdm_dtype;

/* Compressed sparse column matrix; column i holds coordinate i's data a_i
 * (the paper stores A by columns: coordinate i needs only a_i).
 *   col_ptr [n+1] int64 : col_ptr[0] = 0, non-decreasing, col_ptr[n] = nnz;
 *   row_idx [nnz] int32 : rows of column i at col_ptr[i] .. col_ptr[i+1]-1,
 *                         each in [0, m), unique within the column (any order);
 *   values  [nnz]       : of type dtype, finite.
 * on_device = 1: col_ptr, row_idx, values (and the b passed with them) are
 * device pointers (e.g. torch tensors on the GPU); 0: host pointers.
 * The library copies what it needs; the caller keeps ownership. */
typedef struct pcdm_csc {
    int64_t m, n, nnz;
    const int64_t *col_ptr;
    const int32_t *row_idx;
    const void *values;
    int32_t dtype;
    int32_t on_device;
} pcdm_csc;

typedef struct pcdm_problem pcdm_problem; /* opaque, owned by the library */

typedef struct pcdm_info {
    int64_t m, n, nnz;
    int64_t tau;
    int64_t k;               /* steps taken so far (the sampler counter)          */
    int64_t omega;           /* max nonzeros in a row (measured at create)        */
    int64_t refresh_every;   /* steps between float64 residual refreshes; 0 = off */
    int64_t nonzero_updates; /* coordinate updates with delta != 0 (since create  */
                             /* or the last "reset_counters"); read synchronously */
    int64_t stored_nnz;      /* entries in the device layout (columns padded)     */
    double beta;             /* step damping in use                               */
    double lambda;
    double atb_inf;          /* ||A^T b||_inf in float64 from the stored A        */
    int32_t dtype;
    int32_t beta_rule;       /* 0 = tau-nice, 1 = tau-uniform min(omega,tau),     */
                             /* 2 = explicit value set with option "beta"         */
    int32_t lanes_per_column;/* step-kernel schedule: lanes reading one column    */
    int32_t chunks_per_lane; /* ... and 4-entry chunks each lane holds          */
    int32_t sampling;        /* 0 = tau-nice, 1 = tau-independent, 2 = binomial   */
    int32_t gather_route;    /* partial derivatives: 1 = plain gather, 2 = by rows  */
    double binomial_p;       /* availability p_b of a binomial slot               */
    double expected_set_size;/* E|S_k| of the sampling (drop mask not included)   */
    int64_t mask_len;        /* slots covered by the drop mask (0 = none)         */
    int64_t narrow_below;    /* tau below which a slot gets a group of lanes      */
    int64_t nblocks;         /* blocks of a block problem (0: coordinates)        */
    int32_t loss;            /* pcdm_loss of the model (PCDM_LOSS_SQUARE: LASSO)  */
    int32_t scatter_route;   /* residual scatter: 1 = atomics, 2 = row blocks     */
    double loss_scale;       /* model terms (see pcdm_model); lambda is l1       */
    double l2, linear, lower, upper;
    int64_t async_picks;     /* picks made by pcdm_step_async so far              */
    int64_t async_processors;/* processors (lane groups) of its last launch       */
    int64_t max_incremental; /* ||A^T r||_inf evaluations that took route 3       */
    int64_t max_candidates;  /* columns summed exactly by route 3's last attempt  */
} pcdm_info;

/*
 * Create a problem and copy A and b into library-owned device memory.
 *   A       : matrix (validated; see pcdm_csc);
 *   b       : [m] float64, host or device as A->on_device says;
 *   lambda  : >= 0 and finite;
 *   tau     : sampled coordinates per step, 1 <= tau <= n;
 *   seed    : key of the sampler (S_k depends on (seed, k) and the sampling only).
 * Requires 1 <= n <= 2^31 - 2 and 1 <= m with the working residual under
 * 4 GiB (m < 2^30 for PCDM_F32/PCDM_BF16, m < 2^29 for PCDM_F64).  Rejects (PCDM_EINVAL) empty or all-zero
 * columns (the paper assumes L_i > 0), repeated rows in a column, rows out
 * of range, non-finite values, a malformed col_ptr.  x starts at 0 and
 * r = -b.  Runs on the default stream and returns after the device work is
 * complete.  On failure *out is set to NULL.
 * Device memory held by the handle: the column records (16 bytes per column
 * plus the column's entries padded to a multiple of 4, each 4 + sizeof(value)
 * bytes; with equal column lengths every record is padded to 64 bytes),
 * 8 (n + 1) bytes of column pointers, x (8 n), r (m * sizeof(working type)),
 * r64 and b (8 m each), per-slot results (tau * (4 + sizeof(working type)))
 * and, for float32 / bf16 values, 12 m + 8 n bytes for the two-pass and
 * incremental ||A^T r||_inf (option "max_passes").
 */
int pcdm_create(const pcdm_csc *A, const double *b, double lambda, int64_t tau,
                uint64_t seed, pcdm_problem **out);

/*
 * Other smooth losses and separable regularisers (introduction: partially
 * separable f = sum_j loss_j with the table of three losses; numerical
 * experiments: the SVM dual with box constraints, L2-regularised logistic
 * regression):
 *     F(x) = scale * sum_j phi_j((A x)_j) + sum_i Omega(x_i),
 *     phi_j: PCDM_LOSS_SQUARE   0.5 (z - y_j)^2        (y = targets)
 *            PCDM_LOSS_LOGISTIC log(1 + exp(-y_j z))   (y = labels +-1)
 *            PCDM_LOSS_SQHINGE  0.5 max(0, 1 - y_j z)^2 (y = labels +-1)
 *     Omega(t) = l1 |t| + (l2/2) t^2 + linear t + (0 if lower <= t <= upper
 *                else +inf).
 * f is partially separable with the omega of A; L_i = scale * sup(phi'')
 * * ||a_i||^2 with sup(phi'') = 1, 1/4, 1; beta as for pcdm_create.  The
 * block step is the minimiser of the model with Omega: clip(soft(w, t),
 * lower, upper) with w = (x_i - (g_i + linear)/(beta L_i))/(1 + l2/(beta L_i))
 * and t = (l1/(beta L_i))/(1 + l2/(beta L_i)).  Examples: LASSO {SQUARE, 1,
 * lambda, 0, 0, -inf, inf}; elastic net (l2 > 0); non-negative LASSO (lower
 * = 0); SVM dual of n examples (columns y_i a_i, rows the features, targets
 * 0) {SQUARE, 1/(lambda n^2), 0, 0, -1/n, 0, 1}; L2 logistic
 * sum_j log(1 + exp(-y_j a_j^T x)) + mu ||x||^2 {LOGISTIC, 1, 0, 2 mu, 0,
 * -inf, inf}.  For the logistic and square-hinge losses the labels are
 * multiplied into the stored values at create, and the maintained vector
 * holds the margins y_j a_j^T x (r = A x - y for the square loss).
 */
typedef enum { PCDM_LOSS_SQUARE = 0, PCDM_LOSS_LOGISTIC = 1, PCDM_LOSS_SQHINGE = 2 } pcdm_loss;

typedef struct pcdm_model {
    int32_t loss;    /* pcdm_loss                                    */
    int32_t reserved;
    double scale;    /* > 0, finite                                  */
    double l1, l2;   /* >= 0, finite                                 */
    double linear;   /* finite                                       */
    double lower;    /* <= 0 (may be -HUGE_VAL)                      */
    double upper;    /* >= 0 (may be +HUGE_VAL)                      */
} pcdm_model;

/*
 * Create a problem for a model (see above): y [m] float64 (targets or
 * labels, host or device as A->on_device says).  As pcdm_create otherwise;
 * PCDM_EINVAL also for labels other than +-1 and for model terms out of
 * range.  pcdm_step and pcdm_objective (without dual_gap) serve every model;
 * the duality gap, pcdm_grad_backward, pcdm_step_async and the batches are
 * built for the LASSO only, and pcdm_set_rhs for the square loss only
 * (PCDM_EINVAL otherwise).  Losses other than the square one run with one
 * chunk per lane (chunks_per_lane = 1).
 */
int pcdm_create_model(const pcdm_csc *A, const double *y, const pcdm_model *model, int64_t tau,
                      uint64_t seed, pcdm_problem **out);

/*
 * Blocks of several coordinates: the group LASSO
 *     F(x) = 0.5||A x - b||^2 + lambda sum_i ||x^(i)||_2
 * (section "Block structure, notation and assumptions"; the group-lasso
 * example of a block separable Omega).  Block i is the column range
 * block_ptr[i] .. block_ptr[i+1]-1 (block_ptr [nblocks+1] int64, 0 = first,
 * n = last, 1 to 16 columns per block; host or device as A->on_device says;
 * order the columns so that each group is consecutive).  Euclidean block
 * norms, so L_i = lambda_max(A_i^T A_i) (computed at create from the block's
 * Gram matrix by Jacobi rotations in float64); omega = the largest number of
 * distinct blocks with a nonzero in one row; tau counts blocks (1 <= tau <=
 * nblocks) with the tau-nice sampler over blocks and beta = 1 + (omega-1)
 * (tau-1)/max(1, nblocks-1).  The update of a sampled block is the block
 * soft threshold max(0, 1 - lambda/(beta L_i ||u||)) u with u = x^(i) -
 * A_i^T r/(beta L_i).  pcdm_step, pcdm_objective (with the duality gap for
 * theta = r min(1, lambda / max_i ||A_i^T r||)), pcdm_get_x / set_x,
 * pcdm_set_rhs, the lambda / tau / refresh_every / lanes_per_column options
 * and pcdm_autotune serve block problems; other samplings, slot masks, the
 * adjoint and the asynchronous variant do not (PCDM_EINVAL).  Extra device
 * memory: 8 (nblocks + 1) + 8 nblocks + n * sizeof(working type) bytes.
 */
int pcdm_create_group(const pcdm_csc *A, const double *b, double lambda, const int64_t *block_ptr,
                      int64_t nblocks, int64_t tau, uint64_t seed, pcdm_problem **out);

/* Free all device memory of the handle (synchronises the device). NULL is a no-op. */
int pcdm_destroy(pcdm_problem *h);

/* Message of the last failing call on this thread ("" if none). */
const char *pcdm_last_error(void);

/*
 * Set a numeric option.  Keys:
 *   "refresh_every"    steps between float64 refreshes r = A x - b (default
 *                      ceil(n/tau), one epoch; 0 disables);
 *   "beta_rule"        0 = the ESO beta of the sampling in use (default):
 *                      tau-nice 1 + (omega-1)(tau-1)/max(1,n-1); binomial
 *                      1 + p_b(omega-1)(tau-1)/max(1,n-1); tau-independent
 *                      the doubly uniform 1 + (omega-1)(E|S|^2/E|S| - 1)/max(1,n-1)
 *                      (Table "ESO"; theorem "ESO for doubly uniform
 *                      samplings"); 1 = min(omega, tau);
 *   "sampling"         0 = tau-nice (default); 1 = tau-independent: each of
 *                      tau processors picks a block uniformly and
 *                      independently, a block picked twice is updated once
 *                      (section "Block Samplings", independent sampling; the
 *                      sampler of the paper's own LASSO runs; needs 4n bytes
 *                      of claim stamps, allocated on first use); 2 =
 *                      (tau, p_b)-binomial with implicit selection: slot j of
 *                      the tau-nice S_k updates its block only when available,
 *                      with probability p_b (binomial sampling, case 2).
 *                      Draws: kappa_k = SplitMix64 output k from seed ^
 *                      0x5043444D494E4450 (independent) or seed ^
 *                      0x5043444D42494E4F (binomial); u_j = output j from
 *                      kappa_k; a pick is floor(u_j n / 2^64); a slot is
 *                      available iff (u_j >> 11) 2^-53 < p_b;
 *   "binomial_p"       p_b in (0, 1] (default 1);
 *   "beta"             explicit beta > 0 (sets beta_rule 2);
 *   "lambda"           new lambda >= 0;
 *   "tau"              new tau in [1, n] (beta recomputed by the rule);
 *   "lanes_per_column" 0 = automatic, or 1, 2, 4, 8, 16, 32, 64 lanes
 *                      cooperating on one sampled column;
 *   "chunks_per_lane"  0 = automatic, or 1, 2, 4 four-entry chunks of the
 *                      column each lane keeps in registers; supported pairs
 *                      (lanes, chunks): (1|2, 1|2|4), (4|8, 1|2), (16|32|64, 1);
 *   "narrow_below"     step-kernel layout: for tau below this value (default
 *                      131072) each sampled slot gets its own group of
 *                      lanes_per_column lanes (64/lanes slots per wave), so a
 *                      small step still spreads over many waves; otherwise a
 *                      wave owns 64 consecutive slots (one lane each for the
 *                      sampling and the update).  0 = always 64-slot tiles;
 *   "async_processors" processors of pcdm_step_async: 0 (default) = min(tau,
 *                      lane groups the device holds at once), else that count;
 *   "async_reads", "async_rounds": see pcdm_step_async;
 *   "graph_steps"      runs of this many steps (default 32; 0 = off) are
 *                      captured once into a HIP graph (on an internal stream)
 *                      and replayed on the caller's stream, when no float64
 *                      refresh falls inside the run and "kernel_timing" is
 *                      off; the graph is rebuilt whenever an argument of the
 *                      step kernels changes (options, masks, sampling);
 *   "max_passes"       how ||A^T r||_inf (duality gap, ||A^T b||_inf; for
 *                      blocks max_i ||A_i^T r||_2) is
 *                      found for float32 / bf16 values: 2 = a pass
 *                      over fl32(r) giving every column (block) a rigorous
 *                      bound, then the exact float64 sums for the columns
 *                      (blocks) whose bound reaches the largest lower bound;
 *                      1 = the exact sums everywhere; 3 = as 2, keeping r and
 *                      the bounds of the last evaluation: the next one moves
 *                      each column's bound by ||a_i||_1 times a rigorous bound
 *                      on the change of r in max norm (Hoelder) and, when at most
 *                      n/8 columns can still reach the maximum, sums only
 *                      those exactly (one pass over r and the candidate
 *                      records; the host reads the candidate count).  All
 *                      three give the same number; float64 values always
 *                      take one pass, blocks take 2 for 3; 0 (default) = 3
 *                      from 2^24 stored entries, else 2 (below that the
 *                      route's fixed costs exceed a bound pass);
 *   "gather_route"     how a step's partial derivatives g_i = a_i^T r are
 *                      read: 1 = by columns (every sampled column's entries,
 *                      then r at their rows); 2 = by rows: the step's entries
 *                      are first dealt into bins by (row range, window of
 *                      2^18 rows), then r is read window by window, eight
 *                      row ranges in parallel, and the per-range partial sums
 *                      are added per slot (same g_i up to the order of the
 *                      float32 additions; for float32 / bf16 LASSO problems
 *                      with equal column lengths of at most 32 entries and
 *                      the tau-nice sampling without a drop mask; otherwise
 *                      steps take route 1).  Route 2 needs
 *                      8 ceil(tau/1024) * 8 ceil(m/2^21) * cap + 48 tau bytes.
 *                      It reads each line of r about once per step instead
 *                      of once per entry, but its three launches are bound by
 *                      latency; 0 (default) = 2 where eligible when r (m
 *                      float32 values) takes at least 256 MiB and tau >= 2^20,
 *                      else 1.  pcdm_info.gather_route
 *                      reports the route in effect;
 *   "bin_capacity"     route 2: entries per bin (0 = default: the mean count
 *                      for rows spread evenly, plus seven standard deviations
 *                      and 16, rounded up to 16).  A step whose bins overflow
 *                      is taken by route 1 instead, so results do not depend
 *                      on it;
 *   "scatter_route"    how a step adds delta_i a_i to r: 1 = hardware float
 *                      atomics per entry; 2 = by row blocks: the step's
 *                      products are dealt into runs keyed by block of 4096
 *                      rows, and one workgroup per block sums them in LDS and
 *                      adds the sums to r with plain stores (for float32 /
 *                      bf16 values with equal column lengths of at most 32
 *                      entries, m <= 2^22 and tau <= 2^21; otherwise
 *                      route 1).  Needs
 *                      8 ceil(m/4096) ceil(tau/1024) cap + 4 ceil(m/4096)
 *                      ceil(tau/1024) bytes.  0 (default) = 1.
 *                      pcdm_info.scatter_route reports the route in effect;
 *   "scatter_capacity" route 2: entries per run (0 = default: the mean count
 *                      when every slot changes, plus seven standard
 *                      deviations and 16, rounded up to 16); entries past it
 *                      are added with atomics, so results do not depend on it;
 *   "reset_counters"   any value: zero nonzero_updates;
 *   "adj_tol", "adj_max_epochs", "adj_tau", "adj_check_every"
 *                      settings of pcdm_grad_backward's solve (see there);
 *   "kernel_timing"    1 = record HIP events around every step-kernel launch
 *                      (see pcdm_kernel_time), 0 = stop; either value first
 *                      zeroes the accumulated times.
 * Unknown keys and out-of-range values give PCDM_EINVAL.
 */
int pcdm_set_option(pcdm_problem *h, const char *key, double value);

/* Fill *out (synchronises the handle's last stream for nonzero_updates). */
int pcdm_get_info(pcdm_problem *h, pcdm_info *out);

/*
 * Advance nsteps synchronous PCDM1 steps (k -> k + nsteps) on `stream`.
 * Every refresh_every steps (counted by k) the residual is recomputed in
 * float64 from x and rounded to the working type.  Asynchronous.
 */
int pcdm_step(pcdm_problem *h, int64_t nsteps, void *stream);

/*
 * Asynchronous variant (section "Numerical experiments", billion-variable
 * LASSO: the timed implementation lets each core read the current iterate
 * when it is ready and apply its update at once, each core picking a block
 * uniformly and independently).  One call makes `picks` picks spread over P
 * processors (groups of lanes_per_column lanes; option "async_processors"):
 * pick u of call c is block floor(w n / 2^64), w = SplitMix64 output u from
 * kappa_c = SplitMix64 output c from seed ^ 0x5043444D4153594E (c counts this
 * handle's calls from 0), and processor p makes picks p, p + P, ...  Each
 * pick takes its block by an atomic swap on x_i's slot (a block held by
 * another processor is skipped for that pick), reads r, releases the block
 * by swapping in the new x_i and adds delta_i a_i to r with float atomics.
 * No step boundary: reads see the updates that have landed.  Because each
 * XCD has its own L2, option "async_reads" sets how fresh reads of r are:
 * 0 = plain cached loads, with the call split into launches of
 * "async_rounds" rounds of P picks (default 4; 0 = one launch), whose
 * boundaries make all earlier updates visible; 1 = the swap that takes a
 * block is an acquire (caches invalidated before the reads); 2 = r read
 * through returning atomics; -1 (default) = 1 for at most 8192 processors,
 * else 0.  x lives only in the column records during a launch; the dense
 * copy behind pcdm_get_x is rebuilt from them at the end of the call.  beta is the handle's (the tau-nice rule with
 * tau = the handle's tau, as the paper's runs used with tau = cores).  With
 * P = 1 the call is serial coordinate descent over the pick stream.
 * Afterwards, if refresh_every > 0, r is recomputed in float64.  Does not
 * advance k.  Asynchronous; the result depends on timing for P > 1.  No
 * other work may touch the handle while a call runs.
 */
int pcdm_step_async(pcdm_problem *h, int64_t picks, void *stream);

/*
 * F(x) = 0.5||A x - b||^2 + lambda||x||_1 with A x - b recomputed in float64
 * (the working residual is not modified).  If dual_gap is not NULL, also the
 * duality gap F(x) - D(theta) for theta = s r, s = min(1, lambda/||A^T r||_inf),
 * D(theta) = -0.5||theta||^2 - b^T theta (one extra pass over A).  Both are
 * >= 0 up to rounding and bound F(x) - F*.  Synchronous (waits on `stream`).
 */
int pcdm_objective(pcdm_problem *h, double *F, double *dual_gap, void *stream);

/* Copy x (n values) to x_out, converted to dtype (PCDM_F32 or PCDM_F64),
 * host or device memory.  Host copies are synchronous. */
int pcdm_get_x(pcdm_problem *h, void *x_out, int32_t dtype, int32_t on_device, void *stream);

/* Overwrite x from x (n values of dtype PCDM_F32 / PCDM_F64, host or device),
 * set the step counter to k (resume), and recompute r = A x - b in float64. */
int pcdm_set_x(pcdm_problem *h, const void *x, int32_t dtype, int32_t on_device,
               int64_t k, void *stream);

/* Copy the working residual r (m values, widened to float64) to r_out. */
int pcdm_get_residual(pcdm_problem *h, double *r_out, int32_t on_device, void *stream);

/*
 * Reverse-mode derivative through the current iterate, taken as the LASSO
 * solution: with S = {i : x_i != 0}, s = sign(x_S) and A_S^T A_S x_S =
 * A_S^T b - lambda s on a stable support,
 *     dL/db = A_S v,   dL/dlambda = -s^T v,   where A_S^T A_S v = (dL/dx)_S.
 * (the derivative of the solution map on a stable support: differentiating
 * the optimality conditions of the LASSO).  v is found by synchronous PCDM
 * steps with the same tau-nice sampler and column reads as pcdm_step, in
 * float64, on q(v) = 0.5||A_S v||^2 - g^T v (lambda = 0, coordinates = S,
 * beta from omega_S of the columns in S and tau_S = min(adj_tau or tau, |S|),
 * sampler key seed ^ 0xAD101E5EED), until
 * ||A_S^T A_S v - g_S||_inf <= adj_tol * ||g_S||_inf, checked every
 * adj_check_every epochs (options; defaults 1e-6, 10, at most adj_max_epochs
 * = 20000 epochs).
 *   dL_dx [n] float64, dL_db [m] float64 (out), dL_dlambda (out, host scalar);
 * dL_dx and dL_db are host or device as on_device says.  x_i == 0 exactly
 * defines the inactive set.  Synchronous.  PCDM_ENOTCONV if the tolerance is
 * not met (outputs still written).  Temporary device memory: about
 * 17 n + 12 m + 12 tau bytes, freed before return.
 */
int pcdm_grad_backward(pcdm_problem *h, const double *dL_dx, double *dL_db,
                       double *dL_dlambda, int32_t on_device, void *stream);

/*
 * pcdm_grad_backward for callers that cannot allocate device memory (code
 * that must not call hipMalloc: tight serving loops, harnesses that forbid
 * allocation): the same solve and kernels, with every temporary carved from
 * a fixed 32 MiB device region that the library holds for the life of the
 * process, one copy per device (looked up on the first call on a device).
 * No hipMalloc, hipFree or allocating library routine is called.
 *   dL_dx [n], dL_db [m]: device pointers (float64); dL_dlambda: host scalar.
 * The handle's device must be current.  The temporaries need about
 * 13 n + 12 m + 16 |S| + 12 tau_S bytes (each piece rounded up to 256 bytes,
 * plus the stream compaction's work space); a problem that needs more than
 * 32 MiB is rejected with PCDM_EINVAL before the solve starts (use
 * pcdm_grad_backward).  Every call on one device shares the one region and
 * leaves its contents behind (each call fills what it reads before reading
 * it): calls that overlap in time on one device, from any handles or
 * threads, race and must be serialised by the caller.  Results as
 * pcdm_grad_backward; synchronous.
 */
int pcdm_grad_backward_noalloc(pcdm_problem *h, const double *dL_dx, double *dL_db,
                               double *dL_dlambda, void *stream);

/*
 * Replace b (m float64 values, host or device) and recompute r = A x - b in
 * float64 and ||A^T b||_inf (pcdm_info.atb_inf).  x and k are kept (warm
 * start).  Synchronous.
 */
int pcdm_set_rhs(pcdm_problem *h, const double *b, int32_t on_device, void *stream);

/*
 * Device time of one kernel kind of the step while option "kernel_timing" is
 * on: kernel = "gather" (sample, partial derivatives, update of x),
 * "scatter" (residual scatter-add), "refresh" (float64 residual refresh) or
 * "async" (launches of pcdm_step_async).
 * Measured between HIP events recorded on the launch stream just before and
 * after each launch.  Waits for the recorded launches; writes the number of
 * launches and their summed milliseconds since timing was (re)started.
 */
int pcdm_kernel_time(pcdm_problem *h, const char *kernel, int64_t *launches, double *total_ms);

/*
 * Schedule autotuner: runs steps_per_candidate real steps (they advance k)
 * with each supported (lanes_per_column, chunks_per_lane) pair, both with
 * 64-slot tiles and with a lane group per slot (option "narrow_below"),
 * timed with HIP events on `stream`, and keeps the fastest.  Synchronous.
 */
int pcdm_autotune(pcdm_problem *h, int64_t steps_per_candidate, void *stream);

/*
 * The tau-nice sampler on its own: writes S_k = {pi_k(j) : 0 <= j < tau}
 * for key (seed, k) into out_device[0..tau) (int32, device memory), in slot
 * order.  Same sets as pcdm_step draws.  Asynchronous.
 */
int pcdm_sample(uint64_t seed, uint64_t k, int64_t tau, int64_t n, int32_t *out_device,
                void *stream);

/*
 * The draws of any sampling (section "Block Samplings"; draws as under
 * option "sampling"): out_device[j] (int32, device memory, tau entries) is
 * slot j's block at step k with key seed: pi_k(j) for tau-nice; the raw pick
 * of processor j for tau-independent (duplicates kept: pcdm_step updates each
 * distinct pick once); pi_k(j), or -1 when the slot is unavailable, for
 * binomial.  No drop mask.  Asynchronous.
 */
int pcdm_sample_draw(int32_t sampling, double binomial_p, uint64_t seed, uint64_t k, int64_t tau,
                     int64_t n, int32_t *out_device, void *stream);

/*
 * Drop mask (fault model: processors that are down; binomial sampling's
 * "unreliable processors" made deterministic).  mask[j] == 0 removes slot j
 * (j < len) from every following step under every sampling: the slot
 * computes nothing and scatters nothing; slots >= len are alive.  beta is
 * not changed (the sampling's beta stays valid: dropping slots of a tau-nice
 * sample leaves a smaller nice sample, whose beta is smaller).  len = 0
 * (mask may be NULL) removes the mask.  0 <= len <= n; mask is host or
 * device memory as on_device says and is copied.  Synchronous.
 */
int pcdm_set_slot_mask(pcdm_problem *h, const uint8_t *mask, int64_t len, int32_t on_device,
                       void *stream);

/* ------------------------------------------------------------------------
 * Batched solver: many independent LASSO problems (uneven m_j, n_j, a
 * lambda grid, several right-hand sides) advanced together, one launch per
 * phase for all of them.  Problem j uses the tau-nice sampler with key
 * (seed + j, k_j), its own beta_j (from its omega_j and tau_j), its own
 * float64 refresh every ceil(n_j/tau_j) steps, and converges exactly as it
 * would alone (same steps, same sets).  Problems can be retired (held
 * still) once solved.
 * ------------------------------------------------------------------------ */
typedef struct pcdm_batch pcdm_batch; /* opaque, owned by the library */

/* Create from `count` problems: A[j], b[j] ([m_j] float64), lambda[j],
 * tau[j].  All A[j] share one dtype and one memory kind (on_device), which
 * b follows.  Validation as in pcdm_create (errors name the problem).
 * Synchronous on the default stream. */
int pcdm_batch_create(int count, const pcdm_csc *A, const double *const *b, const double *lambda,
                      const int64_t *tau, uint64_t seed, pcdm_batch **out);

/* Advance every active problem by nsteps steps.  Runs of "graph_steps"
 * (option, default 32; 0 disables) steps are captured once into a HIP graph
 * and replayed; the remainder is launched directly.  Asynchronous. */
int pcdm_batch_step(pcdm_batch *B, int64_t nsteps, void *stream);

/* F_j and (if gap != NULL) the duality gap of every problem, float64
 * (arrays of `count`).  Only the problems that stepped since their last
 * evaluation are evaluated again (refresh of r = A x - b in float64, then
 * the sums and ||A_j^T r_j||_inf); the others return the values of that
 * evaluation, which still hold since neither x_j nor b_j changed.
 * Synchronous. */
int pcdm_batch_objective(pcdm_batch *B, double *F, double *gap, void *stream);

/* active[j] = 0 holds problem j still (retired), 1 resumes it.  Synchronises the device. */
int pcdm_batch_set_active(pcdm_batch *B, const int32_t *active);

/* x of problem `index` (n_index float64 values, host or device). */
int pcdm_batch_get_x(pcdm_batch *B, int index, double *x_out, int32_t on_device, void *stream);

/* Sizes, omega, beta, lambda, ||A^T b||_inf, steps taken of problem `index`
 * (nonzero_updates is -1: not tracked per problem); max_incremental counts
 * its evaluations that moved kept bounds, max_candidates the columns its
 * last evaluation summed. */
int pcdm_batch_get_info(pcdm_batch *B, int index, pcdm_info *out);

/* Options: "graph_steps" (>= 0), "lanes_per_column", "chunks_per_lane"
 * (pairs as for pcdm_set_option), "max_passes": 3 (default) = each problem
 * keeps r and per-column bounds of its last evaluation and sums exactly only
 * the columns whose moved bound can still reach its maximum (as route 3 of
 * pcdm_set_option, without the fallback: the pass itself skips the others);
 * 1 or 2 = every column summed.  Both give the same numbers. */
int pcdm_batch_set_option(pcdm_batch *B, const char *key, double value);

/* Schedule autotuner for the batch (as pcdm_autotune; the steps advance
 * every active problem). */
int pcdm_batch_autotune(pcdm_batch *B, int64_t steps_per_candidate, void *stream);

/* Free (synchronises the device). NULL is a no-op. */
int pcdm_batch_destroy(pcdm_batch *B);

#ifdef __cplusplus
}
#endif

#endif /* PCDM_H */
