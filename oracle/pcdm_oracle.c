/*
 * pcdm_oracle.c -- plain, serial, float64 reference of synchronous PCDM1 on the
 * LASSO objective  F(x) = 0.5*||A x - b||^2 + lambda*||x||_1 .
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code, header, table or constant generator with the HIP library; the
 * sampler below is written from the published definitions of its parts.
 *
 * What each function follows (Richtarik & Takac, "Parallel Coordinate Descent
 * Methods for Big Data Optimization"):
 *   - beta for the tau-nice sampling: Table "ESO" (tau-nice row) and the
 *     theorem "ESO for nice samplings"; beta = 1 + (omega-1)(tau-1)/max(1,n-1).
 *   - beta for tau-uniform samplings: Table "ESO" (tau-uniform row) and the
 *     theorem on proper uniform samplings; beta = min(omega, tau).
 *   - omega = max number of nonzeros in a row of A (introduction, examples of
 *     partially separable functions; contributions, item "partial separability").
 *   - L_i = ||a_i||_2^2, w = L (contributions, "partial separability"; the
 *     LASSO experiment uses w = L).
 *   - the step: Algorithm PCDM1 with the update h(x) = argmin H_{beta,w}(x,.)
 *     (eqs. h(x) and H_{beta,w}); for Omega = lambda*|.| and blocks of size 1
 *     the block minimiser is a soft threshold (derivation in the function).
 *   - every i in S_k is updated from the same x_k (Step 4 "in parallel").
 *   - the tau-independent and (tau, p_b)-binomial samplings: section "Block
 *     Samplings" (items "independent sampling", "binomial sampling", implicit
 *     selection); their beta: Table "ESO" (doubly uniform and binomial rows),
 *     theorem "ESO for doubly uniform samplings".
 *   - the asynchronous variant with one processor: section "Numerical
 *     experiments" (billion-variable LASSO), serial over independent picks.
 *   - other losses and regularisers: the table of three losses
 *     (introduction), the SVM dual with box constraints and L2-regularised
 *     logistic regression (numerical experiments); block minimisers derived
 *     in orc_model_prox.
 *   - the dual bound for the duality gap is standard LASSO duality.
 *
 * Numerics: float64, round to nearest, sums in ascending index order, no
 * blocking or reordering beyond what is stated.  Scatter order inside a step:
 * ascending coordinate index.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Step damping (Table ESO).                                                 */
/* ------------------------------------------------------------------------ */

/* tau-nice sampling: beta = 1 + (omega-1)(tau-1)/max(1, n-1), w = L. */
double orc_beta_nice(int64_t omega, int64_t tau, int64_t n)
{
    double den = (n - 1 > 1) ? (double)(n - 1) : 1.0;
    return 1.0 + ((double)(omega - 1) * (double)(tau - 1)) / den;
}

/* any tau-uniform sampling: beta = min(omega, tau), w = L (monotone ESO). */
double orc_beta_uniform(int64_t omega, int64_t tau)
{
    return (double)(omega < tau ? omega : tau);
}

/* (tau, p_b)-binomial sampling: beta = 1 + p_b(omega-1)(tau-1)/max(1, n-1). */
double orc_beta_binomial(int64_t omega, int64_t tau, int64_t n, double pb)
{
    double den = (n - 1 > 1) ? (double)(n - 1) : 1.0;
    return 1.0 + pb * ((double)(omega - 1) * (double)(tau - 1)) / den;
}

/* ------------------------------------------------------------------------ */
/* Structure of f.                                                           */
/* ------------------------------------------------------------------------ */

/* omega = max_j #{i : A_ji != 0}: the degree of partial separability of
 * 0.5*||Ax-b||^2 (each row term depends on the coordinates it touches). */
int64_t orc_omega(int64_t m, int64_t n, const int64_t *col_ptr,
                  const int32_t *row_idx, const double *val)
{
    int64_t *cnt = (int64_t *)calloc((size_t)(m > 0 ? m : 1), sizeof(int64_t));
    int64_t best = 0;
    if (!cnt)
        return -1;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = col_ptr[i]; p < col_ptr[i + 1]; ++p)
            if (val[p] != 0.0)
                cnt[row_idx[p]] += 1;
    for (int64_t j = 0; j < m; ++j)
        if (cnt[j] > best)
            best = cnt[j];
    free(cnt);
    return best;
}

/* Block Lipschitz constants of grad f: L_i = ||a_i||^2. */
void orc_lipschitz(int64_t n, const int64_t *col_ptr, const double *val, double *L)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t p = col_ptr[i]; p < col_ptr[i + 1]; ++p)
            s += val[p] * val[p];
        L[i] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* omega and ||A^T b||_inf of a matrix too large to hold as float64.         */
/*                                                                           */
/* The caller streams A in column slices with the stored float32 values     */
/* (widened exactly); each call adds the slice's nonzeros to per-row counts */
/* (omega is the largest count once every slice is in) and returns the      */
/* largest |a_i^T b| of the slice (the lambda rule of the experiments is a  */
/* multiple of ||A^T b||_inf).  Columns are split over threads: a row count */
/* is a sum of increments and a maximum does not depend on the order, so    */
/* the results equal those of one serial pass.  Each a_i^T b is summed in   */
/* ascending entry order in float64.                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t c0, c1;
    const int64_t *col_ptr;
    const int32_t *row_idx;
    const float *val;
    const double *b;
    int64_t m;
    int32_t *counts;
    double best;
    int bad;
} orc_stats_job;

static void *orc_stats_worker(void *arg)
{
    orc_stats_job *J = (orc_stats_job *)arg;
    for (int64_t i = J->c0; i < J->c1; ++i) {
        double s = 0.0;
        for (int64_t p = J->col_ptr[i]; p < J->col_ptr[i + 1]; ++p) {
            const int32_t row = J->row_idx[p];
            if (row < 0 || (int64_t)row >= J->m) {
                J->bad = 1;
                return NULL;
            }
            s += (double)J->val[p] * J->b[row];
            if (J->val[p] != 0.0f)
                __atomic_fetch_add(&J->counts[row], 1, __ATOMIC_RELAXED);
        }
        if (fabs(s) > J->best)
            J->best = fabs(s);
    }
    return NULL;
}

/* Slice of ncols columns: entries col_ptr[i] .. col_ptr[i+1]-1 of row_idx and
 * val belong to the slice's column i.  counts[m] accumulates; *absdot_max
 * receives the slice's largest |a_i^T b|.  A thread that cannot be started
 * has its share run on the calling thread.  Returns 0, or -1 on a row out of
 * range. */
int orc_column_stats_f32(int64_t ncols, const int64_t *col_ptr, const int32_t *row_idx, const float *val,
                         const double *b, int64_t m, int32_t *counts, double *absdot_max, int nthreads)
{
    orc_stats_job jobs[64];
    pthread_t th[64];
    int started[64];
    int nt = nthreads < 1 ? 1 : (nthreads > 64 ? 64 : nthreads);
    double best = 0.0;
    int bad = 0;
    if (ncols < 0)
        return -1;
    for (int t = 0; t < nt; ++t) {
        jobs[t].c0 = ncols * t / nt;
        jobs[t].c1 = ncols * (t + 1) / nt;
        jobs[t].col_ptr = col_ptr;
        jobs[t].row_idx = row_idx;
        jobs[t].val = val;
        jobs[t].b = b;
        jobs[t].m = m;
        jobs[t].counts = counts;
        jobs[t].best = 0.0;
        jobs[t].bad = 0;
        started[t] = pthread_create(&th[t], NULL, orc_stats_worker, &jobs[t]) == 0;
        if (!started[t])
            orc_stats_worker(&jobs[t]);
    }
    for (int t = 0; t < nt; ++t) {
        if (started[t])
            pthread_join(th[t], NULL);
        bad |= jobs[t].bad;
        if (jobs[t].best > best)
            best = jobs[t].best;
    }
    *absdot_max = best;
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* tau-nice sampler.                                                         */
/*                                                                           */
/* The paper fixes only the law: every subset of size tau is equally likely. */
/* Concrete generator (written independently on the GPU side):              */
/*   * SplitMix64 (Steele, Lea & Flood, 2014): output number t of the stream */
/*     started at state s is mix64(s + (t+1)*0x9E3779B97F4A7C15) with        */
/*     mix64(z): z=(z^(z>>30))*0xBF58476D1CE4E5B9; z=(z^(z>>27))*            */
/*     0x94D049BB133111EB; return z^(z>>31).                                  */
/*   * MurmurHash3's 32-bit finaliser fmix32 (Appleby) as Feistel round     */
/*     function.                                                             */
/*   * Step k's round keys: K_rho = low 32 bits of SplitMix64 output number  */
/*     10k+rho of the stream started at seed XOR 0x5043444D4E494345,         */
/*     rho = 0..9.                                                           */
/*   * E_k: balanced 10-round Feistel network on [0, 4^h), h >= 1 minimal    */
/*     with 4^h >= n; x -> (L,R) = (x >> h, x & (2^h-1)); each round         */
/*     (L,R) <- (R, L ^ (fmix32(R ^ K_rho) & (2^h-1))); result (L<<h)|R.    */
/*   * pi_k(j): cycle walking (Black & Rogaway, 2002): y = E_k(j), repeat    */
/*     y = E_k(y) while y >= n.  pi_k is a permutation of [0, n).            */
/*   * S_k = { pi_k(j) : 0 <= j < tau } (slot j holds pi_k(j)).              */
/*   Ten rounds, not four: on the tiny domains of small n (4^h = 16 for      */
/*   n = 6) four rounds give a subset law measurably far from uniform.       */
/* ------------------------------------------------------------------------ */

static int orc_cmp_i64_fwd(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

static uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t orc_splitmix64(uint64_t state, uint64_t t)
{
    return orc_mix64(state + (t + 1) * 0x9E3779B97F4A7C15ULL);
}

uint32_t orc_fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6BU;
    h ^= h >> 13;
    h *= 0xC2B2AE35U;
    h ^= h >> 16;
    return h;
}

static int orc_half_bits(int64_t n)
{
    int h = 1;
    while ((((uint64_t)1) << (2 * h)) < (uint64_t)n)
        ++h;
    return h;
}

static uint64_t orc_feistel(uint64_t x, int h, const uint32_t key[10])
{
    uint32_t mask = (uint32_t)((((uint64_t)1) << h) - 1);
    uint32_t left = (uint32_t)(x >> h), right = (uint32_t)(x & mask);
    for (int rho = 0; rho < 10; ++rho) {
        uint32_t t = left ^ (orc_fmix32(right ^ key[rho]) & mask);
        left = right;
        right = t;
    }
    return ((uint64_t)left << h) | right;
}

/* Writes S_k into out[0..tau).  Returns 0, or -1 for bad arguments. */
int orc_sample_nice(uint64_t seed, uint64_t k, int64_t tau, int64_t n, int64_t *out)
{
    uint32_t key[10];
    int h;
    if (n < 1 || n > 2147483647LL || tau < 0 || tau > n)
        return -1;
    for (int rho = 0; rho < 10; ++rho)
        key[rho] = (uint32_t)orc_splitmix64(seed ^ 0x5043444D4E494345ULL, 10 * k + (uint64_t)rho);
    h = orc_half_bits(n);
    for (int64_t j = 0; j < tau; ++j) {
        uint64_t y = orc_feistel((uint64_t)j, h, key);
        while (y >= (uint64_t)n)
            y = orc_feistel(y, h, key);
        out[j] = (int64_t)y;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Other doubly uniform samplings (section "Block Samplings": the           */
/* tau-independent and (tau, p_b)-binomial samplings) and their beta        */
/* (Table ESO, doubly uniform row; theorem "ESO for doubly uniform          */
/* samplings").                                                              */
/*                                                                           */
/* Concrete draws (written independently on the GPU side):                  */
/*   * kappa_k = SplitMix64 output number k of the stream started at        */
/*     seed XOR C, with C = 0x5043444D494E4450 for independent picks and    */
/*     C = 0x5043444D42494E4F for binomial availability draws;               */
/*   * u_j = SplitMix64 output number j of the stream started at kappa_k.   */
/*   * tau-independent: processor j (j < tau) picks block                   */
/*     floor(u_j * n / 2^64) (Lemire's multiply-shift reduction, 2019);     */
/*     S_k is the set of distinct picks (a block picked twice is updated    */
/*     once: the other processors idle).                                     */
/*   * (tau, p_b)-binomial, implicit selection: slot j holds pi_k(j) of the */
/*     tau-nice sampler and is available iff (u_j >> 11) * 2^-53 < p_b.     */
/*     S_k is the set of available slots' blocks.                            */
/* A drop mask models processors that are down: slot j (j < mask_len) with  */
/* mask[j] == 0 contributes nothing, under every sampling.                  */
/* ------------------------------------------------------------------------ */

static uint64_t orc_draw(uint64_t seed, uint64_t stream_const, uint64_t k, uint64_t j)
{
    uint64_t kappa = orc_splitmix64(seed ^ stream_const, k);
    return orc_splitmix64(kappa, j);
}

/* Raw picks of the tau processors of step k (slot order, duplicates kept). */
int orc_draw_independent(uint64_t seed, uint64_t k, int64_t tau, int64_t n, int64_t *out)
{
    if (n < 1 || n > 2147483647LL || tau < 0 || tau > n)
        return -1;
    for (int64_t j = 0; j < tau; ++j) {
        uint64_t u = orc_draw(seed, 0x5043444D494E4450ULL, k, (uint64_t)j);
        out[j] = (int64_t)(((unsigned __int128)u * (uint64_t)n) >> 64);
    }
    return 0;
}

/* Slot j's block for the binomial sampling, or -1 when the slot is not
 * available at step k. */
int orc_draw_binomial(uint64_t seed, uint64_t k, int64_t tau, int64_t n, double pb, int64_t *out)
{
    if (orc_sample_nice(seed, k, tau, n, out) != 0 || !(pb > 0.0 && pb <= 1.0))
        return -1;
    for (int64_t j = 0; j < tau; ++j) {
        uint64_t u = orc_draw(seed, 0x5043444D42494E4FULL, k, (uint64_t)j);
        if (!((double)(u >> 11) * 0x1.0p-53 < pb))
            out[j] = -1;
    }
    return 0;
}

/*
 * S_k of the given sampling (0 = tau-nice, 1 = tau-independent,
 * 2 = (tau, p_b)-binomial) with the drop mask applied, written to out in
 * ascending order without duplicates.  Returns |S_k|, or -1 for bad
 * arguments.  out needs room for tau entries.
 */
int64_t orc_sample_set(int sampling, double pb, uint64_t seed, uint64_t k, int64_t tau, int64_t n,
                       const uint8_t *mask, int64_t mask_len, int64_t *out)
{
    int rc;
    int64_t cnt = 0;
    if (sampling == 0)
        rc = orc_sample_nice(seed, k, tau, n, out);
    else if (sampling == 1)
        rc = orc_draw_independent(seed, k, tau, n, out);
    else if (sampling == 2)
        rc = orc_draw_binomial(seed, k, tau, n, pb, out);
    else
        return -1;
    if (rc != 0)
        return -1;
    for (int64_t j = 0; j < tau; ++j) {
        if (out[j] < 0 || (mask && j < mask_len && mask[j] == 0))
            continue;
        out[cnt++] = out[j];
    }
    qsort(out, (size_t)cnt, sizeof(int64_t), orc_cmp_i64_fwd);
    {
        int64_t u = 0;
        for (int64_t t = 0; t < cnt; ++t)
            if (t == 0 || out[t] != out[t - 1])
                out[u++] = out[t];
        cnt = u;
    }
    return cnt;
}

/*
 * First two moments of |S| for the tau-independent sampling.  Block i is
 * missed by all tau processors with probability (1 - 1/n)^tau, and blocks
 * i != j both by all with probability (1 - 2/n)^tau, so by inclusion and
 * exclusion
 *     E|S|   = n (1 - (1-1/n)^tau),
 *     E|S|^2 = E|S| + n(n-1) (1 - 2(1-1/n)^tau + (1-2/n)^tau).
 * The last bracket cancels badly when tau << n; it is evaluated as
 * (1-a)^2 - (a^2 - c) with a = (1-1/n)^tau, c = (1-2/n)^tau and
 * a^2 - c = c ((1 + 1/(n(n-2)))^tau - 1), using log1p / expm1.
 */
void orc_independent_moments(int64_t tau, int64_t n, double *e1, double *e2)
{
    double nn = (double)n, t = (double)tau, one_minus_a, pair;
    if (n == 1) {
        *e1 = 1.0;
        *e2 = 1.0;
        return;
    }
    one_minus_a = -expm1(t * log1p(-1.0 / nn));
    if (n == 2) {
        pair = 1.0 - 2.0 * pow(0.5, t);
    } else {
        double c = exp(t * log1p(-2.0 / nn));
        pair = one_minus_a * one_minus_a - c * expm1(t * log1p(1.0 / (nn * (nn - 2.0))));
    }
    *e1 = nn * one_minus_a;
    *e2 = *e1 + nn * (nn - 1.0) * pair;
}

/* Doubly uniform sampling with moments E|S| = e1, E|S|^2 = e2:
 * beta = 1 + (omega-1)(e2/e1 - 1)/max(1, n-1), w = L. */
double orc_beta_du(int64_t omega, int64_t n, double e1, double e2)
{
    double den = (n - 1 > 1) ? (double)(n - 1) : 1.0;
    return 1.0 + (double)(omega - 1) * (e2 / e1 - 1.0) / den;
}

/* ------------------------------------------------------------------------ */
/* Objective pieces.                                                         */
/* ------------------------------------------------------------------------ */

/* soft(u, c) = sign(u) * max(|u| - c, 0); soft(+-c, c) = 0. */
double orc_soft(double u, double c)
{
    if (u > c)
        return u - c;
    if (u < -c)
        return u + c;
    return 0.0;
}

/* r = A x - b. */
void orc_residual(int64_t m, int64_t n, const int64_t *col_ptr, const int32_t *row_idx,
                  const double *val, const double *x, const double *b, double *r)
{
    for (int64_t j = 0; j < m; ++j)
        r[j] = -b[j];
    for (int64_t i = 0; i < n; ++i) {
        if (x[i] == 0.0)
            continue;
        for (int64_t p = col_ptr[i]; p < col_ptr[i + 1]; ++p)
            r[row_idx[p]] += val[p] * x[i];
    }
}

/* F(x) = 0.5*||r||^2 + lambda*||x||_1 with r = A x - b given. */
double orc_objective(int64_t m, int64_t n, const double *r, const double *x, double lambda)
{
    double s = 0.0, t = 0.0;
    for (int64_t j = 0; j < m; ++j)
        s += r[j] * r[j];
    for (int64_t i = 0; i < n; ++i)
        t += fabs(x[i]);
    return 0.5 * s + lambda * t;
}

/* g_i = grad_i f(x) = a_i^T r for all i. */
void orc_gradient(int64_t n, const int64_t *col_ptr, const int32_t *row_idx,
                  const double *val, const double *r, double *g)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t p = col_ptr[i]; p < col_ptr[i + 1]; ++p)
            s += val[p] * r[row_idx[p]];
        g[i] = s;
    }
}

/* LASSO dual: D(theta) = -0.5*||theta||^2 - b^T theta on ||A^T theta||_inf <= lambda.
 * theta = s*r with s = min(1, lambda/||A^T r||_inf) is dual feasible; returns
 * the gap F(x) - D(theta) >= 0 (weak duality) and writes F and D. */
double orc_dual_gap(int64_t m, int64_t n, const int64_t *col_ptr, const int32_t *row_idx,
                    const double *val, const double *b, const double *x, const double *r,
                    double lambda, double *F_out, double *D_out)
{
    double gmax = 0.0, rr = 0.0, br = 0.0, s, F, D;
    for (int64_t i = 0; i < n; ++i) {
        double g = 0.0;
        for (int64_t p = col_ptr[i]; p < col_ptr[i + 1]; ++p)
            g += val[p] * r[row_idx[p]];
        if (fabs(g) > gmax)
            gmax = fabs(g);
    }
    for (int64_t j = 0; j < m; ++j) {
        rr += r[j] * r[j];
        br += b[j] * r[j];
    }
    s = (gmax > lambda) ? lambda / gmax : 1.0;
    F = orc_objective(m, n, r, x, lambda);
    D = -0.5 * s * s * rr - s * br;
    if (F_out)
        *F_out = F;
    if (D_out)
        *D_out = D;
    return F - D;
}

/* ------------------------------------------------------------------------ */
/* PCDM1 step.                                                               */
/* ------------------------------------------------------------------------ */

static int orc_cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/*
 * One synchronous step x <- x + (h(x))_[S] on the given set S (size tau), with
 * r = A x - b maintained.
 *
 * h(x)^(i) minimises  g_i t + (beta L_i / 2) t^2 + lambda |x_i + t|  over t
 * (the block form of H_{beta,w} with w = L, N_i = 1).  With u = x_i - g_i/(beta L_i)
 * the minimiser of (beta L_i/2)(x_i + t - u)^2 + lambda|x_i + t| is
 * x_i + t = soft(u, lambda/(beta L_i)).
 *
 * All g_i use the same r (= A x_k - b).  Afterwards x and r are updated in
 * ascending coordinate order.  Returns -1 if S holds a duplicate or an index
 * out of range, else the number of coordinates whose value changed.
 */
int64_t orc_step_with_set(int64_t m, int64_t n, const int64_t *col_ptr, const int32_t *row_idx,
                          const double *val, const double *L, double lambda, double beta,
                          int64_t tau, const int64_t *S, double *x, double *r)
{
    int64_t *ids = (int64_t *)malloc((size_t)(tau > 0 ? tau : 1) * sizeof(int64_t));
    double *delta = (double *)malloc((size_t)(tau > 0 ? tau : 1) * sizeof(double));
    int64_t changed = 0;
    (void)m;
    if (!ids || !delta) {
        free(ids);
        free(delta);
        return -1;
    }
    memcpy(ids, S, (size_t)tau * sizeof(int64_t));
    qsort(ids, (size_t)tau, sizeof(int64_t), orc_cmp_i64);
    for (int64_t t = 0; t < tau; ++t) {
        if (ids[t] < 0 || ids[t] >= n || (t > 0 && ids[t] == ids[t - 1])) {
            free(ids);
            free(delta);
            return -1;
        }
    }
    /* phase 1: every update from the same residual */
    for (int64_t t = 0; t < tau; ++t) {
        int64_t i = ids[t];
        double g = 0.0, u, xn;
        for (int64_t p = col_ptr[i]; p < col_ptr[i + 1]; ++p)
            g += val[p] * r[row_idx[p]];
        u = x[i] - g / (beta * L[i]);
        xn = orc_soft(u, lambda / (beta * L[i]));
        delta[t] = xn - x[i];
    }
    /* phase 2: apply */
    for (int64_t t = 0; t < tau; ++t) {
        int64_t i = ids[t];
        if (delta[t] == 0.0)
            continue;
        ++changed;
        x[i] += delta[t];
        for (int64_t p = col_ptr[i]; p < col_ptr[i + 1]; ++p)
            r[row_idx[p]] += delta[t] * val[p];
    }
    free(ids);
    free(delta);
    return changed;
}

/*
 * nsteps steps of PCDM1 with the tau-nice sampler, steps k0 .. k0+nsteps-1.
 * x and r (= A x - b on entry) are updated in place.  Returns the total count
 * of coordinates that changed, or -1 on error.
 */
int64_t orc_pcdm_run(int64_t m, int64_t n, const int64_t *col_ptr, const int32_t *row_idx,
                     const double *val, const double *L, double lambda, double beta,
                     int64_t tau, uint64_t seed, int64_t k0, int64_t nsteps,
                     double *x, double *r)
{
    int64_t *S = (int64_t *)malloc((size_t)(tau > 0 ? tau : 1) * sizeof(int64_t));
    int64_t total = 0;
    if (!S)
        return -1;
    for (int64_t k = k0; k < k0 + nsteps; ++k) {
        int64_t c;
        if (orc_sample_nice(seed, (uint64_t)k, tau, n, S) != 0) {
            free(S);
            return -1;
        }
        c = orc_step_with_set(m, n, col_ptr, row_idx, val, L, lambda, beta, tau, S, x, r);
        if (c < 0) {
            free(S);
            return -1;
        }
        total += c;
    }
    free(S);
    return total;
}

/*
 * As orc_pcdm_run, with S_k drawn by orc_sample_set (sampling, p_b, drop
 * mask).  beta is the caller's.
 */
int64_t orc_pcdm_run_sampling(int64_t m, int64_t n, const int64_t *col_ptr, const int32_t *row_idx,
                              const double *val, const double *L, double lambda, double beta,
                              int64_t tau, uint64_t seed, int64_t k0, int64_t nsteps, int sampling,
                              double pb, const uint8_t *mask, int64_t mask_len, double *x, double *r)
{
    int64_t *S = (int64_t *)malloc((size_t)(tau > 0 ? tau : 1) * sizeof(int64_t));
    int64_t total = 0;
    if (!S)
        return -1;
    for (int64_t k = k0; k < k0 + nsteps; ++k) {
        int64_t cnt = orc_sample_set(sampling, pb, seed, (uint64_t)k, tau, n, mask, mask_len, S);
        int64_t c;
        if (cnt < 0) {
            free(S);
            return -1;
        }
        c = orc_step_with_set(m, n, col_ptr, row_idx, val, L, lambda, beta, cnt, S, x, r);
        if (c < 0) {
            free(S);
            return -1;
        }
        total += c;
    }
    free(S);
    return total;
}

/*
 * Asynchronous variant with one processor (section "Numerical experiments",
 * LASSO with a billion variables: the implementation there lets each core
 * read the current iterate when it is ready and apply its update at once,
 * each core picking a block uniformly and independently).  With a single
 * processor every update sees all earlier ones, so the run is serial
 * coordinate descent over the pick stream
 *     i_u = floor(u64 * n / 2^64),  u64 = SplitMix64 output u of the stream
 *     started at kappa, kappa = SplitMix64 output `launch` of the stream
 *     started at seed XOR 0x5043444D4153594E,
 * for updates u = 0 .. nupdates-1 of launch number `launch`.  Each update is
 * the damped soft-threshold step of PCDM1 with the given beta.  x and
 * r = A x - b are updated in place.  Returns the number of changed
 * coordinates' updates, or -1.
 */
int64_t orc_async_serial_run(int64_t m, int64_t n, const int64_t *col_ptr, const int32_t *row_idx,
                             const double *val, const double *L, double lambda, double beta, uint64_t seed,
                             uint64_t launch, int64_t nupdates, double *x, double *r)
{
    uint64_t kappa = orc_splitmix64(seed ^ 0x5043444D4153594EULL, launch);
    int64_t changed = 0;
    (void)m;
    if (n < 1 || n > 2147483647LL || nupdates < 0)
        return -1;
    for (int64_t u = 0; u < nupdates; ++u) {
        uint64_t w = orc_splitmix64(kappa, (uint64_t)u);
        int64_t i = (int64_t)(((unsigned __int128)w * (uint64_t)n) >> 64);
        double g = 0.0, xn, d;
        for (int64_t p = col_ptr[i]; p < col_ptr[i + 1]; ++p)
            g += val[p] * r[row_idx[p]];
        xn = orc_soft(x[i] - g / (beta * L[i]), lambda / (beta * L[i]));
        d = xn - x[i];
        if (d == 0.0)
            continue;
        ++changed;
        x[i] = xn;
        for (int64_t p = col_ptr[i]; p < col_ptr[i + 1]; ++p)
            r[row_idx[p]] += d * val[p];
    }
    return changed;
}

/* ------------------------------------------------------------------------ */
/* Other smooth losses and separable regularisers (introduction: examples  */
/* of partially separable functions and the table of three losses; the     */
/* experiments on the SVM dual with box constraints and on L2-regularised  */
/* logistic regression).                                                    */
/*                                                                           */
/*   f(x) = s * sum_j phi(z_j, y_j),   z = A x,                              */
/*   phi: 0 square        0.5 (z - y)^2            phi'' <= 1               */
/*        1 logistic      log(1 + exp(-y z))       phi'' <= 1/4             */
/*        2 square hinge  0.5 max(0, 1 - y z)^2    phi'' <= 1 (y = +-1)     */
/*   Omega_i(t) = l1 |t| + (l2/2) t^2 + c t + [lo <= t <= hi].               */
/* f is partially separable with the omega of A, and its block Lipschitz   */
/* constants are L_i = s * sup(phi'') * ||a_i||^2, so PCDM1 applies with the  */
/* same beta and w = L.                                                      */
/* ------------------------------------------------------------------------ */

static double orc_phi(int loss, double z, double y)
{
    if (loss == 0)
        return 0.5 * (z - y) * (z - y);
    if (loss == 1) {
        double t = -y * z; /* log(1 + e^t), evaluated without overflow */
        return t > 0.0 ? t + log1p(exp(-t)) : log1p(exp(t));
    }
    {
        double h = 1.0 - y * z;
        return h > 0.0 ? 0.5 * h * h : 0.0;
    }
}

/* d phi / d z */
static double orc_dphi(int loss, double z, double y)
{
    if (loss == 0)
        return z - y;
    if (loss == 1) {
        double t = y * z; /* -y / (1 + e^{t}) */
        return t > 0.0 ? -y * exp(-t) / (1.0 + exp(-t)) : -y / (1.0 + exp(t));
    }
    {
        double h = 1.0 - y * z;
        return h > 0.0 ? -y * h : 0.0;
    }
}

double orc_loss_value(int loss, double z, double y) { return orc_phi(loss, z, y); }
double orc_loss_deriv(int loss, double z, double y) { return orc_dphi(loss, z, y); }

double orc_loss_curvature_bound(int loss) { return loss == 1 ? 0.25 : 1.0; }

/*
 * The block minimiser for Omega_i: with v = x_i - g/(beta L_i) the update
 * minimises (beta L_i / 2)(u - v)^2 + l1|u| + (l2/2)u^2 + c u over
 * lo <= u <= hi.  Completing the square, the smooth part is
 * ((beta L_i + l2)/2)(u - w)^2 + const with w = (beta L_i v - c)/(beta L_i + l2);
 * the unconstrained minimiser of that plus l1|u| is soft(w, l1/(beta L_i + l2)),
 * and for a convex function of one variable the minimiser over [lo, hi] is
 * that point clipped to the interval.
 */
double orc_model_prox(double v, double bl, double l1, double l2, double c, double lo, double hi)
{
    double den = bl + l2;
    double w = (bl * v - c) / den;
    double u = orc_soft(w, l1 / den);
    if (u < lo)
        u = lo;
    if (u > hi)
        u = hi;
    return u;
}

/* Omega_i summed over x (infinite outside the box). */
double orc_model_omega(int64_t n, const double *x, double l1, double l2, double c, double lo, double hi)
{
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (x[i] < lo || x[i] > hi)
            return INFINITY;
        acc += l1 * fabs(x[i]) + 0.5 * l2 * x[i] * x[i] + c * x[i];
    }
    return acc;
}

/* F(x) = s sum_j phi(z_j, y_j) + sum_i Omega_i(x_i) for z = A x. */
double orc_model_objective(int64_t m, int64_t n, const double *z, const double *y, const double *x, int loss,
                           double s, double l1, double l2, double c, double lo, double hi)
{
    double acc = 0.0;
    for (int64_t j = 0; j < m; ++j)
        acc += orc_phi(loss, z[j], y[j]);
    return s * acc + orc_model_omega(n, x, l1, l2, c, lo, hi);
}

/*
 * One synchronous PCDM1 step on the set S for the model above: every
 * g_i = s * sum_p a_pi * phi'(z_{row p}, y_{row p}) from the same z = A x_k,
 * then x_i <- prox (with beta L_i), then z += delta_i a_i in ascending i.
 * L holds s * sup(phi'') * ||a_i||^2.  Returns the count of changed
 * coordinates or -1 (duplicate / out-of-range index).
 */
int64_t orc_model_step_with_set(int64_t m, int64_t n, const int64_t *col_ptr, const int32_t *row_idx,
                                const double *val, const double *L, const double *y, int loss, double s,
                                double l1, double l2, double c, double lo, double hi, double beta, int64_t tau,
                                const int64_t *S, double *x, double *z)
{
    int64_t *ids = (int64_t *)malloc((size_t)(tau > 0 ? tau : 1) * sizeof(int64_t));
    double *delta = (double *)malloc((size_t)(tau > 0 ? tau : 1) * sizeof(double));
    int64_t changed = 0;
    (void)m;
    if (!ids || !delta) {
        free(ids);
        free(delta);
        return -1;
    }
    memcpy(ids, S, (size_t)tau * sizeof(int64_t));
    qsort(ids, (size_t)tau, sizeof(int64_t), orc_cmp_i64);
    for (int64_t t = 0; t < tau; ++t) {
        if (ids[t] < 0 || ids[t] >= n || (t > 0 && ids[t] == ids[t - 1])) {
            free(ids);
            free(delta);
            return -1;
        }
    }
    for (int64_t t = 0; t < tau; ++t) {
        int64_t i = ids[t];
        double g = 0.0, bl = beta * L[i];
        for (int64_t p = col_ptr[i]; p < col_ptr[i + 1]; ++p)
            g += val[p] * orc_dphi(loss, z[row_idx[p]], y[row_idx[p]]);
        g *= s;
        delta[t] = orc_model_prox(x[i] - g / bl, bl, l1, l2, c, lo, hi) - x[i];
    }
    for (int64_t t = 0; t < tau; ++t) {
        int64_t i = ids[t];
        if (delta[t] == 0.0)
            continue;
        ++changed;
        x[i] += delta[t];
        for (int64_t p = col_ptr[i]; p < col_ptr[i + 1]; ++p)
            z[row_idx[p]] += delta[t] * val[p];
    }
    free(ids);
    free(delta);
    return changed;
}

/* nsteps tau-nice steps k0 .. k0+nsteps-1 of the model (z = A x on entry). */
int64_t orc_model_run(int64_t m, int64_t n, const int64_t *col_ptr, const int32_t *row_idx, const double *val,
                      const double *L, const double *y, int loss, double s, double l1, double l2, double c,
                      double lo, double hi, double beta, int64_t tau, uint64_t seed, int64_t k0, int64_t nsteps,
                      double *x, double *z)
{
    int64_t *S = (int64_t *)malloc((size_t)(tau > 0 ? tau : 1) * sizeof(int64_t));
    int64_t total = 0;
    if (!S)
        return -1;
    for (int64_t k = k0; k < k0 + nsteps; ++k) {
        int64_t cnt;
        if (orc_sample_nice(seed, (uint64_t)k, tau, n, S) != 0) {
            free(S);
            return -1;
        }
        cnt = orc_model_step_with_set(m, n, col_ptr, row_idx, val, L, y, loss, s, l1, l2, c, lo, hi, beta, tau, S,
                                      x, z);
        if (cnt < 0) {
            free(S);
            return -1;
        }
        total += cnt;
    }
    free(S);
    return total;
}
