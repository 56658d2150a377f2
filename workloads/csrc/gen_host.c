/* gen_host.c -- the host build of gen_common.h: regenerate any column, any
 * planted entry and any noise term on the CPU (input construction only). */
#include "gen_common.h"

#include <pthread.h>
#include <stdlib.h>

int gen_host_column(uint64_t seed, uint64_t m, uint64_t n, int d, uint64_t i, int32_t *rows, double *vals)
{
    if (d < 1 || d > GEN_MAX_D || (uint64_t)d > m || i >= n)
        return -1;
    gen_column(seed, m, n, d, i, rows, vals);
    return 0;
}

void gen_host_xstar(uint64_t seed, uint64_t n, uint64_t j, uint64_t *pos, double *val)
{
    gen_xstar(seed, n, j, pos, val);
}

double gen_host_noise(uint64_t seed, uint64_t row, double sigma) { return gen_noise(seed, row, sigma); }

static double gen_round(double v, int dtype)
{
    if (dtype == 0)
        return (double)(float)v;
    if (dtype == 1) {
        union {
            float f;
            uint32_t u;
        } c;
        c.f = (float)v;
        c.u += ((c.u >> 16) & 1u) + 0x7FFFu;
        c.u &= 0xFFFF0000u;
        return (double)c.f;
    }
    return v;
}

/* Column i with values rounded to the storage dtype (0 f32, 1 bf16, 2 f64). */
int gen_host_column_stored(uint64_t seed, uint64_t m, uint64_t n, int d, uint64_t i, int dtype, int32_t *rows,
                           double *vals)
{
    int st = gen_host_column(seed, m, n, d, i, rows, vals);
    for (int t = 0; st == 0 && t < d; ++t)
        vals[t] = gen_round(vals[t], dtype);
    return st;
}

/* ax[0..m) += A x* (stored values), and the planted entries' positions/values. */
int gen_host_plant(uint64_t seed, uint64_t m, uint64_t n, int d, uint64_t K, int dtype, double *ax,
                   uint64_t *pos_out, double *val_out)
{
    int32_t r[GEN_MAX_D];
    double v[GEN_MAX_D];
    if (d < 1 || d > GEN_MAX_D || (uint64_t)d > m || K > n)
        return -1;
    for (uint64_t j = 0; j < K; ++j) {
        uint64_t pos;
        double xv;
        gen_xstar(seed, n, j, &pos, &xv);
        if (pos_out)
            pos_out[j] = pos;
        if (val_out)
            val_out[j] = xv;
        gen_column(seed, m, n, d, pos, r, v);
        for (int t = 0; t < d; ++t)
            ax[r[t]] += xv * gen_round(v[t], dtype);
    }
    return 0;
}

void gen_host_noise_rows(uint64_t seed, const int64_t *rows, int64_t cnt, double sigma, double *out)
{
    for (int64_t q = 0; q < cnt; ++q)
        out[q] = gen_noise(seed, (uint64_t)rows[q], sigma);
}

/* Whole CSC on the host (rows [n*d], stored values [n*d] as float64). */
int gen_host_csc(uint64_t seed, uint64_t m, uint64_t n, int d, int dtype, int32_t *rows, double *vals)
{
    for (uint64_t i = 0; i < n; ++i) {
        int st = gen_host_column_stored(seed, m, n, d, i, dtype, rows + (uint64_t)d * i, vals + (uint64_t)d * i);
        if (st)
            return st;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Threaded regeneration for instances too large to build whole on the host: */
/* a column range or a column list (rows and stored values), and all of b.  */
/* Threads split the work by columns or rows; every output element is       */
/* written by exactly one thread, so results do not depend on the split.   */
/* A thread that cannot be started has its share run on the calling thread. */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t seed, m, n, K;
    int d, dtype;
    int64_t q0, q1;        /* [q0, q1) of the work items */
    uint64_t i0;           /* first column (range form) */
    const int64_t *cols;   /* column list (list form), or NULL */
    int32_t *rows;
    float *vals32;         /* stored values as float32 (f32 / bf16), or NULL */
    double *vals64;        /* stored values as float64, or NULL */
    double *b;             /* rows form: b[q0..q1) (noise part added) */
    double sigma;
    int bad;
} gen_job;

static void *gen_cols_worker(void *arg)
{
    gen_job *J = (gen_job *)arg;
    double v[GEN_MAX_D];
    for (int64_t q = J->q0; q < J->q1; ++q) {
        const uint64_t col = J->cols ? (uint64_t)J->cols[q] : J->i0 + (uint64_t)q;
        int32_t *r = J->rows + (uint64_t)J->d * (uint64_t)q;
        if (gen_host_column_stored(J->seed, J->m, J->n, J->d, col, J->dtype, r, v) != 0) {
            J->bad = 1;
            return NULL;
        }
        for (int t = 0; t < J->d; ++t) {
            if (J->vals32)
                J->vals32[(uint64_t)J->d * (uint64_t)q + t] = (float)v[t];
            if (J->vals64)
                J->vals64[(uint64_t)J->d * (uint64_t)q + t] = v[t];
        }
    }
    return NULL;
}

static void *gen_noise_worker(void *arg)
{
    gen_job *J = (gen_job *)arg;
    for (int64_t q = J->q0; q < J->q1; ++q)
        J->b[q] += gen_noise(J->seed, (uint64_t)q, J->sigma);
    return NULL;
}

static int gen_run(gen_job *proto, int64_t items, int nthreads, void *(*fn)(void *))
{
    gen_job jobs[64];
    pthread_t th[64];
    int started[64];
    const int nt = nthreads < 1 ? 1 : (nthreads > 64 ? 64 : nthreads);
    int bad = 0;
    for (int t = 0; t < nt; ++t) {
        jobs[t] = *proto;
        jobs[t].q0 = items * t / nt;
        jobs[t].q1 = items * (t + 1) / nt;
        jobs[t].bad = 0;
        started[t] = pthread_create(&th[t], NULL, fn, &jobs[t]) == 0;
        if (!started[t])
            fn(&jobs[t]);
    }
    for (int t = 0; t < nt; ++t) {
        if (started[t])
            pthread_join(th[t], NULL);
        bad |= jobs[t].bad;
    }
    return bad ? -1 : 0;
}

/* Columns [i0, i0 + count): rows[count*d] (sorted per column) and the stored
 * values as float32 (vals32, for dtype f32 / bf16, exact) and/or float64
 * (vals64); either pointer may be NULL. */
int gen_host_columns(uint64_t seed, uint64_t m, uint64_t n, int d, int dtype, uint64_t i0, int64_t count,
                     int32_t *rows, float *vals32, double *vals64, int nthreads)
{
    if (count < 0 || i0 + (uint64_t)count > n || (vals32 && dtype == 2))
        return -1;
    gen_job J = {seed, m, n, 0, d, dtype, 0, 0, i0, NULL, rows, vals32, vals64, NULL, 0.0, 0};
    return gen_run(&J, count, nthreads, gen_cols_worker);
}

/* The columns cols[0..count) (any order, each < n), as gen_host_columns. */
int gen_host_column_list(uint64_t seed, uint64_t m, uint64_t n, int d, int dtype, const int64_t *cols,
                         int64_t count, int32_t *rows, float *vals32, double *vals64, int nthreads)
{
    if (count < 0 || (vals32 && dtype == 2))
        return -1;
    for (int64_t q = 0; q < count; ++q)
        if (cols[q] < 0 || (uint64_t)cols[q] >= n)
            return -1;
    gen_job J = {seed, m, n, 0, d, dtype, 0, 0, 0, cols, rows, vals32, vals64, NULL, 0.0, 0};
    return gen_run(&J, count, nthreads, gen_cols_worker);
}

/* All of b [m]: A x* with the stored values, plus the noise of every row. */
int gen_host_b(uint64_t seed, uint64_t m, uint64_t n, int d, uint64_t K, double sigma, int dtype, double *b,
               int nthreads)
{
    for (uint64_t j = 0; j < m; ++j)
        b[j] = 0.0;
    if (gen_host_plant(seed, m, n, d, K, dtype, b, NULL, NULL) != 0)
        return -1;
    gen_job J = {seed, m, n, K, d, dtype, 0, 0, 0, NULL, NULL, NULL, NULL, b, sigma, 0};
    return gen_run(&J, (int64_t)m, nthreads, gen_noise_worker);
}
