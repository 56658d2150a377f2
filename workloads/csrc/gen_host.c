/* gen_host.c -- the host build of gen_common.h: regenerate any column, any
 * planted entry and any noise term on the CPU (input construction only). */
#include "gen_common.h"

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
