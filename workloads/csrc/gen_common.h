/*
 * gen_common.h -- counter-based generator of large synthetic LASSO inputs
 * (input construction only; none of the coordinate-descent arithmetic).
 * Compiled twice from this one source: into a HIP kernel library that
 * writes the arrays on the device, and into a host library that regenerates
 * any column, any entry of x* and any entry of b on the CPU, so a checker can
 * rebuild sampled inputs without reading device memory.
 *
 * Recipe (seed s, m rows, n columns, d entries per column):
 *   - entry slot p = d*i + t of column i is dealt to row
 *     perm(p) mod m, perm a keyed bijection of [0, n*d) (balanced slots: every
 *     row receives floor or ceil of n*d/m slots); a row repeated inside one
 *     column is redrawn as hash(s, i, t, attempt) mod m until distinct; rows
 *     of a column are sorted;
 *   - values N(0,1) by Box-Muller from two 53-bit uniforms per entry, the
 *     column scaled to unit norm in float64;
 *   - x*: K entries at perm'(j), j < K (a second keyed bijection of [0, n)),
 *     value sign * (1 + U), U uniform on [0, 1), fair sign;
 *   - b = A x* + sigma * N(0,1) per row.
 * Random words: SplitMix64 (Steele, Lea & Flood, 2014) outputs of streams
 * keyed by (s, purpose); bijections: balanced 6-round Feistel networks with
 * the SplitMix64 finaliser as round function, restricted by cycle walking
 * (Black & Rogaway, 2002).
 */
#ifndef GEN_COMMON_H
#define GEN_COMMON_H

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define GEN_FN __host__ __device__ static inline
#else
#define GEN_FN static inline
#endif

#define GEN_MAX_D 64

GEN_FN uint64_t gen_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* output t of the SplitMix64 stream started at `state` */
GEN_FN uint64_t gen_word(uint64_t state, uint64_t t) { return gen_mix(state + (t + 1) * 0x9E3779B97F4A7C15ull); }

/* stream keys per purpose */
GEN_FN uint64_t gen_key(uint64_t seed, uint64_t purpose) { return gen_word(seed ^ 0x47454E4C4153534Full, purpose); }

enum { GEN_SLOTS = 1, GEN_REDRAW = 2, GEN_VALUES = 3, GEN_XPOS = 4, GEN_XVAL = 5, GEN_NOISE = 6 };

typedef struct {
    uint64_t key[6];
    int half;
    uint64_t size;
} gen_perm;

GEN_FN gen_perm gen_perm_make(uint64_t stream, uint64_t size)
{
    gen_perm P;
    int h = 1;
    while (h < 32 && (((uint64_t)1) << (2 * h)) < size)
        ++h;
    P.half = h;
    P.size = size;
    for (int q = 0; q < 6; ++q)
        P.key[q] = gen_word(stream, (uint64_t)q);
    return P;
}

GEN_FN uint64_t gen_perm_once(const gen_perm *P, uint64_t v)
{
    const uint64_t mask = (((uint64_t)1) << P->half) - 1;
    uint64_t hi = v >> P->half, lo = v & mask;
    for (int q = 0; q < 6; ++q) {
        const uint64_t t = hi ^ (gen_mix(lo ^ P->key[q]) & mask);
        hi = lo;
        lo = t;
    }
    return (hi << P->half) | lo;
}

GEN_FN uint64_t gen_perm_apply(const gen_perm *P, uint64_t v)
{
    uint64_t y = gen_perm_once(P, v);
    while (y >= P->size)
        y = gen_perm_once(P, y);
    return y;
}

GEN_FN double gen_unit(uint64_t w) { return (double)(w >> 11) * (1.0 / 9007199254740992.0); }

/* standard normal for counter c of a stream (Box-Muller, cosine branch) */
GEN_FN double gen_normal(uint64_t stream, uint64_t c)
{
    double u1 = gen_unit(gen_word(stream, 2 * c));
    const double u2 = gen_unit(gen_word(stream, 2 * c + 1));
    if (u1 <= 0.0)
        u1 = 1.0 / 9007199254740992.0;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* Rows (sorted, distinct) and float64 values (unit column norm) of column i. */
GEN_FN void gen_column(uint64_t seed, uint64_t m, uint64_t n, int d, uint64_t i, int32_t *rows, double *vals)
{
    const gen_perm P = gen_perm_make(gen_key(seed, GEN_SLOTS), n * (uint64_t)d);
    const uint64_t rs = gen_key(seed, GEN_REDRAW), vs = gen_key(seed, GEN_VALUES);
    for (int t = 0; t < d; ++t) {
        uint64_t r = gen_perm_apply(&P, (uint64_t)d * i + (uint64_t)t) % m;
        for (uint64_t a = 0;; ++a) {
            int dup = 0;
            for (int q = 0; q < t; ++q)
                dup |= rows[q] == (int32_t)r;
            if (!dup)
                break;
            r = gen_word(rs, ((uint64_t)d * i + (uint64_t)t) * 64 + a) % m;
        }
        rows[t] = (int32_t)r;
    }
    /* insertion sort of the rows */
    for (int t = 1; t < d; ++t) {
        const int32_t v = rows[t];
        int q = t - 1;
        while (q >= 0 && rows[q] > v) {
            rows[q + 1] = rows[q];
            --q;
        }
        rows[q + 1] = v;
    }
    double ss = 0.0;
    for (int t = 0; t < d; ++t) {
        vals[t] = gen_normal(vs, (uint64_t)d * i + (uint64_t)t);
        ss += vals[t] * vals[t];
    }
    const double inv = 1.0 / sqrt(ss);
    for (int t = 0; t < d; ++t)
        vals[t] *= inv;
}

/* j-th planted entry: position and value */
GEN_FN void gen_xstar(uint64_t seed, uint64_t n, uint64_t j, uint64_t *pos, double *val)
{
    const gen_perm P = gen_perm_make(gen_key(seed, GEN_XPOS), n);
    *pos = gen_perm_apply(&P, j);
    const uint64_t w = gen_word(gen_key(seed, GEN_XVAL), j);
    const double mag = 1.0 + gen_unit(gen_word(gen_key(seed, GEN_XVAL), j + 0x100000000ull));
    *val = (w & 1) ? -mag : mag;
}

GEN_FN double gen_noise(uint64_t seed, uint64_t row, double sigma) { return sigma * gen_normal(gen_key(seed, GEN_NOISE), row); }

#endif
