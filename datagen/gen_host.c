/*
 * gen_host.c -- host side of the seeded column generator (see gen_core.h).
 *
 * Exports:
 *   gg_zipf_cdf     integer CDF table of a bounded Zipf law (shared by the host
 *                   and device fills, so both draw identical ranks)
 *   gg_stream_seed_host
 *   gg_fill_host    rows [row0, row0 + n) of one column into a typed buffer
 *
 * Built with gcc into datagen/libgacegen_host.so.
 */
#define GG_FN static inline
#include "gen_core.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* Bounded Zipf: P(rank r) = r^-s / H(n, s), r = 1..n; table entry r-1 holds
   round(2^53 * P(rank <= r)), with the last entry forced to 2^53 and the
   table made non-decreasing.  Summation is compensated (Neumaier) so the
   table does not depend on the order of a parallel sum. */
int gg_zipf_cdf(double s, uint64_t n, uint64_t* out) {
    if (n == 0 || !out || !(s >= 0.0)) return -1;
    double sum = 0.0, comp = 0.0;
    for (uint64_t r = 1; r <= n; ++r) {
        double w = pow((double)r, -s);
        double t = sum + w;
        if (fabs(sum) >= fabs(w)) comp += (sum - t) + w; else comp += (w - t) + sum;
        sum = t;
    }
    double total = sum + comp;
    const double scale = 9007199254740992.0; /* 2^53 */
    sum = 0.0; comp = 0.0;
    uint64_t prev = 0;
    for (uint64_t r = 1; r <= n; ++r) {
        double w = pow((double)r, -s);
        double t = sum + w;
        if (fabs(sum) >= fabs(w)) comp += (sum - t) + w; else comp += (w - t) + sum;
        sum = t;
        double q = (sum + comp) / total * scale;
        uint64_t v = q >= scale ? (uint64_t)scale : (uint64_t)llround(q);
        if (v < prev) v = prev;
        out[r - 1] = v;
        prev = v;
    }
    out[n - 1] = (uint64_t)scale;
    return 0;
}

uint64_t gg_stream_seed_host(uint64_t seed, uint32_t table, uint32_t col, uint32_t draw) {
    return gg_stream_seed(seed, table, col, draw);
}

int64_t gg_value_host(const gg_col* c, uint64_t row) { return gg_value(c, row); }

typedef struct {
    const gg_col* c;
    uint64_t row0, begin, end;
    void* out;
} fill_job;

static void fill_range(const gg_col* c, uint64_t row0, uint64_t b, uint64_t e, void* out) {
    if (c->dtype == GG_I32) {
        int32_t* o = (int32_t*)out;
        for (uint64_t i = b; i < e; ++i) o[i] = (int32_t)gg_value(c, row0 + i);
    } else if (c->dtype == GG_I64) {
        int64_t* o = (int64_t*)out;
        for (uint64_t i = b; i < e; ++i) o[i] = gg_value(c, row0 + i);
    } else {
        uint32_t* o = (uint32_t*)out;
        for (uint64_t i = b; i < e; ++i) o[i] = (uint32_t)gg_value(c, row0 + i);
    }
}

static void* fill_worker(void* p) {
    fill_job* j = (fill_job*)p;
    fill_range(j->c, j->row0, j->begin, j->end, j->out);
    return NULL;
}

/* Fill out[0..n) with rows row0..row0+n-1 of column c using up to nthreads
   threads.  Returns 0, or -1 on a bad argument. */
int gg_fill_host(const gg_col* c, uint64_t row0, uint64_t n, void* out, int nthreads) {
    if (!c || (!out && n)) return -1;
    if (c->kind == GG_ZIPF && (!c->cdf || c->ncdf == 0)) return -1;
    if (c->kind == GG_UNIFORM && c->span == 0) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    if (n < 65536 || nthreads == 1) { fill_range(c, row0, 0, n, out); return 0; }
    pthread_t th[64];
    fill_job jobs[64];
    uint64_t per = (n + (uint64_t)nthreads - 1) / (uint64_t)nthreads;
    int started = 0;
    for (int t = 0; t < nthreads; ++t) {
        uint64_t b = per * (uint64_t)t, e = b + per > n ? n : b + per;
        if (b >= e) break;
        jobs[t].c = c; jobs[t].row0 = row0; jobs[t].begin = b; jobs[t].end = e; jobs[t].out = out;
        if (pthread_create(&th[t], NULL, fill_worker, &jobs[t]) != 0) {
            fill_range(c, row0, b, e, out);
            jobs[t].out = NULL;
        }
        started = t + 1;
    }
    for (int t = 0; t < started; ++t)
        if (jobs[t].out) pthread_join(th[t], NULL);
    return 0;
}

/* out[i] = value of column c at rows[i] (integers widened to int64, f32 as
   raw bits in the low 32 bits). */
int gg_values_at(const gg_col* c, const uint64_t* rows, uint64_t n, int64_t* out) {
    if (!c || (n && (!rows || !out))) return -1;
    if (c->kind == GG_ZIPF && (!c->cdf || c->ncdf == 0)) return -1;
    for (uint64_t i = 0; i < n; ++i) out[i] = gg_value(c, rows[i]);
    return 0;
}
