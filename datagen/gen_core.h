/*
 * gen_core.h -- the seeded, counter-based column generator used to build the
 * synthetic inputs of every workload.
 *
 * This file holds no part of the probe method (no sampler, no predicate
 * evaluation, no counting, no hashing of keys): it only turns
 * (stream seed, row) into a column value, so that any row range of a table can
 * be regenerated on the host or on the device, byte for byte the same.
 *
 * The includer defines GG_FN (the function qualifier: plain `static inline` in
 * C host code, `__device__ static inline` in device code) and, for Zipf
 * columns, passes the integer CDF table built by gg_zipf_cdf() on the host.
 *
 * Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014).  Output i of stream s is
 * mix64(s + (i + 1) * 0x9E3779B97F4A7C15).
 */
#ifndef GACE_GEN_CORE_H
#define GACE_GEN_CORE_H

#include <stdint.h>

#ifndef GG_FN
#error "define GG_FN before including gen_core.h"
#endif

/* column value laws */
#define GG_UNIFORM 1u  /* lo + floor(u * span / 2^64)                        */
#define GG_ZIPF    2u  /* lo + r, r = rank drawn from a bounded Zipf CDF      */
#define GG_F32UNIT 3u  /* (u >> 40) * 2^-24, a float in [0, 1)                */

/* storage types (same codes as the probe library's column dtypes) */
#define GG_I32 1u
#define GG_I64 2u
#define GG_F32 3u

#define GG_GAMMA 0x9E3779B97F4A7C15ull

typedef struct gg_col {
    uint32_t kind;        /* GG_UNIFORM / GG_ZIPF / GG_F32UNIT                     */
    uint32_t dtype;       /* GG_I32 / GG_I64 / GG_F32                             */
    uint64_t seed;        /* stream seed of the base law (gg_stream_seed)          */
    int64_t lo;           /* UNIFORM and ZIPF: offset added to the drawn value     */
    uint64_t span;        /* UNIFORM: number of values (>= 1)                      */
    const uint64_t* cdf;  /* ZIPF: ncdf cumulative thresholds on a 2^53 scale      */
    uint64_t ncdf;        /* ZIPF: domain size                                     */
    uint64_t noise_seed;  /* additive integer noise stream (used if noise_span>0)  */
    int64_t noise_lo;     /* noise = noise_lo + floor(u * noise_span / 2^64)       */
    uint64_t noise_span;
} gg_col;

GG_FN uint64_t gg_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Stream seed for (user seed, table, column, draw index). */
GG_FN uint64_t gg_stream_seed(uint64_t seed, uint32_t table, uint32_t col, uint32_t draw) {
    uint64_t tag = ((uint64_t)table << 32) ^ ((uint64_t)col << 8) ^ (uint64_t)draw;
    return gg_mix64(seed ^ gg_mix64(tag + GG_GAMMA));
}

GG_FN uint64_t gg_u64(uint64_t stream, uint64_t row) {
    return gg_mix64(stream + (row + 1u) * GG_GAMMA);
}

/* high 64 bits of a 64x64 product, written with 32-bit limbs so host and
   device code are the same arithmetic */
GG_FN uint64_t gg_mulhi64(uint64_t a, uint64_t b) {
    uint64_t a0 = a & 0xFFFFFFFFull, a1 = a >> 32;
    uint64_t b0 = b & 0xFFFFFFFFull, b1 = b >> 32;
    uint64_t p00 = a0 * b0, p01 = a0 * b1, p10 = a1 * b0, p11 = a1 * b1;
    uint64_t mid = (p00 >> 32) + (p01 & 0xFFFFFFFFull) + (p10 & 0xFFFFFFFFull);
    return p11 + (p01 >> 32) + (p10 >> 32) + (mid >> 32);
}

/* smallest r in [0, n) with x < cdf[r]; cdf[n-1] == 2^53 > x always */
GG_FN uint64_t gg_zipf_rank(const uint64_t* cdf, uint64_t n, uint64_t x) {
    uint64_t a = 0, b = n - 1u;
    while (a < b) {
        uint64_t m = a + ((b - a) >> 1);
        if (x < cdf[m]) b = m; else a = m + 1u;
    }
    return a;
}

/* The value of column c at row `row`, widened to int64 (integer columns) or
   returned as raw float bits in the low 32 bits (GG_F32UNIT). */
GG_FN int64_t gg_value(const gg_col* c, uint64_t row) {
    uint64_t u = gg_u64(c->seed, row);
    int64_t v;
    if (c->kind == GG_F32UNIT) {
        float f = (float)(uint32_t)(u >> 40) * 5.9604644775390625e-08f; /* 2^-24 */
        union { float f; uint32_t b; } cv;
        cv.f = f;
        return (int64_t)cv.b;
    } else if (c->kind == GG_ZIPF) {
        v = c->lo + (int64_t)gg_zipf_rank(c->cdf, c->ncdf, u >> 11);
    } else {
        v = c->lo + (int64_t)gg_mulhi64(u, c->span);
    }
    if (c->noise_span) {
        uint64_t w = gg_u64(c->noise_seed, row);
        v += c->noise_lo + (int64_t)gg_mulhi64(w, c->noise_span);
    }
    return v;
}

#endif /* GACE_GEN_CORE_H */
