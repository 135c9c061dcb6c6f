/*
 * oracle.h -- plain CPU oracle for the sampled predicate-count probe and the
 * key-only join-key frequency probe of the GACE Measurement Engine
 * (Chang, "Risk-Aware GPU-Assisted Cardinality Estimation for Cost-Based Query
 * Optimizers", arXiv 2512.19750, Sec. III-B).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may call this code.  The product library never
 * links, loads or calls it, and it shares no code with the device path.
 *
 * Every function computes the plain definition, slowly and visibly:
 *   - sampling: block b of B rows is kept iff word 0 of Philox4x32-10
 *     (Salmon, Moraes, Dror, Shaw, SC'11) under key = seed and counter =
 *     (b_lo, b_hi, table_id, 0) is below thr = floor(rate * 2^32); rate 1
 *     keeps every block;
 *   - a predicate is a conjunction of terms; count[p] is the number of kept
 *     rows on which every term of p holds (S_probe = count / sampled, Eq. 2);
 *   - join: f_X(k) is the number of sampled occurrences of key k in X;
 *     NDV_X = |{k : f_X(k) > 0}| (the NDV of Eq. 1); join = sum_k f_R(k) f_S(k).
 */
#ifndef GACE_ORACLE_H
#define GACE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_I32 = 1, ORC_I64 = 2, ORC_F32 = 3 };
enum { ORC_RANGE = 1, ORC_EQ = 2, ORC_IN = 3 };

typedef struct { const void* data; uint32_t dtype; uint32_t pad; } orc_col;

/* RANGE: v[0] <= x < v[1]; EQ: x == v[0]; IN: x equals one of v[0..n_vals).
   Integer columns compare in int64 (int32 values sign-extended).  Float
   columns take the float whose bit pattern is the low 32 bits of v[i] and
   compare with IEEE semantics (NaN never matches, -0.0 == +0.0). */
typedef struct { uint32_t col, op, n_vals, pad; int64_t v[8]; } orc_term;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint64_t orc_threshold(double rate);   /* 2^32 means "keep all" */
int orc_block_kept(uint64_t seed, uint32_t table_id, uint64_t block, uint64_t thr);

/* indices of kept blocks of an n_rows table, in increasing order; returns the
   count (writes at most cap entries) */
uint64_t orc_kept_blocks(uint64_t n_rows, uint64_t seed, uint32_t table_id, double rate,
                         uint32_t block_rows, uint64_t* out, uint64_t cap);

/* 0 on success, -1 on an invalid argument. */
int orc_probe_selectivity(uint64_t n_rows, const orc_col* cols, uint32_t n_cols, uint32_t table_id,
                          const orc_term* terms, const uint32_t* pred_off, uint32_t n_preds,
                          uint64_t seed, double rate, uint32_t block_rows,
                          uint64_t* counts, uint64_t* sampled_rows, uint64_t* kept_blocks,
                          int nthreads);

/* out = {join, ndv_R, ndv_S, n_R, n_S, f1_R, f1_S, f2_R, f2_S}, where f1 / f2
   count the distinct sampled keys seen exactly once / twice on that side;
   0, -1 (invalid) or -3 (overflow). */
int orc_join_freq(const int64_t* keys_r, uint64_t n_r, uint32_t tid_r, uint64_t seed_r, double rate_r,
                  uint32_t block_rows_r,
                  const int64_t* keys_s, uint64_t n_s, uint32_t tid_s, uint64_t seed_s, double rate_s,
                  uint32_t block_rows_s, uint64_t out[9]);

/* sorts int64 keys ascending in place (step of orc_join_freq, exported for tests) */
int orc_sort_i64(int64_t* keys, uint64_t n);

#ifdef __cplusplus
}
#endif

#endif
