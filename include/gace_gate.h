/*
 * gace_gate.h -- host-side decision layer over the probe library (gace.h):
 * the Risky Gate's trust metrics, the measurement-cost model with its
 * break-even point, and a cache of probe results.
 *
 * The Risky Gate (Sec. III-A) sends a query to the GPU Measurement Engine
 * only when one of its risk signals crosses a threshold (Sec. III-C):
 *   drift        D = |NDV_hist - NDV_est| / NDV_hist,  trigger when D >= 0.25  (Eq. 1)
 *   selectivity  |S_est - S_probe| > 0.01                                      (Eq. 2)
 *   correlation  PCS = P(A,B) / (P(A) P(B)), breach when > 1.6 or < 0.7        (Eq. 3)
 * The measurement cost is modelled from measured kernel latencies (Eq. 4
 * quotes a constant of 0.85 ms; here it is the prior until latencies are
 * observed), and a break-even sample size in the number of candidate
 * conditions and the sample size decides whether offloading pays (Sec. V,
 * item 2).  Probe results are cached by bind value (Sec. V, item 3).
 *
 * Everything here runs on the host and touches no device memory, except
 * gace_probe_pcs, gace_probe_selectivity_cached and gace_join_freq_cached,
 * which run probes through the context exactly like gace_probe_selectivity /
 * gace_join_freq (same argument rules, ownership, streams and errors).
 * Errors follow gace.h: a negative gace_status, outputs untouched,
 * gace_last_error() set.  Objects are thread-safe (one mutex each).
 */
#ifndef GACE_GATE_H
#define GACE_GATE_H

#include "gace.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- Risky Gate */
/* signal bits: in gace_gate_in.have (which inputs are supplied) and in
   gace_gate_out.flags (which thresholds were crossed) / .undefined */
#define GACE_GATE_DRIFT 1u   /* Eq. 1 */
#define GACE_GATE_SELERR 2u  /* Eq. 2 */
#define GACE_GATE_PCS 4u     /* Eq. 3, inputs */
#define GACE_GATE_PCS_HI 4u  /* Eq. 3: PCS above pcs_hi (underestimation risk) */
#define GACE_GATE_PCS_LO 8u  /* Eq. 3: PCS below pcs_lo (overestimation risk) */

/* Thresholds.  The PCS bounds are rationals so that the breach test is
   exact on the integer counts. */
typedef struct {
    double drift_min;       /* D >= drift_min triggers (Sec. III-C: 0.25) */
    double sel_err_max;     /* |S_est - S_probe| > sel_err_max triggers (0.01) */
    uint32_t pcs_hi_num, pcs_hi_den;  /* 8 / 5 = 1.6 */
    uint32_t pcs_lo_num, pcs_lo_den;  /* 7 / 10 = 0.7 */
} gace_gate_cfg;

/* Inputs.  Only the signals whose bit is set in `have` are read. */
typedef struct {
    uint32_t have;
    uint32_t reserved;
    double ndv_hist;        /* Eq. 1: the optimizer's histogram NDV (> 0) */
    double ndv_est;         /* Eq. 1: the estimated NDV (>= 0) */
    double s_est;           /* Eq. 2: the optimizer's selectivity estimate, in [0, 1] */
    uint64_t count, n;      /* Eq. 2: S_probe = count / n (count <= n) */
    uint64_t c_ab, c_a, c_b, n_pcs;  /* Eq. 3: rows satisfying A and B, A, B, of n_pcs sampled rows */
} gace_gate_in;

/* Outputs.  drift = |ndv_hist - ndv_est| / ndv_hist and
   sel_err = |s_est - count / n| are evaluated in IEEE binary64 in that order
   and compared with the thresholds in binary64.  pcs = (c_ab * n_pcs) /
   (c_a * c_b) in binary64 is informative only: the PCS flags are decided
   exactly on the integers (5 c_ab n > 8 c_a c_b for 8/5).  A supplied signal
   that has no value (n == 0; c_a == 0 or c_b == 0, where PCS is 0/0) sets its
   bit in `undefined`, raises no flag, and reports NaN. */
typedef struct {
    double drift, sel_err, pcs;
    uint32_t flags;         /* GACE_GATE_DRIFT | GACE_GATE_SELERR | GACE_GATE_PCS_HI | GACE_GATE_PCS_LO */
    uint32_t undefined;     /* GACE_GATE_SELERR | GACE_GATE_PCS */
    uint32_t trigger;       /* 1 iff flags != 0: send the query to the Measurement Engine */
    uint32_t reserved;
} gace_gate_out;

/* The paper's thresholds (0.25, 0.01, 8/5, 7/10). */
gace_status gace_gate_default_cfg(gace_gate_cfg* out);
/* Evaluate the supplied signals.  GACE_EINVAL for: NULL pointers; a
   threshold that is NaN, negative or infinite, a zero denominator, or
   pcs_lo > pcs_hi; ndv_hist not finite or <= 0; ndv_est NaN, infinite or < 0;
   s_est NaN or outside [0, 1]; count > n; counts that no sample can have
   (c_ab > c_a, c_ab > c_b, c_a > n_pcs, c_b > n_pcs, c_a + c_b - c_ab > n_pcs);
   n or n_pcs >= 2^48. */
gace_status gace_gate_evaluate(const gace_gate_cfg* cfg, const gace_gate_in* in, gace_gate_out* out);

/* Joint and marginal counts for Eq. 3 from ONE probe: predicates A and B
   (pair = exactly 2 predicates in CSR form, together at most 16 terms) are
   measured as the three candidate conditions {A, B, A AND B} on one sample.
   out: c_a, c_b, c_ab and n_pcs (= sampled rows) of a gace_gate_in; its
   `have` gains GACE_GATE_PCS and its other fields are left as they were. */
gace_status gace_probe_pcs(gace_ctx* ctx, const gace_table* table, const gace_predicates* pair,
                           const gace_sample_spec* spec, gace_gate_in* out, void* stream);

/* ---------------------------------------------------------------- cost model */
/* Measurement cost of one probe, modelled as
     ms = c[0] + c[1] * (n_rows * row_bytes) + c[2] * (n_rows * terms),
   c >= 0 fitted by non-negative least squares to observed (features, ms)
   pairs (the last `window` of them).  With fewer than 3 observations the
   model is the prior: c = (prior_ms, 0, 0), Eq. 4's constant cost. */
typedef struct gace_cost_model gace_cost_model;

typedef struct {
    double n_rows;      /* N: sampled rows read */
    double row_bytes;   /* bytes per row of the referenced columns (key-only) */
    double terms;       /* predicate terms evaluated per row: sum over the candidate conditions */
    double reserved;
} gace_cost_features;

gace_status gace_cost_create(double prior_ms, uint32_t window, gace_cost_model** out);
gace_status gace_cost_destroy(gace_cost_model* m);
/* Record one measured latency (ms >= 0 and finite; features >= 0 and finite). */
gace_status gace_cost_observe(gace_cost_model* m, const gace_cost_features* f, double ms);
/* Current coefficients (refitted when observations changed) and the number
   of observations they rest on. */
gace_status gace_cost_coef(gace_cost_model* m, double coef[3], uint32_t* n_obs);
gace_status gace_cost_predict(gace_cost_model* m, const gace_cost_features* f, double* ms);
/* Features of a selectivity request before it runs: n_rows = rate x table
   rows (the expected sample), row_bytes = widths of the referenced columns,
   terms = total terms over its predicates. */
gace_status gace_cost_features_of(const gace_request* req, gace_cost_features* out);
/* Break-even sample size of offloading: the smallest N >= 0 at which the
   device model's prediction is at most the host model's, for a request of
   row_bytes and terms per row.  +infinity when the device never pays (its
   per-row slope is not below the host's and its fixed cost is higher). */
gace_status gace_cost_breakeven(gace_cost_model* device, gace_cost_model* host, double row_bytes, double terms,
                                double* n_star);

/* ---------------------------------------------------------------- result cache */
/* Results cached by bind value: one entry per (table identity, sample,
   predicate), where the table identity is its table_id, row count and the
   addresses and types of the columns the predicate reads, the sample is
   (seed, rate threshold, block_rows), and the predicate is its set of terms
   with their values (IN lists as sets).  A join entry is keyed by both
   sides' (keys address, length, table_id, sample).  Entries are evicted
   least recently used beyond `capacity`.  The caller invalidates a table
   when its data changes. */
typedef struct gace_cache gace_cache;

typedef struct {
    uint64_t hits, misses, inserts, evictions, invalidated, entries;
} gace_cache_stats;

gace_status gace_cache_create(uint64_t capacity, gace_cache** out);
gace_status gace_cache_destroy(gace_cache* c);
/* Per predicate p: hit[p] = 1 and counts[p] filled when cached, else
   hit[p] = 0 and counts[p] untouched.  *n_hit = number of hits; info (may
   be NULL) is filled when at least one predicate hits.  Requests are
   validated as by gace_check_request. */
gace_status gace_cache_lookup(gace_cache* c, const gace_table* table, const gace_predicates* preds,
                              const gace_sample_spec* spec, uint64_t* counts, uint8_t* hit,
                              gace_probe_info* info, uint32_t* n_hit);
gace_status gace_cache_insert(gace_cache* c, const gace_table* table, const gace_predicates* preds,
                              const gace_sample_spec* spec, const uint64_t* counts, const gace_probe_info* info);
/* Drop every entry that reads table_id (either join side included). */
gace_status gace_cache_invalidate(gace_cache* c, uint32_t table_id);
gace_status gace_cache_stats_get(gace_cache* c, gace_cache_stats* out);

/* gace_probe_selectivity through the cache: the predicates that miss are
   measured in one probe and inserted; *n_hit (may be NULL) receives the
   number answered from the cache.  Results equal gace_probe_selectivity's. */
gace_status gace_probe_selectivity_cached(gace_ctx* ctx, gace_cache* c, const gace_table* table,
                                          const gace_predicates* preds, const gace_sample_spec* spec,
                                          uint64_t* counts, gace_probe_info* info, uint32_t* n_hit,
                                          void* stream);
/* gace_join_freq through the cache; *hit (may be NULL) = 1 when cached. */
gace_status gace_join_freq_cached(gace_ctx* ctx, gace_cache* c, const gace_keys* R, const gace_keys* S,
                                  gace_join_result* out, uint32_t* hit, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GACE_GATE_H */
