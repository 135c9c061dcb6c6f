/*
 * gace_est.h -- sample-scaled estimates from the probe's exact sample counts
 * (host arithmetic only; no device access).
 *
 * The probe returns exact integers on a block-Bernoulli sample (gace.h).  The
 * optimizer needs population quantities: the selectivity and cardinality of
 * a condition, the size of an equi-join, the NDV of a join key (Eq. 1's
 * NDV_est).  These calls scale the sample counts:
 *   selectivity   S = count / sampled_rows           (S_probe of Eq. 2; ratio estimator)
 *   cardinality   count / p                          (Horvitz-Thompson; p = thr / 2^32 is
 *                                                     every row's inclusion probability,
 *                                                     thr = floor(rate * 2^32))
 *   join size     join_card / (p_R p_S)              (Horvitz-Thompson over row pairs; the two
 *                                                     samples are drawn independently)
 *   NDV           GEE: sqrt(n / r) f_1 + (d - f_1)   (Charikar, Chaudhuri, Motwani, Narasayya,
 *                                                     PODS 2000; n table rows, r sampled rows,
 *                                                     d sampled distinct keys, f_1 keys seen once)
 * The paper's Exp. B measures the spread of such estimates across sampling
 * seeds (Est.CV) against the probing budget.
 *
 * All arithmetic is IEEE binary64 in the order written above.  Errors:
 * GACE_EINVAL for NULL pointers, a spec that gace_check_request would reject,
 * or counts that no sample can have (count > sampled_rows, sampled_rows >
 * n_rows, f_1 > d, d > r, r > n).
 */
#ifndef GACE_EST_H
#define GACE_EST_H

#include "gace.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double p;          /* row inclusion probability thr / 2^32 (1 when rate is 1) */
    double sel;        /* count / sampled_rows (NaN when nothing was sampled) */
    double card;       /* sel * n_rows (NaN when nothing was sampled) */
    double card_ht;    /* count / p (NaN when p = 0) */
} gace_sel_estimate;

/* Estimates of one predicate of a selectivity probe of a table of n_rows
   rows (spec NULL: rate 1). */
gace_status gace_estimate_selectivity(uint64_t count, const gace_probe_info* info, uint64_t n_rows,
                                      const gace_sample_spec* spec, gace_sel_estimate* out);

typedef struct {
    double p_R, p_S;       /* inclusion probabilities */
    double join_ht;        /* join_card / (p_R p_S) (NaN when either p is 0) */
    double ndv_R, ndv_S;   /* GEE scale-up of the sampled NDVs (0 when nothing was sampled) */
} gace_join_estimate;

/* Estimates from a join-frequency probe of R (n_rows_R keys) and S. */
gace_status gace_estimate_join(const gace_join_result* r, uint64_t n_rows_R, const gace_sample_spec* spec_R,
                               uint64_t n_rows_S, const gace_sample_spec* spec_S, gace_join_estimate* out);

#ifdef __cplusplus
}
#endif

#endif /* GACE_EST_H */
