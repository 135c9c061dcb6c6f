/*
 * gace_host.h -- selectivity probes of tables that live in host memory, the
 * setting of the paper's Exp. A: the sample is moved host-to-device before
 * the kernel runs, either only the columns the predicates read ("Key-only",
 * the default principle of Sec. V item 1) or every column of each sampled
 * row (the full-row transfer Exp. A compares against).
 *
 * Pipeline (all on the context of gace.h):
 *   1. the block sampler runs on the device (one kernel over the table's
 *      block count, the same Philox4x32-10 decision as gace_probe_selectivity)
 *      and its kept-block bit mask is copied back;
 *   2. host threads gather the kept rows of the transferred columns into
 *      pinned staging, in chunks of at most chunk_rows rows;
 *   3. each chunk is copied host-to-device on a copy stream while the
 *      previous chunk is probed and the next one gathered (two staging slots
 *      on each side);
 *   4. each chunk is probed with the plain path's kernels (every staged row
 *      is a sampled row) and its counts are added on the host.
 * The result equals gace_probe_selectivity's on the same data, spec and
 * predicates: counts, sampled_rows and kept_blocks.
 *
 * Ownership and errors: column pointers are HOST pointers (pinned or
 * pageable), owned by the caller, 16-byte aligned, read only, valid until
 * the call returns.  Validation and error codes are those of
 * gace_probe_selectivity; GACE_ENOMEM if the context's workspace cannot hold
 * the two device staging slots plus the kept-block mask (the message gives
 * the bytes), GACE_EINVAL for bad options.  The call is synchronous and uses
 * the context's workspace: calls on one context must not overlap.
 */
#ifndef GACE_HOST_H
#define GACE_HOST_H

#include "gace.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    uint32_t key_only;        /* 1: transfer the columns the predicates read; 0: every column */
    uint32_t gather_threads;  /* host threads gathering kept rows (0 = 8; at most 64) */
    uint64_t chunk_rows;      /* sampled rows per staged chunk (0 = 2^22; 4096 .. 2^30) */
} gace_host_opts;

/* Where the time of one call went (Exp. A's decomposition).  Device phases
   are HIP-event times summed over chunks; host phases are wall times; with
   the pipeline they overlap, so the phases can sum to more than total_ms. */
typedef struct {
    double total_ms;    /* wall time of the call */
    double sample_ms;   /* sampler kernel + kept-block mask download + run list */
    double gather_ms;   /* host: kept rows into pinned staging */
    double h2d_ms;      /* device: host-to-device copies of the chunks */
    double kernel_ms;   /* device: probe kernels */
    double d2h_ms;      /* device: per-chunk count downloads */
    double reduce_ms;   /* host: summing the chunks' counts */
    uint64_t h2d_bytes; /* bytes copied host to device (chunks only) */
    uint32_t chunks;
    uint32_t reserved;
} gace_transfer_stats;

/* opts and stats may be NULL (defaults; no statistics). */
gace_status gace_probe_selectivity_host(gace_ctx* ctx, const gace_table* table, const gace_predicates* preds,
                                        const gace_sample_spec* spec, const gace_host_opts* opts,
                                        uint64_t* counts, gace_probe_info* info, gace_transfer_stats* stats,
                                        void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GACE_HOST_H */
