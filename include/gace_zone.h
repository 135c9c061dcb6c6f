/*
 * gace_zone.h -- block-level summaries (zone maps) of a device-resident table
 * and selectivity probes that use them to skip work (the "block-level
 * summaries" the Measurement Engine may use, Sec. III-B).
 *
 * A zone map holds, for every column and every zone of 4096 consecutive rows,
 * the smallest and the largest value (float32: of the non-NaN values; a zone
 * of NaNs only holds min = +inf, max = -inf and no condition can hold on it).
 * A probe with a zone map first marks, with one device pass over the zones,
 * those on which no candidate condition can hold: for every predicate some
 * term's interval misses the zone's [min, max] of its column.  Kept blocks
 * that lie entirely in such zones are still sampled (they count in
 * sampled_rows and kept_blocks) but are not read.  The counts are exactly
 * those of gace_probe_selectivity.
 *
 * Ownership: the zone map owns its device memory (2 values per column and
 * zone) until gace_zonemap_destroy.  It describes the table's data at build
 * time: the caller rebuilds it after changing the data.  A probe checks that
 * the table has the zone map's row count and column addresses and types
 * (GACE_EINVAL otherwise).  Validation and errors of the probe are those of
 * gace_probe_selectivity; the probe uses the context's workspace (calls on one
 * context must not overlap).
 */
#ifndef GACE_ZONE_H
#define GACE_ZONE_H

#include "gace.h"

#ifdef __cplusplus
extern "C" {
#endif

#define GACE_ZONE_ROWS 4096u

typedef struct gace_zonemap gace_zonemap;

/* One device pass over every column of `table` (validated as a selectivity
   table: known dtypes, 16-byte aligned columns). */
gace_status gace_zonemap_build(gace_ctx* ctx, const gace_table* table, gace_zonemap** out, void* stream);
gace_status gace_zonemap_destroy(gace_zonemap* zm);
/* Number of zones (ceil(n_rows / 4096)). */
gace_status gace_zonemap_info(const gace_zonemap* zm, uint64_t* n_zones);
/* Copy column col's per-zone minima and maxima into host arrays of n_zones
   values of the column's type (int32, int64 or float32). */
gace_status gace_zonemap_read(const gace_zonemap* zm, uint32_t col, void* zmin, void* zmax);

/* gace_probe_selectivity with zone pruning.  zones_skipped (may be NULL)
   receives the number of zones on which no predicate can hold. */
gace_status gace_probe_selectivity_zm(gace_ctx* ctx, const gace_table* table, const gace_zonemap* zm,
                                      const gace_predicates* preds, const gace_sample_spec* spec, uint64_t* counts,
                                      gace_probe_info* info, uint64_t* zones_skipped, void* stream);

/* Batched and served scans.  A zone map attached to a context is used by
   every later gace_batch_run and gace_probe_selectivity on that context
   whose table it matches (same row count, column addresses and types); one
   attached to a server, by every later batch the server launches.  A shared
   scan skips a zone only when no predicate of any request sharing the scan
   can hold there, so every count equals the unpruned one.  The zone data
   (skip bitmap and the scan's predicates, a few bytes per zone and 80 per
   term) takes arena space after the batch's join tables; a batch where it
   does not fit runs unpruned.  The zone map must stay alive while attached
   (detach before gace_zonemap_destroy); attaching it again is a no-op.
   gace_kernel_stats.zones_skipped reports the zones the last batch skipped.
   Errors: GACE_EINVAL (NULL argument, zone map of another device, detach of
   a map that is not attached). */
gace_status gace_zonemap_attach(gace_ctx* ctx, const gace_zonemap* zm);
gace_status gace_zonemap_detach(gace_ctx* ctx, const gace_zonemap* zm);
gace_status gace_server_attach_zonemap(gace_server* srv, const gace_zonemap* zm);

#ifdef __cplusplus
}
#endif

#endif /* GACE_ZONE_H */
