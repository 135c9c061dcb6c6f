// plan.h -- device-visible layout of a compiled probe batch.
//
// The host compiler (compile.cpp) turns selectivity requests into "scans"
// (one pass over the kept blocks of one table under one sampler, shared by
// every request on that table, seed and block size), each scan's predicates
// into 64-bit "groups", and each group's conditions into per-column interval
// programs (value -> interval index -> 64-bit predicate mask).  Join requests
// become join descriptors.  The plan is one device buffer addressed by byte
// offsets from its base, uploaded with a single copy.
#pragma once
#include <stdint.h>

namespace gace {

constexpr uint32_t kMaxTermsPerPred = 16;
constexpr uint32_t kMaxInVals = 8;
constexpr uint32_t kMaxPredsPerReq = 65536;
constexpr uint64_t kThrAll = 1ull << 32;               // threshold meaning "keep every block"
constexpr uint32_t kLutMaxEntries = 2048;              // LUT programs up to this many entries
constexpr uint32_t kGroupTabBudget = 40u << 10;        // group tables staged in LDS up to this size
constexpr uint64_t kEmptyKey = 0x8000000000000000ull;  // sentinel key (INT64_MIN), counted out of band
// Partition buffers and aggregation tables hold the 64-bit MurmurHash3
// finalizer of each key instead of the key: the finalizer is a bijection, so
// equal hashes mean equal keys.  The sentinel key's hash marks empty slots
// (no partitioned entry can carry it).
constexpr uint64_t kEmptyHash = 0x8f780810af31a493ull;
constexpr uint32_t kPartBitsMax = 13;                  // at most 8192 hash partitions per join
constexpr uint32_t kAggSlots = 4096;                   // LDS key-table slots of one aggregation pass, at most
constexpr uint32_t kAggMinSlots = 256;                 // ... and at least (a unit sizes its table to its keys)
constexpr uint32_t kChunkKeys = 1u << 17;              // a partition with more keys is split into chunks + merge
constexpr uint32_t kTileKeys = 4096;                   // keys staged in LDS per partitioning tile
constexpr uint32_t kPass1BitsMax = 7;                  // first-pass fan-out at most 128 buckets
// a fan-out of 2^b partitions is split into 2^(b - b/2) first-pass buckets
// of 2^(b/2) partitions; both passes partition at most 128 ways
static_assert(kPartBitsMax - kPartBitsMax / 2 <= kPass1BitsMax && kPartBitsMax / 2 <= 7,
              "partition passes wider than 128 ways");
constexpr uint32_t kUnit2Keys = 1u << 17;              // target keys per second-pass unit
// heavy hitters: keys whose hash holds a slot of a join's direct-mapped
// table (slot = low hash bits) are counted per slot and never partitioned;
// the table is filled from kHeavySample keys of each side, with the hashes
// seen at least kHeavyMin times there
constexpr uint32_t kHeavySlots = 1024;
constexpr uint32_t kHeavySample = 4096;
constexpr uint32_t kHeavyCount = 2048;                 // LDS counting-table slots for one side's sample
constexpr uint32_t kHeavyMin = 2;

// column program kinds
enum : uint32_t { CP_LUT32 = 1, CP_RANK32 = 2, CP_RANK64 = 3 };
// value -> order-preserving unsigned key transforms
enum : uint32_t { XF_I32 = 1, XF_F32 = 2, XF_I64 = 3 };

struct PlanHdr {
    uint32_t n_scans, n_groups, n_cols, n_joins;
    uint32_t scans_off, groups_off, cols_off, slots_off;   // byte offsets from the plan base
    uint32_t reqthr_off, reqcum_off, joins_off, total_bytes;
    uint32_t n_counts, n_hist, n_items, n_scan_items;   // items [0, n_scan_items) are scans
    uint64_t arena_static;   // bytes of the arena holding the joins' per-item tables
    uint32_t trace;          // nonzero: kernels write one TraceRec per item
    uint32_t n_join_end;     // items [n_scan_items, n_join_end) are join partitioning items, the rest aggregation
    uint32_t early;          // nonzero: the scans and each join publish their results to the host when done
    uint32_t seq;            // ... raising their host flags to this batch number
    uint32_t wg_done_off;    // hist entry counting the scan kernel's finished workgroups
    uint32_t items_off;      // byte offset of the work items in the plan buffer (0: in their own region)
    uint32_t has_spill;      // some scan passes kept blocks beyond an item's first to the spill list
    uint32_t spill_cap;      // spill-list entries available after the items (0: no list, blocks stay local)
    uint32_t err_off;        // hist entry counting scan-kernel waits that gave up (nonzero fails the scans)
    uint32_t reserved;
};

// Sparse scans in a small batch: an item scans the first kept block of its
// 64-block chunk and appends the chunk's other kept blocks to a spill list in
// the item region, after the items (an Item each: kind, scan index, the
// block's predicate bits in `side`, block range; `sub` becomes 1 once the
// entry is written).  Workgroups that find the item queue empty run the
// list, so a probe's kept tiles spread one per workgroup instead of queueing
// behind each other inside one item.
constexpr uint64_t kInitCopyMax = 64ull << 10;        // plans up to this size are copied by the init kernel
constexpr uint32_t kSpillMax = 16384;                  // spill-list entries per batch, at most
constexpr uint32_t kSpillChunkKept = 8;                // spill when at most this many kept blocks per 64 expected
constexpr uint64_t kSpillPolls = 1ull << 26;           // a drain wait gives up after this many polls

// Per-request completion.  When a plan asks for it, the last workgroup of
// the scan kernel to finish copies all counters and sample histograms, and
// the last aggregation worker of a join copies its JoinAcc, into the
// context's pinned result buffer (the layout of the end-of-batch download:
// counters at 0, histogram at kHostHistOff, accumulators at kHostAccsOff),
// then stores the batch number into host flag 0 (every selectivity request)
// or 1 + j (join j).  One release fence per workgroup orders the counter
// atomics before its exit count; a fence per item would write back and
// invalidate the L2 hundreds of times per probe.
constexpr uint64_t kHostHistOff = 8ull << 20;
constexpr uint64_t kHostAccsOff = 12ull << 20;
constexpr uint32_t kMaxFlags = 1u << 16;

// per-item trace record (same layout as gace_trace_rec)
struct TraceRec {
    uint32_t kind, index, wg, xcc;
    uint64_t t_begin, t_ready, t_end;   // steady-counter ticks: popped, dependencies met, done
    uint64_t work;                      // item-specific: aggregation units << 32 | table passes
};

// one shared pass over one table's kept blocks
struct ScanDesc {
    uint64_t n_rows;
    uint64_t seed;
    uint64_t thr_max;        // largest threshold among the scan's requests
    uint64_t n_blocks;
    uint32_t table_id, log2B;
    uint32_t group_begin, n_groups;
    uint32_t req_begin, n_req;    // thresholds sorted descending (reqthr) and bit prefix sums (reqcum)
    uint32_t hist_off;            // (n_req + 1) x 2 u64: rows, blocks by number of active requests
    uint32_t row_bytes;           // bytes per row over the referenced columns
    uint64_t zskip;               // device address of a zone-skip bit map (bit z set: no predicate of the
                                  // scan can hold on zone z, kZoneRows rows); 0: no zone map
    uint64_t n_zones;
    uint32_t fine;                // blocks under 4096 rows decided row by row in whole tiles (items tile-aligned)
    uint32_t spill;               // items are 64-block chunks whose kept blocks beyond the first are spilled
};

constexpr uint32_t kZoneLog2 = 12;                     // zone-map zones of 4096 rows
constexpr uint64_t kZoneRows = 1ull << kZoneLog2;

// 64 predicate bits of one scan (bits are in request order, requests sorted by
// threshold descending, so the bits active on a block are a prefix)
struct GroupDesc {
    uint64_t base_mask;      // bits whose constant-folded conditions can hold; unused bits 0
    uint32_t col_begin, col_end;
    uint32_t slot_index;     // counts slot of bit i is slots[slot_index + i]
    uint32_t tab_off;        // byte offset of the group's table region in the plan
    uint32_t tab_bytes;      // size of that region (staged into LDS when <= kGroupTabBudget)
    uint32_t n_used;         // used bit positions (1..64)
};

// one referenced column of a group: value -> interval index -> 64-bit mask
struct ColProg {
    const void* data;        // device column base
    uint32_t kind;           // CP_*
    uint32_t xform;          // XF_*
    uint32_t lo, hi;         // LUT32: clamp range of the 32-bit key (index = clamp(key) - lo)
    uint32_t nb;             // RANK: number of boundaries
    uint32_t step;           // RANK: largest power of two <= nb
    uint32_t mask_off;       // byte offset of the masks inside the group's table region
    uint32_t bnd_off;        // RANK: byte offset of the sorted boundaries inside the region
};

struct JoinSide {
    const int64_t* keys;
    uint64_t n;
    uint64_t seed;
    uint64_t thr;
    uint64_t n_blocks;
    uint32_t table_id, log2B;
    uint32_t item_begin, n_items;   // this side's rows in the join's per-item tables
};

struct JoinDesc {
    JoinSide side[2];        // 0 = R, 1 = S
    uint32_t acc;            // index of this join's JoinAcc
    uint32_t log2P;          // hash partitions: P = 2^log2P (top bits of the key hash)
    uint32_t n_items;        // histogram / first-pass scatter items (R then S)
    uint32_t n_off;          // offset items (64 partitions each)
    uint32_t n_agg;          // aggregation workers
    uint32_t log2P2;         // second-pass fan-out bits (0: one pass writes the final partitions)
    uint32_t group_items;    // second pass: items of one side per unit
    uint32_t n_groups[2];    // second pass: item groups per side
    uint32_t n_units2;       // second-pass units: (side, item group, first-pass bucket)
    uint32_t n_s2;           // second-pass workers
    uint64_t rows_off;       // arena offset: per-item partition counts, then offsets, [n_items][P] u32
    uint64_t base_off;       // arena offset: [2][P + 1] u32 partition starts per side
    uint64_t stats_off;      // arena offset: per item {sampled keys, sentinel keys} u64
    uint64_t units_off;      // arena offset: aggregation units (AggUnit), capacity max_units
    uint64_t chunk_off;      // arena offset: per chunk slot, u32 entries emitted
    uint64_t done_off;       // arena offset: per split partition, u32 finished chunks
    uint64_t heavy_off;      // arena offset: [kHeavySlots] u64 heavy hashes, then [2][kHeavySlots] u32 counts
    uint32_t max_units, max_chunks;
};

// aggregation work unit: a whole partition, one chunk of a split partition, or
// the merge of a split partition's chunk tables
enum : uint32_t { AU_SMALL = 0, AU_CHUNK = 1, AU_MERGE = 2 };
struct AggUnit {
    uint32_t part;
    uint32_t kind;
    uint32_t a;              // CHUNK: chunk index in the partition; MERGE: first chunk slot
    uint32_t b;              // CHUNK: chunk slot; MERGE: number of chunks
    uint32_t ord;            // CHUNK / MERGE: split-partition ordinal (done counter)
    uint32_t reserved[3];
};

// entry of a chunk table handed to the merge
struct MergeEntry {
    uint64_t key;            // the key's hash
    uint32_t c0, c1;
};

// per-join device accumulators and phase counters (zeroed before each batch)
struct JoinAcc {
    unsigned long long join, ndv[2], n[2], sent[2];
    unsigned long long buf_off;             // arena offset of the partitioned keys (R then S)
    unsigned long long nkeys[2];            // sampled keys per side other than the sentinel value
    unsigned long long status;              // 0 ok, 2 arena exhausted, 3 aggregation stack overflow, 4 a wait gave up
    unsigned long long merge_off;           // arena offset of the chunk tables (kChunkKeys entries per slot)
    unsigned long long tmp_off;             // arena offset of the first-pass buffer (two-pass partitioning)
    uint32_t next_unit, n_units;
    uint32_t hist_done, off_done, base_done, scatter_done, agg_done, s2_done;
    uint32_t next_s2, heavy_done;
    unsigned long long f1[2], f2[2];        // distinct keys seen exactly once / twice per side
};

static_assert(sizeof(JoinAcc) % 8 == 0, "JoinAcc is published to the host as 64-bit words");

struct Arena {                              // bump allocator for partition buffers
    unsigned long long used, size;
};

// work item of the persistent batch kernel
enum : uint32_t {
    IT_SCAN = 1, IT_JHIST = 2, IT_JOFF = 3, IT_JBASE = 4, IT_JSCATTER = 5, IT_JAGG = 6, IT_JSCATTER2 = 7, IT_JHEAVY = 8
};
struct Item {
    uint32_t kind;
    uint32_t idx;            // scan or join index
    uint32_t side;           // JHIST / JSCATTER: 0 = R, 1 = S
    uint32_t sub;            // JHIST / JSCATTER: item row; JOFF: 64-partition chunk; JAGG: worker
    uint64_t begin, end;     // block range (SCAN, JHIST, JSCATTER)
};

}  // namespace gace
