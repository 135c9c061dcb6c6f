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
constexpr uint64_t kEmptyKey = 0x8000000000000000ull;  // hash-table sentinel (INT64_MIN), counted out of band
constexpr uint32_t kHllBits = 12;                      // 4096 HyperLogLog registers (table sizing only)
constexpr uint32_t kSketchRowsPerJoin = 64;            // max sketch items per join
constexpr uint32_t kSlotChunks = 64;                   // init / final items per join

// column program kinds
enum : uint32_t { CP_LUT32 = 1, CP_RANK32 = 2, CP_RANK64 = 3 };
// value -> order-preserving unsigned key transforms
enum : uint32_t { XF_I32 = 1, XF_F32 = 2, XF_I64 = 3 };

struct PlanHdr {
    uint32_t n_scans, n_groups, n_cols, n_joins;
    uint32_t scans_off, groups_off, cols_off, slots_off;   // byte offsets from the plan base
    uint32_t reqthr_off, reqcum_off, joins_off, total_bytes;
    uint32_t n_counts, n_hist, n_items, reserved;
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
};

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
};

struct JoinDesc {
    JoinSide side[2];        // 0 = R, 1 = S
    uint64_t cap_max;        // slot cap the sampled-key bound allows (power of two)
    uint32_t acc;            // index of this join's JoinAcc
    uint32_t n_sketch, n_build, reserved;
    uint64_t sketch_off;     // byte offset of n_sketch x 4096 u8 HLL rows in the join workspace
};

// hash-table slot: key + per-side counts
struct Slot {
    uint64_t key;
    uint32_t cnt[2];
};

// per-join device accumulators and phase counters (zeroed before each batch)
struct JoinAcc {
    unsigned long long join, ndv[2], n[2], sent[2];
    unsigned long long table_off, cap;      // chosen after the sketch phase
    unsigned long long status;              // 0 ok, 1 table full (rerun), 2 arena exhausted
    uint32_t sketch_done, size_done, init_done, build_done;
    uint32_t final_done, reserved[3];
};

struct Arena {                              // bump allocator for hash tables
    unsigned long long used, size;
};

// work item of the persistent batch kernel
enum : uint32_t { IT_SCAN = 1, IT_JSKETCH = 2, IT_JSIZE = 3, IT_JINIT = 4, IT_JBUILD = 5, IT_JFINAL = 6 };
struct Item {
    uint32_t kind;
    uint32_t idx;            // scan or join index
    uint32_t side;           // JSKETCH / JBUILD: 0 = R, 1 = S
    uint32_t sub;            // JSKETCH: sketch row; JINIT / JFINAL: chunk
    uint64_t begin, end;     // block range (SCAN, JSKETCH, JBUILD)
};

}  // namespace gace
