// compile.h -- host-side validation and compilation of probe requests into a
// device plan (see plan.h).  No HIP calls: usable without a GPU.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/gace.h"
#include "plan.h"

namespace gace {

uint64_t rate_threshold(double rate);

gace_status check_spec(const gace_sample_spec* s, std::string& msg);
gace_status check_selectivity(const gace_table* t, const gace_predicates* p, const gace_sample_spec* s,
                              std::string& msg);
gace_status check_join(const gace_keys* R, const gace_keys* S, std::string& msg);
gace_status check_request(const gace_request* r, std::string& msg);

struct CompileOptions {
    uint32_t item_rows = 65536;      // target sampled rows per work item
    uint32_t join_part_keys = 1024;  // expected sampled keys per join hash partition
    uint32_t workers = 0;            // scan workgroups of the launch (0: items of item_rows regardless)
};

// host bookkeeping that maps plan results back to the requests
struct SelOut {
    uint32_t req;                    // index in the caller's request array
    uint32_t scan;
    uint32_t rank;                   // position among the scan's requests (threshold descending)
    uint32_t count_off;
    uint32_t n_preds;
};

struct JoinOut {
    uint32_t req;
    uint32_t join;                   // index of the JoinDesc / JoinAcc
};

struct CompiledBatch {
    std::vector<uint8_t> plan;       // PlanHdr + descriptors + tables
    std::vector<Item> items;
    std::vector<SelOut> sel;
    std::vector<JoinOut> joins;
    std::vector<ScanDesc> scans;     // host copies
    std::vector<JoinDesc> jdesc;
    std::vector<gace_status> status; // per caller request (validation result)
    std::vector<std::string> errors;
    uint32_t n_counts = 0, n_hist = 0;
    uint32_t err_off = 0;            // hist entry counting the scan kernel's waits that gave up
    uint64_t arena_static = 0;       // joins' per-item tables at the start of the arena
    double est_scan_bytes = 0.0;     // expected bytes the scans read (sum of the items' costs)
    double est_join_keys = 0.0;      // expected sampled keys of the joins
};

// Validate every request; compile the valid ones.  Never throws.
void compile_batch(const gace_request* reqs, uint32_t n, const CompileOptions& opt, CompiledBatch& out);

}  // namespace gace
