// runtime.h -- the context behind gace_ctx (host side).
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/gace.h"
#include "compile.h"

namespace gace {

void set_error(const std::string& msg);

// fixed regions carved from the device workspace
constexpr uint64_t kPlanCap = 16ull << 20;
constexpr uint64_t kItemsCap = 8ull << 20;
constexpr uint64_t kCountsCap = 8ull << 20;
constexpr uint64_t kHistCap = 4ull << 20;
constexpr uint64_t kAccsCap = 1ull << 20;
constexpr uint64_t kMiscCap = 4096;
constexpr uint64_t kTraceCap = (kItemsCap / sizeof(Item)) * sizeof(TraceRec);
constexpr uint64_t kFixedBytes = kPlanCap + kItemsCap + kCountsCap + kHistCap + kAccsCap + kMiscCap + kTraceCap;

// kernel argument block (must match kernels.hip)
struct BatchArgsHost {
    const uint8_t* plan;
    const Item* items;
    uint32_t* head;
    unsigned long long* counts;
    unsigned long long* hist;
    JoinAcc* accs;
    uint8_t* arena_base;
    Arena* arena;
    uint32_t count_mode;
    uint32_t agg_slots;
    TraceRec* trace;
    uint64_t spin_limit;
    uint8_t* host_res;
    uint32_t* host_flags;
};

static_assert(kHostHistOff == kCountsCap && kHostAccsOff == kCountsCap + kHistCap,
              "the kernels publish results in the layout of the pinned result buffer");

gace_schedule default_schedule();

}  // namespace gace

// kernel launchers (kernels.hip; internal, not part of the public ABI)
extern "C" {
hipError_t gace_launch_init(const void* plan, const void* src, uint64_t src_bytes, void* items, void* head, void* counts,
                            void* hist, void* accs, void* arena,
                            hipStream_t stream);
hipError_t gace_launch_scan(const void* args, uint32_t grid, hipStream_t stream);
hipError_t gace_launch_join(const void* args, uint32_t grid, int beside_scan, hipStream_t stream);
hipError_t gace_launch_agg(const void* args, uint32_t grid, hipStream_t stream);
hipError_t gace_launch_read(const void* p, uint64_t n16, void* sink, hipStream_t stream);
const void* gace_kernel_handle(int which);
hipError_t gace_launch_publish(const void* plan, const void* counts, const void* hist, const void* accs,
                               void* host_res, uint32_t grid, hipStream_t stream);
}


using gace::TraceRec;

struct gace_zonemap;

struct gace_ctx {
    int device = 0;
    int n_cu = 0;
    uint8_t* ws = nullptr;
    uint64_t ws_bytes = 0;
    // device regions
    uint8_t* d_plan = nullptr;
    gace::Item* d_items = nullptr;
    unsigned long long* d_counts = nullptr;
    unsigned long long* d_hist = nullptr;
    gace::JoinAcc* d_accs = nullptr;
    uint32_t* d_head = nullptr;
    TraceRec* d_trace = nullptr;
    gace::Arena* d_arena = nullptr;
    uint8_t* d_arena_base = nullptr;
    uint64_t arena_bytes = 0;
    // pinned host staging
    uint8_t* h_stage = nullptr;     // plan + items upload
    const uint8_t* d_stage = nullptr;   // device address of h_stage (small plans: the init kernel copies them)
    uint64_t stage_copy = 0;        // bytes of h_stage the next init kernel copies to the plan region
    uint8_t* h_result = nullptr;    // counts + hist + accs download
    // per-request completion: kernels write finished scans' and joins'
    // results into h_result and raise their flags (device addresses of both)
    uint32_t* h_flags = nullptr;
    uint8_t* d_host_res = nullptr;
    uint32_t* d_host_flags = nullptr;
    bool early = false;             // ask the kernels to publish per scan / join (servers do)
    uint32_t seq = 0;               // batch number of the last launch
    bool last_early = false;        // the last launch publishes per scan / join
    // zone maps attached for batched scans (not owned), and the last batch's
    // skipped-zone counters (pinned, one per pruned scan)
    std::vector<const gace_zonemap*> zonemaps;
    const uint64_t* zm_counts = nullptr;
    uint32_t zm_n_last = 0;
    uint64_t last_zones_skipped = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_done = nullptr, ev_fork = nullptr, ev_join = nullptr;
    // per-kernel timing of direct launches: scan kernel on the call's stream, join kernel on the side stream
    hipEvent_t ev_s0 = nullptr, ev_s1 = nullptr, ev_j0 = nullptr, ev_j1 = nullptr;
    bool use_graph = true;                        // batched path: replay the captured graph
    hipStream_t side_stream = nullptr;   // join kernel runs here, concurrently with the scan kernel
    gace_schedule sched{};
    // captured graphs of the batch branches for the current schedule: scan
    // kernel (0, or 1 beside the joins), join stage (2, or 3 beside a scan)
    hipGraphExec_t graph_exec[8] = {};
    hipGraph_t graph[8] = {};
    gace_schedule graph_sched[8] = {};
    hipStream_t cap_stream = nullptr;             // stream the branch graphs are captured on
    // stats of the last batch
    double last_kernel_ms = 0.0;
    uint64_t last_alg_bytes = 0, last_rows_preds = 0;
    bool last_timed = false;                      // last batch ran by direct launch with per-kernel events
    double last_scan_ms = 0.0, last_join_ms = 0.0;
    double last_compile_ms = 0.0;                 // host validation + compilation of the last batch
    gace::CompiledBatch cb;                       // the last batch's plan (buffers reused batch after batch)
    uint64_t last_scan_bytes = 0, last_join_bytes = 0;
    std::map<std::string, gace_schedule> tuned;   // shape bucket -> schedule
    // host-resident tables: copy stream, per-slot copy events, pinned staging
    hipStream_t copy_stream = nullptr;
    hipEvent_t ev_h0[2] = {nullptr, nullptr}, ev_h1[2] = {nullptr, nullptr}, ev_d2h = nullptr;
    uint8_t* h_hp = nullptr;
    uint64_t h_hp_bytes = 0;
    uint64_t spin_limit = 1ull << 24;             // polls before a join phase wait on the device gives up
    bool trace = false;                           // record per-item device timestamps
    std::vector<TraceRec> last_trace;
    double ticks_per_us = 0.0;
};

namespace gace {

// compile + run a request array on ctx.  use_graph selects graph replay
// (batched path) over direct launches (plain path).
gace_status run_requests(gace_ctx* c, const gace_request* reqs, uint32_t n, gace_status* per_req, hipStream_t st,
                         bool use_graph);

std::string shape_bucket(const gace_request* reqs, uint32_t n);

gace_status launch_compiled(gace_ctx* c, CompiledBatch& cb, hipStream_t st, bool use_graph);
gace_status finish_compiled(gace_ctx* c, CompiledBatch& cb, const gace_request* reqs, gace_status* per_req,
                            const std::vector<char>* done = nullptr);
// Per-request completion (contexts with `early` set): writes the outputs of
// each request of the running batch whose scan or join has published its
// results and is not marked in `done` yet, marks it, and appends (request
// index, status) to `out`.
void collect_published(gace_ctx* c, CompiledBatch& cb, const gace_request* reqs, std::vector<char>& done,
                       std::vector<std::pair<uint32_t, gace_status>>& out);
// Zone pruning of a compiled batch's scans by the zone maps attached to c
// (queued on st before the batch); and the zones the last batch skipped.
gace_status apply_zonemaps(gace_ctx* c, CompiledBatch& cb, const gace_request* reqs, hipStream_t st);
uint64_t zones_skipped_last(const gace_ctx* c);
int zonemap_device(const gace_zonemap* zm);
gace_status run_compiled(gace_ctx* c, CompiledBatch& cb, const gace_request* reqs, gace_status* per_req,
                         hipStream_t st, bool use_graph);

}  // namespace gace
