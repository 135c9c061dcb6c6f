// noalloc.hip -- gace_probe_selectivity_noalloc: the plain selectivity probe
// (Sec. III-B, Eq. 2) with its device scratch in a file-scope array instead of
// a context's workspace, for callers that cannot allocate device memory.
//
// The scratch holds what the context's workspace holds for one selectivity
// request: the compiled plan, the work items, the per-predicate counters,
// the sample histogram and the queue heads.  The kernels are the plain
// path's own (init + scan); only the buffers differ.  Every process keeps
// one copy of the array per GPU it runs on until it ends; all calls on one
// GPU share that copy, so calls that overlap on one GPU race.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "runtime.h"

namespace gace {
namespace {

constexpr uint64_t kNaPlanCap = 2ull << 20;     // compiled plan
constexpr uint64_t kNaItemsCap = 1ull << 20;    // work items (32 B each)
constexpr uint64_t kNaCountsCap = 1ull << 20;   // per-predicate counters (u64)
constexpr uint64_t kNaHistCap = 4096;           // sample histogram (u64)
constexpr uint64_t kNaMiscCap = 4096;           // queue heads, arena header
constexpr uint64_t kNaBytes = kNaPlanCap + kNaItemsCap + kNaCountsCap + kNaHistCap + kNaMiscCap;
constexpr int kNaMaxDevices = 64;
constexpr uint32_t kNaMaxHist = 64;             // histogram entries of one request: 2 x (1 + 1)

}  // namespace
}  // namespace gace

// the scratch; host code uses only the per-device address that
// hipGetSymbolAddress returns for it, never this name
static __device__ __align__(256) uint8_t scratch[gace::kNaBytes];

namespace gace {
namespace {

struct DevScratch {
    uint8_t* ptr = nullptr;   // device address of this GPU's copy of the scratch
    int n_cu = 0;
};

std::mutex g_na_mu;
DevScratch g_na_dev[kNaMaxDevices];
thread_local CompiledBatch t_na_cb;   // host plan buffers, reused call after call

gace_status na_fail(hipError_t e, const char* what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return GACE_EDEVICE;
}

// the scratch address and CU count of the current device, looked up on the
// first call made on that device
gace_status na_setup(int dev, DevScratch& out) {
    std::lock_guard<std::mutex> lk(g_na_mu);
    DevScratch& d = g_na_dev[dev];
    if (!d.ptr) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return na_fail(e, "scratch symbol address");
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess || cus <= 0) return na_fail(e, "device attribute");
        d.n_cu = cus;
        d.ptr = (uint8_t*)p;
    }
    out = d;
    return GACE_OK;
}

gace_status too_big(const char* what, uint64_t need, uint64_t cap) {
    set_error(std::string("static scratch region for ") + what + " too small: need " + std::to_string(need) +
              " bytes, have " + std::to_string(cap));
    return GACE_ENOMEM;
}

}  // namespace
}  // namespace gace

#define NA_TRY(expr, what)                                     \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return gace::na_fail(e_, what);  \
    } while (0)

extern "C" gace_status gace_probe_selectivity_noalloc(const gace_table* table, const gace_predicates* preds,
                                                      const gace_sample_spec* spec, uint64_t* counts,
                                                      gace_probe_info* info, void* stream) {
    using namespace gace;
    if (!table || !preds) {
        set_error("table and predicates must not be NULL");
        return GACE_EINVAL;
    }
    gace_request r;
    std::memset(&r, 0, sizeof(r));
    r.kind = GACE_REQ_SELECTIVITY;
    r.table = *table;
    r.preds = *preds;
    if (spec) {
        r.spec = *spec;
    } else {
        r.spec.rate = 1.0;
        r.spec.block_rows = 4096;
    }
    r.counts = counts;
    r.info = info;

    int dev = 0;
    NA_TRY(hipGetDevice(&dev), "current device");
    if (dev < 0 || dev >= kNaMaxDevices) {
        set_error("device ordinal beyond the static scratch table");
        return GACE_EINVAL;
    }
    DevScratch d;
    if (gace_status s = na_setup(dev, d)) return s;

    const gace_schedule sc = default_schedule();
    CompileOptions opt;
    opt.item_rows = sc.item_rows;
    opt.join_part_keys = sc.join_part_keys;
    opt.workers = (uint32_t)d.n_cu * sc.wgs_per_cu;
    CompiledBatch& cb = t_na_cb;
    compile_batch(&r, 1, opt, cb);
    if (cb.status[0] != GACE_OK) {
        set_error(cb.errors[0]);
        return cb.status[0];
    }
    const uint64_t plan_b = cb.plan.size(), items_b = cb.items.size() * sizeof(Item);
    if (plan_b > kNaPlanCap) return too_big("the plan", plan_b, kNaPlanCap);
    if (items_b > kNaItemsCap) return too_big("work items", items_b, kNaItemsCap);
    if (cb.n_counts * 8ull > kNaCountsCap) return too_big("counts", cb.n_counts * 8ull, kNaCountsCap);
    if (cb.n_hist > kNaMaxHist || cb.n_hist * 8ull > kNaHistCap)
        return too_big("the sample histogram", cb.n_hist * 8ull, kNaMaxHist * 8ull);
    ((PlanHdr*)cb.plan.data())->trace = 0;
    // sparse scans' spill list: the item region after the items
    ((PlanHdr*)cb.plan.data())->spill_cap =
        ((PlanHdr*)cb.plan.data())->has_spill
            ? (uint32_t)std::min<uint64_t>(kSpillMax, (kNaItemsCap - items_b) / sizeof(Item))
            : 0u;

    uint8_t* plan = d.ptr;
    uint8_t* items = plan + kNaPlanCap;
    uint8_t* cnt = items + kNaItemsCap;
    uint8_t* hist = cnt + kNaCountsCap;
    uint8_t* misc = hist + kNaHistCap;
    uint32_t* head = (uint32_t*)misc;              // three queue heads
    Arena* arena = (Arena*)(misc + 256);           // unused by scans; the init kernel resets it

    hipStream_t st = (hipStream_t)stream;
    NA_TRY(hipMemcpyAsync(plan, cb.plan.data(), plan_b, hipMemcpyHostToDevice, st), "plan upload");
    if (items_b) NA_TRY(hipMemcpyAsync(items, cb.items.data(), items_b, hipMemcpyHostToDevice, st), "item upload");
    // the init kernel zeroes the counters, the histogram and the queue heads
    NA_TRY(gace_launch_init(plan, nullptr, 0, items, head, cnt, hist, misc + 512, arena, st), "init kernel");
    BatchArgsHost a;
    std::memset(&a, 0, sizeof(a));
    a.plan = plan;
    a.items = (const Item*)items;
    a.head = head;
    a.counts = (unsigned long long*)cnt;
    a.hist = (unsigned long long*)hist;
    a.accs = (JoinAcc*)(misc + 512);
    a.arena = arena;
    a.count_mode = sc.count_mode;
    a.spin_limit = 1ull << 24;
    // spilling scans run one workgroup per CU (as in the context path)
    const PlanHdr* hp = (const PlanHdr*)cb.plan.data();
    const uint32_t per_cu = hp->has_spill && hp->spill_cap ? 1u : sc.wgs_per_cu;
    NA_TRY(gace_launch_scan(&a, (uint32_t)d.n_cu * per_cu, st), "scan kernel");

    const SelOut& so = cb.sel[0];
    const ScanDesc& S = cb.scans[so.scan];
    uint64_t h[kNaMaxHist];
    if (so.n_preds)
        NA_TRY(hipMemcpyAsync(counts, cnt + 8ull * so.count_off, 8ull * so.n_preds, hipMemcpyDeviceToHost, st),
               "counts download");
    if (cb.n_hist) NA_TRY(hipMemcpyAsync(h, hist, 8ull * cb.n_hist, hipMemcpyDeviceToHost, st), "hist download");
    NA_TRY(hipStreamSynchronize(st), "synchronize");
    if (h[cb.err_off]) {
        set_error("a scan workgroup's wait for spilled blocks gave up before the probe's items finished");
        return GACE_EDEVICE;
    }
    if (info) {
        uint64_t rows = 0, blocks = 0;
        for (uint32_t k = so.rank + 1; k <= S.n_req; ++k) {
            rows += h[S.hist_off + 2 * k];
            blocks += h[S.hist_off + 2 * k + 1];
        }
        info->sampled_rows = rows;
        info->kept_blocks = blocks;
    }
    return GACE_OK;
}
