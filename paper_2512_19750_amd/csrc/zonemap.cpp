// zonemap.cpp -- zone maps (per-zone min / max of every column) and the
// selectivity probe that skips zones on which no predicate can hold.
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gace_zone.h"
#include "compile.h"
#include "runtime.h"

extern "C" {
hipError_t gace_launch_zone_build(const void* col, uint32_t dtype, uint64_t n_rows, void* zmin, void* zmax,
                                  hipStream_t stream);
hipError_t gace_launch_zone_prune(const void* zc, const void* terms, const uint32_t* pred_off, uint32_t n_preds,
                                  uint64_t n_zones, uint32_t* skip, void* n_skip, hipStream_t stream);
}

using gace::set_error;

struct gace_zonemap {
    int device = 0;
    uint64_t n_rows = 0, n_zones = 0;
    uint32_t n_cols = 0;
    std::vector<const void*> data;     // the columns it describes
    std::vector<uint32_t> dtype;
    uint8_t* d_mem = nullptr;          // per column: min[n_zones], max[n_zones]; then the ZoneCol array
    std::vector<uint64_t> off;         // byte offset of column c's minima (maxima follow)
    uint64_t zc_off = 0;
};

namespace {

// layout of the kernels' per-column record
struct ZoneColHost {
    const void* zmin;
    const void* zmax;
    uint32_t dtype;
    uint32_t reserved;
};

uint64_t width(uint32_t dtype) { return dtype == GACE_I64 ? 8 : 4; }
uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

gace_status hip_err(hipError_t e, const char* what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return GACE_EDEVICE;
}

#define ZTRY(expr, what)                               \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return hip_err(e_, what); \
    } while (0)

}  // namespace

extern "C" gace_status gace_zonemap_build(gace_ctx* ctx, const gace_table* table, gace_zonemap** out, void* stream) {
    if (!ctx || !table || !out) {
        set_error("NULL argument");
        return GACE_EINVAL;
    }
    gace_predicates none;
    std::memset(&none, 0, sizeof(none));
    gace_sample_spec sp;
    std::memset(&sp, 0, sizeof(sp));
    sp.rate = 1.0;
    sp.block_rows = 4096;
    std::string msg;
    if (gace_status st = gace::check_selectivity(table, &none, &sp, msg)) {
        set_error(msg);
        return st;
    }
    ZTRY(hipSetDevice(ctx->device), "set device");
    gace_zonemap* zm = new gace_zonemap();
    zm->device = ctx->device;
    zm->n_rows = table->n_rows;
    zm->n_zones = (table->n_rows + GACE_ZONE_ROWS - 1) / GACE_ZONE_ROWS;
    zm->n_cols = table->n_cols;
    uint64_t bytes = 0;
    std::vector<ZoneColHost> zc(table->n_cols);
    for (uint32_t c = 0; c < table->n_cols; ++c) {
        zm->data.push_back(table->cols[c].data);
        zm->dtype.push_back(table->cols[c].dtype);
        zm->off.push_back(bytes);
        bytes += 2 * align256(zm->n_zones * width(table->cols[c].dtype));
    }
    zm->zc_off = bytes;
    bytes += align256(std::max<size_t>(1, zc.size()) * sizeof(ZoneColHost));
    hipError_t e = hipMalloc((void**)&zm->d_mem, bytes);
    if (e != hipSuccess) {
        delete zm;
        set_error("zone map allocation of " + std::to_string(bytes) + " bytes failed");
        return GACE_ENOMEM;
    }
    hipStream_t st = (hipStream_t)stream;
    for (uint32_t c = 0; c < table->n_cols; ++c) {
        const uint64_t w = width(zm->dtype[c]);
        uint8_t* mn = zm->d_mem + zm->off[c];
        uint8_t* mx = mn + align256(zm->n_zones * w);
        zc[c].zmin = mn;
        zc[c].zmax = mx;
        zc[c].dtype = zm->dtype[c];
        zc[c].reserved = 0;
        e = gace_launch_zone_build(table->cols[c].data, zm->dtype[c], zm->n_rows, mn, mx, st);
        if (e != hipSuccess) {
            gace_zonemap_destroy(zm);
            return hip_err(e, "zone map kernel");
        }
    }
    if (!zc.empty()) {
        e = hipMemcpyAsync(zm->d_mem + zm->zc_off, zc.data(), zc.size() * sizeof(ZoneColHost), hipMemcpyHostToDevice,
                           st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    } else {
        e = hipStreamSynchronize(st);
    }
    if (e != hipSuccess) {
        gace_zonemap_destroy(zm);
        return hip_err(e, "zone map upload");
    }
    *out = zm;
    return GACE_OK;
}

extern "C" gace_status gace_zonemap_destroy(gace_zonemap* zm) {
    if (!zm) return GACE_OK;
    (void)hipSetDevice(zm->device);
    if (zm->d_mem) (void)hipFree(zm->d_mem);
    delete zm;
    return GACE_OK;
}

extern "C" gace_status gace_zonemap_info(const gace_zonemap* zm, uint64_t* n_zones) {
    if (!zm || !n_zones) {
        set_error("NULL argument");
        return GACE_EINVAL;
    }
    *n_zones = zm->n_zones;
    return GACE_OK;
}

extern "C" gace_status gace_zonemap_read(const gace_zonemap* zm, uint32_t col, void* zmin, void* zmax) {
    if (!zm || col >= zm->n_cols || (zm->n_zones && (!zmin || !zmax))) {
        set_error("zone map read needs a zone map, a column index in range and two host arrays");
        return GACE_EINVAL;
    }
    ZTRY(hipSetDevice(zm->device), "set device");
    const uint64_t b = zm->n_zones * width(zm->dtype[col]);
    const uint8_t* mn = zm->d_mem + zm->off[col];
    if (b) {
        ZTRY(hipMemcpy(zmin, mn, b, hipMemcpyDeviceToHost), "zone map download");
        ZTRY(hipMemcpy(zmax, mn + align256(b), b, hipMemcpyDeviceToHost), "zone map download");
    }
    return GACE_OK;
}

// ---------------------------------------------------------------- batches
namespace gace {

static bool zm_matches(const gace_zonemap* zm, const gace_table& t, int device) {
    if (zm->n_rows != t.n_rows || zm->n_cols != t.n_cols || zm->device != device) return false;
    for (uint32_t c = 0; c < t.n_cols; ++c)
        if (zm->data[c] != t.cols[c].data || zm->dtype[c] != t.cols[c].dtype) return false;
    return true;
}

// Zone pruning for the shared scans of a compiled batch.  For each scan on a
// table with an attached zone map, the union of every predicate of every
// request sharing the scan goes to the prune kernel, so a zone is skipped only
// when no request of the scan can match in it.  The skip bitmaps, the staged
// predicates and the skipped-zone counters sit in the arena after the joins'
// per-item tables (the batch's static arena grows by their size); the plan's
// scan descriptors get the bitmaps' addresses.  A batch whose zone data does
// not fit the arena runs unpruned, with the same counts.
gace_status apply_zonemaps(gace_ctx* c, CompiledBatch& cb, const gace_request* reqs, hipStream_t st) {
    c->zm_n_last = 0;
    if (c->zonemaps.empty() || cb.scans.empty()) return GACE_OK;
    std::vector<std::vector<uint32_t>> members(cb.scans.size());
    for (const SelOut& so : cb.sel) members[so.scan].push_back(so.req);
    struct Z {
        uint32_t scan;
        const gace_zonemap* zm;
        uint64_t skip_off, terms_off, off_off;
        uint32_t np, nt;
    };
    std::vector<Z> zs;
    for (uint32_t s = 0; s < cb.scans.size(); ++s) {
        if (members[s].empty()) continue;
        const gace_table& t = reqs[members[s][0]].table;
        for (const gace_zonemap* zm : c->zonemaps)
            if (zm_matches(zm, t, c->device)) {
                Z z{};
                z.scan = s;
                z.zm = zm;
                for (uint32_t q : members[s]) {
                    const gace_predicates& p = reqs[q].preds;
                    z.np += p.n_preds;
                    z.nt += p.n_preds ? p.pred_off[p.n_preds] : 0;
                }
                zs.push_back(z);
                break;
            }
    }
    if (zs.empty()) return GACE_OK;
    // layout: counters (one u64 per zoned scan), then per scan its bitmap, terms and offsets
    const uint64_t base = align256(cb.arena_static);
    uint64_t at = base + align256(8 * zs.size());
    for (Z& z : zs) {
        z.skip_off = at;
        at += align256((z.zm->n_zones + 31) / 32 * 4);
        z.terms_off = at;
        at += align256((uint64_t)std::max<uint32_t>(z.nt, 1) * sizeof(gace_term));
        z.off_off = at;
        at += align256(((uint64_t)z.np + 1) * 4);
    }
    if (at > c->arena_bytes) return GACE_OK;
    const uint64_t up_b = at - base, down_off = align256(up_b);
    const uint64_t h_need = down_off + 8 * zs.size();
    if (c->h_hp_bytes < h_need) {
        if (c->h_hp) (void)hipHostFree(c->h_hp);
        c->h_hp = nullptr;
        c->h_hp_bytes = 0;
        ZTRY(hipHostMalloc((void**)&c->h_hp, h_need, hipHostMallocDefault), "pinned staging");
        c->h_hp_bytes = h_need;
    }
    uint8_t* h = c->h_hp;
    std::memset(h, 0, up_b);   // zero counters; the bitmaps are written whole by the kernel
    for (Z& z : zs) {
        gace_term* T = (gace_term*)(h + (z.terms_off - base));
        uint32_t* O = (uint32_t*)(h + (z.off_off - base));
        uint32_t nt = 0, np = 0;
        O[0] = 0;
        for (uint32_t q : members[z.scan]) {
            const gace_predicates& p = reqs[q].preds;
            const uint32_t pt = p.n_preds ? p.pred_off[p.n_preds] : 0;
            if (pt) std::memcpy(T + nt, p.terms, (uint64_t)pt * sizeof(gace_term));
            for (uint32_t i = 1; i <= p.n_preds; ++i) O[np + i] = nt + p.pred_off[i];
            nt += pt;
            np += p.n_preds;
        }
    }
    ZTRY(hipMemcpyAsync(c->d_arena_base + base, h, up_b, hipMemcpyHostToDevice, st), "zone predicate upload");
    PlanHdr H;
    std::memcpy(&H, cb.plan.data(), sizeof(H));
    ScanDesc* sd = (ScanDesc*)(cb.plan.data() + H.scans_off);
    for (size_t i = 0; i < zs.size(); ++i) {
        const Z& z = zs[i];
        uint8_t* a = c->d_arena_base;
        ZTRY(gace_launch_zone_prune(z.zm->d_mem + z.zm->zc_off, a + z.terms_off, (const uint32_t*)(a + z.off_off),
                                    z.np, z.zm->n_zones, (uint32_t*)(a + z.skip_off), a + base + 8 * i, st),
             "zone prune kernel");
        sd[z.scan].zskip = (uint64_t)(uintptr_t)(a + z.skip_off);
        sd[z.scan].n_zones = z.zm->n_zones;
        cb.scans[z.scan].zskip = sd[z.scan].zskip;
        cb.scans[z.scan].n_zones = sd[z.scan].n_zones;
    }
    ZTRY(hipMemcpyAsync(h + down_off, c->d_arena_base + base, 8 * zs.size(), hipMemcpyDeviceToHost, st),
         "zone counter download");
    c->zm_counts = (const uint64_t*)(h + down_off);
    c->zm_n_last = (uint32_t)zs.size();
    cb.arena_static = at;
    H.arena_static = at;
    std::memcpy(cb.plan.data(), &H, sizeof(H));
    return GACE_OK;
}

int zonemap_device(const gace_zonemap* zm) { return zm->device; }

uint64_t zones_skipped_last(const gace_ctx* c) {
    uint64_t n = 0;
    for (uint32_t i = 0; i < c->zm_n_last; ++i) n += c->zm_counts[i];
    return n;
}

}  // namespace gace

extern "C" gace_status gace_zonemap_attach(gace_ctx* ctx, const gace_zonemap* zm) {
    if (!ctx || !zm) {
        set_error("NULL argument");
        return GACE_EINVAL;
    }
    if (zm->device != ctx->device) {
        set_error("the zone map is on another device than the context");
        return GACE_EINVAL;
    }
    for (const gace_zonemap* z : ctx->zonemaps)
        if (z == zm) return GACE_OK;
    ctx->zonemaps.push_back(zm);
    return GACE_OK;
}

extern "C" gace_status gace_zonemap_detach(gace_ctx* ctx, const gace_zonemap* zm) {
    if (!ctx || !zm) {
        set_error("NULL argument");
        return GACE_EINVAL;
    }
    for (size_t i = 0; i < ctx->zonemaps.size(); ++i)
        if (ctx->zonemaps[i] == zm) {
            ctx->zonemaps.erase(ctx->zonemaps.begin() + (long)i);
            return GACE_OK;
        }
    set_error("zone map not attached to this context");
    return GACE_EINVAL;
}

extern "C" gace_status gace_probe_selectivity_zm(gace_ctx* ctx, const gace_table* table, const gace_zonemap* zm,
                                                 const gace_predicates* preds, const gace_sample_spec* spec,
                                                 uint64_t* counts, gace_probe_info* info, uint64_t* zones_skipped,
                                                 void* stream) {
    if (!ctx || !table || !zm || !preds) {
        set_error("NULL argument");
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
    std::string msg;
    if (gace_status st = gace::check_request(&r, msg)) {
        set_error(msg);
        return st;
    }
    bool same = zm->n_rows == table->n_rows && zm->n_cols == table->n_cols && zm->device == ctx->device;
    for (uint32_t c = 0; same && c < table->n_cols; ++c)
        same = zm->data[c] == table->cols[c].data && zm->dtype[c] == table->cols[c].dtype;
    if (!same) {
        set_error("the zone map was built for another table (rows, column addresses or types differ)");
        return GACE_EINVAL;
    }
    const uint32_t np = preds->n_preds, nt = np ? preds->pred_off[np] : 0;
    // device workspace: skip bits | skipped-zone counter | terms | pred_off;
    // the counter, terms and offsets go up in one copy, the counter as zero
    const uint64_t skip_b = align256((zm->n_zones + 31) / 32 * 4);
    const uint64_t cnt_b = 256;
    const uint64_t term_b = align256((uint64_t)std::max<uint32_t>(nt, 1) * sizeof(gace_term));
    const uint64_t off_b = align256(((uint64_t)np + 1) * 4);
    const uint64_t up_b = cnt_b + term_b + off_b;
    const uint64_t need = skip_b + up_b;
    if (need > ctx->arena_bytes) {
        set_error("workspace too small for the zone-skip map: need " + std::to_string(need) + " bytes");
        return GACE_ENOMEM;
    }
    ZTRY(hipSetDevice(ctx->device), "set device");
    // pinned host staging: 256 B for the counter's download, then the upload
    const uint64_t h_need = 256 + up_b;
    if (ctx->h_hp_bytes < h_need) {
        if (ctx->h_hp) (void)hipHostFree(ctx->h_hp);
        ctx->h_hp = nullptr;
        ctx->h_hp_bytes = 0;
        ZTRY(hipHostMalloc((void**)&ctx->h_hp, h_need, hipHostMallocDefault), "pinned staging");
        ctx->h_hp_bytes = h_need;
    }
    hipStream_t st = (hipStream_t)stream;
    uint32_t* d_skip = (uint32_t*)ctx->d_arena_base;
    uint8_t* d_cnt = ctx->d_arena_base + skip_b;
    uint8_t* d_terms = d_cnt + cnt_b;
    uint32_t* d_off = (uint32_t*)(d_terms + term_b);
    uint64_t* h_cnt = (uint64_t*)ctx->h_hp;
    uint8_t* h_up = ctx->h_hp + 256;
    std::memset(h_up, 0, cnt_b);
    if (nt) std::memcpy(h_up + cnt_b, preds->terms, (uint64_t)nt * sizeof(gace_term));
    if (np) std::memcpy(h_up + cnt_b + term_b, preds->pred_off, ((uint64_t)np + 1) * 4);
    ZTRY(hipMemcpyAsync(d_cnt, h_up, up_b, hipMemcpyHostToDevice, st), "term upload");
    ZTRY(gace_launch_zone_prune(zm->d_mem + zm->zc_off, d_terms, d_off, np, zm->n_zones, d_skip, d_cnt, st),
         "zone prune kernel");
    if (zones_skipped) ZTRY(hipMemcpyAsync(h_cnt, d_cnt, 8, hipMemcpyDeviceToHost, st), "skip count download");

    gace::CompileOptions opt;
    opt.item_rows = ctx->sched.item_rows;
    opt.join_part_keys = ctx->sched.join_part_keys;
    opt.workers = (uint32_t)ctx->n_cu * ctx->sched.wgs_per_cu;
    gace::CompiledBatch& cb = ctx->cb;
    gace::compile_batch(&r, 1, opt, cb);
    if (cb.status[0] != GACE_OK) {
        set_error(cb.errors[0]);
        (void)hipStreamSynchronize(st);
        return cb.status[0];
    }
    if (cb.scans.size() == 1) {
        gace::PlanHdr H;
        std::memcpy(&H, cb.plan.data(), sizeof(H));
        gace::ScanDesc* sd = (gace::ScanDesc*)(cb.plan.data() + H.scans_off);
        sd->zskip = (uint64_t)(uintptr_t)d_skip;
        sd->n_zones = zm->n_zones;
        cb.scans[0].zskip = sd->zskip;
        cb.scans[0].n_zones = sd->n_zones;
    }
    // the batch's done event follows the count download on the same stream
    if (!cb.sel.empty()) {
        if (gace_status e = gace::run_compiled(ctx, cb, &r, nullptr, st, false)) return e;
    } else {
        ZTRY(hipStreamSynchronize(st), "synchronize");
    }
    if (zones_skipped) *zones_skipped = *h_cnt;
    return GACE_OK;
}
