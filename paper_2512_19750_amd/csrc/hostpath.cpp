// hostpath.cpp -- selectivity probes of host-resident tables (Exp. A):
// device-side block sampler, host gather of the kept rows into pinned
// staging, chunked host-to-device copies overlapped with the probe kernels.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <thread>
#include <vector>

#include "../../include/gace_host.h"
#include "compile.h"
#include "runtime.h"

extern "C" hipError_t gace_launch_sample_mask(uint64_t n_blocks, uint64_t seed, uint32_t table_id, uint64_t thr,
                                              void* mask, hipStream_t stream);

using gace::set_error;

namespace {

using clk = std::chrono::steady_clock;

double ms_since(clk::time_point t) { return std::chrono::duration<double, std::milli>(clk::now() - t).count(); }

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

gace_status hip_err(hipError_t e, const char* what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return GACE_EDEVICE;
}

#define HTRY(expr, what)                              \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return hip_err(e_, what); \
    } while (0)

// a contiguous range of kept rows: source row, rows, position in its chunk
struct Piece {
    uint64_t row0, rows, dst;
};

struct Chunk {
    size_t p0, p1;   // pieces [p0, p1)
    uint64_t rows;
};

// copy the chunk's pieces of every transferred column into a host slot,
// split over `threads` workers by rows
void gather(const std::vector<Piece>& pieces, const Chunk& ch, const std::vector<const uint8_t*>& src,
            const std::vector<uint32_t>& width, const std::vector<uint64_t>& col_off, uint8_t* slot,
            uint32_t threads) {
    const uint64_t per = std::max<uint64_t>(1, (ch.rows + threads - 1) / threads);
    auto work = [&](uint64_t lo, uint64_t hi) {   // rows [lo, hi) of the chunk
        for (size_t i = ch.p0; i < ch.p1; ++i) {
            const Piece& p = pieces[i];
            const uint64_t a = std::max(lo, p.dst), b = std::min(hi, p.dst + p.rows);
            if (a >= b) continue;
            for (size_t c = 0; c < src.size(); ++c) {
                const uint64_t w = width[c];
                std::memcpy(slot + col_off[c] + a * w, src[c] + (p.row0 + (a - p.dst)) * w, (b - a) * w);
            }
        }
    };
    if (threads <= 1 || ch.rows < 65536) {
        work(0, ch.rows);
        return;
    }
    std::vector<std::thread> ts;
    for (uint32_t t = 0; t < threads; ++t) {
        const uint64_t lo = t * per, hi = std::min(ch.rows, lo + per);
        if (lo >= hi) break;
        ts.emplace_back(work, lo, hi);
    }
    for (auto& t : ts) t.join();
}

struct Joiner {
    std::thread t;
    ~Joiner() {
        if (t.joinable()) t.join();
    }
};

}  // namespace

extern "C" gace_status gace_probe_selectivity_host(gace_ctx* ctx, const gace_table* table,
                                                   const gace_predicates* preds, const gace_sample_spec* spec,
                                                   const gace_host_opts* opts, uint64_t* counts,
                                                   gace_probe_info* info, gace_transfer_stats* stats,
                                                   void* stream) {
    const clk::time_point t_call = clk::now();
    if (!ctx || !table || !preds || (preds->n_preds && !counts)) {
        set_error("NULL argument");
        return GACE_EINVAL;
    }
    gace_sample_spec sp;
    std::memset(&sp, 0, sizeof(sp));
    sp.rate = 1.0;
    sp.block_rows = 4096;
    if (spec) sp = *spec;
    std::string msg;
    if (gace_status st = gace::check_selectivity(table, preds, &sp, msg)) {
        set_error(msg);
        return st;
    }
    gace_host_opts o;
    std::memset(&o, 0, sizeof(o));
    o.key_only = 1;
    if (opts) o = *opts;
    if (o.chunk_rows == 0) o.chunk_rows = 1ull << 22;
    if (o.gather_threads == 0) o.gather_threads = 8;
    if (o.key_only > 1 || o.chunk_rows < 4096 || o.chunk_rows > (1ull << 30) || o.gather_threads > 64) {
        set_error("host options: key_only 0 or 1, chunk_rows in [4096, 2^30], gather_threads <= 64");
        return GACE_EINVAL;
    }
    const uint32_t np = preds->n_preds;
    const uint64_t n_rows = table->n_rows, B = sp.block_rows;
    const uint64_t n_blocks = (n_rows + B - 1) / B;

    // transferred columns and their staging layout
    std::vector<uint8_t> used(table->n_cols, o.key_only ? 0 : 1);
    for (uint32_t t = 0; np && t < preds->pred_off[np]; ++t) used[preds->terms[t].col] = 1;
    std::vector<uint32_t> cols, width;
    std::vector<const uint8_t*> src;
    std::vector<uint64_t> col_off;
    uint64_t slot_bytes = 0;
    for (uint32_t c = 0; c < table->n_cols; ++c) {
        if (!used[c]) continue;
        const uint32_t w = table->cols[c].dtype == GACE_I64 ? 8u : 4u;
        cols.push_back(c);
        width.push_back(w);
        src.push_back((const uint8_t*)table->cols[c].data);
        col_off.push_back(slot_bytes);
        slot_bytes += align256(o.chunk_rows * w);
    }
    slot_bytes = std::max<uint64_t>(slot_bytes, 256);
    const uint64_t mask_bytes = align256((n_blocks + 31) / 32 * 4);
    const uint64_t need = mask_bytes + 2 * slot_bytes;
    if (need > ctx->arena_bytes) {
        set_error("workspace too small for host-table staging: need " + std::to_string(need) + " bytes, have " +
                  std::to_string(ctx->arena_bytes));
        return GACE_ENOMEM;
    }
    HTRY(hipSetDevice(ctx->device), "set device");
    if (ctx->h_hp_bytes < need) {
        if (ctx->h_hp) (void)hipHostFree(ctx->h_hp);
        ctx->h_hp = nullptr;
        ctx->h_hp_bytes = 0;
        HTRY(hipHostMalloc((void**)&ctx->h_hp, need, hipHostMallocDefault), "pinned staging");
        ctx->h_hp_bytes = need;
    }
    if (!ctx->copy_stream) {
        HTRY(hipStreamCreateWithFlags(&ctx->copy_stream, hipStreamNonBlocking), "copy stream");
        for (int s = 0; s < 2; ++s) {
            HTRY(hipEventCreate(&ctx->ev_h0[s]), "event");
            HTRY(hipEventCreate(&ctx->ev_h1[s]), "event");
        }
        HTRY(hipEventCreate(&ctx->ev_d2h), "event");
    }
    hipStream_t st = (hipStream_t)stream;
    uint8_t* d_mask = ctx->d_arena_base;
    uint8_t* d_slot[2] = {ctx->d_arena_base + mask_bytes, ctx->d_arena_base + mask_bytes + slot_bytes};
    uint32_t* h_mask = (uint32_t*)ctx->h_hp;
    uint8_t* h_slot[2] = {ctx->h_hp + mask_bytes, ctx->h_hp + mask_bytes + slot_bytes};
    gace_transfer_stats S;
    std::memset(&S, 0, sizeof(S));

    // 1. sampler on the device; kept rows as contiguous runs, cut into chunks
    clk::time_point t0 = clk::now();
    if (n_blocks) {
        HTRY(gace_launch_sample_mask(n_blocks, sp.seed, table->table_id, gace::rate_threshold(sp.rate), d_mask, st),
             "sampler kernel");
        HTRY(hipMemcpyAsync(h_mask, d_mask, (n_blocks + 31) / 32 * 4, hipMemcpyDeviceToHost, st), "mask download");
        HTRY(hipStreamSynchronize(st), "synchronize");
    }
    std::vector<Piece> pieces;
    std::vector<Chunk> chunks;
    uint64_t kept_blocks = 0, total_rows = 0;
    {
        uint64_t run0 = 0, run_rows = 0;
        auto emit = [&](uint64_t r0, uint64_t rows) {   // cut a run at chunk boundaries
            while (rows) {
                if (chunks.empty() || chunks.back().rows == o.chunk_rows)
                    chunks.push_back({pieces.size(), pieces.size(), 0});
                Chunk& ch = chunks.back();
                const uint64_t take = std::min(rows, o.chunk_rows - ch.rows);
                pieces.push_back({r0, take, ch.rows});
                ch.p1 = pieces.size();
                ch.rows += take;
                r0 += take;
                rows -= take;
            }
        };
        for (uint64_t w = 0; w < (n_blocks + 31) / 32; ++w) {
            uint32_t bits = h_mask[w];
            while (bits) {
                const uint64_t b = w * 32 + (uint64_t)__builtin_ctz(bits);
                bits &= bits - 1;
                const uint64_t r0 = b * B, rows = std::min(n_rows, r0 + B) - r0;
                kept_blocks += 1;
                total_rows += rows;
                if (run_rows && run0 + run_rows == r0) {
                    run_rows += rows;
                } else {
                    if (run_rows) emit(run0, run_rows);
                    run0 = r0;
                    run_rows = rows;
                }
            }
        }
        if (run_rows) emit(run0, run_rows);
    }
    S.sample_ms = ms_since(t0);

    // 2-4. gather -> copy -> probe, two slots deep
    std::vector<unsigned long long> acc(np, 0);
    std::vector<gace_column> dcols(table->n_cols);
    std::vector<uint64_t> part(std::max<uint32_t>(np, 1), 0);
    auto h2d = [&](size_t k) -> gace_status {
        const int s = (int)(k & 1);
        HTRY(hipEventRecord(ctx->ev_h0[s], ctx->copy_stream), "event");
        for (size_t c = 0; c < cols.size(); ++c)
            HTRY(hipMemcpyAsync(d_slot[s] + col_off[c], h_slot[s] + col_off[c], chunks[k].rows * width[c],
                                hipMemcpyHostToDevice, ctx->copy_stream), "chunk upload");
        HTRY(hipEventRecord(ctx->ev_h1[s], ctx->copy_stream), "event");
        for (size_t c = 0; c < cols.size(); ++c) S.h2d_bytes += chunks[k].rows * width[c];
        return GACE_OK;
    };
    auto gather_k = [&](size_t k, double* ms) {
        const clk::time_point g0 = clk::now();
        gather(pieces, chunks[k], src, width, col_off, h_slot[k & 1], o.gather_threads);
        *ms += ms_since(g0);
    };
    auto probe = [&](size_t k) -> gace_status {
        const int s = (int)(k & 1);
        HTRY(hipStreamWaitEvent(st, ctx->ev_h1[s], 0), "wait for chunk");
        for (uint32_t c = 0; c < table->n_cols; ++c) {
            dcols[c].dtype = table->cols[c].dtype;
            dcols[c].reserved = 0;
            dcols[c].data = d_slot[s];          // columns that are not transferred are never read
        }
        for (size_t c = 0; c < cols.size(); ++c) dcols[cols[c]].data = d_slot[s] + col_off[c];
        gace_request r;
        std::memset(&r, 0, sizeof(r));
        r.kind = GACE_REQ_SELECTIVITY;
        r.table.n_rows = chunks[k].rows;
        r.table.cols = dcols.data();
        r.table.n_cols = table->n_cols;
        r.table.table_id = table->table_id;
        r.preds = *preds;
        r.spec.rate = 1.0;                      // every staged row is a sampled row
        r.spec.block_rows = 4096;
        r.counts = part.data();
        gace::CompileOptions co;
        co.item_rows = ctx->sched.item_rows;
        co.join_part_keys = ctx->sched.join_part_keys;
        co.workers = (uint32_t)ctx->n_cu * ctx->sched.wgs_per_cu;
        gace::CompiledBatch cb;
        gace::compile_batch(&r, 1, co, cb);
        if (cb.status[0] != GACE_OK) {
            set_error(cb.errors[0]);
            return cb.status[0];
        }
        if (gace_status e = gace::launch_compiled(ctx, cb, st, false)) return e;
        HTRY(hipEventRecord(ctx->ev_d2h, st), "event");
        HTRY(hipEventSynchronize(ctx->ev_d2h), "synchronize");
        if (gace_status e = gace::finish_compiled(ctx, cb, &r, nullptr)) return e;
        float ms = 0.f;
        S.kernel_ms += ctx->last_kernel_ms;
        if (hipEventElapsedTime(&ms, ctx->ev1, ctx->ev_d2h) == hipSuccess) S.d2h_ms += ms;
        if (hipEventElapsedTime(&ms, ctx->ev_h0[s], ctx->ev_h1[s]) == hipSuccess) S.h2d_ms += ms;
        const clk::time_point r0 = clk::now();
        for (uint32_t p = 0; p < np; ++p) acc[p] += part[p];
        S.reduce_ms += ms_since(r0);
        return GACE_OK;
    };
    const size_t nc = np ? chunks.size() : 0;   // no predicates: nothing to count, nothing to move
    if (nc) {
        gather_k(0, &S.gather_ms);
        if (gace_status e = h2d(0)) return e;
        if (nc > 1) gather_k(1, &S.gather_ms);
    }
    double bg_ms = 0.0;
    for (size_t k = 0; k < nc; ++k) {
        if (k + 1 < nc)
            if (gace_status e = h2d(k + 1)) return e;
        Joiner j;
        if (k + 2 < nc) {
            // host slot k & 1 is free once chunk k's copy has finished
            HTRY(hipEventSynchronize(ctx->ev_h1[k & 1]), "synchronize");
            j.t = std::thread(gather_k, k + 2, &bg_ms);
        }
        if (gace_status e = probe(k)) return e;
    }
    S.gather_ms += bg_ms;
    S.chunks = (uint32_t)nc;
    for (uint32_t p = 0; p < np; ++p) counts[p] = acc[p];
    if (info) {
        info->sampled_rows = total_rows;
        info->kept_blocks = kept_blocks;
    }
    S.total_ms = ms_since(t_call);
    if (stats) *stats = S;
    return GACE_OK;
}
