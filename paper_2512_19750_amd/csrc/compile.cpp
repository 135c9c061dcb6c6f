// compile.cpp -- request validation and compilation (host only).
//
// A conjunctive predicate is turned into per-column programs: on each column
// the terms' accepted values form intervals on an order-preserving unsigned
// key line (int32 and float32 map to 32-bit keys, int64 to 64-bit keys).  All
// interval endpoints of a 64-predicate group on a column cut the key line into
// elementary intervals on which every term is constant; each elementary
// interval gets a 64-bit mask with bit p set when predicate p's terms on that
// column all accept it.  At run time a row's mask is the AND over the
// referenced columns of mask[interval(value)], so the per-row work is one
// lookup per column instead of one comparison per term (Sec. III-B "Key-Only
// + Bitmask": only the referenced columns are read; bits are never stored).
#include "compile.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>

namespace gace {

typedef unsigned __int128 u128;

uint64_t rate_threshold(double rate) {
    if (rate >= 1.0) return kThrAll;
    if (!(rate > 0.0)) return 0;
    return (uint64_t)std::floor(rate * 4294967296.0);
}

static float f32_of(int64_t v) {
    uint32_t b = (uint32_t)(uint64_t)v;
    float f;
    std::memcpy(&f, &b, 4);
    return f;
}

static uint32_t f32_key(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u << 1) == 0u) u = 0u;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// ------------------------------------------------------------------ checks
gace_status check_spec(const gace_sample_spec* s, std::string& msg) {
    if (!s) return GACE_OK;
    if (!(s->rate >= 0.0 && s->rate <= 1.0)) {
        msg = "sample rate must be in [0, 1]";
        return GACE_EINVAL;
    }
    const uint32_t b = s->block_rows;
    if (b == 0 || b > (1u << 20) || (b & (b - 1))) {
        msg = "block_rows must be a power of two in [1, 2^20]";
        return GACE_EINVAL;
    }
    return GACE_OK;
}

gace_status check_selectivity(const gace_table* t, const gace_predicates* p, const gace_sample_spec* s,
                              std::string& msg) {
    if (!t || !p) {
        msg = "table and predicates must not be NULL";
        return GACE_EINVAL;
    }
    if (gace_status st = check_spec(s, msg)) return st;
    if (t->n_cols && !t->cols) {
        msg = "table has columns but a NULL column array";
        return GACE_EINVAL;
    }
    for (uint32_t c = 0; c < t->n_cols; ++c) {
        const gace_column& col = t->cols[c];
        if (col.dtype < GACE_I32 || col.dtype > GACE_F32) {
            msg = "column " + std::to_string(c) + " has an unknown dtype";
            return GACE_EINVAL;
        }
        if (t->n_rows && !col.data) {
            msg = "column " + std::to_string(c) + " has a NULL data pointer";
            return GACE_EINVAL;
        }
        if (((uintptr_t)col.data) & 15u) {
            msg = "column " + std::to_string(c) + " is not 16-byte aligned";
            return GACE_EINVAL;
        }
    }
    if (p->n_preds > kMaxPredsPerReq) {
        msg = "more than 65536 predicates in one request";
        return GACE_EINVAL;
    }
    if (p->n_preds && (!p->pred_off || !p->terms)) {
        msg = "predicates with a NULL term or offset array";
        return GACE_EINVAL;
    }
    if (p->n_preds && p->pred_off[0] != 0) {
        msg = "pred_off[0] must be 0";
        return GACE_EINVAL;
    }
    for (uint32_t q = 0; q < p->n_preds; ++q) {
        const uint32_t a = p->pred_off[q], b = p->pred_off[q + 1];
        if (b <= a || b - a > kMaxTermsPerPred) {
            msg = "predicate " + std::to_string(q) + " must have 1..16 terms";
            return GACE_EINVAL;
        }
        for (uint32_t i = a; i < b; ++i) {
            const gace_term& tm = p->terms[i];
            if (tm.col >= t->n_cols) {
                msg = "term column index out of range";
                return GACE_EINVAL;
            }
            if (tm.op == GACE_RANGE) {
                if (tm.n_vals != 2) { msg = "RANGE needs exactly 2 values"; return GACE_EINVAL; }
            } else if (tm.op == GACE_EQ) {
                if (tm.n_vals != 1) { msg = "EQ needs exactly 1 value"; return GACE_EINVAL; }
            } else if (tm.op == GACE_IN) {
                if (tm.n_vals < 1 || tm.n_vals > kMaxInVals) { msg = "IN needs 1..8 values"; return GACE_EINVAL; }
            } else {
                msg = "unknown term operator";
                return GACE_EINVAL;
            }
            if (t->cols[tm.col].dtype == GACE_F32)
                for (uint32_t k = 0; k < tm.n_vals; ++k)
                    if (std::isnan(f32_of(tm.v[k]))) { msg = "NaN float bound"; return GACE_EINVAL; }
        }
    }
    return GACE_OK;
}

static gace_status check_side(const gace_keys* k, const char* name, std::string& msg) {
    if (!k) { msg = std::string(name) + " is NULL"; return GACE_EINVAL; }
    if (k->n && !k->keys) { msg = std::string(name) + " has keys but a NULL pointer"; return GACE_EINVAL; }
    if (((uintptr_t)k->keys) & 7u) { msg = std::string(name) + " keys are not 8-byte aligned"; return GACE_EINVAL; }
    if (k->n > 0xFFFFFFFFull) { msg = std::string(name) + " has more than 2^32 - 1 keys"; return GACE_EINVAL; }
    return check_spec(&k->spec, msg);
}

gace_status check_join(const gace_keys* R, const gace_keys* S, std::string& msg) {
    if (gace_status st = check_side(R, "R", msg)) return st;
    // each side holds fewer than 2^32 keys, so n_R * n_S < 2^64 bounds sum f_R f_S
    return check_side(S, "S", msg);
}

gace_status check_request(const gace_request* r, std::string& msg) {
    if (!r) { msg = "NULL request"; return GACE_EINVAL; }
    if (r->kind == GACE_REQ_SELECTIVITY) {
        if (gace_status st = check_selectivity(&r->table, &r->preds, &r->spec, msg)) return st;
        if (r->preds.n_preds && !r->counts) { msg = "NULL counts output"; return GACE_EINVAL; }
        return GACE_OK;
    }
    if (r->kind == GACE_REQ_JOIN) {
        if (gace_status st = check_join(&r->R, &r->S, msg)) return st;
        if (!r->join) { msg = "NULL join output"; return GACE_EINVAL; }
        return GACE_OK;
    }
    msg = "unknown request kind";
    return GACE_EINVAL;
}

// ------------------------------------------------------------------ intervals
struct Iv {
    u128 a, b;   // [a, b) on the key line; b == END means "to the end"
};

static void term_intervals(uint32_t dtype, const gace_term& t, std::vector<Iv>& out) {
    out.clear();
    if (dtype == GACE_I32) {
        const int64_t lo32 = INT32_MIN, end32 = (int64_t)INT32_MAX + 1;
        const u128 bias = (u128)1 << 31;
        if (t.op == GACE_RANGE) {
            const int64_t l = std::max(t.v[0], lo32), h = std::min(t.v[1], end32);
            if (l < h) out.push_back({(u128)(l + (int64_t)bias), (u128)(h + (int64_t)bias)});
        } else {
            for (uint32_t i = 0; i < t.n_vals; ++i)
                if (t.v[i] >= lo32 && t.v[i] < end32) {
                    const u128 k = (u128)(t.v[i] + (int64_t)bias);
                    out.push_back({k, k + 1});
                }
        }
    } else if (dtype == GACE_F32) {
        if (t.op == GACE_RANGE) {
            const float fl = f32_of(t.v[0]), fh = f32_of(t.v[1]);
            if (fl < fh) out.push_back({(u128)f32_key(fl), (u128)f32_key(fh)});
        } else {
            for (uint32_t i = 0; i < t.n_vals; ++i) {
                const u128 k = f32_key(f32_of(t.v[i]));
                out.push_back({k, k + 1});
            }
        }
    } else {
        const uint64_t flip = 0x8000000000000000ull;
        if (t.op == GACE_RANGE) {
            if (t.v[0] < t.v[1]) out.push_back({(u128)((uint64_t)t.v[0] ^ flip), (u128)((uint64_t)t.v[1] ^ flip)});
        } else {
            for (uint32_t i = 0; i < t.n_vals; ++i) {
                const u128 k = (u128)((uint64_t)t.v[i] ^ flip);
                out.push_back({k, k + 1});
            }
        }
    }
    // merge overlapping intervals (IN lists may repeat values)
    std::sort(out.begin(), out.end(), [](const Iv& x, const Iv& y) { return x.a < y.a; });
    size_t w = 0;
    for (size_t i = 0; i < out.size(); ++i) {
        if (w && out[i].a <= out[w - 1].b) {
            if (out[i].b > out[w - 1].b) out[w - 1].b = out[i].b;
        } else {
            out[w++] = out[i];
        }
    }
    out.resize(w);
}

// ------------------------------------------------------------------ groups
struct BitRef {
    const gace_table* table;
    const gace_term* terms;   // the predicate's terms
    uint32_t n_terms;
};

struct ColBuild {
    uint32_t col;
    ColProg prog;
    std::vector<uint64_t> masks;
    std::vector<uint64_t> bnd;   // boundaries (stored as u32 or u64)
    bool wide;
};

static uint32_t align_up(uint32_t x, uint32_t a) { return (x + a - 1) / a * a; }

// Build the programs of one group of <= 64 bits.  Returns the group descriptor
// (offsets relative to its own table region) and appends its ColProgs.
static void build_group(const std::vector<BitRef>& bits, const gace_table* table, GroupDesc& G,
                        std::vector<ColProg>& cols_out, std::vector<uint8_t>& tab_out) {
    const uint32_t nb = (uint32_t)bits.size();
    uint64_t base = nb == 64 ? ~0ull : ((1ull << nb) - 1);
    // referenced columns, in ascending order
    std::vector<uint32_t> refcols;
    for (const BitRef& b : bits)
        for (uint32_t i = 0; i < b.n_terms; ++i) refcols.push_back(b.terms[i].col);
    std::sort(refcols.begin(), refcols.end());
    refcols.erase(std::unique(refcols.begin(), refcols.end()), refcols.end());

    std::vector<ColBuild> builds;
    std::vector<Iv> iv;
    // the term intervals on one column, in (bit, term) order: one flat list
    // reused across columns (this runs for every group of every batch)
    struct TermIv {
        uint32_t bit, term;
        Iv x;
    };
    std::vector<TermIv> tiv;
    // interval boundaries: every stored one is below END <= 2^64, so they
    // sort and search as 64-bit integers
    std::vector<uint64_t> B;
    std::vector<uint32_t> nterm(nb);
    std::vector<Iv> cur, nxt;
    for (uint32_t col : refcols) {
        const uint32_t dt = table->cols[col].dtype;
        const bool wide = dt == GACE_I64;
        const u128 END = wide ? ((u128)1 << 64) : ((u128)1 << 32);
        tiv.clear();
        B.clear();
        for (uint32_t i = 0; i < nb; ++i) {
            nterm[i] = 0;
            for (uint32_t t = 0; t < bits[i].n_terms; ++t)
                if (bits[i].terms[t].col == col) {
                    term_intervals(dt, bits[i].terms[t], iv);
                    for (const Iv& x : iv) {
                        if (x.a > 0) B.push_back((uint64_t)x.a);
                        if (x.b < END) B.push_back((uint64_t)x.b);
                        tiv.push_back({i, nterm[i], x});
                    }
                    ++nterm[i];
                }
        }
        std::sort(B.begin(), B.end());
        B.erase(std::unique(B.begin(), B.end()), B.end());
        const uint32_t m = (uint32_t)B.size();
        auto idx = [&](u128 x) -> uint32_t {
            if (x >= END) return m + 1;
            return (uint32_t)(std::upper_bound(B.begin(), B.end(), (uint64_t)x) - B.begin());
        };
        // acceptance: bit set on interval j when all the bit's terms on this column hold there
        std::vector<uint64_t> mask(m + 1, 0);
        std::vector<uint64_t> diff(m + 2, 0);
        uint64_t no_term = 0;
        size_t e = 0;   // cursor into tiv
        for (uint32_t i = 0; i < nb; ++i) {
            const uint64_t bit = 1ull << i;
            if (nterm[i] == 0) { no_term |= bit; continue; }
            const size_t e0 = e;
            while (e < tiv.size() && tiv[e].bit == i) ++e;
            if (nterm[i] == 1) {
                for (size_t k = e0; k < e; ++k) {
                    diff[idx(tiv[k].x.a)] ^= bit;
                    diff[idx(tiv[k].x.b)] ^= bit;
                }
                continue;
            }
            // several terms on this column: intersect their sorted, disjoint
            // interval lists (a term with no interval empties the result),
            // then mark the result like a single term's intervals
            cur.clear();
            bool first = true;
            for (size_t k = e0; k < e;) {
                const uint32_t t = tiv[k].term;
                const size_t k0 = k;
                while (k < e && tiv[k].term == t) ++k;
                if (first) {
                    for (size_t q = k0; q < k; ++q) cur.push_back(tiv[q].x);
                    first = false;
                    continue;
                }
                nxt.clear();
                size_t a = 0, q = k0;
                while (a < cur.size() && q < k) {
                    const u128 lo = std::max(cur[a].a, tiv[q].x.a), hi = std::min(cur[a].b, tiv[q].x.b);
                    if (lo < hi) nxt.push_back({lo, hi});
                    if (cur[a].b < tiv[q].x.b) ++a; else ++q;
                }
                cur.swap(nxt);
            }
            // a term with no interval on the line (an empty range) accepts nothing
            uint32_t seen_terms = 0;
            for (size_t k = e0; k < e; ++k)
                if (k == e0 || tiv[k].term != tiv[k - 1].term) ++seen_terms;
            if (seen_terms < nterm[i]) cur.clear();
            for (const Iv& x : cur) {
                diff[idx(x.a)] ^= bit;
                diff[idx(x.b)] ^= bit;
            }
        }
        uint64_t run = 0;
        for (uint32_t j = 0; j <= m; ++j) {
            run ^= diff[j];
            mask[j] |= run | no_term;
        }
        if (m == 0) {            // constant column: fold into the base mask
            base &= mask[0];
            continue;
        }
        ColBuild cb;
        cb.col = col;
        cb.wide = wide;
        std::memset(&cb.prog, 0, sizeof(cb.prog));
        cb.prog.data = table->cols[col].data;
        cb.prog.xform = dt == GACE_I32 ? XF_I32 : (dt == GACE_F32 ? XF_F32 : XF_I64);
        cb.masks = std::move(mask);
        cb.bnd.resize(m);
        for (uint32_t j = 0; j < m; ++j) cb.bnd[j] = B[j];
        builds.push_back(std::move(cb));
    }

    // choose LUT or RANK per column within the LDS budget
    auto rank_bytes = [](const ColBuild& c) {
        return align_up((uint32_t)c.masks.size() * 8, 8) + align_up((uint32_t)c.bnd.size() * (c.wide ? 8 : 4), 8);
    };
    auto lut_entries = [](const ColBuild& c) -> uint64_t {
        if (c.wide) return ~0ull;
        return c.bnd.back() - c.bnd.front() + 2;
    };
    uint32_t total = 0;
    for (const ColBuild& c : builds) total += rank_bytes(c);
    std::vector<bool> use_lut(builds.size(), false);
    for (size_t i = 0; i < builds.size(); ++i) {
        const uint64_t e = lut_entries(builds[i]);
        if (e > kLutMaxEntries) continue;
        const uint32_t lb = align_up((uint32_t)e * 8, 8);
        if (total - rank_bytes(builds[i]) + lb <= kGroupTabBudget) {
            total = total - rank_bytes(builds[i]) + lb;
            use_lut[i] = true;
        }
    }

    std::vector<uint8_t> tab;
    tab.reserve(total + 8 * (2 * builds.size() + 2));
    auto put = [&](const void* p, size_t n) -> uint32_t {
        const uint32_t off = align_up((uint32_t)tab.size(), 8);
        tab.resize(off + n);
        std::memcpy(tab.data() + off, p, n);
        return off;
    };
    G.col_begin = (uint32_t)cols_out.size();
    for (size_t i = 0; i < builds.size(); ++i) {
        ColBuild& c = builds[i];
        ColProg P = c.prog;
        if (use_lut[i]) {
            const uint32_t lo = (uint32_t)c.bnd.front() - 1u, hi = (uint32_t)c.bnd.back();
            std::vector<uint64_t> lut(hi - lo + 1);
            uint32_t j = 0;   // interval index of key lo + e
            for (uint64_t e = 0; e < lut.size(); ++e) {
                const uint64_t key = (uint64_t)lo + e;
                while (j < c.bnd.size() && c.bnd[j] <= key) ++j;
                lut[e] = c.masks[j];
            }
            P.kind = CP_LUT32;
            P.lo = lo;
            P.hi = hi;
            P.mask_off = put(lut.data(), lut.size() * 8);
        } else {
            P.kind = c.wide ? CP_RANK64 : CP_RANK32;
            P.nb = (uint32_t)c.bnd.size();
            P.step = 1;
            while (P.step * 2 <= P.nb) P.step *= 2;
            P.mask_off = put(c.masks.data(), c.masks.size() * 8);
            if (c.wide) {
                P.bnd_off = put(c.bnd.data(), c.bnd.size() * 8);
            } else {
                std::vector<uint32_t> b32(c.bnd.begin(), c.bnd.end());
                P.bnd_off = put(b32.data(), b32.size() * 4);
            }
        }
        cols_out.push_back(P);
    }
    G.col_end = (uint32_t)cols_out.size();
    tab.resize(align_up((uint32_t)tab.size(), 16));
    G.base_mask = base;
    G.n_used = nb;
    G.tab_bytes = (uint32_t)tab.size();
    tab_out = std::move(tab);
}

// ------------------------------------------------------------------ host threads
// Worker threads that outlive a compilation: starting and joining 15 threads
// costs a few hundred microseconds, next to ~1 ms of compilation.  run(n, f)
// calls f on n threads (the caller and n - 1 workers) and returns when all
// have returned; one run at a time.  The pool is never destroyed: its
// workers wait on its condition variable until the process ends.
class HostPool {
public:
    void run(uint32_t n, const std::function<void()>& f) {
        std::lock_guard<std::mutex> one(run_m_);
        {
            std::lock_guard<std::mutex> lk(m_);
            while (threads_.size() + 1 < n) {
                const uint32_t id = (uint32_t)threads_.size();
                threads_.emplace_back([this, id] { worker(id); });
            }
            job_ = &f;
            want_ = n - 1;
            pending_ = n - 1;
            ++gen_;
        }
        cv_start_.notify_all();
        f();
        std::unique_lock<std::mutex> lk(m_);
        cv_done_.wait(lk, [this] { return pending_ == 0; });
        job_ = nullptr;
    }

private:
    void worker(uint32_t id) {
        uint64_t seen = 0;
        std::unique_lock<std::mutex> lk(m_);
        for (;;) {
            cv_start_.wait(lk, [&] { return gen_ != seen; });
            seen = gen_;
            if (id >= want_) continue;
            const std::function<void()>* f = job_;
            lk.unlock();
            (*f)();
            lk.lock();
            if (--pending_ == 0) cv_done_.notify_all();
        }
    }
    std::mutex run_m_, m_;
    std::condition_variable cv_start_, cv_done_;
    std::vector<std::thread> threads_;
    const std::function<void()>* job_ = nullptr;
    uint64_t gen_ = 0;
    uint32_t want_ = 0, pending_ = 0;
};

static HostPool& host_pool() {
    static HostPool* p = new HostPool;
    return *p;
}

// ------------------------------------------------------------------ batch
static uint32_t log2u(uint32_t x) {
    uint32_t l = 0;
    while ((1u << l) < x) ++l;
    return l;
}

static uint64_t bpi_for(uint64_t thr, uint32_t log2B, uint32_t item_rows) {
    const double p = thr >= kThrAll ? 1.0 : (double)thr / 4294967296.0;
    if (p <= 0.0) return 0;
    double want = (double)item_rows / ((double)(1ull << log2B) * p);
    uint64_t b = want < 1.0 ? 1 : (uint64_t)want;
    if (b > 64) b = (b + 63) / 64 * 64;   // whole 64-block decision chunks
    if (b > (1ull << 30)) b = 1ull << 30;
    return b;
}

void compile_batch(const gace_request* reqs, uint32_t n, const CompileOptions& opt, CompiledBatch& out) {
    // clear, keeping the vectors' capacity: a context compiles batch after
    // batch, and fresh multi-megabyte buffers cost more in page faults than
    // the compilation itself
    out.plan.clear();
    out.items.clear();
    out.sel.clear();
    out.joins.clear();
    out.scans.clear();
    out.jdesc.clear();
    out.n_counts = out.n_hist = 0;
    out.err_off = 0;
    out.arena_static = 0;
    out.est_scan_bytes = out.est_join_keys = 0.0;
    out.status.assign(n, GACE_OK);
    out.errors.assign(n, std::string());

    struct ScanReq { uint32_t req; uint64_t thr; };
    std::map<std::vector<uint64_t>, uint32_t> scan_of;
    std::vector<std::vector<ScanReq>> scan_reqs;
    std::vector<uint32_t> join_reqs;
    for (uint32_t i = 0; i < n; ++i) {
        std::string msg;
        gace_status st = check_request(&reqs[i], msg);
        out.status[i] = st;
        out.errors[i] = msg;
        if (st != GACE_OK) continue;
        const gace_request& r = reqs[i];
        if (r.kind == GACE_REQ_JOIN) {
            join_reqs.push_back(i);
            continue;
        }
        const uint32_t B = r.spec.block_rows;
        std::vector<uint64_t> key = {r.table.n_rows, r.table.table_id, r.spec.seed, B, r.table.n_cols};
        for (uint32_t c = 0; c < r.table.n_cols; ++c) {
            key.push_back((uint64_t)(uintptr_t)r.table.cols[c].data);
            key.push_back(r.table.cols[c].dtype);
        }
        auto it = scan_of.find(key);
        uint32_t s;
        if (it == scan_of.end()) {
            s = (uint32_t)scan_reqs.size();
            scan_of.emplace(key, s);
            scan_reqs.emplace_back();
        } else {
            s = it->second;
        }
        scan_reqs[s].push_back({i, rate_threshold(r.spec.rate)});
    }

    // ---- selectivity scans
    std::vector<ScanDesc> scans;
    std::vector<GroupDesc> groups;
    std::vector<ColProg> cols;
    std::vector<uint32_t> slots;
    std::vector<uint64_t> rthr;
    std::vector<uint32_t> rcum;
    std::vector<std::vector<uint8_t>> tabs;
    struct GroupJob {
        std::vector<BitRef> bits;
        const gace_table* table;
        GroupDesc G;
        std::vector<ColProg> cols;
        std::vector<uint8_t> tab;
    };
    std::vector<GroupJob> jobs;
    uint32_t n_counts = 0, n_hist = 0;
    for (uint32_t s = 0; s < scan_reqs.size(); ++s) {
        auto& sr = scan_reqs[s];
        std::stable_sort(sr.begin(), sr.end(), [](const ScanReq& x, const ScanReq& y) { return x.thr > y.thr; });
        const gace_request& r0 = reqs[sr[0].req];
        ScanDesc S;
        std::memset(&S, 0, sizeof(S));
        S.n_rows = r0.table.n_rows;
        S.seed = r0.spec.seed;
        S.thr_max = sr[0].thr;
        S.log2B = log2u(r0.spec.block_rows);
        S.n_blocks = (S.n_rows + (1ull << S.log2B) - 1) >> S.log2B;
        S.table_id = r0.table.table_id;
        S.req_begin = (uint32_t)rthr.size();
        S.n_req = (uint32_t)sr.size();
        S.hist_off = n_hist;
        n_hist += 2 * (S.n_req + 1);
        S.group_begin = (uint32_t)jobs.size();

        std::vector<BitRef> bits;
        std::vector<uint32_t> bit_slot;
        std::vector<bool> used_col(r0.table.n_cols, false);
        uint32_t cum = 0;
        rcum.push_back(0);
        for (uint32_t q = 0; q < sr.size(); ++q) {
            const gace_request& r = reqs[sr[q].req];
            rthr.push_back(sr[q].thr);
            SelOut so;
            so.req = sr[q].req;
            so.scan = s;
            so.rank = q;
            so.count_off = n_counts;
            so.n_preds = r.preds.n_preds;
            out.sel.push_back(so);
            for (uint32_t p = 0; p < r.preds.n_preds; ++p) {
                const uint32_t a = r.preds.pred_off[p], b = r.preds.pred_off[p + 1];
                bits.push_back({&r.table, r.preds.terms + a, b - a});
                bit_slot.push_back(n_counts + p);
                for (uint32_t t = a; t < b; ++t) used_col[r.preds.terms[t].col] = true;
            }
            n_counts += r.preds.n_preds;
            cum += r.preds.n_preds;
            if (q + 1 < sr.size()) rcum.push_back(cum);
        }
        rcum.push_back(cum);
        // rcum for this scan has n_req + 1 entries; rthr has n_req
        for (uint32_t c = 0; c < r0.table.n_cols; ++c)
            if (used_col[c]) S.row_bytes += r0.table.cols[c].dtype == GACE_I64 ? 8 : 4;

        for (uint32_t g0 = 0; g0 < bits.size(); g0 += 64) {
            const uint32_t g1 = std::min<uint32_t>((uint32_t)bits.size(), g0 + 64);
            GroupJob job;
            job.bits.assign(bits.begin() + g0, bits.begin() + g1);
            job.table = &r0.table;
            std::memset(&job.G, 0, sizeof(job.G));
            job.G.slot_index = (uint32_t)slots.size();
            for (uint32_t i = g0; i < g0 + 64; ++i) slots.push_back(i < g1 ? bit_slot[i] : 0);
            jobs.push_back(std::move(job));
        }
        S.n_groups = (uint32_t)jobs.size() - S.group_begin;
        scans.push_back(S);
    }
    // the groups compile independently: spread them over a few host threads,
    // then append their column programs and tables in group order
    {
        std::atomic<uint32_t> next{0};
        auto work = [&] {
            for (uint32_t j; (j = next.fetch_add(1)) < jobs.size();)
                build_group(jobs[j].bits, jobs[j].table, jobs[j].G, jobs[j].cols, jobs[j].tab);
        };
        const uint32_t hw = std::max(1u, std::thread::hardware_concurrency());
        const uint32_t nt = std::min<uint32_t>({hw, 16u, (uint32_t)(jobs.size() + 7) / 8});
        if (nt > 1)
            host_pool().run(nt, work);
        else
            work();
        for (GroupJob& job : jobs) {
            GroupDesc G = job.G;
            G.col_begin += (uint32_t)cols.size();
            G.col_end += (uint32_t)cols.size();
            cols.insert(cols.end(), job.cols.begin(), job.cols.end());
            groups.push_back(G);
            tabs.push_back(std::move(job.tab));
        }
    }
    // the reqcum array interleaves per scan: entries [req_begin + scan_index, ...) -- keep it simple by
    // rebuilding it with explicit per-scan offsets
    std::vector<uint32_t> rcum_flat;
    {
        size_t pos = 0;
        for (uint32_t s = 0; s < scans.size(); ++s) {
            const uint32_t nr = scans[s].n_req;
            scans[s].req_begin = (uint32_t)rcum_flat.size();   // same start for thresholds (copied below)
            for (uint32_t i = 0; i <= nr; ++i) rcum_flat.push_back(rcum[pos + i]);
            pos += nr + 1;
        }
    }
    // thresholds laid out with the same per-scan start as rcum_flat (n_req + 1 stride, last unused)
    std::vector<uint64_t> rthr_flat;
    {
        size_t pos = 0;
        for (uint32_t s = 0; s < scans.size(); ++s) {
            const uint32_t nr = scans[s].n_req;
            for (uint32_t i = 0; i < nr; ++i) rthr_flat.push_back(rthr[pos + i]);
            rthr_flat.push_back(0);
            pos += nr;
        }
    }

    // ---- joins: hash-partitioned key aggregation
    std::vector<JoinDesc> joins;
    std::vector<Item> heavy_items, hist_items, off_items, base_items, scatter_items, scatter2_items, agg_items;
    uint64_t arena_static = 0;
    auto carve = [&](uint64_t bytes) {
        const uint64_t off = arena_static;
        arena_static += (bytes + 255) / 256 * 256;
        return off;
    };
    // Small join batches spread over the partitioning workers: items shrink
    // below item_rows keys only while the batch would have fewer items than
    // the workers, and second-pass units shrink to ~2 per worker.  A large
    // batch keeps items of item_rows keys and units of kUnit2Keys; a lone
    // join of 12.7 M keys gets one item per worker (512 instead of 49) and
    // units of a few thousand keys, so a Zipf-hot bucket no longer stalls its
    // second pass.  (Smaller items for a join that already has more items
    // than workers made its offset phases longer: 250 M keys, 8.1 -> 8.5 ms.)
    double batch_keys = 0.0;
    for (uint32_t j = 0; j < join_reqs.size(); ++j) {
        const gace_request& r = reqs[join_reqs[j]];
        for (const gace_keys* k : {&r.R, &r.S}) {
            const uint64_t thr = rate_threshold(k->spec.rate);
            batch_keys += (double)k->n * (thr >= kThrAll ? 1.0 : (double)thr / 4294967296.0);
        }
    }
    const double workers = std::max<uint32_t>(opt.workers, 1);
    const double item_share = batch_keys / workers, unit_share = batch_keys / (2.0 * workers);
    for (uint32_t j = 0; j < join_reqs.size(); ++j) {
        const gace_request& r = reqs[join_reqs[j]];
        JoinDesc J;
        std::memset(&J, 0, sizeof(J));
        const gace_keys* sides[2] = {&r.R, &r.S};
        double expect = 0.0, side_p[2];
        for (uint32_t sd = 0; sd < 2; ++sd) {
            JoinSide& D = J.side[sd];
            D.keys = sides[sd]->keys;
            D.n = sides[sd]->n;
            D.seed = sides[sd]->spec.seed;
            D.thr = rate_threshold(sides[sd]->spec.rate);
            D.log2B = log2u(sides[sd]->spec.block_rows);
            D.n_blocks = (D.n + (1ull << D.log2B) - 1) >> D.log2B;
            D.table_id = sides[sd]->table_id;
            side_p[sd] = D.thr >= kThrAll ? 1.0 : (double)D.thr / 4294967296.0;
            expect += (double)D.n * side_p[sd];
        }
        out.est_join_keys += expect;
        uint32_t log2P = 0;
        while (log2P < kPartBitsMax && (double)(1u << log2P) * (double)opt.join_part_keys < expect) ++log2P;
        const uint32_t P = 1u << log2P;
        // two passes when the fan-out is too wide for one LDS-staged pass:
        // first 2^log2P1 buckets, then 2^log2P2 partitions inside each bucket
        const uint32_t log2P2 = log2P > 6 ? log2P / 2 : 0;
        const uint32_t log2P1 = log2P - log2P2;
        // items large enough that the per-item partition counts (4 P bytes)
        // stay small next to the item's keys (at most a quarter of their 8 B
        // each; a floor of 8 P keys left a lone 12.7 M-key join 192 items
        // for 512 workers: 1.62 against 1.33 ms)
        const uint32_t item_keys =
            std::max<uint32_t>((uint32_t)std::min<double>(opt.item_rows, item_share), 2u * P);
        uint32_t item = 0;
        std::vector<Item> my_items;
        double keys_per_item = 1.0;
        for (uint32_t sd = 0; sd < 2; ++sd) {
            JoinSide& D = J.side[sd];
            D.item_begin = item;
            const uint64_t bb = bpi_for(D.thr, D.log2B, item_keys);
            if (bb && D.n) {
                for (uint64_t b = 0; b < D.n_blocks; b += bb) {
                    Item it = {IT_JHIST, j, sd, item++, b, std::min(D.n_blocks, b + bb)};
                    my_items.push_back(it);
                }
                keys_per_item = std::max(keys_per_item, (double)bb * (double)(1ull << D.log2B) * side_p[sd]);
            }
            D.n_items = item - D.item_begin;
        }
        J.log2P = log2P;
        J.log2P2 = log2P2;
        J.acc = j;
        J.n_items = item;
        J.n_off = (P + 63) / 64;
        J.n_agg = std::min<uint32_t>(512, std::max<uint32_t>(1, (P + 15) / 16));
        if (log2P2) {
            // second-pass unit: one first-pass bucket of a group of items
            const double unit_keys = std::min<double>(kUnit2Keys, std::max(4096.0, unit_share));
            const double g = unit_keys * (double)(1u << log2P1) / keys_per_item;
            J.group_items = (uint32_t)std::min(1e6, std::max(1.0, g));
            for (uint32_t sd = 0; sd < 2; ++sd)
                J.n_groups[sd] = (J.side[sd].n_items + J.group_items - 1) / J.group_items;
            J.n_units2 = (J.n_groups[0] + J.n_groups[1]) << log2P1;
            J.n_s2 = std::min<uint32_t>(512, std::max<uint32_t>(1, J.n_units2 / 4));
        }
        J.rows_off = carve((uint64_t)item * P * 4);
        J.base_off = carve(2ull * (P + 1) * 4);
        J.stats_off = carve((uint64_t)item * 16);
        // partitions above kChunkKeys keys become chunks + a merge: at most
        // 2 N / kChunkKeys chunks and N / kChunkKeys merges for N keys
        const uint64_t nk = J.side[0].n + J.side[1].n;
        const uint64_t big = nk / kChunkKeys + 1;
        J.max_chunks = (uint32_t)std::min<uint64_t>(2 * big + 8, 0xFFFFFFF0u);
        J.max_units = (uint32_t)std::min<uint64_t>((uint64_t)P + J.max_chunks + big + 8, 0xFFFFFFF0u);
        J.units_off = carve((uint64_t)J.max_units * sizeof(AggUnit));
        J.chunk_off = carve((uint64_t)J.max_chunks * 4);
        J.done_off = carve(big * 4 + 64);
        J.heavy_off = carve((uint64_t)kHeavySlots * 16);
        heavy_items.push_back({IT_JHEAVY, j, 0, 0, 0, 0});
        for (const Item& it : my_items) {
            hist_items.push_back(it);
            Item sc = it;
            sc.kind = IT_JSCATTER;
            scatter_items.push_back(sc);
        }
        for (uint32_t c = 0; c < J.n_off; ++c) off_items.push_back({IT_JOFF, j, 0, c, 0, 0});
        base_items.push_back({IT_JBASE, j, 0, 0, 0, 0});
        for (uint32_t w = 0; w < J.n_s2; ++w) scatter2_items.push_back({IT_JSCATTER2, j, 0, w, 0, 0});
        for (uint32_t w = 0; w < J.n_agg; ++w) agg_items.push_back({IT_JAGG, j, 0, w, 0, 0});
        joins.push_back(J);
        JoinOut jo;
        jo.req = join_reqs[j];
        jo.join = j;
        out.joins.push_back(jo);
    }

    // one histogram entry counts the scan kernel's finished workgroups (per-request completion),
    // the next its waits that gave up
    const uint32_t wg_done_off = n_hist;
    n_hist += 2;

    // ---- items
    // A kept block streams predicate group g only when its draw is below the
    // threshold of the first request owning a bit of g, so a scan's work per
    // kept row is its row width times the expected groups per kept block.
    // Items are sized to about item_rows rows of one group each and queued
    // costliest first, so the tail of the queue is short items.
    std::vector<Item> scan_items;
    std::vector<double> item_cost;
    // one request on blocks under 4096 rows, with more than one kept block per
    // 4096 rows expected (thr_max / 2^32 > B / 4096): decided row by row in
    // whole tiles, which read every row of the item
    auto is_fine = [](const ScanDesc& S) {
        return S.n_req == 1 && S.log2B < kZoneLog2 && S.thr_max > (1ull << (S.log2B + 20));
    };
    // a small batch (a single probe, a short served batch) still gets about
    // four items per worker, down to items of 1024 expected kept rows: in a
    // sparse sample (1 % of 4096-row blocks) an item then spans ~25 blocks and
    // holds a kept block one time in four, so the work queue spreads the
    // kept tiles about one per workgroup instead of stacking several in one
    // item (an item with no kept block costs one sampling decision); the
    // rows an item reads are its kept rows, or all its rows for the
    // row-by-row scan
    uint32_t item_rows = opt.item_rows;
    bool small_batch = false;
    if (opt.workers) {
        double rows_read = 0.0;
        for (const ScanDesc& S : scans)
            rows_read += (double)S.n_rows *
                         (is_fine(S) || S.thr_max >= kThrAll ? 1.0 : (double)S.thr_max / 4294967296.0);
        const double cap = std::max(1024.0, rows_read / (4.0 * opt.workers));
        if (cap < item_rows) {
            item_rows = (uint32_t)cap;
            small_batch = true;
        }
    }
    bool any_spill = false;
    for (uint32_t s = 0; s < scans.size(); ++s) {
        ScanDesc& S = scans[s];
        const uint32_t* rc = rcum_flat.data() + S.req_begin;
        const uint64_t* rt = rthr_flat.data() + S.req_begin;
        double gpb = 0.0;
        uint32_t k = 0;
        for (uint64_t g = 0; 64 * g < rc[S.n_req]; ++g) {
            while (k + 1 <= S.n_req && rc[k + 1] <= 64 * g) ++k;
            gpb += S.thr_max ? (double)rt[k] / (double)S.thr_max : 0.0;
        }
        if (gpb < 1.0) gpb = 1.0;
        const uint32_t rows = std::max<uint32_t>(1024u, (uint32_t)((double)item_rows / gpb));
        if (S.thr_max == 0) continue;
        // the row-by-row scan reads every row of its items: they are sized by
        // rows and cut on tile boundaries
        S.fine = is_fine(S) ? 1u : 0u;
        uint64_t bb;
        if (S.fine) {
            const uint64_t per_tile = kZoneRows >> S.log2B;
            const uint64_t want = std::max<uint64_t>(kZoneRows, rows) >> S.log2B;
            bb = (want + per_tile - 1) / per_tile * per_tile;
        } else {
            bb = bpi_for(S.thr_max, S.log2B, rows);
            // a sparse scan in a small batch: items of one 64-block sampling
            // chunk, whose kept blocks beyond the first are spilled
            const double p_keep = S.thr_max >= kThrAll ? 1.0 : (double)S.thr_max / 4294967296.0;
            if (small_batch && p_keep * 64.0 <= (double)kSpillChunkKept) {
                S.spill = 1;
                any_spill = true;
                bb = 64;
            }
        }
        if (bb == 0) continue;
        const double p = S.fine ? 1.0 : S.thr_max >= kThrAll ? 1.0 : (double)S.thr_max / 4294967296.0;
        for (uint64_t b = 0; b < S.n_blocks; b += bb) {
            Item it = {IT_SCAN, s, 0, 0, b, std::min(S.n_blocks, b + bb)};
            scan_items.push_back(it);
            item_cost.push_back((double)(it.end - it.begin) * (double)(1ull << S.log2B) * p * S.row_bytes * gpb);
            out.est_scan_bytes += item_cost.back();
        }
    }
    {
        std::vector<uint32_t> order(scan_items.size());
        for (uint32_t i = 0; i < order.size(); ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(),
                         [&](uint32_t x, uint32_t y) { return item_cost[x] > item_cost[y]; });
        std::vector<Item> sorted;
        sorted.reserve(order.size());
        for (uint32_t i : order) sorted.push_back(scan_items[i]);
        scan_items.swap(sorted);
    }
    // scans form the first queue; the join partitioning queue follows in
    // phase order, so a join item only ever waits for items earlier in its
    // queue; the aggregation queue comes last (its kernel runs after the
    // partitioning kernel on the same stream)
    out.items.insert(out.items.end(), scan_items.begin(), scan_items.end());
    const uint32_t n_scan_items = (uint32_t)out.items.size();
    for (auto* v : {&heavy_items, &hist_items, &off_items, &base_items, &scatter_items, &scatter2_items})
        out.items.insert(out.items.end(), v->begin(), v->end());
    const uint32_t n_join_end = (uint32_t)out.items.size();
    out.items.insert(out.items.end(), agg_items.begin(), agg_items.end());

    // ---- plan blob
    PlanHdr H;
    std::memset(&H, 0, sizeof(H));
    H.n_scans = (uint32_t)scans.size();
    H.n_groups = (uint32_t)groups.size();
    H.n_cols = (uint32_t)cols.size();
    H.n_joins = (uint32_t)joins.size();
    H.n_counts = n_counts;
    H.n_hist = n_hist;
    H.n_items = (uint32_t)out.items.size();
    H.n_scan_items = n_scan_items;
    H.n_join_end = n_join_end;
    H.wg_done_off = wg_done_off;
    H.err_off = wg_done_off + 1;
    out.err_off = H.err_off;
    H.has_spill = any_spill ? 1u : 0u;
    H.spill_cap = 0;   // set at launch, from the room left in the item region
    H.arena_static = arena_static;
    std::vector<uint8_t>& blob = out.plan;
    {
        size_t est = sizeof(PlanHdr) + 16 * 16 + scans.size() * sizeof(ScanDesc) + groups.size() * sizeof(GroupDesc) +
                     cols.size() * sizeof(ColProg) + slots.size() * 4 + rthr_flat.size() * 8 + rcum_flat.size() * 4 +
                     joins.size() * sizeof(JoinDesc);
        for (const auto& t : tabs) est += t.size() + 16;
        blob.reserve(est);
    }
    blob.assign(sizeof(PlanHdr), 0);
    auto put = [&](const void* p, size_t nbytes) -> uint32_t {
        const uint32_t off = align_up((uint32_t)blob.size(), 16);
        blob.resize(off + nbytes);
        if (nbytes) std::memcpy(blob.data() + off, p, nbytes);
        return off;
    };
    // group tables first so their offsets are known when groups are written
    for (uint32_t g = 0; g < groups.size(); ++g) groups[g].tab_off = put(tabs[g].data(), tabs[g].size());
    H.scans_off = put(scans.data(), scans.size() * sizeof(ScanDesc));
    H.groups_off = put(groups.data(), groups.size() * sizeof(GroupDesc));
    H.cols_off = put(cols.data(), cols.size() * sizeof(ColProg));
    H.slots_off = put(slots.data(), slots.size() * sizeof(uint32_t));
    H.reqthr_off = put(rthr_flat.data(), rthr_flat.size() * sizeof(uint64_t));
    H.reqcum_off = put(rcum_flat.data(), rcum_flat.size() * sizeof(uint32_t));
    H.joins_off = put(joins.data(), joins.size() * sizeof(JoinDesc));
    blob.resize(align_up((uint32_t)blob.size(), 16));
    H.total_bytes = (uint32_t)blob.size();
    std::memcpy(blob.data(), &H, sizeof(H));

    out.scans = scans;
    out.jdesc = joins;
    out.n_counts = n_counts;
    out.n_hist = n_hist;
    out.arena_static = arena_static;
}

}  // namespace gace
