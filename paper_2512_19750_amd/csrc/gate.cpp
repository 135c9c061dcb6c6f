// gate.cpp -- the Risky Gate's trust metrics (Sec. III-C, Eqs. 1-3), the
// measurement-cost model and break-even point (Eq. 4, Sec. V item 2) and the
// probe-result cache (Sec. V item 3).  Host code over the probe library.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <deque>
#include <limits>
#include <list>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/gace_gate.h"
#include "compile.h"
#include "runtime.h"

using gace::set_error;

namespace {

constexpr uint64_t kCountLimit = 1ull << 48;   // keeps c_ab * n * den below 2^128

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

gace_sample_spec spec_or_default(const gace_sample_spec* s) {
    gace_sample_spec d;
    std::memset(&d, 0, sizeof(d));
    d.rate = 1.0;
    d.block_rows = 4096;
    return s ? *s : d;
}

}  // namespace

// ---------------------------------------------------------------- Risky Gate
extern "C" gace_status gace_gate_default_cfg(gace_gate_cfg* out) {
    if (!out) {
        set_error("NULL output");
        return GACE_EINVAL;
    }
    std::memset(out, 0, sizeof(*out));
    out->drift_min = 0.25;     // Sec. III-C, Eq. 1
    out->sel_err_max = 0.01;   // Eq. 2
    out->pcs_hi_num = 8;       // Eq. 3: 1.6
    out->pcs_hi_den = 5;
    out->pcs_lo_num = 7;       // Eq. 3: 0.7
    out->pcs_lo_den = 10;
    return GACE_OK;
}

extern "C" gace_status gace_gate_evaluate(const gace_gate_cfg* cfg, const gace_gate_in* in, gace_gate_out* out) {
    if (!cfg || !in || !out) {
        set_error("NULL argument");
        return GACE_EINVAL;
    }
    if (!finite_nonneg(cfg->drift_min) || !finite_nonneg(cfg->sel_err_max) || !cfg->pcs_hi_den ||
        !cfg->pcs_lo_den) {
        set_error("thresholds must be finite and >= 0, with nonzero PCS denominators");
        return GACE_EINVAL;
    }
    using u128 = unsigned __int128;
    if ((u128)cfg->pcs_lo_num * cfg->pcs_hi_den > (u128)cfg->pcs_hi_num * cfg->pcs_lo_den) {
        set_error("pcs_lo must not exceed pcs_hi");
        return GACE_EINVAL;
    }
    const double nan = std::numeric_limits<double>::quiet_NaN();
    gace_gate_out o;
    std::memset(&o, 0, sizeof(o));
    o.drift = o.sel_err = o.pcs = nan;
    if (in->have & GACE_GATE_DRIFT) {
        if (!std::isfinite(in->ndv_hist) || in->ndv_hist <= 0.0 || !finite_nonneg(in->ndv_est)) {
            set_error("drift needs a finite ndv_hist > 0 and a finite ndv_est >= 0");
            return GACE_EINVAL;
        }
        // Eq. 1
        o.drift = std::fabs(in->ndv_hist - in->ndv_est) / in->ndv_hist;
        if (o.drift >= cfg->drift_min) o.flags |= GACE_GATE_DRIFT;
    }
    if (in->have & GACE_GATE_SELERR) {
        if (!(in->s_est >= 0.0 && in->s_est <= 1.0) || in->count > in->n || in->n >= kCountLimit) {
            set_error("selectivity needs s_est in [0, 1], count <= n and n < 2^48");
            return GACE_EINVAL;
        }
        if (in->n == 0) {
            o.undefined |= GACE_GATE_SELERR;
        } else {
            // Eq. 2 with S_probe = count / n
            const double s_probe = (double)in->count / (double)in->n;
            o.sel_err = std::fabs(in->s_est - s_probe);
            if (o.sel_err > cfg->sel_err_max) o.flags |= GACE_GATE_SELERR;
        }
    }
    if (in->have & GACE_GATE_PCS) {
        const uint64_t ab = in->c_ab, a = in->c_a, b = in->c_b, n = in->n_pcs;
        if (n >= kCountLimit || ab > a || ab > b || a > n || b > n || a + b - ab > n) {
            set_error("correlation counts are inconsistent (need c_ab <= c_a, c_b <= n_pcs, "
                      "c_a + c_b - c_ab <= n_pcs, n_pcs < 2^48)");
            return GACE_EINVAL;
        }
        if (a == 0 || b == 0) {
            o.undefined |= GACE_GATE_PCS;
        } else {
            // Eq. 3: PCS = (c_ab / n) / ((c_a / n) (c_b / n)) = c_ab n / (c_a c_b),
            // compared with num / den exactly: c_ab n den  vs  num c_a c_b
            const u128 lhs = (u128)ab * n, rhs = (u128)a * b;
            if (lhs * cfg->pcs_hi_den > rhs * cfg->pcs_hi_num) o.flags |= GACE_GATE_PCS_HI;
            if (lhs * cfg->pcs_lo_den < rhs * cfg->pcs_lo_num) o.flags |= GACE_GATE_PCS_LO;
            o.pcs = ((double)ab * (double)n) / ((double)a * (double)b);
        }
    }
    o.trigger = o.flags ? 1u : 0u;
    *out = o;
    return GACE_OK;
}

extern "C" gace_status gace_probe_pcs(gace_ctx* ctx, const gace_table* table, const gace_predicates* pair,
                                      const gace_sample_spec* spec, gace_gate_in* out, void* stream) {
    if (!ctx || !table || !pair || !out || (pair->n_preds && (!pair->terms || !pair->pred_off))) {
        set_error("NULL argument");
        return GACE_EINVAL;
    }
    if (pair->n_preds != 2 || pair->pred_off[0] != 0 || pair->pred_off[1] > pair->pred_off[2]) {
        set_error("the PCS probe takes exactly two predicates A and B in CSR form");
        return GACE_EINVAL;
    }
    const uint32_t na = pair->pred_off[1], nb = pair->pred_off[2] - na;
    // candidate conditions {A, B, A AND B}: one sample, three counts
    std::vector<gace_term> terms(pair->terms, pair->terms + na + nb);
    terms.insert(terms.end(), pair->terms, pair->terms + na + nb);
    const uint32_t off[4] = {0, na, na + nb, 2 * (na + nb)};
    gace_predicates three;
    std::memset(&three, 0, sizeof(three));
    three.terms = terms.data();
    three.pred_off = off;
    three.n_preds = 3;
    uint64_t counts[3] = {0, 0, 0};
    gace_probe_info info{};
    const gace_status st = gace_probe_selectivity(ctx, table, &three, spec, counts, &info, stream);
    if (st != GACE_OK) return st;
    out->have |= GACE_GATE_PCS;
    out->c_a = counts[0];
    out->c_b = counts[1];
    out->c_ab = counts[2];
    out->n_pcs = info.sampled_rows;
    return GACE_OK;
}

// ---------------------------------------------------------------- cost model
struct gace_cost_model {
    std::mutex mu;
    double prior_ms = 0.85;
    uint32_t window = 0;
    std::deque<std::array<double, 4>> obs;    // x0 = 1, x1 = N * row_bytes, x2 = N * terms, y = ms
    double coef[3] = {0.0, 0.0, 0.0};
    bool dirty = true;
};

namespace {

// least squares on the feature subset `mask` (columns scaled to unit RMS);
// false when the subset's normal matrix is singular
bool lsq_subset(const std::deque<std::array<double, 4>>& obs, unsigned mask, const long double scale[3],
                long double beta[3], long double* rss) {
    int idx[3], k = 0;
    for (int j = 0; j < 3; ++j)
        if (mask & (1u << j)) idx[k++] = j;
    long double A[3][4] = {};
    for (const auto& o : obs) {
        long double x[3];
        for (int a = 0; a < k; ++a) x[a] = (long double)o[idx[a]] / scale[idx[a]];
        for (int a = 0; a < k; ++a) {
            for (int b = 0; b < k; ++b) A[a][b] += x[a] * x[b];
            A[a][k] += x[a] * (long double)o[3];
        }
    }
    long double trace = 0.0L;
    for (int a = 0; a < k; ++a) trace += A[a][a];
    // Gaussian elimination with partial pivoting
    for (int c = 0; c < k; ++c) {
        int p = c;
        for (int r = c + 1; r < k; ++r)
            if (fabsl(A[r][c]) > fabsl(A[p][c])) p = r;
        if (fabsl(A[p][c]) <= 1e-13L * (trace > 0 ? trace : 1.0L)) return false;
        if (p != c)
            for (int j = 0; j <= k; ++j) std::swap(A[p][j], A[c][j]);
        for (int r = c + 1; r < k; ++r) {
            const long double f = A[r][c] / A[c][c];
            for (int j = c; j <= k; ++j) A[r][j] -= f * A[c][j];
        }
    }
    long double sol[3] = {0.0L, 0.0L, 0.0L};
    for (int c = k - 1; c >= 0; --c) {
        long double s = A[c][k];
        for (int j = c + 1; j < k; ++j) s -= A[c][j] * sol[j];
        sol[c] = s / A[c][c];
    }
    for (int j = 0; j < 3; ++j) beta[j] = 0.0L;
    for (int a = 0; a < k; ++a) beta[idx[a]] = sol[a] / scale[idx[a]];
    long double r2 = 0.0L;
    for (const auto& o : obs) {
        const long double e = (long double)o[3] - (beta[0] * o[0] + beta[1] * o[1] + beta[2] * o[2]);
        r2 += e * e;
    }
    *rss = r2;
    return true;
}

// non-negative least squares for three unknowns: the optimum is the plain
// least-squares solution on its own support, so the best feasible one over
// all supports is it
void refit(gace_cost_model* m) {
    if (!m->dirty) return;
    m->dirty = false;
    if (m->obs.size() < 3) {
        m->coef[0] = m->prior_ms;
        m->coef[1] = m->coef[2] = 0.0;
        return;
    }
    long double scale[3] = {0.0L, 0.0L, 0.0L};
    for (const auto& o : m->obs)
        for (int j = 0; j < 3; ++j) scale[j] += (long double)o[j] * o[j];
    for (int j = 0; j < 3; ++j) scale[j] = scale[j] > 0 ? sqrtl(scale[j] / m->obs.size()) : 1.0L;
    long double best_rss = 0.0L;
    long double y2 = 0.0L;
    for (const auto& o : m->obs) y2 += (long double)o[3] * o[3];
    best_rss = y2;                       // the empty support: c = 0
    long double best[3] = {0.0L, 0.0L, 0.0L};
    for (unsigned mask = 1; mask < 8; ++mask) {
        long double beta[3], rss;
        if (!lsq_subset(m->obs, mask, scale, beta, &rss)) continue;
        if (beta[0] < 0 || beta[1] < 0 || beta[2] < 0) continue;
        if (rss < best_rss) {
            best_rss = rss;
            for (int j = 0; j < 3; ++j) best[j] = beta[j];
        }
    }
    for (int j = 0; j < 3; ++j) m->coef[j] = (double)best[j];
}

bool features_ok(const gace_cost_features* f) {
    return f && finite_nonneg(f->n_rows) && finite_nonneg(f->row_bytes) && finite_nonneg(f->terms);
}

}  // namespace

extern "C" gace_status gace_cost_create(double prior_ms, uint32_t window, gace_cost_model** out) {
    if (!out || !finite_nonneg(prior_ms) || window < 3 || window > (1u << 20)) {
        set_error("cost model needs an output pointer, a finite prior_ms >= 0 and 3 <= window <= 2^20");
        return GACE_EINVAL;
    }
    gace_cost_model* m = new (std::nothrow) gace_cost_model();
    if (!m) {
        set_error("out of host memory");
        return GACE_ENOMEM;
    }
    m->prior_ms = prior_ms;
    m->window = window;
    *out = m;
    return GACE_OK;
}

extern "C" gace_status gace_cost_destroy(gace_cost_model* m) {
    delete m;
    return GACE_OK;
}

extern "C" gace_status gace_cost_observe(gace_cost_model* m, const gace_cost_features* f, double ms) {
    if (!m || !features_ok(f) || !finite_nonneg(ms)) {
        set_error("observation needs finite, non-negative features and latency");
        return GACE_EINVAL;
    }
    std::lock_guard<std::mutex> g(m->mu);
    m->obs.push_back({1.0, f->n_rows * f->row_bytes, f->n_rows * f->terms, ms});
    while (m->obs.size() > m->window) m->obs.pop_front();
    m->dirty = true;
    return GACE_OK;
}

extern "C" gace_status gace_cost_coef(gace_cost_model* m, double coef[3], uint32_t* n_obs) {
    if (!m || !coef) {
        set_error("NULL argument");
        return GACE_EINVAL;
    }
    std::lock_guard<std::mutex> g(m->mu);
    refit(m);
    for (int j = 0; j < 3; ++j) coef[j] = m->coef[j];
    if (n_obs) *n_obs = (uint32_t)m->obs.size();
    return GACE_OK;
}

extern "C" gace_status gace_cost_predict(gace_cost_model* m, const gace_cost_features* f, double* ms) {
    if (!m || !features_ok(f) || !ms) {
        set_error("prediction needs a model, finite non-negative features and an output");
        return GACE_EINVAL;
    }
    std::lock_guard<std::mutex> g(m->mu);
    refit(m);
    *ms = m->coef[0] + m->coef[1] * (f->n_rows * f->row_bytes) + m->coef[2] * (f->n_rows * f->terms);
    return GACE_OK;
}

extern "C" gace_status gace_cost_features_of(const gace_request* req, gace_cost_features* out) {
    if (!req || !out) {
        set_error("NULL argument");
        return GACE_EINVAL;
    }
    std::string msg;
    const gace_status st = gace::check_request(req, msg);
    if (st != GACE_OK) {
        set_error(msg);
        return st;
    }
    gace_cost_features f;
    std::memset(&f, 0, sizeof(f));
    if (req->kind == GACE_REQ_SELECTIVITY) {
        const gace_predicates& p = req->preds;
        std::vector<uint8_t> used(req->table.n_cols, 0);
        for (uint32_t t = 0; t < p.pred_off[p.n_preds]; ++t) used[p.terms[t].col] = 1;
        for (uint32_t c = 0; c < req->table.n_cols; ++c)
            if (used[c]) f.row_bytes += req->table.cols[c].dtype == GACE_I64 ? 8.0 : 4.0;
        f.terms = (double)p.pred_off[p.n_preds];
        f.n_rows = req->spec.rate * (double)req->table.n_rows;
    } else {
        f.row_bytes = 8.0;
        f.n_rows = req->R.spec.rate * (double)req->R.n + req->S.spec.rate * (double)req->S.n;
    }
    *out = f;
    return GACE_OK;
}

extern "C" gace_status gace_cost_breakeven(gace_cost_model* device, gace_cost_model* host, double row_bytes,
                                           double terms, double* n_star) {
    if (!device || !host || !n_star || !finite_nonneg(row_bytes) || !finite_nonneg(terms)) {
        set_error("break-even needs two models, finite non-negative row_bytes / terms and an output");
        return GACE_EINVAL;
    }
    double g[3], h[3];
    gace_cost_coef(device, g, nullptr);
    gace_cost_coef(host, h, nullptr);
    // offloading pays for every N >= N*: g0 + sg N <= h0 + sh N
    const double sg = g[1] * row_bytes + g[2] * terms, sh = h[1] * row_bytes + h[2] * terms;
    if (sg < sh) {
        *n_star = std::max(0.0, (g[0] - h[0]) / (sh - sg));
    } else if (sg == sh && g[0] <= h[0]) {
        *n_star = 0.0;
    } else {
        *n_star = std::numeric_limits<double>::infinity();
    }
    return GACE_OK;
}

// ---------------------------------------------------------------- result cache
struct gace_cache {
    struct Entry {
        uint32_t table_ids[2];
        uint32_t n_tables;
        uint64_t count;
        gace_probe_info info;
        gace_join_result join;
        std::list<std::string>::iterator lru;
    };
    std::mutex mu;
    uint64_t capacity = 0;
    std::list<std::string> order;                         // most recent first
    std::unordered_map<std::string, Entry> map;
    gace_cache_stats st{};
};

namespace {

void put(std::string& s, const void* p, size_t n) { s.append((const char*)p, n); }
template <typename T>
void put(std::string& s, T v) { put(s, &v, sizeof(v)); }

void put_sample(std::string& s, const gace_sample_spec& sp) {
    put(s, sp.seed);
    put(s, (uint64_t)gace::rate_threshold(sp.rate));
    put(s, sp.block_rows);
}

// key of predicate p: the table identity, the sample and the predicate's
// terms as a sorted list (a conjunction does not depend on term order; an
// IN list is a set)
std::string sel_key(const gace_table* t, const gace_predicates* ps, const gace_sample_spec& sp, uint32_t p) {
    std::vector<std::string> terms;
    for (uint32_t i = ps->pred_off[p]; i < ps->pred_off[p + 1]; ++i) {
        const gace_term& tm = ps->terms[i];
        std::vector<int64_t> v(tm.v, tm.v + tm.n_vals);
        if (tm.op == GACE_IN) {
            std::sort(v.begin(), v.end());
            v.erase(std::unique(v.begin(), v.end()), v.end());
        }
        std::string e;
        put(e, (uint64_t)(uintptr_t)t->cols[tm.col].data);
        put(e, t->cols[tm.col].dtype);
        put(e, tm.op);
        put(e, (uint32_t)v.size());
        for (int64_t x : v) put(e, x);
        terms.push_back(std::move(e));
    }
    std::sort(terms.begin(), terms.end());
    std::string k("S");
    put(k, t->table_id);
    put(k, t->n_rows);
    put_sample(k, sp);
    put(k, (uint32_t)terms.size());
    for (const std::string& e : terms) {
        put(k, (uint32_t)e.size());
        k += e;
    }
    return k;
}

std::string join_key(const gace_keys* R, const gace_keys* S) {
    std::string k("J");
    for (const gace_keys* s : {R, S}) {
        put(k, (uint64_t)(uintptr_t)s->keys);
        put(k, s->n);
        put(k, s->table_id);
        put_sample(k, s->spec);
    }
    return k;
}

gace_cache::Entry* find(gace_cache* c, const std::string& k) {
    auto it = c->map.find(k);
    if (it == c->map.end()) return nullptr;
    c->order.splice(c->order.begin(), c->order, it->second.lru);
    return &it->second;
}

void store(gace_cache* c, const std::string& k, const gace_cache::Entry& e) {
    auto it = c->map.find(k);
    if (it != c->map.end()) {
        auto lru = it->second.lru;
        it->second = e;
        it->second.lru = lru;
        c->order.splice(c->order.begin(), c->order, lru);
    } else {
        c->order.push_front(k);
        gace_cache::Entry x = e;
        x.lru = c->order.begin();
        c->map.emplace(k, x);
    }
    c->st.inserts += 1;
    while (c->map.size() > c->capacity) {
        c->map.erase(c->order.back());
        c->order.pop_back();
        c->st.evictions += 1;
    }
}

gace_status check_sel(const gace_table* t, const gace_predicates* p, const gace_sample_spec& sp) {
    std::string msg;
    const gace_status st = gace::check_selectivity(t, p, &sp, msg);
    if (st != GACE_OK) set_error(msg);
    return st;
}

}  // namespace

extern "C" gace_status gace_cache_create(uint64_t capacity, gace_cache** out) {
    if (!out || capacity == 0) {
        set_error("cache needs an output pointer and a capacity >= 1");
        return GACE_EINVAL;
    }
    gace_cache* c = new (std::nothrow) gace_cache();
    if (!c) {
        set_error("out of host memory");
        return GACE_ENOMEM;
    }
    c->capacity = capacity;
    *out = c;
    return GACE_OK;
}

extern "C" gace_status gace_cache_destroy(gace_cache* c) {
    delete c;
    return GACE_OK;
}

extern "C" gace_status gace_cache_lookup(gace_cache* c, const gace_table* table, const gace_predicates* preds,
                                         const gace_sample_spec* spec, uint64_t* counts, uint8_t* hit,
                                         gace_probe_info* info, uint32_t* n_hit) {
    if (!c || !table || !preds || (preds->n_preds && (!counts || !hit)) || !n_hit) {
        set_error("NULL argument");
        return GACE_EINVAL;
    }
    const gace_sample_spec sp = spec_or_default(spec);
    gace_status st = check_sel(table, preds, sp);
    if (st != GACE_OK) return st;
    std::lock_guard<std::mutex> g(c->mu);
    uint32_t nh = 0;
    const gace_cache::Entry* any = nullptr;
    for (uint32_t p = 0; p < preds->n_preds; ++p) {
        const gace_cache::Entry* e = find(c, sel_key(table, preds, sp, p));
        hit[p] = e ? 1 : 0;
        if (e) {
            counts[p] = e->count;
            any = e;
            nh += 1;
        }
    }
    c->st.hits += nh;
    c->st.misses += preds->n_preds - nh;
    if (any && info) *info = any->info;
    *n_hit = nh;
    return GACE_OK;
}

extern "C" gace_status gace_cache_insert(gace_cache* c, const gace_table* table, const gace_predicates* preds,
                                         const gace_sample_spec* spec, const uint64_t* counts,
                                         const gace_probe_info* info) {
    if (!c || !table || !preds || (preds->n_preds && !counts) || !info) {
        set_error("NULL argument");
        return GACE_EINVAL;
    }
    const gace_sample_spec sp = spec_or_default(spec);
    gace_status st = check_sel(table, preds, sp);
    if (st != GACE_OK) return st;
    std::lock_guard<std::mutex> g(c->mu);
    for (uint32_t p = 0; p < preds->n_preds; ++p) {
        gace_cache::Entry e{};
        e.table_ids[0] = table->table_id;
        e.n_tables = 1;
        e.count = counts[p];
        e.info = *info;
        store(c, sel_key(table, preds, sp, p), e);
    }
    c->st.entries = c->map.size();
    return GACE_OK;
}

extern "C" gace_status gace_cache_invalidate(gace_cache* c, uint32_t table_id) {
    if (!c) {
        set_error("NULL cache");
        return GACE_EINVAL;
    }
    std::lock_guard<std::mutex> g(c->mu);
    for (auto it = c->map.begin(); it != c->map.end();) {
        const gace_cache::Entry& e = it->second;
        bool drop = false;
        for (uint32_t i = 0; i < e.n_tables; ++i) drop |= e.table_ids[i] == table_id;
        if (drop) {
            c->order.erase(e.lru);
            it = c->map.erase(it);
            c->st.invalidated += 1;
        } else {
            ++it;
        }
    }
    c->st.entries = c->map.size();
    return GACE_OK;
}

extern "C" gace_status gace_cache_stats_get(gace_cache* c, gace_cache_stats* out) {
    if (!c || !out) {
        set_error("NULL argument");
        return GACE_EINVAL;
    }
    std::lock_guard<std::mutex> g(c->mu);
    c->st.entries = c->map.size();
    *out = c->st;
    return GACE_OK;
}

extern "C" gace_status gace_probe_selectivity_cached(gace_ctx* ctx, gace_cache* c, const gace_table* table,
                                                     const gace_predicates* preds, const gace_sample_spec* spec,
                                                     uint64_t* counts, gace_probe_info* info, uint32_t* n_hit,
                                                     void* stream) {
    if (!ctx || !c || !table || !preds || (preds->n_preds && !counts)) {
        set_error("NULL argument");
        return GACE_EINVAL;
    }
    const uint32_t np = preds->n_preds;
    std::vector<uint64_t> got(np, 0);
    std::vector<uint8_t> hit(np, 0);
    gace_probe_info hinfo{};
    uint32_t nh = 0;
    gace_status st = gace_cache_lookup(c, table, preds, spec, got.data(), hit.data(), &hinfo, &nh);
    if (st != GACE_OK) return st;
    gace_probe_info pinfo = hinfo;
    if (nh < np || np == 0) {
        // one probe of the predicates that missed
        std::vector<gace_term> terms;
        std::vector<uint32_t> off(1, 0);
        std::vector<uint32_t> which;
        for (uint32_t p = 0; p < np; ++p) {
            if (hit[p]) continue;
            terms.insert(terms.end(), preds->terms + preds->pred_off[p], preds->terms + preds->pred_off[p + 1]);
            off.push_back((uint32_t)terms.size());
            which.push_back(p);
        }
        gace_predicates miss;
        std::memset(&miss, 0, sizeof(miss));
        miss.terms = terms.data();
        miss.pred_off = off.data();
        miss.n_preds = (uint32_t)which.size();
        std::vector<uint64_t> mc(std::max<size_t>(which.size(), 1), 0);
        st = gace_probe_selectivity(ctx, table, &miss, spec, mc.data(), &pinfo, stream);
        if (st != GACE_OK) return st;
        st = gace_cache_insert(c, table, &miss, spec, mc.data(), &pinfo);
        if (st != GACE_OK) return st;
        for (size_t i = 0; i < which.size(); ++i) got[which[i]] = mc[i];
    }
    for (uint32_t p = 0; p < np; ++p) counts[p] = got[p];
    if (info) *info = pinfo;
    if (n_hit) *n_hit = nh;
    return GACE_OK;
}

extern "C" gace_status gace_join_freq_cached(gace_ctx* ctx, gace_cache* c, const gace_keys* R, const gace_keys* S,
                                             gace_join_result* out, uint32_t* hit, void* stream) {
    if (!ctx || !c || !R || !S || !out) {
        set_error("NULL argument");
        return GACE_EINVAL;
    }
    std::string msg;
    gace_status st = gace::check_join(R, S, msg);
    if (st != GACE_OK) {
        set_error(msg);
        return st;
    }
    const std::string k = join_key(R, S);
    {
        std::lock_guard<std::mutex> g(c->mu);
        const gace_cache::Entry* e = find(c, k);
        if (e) {
            c->st.hits += 1;
            *out = e->join;
            if (hit) *hit = 1;
            return GACE_OK;
        }
        c->st.misses += 1;
    }
    gace_join_result r{};
    st = gace_join_freq(ctx, R, S, &r, stream);
    if (st != GACE_OK) return st;
    {
        std::lock_guard<std::mutex> g(c->mu);
        gace_cache::Entry e{};
        e.table_ids[0] = R->table_id;
        e.table_ids[1] = S->table_id;
        e.n_tables = 2;
        e.join = r;
        store(c, k, e);
        c->st.entries = c->map.size();
    }
    *out = r;
    if (hit) *hit = 0;
    return GACE_OK;
}
