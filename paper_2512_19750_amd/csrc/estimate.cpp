// estimate.cpp -- population estimates scaled from the probe's sample counts
// (selectivity, Horvitz-Thompson cardinality and join size, GEE NDV).
#include <cmath>
#include <cstring>
#include <limits>
#include <string>

#include "../../include/gace_est.h"
#include "compile.h"
#include "runtime.h"

using gace::set_error;

namespace {

// inclusion probability of every row under block-Bernoulli sampling at the
// spec's threshold
bool inclusion(const gace_sample_spec* spec, double* p) {
    gace_sample_spec s;
    std::memset(&s, 0, sizeof(s));
    s.rate = 1.0;
    s.block_rows = 4096;
    if (spec) s = *spec;
    std::string msg;
    if (gace::check_spec(&s, msg) != GACE_OK) {
        set_error(msg);
        return false;
    }
    const uint64_t thr = gace::rate_threshold(s.rate);
    *p = thr >= (1ull << 32) ? 1.0 : (double)thr / 4294967296.0;
    return true;
}

// GEE (Charikar et al., PODS 2000): sqrt(n / r) f1 + (d - f1)
double gee(uint64_t n, uint64_t r, uint64_t d, uint64_t f1) {
    if (r == 0) return 0.0;
    return std::sqrt((double)n / (double)r) * (double)f1 + (double)(d - f1);
}

}  // namespace

extern "C" gace_status gace_estimate_selectivity(uint64_t count, const gace_probe_info* info, uint64_t n_rows,
                                                 const gace_sample_spec* spec, gace_sel_estimate* out) {
    if (!info || !out) {
        set_error("NULL argument");
        return GACE_EINVAL;
    }
    if (count > info->sampled_rows || info->sampled_rows > n_rows) {
        set_error("need count <= sampled_rows <= n_rows");
        return GACE_EINVAL;
    }
    double p = 0.0;
    if (!inclusion(spec, &p)) return GACE_EINVAL;
    const double nan = std::numeric_limits<double>::quiet_NaN();
    gace_sel_estimate e;
    e.p = p;
    e.sel = info->sampled_rows ? (double)count / (double)info->sampled_rows : nan;
    e.card = info->sampled_rows ? e.sel * (double)n_rows : nan;
    e.card_ht = p > 0.0 ? (double)count / p : nan;
    *out = e;
    return GACE_OK;
}

extern "C" gace_status gace_estimate_join(const gace_join_result* r, uint64_t n_rows_R, const gace_sample_spec* spec_R,
                                          uint64_t n_rows_S, const gace_sample_spec* spec_S, gace_join_estimate* out) {
    if (!r || !out || !spec_R || !spec_S) {
        set_error("NULL argument");
        return GACE_EINVAL;
    }
    if (r->n_R > n_rows_R || r->n_S > n_rows_S || r->ndv_R > r->n_R || r->ndv_S > r->n_S ||
        r->f1_R > r->ndv_R || r->f1_S > r->ndv_S || r->f2_R > r->ndv_R - r->f1_R ||
        r->f2_S > r->ndv_S - r->f1_S) {
        set_error("join counts inconsistent with the table sizes (need f1 + f2 <= ndv <= n <= rows)");
        return GACE_EINVAL;
    }
    gace_join_estimate e;
    if (!inclusion(spec_R, &e.p_R) || !inclusion(spec_S, &e.p_S)) return GACE_EINVAL;
    e.join_ht = e.p_R > 0.0 && e.p_S > 0.0 ? (double)r->join_card / (e.p_R * e.p_S)
                                           : std::numeric_limits<double>::quiet_NaN();
    e.ndv_R = gee(n_rows_R, r->n_R, r->ndv_R, r->f1_R);
    e.ndv_S = gee(n_rows_S, r->n_S, r->ndv_S, r->f1_S);
    *out = e;
    return GACE_OK;
}
