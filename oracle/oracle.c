/*
 * oracle.c -- plain CPU oracle (test infrastructure only; see oracle.h).
 *
 * Follows the problem statement of the Measurement Engine (arXiv 2512.19750,
 * Sec. III-B: selectivity and distribution of candidate conditions measured on
 * a sample, key-only aggregation) and the quantities the gate consumes (Eq. 1
 * NDV, Eq. 2 S_probe = count / n, Eq. 3 joint vs marginal probabilities).
 * No blocking, fusion or reordering beyond "for every kept row, for every
 * predicate, for every term".
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of the 4x32 Philox S-box, the key    */
/* bumped by the Weyl constants between rounds.                              */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* P(keep) = thr / 2^32 exactly; rate 1 means every block. */
uint64_t orc_threshold(double rate) {
    if (rate >= 1.0) return 4294967296ull;
    if (!(rate > 0.0)) return 0;
    return (uint64_t)floor(rate * 4294967296.0);
}

int orc_block_kept(uint64_t seed, uint32_t table_id, uint64_t block, uint64_t thr) {
    if (thr >= 4294967296ull) return 1;
    uint32_t ctr[4] = {(uint32_t)block, (uint32_t)(block >> 32), table_id, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return (uint64_t)out[0] < thr;
}

static int valid_block_rows(uint32_t b) { return b >= 1 && b <= (1u << 20) && (b & (b - 1)) == 0; }
static int valid_rate(double r) { return r >= 0.0 && r <= 1.0; }

uint64_t orc_kept_blocks(uint64_t n_rows, uint64_t seed, uint32_t table_id, double rate,
                         uint32_t block_rows, uint64_t* out, uint64_t cap) {
    if (!valid_block_rows(block_rows) || !valid_rate(rate)) return 0;
    uint64_t thr = orc_threshold(rate);
    uint64_t nb = (n_rows + block_rows - 1) / block_rows, k = 0;
    for (uint64_t b = 0; b < nb; ++b)
        if (orc_block_kept(seed, table_id, b, thr)) {
            if (k < cap) out[k] = b;
            ++k;
        }
    return k;
}

/* ------------------------------------------------------------------------ */
/* predicate terms                                                           */
/* ------------------------------------------------------------------------ */
static float bits_to_float(int64_t v) {
    union { uint32_t u; float f; } c;
    c.u = (uint32_t)(uint64_t)v;
    return c.f;
}

static int term_holds(const orc_term* t, const orc_col* cols, uint64_t row) {
    const orc_col* c = &cols[t->col];
    if (c->dtype == ORC_F32) {
        float x = ((const float*)c->data)[row];
        if (t->op == ORC_RANGE) return x >= bits_to_float(t->v[0]) && x < bits_to_float(t->v[1]);
        for (uint32_t i = 0; i < t->n_vals; ++i)
            if (x == bits_to_float(t->v[i])) return 1;
        return 0;
    }
    int64_t x = c->dtype == ORC_I32 ? (int64_t)((const int32_t*)c->data)[row]
                                    : ((const int64_t*)c->data)[row];
    if (t->op == ORC_RANGE) return t->v[0] <= x && x < t->v[1];
    for (uint32_t i = 0; i < t->n_vals; ++i)
        if (x == t->v[i]) return 1;
    return 0;
}

static int valid_terms(const orc_col* cols, uint32_t n_cols, const orc_term* terms,
                       const uint32_t* pred_off, uint32_t n_preds) {
    for (uint32_t c = 0; c < n_cols; ++c)
        if (cols[c].dtype < ORC_I32 || cols[c].dtype > ORC_F32) return 0;
    if (n_preds && (!terms || !pred_off || pred_off[0] != 0)) return 0;
    for (uint32_t p = 0; p < n_preds; ++p) {
        uint32_t a = pred_off[p], b = pred_off[p + 1];
        if (b <= a || b - a > 16) return 0;
        for (uint32_t i = a; i < b; ++i) {
            const orc_term* t = &terms[i];
            if (t->col >= n_cols) return 0;
            if (t->op == ORC_RANGE) { if (t->n_vals != 2) return 0; }
            else if (t->op == ORC_EQ) { if (t->n_vals != 1) return 0; }
            else if (t->op == ORC_IN) { if (t->n_vals < 1 || t->n_vals > 8) return 0; }
            else return 0;
            if (cols[t->col].dtype == ORC_F32)
                for (uint32_t k = 0; k < t->n_vals; ++k)
                    if (isnan(bits_to_float(t->v[k]))) return 0;
        }
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* selectivity probe                                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t n_rows, b_begin, b_end, thr, seed;
    uint32_t block_rows, table_id, n_preds;
    const orc_col* cols;
    const orc_term* terms;
    const uint32_t* pred_off;
    uint64_t* counts;      /* n_preds partials owned by this worker */
    uint64_t sampled, kept;
} sel_job;

static void* sel_worker(void* arg) {
    sel_job* j = (sel_job*)arg;
    for (uint64_t b = j->b_begin; b < j->b_end; ++b) {
        if (!orc_block_kept(j->seed, j->table_id, b, j->thr)) continue;
        j->kept += 1;
        uint64_t r0 = b * j->block_rows;
        uint64_t r1 = r0 + j->block_rows < j->n_rows ? r0 + j->block_rows : j->n_rows;
        for (uint64_t r = r0; r < r1; ++r) {
            j->sampled += 1;
            for (uint32_t p = 0; p < j->n_preds; ++p) {
                int all = 1;
                for (uint32_t t = j->pred_off[p]; t < j->pred_off[p + 1]; ++t)
                    if (!term_holds(&j->terms[t], j->cols, r)) { all = 0; break; }
                j->counts[p] += (uint64_t)all;
            }
        }
    }
    return NULL;
}

int orc_probe_selectivity(uint64_t n_rows, const orc_col* cols, uint32_t n_cols, uint32_t table_id,
                          const orc_term* terms, const uint32_t* pred_off, uint32_t n_preds,
                          uint64_t seed, double rate, uint32_t block_rows,
                          uint64_t* counts, uint64_t* sampled_rows, uint64_t* kept_blocks,
                          int nthreads) {
    if (!valid_block_rows(block_rows) || !valid_rate(rate)) return -1;
    if (n_cols && !cols) return -1;
    if (!valid_terms(cols, n_cols, terms, pred_off, n_preds)) return -1;
    if (n_rows && n_cols) {
        for (uint32_t c = 0; c < n_cols; ++c) if (!cols[c].data) return -1;
    }
    uint64_t thr = orc_threshold(rate);
    uint64_t nb = (n_rows + block_rows - 1) / block_rows;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((uint64_t)nthreads > nb) nthreads = nb ? (int)nb : 1;

    sel_job* jobs = (sel_job*)calloc((size_t)nthreads, sizeof(sel_job));
    uint64_t* part = (uint64_t*)calloc((size_t)nthreads * (n_preds ? n_preds : 1), sizeof(uint64_t));
    pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
    char* started = (char*)calloc((size_t)nthreads, 1);
    if (!jobs || !part || !th || !started) { free(jobs); free(part); free(th); free(started); return -2; }
    uint64_t per = (nb + (uint64_t)nthreads - 1) / (uint64_t)nthreads;
    for (int t = 0; t < nthreads; ++t) {
        sel_job* j = &jobs[t];
        j->n_rows = n_rows; j->thr = thr; j->seed = seed;
        j->b_begin = per * (uint64_t)t < nb ? per * (uint64_t)t : nb;
        j->b_end = j->b_begin + per < nb ? j->b_begin + per : nb;
        j->block_rows = block_rows; j->table_id = table_id; j->n_preds = n_preds;
        j->cols = cols; j->terms = terms; j->pred_off = pred_off;
        j->counts = part + (size_t)t * (n_preds ? n_preds : 1);
        if (nthreads > 1 && pthread_create(&th[t], NULL, sel_worker, j) == 0) started[t] = 1;
        else sel_worker(j);
    }
    uint64_t sampled = 0, kept = 0;
    for (uint32_t p = 0; p < n_preds; ++p) counts[p] = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (started[t]) pthread_join(th[t], NULL);
        sampled += jobs[t].sampled;
        kept += jobs[t].kept;
        for (uint32_t p = 0; p < n_preds; ++p) counts[p] += jobs[t].counts[p];
    }
    if (sampled_rows) *sampled_rows = sampled;
    if (kept_blocks) *kept_blocks = kept;
    free(jobs); free(part); free(th); free(started);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* join-key frequencies                                                      */
/* ------------------------------------------------------------------------ */

/* LSD radix sort on the order-preserving unsigned image of int64
   (sign bit flipped), four passes of 16 bits. */
int orc_sort_i64(int64_t* keys, uint64_t n) {
    if (n < 2) return 0;
    uint64_t* a = (uint64_t*)malloc(n * sizeof(uint64_t));
    uint64_t* b = (uint64_t*)malloc(n * sizeof(uint64_t));
    uint64_t* cnt = (uint64_t*)malloc(65536 * sizeof(uint64_t));
    if (!a || !b || !cnt) { free(a); free(b); free(cnt); return -2; }
    for (uint64_t i = 0; i < n; ++i) a[i] = (uint64_t)keys[i] ^ 0x8000000000000000ull;
    for (int pass = 0; pass < 4; ++pass) {
        int shift = 16 * pass;
        memset(cnt, 0, 65536 * sizeof(uint64_t));
        for (uint64_t i = 0; i < n; ++i) cnt[(a[i] >> shift) & 0xFFFF] += 1;
        uint64_t sum = 0;
        for (int d = 0; d < 65536; ++d) { uint64_t c = cnt[d]; cnt[d] = sum; sum += c; }
        for (uint64_t i = 0; i < n; ++i) b[cnt[(a[i] >> shift) & 0xFFFF]++] = a[i];
        uint64_t* t = a; a = b; b = t;
    }
    for (uint64_t i = 0; i < n; ++i) keys[i] = (int64_t)(a[i] ^ 0x8000000000000000ull);
    free(a); free(b); free(cnt);
    return 0;
}

/* copy the keys of the kept blocks (in block order) into a new array */
static int64_t* sample_keys(const int64_t* keys, uint64_t n, uint32_t tid, uint64_t seed, double rate,
                            uint32_t block_rows, uint64_t* n_out) {
    uint64_t thr = orc_threshold(rate);
    uint64_t nb = (n + block_rows - 1) / block_rows, m = 0;
    for (uint64_t b = 0; b < nb; ++b)
        if (orc_block_kept(seed, tid, b, thr)) {
            uint64_t r0 = b * block_rows, r1 = r0 + block_rows < n ? r0 + block_rows : n;
            m += r1 - r0;
        }
    int64_t* out = (int64_t*)malloc((m ? m : 1) * sizeof(int64_t));
    if (!out) return NULL;
    uint64_t k = 0;
    for (uint64_t b = 0; b < nb; ++b)
        if (orc_block_kept(seed, tid, b, thr)) {
            uint64_t r0 = b * block_rows, r1 = r0 + block_rows < n ? r0 + block_rows : n;
            for (uint64_t r = r0; r < r1; ++r) out[k++] = keys[r];
        }
    *n_out = m;
    return out;
}

int orc_join_freq(const int64_t* keys_r, uint64_t n_r, uint32_t tid_r, uint64_t seed_r, double rate_r,
                  uint32_t block_rows_r,
                  const int64_t* keys_s, uint64_t n_s, uint32_t tid_s, uint64_t seed_s, double rate_s,
                  uint32_t block_rows_s, uint64_t out[9]) {
    if (!valid_block_rows(block_rows_r) || !valid_block_rows(block_rows_s)) return -1;
    if (!valid_rate(rate_r) || !valid_rate(rate_s)) return -1;
    if ((n_r && !keys_r) || (n_s && !keys_s) || !out) return -1;
    /* sum f_R f_S <= n_R * n_S; refuse inputs where that bound is >= 2^64 */
    if (n_r && n_s && n_r > UINT64_MAX / n_s) return -3;

    uint64_t mr = 0, ms = 0;
    int64_t* r = sample_keys(keys_r, n_r, tid_r, seed_r, rate_r, block_rows_r, &mr);
    int64_t* s = sample_keys(keys_s, n_s, tid_s, seed_s, rate_s, block_rows_s, &ms);
    if (!r || !s || orc_sort_i64(r, mr) || orc_sort_i64(s, ms)) { free(r); free(s); return -2; }

    /* runs of equal keys in the sorted samples are the frequencies f(k);
       walk both run lists in key order */
    uint64_t ndv_r = 0, ndv_s = 0, join = 0, i = 0, j = 0;
    uint64_t f1_r = 0, f1_s = 0, f2_r = 0, f2_s = 0;   /* keys seen exactly once / twice */
    while (i < mr || j < ms) {
        int take_r, take_s;
        if (i < mr && j < ms) { take_r = r[i] <= s[j]; take_s = s[j] <= r[i]; }
        else { take_r = i < mr; take_s = j < ms; }
        int64_t k = take_r ? r[i] : s[j];
        uint64_t fr = 0, fs = 0;
        if (take_r) { while (i < mr && r[i] == k) { ++fr; ++i; } ndv_r += 1; }
        if (take_s) { while (j < ms && s[j] == k) { ++fs; ++j; } ndv_s += 1; }
        join += fr * fs;
        f1_r += fr == 1; f2_r += fr == 2;
        f1_s += fs == 1; f2_s += fs == 2;
    }
    out[0] = join; out[1] = ndv_r; out[2] = ndv_s; out[3] = mr; out[4] = ms;
    out[5] = f1_r; out[6] = f1_s; out[7] = f2_r; out[8] = f2_s;
    free(r); free(s);
    return 0;
}
