// kernels.hip -- gfx950 kernels of the probe library.
//
// One persistent kernel serves every request of a batch: workgroups pop work
// items from a device queue (plain calls are batches of one).  Item kinds:
//   SCAN     kept blocks of one table, all predicates of the requests sharing
//            the scan (selectivity probe, Sec. III-B; Exp. D "Key-Only +
//            Bitmask": only referenced columns are read, per-row predicate
//            bits are reduced in registers and never stored)
//   JSKETCH  HyperLogLog registers of the sampled join keys (sizes the table)
//   JSIZE    table capacity from the sketch, carved from the arena
//   JINIT    clear a slice of the join hash table
//   JBUILD   sampled keys -> per-workgroup LDS key cache -> global open-
//            addressing table (key-only aggregation, Sec. III-B)
//   JFINAL   slice of the table -> NDV (Eq. 1) and sum f_R f_S
// Items of a join wait on the previous phase's completion counter; the host
// orders the queue by phase, so every awaited item was popped earlier by a
// running workgroup and the waits always end.
#include <hip/hip_runtime.h>

#include "plan.h"

namespace gace {

constexpr int kWG = 256;
constexpr int kWaves = kWG / 64;
constexpr uint32_t kScanLdsGroups = 16;          // per-item LDS counters for the first 16 groups
constexpr uint32_t kLdsMisc = 512;
constexpr uint32_t kLdsCnt = kScanLdsGroups * 64 * 4;
constexpr uint32_t kLdsBytes = kLdsMisc + kLdsCnt + kGroupTabBudget;   // 45.5 KiB

struct BatchArgs {
    const uint8_t* plan;
    const Item* items;
    uint32_t* head;
    unsigned long long* counts;
    unsigned long long* hist;
    JoinAcc* accs;
    uint8_t* sketch;           // HLL rows
    uint8_t* arena_base;       // hash tables
    Arena* arena;
    uint32_t count_mode;       // 0 auto, 1 ballot, 2 transpose
    uint32_t cache_slots;      // join LDS key-cache slots (power of two <= 2048, 0 = off)
    uint64_t force_cap;        // nonzero: skip the sketch estimate and use this capacity
};

// ------------------------------------------------------------------ sampler
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): word 0 of the output
// for key = seed and counter = (block lo, block hi, table id, 0).
__device__ __forceinline__ uint32_t block_word0(uint64_t block, uint32_t table_id, uint64_t seed) {
    uint32_t x0 = (uint32_t)block, x1 = (uint32_t)(block >> 32), x2 = table_id, x3 = 0u;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t a = 0xD2511F53u * x0, ah = __umulhi(0xD2511F53u, x0);
        const uint32_t b = 0xCD9E8D57u * x2, bh = __umulhi(0xCD9E8D57u, x2);
        x0 = bh ^ x1 ^ k0;
        x2 = ah ^ x3 ^ k1;
        x1 = b;
        x3 = a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return x0;
}

// ------------------------------------------------------------------ keys
__device__ __forceinline__ uint32_t key32(uint32_t v, uint32_t xf) {
    if (xf == XF_I32) return v ^ 0x80000000u;
    if ((v << 1) == 0u) v = 0u;                       // -0.0 -> +0.0
    return (v & 0x80000000u) ? ~v : (v | 0x80000000u);
}

__device__ __forceinline__ uint32_t rank32(const uint32_t* bnd, uint32_t nb, uint32_t step, uint32_t k) {
    uint32_t pos = 0;
    for (; step; step >>= 1)
        if (pos + step <= nb && bnd[pos + step - 1] <= k) pos += step;
    return pos;
}

__device__ __forceinline__ uint32_t rank64(const uint64_t* bnd, uint32_t nb, uint32_t step, uint64_t k) {
    uint32_t pos = 0;
    for (; step; step >>= 1)
        if (pos + step <= nb && bnd[pos + step - 1] <= k) pos += step;
    return pos;
}

// predicate mask of row r for one group (bits of predicates whose every
// term on these columns holds)
__device__ __forceinline__ uint64_t eval_row(const ColProg* cp, uint32_t c0, uint32_t c1, const uint8_t* tab,
                                             uint64_t r) {
    uint64_t m = ~0ull;
    for (uint32_t c = c0; c < c1; ++c) {
        const ColProg P = cp[c];
        uint32_t idx;
        if (P.kind == CP_LUT32) {
            uint32_t k = key32(__builtin_nontemporal_load((const uint32_t*)P.data + r), P.xform);
            idx = min(max(k, P.lo), P.hi) - P.lo;
        } else if (P.kind == CP_RANK32) {
            uint32_t k = key32(__builtin_nontemporal_load((const uint32_t*)P.data + r), P.xform);
            idx = rank32((const uint32_t*)(tab + P.bnd_off), P.nb, P.step, k);
        } else {
            uint64_t k = __builtin_nontemporal_load((const uint64_t*)P.data + r) ^ 0x8000000000000000ull;
            idx = rank64((const uint64_t*)(tab + P.bnd_off), P.nb, P.step, k);
        }
        m &= ((const uint64_t*)(tab + P.mask_off))[idx];
    }
    return m;
}

// ------------------------------------------------------------------ counting
// 64x64 bit transpose across the wave: lane i holds row i's 64 predicate
// bits; afterwards lane j holds predicate j's bit for each of the 64 rows.
__device__ __forceinline__ void transpose64(uint32_t& lo, uint32_t& hi, int lane) {
    {
        const bool up = lane & 32;
        uint32_t r = __shfl_xor(up ? lo : hi, 32);
        if (up) lo = r; else hi = r;
    }
#define GACE_TSTAGE(S, M)                                                       \
    {                                                                           \
        const bool up = lane & S;                                               \
        const uint32_t km = up ? ~(uint32_t)(M) : (uint32_t)(M);                \
        uint32_t rl = __shfl_xor(lo & ~km, S);                                  \
        uint32_t rh = __shfl_xor(hi & ~km, S);                                  \
        lo = (lo & km) | (up ? (rl >> S) : (rl << S));                          \
        hi = (hi & km) | (up ? (rh >> S) : (rh << S));                          \
    }
    GACE_TSTAGE(16, 0x0000FFFFu)
    GACE_TSTAGE(8, 0x00FF00FFu)
    GACE_TSTAGE(4, 0x0F0F0F0Fu)
    GACE_TSTAGE(2, 0x33333333u)
    GACE_TSTAGE(1, 0x55555555u)
#undef GACE_TSTAGE
}

// add the 64 rows' bits to the per-lane counter (lane p counts predicate p)
__device__ __forceinline__ void count_rows(uint64_t m, uint64_t active, uint32_t& cnt, int lane, uint32_t mode) {
    const int na = __popcll(active);
    if (mode == 1 || (mode == 0 && na <= 6)) {
        uint64_t a = active;
        while (a) {
            const int p = __ffsll((long long)a) - 1;
            a &= a - 1;
            const uint32_t c = (uint32_t)__popcll(__ballot((m >> p) & 1ull));
            if (lane == p) cnt += c;
        }
    } else {
        uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
        transpose64(lo, hi, lane);
        cnt += (uint32_t)(__popc(lo) + __popc(hi));
    }
}

// wave 0 decides 64 consecutive blocks; fills s_w0[0..64) and s_keep
__device__ __forceinline__ void decide_blocks(uint64_t cb, uint64_t b_end, uint64_t thr, uint32_t table_id,
                                              uint64_t seed, uint32_t* s_w0, unsigned long long* s_keep) {
    if (threadIdx.x < 64) {
        const uint64_t b = cb + threadIdx.x;
        bool keep = false;
        uint32_t w0 = 0xFFFFFFFFu;
        if (b < b_end) {
            w0 = block_word0(b, table_id, seed);
            keep = (uint64_t)w0 < thr;
        }
        s_w0[threadIdx.x] = w0;
        const unsigned long long bal = __ballot(keep);
        if (threadIdx.x == 0) *s_keep = bal;
    }
}

// ------------------------------------------------------------------ scan item
__device__ void scan_item(const BatchArgs& a, const PlanHdr& H, const Item& it, uint8_t* lds) {
    const ScanDesc S = ((const ScanDesc*)(a.plan + H.scans_off))[it.idx];
    const GroupDesc* groups = (const GroupDesc*)(a.plan + H.groups_off) + S.group_begin;
    const ColProg* cols = (const ColProg*)(a.plan + H.cols_off);
    const uint32_t* slots = (const uint32_t*)(a.plan + H.slots_off);
    const uint64_t* rthr = (const uint64_t*)(a.plan + H.reqthr_off) + S.req_begin;
    const uint32_t* rcum = (const uint32_t*)(a.plan + H.reqcum_off) + S.req_begin;

    uint32_t* s_w0 = (uint32_t*)lds;
    unsigned long long* s_keep = (unsigned long long*)(lds + 256);
    int* s_staged = (int*)(lds + 264);
    uint32_t* s_cnt = (uint32_t*)(lds + kLdsMisc);
    uint8_t* s_tab = lds + kLdsMisc + kLdsCnt;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t n_lds_groups = S.n_groups < kScanLdsGroups ? S.n_groups : kScanLdsGroups;
    for (uint32_t i = threadIdx.x; i < n_lds_groups * 64; i += kWG) s_cnt[i] = 0;
    if (threadIdx.x == 0) *s_staged = -1;
    __syncthreads();

    const uint64_t B = 1ull << S.log2B;
    for (uint64_t cb = it.begin; cb < it.end; cb += 64) {
        decide_blocks(cb, it.end, S.thr_max, S.table_id, S.seed, s_w0, s_keep);
        __syncthreads();
        unsigned long long keep = *s_keep;
        while (keep) {
            const int j = __ffsll((long long)keep) - 1;
            keep &= keep - 1;
            const uint64_t b = cb + (uint64_t)j;
            const uint64_t w0 = s_w0[j];
            const uint64_t r0 = b * B;
            const uint64_t r1 = (r0 + B < S.n_rows) ? r0 + B : S.n_rows;
            // k = number of requests whose threshold exceeds word 0 (sorted descending)
            uint32_t k = 0;
            for (uint32_t step = 1u << 31; step; step >>= 1)
                if (k + step <= S.n_req && rthr[k + step - 1] > w0) k += step;
            if (threadIdx.x == 0) {
                atomicAdd(&a.hist[S.hist_off + 2 * k], (unsigned long long)(r1 - r0));
                atomicAdd(&a.hist[S.hist_off + 2 * k + 1], 1ull);
            }
            const uint32_t act_bits = rcum[k];
            for (uint32_t g = 0; g * 64 < act_bits; ++g) {
                const GroupDesc G = groups[g];
                const uint32_t na = act_bits - g * 64;
                const uint64_t active = G.base_mask & (na >= 64 ? ~0ull : ((1ull << na) - 1));
                if (active == 0) continue;
                const uint8_t* tab = a.plan + G.tab_off;
                if (G.tab_bytes <= kGroupTabBudget) {
                    if (*s_staged != (int)g) {
                        __syncthreads();
                        const uint4* src = (const uint4*)(a.plan + G.tab_off);
                        uint4* dst = (uint4*)s_tab;
                        for (uint32_t i = threadIdx.x; i < G.tab_bytes / 16; i += kWG) dst[i] = src[i];
                        __syncthreads();
                        if (threadIdx.x == 0) *s_staged = (int)g;
                    }
                    tab = s_tab;
                }
                uint32_t cnt = 0;
                for (uint64_t base = r0 + (uint64_t)wave * 64; base < r1; base += kWG) {
                    const uint64_t r = base + (uint64_t)lane;
                    uint64_t m = 0;
                    if (r < r1) m = eval_row(cols, G.col_begin, G.col_end, tab, r) & active;
                    count_rows(m, active, cnt, lane, a.count_mode);
                }
                if (cnt) {
                    if (g < n_lds_groups) atomicAdd(&s_cnt[g * 64 + lane], cnt);
                    else atomicAdd(&a.counts[slots[G.slot_index + lane]], (unsigned long long)cnt);
                }
                __syncthreads();   // the staged table may be replaced by the next group
            }
        }
        __syncthreads();
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n_lds_groups * 64; i += kWG) {
        const uint32_t c = s_cnt[i];
        if (c) atomicAdd(&a.counts[slots[groups[i >> 6].slot_index + (i & 63)]], (unsigned long long)c);
    }
}

// ------------------------------------------------------------------ joins
// MurmurHash3 64-bit finalizer (Appleby, public domain): a bijection on keys
__device__ __forceinline__ uint64_t mix_key(uint64_t k) {
    k ^= k >> 33;
    k *= 0xFF51AFD7ED558CCDull;
    k ^= k >> 33;
    k *= 0xC4CEB9FE1A85EC53ull;
    k ^= k >> 33;
    return k;
}

__device__ __forceinline__ bool table_add(Slot* T, uint64_t mask, uint64_t h, uint64_t key, int side, uint32_t c) {
    uint64_t i = h & mask;
    for (uint64_t p = 0; p <= mask; ++p) {
        unsigned long long* kp = (unsigned long long*)&T[i].key;
        unsigned long long k = __hip_atomic_load(kp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (k == key) {
            atomicAdd(&T[i].cnt[side], c);
            return true;
        }
        if (k == kEmptyKey) {
            unsigned long long prev = atomicCAS(kp, (unsigned long long)kEmptyKey, (unsigned long long)key);
            if (prev == kEmptyKey || prev == key) {
                atomicAdd(&T[i].cnt[side], c);
                return true;
            }
        }
        i = (i + 1) & mask;
    }
    return false;
}

__device__ __forceinline__ unsigned long long block_sum(unsigned long long v, unsigned long long* s_red) {
    for (int o = 32; o; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned long long t = 0;
    for (int w = 0; w < kWaves; ++w) t += s_red[w];
    return t;
}

__device__ void jsketch_item(const BatchArgs& a, const PlanHdr& H, const Item& it, uint8_t* lds) {
    const JoinDesc J = ((const JoinDesc*)(a.plan + H.joins_off))[it.idx];
    const JoinSide& D = J.side[it.side];
    uint32_t* s_w0 = (uint32_t*)lds;
    unsigned long long* s_keep = (unsigned long long*)(lds + 256);
    uint32_t* reg = (uint32_t*)(lds + kLdsMisc);
    const uint32_t M = 1u << kHllBits;
    for (uint32_t i = threadIdx.x; i < M; i += kWG) reg[i] = 0;
    __syncthreads();
    const uint64_t B = 1ull << D.log2B;
    for (uint64_t cb = it.begin; cb < it.end; cb += 64) {
        decide_blocks(cb, it.end, D.thr, D.table_id, D.seed, s_w0, s_keep);
        __syncthreads();
        unsigned long long keep = *s_keep;
        while (keep) {
            const int j = __ffsll((long long)keep) - 1;
            keep &= keep - 1;
            const uint64_t r0 = (cb + (uint64_t)j) * B;
            const uint64_t r1 = (r0 + B < D.n) ? r0 + B : D.n;
            for (uint64_t r = r0 + threadIdx.x; r < r1; r += kWG) {
                const uint64_t h = mix_key((uint64_t)__builtin_nontemporal_load(D.keys + r));
                const uint32_t idx = (uint32_t)(h >> (64 - kHllBits));
                const uint64_t w = h << kHllBits;
                const uint32_t rho = w ? (uint32_t)__clzll((long long)w) + 1u : (uint32_t)(65 - kHllBits);
                atomicMax(&reg[idx], rho);
            }
        }
        __syncthreads();
    }
    uint8_t* row = a.sketch + J.sketch_off + (uint64_t)it.sub * M;
    for (uint32_t i = threadIdx.x; i < M; i += kWG) row[i] = (uint8_t)reg[i];
}

__device__ void jsize_item(const BatchArgs& a, const PlanHdr& H, const Item& it, uint8_t* lds) {
    const JoinDesc J = ((const JoinDesc*)(a.plan + H.joins_off))[it.idx];
    JoinAcc& acc = a.accs[J.acc];
    double* s_sum = (double*)(lds + kLdsMisc);
    uint32_t* s_zero = (uint32_t*)(lds + kLdsMisc + kWG * 8);
    const uint32_t M = 1u << kHllBits;
    double sum = 0.0;
    uint32_t zeros = 0;
    for (uint32_t i = threadIdx.x; i < M; i += kWG) {
        uint32_t mx = 0;
        for (uint32_t s = 0; s < J.n_sketch; ++s) {
            const uint32_t v = a.sketch[J.sketch_off + (uint64_t)s * M + i];
            mx = v > mx ? v : mx;
        }
        sum += ldexp(1.0, -(int)mx);
        zeros += mx == 0;
    }
    s_sum[threadIdx.x] = sum;
    s_zero[threadIdx.x] = zeros;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        uint32_t z = 0;
        for (int i = 0; i < kWG; ++i) { t += s_sum[i]; z += s_zero[i]; }
        const double m = (double)M;
        double est = (0.7213 / (1.0 + 1.079 / m)) * m * m / t;          // Flajolet et al. 2007
        if (est <= 2.5 * m && z > 0) est = m * log(m / (double)z);       // small-range correction
        uint64_t want = (uint64_t)(2.5 * est) + 2048;
        uint64_t cap = 2048;
        while (cap < want && cap < J.cap_max) cap <<= 1;
        if (a.force_cap) cap = a.force_cap;
        if (cap > J.cap_max) cap = J.cap_max;
        const unsigned long long bytes = (unsigned long long)cap * sizeof(Slot);
        const unsigned long long off = atomicAdd(&a.arena->used, bytes);
        if (off + bytes > a.arena->size) acc.status = 2;
        acc.table_off = off;
        acc.cap = cap;
    }
}

__device__ void jinit_item(const BatchArgs& a, const PlanHdr& H, const Item& it) {
    const JoinDesc J = ((const JoinDesc*)(a.plan + H.joins_off))[it.idx];
    JoinAcc& acc = a.accs[J.acc];
    if (__hip_atomic_load(&acc.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const uint64_t cap = acc.cap;
    Slot* T = (Slot*)(a.arena_base + acc.table_off);
    const uint64_t s0 = cap * it.sub / kSlotChunks, s1 = cap * (it.sub + 1) / kSlotChunks;
    for (uint64_t i = s0 + threadIdx.x; i < s1; i += kWG) {
        Slot s;
        s.key = kEmptyKey;
        s.cnt[0] = 0;
        s.cnt[1] = 0;
        T[i] = s;
    }
}

__device__ void jbuild_item(const BatchArgs& a, const PlanHdr& H, const Item& it, uint8_t* lds) {
    const JoinDesc J = ((const JoinDesc*)(a.plan + H.joins_off))[it.idx];
    const JoinSide& D = J.side[it.side];
    JoinAcc& acc = a.accs[J.acc];
    const bool dead = __hip_atomic_load(&acc.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    const uint64_t mask = acc.cap - 1;
    Slot* T = (Slot*)(a.arena_base + acc.table_off);
    const int side = (int)it.side;

    uint32_t* s_w0 = (uint32_t*)lds;
    unsigned long long* s_keep = (unsigned long long*)(lds + 256);
    unsigned long long* s_red = (unsigned long long*)(lds + 320);
    const uint32_t CS = a.cache_slots;
    unsigned long long* ckey = (unsigned long long*)(lds + kLdsMisc);
    uint32_t* ccnt = (uint32_t*)(lds + kLdsMisc + (size_t)CS * 8);
    for (uint32_t i = threadIdx.x; i < CS; i += kWG) {
        ckey[i] = kEmptyKey;
        ccnt[i] = 0;
    }
    __syncthreads();

    unsigned long long n_local = 0, sent_local = 0, fail = 0;
    const uint64_t B = 1ull << D.log2B;
    for (uint64_t cb = it.begin; cb < it.end; cb += 64) {
        decide_blocks(cb, it.end, D.thr, D.table_id, D.seed, s_w0, s_keep);
        __syncthreads();
        unsigned long long keep = *s_keep;
        while (keep) {
            const int j = __ffsll((long long)keep) - 1;
            keep &= keep - 1;
            const uint64_t r0 = (cb + (uint64_t)j) * B;
            const uint64_t r1 = (r0 + B < D.n) ? r0 + B : D.n;
            for (uint64_t r = r0 + threadIdx.x; r < r1; r += kWG) {
                const uint64_t key = (uint64_t)__builtin_nontemporal_load(D.keys + r);
                n_local += 1;
                if (key == kEmptyKey) { sent_local += 1; continue; }
                if (dead) continue;
                const uint64_t h = mix_key(key);
                bool done = false;
                if (CS) {
                    uint32_t i = (uint32_t)(h >> 40) & (CS - 1);
                    for (int p = 0; p < 8 && !done; ++p) {
                        unsigned long long k = ckey[i];
                        if (k == kEmptyKey) k = atomicCAS(&ckey[i], (unsigned long long)kEmptyKey, key);
                        if (k == kEmptyKey || k == key) {
                            atomicAdd(&ccnt[i], 1u);
                            done = true;
                        }
                        i = (i + 1) & (CS - 1);
                    }
                }
                if (!done && !table_add(T, mask, h, key, side, 1u)) fail += 1;
            }
        }
        __syncthreads();
    }
    if (!dead) {
        for (uint32_t i = threadIdx.x; i < CS; i += kWG) {
            const unsigned long long k = ckey[i];
            if (k != kEmptyKey && ccnt[i] && !table_add(T, mask, mix_key(k), k, side, ccnt[i])) fail += 1;
        }
    }
    const unsigned long long n = block_sum(n_local, s_red);
    const unsigned long long sent = block_sum(sent_local, s_red);
    const unsigned long long f = block_sum(fail, s_red);
    if (threadIdx.x == 0) {
        atomicAdd(&acc.n[side], n);
        if (sent) atomicAdd(&acc.sent[side], sent);
        if (f) atomicMax(&acc.status, 1ull);
    }
}

__device__ void jfinal_item(const BatchArgs& a, const PlanHdr& H, const Item& it, uint8_t* lds) {
    const JoinDesc J = ((const JoinDesc*)(a.plan + H.joins_off))[it.idx];
    JoinAcc& acc = a.accs[J.acc];
    unsigned long long* s_red = (unsigned long long*)(lds + 320);
    unsigned long long jn = 0, n0 = 0, n1 = 0;
    if (!__hip_atomic_load(&acc.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        const uint64_t cap = acc.cap;
        const Slot* T = (const Slot*)(a.arena_base + acc.table_off);
        const uint64_t s0 = cap * it.sub / kSlotChunks, s1 = cap * (it.sub + 1) / kSlotChunks;
        for (uint64_t i = s0 + threadIdx.x; i < s1; i += kWG) {
            const Slot s = T[i];
            if (s.key != kEmptyKey) {
                n0 += s.cnt[0] != 0;
                n1 += s.cnt[1] != 0;
                jn += (unsigned long long)s.cnt[0] * s.cnt[1];
            }
        }
    }
    jn = block_sum(jn, s_red);
    n0 = block_sum(n0, s_red);
    n1 = block_sum(n1, s_red);
    if (threadIdx.x == 0) {
        if (jn) atomicAdd(&acc.join, jn);
        if (n0) atomicAdd(&acc.ndv[0], n0);
        if (n1) atomicAdd(&acc.ndv[1], n1);
        __threadfence();
        if (atomicAdd(&acc.final_done, 1u) == kSlotChunks - 1) {
            // last slice: the sentinel key, counted outside the table
            __threadfence();
            const unsigned long long s0 = atomicAdd(&acc.sent[0], 0ull), s1 = atomicAdd(&acc.sent[1], 0ull);
            if (s0 && s1) atomicAdd(&acc.join, s0 * s1);
            if (s0) atomicAdd(&acc.ndv[0], 1ull);
            if (s1) atomicAdd(&acc.ndv[1], 1ull);
        }
    }
}

// ------------------------------------------------------------------ kernels
__device__ __forceinline__ void wait_count(uint32_t* p, uint32_t target) {
    if (threadIdx.x == 0) {
        while (__hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target)
            __builtin_amdgcn_s_sleep(2);
    }
    __syncthreads();
    __threadfence();
}

__device__ __forceinline__ void signal_count(uint32_t* p) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(p, 1u);
    }
}

__global__ void __launch_bounds__(kWG) gace_batch_kernel(BatchArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    __shared__ uint32_t s_item;
    const PlanHdr H = *(const PlanHdr*)a.plan;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.head, 1u);
        __syncthreads();
        const uint32_t idx = s_item;
        __syncthreads();
        if (idx >= H.n_items) break;
        const Item it = a.items[idx];
        if (it.kind == IT_SCAN) {
            scan_item(a, H, it, lds);
            __syncthreads();
            continue;
        }
        const JoinDesc* jd = (const JoinDesc*)(a.plan + H.joins_off) + it.idx;
        JoinAcc& acc = a.accs[jd->acc];
        switch (it.kind) {
            case IT_JSKETCH:
                jsketch_item(a, H, it, lds);
                signal_count(&acc.sketch_done);
                break;
            case IT_JSIZE:
                wait_count(&acc.sketch_done, jd->n_sketch);
                jsize_item(a, H, it, lds);
                signal_count(&acc.size_done);
                break;
            case IT_JINIT:
                wait_count(&acc.size_done, 1);
                jinit_item(a, H, it);
                signal_count(&acc.init_done);
                break;
            case IT_JBUILD:
                wait_count(&acc.init_done, kSlotChunks);
                jbuild_item(a, H, it, lds);
                signal_count(&acc.build_done);
                break;
            case IT_JFINAL:
                wait_count(&acc.build_done, jd->n_build);
                jfinal_item(a, H, it, lds);
                break;
            default:
                break;
        }
        __syncthreads();
    }
}

// zero the per-batch accumulators (a kernel, not a memset, so it can be
// captured in a graph and replayed)
__global__ void __launch_bounds__(kWG) gace_init_kernel(const uint8_t* plan, uint32_t* head,
                                                        unsigned long long* counts, unsigned long long* hist,
                                                        JoinAcc* accs, Arena* arena) {
    const PlanHdr H = *(const PlanHdr*)plan;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = tid; i < H.n_counts; i += stride) counts[i] = 0;
    for (uint64_t i = tid; i < H.n_hist; i += stride) hist[i] = 0;
    const uint64_t nacc = (uint64_t)H.n_joins * (sizeof(JoinAcc) / 8);
    for (uint64_t i = tid; i < nacc; i += stride) ((unsigned long long*)accs)[i] = 0;
    if (tid == 0) {
        *head = 0;
        arena->used = 0;
    }
}

}  // namespace gace

extern "C" {

// launchers used by the host runtime (internal; not part of the public ABI)
hipError_t gace_launch_init(const void* plan, void* head, void* counts, void* hist, void* accs, void* arena,
                            hipStream_t stream) {
    hipLaunchKernelGGL(gace::gace_init_kernel, dim3(256), dim3(gace::kWG), 0, stream, (const uint8_t*)plan,
                       (uint32_t*)head, (unsigned long long*)counts, (unsigned long long*)hist,
                       (gace::JoinAcc*)accs, (gace::Arena*)arena);
    return hipGetLastError();
}

hipError_t gace_launch_batch(const void* args, uint32_t grid, hipStream_t stream) {
    const gace::BatchArgs& a = *(const gace::BatchArgs*)args;
    hipLaunchKernelGGL(gace::gace_batch_kernel, dim3(grid), dim3(gace::kWG), gace::kLdsBytes, stream, a);
    return hipGetLastError();
}

uint32_t gace_batch_lds_bytes(void) { return gace::kLdsBytes; }
uint32_t gace_batch_wg_threads(void) { return gace::kWG; }

}
