// kernels.hip -- gfx950 kernels of the probe library.
//
// One persistent kernel serves every request of a batch: workgroups pop work
// items from a device queue (plain calls are batches of one).  Item kinds:
//   SCAN     kept blocks of one table, all predicates of the requests sharing
//            the scan (selectivity probe, Sec. III-B; Exp. D "Key-Only +
//            Bitmask": only referenced columns are read, per-row predicate
//            bits are reduced in registers and never stored); in a small
//            batch, a sparse scan's item keeps its chunk's first kept block
//            and spills the others to a list that idle workgroups run
//   JHEAVY   a join's heavy-hitter table, from a small sample of its keys
//   JHIST    per-item hash-partition counts of the sampled join keys (heavy
//            keys counted per table slot instead)
//   JOFF     per-item offsets inside each partition
//   JBASE    partition starts; the partition buffer is carved from the arena
//   JSCATTER sampled keys other than heavy ones -> their hash partitions
//            (or first-pass buckets when the fan-out needs two passes)
//   JSCATTER2 each first-pass bucket of a group of items -> its partitions
//   JAGG     each partition aggregated in an LDS key table -> f_R(k), f_S(k)
//            -> NDV (Eq. 1) and sum f_R f_S (key-only aggregation, Sec. III-B)
// Items of a join wait on the previous phase's completion counter; the host
// orders the queue by phase, so every awaited item was popped earlier by a
// running workgroup and the waits always end.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "plan.h"

namespace gace {

constexpr int kWG = 256;
constexpr int kHeads = 6;                        // queue heads and counters (BatchArgs::head)
constexpr int kWaves = kWG / 64;
constexpr uint32_t kScanLdsGroups = 32;          // per-item LDS counters for the first 32 groups
constexpr uint32_t kScanLdsHist = 128;           // per-item LDS sample histogram for scans of < 128 requests
constexpr uint32_t kLdsMisc = 768;
constexpr uint32_t kLdsCnt = kScanLdsGroups * 64 * 4;
constexpr uint32_t kLdsHist = kScanLdsHist * 2 * 8;
constexpr uint32_t kLdsThr = kScanLdsHist * 8 + 640;                             // thresholds + bit prefix sums
constexpr uint32_t kLdsBytes = kLdsMisc + kLdsCnt + kLdsHist + kLdsThr + kGroupTabBudget;   // scan kernel
// partitioning tiles: kWG * KP keys, KP staged keys per thread (kTileKeys
// or half of it; see gace_join_kernel)
constexpr int kPerBig = kTileKeys / kWG;
constexpr int kPerSmall = kTileKeys / 2 / kWG;
constexpr uint32_t tile_lds_bytes(uint32_t keys) { return 3 * 132 * 4 + keys * 12; }   // cursors, counts, starts, tile
constexpr uint32_t kBaseLdsBytes = ((1u << kPartBitsMax) + 1) * 4;                     // one side's partition starts
constexpr uint32_t lds_max(uint32_t x, uint32_t y) { return x > y ? x : y; }
// the heavy-hitter table (hashes, then the histogram items' per-slot counts)
// sits above both a partitioning tile and a histogram row of the most
// partitions; the sampling phase's counting table fits below it
constexpr uint32_t heavy_lds_off(uint32_t keys) {
    return (kLdsMisc + lds_max(tile_lds_bytes(keys), lds_max(kBaseLdsBytes, (1u << kPartBitsMax) * 4)) + 15) / 16 * 16;
}
constexpr uint32_t join_lds_bytes(uint32_t keys) { return heavy_lds_off(keys) + kHeavySlots * 12; }
static_assert(kHeavyCount * 12 <= (1u << kPartBitsMax) * 4 && heavy_lds_off(kTileKeys / 2) % 16 == 0 &&
                  heavy_lds_off(kTileKeys) % 16 == 0,
              "heavy-hitter LDS layout");

// explicit address spaces: pointers read from the plan are generic to the
// compiler; global loads through them must not become flat loads, which would
// make every LDS wait also wait for the loads in flight
#define GACE_GLOBAL __attribute__((address_space(1)))
// the plan is written before a launch and only read by the kernels: read
// through the constant address space, uniform plan fields become scalar loads,
// which do not wait behind the vector loads a wave has in flight
#define GACE_CONST __attribute__((address_space(4)))
#define GACE_LDS __attribute__((address_space(3)))

struct BatchArgs {
    const uint8_t* plan;
    const Item* items;
    uint32_t* head;            // [0] scan queue, [1] join partitioning queue, [2] aggregation queue,
                               // [3] spill entries claimed, [4] spill entries taken, [5] scan items done
    unsigned long long* counts;
    unsigned long long* hist;
    JoinAcc* accs;
    uint8_t* arena_base;       // join tables and partition buffers
    Arena* arena;
    uint32_t count_mode;       // 0 auto, 1 ballot, 2 adder tree + transpose per bit plane
    uint32_t agg_slots;        // aggregation kernel: LDS table slots (power of two)
    TraceRec* trace;           // one record per item when the plan asks for tracing
    uint64_t spin_limit;       // polls before a join's phase wait gives up (0: at once)
    uint8_t* host_res;         // device address of the pinned result buffer (per-request completion)
    uint32_t* host_flags;      // device address of the pinned completion flags
};

// the batch's work items: in the plan buffer after the descriptors when they
// fit there (one upload), else in their own region
__device__ __forceinline__ const Item* batch_items(const BatchArgs& a, const PlanHdr& H) {
    return H.items_off ? (const Item*)(a.plan + H.items_off) : a.items;
}

// relaxed device-scope read of a value other workgroups updated with atomics
__device__ __forceinline__ unsigned long long load_agent(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-request completion: n 64-bit words at src (device) copied into the
// pinned host buffer at byte offset off, by the whole workgroup or (one) by
// thread 0 alone.  The caller has made the words final: every producer fenced
// its atomics before announcing its part done.
__device__ __forceinline__ void copy_to_host(const BatchArgs& a, const unsigned long long* src, uint64_t n,
                                             uint64_t off, bool one) {
    unsigned long long* dst = (unsigned long long*)(a.host_res + off);
    const uint32_t t0 = one ? 0u : threadIdx.x, step = one ? 1u : kWG;
    for (uint64_t i = t0; i < n; i += step) dst[i] = load_agent(src + i);
}

// ... then host flag f is raised to the batch number, after the copies
__device__ __forceinline__ void raise_flag(const BatchArgs& a, const PlanHdr& H, uint32_t f, bool one) {
    __threadfence_system();
    if (!one) __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(&a.host_flags[f], H.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// hardware register XCC_ID (s_getreg: id 20, offset 0, 4 bits): which XCD runs this wave
__device__ __forceinline__ uint32_t xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | 20) & 15u; }

__device__ __forceinline__ void trace_item(const BatchArgs& a, const PlanHdr& H, uint32_t idx, const Item& it,
                                           uint64_t t0, uint64_t t1, uint64_t work = 0) {
    if (!H.trace || threadIdx.x) return;
    TraceRec r;
    r.kind = it.kind;
    r.index = it.idx;
    r.wg = blockIdx.x;
    r.xcc = xcc_id();
    r.t_begin = t0;
    r.t_ready = t1;
    r.t_end = (uint64_t)wall_clock64();
    r.work = work;
    a.trace[idx] = r;
}

// Thread 0 polls *p until it reaches target, at most `limit` times (0: it
// gives up at once); true when the target was reached.  The polls are
// relaxed loads and the acquire fence comes once, after the last: on gfx950
// an agent-scope acquire invalidates the CU's vector L1, and hundreds of
// waiting workgroups polling with acquire kept flushing the L1 of the CUs
// doing the work (config 3's join stage: 6.05 -> 4.97 ms at rate 1, 1.28 ->
// 0.77 ms at rate 0.05).
__device__ __forceinline__ bool poll_count(const uint32_t* p, uint32_t target, uint64_t limit) {
    if (limit == 0) return false;
    for (uint64_t polls = 1; __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target; ++polls) {
        if (polls >= limit) return false;
        __builtin_amdgcn_s_sleep(20);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

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

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

// value -> elementary-interval index of one column program; AS is the
// address space of the group's tables (LDS when staged, else global)
// field-wise copies of plan descriptors read through the constant address space
__device__ __forceinline__ ColProg cprog(const GACE_CONST ColProg* p) {
    ColProg P;
    P.data = p->data;
    P.kind = p->kind;
    P.xform = p->xform;
    P.lo = p->lo;
    P.hi = p->hi;
    P.nb = p->nb;
    P.step = p->step;
    P.mask_off = p->mask_off;
    P.bnd_off = p->bnd_off;
    return P;
}

__device__ __forceinline__ GroupDesc cgroup(const GACE_CONST GroupDesc* p) {
    GroupDesc G;
    G.base_mask = p->base_mask;
    G.col_begin = p->col_begin;
    G.col_end = p->col_end;
    G.slot_index = p->slot_index;
    G.tab_off = p->tab_off;
    G.tab_bytes = p->tab_bytes;
    G.n_used = p->n_used;
    return G;
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

// ballot count of one row slot: for each active predicate p, the number of
// the wave's 64 rows (one per lane) whose bit p is set goes to lane p
__device__ __forceinline__ void count_ballot(uint64_t m, uint64_t active, uint32_t& cnt, int lane) {
    uint64_t a = active;
    while (a) {
        const int p = __ffsll((long long)a) - 1;
        a &= a - 1;
        const uint32_t c = (uint32_t)__popcll(__ballot((m >> p) & 1ull));
        if (lane == p) cnt += c;
    }
}

// a + b + c at every bit position: carry (weight 2) and sum (weight 1) words
__device__ __forceinline__ void csa(uint64_t& carry, uint64_t& sum, uint64_t a, uint64_t b, uint64_t c) {
    const uint64_t u = a ^ b;
    carry = (a & b) | (u & c);
    sum = u ^ c;
}

// The lane's 16 row masks summed at every bit position into a 5-bit count,
// bit plane p[k] of weight 2^k, by a carry-save adder tree: 11 full and 4
// half adders, 63 word operations for 16 rows.
__device__ __forceinline__ void add16(const uint64_t (&d)[16], uint64_t (&p)[5]) {
    uint64_t c2[8], s1[5], t1[2];
    csa(c2[0], s1[0], d[0], d[1], d[2]);
    csa(c2[1], s1[1], d[3], d[4], d[5]);
    csa(c2[2], s1[2], d[6], d[7], d[8]);
    csa(c2[3], s1[3], d[9], d[10], d[11]);
    csa(c2[4], s1[4], d[12], d[13], d[14]);
    csa(c2[5], t1[0], s1[0], s1[1], s1[2]);
    csa(c2[6], t1[1], s1[3], s1[4], d[15]);
    p[0] = t1[0] ^ t1[1];
    c2[7] = t1[0] & t1[1];
    uint64_t c4[4], s2[3];
    csa(c4[0], s2[0], c2[0], c2[1], c2[2]);
    csa(c4[1], s2[1], c2[3], c2[4], c2[5]);
    csa(c4[2], s2[2], s2[0], s2[1], c2[6]);
    p[1] = s2[2] ^ c2[7];
    c4[3] = s2[2] & c2[7];
    uint64_t c8[2], s4;
    csa(c8[0], s4, c4[0], c4[1], c4[2]);
    p[2] = s4 ^ c4[3];
    c8[1] = s4 & c4[3];
    p[3] = c8[0] ^ c8[1];
    p[4] = c8[0] & c8[1];
}

// a tile's 16 row masks per lane (rows out of range already 0) added to the
// per-lane counters (lane p counts predicate p).  Ballot per active predicate
// for few of them (mode 1, or mode 0 with at most 6); else (mode 2, or mode
// 0) the adder tree, then one 64x64 wave transpose per bit plane: 5
// transposes per 16 rows instead of one per row.
__device__ __forceinline__ void count_tile(const uint64_t (&d)[16], uint64_t active, uint32_t& cnt, int lane,
                                           uint32_t mode) {
    if (mode == 1 || (mode == 0 && __popcll(active) <= 6)) {
#pragma unroll
        for (int i = 0; i < 16; ++i) count_ballot(d[i], active, cnt, lane);
        return;
    }
    uint64_t p[5];
    add16(d, p);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        uint32_t lo = (uint32_t)p[k], hi = (uint32_t)(p[k] >> 32);
        transpose64(lo, hi, lane);
        cnt += (uint32_t)(__popc(lo) + __popc(hi)) << k;
    }
}

// rows [r0, r1) of one block for one group.  The WG walks the rows in tiles
// of 4096: wave w takes rows [tile + 1024 w, tile + 1024 (w + 1)), each lane 16
// of them (4 quads of 4 consecutive rows, 256 rows apart).  For a 32-bit
// column the lane issues its 4 quad loads (16 B each) at once, and the next
// 32-bit column's loads are issued before this column's lookups, so up to 8
// loads per lane are in flight while masks are combined.  64-bit columns are
// loaded and looked up one quad at a time.  tab points at the group's
// masks/boundaries in address space AS (LDS when staged, else global).
constexpr int kQuads = 4;
constexpr int kRows = kQuads * 4;

__device__ __forceinline__ void load32(const ColProg& P, uint64_t q0, uint64_t r1, uint32_t (&v)[kRows]) {
#pragma unroll
    for (int j = 0; j < kQuads; ++j) {
        const uint64_t rq = q0 + 256ull * j;
        const int nv = rq < r1 ? (int)min((uint64_t)4, r1 - rq) : 0;
        const GACE_GLOBAL uint32_t* p = (const GACE_GLOBAL uint32_t*)P.data + rq;
        if (nv == 4 && (rq & 3) == 0) {
            const u32x4 x = __builtin_nontemporal_load((const GACE_GLOBAL u32x4*)p);
            v[4 * j + 0] = x.x; v[4 * j + 1] = x.y; v[4 * j + 2] = x.z; v[4 * j + 3] = x.w;
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) v[4 * j + t] = t < nv ? p[t] : 0u;
        }
    }
}

// binary searches of n keys advanced together: each step issues n
// independent boundary reads instead of n dependent chains
template <int N, typename B, typename K>
__device__ __forceinline__ void rank_many(const B* bnd, uint32_t nb, uint32_t step, const K (&k)[N],
                                          uint32_t (&pos)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) pos[i] = 0;
    for (; step; step >>= 1) {
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (pos[i] + step <= nb && bnd[pos[i] + step - 1] <= k[i]) pos[i] += step;
    }
}

// the column's kind and key transform are dispatched once for all rows
template <int AS>
__device__ __forceinline__ void lookup32(const ColProg& P, const uint8_t* tab, const uint32_t (&v)[kRows],
                                         uint64_t (&m)[kRows]) {
    typedef __attribute__((address_space(AS))) const uint64_t TM;
    typedef __attribute__((address_space(AS))) const uint32_t TB;
    TM* masks = (TM*)(tab + P.mask_off);
    uint32_t k[kRows];
    if (P.xform == XF_I32) {
#pragma unroll
        for (int i = 0; i < kRows; ++i) k[i] = v[i] ^ 0x80000000u;
    } else {
#pragma unroll
        for (int i = 0; i < kRows; ++i) k[i] = key32(v[i], XF_F32);
    }
    if (P.kind == CP_LUT32) {
#pragma unroll
        for (int i = 0; i < kRows; ++i) m[i] &= masks[min(max(k[i], P.lo), P.hi) - P.lo];
    } else {
        uint32_t pos[kRows];
        rank_many<kRows>((TB*)(tab + P.bnd_off), P.nb, P.step, k, pos);
#pragma unroll
        for (int i = 0; i < kRows; ++i) m[i] &= masks[pos[i]];
    }
}

template <int AS>
__device__ __forceinline__ void lookup64(const ColProg& P, const uint8_t* tab, uint64_t q0, uint64_t r1,
                                         uint64_t (&m)[kRows]) {
    typedef __attribute__((address_space(AS))) const uint64_t TM;
    TM* masks = (TM*)(tab + P.mask_off);
#pragma unroll
    for (int j = 0; j < kQuads; ++j) {
        const uint64_t rq = q0 + 256ull * j;
        const int nv = rq < r1 ? (int)min((uint64_t)4, r1 - rq) : 0;
        const GACE_GLOBAL uint64_t* p = (const GACE_GLOBAL uint64_t*)P.data + rq;
        uint64_t w[4] = {0, 0, 0, 0};
        if (nv == 4 && (rq & 3) == 0) {
            const u64x2 x = __builtin_nontemporal_load((const GACE_GLOBAL u64x2*)p);
            const u64x2 y = __builtin_nontemporal_load((const GACE_GLOBAL u64x2*)p + 1);
            w[0] = x.x; w[1] = x.y; w[2] = y.x; w[3] = y.y;
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) w[t] = t < nv ? p[t] : 0ull;
        }
        uint64_t kk[4];
        uint32_t pos[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) kk[t] = w[t] ^ 0x8000000000000000ull;
        typedef __attribute__((address_space(AS))) const uint64_t TB;
        rank_many<4>((TB*)(tab + P.bnd_off), P.nb, P.step, kk, pos);
#pragma unroll
        for (int t = 0; t < 4; ++t) m[4 * j + t] &= masks[pos[t]];
    }
}

// tiles of 4096 rows over a set of kept blocks of one 64-block chunk
struct TileIt {
    uint64_t start, end;        // tile start row, end row of its block
    uint32_t j;                 // the block's index in the chunk
};

__device__ __forceinline__ bool tile_first(TileIt& t, unsigned long long& rest, uint64_t cb, uint64_t B,
                                           uint64_t n) {
    if (!rest) return false;
    const int j = __ffsll((long long)rest) - 1;
    rest &= rest - 1;
    t.start = (cb + (uint64_t)j) * B;
    t.end = t.start + B < n ? t.start + B : n;
    t.j = (uint32_t)j;
    return true;
}

// predicate bits of group g active for a block whose requests own the first
// act_bits predicate bits of the scan
__device__ __forceinline__ uint64_t group_prefix(uint32_t act_bits, uint32_t g) {
    if (act_bits <= g * 64) return 0ull;
    const uint32_t na = act_bits - g * 64;
    return na >= 64 ? ~0ull : ((1ull << na) - 1ull);
}

__device__ __forceinline__ bool tile_next(TileIt& t, unsigned long long& rest, uint64_t cb, uint64_t B,
                                          uint64_t n) {
    t.start += (uint64_t)kWG * kRows;
    if (t.start < t.end) return true;
    return tile_first(t, rest, cb, B, n);
}

// all rows of the blocks in `blocks` (bit j = block cb + j) for group g: a
// block's active predicates are the group's bits among the first s_act[j]
// predicate bits of the scan.  tab points at the group's masks/boundaries in
// address space AS (LDS when staged, else global).
//
// Full tiles (4096 rows inside one block) form a stream of units (tile,
// 32-bit column) with two register buffers that alternate, so a unit's four
// 16-byte loads per lane are in flight while the previous unit is looked up;
// their loads have one form and no bounds, so nothing makes the wave wait for
// them early.  Short tiles (blocks of fewer than 4096 rows, a table's last
// block) take a second, unpipelined pass with per-row bounds.  64-bit columns
// are loaded and looked up at the end of each tile.
struct ScanUnit {
    TileIt t;
    unsigned long long rest;    // blocks after t's block
    uint32_t c;                 // column
    bool valid;
};

__device__ __forceinline__ bool tile_full(const TileIt& t) { return t.end - t.start >= (uint64_t)kWG * kRows; }

// next tile of the requested kind (full or short) after t, or of blocks in rest
__device__ __forceinline__ bool tile_next_kind(TileIt& t, unsigned long long& rest, uint64_t cb, uint64_t B,
                                               uint64_t n, bool full, bool first) {
    bool ok = first ? tile_first(t, rest, cb, B, n) : tile_next(t, rest, cb, B, n);
    while (ok && tile_full(t) != full) ok = tile_next(t, rest, cb, B, n);
    return ok;
}

__device__ __forceinline__ void load32_full(const ColProg& P, uint64_t q0, uint32_t (&v)[kRows]) {
#pragma unroll
    for (int j = 0; j < kQuads; ++j) {
        const GACE_GLOBAL u32x4* p = (const GACE_GLOBAL u32x4*)((const GACE_GLOBAL uint32_t*)P.data + q0 + 256ull * j);
        const u32x4 x = __builtin_nontemporal_load(p);
        v[4 * j + 0] = x.x;
        v[4 * j + 1] = x.y;
        v[4 * j + 2] = x.z;
        v[4 * j + 3] = x.w;
    }
}

template <int AS>
__device__ __forceinline__ uint32_t scan_blocks(const GACE_CONST ColProg* cols, uint32_t c_begin, uint32_t c_end,
                                                const uint8_t* tab, unsigned long long blocks, uint64_t cb,
                                                uint64_t B, uint64_t n, uint64_t base_mask, const uint32_t* s_act,
                                                uint32_t g, int lane, int wave, uint32_t mode) {
    uint32_t cnt = 0;
    auto next32 = [&](uint32_t c) __attribute__((always_inline)) {
        while (c < c_end && cols[c].kind == CP_RANK64) ++c;
        return c;
    };
    const uint32_t first32 = next32(c_begin);
    bool any64 = false;
    for (uint32_t c = c_begin; c < c_end; ++c) any64 |= cols[c].kind == CP_RANK64;
    const uint64_t lane_off = (uint64_t)wave * 256 * kQuads + 4ull * (uint64_t)lane;
    uint64_t m[kRows];
    // end of a tile: 64-bit columns, then count the tile's rows
    auto finish_tile = [&](const TileIt& t, uint64_t active) __attribute__((always_inline)) {
        const uint64_t q0 = t.start + lane_off, r1 = t.end;
        if (any64)
            for (uint32_t c64 = c_begin; c64 < c_end; ++c64)
                if (cols[c64].kind == CP_RANK64) {
                    const ColProg P64 = cprog(cols + c64);
                    lookup64<AS>(P64, tab, q0, r1, m);
                }
#pragma unroll
        for (int j = 0; j < kQuads; ++j) {
            const uint64_t rq = q0 + 256ull * j;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (rq + u >= r1) m[4 * j + u] = 0ull;
        }
        count_tile(m, active, cnt, lane, mode);
    };

    // ---- full tiles, pipelined over (tile, column) units
    if (first32 < c_end) {
        ScanUnit u0;
        u0.rest = blocks;
        u0.valid = tile_next_kind(u0.t, u0.rest, cb, B, n, true, true);
        u0.c = first32;
        auto advance = [&](ScanUnit u) __attribute__((always_inline)) {
            u.c = next32(u.c + 1);
            if (u.c >= c_end) {
                u.valid = tile_next_kind(u.t, u.rest, cb, B, n, true, false);
                u.c = first32;
            }
            return u;
        };
        // a tile's first column starts its masks, its last one finishes it
        auto consume = [&](const ScanUnit& u, const uint32_t (&v)[kRows]) __attribute__((always_inline)) {
            const uint64_t active = base_mask & group_prefix(s_act[u.t.j], g);
            if (u.c == first32) {
#pragma unroll
                for (int i = 0; i < kRows; ++i) m[i] = active;
            }
            const ColProg Pc = cprog(cols + u.c);
            lookup32<AS>(Pc, tab, v, m);
            if (next32(u.c + 1) >= c_end) finish_tile(u.t, active);
        };
        if (u0.valid) {
            uint32_t va[kRows], vb[kRows];
            {
                const ColProg P = cprog(cols + u0.c);
                load32_full(P, u0.t.start + lane_off, va);
            }
            for (;;) {
                const ScanUnit u1 = advance(u0);
                if (u1.valid) {
                    const ColProg P = cprog(cols + u1.c);
                    load32_full(P, u1.t.start + lane_off, vb);
                }
                consume(u0, va);
                if (!u1.valid) break;
                const ScanUnit u2 = advance(u1);
                if (u2.valid) {
                    const ColProg P = cprog(cols + u2.c);
                    load32_full(P, u2.t.start + lane_off, va);
                }
                consume(u1, vb);
                if (!u2.valid) break;
                u0 = u2;
            }
        }
    }

    // ---- short tiles (and groups with only 64-bit columns): one at a time
    {
        const bool only64 = first32 >= c_end;
        TileIt t;
        unsigned long long rest = blocks;
        bool ok = only64 ? tile_first(t, rest, cb, B, n) : tile_next_kind(t, rest, cb, B, n, false, true);
        while (ok) {
            const uint64_t active = base_mask & group_prefix(s_act[t.j], g);
#pragma unroll
            for (int i = 0; i < kRows; ++i) m[i] = active;
            for (uint32_t c = first32; c < c_end; c = next32(c + 1)) {
                const ColProg P = cprog(cols + c);
                uint32_t v[kRows];
                load32(P, t.start + lane_off, t.end, v);
                lookup32<AS>(P, tab, v, m);
            }
            finish_tile(t, active);
            ok = only64 ? tile_next(t, rest, cb, B, n) : tile_next_kind(t, rest, cb, B, n, false, false);
        }
    }
    return cnt;
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

// ------------------------------------------------------------------ fine scan
// One request on blocks of fewer than 4096 rows, with at least one block in
// 4096 / B kept on average: the item's rows are walked in aligned 4096-row
// tiles and every row's block is decided by the lane that holds the row (one
// Philox per distinct block of the lane's rows), so a tile costs one pass
// however its kept blocks are spread.  A lane keeps a 16-bit mask of its kept
// rows; the lane holding a block's first row counts the block.  Counts and
// sample histogram equal the block-by-block path's.
template <int AS>
__device__ __forceinline__ void fine_group(const GACE_CONST ColProg* cols, const GroupDesc& G, const uint8_t* tab,
                                           uint32_t g, uint32_t km, uint32_t all_bits, uint64_t q0, uint64_t r1,
                                           int lane, uint32_t mode, uint32_t& cnt) {
    const uint64_t active = G.base_mask & group_prefix(all_bits, g);
    uint64_t m[kRows];
#pragma unroll
    for (int i = 0; i < kRows; ++i) m[i] = ((km >> i) & 1u) ? active : 0ull;
    for (uint32_t c = G.col_begin; c < G.col_end; ++c) {
        const ColProg P = cprog(cols + c);
        if (P.kind == CP_RANK64) {
            lookup64<AS>(P, tab, q0, r1, m);
        } else {
            uint32_t v[kRows];
            load32(P, q0, r1, v);
            lookup32<AS>(P, tab, v, m);
        }
    }
    count_tile(m, active, cnt, lane, mode);
}

__device__ __forceinline__ void scan_fine(const BatchArgs& a, const ScanDesc& S, const GACE_CONST GroupDesc* groups,
                                          const GACE_CONST ColProg* cols, const uint32_t* slots, uint32_t all_bits,
                                          unsigned long long* s_hist, uint32_t* s_cnt, uint8_t* s_tab, int* s_staged,
                                          uint32_t n_lds_groups, uint64_t b_begin, uint64_t b_end, int lane,
                                          int wave) {
    const uint32_t log2B = S.log2B;
    const uint64_t B = 1ull << log2B;
    const uint64_t r_begin = b_begin << log2B;
    const uint64_t r_end = min(b_end << log2B, S.n_rows);
    const uint64_t lane_off = (uint64_t)wave * 256 * kQuads + 4ull * (uint64_t)lane;
    for (uint64_t t = r_begin; t < r_end; t += kZoneRows) {
        const uint64_t q0 = t + lane_off;
        const uint64_t r1 = t + kZoneRows < r_end ? t + kZoneRows : r_end;
        uint32_t km = 0;   // bit i: row i of this lane is in a kept block
        uint32_t hrows = 0, hblocks = 0;
#pragma unroll
        for (int i = 0; i < kRows; ++i) {
            const uint64_t r = q0 + 256ull * (i >> 2) + (i & 3);
            // rows of one quad share a block when B >= 4: decide it once
            if ((i & 3) == 0 || log2B < 2) {
                bool kept = false;
                if (r < r1) {
                    kept = (uint64_t)block_word0(r >> log2B, S.table_id, S.seed) < S.thr_max;
                    if (kept && (r & (B - 1)) == 0) {
                        hrows += (uint32_t)((r + B < S.n_rows ? r + B : S.n_rows) - r);
                        hblocks += 1;
                    }
                }
                if (kept) km |= (log2B < 2 ? 1u : 15u) << i;
            }
        }
        if (log2B >= 2) {   // drop the rows of a quad past the end
#pragma unroll
            for (int i = 0; i < kRows; ++i)
                if (q0 + 256ull * (i >> 2) + (i & 3) >= r1) km &= ~(1u << i);
        }
        // the tile's kept rows and blocks, one LDS add per wave
        for (int o = 32; o; o >>= 1) {
            hrows += __shfl_xor(hrows, o);
            hblocks += __shfl_xor(hblocks, o);
        }
        if (lane == 0 && hblocks) {
            atomicAdd(&s_hist[2], (unsigned long long)hrows);
            atomicAdd(&s_hist[3], (unsigned long long)hblocks);
        }
        if (S.zskip) {
            const GACE_GLOBAL uint32_t* zs = (const GACE_GLOBAL uint32_t*)S.zskip;
            const uint64_t z = t >> kZoneLog2;
            if ((zs[z >> 5] >> (z & 31)) & 1u) continue;   // sampled, but no predicate can hold here
        }
        const bool any = km != 0;
        for (uint32_t g = 0; g * 64 < all_bits; ++g) {
            if (!__syncthreads_or(any)) break;
            const GroupDesc G = cgroup(groups + g);
            uint32_t cnt = 0;
            if (G.tab_bytes <= kGroupTabBudget) {
                if (*s_staged != (int)g) {
                    __syncthreads();
                    const uint4* src = (const uint4*)(a.plan + G.tab_off);
                    uint4* dst = (uint4*)s_tab;
                    for (uint32_t i = threadIdx.x; i < G.tab_bytes / 16; i += kWG) dst[i] = src[i];
                    __syncthreads();
                    if (threadIdx.x == 0) *s_staged = (int)g;
                }
                if (__ballot(any)) fine_group<3>(cols, G, s_tab, g, km, all_bits, q0, r1, lane, a.count_mode, cnt);
            } else if (__ballot(any)) {
                fine_group<1>(cols, G, a.plan + G.tab_off, g, km, all_bits, q0, r1, lane, a.count_mode, cnt);
            }
            if (cnt) {
                if (g < n_lds_groups) atomicAdd(&s_cnt[g * 64 + lane], cnt);
                else atomicAdd(&a.counts[slots[G.slot_index + lane]], (unsigned long long)cnt);
            }
            if (S.n_groups > 1) __syncthreads();   // the staged table may be replaced by the next group
        }
    }
}

// Group-major pass over the blocks in scan_keep (bit j = block cb + j) of
// one chunk: group g streams every block whose requests reach into it, each
// with its own active bits (s_act[j]).  Counts of the first n_lds_groups
// groups go to the LDS counters, the rest straight to the global ones.
__device__ __forceinline__ void scan_groups(const BatchArgs& a, const ScanDesc& S,
                                            const GACE_CONST GroupDesc* groups, const GACE_CONST ColProg* cols,
                                            const uint32_t* slots, uint32_t n_lds_groups, unsigned long long scan_keep,
                                            uint64_t cb, const uint32_t* s_act, uint32_t* s_cnt, uint8_t* s_tab,
                                            int* s_staged, int lane, int wave) {
    const uint64_t B = 1ull << S.log2B;
    for (uint32_t g = 0;; ++g) {
        const unsigned long long blocks_g = __ballot(((scan_keep >> lane) & 1ull) && s_act[lane] > g * 64);
        if (!blocks_g) break;
        const GroupDesc G = cgroup(groups + g);
        uint32_t cnt;
        if (G.tab_bytes <= kGroupTabBudget) {
            if (*s_staged != (int)g) {
                __syncthreads();
                const uint4* src = (const uint4*)(a.plan + G.tab_off);
                uint4* dst = (uint4*)s_tab;
                for (uint32_t i = threadIdx.x; i < G.tab_bytes / 16; i += kWG) dst[i] = src[i];
                __syncthreads();
                if (threadIdx.x == 0) *s_staged = (int)g;
            }
            cnt = scan_blocks<3>(cols, G.col_begin, G.col_end, s_tab, blocks_g, cb, B, S.n_rows, G.base_mask, s_act,
                                 g, lane, wave, a.count_mode);
        } else {
            cnt = scan_blocks<1>(cols, G.col_begin, G.col_end, a.plan + G.tab_off, blocks_g, cb, B, S.n_rows,
                                 G.base_mask, s_act, g, lane, wave, a.count_mode);
        }
        if (cnt) {
            if (g < n_lds_groups) atomicAdd(&s_cnt[g * 64 + lane], cnt);
            else atomicAdd(&a.counts[slots[G.slot_index + lane]], (unsigned long long)cnt);
        }
        if (S.n_groups > 1) __syncthreads();   // the staged table may be replaced by the next group
    }
}

// the spill list: the item region after the items kept there
__device__ __forceinline__ Item* spill_list(const BatchArgs& a, const PlanHdr& H) {
    return const_cast<Item*>(a.items) + (H.items_off ? 0u : H.n_items);
}

// Wave 0 appends every kept block of the chunk after the first to the spill
// list (an entry per block: scan, block, its predicate bits; its ready word
// stored last, with release); blocks that find the list full stay.  Returns
// the blocks this item still scans.
__device__ __forceinline__ unsigned long long spill_blocks(const BatchArgs& a, const PlanHdr& H, uint32_t scan,
                                                           uint64_t cb, unsigned long long scan_keep,
                                                           const uint32_t* s_act, unsigned long long* s_keep2) {
    if (threadIdx.x < 64) {
        const uint32_t lane = threadIdx.x;
        const unsigned long long first = scan_keep & (~scan_keep + 1ull);
        bool moved = false;
        if (((scan_keep >> lane) & 1ull) && !((first >> lane) & 1ull)) {
            const uint32_t slot = atomicAdd(&a.head[3], 1u);
            if (slot < H.spill_cap) {
                Item* e = spill_list(a, H) + slot;
                e->kind = IT_SCAN;
                e->idx = scan;
                e->side = s_act[lane];
                e->begin = cb + lane;
                e->end = cb + lane + 1;
                __hip_atomic_store(&e->sub, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                moved = true;
            }
        }
        const unsigned long long out = __ballot(moved);
        if (lane == 0) *s_keep2 = scan_keep & ~out;
    }
    __syncthreads();
    return *s_keep2;
}

// ------------------------------------------------------------------ scan item
__device__ __forceinline__ void scan_item(const BatchArgs& a, const PlanHdr& H, const Item& it, uint8_t* lds) {
    const ScanDesc S = ((const ScanDesc*)(a.plan + H.scans_off))[it.idx];
    const GACE_CONST GroupDesc* groups = (const GACE_CONST GroupDesc*)(a.plan + H.groups_off) + S.group_begin;
    const GACE_CONST ColProg* cols = (const GACE_CONST ColProg*)(a.plan + H.cols_off);
    const uint32_t* slots = (const uint32_t*)(a.plan + H.slots_off);
    const uint64_t* rthr = (const uint64_t*)(a.plan + H.reqthr_off) + S.req_begin;
    const uint32_t* rcum = (const uint32_t*)(a.plan + H.reqcum_off) + S.req_begin;

    uint32_t* s_w0 = (uint32_t*)lds;
    unsigned long long* s_keep = (unsigned long long*)(lds + 256);
    int* s_staged = (int*)(lds + 264);
    unsigned long long* s_keep2 = (unsigned long long*)(lds + 272);
    uint32_t* s_k = (uint32_t*)(lds + 384);
    uint32_t* s_act = s_w0;   // per block: predicate bits its requests own (replaces w0 once k is known)
    uint32_t* s_cnt = (uint32_t*)(lds + kLdsMisc);
    unsigned long long* s_hist = (unsigned long long*)(lds + kLdsMisc + kLdsCnt);
    uint64_t* s_thr = (uint64_t*)(lds + kLdsMisc + kLdsCnt + kLdsHist);
    uint32_t* s_cum = (uint32_t*)(lds + kLdsMisc + kLdsCnt + kLdsHist + kScanLdsHist * 8);
    uint8_t* s_tab = lds + kLdsMisc + kLdsCnt + kLdsHist + kLdsThr;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t n_lds_groups = S.n_groups < kScanLdsGroups ? S.n_groups : kScanLdsGroups;
    // scans of fewer than 128 requests keep thresholds, bit prefix sums and
    // the sample histogram in LDS for the whole item
    const bool small = S.n_req < kScanLdsHist;
    for (uint32_t i = threadIdx.x; i < n_lds_groups * 64; i += kWG) s_cnt[i] = 0;
    if (small) {
        for (uint32_t i = threadIdx.x; i < 2 * (S.n_req + 1); i += kWG) s_hist[i] = 0;
        for (uint32_t i = threadIdx.x; i < S.n_req; i += kWG) s_thr[i] = rthr[i];
        for (uint32_t i = threadIdx.x; i <= S.n_req; i += kWG) s_cum[i] = rcum[i];
    }
    if (threadIdx.x == 0) *s_staged = -1;
    __syncthreads();

    const uint64_t B = 1ull << S.log2B;
    if (S.fine)
        scan_fine(a, S, groups, cols, slots, small ? s_cum[1] : rcum[1], s_hist, s_cnt, s_tab, s_staged,
                  n_lds_groups, it.begin, it.end, lane, wave);
    for (uint64_t cb = it.begin; cb < it.end && !S.fine; cb += 64) {
        decide_blocks(cb, it.end, S.thr_max, S.table_id, S.seed, s_w0, s_keep);
        __syncthreads();
        const unsigned long long keep = *s_keep;
        // wave 0: k(b) = number of requests whose threshold exceeds word 0
        // (thresholds sorted descending), and the sample histogram
        if (threadIdx.x < 64 && ((keep >> threadIdx.x) & 1ull)) {
            const uint64_t w0 = s_w0[threadIdx.x];
            uint32_t k = 0;
            for (uint32_t step = 1u << 31; step; step >>= 1)
                if (k + step <= S.n_req && (small ? s_thr[k + step - 1] : rthr[k + step - 1]) > w0) k += step;
            s_k[threadIdx.x] = k;
            s_act[threadIdx.x] = small ? s_cum[k] : rcum[k];
            const uint64_t r0 = (cb + threadIdx.x) * B;
            const uint64_t rows = (r0 + B < S.n_rows ? r0 + B : S.n_rows) - r0;
            if (small) {
                atomicAdd(&s_hist[2 * k], (unsigned long long)rows);
                atomicAdd(&s_hist[2 * k + 1], 1ull);
            } else {
                atomicAdd(&a.hist[S.hist_off + 2 * k], (unsigned long long)rows);
                atomicAdd(&a.hist[S.hist_off + 2 * k + 1], 1ull);
            }
        }
        __syncthreads();
        // zone map: kept blocks on which no predicate can hold are sampled
        // (counted above) but not scanned
        unsigned long long scan_keep = keep;
        if (S.zskip) {
            const GACE_GLOBAL uint32_t* zs = (const GACE_GLOBAL uint32_t*)S.zskip;
            bool skip = false;
            if ((keep >> lane) & 1ull) {
                const uint64_t r0 = (cb + (uint64_t)lane) * B;
                const uint64_t r1 = (r0 + B < S.n_rows ? r0 + B : S.n_rows) - 1;
                skip = true;
                for (uint64_t z = r0 >> kZoneLog2; z <= (r1 >> kZoneLog2) && skip; ++z)
                    skip = (zs[z >> 5] >> (z & 31)) & 1u;
            }
            scan_keep = keep & ~__ballot(skip);
        }
        // a sparse scan keeps the chunk's first kept block and spills the rest
        if (S.spill && H.spill_cap) scan_keep = spill_blocks(a, H, it.idx, cb, scan_keep, s_act, s_keep2);
        scan_groups(a, S, groups, cols, slots, n_lds_groups, scan_keep, cb, s_act, s_cnt, s_tab, s_staged, lane,
                    wave);
        __syncthreads();
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n_lds_groups * 64; i += kWG) {
        const uint32_t c = s_cnt[i];
        if (c) atomicAdd(&a.counts[slots[groups[i >> 6].slot_index + (i & 63)]], (unsigned long long)c);
    }
    if (small)
        for (uint32_t i = threadIdx.x; i < 2 * (S.n_req + 1); i += kWG) {
            const unsigned long long v = s_hist[i];
            if (v) atomicAdd(&a.hist[S.hist_off + i], v);
        }
}

// One spilled block: the group-major pass over it alone (its sample
// histogram entry was counted by the item that decided it).
__device__ __forceinline__ void scan_spill_task(const BatchArgs& a, const PlanHdr& H, uint32_t scan, uint64_t block,
                                                uint32_t act, uint8_t* lds) {
    const ScanDesc S = ((const ScanDesc*)(a.plan + H.scans_off))[scan];
    const GACE_CONST GroupDesc* groups = (const GACE_CONST GroupDesc*)(a.plan + H.groups_off) + S.group_begin;
    const GACE_CONST ColProg* cols = (const GACE_CONST ColProg*)(a.plan + H.cols_off);
    const uint32_t* slots = (const uint32_t*)(a.plan + H.slots_off);
    uint32_t* s_act = (uint32_t*)lds;
    int* s_staged = (int*)(lds + 264);
    uint32_t* s_cnt = (uint32_t*)(lds + kLdsMisc);
    uint8_t* s_tab = lds + kLdsMisc + kLdsCnt + kLdsHist + kLdsThr;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t n_lds_groups = S.n_groups < kScanLdsGroups ? S.n_groups : kScanLdsGroups;
    for (uint32_t i = threadIdx.x; i < n_lds_groups * 64; i += kWG) s_cnt[i] = 0;
    if (threadIdx.x == 0) {
        *s_staged = -1;
        s_act[0] = act;
    }
    __syncthreads();
    scan_groups(a, S, groups, cols, slots, n_lds_groups, 1ull, block, s_act, s_cnt, s_tab, s_staged, lane, wave);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n_lds_groups * 64; i += kWG) {
        const uint32_t c = s_cnt[i];
        if (c) atomicAdd(&a.counts[slots[groups[i >> 6].slot_index + (i & 63)]], (unsigned long long)c);
    }
}

// ------------------------------------------------------------------ joins
// Key-only aggregation by hash partitioning: per-item partition counts of the
// sampled keys (JHIST) -> per-partition offsets (JOFF, JBASE) -> keys
// scattered into their partitions (JSCATTER) -> each partition aggregated in
// an LDS key table (JAGG), which gives f_R(k), f_S(k) for every key of the
// partition, hence NDV and sum f_R f_S.  A partition with more distinct keys
// than one LDS table holds is split into residue classes of the hash and
// aggregated in several passes, so the result is exact for any input.
// Keys whose hash sits in the join's heavy-hitter table (JHEAVY) are counted
// per slot by the histogram items, like the sentinel key, and skip the
// partitioning and the LDS tables; the offset phase adds their share of the
// results.  Under Zipf skew they are a large part of the keys.

// MurmurHash3 64-bit finalizer (Appleby, public domain): a bijection on keys
__device__ __forceinline__ uint64_t mix_key(uint64_t k) {
    k ^= k >> 33;
    k *= 0xFF51AFD7ED558CCDull;
    k ^= k >> 33;
    k *= 0xC4CEB9FE1A85EC53ull;
    k ^= k >> 33;
    return k;
}

__device__ __forceinline__ uint32_t part_of(uint64_t h, uint32_t log2P) {
    return log2P ? (uint32_t)(h >> (64 - log2P)) : 0u;
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

// calls f(k, ok) for the sampled keys of blocks [b0, b1) of one side, N
// per thread at a time (k[u] is a key where ok[u]); the N loads are issued
// before use
template <int N, typename F>
__device__ __forceinline__ void for_each_sampled_key(const JoinSide* D, uint64_t b0, uint64_t b1, uint8_t* lds,
                                                     F&& f) {
    uint32_t* s_w0 = (uint32_t*)lds;
    unsigned long long* s_keep = (unsigned long long*)(lds + 256);
    const uint64_t B = 1ull << D->log2B, n = D->n;
    const GACE_GLOBAL int64_t* keys = (const GACE_GLOBAL int64_t*)D->keys;
    for (uint64_t cb = b0; cb < b1; cb += 64) {
        decide_blocks(cb, b1, D->thr, D->table_id, D->seed, s_w0, s_keep);
        __syncthreads();
        unsigned long long keep = *s_keep;
        while (keep) {
            const int j = __ffsll((long long)keep) - 1;
            keep &= keep - 1;
            const uint64_t r0 = (cb + (uint64_t)j) * B;
            const uint64_t r1 = (r0 + B < n) ? r0 + B : n;
            for (uint64_t r = r0 + threadIdx.x; r < r1; r += (uint64_t)N * kWG) {
                uint64_t k[N];
                // unconditional loads (clamped in range): no branch makes the
                // wave wait for one load before issuing the next
#pragma unroll
                for (int u = 0; u < N; ++u) {
                    const uint64_t rr = r + (uint64_t)u * kWG;
                    k[u] = (uint64_t)__builtin_nontemporal_load(keys + (rr < r1 ? rr : r1 - 1));
                }
                bool ok[N];
#pragma unroll
                for (int u = 0; u < N; ++u) ok[u] = r + (uint64_t)u * kWG < r1;
                f(k, ok);
            }
        }
        __syncthreads();
    }
}

// Heavy hitters of one join, ahead of its histogram items.  Each side
// contributes up to kHeavySample keys: all of them for a short side, else 8
// runs of kWG consecutive rows spread evenly over the column (any rows would
// do: the table only decides which keys skip the partitioning, never a
// count).  A side's sample is counted in an LDS table (linear probing; a key
// that finds no slot in 16 probes is left out); each hash seen at least
// kHeavyMin times bids for its slot of the join's direct-mapped heavy table,
// the higher count winning (ties: the later side, then the larger table
// index).  The winners and zeroed per-slot counts go to the arena.
template <int KP>
__device__ void jheavy_item(const BatchArgs& a, const JoinDesc* jd, uint8_t* lds) {
    unsigned long long* s_key = (unsigned long long*)(lds + kLdsMisc);          // [kHeavyCount]
    uint32_t* s_cnt = (uint32_t*)(s_key + kHeavyCount);                          // [kHeavyCount]
    unsigned long long* s_win = (unsigned long long*)(lds + heavy_lds_off(KP * kWG));   // [kHeavySlots]
    uint32_t* s_best = (uint32_t*)(s_win + kHeavySlots);                         // [kHeavySlots]
    for (uint32_t i = threadIdx.x; i < kHeavySlots; i += kWG) {
        s_win[i] = kEmptyHash;
        s_best[i] = 0;
    }
    for (uint32_t sd = 0; sd < 2; ++sd) {
        for (uint32_t i = threadIdx.x; i < kHeavyCount; i += kWG) {
            s_key[i] = kEmptyHash;
            s_cnt[i] = 0;
        }
        __syncthreads();
        const JoinSide& D = jd->side[sd];
        const uint64_t n = D.n;
        const GACE_GLOBAL int64_t* keys = (const GACE_GLOBAL int64_t*)D.keys;
        constexpr uint32_t kRuns = kHeavySample / kWG;
        // four keys at a time: fully unrolled, this phase's registers would
        // raise the whole kernel's allocation past the partitioning tiles'
        constexpr uint32_t kLoads = 4;
        static_assert(kRuns % kLoads == 0, "sample runs in groups of four");
#pragma unroll 1
        for (uint32_t u0 = 0; u0 < kRuns; u0 += kLoads) {
            int64_t key4[kLoads];
#pragma unroll
            for (uint32_t v = 0; v < kLoads; ++v) {
                const uint32_t u = u0 + v;
                const uint64_t row = n <= kHeavySample ? (uint64_t)u * kWG + threadIdx.x
                                                       : (n - kWG) * u / (kRuns - 1) + threadIdx.x;
                key4[v] = row < n ? keys[row] : (int64_t)kEmptyKey;
            }
#pragma unroll
            for (uint32_t v = 0; v < kLoads; ++v) {
                if ((uint64_t)key4[v] == kEmptyKey) continue;
                const uint64_t h = mix_key((uint64_t)key4[v]);
                uint32_t sl = (uint32_t)(h >> 21) & (kHeavyCount - 1);
                for (int probe = 0; probe < 16; ++probe, sl = (sl + 1) & (kHeavyCount - 1)) {
                    unsigned long long cur = s_key[sl];
                    if (cur == kEmptyHash) cur = atomicCAS(&s_key[sl], (unsigned long long)kEmptyHash, h);
                    if (cur == kEmptyHash || cur == h) {
                        atomicAdd(&s_cnt[sl], 1u);
                        break;
                    }
                }
            }
        }
        __syncthreads();
        // bid: count above the side and the table index (unique per candidate)
        for (uint32_t i = threadIdx.x; i < kHeavyCount; i += kWG) {
            const uint32_t c = s_cnt[i];
            if (c >= kHeavyMin) atomicMax(&s_best[(uint32_t)s_key[i] & (kHeavySlots - 1)], c << 12 | sd << 11 | i);
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < kHeavyCount; i += kWG) {
            const uint32_t c = s_cnt[i];
            const uint32_t hs = (uint32_t)s_key[i] & (kHeavySlots - 1);
            if (c >= kHeavyMin && s_best[hs] == (c << 12 | sd << 11 | i)) s_win[hs] = s_key[i];
        }
        __syncthreads();
    }
    GACE_GLOBAL unsigned long long* gh = (GACE_GLOBAL unsigned long long*)(a.arena_base + jd->heavy_off);
    GACE_GLOBAL uint32_t* gc = (GACE_GLOBAL uint32_t*)(gh + kHeavySlots);
    for (uint32_t i = threadIdx.x; i < kHeavySlots; i += kWG) {
        gh[i] = s_win[i];
        gc[i] = 0;
        gc[kHeavySlots + i] = 0;
    }
}

// the join's heavy-hitter hashes staged in LDS
__device__ __forceinline__ void stage_heavy(const BatchArgs& a, const JoinDesc* jd, unsigned long long* s_hh) {
    const GACE_GLOBAL u64x2* gh = (const GACE_GLOBAL u64x2*)(a.arena_base + jd->heavy_off);
    for (uint32_t i = threadIdx.x; i < kHeavySlots / 2; i += kWG) ((u64x2*)s_hh)[i] = gh[i];
}

// Partition counts of an item's sampled keys; keys of the heavy table are
// counted per slot instead (added to the join's per-slot counts at the end).
// hist_keys(KP) loads per thread are in flight at once: the pass runs at the
// partitioning kernel's occupancy, so its bytes in flight per CU come from
// the loads per thread.  The 2048-key-tile variant keeps eight, which fit
// its register budget beside a scan workgroup.
constexpr int hist_keys(int kp) { return kp == kPerBig ? 16 : 8; }
template <int KP>
__device__ void jhist_item(const BatchArgs& a, const JoinDesc* jd, const Item& it, uint8_t* lds) {
    const JoinSide* D = &jd->side[it.side];
    JoinAcc& acc = a.accs[jd->acc];
    const uint32_t log2P = jd->log2P, P = 1u << log2P;
    unsigned long long* s_red = (unsigned long long*)(lds + 320);
    uint32_t* cnt = (uint32_t*)(lds + kLdsMisc);
    unsigned long long* s_hh = (unsigned long long*)(lds + heavy_lds_off(KP * kWG));
    uint32_t* s_hc = (uint32_t*)(s_hh + kHeavySlots);
    stage_heavy(a, jd, s_hh);
    for (uint32_t i = threadIdx.x; i < kHeavySlots; i += kWG) s_hc[i] = 0;
    for (uint32_t i = threadIdx.x; i < P; i += kWG) cnt[i] = 0;
    __syncthreads();
    unsigned long long nall = 0, nsent = 0;
    // a key's count goes to its heavy slot or to its partition through one
    // atomic on a per-lane address: two guarded atomics would make every
    // wave issue both
    constexpr int N = hist_keys(KP);
    for_each_sampled_key<N>(D, it.begin, it.end, lds, [&](const uint64_t (&k)[N], const bool (&ok)[N]) {
        uint64_t h[N], m[N];
#pragma unroll
        for (int u = 0; u < N; ++u) {
            h[u] = mix_key(k[u]);
            m[u] = s_hh[(uint32_t)h[u] & (kHeavySlots - 1)];
        }
#pragma unroll
        for (int u = 0; u < N; ++u) {
            const bool sent = k[u] == kEmptyKey;
            nall += ok[u];
            nsent += ok[u] && sent;
            uint32_t* c = m[u] == h[u] ? &s_hc[(uint32_t)h[u] & (kHeavySlots - 1)] : &cnt[part_of(h[u], log2P)];
            if (ok[u] && !sent) atomicAdd(c, 1u);
        }
    });
    __syncthreads();
    GACE_GLOBAL uint32_t* row = (GACE_GLOBAL uint32_t*)(a.arena_base + jd->rows_off) + (uint64_t)it.sub * P;
    for (uint32_t i = threadIdx.x; i < P; i += kWG) row[i] = cnt[i];
    uint32_t* gc = (uint32_t*)(a.arena_base + jd->heavy_off + kHeavySlots * 8) + (uint64_t)it.side * kHeavySlots;
    for (uint32_t i = threadIdx.x; i < kHeavySlots; i += kWG) {
        const uint32_t c = s_hc[i];
        if (c) atomicAdd(&gc[i], c);
    }
    nall = block_sum(nall, s_red);
    nsent = block_sum(nsent, s_red);
    if (threadIdx.x == 0) {
        GACE_GLOBAL unsigned long long* st = (GACE_GLOBAL unsigned long long*)(a.arena_base + jd->stats_off);
        st[2 * it.sub] = nall;
        st[2 * it.sub + 1] = nsent;
    }
    (void)acc;
}

// offsets of each item inside each partition of 64 partitions (in place:
// a row's counts become its offsets); the partition totals go to base[]
__device__ void joff_item(const BatchArgs& a, const JoinDesc* jd, const Item& it, uint8_t* lds) {
    const uint32_t P = 1u << jd->log2P;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t p = it.sub * 64 + (uint32_t)lane;
    uint32_t* s_part = (uint32_t*)(lds + kLdsMisc);
    GACE_GLOBAL uint32_t* rows = (GACE_GLOBAL uint32_t*)(a.arena_base + jd->rows_off);
    GACE_GLOBAL uint32_t* base = (GACE_GLOBAL uint32_t*)(a.arena_base + jd->base_off);
    for (int s = 0; s < 2; ++s) {
        const JoinSide* D = &jd->side[s];
        const uint32_t ib = D->item_begin, ni = D->n_items;
        const uint32_t q = (ni + kWaves - 1) / kWaves;
        const uint32_t i0 = ib + min(ni, (uint32_t)wave * q), i1 = ib + min(ni, (uint32_t)(wave + 1) * q);
        // 8 independent loads in flight per lane
        uint32_t sum = 0;
        if (p < P) {
            uint32_t i = i0;
            for (; i + 8 <= i1; i += 8) {
                uint32_t v[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) v[k] = rows[(uint64_t)(i + k) * P + p];
#pragma unroll
                for (int k = 0; k < 8; ++k) sum += v[k];
            }
            for (; i < i1; ++i) sum += rows[(uint64_t)i * P + p];
        }
        s_part[wave * 64 + lane] = sum;
        __syncthreads();
        uint32_t run = 0, total = 0;
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t v = s_part[w * 64 + lane];
            if (w < wave) run += v;
            total += v;
        }
        if (p < P) {
            uint32_t i = i0;
            for (; i + 8 <= i1; i += 8) {
                uint32_t v[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) v[k] = rows[(uint64_t)(i + k) * P + p];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    rows[(uint64_t)(i + k) * P + p] = run;
                    run += v[k];
                }
            }
            for (; i < i1; ++i) {
                GACE_GLOBAL uint32_t* e = &rows[(uint64_t)i * P + p];
                const uint32_t v = *e;
                *e = run;
                run += v;
            }
            if (wave == 0) base[(uint64_t)s * (P + 1) + p] = total;
        }
        __syncthreads();
    }
}

// block-wide exclusive prefix of one value per thread (wave scans + the
// waves' totals); *total receives the sum over the block
__device__ __forceinline__ unsigned long long block_excl(unsigned long long v, unsigned long long* s_w,
                                                         unsigned long long* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long y = __shfl_up(x, (unsigned)o);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    unsigned long long pre = 0, all = 0;
    for (int w = 0; w < kWaves; ++w) {
        const unsigned long long t = s_w[w];
        if (w < wave) pre += t;
        all += t;
    }
    *total = all;
    return pre + x - v;
}

__device__ __forceinline__ void put_unit(GACE_GLOBAL AggUnit* u, uint32_t part, uint32_t kind, uint32_t a,
                                         uint32_t b, uint32_t ord) {
    u->part = part;
    u->kind = kind;
    u->a = a;
    u->b = b;
    u->ord = ord;
}

// partition starts per side (exclusive prefix of the totals), per-side key
// totals, the partition buffer and chunk tables carved from the arena, and
// the list of aggregation units: partitions with more than kChunkKeys keys
// are split into chunks followed by one merge unit
// exclusive prefix of s_b[0..P) in place (contiguous chunks per thread);
// s_b[P] receives the total, which is also returned
__device__ __forceinline__ unsigned long long lds_prefix(uint32_t* s_b, uint32_t P, unsigned long long* s_w) {
    const uint32_t chunk = (P + kWG - 1) / kWG;
    const uint32_t lo = min(P, threadIdx.x * chunk), hi = min(P, lo + chunk);
    unsigned long long local = 0, tot = 0;
    for (uint32_t i = lo; i < hi; ++i) local += s_b[i];
    unsigned long long run = block_excl(local, s_w, &tot);
    for (uint32_t i = lo; i < hi; ++i) {
        const uint32_t v = s_b[i];
        s_b[i] = (uint32_t)run;
        run += v;
    }
    if (threadIdx.x == 0) s_b[P] = (uint32_t)tot;
    __syncthreads();
    return tot;
}

// Partition starts per side (exclusive prefix of the totals), per-side key
// totals, the partition buffers and chunk tables carved from the arena, and
// the list of aggregation units: partitions with more than kChunkKeys keys
// are split into chunks followed by one merge unit.  One side's starts are
// staged in LDS at a time; the units are counted while side 1's starts are
// in LDS and side 0 still holds its totals in global memory.
__device__ void jbase_item(const BatchArgs& a, const JoinDesc* jd, uint8_t* lds) {
    JoinAcc& acc = a.accs[jd->acc];
    const uint32_t P = 1u << jd->log2P;
    GACE_GLOBAL uint32_t* base = (GACE_GLOBAL uint32_t*)(a.arena_base + jd->base_off);
    GACE_GLOBAL uint32_t* b0 = base;               // side 0: totals, then starts
    GACE_GLOBAL uint32_t* b1 = base + (P + 1);     // side 1
    unsigned long long* s_w = (unsigned long long*)(lds + 320);     // kWaves wave totals
    uint32_t* s_b = (uint32_t*)(lds + kLdsMisc);                    // [P + 1] staged in LDS
    unsigned long long tot[2];
    // loads of totals go out eight per thread at a time: one memory round
    // trip per eight partitions of a thread instead of one per partition
    constexpr uint32_t kBatch = 8;
    auto stage = [&](const GACE_GLOBAL uint32_t* src) __attribute__((always_inline)) {
        for (uint32_t i0 = threadIdx.x; i0 < P; i0 += kBatch * kWG) {
            uint32_t v[kBatch];
#pragma unroll
            for (uint32_t u = 0; u < kBatch; ++u) v[u] = i0 + u * kWG < P ? src[i0 + u * kWG] : 0u;
#pragma unroll
            for (uint32_t u = 0; u < kBatch; ++u)
                if (i0 + u * kWG < P) s_b[i0 + u * kWG] = v[u];
        }
    };
    // side 1 starts
    stage(b1);
    __syncthreads();
    tot[1] = lds_prefix(s_b, P, s_w);
    for (uint32_t i = threadIdx.x; i <= P; i += kWG) b1[i] = s_b[i];
    // aggregation units (partitions interleaved over threads: coalesced reads;
    // the unit order only needs chunks, then whole partitions, then merges)
    auto np_of = [&](uint32_t p, uint32_t t0) { return (uint64_t)t0 + (s_b[p + 1] - s_b[p]); };
    unsigned long long n_chunk = 0, n_small = 0, n_split = 0;
    for (uint32_t p0 = threadIdx.x; p0 < P; p0 += kBatch * kWG) {
        uint32_t v[kBatch];
#pragma unroll
        for (uint32_t u = 0; u < kBatch; ++u) v[u] = p0 + u * kWG < P ? b0[p0 + u * kWG] : 0u;
#pragma unroll
        for (uint32_t u = 0; u < kBatch; ++u) {
            const uint32_t p = p0 + u * kWG;
            if (p >= P) break;
            const uint64_t np = np_of(p, v[u]);
            if (np > kChunkKeys) {
                n_chunk += (np + kChunkKeys - 1) / kChunkKeys;
                n_split += 1;
            } else if (np) {
                n_small += 1;
            }
        }
    }
    unsigned long long t_chunk, t_small, t_split;
    unsigned long long c_at = block_excl(n_chunk, s_w, &t_chunk);
    unsigned long long s_at = block_excl(n_small, s_w, &t_small) + t_chunk;
    unsigned long long m_ord = block_excl(n_split, s_w, &t_split);
    GACE_GLOBAL AggUnit* units = (GACE_GLOBAL AggUnit*)(a.arena_base + jd->units_off);
    GACE_GLOBAL uint32_t* done = (GACE_GLOBAL uint32_t*)(a.arena_base + jd->done_off);
    const bool fits = t_chunk <= jd->max_chunks && t_chunk + t_small + t_split <= jd->max_units;
    if (fits) {
        for (uint32_t p0 = threadIdx.x; p0 < P; p0 += kBatch * kWG) {
            uint32_t v[kBatch];
#pragma unroll
            for (uint32_t u = 0; u < kBatch; ++u) v[u] = p0 + u * kWG < P ? b0[p0 + u * kWG] : 0u;
            for (uint32_t u = 0; u < kBatch; ++u) {
                const uint32_t p = p0 + u * kWG;
                if (p >= P) break;
                const uint64_t np = np_of(p, v[u]);
                if (np > kChunkKeys) {
                    const uint32_t nc = (uint32_t)((np + kChunkKeys - 1) / kChunkKeys);
                    for (uint32_t c = 0; c < nc; ++c)
                        put_unit(units + c_at + c, p, AU_CHUNK, c, (uint32_t)(c_at + c), (uint32_t)m_ord);
                    put_unit(units + t_chunk + t_small + m_ord, p, AU_MERGE, (uint32_t)c_at, nc, (uint32_t)m_ord);
                    done[m_ord] = 0;
                    c_at += nc;
                    m_ord += 1;
                } else if (np) {
                    put_unit(units + s_at, p, AU_SMALL, 0, 0, 0);
                    ++s_at;
                }
            }
        }
    }
    __syncthreads();
    // side 0 starts
    stage(b0);
    __syncthreads();
    tot[0] = lds_prefix(s_b, P, s_w);
    for (uint32_t i = threadIdx.x; i <= P; i += kWG) b0[i] = s_b[i];
    // per-side sampled and sentinel key counts from the histogram items
    {
        const GACE_GLOBAL unsigned long long* st =
            (const GACE_GLOBAL unsigned long long*)(a.arena_base + jd->stats_off);
        unsigned long long v[4] = {0, 0, 0, 0};
        for (int sd = 0; sd < 2; ++sd)
            for (uint32_t i = jd->side[sd].item_begin + threadIdx.x;
                 i < jd->side[sd].item_begin + jd->side[sd].n_items; i += kWG) {
                v[2 * sd] += st[2 * i];
                v[2 * sd + 1] += st[2 * i + 1];
            }
        unsigned long long* s_red = (unsigned long long*)(lds + 320);
        for (int k = 0; k < 4; ++k) v[k] = block_sum(v[k], s_red);
        if (threadIdx.x == 0) {
            acc.n[0] = v[0];
            acc.sent[0] = v[1];
            acc.n[1] = v[2];
            acc.sent[1] = v[3];
        }
    }
    // the heavy table's keys, counted outside the partitions: their share of
    // the join size, the distinct counts and the keys seen once or twice
    {
        const GACE_GLOBAL uint32_t* gc = (const GACE_GLOBAL uint32_t*)(a.arena_base + jd->heavy_off + kHeavySlots * 8);
        unsigned long long v[7] = {0, 0, 0, 0, 0, 0, 0};
        for (uint32_t i = threadIdx.x; i < kHeavySlots; i += kWG) {
            const uint32_t x = gc[i], y = gc[kHeavySlots + i];
            v[0] += (unsigned long long)x * y;
            v[1] += x != 0;
            v[2] += y != 0;
            v[3] += x == 1;
            v[4] += y == 1;
            v[5] += x == 2;
            v[6] += y == 2;
        }
        unsigned long long* s_red = (unsigned long long*)(lds + 320);
        for (int k = 0; k < 7; ++k) v[k] = block_sum(v[k], s_red);
        if (threadIdx.x == 0) {
            if (v[0]) atomicAdd(&acc.join, v[0]);
            if (v[1]) atomicAdd(&acc.ndv[0], v[1]);
            if (v[2]) atomicAdd(&acc.ndv[1], v[2]);
            if (v[3]) atomicAdd(&acc.f1[0], v[3]);
            if (v[4]) atomicAdd(&acc.f1[1], v[4]);
            if (v[5]) atomicAdd(&acc.f2[0], v[5]);
            if (v[6]) atomicAdd(&acc.f2[1], v[6]);
        }
    }
    if (threadIdx.x == 0) {
        acc.nkeys[0] = tot[0];
        acc.nkeys[1] = tot[1];
        acc.n_units = (uint32_t)(t_chunk + t_small + t_split);
        const unsigned long long kbytes = 8ull * (tot[0] + tot[1]);
        const unsigned long long tbytes = jd->log2P2 ? kbytes : 0ull;
        const unsigned long long mbytes = t_chunk * (unsigned long long)kChunkKeys * sizeof(MergeEntry);
        const unsigned long long off = atomicAdd(&a.arena->used, kbytes + tbytes + mbytes);
        if (!fits || off + kbytes + tbytes + mbytes > a.arena->size) acc.status = 2;
        acc.buf_off = off;
        acc.tmp_off = off + kbytes;
        acc.merge_off = off + kbytes + tbytes;
    }
}

// ---- LDS-staged partitioning
// A tile of up to kWG * KP keys is counting-sorted by digit in LDS and each
// digit's run is written to its output cursor with consecutive lanes on
// consecutive addresses, so the partition writes are whole cache lines
// instead of one scattered 8-byte store per key.
struct TileLds {
    uint32_t* cur;               // [F] output cursor per digit (keys from the side's buffer start)
    uint32_t* cnt;               // [F] tile count per digit
    uint32_t* start;             // [F + 1] tile start per digit; start[F] = keys in the tile
    unsigned long long* key;     // [kWG * KP] keys sorted by digit
    uint32_t* dest;              // [kWG * KP] their output index
};

template <int KP>
__device__ __forceinline__ TileLds tile_lds(uint8_t* lds) {
    TileLds L;
    L.cur = (uint32_t*)(lds + kLdsMisc);
    L.cnt = L.cur + 132;
    L.start = L.cnt + 132;
    L.key = (unsigned long long*)(lds + kLdsMisc + 3 * 132 * 4);
    L.dest = (uint32_t*)(L.key + (uint32_t)KP * kWG);
    return L;
}

// The tile's entries are keys (first pass: hashed here, sentinel keys and
// keys of the heavy table hh dropped) or hashes (second pass); the hashes are
// written out.  Digit of a
// hash: (hash >> shift) mod F (F a power of two <= 128).  All digits are
// computed first and the rank atomics issued back to back, so their LDS
// latencies overlap; each entry's output index is recorded beside it, so the
// copy-out reads two independent LDS words per entry.
// L.cnt must be zero on entry (it is again on return).
template <bool kKeys, int KP>
__device__ void tile_partition(uint64_t (&k)[KP], uint32_t nt, uint32_t shift, uint32_t F,
                               GACE_GLOBAL int64_t* dst, const TileLds& L, const unsigned long long* hh) {
    uint32_t d[KP], r[KP];   // digit (~0: no entry at this position) and rank within it
#pragma unroll
    for (int u = 0; u < KP; ++u) {
        const uint32_t pos = threadIdx.x + (uint32_t)u * kWG;
        bool ok = pos < nt && (!kKeys || k[u] != kEmptyKey);
        if (kKeys) {
            k[u] = mix_key(k[u]);
            const bool heavy = hh[(uint32_t)k[u] & (kHeavySlots - 1)] == k[u];   // read for every position
            ok = ok && !heavy;
        }
        const uint32_t dg = F > 1 ? (uint32_t)(k[u] >> shift) & (F - 1) : 0u;
        d[u] = ok ? dg : ~0u;
    }
#pragma unroll
    for (int u = 0; u < KP; ++u) r[u] = d[u] != ~0u ? atomicAdd(&L.cnt[d[u]], 1u) : 0u;
    __syncthreads();
    if (threadIdx.x < 64) {
        const uint32_t lane = threadIdx.x;
        const uint32_t a0 = 2 * lane < F ? L.cnt[2 * lane] : 0u;
        const uint32_t a1 = 2 * lane + 1 < F ? L.cnt[2 * lane + 1] : 0u;
        uint32_t x = a0 + a1;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if ((int)lane >= o) x += y;
        }
        const uint32_t ex = x - a0 - a1;
        if (2 * lane < F) L.start[2 * lane] = ex;
        if (2 * lane + 1 < F) L.start[2 * lane + 1] = ex + a0;
        if (lane == 63) L.start[F] = x;
    }
    __syncthreads();
    // all LDS reads of a step are issued before any dependent write, so their
    // latencies overlap (indices are clamped in range; writes stay guarded)
    {
        uint32_t st[KP], cu[KP];
#pragma unroll
        for (int u = 0; u < KP; ++u) {
            const uint32_t dd = d[u] != ~0u ? d[u] : 0u;
            st[u] = L.start[dd];
            cu[u] = L.cur[dd];
        }
#pragma unroll
        for (int u = 0; u < KP; ++u) {
            if (d[u] != ~0u) {
                const uint32_t at = st[u] + r[u];
                L.key[at] = k[u];
                L.dest[at] = cu[u] + r[u];
            }
        }
    }
    __syncthreads();
    {
        const uint32_t m = L.start[F];
        uint32_t de[KP];
        unsigned long long kk[KP];
#pragma unroll
        for (int u = 0; u < KP; ++u) {
            const uint32_t i = threadIdx.x + (uint32_t)u * kWG;
            const uint32_t ic = i < m ? i : 0u;
            de[u] = L.dest[ic];
            kk[u] = L.key[ic];
        }
#pragma unroll
        for (int u = 0; u < KP; ++u) {
            const uint32_t i = threadIdx.x + (uint32_t)u * kWG;
            if (i < m) dst[de[u]] = (int64_t)kk[u];
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < F; i += kWG) {
        L.cur[i] += L.cnt[i];
        L.cnt[i] = 0;
    }
    __syncthreads();
}

// calls f(k, nt) for consecutive tiles of the sampled keys of blocks [b0, b1)
// of one side: tile position t (thread + u * kWG) holds k[u] when t < nt.
// Tiles run over the concatenated rows of the kept blocks of each 64-block
// decision chunk, so small blocks still fill whole tiles.
template <int KP, typename F>
__device__ void for_each_tile(const JoinSide* D, uint64_t b0, uint64_t b1, uint8_t* lds, F&& f) {
    constexpr uint64_t kTile = (uint64_t)KP * kWG;
    uint32_t* s_w0 = (uint32_t*)lds;
    unsigned long long* s_keep = (unsigned long long*)(lds + 256);
    uint32_t* s_kidx = (uint32_t*)(lds + 384);
    const uint32_t log2B = D->log2B;
    const uint64_t B = 1ull << log2B, n = D->n;
    const GACE_GLOBAL int64_t* keys = (const GACE_GLOBAL int64_t*)D->keys;
    for (uint64_t cb = b0; cb < b1; cb += 64) {
        decide_blocks(cb, b1, D->thr, D->table_id, D->seed, s_w0, s_keep);
        __syncthreads();
        const unsigned long long keep = *s_keep;
        if (threadIdx.x < 64 && ((keep >> threadIdx.x) & 1ull))
            s_kidx[__popcll(keep & ((1ull << threadIdx.x) - 1ull))] = threadIdx.x;
        __syncthreads();
        const uint32_t c = (uint32_t)__popcll(keep);
        if (c) {
            // only the side's final block can be short, and it is the chunk's last kept block
            const uint64_t last = (cb + s_kidx[c - 1]) << log2B;
            const uint64_t total = (uint64_t)(c - 1) * B + min(B, n - last);
            // the next tile's keys are loaded while this tile is partitioned
            // positions past the end are clamped to the last one (loads stay
            // unconditional); the partitioner ignores them
            auto load = [&](uint64_t t0, uint64_t (&k)[KP]) {
#pragma unroll
                for (int u = 0; u < KP; ++u) {
                    uint64_t pos = t0 + threadIdx.x + (uint64_t)u * kWG;
                    pos = pos < total ? pos : total - 1;
                    const uint64_t row = ((cb + s_kidx[pos >> log2B]) << log2B) + (pos & (B - 1));
                    k[u] = (uint64_t)__builtin_nontemporal_load(keys + row);
                }
            };
            uint64_t k[KP], kn[KP];
            load(0, k);
            for (uint64_t t0 = 0; t0 < total; t0 += kTile) {
                const uint32_t nt = (uint32_t)min((uint64_t)kTile, total - t0);
                const bool more = t0 + kTile < total;
                if (more) load(t0 + kTile, kn);
                f(k, nt);
                if (more) {
#pragma unroll
                    for (int u = 0; u < KP; ++u) k[u] = kn[u];
                }
            }
        }
        __syncthreads();
    }
}

// first pass: each item's keys go to their first-pass bucket (top log2P1
// hash bits) in the temporary buffer, or straight to their partition when one
// pass suffices.  An item's run inside a bucket starts at the sum of its
// offsets in the bucket's partitions, so both passes place keys in item order.
template <int KP>
__device__ void jscatter_item(const BatchArgs& a, const JoinDesc* jd, const Item& it, uint8_t* lds) {
    JoinAcc& acc = a.accs[jd->acc];
    const uint32_t log2P = jd->log2P, P = 1u << log2P, log2P2 = jd->log2P2, log2P1 = log2P - log2P2;
    const uint32_t F1 = 1u << log2P1;
    const GACE_GLOBAL uint32_t* base =
        (const GACE_GLOBAL uint32_t*)(a.arena_base + jd->base_off) + (uint64_t)it.side * (P + 1);
    const GACE_GLOBAL uint32_t* row = (const GACE_GLOBAL uint32_t*)(a.arena_base + jd->rows_off) + (uint64_t)it.sub * P;
    const TileLds L = tile_lds<KP>(lds);
    unsigned long long* s_hh = (unsigned long long*)(lds + heavy_lds_off(KP * kWG));
    stage_heavy(a, jd, s_hh);
    for (uint32_t i = threadIdx.x; i < F1; i += kWG) {
        L.cur[i] = 0;
        L.cnt[i] = 0;
    }
    __syncthreads();
    for (uint32_t p = threadIdx.x; p < P; p += kWG) atomicAdd(&L.cur[p >> log2P2], row[p]);
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < F1; b += kWG) L.cur[b] += base[b << log2P2];
    __syncthreads();
    if (__hip_atomic_load(&acc.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    GACE_GLOBAL int64_t* dst = (GACE_GLOBAL int64_t*)(a.arena_base + (log2P2 ? acc.tmp_off : acc.buf_off)) +
                               (it.side ? acc.nkeys[0] : 0ull);
    const uint32_t shift = 64 - log2P1;
    for_each_tile<KP>(&jd->side[it.side], it.begin, it.end, lds,
                      [&](uint64_t (&k)[KP], uint32_t nt) { tile_partition<true, KP>(k, nt, shift, F1, dst, L, s_hh); });
}

// second pass: a unit is one first-pass bucket of a group of consecutive
// items of one side; its keys are contiguous in the temporary buffer and are
// partitioned by the next log2P2 hash bits into their final partitions, where
// the group's run starts at the first item's offsets
template <int KP>
__device__ void jscatter2_item(const BatchArgs& a, const JoinDesc* jd, uint8_t* lds) {
    constexpr uint64_t kTile = (uint64_t)KP * kWG;
    JoinAcc& acc = a.accs[jd->acc];
    const uint32_t log2P = jd->log2P, P = 1u << log2P, log2P2 = jd->log2P2, log2P1 = log2P - log2P2;
    const uint32_t F1 = 1u << log2P1, F2 = 1u << log2P2;
    const GACE_GLOBAL uint32_t* rows = (const GACE_GLOBAL uint32_t*)(a.arena_base + jd->rows_off);
    uint32_t* s_ctl = (uint32_t*)(lds + 352);
    const TileLds L = tile_lds<KP>(lds);
    if (__hip_atomic_load(&acc.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const uint32_t units0 = jd->n_groups[0] << log2P1;
    const uint32_t shift = 64 - log2P;
    for (;;) {
        if (threadIdx.x == 0) s_ctl[2] = atomicAdd(&acc.next_s2, 1u);
        __syncthreads();
        const uint32_t u = s_ctl[2];
        __syncthreads();
        if (u >= jd->n_units2) break;
        const uint32_t side = u >= units0 ? 1u : 0u;
        const uint32_t uu = side ? u - units0 : u;
        const uint32_t g = uu >> log2P1, b = uu & (F1 - 1);
        const JoinSide& D = jd->side[side];
        const uint32_t i0 = D.item_begin + g * jd->group_items;
        const uint32_t iend = D.item_begin + D.n_items;
        const uint32_t i1 = min(iend, i0 + jd->group_items);
        const GACE_GLOBAL uint32_t* base = (const GACE_GLOBAL uint32_t*)(a.arena_base + jd->base_off) +
                                           (uint64_t)side * (P + 1);
        const uint32_t p0 = b << log2P2;
        // F2 <= 128 sub-partitions: one per thread of the first two waves,
        // each wave's sums of the group's start and end offsets in s_ctl[4..7]
        if (threadIdx.x < 128) {
            const uint32_t q = threadIdx.x;
            uint32_t o0 = 0, o1 = 0;
            L.cnt[q] = 0;
            if (q < F2) {
                o0 = rows[(uint64_t)i0 * P + p0 + q];
                o1 = i1 < iend ? rows[(uint64_t)i1 * P + p0 + q] : base[p0 + q + 1] - base[p0 + q];
                L.cur[q] = base[p0 + q] + o0;
            }
            for (int o = 32; o; o >>= 1) {
                o0 += __shfl_xor(o0, o);
                o1 += __shfl_xor(o1, o);
            }
            if ((q & 63) == 0) {
                s_ctl[4 + 2 * (q >> 6)] = o0;
                s_ctl[5 + 2 * (q >> 6)] = o1;
            }
        }
        __syncthreads();
        const uint64_t side_off = side ? acc.nkeys[0] : 0ull;
        const GACE_GLOBAL int64_t* src = (const GACE_GLOBAL int64_t*)(a.arena_base + acc.tmp_off) + side_off;
        GACE_GLOBAL int64_t* dst = (GACE_GLOBAL int64_t*)(a.arena_base + acc.buf_off) + side_off;
        const uint64_t lo = (uint64_t)base[p0] + s_ctl[4] + s_ctl[6];
        const uint64_t hi = (uint64_t)base[p0] + s_ctl[5] + s_ctl[7];
        __syncthreads();
        auto load = [&](uint64_t t0, uint64_t (&k)[KP]) {
#pragma unroll
            for (int u2 = 0; u2 < KP; ++u2) {
                const uint64_t pos = t0 + threadIdx.x + (uint64_t)u2 * kWG;
                k[u2] = (uint64_t)__builtin_nontemporal_load(src + (pos < hi ? pos : hi - 1));
            }
        };
        uint64_t k[KP], kn[KP];
        if (lo < hi) load(lo, k);
        for (uint64_t t0 = lo; t0 < hi; t0 += kTile) {
            const uint32_t nt = (uint32_t)min((uint64_t)kTile, hi - t0);
            const bool more = t0 + kTile < hi;
            if (more) load(t0 + kTile, kn);
            tile_partition<false, KP>(k, nt, shift, F2, dst, L, nullptr);
            if (more) {
#pragma unroll
                for (int u2 = 0; u2 < KP; ++u2) k[u2] = kn[u2];
            }
        }
    }
}

// LDS table of one aggregation pass: `slots` (a power of two) entries of
// which at most `limit` (3/4) may be claimed
struct AggLds {
    unsigned long long* key;
    uint32_t* c0;
    uint32_t* c1;
    uint32_t slots, limit;
};

// table size for a unit of n entries: a power of two with n <= 3/4 of it when
// it fits, so a unit of at most 3/4 of the largest table never overflows
__device__ __forceinline__ void agg_size(AggLds& T, uint64_t n, uint32_t cap) {
    uint32_t s = kAggMinSlots;
    while (s < cap && (uint64_t)s * 3 < n * 4) s <<= 1;
    T.slots = s;
    T.limit = s / 4 * 3;
}

// Insert entries whose hash lies in residue class res mod m.
// Each lane loads kAggBatch entries, then all of them probe together: every
// step issues the pending entries' slot reads at once, then their claims of
// empty slots (compare-and-swap) at once, so a step costs two LDS round
// trips for all of them.  Claimed slots are counted once per wave; past 3/4
// of the table the pass is abandoned (the spare quarter absorbs the keys
// inserted before the count catches up) and redone on split residue classes;
// so is a pass that finds the table full.
constexpr int kAggBatch = 2;

// Probe kAggBatch entries per lane into the table.  Slots are paired into
// buckets read with one 16-byte LDS load: an entry matches either slot of
// its bucket, or claims the bucket's first empty slot, or, when the bucket
// is full of other hashes, moves to the next bucket (slots only ever fill,
// so a hash is always in the first bucket that had room for it).  Counts
// the wave's claimed slots and flags an overflow in s_ctl[1].
__device__ __forceinline__ void agg_probe(AggLds& T, const uint64_t (&h)[kAggBatch], const uint32_t (&c0)[kAggBatch],
                                          const uint32_t (&c1)[kAggBatch], uint64_t m, uint64_t res,
                                          uint32_t* s_ctl) {
    const int lane = threadIdx.x & 63;
    const uint32_t nb = T.slots / 2, bmask = nb - 1;
    uint32_t bk[kAggBatch];
    bool pend[kAggBatch];
#pragma unroll
    for (int u = 0; u < kAggBatch; ++u) {
        pend[u] = (c0[u] | c1[u]) != 0u && (h[u] & (m - 1)) == res;
        bk[u] = (uint32_t)(h[u] >> 20) & bmask;
    }
    uint32_t took = 0;
    for (uint32_t probe = 0;; ++probe) {
        bool any = false;
#pragma unroll
        for (int u = 0; u < kAggBatch; ++u) any |= pend[u];
        if (!__ballot(any)) break;
        if (probe >= nb) {               // every bucket probed: the table is full
            s_ctl[1] = 1;
            break;
        }
        u64x2 cur[kAggBatch];
#pragma unroll
        for (int u = 0; u < kAggBatch; ++u)
            cur[u] = pend[u] ? *(const u64x2*)(T.key + 2 * bk[u]) : u64x2{0ull, 0ull};
        int at[kAggBatch];
#pragma unroll
        for (int u = 0; u < kAggBatch; ++u) {
            at[u] = -1;
            if (!pend[u]) continue;
            if (cur[u].x == h[u]) {
                at[u] = 0;
            } else if (cur[u].y == h[u]) {
                at[u] = 1;
            } else if (cur[u].x == kEmptyHash || cur[u].y == kEmptyHash) {
                const int t = cur[u].x == kEmptyHash ? 0 : 1;
                unsigned long long o =
                    atomicCAS(&T.key[2 * bk[u] + t], (unsigned long long)kEmptyHash, (unsigned long long)h[u]);
                if (o == kEmptyHash) {
                    at[u] = t;
                    ++took;
                } else if (o == h[u]) {
                    at[u] = t;
                } else if (t == 0 && cur[u].y == kEmptyHash) {
                    o = atomicCAS(&T.key[2 * bk[u] + 1], (unsigned long long)kEmptyHash, (unsigned long long)h[u]);
                    if (o == kEmptyHash) {
                        at[u] = 1;
                        ++took;
                    } else if (o == h[u]) {
                        at[u] = 1;
                    }
                }
                // a lost claim re-reads the same bucket next step
            } else {
                bk[u] = (bk[u] + 1) & bmask;   // bucket full of other hashes
            }
        }
#pragma unroll
        for (int u = 0; u < kAggBatch; ++u)
            if (pend[u] && at[u] >= 0) {
                const uint32_t sl = 2 * bk[u] + (uint32_t)at[u];
                if (c0[u]) atomicAdd(&T.c0[sl], c0[u]);
                if (c1[u]) atomicAdd(&T.c1[sl], c1[u]);
                pend[u] = false;
            }
    }
    uint32_t wt = took;
    for (int o = 32; o; o >>= 1) wt += __shfl_xor(wt, o);
    if (lane == 0 && wt && atomicAdd(&s_ctl[0], wt) + wt > T.limit) s_ctl[1] = 1;
}

// chunk-table entries (merge units): one batch at a time
__device__ __forceinline__ void agg_entries(AggLds& T, const GACE_GLOBAL MergeEntry* ent, uint64_t n, uint64_t m,
                                            uint64_t res, uint32_t* s_ctl) {
    for (uint64_t e0 = 0; e0 < n; e0 += (uint64_t)kWG * kAggBatch) {
        if (__hip_atomic_load(&s_ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
        uint64_t h[kAggBatch];
        uint32_t c0[kAggBatch], c1[kAggBatch];
#pragma unroll
        for (int u = 0; u < kAggBatch; ++u) {
            const uint64_t e = e0 + (uint64_t)u * kWG + threadIdx.x;
            h[u] = e < n ? ent[e].key : kEmptyHash;
            c0[u] = e < n ? ent[e].c0 : 0u;
            c1[u] = e < n ? ent[e].c1 : 0u;
        }
        agg_probe(T, h, c0, c1, m, res, s_ctl);
    }
}

// bare hashes of a unit: nR of side R then nS of side S, as one stream whose
// next batch is loaded while the current one probes
__device__ __forceinline__ void agg_bare(AggLds& T, const GACE_GLOBAL int64_t* hr, uint64_t nR,
                                         const GACE_GLOBAL int64_t* hs, uint64_t nS, uint64_t m, uint64_t res,
                                         uint32_t* s_ctl) {
    const uint64_t total = nR + nS;
    // one unconditional load per entry (positions past the end are clamped
    // to the last entry and carry zero counts)
    auto load = [&](uint64_t e0, uint64_t (&h)[kAggBatch]) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < kAggBatch; ++u) {
            uint64_t e = e0 + (uint64_t)u * kWG + threadIdx.x;
            e = e < total ? e : total - 1;
            const GACE_GLOBAL int64_t* p = e < nR ? hr + e : hs + (e - nR);
            h[u] = (uint64_t)__builtin_nontemporal_load(p);
        }
    };
    if (total == 0) return;
    uint64_t h[kAggBatch], hn[kAggBatch];
    load(0, h);
    for (uint64_t e0 = 0; e0 < total; e0 += (uint64_t)kWG * kAggBatch) {
        if (__hip_atomic_load(&s_ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
        const uint64_t e1 = e0 + (uint64_t)kWG * kAggBatch;
        if (e1 < total) load(e1, hn);
        uint32_t c0[kAggBatch], c1[kAggBatch];
#pragma unroll
        for (int u = 0; u < kAggBatch; ++u) {
            const uint64_t e = e0 + (uint64_t)u * kWG + threadIdx.x;
            c0[u] = e < nR ? 1u : 0u;
            c1[u] = e >= nR && e < total ? 1u : 0u;
        }
        agg_probe(T, h, c0, c1, m, res, s_ctl);
        if (e1 < total) {
#pragma unroll
            for (int u = 0; u < kAggBatch; ++u) h[u] = hn[u];
        }
    }
}

// The LDS table is clean (every slot empty, counts zero) whenever no pass is
// running: a pass that completes resets each slot as it reads it out, one
// that overflows clears the slots it used.  The worker clears the whole
// region once before its first unit.
__device__ __forceinline__ void agg_clear(AggLds& T, uint32_t slots) {
    for (uint32_t i = threadIdx.x; i < slots; i += kWG) {
        T.key[i] = kEmptyHash;
        T.c0[i] = 0;
        T.c1[i] = 0;
    }
}

// pass(m, res) inserts every entry of the unit in residue class res mod m
template <typename Pass>
__device__ void aggregate(AggLds& T, Pass&& pass, uint32_t* s_ctl, uint32_t* stack,
                          GACE_GLOBAL MergeEntry* emit, unsigned long long& n0, unsigned long long& n1,
                          unsigned long long& jn, uint32_t (&ff)[4], JoinAcc& acc, uint32_t& passes) {
    const int lane = threadIdx.x & 63;
    if (threadIdx.x == 0) {
        stack[0] = 1;
        stack[1] = 0;
        s_ctl[3] = 1;
        s_ctl[6] = 0;
    }
    __syncthreads();
    while (s_ctl[3] > 0) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t sp = s_ctl[3] - 1;
            s_ctl[4] = stack[2 * sp];
            s_ctl[5] = stack[2 * sp + 1];
            s_ctl[3] = sp;
            s_ctl[0] = 0;
            s_ctl[1] = 0;
        }
        __syncthreads();
        const uint64_t m = s_ctl[4], res = s_ctl[5];
        ++passes;
        pass(m, res);
        __syncthreads();
        if (s_ctl[1]) {
            agg_clear(T, T.slots);
            if (threadIdx.x == 0) {
                const uint32_t sp = s_ctl[3];
                if (m < (1u << 20) && sp + 2 <= 64) {
                    stack[2 * sp] = 2 * (uint32_t)m;
                    stack[2 * sp + 1] = (uint32_t)res;
                    stack[2 * sp + 2] = 2 * (uint32_t)m;
                    stack[2 * sp + 3] = (uint32_t)(res + m);
                    s_ctl[3] = sp + 2;
                } else {
                    atomicMax(&acc.status, 3ull);
                    s_ctl[3] = 0;
                }
            }
        } else {
            for (uint32_t i0 = 0; i0 < T.slots; i0 += kWG) {
                const uint32_t i = i0 + threadIdx.x;
                unsigned long long k = kEmptyHash;
                uint32_t x = 0, y = 0;
                if (i < T.slots) {
                    k = T.key[i];
                    x = T.c0[i];
                    y = T.c1[i];
                    if (k != kEmptyHash) {
                        T.key[i] = kEmptyHash;
                        T.c0[i] = 0;
                        T.c1[i] = 0;
                    }
                }
                const bool full = k != kEmptyHash;
                if (emit) {
                    // one slot claim per wave for its entries
                    const unsigned long long fb = __ballot(full);
                    uint32_t base = 0;
                    if (lane == 0 && fb) base = atomicAdd(&s_ctl[6], (uint32_t)__popcll(fb));
                    base = __shfl(base, 0);
                    if (full) {
                        const uint32_t at = base + (uint32_t)__popcll(fb & ((1ull << lane) - 1ull));
                        emit[at].key = k;
                        emit[at].c0 = x;
                        emit[at].c1 = y;
                    }
                } else if (full) {
                    n0 += x != 0;
                    n1 += y != 0;
                    jn += (unsigned long long)x * y;
                    ff[0] += x == 1;      // keys seen once / twice per side
                    ff[1] += y == 1;
                    ff[2] += x == 2;
                    ff[3] += y == 2;
                }
            }
        }
        __syncthreads();
    }
}

// work: aggregation units taken << 32 | table passes made
__device__ void jagg_item(const BatchArgs& a, const JoinDesc* jd, const Item& it, uint8_t* lds, uint64_t& work) {
    uint32_t n_taken = 0, passes = 0;
    JoinAcc& acc = a.accs[jd->acc];
    const uint32_t P = 1u << jd->log2P;
    unsigned long long* s_red = (unsigned long long*)(lds + 320);
    uint32_t* s_ctl = (uint32_t*)(lds + 352);   // [0] claims [1] over [2] unit [3] sp [4] m [5] r [6] emitted [7] merge ready
    AggLds T;
    const uint32_t cap = a.agg_slots;
    T.key = (unsigned long long*)(lds + kLdsMisc);
    T.c0 = (uint32_t*)(lds + kLdsMisc + cap * 8);
    T.c1 = (uint32_t*)(lds + kLdsMisc + cap * 12);
    uint32_t* stack = (uint32_t*)(lds + kLdsMisc + cap * 16);   // 64 x (m, r)
    const GACE_GLOBAL uint32_t* base0 = (const GACE_GLOBAL uint32_t*)(a.arena_base + jd->base_off);
    const GACE_GLOBAL uint32_t* base1 = base0 + (P + 1);
    const GACE_GLOBAL AggUnit* units = (const GACE_GLOBAL AggUnit*)(a.arena_base + jd->units_off);
    GACE_GLOBAL uint32_t* chunk_cnt = (GACE_GLOBAL uint32_t*)(a.arena_base + jd->chunk_off);
    uint32_t* done = (uint32_t*)(a.arena_base + jd->done_off);
    unsigned long long jn = 0, n0 = 0, n1 = 0;
    uint32_t ff[4] = {0, 0, 0, 0};
    const bool dead = __hip_atomic_load(&acc.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    const GACE_GLOBAL int64_t* bufR = (const GACE_GLOBAL int64_t*)(a.arena_base + acc.buf_off);
    const GACE_GLOBAL int64_t* bufS = bufR + acc.nkeys[0];
    GACE_GLOBAL MergeEntry* merge = (GACE_GLOBAL MergeEntry*)(a.arena_base + acc.merge_off);
    const uint32_t n_units = acc.n_units;
    if (!dead) agg_clear(T, a.agg_slots);
    // thread 0 claims the next unit while the current one is aggregated
    uint32_t claim_next = 0;
    if (threadIdx.x == 0) s_ctl[2] = dead ? ~0u : atomicAdd(&acc.next_unit, 1u);
    __syncthreads();
    while (!dead) {
        const uint32_t u = s_ctl[2];
        __syncthreads();
        if (u >= n_units) break;
        if (threadIdx.x == 0) claim_next = atomicAdd(&acc.next_unit, 1u);
        AggUnit U;
        U.part = units[u].part;
        U.kind = units[u].kind;
        U.a = units[u].a;
        U.b = units[u].b;
        U.ord = units[u].ord;
        const uint32_t p = U.part;
        const uint64_t bR = base0[p], nR = base0[p + 1] - bR, bS = base1[p], nS = base1[p + 1] - bS;
        if (U.kind == AU_MERGE) {
            // wait until every chunk of this partition has emitted its table
            // (bounded like the phase waits: giving up fails the join)
            if (threadIdx.x == 0) {
                const bool ok = poll_count(&done[U.ord], U.b, a.spin_limit);
                if (!ok) atomicMax(&acc.status, 4ull);
                s_ctl[7] = ok ? 1u : 0u;
            }
            __syncthreads();
            __threadfence();
            if (!s_ctl[7]) {
                ++n_taken;
                if (threadIdx.x == 0) s_ctl[2] = claim_next;
                __syncthreads();
                continue;
            }
            agg_size(T, (uint64_t)a.agg_slots, a.agg_slots);
            aggregate(
                T,
                [&](uint64_t m, uint64_t res) {
                    for (uint32_t c = 0; c < U.b; ++c)
                        agg_entries(T, merge + (uint64_t)(U.a + c) * kChunkKeys, chunk_cnt[U.a + c], m, res, s_ctl);
                },
                s_ctl, stack, nullptr, n0, n1, jn, ff, acc, passes);
            ++n_taken;
            if (threadIdx.x == 0) s_ctl[2] = claim_next;
            __syncthreads();
            continue;
        }
        uint64_t lo = 0, hi = nR + nS;
        if (U.kind == AU_CHUNK) {
            lo = (uint64_t)U.a * kChunkKeys;
            hi = min(hi, lo + kChunkKeys);
        }
        // the unit's entries: [lo, hi) of the partition's R hashes followed by its S hashes
        const uint64_t r0 = lo < nR ? lo : nR, r1 = hi < nR ? hi : nR;
        const uint64_t s0 = lo > nR ? lo - nR : 0, s1 = hi > nR ? hi - nR : 0;
        auto pass = [&](uint64_t m, uint64_t res) {
            agg_bare(T, bufR + bR + r0, r1 - r0, bufS + bS + s0, s1 - s0, m, res, s_ctl);
        };
        agg_size(T, hi - lo, a.agg_slots);
        if (U.kind == AU_CHUNK) {
            aggregate(T, pass, s_ctl, stack, merge + (uint64_t)U.b * kChunkKeys, n0, n1, jn, ff, acc, passes);
            if (threadIdx.x == 0) {
                chunk_cnt[U.b] = s_ctl[6];
                __threadfence();
                atomicAdd(&done[U.ord], 1u);
            }
        } else {
            aggregate(T, pass, s_ctl, stack, nullptr, n0, n1, jn, ff, acc, passes);
        }
        ++n_taken;
        if (threadIdx.x == 0) s_ctl[2] = claim_next;
        __syncthreads();
    }
    work = (uint64_t)n_taken << 32 | passes;
    jn = block_sum(jn, s_red);
    n0 = block_sum(n0, s_red);
    n1 = block_sum(n1, s_red);
    unsigned long long fs[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) fs[k] = block_sum((unsigned long long)ff[k], s_red);
    if (threadIdx.x == 0) {
        if (jn) atomicAdd(&acc.join, jn);
        if (n0) atomicAdd(&acc.ndv[0], n0);
        if (n1) atomicAdd(&acc.ndv[1], n1);
        if (fs[0]) atomicAdd(&acc.f1[0], fs[0]);
        if (fs[1]) atomicAdd(&acc.f1[1], fs[1]);
        if (fs[2]) atomicAdd(&acc.f2[0], fs[2]);
        if (fs[3]) atomicAdd(&acc.f2[1], fs[3]);
        __threadfence();
        if (atomicAdd(&acc.agg_done, 1u) == jd->n_agg - 1) {
            // last worker: the sentinel key, counted outside the tables
            __threadfence();
            const unsigned long long s0 = atomicAdd(&acc.sent[0], 0ull), s1 = atomicAdd(&acc.sent[1], 0ull);
            if (s0 && s1) atomicAdd(&acc.join, s0 * s1);
            if (s0) atomicAdd(&acc.ndv[0], 1ull);
            if (s1) atomicAdd(&acc.ndv[1], 1ull);
            if (s0 == 1) atomicAdd(&acc.f1[0], 1ull);
            if (s1 == 1) atomicAdd(&acc.f1[1], 1ull);
            if (s0 == 2) atomicAdd(&acc.f2[0], 1ull);
            if (s1 == 2) atomicAdd(&acc.f2[1], 1ull);
            const PlanHdr& H = *(const PlanHdr*)a.plan;
            if (H.early) {
                // every worker fenced its adds before counting itself done
                __threadfence();
                copy_to_host(a, (const unsigned long long*)&acc, sizeof(JoinAcc) / 8,
                             kHostAccsOff + (uint64_t)jd->acc * sizeof(JoinAcc), true);
                raise_flag(a, H, 1 + jd->acc, true);
            }
        }
    }
}

// ------------------------------------------------------------------ kernels
// Waits for a join phase counter, bounded: a wait that gives up marks the
// join failed (status 4, reported to the host as a device error) and returns
// false, so a lost signal ends the kernel instead of hanging it.  A join
// whose status is already set skips its remaining phases the same way.
__device__ __forceinline__ bool wait_count(const BatchArgs& a, uint32_t* p, uint32_t target, JoinAcc& acc,
                                           uint32_t* s_flag) {
    if (threadIdx.x == 0) {
        const bool ok = poll_count(p, target, a.spin_limit);
        if (!ok) atomicMax(&acc.status, 4ull);
        *s_flag = ok && __hip_atomic_load(&acc.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0 ? 1u : 0u;
    }
    __syncthreads();
    __threadfence();
    return *s_flag != 0;
}

__device__ __forceinline__ void signal_count(uint32_t* p) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(p, 1u);
    }
}

// pop the next item of one queue (items [first, last) of the plan's list)
__device__ __forceinline__ uint32_t pop_item(uint32_t* head, uint32_t first, uint32_t* s_item) {
    if (threadIdx.x == 0) *s_item = first + atomicAdd(head, 1u);
    __syncthreads();
    const uint32_t idx = *s_item;
    __syncthreads();
    return idx;
}

// selectivity scans (queue 0: items [0, n_scan_items))
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(3, 8))) gace_scan_kernel(BatchArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    __shared__ uint32_t s_item;
    const PlanHdr H = *(const PlanHdr*)a.plan;
    const bool spill = H.has_spill && H.spill_cap;
    bool worked = false;
    for (;;) {
        const uint32_t idx = pop_item(&a.head[0], 0, &s_item);
        if (idx >= H.n_scan_items) break;
        const uint64_t t0 = (uint64_t)wall_clock64();
        const Item it = batch_items(a, H)[idx];
        scan_item(a, H, it, lds);
        worked = true;
        __syncthreads();
        trace_item(a, H, idx, it, t0, t0);
        if (spill && threadIdx.x == 0) {
            // this item's spill claims and entries come before its count
            __threadfence();
            atomicAdd(&a.head[5], 1u);
        }
    }
    if (spill) {
        // Run spilled blocks: a ticket names an entry; it is run once it is
        // written, and the workgroup leaves when every item is done and the
        // ticket lies past the entries claimed.  The items never wait, so
        // the wait ends; it gives up, failing the scans, after kSpillPolls.
        __shared__ uint32_t s_ok;
        __shared__ uint32_t s_task[2];
        __shared__ unsigned long long s_block;
        Item* list = spill_list(a, H);
        for (;;) {
            if (threadIdx.x == 0) {
                const uint32_t t = atomicAdd(&a.head[4], 1u);
                uint32_t ok = 0;   // 1: run entry t, 0: no entry left, 2: gave up
                for (uint64_t polls = 0;; ++polls) {
                    if (t < H.spill_cap &&
                        __hip_atomic_load(&list[t].sub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 1u) {
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                        ok = 1;
                        break;
                    }
                    if (__hip_atomic_load(&a.head[5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= H.n_scan_items) {
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                        const uint32_t claimed = __hip_atomic_load(&a.head[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (t >= (claimed < H.spill_cap ? claimed : H.spill_cap)) break;
                    }
                    if (polls >= kSpillPolls) {
                        ok = 2;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                if (ok == 1) {
                    s_task[0] = list[t].idx;
                    s_task[1] = list[t].side;
                    s_block = list[t].begin;
                }
                if (ok == 2) atomicAdd(&a.hist[H.err_off], 1ull);
                s_ok = ok;
            }
            __syncthreads();
            if (s_ok != 1) break;
            scan_spill_task(a, H, s_task[0], s_block, s_task[1], lds);
            worked = true;
            __syncthreads();
        }
    }
    if (H.early && H.n_scan_items) {
        // the last workgroup to finish publishes every counter and histogram;
        // a workgroup that ran no item has no atomics to release
        if (worked) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0)
            s_item = atomicAdd(&a.hist[H.wg_done_off], 1ull) + 1 == gridDim.x ? 1u : 0u;
        __syncthreads();
        if (s_item) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            copy_to_host(a, a.counts, H.n_counts, 0, false);
            copy_to_host(a, a.hist, H.n_hist, kHostHistOff, false);
            raise_flag(a, H, 0, false);
        }
    }
}

// join phases (queue 1: items [n_scan_items, n_items), in phase order).
// KP staged keys per thread in the partitioning tiles: kPerBig when the join
// kernel has the GPU to itself; kPerSmall (160 instead of 240 VGPRs) when a
// scan kernel runs beside it, so a CU that holds a scan workgroup still fits
// two join waves per SIMD.
template <int KP>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(2, 8))) gace_join_kernel(BatchArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    __shared__ uint32_t s_item, s_flag;
    const PlanHdr H = *(const PlanHdr*)a.plan;
    for (;;) {
        const uint32_t idx = pop_item(&a.head[1], H.n_scan_items, &s_item);
        if (idx >= H.n_join_end) break;
        const uint64_t t0 = (uint64_t)wall_clock64();
        uint64_t t1 = t0, work = 0;
        const Item it = batch_items(a, H)[idx];
        const JoinDesc* jd = (const JoinDesc*)(a.plan + H.joins_off) + it.idx;
        JoinAcc& acc = a.accs[jd->acc];
        switch (it.kind) {
            case IT_JHEAVY:
                jheavy_item<KP>(a, jd, lds);
                signal_count(&acc.heavy_done);
                break;
            case IT_JHIST:
                if (wait_count(a, &acc.heavy_done, 1, acc, &s_flag)) {
                    t1 = (uint64_t)wall_clock64();
                    jhist_item<KP>(a, jd, it, lds);
                }
                signal_count(&acc.hist_done);
                break;
            case IT_JOFF:
                if (wait_count(a, &acc.hist_done, jd->n_items, acc, &s_flag)) {
                    t1 = (uint64_t)wall_clock64();
                    joff_item(a, jd, it, lds);
                }
                signal_count(&acc.off_done);
                break;
            case IT_JBASE:
                if (wait_count(a, &acc.off_done, jd->n_off, acc, &s_flag)) {
                    t1 = (uint64_t)wall_clock64();
                    jbase_item(a, jd, lds);
                }
                signal_count(&acc.base_done);
                break;
            case IT_JSCATTER:
                if (wait_count(a, &acc.base_done, 1, acc, &s_flag)) {
                    t1 = (uint64_t)wall_clock64();
                    jscatter_item<KP>(a, jd, it, lds);
                }
                signal_count(&acc.scatter_done);
                break;
            case IT_JSCATTER2:
                if (wait_count(a, &acc.scatter_done, jd->n_items, acc, &s_flag)) {
                    t1 = (uint64_t)wall_clock64();
                    jscatter2_item<KP>(a, jd, lds);
                }
                signal_count(&acc.s2_done);
                break;
            default:
                break;
        }
        __syncthreads();
        trace_item(a, H, idx, it, t0, t1, work);
    }
}

// join aggregation (queue 2: items [n_join_end, n_items)); launched after
// the partitioning kernel on the same stream, so every partition is final
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(4, 8))) gace_agg_kernel(BatchArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    __shared__ uint32_t s_item;
    const PlanHdr H = *(const PlanHdr*)a.plan;
    for (;;) {
        const uint32_t idx = pop_item(&a.head[2], H.n_join_end, &s_item);
        if (idx >= H.n_items) break;
        const uint64_t t0 = (uint64_t)wall_clock64();
        uint64_t work = 0;
        const Item it = batch_items(a, H)[idx];
        const JoinDesc* jd = (const JoinDesc*)(a.plan + H.joins_off) + it.idx;
        jagg_item(a, jd, it, lds, work);
        __syncthreads();
        trace_item(a, H, idx, it, t0, t0, work);
    }
}

// zero the per-batch accumulators (a kernel, not a memset, so it can be
// captured in a graph and replayed)
__global__ void __launch_bounds__(kWG) gace_init_kernel(uint8_t* plan, const uint8_t* src, uint64_t src_bytes,
                                                        Item* items, uint32_t* head, unsigned long long* counts,
                                                        unsigned long long* hist, JoinAcc* accs, Arena* arena) {
    const PlanHdr H = *(const PlanHdr*)(src_bytes ? src : plan);
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // a small plan comes from the pinned staging buffer (16-byte words)
    for (uint64_t i = tid; i < src_bytes / 16; i += stride) ((uint4*)plan)[i] = ((const uint4*)src)[i];
    if (tid < (src_bytes & 15)) plan[src_bytes / 16 * 16 + tid] = src[src_bytes / 16 * 16 + tid];
    for (uint64_t i = tid; i < H.n_counts; i += stride) counts[i] = 0;
    for (uint64_t i = tid; i < H.n_hist; i += stride) hist[i] = 0;
    const uint64_t nacc = (uint64_t)H.n_joins * (sizeof(JoinAcc) / 8);
    for (uint64_t i = tid; i < nacc; i += stride) ((unsigned long long*)accs)[i] = 0;
    // spill-list entries start unwritten (their ready words cleared)
    Item* spill = items + (H.items_off ? 0u : H.n_items);
    for (uint64_t i = tid; i < H.spill_cap; i += stride) spill[i].sub = 0;
    if (tid == 0) {
        for (int q = 0; q < kHeads; ++q) head[q] = 0;
        arena->used = H.arena_static;
    }
}

// After a batch: its counters, histograms and join accumulators copied into
// the pinned host result buffer (one small kernel instead of three copies;
// the launch boundary orders it after the batch's kernels)
__global__ void __launch_bounds__(kWG) gace_publish_kernel(const uint8_t* plan, const unsigned long long* counts,
                                                           const unsigned long long* hist, const JoinAcc* accs,
                                                           uint8_t* host_res) {
    const PlanHdr H = *(const PlanHdr*)plan;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long* hc = (unsigned long long*)host_res;
    unsigned long long* hh = (unsigned long long*)(host_res + kHostHistOff);
    unsigned long long* ha = (unsigned long long*)(host_res + kHostAccsOff);
    for (uint64_t i = tid; i < H.n_counts; i += stride) hc[i] = counts[i];
    for (uint64_t i = tid; i < H.n_hist; i += stride) hh[i] = hist[i];
    const uint64_t na = (uint64_t)H.n_joins * (sizeof(JoinAcc) / 8);
    for (uint64_t i = tid; i < na; i += stride) ha[i] = ((const unsigned long long*)accs)[i];
}

// Kept-block bit mask for a host-resident table: bit (b mod 32) of word b / 32
// is set iff block b is kept (the same decision as decide_blocks).  One
// thread per 32-bit word, so every word is written whole with one store.
__global__ void __launch_bounds__(kWG) gace_sample_mask_kernel(uint64_t n_blocks, uint64_t seed, uint32_t table_id,
                                                               uint64_t thr, uint32_t* mask) {
    const uint64_t w = (uint64_t)blockIdx.x * kWG + threadIdx.x;
    if (w >= (n_blocks + 31) / 32) return;
    uint32_t bits = 0;
    for (uint32_t j = 0; j < 32; ++j) {
        const uint64_t b = w * 32 + j;
        if (b < n_blocks && (uint64_t)block_word0(b, table_id, seed) < thr) bits |= 1u << j;
    }
    mask[w] = bits;
}

// ------------------------------------------------------------------ zone maps
// Per column and zone of kZoneRows rows: the smallest and largest value (for
// float32: of the non-NaN values; an all-NaN zone gets min = +inf, max = -inf,
// which no condition overlaps).  One workgroup per zone; each lane reads
// 16-byte quads, coalesced across the wave, folding into min / max started at
// the type's extremes, then wave shuffles and one LDS step reduce them.
template <typename T> struct ZoneLim;
template <> struct ZoneLim<int32_t> {
    static __device__ int32_t lo() { return 0x7FFFFFFF; }
    static __device__ int32_t hi() { return (int32_t)0x80000000; }
};
template <> struct ZoneLim<int64_t> {
    static __device__ int64_t lo() { return 0x7FFFFFFFFFFFFFFFll; }
    static __device__ int64_t hi() { return (int64_t)0x8000000000000000ull; }
};
template <> struct ZoneLim<float> {
    static __device__ float lo() { return __builtin_huge_valf(); }
    static __device__ float hi() { return -__builtin_huge_valf(); }
};

template <typename T>
__device__ __forceinline__ void zone_fold(T x, T& lo, T& hi) {
    if constexpr (std::is_same<T, float>::value) {
        if (x != x) return;   // NaN satisfies no condition
    }
    lo = x < lo ? x : lo;
    hi = x > hi ? x : hi;
}

template <typename T>
__device__ void zone_minmax(const T* col, uint64_t n_rows, T* zmin, T* zmax, uint8_t* lds) {
    constexpr uint32_t kPerQuad = 16 / sizeof(T);
    constexpr uint32_t kQuadsPerZone = (uint32_t)(kZoneRows / kPerQuad);
    const uint64_t z = blockIdx.x;
    const uint64_t r0 = z * kZoneRows;
    T lo = ZoneLim<T>::lo(), hi = ZoneLim<T>::hi();
    for (uint32_t q = threadIdx.x; q < kQuadsPerZone; q += kWG) {
        const uint64_t r = r0 + (uint64_t)q * kPerQuad;
        if (r + kPerQuad <= n_rows) {
            const u32x4 v = __builtin_nontemporal_load((const GACE_GLOBAL u32x4*)(col + r));
            T e[kPerQuad];
            __builtin_memcpy(e, &v, 16);
#pragma unroll
            for (uint32_t i = 0; i < kPerQuad; ++i) zone_fold(e[i], lo, hi);
        } else {
            for (uint64_t i = r; i < n_rows; ++i) zone_fold(col[i], lo, hi);
        }
    }
    for (int o = 32; o; o >>= 1) {
        const T l2 = __shfl_xor(lo, o), h2 = __shfl_xor(hi, o);
        lo = l2 < lo ? l2 : lo;
        hi = h2 > hi ? h2 : hi;
    }
    T* s_lo = (T*)lds;
    T* s_hi = s_lo + kWaves;
    if ((threadIdx.x & 63) == 0) {
        s_lo[threadIdx.x >> 6] = lo;
        s_hi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kWaves; ++w) {
            lo = s_lo[w] < lo ? s_lo[w] : lo;
            hi = s_hi[w] > hi ? s_hi[w] : hi;
        }
        zmin[z] = lo;
        zmax[z] = hi;
    }
}

// HBM read ceiling: workgroup w reads the 16-byte words [w, w + 1) x kWG x
// kReadUnroll of the buffer (clipped at n16), each thread kReadUnroll words
// kWG apart with nontemporal loads, all in flight at once, folded with XOR.
// A thread stores only when its fold is all ones, which never happens on the
// zero-filled buffers it is measured on: the kernel reads and does not write.
constexpr uint32_t kReadUnroll = 16;
__global__ void __launch_bounds__(kWG) gace_read_kernel(const u32x4* p, uint64_t n16, uint32_t* sink) {
    const uint64_t base = (uint64_t)blockIdx.x * kWG * kReadUnroll + threadIdx.x;
    const GACE_GLOBAL u32x4* q = (const GACE_GLOBAL u32x4*)p;
    u32x4 acc = {0u, 0u, 0u, 0u};
    if (base + (uint64_t)(kReadUnroll - 1) * kWG < n16) {
        u32x4 v[kReadUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kReadUnroll; ++u) v[u] = __builtin_nontemporal_load(q + base + u * kWG);
#pragma unroll
        for (uint32_t u = 0; u < kReadUnroll; ++u) acc ^= v[u];
    } else {
        for (uint32_t u = 0; u < kReadUnroll; ++u)
            if (base + u * kWG < n16) acc ^= __builtin_nontemporal_load(q + base + u * kWG);
    }
    const uint32_t f = acc[0] ^ acc[1] ^ acc[2] ^ acc[3];
    if (f == 0xffffffffu) sink[0] = f;
}

__global__ void __launch_bounds__(kWG) gace_zone_build_kernel(const void* col, uint32_t dtype, uint64_t n_rows,
                                                              void* zmin, void* zmax) {
    __shared__ __align__(16) uint8_t lds[2 * kWaves * 8];
    if (dtype == 2u)
        zone_minmax<int64_t>((const int64_t*)col, n_rows, (int64_t*)zmin, (int64_t*)zmax, lds);
    else if (dtype == 3u)
        zone_minmax<float>((const float*)col, n_rows, (float*)zmin, (float*)zmax, lds);
    else
        zone_minmax<int32_t>((const int32_t*)col, n_rows, (int32_t*)zmin, (int32_t*)zmax, lds);
}

// one column's zone arrays, as the prune kernel reads them
struct ZoneCol {
    const void* zmin;
    const void* zmax;
    uint32_t dtype;
    uint32_t reserved;
};

// a term of the request (the ABI's gace_term layout)
struct ZTerm {
    uint32_t col, op, n_vals, reserved;
    int64_t v[8];
};

// can some value in [lo, hi] satisfy the term?  Integers compare in int64,
// floats as IEEE binary32 (an empty float zone has lo > hi and fails every test)
__device__ __forceinline__ bool zterm_may(const ZTerm& t, const ZoneCol& c, uint64_t z) {
    if (c.dtype == 3u) {
        const float lo = ((const float*)c.zmin)[z], hi = ((const float*)c.zmax)[z];
        auto fv = [&](int k) { return __uint_as_float((uint32_t)(uint64_t)t.v[k]); };
        if (t.op == 1u) return hi >= fv(0) && lo < fv(1) && lo <= hi;
        for (uint32_t k = 0; k < t.n_vals; ++k)
            if (lo <= fv(k) && fv(k) <= hi) return true;
        return false;
    }
    int64_t lo, hi;
    if (c.dtype == 2u) {
        lo = ((const int64_t*)c.zmin)[z];
        hi = ((const int64_t*)c.zmax)[z];
    } else {
        lo = ((const int32_t*)c.zmin)[z];
        hi = ((const int32_t*)c.zmax)[z];
    }
    if (t.op == 1u) return hi >= t.v[0] && lo < t.v[1];
    for (uint32_t k = 0; k < t.n_vals; ++k)
        if (lo <= t.v[k] && t.v[k] <= hi) return true;
    return false;
}

// bit z of skip: no predicate can hold on zone z.  One thread per zone; each
// wave's 64 bits are written as two whole 32-bit words.  The number of set
// bits is added to *n_skip (zeroed by the caller), one atomic per workgroup.
__global__ void __launch_bounds__(kWG) gace_zone_prune_kernel(const ZoneCol* zc, const ZTerm* terms,
                                                              const uint32_t* pred_off, uint32_t n_preds,
                                                              uint64_t n_zones, uint32_t* skip,
                                                              unsigned long long* n_skip) {
    __shared__ uint32_t s_n;
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    const uint64_t z = (uint64_t)blockIdx.x * kWG + threadIdx.x;
    bool may = false;
    if (z < n_zones) {
        for (uint32_t p = 0; p < n_preds && !may; ++p) {
            bool all = true;
            for (uint32_t i = pred_off[p]; i < pred_off[p + 1] && all; ++i) all = zterm_may(terms[i], zc[terms[i].col], z);
            may = all;
        }
    }
    const unsigned long long sk = __ballot(z < n_zones && !may);
    const uint64_t w0 = (z >> 6) * 2;                    // first 32-bit word of this wave
    if ((threadIdx.x & 63) == 0 && w0 * 32 < n_zones) {
        skip[w0] = (uint32_t)sk;
        if ((w0 + 1) * 32 < n_zones) skip[w0 + 1] = (uint32_t)(sk >> 32);
        if (sk) atomicAdd(&s_n, (uint32_t)__popcll(sk));
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_n) atomicAdd(n_skip, (unsigned long long)s_n);
}

}  // namespace gace

extern "C" {

hipError_t gace_launch_zone_build(const void* col, uint32_t dtype, uint64_t n_rows, void* zmin, void* zmax,
                                  hipStream_t stream) {
    const uint64_t zones = (n_rows + gace::kZoneRows - 1) / gace::kZoneRows;
    if (zones == 0) return hipSuccess;
    (void)hipGetLastError();   // report this launch's error, not an earlier call's
    hipLaunchKernelGGL(gace::gace_zone_build_kernel, dim3((uint32_t)zones), dim3(gace::kWG), 0, stream, col, dtype,
                       n_rows, zmin, zmax);
    return hipGetLastError();
}

hipError_t gace_launch_zone_prune(const void* zc, const void* terms, const uint32_t* pred_off, uint32_t n_preds,
                                  uint64_t n_zones, uint32_t* skip, void* n_skip, hipStream_t stream) {
    const uint64_t grid = (n_zones + gace::kWG - 1) / gace::kWG;
    if (grid == 0) return hipSuccess;
    (void)hipGetLastError();   // report this launch's error, not an earlier call's
    hipLaunchKernelGGL(gace::gace_zone_prune_kernel, dim3((uint32_t)grid), dim3(gace::kWG), 0, stream,
                       (const gace::ZoneCol*)zc, (const gace::ZTerm*)terms, pred_off, n_preds, n_zones, skip,
                       (unsigned long long*)n_skip);
    return hipGetLastError();
}

hipError_t gace_launch_sample_mask(uint64_t n_blocks, uint64_t seed, uint32_t table_id, uint64_t thr, void* mask,
                                   hipStream_t stream) {
    const uint64_t words = (n_blocks + 31) / 32;
    const uint64_t grid = (words + gace::kWG - 1) / gace::kWG;
    if (grid == 0) return hipSuccess;
    (void)hipGetLastError();   // report this launch's error, not an earlier call's
    hipLaunchKernelGGL(gace::gace_sample_mask_kernel, dim3((uint32_t)grid), dim3(gace::kWG), 0, stream, n_blocks,
                       seed, table_id, thr, (uint32_t*)mask);
    return hipGetLastError();
}

hipError_t gace_launch_read(const void* p, uint64_t n16, void* sink, hipStream_t stream) {
    const uint64_t per = (uint64_t)gace::kWG * gace::kReadUnroll;
    const uint64_t grid = (n16 + per - 1) / per;
    if (grid == 0) return hipSuccess;
    (void)hipGetLastError();   // report this launch's error, not an earlier call's
    hipLaunchKernelGGL(gace::gace_read_kernel, dim3((uint32_t)grid), dim3(gace::kWG), 0, stream,
                       (const gace::u32x4*)p, n16, (uint32_t*)sink);
    return hipGetLastError();
}

// host-side handles of the batch kernels, as the kernel nodes of a captured
// graph name them: 0 scan, 1 join (large tiles), 2 join (small tiles), 3
// aggregation
const void* gace_kernel_handle(int which) {
    switch (which) {
        case 0: return reinterpret_cast<const void*>(&gace::gace_scan_kernel);
        case 1: return reinterpret_cast<const void*>(&gace::gace_join_kernel<gace::kPerBig>);
        case 2: return reinterpret_cast<const void*>(&gace::gace_join_kernel<gace::kPerSmall>);
        case 3: return reinterpret_cast<const void*>(&gace::gace_agg_kernel);
        default: return nullptr;
    }
}

// launchers used by the host runtime (internal; not part of the public ABI)
hipError_t gace_launch_init(const void* plan, const void* src, uint64_t src_bytes, void* items, void* head,
                            void* counts, void* hist, void* accs, void* arena, hipStream_t stream) {
    (void)hipGetLastError();   // report this launch's error, not an earlier call's
    hipLaunchKernelGGL(gace::gace_init_kernel, dim3(256), dim3(gace::kWG), 0, stream, (uint8_t*)plan,
                       (const uint8_t*)src, src_bytes, (gace::Item*)items, (uint32_t*)head, (unsigned long long*)counts, (unsigned long long*)hist,
                       (gace::JoinAcc*)accs, (gace::Arena*)arena);
    return hipGetLastError();
}

hipError_t gace_launch_publish(const void* plan, const void* counts, const void* hist, const void* accs,
                               void* host_res, uint32_t grid, hipStream_t stream) {
    (void)hipGetLastError();   // report this launch's error, not an earlier call's
    hipLaunchKernelGGL(gace::gace_publish_kernel, dim3(grid), dim3(gace::kWG), 0, stream, (const uint8_t*)plan,
                       (const unsigned long long*)counts, (const unsigned long long*)hist,
                       (const gace::JoinAcc*)accs, (uint8_t*)host_res);
    return hipGetLastError();
}

hipError_t gace_launch_scan(const void* args, uint32_t grid, hipStream_t stream) {
    const gace::BatchArgs& a = *(const gace::BatchArgs*)args;
    (void)hipGetLastError();   // report this launch's error, not an earlier call's
    hipLaunchKernelGGL(gace::gace_scan_kernel, dim3(grid), dim3(gace::kWG), gace::kLdsBytes, stream, a);
    return hipGetLastError();
}

hipError_t gace_launch_agg(const void* args, uint32_t grid, hipStream_t stream) {
    const gace::BatchArgs& a = *(const gace::BatchArgs*)args;
    const uint32_t lds = gace::kLdsMisc + a.agg_slots * 16 + 512;
    (void)hipGetLastError();   // report this launch's error, not an earlier call's
    hipLaunchKernelGGL(gace::gace_agg_kernel, dim3(grid), dim3(gace::kWG), lds, stream, a);
    return hipGetLastError();
}

hipError_t gace_launch_join(const void* args, uint32_t grid, int beside_scan, hipStream_t stream) {
    const gace::BatchArgs& a = *(const gace::BatchArgs*)args;
    (void)hipGetLastError();   // report this launch's error, not an earlier call's
    if (beside_scan)
        hipLaunchKernelGGL(gace::gace_join_kernel<gace::kPerSmall>, dim3(grid), dim3(gace::kWG),
                           gace::join_lds_bytes(gace::kPerSmall * gace::kWG), stream, a);
    else
        hipLaunchKernelGGL(gace::gace_join_kernel<gace::kPerBig>, dim3(grid), dim3(gace::kWG),
                           gace::join_lds_bytes(gace::kPerBig * gace::kWG), stream, a);
    return hipGetLastError();
}

}
