// Match-count scan and count priority queue (c-PQ) on gfx950.
//
// One workgroup owns one (query, object tile) pair.  The tile's counters --
// the Bitmap Counter of Section 3.3.1, b bits per object packed into 32-bit
// LDS words -- and the Gate (ZipperArray ZA, AuditThreshold AT) and Hash
// Table of that tile live in LDS.  The workgroup streams every posting run
// of the query's items inside the tile (Section 3.2: scan the lists of every
// keyword an item covers; Definition 2.1: each posting adds one), applying
// Algorithm 1 per posting with an LDS atomic add that returns the previous
// count.  At the end, Theorem 3.1 gives the tile's k-th count as AT - 1; the
// tile emits its exact top-k under (count desc, id asc): the objects of
// count >= AT found through the Hash Table, then the smallest ids of count
// AT - 1 read from the counters (the Hash Table need not hold every tied
// object).  A second kernel merges the per-tile lists of each query; the
// global top-k is inside the union of the tile top-k lists because the
// order is total.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace genie {
namespace {

struct ScanParams {
    const uint16_t *post;
    const uint64_t *tile_base;
    const uint2 *map_ck;    // Position Map: per tile, nkeys + 1 pairs {offset, pads}, or in
                            // the compact form map_groups checkpoints {offset, pads}
    const uint4 *map_len;   // ... and per group the 8 keywords' run lengths (uint16)
    uint32_t map_compact;   // 1: the compact form
    uint64_t n;
    uint64_t nkeys;         // keywords
    uint64_t map_groups;    // Position Map groups per tile
    uint32_t d, V, n_tiles;
    const uint64_t *q_off;
    const uint32_t *items;  // 3 words per item
    uint64_t n_items;       // items available at items
    uint32_t nq, k, max_items, ht_log2;
    uint64_t per_xcd;       // (query, tile) pairs handled per XCD slice
    uint64_t *cand;         // [nq][n_tiles][k] packed keys
    uint32_t *tile_kth;     // [nq][n_tiles]
    uint4 *pair_stats;      // [nq][n_tiles] statistics of each pair, or null (count dump:
                            // added to the status block directly)
    uint32_t *full_counts;  // [nq][n] (count dump mode) or null
    uint32_t *status;       // flags word; stats as uint64 at status + 2
    const float *gate;      // predicted k-th count per query (gated search) or null
    float gate_delta;       // safety margin subtracted from the prediction
    const uint32_t *qlist;  // query of each row (fallback pass) or null
    const uint32_t *qcount; // rows in qlist (device) or null
    uint32_t *work;         // persistent schedule: 8 per-XCD pair counters (zeroed), or null
    // Index parts searched one after another into one candidate array
    // (multiple loadings): ids of this part start at id_base, its tiles at
    // column tile_off of rows of tiles_total tiles.  A single index: 0, 0,
    // n_tiles.
    uint64_t id_base;
    uint32_t tile_off, tiles_total;
    uint32_t spq;           // 1: GEN-SPQ ablation (count everything, then select)
    uint32_t key_sets;      // 1: keyword-set index, every item names one keyword
    uint32_t rows_loop;     // 1: the pairs of the qcount rows only, by resident workgroups
};

// Schedules of the scan kernel: one workgroup per pair; persistent
// workgroups over per-XCD pair counters; resident workgroups looping over
// the pairs of the rows counted on the device (the gated search's fallback
// pass, which usually has none).
enum : int { kSchedGrid = 0, kSchedQueue = 1, kSchedRows = 2 };

struct MergeParams {
    const uint64_t *cand;
    const uint32_t *tile_kth;
    const uint4 *pair_stats;  // per-pair statistics, summed per query into the status block
    uint32_t *status;
    uint64_t n;
    uint32_t n_tiles, k;
    uint32_t *out_ids, *out_counts;
    uint32_t *fb_count;      // gated search: queries to answer again (device counter)
    uint32_t *fb_list;       // ... and their indices
    const uint32_t *qlist;   // fallback pass: query of each block
    const uint32_t *qcount;
};

// Answer order key: larger is better; count in the high word, then smaller
// id.  Key 0 is the padding entry (count 0, id UINT32_MAX).
__device__ __forceinline__ uint64_t make_key(uint32_t count, uint32_t gid) {
    return ((uint64_t)count << 32) | (uint64_t)(0xFFFFFFFFu - gid);
}

__device__ __forceinline__ uint32_t lds_load(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t lds_add(uint32_t *p, uint32_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t lds_or(uint32_t *p, uint32_t v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t lds_max(uint32_t *p, uint32_t v) {
    return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ bool lds_cas(uint32_t *p, uint32_t expect, uint32_t desired) {
    return __hip_atomic_compare_exchange_strong(p, &expect, desired, __ATOMIC_RELAXED,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The run holding stream position p0, for a cursor at run `si` that ends at
// or before p0 (p0 < sp_cum[s]): the ends of the next 64 runs, one per lane
// (lane 0 reads the cursor's own end); the first end past p0 closes the run
// holding p0.  Returns that run and its bounds {run, start, end}.  Kept out
// of line: it serves the long jumps of the run cursor over short runs.
// Wave-uniform call with every lane active.
typedef __attribute__((address_space(3))) const uint32_t lds_u32;   // an LDS word
__device__ __attribute__((noinline)) uint3 run_holding(lds_u32 *sp_cum, uint32_t si, uint32_t s,
                                                       uint32_t p0) {
    const uint32_t lane = threadIdx.x & 63;
    for (;;) {
        const uint32_t idx = si + 1 + lane;
        const uint32_t w = idx <= s ? sp_cum[idx] : 0xFFFFFFFFu;
        const uint64_t m = __ballot(w > p0);
        if (m) {
            const uint32_t j = (uint32_t)__builtin_ctzll(m);   // >= 1
            return make_uint3(si + j, __builtin_amdgcn_readlane(w, j - 1),
                              __builtin_amdgcn_readlane(w, j));
        }
        si += 63;   // run si + 63 ends at or before p0
    }
}

// misc words at the start of the LDS block
enum : int {
    M_AT = 0, M_NABOVE = 1, M_OVERFLOW = 2, M_INSERTS = 3, M_SCANNED = 4, M_PASSES = 5,
    M_PREFETCH = 6, M_TAIL = 7, M_WAVESUM = 8,
    // cleared for every pair: words below M_KEEP; the persistent schedule keeps
    // its state above: two run-table slot headers and its claim cursor
    M_KEEP = 24, M_SLOT = 24, M_XCD = 30, M_SPENT = 31
};
// Header of a prepared run table (persistent schedule): its pair, its item
// count with the flags of a query answered with padding, postings scanned.
enum : uint32_t { H_PAIR = 0, H_S = 1, H_SCANNED = 2, H_WORDS = 3 };
constexpr uint32_t kNoPair = 0xFFFFFFFFu;
constexpr uint32_t kTooManyFlag = 1u << 30, kBadOffsetsFlag = 1u << 31;

// Position Map entry of keyword `key` in tile t: {padded offset of its run
// in the tile, padded runs before it}: one 8-byte read.  In the compact form
// the map keeps one checkpoint per group of 8 keywords and the group's real
// run lengths (uint16); the entry is the checkpoint plus the padded lengths
// (and odd lengths) of the group's keywords before `key`: one 8-byte and
// one 16-byte read.
// `own` (compact form) receives the real run length of `key` itself.
__device__ __forceinline__ uint2 map_entry(const ScanParams &p, uint32_t t, uint64_t key,
                                           uint32_t *own = nullptr) {
    if (!p.map_compact)
        return p.map_ck[(uint64_t)t * (p.nkeys + 1) + key];
    const uint64_t g = (uint64_t)t * p.map_groups + (key >> 3);
    const uint2 c = p.map_ck[g];
    const uint4 L = p.map_len[g];
    const uint32_t r = (uint32_t)(key & 7);
    const uint32_t w[4] = {L.x, L.y, L.z, L.w};
    uint32_t off = c.x, pads = c.y, mine = 0;
#pragma unroll
    for (uint32_t j = 0; j < 8; j++) {
        const uint32_t len = (w[j >> 1] >> ((j & 1) * 16)) & 0xFFFFu, odd = len & 1u;
        if (j < r) {
            off += len + odd;
            pads += odd;
        }
        mine = j == r ? len : mine;
    }
    if (own)
        *own = mine;
    return make_uint2(off, pads);
}

// The run of item `it` (dim, lo, hi) in tile t: [b, e) in padded elements
// of the tile, with `pads` padding elements inside.  The keywords of one
// dim are adjacent in the tile (Section 3.2, Position Map restricted to the
// tile), so an item is the single run [off(dim*V+lo), off(dim*V+hi+1)).
__device__ __forceinline__ void item_run(const ScanParams &p, uint32_t t, const uint32_t *it,
                                         uint32_t &b, uint32_t &e, uint32_t &pads) {
    uint32_t dim = it[0], lo = it[1], hi = it[2];
    b = e = pads = 0;
    if (dim >= p.d) {
        if (t == 0)
            atomicOr(p.status, GENIE_STATUS_BAD_DIM);
    } else {
        hi = min(hi, p.V - 1);
        if (p.key_sets && lo < hi) {
            // an object holds a keyword at most once, so one keyword per
            // item keeps every count at most the number of items
            if (t == 0)
                atomicOr(p.status, GENIE_STATUS_RANGE_ON_SET);
        } else if (lo <= hi) {
            const uint64_t key = (uint64_t)dim * p.V;
            if (p.map_compact && lo == hi) {   // one keyword: its own length ends the run
                uint32_t len = 0;
                b = map_entry(p, t, key + lo, &len).x;
                e = b + len + (len & 1u);
                pads = len & 1u;
            } else {
                const uint2 x0 = map_entry(p, t, key + lo), x1 = map_entry(p, t, key + hi + 1);
                b = x0.x;
                e = x1.x;
                pads = x1.y - x0.y;
            }
        }
    }
}

__device__ __forceinline__ uint32_t ht_home(uint32_t lid, uint32_t lg) {
    return (lid * 2654435761u) >> (32 - lg);
}

// Hash Table insert with the modified Robin Hood scheme (Section 3.3.2).
// Entry = count << 16 | local id (0 = empty).  Robin Hood: a probing entry
// that is farther from its home slot than the resident takes the slot and
// carries the resident on.  Modification: an entry that can no longer be
// among the objects of count >= AT is overwritten (or dropped, when carried)
// regardless of hashing.  The paper expires entries below AT - 1; here the
// objects tied at AT - 1 are taken from the exact counters at selection
// time, so the table only has to keep entries of count >= AT and expires
// everything below AT.  The same object may end up in two slots when races
// interleave; selection removes duplicates.  Returns false when a full sweep
// finds no free slot (the tile then selects from the counters alone, which
// hold every exact count).
__device__ bool ht_insert(uint32_t *ht, uint32_t lg, uint32_t *misc, uint32_t lid, uint32_t val) {
    const uint32_t mask = (1u << lg) - 1;
    uint32_t entry = (val << 16) | lid;
    uint32_t pos = ht_home(lid, lg);
    uint32_t dist = 0;
    for (uint32_t step = 0; step < 2u * (mask + 1) + 16; step++) {
        const uint32_t at = lds_load(&misc[M_AT]);
        if ((entry >> 16) < at)
            return true;  // the carried entry has expired
        const uint32_t cur = lds_load(&ht[pos]);
        if (cur == 0 || (cur >> 16) < at) {
            if (lds_cas(&ht[pos], cur, entry))
                return true;
            continue;  // slot changed under us: look again
        }
        if ((cur & 0xFFFFu) == (entry & 0xFFFFu)) {
            if ((cur >> 16) >= (entry >> 16))
                return true;
            if (lds_cas(&ht[pos], cur, entry))
                return true;
            continue;
        }
        const uint32_t cdist = (pos - ht_home(cur & 0xFFFFu, lg)) & mask;
        if (cdist < dist) {
            if (!lds_cas(&ht[pos], cur, entry))
                continue;
            entry = cur;
            dist = cdist;
        }
        pos = (pos + 1) & mask;
        dist++;
    }
    return false;
}

// Algorithm 1 after the gate check, part 1: advance AT while ZA[AT] >= k
// (the caller has just added to ZA).  A stale AT only lets extra increments
// through the gate; AT never passes the k-th count because ZA[v] never
// exceeds the objects that reached v (each (object, value) pair is counted
// once: val comes from an atomic increment).  s is the query's item count
// (the largest possible count); ZA[s+1] stays 0, so AT stops at s + 1.
__device__ void advance_at(uint32_t *za, uint32_t *misc, uint32_t k, uint32_t s) {
    uint32_t a = lds_load(&misc[M_AT]);
    while (a <= s && lds_load(&za[a]) >= k) {
        lds_max(&misc[M_AT], a + 1);
        a = lds_load(&misc[M_AT]);
    }
}

// Algorithm 1, part 2: put (object, val) into the HT.  Callers run it some
// time after the increment (queued per wave); an increment that AT has left
// behind by then (val < AT) is not stored, which keeps the table small.
// Every object whose final count reaches the final AT is stored by its last
// increment, because AT never exceeds its final value.
__device__ void ht_put(uint32_t *ht, uint32_t lg, uint32_t *misc, uint32_t lid, uint32_t val) {
    if (val >= lds_load(&misc[M_AT]) && lds_load(&misc[M_OVERFLOW]) == 0) {
        lds_add(&misc[M_INSERTS], 1);
        if (!ht_insert(ht, lg, misc, lid, val))
            misc[M_OVERFLOW] = 1;
    }
}

// The BITS-bit fields of `word` equal to v among those whose ids (first,
// first + 1, ...) are below n, as the high bit of each such field.  Exact
// zero-field test: in x = word xor (v in every field), a field is non-zero
// iff its high bit is set or its low bits are; adding the low-bits mask to
// the low bits sets the high bit exactly when they are non-zero (no carry
// leaves a field).
template <int BITS>
__device__ __forceinline__ uint32_t fields_equal_mask(uint32_t word, uint32_t v, uint32_t n,
                                                      uint32_t first) {
    constexpr uint32_t CPW = 32 / BITS;
    constexpr uint32_t ONES = BITS == 4 ? 0x11111111u : (BITS == 8 ? 0x01010101u : 0x00010001u);
    constexpr uint32_t HI = ONES << (BITS - 1);
    const uint32_t x = word ^ (v * ONES);
    const uint32_t nonzero = (((x & ~HI) + ~HI) | x) & HI;
    uint32_t zero = ~nonzero & HI;
    if (first + CPW > n)   // fields at or past n are not objects of the tile
        zero &= n > first ? HI >> ((CPW - (n - first)) * BITS) : 0u;
    return zero;
}

// Number of those fields.
template <int BITS>
__device__ __forceinline__ uint32_t fields_equal(uint32_t word, uint32_t v, uint32_t n,
                                                 uint32_t first) {
    return __popc(fields_equal_mask<BITS>(word, v, n, first));
}

constexpr uint32_t ilog2(uint32_t x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }


// Inclusive prefix sum over the 64 lanes of a wave by DPP moves, which stay
// in the VALU (a shuffle is an LDS instruction and would queue behind the
// counting atomics of the workgroup sharing the CU): shifts by 1, 2, 4 and 8
// lanes inside each row of 16, then the last lane of a row added into the
// next row (row_bcast:15) and lane 31 into the upper half (row_bcast:31).
// Every lane in the wave must be active.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t x) {
    const uint32_t lane = threadIdx.x & 63, row_lane = lane & 15;
    int v = (int)x, t;
    t = __builtin_amdgcn_mov_dpp(v, 0x111, 0xF, 0xF, false);   // row_shr:1
    v += row_lane >= 1 ? t : 0;
    t = __builtin_amdgcn_mov_dpp(v, 0x112, 0xF, 0xF, false);   // row_shr:2
    v += row_lane >= 2 ? t : 0;
    t = __builtin_amdgcn_mov_dpp(v, 0x114, 0xF, 0xF, false);   // row_shr:4
    v += row_lane >= 4 ? t : 0;
    t = __builtin_amdgcn_mov_dpp(v, 0x118, 0xF, 0xF, false);   // row_shr:8
    v += row_lane >= 8 ? t : 0;
    t = __builtin_amdgcn_mov_dpp(v, 0x142, 0xF, 0xF, false);   // row_bcast:15
    v += (lane & 31) >= 16 ? t : 0;
    t = __builtin_amdgcn_mov_dpp(v, 0x143, 0xF, 0xF, false);   // row_bcast:31
    v += lane >= 32 ? t : 0;
    return (uint32_t)v;
}

// Exclusive prefix sum over the workgroup; returns the total in *total.
// TRAIL: end with a barrier, so that wave_sums may be written again at once
// (callers that reach another barrier before the next write leave it out).
template <int NT, bool TRAIL = true>
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *wave_sums, uint32_t *total) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t incl = wave_inclusive_sum(v);
    if (lane == 63)
        wave_sums[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; w++) {
        uint32_t ws = wave_sums[w];
        before += (w < (int)wave) ? ws : 0;
        all += ws;
    }
    if (TRAIL)
        __syncthreads();
    *total = all;
    return before + incl - v;
}

// Persistent schedule: the next pair of this workgroup, from the per-XCD
// pair counters (one device-scope atomic per pair): the workgroup's own
// XCD slice first, then the others in turn.  Called by one lane; the cursor
// lives in LDS (misc M_XCD, M_SPENT).
__device__ uint32_t claim_pair(const ScanParams &p, uint32_t *misc) {
    const uint64_t npairs = (uint64_t)p.nq * p.n_tiles;
    uint32_t x = misc[M_XCD], spent = misc[M_SPENT], pair = kNoPair;
    while (spent < 8) {
        const uint32_t idx = atomicAdd(&p.work[x], 1u);
        const uint64_t first = (uint64_t)x * p.per_xcd;
        const uint64_t slice = first >= npairs ? 0 : min<uint64_t>(p.per_xcd, npairs - first);
        if (idx < slice) {
            pair = (uint32_t)(first + idx);
            if (p.qcount && pair % p.nq >= *p.qcount) {
                pair = kNoPair;   // a row past the live count: take the next pair
                continue;
            }
            break;
        }
        x = (x + 1) & 7;
        spent++;
    }
    misc[M_XCD] = x;
    misc[M_SPENT] = spent;
    return pair;
}

// One wave claims the workgroup's next pair and builds its run table into a
// slot (run starts sp_dw, prefix dword counts sp_cum, header hdr), 64 items
// per round with a wave prefix sum.  Every lane of the wave must be active.
__device__ void prepare_pair(const ScanParams &p, uint32_t *misc, uint32_t *sp_dw,
                             uint32_t *sp_cum, uint32_t *hdr) {
    const uint32_t lane = threadIdx.x & 63;
    uint32_t pair = 0;
    if (lane == 0)
        pair = claim_pair(p, misc);
    pair = __builtin_amdgcn_readfirstlane(pair);
    if (pair == kNoPair) {
        if (lane == 0)
            hdr[H_PAIR] = kNoPair;
        return;
    }
    const uint32_t t = pair / p.nq, q = pair % p.nq;
    const uint64_t i0 = p.q_off[q], i1 = p.q_off[q + 1];
    const bool bad_offsets = i1 < i0 || i1 > p.n_items;
    const uint64_t s64 = bad_offsets ? 0 : i1 - i0;
    const bool too_many = bad_offsets || s64 > p.max_items;
    const uint32_t s = too_many ? 0 : (uint32_t)s64;
    uint32_t carry = 0, scanned = 0;
    for (uint32_t c = 0; c < s; c += 64) {
        const uint32_t i = c + lane;
        uint32_t b = 0, e = 0, pads = 0;
        if (i < s)
            item_run(p, t, p.items + 3 * (i0 + i), b, e, pads);
        const uint32_t dw = (e - b) >> 1;
        const uint32_t incl = wave_inclusive_sum(dw);
        if (i < s) {
            sp_dw[i] = b >> 1;
            sp_cum[i] = carry + incl - dw;
        }
        carry += __builtin_amdgcn_readlane(incl, 63);
        scanned += (e - b) - pads;
    }
    scanned = __builtin_amdgcn_readlane(wave_inclusive_sum(scanned), 63);
    if (lane == 0) {
        sp_cum[s] = carry;
        hdr[H_PAIR] = pair;
        hdr[H_S] = s | (too_many ? kTooManyFlag : 0u) | (bad_offsets ? kBadOffsetsFlag : 0u);
        hdr[H_SCANNED] = scanned;
    }
}

// Occupancy: when the counters take at most 64 KB of LDS (2^LG counters of
// BITS bits), the workgroup's LDS (counters plus the gate, queues and
// table) lets two 1024-thread workgroups share a CU, i.e. 8 waves per SIMD,
// if the kernel fits 64 VGPRs; the scan is bound by the latency of its loads
// and LDS atomics, so that occupancy is asked for explicitly.  Likewise four
// 512-thread workgroups with at most 32 KB of counters (8-bit counters over
// 2^15 ids).  128 KB of counters (16-bit counters over 2^16 ids) allow one
// workgroup per CU.
template <int BITS, int NT, int LG>
constexpr int scan_waves_per_eu() {
    return ((NT == 1024 && (BITS << LG) <= (8 << 16)) || (NT == 512 && (BITS << LG) <= (8 << 15)))
               ? 8 : 1;
}

// One (query, tile) pair: the whole of Algorithm 1 over the tile's part of
// the query's lists, then the tile's exact top-k.  `bc` is the workgroup's
// static counter array; `smem` the dynamic LDS block.  PF (persistent
// schedule): the pair's run table was prepared in run-table slot `slot`
// while the workgroup's previous pair was counted, and the first wave to
// finish counting this pair prepares the next one in the other slot.
template <int BITS, int NT, int U, bool DUMP, int LG, bool SPQ = false, bool PF = false>
__device__ __forceinline__ void scan_pair(const ScanParams &p, uint64_t pair, uint32_t *bc,
                                          uint32_t *smem, uint32_t slot = 0) {
    static_assert(BITS == 4 || BITS == 8 || BITS == 16, "power-of-two counter width");
    constexpr uint32_t CPW = 32 / BITS;                   // counters per word
    constexpr uint32_t LBITS = BITS == 4 ? 2 : (BITS == 8 ? 3 : 4);  // log2(BITS)
    constexpr uint32_t MASK = (1u << BITS) - 1;           // also the "emitted" mark
    constexpr uint32_t TILE = (1u << LG) - 1;             // objects per tile
    constexpr uint32_t SENT = TILE;                       // the padding id
    constexpr uint32_t NW = (1u << LG) / CPW;             // a counter for every LG-bit id
    constexpr uint32_t NWAVE = NT / 64;
    constexpr uint32_t CH = 64 * U;                       // dwords per wave per step

    uint32_t *misc = smem;
    const uint32_t lg = p.ht_log2, cap = 1u << lg;
    uint32_t *ht = smem + 32;
    uint32_t *za = ht + cap;
    // run table: first dword of each item's run (tile-relative) and the
    // prefix counts of the runs' dwords (two slots in the persistent schedule)
    const uint32_t table_words = 2 * p.max_items + 1;
    uint32_t *tables = za + (p.max_items + 2);
    uint32_t *sp_dw = tables + (PF ? slot * table_words : 0u);
    uint32_t *sp_cum = sp_dw + p.max_items;               // max_items + 1 entries
    // per-wave queue of (count << 16 | local id) pairs that passed the gate
    uint32_t *gq = tables + (PF ? 2u : 1u) * table_words + ((threadIdx.x >> 6) * kGateQueue);
    // the next pair's table (persistent schedule), prepared by one wave
    auto prepare_next = [&]() {
        const uint32_t nslot = slot ^ 1u;
        uint32_t *ndw = tables + nslot * table_words;
        prepare_pair(p, misc, ndw, ndw + p.max_items, misc + M_SLOT + nslot * H_WORDS);
    };

    const uint32_t t = (uint32_t)(pair / p.nq);
    const uint32_t qrow = (uint32_t)(pair % p.nq);
    if (p.qcount && qrow >= *p.qcount)
        return;
    const uint32_t q = p.qlist ? p.qlist[qrow] : qrow;
    const uint32_t tid = threadIdx.x;

    const uint64_t tile0 = (uint64_t)t * TILE;
    const uint32_t tile_n = (uint32_t)min<uint64_t>(TILE, p.n - tile0);
    bool bad_offsets, too_many;
    uint32_t s;
    uint64_t i0 = 0;
    if constexpr (PF) {   // from the prepared slot's header
        const uint32_t hs = misc[M_SLOT + slot * H_WORDS + H_S];
        bad_offsets = (hs & kBadOffsetsFlag) != 0;
        too_many = (hs & kTooManyFlag) != 0;
        s = hs & 0xFFFFu;
    } else {
        i0 = p.q_off[q];
        const uint64_t i1 = p.q_off[q + 1];
        bad_offsets = i1 < i0 || i1 > p.n_items;
        const uint64_t s64 = bad_offsets ? 0 : i1 - i0;
        too_many = bad_offsets || s64 > p.max_items;
        s = too_many ? 0 : (uint32_t)s64;
    }

    for (uint32_t i = tid; i < NW; i += NT)
        bc[i] = 0;
    for (uint32_t i = tid; i < cap; i += NT)
        ht[i] = 0;
    for (uint32_t i = tid; i < p.max_items + 2; i += NT)
        za[i] = 0;
    // AuditThreshold starts at 1 (Algorithm 1), or, in the gated search, at
    // the predicted k-th count minus a margin (never above s + 1)
    uint32_t at0 = 1;
    if (p.gate) {
        const float g = fminf(p.gate[q] - p.gate_delta, (float)(s + 1));
        at0 = g >= 2.0f ? (uint32_t)floorf(g) : 1u;   // NaN and low values give 1
    }
    // misc words from M_KEEP up hold the persistent schedule's state
    if (tid < M_KEEP)
        misc[tid] = (tid == M_AT) ? at0 : (PF && tid == M_SCANNED)
                                              ? misc[M_SLOT + slot * H_WORDS + H_SCANNED] : 0u;
    // Position Map lookup (Section 3.2), restricted to this tile, item by
    // item (item_run).  The lookup writes only the run table (the counters
    // are cleared meanwhile); a thread's share of the scanned postings
    // reaches misc after a barrier.  A prepared pair has its table already.
    auto lookup = [&](uint32_t i, uint32_t &b, uint32_t &e, uint32_t &pads) {
        item_run(p, t, p.items + 3 * (i0 + i), b, e, pads);
    };
    if (PF) {
        __syncthreads();
    } else if (s <= 64) {
        // one item per lane of wave 0 and a wave prefix sum of the runs'
        // dwords: the run table needs no barrier of its own
        if (tid < 64) {
            uint32_t b = 0, e = 0, pads = 0;
            if (tid < s)
                lookup(tid, b, e, pads);
            const uint32_t dw = (e - b) >> 1;
            const uint32_t incl = wave_inclusive_sum(dw);
            if (tid < s) {
                sp_dw[tid] = b >> 1;
                sp_cum[tid] = incl - dw;
            }
            if (tid == 63)
                sp_cum[s] = incl;
            if (e - b - pads)   // misc was cleared by this wave above
                lds_add(&misc[M_SCANNED], (e - b) - pads);
        }
        __syncthreads();
    } else {
        uint32_t my_scanned = 0;
        for (uint32_t i = tid; i < s; i += NT) {
            uint32_t b, e, pads;
            lookup(i, b, e, pads);
            sp_dw[i] = b >> 1;
            sp_cum[i] = (e - b) >> 1;   // dwords of the run (temporary)
            my_scanned += (e - b) - pads;
        }
        __syncthreads();
        if (my_scanned)
            lds_add(&misc[M_SCANNED], my_scanned);
        // prefix counts of the runs' dwords (at most 1024 runs, 2 per thread)
        const uint32_t a0 = 2 * tid, a1 = 2 * tid + 1;
        const uint32_t c0 = a0 < s ? sp_cum[a0] : 0u, c1 = a1 < s ? sp_cum[a1] : 0u;
        uint32_t total = 0;
        // the wave totals are next written after the barrier below
        const uint32_t ex = block_exclusive_scan<NT, false>(c0 + c1, misc + M_WAVESUM, &total);
        if (a0 < s)
            sp_cum[a0] = ex;
        if (a1 < s)
            sp_cum[a1] = ex + c0;
        if (tid == 0)
            sp_cum[s] = total;
        __syncthreads();
    }

    const uint64_t row = (uint64_t)q * p.tiles_total + p.tile_off + t;
    const uint64_t gid0 = p.id_base + tile0;   // global id of the tile's first object
    if (too_many) {
        // counts could overflow the packed width: answer with padding only
        if (tid == 0)
            atomicOr(p.status, bad_offsets ? GENIE_STATUS_BAD_OFFSETS : GENIE_STATUS_TOO_MANY_ITEMS);
        if (DUMP) {
            for (uint32_t i = tid; i < tile_n; i += NT)
                p.full_counts[(uint64_t)q * p.n + tile0 + i] = 0;
        } else {
            for (uint32_t i = tid; i < p.k; i += NT)
                p.cand[row * p.k + i] = 0;
            if (tid == 0) {
                p.tile_kth[row] = 0;
                p.pair_stats[row] = make_uint4(0u, 0u, 0u, 0u);
            }
        }
        if (PF && tid < 64)
            prepare_next();
        return;
    }

    // ---- scan: every posting of every run adds one to its object's count.
    // The runs' dwords form one stream cut into 64-dword pieces; a wave's
    // step takes U consecutive pieces (a chunk of CH dwords), and lane l
    // takes dword l of each piece (two postings); the build orders each run
    // so that the ids the lanes of one step touch sit in different LDS
    // banks.  The run cursor is the same in every lane: a piece inside one
    // run is addressed as cursor + lane.  Runs are padded with the
    // reserved padding id 2^LG - 1, whose counter is a dummy (the top field of the
    // last word, where carries fall off), so every element is counted
    // without a bounds test; lanes past the end read the tile's trailing
    // all-sentinel dwords.
    const char *tile_bytes = reinterpret_cast<const char *>(p.post) + 2 * p.tile_base[t];
    // the tile's trailing sentinel dwords start where the last keyword's run ends
    const uint32_t sent_dw = map_entry(p, t, p.nkeys).x >> 1;
    const uint32_t k = p.k;
    // wave-uniform values, so that the run cursor lives in scalar registers
    const uint32_t total_dw = __builtin_amdgcn_readfirstlane(sp_cum[s]);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    uint32_t qn = 0;       // pairs in this wave's gate queue (same in every lane)
    uint32_t passes = 0;   // increments this wave let through the gate
    uint32_t si = 0, c_lo = 0;
    uint32_t c_hi = s ? __builtin_amdgcn_readfirstlane(sp_cum[1]) : 0u;
    uint32_t dwb = s ? __builtin_amdgcn_readfirstlane(sp_dw[0]) : 0u;
    // A wave's next chunk lies NWAVE chunks ahead (or further, for a chunk
    // claimed at the tail); when the runs average fewer than 256 dwords that
    // is past 16 runs or more on average, and the cursor finds its run from
    // the ends of the next 64 runs at once (run_holding) instead of run by
    // run.
    const bool short_runs = total_dw < 256u * s;
    // move the cursor to the run holding stream position p0 < total_dw
    auto seek = [&](uint32_t p0) {
        if (p0 >= c_hi) {
            si++;
            c_lo = c_hi;
            c_hi = __builtin_amdgcn_readfirstlane(sp_cum[si + 1]);
            if (p0 >= c_hi) {
                if (short_runs) {
                    const uint3 r = run_holding((lds_u32 *)sp_cum, si, s, p0);
                    si = __builtin_amdgcn_readfirstlane(r.x);
                    c_lo = __builtin_amdgcn_readfirstlane(r.y);
                    c_hi = __builtin_amdgcn_readfirstlane(r.z);
                } else {
                    while (p0 >= c_hi) {   // runs of no dwords are skipped
                        si++;
                        c_lo = c_hi;
                        c_hi = __builtin_amdgcn_readfirstlane(sp_cum[si + 1]);
                    }
                }
            }
            dwb = __builtin_amdgcn_readfirstlane(sp_dw[si]);
        }
    };
    // Byte offsets (from the tile's first posting) of the lane's dword in
    // each of the U pieces of the wave's step at stream position cb; the
    // cursor only moves forward, and pieces past the end read the tile's
    // trailing padding dwords.  When the step's CH dwords lie inside one run
    // (the common case with long runs) an offset is one scalar base plus the
    // lane's fixed offset, a single vector add; otherwise each piece is
    // placed on its own, and a piece that reaches into later runs or past
    // the end is placed lane by lane.
    const uint32_t lane4 = lane * 4;
    uint32_t off4[U];
    auto step_offsets = [&](uint32_t cb) {
        if (cb < total_dw)
            seek(cb);
        if (cb + CH <= c_hi) {
            const uint32_t sb = (dwb + (cb - c_lo)) * 4;
#pragma unroll
            for (int u = 0; u < U; u++)
                off4[u] = (sb + 256u * u) + lane4;
            return;
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint32_t p0 = cb + u * 64;
            uint32_t off;
            if (p0 >= total_dw) {
                off = sent_dw + lane;
            } else {
                seek(p0);
                if (p0 + 64 <= c_hi) {
                    off = (dwb + (p0 - c_lo)) + lane;   // scalar part + lane
                } else {
                    const uint32_t pos = p0 + lane;
                    if (pos < total_dw) {
                        uint32_t li = si, l_lo = c_lo, l_hi = c_hi, l_dwb = dwb;
                        while (pos >= l_hi) {
                            li++;
                            l_lo = l_hi;
                            l_hi = sp_cum[li + 1];
                            l_dwb = sp_dw[li];
                        }
                        off = l_dwb + (pos - l_lo);
                    } else {
                        off = sent_dw + lane;
                    }
                }
            }
            off4[u] = off * 4;
        }
    };
    // Software pipelining: each step issues the next step's posting loads
    // before its own counting, so the load latency (from L2, the Infinity
    // Cache or HBM) overlaps the LDS atomics; the scheduling barrier keeps
    // the compiler from sinking those loads below the atomics.
    // Chunks of CH dwords: the first ones go to the waves in turn, the last
    // quarter (at least one per wave) is taken by the waves that get there
    // first, one LDS claim per chunk, so the waves end together.
    const uint32_t n_chunks = (total_dw + CH - 1) / CH;
    const uint32_t tail = max(n_chunks / 4, (uint32_t)NWAVE);
    const uint32_t c_static = n_chunks > tail ? n_chunks - tail : 0u;
    auto next_chunk = [&](uint32_t c) -> uint32_t {
        if (c + NWAVE < c_static)
            return c + NWAVE;
        uint32_t x = 0;
        if (lane == 0)
            x = lds_add(&misc[M_TAIL], 1u);
        return c_static + __builtin_amdgcn_readfirstlane(x);
    };
    uint32_t cc = wave < c_static ? wave : next_chunk(c_static);
    uint32_t nv[U];
    step_offsets(cc * CH);
#pragma unroll
    for (int u = 0; u < U; u++)   // uniform 64-bit base + 32-bit byte offset
        nv[u] = *reinterpret_cast<const uint32_t *>(tile_bytes + off4[u]);
    for (; cc < n_chunks;) {
        uint32_t v[U];
#pragma unroll
        for (int u = 0; u < U; u++)
            v[u] = nv[u];
        cc = next_chunk(cc);
        step_offsets(cc * CH);
#pragma unroll
        for (int u = 0; u < U; u++)
            nv[u] = *reinterpret_cast<const uint32_t *>(tile_bytes + off4[u]);
        __builtin_amdgcn_sched_barrier(0);
        uint32_t at_reg = lds_load(&misc[M_AT]);
        const uint32_t at_m1 = at_reg - 1;   // val = f + 1 >= AT  <=>  f >= AT - 1
        // all increments first (no branch between the LDS atomics, so their
        // latencies overlap), then the gate check
        uint32_t f[2 * U], shs[2 * U];
#pragma unroll
        for (int u = 0; u < U; u++) {
#pragma unroll
            for (int h = 0; h < 2; h++) {
                // The counter of id x sits in word x >> log2(CPW), field
                // (x mod CPW) * BITS, which is the low 5 bits of x << log2(BITS)
                // (shifts and bit-field extracts read only those bits), so
                // the field offset and the word's byte address come straight
                // from the posting dword, without isolating the id first.
                const uint32_t w = v[u];
                uint32_t sh, a;
                if (h == 0) {
                    sh = w << LBITS;
                    a = BITS == 8 ? (w & 0xFFFCu) : BITS == 4 ? ((w >> 1) & 0x7FFCu) : ((w << 1) & 0x1FFFCu);
                } else {
                    sh = (w >> 16) << LBITS;
                    a = BITS == 8 ? ((w >> 16) & 0xFFFCu) : BITS == 4 ? ((w >> 17) & 0x7FFCu) : ((w >> 15) & 0x1FFFCu);
                }
                uint32_t inc;   // 1 << (sh mod 32): the shift unit masks the amount
                asm("v_lshlrev_b32 %0, %1, 1" : "=v"(inc) : "v"(sh));
                uint32_t *cw = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(bc) + a);
                if constexpr (SPQ) {   // count only: no value returned, no gate
                    __hip_atomic_fetch_add(cw, inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    f[2 * u + h] = 0;
                } else {
                    f[2 * u + h] = lds_add(cw, inc);   // the word before the add
                    shs[2 * u + h] = sh;
                }
            }
        }
        // Every atomic of the step is issued before the first returned word
        // is used: left to itself the compiler extracts the first fields early
        // and waits for the first atomics before issuing the later ones.
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (!SPQ) {
#pragma unroll
            for (int j = 0; j < 2 * U; j++)
                f[j] = __builtin_amdgcn_ubfe(f[j], shs[j], BITS);
        }
        // Algorithm 1's gate check, first for the whole wave at once: the
        // largest previous count of the lane's postings against AT - 1
        if constexpr (SPQ)
            continue;
        uint32_t fmax = f[0];
#pragma unroll
        for (int j = 1; j < 2 * U; j++)
            fmax = max(fmax, f[j]);
        if (__ballot(fmax >= at_m1)) {
            // Per posting slot j: the passing lanes (not the padding id) add
            // to ZA[val] at once, and the AT advance runs as soon as a level
            // fills, so AT stays current for the next gate checks.  The HT
            // puts go to the wave's queue (a ballot gives the passing lanes
            // and mbcnt each lane's place) and run in rounds of 64, so the
            // wave does not serialise on the few lanes that pass.
#pragma unroll
            for (int u = 0; u < U; u++)
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    // a slot none of whose lanes reach AT costs one compare
                    if (!__ballot(f[2 * u + h] + 1 >= at_reg))
                        continue;
                    const uint32_t lid = h ? (v[u] >> 16) : (v[u] & 0xFFFFu);
                    const uint32_t val = f[2 * u + h] + 1;
                    const bool pass = val >= at_reg && lid != SENT;
                    const uint64_t m = __ballot(pass);
                    if (m) {
                        passes += (uint32_t)__popcll(m);
                        // the ZA add and the AT read go out together (one
                        // LDS round trip); AT is read again only after an
                        // advance of this wave's own
                        const uint32_t zc = pass ? lds_add(&za[val], 1u) + 1 : 0u;
                        at_reg = lds_load(&misc[M_AT]);
                        if (__ballot(zc >= k)) {
                            advance_at(za, misc, k, s);
                            at_reg = lds_load(&misc[M_AT]);
                        }
                        const bool keep = pass && val >= at_reg;
                        const uint64_t mk = __ballot(keep);
                        if (mk) {
                            const uint32_t r = __builtin_amdgcn_mbcnt_hi(
                                (uint32_t)(mk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
                            if (keep)
                                gq[qn + r] = (val << 16) | lid;
                            qn += (uint32_t)__popcll(mk);
                            if (qn >= 64) {   // one full round of HT puts
                                const uint32_t e = gq[qn - 64 + lane];
                                ht_put(ht, lg, misc, e & 0xFFFFu, e >> 16);
                                qn -= 64;
                            }
                        }
                    }
                }
        }
    }
    // drain the queue
    for (uint32_t i0q = 0; i0q < qn; i0q += 64)
        if (i0q + lane < qn) {
            const uint32_t e = gq[i0q + lane];
            ht_put(ht, lg, misc, e & 0xFFFFu, e >> 16);
        }
    if (lane == 0 && passes)
        lds_add(&misc[M_PASSES], passes);
    if constexpr (PF) {
        // the first wave to finish counting prepares the next pair (its
        // loads overlap the counting of the waves still running)
        uint32_t first = 1;
        if (lane == 0)
            first = lds_add(&misc[M_PREFETCH], 1u);
        if (__builtin_amdgcn_readfirstlane(first) == 0)
            prepare_next();
    }
    __syncthreads();
    uint32_t spq_thr = 0;
    if constexpr (SPQ) {
        // GEN-SPQ (the c-PQ ablation of Section 6.3): the counters hold every
        // exact count; the tile's k-th count is found by bisection over them
        // (the largest c with at least min(k, tile_n) objects of count >= c,
        // 0 when fewer objects than that were hit), and selection below then
        // reads the counters alone, as after a Hash Table overflow.
        const uint32_t kk_t = min(p.k, tile_n);
        uint32_t lo = 0, hi = s;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) / 2;
            uint32_t mine = 0;
            for (uint32_t w = tid; w < NW; w += NT) {
                const uint32_t word = bc[w];
#pragma unroll
                for (uint32_t fi = 0; fi < CPW; fi++)
                    mine += (w * CPW + fi < tile_n && ((word >> (fi * BITS)) & MASK) >= mid) ? 1u
                                                                                            : 0u;
            }
            uint32_t total = 0;
            block_exclusive_scan<NT>(mine, misc + M_WAVESUM, &total);
            if (total >= kk_t)
                lo = mid;
            else
                hi = mid - 1;
        }
        spq_thr = lo;
    }
    // settle: AT advances that raced with ZA increments are finished here.
    // ZA is final after the barrier above, and the walk ends at the same AT
    // from any start at or below it, so every thread settles for itself and
    // the selection needs no barrier of its own.
    uint32_t AT = lds_load(&misc[M_AT]);
    while (AT <= s && lds_load(&za[AT]) >= k)
        AT++;
    // select from the counters after a Hash Table overflow (and in GEN-SPQ)
    const bool from_counters = SPQ || lds_load(&misc[M_OVERFLOW]) != 0;
    if constexpr (SPQ)
        AT = spq_thr + 1;
    if (tid == 0) {
        // the pair's statistics: a plain store, summed per query by the merge
        // (one device-scope atomic per pair and counter serialises across
        // the chip); the count dump has no merge and adds them here
        const uint32_t scanned = misc[M_SCANNED], ovf = (from_counters && !SPQ) ? 1u : 0u;
        if (p.pair_stats) {
            p.pair_stats[row] = make_uint4(scanned, ovf, misc[M_INSERTS], misc[M_PASSES]);
        } else {
            unsigned long long *stats = reinterpret_cast<unsigned long long *>(p.status + 2);
            atomicAdd(&stats[0], (unsigned long long)scanned);
            if (ovf)
                atomicAdd(&stats[1], 1ull);
            atomicAdd(&stats[2], (unsigned long long)misc[M_INSERTS]);
            atomicAdd(&stats[3], (unsigned long long)misc[M_PASSES]);
        }
    }

    if (DUMP) {
        for (uint32_t i = tid; i < tile_n; i += NT) {
            const uint32_t word = i / CPW, sh = (i - word * CPW) * BITS;
            p.full_counts[(uint64_t)q * p.n + tile0 + i] = (bc[word] >> sh) & MASK;
        }
        return;
    }

    // ---- select (Theorem 3.1): AT - 1 is the tile's k-th count
    const uint32_t thr = AT - 1;
    const uint32_t kk = min(k, tile_n);
    uint64_t *out = p.cand + row * k;
    // (1) count >= AT: fewer than k objects (Lemma 3.1), all in the HT.
    //     Each is read back from the counters (exact) and marked emitted, so
    //     duplicate HT slots are emitted once.
    auto claim = [&](uint32_t lid) {
        const uint32_t word = lid / CPW, sh = (lid - word * CPW) * BITS;
        const uint32_t c = (lds_load(&bc[word]) >> sh) & MASK;
        if (c == MASK || c < AT)
            return;
        const uint32_t old = (lds_or(&bc[word], MASK << sh) >> sh) & MASK;
        if (old == MASK)
            return;
        const uint32_t pos = lds_add(&misc[M_NABOVE], 1);
        if (pos < kk)
            out[pos] = make_key(old, (uint32_t)(gid0 + lid));
    };
    if (!from_counters) {
        for (uint32_t slot = tid; slot < cap; slot += NT) {
            const uint32_t cur = ht[slot];
            if (cur != 0 && (cur & 0xFFFFu) < tile_n)
                claim(cur & 0xFFFFu);
        }
    } else {
        for (uint32_t lid = tid; lid < tile_n; lid += NT)
            claim(lid);
    }
    // (2) count == AT - 1: the smallest ids, read from the counters in id
    //     order.  Thread t owns a contiguous range of counter words; a
    //     workgroup prefix count of the ties turns local order into the rank
    //     in id order.  The ties are counted in the same phase as the claims
    //     above: a claim only turns a count >= AT into the emitted mark, a
    //     field the tie count does not look at.
    uint32_t emitted;
    {
        constexpr uint32_t WPT = NW / NT;  // words per thread
        static_assert(WPT * NT == NW && WPT <= 64 && (WPT & (WPT - 1)) == 0, "tie pass layout");
        const uint32_t wb = tid * WPT, we = wb + WPT;
        // Counting is order-free, so each thread visits its words rotated by
        // its lane group: lane a * (64 / WPT) + b reads word b * WPT +
        // ((j + a) mod WPT) of the wave's block at step j, and the 64 lanes
        // of one read hit 64 different LDS banks (in id order they would
        // share 64 / WPT banks, stalling the counting of the workgroup that
        // shares the CU).
        const uint32_t rot = (tid & 63) >> (6 - ilog2(WPT));
        uint32_t mine = 0;
#pragma unroll 8
        for (uint32_t j = 0; j < WPT; j++) {
            const uint32_t w = wb + ((j + rot) & (WPT - 1));
            // claims may be updating other fields of this word: atomic read
            mine += fields_equal<BITS>(lds_load(&bc[w]), thr, tile_n, w * CPW);
        }
        // rank of the thread's first tie in id order: a wave prefix sum, then
        // the wave totals through LDS (one barrier, which also completes the
        // claims; the totals are not written again before the next pair's
        // barriers)
        const uint32_t incl = wave_inclusive_sum(mine);
        uint32_t *wsum = misc + M_WAVESUM;
        if ((tid & 63) == 63)
            wsum[tid >> 6] = incl;
        __syncthreads();
        const uint32_t n_above = min(misc[M_NABOVE], kk);
        const uint32_t need = kk - n_above;
        uint32_t before = 0, total = 0;
#pragma unroll
        for (uint32_t w = 0; w < NWAVE; w++) {
            const uint32_t v = wsum[w];
            before += w < (tid >> 6) ? v : 0u;
            total += v;
        }
        uint32_t r = before + incl - mine;
        // fewer than need only when AT started above the tile's k-th count
        emitted = n_above + min(need, total);
        if (mine && r < need) {
            // the thread's words in id order, read a batch at a time so that
            // the LDS latencies overlap
            constexpr uint32_t B = WPT < 8 ? WPT : 8;
            for (uint32_t w0 = wb; w0 < we && r < need; w0 += B) {
                uint32_t wd[B];
#pragma unroll
                for (uint32_t u = 0; u < B; u++)
                    wd[u] = bc[w0 + u];
#pragma unroll
                for (uint32_t u = 0; u < B; u++) {
                    // the word's tied fields in id order, one bit each
                    uint32_t z = fields_equal_mask<BITS>(wd[u], thr, tile_n, (w0 + u) * CPW);
                    while (z != 0 && r < need) {
                        const uint32_t f = (uint32_t)__builtin_ctz(z) >> LBITS;
                        z &= z - 1;
                        out[n_above + r] = make_key(thr, (uint32_t)(gid0 + (w0 + u) * CPW + f));
                        r++;
                    }
                }
            }
        }
    }
    for (uint32_t i = emitted + tid; i < k; i += NT)
        out[i] = 0;
    if (tid == 0)
        p.tile_kth[row] = thr;
}

template <int BITS, int NT, int U, bool DUMP, int LG, int SCHED, bool SPQ = false>
__global__ __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(scan_waves_per_eu<BITS, NT, LG>())))
void scan_cpq_kernel(ScanParams p) {
    constexpr uint32_t CPW = 32 / BITS;
    constexpr uint32_t NW = (1u << LG) / CPW;
    // The Bitmap Counter has a fixed size per counter width; as a static
    // array at LDS offset 0 its addresses need no base register.
    __shared__ uint32_t bc[NW];
    extern __shared__ uint32_t smem[];
    // XCD-aware mapping: consecutive workgroup ids go to different XCDs, so
    // each XCD gets a contiguous slice of the (tile, query) pairs, tile-major,
    // and its L2 keeps serving the same tile's postings.
    const uint32_t bid = blockIdx.x;
    const uint64_t npairs = (uint64_t)p.nq * p.n_tiles;
    if constexpr (SCHED == kSchedGrid) {   // one workgroup per pair
        const uint64_t pair = (uint64_t)(bid & 7) * p.per_xcd + (bid >> 3);
        if (pair < npairs)
            scan_pair<BITS, NT, U, DUMP, LG, SPQ>(p, pair, bc, smem);
    } else if constexpr (SCHED == kSchedRows) {
        // only the pairs of the qcount rows: pair index i is tile i / qc of
        // row i mod qc; no work, and no dispatch of one workgroup per pair,
        // when the count is 0
        const uint32_t qc = *p.qcount;
        const uint64_t n = (uint64_t)qc * p.n_tiles;
        for (uint64_t i = bid; i < n; i += gridDim.x) {
            const uint64_t t = i / qc, qrow = i - t * qc;
            scan_pair<BITS, NT, U, DUMP, LG, SPQ>(p, t * p.nq + qrow, bc, smem);
            __syncthreads();   // the next pair reuses the LDS
        }
    } else {
        // Persistent schedule: as many workgroups as fit the device at once,
        // each taking the next pair of its XCD's slice from that slice's
        // counter (one atomic per pair), then helping the other slices in
        // turn (claim_pair).  A pair's claim and run table are prepared while
        // the workgroup still counts the pair before it, in the other of two
        // run-table slots.  Every workgroup leaves once all eight counters
        // have run past their slices.
        (void)npairs;
        if (threadIdx.x == 0) {
            smem[M_XCD] = bid & 7;
            smem[M_SPENT] = 0;
        }
        __syncthreads();
        uint32_t *tables = smem + 32 + (1u << p.ht_log2) + (p.max_items + 2);
        if (threadIdx.x < 64)
            prepare_pair(p, smem, tables, tables + p.max_items, smem + M_SLOT);
        __syncthreads();
        for (uint32_t slot = 0;; slot ^= 1u) {
            const uint32_t pair =
                __builtin_amdgcn_readfirstlane(smem[M_SLOT + slot * H_WORDS + H_PAIR]);
            if (pair == kNoPair)
                break;
            scan_pair<BITS, NT, U, DUMP, LG, SPQ, true>(p, pair, bc, smem, slot);
            __syncthreads();   // the next pair reuses the LDS
        }
    }
}

// Per query: the largest tile k-th count is a floor of the global k-th
// count; a histogram of the candidates' counts above the floor gives the
// global k-th count itself (or a floor of it when it lies past the top bin).
// Only candidates reaching it are sorted by key; emit the top k.
constexpr int kMergeBuf = 4096;   // keys held in LDS
constexpr int kMergeChunk = 2048; // candidates read per round
constexpr int kMergeBins = 256;   // counts floor .. floor + 254, and above
template <int NT>
__global__ __launch_bounds__(NT) void merge_kernel(MergeParams p) {
    static_assert(NT >= 64 && NT % 64 == 0, "wave 0 reads the histogram");
    __shared__ uint64_t buf[kMergeBuf];
    __shared__ uint32_t hist[kMergeBins];
    __shared__ uint32_t s_cnt, s_floor, s_thr, s_reached;
    __shared__ unsigned long long s_stats[4];
    if (p.qcount && blockIdx.x >= *p.qcount)
        return;
    const uint32_t q = p.qlist ? p.qlist[blockIdx.x] : blockIdx.x;
    const uint32_t tid = threadIdx.x, k = p.k;
    const uint64_t ncand = (uint64_t)p.n_tiles * k;
    const uint64_t *cand = p.cand + (uint64_t)q * ncand;
    if (tid == 0) {
        s_floor = 0;
        s_cnt = 0;
    }
    if (tid < 4)
        s_stats[tid] = 0;
    for (uint32_t b = tid; b < kMergeBins; b += NT)
        hist[b] = 0;
    __syncthreads();
    uint32_t fl = 0;
    unsigned long long st0 = 0, st1 = 0, st2 = 0, st3 = 0;
    for (uint32_t t = tid; t < p.n_tiles; t += NT) {
        fl = max(fl, p.tile_kth[(uint64_t)q * p.n_tiles + t]);
        const uint4 v = p.pair_stats[(uint64_t)q * p.n_tiles + t];
        st0 += v.x;
        st1 += v.y;
        st2 += v.z;
        st3 += v.w;
    }
    atomicMax(&s_floor, fl);
    if (st0 | st1 | st2 | st3) {
        atomicAdd(&s_stats[0], st0);
        atomicAdd(&s_stats[1], st1);
        atomicAdd(&s_stats[2], st2);
        atomicAdd(&s_stats[3], st3);
    }
    __syncthreads();
    if (tid < 4 && s_stats[tid]) {   // the query's statistics into the status block
        unsigned long long *stats = reinterpret_cast<unsigned long long *>(p.status + 2);
        atomicAdd(&stats[tid], s_stats[tid]);
    }
    const uint32_t floor_count = s_floor;
    for (uint64_t i = tid; i < ncand; i += NT) {
        const uint64_t key = cand[i];
        const uint32_t c = (uint32_t)(key >> 32);
        if (key != 0 && c >= floor_count)
            atomicAdd(&hist[min(c - floor_count, (uint32_t)kMergeBins - 1u)], 1u);
    }
    __syncthreads();
    if (tid < 64) {
        // lane l holds bins 4(63 - l) .. 4(63 - l) + 3, so the wave's
        // inclusive sum is the number of candidates at or above each lane's
        // lowest bin; the first lane to reach k holds the k-th count
        const uint32_t b0 = 4u * (63u - tid);
        const uint32_t h0 = hist[b0], h1 = hist[b0 + 1], h2 = hist[b0 + 2], h3 = hist[b0 + 3];
        const uint32_t v = h0 + h1 + h2 + h3;
        const uint32_t at_or_above = wave_inclusive_sum(v);
        const uint64_t hit = __ballot(at_or_above >= k);
        if (tid == 63)
            s_reached = at_or_above;
        if (hit == 0) {
            if (tid == 0)
                s_thr = floor_count;   // fewer than k candidates: keep them all
        } else if (tid == (uint32_t)(__ffsll((unsigned long long)hit) - 1)) {
            uint32_t above = at_or_above - v + h3, b = b0 + 3;
            if (above < k) {
                above += h2;
                b--;
                if (above < k) {
                    above += h1;
                    b--;
                    if (above < k)
                        b--;
                }
            }
            s_thr = floor_count + b;
        }
    }
    __syncthreads();
    const uint32_t thr = s_thr;
    const uint32_t kept = s_reached;   // candidates that reached the floor
    uint32_t kc = 0;     // valid keys at the front of buf, sorted descending
    for (uint64_t c0 = 0; c0 < ncand; c0 += kMergeChunk) {
        const uint64_t c1 = min<uint64_t>(ncand, c0 + kMergeChunk);
        for (uint64_t i = c0 + tid; i < c1; i += NT) {
            const uint64_t key = cand[i];
            if (key != 0 && (uint32_t)(key >> 32) >= thr) {
                const uint32_t pos = atomicAdd(&s_cnt, 1u);
                buf[kc + pos] = key;
            }
        }
        __syncthreads();
        const uint32_t added = s_cnt;
        __syncthreads();
        if (tid == 0)
            s_cnt = 0;
        __syncthreads();
        if (added == 0)
            continue;
        const uint32_t m = kc + added;
        uint32_t np2 = 1;
        while (np2 < m)
            np2 <<= 1;
        for (uint32_t i = m + tid; i < np2; i += NT)
            buf[i] = 0;
        __syncthreads();
        // bitonic sort, descending
        for (uint32_t size = 2; size <= np2; size <<= 1) {
            for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                for (uint32_t i = tid; i < np2 / 2; i += NT) {
                    const uint32_t lo = 2 * i - (i & (stride - 1));
                    const uint32_t hi = lo + stride;
                    const bool desc = (lo & size) == 0;
                    const uint64_t a = buf[lo], b = buf[hi];
                    if ((a < b) == desc) {
                        buf[lo] = b;
                        buf[hi] = a;
                    }
                }
                __syncthreads();
            }
        }
        kc = min(m, k);
    }
    // Gated search: when fewer than min(k, n) candidates reached the floor,
    // the query's k-th count lies below where its AT started; it is answered
    // again with AT = 1.
    if (p.fb_count && kept < min<uint64_t>(k, p.n)) {
        if (tid == 0)
            p.fb_list[atomicAdd(p.fb_count, 1u)] = q;
        return;
    }
    for (uint32_t i = tid; i < k; i += NT) {
        const uint64_t key = i < kc ? buf[i] : 0ull;
        p.out_ids[(uint64_t)q * k + i] = 0xFFFFFFFFu - (uint32_t)key;
        p.out_counts[(uint64_t)q * k + i] = (uint32_t)(key >> 32);
    }
}

// Status block: flags, statistics, the fallback count and the persistent
// schedule's pair counters (words 16..23; words 24..31 are spare).
constexpr uint32_t kStatusWords = 32;
constexpr uint64_t kPersistentMinPairs = 1024;   // below: one workgroup per pair
constexpr uint32_t kWorkWord = 16;
__global__ void clear_status_kernel(uint32_t *status) {
    if (threadIdx.x < kStatusWords)
        status[threadIdx.x] = 0;
}

template <int BITS, int NT, int U, int LG>
int launch_scan(const ScanParams &sp, bool dump, size_t lds, uint64_t grid, hipStream_t st) {
    // the count dump (match-count entry point) always runs 1024 x 4, one
    // workgroup per pair
    // (the GEN-SPQ ablation likewise)
    const void *kern =
        dump ? (const void *)scan_cpq_kernel<BITS, 1024, 4, true, LG, kSchedGrid>
        : sp.spq ? (const void *)scan_cpq_kernel<BITS, 1024, 4, false, LG, kSchedGrid, true>
        : sp.rows_loop ? (const void *)scan_cpq_kernel<BITS, NT, U, false, LG, kSchedRows>
        : sp.work ? (const void *)scan_cpq_kernel<BITS, NT, U, false, LG, kSchedQueue>
                  : (const void *)scan_cpq_kernel<BITS, NT, U, false, LG, kSchedGrid>;
    const int nt = (dump || sp.spq) ? 1024 : NT;
    GENIE_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    if ((sp.work || sp.rows_loop) && !dump && !sp.spq) {
        // persistent and row schedules: the workgroups that fit the device at once
        // (a multiple of 8, so that every XCD has the same number)
        int dev = 0, cus = 0, per_cu = 0;
        GENIE_HIP(hipGetDevice(&dev));
        GENIE_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        GENIE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, nt, lds));
        const uint64_t resident = std::max<uint64_t>(8, (uint64_t)cus * std::max(per_cu, 1) / 8 * 8);
        grid = std::min<uint64_t>(grid, resident);
    }
    ScanParams arg = sp;
    void *args[] = {&arg};
    void *ev = timing_begin(st);
    GENIE_HIP(hipLaunchKernel(kern, dim3((uint32_t)grid), dim3(nt), args, lds, st));
    timing_end(ev, st, sp.rows_loop ? 2 : 0);   // the row schedule is the fallback pass
    GENIE_HIP(hipGetLastError());
    return GENIE_OK;
}

template <int BITS, int LG>
int dispatch_shape(int nt, int u, const ScanParams &sp, bool dump, size_t lds, uint64_t grid,
                   hipStream_t st) {
    if (nt == 512 && u == 4) return launch_scan<BITS, 512, 4, LG>(sp, dump, lds, grid, st);
    if (nt == 512 && u == 8) return launch_scan<BITS, 512, 8, LG>(sp, dump, lds, grid, st);
    if (nt == 1024 && u == 4) return launch_scan<BITS, 1024, 4, LG>(sp, dump, lds, grid, st);
    if (nt == 1024 && u == 8) return launch_scan<BITS, 1024, 8, LG>(sp, dump, lds, grid, st);
    set_error("no scan kernel for %d threads x %d dwords", nt, u);
    return GENIE_EINVAL;
}

template <int LG>
int dispatch_bits(int bits, int nt, int u, const ScanParams &sp, bool dump, size_t lds,
                  uint64_t grid, hipStream_t st) {
    switch (bits) {
    case 4: return dispatch_shape<4, LG>(nt, u, sp, dump, lds, grid, st);
    case 8: return dispatch_shape<8, LG>(nt, u, sp, dump, lds, grid, st);
    case 16: return dispatch_shape<16, LG>(nt, u, sp, dump, lds, grid, st);
    default: set_error("no kernel for %d-bit counters", bits); return GENIE_ERANGE;
    }
}

int dispatch_scan(int bits, int nt, int u, uint32_t tile_log2, const ScanParams &sp, bool dump,
                  size_t lds, uint64_t grid, hipStream_t st) {
    switch (tile_log2) {
    case 15: return dispatch_bits<15>(bits, nt, u, sp, dump, lds, grid, st);
    case 16: return dispatch_bits<16>(bits, nt, u, sp, dump, lds, grid, st);
    default: set_error("no kernel for tiles of 2^%u - 1 objects", tile_log2); return GENIE_ERANGE;
    }
}

}  // namespace

int launch_clear_status(void *d_workspace, hipStream_t stream) {
    hipLaunchKernelGGL(clear_status_kernel, dim3(1), dim3(64), 0, stream,
                       static_cast<uint32_t *>(d_workspace));
    GENIE_HIP(hipGetLastError());
    return GENIE_OK;
}

int launch_part_scan(const IndexView &v, uint64_t id_base, uint32_t tile_off,
                     uint32_t tiles_total, const uint64_t *d_q_offsets, const genie_item *d_items,
                     uint64_t n_items, uint32_t n_queries, uint32_t max_items, uint32_t k,
                     void *d_workspace, hipStream_t stream) {
    const WorkspaceLayout L = workspace_layout_tiles(tiles_total, n_queries, k);
    SearchShape shape;
    int rc = search_shape(max_items, k, v.scan_threads, v.tile_log2, &shape);
    if (rc)
        return rc;
    char *ws = static_cast<char *>(d_workspace);
    ScanParams sp{};
    sp.post = v.post;
    sp.tile_base = v.tile_base;
    sp.map_ck = reinterpret_cast<const uint2 *>(v.tix);
    sp.map_len = reinterpret_cast<const uint4 *>(v.tix + map_ck_bytes(v.n_tiles, v.nkeys));
    sp.map_groups = map_groups(v.nkeys);
    sp.map_compact = v.map_compact ? 1u : 0u;
    sp.n = v.n;
    sp.nkeys = v.nkeys;
    sp.d = v.d;
    sp.V = v.V;
    sp.n_tiles = v.n_tiles;
    sp.id_base = id_base;
    sp.tile_off = tile_off;
    sp.tiles_total = tiles_total;
    sp.q_off = d_q_offsets;
    sp.items = reinterpret_cast<const uint32_t *>(d_items);
    sp.n_items = n_items;
    sp.nq = n_queries;
    sp.k = k;
    sp.max_items = max_items;
    sp.ht_log2 = shape.ht_log2;
    const uint64_t pairs = (uint64_t)n_queries * v.n_tiles;
    sp.per_xcd = (pairs + 7) / 8;
    sp.cand = reinterpret_cast<uint64_t *>(ws + L.cand);
    sp.tile_kth = reinterpret_cast<uint32_t *>(ws + L.tile_kth);
    sp.pair_stats = reinterpret_cast<uint4 *>(ws + L.pair_stats);
    sp.status = reinterpret_cast<uint32_t *>(ws + L.status);
    const uint64_t grid = sp.per_xcd * 8;
    if (grid > 0x7FFFFFFFull) {
        set_error("too many (query, tile) pairs in one call");
        return GENIE_ERANGE;
    }
    return dispatch_scan(shape.bits, v.scan_threads, v.scan_unroll, v.tile_log2, sp, false,
                         shape.lds_bytes, grid, stream);
}

int launch_part_merge(uint64_t n_total, uint32_t tiles_total, uint32_t n_queries, uint32_t k,
                      void *d_workspace, uint32_t *d_out_ids, uint32_t *d_out_counts,
                      hipStream_t stream) {
    const WorkspaceLayout L = workspace_layout_tiles(tiles_total, n_queries, k);
    char *ws = static_cast<char *>(d_workspace);
    MergeParams mp{};
    mp.cand = reinterpret_cast<uint64_t *>(ws + L.cand);
    mp.tile_kth = reinterpret_cast<uint32_t *>(ws + L.tile_kth);
    mp.pair_stats = reinterpret_cast<const uint4 *>(ws + L.pair_stats);
    mp.status = reinterpret_cast<uint32_t *>(ws + L.status);
    mp.n = n_total;
    mp.n_tiles = tiles_total;
    mp.k = k;
    mp.out_ids = d_out_ids;
    mp.out_counts = d_out_counts;
    void *ev = timing_begin(stream);
    hipLaunchKernelGGL(merge_kernel<256>, dim3(n_queries), dim3(256), 0, stream, mp);
    timing_end(ev, stream, 1);
    GENIE_HIP(hipGetLastError());
    return GENIE_OK;
}

int launch_search(const genie_index *ix, const uint64_t *d_q_offsets, const genie_item *d_items,
                  uint64_t n_items, uint32_t n_queries, uint32_t max_items, uint32_t k, uint32_t *d_out_ids,
                  uint32_t *d_out_counts, uint32_t *d_full_counts, void *d_workspace,
                  size_t workspace_bytes, hipStream_t stream, const float *d_gate,
                  float gate_delta, const uint32_t *d_rows, bool spq) {
    const bool dump = d_full_counts != nullptr;
    const WorkspaceLayout L = workspace_layout(ix, n_queries, k);
    if (workspace_bytes < L.total) {
        set_error("workspace of %zu bytes is smaller than the %zu needed", workspace_bytes,
                  L.total);
        return GENIE_EINVAL;
    }
    SearchShape shape;
    // the count dump and the GEN-SPQ ablation run 1024 x 4
    const int threads = (dump || spq) ? 1024 : ix->scan_threads;
    // the persistent schedule keeps a second run table in LDS; where that
    // does not fit, the search runs one workgroup per pair instead.  A
    // search over a device row count (graph replay at a fixed capacity) also
    // runs one workgroup per pair: the pairs of rows past the count exit at
    // once there, while persistent workgroups would claim every one of them
    // through the device counters.  Under the automatic schedule (2), so
    // does a batch of fewer pairs than about two rounds of resident
    // workgroups, where a workgroup would count one pair and gain nothing
    // from preparing the next.
    bool persistent = ix->scan_persistent && !dump && !spq && !d_rows &&
                      (ix->scan_persistent == 1 ||
                       (uint64_t)n_queries * ix->n_tiles >= kPersistentMinPairs);
    int rc = search_shape(max_items, k, threads, ix->tile_log2, &shape, ix->ht_log2_cap,
                          persistent);
    if (rc && persistent) {
        persistent = false;
        rc = search_shape(max_items, k, threads, ix->tile_log2, &shape, ix->ht_log2_cap);
    }
    if (rc)
        return rc;
    char *ws = static_cast<char *>(d_workspace);
    ScanParams sp{};
    sp.post = ix->post;
    sp.tile_base = ix->tile_base;
    sp.map_ck = reinterpret_cast<const uint2 *>(ix->tix);
    sp.map_len = reinterpret_cast<const uint4 *>(ix->tix + map_ck_bytes(ix->n_tiles, ix->nkeys));
    sp.map_groups = map_groups(ix->nkeys);
    sp.map_compact = ix->map_compact ? 1u : 0u;
    sp.n = ix->n;
    sp.nkeys = ix->nkeys;
    sp.d = ix->d;
    sp.V = ix->V;
    sp.key_sets = ix->key_sets ? 1u : 0u;
    sp.n_tiles = ix->n_tiles;
    sp.id_base = 0;
    sp.tile_off = 0;
    sp.tiles_total = ix->n_tiles;
    sp.q_off = d_q_offsets;
    sp.items = reinterpret_cast<const uint32_t *>(d_items);
    sp.n_items = n_items;
    sp.nq = n_queries;
    sp.k = k;
    sp.max_items = max_items;
    sp.ht_log2 = shape.ht_log2;
    const uint64_t pairs = (uint64_t)n_queries * ix->n_tiles;
    sp.per_xcd = (pairs + 7) / 8;
    sp.cand = reinterpret_cast<uint64_t *>(ws + L.cand);
    sp.tile_kth = reinterpret_cast<uint32_t *>(ws + L.tile_kth);
    sp.pair_stats = dump ? nullptr : reinterpret_cast<uint4 *>(ws + L.pair_stats);
    sp.full_counts = d_full_counts;
    sp.status = reinterpret_cast<uint32_t *>(ws + L.status);
    sp.gate = d_gate;
    sp.gate_delta = gate_delta;
    sp.spq = spq ? 1u : 0u;
    sp.work = persistent ? sp.status + kWorkWord : nullptr;
    sp.qcount = d_rows;   // live rows (device), or null: all n_queries
    const uint64_t grid = sp.per_xcd * 8;
    if (grid > 0x7FFFFFFFull) {
        set_error("too many (query, tile) pairs in one call");
        return GENIE_ERANGE;
    }
    hipLaunchKernelGGL(clear_status_kernel, dim3(1), dim3(64), 0, stream, sp.status);
    GENIE_HIP(hipGetLastError());
    rc = dispatch_scan(shape.bits, ix->scan_threads, ix->scan_unroll, ix->tile_log2, sp, dump,
                       shape.lds_bytes, grid, stream);
    if (rc || dump)
        return rc;
    MergeParams mp{};
    mp.cand = sp.cand;
    mp.tile_kth = sp.tile_kth;
    mp.pair_stats = sp.pair_stats;
    mp.status = sp.status;
    mp.n = ix->n;
    mp.n_tiles = ix->n_tiles;
    mp.k = k;
    mp.out_ids = d_out_ids;
    mp.out_counts = d_out_counts;
    mp.qcount = d_rows;
    uint32_t *fb_count = sp.status + kStatusFallbackWord;
    uint32_t *fb_list = reinterpret_cast<uint32_t *>(ws + L.fb_list);
    if (d_gate) {
        mp.fb_count = fb_count;
        mp.fb_list = fb_list;
    }
    void *ev = timing_begin(stream);
    hipLaunchKernelGGL(merge_kernel<256>, dim3(n_queries), dim3(256), 0, stream, mp);
    timing_end(ev, stream, 1);
    GENIE_HIP(hipGetLastError());
    if (!d_gate)
        return GENIE_OK;
    // fallback pass: the flagged queries again with AT = 1 (workgroups past
    // the device-side count exit at once)
    ScanParams fp = sp;
    fp.gate = nullptr;
    fp.qlist = fb_list;
    fp.qcount = fb_count;
    fp.work = nullptr;
    fp.rows_loop = 1;   // resident workgroups over the flagged rows' pairs only
    rc = dispatch_scan(shape.bits, ix->scan_threads, ix->scan_unroll, ix->tile_log2, fp, false,
                       shape.lds_bytes, grid, stream);
    if (rc)
        return rc;
    MergeParams fm = mp;
    fm.fb_count = nullptr;
    fm.fb_list = nullptr;
    fm.qlist = fb_list;
    fm.qcount = fb_count;
    hipLaunchKernelGGL(merge_kernel<256>, dim3(n_queries), dim3(256), 0, stream, fm);
    GENIE_HIP(hipGetLastError());
    return GENIE_OK;
}

// ---------------------------------------------------------------------------
// Workspace held by the library for callers that cannot allocate device
// memory (genie_search_noalloc_async).  Every GPU the library runs on gets
// its own copy of this array when the code object is loaded there, at its
// own address, and keeps it until the process ends.  In host code the
// array's name is only a host-side stand-in; the device address comes from
// hipGetSymbolAddress, asked once per device with that device current.
// ---------------------------------------------------------------------------
namespace {
__device__ __align__(256) uint8_t scratch[GENIE_NOALLOC_WORKSPACE_BYTES];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

int noalloc_workspace(int device, void **out) {
    if (device < 0 || device >= kMaxScratchDevices) {
        set_error("device %d outside the %d devices the held workspace supports", device,
                  kMaxScratchDevices);
        return GENIE_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        GENIE_HIP(hipGetDevice(&cur));
        if (cur != device) {
            set_error("device %d is not current (current: %d)", device, cur);
            return GENIE_EINVAL;
        }
        void *ptr = nullptr;
        GENIE_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr || ((uintptr_t)ptr & 255) != 0) {
            set_error("held workspace has no usable device address");
            return GENIE_EDEVICE;
        }
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return GENIE_OK;
}

}  // namespace genie
