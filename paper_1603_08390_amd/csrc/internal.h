// Internal declarations of libgenie (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "genie.h"

// Tiles of 2^L - 1 objects (L = tile_log2, 15 or 16).  Local ids inside a
// tile fit L bits, so postings are stored as uint16 and a tile's counters
// (2^L of them) fit one workgroup's LDS.  The id 2^L - 1 is never an
// object: it pads keyword runs to an even length.
constexpr uint32_t kTileLog2Default = 16;
constexpr uint32_t tile_objects_of(uint32_t tile_log2) { return (1u << tile_log2) - 1u; }
static_assert(tile_objects_of(kTileLog2Default) == GENIE_TILE_OBJECTS, "default tiling");
constexpr uint64_t kSentinelDwords = 64;   // all-sentinel dwords after each tile's runs

// LDS available to one workgroup on gfx950.
constexpr size_t kMaxLdsBytes = 160 * 1024;

// Scan kernel launch shapes compiled in: threads per workgroup in {512,
// 1024} (at least 512: the run table prefix sum gives each thread two of at
// most 1024 runs) and posting dwords each thread loads per step in {4, 8}.
// The default is the fastest measured on the relational workload; an index
// can be given another one (genie_index_set_scan_shape).
constexpr int kScanThreadsDefault = 1024;
constexpr int kScanUnrollDefault = 4;
// Gate queue entries per wave (LDS words): fewer than 64 wait between
// rounds, and one posting slot adds at most 64.
constexpr uint32_t kGateQueue = 128;

struct genie_index {
    uint64_t n = 0;          // objects
    uint32_t d = 0;          // dimensions
    uint32_t V = 0;          // buckets (values) per dimension
    uint32_t tile_log2 = kTileLog2Default;
    uint32_t tile_objects = tile_objects_of(kTileLog2Default);   // also the padding id
    uint32_t n_tiles = 0;    // ceil(n / tile_objects)
    uint64_t nkeys = 0;      // d * V keywords
    uint64_t n_postings = 0; // n * d
    // device arrays
    uint16_t *post = nullptr;      // tile-major, keyword-major, ascending local ids (+ pad)
    uint64_t *tile_base = nullptr; // n_tiles + 1 element offsets of each tile in post
    // Position Map per tile (offsets relative to tile_base): n_tiles rows of
    // nkeys + 1 pairs {padded offset, padded runs before} (one 8-byte read per
    // lookup), or, where that would exceed a quarter of the postings' bytes,
    // the compact form of compact_offsets (3 bytes per keyword)
    uint8_t *tix = nullptr;
    bool map_compact = false;
    uint64_t map_bytes = 0;
    uint64_t *kcum = nullptr;      // nkeys + 1 prefix counts of postings per keyword (all tiles)
    uint64_t stored_postings = 0;  // elements in post (real + padding + trailing sentinels)
    uint64_t device_bytes = 0;
    int device = 0;
    int scan_threads = kScanThreadsDefault;   // launch shape of the scan kernel
    int scan_unroll = kScanUnrollDefault;
    int scan_persistent = 2;                  // 0: a workgroup per pair; 1: persistent
                                              // workgroups; 2: persistent for large calls
    uint32_t ht_log2_cap = 0;                 // Hash Table slots capped at 2^cap (0: no cap)
    bool key_sets = false;                    // built from keyword sets: d = 1, V = keywords
};

namespace genie {

// An index built in host memory (the layout of genie_index's device arrays).
struct HostIndex {
    uint64_t n = 0, nkeys = 0, n_postings = 0;
    uint32_t d = 0, V = 0, n_tiles = 0, tile_log2 = 0;
    std::vector<uint16_t> post;
    std::vector<uint64_t> tile_base, kcum;
    std::vector<uint32_t> toff, tpad;
    bool key_sets = false;
};
int build_host_index(const uint32_t *values, uint64_t n, uint32_t d, uint32_t V,
                     uint32_t tile_log2, HostIndex *h);
// Objects given as keyword sets: object o holds keys[obj_offsets[o] ..
// obj_offsets[o+1]), each below n_keys.  The index has d = 1 and V = n_keys,
// so the item (0, key, key) is the list of one keyword.
int build_host_index_sets(const uint64_t *obj_offsets, const uint32_t *keys, uint64_t n,
                          uint32_t n_keys, uint32_t tile_log2, HostIndex *h);
int upload_host_index(const HostIndex &h, genie_index **out);

// Device form of the Position Map (Section 3.2), restricted per tile: for
// each tile, keywords 0..nkeys in groups of 8, each group one 8-byte
// checkpoint {padded offset, padded runs before} of its first keyword and
// one 16-byte record of the 8 keywords' real run lengths (uint16: a tile
// holds fewer than 2^16 objects, each at most once per keyword).  A
// keyword's offset is its group's checkpoint plus the padded lengths of the
// keywords before it in the group.  3 bytes per (tile, keyword) instead of
// 8.  Layout: checkpoints of every tile's groups (padded to 16 bytes), then
// the length records.
constexpr uint64_t kMapGroup = 8;
inline uint64_t map_groups(uint64_t nkeys) { return nkeys / kMapGroup + 1; }
inline size_t map_ck_bytes(uint64_t n_tiles, uint64_t nkeys) {
    return (size_t)((n_tiles * map_groups(nkeys) * 8 + 15) & ~uint64_t(15));
}
inline size_t map_bytes(uint64_t n_tiles, uint64_t nkeys) {
    return map_ck_bytes(n_tiles, nkeys) + (size_t)(n_tiles * map_groups(nkeys) * 16);
}
// Writes h's Position Map in that device form (map_bytes(n_tiles, nkeys)).
void compact_offsets(const HostIndex &h, uint8_t *dst);
// The 8-byte form: n_tiles * (nkeys + 1) pairs {toff[i], tpad[i]}.
void interleave_offsets(const HostIndex &h, uint32_t *dst);
inline size_t full_map_bytes(uint64_t n_tiles, uint64_t nkeys) {
    return (size_t)(n_tiles * (nkeys + 1) * 8);
}
// The form an index uses: compact where the 8-byte form would exceed a
// quarter of the postings' bytes.
inline bool use_compact_map(const HostIndex &h) {
    return full_map_bytes(h.n_tiles, h.nkeys) * 4 > h.post.size() * sizeof(uint16_t);
}
inline size_t device_map_bytes(const HostIndex &h) {
    return use_compact_map(h) ? map_bytes(h.n_tiles, h.nkeys) : full_map_bytes(h.n_tiles, h.nkeys);
}
// Writes h's Position Map in the form use_compact_map picks.
void write_offsets(const HostIndex &h, uint8_t *dst);

void set_error(const char *fmt, ...);
void clear_error();
int hip_fail(hipError_t e, const char *what);

#define GENIE_HIP(call)                                                      \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess)                                                \
            return ::genie::hip_fail(e_, #call);                             \
    } while (0)

// Workspace layout of one search call (all offsets 256-byte aligned).
struct WorkspaceLayout {
    size_t status = 0;     // uint32 flags + pad, uint64 stats[4], uint32 fallback count
    size_t tile_kth = 0;   // uint32 [n_queries * n_tiles]
    size_t cand = 0;       // uint64 [n_queries * n_tiles * k]
    size_t pair_stats = 0; // uint32 x 4 [n_queries * n_tiles]: postings scanned, hash-table
                           // overflow (0/1), insertions, gate passes of each pair
    size_t fb_list = 0;    // uint32 [n_queries] (gated search)
    size_t total = 0;
};
// uint32 word of the status block that counts fallback queries
constexpr uint32_t kStatusFallbackWord = 10;
WorkspaceLayout workspace_layout(const genie_index *ix, uint32_t n_queries, uint32_t k);
WorkspaceLayout workspace_layout_tiles(uint64_t n_tiles, uint32_t n_queries, uint32_t k);

// Counter width and table sizes picked for one search call.
struct SearchShape {
    int bits = 0;          // bits per packed counter
    uint32_t ht_log2 = 0;  // hash-table slots = 1 << ht_log2
    size_t lds_bytes = 0;  // dynamic LDS of the scan kernel (the counters are static)
};
int search_shape(uint32_t max_items, uint32_t k, int threads, uint32_t tile_log2,
                 SearchShape *out, uint32_t ht_log2_cap = 0, bool two_tables = false);

int launch_search(const genie_index *ix, const uint64_t *d_q_offsets, const genie_item *d_items,
                  uint64_t n_items, uint32_t n_queries, uint32_t max_items, uint32_t k, uint32_t *d_out_ids,
                  uint32_t *d_out_counts, uint32_t *d_full_counts, void *d_workspace,
                  size_t workspace_bytes, hipStream_t stream, const float *d_gate = nullptr,
                  float gate_delta = 0.0f, const uint32_t *d_rows = nullptr,
                  bool spq = false);

// Multiple loadings: device arrays of one index part (in a streaming slot),
// scanned into columns [tile_off, tile_off + n_tiles) of candidate rows of
// tiles_total tiles, with object ids offset by id_base; one merge over all
// columns afterwards.
struct IndexView {
    const uint16_t *post = nullptr;
    const uint64_t *tile_base = nullptr;
    const uint8_t *tix = nullptr;   // Position Map, as in genie_index
    bool map_compact = false;
    uint64_t n = 0, nkeys = 0;
    uint32_t d = 0, V = 0, n_tiles = 0, tile_log2 = 0;
    int scan_threads = kScanThreadsDefault, scan_unroll = kScanUnrollDefault;
};
int launch_clear_status(void *d_workspace, hipStream_t stream);
int launch_part_scan(const IndexView &v, uint64_t id_base, uint32_t tile_off,
                     uint32_t tiles_total, const uint64_t *d_q_offsets, const genie_item *d_items,
                     uint64_t n_items, uint32_t n_queries, uint32_t max_items, uint32_t k,
                     void *d_workspace, hipStream_t stream);
int launch_part_merge(uint64_t n_total, uint32_t tiles_total, uint32_t n_queries, uint32_t k,
                      void *d_workspace, uint32_t *d_out_ids, uint32_t *d_out_counts,
                      hipStream_t stream);

// Device address of this device's held workspace of
// GENIE_NOALLOC_WORKSPACE_BYTES (search.hip); `device` must be current on the
// first call for it.  Allocates nothing.
int noalloc_workspace(int device, void **out);

// Opt-in kernel timing (timing.cpp): begin returns an event handle or null.
void *timing_begin(hipStream_t st);
void timing_end(void *start, hipStream_t st, int kind);

}  // namespace genie
