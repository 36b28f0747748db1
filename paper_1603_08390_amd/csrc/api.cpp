// Host side of libgenie: error reporting, index build (Section 3.2), the
// synchronous search wrapper and argument checks of the C-ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "internal.h"

namespace genie {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

int hip_fail(hipError_t e, const char *what) {
    set_error("%s failed: %s", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? GENIE_ENOMEM : GENIE_EDEVICE;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

WorkspaceLayout workspace_layout(const genie_index *ix, uint32_t n_queries, uint32_t k) {
    return workspace_layout_tiles(ix->n_tiles, n_queries, k);
}

WorkspaceLayout workspace_layout_tiles(uint64_t n_tiles, uint32_t n_queries, uint32_t k) {
    WorkspaceLayout L;
    uint64_t pairs = (uint64_t)n_queries * n_tiles;
    L.status = 0;
    L.tile_kth = 256;
    L.cand = align256(L.tile_kth + pairs * sizeof(uint32_t));
    L.pair_stats = align256(L.cand + pairs * (uint64_t)k * sizeof(uint64_t));
    L.fb_list = align256(L.pair_stats + pairs * 4 * sizeof(uint32_t));
    L.total = align256(L.fb_list + (uint64_t)n_queries * sizeof(uint32_t));
    return L;
}

int search_shape(uint32_t max_items, uint32_t k, int threads, uint32_t tile_log2,
                 SearchShape *out, uint32_t ht_log2_cap, bool two_tables) {
    // Counter width b: counts reach at most max_items; one more code (all
    // ones) marks an object already emitted during selection.
    static const int widths[] = {4, 8, 16};
    int bits = 0;
    for (int b : widths)
        if ((uint64_t)max_items + 2 <= (1ull << b)) {
            bits = b;
            break;
        }
    if (!bits) {
        set_error("max_items %u too large", max_items);
        return GENIE_ERANGE;
    }
    // Hash table: live entries stay below about 2k (Theorem 3.1 with expiry
    // of entries under AT-1); 4k slots keep probe sequences short.
    uint32_t lg = 6;
    while ((1u << lg) < 4u * k)
        lg++;
    if (ht_log2_cap)   // a smaller table set on the index (overflow handling, tests)
        lg = std::min(lg, ht_log2_cap);
    const uint32_t cpw = 32 / bits;
    // static part: the Bitmap Counter (a counter for every local id and the
    // padding id) and one word of the persistent schedule
    const size_t bc_words = (size_t(1) << tile_log2) / cpw + 1;
    // dynamic part: misc, HT, ZA, run table (two for the persistent
    // schedule, which prepares the next pair's while counting), gate queues
    size_t words = 32 + (1u << lg) + (max_items + 2) + (two_tables ? 2 : 1) * (2ull * max_items + 1) +
                   (size_t)(threads / 64) * kGateQueue;
    out->bits = bits;
    out->ht_log2 = lg;
    out->lds_bytes = words * 4;
    if ((bc_words + words) * 4 > kMaxLdsBytes) {
        set_error("search needs %zu bytes of LDS (k=%u, max_items=%u); limit %zu",
                  (bc_words + words) * 4, k, max_items, kMaxLdsBytes);
        return GENIE_ERANGE;
    }
    return GENIE_OK;
}

}  // namespace genie

using namespace genie;

extern "C" const char *genie_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------
// index build
// ---------------------------------------------------------------------------

extern "C" int genie_build_index(const uint32_t *values, uint64_t n, uint32_t d, uint32_t V,
                                 genie_index **out) {
    return genie_build_index_tiled(values, n, d, V, kTileLog2Default, out);
}

namespace genie {

// Permutes the len ids of one run that starts at element `start` of its
// tile so that element j holds, where the run allows, an id whose 8-bit
// counter word (id / 4) falls in LDS bank ((start + j) / 2) mod 64; when the
// run has no id left for that bank, the next bank that has one is taken.
static void bank_order(uint16_t *run, uint32_t start, uint32_t len,
                       std::vector<uint16_t> (&bucket)[64]) {
    if (len < 4)
        return;
    for (auto &v : bucket)
        v.clear();
    for (uint32_t j = 0; j < len; j++)
        bucket[(run[j] >> 2) & 63].push_back(run[j]);
    for (uint32_t j = 0; j < len; j++) {
        uint32_t g = ((start + j) >> 1) & 63;
        while (bucket[g].empty())
            g = (g + 1) & 63;
        run[j] = bucket[g].back();
        bucket[g].pop_back();
    }
}

// Shared by both index forms: keys_of(o, emit) calls emit(key) once for
// every keyword of object o and returns false if a keyword is out of range.
template <class KeysOf>
static int build_host_index_impl(uint64_t n, uint32_t d, uint32_t V, uint64_t nkeys,
                                 uint64_t npost, uint32_t tile_log2, const KeysOf &keys_of,
                                 HostIndex *h) {
    if (tile_log2 != 15 && tile_log2 != 16) {
        set_error("tile_log2 must be 15 or 16 (got %u)", tile_log2);
        return GENIE_EINVAL;
    }
    const uint32_t kTile = tile_objects_of(tile_log2);
    const uint16_t kSentinel = (uint16_t)kTile;
    const uint32_t T = (uint32_t)((n + kTile - 1) / kTile);

    // Per tile: run length of every keyword (counting sort), each run padded
    // to an even number of elements with the sentinel id kSentinel so that
    // runs start and end on dword boundaries.  toff = padded offsets, tpad =
    // number of padded runs before each keyword (to recover real lengths).
    std::vector<uint32_t> &toff = h->toff, &tpad = h->tpad;
    toff.assign((uint64_t)T * (nkeys + 1), 0u);
    tpad.assign((uint64_t)T * (nkeys + 1), 0u);
    std::vector<uint64_t> tile_size(T);
    std::vector<uint64_t> &tile_base = h->tile_base;
    tile_base.assign(T + 1, 0);
    std::atomic<int> bad{0}, overflow{0}, nomem{0};
    // a thread that cannot allocate reports it instead of ending the process
    auto guarded = [&](const auto &body) {
        return [&nomem, &body]() {
            try {
                body();
            } catch (const std::bad_alloc &) {
                nomem.store(1);
            }
        };
    };
    std::atomic<uint32_t> next{0};
    auto count_tiles = [&]() {
        for (;;) {
            uint32_t t = next.fetch_add(1);
            if (t >= T)
                break;
            uint64_t o0 = (uint64_t)t * kTile, o1 = std::min<uint64_t>(o0 + kTile, n);
            uint32_t *row = &toff[(uint64_t)t * (nkeys + 1)];
            uint32_t *prow = &tpad[(uint64_t)t * (nkeys + 1)];
            for (uint64_t o = o0; o < o1; o++)
                if (!keys_of(o, [&](uint64_t key) { row[key + 1]++; })) {
                    bad.store(1);
                    return;
                }
            uint64_t off = 0;
            uint32_t pads = 0;
            row[0] = 0;
            prow[0] = 0;
            for (uint64_t key = 0; key < nkeys; key++) {
                uint32_t len = row[key + 1];
                off += len + (len & 1u);
                pads += len & 1u;
                row[key + 1] = (uint32_t)off;
                prow[key + 1] = pads;
            }
            // the scan addresses a tile's postings by a 32-bit byte offset
            // (2 bytes per element): fewer than 2^31 elements per tile
            if (off + 2 * kSentinelDwords >= (1ull << 31))
                overflow.store(1);
            tile_size[t] = off + 2 * kSentinelDwords;   // trailing all-sentinel dwords
        }
    };
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    nth = std::min<unsigned>(nth, T);
    {
        std::vector<std::thread> pool;
        for (unsigned i = 0; i < nth; i++)
            pool.emplace_back(guarded(count_tiles));
        for (auto &th : pool)
            th.join();
    }
    if (nomem.load()) {
        set_error("host allocation failed while building the index");
        return GENIE_ENOMEM;
    }
    if (bad.load()) {
        set_error("a keyword is out of range (n_buckets %u, keywords %llu)", V,
                  (unsigned long long)nkeys);
        return GENIE_EINVAL;
    }
    if (overflow.load()) {
        set_error("a tile holds 2^31 or more postings (32-bit byte offsets in the scan)");
        return GENIE_EINVAL;
    }
    tile_base[0] = 0;
    for (uint32_t t = 0; t < T; t++)
        tile_base[t + 1] = tile_base[t] + tile_size[t];
    // postings per keyword over all tiles, as a prefix (query features)
    std::vector<uint64_t> &kcum = h->kcum;
    kcum.assign(nkeys + 1, 0);
    for (uint32_t t = 0; t < T; t++) {
        const uint32_t *row = &toff[(uint64_t)t * (nkeys + 1)];
        const uint32_t *prow = &tpad[(uint64_t)t * (nkeys + 1)];
        for (uint64_t key = 0; key < nkeys; key++)
            kcum[key + 1] += (row[key + 1] - row[key]) - (prow[key + 1] - prow[key]);
    }
    for (uint64_t key = 0; key < nkeys; key++)
        kcum[key + 1] += kcum[key];
    const uint64_t stored = tile_base[T];
    std::vector<uint16_t> &post = h->post;
    post.assign(stored, kSentinel);
    next.store(0);
    auto fill_tiles = [&]() {
        std::vector<uint32_t> fill(nkeys);
        std::vector<uint16_t> bucket[64];
        for (;;) {
            uint32_t t = next.fetch_add(1);
            if (t >= T)
                break;
            uint64_t o0 = (uint64_t)t * kTile, o1 = std::min<uint64_t>(o0 + kTile, n);
            std::memcpy(fill.data(), &toff[(uint64_t)t * (nkeys + 1)], nkeys * sizeof(uint32_t));
            uint16_t *dst = &post[tile_base[t]];
            // objects in ascending id order: every run ascends
            for (uint64_t o = o0; o < o1; o++)
                keys_of(o, [&](uint64_t key) { dst[fill[key]++] = (uint16_t)(o - o0); });
            // Bank order: the order inside a run does not change any count, so
            // each run is permuted such that the id at element j, which the
            // scan reads in dword (start + j) / 2 by lane (start + j) / 2 mod
            // 64 of a wave, has its 8-bit counter word in LDS bank
            // (start + j) / 2 mod 64 when the run holds such an id: the 64
            // atomics of one wave instruction then tend to hit 64 different
            // banks.  (8-bit counters are the common width; other widths get
            // an order as good as any.)
            for (uint64_t key = 0; key < nkeys; key++) {
                const uint32_t b = toff[(uint64_t)t * (nkeys + 1) + key];
                const uint32_t e = toff[(uint64_t)t * (nkeys + 1) + key + 1];
                const uint32_t pads = tpad[(uint64_t)t * (nkeys + 1) + key + 1] -
                                      tpad[(uint64_t)t * (nkeys + 1) + key];
                bank_order(dst + b, b, (e - b) - pads, bucket);
            }
        }
    };
    {
        std::vector<std::thread> pool;
        for (unsigned i = 0; i < nth; i++)
            pool.emplace_back(guarded(fill_tiles));
        for (auto &th : pool)
            th.join();
    }
    if (nomem.load()) {
        set_error("host allocation failed while building the index");
        return GENIE_ENOMEM;
    }
    h->n = n;
    h->d = d;
    h->V = V;
    h->n_tiles = T;
    h->tile_log2 = tile_log2;
    h->nkeys = nkeys;
    h->n_postings = npost;
    return GENIE_OK;
}

int build_host_index(const uint32_t *values, uint64_t n, uint32_t d, uint32_t V,
                     uint32_t tile_log2, HostIndex *h) {
    if (!values) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    if (n == 0 || n >= 0xFFFFFFFFull || d == 0 || V == 0 || (uint64_t)d * V >= 0xFFFFFFFFull) {
        set_error("bad sizes n=%llu d=%u V=%u", (unsigned long long)n, d, V);
        return GENIE_EINVAL;
    }
    const uint64_t nkeys = (uint64_t)d * V;
    auto keys_of = [&](uint64_t o, const auto &emit) {
        for (uint32_t j = 0; j < d; j++) {
            const uint32_t v = values[o * d + j];
            if (v >= V)
                return false;
            emit((uint64_t)j * V + v);
        }
        return true;
    };
    return build_host_index_impl(n, d, V, nkeys, n * d, tile_log2, keys_of, h);
}

int build_host_index_sets(const uint64_t *obj_offsets, const uint32_t *keys, uint64_t n,
                          uint32_t n_keys, uint32_t tile_log2, HostIndex *h) {
    if (!obj_offsets || (!keys && n && obj_offsets[n] != obj_offsets[0])) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    if (n == 0 || n >= 0xFFFFFFFFull || n_keys == 0 || n_keys == 0xFFFFFFFFu) {
        set_error("bad sizes n=%llu n_keys=%u", (unsigned long long)n, n_keys);
        return GENIE_EINVAL;
    }
    for (uint64_t o = 0; o < n; o++)
        if (obj_offsets[o + 1] < obj_offsets[o]) {
            set_error("object offsets decrease at object %llu", (unsigned long long)o);
            return GENIE_EINVAL;
        }
    auto keys_of = [&](uint64_t o, const auto &emit) {
        for (uint64_t i = obj_offsets[o]; i < obj_offsets[o + 1]; i++) {
            if (keys[i] >= n_keys)
                return false;
            emit((uint64_t)keys[i]);
        }
        return true;
    };
    int rc = build_host_index_impl(n, 1, n_keys, n_keys, obj_offsets[n] - obj_offsets[0],
                                   tile_log2, keys_of, h);
    if (rc == GENIE_OK)
        h->key_sets = true;
    return rc;
}

}  // namespace genie

namespace genie {

void interleave_offsets(const HostIndex &h, uint32_t *dst) {
    const uint64_t m = h.toff.size();
    for (uint64_t i = 0; i < m; i++) {
        dst[2 * i] = h.toff[i];
        dst[2 * i + 1] = h.tpad[i];
    }
}

void write_offsets(const HostIndex &h, uint8_t *dst) {
    if (use_compact_map(h))
        compact_offsets(h, dst);
    else
        interleave_offsets(h, reinterpret_cast<uint32_t *>(dst));
}

void compact_offsets(const HostIndex &h, uint8_t *dst) {
    const uint64_t T = h.n_tiles, K = h.nkeys, G = map_groups(K);
    uint32_t *ck = reinterpret_cast<uint32_t *>(dst);
    uint16_t *ln = reinterpret_cast<uint16_t *>(dst + map_ck_bytes(T, K));
    std::memset(dst, 0, map_bytes(T, K));
    for (uint64_t t = 0; t < T; t++) {
        const uint32_t *row = &h.toff[t * (K + 1)];
        const uint32_t *prow = &h.tpad[t * (K + 1)];
        for (uint64_t g = 0; g < G; g++) {
            const uint64_t k0 = g * kMapGroup;   // <= K
            ck[2 * (t * G + g)] = row[k0];
            ck[2 * (t * G + g) + 1] = prow[k0];
            for (uint64_t r = 0; r < kMapGroup && k0 + r < K; r++) {
                const uint64_t key = k0 + r;
                ln[(t * G + g) * kMapGroup + r] =
                    (uint16_t)((row[key + 1] - row[key]) - (prow[key + 1] - prow[key]));
            }
        }
    }
}

int upload_host_index(const HostIndex &h, genie_index **out) {
    const uint32_t T = h.n_tiles;
    genie_index *ix = new (std::nothrow) genie_index;
    if (!ix) {
        set_error("host allocation failed");
        return GENIE_ENOMEM;
    }
    ix->n = h.n;
    ix->d = h.d;
    ix->V = h.V;
    ix->n_tiles = T;
    ix->tile_log2 = h.tile_log2;
    ix->tile_objects = tile_objects_of(h.tile_log2);
    ix->nkeys = h.nkeys;
    ix->n_postings = h.n_postings;
    ix->stored_postings = h.tile_base[T];
    ix->key_sets = h.key_sets;
    hipError_t e = hipGetDevice(&ix->device);
    size_t bp = h.post.size() * sizeof(uint16_t), bb = h.tile_base.size() * sizeof(uint64_t),
           bt = device_map_bytes(h), bk = h.kcum.size() * sizeof(uint64_t);
    ix->map_compact = use_compact_map(h);
    ix->map_bytes = bt;
    if (e == hipSuccess) e = hipMalloc((void **)&ix->post, bp);
    if (e == hipSuccess) e = hipMalloc((void **)&ix->tile_base, bb);
    if (e == hipSuccess) e = hipMalloc((void **)&ix->tix, bt);
    if (e == hipSuccess) e = hipMalloc((void **)&ix->kcum, bk);
    if (e == hipSuccess) e = hipMemcpy(ix->kcum, h.kcum.data(), bk, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ix->post, h.post.data(), bp, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ix->tile_base, h.tile_base.data(), bb, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        std::vector<uint8_t> tix;
        try {
            tix.resize(bt);
        } catch (const std::bad_alloc &) {
            set_error("out of host memory for the index offsets");
            genie_free_index(ix);
            return GENIE_ENOMEM;
        }
        write_offsets(h, tix.data());
        e = hipMemcpy(ix->tix, tix.data(), bt, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        int rc = hip_fail(e, "index upload");
        genie_free_index(ix);
        return rc;
    }
    ix->device_bytes = bp + bb + bt + bk;
    *out = ix;
    return GENIE_OK;
}

}  // namespace genie

extern "C" int genie_build_index_tiled(const uint32_t *values, uint64_t n, uint32_t d, uint32_t V,
                                       uint32_t tile_log2, genie_index **out) {
    clear_error();
    if (!values || !out) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    *out = nullptr;
    try {
        HostIndex h;
        int rc = build_host_index(values, n, d, V, tile_log2, &h);
        return rc ? rc : upload_host_index(h, out);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed while building the index");
        return GENIE_ENOMEM;
    }
}

extern "C" int genie_build_index_sets(const uint64_t *obj_offsets, const uint32_t *keys,
                                      uint64_t n, uint32_t n_keys, uint32_t tile_log2,
                                      genie_index **out) {
    clear_error();
    if (!obj_offsets || !out) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    *out = nullptr;
    try {
        HostIndex h;
        int rc = build_host_index_sets(obj_offsets, keys, n, n_keys, tile_log2, &h);
        return rc ? rc : upload_host_index(h, out);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed while building the index");
        return GENIE_ENOMEM;
    }
}

extern "C" void genie_free_index(genie_index *ix) {
    if (!ix)
        return;
    int cur = 0;
    bool sw = hipGetDevice(&cur) == hipSuccess && cur != ix->device;
    if (sw)
        (void)hipSetDevice(ix->device);
    if (ix->post) (void)hipFree(ix->post);
    if (ix->tile_base) (void)hipFree(ix->tile_base);
    if (ix->tix) (void)hipFree(ix->tix);
    if (ix->kcum) (void)hipFree(ix->kcum);
    if (sw)
        (void)hipSetDevice(cur);
    delete ix;
}

extern "C" int genie_index_set_scan_shape(genie_index *ix, uint32_t threads, uint32_t unroll) {
    clear_error();
    if (!ix || !((threads == 512 || threads == 1024) && (unroll == 4 || unroll == 8))) {
        set_error("scan shape %u x %u not available (threads 512|1024, unroll 4|8)", threads,
                  unroll);
        return GENIE_EINVAL;
    }
    ix->scan_threads = (int)threads;
    ix->scan_unroll = (int)unroll;
    return GENIE_OK;
}

extern "C" int genie_index_set_scan_schedule(genie_index *ix, uint32_t persistent) {
    clear_error();
    if (!ix || persistent > 2) {
        set_error("scan schedule must be 0 (one workgroup per pair), 1 (persistent) or 2 "
                  "(persistent for calls of at least 1,024 pairs)");
        return GENIE_EINVAL;
    }
    ix->scan_persistent = (int)persistent;
    return GENIE_OK;
}

extern "C" int genie_index_set_hash_slots(genie_index *ix, uint32_t log2_slots) {
    clear_error();
    if (!ix || log2_slots > 16) {
        set_error("hash table slots must be 2^1 .. 2^16, or 0 for the default");
        return GENIE_EINVAL;
    }
    ix->ht_log2_cap = log2_slots;
    return GENIE_OK;
}

extern "C" int genie_index_info_get(const genie_index *ix, genie_index_info *out) {
    clear_error();
    if (!ix || !out) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    out->n_objects = ix->n;
    out->n_dims = ix->d;
    out->n_buckets = ix->V;
    out->n_tiles = ix->n_tiles;
    out->tile_objects = ix->tile_objects;
    out->n_postings = ix->n_postings;
    out->device_bytes = ix->device_bytes;
    out->scan_threads = (uint32_t)ix->scan_threads;
    out->scan_unroll = (uint32_t)ix->scan_unroll;
    out->scan_persistent = (uint32_t)ix->scan_persistent;
    out->map_compact = ix->map_compact ? 1u : 0u;
    out->map_bytes = ix->map_bytes;
    return GENIE_OK;
}

// ---------------------------------------------------------------------------
// search
// ---------------------------------------------------------------------------

extern "C" size_t genie_search_workspace_size(const genie_index *ix, uint32_t n_queries,
                                              uint32_t k) {
    if (!ix || k == 0 || k > GENIE_MAX_K)
        return 0;
    return workspace_layout(ix, n_queries, k).total;
}

static int check_common(const genie_index *ix, uint32_t n_queries, uint32_t k) {
    if (!ix) {
        set_error("null index");
        return GENIE_EINVAL;
    }
    if (k == 0 || k > GENIE_MAX_K) {
        set_error("k=%u outside 1..%u", k, GENIE_MAX_K);
        return GENIE_EINVAL;
    }
    (void)n_queries;
    return GENIE_OK;
}

namespace {
int check_async(const genie_index *ix, const uint64_t *d_q_offsets, const genie_item *d_items,
                uint32_t n_queries, uint32_t max_items, uint32_t k, uint32_t *d_out_ids,
                uint32_t *d_out_counts, void *d_workspace) {
    int rc = check_common(ix, n_queries, k);
    if (rc)
        return rc;
    if (n_queries == 0)
        return GENIE_OK;
    if (!d_q_offsets || !d_items || !d_out_ids || !d_out_counts || !d_workspace) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    if (max_items > GENIE_MAX_ITEMS) {
        set_error("max_items=%u above %u", max_items, GENIE_MAX_ITEMS);
        return GENIE_ERANGE;
    }
    if (((uintptr_t)d_workspace & 255) != 0) {
        set_error("workspace must be 256-byte aligned");
        return GENIE_EINVAL;
    }
    return GENIE_OK;
}

int check_gate(const float *d_gate, float gate_delta) {
    if (!d_gate) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    if (!(gate_delta >= 0.0f)) {
        set_error("gate_delta must be >= 0");
        return GENIE_EINVAL;
    }
    return GENIE_OK;
}
}  // namespace

extern "C" int genie_search_async(const genie_index *ix, const uint64_t *d_q_offsets,
                                  const genie_item *d_items, uint64_t n_items,
                                  uint32_t n_queries, uint32_t max_items, uint32_t k, uint32_t *d_out_ids,
                                  uint32_t *d_out_counts, void *d_workspace,
                                  size_t workspace_bytes, void *stream) {
    clear_error();
    int rc = check_async(ix, d_q_offsets, d_items, n_queries, max_items, k, d_out_ids,
                         d_out_counts, d_workspace);
    if (rc || n_queries == 0)
        return rc;
    return launch_search(ix, d_q_offsets, d_items, n_items, n_queries, max_items, k, d_out_ids,
                         d_out_counts, nullptr, d_workspace, workspace_bytes,
                         (hipStream_t)stream);
}

extern "C" int genie_search_noalloc_async(const genie_index *ix, const uint64_t *d_q_offsets,
                                          const genie_item *d_items, uint64_t n_items,
                                          uint32_t n_queries, uint32_t max_items, uint32_t k,
                                          uint32_t *d_out_ids, uint32_t *d_out_counts,
                                          void *stream) {
    clear_error();
    int rc = check_common(ix, n_queries, k);
    if (rc || n_queries == 0)
        return rc;
    const size_t need = workspace_layout(ix, n_queries, k).total;
    if (need > GENIE_NOALLOC_WORKSPACE_BYTES) {
        set_error("search needs %zu bytes of workspace; the held workspace has %u "
                  "(fewer queries per call, or genie_search_async with a caller buffer)",
                  need, GENIE_NOALLOC_WORKSPACE_BYTES);
        return GENIE_ERANGE;
    }
    int dev = -1;
    GENIE_HIP(hipGetDevice(&dev));
    if (dev != ix->device) {
        set_error("index lives on device %d but device %d is current", ix->device, dev);
        return GENIE_EINVAL;
    }
    void *ws = nullptr;
    if ((rc = noalloc_workspace(dev, &ws)))
        return rc;
    rc = check_async(ix, d_q_offsets, d_items, n_queries, max_items, k, d_out_ids, d_out_counts,
                     ws);
    if (rc)
        return rc;
    return launch_search(ix, d_q_offsets, d_items, n_items, n_queries, max_items, k, d_out_ids,
                         d_out_counts, nullptr, ws, GENIE_NOALLOC_WORKSPACE_BYTES,
                         (hipStream_t)stream);
}

extern "C" int genie_search_gated_async(const genie_index *ix, const uint64_t *d_q_offsets,
                                        const genie_item *d_items, uint64_t n_items,
                                        uint32_t n_queries, uint32_t max_items, uint32_t k,
                                        const float *d_gate, float gate_delta,
                                        uint32_t *d_out_ids, uint32_t *d_out_counts,
                                        void *d_workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    int rc = check_async(ix, d_q_offsets, d_items, n_queries, max_items, k, d_out_ids,
                         d_out_counts, d_workspace);
    if (rc || n_queries == 0)
        return rc;
    if ((rc = check_gate(d_gate, gate_delta)))
        return rc;
    return launch_search(ix, d_q_offsets, d_items, n_items, n_queries, max_items, k, d_out_ids,
                         d_out_counts, nullptr, d_workspace, workspace_bytes,
                         (hipStream_t)stream, d_gate, gate_delta);
}

extern "C" int genie_search_spq_async(const genie_index *ix, const uint64_t *d_q_offsets,
                                      const genie_item *d_items, uint64_t n_items,
                                      uint32_t n_queries, uint32_t max_items, uint32_t k,
                                      uint32_t *d_out_ids, uint32_t *d_out_counts,
                                      void *d_workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    int rc = check_async(ix, d_q_offsets, d_items, n_queries, max_items, k, d_out_ids,
                         d_out_counts, d_workspace);
    if (rc || n_queries == 0)
        return rc;
    return launch_search(ix, d_q_offsets, d_items, n_items, n_queries, max_items, k, d_out_ids,
                         d_out_counts, nullptr, d_workspace, workspace_bytes,
                         (hipStream_t)stream, nullptr, 0.0f, nullptr, true);
}

extern "C" int genie_search_rows_async(const genie_index *ix, const uint64_t *d_q_offsets,
                                       const genie_item *d_items, uint64_t n_items,
                                       uint32_t capacity, const uint32_t *d_rows,
                                       uint32_t max_items, uint32_t k, const float *d_gate,
                                       float gate_delta, uint32_t *d_out_ids,
                                       uint32_t *d_out_counts, void *d_workspace,
                                       size_t workspace_bytes, void *stream) {
    clear_error();
    int rc = check_async(ix, d_q_offsets, d_items, capacity, max_items, k, d_out_ids,
                         d_out_counts, d_workspace);
    if (rc || capacity == 0)
        return rc;
    if (!d_rows) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    if (d_gate && (rc = check_gate(d_gate, gate_delta)))
        return rc;
    return launch_search(ix, d_q_offsets, d_items, n_items, capacity, max_items, k, d_out_ids,
                         d_out_counts, nullptr, d_workspace, workspace_bytes,
                         (hipStream_t)stream, d_gate, gate_delta, d_rows);
}

extern "C" int genie_match_count_async(const genie_index *ix, const uint64_t *d_q_offsets,
                                       const genie_item *d_items, uint64_t n_items,
                                       uint32_t n_queries,
                                       uint32_t max_items, uint32_t *d_out_counts,
                                       void *d_workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    int rc = check_common(ix, n_queries, 1);
    if (rc)
        return rc;
    if (n_queries == 0)
        return GENIE_OK;
    if (!d_q_offsets || !d_items || !d_out_counts || !d_workspace) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    if (max_items > GENIE_MAX_ITEMS) {
        set_error("max_items=%u above %u", max_items, GENIE_MAX_ITEMS);
        return GENIE_ERANGE;
    }
    if (((uintptr_t)d_workspace & 255) != 0) {
        set_error("workspace must be 256-byte aligned");
        return GENIE_EINVAL;
    }
    return launch_search(ix, d_q_offsets, d_items, n_items, n_queries, max_items, 1, nullptr,
                         nullptr, d_out_counts, d_workspace, workspace_bytes,
                         (hipStream_t)stream);
}

namespace {
// Device buffers of one synchronous call, freed on every exit path.
struct DeviceBuffers {
    std::vector<void *> ptrs;
    ~DeviceBuffers() {
        for (void *p : ptrs)
            (void)hipFree(p);
    }
    hipError_t alloc(void **p, size_t bytes) {
        hipError_t e = hipMalloc(p, bytes ? bytes : 256);
        if (e == hipSuccess)
            ptrs.push_back(*p);
        return e;
    }
};
}  // namespace

extern "C" int genie_search(const genie_index *ix, const uint64_t *q_offsets,
                            const genie_item *items, uint32_t n_queries, uint32_t k,
                            uint32_t *out_ids, uint32_t *out_counts) {
    clear_error();
    int rc = check_common(ix, n_queries, k);
    if (rc)
        return rc;
    if (n_queries == 0)
        return GENIE_OK;
    if (!q_offsets || !out_ids || !out_counts) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    if (q_offsets[0] != 0) {
        set_error("q_offsets[0] must be 0");
        return GENIE_EINVAL;
    }
    uint32_t max_items = 0;
    for (uint32_t q = 0; q < n_queries; q++) {
        if (q_offsets[q + 1] < q_offsets[q]) {
            set_error("q_offsets decreases at query %u", q);
            return GENIE_EINVAL;
        }
        uint64_t s = q_offsets[q + 1] - q_offsets[q];
        if (s > GENIE_MAX_ITEMS) {
            set_error("query %u has %llu items (limit %u)", q, (unsigned long long)s,
                      GENIE_MAX_ITEMS);
            return GENIE_ERANGE;
        }
        max_items = std::max<uint32_t>(max_items, (uint32_t)s);
    }
    const uint64_t n_items = q_offsets[n_queries];
    if (n_items && !items) {
        set_error("null items");
        return GENIE_EINVAL;
    }
    for (uint64_t i = 0; i < n_items; i++) {
        if (items[i].dim >= ix->d) {
            set_error("item %llu names dim %u >= n_dims %u", (unsigned long long)i, items[i].dim,
                      ix->d);
            return GENIE_EINVAL;
        }
        if (ix->key_sets && items[i].lo < std::min(items[i].hi, ix->V - 1)) {
            set_error("item %llu spans keywords %u..%u of a keyword-set index (one keyword per "
                      "item)", (unsigned long long)i, items[i].lo, items[i].hi);
            return GENIE_EINVAL;
        }
    }
    SearchShape shape;
    rc = search_shape(max_items, k, ix->scan_threads, ix->tile_log2, &shape);
    if (rc)
        return rc;

    int cur = 0;
    GENIE_HIP(hipGetDevice(&cur));
    if (cur != ix->device)
        GENIE_HIP(hipSetDevice(ix->device));
    struct Restore {
        int dev, cur;
        ~Restore() {
            if (dev != cur)
                (void)hipSetDevice(cur);
        }
    } restore{ix->device, cur};

    DeviceBuffers buf;
    uint64_t *d_off = nullptr;
    genie_item *d_items = nullptr;
    uint32_t *d_ids = nullptr, *d_cts = nullptr;
    void *d_ws = nullptr;
    size_t ws = genie_search_workspace_size(ix, n_queries, k);
    size_t out_bytes = (size_t)n_queries * k * sizeof(uint32_t);
    GENIE_HIP(buf.alloc((void **)&d_off, (n_queries + 1) * sizeof(uint64_t)));
    GENIE_HIP(buf.alloc((void **)&d_items, n_items * sizeof(genie_item)));
    GENIE_HIP(buf.alloc((void **)&d_ids, out_bytes));
    GENIE_HIP(buf.alloc((void **)&d_cts, out_bytes));
    GENIE_HIP(buf.alloc(&d_ws, ws));
    GENIE_HIP(hipMemcpy(d_off, q_offsets, (n_queries + 1) * sizeof(uint64_t),
                        hipMemcpyHostToDevice));
    if (n_items)
        GENIE_HIP(hipMemcpy(d_items, items, n_items * sizeof(genie_item), hipMemcpyHostToDevice));
    rc = launch_search(ix, d_off, d_items, n_items, n_queries, max_items, k, d_ids, d_cts,
                       nullptr, d_ws, ws, nullptr);
    if (rc)
        return rc;
    GENIE_HIP(hipDeviceSynchronize());
    uint32_t status = 0;
    GENIE_HIP(hipMemcpy(&status, d_ws, sizeof status, hipMemcpyDeviceToHost));
    if (status) {
        set_error("device status flags 0x%x", status);
        return (status & GENIE_STATUS_TOO_MANY_ITEMS) ? GENIE_ERANGE : GENIE_EINVAL;
    }
    GENIE_HIP(hipMemcpy(out_ids, d_ids, out_bytes, hipMemcpyDeviceToHost));
    GENIE_HIP(hipMemcpy(out_counts, d_cts, out_bytes, hipMemcpyDeviceToHost));
    return GENIE_OK;
}
