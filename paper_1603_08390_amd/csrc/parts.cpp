// Multiple loadings (Section 3.4): an index too large for the device is cut
// into parts by object range, each built once into pinned host memory.  A
// search streams the parts through two device slots: part p is copied into
// slot p mod 2 on a copy stream while the scan of part p - 1 runs on the
// search stream, and every part's scan writes its tiles' exact top-k lists
// into its own columns of one candidate array, ids offset by the part's
// first object.  One merge over all columns then gives the exact answer:
// the global top-k is inside the union of the tile lists (the order is
// total), which is the paper's merge of the parts' results, done on the
// device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

using namespace genie;

namespace {

struct PartHost {
    uint64_t id_base = 0, n = 0;
    uint32_t n_tiles = 0, tile_off = 0;
    uint64_t nkeys = 0;
    uint16_t *post = nullptr;       // pinned host arrays of the part's index
    uint64_t *tile_base = nullptr;
    uint8_t *tix = nullptr;         // Position Map, as in genie_index
    bool map_compact = false;
    size_t post_bytes = 0, base_bytes = 0, off_bytes = 0;
};

struct Slot {
    uint16_t *post = nullptr;
    uint64_t *tile_base = nullptr;
    uint8_t *tix = nullptr;
    hipEvent_t copied = nullptr, scanned = nullptr;
};

}  // namespace

struct genie_parts {
    uint64_t n = 0;
    uint32_t d = 0, V = 0, tile_log2 = 0, tiles_total = 0;
    uint64_t part_objects = 0;
    std::vector<PartHost> parts;
    Slot slot[2];
    hipStream_t copy_stream = nullptr;
    int device = 0;
    uint64_t host_bytes = 0, device_bytes = 0;
};

namespace {

void free_parts(genie_parts *ps) {
    for (PartHost &p : ps->parts) {
        if (p.post) (void)hipHostFree(p.post);
        if (p.tile_base) (void)hipHostFree(p.tile_base);
        if (p.tix) (void)hipHostFree(p.tix);
    }
    for (Slot &s : ps->slot) {
        if (s.post) (void)hipFree(s.post);
        if (s.tile_base) (void)hipFree(s.tile_base);
        if (s.tix) (void)hipFree(s.tix);
        if (s.copied) (void)hipEventDestroy(s.copied);
        if (s.scanned) (void)hipEventDestroy(s.scanned);
    }
    if (ps->copy_stream) (void)hipStreamDestroy(ps->copy_stream);
    delete ps;
}

}  // namespace

extern "C" int genie_parts_build(const uint32_t *values, uint64_t n, uint32_t d, uint32_t V,
                                 uint64_t part_objects, uint32_t tile_log2, genie_parts **out) {
    clear_error();
    if (!values || !out) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    *out = nullptr;
    if (part_objects == 0 || n == 0 || n >= 0xFFFFFFFFull) {
        set_error("bad sizes n=%llu part_objects=%llu", (unsigned long long)n,
                  (unsigned long long)part_objects);
        return GENIE_EINVAL;
    }
    genie_parts *ps = new (std::nothrow) genie_parts;
    if (!ps) {
        set_error("host allocation failed");
        return GENIE_ENOMEM;
    }
    ps->n = n;
    ps->d = d;
    ps->V = V;
    ps->tile_log2 = tile_log2;
    ps->part_objects = part_objects;
    size_t max_post = 0, max_base = 0, max_off = 0;
    uint32_t tiles = 0;
    hipError_t e = hipGetDevice(&ps->device);
    for (uint64_t o0 = 0; o0 < n && e == hipSuccess; o0 += part_objects) {
        const uint64_t np = std::min<uint64_t>(part_objects, n - o0);
        HostIndex h;
        int rc = build_host_index(values + o0 * d, np, d, V, tile_log2, &h);
        if (rc) {
            free_parts(ps);
            return rc;
        }
        PartHost p;
        p.id_base = o0;
        p.n = np;
        p.n_tiles = h.n_tiles;
        p.tile_off = tiles;
        p.nkeys = h.nkeys;
        p.post_bytes = h.post.size() * sizeof(uint16_t);
        p.base_bytes = h.tile_base.size() * sizeof(uint64_t);
        p.off_bytes = device_map_bytes(h);
        p.map_compact = use_compact_map(h);
        // pinned host copies: the copies to the device run asynchronously
        e = hipHostMalloc((void **)&p.post, p.post_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void **)&p.tile_base, p.base_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void **)&p.tix, p.off_bytes, hipHostMallocDefault);
        ps->parts.push_back(p);
        if (e != hipSuccess)
            break;
        PartHost &q = ps->parts.back();
        std::memcpy(q.post, h.post.data(), q.post_bytes);
        std::memcpy(q.tile_base, h.tile_base.data(), q.base_bytes);
        write_offsets(h, q.tix);
        ps->host_bytes += q.post_bytes + q.base_bytes + q.off_bytes;
        max_post = std::max(max_post, q.post_bytes);
        max_base = std::max(max_base, q.base_bytes);
        max_off = std::max(max_off, q.off_bytes);
        tiles += h.n_tiles;
    }
    ps->tiles_total = tiles;
    for (Slot &s : ps->slot) {
        if (e == hipSuccess) e = hipMalloc((void **)&s.post, max_post);
        if (e == hipSuccess) e = hipMalloc((void **)&s.tile_base, max_base);
        if (e == hipSuccess) e = hipMalloc((void **)&s.tix, max_off);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.copied, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.scanned, hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ps->copy_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        int rc = hip_fail(e, "index parts");
        free_parts(ps);
        return rc;
    }
    ps->device_bytes = 2 * (max_post + max_base + max_off);
    *out = ps;
    return GENIE_OK;
}

extern "C" void genie_parts_free(genie_parts *ps) {
    if (!ps)
        return;
    // wait for the copies and for the scans that read the slots
    (void)hipStreamSynchronize(ps->copy_stream);
    for (Slot &s : ps->slot)
        if (s.scanned)
            (void)hipEventSynchronize(s.scanned);
    free_parts(ps);
}

extern "C" int genie_parts_info_get(const genie_parts *ps, genie_parts_info *out) {
    clear_error();
    if (!ps || !out) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    out->n_objects = ps->n;
    out->n_parts = (uint32_t)ps->parts.size();
    out->tiles_total = ps->tiles_total;
    out->part_objects = ps->part_objects;
    out->host_bytes = ps->host_bytes;
    out->device_bytes = ps->device_bytes;
    return GENIE_OK;
}

extern "C" size_t genie_parts_workspace_size(const genie_parts *ps, uint32_t n_queries,
                                             uint32_t k) {
    if (!ps)
        return 0;
    return workspace_layout_tiles(ps->tiles_total, n_queries, k).total;
}

extern "C" int genie_parts_search_async(genie_parts *ps, const uint64_t *d_q_offsets,
                                        const genie_item *d_items, uint64_t n_items,
                                        uint32_t n_queries, uint32_t max_items, uint32_t k,
                                        uint32_t *d_out_ids, uint32_t *d_out_counts,
                                        void *d_workspace, size_t workspace_bytes,
                                        void *stream) {
    clear_error();
    if (!ps || k == 0 || k > GENIE_MAX_K) {
        set_error("bad arguments (k must be 1..%d)", GENIE_MAX_K);
        return GENIE_EINVAL;
    }
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
    if (((uintptr_t)d_workspace & 255) != 0 ||
        workspace_bytes < workspace_layout_tiles(ps->tiles_total, n_queries, k).total) {
        set_error("workspace too small or not 256-byte aligned");
        return GENIE_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    int rc = launch_clear_status(d_workspace, st);
    if (rc)
        return rc;
    for (size_t i = 0; i < ps->parts.size(); i++) {
        const PartHost &p = ps->parts[i];
        Slot &s = ps->slot[i & 1];
        // the slot is free once the scan that last read it has finished
        GENIE_HIP(hipStreamWaitEvent(ps->copy_stream, s.scanned, 0));
        GENIE_HIP(hipMemcpyAsync(s.post, p.post, p.post_bytes, hipMemcpyHostToDevice,
                                 ps->copy_stream));
        GENIE_HIP(hipMemcpyAsync(s.tile_base, p.tile_base, p.base_bytes, hipMemcpyHostToDevice,
                                 ps->copy_stream));
        GENIE_HIP(hipMemcpyAsync(s.tix, p.tix, p.off_bytes, hipMemcpyHostToDevice,
                                 ps->copy_stream));
        GENIE_HIP(hipEventRecord(s.copied, ps->copy_stream));
        GENIE_HIP(hipStreamWaitEvent(st, s.copied, 0));
        IndexView v;
        v.post = s.post;
        v.tile_base = s.tile_base;
        v.tix = s.tix;
        v.map_compact = p.map_compact;
        v.n = p.n;
        v.nkeys = p.nkeys;
        v.d = ps->d;
        v.V = ps->V;
        v.n_tiles = p.n_tiles;
        v.tile_log2 = ps->tile_log2;
        rc = launch_part_scan(v, p.id_base, p.tile_off, ps->tiles_total, d_q_offsets, d_items,
                              n_items, n_queries, max_items, k, d_workspace, st);
        if (rc)
            return rc;
        GENIE_HIP(hipEventRecord(s.scanned, st));
    }
    return launch_part_merge(ps->n, ps->tiles_total, n_queries, k, d_workspace, d_out_ids,
                             d_out_counts, st);
}
