/*
 * libgenie -- match-count search with a count priority queue on MI355X (gfx950).
 *
 * The method (GENIE, "A Generic Inverted Index Framework for Similarity
 * Search on the GPU"):
 *   - Section 2.1, Definition 2.1: an object is one value per dimension; a
 *     query is a list of items (dim, lo, hi); MC(Q, O) counts the items that
 *     contain O's value on the item's dimension (ranges inclusive, Example
 *     2.1).  The answer is the k objects of largest MC.
 *   - Section 3.2: an inverted index on the GPU, keyword = (dim, value),
 *     postings = ids of the objects holding that keyword.
 *   - Section 3.3: the count priority queue (c-PQ): Bitmap Counter, Gate
 *     (ZipperArray + AuditThreshold, Algorithm 1), Hash Table with a modified
 *     Robin Hood scheme; Theorem 3.1 gives MC_k = AT - 1.
 *   - Section 4.1.2 / 4.2.3: LSH signatures (E2LSH, then a re-hash into D
 *     buckets) turn points into match-count objects for tau-ANN search.
 *
 * Answer order: count descending, then id ascending (the paper breaks ties
 * at the k-th count randomly; a fixed order makes every answer unique and
 * checkable bit for bit).  Row q lists min(k, n) objects over ALL n objects
 * (objects with count 0 included, smallest ids first); slots past n hold
 * (id = UINT32_MAX, count = 0).
 *
 * Conventions for every call:
 *   - Return value: GENIE_OK (0) or a negative GENIE_E* code.  No exception
 *     or abort crosses this interface.  On error, output contents are
 *     unspecified and genie_last_error() describes the failure.
 *   - The caller owns every buffer it passes and keeps it alive for the
 *     call (for *_async calls: until the stream has passed the call).  The
 *     library owns an index from genie_build_index until genie_free_index.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory of the current device (for example a torch tensor's
 *     data_ptr()).  Streams are hipStream_t passed as void*; NULL means the
 *     default (null) stream.
 *   - A const genie_index* may be searched concurrently from several host
 *     threads and streams, each with its own workspace.
 */
#ifndef GENIE_H
#define GENIE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GENIE_OK 0
#define GENIE_EINVAL (-22)   /* bad pointer, size, dimension, k, ... */
#define GENIE_ENOMEM (-12)   /* host or device allocation failed */
#define GENIE_EDEVICE (-5)   /* a HIP call failed */
#define GENIE_ERANGE (-34)   /* a query exceeds the limits below */

/* Limits of one search call. */
#define GENIE_MAX_K 1024          /* results per query */
#define GENIE_MAX_ITEMS 1024      /* items per query (bounds the count) */
#define GENIE_TILE_OBJECTS 65535  /* objects per tile of genie_build_index (16-bit local ids, 0xFFFF reserved) */

/* Device status flags, OR-ed into the first word of a search workspace. */
#define GENIE_STATUS_BAD_DIM 1u       /* an item named dim >= n_dims (treated as empty) */
#define GENIE_STATUS_TOO_MANY_ITEMS 2u /* a query had more items than max_items (row padded) */
#define GENIE_STATUS_BAD_OFFSETS 4u    /* a query's offsets were invalid (row padded) */
#define GENIE_STATUS_RANGE_ON_SET 8u   /* an item on a keyword-set index spanned several keywords (treated as empty) */

typedef struct genie_index genie_index; /* opaque, owned by the library */

/* One query item: the keywords (dim, v) with lo <= v <= hi (Example 2.1).
 * hi is capped at n_buckets-1; lo > hi (after the cap) is an empty item.
 * Several items may name the same dim; each contributes on its own
 * (MC sums over items, Definition 2.1). */
typedef struct {
    uint32_t dim, lo, hi;
} genie_item;

typedef struct {
    uint64_t n_objects;
    uint32_t n_dims;
    uint32_t n_buckets;
    uint32_t n_tiles;          /* ceil(n_objects / tile_objects) */
    uint32_t tile_objects;     /* objects per tile: 2^tile_log2 - 1 */
    uint64_t n_postings;       /* n_objects * n_dims */
    uint64_t device_bytes;     /* device memory held by the index */
    uint32_t scan_threads;     /* scan kernel launch shape in use (see */
    uint32_t scan_unroll;      /* genie_index_set_scan_shape) */
    uint32_t scan_persistent;  /* schedule 0, 1 or 2 (genie_index_set_scan_schedule) */
    uint32_t map_compact;      /* 1: Position Map in the compact form (3 bytes per tile
                                  and keyword, chosen where the 8-byte form would
                                  exceed a quarter of the postings' bytes) */
    uint64_t map_bytes;        /* device bytes of the Position Map */
} genie_index_info;

/*
 * Build the inverted index of Section 3.2 (List Array + Position Map) and
 * upload it to the current device.
 *   values:    host, n_objects * n_dims uint32, row-major (object-major);
 *              values[o*n_dims + j] is object o's value on dim j, which must
 *              be < n_buckets (keyword = (j, value), Section 2.1).
 *   n_objects: 1 .. 2^32 - 1; n_dims >= 1; n_buckets >= 1;
 *              n_dims * n_buckets < 2^32.
 *   out:       receives the new index.
 * Layout on the device: objects are cut into tiles of GENIE_TILE_OBJECTS;
 * postings are stored tile-major, then keyword-major, as 16-bit ids local to
 * the tile in ascending order, so that every keyword list restricted to a
 * tile is one contiguous run and the runs of one dimension are adjacent;
 * each run is padded to an even length with the reserved id 0xFFFF.
 * Errors: GENIE_EINVAL (null pointer, size, value >= n_buckets),
 * GENIE_ENOMEM, GENIE_EDEVICE.
 */
int genie_build_index(const uint32_t *values, uint64_t n_objects, uint32_t n_dims,
                      uint32_t n_buckets, genie_index **out);

/*
 * genie_build_index with tiles of 2^tile_log2 - 1 objects (tile_log2 = 15
 * or 16; 16 is genie_build_index); the reserved padding id is
 * 2^tile_log2 - 1.  A search keeps one counter per id of a tile in LDS, so
 * smaller tiles halve that footprint (16-bit counters: 64 KB instead of
 * 128 KB, which lets two workgroups share a compute unit) at the price of
 * twice the tiles, each with its own per-query overhead and candidate list.
 * Results do not depend on the tiling.  Other arguments and errors as
 * genie_build_index; GENIE_EINVAL for another tile_log2.
 */
int genie_build_index_tiled(const uint32_t *values, uint64_t n_objects, uint32_t n_dims,
                            uint32_t n_buckets, uint32_t tile_log2, genie_index **out);

/* Free an index and its device memory.  NULL is ignored. */
void genie_free_index(genie_index *ix);

/*
 * Launch shape of the scan kernel for searches on this index: threads per
 * workgroup (512 or 1024) and posting dwords each thread loads per step (4
 * or 8); a new index starts at 1024 x 4.  Results do not depend on it;
 * speed does (an autotuner picks it).
 * Not to be changed while a search on the index is being enqueued.
 * Errors: GENIE_EINVAL.
 */
int genie_index_set_scan_shape(genie_index *ix, uint32_t threads, uint32_t unroll);

/*
 * Schedule of the scan kernel for searches on this index.  0: one
 * workgroup per (query, tile) pair, the hardware dispatcher hands pairs to
 * compute units as workgroups finish.  1: persistent
 * workgroups, as many as fit the device at once, each taking pairs from its
 * XCD's slice of the pair list through a device counter and then helping
 * the other slices (Section 3.2.1's load balancing: work goes to whichever
 * workgroup is free); a workgroup claims its next pair and looks up that
 * pair's runs while it still counts the current one.  2 (the default):
 * schedule 1 for calls of at least 1,024 (query, tile) pairs, schedule 0
 * below (a workgroup would count one pair and gain nothing from preparing
 * the next).  Where the second run table of schedule 1 does not fit in LDS,
 * and for genie_search_rows_async (whose rows past the live count would all
 * be claimed), a search runs with schedule 0.
 * Results do not depend on it; speed may (the autotuner picks it).  Not to
 * be changed while a search on the index is being enqueued.
 * Errors: GENIE_EINVAL.
 */
int genie_index_set_scan_schedule(genie_index *ix, uint32_t persistent);

/*
 * Caps the Hash Table of the count priority queue (Section 3.3.2) at
 * 2^log2_slots slots for later searches on this index; 0 restores the
 * default (the smallest power of two >= 4k, at least 64).  The paper sizes
 * the table only as O(k x largest count); a tile whose table runs out of
 * slots flags the overflow and selects its top-k from its exact counters
 * instead, with the same answers (the statistic "tiles whose hash table
 * overflowed" counts such tiles).  For tests of that fallback and for
 * measurement.  log2_slots <= 16.  Errors: GENIE_EINVAL.
 */
int genie_index_set_hash_slots(genie_index *ix, uint32_t log2_slots);

/* Describe an index.  Errors: GENIE_EINVAL. */
int genie_index_info_get(const genie_index *ix, genie_index_info *out);

/*
 * Top-k match-count search (Definition 2.1 scored, c-PQ of Section 3.3
 * selecting), synchronous, host buffers.
 *   q_offsets: host, n_queries+1 uint64; query q owns
 *              items[q_offsets[q] .. q_offsets[q+1]-1]; q_offsets[0] = 0,
 *              non-decreasing.
 *   items:     host, q_offsets[n_queries] items.
 *   k:         1 .. GENIE_MAX_K.  Each query has at most GENIE_MAX_ITEMS items.
 *   out_ids, out_counts: host, n_queries * k uint32 each, row q at q*k.
 * Errors: GENIE_EINVAL (dim >= n_dims, k out of range, bad offsets, null
 * pointer with n_queries > 0), GENIE_ERANGE (too many items), GENIE_ENOMEM,
 * GENIE_EDEVICE.  n_queries = 0 is a no-op.
 */
int genie_search(const genie_index *ix, const uint64_t *q_offsets, const genie_item *items,
                 uint32_t n_queries, uint32_t k, uint32_t *out_ids, uint32_t *out_counts);

/*
 * Bytes of device workspace that genie_search_async needs for n_queries
 * queries at this k (0 on bad arguments).
 */
size_t genie_search_workspace_size(const genie_index *ix, uint32_t n_queries, uint32_t k);

/*
 * Same search, enqueued on a stream, all buffers on the device.
 *   d_q_offsets, d_items, d_out_ids, d_out_counts: as in genie_search, device.
 *   n_items:     number of items in d_items.  A query whose offsets are
 *                decreasing or reach past n_items is answered with padding
 *                and flags GENIE_STATUS_BAD_OFFSETS; no item outside
 *                d_items is read.
 *   max_items:   an upper bound on the items of every query in this call
 *                (1 .. GENIE_MAX_ITEMS; it fixes the counter width).  A query
 *                with more items is answered with padding and flags
 *                GENIE_STATUS_TOO_MANY_ITEMS.
 *   d_workspace: device, >= genie_search_workspace_size(ix, n_queries, k)
 *                bytes, 256-byte aligned.  After the stream passes the call,
 *                its first uint32 holds the OR of GENIE_STATUS_* flags, and
 *                the uint64 words at byte offsets 8, 16, 24 and 32 hold:
 *                postings scanned, tiles whose hash table overflowed (answered
 *                exactly from the counters), hash-table insertions, and
 *                increments that passed the gate.  Calls that share a
 *                workspace must be ordered on one stream.
 *   stream:      hipStream_t or NULL.
 * Host-side checks only (k, max_items, pointers); item contents are checked
 * on the device (bad dims flag GENIE_STATUS_BAD_DIM and act as empty items).
 */
int genie_search_async(const genie_index *ix, const uint64_t *d_q_offsets,
                       const genie_item *d_items, uint64_t n_items, uint32_t n_queries,
                       uint32_t max_items,
                       uint32_t k, uint32_t *d_out_ids, uint32_t *d_out_counts,
                       void *d_workspace, size_t workspace_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * genie_search_async with its workspace taken from a device array that the
 * library holds instead of a caller buffer.  The array is
 * GENIE_NOALLOC_WORKSPACE_BYTES on every GPU the library runs on, one copy
 * per GPU, kept until the process ends; the call allocates nothing.
 *   Arguments, results and errors as genie_search_async without the
 *   workspace.  The index's GPU must be the current device.
 *   Limit: genie_search_workspace_size(ix, n_queries, k) must not exceed
 *   GENIE_NOALLOC_WORKSPACE_BYTES, else GENIE_ERANGE and nothing is
 *   enqueued (e.g. 1,024 queries at k = 100 over 16 tiles take 13.2 MB).
 *   Every call on one GPU shares that GPU's array, which keeps the last
 *   call's contents (each call clears what must start at zero on its stream
 *   before its kernels read it): calls that overlap on one GPU -- on
 *   different streams, or from threads without ordering -- race and give
 *   undefined results.  Order them on one stream.
 */
#define GENIE_NOALLOC_WORKSPACE_BYTES (64u << 20)
int genie_search_noalloc_async(const genie_index *ix, const uint64_t *d_q_offsets,
                               const genie_item *d_items, uint64_t n_items, uint32_t n_queries,
                               uint32_t max_items, uint32_t k, uint32_t *d_out_ids,
                               uint32_t *d_out_counts, void *stream);

/*
 * Search with a learned initial gate (an extension of Algorithm 1: the paper
 * starts the AuditThreshold at 1).  For each query the AuditThreshold starts
 * at max(1, floor(d_gate[q] - gate_delta)), capped at s + 1, where d_gate[q]
 * is a prediction of the query's k-th match count (genie_gate_forward_async).
 * Fewer increments then pass the gate.  Results are identical to
 * genie_search_async: a query whose k-th count lies below its start is
 * detected after the scan and answered again with AT = 1 on the device (the
 * number of such queries is left as a uint32 at byte offset 40 of the
 * workspace).
 *   d_gate: device, n_queries float32.  gate_delta >= 0.
 *   Other arguments and the workspace as genie_search_async.
 */
int genie_search_gated_async(const genie_index *ix, const uint64_t *d_q_offsets,
                             const genie_item *d_items, uint64_t n_items, uint32_t n_queries,
                             uint32_t max_items, uint32_t k, const float *d_gate,
                             float gate_delta, uint32_t *d_out_ids, uint32_t *d_out_counts,
                             void *d_workspace, size_t workspace_bytes, void *stream);

/*
 * GEN-SPQ, the c-PQ ablation of Section 6.3: the same index and counters,
 * but without the Gate and the Hash Table of Section 3.3.  Every posting
 * only increments its object's counter; afterwards each tile finds its k-th
 * count from the exact counters (the largest c with at least min(k, tile
 * objects) objects of count >= c, found by bisection: the bucket selection
 * of the paper's appendix collapses to this on small integer counts) and
 * selects from the counters alone.  Results are identical to
 * genie_search_async; it exists to measure what c-PQ saves.  Arguments,
 * workspace and errors as genie_search_async (it always runs 1024 threads
 * x 4 dwords, one workgroup per pair).
 */
int genie_search_spq_async(const genie_index *ix, const uint64_t *d_q_offsets,
                           const genie_item *d_items, uint64_t n_items, uint32_t n_queries,
                           uint32_t max_items, uint32_t k, uint32_t *d_out_ids,
                           uint32_t *d_out_counts, void *d_workspace, size_t workspace_bytes,
                           void *stream);

/*
 * genie_search_async (d_gate NULL) or genie_search_gated_async (d_gate set)
 * over the first *d_rows of a batch laid out for `capacity` queries, the
 * count read on the device when the kernels run.  For callers that record
 * the launches once in a HIP graph and replay them on batches of any size
 * up to the capacity (the buffers and the workspace are sized for it): rows
 * at or past *d_rows are neither scanned nor written.
 *   d_q_offsets: device, capacity + 1 uint64 (entries past the live rows
 *                are not read by the search); d_gate: capacity float32.
 *   d_rows: device, one uint32 <= capacity.
 *   Other arguments, the workspace and errors as genie_search_async with
 *   n_queries = capacity.
 */
int genie_search_rows_async(const genie_index *ix, const uint64_t *d_q_offsets,
                            const genie_item *d_items, uint64_t n_items, uint32_t capacity,
                            const uint32_t *d_rows, uint32_t max_items, uint32_t k,
                            const float *d_gate, float gate_delta, uint32_t *d_out_ids,
                            uint32_t *d_out_counts, void *d_workspace, size_t workspace_bytes,
                            void *stream);

/*
 * Random binning hashing (RBH) signatures for ANN in the Laplacian kernel
 * space (Section 4.1.3): for every point p and function f, the bin
 * floor((p_j - u[f][j]) / g[f][j]) on every dimension j (float32, correctly
 * rounded division; clamped to int32), the bin vector taken as int32
 * blocks in ascending j and re-hashed by MurmurHash3_x86_32 with seed
 * seeds[f]; out_sig[p][f] = the hash's top log2_buckets bits.  With g drawn
 * from Gamma(2, sigma) and u uniformly from [0, g) per function and
 * dimension, two points collide in a function with probability
 * exp(-||p - q||_1 / sigma).  Each signature depends on its own point and
 * function only.  Queries then use genie_lsh_items_async as for E2LSH.
 *   d_points: device, n * dim float32; d_g, d_u: device, m * dim float32
 *   (g > 0); d_seeds: device, m uint32; d_out_sig: device, n * m uint32.
 *   1 <= log2_buckets <= 32.  Errors: GENIE_EINVAL.
 */
int genie_rbh_signatures(const float *d_points, uint64_t n, uint32_t dim, const float *d_g,
                         const float *d_u, const uint32_t *d_seeds, uint32_t m,
                         uint32_t log2_buckets, uint32_t *d_out_sig, void *stream);

/* ---- multiple loadings: an index streamed to the device in parts -------- */

typedef struct genie_parts genie_parts; /* opaque, owned by the library */

typedef struct {
    uint64_t n_objects;
    uint32_t n_parts;
    uint32_t tiles_total;      /* tiles over all parts */
    uint64_t part_objects;
    uint64_t host_bytes;       /* pinned host memory holding the parts' indexes */
    uint64_t device_bytes;     /* the two device slots the parts stream through */
} genie_parts_info;

/*
 * Multiple loadings (Section 3.4), for an index larger than the device
 * memory the caller gives it: objects [p * part_objects, (p + 1) *
 * part_objects) form part p, whose index (the layout of genie_build_index,
 * tiles of 2^tile_log2 - 1 objects, tile_log2 = 15 or 16) is built once into
 * pinned host memory.  Two device slots, each sized for the largest part,
 * are allocated here.  values, n_objects, n_dims, n_buckets as
 * genie_build_index; part_objects >= 1.
 * Errors: GENIE_EINVAL, GENIE_ENOMEM, GENIE_EDEVICE.
 */
int genie_parts_build(const uint32_t *values, uint64_t n_objects, uint32_t n_dims,
                      uint32_t n_buckets, uint64_t part_objects, uint32_t tile_log2,
                      genie_parts **out);

/* Free the parts, their pinned host memory and device slots.  NULL is ignored. */
void genie_parts_free(genie_parts *parts);

/* Describe a parts index.  Errors: GENIE_EINVAL. */
int genie_parts_info_get(const genie_parts *parts, genie_parts_info *out);

/* Workspace bytes for genie_parts_search_async (0 for a NULL parts index). */
size_t genie_parts_workspace_size(const genie_parts *parts, uint32_t n_queries, uint32_t k);

/*
 * Top-k match-count search over all parts, identical to genie_search_async
 * on one index of all the objects.  Each part is copied into one of the two
 * slots on the library's own copy stream while the previous part is
 * scanned on `stream` (events order the copy into a slot after the last
 * scan that read it); every part's scan writes its tiles' exact top-k lists
 * into its own columns of one candidate array, ids offset by the part's
 * first object, and one merge over all columns on `stream` gives the answer
 * (Section 3.4's merge of the parts' results, on the device).  Arguments,
 * layout and errors as genie_search_async; the workspace has
 * genie_parts_workspace_size bytes.  Calls on one parts index run one at a
 * time: make them on one stream, or wait for a call before starting another.
 */
int genie_parts_search_async(genie_parts *parts, const uint64_t *d_q_offsets,
                             const genie_item *d_items, uint64_t n_items, uint32_t n_queries,
                             uint32_t max_items, uint32_t k, uint32_t *d_out_ids,
                             uint32_t *d_out_counts, void *d_workspace, size_t workspace_bytes,
                             void *stream);

/*
 * Queries of the LSH transform (Section 4.1.1): query q is the items
 * (i, sig[q][i], sig[q][i]) for i = 0..m-1, i.e. one exact keyword per hash
 * function.
 *   d_sig: device, n_queries * m uint32 (genie_lsh_signatures output).
 *   d_items: device, n_queries * m items; d_q_offsets: device, n_queries + 1.
 */
int genie_lsh_items_async(const uint32_t *d_sig, uint32_t n_queries, uint32_t m,
                          genie_item *d_items, uint64_t *d_q_offsets, void *stream);

/* ---- learned initial gate: features and a 64-128-128-1 MLP ------------- */

#define GENIE_GATE_FEATURES 64
#define GENIE_GATE_PARAMS 24961 /* W1[128][64] b1[128] W2[128][128] b2[128] w3[128] b3 */

/*
 * The 64 features of each query, from the posting counts L_i of the keywords
 * each item covers (an index lookup per item, no scan).  With p_i = L_i / n,
 * mu = sum p_i, sigma^2 = sum p_i (1 - p_i) and z the upper k/n quantile of
 * the standard normal:
 *   0 s/512 (s = items)  1 mu/64  2 sigma/8  3 (mu + z sigma)/64  4 max p_i
 *   5 sum p_i^2/64  6 sum p_i^3/64  7 z/8
 *   8..23  items with L_i > 0 by the largest b <= 15 with L_i 2^b <= n, /64
 *   24..55 the 32 largest p_i, descending (0 past s)
 *   56 items with L_i = 0, /64   57 items with 4 L_i >= n, /64   58..63 zero
 * Sums are formed in float64 in a fixed order and stored as float32.
 *   d_features: device, n_queries * 64 float32, row-major.
 * Errors: GENIE_EINVAL.
 */
int genie_gate_features_async(const genie_index *ix, const uint64_t *d_q_offsets,
                              const genie_item *d_items, uint64_t n_items, uint32_t n_queries,
                              uint32_t k, float *d_features, void *stream);

/*
 * Predictions out[i] = w3 . relu(W2 relu(W1 x_i + b1) + b2) + b3, float32
 * arithmetic, each dot product summed in index order (a row's prediction does
 * not depend on the other rows).  Weights: exactly one of d_w_bf16 (bfloat16
 * bit patterns) or d_w_f32, GENIE_GATE_PARAMS values in the layout above.
 *   d_x: device, n * 64 float32; d_out: device, n float32.
 */
int genie_gate_forward_async(const uint16_t *d_w_bf16, const float *d_w_f32, const float *d_x,
                             uint32_t n, float *d_out, void *stream);

/* Workspace bytes for genie_gate_backward_async over n samples. */
size_t genie_gate_workspace_size(uint32_t n);

/*
 * Gradient of the mean pinball (quantile tau) loss over n samples,
 * L = mean(tau r if r >= 0 else (tau - 1) r), r = y - prediction, with
 * respect to the parameters (layout above), into d_grad (GENIE_GATE_PARAMS
 * float32), and the loss into *d_loss (may be NULL).  Per-workgroup partial
 * sums are added in a fixed order.  0 < tau < 1.
 */
int genie_gate_backward_async(const uint16_t *d_w_bf16, const float *d_w_f32, const float *d_x,
                              const float *d_y, uint32_t n, float tau, float *d_grad,
                              float *d_loss, void *d_workspace, size_t workspace_bytes,
                              void *stream);

/*
 * One Adam step on the float32 master weights (moments d_m, d_v; step counts
 * from 1), then d_w_bf16 (may be NULL) = master rounded to nearest bfloat16,
 * ties to even.
 */
int genie_gate_adam_async(float *d_master, uint16_t *d_w_bf16, const float *d_grad, float *d_m,
                          float *d_v, uint32_t step, float lr, float beta1, float beta2, float eps,
                          void *stream);

/*
 * Full match-count vectors (the scan-and-count step of Section 3.2 with the
 * Bitmap Counter of Section 3.3.1), for checking and analysis.
 *   d_out_counts: device, n_queries * n_objects uint32; row q at q*n_objects.
 * Other arguments as genie_search_async (workspace from
 * genie_search_workspace_size(ix, n_queries, 1)).
 */
int genie_match_count_async(const genie_index *ix, const uint64_t *d_q_offsets,
                            const genie_item *d_items, uint64_t n_items, uint32_t n_queries,
                            uint32_t max_items, uint32_t *d_out_counts,
                            void *d_workspace, size_t workspace_bytes, void *stream);

/*
 * LSH signatures (Section 4.1.2 object transform with the E2LSH family of
 * Section 4.2.3):  h_i(p) = floor((a_i . p + b_i) / w), computed in float32
 * (products and a sum in a fixed order), then re-hashed into
 * [0, 2^log2_buckets):  u = the 32-bit two's complement pattern of h_i
 * zero-extended to 64 bits,  r_i = ((A_i * u + B_i) mod 2^64) >> (64 - log2_buckets).
 *   d_points: device, n * dim float32, row-major.
 *   d_a:      device, m * dim float32 (row i = a_i).
 *   d_b:      device, m float32.
 *   w:        bucket width > 0.
 *   d_rehash: device, 2*m uint64, (A_0, B_0, A_1, B_1, ...).
 *   log2_buckets: 1 .. 32.
 *   d_out_sig: device, n * m uint32, row-major (object = [r_1(h_1(p)), ...]).
 * Errors: GENIE_EINVAL, GENIE_EDEVICE.
 */
int genie_lsh_signatures(const float *d_points, uint64_t n, uint32_t dim, const float *d_a,
                         const float *d_b, float w, uint32_t m, const uint64_t *d_rehash,
                         uint32_t log2_buckets, uint32_t *d_out_sig, void *stream);

/*
 * Index over keyword sets (the Shotgun-and-Assembly scheme of Section 2.2
 * and Section 5: an object is a set of keywords, such as the words of a
 * short document, Section 5.2, or the ordered n-grams of a sequence,
 * Section 5.1.1).  Object o holds the keywords keys[obj_offsets[o] ..
 * obj_offsets[o+1]), each below n_keys and each at most once per object.
 *   obj_offsets: host, n_objects + 1 uint64, non-decreasing.
 *   keys:        host, obj_offsets[n_objects] - obj_offsets[0] uint32
 *                (may be NULL when that is 0).
 *   n_objects: 1 .. 2^32 - 2; n_keys: 1 .. 2^32 - 2; tile_log2: 15 or 16.
 * The index has n_dims = 1 and n_buckets = n_keys: the query item
 * (0, key, key) is the list of one keyword.  Every item on this index must
 * name one keyword (lo == hi) or be empty, which keeps every count at most
 * the number of items; a range item is an error of genie_search and is
 * treated as empty by the asynchronous searches, which then raise
 * GENIE_STATUS_RANGE_ON_SET.  Device layout and errors as
 * genie_build_index_tiled (GENIE_EINVAL also for a key >= n_keys or
 * decreasing offsets).
 */
int genie_build_index_sets(const uint64_t *obj_offsets, const uint32_t *keys, uint64_t n_objects,
                           uint32_t n_keys, uint32_t tile_log2, genie_index **out);

/*
 * Similarity search on sequences under edit distance (Section 5.1).
 * A sequence is a string of bytes; the edit distance counts unit-cost
 * single-byte insertions, deletions and substitutions.
 */
typedef struct genie_seq_index genie_seq_index; /* opaque, owned by the library */

typedef struct {
    uint64_t n_sequences;
    uint64_t n_chars;          /* bytes of all sequences */
    uint64_t n_windows;        /* ordered n-grams of all sequences (postings) */
    uint32_t gram;             /* n of the n-grams */
    uint32_t alphabet;         /* distinct byte values in the data */
    uint32_t n_grams;          /* distinct n-grams in the data */
    uint32_t n_keys;           /* distinct ordered n-grams (keywords of the index) */
    uint32_t max_occurrences;  /* most occurrences of one n-gram in one sequence */
    uint32_t n_tiles;
    uint64_t device_bytes;     /* index, sequences and n-gram table on the device */
} genie_seq_info;

/*
 * Shotgun (Section 5.1.1): decompose every sequence into its ordered
 * n-grams G(S) (Example 5.1) and build the match-count index over them,
 * keeping the sequences on the device for verification.
 *   chars:   host, offsets[n_sequences] bytes: the sequences back to back.
 *   offsets: host, n_sequences + 1 uint64, offsets[0] = 0, non-decreasing;
 *            sequence i is chars[offsets[i] .. offsets[i+1]).
 *   gram:    n, 1..8.  alphabet^gram (alphabet = distinct byte values of
 *            the data) must be at most 2^24 (GENIE_ERANGE otherwise).
 *   tile_log2: 15 or 16 (tiles of the match-count index).
 * Errors: GENIE_EINVAL, GENIE_ERANGE, GENIE_ENOMEM, GENIE_EDEVICE.
 */
int genie_seq_build(const uint8_t *chars, const uint64_t *offsets, uint64_t n_sequences,
                    uint32_t gram, uint32_t tile_log2, genie_seq_index **out);

/* Free a sequence index and its device memory.  NULL is ignored. */
void genie_seq_free(genie_seq_index *sx);

/* Describe a sequence index.  Errors: GENIE_EINVAL. */
int genie_seq_info_get(const genie_seq_index *sx, genie_seq_info *out);

/* The match-count index of a sequence index (owned by it; NULL for NULL). */
genie_index *genie_seq_match_index(genie_seq_index *sx);

/*
 * Query decomposition (Section 5.1.2): the items of every query's ordered
 * n-grams on the index of genie_seq_match_index.  Item r of query q is
 * written at d_items[d_qoffsets[q] + r] (one item per query byte): window r
 * gives (0, key, key) for the keyword of its ordered n-gram, or the empty
 * item (0, 1, 0) when no data sequence holds that ordered n-gram; the last
 * gram - 1 bytes of a query start no window and give empty items.  So the
 * query offsets are also the item offsets, and the match count of a
 * sequence S is |G(S) and G(Q)| (Lemma 5.1).
 *   d_qchars: device, n_qchars bytes; d_qoffsets: device, n_queries + 1,
 *   non-decreasing, d_qoffsets[n_queries] <= n_qchars; d_items: device,
 *   n_qchars items.  A query whose offsets are invalid gets no items; one
 *   longer than GENIE_MAX_ITEMS gets empty items (the search pads its row).
 * Errors: GENIE_EINVAL (null pointer); launch errors GENIE_EDEVICE.
 */
int genie_seq_decompose_async(const genie_seq_index *sx, const uint8_t *d_qchars,
                              const uint64_t *d_qoffsets, uint64_t n_qchars, uint32_t n_queries,
                              genie_item *d_items, void *stream);

/*
 * Verification (Algorithm 2, Section 5.1.2) of K candidates per query,
 * given in count order (genie_search_async's output on the match index).
 * Answer: the k candidates of smallest edit distance to the query, ties to
 * the earlier candidate (Algorithm 2 with k = 1; its filtering bound and
 * length filter skip only candidates that cannot change this answer).
 *   d_cand_ids, d_cand_counts: device, n_queries * K; ids >= n_sequences
 *     are empty slots (distance UINT32_MAX).
 *   max_qlen: at least every query's length, at most GENIE_MAX_ITEMS.
 *   d_out_ids, d_out_dist: device, n_queries * k, best first; slots past
 *     the valid candidates hold UINT32_MAX.
 *   d_out_cert: device, n_queries: 1 if Theorem 5.2 certifies the answer as
 *     the true k nearest sequences of the whole data set (c_K <
 *     |Q| - n + 1 - tau_k' n, c_K the K-th candidate's count, tau_k' the
 *     k-th answer's distance), or if K >= n_sequences; else 0.
 * A query with invalid offsets or longer than max_qlen's bit-vector width
 * gets UINT32_MAX answers and certificate 0.
 * Errors: GENIE_EINVAL (null pointer; need 1 <= k <= K <= GENIE_MAX_K),
 * GENIE_ERANGE (max_qlen), GENIE_EDEVICE.
 */
int genie_seq_verify_async(const genie_seq_index *sx, const uint8_t *d_qchars,
                           const uint64_t *d_qoffsets, uint64_t n_qchars, uint32_t n_queries,
                           uint32_t max_qlen, const uint32_t *d_cand_ids,
                           const uint32_t *d_cand_counts, uint32_t K, uint32_t k,
                           uint32_t *d_out_ids, uint32_t *d_out_dist, uint32_t *d_out_cert,
                           void *stream);

/* Workspace bytes for genie_seq_search_async (0 for a NULL index). */
size_t genie_seq_workspace_size(const genie_seq_index *sx, uint32_t n_queries, uint64_t n_qchars,
                                uint32_t K);

/*
 * Sequence search (Section 5.1): decomposition, top-K match-count search
 * (c-PQ, as genie_search_async) and verification, on `stream`, writing
 * what genie_seq_verify_async writes.  The workspace (device, 256-byte
 * aligned, genie_seq_workspace_size bytes) starts with the search
 * workspace, so its status word and statistics are read as for
 * genie_search_async; it also holds the items and the K candidates.
 * Arguments and errors as genie_seq_decompose_async and
 * genie_seq_verify_async.
 */
int genie_seq_search_async(const genie_seq_index *sx, const uint8_t *d_qchars,
                           const uint64_t *d_qoffsets, uint64_t n_qchars, uint32_t n_queries,
                           uint32_t max_qlen, uint32_t K, uint32_t k, uint32_t *d_out_ids,
                           uint32_t *d_out_dist, uint32_t *d_out_cert, void *d_workspace,
                           size_t workspace_bytes, void *stream);

/*
 * Per-kernel timing for measurement.  While enabled, every search call
 * records a HIP event pair around its scan kernel, around its merge kernel
 * and (gated search) around its fallback scan, on the stream of the call.  genie_kernel_timing_read waits for the
 * recorded events, adds up their elapsed times and (if reset != 0) clears the
 * totals.  Disabled by default; process-wide; thread-safe.
 */
typedef struct {
    uint64_t scan_launches;
    double scan_ms;      /* summed event time of the scan + c-PQ kernel */
    uint64_t merge_launches;
    double merge_ms;     /* summed event time of the per-query merge kernel */
    uint64_t fallback_launches;
    double fallback_ms;  /* summed event time of the gated search's fallback scan */
} genie_kernel_times;

int genie_kernel_timing_enable(int on);
int genie_kernel_timing_read(genie_kernel_times *out, int reset);

/*
 * Measurement probes (not part of the search): the peak rates the search
 * kernels are priced against, measured on the current device.  Both run on
 * the null stream and wait for their own kernels.
 *
 * genie_probe_lds_atomics: n_blocks workgroups of 1024 threads, 64 KB of LDS
 * each (two share a CU, as the scan kernel's at 8-bit counters), every lane
 * issuing steps x 8 32-bit LDS atomic adds, 8 independent ones at a time.
 *   mode 0: with return, lane-consecutive words (no bank conflicts);
 *   mode 1: with return, pseudo-random words of the 64 KB;
 *   mode 2: without return, pseudo-random words;
 *   mode 3: with return, lane l at word l of a pseudo-random 64-word row
 *           (one bank per lane, rows scattered).
 *   Modes 1-3 draw per-lane random words once and move them every step by
 *   XOR with a step-dependent value shared by the wave (one vector op per
 *   atomic), which keeps mode 3's lane-to-bank relation.
 *   d_sink: device, n_blocks * 1024 uint32 (written; keeps results live).
 *   *out_per_s: atomic adds per second over the chip (one untimed launch,
 *   then one timed by HIP events).
 * genie_probe_hbm: a streaming read of `bytes` at d_src (16-byte loads,
 * grid-stride), `reps` launches timed together -> *out_read_gbs; with d_dst
 * set, a copy of d_src into d_dst likewise -> *out_copy_gbs (bytes read plus
 * bytes written).  bytes: a multiple of 16, well above the 256 MB of
 * Infinity Cache for an HBM figure.  d_sink: device, >= 1 uint32.
 * Errors: GENIE_EINVAL (bad arguments), GENIE_EDEVICE.
 */
int genie_probe_lds_atomics(int mode, uint32_t steps, uint32_t n_blocks, uint32_t *d_sink,
                            double *out_per_s);
int genie_probe_hbm(const void *d_src, void *d_dst, uint64_t bytes, uint32_t reps,
                    uint32_t *d_sink, double *out_read_gbs, double *out_copy_gbs);

/* Message of the last failure on the calling thread ("" if none). */
const char *genie_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GENIE_H */
