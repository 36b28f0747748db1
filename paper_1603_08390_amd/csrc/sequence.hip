// Similarity search on sequences under edit distance with the
// Shotgun-and-Assembly scheme (Section 5.1).
//
// Shotgun (Section 5.1.1): every sequence is cut by a sliding window into
// its ordered n-grams G(S), the pairs (n-gram, i) with i the number of
// earlier windows holding the same n-gram (Example 5.1).  Each distinct pair
// is one keyword, and the inverted index holds every sequence under the
// keywords of its ordered n-grams (a keyword-set index, d = 1).  Keywords
// are numbered per n-gram: n-gram g with at most c occurrences in any one
// sequence owns the keywords first[g] .. first[g] + c - 1, occurrence i
// being first[g] + i.  An n-gram is coded in base A over the data's
// alphabet (the distinct byte values of the data), and a table with one
// entry per code (A^n entries) gives (first, c), with c = 0 for n-grams that
// no sequence holds.
//
// Assembly (Section 5.1.2): a query's ordered n-grams become one item per
// window, so that its match count against S is |G(S) and G(Q)|, which is
// Lemma 5.1's sum of min(c_s, c_q).  The match-count search returns the K
// candidates of largest count (count desc, id asc).  Verification computes
// the edit distance of the query to the candidates and keeps the k closest,
// Algorithm 2's answer: the candidates' distances are computed in parallel
// lanes, one candidate per lane, and the answer is the k first candidates
// in the order (distance, candidate position).  Algorithm 2 visits the
// candidates in count order and stops or skips only where Theorem 5.1 shows
// that no closer candidate can follow (the filtering bound) or that the
// candidate is farther (the length filter), so its answer is that order's
// first k: computing all K distances at once yields the same answer.
// Theorem 5.2 then certifies the answer as the true top-k of the whole data
// set when the K-th candidate's count is below |Q| - n + 1 - tau_k' n.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <new>
#include <thread>
#include <vector>

#include "bitvector_ed.h"
#include "internal.h"

using namespace genie;

struct genie_seq_index {
    genie_index *ix = nullptr;     // match-count index over the ordered n-grams
    uint8_t *chars = nullptr;      // device: the sequences back to back
    uint64_t *offsets = nullptr;   // device: n + 1 offsets into chars
    int32_t *sym = nullptr;        // device: 256 entries, symbol of a byte or -1
    uint32_t *grams = nullptr;     // device: 2 words per n-gram code (first keyword, occurrences)
    uint64_t n = 0, n_chars = 0, n_windows = 0, table_entries = 0;
    uint32_t gram = 0, alphabet = 0, n_grams = 0, n_keys = 0, max_occurrences = 0;
    uint64_t device_bytes = 0;
    int device = 0;
};

namespace {

constexpr uint32_t kNoGram = 0xFFFFFFFFu;
constexpr uint64_t kMaxTable = 1ull << 24;   // n-gram codes (A^n)

struct DecomposeParams {
    const uint8_t *qchars;
    const uint64_t *qoff;
    uint64_t n_qchars;
    uint32_t nq, gram, alphabet;
    const int32_t *sym;
    const uint32_t *grams;
    uint32_t *items;        // 3 words per query character
};

// One wave per query.  Window p of the query gives the item of its ordered
// n-gram (0, key, key), or an empty item (0, 1, 0) when no sequence holds it;
// the last gram - 1 characters of a query start no window and give empty
// items, so item r of the query sits at character offset r.
__global__ __launch_bounds__(64) void seq_decompose_kernel(DecomposeParams p) {
    __shared__ uint32_t code[GENIE_MAX_ITEMS];
    const uint32_t q = blockIdx.x, lane = threadIdx.x;
    const uint64_t c0 = p.qoff[q], c1 = p.qoff[q + 1];
    if (c1 < c0 || c1 > p.n_qchars)
        return;   // the search reports these offsets (GENIE_STATUS_BAD_OFFSETS)
    const uint64_t len64 = c1 - c0;
    uint32_t *out = p.items + 3 * c0;
    if (len64 > GENIE_MAX_ITEMS) {
        // the search pads this row (GENIE_STATUS_TOO_MANY_ITEMS); keep the
        // items defined
        for (uint64_t r = lane; r < len64; r += 64) {
            out[3 * r] = 0;
            out[3 * r + 1] = 1;
            out[3 * r + 2] = 0;
        }
        return;
    }
    const uint32_t L = (uint32_t)len64;
    const uint32_t nw = L >= p.gram ? L - p.gram + 1 : 0;
    for (uint32_t w = lane; w < nw; w += 64) {
        uint32_t c = 0;
        bool ok = true;
        for (uint32_t i = 0; i < p.gram; i++) {
            const int32_t s = p.sym[p.qchars[c0 + w + i]];
            ok = ok && s >= 0;
            c = c * p.alphabet + (uint32_t)max(s, 0);
        }
        code[w] = ok ? c : kNoGram;
    }
    __syncthreads();
    for (uint32_t w = lane; w < L; w += 64) {
        uint32_t lo = 1, hi = 0;
        if (w < nw && code[w] != kNoGram) {
            const uint32_t c = code[w];
            uint32_t occ = 0;
            for (uint32_t r = 0; r < w; r++)
                occ += code[r] == c ? 1u : 0u;
            const uint32_t first = p.grams[2 * (uint64_t)c], count = p.grams[2 * (uint64_t)c + 1];
            if (occ < count)
                lo = hi = first + occ;
        }
        out[3 * w] = 0;
        out[3 * w + 1] = lo;
        out[3 * w + 2] = hi;
    }
}

struct VerifyParams {
    const uint8_t *qchars;
    const uint64_t *qoff;
    uint64_t n_qchars;
    const uint8_t *chars;
    const uint64_t *offsets;
    uint64_t n;
    uint32_t nq, gram, K, k;
    const uint32_t *cand_ids;      // [nq][K]
    const uint32_t *cand_counts;   // [nq][K]
    uint32_t *out_ids, *out_dist;  // [nq][k]
    uint32_t *out_cert;            // [nq]
};

constexpr uint32_t kTextChunk = 16;   // text bytes loaded ahead of the bit-vector steps

// One wave per query; pattern = query (at most 64*W characters).
template <int W>
__global__ __launch_bounds__(64) void seq_verify_kernel(VerifyParams p) {
    __shared__ uint64_t peq[256 * W];
    __shared__ uint8_t qs[64 * W];
    __shared__ uint32_t dist[GENIE_MAX_K];
    __shared__ uint32_t tau_k;
    const uint32_t q = blockIdx.x, lane = threadIdx.x;
    const uint64_t c0 = p.qoff[q], c1 = p.qoff[q + 1];
    uint32_t *oid = p.out_ids + (uint64_t)q * p.k, *odist = p.out_dist + (uint64_t)q * p.k;
    if (c1 < c0 || c1 > p.n_qchars || c1 - c0 > 64ull * W) {
        for (uint32_t r = lane; r < p.k; r += 64) {
            oid[r] = UINT32_MAX;
            odist[r] = UINT32_MAX;
        }
        if (lane == 0)
            p.out_cert[q] = 0;
        return;
    }
    const uint32_t m = (uint32_t)(c1 - c0);
    for (uint32_t i = lane; i < m; i += 64)
        qs[i] = p.qchars[c0 + i];
    if (lane == 0)
        tau_k = UINT32_MAX;
    __syncthreads();
    // match masks: lane l builds those of byte values l, l+64, l+128, l+192
    for (uint32_t c = lane; c < 256; c += 64)
#pragma unroll
        for (int b = 0; b < W; b++) {
            uint64_t word = 0;
            const uint32_t i1 = min(m, 64u * (b + 1));
            for (uint32_t i = 64u * b; i < i1; i++)
                word |= (qs[i] == c ? 1ull : 0ull) << (i - 64u * b);
            peq[c * W + b] = word;
        }
    __syncthreads();
    const uint32_t *cid = p.cand_ids + (uint64_t)q * p.K;
    for (uint32_t j = lane; j < p.K; j += 64) {
        const uint32_t id = cid[j];
        uint32_t d = UINT32_MAX;
        if (id < p.n) {
            const uint8_t *t = p.chars + p.offsets[id];
            const uint32_t tn = (uint32_t)(p.offsets[id + 1] - p.offsets[id]);
            if (m == 0) {
                d = tn;
            } else {
                BitVectorEd<W> ed;
                ed.init(m);
                for (uint32_t j0 = 0; j0 < tn; j0 += kTextChunk) {
                    uint8_t buf[kTextChunk];
#pragma unroll
                    for (uint32_t u = 0; u < kTextChunk; u++)
                        buf[u] = j0 + u < tn ? t[j0 + u] : 0;
                    const uint32_t cnt = min(kTextChunk, tn - j0);
                    for (uint32_t u = 0; u < cnt; u++)
                        ed.step(&peq[buf[u] * W]);
                }
                d = ed.score;
            }
        }
        dist[j] = d;
    }
    __syncthreads();
    // rank in (distance, candidate position): the k first are the answer
    for (uint32_t j = lane; j < p.K; j += 64) {
        const uint32_t d = dist[j];
        uint32_t r = 0;
        for (uint32_t t = 0; t < p.K; t++) {
            const uint32_t e = dist[t];
            r += (e < d || (e == d && t < j)) ? 1u : 0u;
        }
        if (r < p.k) {
            oid[r] = d == UINT32_MAX ? UINT32_MAX : cid[j];
            odist[r] = d;
        }
        if (r == p.k - 1)
            tau_k = d;
    }
    __syncthreads();
    if (lane == 0) {
        // Theorem 5.2 (and trivially when every sequence is a candidate)
        uint32_t cert;
        if ((uint64_t)p.K >= p.n) {
            cert = 1;
        } else if (tau_k == UINT32_MAX) {
            cert = 0;
        } else {
            const int64_t c_K = (int64_t)p.cand_counts[(uint64_t)q * p.K + p.K - 1];
            const int64_t bound = (int64_t)m - (int64_t)p.gram + 1 - (int64_t)tau_k * p.gram;
            cert = c_K < bound ? 1u : 0u;
        }
        p.out_cert[q] = cert;
    }
}

int verify_words(uint32_t max_qlen) {
    for (int w : {1, 2, 4, 8, 16})
        if (max_qlen <= 64u * w)
            return w;
    return 0;
}

void free_seq(genie_seq_index *sx) {
    if (sx->ix)
        genie_free_index(sx->ix);
    if (sx->chars) (void)hipFree(sx->chars);
    if (sx->offsets) (void)hipFree(sx->offsets);
    if (sx->sym) (void)hipFree(sx->sym);
    if (sx->grams) (void)hipFree(sx->grams);
    delete sx;
}

struct SeqWorkspace {
    size_t search = 0, items = 0, cand_ids = 0, cand_counts = 0, total = 0;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

SeqWorkspace seq_workspace(const genie_seq_index *sx, uint32_t nq, uint64_t n_qchars,
                           uint32_t K) {
    SeqWorkspace L;
    L.search = 0;
    L.items = align256(workspace_layout(sx->ix, nq, K).total);
    L.cand_ids = align256(L.items + 12 * std::max<uint64_t>(n_qchars, 1));
    L.cand_counts = align256(L.cand_ids + 4ull * nq * K);
    L.total = align256(L.cand_counts + 4ull * nq * K);
    return L;
}

int check_queries(const genie_seq_index *sx, const uint8_t *d_qchars, const uint64_t *d_qoffsets,
                  uint64_t n_qchars, uint32_t nq) {
    if (!sx) {
        set_error("null sequence index");
        return GENIE_EINVAL;
    }
    if (nq && (!d_qoffsets || (!d_qchars && n_qchars))) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    if (nq > 0x7FFFFFFFu) {
        set_error("too many queries (%u)", nq);
        return GENIE_EINVAL;
    }
    return GENIE_OK;
}

int launch_decompose(const genie_seq_index *sx, const uint8_t *d_qchars,
                     const uint64_t *d_qoffsets, uint64_t n_qchars, uint32_t nq,
                     genie_item *d_items, hipStream_t st) {
    DecomposeParams p{d_qchars, d_qoffsets, n_qchars, nq, sx->gram, sx->alphabet, sx->sym,
                      sx->grams, reinterpret_cast<uint32_t *>(d_items)};
    hipLaunchKernelGGL(seq_decompose_kernel, dim3(nq), dim3(64), 0, st, p);
    GENIE_HIP(hipGetLastError());
    return GENIE_OK;
}

int launch_verify(const genie_seq_index *sx, const uint8_t *d_qchars, const uint64_t *d_qoffsets,
                  uint64_t n_qchars, uint32_t nq, uint32_t max_qlen, const uint32_t *d_cand_ids,
                  const uint32_t *d_cand_counts, uint32_t K, uint32_t k, uint32_t *d_out_ids,
                  uint32_t *d_out_dist, uint32_t *d_out_cert, hipStream_t st) {
    const int W = verify_words(max_qlen);
    VerifyParams p{d_qchars, d_qoffsets, n_qchars, sx->chars, sx->offsets, sx->n, nq, sx->gram,
                   K, k, d_cand_ids, d_cand_counts, d_out_ids, d_out_dist, d_out_cert};
    switch (W) {
    case 1: hipLaunchKernelGGL(seq_verify_kernel<1>, dim3(nq), dim3(64), 0, st, p); break;
    case 2: hipLaunchKernelGGL(seq_verify_kernel<2>, dim3(nq), dim3(64), 0, st, p); break;
    case 4: hipLaunchKernelGGL(seq_verify_kernel<4>, dim3(nq), dim3(64), 0, st, p); break;
    case 8: hipLaunchKernelGGL(seq_verify_kernel<8>, dim3(nq), dim3(64), 0, st, p); break;
    default: hipLaunchKernelGGL(seq_verify_kernel<16>, dim3(nq), dim3(64), 0, st, p); break;
    }
    GENIE_HIP(hipGetLastError());
    return GENIE_OK;
}

int check_verify_args(const genie_seq_index *sx, uint32_t max_qlen, uint32_t K, uint32_t k) {
    if (max_qlen > GENIE_MAX_ITEMS) {
        set_error("max_qlen=%u above %u", max_qlen, GENIE_MAX_ITEMS);
        return GENIE_ERANGE;
    }
    if (K == 0 || K > GENIE_MAX_K || k == 0 || k > K) {
        set_error("need 1 <= k <= K <= %d (K=%u, k=%u)", GENIE_MAX_K, K, k);
        return GENIE_EINVAL;
    }
    (void)sx;
    return GENIE_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------

extern "C" int genie_seq_build(const uint8_t *chars, const uint64_t *offsets, uint64_t n,
                               uint32_t gram, uint32_t tile_log2, genie_seq_index **out) {
    clear_error();
    if (!offsets || !out) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    *out = nullptr;
    if (n == 0 || n >= 0xFFFFFFFFull || gram == 0 || gram > 8) {
        set_error("bad sizes n=%llu gram=%u (gram 1..8)", (unsigned long long)n, gram);
        return GENIE_EINVAL;
    }
    if (offsets[0] != 0) {
        set_error("offsets[0] must be 0");
        return GENIE_EINVAL;
    }
    for (uint64_t i = 0; i < n; i++)
        if (offsets[i + 1] < offsets[i]) {
            set_error("offsets decrease at sequence %llu", (unsigned long long)i);
            return GENIE_EINVAL;
        }
    const uint64_t n_chars = offsets[n];
    if (n_chars && !chars) {
        set_error("null chars");
        return GENIE_EINVAL;
    }
    genie_seq_index *sx = new (std::nothrow) genie_seq_index;
    if (!sx) {
        set_error("host allocation failed");
        return GENIE_ENOMEM;
    }
    try {
        sx->n = n;
        sx->n_chars = n_chars;
        sx->gram = gram;
        // alphabet: the byte values present, numbered in increasing order
        std::vector<int32_t> sym(256, -1);
        {
            std::vector<uint8_t> present(256, 0);
            for (uint64_t i = 0; i < n_chars; i++)
                present[chars[i]] = 1;
            uint32_t a = 0;
            for (int b = 0; b < 256; b++)
                if (present[b])
                    sym[b] = (int32_t)a++;
            sx->alphabet = std::max(a, 1u);
        }
        uint64_t table = 1;
        for (uint32_t i = 0; i < gram; i++) {
            table *= sx->alphabet;
            if (table > kMaxTable) {
                set_error("alphabet^gram = %u^%u is above %llu n-gram codes", sx->alphabet, gram,
                          (unsigned long long)kMaxTable);
                free_seq(sx);
                return GENIE_ERANGE;
            }
        }
        sx->table_entries = table;
        // windows of every sequence, as objects' keyword lists
        std::vector<uint64_t> obj_off(n + 1, 0);
        for (uint64_t i = 0; i < n; i++) {
            const uint64_t L = offsets[i + 1] - offsets[i];
            obj_off[i + 1] = obj_off[i] + (L >= gram ? L - gram + 1 : 0);
        }
        const uint64_t nw = obj_off[n];
        sx->n_windows = nw;
        std::vector<uint32_t> key(nw), occ(nw);
        std::vector<std::atomic<uint32_t>> count(table);
        for (auto &c : count)
            c.store(0, std::memory_order_relaxed);
        const unsigned nth =
            std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        auto for_sequences = [&](const auto &body) {
            std::atomic<uint64_t> next{0};
            std::atomic<int> nomem{0};
            const uint64_t chunk = 4096;
            auto worker = [&]() {
                try {   // a thread that cannot allocate reports it
                    std::vector<uint64_t> scratch;
                    for (;;) {
                        const uint64_t s0 = next.fetch_add(chunk);
                        if (s0 >= n || nomem.load())
                            break;
                        for (uint64_t s = s0; s < std::min(n, s0 + chunk); s++)
                            body(s, scratch);
                    }
                } catch (const std::bad_alloc &) {
                    nomem.store(1);
                }
            };
            std::vector<std::thread> pool;
            for (unsigned t = 0; t < nth; t++)
                pool.emplace_back(worker);
            for (auto &th : pool)
                th.join();
            if (nomem.load())
                throw std::bad_alloc();   // caught below: GENIE_ENOMEM
        };
        // codes, then occurrence ranks by sorting (code, window) within a
        // sequence, then the largest occurrence count of every code
        for_sequences([&](uint64_t s, std::vector<uint64_t> &scratch) {
            const uint64_t w0 = obj_off[s], w1 = obj_off[s + 1];
            const uint8_t *c = chars + offsets[s];
            scratch.clear();
            for (uint64_t w = w0; w < w1; w++) {
                uint32_t code = 0;
                for (uint32_t i = 0; i < gram; i++)
                    code = code * sx->alphabet + (uint32_t)sym[c[w - w0 + i]];
                key[w] = code;
                scratch.push_back(((uint64_t)code << 32) | (uint64_t)(w - w0));
            }
            std::sort(scratch.begin(), scratch.end());
            for (size_t i = 0; i < scratch.size(); i++) {
                const uint32_t code = (uint32_t)(scratch[i] >> 32);
                const uint32_t o = (i > 0 && (uint32_t)(scratch[i - 1] >> 32) == code)
                                       ? occ[w0 + (uint32_t)scratch[i - 1]] + 1
                                       : 0u;
                occ[w0 + (uint32_t)scratch[i]] = o;
                uint32_t cur = count[code].load(std::memory_order_relaxed);
                while (cur < o + 1 &&
                       !count[code].compare_exchange_weak(cur, o + 1, std::memory_order_relaxed)) {
                }
            }
        });
        // keywords of each n-gram: first[g] .. first[g] + count[g] - 1
        std::vector<uint32_t> grams(2 * table, 0);
        uint64_t nkeys = 0;
        uint32_t distinct = 0, max_occ = 0;
        for (uint64_t g = 0; g < table; g++) {
            const uint32_t c = count[g].load(std::memory_order_relaxed);
            grams[2 * g] = (uint32_t)std::min<uint64_t>(nkeys, 0xFFFFFFFFu);
            grams[2 * g + 1] = c;
            nkeys += c;
            distinct += c ? 1u : 0u;
            max_occ = std::max(max_occ, c);
        }
        if (nkeys == 0)
            nkeys = 1;   // no windows at all: one keyword nobody holds
        if (nkeys >= 0xFFFFFFFFull) {
            set_error("%llu ordered n-grams: above the 32-bit keyword space",
                      (unsigned long long)nkeys);
            free_seq(sx);
            return GENIE_ERANGE;
        }
        sx->n_grams = distinct;
        sx->n_keys = (uint32_t)nkeys;
        sx->max_occurrences = max_occ;
        for_sequences([&](uint64_t s, std::vector<uint64_t> &) {
            for (uint64_t w = obj_off[s]; w < obj_off[s + 1]; w++)
                key[w] = grams[2 * (uint64_t)key[w]] + occ[w];
        });
        std::vector<uint32_t>().swap(occ);
        HostIndex h;
        int rc = build_host_index_sets(obj_off.data(), key.data(), n, (uint32_t)nkeys, tile_log2,
                                       &h);
        if (rc == GENIE_OK)
            rc = upload_host_index(h, &sx->ix);
        if (rc) {
            free_seq(sx);
            return rc;
        }
        hipError_t e = hipGetDevice(&sx->device);
        const size_t bc = std::max<uint64_t>(n_chars, 1), bo = (n + 1) * sizeof(uint64_t),
                     bs = 256 * sizeof(int32_t), bg = grams.size() * sizeof(uint32_t);
        if (e == hipSuccess) e = hipMalloc((void **)&sx->chars, bc);
        if (e == hipSuccess) e = hipMalloc((void **)&sx->offsets, bo);
        if (e == hipSuccess) e = hipMalloc((void **)&sx->sym, bs);
        if (e == hipSuccess) e = hipMalloc((void **)&sx->grams, bg);
        if (e == hipSuccess && n_chars)
            e = hipMemcpy(sx->chars, chars, n_chars, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(sx->offsets, offsets, bo, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(sx->sym, sym.data(), bs, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(sx->grams, grams.data(), bg, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            rc = hip_fail(e, "sequence index upload");
            free_seq(sx);
            return rc;
        }
        sx->device_bytes = sx->ix->device_bytes + bc + bo + bs + bg;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed while building the sequence index");
        free_seq(sx);
        return GENIE_ENOMEM;
    }
    *out = sx;
    return GENIE_OK;
}

extern "C" void genie_seq_free(genie_seq_index *sx) {
    if (!sx)
        return;
    int cur = 0;
    bool sw = hipGetDevice(&cur) == hipSuccess && cur != sx->device;
    if (sw)
        (void)hipSetDevice(sx->device);
    free_seq(sx);
    if (sw)
        (void)hipSetDevice(cur);
}

extern "C" int genie_seq_info_get(const genie_seq_index *sx, genie_seq_info *out) {
    clear_error();
    if (!sx || !out) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    out->n_sequences = sx->n;
    out->n_chars = sx->n_chars;
    out->n_windows = sx->n_windows;
    out->gram = sx->gram;
    out->alphabet = sx->alphabet;
    out->n_grams = sx->n_grams;
    out->n_keys = sx->n_keys;
    out->max_occurrences = sx->max_occurrences;
    out->n_tiles = sx->ix->n_tiles;
    out->device_bytes = sx->device_bytes;
    return GENIE_OK;
}

extern "C" genie_index *genie_seq_match_index(genie_seq_index *sx) { return sx ? sx->ix : nullptr; }

extern "C" int genie_seq_decompose_async(const genie_seq_index *sx, const uint8_t *d_qchars,
                                         const uint64_t *d_qoffsets, uint64_t n_qchars,
                                         uint32_t n_queries, genie_item *d_items, void *stream) {
    clear_error();
    int rc = check_queries(sx, d_qchars, d_qoffsets, n_qchars, n_queries);
    if (rc || n_queries == 0)
        return rc;
    if (!d_items) {
        set_error("null items");
        return GENIE_EINVAL;
    }
    return launch_decompose(sx, d_qchars, d_qoffsets, n_qchars, n_queries, d_items,
                            (hipStream_t)stream);
}

extern "C" int genie_seq_verify_async(const genie_seq_index *sx, const uint8_t *d_qchars,
                                      const uint64_t *d_qoffsets, uint64_t n_qchars,
                                      uint32_t n_queries, uint32_t max_qlen,
                                      const uint32_t *d_cand_ids, const uint32_t *d_cand_counts,
                                      uint32_t K, uint32_t k, uint32_t *d_out_ids,
                                      uint32_t *d_out_dist, uint32_t *d_out_cert, void *stream) {
    clear_error();
    int rc = check_queries(sx, d_qchars, d_qoffsets, n_qchars, n_queries);
    if (rc || (rc = check_verify_args(sx, max_qlen, K, k)) || n_queries == 0)
        return rc;
    if (!d_cand_ids || !d_cand_counts || !d_out_ids || !d_out_dist || !d_out_cert) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    return launch_verify(sx, d_qchars, d_qoffsets, n_qchars, n_queries, max_qlen, d_cand_ids,
                         d_cand_counts, K, k, d_out_ids, d_out_dist, d_out_cert,
                         (hipStream_t)stream);
}

extern "C" size_t genie_seq_workspace_size(const genie_seq_index *sx, uint32_t n_queries,
                                           uint64_t n_qchars, uint32_t K) {
    if (!sx)
        return 0;
    return seq_workspace(sx, n_queries, n_qchars, K).total;
}

extern "C" int genie_seq_search_async(const genie_seq_index *sx, const uint8_t *d_qchars,
                                      const uint64_t *d_qoffsets, uint64_t n_qchars,
                                      uint32_t n_queries, uint32_t max_qlen, uint32_t K,
                                      uint32_t k, uint32_t *d_out_ids, uint32_t *d_out_dist,
                                      uint32_t *d_out_cert, void *d_workspace,
                                      size_t workspace_bytes, void *stream) {
    clear_error();
    int rc = check_queries(sx, d_qchars, d_qoffsets, n_qchars, n_queries);
    if (rc || (rc = check_verify_args(sx, max_qlen, K, k)) || n_queries == 0)
        return rc;
    if (!d_out_ids || !d_out_dist || !d_out_cert || !d_workspace) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    const SeqWorkspace L = seq_workspace(sx, n_queries, n_qchars, K);
    if (((uintptr_t)d_workspace & 255) != 0 || workspace_bytes < L.total) {
        set_error("workspace too small (%zu < %zu) or not 256-byte aligned", workspace_bytes,
                  L.total);
        return GENIE_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)d_workspace;
    genie_item *items = reinterpret_cast<genie_item *>(ws + L.items);
    uint32_t *cand_ids = reinterpret_cast<uint32_t *>(ws + L.cand_ids);
    uint32_t *cand_counts = reinterpret_cast<uint32_t *>(ws + L.cand_counts);
    if ((rc = launch_decompose(sx, d_qchars, d_qoffsets, n_qchars, n_queries, items, st)))
        return rc;
    // item r of a query sits at its character offset: the query offsets are
    // the item offsets
    rc = launch_search(sx->ix, d_qoffsets, items, n_qchars, n_queries, std::max(max_qlen, 1u), K,
                       cand_ids, cand_counts, nullptr, ws + L.search, L.items - L.search, st);
    if (rc)
        return rc;
    return launch_verify(sx, d_qchars, d_qoffsets, n_qchars, n_queries, max_qlen, cand_ids,
                         cand_counts, K, k, d_out_ids, d_out_dist, d_out_cert, st);
}
