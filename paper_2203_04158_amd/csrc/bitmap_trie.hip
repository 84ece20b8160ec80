// Bitmap trie: a GPU layout of the radix-2^k trie of Sec. IV in which every
// node is one record {base, bitmap of its occurring chunk values}.
//
// Chunks are dispatched from the most significant end (the top chunk holds
// M mod k bits when k does not divide M), so at every level the nodes, and
// the members under each node, come in ascending numeric order.  A node's
// children are then consecutive records of the next level, and the child
// for chunk value c is record base + (number of set bits below c); at the
// last level the same count gives the rank, base being the position of the
// node's first member in the sector's list.  A clear bit means the pattern
// is not a member, so membership needs no read of the state list (the
// packed trie of trie.hip checks states[rank] == alpha after its walk).
//
// Records are 2^s bytes (8 B for k <= 5, 16 B for k = 6, 32 B for k = 7,
// 64 B for k = 8), the same size on every level (the root's short chunk
// included, one record), aligned to their size, so a record never straddles a
// 64-byte line: one line per level and query.  Word 0 is the base; for k >= 6
// one (k = 6, 7) or two (k = 8) words follow with, in byte w, the set bits of
// map words 0..w-1; then the 2^k-bit map.  A step reads the base, the prefix
// byte and one map word, so it costs one popcount whatever k is.
// The top levels that fit 48 KB are staged in LDS.  With k = 8 the sector
// M = 32, N = 16 with >= 6 of orbitals 0-7 occupied needs about 4 M leaf
// records (its packed trie holds 332 M entries).
#include <algorithm>
#include <cstring>
#include <memory>

#include "rank_device.hpp"

namespace {

constexpr unsigned kBlock = 256;
constexpr int kQ = 4;                      // independent walks in flight per lane
constexpr size_t kLdsBudget = 48 * 1024;   // bytes of top levels staged per workgroup
constexpr int kMaxH = 32;

struct BtArgs {
    const uint32_t *rec;      // all levels' records, level after level
    int32_t M, H, lds_levels;
    uint32_t lds_words;       // words of the staged levels
    uint32_t off[kMaxH];      // first word of each level
    uint32_t shift[kMaxH];    // bit offset of each level's chunk
    uint32_t cmask[kMaxH];    // chunk mask
};

// Words before the map in a record of RW words: the base, and the prefix
// bytes of the map words when there is more than one.
__host__ __device__ constexpr int map_offset(int rw) { return rw == 2 ? 1 : rw == 16 ? 3 : 2; }

// One level of the walk: the record at `rec` (RW words), chunk value c.
// Returns whether c occurs; `next` receives base + set bits below c.
template <int RW>
__device__ __forceinline__ bool bt_step(const uint32_t *rec, uint32_t c, uint32_t &next) {
    const uint32_t bit = c & 31;
    uint32_t base, cw, pre;
    if constexpr (RW == 2) {
        const uint2 v = *reinterpret_cast<const uint2 *>(rec);
        base = v.x;
        cw = v.y;
        pre = 0;
    } else {
        const uint4 h = *reinterpret_cast<const uint4 *>(rec);  // base, prefix words (and map words for k = 6)
        const uint32_t word = c >> 5;
        uint32_t pw = h.y;
        if constexpr (RW == 4) {
            cw = word ? h.w : h.z;
        } else {
            cw = rec[map_offset(RW) + word];
            if constexpr (RW == 16) pw = word >= 4 ? h.z : h.y;
        }
        pre = (pw >> (8 * (word & 3))) & 0xffu;
        base = h.x;
    }
    next = base + pre + __popc(cw & ((1u << bit) - 1u));
    return (cw >> bit) & 1u;
}

template <class P, int RW>
__global__ void __launch_bounds__(kBlock) bt_rank_kernel(const P *__restrict__ q, uint64_t n,
                                                         uint32_t *__restrict__ out, BtArgs a) {
    extern __shared__ __align__(16) uint32_t top[];
    stage_to_lds(top, a.rec, (uint64_t)a.lds_words * 4);
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; base < n; base += stride * kQ) {
        P x[kQ];
        uint32_t node[kQ];
        bool ok[kQ];
#pragma unroll
        for (int u = 0; u < kQ; ++u) {
            const uint64_t j = base + u * stride;
            x[u] = j < n ? q[j] : (P)0;
            ok[u] = j < n && (a.M >= (int)(8 * sizeof(P)) || (x[u] >> a.M) == 0);
            node[u] = 0;
        }
        // staged levels from LDS, the rest through the caches; a walk that
        // leaves the sector stays on record 0 of each further level
        int l = 0;
        for (; l < a.lds_levels; ++l) {
#pragma unroll
            for (int u = 0; u < kQ; ++u) {
                uint32_t nx;
                const uint32_t c = (uint32_t)(x[u] >> a.shift[l]) & a.cmask[l];
                ok[u] = bt_step<RW>(top + a.off[l] + node[u] * RW, c, nx) && ok[u];
                node[u] = ok[u] ? nx : 0u;
            }
        }
        for (; l < a.H; ++l) {
            const uint32_t *lv = a.rec + a.off[l];
#pragma unroll
            for (int u = 0; u < kQ; ++u) {
                uint32_t nx;
                const uint32_t c = (uint32_t)(x[u] >> a.shift[l]) & a.cmask[l];
                ok[u] = bt_step<RW>(lv + node[u] * RW, c, nx) && ok[u];  // words < 2^32
                node[u] = ok[u] ? nx : 0u;
            }
        }
#pragma unroll
        for (int u = 0; u < kQ; ++u) {
            const uint64_t j = base + u * stride;
            if (j < n) out[j] = ok[u] ? node[u] : MBR_NOT_FOUND;
        }
    }
}

// Words of a record for k-bit chunks: base, prefix words, map, rounded up to
// a power of two.
uint32_t record_words(int w) {
    const uint32_t map_words = ((1u << w) + 31) / 32;
    const uint32_t pref_words = map_words > 1 ? (map_words + 3) / 4 : 0;
    const uint32_t bytes = 4 * (1 + pref_words + map_words);
    uint32_t r = 8;
    while (r < bytes) r *= 2;
    return r / 4;
}

// Records of every level from the ascending list (one counting pass, one
// filling pass).
template <class P>
mbr_status build_records(BitmapTrie &t, const std::vector<P> &s) {
    const int H = t.H;
    std::vector<uint64_t> nodes(H, 0);
    for (int l = 0; l < H; ++l) {
        const int up = t.shift[l] + t.w[l];
        P prev = 0;
        uint64_t cnt = 0;
        for (size_t i = 0; i < s.size(); ++i) {
            const P pre = up >= (int)(8 * sizeof(P)) ? (P)0 : (P)(s[i] >> up);
            if (i == 0 || pre != prev) ++cnt;
            prev = pre;
        }
        nodes[l] = cnt;
    }
    uint64_t words = 0;
    const int kw = *std::max_element(t.w, t.w + H);
    for (int l = 0; l < H; ++l) {
        t.rw[l] = record_words(kw);  // one record size for all levels (the root's short chunk included)
        words = (words + 15) & ~(uint64_t)15;  // every level starts on a 64-byte line
        t.off[l] = words;
        t.nodes[l] = nodes[l];
        words += nodes[l] * t.rw[l];
    }
    t.off[H] = words;
    if (words >= (1ull << 32)) MBR_FAIL(MBR_EUNSUPPORTED, "bitmap trie of %llu words", (unsigned long long)words);
    std::vector<uint32_t> rec(words, 0u);
    std::vector<int64_t> cur(H, -1);
    std::vector<P> prev(H, 0);
    for (size_t i = 0; i < s.size(); ++i) {
        const P a = s[i];
        for (int l = 0; l < H; ++l) {
            const int up = t.shift[l] + t.w[l];
            const P pre = up >= (int)(8 * sizeof(P)) ? (P)0 : (P)(a >> up);
            if (cur[l] < 0 || pre != prev[l]) {
                ++cur[l];
                prev[l] = pre;
                // first child of a new node: the next record of the level
                // below (created for this member in the same pass), or at the
                // last level the position of its first member
                rec[t.off[l] + (uint64_t)cur[l] * t.rw[l]] = l + 1 < H ? (uint32_t)(cur[l + 1] + 1) : (uint32_t)i;
            }
            const uint32_t c = (uint32_t)(a >> t.shift[l]) & ((1u << t.w[l]) - 1u);
            rec[t.off[l] + (uint64_t)cur[l] * t.rw[l] + map_offset(t.rw[l]) + (c >> 5)] |= 1u << (c & 31);
        }
    }
    // prefix bytes: set bits of the map words before each word
    const uint32_t map_words = ((1u << kw) + 31) / 32;
    if (map_words > 1)
        for (int l = 0; l < H; ++l)
            for (uint64_t nd = 0; nd < nodes[l]; ++nd) {
                uint32_t *r = rec.data() + t.off[l] + nd * t.rw[l];
                const uint32_t *m = r + map_offset(t.rw[l]);
                uint32_t run = 0;
                for (uint32_t w = 0; w < map_words; ++w) {
                    r[1 + w / 4] |= run << (8 * (w % 4));
                    run += (uint32_t)__builtin_popcount(m[w]);
                }
            }
    MBR_TRY(t.table.alloc(words * 4));
    MBR_HIP(hipMemcpy(t.table.p, rec.data(), words * 4, hipMemcpyHostToDevice));
    uint64_t lw = 0;
    int ll = 0;
    while (ll < H && (t.off[ll + 1]) * 4 <= kLdsBudget) {
        lw = t.off[ll + 1];
        ++ll;
    }
    t.lds_levels = ll;
    t.lds_words = lw;
    return MBR_OK;
}

template <class P>
mbr_status launch_bt(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out, hipStream_t s) {
    const BitmapTrie &t = *r->btrie;
    BtArgs a{};
    a.rec = t.table.as<uint32_t>();
    a.M = t.M;
    a.H = t.H;
    a.lds_levels = t.lds_levels;
    a.lds_words = (uint32_t)t.lds_words;
    for (int l = 0; l < t.H; ++l) {
        a.off[l] = (uint32_t)t.off[l];
        a.shift[l] = (uint32_t)t.shift[l];
        a.cmask[l] = (1u << t.w[l]) - 1u;
    }
    const unsigned grid = mbr::grid_for(n, kBlock * kQ, mbr::device_cu_count() * 8);
    const size_t lds = (size_t)t.lds_words * 4;
    const P *qp = static_cast<const P *>(q);
    switch (t.rw[0]) {
    case 2: bt_rank_kernel<P, 2><<<grid, kBlock, lds, s>>>(qp, n, out, a); break;
    case 4: bt_rank_kernel<P, 4><<<grid, kBlock, lds, s>>>(qp, n, out, a); break;
    case 8: bt_rank_kernel<P, 8><<<grid, kBlock, lds, s>>>(qp, n, out, a); break;
    default: bt_rank_kernel<P, 16><<<grid, kBlock, lds, s>>>(qp, n, out, a); break;
    }
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

}  // namespace

void bitmap_trie_free(BitmapTrie *t) { delete t; }

mbr_status rank_bitmap_trie_launch(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out,
                                   hipStream_t s) {
    if (r->width_bits == 32) return launch_bt<uint32_t>(r, q, n, out, s);
    return launch_bt<uint64_t>(r, q, n, out, s);
}

extern "C" mbr_status mbr_build_bitmap_trie(const mbr_sector *sec, int32_t k, mbr_ranker **out, void *stream) {
    using namespace mbr;
    if (!out) MBR_FAIL(MBR_EINVAL, "null output handle");
    *out = nullptr;
    if (!sec) MBR_FAIL(MBR_EINVAL, "null sector");
    if (k < 1 || k > 8) MBR_FAIL(MBR_EINVAL, "k=%d outside 1..8", k);
    if (sec->n == 0) MBR_FAIL(MBR_EINVAL, "empty sector");
    if (sec->n >= 0xFFFFFFFFull) MBR_FAIL(MBR_ERANGE, "sector of %llu states", (unsigned long long)sec->n);
    const int M = sec->M;
    const int H = (M + k - 1) / k;
    if (H > kMaxH) MBR_FAIL(MBR_EUNSUPPORTED, "%d levels (at most %d)", H, kMaxH);
    hipStream_t s = as_stream(stream);
    auto t = std::make_unique<BitmapTrie>();
    t->M = M;
    t->H = H;
    // widths from the top: the short chunk first, then k bits each
    for (int l = 0, below = M; l < H; ++l) {
        t->w[l] = l == 0 ? M - (H - 1) * k : k;
        below -= t->w[l];
        t->shift[l] = below;
    }
    mbr_status st;
    if (sec->width_bits == 32) {
        std::vector<uint32_t> h(sec->n);
        MBR_HIP(hipMemcpyAsync(h.data(), sec->states.p, sec->n * 4, hipMemcpyDeviceToHost, s));
        MBR_HIP(hipStreamSynchronize(s));
        st = build_records<uint32_t>(*t, h);
    } else {
        std::vector<uint64_t> h(sec->n);
        MBR_HIP(hipMemcpyAsync(h.data(), sec->states.p, sec->n * 8, hipMemcpyDeviceToHost, s));
        MBR_HIP(hipStreamSynchronize(s));
        st = build_records<uint64_t>(*t, h);
    }
    if (st != MBR_OK) return st;
    auto *r = new (std::nothrow) mbr_ranker;
    if (!r) MBR_FAIL(MBR_ENOMEM, "host allocation");
    r->kind = MBR_RANKER_BITMAP_TRIE;
    r->M = M;
    r->k = k;
    r->width_bits = sec->width_bits;
    r->n_states = sec->n;
    r->sector = sec;
    (void)hipGetDevice(&r->device);
    r->btrie = t.release();
    *out = r;
    return MBR_OK;
}

extern "C" mbr_status mbr_bitmap_trie_levels(const mbr_ranker *r, uint64_t *records, uint32_t *record_bytes,
                                             int32_t cap, int32_t *levels, int32_t *lds_levels) {
    if (!r || r->kind != MBR_RANKER_BITMAP_TRIE || !r->btrie) MBR_FAIL(MBR_EINVAL, "not a bitmap trie ranker");
    const BitmapTrie &t = *r->btrie;
    if (levels) *levels = t.H;
    if (lds_levels) *lds_levels = t.lds_levels;
    for (int l = 0; l < t.H && l < cap; ++l) {
        if (records) records[l] = t.nodes[l];
        if (record_bytes) record_bytes[l] = 4 * t.rw[l];
    }
    return MBR_OK;
}
