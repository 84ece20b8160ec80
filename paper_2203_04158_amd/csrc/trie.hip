// Packed radix-2^k tries (Sec. IV) for ranking in arbitrary sectors.
//
// Dispatch order is the paper's: chunk 0 holds the k least significant bits,
// chunk l the next k bits, and a final chunk the remaining M mod k bits, so a
// lookup is the chain of the trie-lookup figure: n <- T_0[chunk_0]; n <-
// T_l[n + chunk_l] for the middle levels; rank <- T_{H-1}[n + chunk_{H-1}].
//
// Layout (GPU-specific, not the paper's single depth-first array): one array
// per level, nodes of a level contiguous in the order of their prefixes, each
// node spanning only its first..last occurring chunk value (packing), the
// parent storing start - first (the index shifted back, as in the paper's
// packed form).  Each level array starts with 2^w - 1 zeros and ends with 2^w
// zeros, so stored indices are never negative and a walk with any pattern,
// member or not, stays inside the arrays; unused slots hold 0.  The root is a
// full 2^w0 array.  Membership: the walk's rank i is accepted only when
// i < N_s and states[i] == alpha (the check of Sec. IV).
//
// Level-major arrays keep every level's nodes together: the top levels fit
// LDS and are staged there, the middle levels stay in L2/MALL and only the
// leaf level and the membership check are HBM gathers.
#include <algorithm>
#include <cstring>
#include <memory>

#include "rank_device.hpp"

void trie_free(TrieLevels *t) { delete t; }
uint64_t trie_bytes(const TrieLevels *t) { return t ? t->entries * 4 : 0; }
int32_t trie_levels(const TrieLevels *t) { return t ? t->H : 0; }

namespace {

constexpr unsigned kBlock = 256;
constexpr size_t kLdsBudget = 48 * 1024;  // bytes of top levels staged per workgroup
constexpr int kQ = 4;                       // independent walks in flight per lane

struct TrieArgs {
    const uint32_t *tab;
    const void *states;
    uint64_t ns;
    int32_t M, H;
    uint32_t lds_entries;
    int32_t lds_levels;
    uint32_t wmask[16];
    int32_t shift[16];
    uint64_t off[17];
};

template <class P>
__device__ __forceinline__ bool fits(P x, int M) {
    return (M >= (int)(8 * sizeof(P))) ? true : (x >> M) == 0;
}

template <class P>
__global__ void __launch_bounds__(kBlock) trie_rank_kernel(const P *__restrict__ q, uint64_t n,
                                                           uint32_t *__restrict__ out, TrieArgs a) {
    extern __shared__ __align__(16) uint32_t top[];
    stage_to_lds(top, a.tab, (uint64_t)a.lds_entries * 4);
    __syncthreads();
    const P *states = static_cast<const P *>(a.states);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; base < n;
         base += stride * kQ) {
        P x[kQ];
        uint32_t node[kQ];
        bool ok[kQ];
#pragma unroll
        for (int u = 0; u < kQ; ++u) {
            const uint64_t j = base + u * stride;
            x[u] = j < n ? q[j] : (P)0;
            ok[u] = j < n && fits(x[u], a.M);
            if (!ok[u]) x[u] = 0;
            node[u] = 0;
        }
        // the walks of kQ queries advance level by level side by side; the
        // staged levels and the rest are separate loops, so that LDS is read
        // with LDS loads and the arrays with global loads (one loop choosing
        // per level compiles to flat loads for both)
        int l = 0;
        for (; l < a.lds_levels; ++l) {
#pragma unroll
            for (int u = 0; u < kQ; ++u) {
                const uint32_t c = (uint32_t)(x[u] >> a.shift[l]) & a.wmask[l];
                node[u] = top[a.off[l] + node[u] + c];
            }
        }
        for (; l < a.H; ++l) {
            const uint32_t *lv = a.tab + a.off[l];
#pragma unroll
            for (int u = 0; u < kQ; ++u) {
                const uint32_t c = (uint32_t)(x[u] >> a.shift[l]) & a.wmask[l];
                node[u] = lv[node[u] + c];
            }
        }
        P hit[kQ];
#pragma unroll
        for (int u = 0; u < kQ; ++u) hit[u] = node[u] < a.ns ? states[node[u]] : (P)~x[u];
#pragma unroll
        for (int u = 0; u < kQ; ++u) {
            const uint64_t j = base + u * stride;
            if (j < n) out[j] = (ok[u] && hit[u] == x[u]) ? node[u] : MBR_NOT_FOUND;
        }
    }
}

// LSD radix sort of (key, index) pairs by key.
template <class K>
void radix_sort_pairs(std::vector<K> &key, std::vector<uint32_t> &idx, int key_bits) {
    const size_t n = key.size();
    std::vector<K> k2(n);
    std::vector<uint32_t> i2(n);
    const int D = 11;
    for (int sh = 0; sh < key_bits; sh += D) {
        std::vector<size_t> cnt((1u << D) + 1, 0);
        for (size_t i = 0; i < n; ++i) ++cnt[((key[i] >> sh) & ((1u << D) - 1)) + 1];
        for (size_t d = 0; d < (1u << D); ++d) cnt[d + 1] += cnt[d];
        for (size_t i = 0; i < n; ++i) {
            size_t p = cnt[(key[i] >> sh) & ((1u << D) - 1)]++;
            k2[p] = key[i];
            i2[p] = idx[i];
        }
        key.swap(k2);
        idx.swap(i2);
    }
}

template <class P>
mbr_status build_levels(TrieLevels &t, const std::vector<P> &states) {
    const int M = t.M, H = t.H;
    const size_t n = states.size();
    // chunk-reversed key: chunk 0 becomes the most significant field, so the
    // key order groups patterns by their low-bit prefixes at every level
    std::vector<P> key(n);
    std::vector<uint32_t> idx(n);
    for (size_t i = 0; i < n; ++i) {
        P a = states[i], k = 0;
        int top = M;
        for (int l = 0; l < H; ++l) {
            top -= t.w[l];
            P c = (a >> t.shift[l]) & (P)((1ull << t.w[l]) - 1);
            k |= c << top;
        }
        key[i] = k;
        idx[i] = (uint32_t)i;
    }
    radix_sort_pairs(key, idx, M);
    // field of level l in the key: bits [kb[l], kb[l] + w[l])
    std::vector<int> kb(H);
    {
        int top = M;
        for (int l = 0; l < H; ++l) {
            top -= t.w[l];
            kb[l] = top;
        }
    }
    auto prefix = [&](P k, int l) -> P { return l == 0 ? (P)0 : (P)(k >> (kb[l - 1])); };
    auto chunk = [&](P k, int l) -> uint32_t { return (uint32_t)((k >> kb[l]) & (P)((1ull << t.w[l]) - 1)); };
    // pass 1: node spans and starts per level
    std::vector<std::vector<uint32_t>> nfirst(H), nbase(H);
    uint64_t total = 0;
    for (int l = 0; l < H; ++l) {
        const uint64_t W = 1ull << t.w[l];
        uint64_t pos;
        t.off[l] = total;
        if (l == 0) {
            nfirst[0].push_back(0);
            nbase[0].push_back(0);
            pos = W;
        } else {
            pos = W - 1;  // front padding
            size_t i = 0;
            while (i < n) {
                const P pf = prefix(key[i], l);
                size_t j = i;
                while (j + 1 < n && prefix(key[j + 1], l) == pf) ++j;
                const uint32_t f = chunk(key[i], l), la = chunk(key[j], l);
                nfirst[l].push_back(f);
                nbase[l].push_back((uint32_t)(pos - f));
                pos += (uint64_t)(la - f) + 1;
                i = j + 1;
            }
            pos += W;  // tail padding
        }
        if (pos > 0xFFFFFFFFull) MBR_FAIL(MBR_ERANGE, "trie level %d has %llu entries", l, (unsigned long long)pos);
        total += pos;
    }
    t.off[H] = total;
    t.entries = total;
    std::vector<uint32_t> tab(total, 0);
    // pass 2: entries; the p-th distinct (prefix, chunk) pair of level l is
    // node p of level l + 1
    for (int l = 0; l < H; ++l) {
        uint32_t *lv = tab.data() + t.off[l];
        size_t node = 0, pair = 0;
        size_t i = 0;
        while (i < n) {
            const P pf = prefix(key[i], l);
            size_t j = i;
            while (j < n && prefix(key[j], l) == pf) {
                const uint32_t c = chunk(key[j], l);
                size_t e = j;
                while (e + 1 < n && prefix(key[e + 1], l) == pf && chunk(key[e + 1], l) == c) ++e;
                const uint64_t slot = (uint64_t)nbase[l][node] + c;
                lv[slot] = (l == H - 1) ? idx[j] : nbase[l + 1][pair];
                ++pair;
                j = e + 1;
            }
            ++node;
            i = j;
        }
    }
    // stage the top levels in LDS while they fit
    t.lds_levels = 0;
    t.lds_entries = 0;
    for (int l = 0; l < H; ++l) {
        if (t.off[l + 1] * 4 > kLdsBudget) break;
        t.lds_levels = l + 1;
        t.lds_entries = t.off[l + 1];
    }
    return mbr::upload(t.table, tab.data(), tab.size() * 4, nullptr);
}

template <class P>
mbr_status launch_trie(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out, hipStream_t s) {
    const TrieLevels &t = *r->trie;
    TrieArgs a{};
    a.tab = t.table.as<uint32_t>();
    a.states = r->sector->states.p;
    a.ns = r->sector->n;
    a.M = t.M;
    a.H = t.H;
    a.lds_entries = (uint32_t)t.lds_entries;
    a.lds_levels = (int32_t)t.lds_levels;
    for (int l = 0; l < t.H; ++l) {
        a.wmask[l] = (uint32_t)((1ull << t.w[l]) - 1);
        a.shift[l] = t.shift[l];
        a.off[l] = t.off[l];
    }
    a.off[t.H] = t.off[t.H];
    const size_t lds = t.lds_entries * 4;
    const unsigned grid = mbr::grid_for(n, kBlock * kQ, mbr::device_cu_count() * 8);
    trie_rank_kernel<P><<<grid, kBlock, lds, s>>>(static_cast<const P *>(q), n, out, a);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

}  // namespace

mbr_status rank_trie_launch(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out,
                            hipStream_t s) {
    if (r->width_bits == 32) return launch_trie<uint32_t>(r, q, n, out, s);
    return launch_trie<uint64_t>(r, q, n, out, s);
}

extern "C" mbr_status mbr_trie_level_entries(const mbr_ranker *r, uint64_t *entries, int32_t cap,
                                             int32_t *levels, int32_t *lds_levels) {
    if (!r || r->kind != MBR_RANKER_TRIE || !r->trie) MBR_FAIL(MBR_EINVAL, "not a trie ranker");
    const TrieLevels &t = *r->trie;
    if (levels) *levels = t.H;
    if (lds_levels) *lds_levels = (int32_t)t.lds_levels;
    if (entries)
        for (int l = 0; l < t.H && l < cap; ++l) entries[l] = t.off[l + 1] - t.off[l];
    return MBR_OK;
}

extern "C" mbr_status mbr_build_trie(const mbr_sector *sec, int32_t k, mbr_ranker **out,
                                     void *stream) {
    using namespace mbr;
    if (!out) MBR_FAIL(MBR_EINVAL, "null output handle");
    *out = nullptr;
    if (!sec) MBR_FAIL(MBR_EINVAL, "null sector");
    if (k < 1 || k > 16) MBR_FAIL(MBR_EINVAL, "k=%d outside 1..16", k);
    const int M = sec->M;
    const int H = (M + k - 1) / k;
    if (H > 16) MBR_FAIL(MBR_EUNSUPPORTED, "%d levels (at most 16)", H);
    if (sec->n == 0) MBR_FAIL(MBR_EINVAL, "empty sector");
    hipStream_t s = as_stream(stream);
    auto t = std::make_unique<TrieLevels>();
    t->M = M;
    t->H = H;
    t->width_bits = sec->width_bits;
    for (int l = 0, b = 0; l < H; ++l) {
        t->w[l] = std::min(k, M - b);
        t->shift[l] = b;
        b += t->w[l];
    }
    mbr_status st;
    if (sec->width_bits == 32) {
        std::vector<uint32_t> h(sec->n);
        MBR_HIP(hipMemcpyAsync(h.data(), sec->states.p, sec->n * 4, hipMemcpyDeviceToHost, s));
        MBR_HIP(hipStreamSynchronize(s));
        st = build_levels<uint32_t>(*t, h);
    } else {
        std::vector<uint64_t> h(sec->n);
        MBR_HIP(hipMemcpyAsync(h.data(), sec->states.p, sec->n * 8, hipMemcpyDeviceToHost, s));
        MBR_HIP(hipStreamSynchronize(s));
        st = build_levels<uint64_t>(*t, h);
    }
    if (st != MBR_OK) return st;
    auto *r = new (std::nothrow) mbr_ranker;
    if (!r) MBR_FAIL(MBR_ENOMEM, "host allocation");
    r->kind = MBR_RANKER_TRIE;
    r->M = M;
    r->k = k;
    r->width_bits = sec->width_bits;
    r->n_states = sec->n;
    r->sector = sec;
    (void)hipGetDevice(&r->device);
    r->trie = t.release();
    *out = r;
    return MBR_OK;
}
