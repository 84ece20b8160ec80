// Device-side rank helpers shared by the batched rank kernels and the
// generic operator: the staggered lookup (Fig. fastrank) and a single trie
// walk with its membership check (Fig. trielookup, safe lookup of Sec. IV).
#pragma once

#include "common.hpp"

struct StagArgs {
    int32_t M, k, nch, N;
    int32_t rowoff[16];  // row of (chunk c, N' = 0); may be negative for a trimmed table
    uint64_t nentries;
    uint64_t safe;       // pattern ranked in place of a non-member (its rows exist)
};

template <class P>
__device__ __forceinline__ bool below_width(P x, int M) {
    return (M >= (int)(8 * sizeof(P))) ? true : (x >> M) == 0;
}

// Rank of x within its own particle-number block, Fig. fastrank: add the
// partial rank of each k-bit chunk, advancing N' by the chunk's popcount.
// `tab` is the table (LDS copy or global).
template <class P, class E>
__device__ __forceinline__ uint64_t stag_rank(P x, const E *tab, const StagArgs &a) {
    uint64_t rank = 0;
    int np = 0;
    const P cm = (P)((1ull << a.k) - 1);
#pragma unroll 4
    for (int c = 0; c < a.nch; ++c) {
        P r = (x >> (c * a.k)) & cm;
        rank += (uint64_t)tab[((uint32_t)(a.rowoff[c] + np) << a.k) + (uint32_t)r];
        np += (sizeof(P) == 8) ? __popcll((uint64_t)r) : __popc((uint32_t)r);
    }
    return rank;
}

// Copy `bytes` from global memory to LDS with 16-byte accesses (both
// addresses 16-byte aligned), four in flight per lane before the first store,
// then the tail by 4-byte words (bytes is a multiple of 4).  No barrier.
__device__ __forceinline__ void stage_to_lds(void *lds, const void *__restrict__ g, uint64_t bytes) {
    const uint4 *src = static_cast<const uint4 *>(g);
    uint4 *dst = static_cast<uint4 *>(lds);
    const uint64_t n16 = bytes >> 4;
    uint64_t i = threadIdx.x;
    for (; i + 3 * blockDim.x < n16; i += 4 * blockDim.x) {
        const uint4 v0 = src[i], v1 = src[i + blockDim.x], v2 = src[i + 2 * blockDim.x], v3 = src[i + 3 * blockDim.x];
        dst[i] = v0;
        dst[i + blockDim.x] = v1;
        dst[i + 2 * blockDim.x] = v2;
        dst[i + 3 * blockDim.x] = v3;
    }
    for (; i < n16; i += blockDim.x) dst[i] = src[i];
    const uint32_t *s4 = static_cast<const uint32_t *>(g);
    uint32_t *d4 = static_cast<uint32_t *>(lds);
    for (uint64_t k = (n16 << 2) + threadIdx.x; k < (bytes >> 2); k += blockDim.x) d4[k] = s4[k];
}

// A trie in the level-major layout of trie.hip, read from global memory.
struct TrieWalk {
    const uint32_t *tab;
    const void *states;
    uint64_t ns;
    int32_t M, H;
    uint32_t wmask[16];
    int32_t shift[16];
    uint64_t off[17];
};

// Rank of x in the trie's sector, or MBR_NOT_FOUND: the level walk, then the
// membership check against the state list.  Every read stays in bounds for
// any x (the levels are padded).
template <class P>
__device__ __forceinline__ uint32_t trie_rank_one(P x, const TrieWalk &a) {
    if (!below_width(x, a.M)) return MBR_NOT_FOUND;
    uint32_t node = 0;
    for (int l = 0; l < a.H; ++l) node = a.tab[a.off[l] + node + ((uint32_t)(x >> a.shift[l]) & a.wmask[l])];
    const P *st = static_cast<const P *>(a.states);
    return (node < a.ns && st[node] == x) ? node : MBR_NOT_FOUND;
}
