// Device-side rank helpers shared by the batched rank kernels and the
// generic operator: the staggered lookup (Fig. fastrank) and a single trie
// walk with its membership check (Fig. trielookup, safe lookup of Sec. IV).
#pragma once

#include "common.hpp"

struct StagArgs {
    int32_t M, k, nch, N;
    int32_t rowoff[16];
    uint64_t nentries;
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
