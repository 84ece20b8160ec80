// Internal declarations shared by the mbrank translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/mbrank.h"

namespace mbr {

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();

#define MBR_FAIL(code, ...)          \
    do {                             \
        ::mbr::set_error(__VA_ARGS__); \
        return (code);               \
    } while (0)

#define MBR_HIP(call)                                                               \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) {                                                     \
            ::mbr::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                             __FILE__, __LINE__);                                   \
            return MBR_EHIP;                                                        \
        }                                                                           \
    } while (0)

#define MBR_TRY(expr)                 \
    do {                              \
        mbr_status s_ = (expr);       \
        if (s_ != MBR_OK) return s_;  \
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ---------------------------------------------------------------- device buffer
// Owning device allocation used by handles (tables, lists, work space).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes) {
        o.p = nullptr;
        o.bytes = 0;
    }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            bytes = o.bytes;
            o.p = nullptr;
            o.bytes = 0;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    mbr_status alloc(size_t n) {
        release();
        if (n == 0) n = 16;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            set_error("hipMalloc(%zu) failed: %s", n, hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? MBR_ENOMEM : MBR_EHIP;
        }
        bytes = n;
        return MBR_OK;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Allocate and fill from host synchronously on `stream`.
mbr_status upload(DevBuf &b, const void *host, size_t bytes, hipStream_t stream);

// ---------------------------------------------------------------- binomials
// Exact C(n, k) for 0 <= n, k <= 64 (0 when k > n), host side.
uint64_t binom(int n, int k);

// Device copy of the same table (65 x 65 uint64, row n, column k) on the
// current device; uploaded on first use and kept until the process ends.
mbr_status device_binom(const uint64_t **d_table);

// ---------------------------------------------------------------- handles
struct mbr_sector_impl;
int device_cu_count();

// Launch geometry helper: number of workgroups for a grid-stride kernel.
inline unsigned grid_for(uint64_t work, unsigned per_block, unsigned max_blocks) {
    uint64_t b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return static_cast<unsigned>(b);
}

}  // namespace mbr

// Opaque handle definitions (C-ABI names).
struct mbr_sector {
    int32_t M = 0;
    int32_t width_bits = 32;
    uint64_t n = 0;
    int device = 0;
    std::vector<mbr_popc_cons> cons;
    int32_t modulus = 0, residue = 0;  // modular weight constraint (modulus 0: none)
    std::vector<int32_t> weights;      // orbital weights mod modulus (modulus > 0)
    bool from_list = false;            // adopted from a caller's list: no constraint describes it
    mbr::DevBuf states;
};

// Staggered table description, shared by the staggered, spin and Hubbard paths.
struct StagTable {
    int32_t M = 0, k = 0, nmax = 0, nch = 0;
    int32_t entry_bytes = 4;  // 2, 4 or 8
    int32_t rowoff[65] = {0};  // row index of (chunk c, N' = 0)
    int32_t nrows = 0;
    mbr::DevBuf table;         // nrows << k entries
    std::vector<uint64_t> host; // same entries as uint64
    // Fixed particle number N: only the rows a member can reach, N' in
    // [max(0, N - (M - c k)), min(c k, N)] for chunk c; trim_rowoff[c] is the
    // row of N' = 0 in that copy (negative when the first rows are cut).
    mbr::DevBuf trim;
    int32_t trim_rowoff[65] = {0};
    uint64_t trim_entries = 0;
};

mbr_status stag_build(StagTable &t, int32_t M, int32_t k, int32_t nmax, int32_t entry_bytes,
                      hipStream_t stream);

// Packed trie, one uint32 array per level (level-major layout of trie.hip).
struct TrieLevels {
    int32_t M = 0, H = 0, width_bits = 32;
    int32_t w[64] = {0};       // chunk widths, least significant first
    int32_t shift[64] = {0};   // bit offset of chunk l in the pattern
    uint64_t off[65] = {0};    // level l occupies entries off[l] .. off[l+1]-1
    uint64_t entries = 0;
    uint64_t lds_levels = 0;   // levels 0..lds_levels-1 are staged in LDS
    uint64_t lds_entries = 0;
    mbr::DevBuf table;         // uint32 entries of all levels
};

// Bitmap trie (bitmap_trie.hip): records {base, bitmap} per node, levels
// from the most significant chunk.
struct BitmapTrie {
    int32_t M = 0, H = 0;
    int32_t w[32] = {0};        // chunk widths, most significant first
    int32_t shift[32] = {0};    // bit offset of chunk l in the pattern
    uint32_t rw[32] = {0};      // record words of level l
    uint64_t off[33] = {0};     // first word of level l (64-byte aligned)
    uint64_t nodes[32] = {0};   // records of level l
    int32_t lds_levels = 0;     // levels 0..lds_levels-1 are staged in LDS
    uint64_t lds_words = 0;
    mbr::DevBuf table;
};

struct LearnedModel;

struct mbr_ranker {
    int32_t kind = 0;
    int32_t M = 0, k = 0, width_bits = 32;
    int32_t N = -1;            // staggered: particle number or -1
    int32_t n_up = 0, n_dn = 0, L = 0;  // spin ranker
    uint64_t n_states = 0;
    bool rank64 = false;       // staggered: ranks only fit the 64-bit entry point
    int device = 0;
    StagTable stag;            // staggered, spin halves
    mbr::DevBuf unrank_tab;    // spin: half lists (uint16) or binomial table for unranking
    bool unrank_lists = false; // spin: unrank_tab holds the half lists
    TrieLevels *trie = nullptr;
    BitmapTrie *btrie = nullptr;
    LearnedModel *learned = nullptr;
    const mbr_sector *sector = nullptr;
    const mbr_ranker *fallback = nullptr;
    ~mbr_ranker();
};

// Per-kind rank launchers (defined in their translation units).
mbr_status rank_staggered_launch(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out,
                                 hipStream_t s);
mbr_status rank_spin_launch(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out,
                            hipStream_t s);
mbr_status rank_trie_launch(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out,
                            hipStream_t s);
mbr_status rank_learned_launch(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out,
                               hipStream_t s);
mbr_status rank_staggered_launch64(const mbr_ranker *r, const void *q, uint64_t n, uint64_t *out,
                                   hipStream_t s);
mbr_status rank_bisect_launch(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out,
                              hipStream_t s);
// Unranking tables of a spin ranker (unrank.hip).
mbr_status spin_unrank_build(mbr_ranker *r, hipStream_t s);
mbr_status rank_cns_launch(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out,
                           hipStream_t s);
void trie_free(TrieLevels *t);
void bitmap_trie_free(BitmapTrie *t);
mbr_status rank_bitmap_trie_launch(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out,
                                   hipStream_t s);
uint64_t trie_bytes(const TrieLevels *t);
int32_t trie_levels(const TrieLevels *t);
void learned_free(LearnedModel *m);
uint64_t learned_bytes(const LearnedModel *m);
int32_t learned_levels(const LearnedModel *m);  // sampled copies + the list
