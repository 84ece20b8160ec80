/*
 * mbrank — ranking of many-body occupation patterns, on-the-fly Hubbard H·x and
 * Lanczos ground-state search on AMD Instinct MI355X (gfx950).
 *
 * Method: M. Wallerberger and K. Held, "Trie-based ranking of quantum many-body
 * states", arXiv:2203.04158.  Section/equation references below are to that paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - A state is an M-bit occupation pattern: bit i is orbital i (Sec. II).  Patterns
 *    are passed as uint32 (M <= 32) or uint64 (M <= 64) arrays; `width_bits` (32|64)
 *    names which.  For the spin-resolved Hamiltonians orbital i (< L) is site i
 *    spin-down and orbital L+i is site i spin-up (spin-down in the least
 *    significant bits, as assumed for Eq. rankupdown).
 *  - A sector is the set of patterns satisfying a list of popcount windows,
 *    ordered by ascending numeric value, which is the lexicographic order of
 *    Sec. III (c_N first).  rank(alpha) is the position of alpha in that order.
 *  - Every call returns an mbr_status; 0 is success and the negative codes are
 *    listed below.  mbr_last_error() returns a text for the last failing call of
 *    the calling thread.
 *  - Pointers named d_* are device pointers (HIP device memory) owned by the
 *    caller, who keeps them alive until the work queued on `stream` completes.
 *    Other pointers are host memory, read during the call only.
 *  - Handles (mbr_sector, mbr_ranker, mbr_hubbard, mbr_lanczos) are opaque,
 *    owned by the library, hold their own device tables, and are released with
 *    the matching *_destroy.  A handle lives on the device that was current when
 *    it was created.  Read-only use of one handle from several streams is safe.
 *  - `stream` is a hipStream_t passed as void*; NULL is the null stream.  Batched
 *    calls only enqueue work (no host synchronisation) unless stated otherwise.
 *  - Per-element failures are sentinels, not status codes: a pattern outside the
 *    ranker's sector ranks to MBR_NOT_FOUND (all patterns with bits at or above M,
 *    with the wrong particle numbers, or absent from a trie's sector); an unrank
 *    index >= the sector size yields an all-ones pattern.
 */
#ifndef MBRANK_H
#define MBRANK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mbr_status;
#define MBR_OK            0
#define MBR_EINVAL       (-1) /* argument outside its documented range */
#define MBR_ENOMEM       (-2) /* device or host allocation failed */
#define MBR_EHIP         (-3) /* a HIP runtime call failed */
#define MBR_ENOTSORTED   (-4) /* caller-supplied state list not strictly ascending */
#define MBR_EDUP         (-5) /* caller-supplied state list has a repeated entry */
#define MBR_ERANGE       (-6) /* an index or size exceeds what the handle supports */
#define MBR_EUNSUPPORTED (-7) /* valid request the library does not implement */

#define MBR_NOT_FOUND 0xFFFFFFFFu

/* Text for a status code (static storage). */
const char *mbr_status_str(mbr_status s);
/* Detail of the last failing call on this thread ("" if none). */
const char *mbr_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int32_t mbr_version(void);

/* ======================================================================== */
/* Sectors (Sec. II: particle-number blocks, Eq. mvblock; Sec. IV: further   */
/* quantum numbers by filtering)                                            */
/* ======================================================================== */

/* Popcount window: lo <= popcount(alpha AND mask) <= hi. */
typedef struct {
    uint64_t mask;
    int32_t lo;
    int32_t hi;
} mbr_popc_cons;

typedef struct mbr_sector mbr_sector;

/* Enumerate, on the device, every M-bit pattern that satisfies all n_cons
 * windows, in ascending order (this list is the unrank table, Sec. II and
 * Sec. III.A).  M in 1..64; width_bits 32 (needs M <= 32) or 64.  If the windows
 * fix the total particle number (one window on all M bits with lo == hi, or
 * disjoint fixed windows covering all M bits) only the C(M,N) patterns of that
 * number are visited; otherwise M <= 32 and all 2^M patterns are tested.
 * Sectors must hold fewer than 2^32 - 1 states (ERANGE).  Synchronises `stream`
 * (the size must be known to allocate).  *out receives the handle. */
mbr_status mbr_sector_build(int32_t M, int32_t width_bits, int32_t n_cons,
                            const mbr_popc_cons *cons, mbr_sector **out, void *stream);

/* As mbr_sector_build, plus one modular constraint: the weights of the set
 * bits add up to `residue` modulo `modulus` (weights[i] for orbital i, M
 * entries).  With orbital weights equal to lattice momenta this gives the
 * total-momentum sectors of a translation-invariant ring (Sec. V.C, the
 * K_tot sets of Sec. IV). */
mbr_status mbr_sector_build_mod(int32_t M, int32_t width_bits, int32_t n_cons, const mbr_popc_cons *cons,
                                const int32_t *weights, int32_t modulus, int32_t residue,
                                mbr_sector **out, void *stream);

/* Adopt a sector the caller has listed (Sec. IV, last paragraph: sets that
 * only a filter describes, such as the total-momentum blocks, are fed to the
 * trie builder in ascending order).  d_states holds n patterns (device memory,
 * uint32 or uint64 per width_bits, M in 1..64, M <= 32 for 32-bit patterns);
 * they are copied into a new library-owned sector, so the caller may free
 * them on return.  The copy is checked on the device, and the first offending
 * position j decides the status: MBR_ENOTSORTED when entry j is smaller than
 * entry j-1, MBR_EDUP when it equals entry j-1, MBR_EINVAL when entry j has
 * bits at or above M (order is checked before width at one position).
 * MBR_ERANGE for n >= 2^32 - 1.  n = 0 gives an empty sector.  No popcount
 * window describes such a sector, so operators on it always check membership.
 * Synchronises `stream`.  *out receives the handle. */
mbr_status mbr_sector_from_list(int32_t M, int32_t width_bits, const void *d_states, uint64_t n,
                                mbr_sector **out, void *stream);

/* Number of states in the sector. */
mbr_status mbr_sector_size(const mbr_sector *s, uint64_t *n);

/* Borrowed device pointer to the ascending state list (uint32 or uint64 per
 * width_bits), valid until mbr_sector_destroy. */
mbr_status mbr_sector_states(const mbr_sector *s, const void **d_states);

mbr_status mbr_sector_destroy(mbr_sector *s);

/* Unrank by the stored list (Sec. II): d_out[j] = states[d_idx[j]] for j < n,
 * or all ones when d_idx[j] >= size.  d_out has the sector's width. */
mbr_status mbr_unrank_batch(const mbr_sector *s, const uint32_t *d_idx, uint64_t n,
                            void *d_out, void *stream);

/* ======================================================================== */
/* Rankers                                                                   */
/* ======================================================================== */

typedef struct mbr_ranker mbr_ranker;

#define MBR_RANKER_STAGGERED 1
#define MBR_RANKER_SPIN      2
#define MBR_RANKER_TRIE      3
#define MBR_RANKER_LEARNED   4
#define MBR_RANKER_BISECT    5
#define MBR_RANKER_CNS       6
#define MBR_RANKER_SAMPLED   7
#define MBR_RANKER_BITMAP_TRIE 8

typedef struct {
    int32_t kind;       /* MBR_RANKER_* */
    int32_t M;          /* pattern length in bits */
    int32_t k;          /* chunk width (bits per lookup) */
    int32_t width_bits; /* query width: 32 or 64 */
    uint64_t n_states;  /* size of the sector ranked into */
    uint64_t bytes;     /* device bytes of the ranker's tables */
    int32_t levels;     /* lookups per query (chunks or trie levels) */
    int32_t reserved;
} mbr_ranker_info;

/* Staggered lookup (Sec. III.B, Fig. fastrank, Eq. partrank): tables of the
 * partial ranks rank(r, M', N') for chunks of k bits taken from the least
 * significant end, M' = 0, k, 2k, ..., rows N' = 0..min(M', Nmax), chunk value r
 * varying fastest; entries built through Eq. reuse.  When k does not divide M
 * the last chunk holds M mod k bits.  N >= 0 ranks within C^M_N (patterns of
 * other popcount rank to MBR_NOT_FOUND, Nmax = N); N = -1 builds the universal
 * table (Nmax = M) and ranks any pattern within its own particle-number block.
 * M in 1..64 (M <= 63 with N = -1), k in 1..16, width_bits 32|64.  When ranks
 * can reach 2^32 - 1 (large M) they are only available through
 * mbr_rank_batch64; mbr_rank_batch then returns ERANGE. */
mbr_status mbr_build_staggered_tables(int32_t M, int32_t N, int32_t k, int32_t width_bits,
                                      mbr_ranker **out, void *stream);

/* Copy a staggered ranker's table to host memory as uint64 entries:
 * entry (chunk c, N', r) is written at index (row(c, N') << k) + r with
 * row(c, N') = sum_{c' < c} (min(c' k, Nmax) + 1) + N'.  *n_entries receives
 * the count; nothing is written when host_out is NULL or cap is too small.
 * Synchronises `stream`. */
mbr_status mbr_staggered_table_copy(const mbr_ranker *r, uint64_t *host_out, uint64_t cap,
                                    uint64_t *n_entries, void *stream);

/* Spin-resolved rank (Eq. rankupdown, with the multiplier read as the number of
 * spin-down configurations): for a 2L-bit pattern with spin-down in bits 0..L-1,
 * rank = rank_{N_up}(alpha_up) * C(L, n_dn) + rank_{N_dn}(alpha_dn), each half
 * ranked by the staggered lookup with chunk width k.  L in 1..32. */
mbr_status mbr_build_spin_ranker(int32_t L, int32_t n_up, int32_t n_dn, int32_t k,
                                 mbr_ranker **out, void *stream);

/* Unrank in the spin sector of a spin ranker without its state list (the
 * inverse of Eq. rankupdown, each half by Eq. unrank):
 * d_out[j] = (half_up << L) | half_dn with half_up the (i / C(L, n_dn))-th and
 * half_dn the (i mod C(L, n_dn))-th ascending pattern of n_up (n_dn) set bits
 * among L, i = d_idx[j]; all ones when i >= C(L, n_up) C(L, n_dn).  d_out has
 * the ranker's width (32 bits for L <= 16, else 64).  The halves come from
 * lists staged in LDS when both are short (L <= 16, at most 32768 patterns
 * together), else from the greedy inversion of Eq. cns over a binomial table
 * in LDS.  EINVAL for a ranker of another kind. */
mbr_status mbr_unrank_spin_batch(const mbr_ranker *r, const uint32_t *d_idx, uint64_t n, void *d_out,
                                 void *stream);

/* Packed radix-2^k trie over a sector (Sec. IV, Fig. trie, Fig. trielookup):
 * chunks dispatched from the least significant end, one array per level, each
 * node spanning its first to last occurring child, unused slots zero and the
 * arrays padded so that any pattern's walk stays in bounds; after the walk,
 * membership is checked against the sector's list (safe lookup, Sec. IV).
 * k in 1..16.  The trie keeps a reference to `s`: destroy it before `s`. */
mbr_status mbr_build_trie(const mbr_sector *s, int32_t k, mbr_ranker **out, void *stream);

/* Bitmap trie (the radix-2^k trie of Sec. IV in a GPU layout): chunks
 * dispatched from the most significant end (the top chunk holds M mod k bits
 * when k does not divide M), every node one record of a 32-bit base, for
 * k >= 6 the set-bit counts before each 32-bit word of the map (one byte
 * each), and a 2^k-bit map of the chunk values that occur under it: 8, 16, 32
 * or 64 bytes (k <= 5, 6, 7, 8; the same size on every level) aligned to its
 * size.  The child for chunk value c is
 * record base + (set bits below c) of the next level; at the last level that
 * count gives the rank (base = position of the node's first member).  A clear
 * bit means the pattern is not in the sector, so no state list is read.
 * k in 1..8; the sector must be non-empty; the ranker keeps a reference to
 * `s` (destroy it first).  Synchronises `stream`. */
mbr_status mbr_build_bitmap_trie(const mbr_sector *s, int32_t k, mbr_ranker **out, void *stream);

/* Layout of a bitmap trie: *levels levels, the top *lds_levels of them staged
 * in LDS per workgroup; records[l] and record_bytes[l] for l < min(levels, cap). */
mbr_status mbr_bitmap_trie_levels(const mbr_ranker *r, uint64_t *records, uint32_t *record_bytes,
                                  int32_t cap, int32_t *levels, int32_t *lds_levels);

/* The established methods the paper compares against (Sec. III, Sec. V.A).
 * Bisection: lower bound of the pattern in the sector's ascending list, found
 * when the entry equals the pattern; any sector; the ranker keeps a reference
 * to `s` (destroy it first).  Combinadics: Eq. cns, the sum of C(c_k, k)
 * over the occupied positions c_1 < ... < c_N (Sec. III.A), taken position by
 * position, for the particle-number sector of N out of M orbitals; ranks
 * must fit 32 bits (ERANGE).  Both answer MBR_NOT_FOUND outside the sector. */
mbr_status mbr_build_bisect_ranker(const mbr_sector *s, mbr_ranker **out);
mbr_status mbr_build_cns_ranker(int32_t M, int32_t N, int32_t width_bits, mbr_ranker **out,
                                void *stream);

/* Device bytes of a packed or bitmap trie (all levels, padding included):
 * the memory overhead of Sec. IV is f = bytes / (4 N_s).  EINVAL for other
 * rankers. */
mbr_status mbr_trie_bytes(const mbr_ranker *r, uint64_t *bytes);

/* Layout of a trie ranker: *levels = number of levels (chunks), *lds_levels =
 * how many top levels each workgroup stages in LDS, entries[l] = uint32
 * entries of level l (padding included) for l < min(levels, cap). */
mbr_status mbr_trie_level_entries(const mbr_ranker *r, uint64_t *entries, int32_t cap,
                                  int32_t *levels, int32_t *lds_levels);

/* Learned index (extension, not in the paper): a two-stage recursive model
 * index.  Stage 1 is a 32->64->64->1 ReLU network with bf16 weights and fp32
 * accumulation that predicts y ~ rank/size from the 32 bit features; it is
 * trained on the GPU on the sector's own list (Adam, mean squared error).
 * Stage 2 has n_leaves = 2^b leaves (opts->log2_leaves, or about one per
 * four members up to 2^12); leaf floor(y 2^b) records the smallest and
 * largest rank of the members the network sends to it, measured with the
 * query kernel's own arithmetic.  A query takes the lower bound of its
 * pattern in states[lo..hi] of its leaf (through sampled copies of every
 * 16^l-th state, which the ranker holds on the device, about 1/15 of the
 * list), so ranks are exact.  The recorded
 * error e is the widest leaf window hi - lo; when it exceeds opts->max_window,
 * `fallback` answers instead (the fallback must rank the same sector; the
 * learned ranker keeps a reference to it and to `s`).  width_bits must be 32.
 * Synchronises `stream`. */
typedef struct {
    int32_t epochs;     /* passes over the sector list */
    int32_t batch;      /* samples per optimiser step (multiple of 256) */
    float lr;           /* Adam step size (cosine decay over the run) */
    uint64_t seed;      /* weight initialisation and sample order */
    uint64_t max_window;/* largest leaf window e still served by the window search */
    uint64_t samples_per_epoch; /* 0 = whole list */
    int32_t log2_leaves; /* stage-2 leaves 2^b, b in [8, 28]; 0 = about one per four members, at most 2^12 */
} mbr_learned_opts;

mbr_status mbr_learned_train(const mbr_sector *s, const mbr_learned_opts *opts,
                             const mbr_ranker *fallback, mbr_ranker **out, void *stream);

/* The learned ranker's search without its network (extension, not in the
 * paper): the lower bound of a pattern in the whole of the sector's ascending
 * list, by a bisection of the top sampled copy (every 16^H-th state, at most
 * 8192 entries, staged in LDS) and then one aligned line of 16 entries per
 * lower copy and one in the list, found when the entry equals the pattern.
 * It is what a learned ranker's windows are measured against.  width_bits
 * must be 32 and the sector size below MBR_NOT_FOUND (ERANGE); the ranker
 * keeps a reference to `s` (destroy it first) and holds the copies, about
 * 1/15 of the list, on the device.  Answers MBR_NOT_FOUND outside the sector.
 * Synchronises `stream`. */
mbr_status mbr_build_sampled_ranker(const mbr_sector *s, mbr_ranker **out, void *stream);

/* Recorded error e of a learned ranker (widest leaf window, hi - lo), and
 * whether it answers through its own window search (1) or the fallback (0). */
mbr_status mbr_learned_max_error(const mbr_ranker *r, uint64_t *e, int32_t *uses_window);

/* Tune the learned ranker's fallback threshold on the caller's queries: time
 * its window search and its fallback ranker (one untimed launch, then `reps`
 * launches each, 1..1000) on the n device queries d_q and keep the faster for
 * later calls; both give the same ranks, since the window search is exact
 * for any e.  The threshold is then e when the window search wins (it
 * serves) and e - 1 otherwise (the fallback serves).  *ms_window and
 * *ms_fallback (either may be NULL) receive the two average times.  EINVAL
 * for a ranker without a fallback or of another kind.  Synchronises
 * `stream`. */
mbr_status mbr_learned_autotune(mbr_ranker *r, const void *d_q, uint64_t n, int32_t reps,
                                double *ms_window, double *ms_fallback, void *stream);

typedef struct {
    uint64_t n_leaves;            /* stage-2 leaves (a power of two) */
    uint64_t max_window;          /* widest leaf window hi - lo (= e) */
    double mean_window;           /* mean over members of their leaf's hi - lo + 1 */
    uint64_t single_window_error; /* max |rint(size y) - rank| of stage 1 alone */
    int32_t uses_window;
} mbr_learned_info;

/* Statistics of a learned ranker's two stages. */
mbr_status mbr_learned_stats(const mbr_ranker *r, mbr_learned_info *info);

/* Copy the learned ranker's parameters to host memory as fp32 in the order
 * W1[64][32], b1[64], W2[64][64], b2[64], w3[64], b3 (6337 values); these are
 * the bf16-rounded weights the query kernel uses.  Synchronises `stream`. */
mbr_status mbr_learned_params(const mbr_ranker *r, float *host_out, void *stream);

/* Learned-network primitives exposed for checking against an fp64 reference:
 * forward pass (d_pred[B]) and mean-squared-loss gradients (d_grad[6337], same
 * order as mbr_learned_params) for B patterns d_q (uint32) and targets d_tgt,
 * with fp32 parameters d_params (rounded to bf16 inside, as in training).
 * B must be a multiple of 64. */
mbr_status mbr_mlp_forward(const float *d_params, const uint32_t *d_q, int32_t B,
                           float *d_pred, void *stream);
mbr_status mbr_mlp_gradients(const float *d_params, const uint32_t *d_q, const float *d_tgt,
                             int32_t B, float *d_grad, float *d_loss, void *stream);

/* mbr_mlp_gradients without any device allocation and without host
 * synchronisation, for callers that cannot allocate: a training step captured
 * in a HIP graph, or a loop that may not call hipMalloc.  Same arguments,
 * kernels and results as mbr_mlp_gradients; the scratch (rounded weights,
 * per-sample activations, per-64-sample gradient partials) is one static
 * device array of about 11.8 MB that each device holds until the process
 * ends, sized for B <= 8192 (MBR_ERANGE beyond).  Every scratch word a call
 * reads is written earlier in the same call, so nothing needs clearing, but
 * calls that overlap on one device (other streams, other threads) share that
 * array and race: serialise them.  Only enqueues work on `stream`. */
mbr_status mbr_mlp_gradients_noalloc(const float *d_params, const uint32_t *d_q, const float *d_tgt,
                                     int32_t B, float *d_grad, float *d_loss, void *stream);

mbr_status mbr_ranker_info_get(const mbr_ranker *r, mbr_ranker_info *info);

/* Rank n patterns: d_rank[j] = rank of d_q[j] in the ranker's sector or
 * MBR_NOT_FOUND.  d_q has the ranker's width. */
mbr_status mbr_rank_batch(const mbr_ranker *r, const void *d_q, uint64_t n, uint32_t *d_rank,
                          void *stream);

/* 64-bit ranks (Sec. III.B at M up to 64, where sectors exceed 2^32 states):
 * d_rank[j] = rank of d_q[j], or all ones outside the sector.  Staggered
 * rankers only (EUNSUPPORTED otherwise). */
mbr_status mbr_rank_batch64(const mbr_ranker *r, const void *d_q, uint64_t n, uint64_t *d_rank,
                            void *stream);

mbr_status mbr_ranker_destroy(mbr_ranker *r);

/* Rank-side autotuner: the chunk width k (the paper's R, Sec. V.A, where the
 * fastest width is a property of the machine) of one ranker kind for one
 * sector.  kind is MBR_RANKER_STAGGERED (the sector must be exactly C(M, N):
 * one window on all M bits with lo == hi, else EINVAL), MBR_RANKER_TRIE or
 * MBR_RANKER_BITMAP_TRIE.  Candidates are ks[0..n_ks) (n_ks <= 64), or with
 * n_ks = 0 {3,4,5,6,7,8,10,12,14,16}, {4,6,8,10,12} and {4,...,8} for the
 * three kinds; each is capped at M.  Every candidate is built and timed on the
 * caller's n device queries d_q (one untimed launch, then `reps` launches,
 * 1..1000, HIP events on `stream`); candidates that cannot be built or run
 * (device memory, ranks beyond 32 bits) are skipped, and when none is left
 * the first failure is returned.  *out receives the fastest ranker (the
 * caller destroys it; trie kinds keep a reference to `s`), *res its k and
 * average time.  If the environment variable MBR_AUTOTUNE_CACHE names a
 * file, an entry for this device, kind and sector description (M, width,
 * size, windows, modular weight) is used without timing and new results are
 * appended; sectors adopted from a list are never cached; malformed entries
 * are ignored.  Synchronises `stream`. */
typedef struct {
    int32_t kind;       /* the ranker kind tuned */
    int32_t k;          /* the chosen chunk width */
    double ms;          /* its time for one mbr_rank_batch of the n queries (the cached time on a hit) */
    int32_t from_cache; /* 1: read from MBR_AUTOTUNE_CACHE, nothing timed */
    int32_t tried;      /* candidates built and timed */
} mbr_rank_tuning;

mbr_status mbr_rank_autotune(const mbr_sector *s, int32_t kind, const int32_t *ks, int32_t n_ks,
                             const void *d_q, uint64_t n, int32_t reps, mbr_rank_tuning *res,
                             mbr_ranker **out, void *stream);

/* ======================================================================== */
/* General operators from non-branching terms (Sec. II, Eq. H, App. A)       */
/* ======================================================================== */

/* One term as the tuple of Eq. Talpha1 / Eq. Talpha2:
 *   T|a> = v [a & m == r] (-1)^popcount(a & s) |a ^ x>,
 *   <a|T = v [a & m == l] (-1)^popcount(a & s) <a ^ x|. */
typedef struct {
    double v;
    uint64_t m, l, r, x, s;
} mbr_term;

/* Two-body coefficient U_ijkl of Eq. H (the term (1/4) U c+_i c+_j c_l c_k). */
typedef struct {
    int32_t i, j, k, l;
    double U;
} mbr_coulomb;

typedef struct mbr_operator mbr_operator;

/* Tuples of H = -sum_ij t_ij c+_i c_j + 1/4 sum U_ijkl c+_i c+_j c_l c_k (Eq. H)
 * over M orbitals: each term's tuple is built from those of c_i and c+_i
 * (Eqs. ci) by the product rule of App. A, terms with equal (m, l, x, s) are
 * merged by adding their prefactors and zero terms are dropped.  t is M*M
 * row-major (NULL: no one-body part); u holds n_u two-body entries.  *n_out
 * receives the number of tuples; they are written to out when cap suffices.
 * Host only. */
mbr_status mbr_terms_from_hamiltonian(int32_t M, const double *t, int32_t n_u, const mbr_coulomb *u,
                                      mbr_term *out, int64_t cap, int64_t *n_out);

/* An operator on one sector: the term list (copied to the device) and a
 * ranker for that sector, either a staggered ranker of the same C^M_N (the
 * sector built with the single window of N set bits among all M orbitals) or
 * a trie built on `s`.  y = H x is formed in gather form (Eq. Talpha2), one lane
 * per row: y_a = sum_T v [a & m == l] (-1)^popcount(a & s) x[rank(a ^ x_T)];
 * terms that lead out of the sector contribute nothing.  The operator keeps
 * references to `s` and `r`. */
mbr_status mbr_operator_create(const mbr_sector *s, const mbr_ranker *r, const mbr_term *terms,
                               int64_t n_terms, mbr_operator **out, void *stream);

/* y = H x over the sector, fp64 vectors of the sector's size (d_x and d_y must
 * not alias). */
mbr_status mbr_operator_apply(const mbr_operator *op, const double *d_x, double *d_y, void *stream);

/* Lowest eigenvalue of the operator on its sector by plain fp64 Lanczos
 * (three vectors, no reorthogonalisation; the minimum is unaffected by ghost
 * copies): alpha_j = <v_j, H v_j>, w = H v_j - alpha_j v_j - beta_{j-1} v_{j-1},
 * beta_j = |w|, v_{j+1} = w / beta_j, from v_0 = d_v0 / |d_v0| (fp64, the
 * sector's size), for nsteps steps, as many steps as the sector has states,
 * or until beta_j <= tol (|alpha_j| + beta_{j-1}); then the lowest eigenvalue of the tridiagonal matrix (Sturm
 * bisection, as mbr_tridiag_lowest).  Host outputs: *e0, *steps_done, and the
 * coefficients alpha[0..nsteps), beta[0..nsteps) when not NULL (entries from
 * steps_done on are zero).  Allocates
 * three work vectors; synchronises `stream`. */
mbr_status mbr_operator_lanczos(const mbr_operator *op, const double *d_v0, int32_t nsteps, double tol,
                                double *e0, int32_t *steps_done, double *alpha, double *beta, void *stream);

mbr_status mbr_operator_destroy(mbr_operator *op);

/* ======================================================================== */
/* Hubbard-type Hamiltonians applied on the fly (Eq. Talpha, Eq. mvblock,     */
/* Eq. Hring generalised to a bond list)                                     */
/* ======================================================================== */

typedef struct mbr_hubbard mbr_hubbard;

typedef struct {
    int32_t i, j; /* sites, 0 <= i, j < L, i != j */
    double t;     /* amplitude: H contains -t (c+_{i s} c_{j s} + c+_{j s} c_{i s}) */
} mbr_bond;

typedef struct {
    int32_t n_up, n_dn;
} mbr_spin_sector;

#define MBR_F64 0
#define MBR_F32 1

#define MBR_HV_RANK_HALVES 0 /* staggered lookup of the half a hop changes (Eq. rankupdown) */
#define MBR_HV_RANK_TRIE   1 /* packed trie over each sector's full 2L-bit patterns (Sec. IV) */

typedef struct {
    int32_t L;                       /* sites, 1..16 */
    int32_t n_bonds;                 /* 0..48 */
    const mbr_bond *bonds;
    const double *eps;               /* on-site energies [L] or NULL */
    const double *U;                 /* on-site interaction [L] or NULL */
    int32_t n_sectors;               /* 1..1024 spin sectors, concatenated */
    const mbr_spin_sector *sectors;
    int32_t precision;               /* MBR_F64 or MBR_F32 vectors */
    int32_t k;                       /* chunk width, 0 = automatic: of the half-pattern table
                                        (halves), or of the trie, 4..16 (trie; automatic: four levels) */
    int32_t rank_kind;               /* MBR_HV_RANK_HALVES or MBR_HV_RANK_TRIE */
} mbr_hubbard_desc;

/* H = -sum_b t_b sum_s (c+_{i s} c_{j s} + h.c.) + sum_i U_i n_{i up} n_{i dn}
 *     + sum_{i s} eps_i n_{i s}, restricted to the listed (N_up, N_dn) sectors.
 * Vectors are the concatenation of the sectors in list order; within a sector
 * the index is rank_up * C(L, n_dn) + rank_dn (Eq. rankupdown), which is also
 * the position of the pattern (up half << L | down half) in the sector's
 * ascending list.
 * rank_kind selects how hop targets are ranked.  MBR_HV_RANK_HALVES (the
 * default): only the half a hop changes is re-ranked, by staggered lookup on
 * L-bit halves.  MBR_HV_RANK_TRIE: the plain trie method inside H·x (Sec. V.B
 * compares it with staggered lookup): the library builds each sector's list
 * and a packed trie over its full 2L-bit patterns (2L <= 32), reads every row's
 * pattern from the list and ranks every hop target by a trie walk (a hop
 * target of a spin sector is always a member, so no membership read).  Both
 * kinds sum each row's terms in the same order, so their products are
 * bitwise equal.  The trie kind has one launch shape (set_config returns
 * EUNSUPPORTED); its autotune times the trie chunk widths that give two,
 * three and four levels and keeps the fastest. */
mbr_status mbr_hubbard_create(const mbr_hubbard_desc *d, mbr_hubbard **out, void *stream);

/* Total dimension and, if offsets != NULL, the n_sectors+1 sector offsets. */
mbr_status mbr_hubbard_dim(const mbr_hubbard *h, uint64_t *total, uint64_t *offsets);

/* d_y = H d_x in the gather form of Eq. Talpha2: one output row per lane group,
 * no atomics.  x and y are fp64 or fp32 per the descriptor and must not alias. */
mbr_status mbr_hubbard_apply(const mbr_hubbard *h, const void *d_x, void *d_y, void *stream);

mbr_status mbr_hubbard_destroy(mbr_hubbard *h);

/* Launch shape of the H·x kernel (extension: the paper has no GPU layout).
 * k: half-pattern chunk width of the staggered rank; G: -1 selects the flat
 * kernel for every sector (256-lane workgroups, one row per lane at a time,
 * both halves ranked on the fly, no staged x and no barrier between rows);
 * 0 selects the alpha_dn-stationary rows kernel (1024-lane workgroups, one
 * per CU, down-hop lists ranked once per launch shape) for every sector it
 * supports (at most 4095 spin-down configurations and 15 bonds) and the tile
 * kernel with two blocks for the rest; -2 is G = 0 with the sectors of more
 * than 512 spin-down configurations moved to the block kernel (one alpha_up
 * block per 1024-lane workgroup, a workgroup per tile instead of one per CU,
 * up-hop lists of every half state built once per launch shape); G in
 * {1,2,4} selects the tile kernel for every sector, holding G alpha_up
 * blocks per workgroup (the down-hop ranks of a lane are reused G times);
 * block: threads per workgroup of the tile kernel (256 or 512).  Every shape
 * sums each row's terms in the same order, so products are bitwise equal.
 * tuned_ms is the autotuner's best time for one product (0 when not tuned). */
typedef struct {
    int32_t k;
    int32_t G;
    int32_t block;
    int32_t tiles;
    uint64_t lds_bytes;
    double tuned_ms;
} mbr_hubbard_cfg;

mbr_status mbr_hubbard_get_config(const mbr_hubbard *h, mbr_hubbard_cfg *cfg);

/* Set the launch shape (k in 1..L, G in {-2,-1,0,1,2,4}, block in {256,512}); EUNSUPPORTED
 * when the tiles would not fit the LDS.  Lanczos handles created before the
 * change reject further steps (EINVAL): create them afterwards. */
mbr_status mbr_hubbard_set_config(mbr_hubbard *h, int32_t k, int32_t G, int32_t block, void *stream);

/* Time every supported (k, G, block) on this device with `reps` products of
 * scratch vectors and keep the fastest (for a trie-ranked product: the trie's
 * chunk width, rebuilding the tries; get_config then reports it as k).  If the environment variable
 * MBR_AUTOTUNE_CACHE names a file, a matching entry (device, L, bonds,
 * sectors, precision) is used without timing, and new results are appended;
 * unreadable or malformed entries are ignored.  Synchronises `stream`. */
mbr_status mbr_hubbard_autotune(mbr_hubbard *h, int32_t reps, void *stream);

/* ======================================================================== */
/* Lanczos ground-state search over every sector of a Hamiltonian            */
/* ======================================================================== */

typedef struct mbr_lanczos mbr_lanczos;

typedef struct {
    int32_t max_steps;     /* Krylov steps kept per sector, 1..4096 */
    int32_t reorth;        /* 1: full classical Gram-Schmidt each step (fp64 coefficients) */
    int32_t batched;       /* 1: all sectors per kernel launch; 0: one launch set per sector */
    int32_t use_graph;     /* 1: replay a captured hipGraph per step */
    double breakdown_tol;  /* relative beta below which a sector stops (0 = default) */
} mbr_lanczos_opts;

/* Lanczos recurrence u = H v_j - beta_{j-1} v_{j-1}, alpha_j = <v_j, u>,
 * w = u - alpha_j v_j, beta_j = |w|, v_{j+1} = w / beta_j, run independently per
 * sector.  Vectors have the Hamiltonian's precision; alpha, beta and every dot
 * product accumulate in fp64. */
mbr_status mbr_lanczos_create(const mbr_hubbard *h, const mbr_lanczos_opts *o,
                              mbr_lanczos **out);

/* Set the start vector (fp64, the Hamiltonian's total dimension; each sector's
 * part is normalised separately) and reset the step count. */
mbr_status mbr_lanczos_start(mbr_lanczos *lz, const double *d_v0, void *stream);

/* Enqueue nsteps Lanczos steps. */
mbr_status mbr_lanczos_step(mbr_lanczos *lz, int32_t nsteps, void *stream);

/* Lowest Ritz value per sector (tridiagonal solved on the device by Sturm
 * bisection in fp64) and the steps each sector completed.  Either output may be
 * NULL.  Synchronises `stream`. */
mbr_status mbr_lanczos_result(mbr_lanczos *lz, double *e0, int32_t *steps_done, void *stream);

/* Copy alpha and beta (n_sectors x max_steps each, row per sector) to host.
 * Synchronises `stream`. */
mbr_status mbr_lanczos_coeffs(mbr_lanczos *lz, double *alpha, double *beta, void *stream);

mbr_status mbr_lanczos_destroy(mbr_lanczos *lz);

/* Lowest eigenvalue of n_batch symmetric tridiagonal matrices by Sturm-count
 * bisection in fp64: matrix b has diagonal d_alpha[b*ld .. b*ld+len_b-1] and
 * off-diagonal d_beta[b*ld .. b*ld+len_b-2], len_b = d_len[b] (1..ld).
 * Result to d_e0[b]. */
mbr_status mbr_tridiag_lowest(const double *d_alpha, const double *d_beta, const int32_t *d_len,
                              int32_t ld, int32_t n_batch, double *d_e0, void *stream);

/* ======================================================================== */
/* Measurement                                                              */
/* ======================================================================== */

/* Gather probe (a measurement primitive for the rooflines of the gather-bound
 * kernels, not a step of the method): for each j < n, i = d_idx[j] mod
 * entries, then depth times i = d_table[i] mod entries (each read's address
 * comes from the one before, as in a trie walk), and d_out[j] = i.  entries
 * is a power of two up to 2^32 (EINVAL otherwise), depth in 1..64.  lds = 1
 * stages the table in LDS first, for entries <= 16384 (EINVAL beyond).
 * d_table holds `entries` uint32 values, d_idx and d_out n each. */
mbr_status mbr_probe_gather(const uint32_t *d_table, uint64_t entries, const uint32_t *d_idx, uint64_t n,
                            int32_t depth, int32_t lds, uint32_t *d_out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MBRANK_H */
