/*
 * Plain CPU oracle for the many-body ranking hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into oracle/liboracle.so and is
 * loaded by tests/, by __graft_entry__.smoke() and by the cpu_baseline leg of
 * bench.py.  The product library (paper_2203_04158_amd) never includes, links or
 * calls it, and it shares no code with the HIP path.
 *
 * Every routine is a direct, unblocked transcription of a definition from
 * M. Wallerberger and K. Held, "Trie-based ranking of quantum many-body states"
 * (arXiv:2203.04158); the comment above each routine names the passage.
 * Patterns are carried as uint64 throughout, whatever their width.
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

static int popc64(uint64_t a) { return __builtin_popcountll(a); }

/* ---------------------------------------------------------------------------
 * Binomial coefficients C(n,k) for 0 <= n,k <= 64, with C(n,k) = 0 for k > n
 * (convention stated under Eq. cns).  Built by Pascal's rule; C(64,32) < 2^64.
 */
static uint64_t g_binom[65][65];
static int g_binom_ready = 0;

static void binom_init(void)
{
    if (g_binom_ready) return;
    for (int n = 0; n <= 64; ++n) {
        g_binom[n][0] = 1;
        for (int k = 1; k <= 64; ++k)
            g_binom[n][k] = (n == 0) ? 0 : g_binom[n - 1][k - 1] + g_binom[n - 1][k];
    }
    g_binom_ready = 1;
}

uint64_t orc_binom(int n, int k)
{
    binom_init();
    if (n < 0 || k < 0 || n > 64 || k > 64) return 0;
    return g_binom[n][k];
}

/* ---------------------------------------------------------------------------
 * Combinadics rank, Eq. cns with Eq. rank: with the occupied orbitals in
 * increasing position c_1 < c_2 < ... < c_N, the rank is the sum over k of
 * C(c_k, k).  Summed position by position: k counts the occupied orbitals
 * seen so far, and an occupied position adds C(position, k).
 */
uint64_t orc_cns_rank(uint64_t a)
{
    uint64_t rank = 0;
    int k = 0;
    for (int pos = 0; pos < 64; ++pos) {
        if ((a >> pos) & 1u) {
            ++k;
            rank += orc_binom(pos, k);
        }
    }
    return rank;
}

void orc_cns_rank_batch(const uint64_t *q, int64_t n, uint64_t *out)
{
    for (int64_t j = 0; j < n; ++j) out[j] = orc_cns_rank(q[j]);
}

/* Inverse of Eq. cns (Eq. unrank): for k = N..1 pick the largest c with
 * C(c,k) <= remaining index.  Returns the pattern alpha(c_N, ..., c_1). */
uint64_t orc_cns_unrank(uint64_t idx, int N, int M)
{
    uint64_t a = 0;
    int c = M - 1;
    for (int k = N; k >= 1; --k) {
        while (c >= 0 && orc_binom(c, k) > idx) --c;
        if (c < 0) return ~(uint64_t)0;
        a |= (uint64_t)1 << c;
        idx -= orc_binom(c, k);
        --c;
    }
    return a;
}

/* ---------------------------------------------------------------------------
 * Sector membership: a pattern belongs to the sector when, for every
 * constraint j, lo[j] <= popcount(alpha AND mask[j]) <= hi[j].  Particle
 * number (Eq. HNcomm), the (N_up, N_dn) split of Eq. rankupdown and extra
 * occupation restrictions are all of this form (filtering by further quantum
 * numbers, closing paragraph of Sec. IV).
 */
static int in_sector(uint64_t a, int nc, const uint64_t *mask,
                     const int32_t *lo, const int32_t *hi)
{
    for (int j = 0; j < nc; ++j) {
        int h = popc64(a & mask[j]);
        if (h < lo[j] || h > hi[j]) return 0;
    }
    return 1;
}

/* All M-bit patterns of the sector in ascending numeric order, which is the
 * lexicographic order of Sec. III (c_N first).  With fixedN >= 0 the walk
 * visits only N-particle patterns, in increasing order, using Gosper's
 * next-combination step (HAKMEM item 175); otherwise every pattern below 2^M is
 * tested.  Returns the count; writes at most cap entries to out (out may be
 * NULL to count only).  Returns -1 for unsupported sizes. */
int64_t orc_sector_enumerate(int M, int nc, const uint64_t *mask, const int32_t *lo,
                             const int32_t *hi, int fixedN, uint64_t *out, int64_t cap)
{
    int64_t cnt = 0;
    if (M < 0 || M > 40) return -1;
    if (fixedN >= 0) {
        if (fixedN > M) return 0;
        uint64_t lim = (uint64_t)1 << M;
        uint64_t a = (fixedN == 0) ? 0 : (((uint64_t)1 << fixedN) - 1);
        for (;;) {
            if (in_sector(a, nc, mask, lo, hi)) {
                if (out && cnt < cap) out[cnt] = a;
                ++cnt;
            }
            if (a == 0) break; /* N = 0 has the single pattern 0 */
            uint64_t c = a & (~a + 1);
            uint64_t r = a + c;
            a = (((r ^ a) >> 2) / c) | r;
            if (a >= lim) break;
        }
    } else {
        if (M > 34) return -1;
        uint64_t lim = (uint64_t)1 << M;
        for (uint64_t a = 0; a < lim; ++a) {
            if (in_sector(a, nc, mask, lo, hi)) {
                if (out && cnt < cap) out[cnt] = a;
                ++cnt;
            }
        }
    }
    return cnt;
}

/* ---------------------------------------------------------------------------
 * Bisection ranking (the established method, Sec. II end and Sec. III.A):
 * lower bound in the sorted list, then an equality test.  Not found -> -1.
 */
static int64_t bisect(const uint64_t *s, int64_t n, uint64_t a)
{
    int64_t lo = 0, hi = n; /* first index with s[idx] >= a lies in [lo, hi] */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (s[mid] < a) lo = mid + 1; else hi = mid;
    }
    return (lo < n && s[lo] == a) ? lo : -1;
}

void orc_bisect_rank_batch(const uint64_t *states, int64_t n, const uint64_t *q,
                           int64_t nq, int64_t *out)
{
    for (int64_t j = 0; j < nq; ++j) out[j] = bisect(states, n, q[j]);
}

/* ---------------------------------------------------------------------------
 * Staggered lookup entry, Eq. partrank: for a chunk r with set bits
 * c_1 < ... < c_Q, after M' lower flavours holding N' particles,
 * rank(r, M', N') = sum_q C(M' + c_q, N' + q).
 */
uint64_t orc_partrank(uint64_t r, int Mp, int Np)
{
    uint64_t s = 0;
    int q = 1;
    while (r != 0) {
        int c = __builtin_ctzll(r);
        r &= r - 1;
        s += orc_binom(Mp + c, Np + q);
        ++q;
    }
    return s;
}

/* ---------------------------------------------------------------------------
 * Size of the packed linearised trie (Sec. IV, packed representation): every
 * node at level l (which dispatches on chunk l, chunks taken least significant
 * first with the given widths) occupies the slots from its first to its last
 * occurring child value.  The node at level l is identified by the bits below
 * chunk l.  Returns the total number of slots T (so f = T / N_s), or -1 when a
 * level's prefix exceeds 26 bits.  No padding is counted.
 */
int64_t orc_trie_paper_size(const uint64_t *states, int64_t n, int H, const int32_t *widths)
{
    int64_t total = 0;
    int B = 0;
    for (int l = 0; l < H; ++l) {
        int w = widths[l];
        if (B > 26 || w > 16) return -1;
        size_t np = (size_t)1 << B;
        uint16_t *mn = (uint16_t *)malloc(np * sizeof(uint16_t));
        uint16_t *mx = (uint16_t *)malloc(np * sizeof(uint16_t));
        uint8_t *seen = (uint8_t *)calloc(np, 1);
        if (!mn || !mx || !seen) { free(mn); free(mx); free(seen); return -1; }
        uint64_t pmask = np - 1, cmask = ((uint64_t)1 << w) - 1;
        for (int64_t j = 0; j < n; ++j) {
            uint64_t p = states[j] & pmask;
            uint16_t c = (uint16_t)((states[j] >> B) & cmask);
            if (!seen[p]) { seen[p] = 1; mn[p] = c; mx[p] = c; }
            else { if (c < mn[p]) mn[p] = c; if (c > mx[p]) mx[p] = c; }
        }
        for (size_t p = 0; p < np; ++p)
            if (seen[p]) total += (int64_t)mx[p] - (int64_t)mn[p] + 1;
        free(mn); free(mx); free(seen);
        B += w;
    }
    return total;
}

/* ---------------------------------------------------------------------------
 * Gather-form product y = H x restricted to a sector, Eq. mvblock with each
 * term applied from the bra side, Eq. Talpha2:
 *     <alpha| T = v [alpha AND m == l] (-1)^h(alpha AND s) <alpha XOR x|,
 * so y[alpha] = sum_T v [..] (-1)^.. x[rank(alpha XOR x_T)], with the rank found
 * by bisection.  Rows row_begin..row_end-1 are produced; abssum (optional)
 * receives sum_T |v x[..]| per row for error bounds.  Terms leaving the sector
 * are a caller error and make the routine return the offending row + 1 as a
 * negative number.  The sum runs over terms in the order given.
 */
int64_t orc_apply_terms_bra(const uint64_t *states, int64_t n, int nt,
                            const double *tv, const uint64_t *tm, const uint64_t *tl,
                            const uint64_t *tx, const uint64_t *ts,
                            const double *x, double *y, double *abssum,
                            int64_t row_begin, int64_t row_end)
{
    for (int64_t i = row_begin; i < row_end; ++i) {
        uint64_t a = states[i];
        double acc = 0.0, aacc = 0.0;
        for (int t = 0; t < nt; ++t) {
            if ((a & tm[t]) != tl[t]) continue;
            int64_t j = bisect(states, n, a ^ tx[t]);
            if (j < 0) return -(i + 1);
            double sgn = (popc64(a & ts[t]) & 1) ? -1.0 : 1.0;
            double term = tv[t] * sgn * x[j];
            acc += term;
            aacc += (term < 0) ? -term : term;
        }
        y[i - row_begin] = acc;
        if (abssum) abssum[i - row_begin] = aacc;
    }
    return 0;
}

/* Same product, emitted as coordinate triplets (row, column, value) for every
 * non-zero term contribution, so that a sparse matrix can be assembled.
 * Returns the number of triplets, or a negative row + 1 on a sector leak.
 * cap bounds the number written. */
int64_t orc_terms_coo(const uint64_t *states, int64_t n, int nt,
                      const double *tv, const uint64_t *tm, const uint64_t *tl,
                      const uint64_t *tx, const uint64_t *ts,
                      int64_t *rows, int64_t *cols, double *vals, int64_t cap)
{
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t a = states[i];
        for (int t = 0; t < nt; ++t) {
            if ((a & tm[t]) != tl[t]) continue;
            int64_t j = bisect(states, n, a ^ tx[t]);
            if (j < 0) return -(i + 1);
            double sgn = (popc64(a & ts[t]) & 1) ? -1.0 : 1.0;
            if (cnt < cap) { rows[cnt] = i; cols[cnt] = j; vals[cnt] = tv[t] * sgn; }
            ++cnt;
        }
    }
    return cnt;
}

/* ---------------------------------------------------------------------------
 * Plain gather-form H x of a Hubbard-type Hamiltonian with every hop target
 * ranked by bisection in the sector list: the method the paper measures its
 * staggered and trie lookups against inside H v (Sec. V.B).  Used as the
 * timed CPU baseline; its results are checked against orc_apply_terms_bra.
 *
 * H = -sum_b t_b sum_s (c+_{i s} c_{j s} + h.c.) + sum_i U_i n_{i up} n_{i dn}
 *     + sum_{i s} eps_i n_{i s},  spin-down in bits 0..L-1, spin-up in L..2L-1.
 * Row a of the bra form (Eq. Talpha2): the diagonal, plus for every bond and
 * spin whose two orbitals differ in a, -t_b times (-1)^(occupied orbitals
 * strictly between them, on a) times x at the rank of a with both flipped
 * (Eq. cee: <a| c+_p c_q is non-zero for a_p = 1, a_q = 0).
 * Rows row_begin .. row_end-1 go to y[0 ..]; nthreads > 1 splits them over
 * OpenMP threads (static schedule).  Returns 0, or -(row + 1) if a target
 * is missing from the list.
 */
int64_t orc_hubbard_bisect_apply(const uint64_t *states, int64_t n, int L, int nb,
                                 const int32_t *bi, const int32_t *bj, const double *bt,
                                 const double *eps, const double *U, const double *x, double *y,
                                 int64_t row_begin, int64_t row_end, int nthreads)
{
    int64_t bad = 0;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads) reduction(min:bad)
    for (int64_t i = row_begin; i < row_end; ++i) {
        const uint64_t a = states[i];
        double diag = 0.0;
        for (int site = 0; site < L; ++site) {
            const int dn = (int)((a >> site) & 1u), up = (int)((a >> (L + site)) & 1u);
            diag += eps[site] * (dn + up) + U[site] * (dn & up);
        }
        double acc = diag * x[i];
        for (int b = 0; b < nb; ++b) {
            const int lo = bi[b] < bj[b] ? bi[b] : bj[b], hi = bi[b] < bj[b] ? bj[b] : bi[b];
            for (int spin = 0; spin < 2; ++spin) {
                const int off = spin * L;
                const uint64_t pi = (uint64_t)1 << (off + lo), pj = (uint64_t)1 << (off + hi);
                if (((a & pi) != 0) == ((a & pj) != 0)) continue;
                uint64_t between = 0;
                for (int k = lo + 1; k < hi; ++k) between |= (uint64_t)1 << (off + k);
                const int64_t j = bisect(states, n, a ^ pi ^ pj);
                if (j < 0) { bad = bad < -(i + 1) ? bad : -(i + 1); continue; }
                const double sgn = (popc64(a & between) & 1) ? -1.0 : 1.0;
                acc += -bt[b] * sgn * x[j];
            }
        }
        y[i - row_begin] = acc;
    }
    return bad;
}

/* Bisection and combinadics ranks of n queries split over nthreads OpenMP
 * threads (the rank baselines of the timing leg). */
void orc_rank_batch_mt(const uint64_t *states, int64_t ns, const uint64_t *q, int64_t n,
                       int64_t *out, int method, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t j = 0; j < n; ++j)
        out[j] = method == 0 ? bisect(states, ns, q[j]) : (int64_t)orc_cns_rank(q[j]);
}
