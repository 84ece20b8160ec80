// Generic operators from non-branching terms (App. A) applied on the fly.
//
// Every term of Eq. H, a prefactor times a product of creation and
// annihilation operators, acts on an occupation pattern as one tuple
// (v, m, l, r, x, s) (Eq. Talpha1, Eq. Talpha2).  Tuples are built on the host
// from those of the single operators (Eqs. ci) by the product rule of App. A;
// terms with equal (m, l, x, s) are merged by adding their prefactors.
//
// The product is taken in gather form from the bra side (Eq. Talpha2), one
// lane per output row, so no atomics are needed:
//   y_alpha = sum_T v [alpha AND m == l] (-1)^popcount(alpha AND s) x[rank(alpha XOR x_T)]
// with alpha = states[row] and the rank from the operator's ranker: a staggered
// table (sector C^M_N; table staged in LDS when it fits) or a packed trie (any
// sector; walk plus membership check).  Tuples are uniform across the lanes
// and are read through the scalar path.
#include <algorithm>
#include <memory>
#include <tuple>

#include "rank_device.hpp"

namespace {

// ---------------------------------------------------------------- host algebra
struct Tup {
    double v;
    uint64_t m, l, r, x, s;
};

// c_i (Eqs. ci): needs orbital i occupied on the right, leaves it empty on the
// left, flips it, and picks up the parity of the orbitals below i.
Tup annihilator(int i) {
    const uint64_t b = 1ull << i;
    return Tup{1.0, b, 0, b, b, b - 1};
}

// c_i^dagger: the annihilator with its left and right requirements exchanged.
Tup creator(int i) {
    Tup t = annihilator(i);
    std::swap(t.l, t.r);
    return t;
}

// One tuple applied to a ket (Eq. Talpha1): false when it annihilates alpha,
// else the coefficient is multiplied by its signed prefactor and alpha moved to
// its image.
bool act_on(const Tup &t, uint64_t &alpha, double &coef) {
    if ((alpha & t.m) != t.r) return false;
    coef *= (__builtin_popcountll(alpha & t.s) & 1) ? -t.v : t.v;
    alpha ^= t.x;
    return true;
}

// Tuple of the product T_a T_b (T_b acts first), App. A, by running the one
// pattern that can survive through both factors.  The product touches the
// orbitals of m = m_a | m_b: on m_b a surviving pattern must hold r_b, and on
// the rest of m_a, which T_b leaves alone, it must hold r_a; outside m it is
// free.  The pattern holding exactly that (nothing outside m) is pushed
// through T_b and then T_a: if either annihilates it the product vanishes,
// otherwise its image is l and the accumulated coefficient is v.  Outside m
// each factor sees the same occupations, so an orbital there changes the sign
// once per factor whose sign mask holds it: s = (s_a ^ s_b) & ~m.
Tup product(const Tup &a, const Tup &b) {
    Tup t;
    t.m = a.m | b.m;
    t.r = b.r | (a.r & ~b.m);
    t.s = (a.s ^ b.s) & ~t.m;
    uint64_t state = t.r;
    double coef = 1.0;
    if (!act_on(b, state, coef) || !act_on(a, state, coef)) {
        t.v = 0.0;
        t.l = t.x = 0;
        return t;
    }
    t.l = state;
    t.x = t.l ^ t.r;
    t.v = coef;
    return t;
}

Tup product_of(double v, std::initializer_list<Tup> ops) {
    auto it = ops.begin();
    Tup t = *it;
    for (++it; it != ops.end(); ++it) t = product(t, *it);
    t.v *= v;
    return t;
}

// Merge tuples with equal (m, l, x, s), drop zeros; deterministic order.
std::vector<Tup> merge_terms(std::vector<Tup> ts) {
    std::sort(ts.begin(), ts.end(), [](const Tup &a, const Tup &b) {
        return std::tie(a.m, a.l, a.x, a.s) < std::tie(b.m, b.l, b.x, b.s);
    });
    std::vector<Tup> out;
    for (const Tup &t : ts) {
        if (!out.empty() && out.back().m == t.m && out.back().l == t.l && out.back().x == t.x &&
            out.back().s == t.s)
            out.back().v += t.v;
        else
            out.push_back(t);
    }
    out.erase(std::remove_if(out.begin(), out.end(), [](const Tup &t) { return t.v == 0.0; }), out.end());
    return out;
}

// ---------------------------------------------------------------- device apply
constexpr unsigned kBlock = 256;
constexpr size_t kLdsTable = 64 * 1024;

enum RankKind { kStagLds = 0, kStagGlobal = 1, kTrie = 2 };

template <class P>
struct OpArgs {
    const P *states;
    uint64_t ns;
    int64_t nt;
    const double *v;
    const P *m, *l, *x, *s;
    const uint32_t *keep;  // per tuple: every member's target is a member
    const double *xin;
    double *out;
    StagArgs stag;
    const void *stab;
    TrieWalk trie;
};

template <class P, class E, int RK>
__global__ void __launch_bounds__(kBlock) op_apply_kernel(OpArgs<P> a) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const E *tab = static_cast<const E *>(a.stab);
    if constexpr (RK == kStagLds) {
        E *t = reinterpret_cast<E *>(lds_raw);
        for (uint64_t i = threadIdx.x; i < a.stag.nentries; i += blockDim.x) t[i] = tab[i];
        __syncthreads();
        tab = t;
    }
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t row = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; row < a.ns; row += stride) {
        const P al = a.states[row];
        double acc = 0.0;
        for (int64_t t = 0; t < a.nt; ++t) {
            if ((al & a.m[t]) != a.l[t]) continue;
            const P be = al ^ a.x[t];
            uint64_t rr;
            if (a.x[t] == 0) {
                rr = row;
            } else if constexpr (RK == kTrie) {
                if (a.keep[t]) {
                    // the target is a member, so the walk alone gives its rank
                    uint32_t node = 0;
                    for (int lv = 0; lv < a.trie.H; ++lv)
                        node = a.trie.tab[a.trie.off[lv] + node + ((uint32_t)(be >> a.trie.shift[lv]) & a.trie.wmask[lv])];
                    rr = node;
                } else {
                    const uint32_t q = trie_rank_one<P>(be, a.trie);
                    if (q == MBR_NOT_FOUND) continue;  // the term leaves the sector
                    rr = q;
                }
            } else {
                const int h = (sizeof(P) == 8) ? __popcll((uint64_t)be) : __popc((uint32_t)be);
                if (h != a.stag.N || !below_width(be, a.stag.M)) continue;  // leaves C^M_N
                rr = stag_rank<P, E>(be, tab, a.stag);
            }
            const bool odd = ((sizeof(P) == 8) ? __popcll((uint64_t)(al & a.s[t])) : __popc((uint32_t)(al & a.s[t]))) & 1;
            const double c = odd ? -a.v[t] : a.v[t];
            acc = __builtin_fma(c, a.xin[rr], acc);
        }
        a.out[row] = acc;
    }
}

// ---------------------------------------------------------------- Lanczos
// Plain fp64 Lanczos on an operator (three vectors, no reorthogonalisation):
// alpha_j = <v_j, H v_j>; w = H v_j - alpha_j v_j - beta_{j-1} v_{j-1};
// beta_j = |w|; v_{j+1} = w / beta_j.  Dot products are fixed-order two-level
// reductions (kRedBlocks block partials, then one block), so runs repeat
// bitwise.  The recurrence stops (the remaining kernels do nothing) once
// beta_j <= tol (|alpha_j| + beta_{j-1}) or after as many steps as the sector
// has states; *len holds the steps taken.
constexpr unsigned kRedBlocks = 1024;

__device__ __forceinline__ double blk_sum(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
    return s;
}

__global__ void op_start_kernel(int32_t *len, int32_t nsteps) { *len = nsteps; }

__global__ void __launch_bounds__(kBlock) op_dot_parts(const double *__restrict__ a, const double *__restrict__ b,
                                                       uint64_t n, double *parts) {
    __shared__ double red[kBlock / 64];
    double acc = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        acc = __builtin_fma(a[i], b[i], acc);
    const double s = blk_sum(acc, red);
    if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

// out = sum of the kRedBlocks partials (sqrt of it when root != 0).
__global__ void __launch_bounds__(kBlock) op_reduce(const double *parts, double *out, int root) {
    __shared__ double red[kBlock / 64];
    double acc = 0;
    for (unsigned i = threadIdx.x; i < kRedBlocks; i += blockDim.x) acc += parts[i];
    const double s = blk_sum(acc, red);
    if (threadIdx.x == 0) *out = root ? sqrt(s) : s;
}

__global__ void __launch_bounds__(kBlock) op_scale_kernel(const double *__restrict__ v0, double *__restrict__ v,
                                                          double *__restrict__ vp, uint64_t n, const double *norm) {
    const double c = *norm > 0 ? 1.0 / *norm : 0.0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        v[i] = v0[i] * c;
        vp[i] = 0.0;
    }
}

__global__ void __launch_bounds__(kBlock) op_update_kernel(double *__restrict__ w, const double *__restrict__ v,
                                                           const double *__restrict__ vp, uint64_t n,
                                                           const double *al, const double *be, int j,
                                                           const int32_t *len, double *parts) {
    __shared__ double red[kBlock / 64];
    if (j >= *len) return;
    const double a = al[j], b = j > 0 ? be[j - 1] : 0.0;
    double acc = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const double x = w[i] - a * v[i] - b * vp[i];
        w[i] = x;
        acc = __builtin_fma(x, x, acc);
    }
    const double s = blk_sum(acc, red);
    if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock) op_beta_kernel(const double *parts, const double *al, double *be, int j,
                                                         int nsteps, uint64_t dim, double tol, int32_t *len) {
    __shared__ double red[kBlock / 64];
    if (j >= *len) return;
    double acc = 0;
    for (unsigned i = threadIdx.x; i < kRedBlocks; i += blockDim.x) acc += parts[i];
    const double s = blk_sum(acc, red);
    if (threadIdx.x == 0) {
        const double b = sqrt(s);
        const double bprev = j > 0 ? be[j - 1] : 0.0;
        // the Krylov space cannot outgrow the sector
        const bool stop = b <= tol * (fabs(al[j]) + bprev) || j + 1 >= nsteps || (uint64_t)(j + 1) >= dim;
        be[j] = stop ? 0.0 : b;
        if (stop) *len = j + 1;
    }
}

// v_{j+1} = w / beta_j, in place in w's buffer (the caller rotates the buffers).
// Once the recurrence has stopped the buffer is zeroed instead, so the steps
// the host still enqueues work on zero vectors (alpha = 0, nothing grows).
__global__ void __launch_bounds__(kBlock) op_next_kernel(double *__restrict__ w, const double *__restrict__ v,
                                                         const double *__restrict__ vp, uint64_t n,
                                                         const double *be, int j, const int32_t *len) {
    const double c = (j + 1 >= *len) ? 0.0 : 1.0 / be[j];
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        w[i] *= c;
}

}  // namespace

struct mbr_operator {
    const mbr_sector *sec = nullptr;
    const mbr_ranker *rk = nullptr;
    int64_t nt = 0;
    int32_t M = 0, width_bits = 32;
    mbr::DevBuf v, m, l, x, s, keep;
    int device = 0;
};

namespace {

template <class P, class E, int RK>
mbr_status launch_op(const mbr_operator *op, OpArgs<P> a, size_t lds, hipStream_t st) {
    auto kern = op_apply_kernel<P, E, RK>;
    if (lds > 64 * 1024)
        MBR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const unsigned grid = mbr::grid_for(op->sec->n, kBlock, mbr::device_cu_count() * 8);
    kern<<<grid, kBlock, lds, st>>>(a);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

template <class P>
mbr_status apply_t(const mbr_operator *op, const double *x, double *y, hipStream_t st) {
    OpArgs<P> a{};
    a.states = op->sec->states.as<P>();
    a.ns = op->sec->n;
    a.nt = op->nt;
    a.v = op->v.as<double>();
    a.m = op->m.as<P>();
    a.l = op->l.as<P>();
    a.x = op->x.as<P>();
    a.s = op->s.as<P>();
    a.keep = op->keep.as<uint32_t>();
    a.xin = x;
    a.out = y;
    const mbr_ranker *r = op->rk;
    if (r->kind == MBR_RANKER_TRIE) {
        const TrieLevels &t = *r->trie;
        a.trie.tab = t.table.as<uint32_t>();
        a.trie.states = op->sec->states.p;
        a.trie.ns = op->sec->n;
        a.trie.M = t.M;
        a.trie.H = t.H;
        for (int lv = 0; lv < t.H; ++lv) {
            a.trie.wmask[lv] = (uint32_t)((1ull << t.w[lv]) - 1);
            a.trie.shift[lv] = t.shift[lv];
            a.trie.off[lv] = t.off[lv];
        }
        a.trie.off[t.H] = t.off[t.H];
        return launch_op<P, uint32_t, kTrie>(op, a, 0, st);
    }
    const StagTable &tb = r->stag;
    a.stag.M = tb.M;
    a.stag.k = tb.k;
    a.stag.nch = tb.nch;
    a.stag.N = r->N;
    for (int c = 0; c < tb.nch && c < 16; ++c) a.stag.rowoff[c] = tb.rowoff[c];
    a.stag.nentries = (uint64_t)tb.nrows << tb.k;
    a.stab = tb.table.p;
    const size_t lds = a.stag.nentries * tb.entry_bytes;
    const bool in_lds = lds <= kLdsTable;
    switch (tb.entry_bytes) {
        case 2: return in_lds ? launch_op<P, uint16_t, kStagLds>(op, a, lds, st) : launch_op<P, uint16_t, kStagGlobal>(op, a, 0, st);
        case 4: return in_lds ? launch_op<P, uint32_t, kStagLds>(op, a, lds, st) : launch_op<P, uint32_t, kStagGlobal>(op, a, 0, st);
        default: return in_lds ? launch_op<P, uint64_t, kStagLds>(op, a, lds, st) : launch_op<P, uint64_t, kStagGlobal>(op, a, 0, st);
    }
}

}  // namespace

extern "C" {

mbr_status mbr_terms_from_hamiltonian(int32_t M, const double *t, int32_t n_u, const mbr_coulomb *u,
                                      mbr_term *out, int64_t cap, int64_t *n_out) {
    if (M < 1 || M > 64) MBR_FAIL(MBR_EINVAL, "M=%d outside 1..64", M);
    if (n_u < 0 || (n_u > 0 && !u)) MBR_FAIL(MBR_EINVAL, "bad interaction list");
    if (!n_out) MBR_FAIL(MBR_EINVAL, "null count pointer");
    std::vector<Tup> ts;
    if (t) {
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) {
                const double a = t[(size_t)i * M + j];
                if (a != 0.0) ts.push_back(product_of(-a, {creator(i), annihilator(j)}));
            }
    }
    for (int q = 0; q < n_u; ++q) {
        const mbr_coulomb &c = u[q];
        if (c.i < 0 || c.j < 0 || c.k < 0 || c.l < 0 || c.i >= M || c.j >= M || c.k >= M || c.l >= M)
            MBR_FAIL(MBR_EINVAL, "interaction %d has an orbital outside 0..M-1", q);
        if (c.U != 0.0)
            ts.push_back(product_of(0.25 * c.U, {creator(c.i), creator(c.j), annihilator(c.l), annihilator(c.k)}));
    }
    const std::vector<Tup> mt = merge_terms(std::move(ts));
    *n_out = (int64_t)mt.size();
    if (out && cap >= (int64_t)mt.size())
        for (size_t i = 0; i < mt.size(); ++i) out[i] = mbr_term{mt[i].v, mt[i].m, mt[i].l, mt[i].r, mt[i].x, mt[i].s};
    return MBR_OK;
}

mbr_status mbr_operator_create(const mbr_sector *sec, const mbr_ranker *rk, const mbr_term *terms,
                               int64_t n_terms, mbr_operator **out, void *stream) {
    using namespace mbr;
    if (!out) MBR_FAIL(MBR_EINVAL, "null output handle");
    *out = nullptr;
    if (!sec || !rk) MBR_FAIL(MBR_EINVAL, "null sector or ranker");
    if (n_terms < 0 || (n_terms > 0 && !terms)) MBR_FAIL(MBR_EINVAL, "bad term list");
    if (sec->n == 0) MBR_FAIL(MBR_EINVAL, "empty sector");
    if (rk->kind == MBR_RANKER_TRIE) {
        if (rk->sector != sec) MBR_FAIL(MBR_EINVAL, "the trie ranks a different sector");
    } else if (rk->kind == MBR_RANKER_STAGGERED) {
        // the sector must be exactly C^M_N of the table: one window with N set
        // bits among all M orbitals and no other constraint
        const uint64_t full = sec->M >= 64 ? ~0ull : ((1ull << sec->M) - 1);
        const bool cnm = sec->modulus == 0 && sec->cons.size() == 1 && sec->cons[0].mask == full &&
                         sec->cons[0].lo == rk->N && sec->cons[0].hi == rk->N;
        if (rk->N < 0 || rk->M != sec->M || !cnm || rk->n_states != sec->n || rk->width_bits != sec->width_bits)
            MBR_FAIL(MBR_EINVAL, "the staggered ranker does not rank this sector (C^M_N with one window)");
    } else {
        MBR_FAIL(MBR_EUNSUPPORTED, "operators rank with a staggered or trie ranker");
    }
    const uint64_t lim = sec->M >= 64 ? ~0ull : ((1ull << sec->M) - 1);
    for (int64_t i = 0; i < n_terms; ++i) {
        const mbr_term &t = terms[i];
        if ((t.m | t.l | t.x | t.s) & ~lim) MBR_FAIL(MBR_EINVAL, "term %lld touches orbitals >= M", (long long)i);
        if ((t.l & ~t.m) || (t.x & ~t.m)) MBR_FAIL(MBR_EINVAL, "term %lld: l and x must lie inside m", (long long)i);
    }
    auto op = std::make_unique<mbr_operator>();
    op->sec = sec;
    op->rk = rk;
    op->nt = n_terms;
    op->M = sec->M;
    op->width_bits = sec->width_bits;
    (void)hipGetDevice(&op->device);
    const size_t n = (size_t)std::max<int64_t>(n_terms, 1);
    std::vector<double> v(n, 0.0);
    std::vector<uint64_t> f[4];
    for (auto &a : f) a.assign(n, 0);
    for (int64_t i = 0; i < n_terms; ++i) {
        v[i] = terms[i].v;
        f[0][i] = terms[i].m;
        f[1][i] = terms[i].l;
        f[2][i] = terms[i].x;
        f[3][i] = terms[i].s;
    }
    // A tuple keeps the sector when it moves no particle into or out of any
    // constraint's orbitals and leaves the modular weight unchanged: the
    // target of every member is then a member (bits outside m are untouched,
    // and inside m the row holds l and the target l ^ x).
    std::vector<uint32_t> keep(n, 0u);
    for (int64_t i = 0; i < n_terms; ++i) {
        const uint64_t lo = terms[i].l, hi = terms[i].l ^ terms[i].x;
        // a caller's list has no constraints to check a tuple against
        bool k = !sec->from_list;
        for (const mbr_popc_cons &c : sec->cons)
            k = k && __builtin_popcountll(lo & c.mask) == __builtin_popcountll(hi & c.mask);
        if (sec->modulus > 0) {
            int64_t dw = 0;
            for (int b = 0; b < sec->M; ++b) dw += (int64_t)(((hi >> b) & 1) - ((lo >> b) & 1)) * sec->weights[b];
            k = k && dw % sec->modulus == 0;
        }
        keep[i] = k ? 1u : 0u;
    }
    hipStream_t st = as_stream(stream);
    MBR_TRY(upload(op->keep, keep.data(), n * 4, st));
    MBR_TRY(upload(op->v, v.data(), n * 8, st));
    DevBuf *dst[4] = {&op->m, &op->l, &op->x, &op->s};
    for (int k = 0; k < 4; ++k) {
        if (sec->width_bits == 64) {
            MBR_TRY(upload(*dst[k], f[k].data(), n * 8, st));
        } else {
            std::vector<uint32_t> w(f[k].begin(), f[k].end());
            MBR_TRY(upload(*dst[k], w.data(), n * 4, st));
        }
    }
    *out = op.release();
    return MBR_OK;
}

mbr_status mbr_operator_apply(const mbr_operator *op, const double *d_x, double *d_y, void *stream) {
    if (!op) MBR_FAIL(MBR_EINVAL, "null operator");
    if (!d_x || !d_y) MBR_FAIL(MBR_EINVAL, "null vector");
    if (d_x == d_y) MBR_FAIL(MBR_EINVAL, "x and y must not alias (gather form reads x while y is written)");
    hipStream_t st = mbr::as_stream(stream);
    if (op->width_bits == 32) return apply_t<uint32_t>(op, d_x, d_y, st);
    return apply_t<uint64_t>(op, d_x, d_y, st);
}

mbr_status mbr_operator_lanczos(const mbr_operator *op, const double *d_v0, int32_t nsteps, double tol,
                                double *e0, int32_t *steps_done, double *alpha, double *beta, void *stream) {
    using namespace mbr;
    if (!op || !d_v0) MBR_FAIL(MBR_EINVAL, "null operator or start vector");
    if (nsteps < 1 || nsteps > 100000) MBR_FAIL(MBR_EINVAL, "nsteps=%d", nsteps);
    if (!(tol >= 0.0)) MBR_FAIL(MBR_EINVAL, "tolerance must be non-negative");
    hipStream_t st = as_stream(stream);
    const uint64_t n = op->sec->n;
    DevBuf buf[3], parts, sc, d_len, d_e0;
    for (auto &b2 : buf) MBR_TRY(b2.alloc(n * 8));
    MBR_TRY(parts.alloc(kRedBlocks * 8));
    MBR_TRY(sc.alloc((2 * (size_t)nsteps + 2) * 8));
    MBR_TRY(d_len.alloc(4));
    MBR_TRY(d_e0.alloc(8));
    double *al = sc.as<double>(), *be = al + nsteps, *norm = be + nsteps;
    MBR_HIP(hipMemsetAsync(sc.p, 0, (2 * (size_t)nsteps + 2) * 8, st));
    int32_t *len = d_len.as<int32_t>();
    // v_0 = v0 / |v0|; the previous vector starts at zero
    double *vp = buf[0].as<double>(), *v = buf[1].as<double>(), *w = buf[2].as<double>();
    op_start_kernel<<<1, 1, 0, st>>>(len, nsteps);
    op_dot_parts<<<kRedBlocks, kBlock, 0, st>>>(d_v0, d_v0, n, parts.as<double>());
    op_reduce<<<1, kBlock, 0, st>>>(parts.as<double>(), norm, 1);
    op_scale_kernel<<<kRedBlocks, kBlock, 0, st>>>(d_v0, v, vp, n, norm);
    MBR_HIP(hipGetLastError());
    for (int32_t j = 0; j < nsteps; ++j) {
        MBR_TRY(mbr_operator_apply(op, v, w, stream));  // w = H v_j
        op_dot_parts<<<kRedBlocks, kBlock, 0, st>>>(v, w, n, parts.as<double>());
        op_reduce<<<1, kBlock, 0, st>>>(parts.as<double>(), al + j, 0);
        op_update_kernel<<<kRedBlocks, kBlock, 0, st>>>(w, v, vp, n, al, be, j, len, parts.as<double>());
        op_beta_kernel<<<1, kBlock, 0, st>>>(parts.as<double>(), al, be, j, nsteps, n, tol, len);
        op_next_kernel<<<kRedBlocks, kBlock, 0, st>>>(w, v, vp, n, be, j, len);
        MBR_HIP(hipGetLastError());
        double *t = vp;  // v_{j+1} now sits in w's buffer, v_j becomes the previous vector
        vp = v;
        v = w;
        w = t;
    }
    MBR_TRY(mbr_tridiag_lowest(al, be, len, nsteps, 1, d_e0.as<double>(), stream));
    int32_t hl = 0;
    double he = 0;
    MBR_HIP(hipMemcpyAsync(&hl, len, 4, hipMemcpyDeviceToHost, st));
    MBR_HIP(hipMemcpyAsync(&he, d_e0.p, 8, hipMemcpyDeviceToHost, st));
    if (alpha) MBR_HIP(hipMemcpyAsync(alpha, al, (size_t)nsteps * 8, hipMemcpyDeviceToHost, st));
    if (beta) MBR_HIP(hipMemcpyAsync(beta, be, (size_t)nsteps * 8, hipMemcpyDeviceToHost, st));
    MBR_HIP(hipStreamSynchronize(st));
    if (e0) *e0 = he;
    if (steps_done) *steps_done = hl;
    return MBR_OK;
}

mbr_status mbr_operator_destroy(mbr_operator *op) {
    delete op;
    return MBR_OK;
}

}  // extern "C"
