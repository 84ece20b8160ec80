// Staggered lookup (Sec. III.B): partial-rank tables and the rank kernels for
// particle-number sectors and for spin-resolved sectors (Eq. rankupdown).
//
// Table layout: one row per (chunk c, N'), rows of chunk c start at rowoff[c],
// 2^k entries per row with the chunk value fastest (the layout the paper
// recommends so that only the rows a query touches are loaded).  A workgroup
// copies the whole table into LDS once and then ranks a grid-stride share of
// the queries: per query, ceil(M/k) dependent LDS reads and popcounts.
#include "rank_device.hpp"

// ------------------------------------------------------------------ tables

mbr_status stag_build(StagTable &t, int32_t M, int32_t k, int32_t nmax, int32_t entry_bytes,
                      hipStream_t stream) {
    using namespace mbr;
    t.M = M;
    t.k = k;
    t.nmax = nmax;
    t.nch = (M + k - 1) / k;
    t.entry_bytes = entry_bytes;
    int rows = 0;
    for (int c = 0; c < t.nch; ++c) {
        t.rowoff[c] = rows;
        int Mp = c * k;
        rows += (Mp < nmax ? Mp : nmax) + 1;
    }
    t.nrows = rows;
    const uint64_t width = 1ull << k;
    t.host.assign((uint64_t)rows * width, 0);
    // Entry for (c, N', r), Eq. partrank evaluated through Eq. reuse: the
    // combinadics rank of the chunk placed at offset M' above N' set bits,
    // minus nothing (the N' low bits contribute C(j, j+1) = 0).
    for (int c = 0; c < t.nch; ++c) {
        int Mp = c * k;
        int w = (M - Mp < k) ? (M - Mp) : k;
        for (int Np = 0; Np <= (Mp < nmax ? Mp : nmax); ++Np) {
            uint64_t *row = &t.host[(uint64_t)(t.rowoff[c] + Np) * width];
            for (uint64_t r = 0; r < (1ull << w); ++r) {
                uint64_t s = 0;
                int q = Np + 1;
                for (int b = 0; b < w; ++b)
                    if ((r >> b) & 1) s += binom(Mp + b, q++);
                row[r] = s;
            }
        }
    }
    // Entry width: at least the requested one, widened until the largest
    // stored partial rank fits (rows never reached by a valid query included).
    uint64_t maxv = 0;
    for (uint64_t v : t.host) maxv = v > maxv ? v : maxv;
    if (entry_bytes < 4 && maxv > 0xFFFFull) entry_bytes = 4;
    if (entry_bytes < 8 && maxv > 0xFFFFFFFFull) entry_bytes = 8;
    t.entry_bytes = entry_bytes;
    size_t n = t.host.size();
    if (entry_bytes == 8) return upload(t.table, t.host.data(), n * 8, stream);
    if (entry_bytes == 4) {
        std::vector<uint32_t> v(t.host.begin(), t.host.end());
        return upload(t.table, v.data(), n * 4, stream);
    }
    std::vector<uint16_t> v(t.host.begin(), t.host.end());
    return upload(t.table, v.data(), n * 2, stream);
}

// The rows of a fixed-N table that members reach (LDS copies of it are
// smaller; the full table stays the reference layout).
mbr_status stag_trim(StagTable &t, int32_t N, hipStream_t stream) {
    using namespace mbr;
    const uint64_t width = 1ull << t.k;
    std::vector<uint64_t> h;
    int rows = 0;
    for (int c = 0; c < t.nch; ++c) {
        const int Mp = c * t.k;
        const int lo = N - (t.M - Mp) > 0 ? N - (t.M - Mp) : 0, hi = Mp < N ? Mp : N;
        t.trim_rowoff[c] = rows - lo;
        for (int Np = lo; Np <= hi; ++Np) {
            const uint64_t *row = &t.host[(uint64_t)(t.rowoff[c] + Np) * width];
            h.insert(h.end(), row, row + width);
        }
        rows += hi - lo + 1;
    }
    t.trim_entries = h.size();
    if (t.entry_bytes == 8) return upload(t.trim, h.data(), h.size() * 8, stream);
    if (t.entry_bytes == 4) {
        std::vector<uint32_t> v(h.begin(), h.end());
        return upload(t.trim, v.data(), v.size() * 4, stream);
    }
    std::vector<uint16_t> v(h.begin(), h.end());
    return upload(t.trim, v.data(), v.size() * 2, stream);
}

namespace {

// Smallest entry width (bytes) holding every partial rank of a table whose
// ranks stay below C(M, nmax-ish): the largest entry is below max_N C(M, N').
int entry_bytes_for(int M, int nmax) {
    uint64_t mx = 0;
    for (int n = 0; n <= nmax && n <= M; ++n) {
        uint64_t b = mbr::binom(M, n);
        mx = b > mx ? b : mx;
    }
    if (mx <= 0xFFFFull) return 2;
    if (mx <= 0xFFFFFFFFull) return 4;
    return 8;
}

// Workgroups of 1024 lanes: each stages the table once for four times the
// queries of a 256-lane one (2^28 queries: 0.54 -> 0.44 ms).
constexpr unsigned kBlock = 1024;

// The whole table into LDS (16-byte copies; the table's byte size is a
// multiple of 4: 2^k entries per row, k >= 1, entries of 2 bytes or more).
template <class E>
__device__ __forceinline__ void load_table(E *lds, const E *__restrict__ g, uint64_t n) {
    if ((n * sizeof(E)) % 4 == 0) {
        stage_to_lds(lds, g, n * sizeof(E));
    } else {
        for (uint64_t i = threadIdx.x; i < n; i += blockDim.x) lds[i] = g[i];
    }
    __syncthreads();
}

// V consecutive patterns (or ranks) moved by one 16-byte (V = 16 / sizeof(P))
// or scalar (V = 1) access; the launcher picks V = 1 when a pointer is not
// aligned to the vector.
template <class P, int V>
__device__ __forceinline__ void load_vec(const P *__restrict__ q, uint64_t j, P (&x)[V]) {
    if constexpr (V == 1) {
        x[0] = q[j];
    } else {
        typedef P vec_t __attribute__((ext_vector_type(V)));
        const vec_t v = reinterpret_cast<const vec_t *>(q)[j];
#pragma unroll
        for (int i = 0; i < V; ++i) x[i] = v[i];
    }
}

template <class RT, int V>
__device__ __forceinline__ void store_vec(RT *__restrict__ out, uint64_t j, const RT (&r)[V]) {
    if constexpr (V == 1) {
        out[j] = r[0];
    } else {
        typedef RT vec_t __attribute__((ext_vector_type(V)));
        vec_t v;
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = r[i];
        reinterpret_cast<vec_t *>(out)[j] = v;
    }
}

// Rank of one query of a particle-number sector as RT (32 or 64 bits); all
// ones (MBR_NOT_FOUND for 32 bits) outside it.
template <class P, class E, class RT>
__device__ __forceinline__ RT stag_query(P x, const E *tab, const StagArgs &a) {
    const int h = (sizeof(P) == 8) ? __popcll((uint64_t)x) : __popc((uint32_t)x);
    const bool ok = below_width(x, a.M) && (a.N < 0 || h == a.N);
    const uint64_t r = stag_rank<P, E>(ok ? x : (P)a.safe, tab, a);  // a.safe: its rows are in the table
    return ok ? (RT)r : (RT)~(RT)0;
}

// Queries are handled as vectors of V patterns, kVecs vectors per lane and
// batch (grid stride between a lane's vectors, so a wave's accesses stay
// contiguous).  The first batch is loaded before the table is staged so that
// its latency overlaps the staging; the n mod V last queries are ranked one
// per lane at the end.
constexpr int kVecs = 4;

// USE_LDS = false reads the table through the caches instead (tables larger
// than the LDS budget, e.g. k = 16 or 64-bit patterns with wide chunks).
template <class P, class E, bool USE_LDS, int V, class RT>
__global__ void __launch_bounds__(kBlock) rank_staggered_kernel(const P *__restrict__ q, uint64_t n,
                                                                RT *__restrict__ out,
                                                                const E *__restrict__ gtab,
                                                                StagArgs a) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const uint64_t nv = n / V;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    P x[kVecs][V];
    auto load = [&](uint64_t base) {
#pragma unroll
        for (int u = 0; u < kVecs; ++u) {
            const uint64_t j = base + u * stride;
            if (j < nv) load_vec<P, V>(q, j, x[u]);
        }
    };
    load(t0);
    const E *tab = gtab;
    if constexpr (USE_LDS) {
        E *t = reinterpret_cast<E *>(lds_raw);
        load_table(t, gtab, a.nentries);
        tab = t;
    }
    for (uint64_t base = t0; base < nv; base += stride * kVecs) {
        if (base != t0) load(base);
#pragma unroll
        for (int u = 0; u < kVecs; ++u) {
            const uint64_t j = base + u * stride;
            if (j < nv) {
                RT r[V];
#pragma unroll
                for (int i = 0; i < V; ++i) r[i] = stag_query<P, E, RT>(x[u][i], tab, a);
                store_vec<RT, V>(out, j, r);
            }
        }
    }
    if (t0 < n - nv * V) {
        const uint64_t j = nv * V + t0;
        out[j] = stag_query<P, E, RT>(q[j], tab, a);
    }
}

struct SpinArgs {
    StagArgs half;      // table over L-bit halves (universal up to nmax)
    int32_t L, n_up, n_dn;
    uint32_t mult;      // C(L, n_dn)
};

// Eq. rankupdown: rank(alpha_up) C(L, n_dn) + rank(alpha_dn), spin-down in
// the low L bits; MBR_NOT_FOUND outside the sector.
template <class P, class E>
__device__ __forceinline__ uint32_t spin_query(P x, const E *tab, const SpinArgs &a) {
    const P hm = (P)((a.L >= 32 && sizeof(P) == 8) ? 0xFFFFFFFFull : ((1ull << a.L) - 1));
    P dn = x & hm;
    P up = (x >> a.L) & hm;
    const int hd = (sizeof(P) == 8) ? __popcll((uint64_t)dn) : __popc((uint32_t)dn);
    const int hu = (sizeof(P) == 8) ? __popcll((uint64_t)up) : __popc((uint32_t)up);
    const bool ok = below_width(x, 2 * a.L) && hd == a.n_dn && hu == a.n_up;
    if (!ok) {
        dn = 0;
        up = 0;
    }
    const uint64_t rd = stag_rank<P, E>(dn, tab, a.half);
    const uint64_t ru = stag_rank<P, E>(up, tab, a.half);
    return ok ? (uint32_t)(ru * a.mult + rd) : MBR_NOT_FOUND;
}

template <class P, class E, bool USE_LDS, int V>
__global__ void __launch_bounds__(kBlock) rank_spin_kernel(const P *__restrict__ q, uint64_t n,
                                                           uint32_t *__restrict__ out,
                                                           const E *__restrict__ gtab, SpinArgs a) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const uint64_t nv = n / V;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    P x[kVecs][V];
    auto load = [&](uint64_t base) {
#pragma unroll
        for (int u = 0; u < kVecs; ++u) {
            const uint64_t j = base + u * stride;
            if (j < nv) load_vec<P, V>(q, j, x[u]);
        }
    };
    load(t0);
    const E *tab = gtab;
    if constexpr (USE_LDS) {
        E *t = reinterpret_cast<E *>(lds_raw);
        load_table(t, gtab, a.half.nentries);
        tab = t;
    }
    for (uint64_t base = t0; base < nv; base += stride * kVecs) {
        if (base != t0) load(base);
#pragma unroll
        for (int u = 0; u < kVecs; ++u) {
            const uint64_t j = base + u * stride;
            if (j < nv) {
                uint32_t r[V];
#pragma unroll
                for (int i = 0; i < V; ++i) r[i] = spin_query<P, E>(x[u][i], tab, a);
                store_vec<uint32_t, V>(out, j, r);
            }
        }
    }
    if (t0 < n - nv * V) {
        const uint64_t j = nv * V + t0;
        out[j] = spin_query<P, E>(q[j], tab, a);
    }
}

StagArgs make_args(const StagTable &t, int N) {
    StagArgs a{};
    a.M = t.M;
    a.k = t.k;
    a.nch = t.nch;
    a.N = N;
    for (int c = 0; c < t.nch && c < 16; ++c) a.rowoff[c] = t.rowoff[c];
    a.nentries = (uint64_t)t.nrows << t.k;
    return a;
}

// Tables up to this size are staged in LDS (several workgroups per CU still fit).
constexpr size_t kLdsTable = 64 * 1024;

template <class K>
mbr_status set_lds(K kernel, size_t bytes) {
    if (bytes > 64 * 1024)
        MBR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return MBR_OK;
}

// Vector width for a launch: 16-byte accesses when both the queries and the
// ranks are aligned to them, otherwise one pattern per access.
template <class P, class RT = uint32_t>
bool vec_aligned(const void *q, const RT *out) {
    constexpr int V = 16 / sizeof(P);
    return ((uintptr_t)q % 16 == 0) && ((uintptr_t)out % (sizeof(RT) * V) == 0);
}

template <class P, class E, int V, class RT>
mbr_status launch_stag_v(const mbr_ranker *r, const void *q, uint64_t n, RT *out, hipStream_t s) {
    StagArgs a = make_args(r->stag, r->N);
    const E *tab = r->stag.table.as<E>();
    if (r->stag.trim_entries) {
        // fixed N: the trimmed rows, and the lowest member in place of a non-member
        for (int c = 0; c < a.nch; ++c) a.rowoff[c] = r->stag.trim_rowoff[c];
        a.nentries = r->stag.trim_entries;
        a.safe = r->N >= 64 ? ~0ull : ((1ull << r->N) - 1);
        tab = r->stag.trim.as<E>();
    }
    size_t lds = a.nentries * sizeof(E);
    unsigned grid = mbr::grid_for((n + V - 1) / V, kBlock * kVecs, mbr::device_cu_count() * 8);
    if (lds <= kLdsTable) {
        auto kern = rank_staggered_kernel<P, E, true, V, RT>;
        MBR_TRY(set_lds(kern, lds));
        kern<<<grid, kBlock, lds, s>>>(static_cast<const P *>(q), n, out, tab, a);
    } else {
        rank_staggered_kernel<P, E, false, V, RT><<<grid, kBlock, 0, s>>>(static_cast<const P *>(q), n, out,
                                                                         tab, a);
    }
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

template <class P, class E, class RT>
mbr_status launch_stag(const mbr_ranker *r, const void *q, uint64_t n, RT *out, hipStream_t s) {
    if (vec_aligned<P, RT>(q, out)) return launch_stag_v<P, E, 16 / sizeof(P), RT>(r, q, n, out, s);
    return launch_stag_v<P, E, 1, RT>(r, q, n, out, s);
}

template <class P, class E, int V>
mbr_status launch_spin_v(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out,
                         hipStream_t s) {
    SpinArgs a{};
    a.half = make_args(r->stag, -1);
    a.L = r->L;
    a.n_up = r->n_up;
    a.n_dn = r->n_dn;
    a.mult = (uint32_t)mbr::binom(r->L, r->n_dn);
    size_t lds = a.half.nentries * sizeof(E);
    unsigned grid = mbr::grid_for((n + V - 1) / V, kBlock * kVecs, mbr::device_cu_count() * 8);
    if (lds <= kLdsTable) {
        auto kern = rank_spin_kernel<P, E, true, V>;
        MBR_TRY(set_lds(kern, lds));
        kern<<<grid, kBlock, lds, s>>>(static_cast<const P *>(q), n, out, r->stag.table.as<E>(), a);
    } else {
        rank_spin_kernel<P, E, false, V><<<grid, kBlock, 0, s>>>(static_cast<const P *>(q), n, out,
                                                                r->stag.table.as<E>(), a);
    }
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

template <class P, class E>
mbr_status launch_spin(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out,
                       hipStream_t s) {
    if (vec_aligned<P>(q, out)) return launch_spin_v<P, E, 16 / sizeof(P)>(r, q, n, out, s);
    return launch_spin_v<P, E, 1>(r, q, n, out, s);
}

}  // namespace

mbr_status rank_staggered_launch(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out,
                                 hipStream_t s) {
    if (r->rank64) MBR_FAIL(MBR_ERANGE, "ranks of this sector need 64 bits: use mbr_rank_batch64");
    int eb = r->stag.entry_bytes;
    if (r->width_bits == 32) {
        if (eb == 2) return launch_stag<uint32_t, uint16_t>(r, q, n, out, s);
        if (eb == 4) return launch_stag<uint32_t, uint32_t>(r, q, n, out, s);
        return launch_stag<uint32_t, uint64_t>(r, q, n, out, s);
    }
    if (eb == 2) return launch_stag<uint64_t, uint16_t>(r, q, n, out, s);
    if (eb == 4) return launch_stag<uint64_t, uint32_t>(r, q, n, out, s);
    return launch_stag<uint64_t, uint64_t>(r, q, n, out, s);
}

mbr_status rank_staggered_launch64(const mbr_ranker *r, const void *q, uint64_t n, uint64_t *out,
                                   hipStream_t s) {
    int eb = r->stag.entry_bytes;
    if (r->width_bits == 32) {
        if (eb == 2) return launch_stag<uint32_t, uint16_t>(r, q, n, out, s);
        if (eb == 4) return launch_stag<uint32_t, uint32_t>(r, q, n, out, s);
        return launch_stag<uint32_t, uint64_t>(r, q, n, out, s);
    }
    if (eb == 2) return launch_stag<uint64_t, uint16_t>(r, q, n, out, s);
    if (eb == 4) return launch_stag<uint64_t, uint32_t>(r, q, n, out, s);
    return launch_stag<uint64_t, uint64_t>(r, q, n, out, s);
}

mbr_status rank_spin_launch(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out,
                            hipStream_t s) {
    int eb = r->stag.entry_bytes;
    if (r->width_bits == 32) {
        if (eb == 2) return launch_spin<uint32_t, uint16_t>(r, q, n, out, s);
        if (eb == 4) return launch_spin<uint32_t, uint32_t>(r, q, n, out, s);
        return launch_spin<uint32_t, uint64_t>(r, q, n, out, s);
    }
    if (eb == 2) return launch_spin<uint64_t, uint16_t>(r, q, n, out, s);
    if (eb == 4) return launch_spin<uint64_t, uint32_t>(r, q, n, out, s);
    return launch_spin<uint64_t, uint64_t>(r, q, n, out, s);
}

#define MBR_FAIL_DEL(obj, code, ...) \
    do {                             \
        delete (obj);                \
        MBR_FAIL(code, __VA_ARGS__); \
    } while (0)

extern "C" {

mbr_status mbr_build_staggered_tables(int32_t M, int32_t N, int32_t k, int32_t width_bits,
                                      mbr_ranker **out, void *stream) {
    using namespace mbr;
    if (!out) MBR_FAIL(MBR_EINVAL, "null output handle");
    *out = nullptr;
    if (M < 1 || M > 64) MBR_FAIL(MBR_EINVAL, "M=%d outside 1..64", M);
    if (k < 1 || k > 16) MBR_FAIL(MBR_EINVAL, "k=%d outside 1..16", k);
    if (width_bits != 32 && width_bits != 64) MBR_FAIL(MBR_EINVAL, "width_bits=%d", width_bits);
    if (width_bits == 32 && M > 32) MBR_FAIL(MBR_EINVAL, "M=%d needs 64-bit patterns", M);
    if (N < -1 || N > M) MBR_FAIL(MBR_EINVAL, "N=%d outside -1..M", N);
    int nch = (M + k - 1) / k;
    if (nch > 16) MBR_FAIL(MBR_EUNSUPPORTED, "%d chunks (at most 16)", nch);
    int nmax = N < 0 ? M : N;
    uint64_t worst = 0;
    for (int n = (N < 0 ? 0 : N); n <= (N < 0 ? M : N); ++n) worst = binom(M, n) > worst ? binom(M, n) : worst;
    if (M == 64 && N < 0) MBR_FAIL(MBR_ERANGE, "a universal table at M=64 holds 2^64 states");
    auto *r = new (std::nothrow) mbr_ranker;
    if (!r) MBR_FAIL(MBR_ENOMEM, "host allocation");
    r->kind = MBR_RANKER_STAGGERED;
    r->M = M;
    r->k = k;
    r->N = N;
    r->width_bits = width_bits;
    r->n_states = N < 0 ? (1ull << M) : binom(M, N);
    r->rank64 = worst >= 0xFFFFFFFFull;  // ranks need the 64-bit entry point
    (void)hipGetDevice(&r->device);
    if (((uint64_t)(nch * (nmax + 1)) << k) > (1ull << 26))
        MBR_FAIL_DEL(r, MBR_EUNSUPPORTED, "staggered table beyond 2^26 entries");
    mbr_status st = stag_build(r->stag, M, k, nmax, entry_bytes_for(M, nmax), as_stream(stream));
    if (st == MBR_OK && N >= 0) st = stag_trim(r->stag, N, as_stream(stream));
    if (st != MBR_OK) {
        delete r;
        return st;
    }
    *out = r;
    return MBR_OK;
}

mbr_status mbr_staggered_table_copy(const mbr_ranker *r, uint64_t *host_out, uint64_t cap,
                                    uint64_t *n_entries, void *stream) {
    (void)stream;
    if (!r) MBR_FAIL(MBR_EINVAL, "null ranker");
    if (r->kind != MBR_RANKER_STAGGERED && r->kind != MBR_RANKER_SPIN)
        MBR_FAIL(MBR_EINVAL, "not a staggered or spin ranker");
    uint64_t n = (uint64_t)r->stag.nrows << r->stag.k;
    if (n_entries) *n_entries = n;
    if (!host_out || cap < n) return MBR_OK;
    // Read back what the device holds, widened to uint64.
    size_t eb = r->stag.entry_bytes;
    std::vector<unsigned char> raw(n * eb);
    MBR_HIP(hipMemcpy(raw.data(), r->stag.table.p, n * eb, hipMemcpyDeviceToHost));
    for (uint64_t i = 0; i < n; ++i) {
        if (eb == 2) host_out[i] = reinterpret_cast<uint16_t *>(raw.data())[i];
        else if (eb == 4) host_out[i] = reinterpret_cast<uint32_t *>(raw.data())[i];
        else host_out[i] = reinterpret_cast<uint64_t *>(raw.data())[i];
    }
    return MBR_OK;
}

mbr_status mbr_build_spin_ranker(int32_t L, int32_t n_up, int32_t n_dn, int32_t k,
                                 mbr_ranker **out, void *stream) {
    using namespace mbr;
    if (!out) MBR_FAIL(MBR_EINVAL, "null output handle");
    *out = nullptr;
    if (L < 1 || L > 32) MBR_FAIL(MBR_EINVAL, "L=%d outside 1..32", L);
    if (n_up < 0 || n_up > L || n_dn < 0 || n_dn > L) MBR_FAIL(MBR_EINVAL, "particle numbers (%d,%d)", n_up, n_dn);
    if (k < 1 || k > 16) MBR_FAIL(MBR_EINVAL, "k=%d outside 1..16", k);
    uint64_t total = binom(L, n_up) * binom(L, n_dn);
    if (total >= 0xFFFFFFFFull) MBR_FAIL(MBR_ERANGE, "spin sector of %llu states", (unsigned long long)total);
    auto *r = new (std::nothrow) mbr_ranker;
    if (!r) MBR_FAIL(MBR_ENOMEM, "host allocation");
    r->kind = MBR_RANKER_SPIN;
    r->M = 2 * L;
    r->L = L;
    r->k = k;
    r->n_up = n_up;
    r->n_dn = n_dn;
    r->width_bits = (2 * L <= 32) ? 32 : 64;
    r->n_states = total;
    (void)hipGetDevice(&r->device);
    int nmax = n_up > n_dn ? n_up : n_dn;
    int eb = entry_bytes_for(L, nmax);
    if ((L + k - 1) / k > 16) MBR_FAIL_DEL(r, MBR_EUNSUPPORTED, "more than 16 chunks");
    mbr_status st = stag_build(r->stag, L, k, nmax, eb, as_stream(stream));
    if (st == MBR_OK) st = spin_unrank_build(r, as_stream(stream));
    if (st != MBR_OK) {
        delete r;
        return st;
    }
    *out = r;
    return MBR_OK;
}

}  // extern "C"
