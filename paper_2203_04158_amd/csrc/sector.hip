// Sector enumeration on the device and unrank by the stored list.
//
// A sector is every M-bit pattern passing a set of popcount windows, in
// ascending numeric order (Sec. III ordering).  When the particle number N is
// fixed the enumeration walks only the C(M,N) patterns of that number: each
// thread owns a run of consecutive combination indices, positions itself with
// a greedy combinadics unrank (inverse of Eq. cns) and steps to the next larger
// pattern of equal popcount with Gosper's rule.  Runs are visited in increasing
// order, so a count pass, an exclusive scan of the per-run counts and a write
// pass give the sorted list without any sort.
#include <memory>
#include <numeric>

#include "common.hpp"

namespace {

constexpr int kMaxCons = 16;

struct ConsSet {
    uint64_t mask[kMaxCons];
    int32_t lo[kMaxCons];
    int32_t hi[kMaxCons];
    int32_t n;
    int32_t modulus, residue;  // modulus > 0: sum of the weights of the set bits = residue (mod modulus)
    int32_t weight[64];
};

__device__ __forceinline__ bool in_sector(uint64_t a, const ConsSet &cs) {
    bool ok = true;
    for (int j = 0; j < cs.n; ++j) {
        int h = __popcll(a & cs.mask[j]);
        ok = ok && (h >= cs.lo[j]) && (h <= cs.hi[j]);
    }
    if (ok && cs.modulus > 0) {
        int64_t w = 0;
        for (uint64_t m = a; m; m &= m - 1) w += cs.weight[__builtin_ctzll(m)];
        int64_t r = w % cs.modulus;
        if (r < 0) r += cs.modulus;
        ok = r == cs.residue;
    }
    return ok;
}

// Pattern with combinadics index u among N-of-M patterns (greedy inversion of
// Eq. cns: the largest c with C(c, k) <= u is c_k).
__device__ __forceinline__ uint64_t combo_at(uint64_t u, int N, int M, const uint64_t *bt) {
    uint64_t a = 0;
    int c = M - 1;
    for (int k = N; k >= 1; --k) {
        while (bt[c * 65 + k] > u) --c;
        a |= 1ull << c;
        u -= bt[c * 65 + k];
        --c;
    }
    return a;
}

// Next larger pattern with the same popcount (Gosper).
__device__ __forceinline__ uint64_t next_combo(uint64_t a) {
    uint64_t c = a & (~a + 1);
    uint64_t r = a + c;
    int tz = __builtin_ctzll(a);  // c = 2^tz, so the division by c is a shift
    return (((r ^ a) >> 2) >> tz) | r;
}

template <bool FIXED>
__device__ __forceinline__ uint64_t run_start(uint64_t u0, int N, int M, const uint64_t *bt) {
    if constexpr (FIXED) return combo_at(u0, N, M, bt);
    else return u0;
}

template <bool FIXED>
__device__ __forceinline__ uint64_t run_next(uint64_t a) {
    if constexpr (FIXED) return next_combo(a);
    else return a + 1;
}

template <bool FIXED>
__global__ void sector_count_kernel(uint64_t S, uint64_t run, int N, int M, ConsSet cs,
                                    const uint64_t *bt, uint32_t *counts, uint64_t nruns) {
    uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (t >= nruns) return;
    uint64_t u0 = t * run;
    uint64_t len = (S - u0 < run) ? S - u0 : run;
    uint64_t a = run_start<FIXED>(u0, N, M, bt);
    uint32_t cnt = 0;
    for (uint64_t j = 0; j < len; ++j) {
        cnt += in_sector(a, cs) ? 1u : 0u;
        if (j + 1 < len) a = run_next<FIXED>(a);
    }
    counts[t] = cnt;
}

template <bool FIXED, class P>
__global__ void sector_fill_kernel(uint64_t S, uint64_t run, int N, int M, ConsSet cs,
                                   const uint64_t *bt, const uint64_t *offsets, P *out,
                                   uint64_t nruns) {
    uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (t >= nruns) return;
    uint64_t u0 = t * run;
    uint64_t len = (S - u0 < run) ? S - u0 : run;
    uint64_t a = run_start<FIXED>(u0, N, M, bt);
    uint64_t o = offsets[t];
    for (uint64_t j = 0; j < len; ++j) {
        if (in_sector(a, cs)) out[o++] = static_cast<P>(a);
        if (j + 1 < len) a = run_next<FIXED>(a);
    }
}

// First position that breaks a caller's list: for j >= 1, list[j] below its
// predecessor (code 1), equal to it (code 2), or any entry with bits at or
// above M (code 3).  The smallest (position << 2 | code) wins, so the first
// offending position decides and the result does not depend on scheduling.
template <class P>
__global__ void list_check_kernel(const P *__restrict__ a, uint64_t n, int M, unsigned long long *first) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long best = ~0ull;
    for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < n; j += stride) {
        const P v = a[j];
        unsigned code = 0;
        if (M < (int)(8 * sizeof(P)) && (v >> M) != 0) code = 3;
        if (j > 0) {
            const P u = a[j - 1];
            if (u > v) code = 1;
            else if (u == v) code = 2;
        }
        if (code) {
            const unsigned long long key = ((unsigned long long)j << 2) | code;
            best = key < best ? key : best;
            break;  // later positions of this lane cannot be smaller
        }
    }
    if (best != ~0ull) atomicMin(first, best);
}

template <class P>
__global__ void unrank_kernel(const P *__restrict__ states, uint64_t nstates,
                              const uint32_t *__restrict__ idx, uint64_t n, P *__restrict__ out) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < n; j += stride) {
        uint32_t i = idx[j];
        out[j] = (i < nstates) ? states[i] : static_cast<P>(~(P)0);
    }
}

// The fixed particle number implied by the windows, or -1.
int implied_n(int M, const std::vector<mbr_popc_cons> &cons) {
    uint64_t full = (M == 64) ? ~0ull : ((1ull << M) - 1);
    for (auto &c : cons)
        if (c.mask == full && c.lo == c.hi) return c.lo;
    uint64_t covered = 0;
    int n = 0;
    for (auto &c : cons) {
        if (c.lo != c.hi) continue;
        if (covered & c.mask) return -1;
        covered |= c.mask;
        n += c.lo;
    }
    return covered == full ? n : -1;
}

mbr_status sector_build_impl(int32_t M, int32_t width_bits, int32_t n_cons, const mbr_popc_cons *cons,
                             const int32_t *weights, int32_t modulus, int32_t residue, mbr_sector **out,
                             void *stream) {
    using namespace mbr;
    if (!out) MBR_FAIL(MBR_EINVAL, "null output handle");
    *out = nullptr;
    if (M < 1 || M > 64) MBR_FAIL(MBR_EINVAL, "M=%d outside 1..64", M);
    if (width_bits != 32 && width_bits != 64) MBR_FAIL(MBR_EINVAL, "width_bits=%d", width_bits);
    if (width_bits == 32 && M > 32) MBR_FAIL(MBR_EINVAL, "M=%d needs 64-bit patterns", M);
    if (n_cons < 0 || n_cons > kMaxCons) MBR_FAIL(MBR_EINVAL, "n_cons=%d outside 0..%d", n_cons, kMaxCons);
    if (n_cons > 0 && !cons) MBR_FAIL(MBR_EINVAL, "null constraint list");
    uint64_t full = (M == 64) ? ~0ull : ((1ull << M) - 1);
    std::vector<mbr_popc_cons> cv(cons, cons + n_cons);
    for (auto &c : cv) {
        if (c.mask & ~full) MBR_FAIL(MBR_EINVAL, "constraint mask has bits at or above M");
        if (c.lo < 0 || c.hi < c.lo || c.hi > 64) MBR_FAIL(MBR_EINVAL, "constraint window [%d,%d]", c.lo, c.hi);
    }
    if (modulus < 0 || (modulus > 0 && (!weights || residue < 0 || residue >= modulus)))
        MBR_FAIL(MBR_EINVAL, "modular constraint: modulus %d, residue %d", modulus, residue);
    int N = implied_n(M, cv);
    uint64_t S;
    if (N >= 0) {
        if (N > M) MBR_FAIL(MBR_EINVAL, "N=%d exceeds M=%d", N, M);
        S = binom(M, N);
        if (S > (1ull << 40)) MBR_FAIL(MBR_EUNSUPPORTED, "C(%d,%d) patterns to scan", M, N);
    } else {
        if (M > 32) MBR_FAIL(MBR_EUNSUPPORTED, "M=%d without a fixed particle number", M);
        S = 1ull << M;
    }
    hipStream_t s = as_stream(stream);
    const uint64_t *bt = nullptr;
    MBR_TRY(device_binom(&bt));
    uint64_t run = 64;
    while ((S + run - 1) / run > (1ull << 24)) run *= 2;
    uint64_t nruns = (S + run - 1) / run;

    ConsSet cs{};
    cs.n = n_cons;
    for (int j = 0; j < n_cons; ++j) {
        cs.mask[j] = cv[j].mask;
        cs.lo[j] = cv[j].lo;
        cs.hi[j] = cv[j].hi;
    }
    cs.modulus = modulus;
    cs.residue = residue;
    for (int i = 0; i < M && modulus > 0; ++i) cs.weight[i] = weights[i] % modulus;
    DevBuf d_counts, d_off;
    MBR_TRY(d_counts.alloc(nruns * sizeof(uint32_t)));
    unsigned blk = 256;
    unsigned grid = static_cast<unsigned>((nruns + blk - 1) / blk);
    if (N >= 0)
        sector_count_kernel<true><<<grid, blk, 0, s>>>(S, run, N, M, cs, bt, d_counts.as<uint32_t>(), nruns);
    else
        sector_count_kernel<false><<<grid, blk, 0, s>>>(S, run, N, M, cs, bt, d_counts.as<uint32_t>(), nruns);
    MBR_HIP(hipGetLastError());
    std::vector<uint32_t> counts(nruns);
    MBR_HIP(hipMemcpyAsync(counts.data(), d_counts.p, nruns * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    MBR_HIP(hipStreamSynchronize(s));
    std::vector<uint64_t> off(nruns);
    uint64_t total = 0;
    for (uint64_t t = 0; t < nruns; ++t) {
        off[t] = total;
        total += counts[t];
    }
    if (total >= 0xFFFFFFFFull) MBR_FAIL(MBR_ERANGE, "sector of %llu states", (unsigned long long)total);

    auto *sec = new (std::nothrow) mbr_sector;
    if (!sec) MBR_FAIL(MBR_ENOMEM, "host allocation");
    sec->M = M;
    sec->width_bits = width_bits;
    sec->n = total;
    sec->cons = cv;
    sec->modulus = modulus;
    sec->residue = residue;
    for (int i = 0; i < M && modulus > 0; ++i) sec->weights.push_back(cs.weight[i]);
    MBR_HIP(hipGetDevice(&sec->device));
    mbr_status st = sec->states.alloc(total * (width_bits / 8));
    if (st == MBR_OK) st = upload(d_off, off.data(), nruns * sizeof(uint64_t), s);
    if (st != MBR_OK) {
        delete sec;
        return st;
    }
    if (total > 0) {
        if (width_bits == 32) {
            if (N >= 0)
                sector_fill_kernel<true, uint32_t><<<grid, blk, 0, s>>>(S, run, N, M, cs, bt, d_off.as<uint64_t>(), sec->states.as<uint32_t>(), nruns);
            else
                sector_fill_kernel<false, uint32_t><<<grid, blk, 0, s>>>(S, run, N, M, cs, bt, d_off.as<uint64_t>(), sec->states.as<uint32_t>(), nruns);
        } else {
            if (N >= 0)
                sector_fill_kernel<true, uint64_t><<<grid, blk, 0, s>>>(S, run, N, M, cs, bt, d_off.as<uint64_t>(), sec->states.as<uint64_t>(), nruns);
            else
                sector_fill_kernel<false, uint64_t><<<grid, blk, 0, s>>>(S, run, N, M, cs, bt, d_off.as<uint64_t>(), sec->states.as<uint64_t>(), nruns);
        }
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            delete sec;
            MBR_FAIL(MBR_EHIP, "sector fill: %s", hipGetErrorString(e));
        }
    }
    *out = sec;
    return MBR_OK;
}

}  // namespace

extern "C" {

mbr_status mbr_sector_build(int32_t M, int32_t width_bits, int32_t n_cons,
                            const mbr_popc_cons *cons, mbr_sector **out, void *stream) {
    return sector_build_impl(M, width_bits, n_cons, cons, nullptr, 0, 0, out, stream);
}

mbr_status mbr_sector_build_mod(int32_t M, int32_t width_bits, int32_t n_cons, const mbr_popc_cons *cons,
                                const int32_t *weights, int32_t modulus, int32_t residue,
                                mbr_sector **out, void *stream) {
    if (modulus < 1) MBR_FAIL(MBR_EINVAL, "modulus %d must be positive", modulus);
    return sector_build_impl(M, width_bits, n_cons, cons, weights, modulus, residue, out, stream);
}

mbr_status mbr_sector_from_list(int32_t M, int32_t width_bits, const void *d_states, uint64_t n,
                                mbr_sector **out, void *stream) {
    using namespace mbr;
    if (!out) MBR_FAIL(MBR_EINVAL, "null output handle");
    *out = nullptr;
    if (M < 1 || M > 64) MBR_FAIL(MBR_EINVAL, "M=%d outside 1..64", M);
    if (width_bits != 32 && width_bits != 64) MBR_FAIL(MBR_EINVAL, "width_bits=%d", width_bits);
    if (width_bits == 32 && M > 32) MBR_FAIL(MBR_EINVAL, "M=%d needs 64-bit patterns", M);
    if (n > 0 && !d_states) MBR_FAIL(MBR_EINVAL, "null state list");
    if (n >= 0xFFFFFFFFull) MBR_FAIL(MBR_ERANGE, "list of %llu states", (unsigned long long)n);
    hipStream_t s = as_stream(stream);
    auto sec = std::make_unique<mbr_sector>();
    sec->M = M;
    sec->width_bits = width_bits;
    sec->n = n;
    sec->from_list = true;
    MBR_HIP(hipGetDevice(&sec->device));
    const size_t bytes = (size_t)n * (width_bits / 8);
    MBR_TRY(sec->states.alloc(bytes));
    if (n > 0) {
        MBR_HIP(hipMemcpyAsync(sec->states.p, d_states, bytes, hipMemcpyDeviceToDevice, s));
        const unsigned long long none = ~0ull;
        DevBuf flag;
        MBR_TRY(upload(flag, &none, sizeof none, s));
        const unsigned grid = grid_for(n, 256, device_cu_count() * 8);
        if (width_bits == 32)
            list_check_kernel<uint32_t><<<grid, 256, 0, s>>>(sec->states.as<uint32_t>(), n, M,
                                                             flag.as<unsigned long long>());
        else
            list_check_kernel<uint64_t><<<grid, 256, 0, s>>>(sec->states.as<uint64_t>(), n, M,
                                                             flag.as<unsigned long long>());
        MBR_HIP(hipGetLastError());
        unsigned long long first = 0;
        MBR_HIP(hipMemcpyAsync(&first, flag.p, sizeof first, hipMemcpyDeviceToHost, s));
        MBR_HIP(hipStreamSynchronize(s));
        if (first != ~0ull) {
            const unsigned long long pos = first >> 2;
            switch (first & 3) {
                case 1: MBR_FAIL(MBR_ENOTSORTED, "entry %llu is smaller than entry %llu", pos, pos - 1);
                case 2: MBR_FAIL(MBR_EDUP, "entry %llu repeats entry %llu", pos, pos - 1);
                default: MBR_FAIL(MBR_EINVAL, "entry %llu has bits at or above M=%d", pos, M);
            }
        }
    }
    *out = sec.release();
    return MBR_OK;
}

mbr_status mbr_sector_size(const mbr_sector *s, uint64_t *n) {
    if (!s || !n) MBR_FAIL(MBR_EINVAL, "null argument");
    *n = s->n;
    return MBR_OK;
}

mbr_status mbr_sector_states(const mbr_sector *s, const void **d_states) {
    if (!s || !d_states) MBR_FAIL(MBR_EINVAL, "null argument");
    *d_states = s->states.p;
    return MBR_OK;
}

mbr_status mbr_sector_destroy(mbr_sector *s) {
    delete s;
    return MBR_OK;
}

mbr_status mbr_unrank_batch(const mbr_sector *sec, const uint32_t *d_idx, uint64_t n, void *d_out,
                            void *stream) {
    using namespace mbr;
    if (!sec) MBR_FAIL(MBR_EINVAL, "null sector");
    if (n == 0) return MBR_OK;
    if (!d_idx || !d_out) MBR_FAIL(MBR_EINVAL, "null index or output pointer");
    hipStream_t s = as_stream(stream);
    unsigned blk = 256;
    unsigned grid = grid_for(n, blk, 65536);
    if (sec->width_bits == 32)
        unrank_kernel<uint32_t><<<grid, blk, 0, s>>>(sec->states.as<uint32_t>(), sec->n, d_idx, n,
                                                     static_cast<uint32_t *>(d_out));
    else
        unrank_kernel<uint64_t><<<grid, blk, 0, s>>>(sec->states.as<uint64_t>(), sec->n, d_idx, n,
                                                     static_cast<uint64_t *>(d_out));
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

}  // extern "C"
