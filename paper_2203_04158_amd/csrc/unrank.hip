// Unrank in a spin-resolved sector without its state list: the inverse of
// Eq. rankupdown.  Index i splits into r_up = i / C(L, n_dn) and
// r_dn = i mod C(L, n_dn); each half is the r-th pattern of N set bits among L
// in ascending order (Sec. II, Eq. unrank), and the pattern is
// (half_up << L) | half_dn, spin-down in the low L bits.
//
// Two ways to form a half, both with a table staged in LDS:
//  * lists: both halves' ascending patterns as uint16 (L <= 16 and at most
//    kMaxListEntries patterns in the two lists): one LDS read per half;
//  * combinadics: the greedy inversion of Eq. cns over a table of C(c, k),
//    c < L, k <= L: walking c from L - 1 down, bit c is set when C(c, k) does
//    not exceed what is left of r (then r -= C(c, k) and k -= 1).
// Either way the kernel reads 4 bytes of index and writes one pattern per
// query; nothing else leaves the chip.
#include <cstring>

#include "common.hpp"
#include "rank_device.hpp"

namespace {

// Large workgroups, two per CU, each staging its table once: the uint16 lists
// of L = 16 take 51.5 KB, and two such workgroups still fill a CU with 32 waves.
constexpr unsigned kBlock = 1024;
constexpr int kQ = 4;                        // queries in flight per lane
constexpr uint32_t kMaxListEntries = 32768;  // uint16 half lists: 64 KB of LDS

struct SpinUnrankArgs {
    uint64_t total;  // C(L, n_up) C(L, n_dn)
    uint32_t cup, cdn;
    int32_t L, n_up, n_dn;
};

__device__ __forceinline__ uint32_t half_unrank(uint32_t r, int N, const uint32_t *bt, int L) {
    uint32_t x = 0;
    int k = N;
    for (int c = L - 1; c >= 0; --c) {
        if (k > 0) {
            const uint32_t b = bt[c * (L + 1) + k];
            if (r >= b) {
                x |= 1u << c;
                r -= b;
                --k;
            }
        }
    }
    return x;
}

// V queries per lane and vector access: a V-wide load of indices and one
// 16-byte store of patterns (V = 16 / sizeof(P)); V = 1 when the buffers are
// not so aligned.  The first indices are loaded before the table is staged.
template <class P, bool LISTS, int V>
__global__ void __launch_bounds__(kBlock) unrank_spin_kernel(const uint32_t *__restrict__ idx, uint64_t n,
                                                             P *__restrict__ out,
                                                             const void *__restrict__ gtab, uint32_t tab_bytes,
                                                             SpinUnrankArgs a) {
    typedef uint32_t ivec __attribute__((ext_vector_type(V)));
    typedef P pvec __attribute__((ext_vector_type(V)));
    extern __shared__ __align__(16) unsigned char lds[];
    const uint16_t *lists = reinterpret_cast<const uint16_t *>(lds);
    const uint32_t *bt = reinterpret_cast<const uint32_t *>(lds);
    auto one = [&](uint32_t i) -> P {
        if (i >= a.total) return ~(P)0;
        const uint32_t ru = i / a.cdn, rd = i - ru * a.cdn;
        uint32_t hu, hd;
        if constexpr (LISTS) {
            hu = lists[ru];
            hd = lists[a.cup + rd];
        } else {
            hu = half_unrank(ru, a.n_up, bt, a.L);
            hd = half_unrank(rd, a.n_dn, bt, a.L);
        }
        return ((P)hu << a.L) | (P)hd;
    };
    const uint64_t nv = n / V;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    ivec iv[kQ];
    auto load = [&](uint64_t base) {
#pragma unroll
        for (int u = 0; u < kQ; ++u) {
            const uint64_t j = base + u * stride;
            if (j < nv) iv[u] = reinterpret_cast<const ivec *>(idx)[j];
        }
    };
    load(t0);
    stage_to_lds(lds, gtab, tab_bytes);
    __syncthreads();
    for (uint64_t base = t0; base < nv; base += stride * kQ) {
        if (base != t0) load(base);
#pragma unroll
        for (int u = 0; u < kQ; ++u) {
            const uint64_t j = base + u * stride;
            if (j < nv) {
                pvec o;
#pragma unroll
                for (int e = 0; e < V; ++e) o[e] = one(iv[u][e]);
                reinterpret_cast<pvec *>(out)[j] = o;
            }
        }
    }
    if (t0 < n - nv * V) {
        const uint64_t j = nv * V + t0;
        out[j] = one(idx[j]);
    }
}

// Ascending patterns of N set bits among L (Gosper's next-combination step).
void append_half(std::vector<uint16_t> &v, int L, int N) {
    const uint64_t cnt = mbr::binom(L, N);
    uint32_t x = N == 0 ? 0u : ((1u << N) - 1u);
    for (uint64_t t = 0; t < cnt; ++t) {
        v.push_back((uint16_t)x);
        if (x == 0) break;
        const uint32_t c = x & (0u - x), r = x + c;
        x = (((r ^ x) >> 2) / c) | r;
    }
}

template <class P, bool LISTS, int V>
mbr_status launch_v(const mbr_ranker *r, const uint32_t *d_idx, uint64_t n, void *d_out, hipStream_t s) {
    SpinUnrankArgs a{};
    a.total = r->n_states;
    a.cup = (uint32_t)mbr::binom(r->L, r->n_up);
    a.cdn = (uint32_t)mbr::binom(r->L, r->n_dn);
    a.L = r->L;
    a.n_up = r->n_up;
    a.n_dn = r->n_dn;
    const unsigned grid = mbr::grid_for((n + V - 1) / V, kBlock * kQ, mbr::device_cu_count() * 2);
    const uint32_t bytes = (uint32_t)r->unrank_tab.bytes;
    unrank_spin_kernel<P, LISTS, V><<<grid, kBlock, bytes, s>>>(d_idx, n, static_cast<P *>(d_out),
                                                                 r->unrank_tab.p, bytes, a);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

template <class P, bool LISTS>
mbr_status launch(const mbr_ranker *r, const uint32_t *d_idx, uint64_t n, void *d_out, hipStream_t s) {
    constexpr int V = 16 / sizeof(P);
    const bool aligned = reinterpret_cast<uintptr_t>(d_idx) % (4 * V) == 0 &&
                         reinterpret_cast<uintptr_t>(d_out) % 16 == 0;
    return aligned ? launch_v<P, LISTS, V>(r, d_idx, n, d_out, s) : launch_v<P, LISTS, 1>(r, d_idx, n, d_out, s);
}

}  // namespace

mbr_status spin_unrank_build(mbr_ranker *r, hipStream_t s) {
    using namespace mbr;
    const int L = r->L;
    const uint64_t cup = binom(L, r->n_up), cdn = binom(L, r->n_dn);
    std::vector<uint32_t> words;
    if (L <= 16 && cup + cdn <= kMaxListEntries) {
        std::vector<uint16_t> h;
        h.reserve(cup + cdn + 8);
        append_half(h, L, r->n_up);
        append_half(h, L, r->n_dn);
        while (h.size() % 8) h.push_back(0);  // whole 16-byte copies into LDS
        words.resize(h.size() / 2);
        std::memcpy(words.data(), h.data(), h.size() * 2);
        r->unrank_lists = true;
    } else {
        words.assign((size_t)L * (L + 1), 0u);
        for (int c = 0; c < L; ++c)
            for (int k = 0; k <= L; ++k) words[(size_t)c * (L + 1) + k] = (uint32_t)binom(c, k);
        while (words.size() % 4) words.push_back(0);
        r->unrank_lists = false;
    }
    return upload(r->unrank_tab, words.data(), words.size() * 4, s);
}

extern "C" {

mbr_status mbr_unrank_spin_batch(const mbr_ranker *r, const uint32_t *d_idx, uint64_t n, void *d_out,
                                 void *stream) {
    using namespace mbr;
    if (!r) MBR_FAIL(MBR_EINVAL, "null ranker");
    if (r->kind != MBR_RANKER_SPIN) MBR_FAIL(MBR_EINVAL, "ranker kind %d is not a spin ranker", r->kind);
    if (n == 0) return MBR_OK;
    if (!d_idx || !d_out) MBR_FAIL(MBR_EINVAL, "null index or output pointer");
    hipStream_t s = as_stream(stream);
    if (r->width_bits == 32)
        return r->unrank_lists ? launch<uint32_t, true>(r, d_idx, n, d_out, s)
                               : launch<uint32_t, false>(r, d_idx, n, d_out, s);
    return r->unrank_lists ? launch<uint64_t, true>(r, d_idx, n, d_out, s)
                           : launch<uint64_t, false>(r, d_idx, n, d_out, s);
}

}  // extern "C"
