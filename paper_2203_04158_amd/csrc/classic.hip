// The two established ranking methods the paper measures its own against
// (Sec. III, Sec. V.A):
//  * bisection: the lower bound of the pattern in the sector's ascending state
//    list, accepted when the entry equals the pattern (any sector);
//  * combinadics ranking (Eq. cns, Sec. III.A): the sum of C(c_k, k) over the
//    occupied positions c_1 < ... < c_N, taken position by position
//    (particle-number sectors C^M_N only).
// Both keep the batch layout of the other rankers: queries in, ranks out,
// MBR_NOT_FOUND for patterns outside the sector.
#include <memory>

#include "common.hpp"

namespace {

constexpr unsigned kBlock = 256;
constexpr int kQ = 4;  // independent queries in flight per lane

template <class P>
__device__ __forceinline__ bool fits(P x, int M) {
    return (M >= (int)(8 * sizeof(P))) ? true : (x >> M) == 0;
}

// kQ bisections side by side, one probe of each per step, so that their
// dependent loads overlap.
template <class P>
__global__ void __launch_bounds__(kBlock) rank_bisect_kernel(const P *__restrict__ q, uint64_t n,
                                                             uint32_t *__restrict__ out,
                                                             const P *__restrict__ states, uint64_t ns,
                                                             int M) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; base < n; base += stride * kQ) {
        P x[kQ];
        uint64_t lo[kQ], len[kQ];
#pragma unroll
        for (int u = 0; u < kQ; ++u) {
            const uint64_t j = base + u * stride;
            x[u] = j < n ? q[j] : (P)0;
            lo[u] = 0;
            len[u] = ns;
        }
        // lower bound: the first index whose state is not below x
        for (bool more = true; more;) {
            more = false;
#pragma unroll
            for (int u = 0; u < kQ; ++u) {
                if (len[u] > 0) {
                    const uint64_t half = len[u] >> 1;
                    if (states[lo[u] + half] < x[u]) {
                        lo[u] += half + 1;
                        len[u] -= half + 1;
                    } else {
                        len[u] = half;
                    }
                    more = more || len[u] > 0;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kQ; ++u) {
            const uint64_t j = base + u * stride;
            if (j < n) {
                const bool hit = fits(x[u], M) && lo[u] < ns && states[lo[u]] == x[u];
                out[j] = hit ? (uint32_t)lo[u] : MBR_NOT_FOUND;
            }
        }
    }
}

// Binomial rows C(c, k) for c < M, k = 1..N as uint32, row-major by c.
// Members of C^M_N have ranks below C(M, N) < 2^32 and every partial sum of
// Eq. cns is at most the rank, so entries that do not fit 32 bits are never
// read for a member; they are stored saturated.
template <class P>
__global__ void __launch_bounds__(kBlock) rank_cns_kernel(const P *__restrict__ q, uint64_t n,
                                                          uint32_t *__restrict__ out,
                                                          const uint32_t *__restrict__ gtab, int M, int N) {
    extern __shared__ uint32_t tab[];  // [M][N + 1]
    const int ld = N + 1;
    for (int i = threadIdx.x; i < M * ld; i += blockDim.x) tab[i] = gtab[i];
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < n; j += stride) {
        P x = q[j];
        const int h = (sizeof(P) == 8) ? __popcll((uint64_t)x) : __popc((uint32_t)x);
        const bool ok = fits(x, M) && h == N;
        uint32_t r = 0;
        if (ok) {
            // Eq. cns position by position: k counts the occupied orbitals
            // seen so far, and an occupied position c adds C(c, k); k <= N
            // keeps every read inside the table
            int k = 0;
            for (int c = 0; c < M; ++c) {
                const uint32_t occ = (uint32_t)(x >> c) & 1u;
                k += (int)occ;
                r += occ ? tab[c * ld + k] : 0u;
            }
        }
        out[j] = ok ? r : MBR_NOT_FOUND;
    }
}

template <class P>
mbr_status launch_bisect(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out, hipStream_t s) {
    const unsigned grid = mbr::grid_for(n, kBlock * kQ, mbr::device_cu_count() * 8);
    rank_bisect_kernel<P><<<grid, kBlock, 0, s>>>(static_cast<const P *>(q), n, out,
                                                  r->sector->states.as<P>(), r->sector->n, r->M);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

template <class P>
mbr_status launch_cns(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out, hipStream_t s) {
    const unsigned grid = mbr::grid_for(n, kBlock, mbr::device_cu_count() * 8);
    const size_t lds = (size_t)r->M * (r->N + 1) * 4;
    rank_cns_kernel<P><<<grid, kBlock, lds, s>>>(static_cast<const P *>(q), n, out,
                                                 r->stag.table.as<uint32_t>(), r->M, r->N);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

}  // namespace

mbr_status rank_bisect_launch(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out,
                              hipStream_t s) {
    if (r->width_bits == 32) return launch_bisect<uint32_t>(r, q, n, out, s);
    return launch_bisect<uint64_t>(r, q, n, out, s);
}

mbr_status rank_cns_launch(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out,
                           hipStream_t s) {
    if (r->width_bits == 32) return launch_cns<uint32_t>(r, q, n, out, s);
    return launch_cns<uint64_t>(r, q, n, out, s);
}

extern "C" {

mbr_status mbr_build_bisect_ranker(const mbr_sector *sec, mbr_ranker **out) {
    using namespace mbr;
    if (!out) MBR_FAIL(MBR_EINVAL, "null output handle");
    *out = nullptr;
    if (!sec) MBR_FAIL(MBR_EINVAL, "null sector");
    if (sec->n == 0) MBR_FAIL(MBR_EINVAL, "empty sector");
    auto r = std::make_unique<mbr_ranker>();
    r->kind = MBR_RANKER_BISECT;
    r->M = sec->M;
    r->k = 0;
    r->width_bits = sec->width_bits;
    r->n_states = sec->n;
    r->sector = sec;
    (void)hipGetDevice(&r->device);
    *out = r.release();
    return MBR_OK;
}

mbr_status mbr_build_cns_ranker(int32_t M, int32_t N, int32_t width_bits, mbr_ranker **out, void *stream) {
    using namespace mbr;
    if (!out) MBR_FAIL(MBR_EINVAL, "null output handle");
    *out = nullptr;
    if (M < 1 || M > 64) MBR_FAIL(MBR_EINVAL, "M=%d outside 1..64", M);
    if (width_bits != 32 && width_bits != 64) MBR_FAIL(MBR_EINVAL, "width_bits=%d", width_bits);
    if (width_bits == 32 && M > 32) MBR_FAIL(MBR_EINVAL, "M=%d needs 64-bit patterns", M);
    if (N < 0 || N > M) MBR_FAIL(MBR_EINVAL, "N=%d outside 0..M", N);
    if (binom(M, N) >= 0xFFFFFFFFull)
        MBR_FAIL(MBR_ERANGE, "C(%d,%d) ranks do not fit 32 bits", M, N);
    auto r = std::make_unique<mbr_ranker>();
    r->kind = MBR_RANKER_CNS;
    r->M = M;
    r->k = 1;
    r->N = N;
    r->width_bits = width_bits;
    r->n_states = binom(M, N);
    (void)hipGetDevice(&r->device);
    std::vector<uint32_t> t((size_t)M * (N + 1));
    for (int c = 0; c < M; ++c)
        for (int k = 0; k <= N; ++k) {
            const uint64_t b = binom(c, k);
            t[(size_t)c * (N + 1) + k] = b > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)b;
        }
    MBR_TRY(upload(r->stag.table, t.data(), t.size() * 4, as_stream(stream)));
    *out = r.release();
    return MBR_OK;
}

}  // extern "C"
