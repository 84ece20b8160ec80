// Gather probe: the measured ceilings behind the rooflines of the gather-bound
// kernels (trie walks, window searches, the up-hop gathers of H·x).  Each
// lane follows chains of random 4-byte reads through a table of a chosen
// footprint; with depth > 1 every read's address comes from the previous
// read, as in a trie walk.  A measurement primitive, not a step of the method.
#include "rank_device.hpp"

namespace {

constexpr unsigned kBlock = 256;
constexpr int kQ = 4;                     // independent chains in flight per lane
constexpr uint64_t kLdsEntries = 16384;   // 64 KB of LDS

template <bool LDS>
__global__ void __launch_bounds__(kBlock) probe_gather_kernel(const uint32_t *__restrict__ tab, uint32_t mask,
                                                              const uint32_t *__restrict__ idx, uint64_t n,
                                                              int depth, uint32_t *__restrict__ out) {
    extern __shared__ __align__(16) uint32_t lt[];
    if constexpr (LDS) {
        stage_to_lds(lt, tab, ((uint64_t)mask + 1) * 4);
        __syncthreads();
    }
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; base < n; base += stride * kQ) {
        uint32_t i[kQ];
#pragma unroll
        for (int u = 0; u < kQ; ++u) {
            const uint64_t j = base + u * stride;
            i[u] = j < n ? idx[j] & mask : 0u;
        }
        for (int h = 0; h < depth; ++h) {
#pragma unroll
            for (int u = 0; u < kQ; ++u) i[u] = (LDS ? lt[i[u]] : tab[i[u]]) & mask;
        }
#pragma unroll
        for (int u = 0; u < kQ; ++u) {
            const uint64_t j = base + u * stride;
            if (j < n) out[j] = i[u];
        }
    }
}

}  // namespace

extern "C" {

mbr_status mbr_probe_gather(const uint32_t *d_table, uint64_t entries, const uint32_t *d_idx, uint64_t n,
                            int32_t depth, int32_t lds, uint32_t *d_out, void *stream) {
    using namespace mbr;
    if (entries == 0 || (entries & (entries - 1)) != 0 || entries > (1ull << 32))
        MBR_FAIL(MBR_EINVAL, "entries=%llu must be a power of two up to 2^32", (unsigned long long)entries);
    if (depth < 1 || depth > 64) MBR_FAIL(MBR_EINVAL, "depth=%d outside 1..64", depth);
    if (lds && entries > kLdsEntries) MBR_FAIL(MBR_EINVAL, "an LDS table holds at most %llu entries",
                                               (unsigned long long)kLdsEntries);
    if (n == 0) return MBR_OK;
    if (!d_table || !d_idx || !d_out) MBR_FAIL(MBR_EINVAL, "null pointer");
    hipStream_t s = as_stream(stream);
    const uint32_t mask = (uint32_t)(entries - 1);
    const unsigned grid = grid_for(n, kBlock * kQ, device_cu_count() * 8);
    if (lds) {
        const size_t bytes = entries * 4;
        probe_gather_kernel<true><<<grid, kBlock, bytes, s>>>(d_table, mask, d_idx, n, depth, d_out);
    } else {
        probe_gather_kernel<false><<<grid, kBlock, 0, s>>>(d_table, mask, d_idx, n, depth, d_out);
    }
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

}  // extern "C"
