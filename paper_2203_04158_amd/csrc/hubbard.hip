// On-the-fly Hubbard H·x in gather form (Eq. Talpha2 applied from the bra side,
// Eq. mvblock per (N_up, N_dn) sector, index of Eq. rankupdown).
//
// Row i of sector (n_up, n_dn) is i = r_up * C(L, n_dn) + r_dn.  Every row is
// produced by exactly one lane, so there are no atomics:
//   y_i = [sum_s eps n + sum_i U_i n_up n_dn](alpha) x_i
//       + sum over bonds b whose two sites differ in alpha_sigma
//           (-t_b) (-1)^popcount(alpha_sigma AND between_b) x[rank(alpha XOR mask_b)].
// A hop changes one spin half only, so only that half is re-ranked (staggered
// lookup on L-bit halves, table in LDS) and the other rank is kept.
//
// Workgroup = tile of nblk consecutive alpha_up blocks of one sector.
//  * up-hops: alpha_up is uniform across the block, so each target rank and
//    sign is computed once per block (first threads, into LDS); the lanes then
//    gather x[r_up' * C_dn + r_dn], contiguous across lanes.
//  * down-hops: the target rank depends on alpha_dn only, so a lane ranks each
//    down-hop once and applies it to all nblk blocks of the tile, whose x rows
//    are staged in LDS.
// Tiles run in decreasing cost order over a persistent grid.
#include <algorithm>
#include <memory>
#include <numeric>

#include "hubbard.hpp"

using namespace mbr;

struct mbr_hubbard {
    int32_t L = 0, nb = 0, precision = MBR_F64, k = 0, nch = 0;
    std::vector<mbr_bond> bonds;
    std::vector<double> eps, U;
    std::vector<mbr_spin_sector> secs;
    std::vector<HvSector> hsec;
    uint64_t total = 0;
    std::vector<HvTile> tiles;          // launch order (decreasing cost)
    std::vector<HvTile> tiles_by_slot;  // sector-contiguous
    uint32_t n_slots = 0;
    StagTable tab;
    DevBuf d_hs_states, d_hs_energy, d_tiles, d_secs;
    std::vector<uint32_t> hs_off;
    uint32_t xcap = 0, upcap = 0, maxblk = 0;
    size_t lds_bytes = 0;
    int grid = 0;
    int device = 0;
};

namespace mbr {
int hubbard_precision(const mbr_hubbard *h) { return h->precision; }
int hubbard_n_sectors(const mbr_hubbard *h) { return (int)h->secs.size(); }
uint64_t hubbard_total(const mbr_hubbard *h) { return h->total; }
const std::vector<HvSector> &hubbard_sectors(const mbr_hubbard *h) { return h->hsec; }
uint32_t hubbard_n_slots(const mbr_hubbard *h) { return h->n_slots; }
const std::vector<HvTile> &hubbard_tiles(const mbr_hubbard *h) { return h->tiles_by_slot; }
}  // namespace mbr

namespace {

constexpr unsigned kBlock = 512;
constexpr int kG = 2;            // alpha_up blocks per wide tile held in registers
constexpr int kUpPre = 8;        // up-hop gathers issued ahead of the down-hop work
constexpr uint32_t kUpCap = 1024; // up-hop list entries per tile
constexpr uint32_t kMaxBlk = 256; // alpha_up blocks per narrow tile
constexpr uint32_t kWideMin = 128; // C_dn from which lanes run over alpha_dn
constexpr size_t kXBudget = 56 * 1024; // LDS bytes for staged x rows

struct HvArgs {
    const void *x;
    void *out;
    const HvTile *tiles;
    uint32_t n_tiles;
    const HvSector *secs;
    const uint16_t *hs_states;
    const double *hs_energy;
    const uint16_t *rtab;
    uint32_t rtab_entries;
    int32_t nb, k, nch;
    int32_t rowoff[kMaxSites];
    uint32_t bmask[kMaxBonds];
    uint32_t bbetw[kMaxBonds];
    uint32_t bij[kMaxBonds];  // i | j << 8
    double bamp[kMaxBonds];
    double U[kMaxSites];
    uint32_t Umask;
    int32_t U_uniform;
    double U0;
    uint32_t xcap;     // LDS elements for staged x rows
    uint32_t upcap;    // LDS up-hop list entries (max nblk * nb over tiles)
    uint32_t maxblk;   // LDS per-block entries (max nblk over tiles)
    HvEpilogue ep;
};

// Rank of an L-bit half pattern within its own particle-number block, by the
// staggered lookup (Fig. fastrank) on the LDS table.
template <int NCH>
__device__ __forceinline__ uint32_t rank_half(uint32_t beta, const uint16_t *rt, const HvArgs &a) {
    if constexpr (NCH == 1) {
        return rt[beta];
    } else if constexpr (NCH == 0) {  // any chunk count, not unrolled
        uint32_t r = 0;
        int np = 0;
        const uint32_t cm = (1u << a.k) - 1;
        for (int c = 0; c < a.nch; ++c) {
            uint32_t ch = (beta >> (c * a.k)) & cm;
            r += rt[((uint32_t)(a.rowoff[c] + np) << a.k) + ch];
            np += __popc(ch);
        }
        return r;
    } else {
        uint32_t r = 0;
        int np = 0;
        const uint32_t cm = (1u << a.k) - 1;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            uint32_t ch = (beta >> (c * a.k)) & cm;
            r += rt[((uint32_t)(a.rowoff[c] + np) << a.k) + ch];
            np += __popc(ch);
        }
        return r;
    }
}

template <class T>
__device__ __forceinline__ T u_energy(uint32_t both, const HvArgs &a) {
    if (a.U_uniform) return (T)(a.U0 * (double)__popc(both));
    T e = 0;
    uint32_t m = both & a.Umask;
    while (m) {
        int i = __ffs(m) - 1;
        m &= m - 1;
        e += (T)a.U[i];
    }
    return e;
}

__device__ __forceinline__ double block_sum(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
        for (int j = 0; j < (int)(blockDim.x >> 6); ++j) s += red[j];
    return s;
}

template <class T>
struct UpLists {
    const uint32_t *tgt;
    const T *coef;
    const uint32_t *alpha;
    const uint32_t *cnt;
    const T *e;
};

// Rows of a wide tile: lanes over alpha_dn, the tile's alpha_up blocks in
// registers.  xsrc holds the tile's own x rows (the LDS copy or x itself);
// each call site passes a pointer of a single address space.
template <class T, int NCH, bool LZ>
__device__ __forceinline__ double wide_rows(const HvArgs &a, const uint16_t *rt, const T *xsrc,
                                            const T *x, T *out, const T *p, const HvTile &tl,
                                            const HvSector &sc, uint64_t base, const UpLists<T> &ul) {
    const uint32_t cdn = sc.cdn;
    const int nb = a.nb;
    const int nblk = (int)tl.nblk;
    double dot = 0.0;
    for (uint32_t rd = threadIdx.x; rd < cdn; rd += blockDim.x) {
        // 1. issue the global loads first: the first kUpPre up-hop gathers of
        //    every block (contiguous across lanes) and the epilogue operand
        T upv[kG][kUpPre];
        T upc[kG][kUpPre];
        T pv[kG];
#pragma unroll
        for (int g = 0; g < kG; ++g) {
            const uint32_t n = g < nblk ? ul.cnt[g] : 0u;
#pragma unroll
            for (int u = 0; u < kUpPre; ++u) {
                upv[g][u] = 0;
                upc[g][u] = 0;
                if (u < (int)n) {
                    upc[g][u] = ul.coef[g * nb + u];
                    upv[g][u] = x[sc.off + (uint64_t)ul.tgt[g * nb + u] * cdn + rd];
                }
            }
            pv[g] = 0;
            if constexpr (LZ) {
                if (a.ep.c2 && g < nblk) pv[g] = p[base + (uint64_t)g * cdn + rd];
            }
        }
        const uint32_t ad = a.hs_states[sc.hs_dn + rd];
        const T ed = (T)a.hs_energy[sc.hs_dn + rd];
        // 2. down-hops while those loads are in flight: rank each target once
        //    and apply it to every alpha_up block of the tile.  Branch-free:
        //    bonds that do not hop get coefficient 0 and the row's own index.
        T acc[kG];
#pragma unroll
        for (int g = 0; g < kG; ++g) acc[g] = 0;
#pragma unroll 2
        for (int b = 0; b < nb; ++b) {
            const uint32_t bi = a.bij[b] & 0xFF, bj = a.bij[b] >> 8;
            const bool hop = ((ad >> bi) ^ (ad >> bj)) & 1;
            uint32_t rr = rank_half<NCH>(ad ^ a.bmask[b], rt, a);
            rr = hop ? rr : rd;
            T c = (__popc(ad & a.bbetw[b]) & 1) ? (T)a.bamp[b] : -(T)a.bamp[b];
            c = hop ? c : (T)0;
#pragma unroll
            for (int g = 0; g < kG; ++g)
                if (g < nblk) acc[g] += c * xsrc[g * cdn + rr];
        }
        // 3. diagonal, up-hops, epilogue
#pragma unroll
        for (int g = 0; g < kG; ++g) {
            if (g >= nblk) break;
            const uint32_t au = ul.alpha[g];
            const T xv = xsrc[g * cdn + rd];
            T v = acc[g] + (ul.e[g] + ed + u_energy<T>(au & ad, a)) * xv;
#pragma unroll
            for (int u = 0; u < kUpPre; ++u) v += upc[g][u] * upv[g][u];
            const uint32_t n = ul.cnt[g];
            for (uint32_t h = kUpPre; h < n; ++h)
                v += ul.coef[g * nb + h] * x[sc.off + (uint64_t)ul.tgt[g * nb + h] * cdn + rd];
            const uint64_t row = base + (uint64_t)g * cdn + rd;
            if constexpr (LZ) {
                T u = (T)a.ep.c1[tl.sector] * v;
                if (a.ep.c2) u -= (T)a.ep.c2[tl.sector] * pv[g];
                out[row] = u;
                dot += (double)xv * (double)u;
            } else {
                out[row] = v;
            }
        }
    }
    return dot;
}

// LZ: fused Lanczos epilogue (u = c1 H x - c2 p with <x, u> partials);
// otherwise the plain product.
template <class T, int NCH, bool LZ>
__global__ void __launch_bounds__(kBlock) hv_kernel(HvArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    // LDS carve-up: rank table | up-hop targets | up-hop coefficients |
    // per-block alpha_up, energy, hop count | reduction scratch | x rows
    uint16_t *rt = reinterpret_cast<uint16_t *>(smem);
    size_t o = ((size_t)a.rtab_entries * 2 + 15) & ~(size_t)15;
    uint32_t *up_tgt = reinterpret_cast<uint32_t *>(smem + o);
    o += ((size_t)a.upcap * 4 + 15) & ~(size_t)15;
    T *up_coef = reinterpret_cast<T *>(smem + o);
    o += ((size_t)a.upcap * sizeof(T) + 15) & ~(size_t)15;
    uint32_t *up_alpha = reinterpret_cast<uint32_t *>(smem + o);
    o += ((size_t)a.maxblk * 4 + 15) & ~(size_t)15;
    uint32_t *up_cnt = reinterpret_cast<uint32_t *>(smem + o);
    o += ((size_t)a.maxblk * 4 + 15) & ~(size_t)15;
    T *up_e = reinterpret_cast<T *>(smem + o);
    o += ((size_t)a.maxblk * sizeof(T) + 15) & ~(size_t)15;
    double *red = reinterpret_cast<double *>(smem + o);
    o += 16 * sizeof(double);
    T *xs = reinterpret_cast<T *>(smem + o);

    for (uint32_t i = threadIdx.x; i < a.rtab_entries; i += blockDim.x) rt[i] = a.rtab[i];

    const T *x = static_cast<const T *>(a.x);
    T *out = static_cast<T *>(a.out);
    const T *p = static_cast<const T *>(a.ep.p);
    if (a.ep.basis_j) {
        const int64_t j = *a.ep.basis_j;
        x += (uint64_t)j * a.ep.basis_stride;
        p = j > 0 ? x - a.ep.basis_stride : x;
    }
    const int nb = a.nb;

    for (uint32_t ti = blockIdx.x; ti < a.n_tiles; ti += gridDim.x) {
        const HvTile tl = a.tiles[ti];
        const HvSector sc = a.secs[tl.sector];
        __syncthreads();  // LDS from the previous tile (and the table copy) settled
        if (a.ep.active && !a.ep.active[tl.sector]) {
            if (a.ep.partial && threadIdx.x == 0) a.ep.partial[tl.slot] = 0.0;
            continue;
        }
        const uint32_t cdn = sc.cdn;
        const uint32_t rows = tl.nblk * cdn;
        const uint64_t base = sc.off + (uint64_t)tl.rup0 * cdn;
        if (sc.x_lds) {
            // coalesced copy, four independent loads in flight per lane
            const uint32_t step = blockDim.x * 4;
            uint32_t e = threadIdx.x;
            for (; e + 3 * blockDim.x < rows; e += step) {
                T v0 = x[base + e], v1 = x[base + e + blockDim.x];
                T v2 = x[base + e + 2 * blockDim.x], v3 = x[base + e + 3 * blockDim.x];
                xs[e] = v0;
                xs[e + blockDim.x] = v1;
                xs[e + 2 * blockDim.x] = v2;
                xs[e + 3 * blockDim.x] = v3;
            }
            for (; e < rows; e += blockDim.x) xs[e] = x[base + e];
        }
        // up-hop lists, one thread per alpha_up block, bonds in order
        if (threadIdx.x < tl.nblk) {
            const uint32_t g = threadIdx.x;
            const uint32_t hi = sc.hs_up + tl.rup0 + g;
            const uint32_t au = a.hs_states[hi];
            up_alpha[g] = au;
            up_e[g] = (T)a.hs_energy[hi];
            uint32_t cnt = 0;
            for (int b = 0; b < nb; ++b) {
                const uint32_t bi = a.bij[b] & 0xFF, bj = a.bij[b] >> 8;
                if (((au >> bi) ^ (au >> bj)) & 1) {
                    up_tgt[g * nb + cnt] = rank_half<NCH>(au ^ a.bmask[b], rt, a);
                    up_coef[g * nb + cnt] = (__popc(au & a.bbetw[b]) & 1) ? (T)a.bamp[b] : -(T)a.bamp[b];
                    ++cnt;
                }
            }
            up_cnt[g] = cnt;
        }
        __syncthreads();

        double dot = 0.0;
        if (sc.wide) {
            const UpLists<T> ul{up_tgt, up_coef, up_alpha, up_cnt, up_e};
            if (sc.x_lds)
                dot = wide_rows<T, NCH, LZ>(a, rt, xs, x, out, p, tl, sc, base, ul);
            else
                dot = wide_rows<T, NCH, LZ>(a, rt, x + base, x, out, p, tl, sc, base, ul);
        } else {
            for (uint32_t e = threadIdx.x; e < rows; e += blockDim.x) {
                const uint32_t g = e / cdn;
                const uint32_t rd = e - g * cdn;
                const uint32_t ad = a.hs_states[sc.hs_dn + rd];
                const T ed = (T)a.hs_energy[sc.hs_dn + rd];
                const uint32_t au = up_alpha[g];
                const T xv = xs[e];
                T v = (up_e[g] + ed + u_energy<T>(au & ad, a)) * xv;
                for (int b = 0; b < nb; ++b) {
                    const uint32_t bi = a.bij[b] & 0xFF, bj = a.bij[b] >> 8;
                    if (((ad >> bi) ^ (ad >> bj)) & 1) {
                        const uint32_t rr = rank_half<NCH>(ad ^ a.bmask[b], rt, a);
                        const T c = (__popc(ad & a.bbetw[b]) & 1) ? (T)a.bamp[b] : -(T)a.bamp[b];
                        v += c * xs[g * cdn + rr];
                    }
                }
                const uint32_t n = up_cnt[g];
                for (uint32_t h = 0; h < n; ++h)
                    v += up_coef[g * nb + h] * x[sc.off + (uint64_t)up_tgt[g * nb + h] * cdn + rd];
                const uint64_t row = base + e;
                if constexpr (LZ) {
                    T u = (T)a.ep.c1[tl.sector] * v;
                    if (a.ep.c2) u -= (T)a.ep.c2[tl.sector] * p[row];
                    out[row] = u;
                    dot += (double)xv * (double)u;
                } else {
                    out[row] = v;
                }
            }
        }
        if (a.ep.partial) {
            double s = block_sum(dot, red);
            if (threadIdx.x == 0) a.ep.partial[tl.slot] = s;
        }
    }
}

size_t lds_bytes_for(const mbr_hubbard *h, size_t tsz) {
    auto r16 = [](size_t v) { return (v + 15) & ~(size_t)15; };
    size_t o = r16(((size_t)h->tab.nrows << h->tab.k) * 2);
    o += r16((size_t)h->upcap * 4) + r16((size_t)h->upcap * tsz);
    o += 2 * r16((size_t)h->maxblk * 4) + r16((size_t)h->maxblk * tsz) + 16 * sizeof(double);
    return o + (size_t)h->xcap * tsz;
}

template <class T, int NCH>
mbr_status launch_t(const mbr_hubbard *h, const void *x, void *out, const HvEpilogue &ep,
                    hipStream_t s) {
    HvArgs a{};
    a.x = x;
    a.out = out;
    a.tiles = ep.tiles ? ep.tiles : h->d_tiles.as<HvTile>();
    a.n_tiles = ep.tiles ? ep.n_tiles : (uint32_t)h->tiles.size();
    a.secs = h->d_secs.as<HvSector>();
    a.hs_states = h->d_hs_states.as<uint16_t>();
    a.hs_energy = h->d_hs_energy.as<double>();
    a.rtab = h->tab.table.as<uint16_t>();
    a.rtab_entries = (uint32_t)((uint64_t)h->tab.nrows << h->tab.k);
    a.nb = h->nb;
    a.k = h->tab.k;
    a.nch = h->tab.nch;
    for (int c = 0; c < kMaxSites; ++c) a.rowoff[c] = c < h->tab.nch ? h->tab.rowoff[c] : 0;
    for (int b = 0; b < h->nb; ++b) {
        const mbr_bond &bd = h->bonds[b];
        int lo = bd.i < bd.j ? bd.i : bd.j, hi = bd.i < bd.j ? bd.j : bd.i;
        a.bmask[b] = (1u << bd.i) | (1u << bd.j);
        a.bbetw[b] = ((1u << hi) - 1) & ~((1u << (lo + 1)) - 1);
        a.bij[b] = (uint32_t)bd.i | ((uint32_t)bd.j << 8);
        a.bamp[b] = bd.t;
    }
    a.U_uniform = 1;
    a.U0 = h->U.empty() ? 0.0 : h->U[0];
    a.Umask = 0;
    for (int i = 0; i < h->L; ++i) {
        double u = h->U.empty() ? 0.0 : h->U[i];
        a.U[i] = u;
        if (u != 0.0) a.Umask |= 1u << i;
        if (u != a.U0) a.U_uniform = 0;
    }
    a.xcap = h->xcap;
    a.upcap = h->upcap;
    a.maxblk = h->maxblk;
    a.ep = ep;
    auto kern = ep.c1 ? hv_kernel<T, NCH, true> : hv_kernel<T, NCH, false>;
    size_t lds = lds_bytes_for(h, sizeof(T));
    if (lds > 64 * 1024)
        MBR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    unsigned grid = (unsigned)std::min<uint64_t>(a.n_tiles, (uint64_t)h->grid);
    if (grid == 0) return MBR_OK;
    kern<<<grid, kBlock, lds, s>>>(a);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

template <class T>
mbr_status launch_p(const mbr_hubbard *h, const void *x, void *out, const HvEpilogue &ep,
                    hipStream_t s) {
    switch (h->tab.nch) {
        case 1: return launch_t<T, 1>(h, x, out, ep, s);
        case 2: return launch_t<T, 2>(h, x, out, ep, s);
        case 3: return launch_t<T, 3>(h, x, out, ep, s);
        case 4: return launch_t<T, 4>(h, x, out, ep, s);
        default: return launch_t<T, 0>(h, x, out, ep, s);
    }
}

}  // namespace

namespace mbr {
mbr_status hubbard_launch(const mbr_hubbard *h, const void *x, void *out, const HvEpilogue &ep,
                          hipStream_t s) {
    if (h->precision == MBR_F64) return launch_p<double>(h, x, out, ep, s);
    return launch_p<float>(h, x, out, ep, s);
}
}  // namespace mbr

extern "C" {

mbr_status mbr_hubbard_create(const mbr_hubbard_desc *d, mbr_hubbard **out, void *stream) {
    if (!out) MBR_FAIL(MBR_EINVAL, "null output handle");
    *out = nullptr;
    if (!d) MBR_FAIL(MBR_EINVAL, "null descriptor");
    const int L = d->L;
    if (L < 1 || L > kMaxSites) MBR_FAIL(MBR_EINVAL, "L=%d outside 1..%d", L, kMaxSites);
    if (d->n_bonds < 0 || d->n_bonds > kMaxBonds) MBR_FAIL(MBR_EINVAL, "n_bonds=%d outside 0..%d", d->n_bonds, kMaxBonds);
    if (d->n_bonds > 0 && !d->bonds) MBR_FAIL(MBR_EINVAL, "null bond list");
    if (d->n_sectors < 1 || d->n_sectors > 1024 || !d->sectors) MBR_FAIL(MBR_EINVAL, "n_sectors=%d", d->n_sectors);
    if (d->precision != MBR_F64 && d->precision != MBR_F32) MBR_FAIL(MBR_EINVAL, "precision=%d", d->precision);
    if (d->k < 0 || d->k > 16) MBR_FAIL(MBR_EINVAL, "k=%d outside 0..16", d->k);
    for (int b = 0; b < d->n_bonds; ++b) {
        const mbr_bond &bd = d->bonds[b];
        if (bd.i < 0 || bd.i >= L || bd.j < 0 || bd.j >= L || bd.i == bd.j)
            MBR_FAIL(MBR_EINVAL, "bond %d = (%d,%d)", b, bd.i, bd.j);
    }
    auto *h = new (std::nothrow) mbr_hubbard;
    if (!h) MBR_FAIL(MBR_ENOMEM, "host allocation");
    std::unique_ptr<mbr_hubbard> guard(h);
    (void)hipGetDevice(&h->device);
    hipStream_t s = as_stream(stream);
    h->L = L;
    h->nb = d->n_bonds;
    h->precision = d->precision;
    h->bonds.assign(d->bonds, d->bonds + d->n_bonds);
    if (d->eps) h->eps.assign(d->eps, d->eps + L);
    if (d->U) h->U.assign(d->U, d->U + L);
    h->secs.assign(d->sectors, d->sectors + d->n_sectors);
    for (auto &sc : h->secs)
        if (sc.n_up < 0 || sc.n_up > L || sc.n_dn < 0 || sc.n_dn > L)
            MBR_FAIL(MBR_EINVAL, "sector (%d,%d)", sc.n_up, sc.n_dn);
    // half-pattern chunk width: two lookups into a small table by default
    int k = d->k;
    if (k == 0) k = (L + 1) / 2;
    h->k = k;
    MBR_TRY(stag_build(h->tab, L, k, L, 2, s));
    if (h->tab.entry_bytes != 2) MBR_FAIL(MBR_EUNSUPPORTED, "half ranks beyond 16 bits");
    if ((((size_t)h->tab.nrows << k) * 2) > 64 * 1024) MBR_FAIL(MBR_EUNSUPPORTED, "half table over 64 KiB; use a smaller k");
    // half-state lists by particle number, ascending, and their one-body energies
    h->hs_off.assign(L + 2, 0);
    std::vector<uint16_t> hs;
    std::vector<double> he;
    for (int n = 0; n <= L; ++n) {
        h->hs_off[n] = (uint32_t)hs.size();
        for (uint32_t a = 0; a < (1u << L); ++a)
            if (__builtin_popcount(a) == n) {
                hs.push_back((uint16_t)a);
                double e = 0;
                for (int i = 0; i < L; ++i)
                    if ((a >> i) & 1) e += h->eps.empty() ? 0.0 : h->eps[i];
                he.push_back(e);
            }
    }
    h->hs_off[L + 1] = (uint32_t)hs.size();
    MBR_TRY(upload(h->d_hs_states, hs.data(), hs.size() * 2, s));
    MBR_TRY(upload(h->d_hs_energy, he.data(), he.size() * 8, s));
    // sectors and tiles
    const size_t tsz = h->precision == MBR_F64 ? 8 : 4;
    uint64_t off = 0;
    uint32_t slot = 0;
    h->xcap = 0;
    const uint32_t upblk = h->nb > 0 ? kUpCap / (uint32_t)h->nb : kMaxBlk;
    for (size_t si = 0; si < h->secs.size(); ++si) {
        HvSector sc{};
        sc.off = off;
        sc.cup = (uint32_t)binom(L, h->secs[si].n_up);
        sc.cdn = (uint32_t)binom(L, h->secs[si].n_dn);
        sc.hs_up = h->hs_off[h->secs[si].n_up];
        sc.hs_dn = h->hs_off[h->secs[si].n_dn];
        sc.wide = sc.cdn >= kWideMin;
        uint32_t nblk;
        if (sc.wide) {
            uint32_t fit = (uint32_t)(kXBudget / (sc.cdn * tsz));
            sc.x_lds = fit >= 1;
            nblk = sc.x_lds ? std::min<uint32_t>(kG, fit) : 1;
        } else {
            sc.x_lds = 1;
            nblk = std::max<uint32_t>(1, 1024 / sc.cdn);
        }
        nblk = std::min({nblk, upblk, kMaxBlk});
        if (nblk < 1) nblk = 1;
        sc.slot0 = slot;
        for (uint32_t r = 0; r < sc.cup; r += nblk) {
            HvTile t{};
            t.sector = (uint32_t)si;
            t.rup0 = r;
            t.nblk = std::min(nblk, sc.cup - r);
            t.slot = slot++;
            if (sc.x_lds) h->xcap = std::max(h->xcap, t.nblk * sc.cdn);
            h->maxblk = std::max(h->maxblk, t.nblk);
            h->upcap = std::max(h->upcap, t.nblk * (uint32_t)std::max(1, h->nb));
            h->tiles.push_back(t);
        }
        sc.nslots = slot - sc.slot0;
        h->hsec.push_back(sc);
        off += (uint64_t)sc.cup * sc.cdn;
    }
    h->total = off;
    h->n_slots = slot;
    h->tiles_by_slot = h->tiles;
    // decreasing cost, sector order kept among equals (deterministic)
    std::stable_sort(h->tiles.begin(), h->tiles.end(), [&](const HvTile &p, const HvTile &q) {
        return (uint64_t)p.nblk * h->hsec[p.sector].cdn > (uint64_t)q.nblk * h->hsec[q.sector].cdn;
    });
    MBR_TRY(upload(h->d_tiles, h->tiles.data(), h->tiles.size() * sizeof(HvTile), s));
    MBR_TRY(upload(h->d_secs, h->hsec.data(), h->hsec.size() * sizeof(HvSector), s));
    h->lds_bytes = lds_bytes_for(h, tsz);
    if (h->lds_bytes > 160 * 1024) MBR_FAIL(MBR_EUNSUPPORTED, "tile needs %zu bytes of LDS", h->lds_bytes);
    int per_cu = (int)std::min<size_t>(8, (160 * 1024) / h->lds_bytes);
    if (per_cu < 1) per_cu = 1;
    h->grid = (int)std::min<size_t>(h->tiles.size(), (size_t)device_cu_count() * per_cu);
    *out = guard.release();
    return MBR_OK;
}

mbr_status mbr_hubbard_dim(const mbr_hubbard *h, uint64_t *total, uint64_t *offsets) {
    if (!h) MBR_FAIL(MBR_EINVAL, "null handle");
    if (total) *total = h->total;
    if (offsets) {
        for (size_t i = 0; i < h->hsec.size(); ++i) offsets[i] = h->hsec[i].off;
        offsets[h->hsec.size()] = h->total;
    }
    return MBR_OK;
}

mbr_status mbr_hubbard_apply(const mbr_hubbard *h, const void *d_x, void *d_y, void *stream) {
    if (!h) MBR_FAIL(MBR_EINVAL, "null handle");
    if (!d_x || !d_y) MBR_FAIL(MBR_EINVAL, "null vector");
    if (d_x == d_y) MBR_FAIL(MBR_EINVAL, "x and y must not alias");
    HvEpilogue ep{};
    return hubbard_launch(h, d_x, d_y, ep, as_stream(stream));
}

mbr_status mbr_hubbard_destroy(mbr_hubbard *h) {
    delete h;
    return MBR_OK;
}

}  // extern "C"
