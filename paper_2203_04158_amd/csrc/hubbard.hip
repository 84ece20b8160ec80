// On-the-fly Hubbard H·x in gather form (Eq. Talpha2 applied from the bra side,
// Eq. mvblock per (N_up, N_dn) sector, index of Eq. rankupdown).
//
// Row i of sector (n_up, n_dn) is i = r_up * C(L, n_dn) + r_dn.  Every row is
// produced by exactly one lane, so there are no atomics:
//   y_i = [sum eps n + sum_i U_i n_up n_dn](alpha) x_i
//       + sum over bonds b whose two sites differ in alpha_sigma
//           (-t_b) (-1)^popcount(alpha_sigma AND between_b) x[rank(alpha XOR mask_b)].
// A hop changes one spin half only, so only that half is re-ranked (staggered
// lookup on L-bit halves, table in LDS) and the other rank is kept.
//
// Workgroup = tile of nblk <= G consecutive alpha_up blocks of one sector.
//  * up-hops: alpha_up is uniform across a block, so each target rank and
//    sign is computed once per block (into LDS); the lanes then gather
//    x[r_up' * C_dn + r_dn], contiguous across lanes.  These loads are issued
//    before the LDS work so that their latency overlaps it.
//  * down-hops: the target rank depends on alpha_dn only, so a lane ranks each
//    down-hop once and applies it to all nblk blocks of the tile, whose x rows
//    are staged in LDS.
// Scheduling: tiles are split into eight contiguous, cost-balanced ranges in
// the natural (combinadics) order, one per XCD (workgroup w runs on XCD w mod
// 8), so the up-hop sources of neighbouring alpha_up blocks, which are mostly
// close in that order, are reused from the same L2.
#include <algorithm>
#include <cstdlib>
#include <fstream>
#include <memory>
#include <numeric>
#include <sstream>

#include "hubbard.hpp"
#include "rank_device.hpp"

using namespace mbr;

namespace {
constexpr int kXcd = 8;
}

// Trie of one sector for the trie-ranked product: levels of a packed trie
// over the sector's full 2L-bit patterns (level-major layout of trie.hip).
struct HvTrieDesc {
    const uint32_t *tab;     // all levels
    const uint32_t *states;  // the sector's ascending list
    uint32_t H, lds_levels, lds_entries, pad;
    uint32_t wmask[8];
    int32_t shift[8];
    uint64_t off[9];
};

struct mbr_hubbard {
    int32_t L = 0, nb = 0, precision = MBR_F64;
    int32_t rank_kind = MBR_HV_RANK_HALVES;
    std::vector<mbr_sector *> tsecs;    // trie-ranked product: each sector's list and trie
    std::vector<mbr_ranker *> ttries;
    DevBuf d_trie;                      // HvTrieDesc per sector
    uint32_t trie_lds = 0;              // LDS entries the largest staged top levels need
    int32_t trie_k = 0;                 // chunk width of the tries
    ~mbr_hubbard() {
        for (auto *r : ttries) mbr_ranker_destroy(r);
        for (auto *s : tsecs) mbr_sector_destroy(s);
    }
    std::vector<mbr_bond> bonds;
    std::vector<double> eps, U;
    std::vector<mbr_spin_sector> secs;
    // launch shape
    int32_t k = 0, G = 2, block = 512;
    double tuned_ms = 0.0;
    uint32_t generation = 0;
    // derived
    std::vector<HvSector> hsec;
    uint64_t total = 0;
    std::vector<HvTile> tiles_by_slot;  // natural order = slot order
    std::vector<HvTile> tiles_binned;   // tile-kernel tiles, XCD ranges, natural order inside
    uint32_t xoff[kXcd + 1] = {0};
    std::vector<HvTile> rows_tiles;     // alpha_dn-stationary kernel tiles, natural order
    std::vector<HvTile> flat_tiles;     // flat kernel tiles, natural order
    DevBuf d_flat_tiles;
    uint32_t flat_xoff[kXcd + 1] = {0};
    DevBuf d_rdesc, d_rdesc_slot;       // their descriptors, and descriptors in slot order
    uint32_t rows_xoff[kXcd + 1] = {0};
    uint32_t rows_xcap = 0, rows_gmax = 1;
    int rows_R = 1, rows_grid = 0;
    bool t_uniform = true;              // all bonds share one amplitude
    DevBuf d_lists;                     // rows and block kernels: down-hop lists per n_dn
    std::vector<uint32_t> lists_ndn;    // n_dn of each list set, in storage order
    std::vector<uint8_t> lists_blk;     // the set serves block-kernel sectors (their negated-copy offset)
    std::vector<HvTile> block_tiles;    // block kernel (G = -2) tiles, one alpha_up block each, natural order
    DevBuf d_bdesc;                     // their descriptors
    uint32_t block_xoff[kXcd + 1] = {0};
    uint32_t block_xcap = 0;            // largest C_dn + 1 of the block kernel's sectors
    DevBuf d_up_tgt, d_up_coef, d_up_n; // block kernel: up-hop lists of every half state
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
uint32_t hubbard_generation(const mbr_hubbard *h) { return h->generation; }
}  // namespace mbr

namespace {

constexpr int kUpPre = 8;          // up-hop gathers issued ahead of the down-hop work
constexpr uint32_t kWideMin = 128; // C_dn from which lanes run over alpha_dn
constexpr size_t kLdsMax = 160 * 1024;

// Work descriptor of one tile of the alpha_dn-stationary kernel (host-built,
// 32 bytes): first row of the tile and of its sector; C_dn | gp << 12 |
// nblk << 20; half-state index of the first alpha_up | that of the alpha_dn
// list << 16; down-hop list row | sector << 16; partial-sum slot.
struct RowsTileDesc {
    uint64_t base, soff;
    uint32_t w0, w1, w2, slot;
};

struct HvArgs {
    const void *x;
    void *out;
    const HvTile *tiles;
    uint32_t n_tiles;
    uint32_t binned;             // tiles grouped in kXcd ranges xoff[]
    uint32_t xoff[kXcd + 1];
    const HvSector *secs;
    const uint16_t *hs_states;
    const double *hs_energy;
    const uint16_t *rtab;
    uint32_t rtab_entries;
    int32_t nb, k, nch;
    int32_t Lsites;
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
    uint32_t rgmax;    // alpha_dn-stationary kernel: max alpha_up blocks per tile
    int32_t t_uniform; // every bond has the amplitude bamp[0]
    const void *lists;     // alpha_dn-stationary kernel: down-hop lists (hv_lists_kernel)
    const RowsTileDesc *rdesc;  // and its tiles (n_tiles of them)
    HvEpilogue ep;
};

// Rank of an L-bit half pattern within its own particle-number block, by the
// staggered lookup (Fig. fastrank) on the LDS table.  NCH = 0: any chunk count.
template <int NCH>
__device__ __forceinline__ uint32_t rank_half(uint32_t beta, const uint16_t *rt, const HvArgs &a) {
    if constexpr (NCH == 1) {
        return rt[beta];
    } else {
        uint32_t r = 0;
        int np = 0;
        const uint32_t cm = (1u << a.k) - 1;
        const int n = NCH == 0 ? a.nch : NCH;
#pragma unroll
        for (int c = 0; c < n; ++c) {
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

template <class T>
__device__ __forceinline__ T fma_t(T a, T b, T c) {
    if constexpr (sizeof(T) == 8) return __builtin_fma(a, b, c);
    else return __builtin_fmaf(a, b, c);
}

// Fused Lanczos epilogue of one row: c1 (H x)_i - c2 p_i.
template <class T>
__device__ __forceinline__ T lz_out(T hx, T c1, T c2, T pv, bool has_p) {
    const T u = c1 * hx;
    return has_p ? fma_t(-c2, pv, u) : u;
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
template <class T, int NCH, bool LZ, int G>
__device__ __forceinline__ double wide_rows(const HvArgs &a, const uint16_t *rt, const T *xsrc,
                                            const T *x, T *out, const T *p, const HvTile &tl,
                                            const HvSector &sc, uint64_t base, const UpLists<T> &ul) {
    const uint32_t cdn = sc.cdn;
    const int nb = a.nb;
    const int nblk = (int)tl.nblk;
    double dot = 0.0;
    for (uint32_t rd = threadIdx.x; rd < cdn; rd += blockDim.x) {
        // 1. global loads first: the first kUpPre up-hop gathers of every
        //    block (contiguous across lanes) and the epilogue operand
        T upv[G][kUpPre];
        T upc[G][kUpPre];
        T pv[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
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
        T acc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] = 0;
#pragma unroll 2
        for (int b = 0; b < nb; ++b) {
            const uint32_t bi = a.bij[b] & 0xFF, bj = a.bij[b] >> 8;
            const bool hop = ((ad >> bi) ^ (ad >> bj)) & 1;
            uint32_t rr = rank_half<NCH>(ad ^ a.bmask[b], rt, a);
            rr = hop ? rr : rd;
            // uniform amplitude: sum the signed x and scale once, as the rows kernel does
            const T mag = a.t_uniform ? (T)1 : (T)a.bamp[b];
            T c = (__popc(ad & a.bbetw[b]) & 1) ? mag : -mag;
            c = hop ? c : (T)0;
#pragma unroll
            for (int g = 0; g < G; ++g)
                if (g < nblk) acc[g] = fma_t(c, xsrc[g * cdn + rr], acc[g]);
        }
        // 3. diagonal, up-hops, epilogue
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (g >= nblk) break;
            const uint32_t au = ul.alpha[g];
            const T xv = xsrc[g * cdn + rd];
            const T dg = ul.e[g] + ed + u_energy<T>(au & ad, a);
            T v = fma_t(dg, xv, a.t_uniform ? (T)a.bamp[0] * acc[g] : acc[g]);
            const uint32_t n = ul.cnt[g];
#pragma unroll
            for (int u = 0; u < kUpPre; ++u)
                if (u < (int)n) v = fma_t(upc[g][u], upv[g][u], v);
            for (uint32_t h = kUpPre; h < n; ++h)
                v = fma_t(ul.coef[g * nb + h], x[sc.off + (uint64_t)ul.tgt[g * nb + h] * cdn + rd], v);
            const uint64_t row = base + (uint64_t)g * cdn + rd;
            if constexpr (LZ) {
                const T u = lz_out(v, (T)a.ep.c1[tl.sector], a.ep.c2 ? (T)a.ep.c2[tl.sector] : (T)0, pv[g],
                                   a.ep.c2 != nullptr);
                out[row] = u;
                dot = __builtin_fma((double)xv, (double)u, dot);
            } else {
                out[row] = v;
            }
        }
    }
    return dot;
}

// LZ: fused Lanczos epilogue (u = c1 H x - c2 p with <x, u> partials);
// otherwise the plain product.
template <class T, int NCH, bool LZ, int G>
__global__ void __launch_bounds__(512) hv_kernel(HvArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    // LDS carve-up: rank table | up-hop targets | up-hop coefficients |
    // per-block alpha_up, hop count, energy | reduction scratch | x rows
    auto r16 = [](size_t v) { return (v + 15) & ~(size_t)15; };
    uint16_t *rt = reinterpret_cast<uint16_t *>(smem);
    size_t o = r16((size_t)a.rtab_entries * 2);
    uint32_t *up_tgt = reinterpret_cast<uint32_t *>(smem + o);
    o += r16((size_t)a.upcap * 4);
    T *up_coef = reinterpret_cast<T *>(smem + o);
    o += r16((size_t)a.upcap * sizeof(T));
    uint32_t *up_alpha = reinterpret_cast<uint32_t *>(smem + o);
    o += r16((size_t)a.maxblk * 4);
    uint32_t *up_cnt = reinterpret_cast<uint32_t *>(smem + o);
    o += r16((size_t)a.maxblk * 4);
    T *up_e = reinterpret_cast<T *>(smem + o);
    o += r16((size_t)a.maxblk * sizeof(T));
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

    uint32_t t_begin, t_end, t_step;
    if (a.binned) {
        const uint32_t xcd = blockIdx.x % kXcd;
        t_begin = a.xoff[xcd] + blockIdx.x / kXcd;
        t_end = a.xoff[xcd + 1];
        t_step = (gridDim.x - xcd + kXcd - 1) / kXcd;
    } else {
        t_begin = blockIdx.x;
        t_end = a.n_tiles;
        t_step = gridDim.x;
    }
    // A tile's partial of <q_j, u>: each wave leaves its sum in red, and wave 0
    // adds them (a fixed tree) right after the next barrier, so the partial
    // costs no barrier of its own.  red is written again only after the
    // barrier that follows that fold.
    bool pend = false;
    uint32_t pend_slot = 0;
    auto fold = [&]() {
        if (threadIdx.x < 64) {
            double v = threadIdx.x < (blockDim.x >> 6) ? red[threadIdx.x] : 0.0;
            for (int o = 8; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
            if (threadIdx.x == 0) a.ep.partial[pend_slot] = v;
        }
        pend = false;
    };
    for (uint32_t ti = t_begin; ti < t_end; ti += t_step) {
        const HvTile tl = a.tiles[ti];
        const HvSector sc = a.secs[tl.sector];
        __syncthreads();  // LDS from the previous tile (and the table copy) settled
        if (pend) fold();
        if (a.ep.active && !a.ep.active[tl.sector]) {
            if (a.ep.partial && threadIdx.x == 0) a.ep.partial[tl.slot] = 0.0;
            continue;
        }
        const uint32_t cdn = sc.cdn;
        const uint32_t rows = tl.nblk * cdn;
        const uint64_t base = sc.off + (uint64_t)tl.rup0 * cdn;
        if (sc.x_lds) {
            // coalesced copy, four independent loads in flight per lane
            const uint32_t bd = blockDim.x;
            uint32_t e = threadIdx.x;
            for (; e + 3 * bd < rows; e += 4 * bd) {
                T v0 = x[base + e], v1 = x[base + e + bd];
                T v2 = x[base + e + 2 * bd], v3 = x[base + e + 3 * bd];
                xs[e] = v0;
                xs[e + bd] = v1;
                xs[e + 2 * bd] = v2;
                xs[e + 3 * bd] = v3;
            }
            for (; e < rows; e += bd) xs[e] = x[base + e];
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
                dot = wide_rows<T, NCH, LZ, G>(a, rt, xs, x, out, p, tl, sc, base, ul);
            else
                dot = wide_rows<T, NCH, LZ, G>(a, rt, x + base, x, out, p, tl, sc, base, ul);
        } else {
            // narrow tiles (few spin-down configurations): flattened rows
            for (uint32_t e = threadIdx.x; e < rows; e += blockDim.x) {
                const uint32_t g = e / cdn;
                const uint32_t rd = e - g * cdn;
                const uint32_t n = up_cnt[g];
                T upv[kUpPre];
#pragma unroll
                for (int u = 0; u < kUpPre; ++u)
                    upv[u] = (u < (int)n) ? x[sc.off + (uint64_t)up_tgt[g * nb + u] * cdn + rd] : (T)0;
                const uint64_t row = base + e;
                T pv = 0;
                if constexpr (LZ) {
                    if (a.ep.c2) pv = p[row];
                }
                const uint32_t ad = a.hs_states[sc.hs_dn + rd];
                const T ed = (T)a.hs_energy[sc.hs_dn + rd];
                const uint32_t au = up_alpha[g];
                const T xv = xs[e];
                T acc = 0;
                for (int b = 0; b < nb; ++b) {
                    const uint32_t bi = a.bij[b] & 0xFF, bj = a.bij[b] >> 8;
                    if (((ad >> bi) ^ (ad >> bj)) & 1) {
                        const uint32_t rr = rank_half<NCH>(ad ^ a.bmask[b], rt, a);
                        const T mag = a.t_uniform ? (T)1 : (T)a.bamp[b];
                        const T c = (__popc(ad & a.bbetw[b]) & 1) ? mag : -mag;
                        acc = fma_t(c, xs[g * cdn + rr], acc);
                    }
                }
                const T dg = up_e[g] + ed + u_energy<T>(au & ad, a);
                T v = fma_t(dg, xv, a.t_uniform ? (T)a.bamp[0] * acc : acc);
#pragma unroll
                for (int u = 0; u < kUpPre; ++u)
                    if (u < (int)n) v = fma_t(up_coef[g * nb + u], upv[u], v);
                for (uint32_t h = kUpPre; h < n; ++h)
                    v = fma_t(up_coef[g * nb + h], x[sc.off + (uint64_t)up_tgt[g * nb + h] * cdn + rd], v);
                if constexpr (LZ) {
                    const T u = lz_out(v, (T)a.ep.c1[tl.sector], a.ep.c2 ? (T)a.ep.c2[tl.sector] : (T)0, pv,
                                       a.ep.c2 != nullptr);
                    out[row] = u;
                    dot = __builtin_fma((double)xv, (double)u, dot);
                } else {
                    out[row] = v;
                }
            }
        }
        if (a.ep.partial) {
            double v = dot;
            for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
            pend = true;
            pend_slot = tl.slot;
        }
    }
    if (pend) {
        __syncthreads();
        fold();
    }
}

// ------------------------------------------------------------------------
// alpha_dn-stationary kernel.  A workgroup of kRowsBlock lanes sweeps a
// contiguous run of tiles (alpha_up blocks of one sector, or a few small
// sectors).  Lane t owns fixed spin-down configurations of the sector: rows
// t + r kRowsBlock (row slot r < R) of each alpha_up block, or one
// (block, alpha_dn) pair when C_dn is small.
//  * down-hops: the targets of an alpha_dn depend on alpha_dn alone.  They are
//    ranked once per launch shape (staggered lookup, hv_lists_kernel) into a
//    list per alpha_dn in bond order of 16-bit LDS byte offsets: the tile's x
//    rows are staged twice, as x and as -x, and the offset selects the copy
//    that carries the hop's fermion sign, so a down hop costs one LDS gather
//    and one add.  Lists are padded with the offset of a zero stored after
//    every block; the trip count of a row slot is the wave's longest list.
//  * up-hops: alpha_up is uniform across a block; its targets are ranked once
//    per tile (one lane per bond, ballot compaction in bond order) and read
//    into scalar registers, so each gather is a scalar base plus the lane's
//    offset.
//  * pipelining: the global loads of row slot r + 1 (up-hop rows, the list,
//    the alpha_dn pattern and energy, the epilogue operand) are issued before
//    the LDS work of slot r, and the next tile's x rows are loaded into
//    registers while this one computes and stored to the other half of a
//    double-buffered LDS tile at its end.
// Tiles are visited in the XCD-binned order of the tile kernel.  Per row the
// terms are summed in the same order and with the same fused operations as in
// the tile kernel, so both give bitwise identical products.
// ------------------------------------------------------------------------
constexpr int kRowsBlock = 1024;
constexpr int kRowsWaves = kRowsBlock / 64;
constexpr int kRowsNB = 16;           // bonds
constexpr int kRowsMaxG = 64;         // alpha_up blocks per tile when C_dn is small
constexpr int kRowsMaxR = 4;          // alpha_dn per lane
constexpr int kUpMax = 8;             // up-hop gathers in flight per row (more run in a tail loop)
constexpr int kRowsDownFixed = 12;    // down-hop entries summed without a branch (padding adds zeros)
constexpr uint32_t kRowsMaxX = 4096;  // staged elements per tile (blocks of C_dn + 1): offsets fit 16 bits
constexpr uint32_t kRowsSlots = 4;    // fp32: alpha_up blocks per tile when each takes a row slot (512 < C_dn <= 1024)
constexpr uint32_t kRowsSlotsUT = 3;  // the same with uniform hopping (R = 4 would spill there)
__host__ __device__ constexpr uint32_t rows_slots(bool ut) { return ut ? kRowsSlotsUT : kRowsSlots; }
static_assert(kRowsMaxX <= (uint32_t)(kRowsMaxR * kRowsBlock), "R slots cover a block");

// LDS layout: rank table | bond amplitudes | on-site U | reduction scratch |
// two buffers.
// A buffer holds the tile's blocks with stride C_dn + 1 (x rows, then a zero)
// from byte 0, the negated rows at byte cs, then up-hop targets |
// coefficients | alpha_up | energies | counts for up to gmax blocks.
struct RowsLds {
    size_t rt, amp, ul, red, buf0, bstride, cs, ut, uc, ua, ue, un, total;
};

__host__ __device__ inline RowsLds rows_lds_layout(uint32_t rtab_entries, uint32_t xcap, uint32_t gmax,
                                                   size_t tsz) {
    auto r16 = [](size_t v) { return (v + 15) & ~(size_t)15; };
    RowsLds L{};
    size_t o = 0;
    L.rt = o;
    o += r16((size_t)rtab_entries * 2);
    L.amp = o;
    o += r16(kRowsNB * tsz);
    L.ul = o;
    o += r16(kMaxSites * tsz);
    L.red = o;
    o += 32 * sizeof(double);
    L.buf0 = o;
    L.cs = r16((size_t)xcap * tsz);
    size_t b = 2 * L.cs;
    L.ut = b;
    b += r16((size_t)gmax * kRowsNB * 4);
    L.uc = b;
    b += r16((size_t)gmax * kRowsNB * tsz);
    L.ua = b;
    b += r16((size_t)gmax * 4);
    L.ue = b;
    b += r16((size_t)gmax * tsz);
    L.un = b;
    b += r16((size_t)gmax * 4);
    L.bstride = b;
    L.total = o + 2 * b;
    return L;
}

template <class T>
__device__ __forceinline__ T uniform_val(T v) {
    if constexpr (sizeof(T) == 8) {
        uint64_t u;
        __builtin_memcpy(&u, &v, 8);
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
        u = ((uint64_t)hi << 32) | lo;
        T r;
        __builtin_memcpy(&r, &u, 8);
        return r;
    } else {
        uint32_t u;
        __builtin_memcpy(&u, &v, 4);
        u = __builtin_amdgcn_readfirstlane(u);
        T r;
        __builtin_memcpy(&r, &u, 4);
        return r;
    }
}

// Staged-row byte offset of down-hop target rr (negated copy for an even
// number of fermions between the bond's sites, i.e. coefficient -t).
__device__ __forceinline__ uint32_t rows_entry(uint32_t rr, bool odd, uint32_t tsz, uint32_t cs) {
    return rr * tsz + (odd ? 0u : cs);
}

// Down-hop lists of one rows-kernel sector: row rd of `lists` holds the
// entries of alpha_dn number rd (kRowsNB - 1 of them, 16-bit offsets two per
// word when every bond has the same amplitude, else one per word with the bond
// in the high half), padded with the offset of the block's zero, and the list
// length in the last entry.
template <bool UT>
__global__ void __launch_bounds__(256) hv_lists_kernel(HvArgs a, uint32_t hs_dn, uint32_t cdn, uint32_t tsz,
                                                       uint32_t cs, uint32_t *lists) {
    const uint32_t rd = blockIdx.x * blockDim.x + threadIdx.x;
    if (rd >= cdn) return;
    constexpr int kWords = UT ? kRowsNB / 2 : kRowsNB;
    const uint32_t ad = a.hs_states[hs_dn + rd];
    const uint32_t zero = cdn * tsz;
    uint32_t w[kWords];
    for (int u = 0; u < kWords; ++u) w[u] = UT ? (zero | (zero << 16)) : zero;
    uint32_t n = 0;
    for (int b = 0; b < a.nb; ++b) {
        const uint32_t bi = a.bij[b] & 0xFF, bj = a.bij[b] >> 8;
        if (!(((ad >> bi) ^ (ad >> bj)) & 1)) continue;
        const uint32_t rr = rank_half<0>(ad ^ a.bmask[b], a.rtab, a);
        uint32_t e = rows_entry(rr, __popc(ad & a.bbetw[b]) & 1, tsz, cs);
        if constexpr (UT) {
            const int wd = n >> 1, sh = (n & 1) * 16;
            w[wd] = (w[wd] & ~(0xFFFFu << sh)) | (e << sh);
        } else {
            w[n] = e | ((uint32_t)b << 16);
        }
        ++n;
    }
    // the last entry holds the length (at most kRowsNB - 1 bonds in this mode)
    if constexpr (UT) w[kWords - 1] = (w[kWords - 1] & 0xFFFFu) | (n << 16);
    else w[kWords - 1] = n;
    for (int u = 0; u < kWords; ++u) lists[(size_t)rd * kWords + u] = w[u];
}

// On-site U energy of a doubly occupied pattern, as u_energy but with the
// site values read from LDS (same order of summation).
template <class T>
__device__ __forceinline__ T rows_u_energy(uint32_t both, const HvArgs &a, const T *ul) {
    if (a.U_uniform) return (T)(a.U0 * (double)__popc(both));
    T e = 0;
    uint32_t m = both & a.Umask;
    while (m) {
        const int i = __ffs(m) - 1;
        m &= m - 1;
        e += ul[i];
    }
    return e;
}

// Up-hop lists of a tile's blocks into buffer bb: lane t ranks bond t % 16 of
// block t / 16 (16-lane groups stay inside a wave) and the hops are compacted
// in bond order with a ballot.  au, eu: the block's alpha_up and its energy,
// loaded ahead by the caller.
template <class T>
__device__ __forceinline__ void rows_uplists(const HvArgs &a, const uint16_t *rt, uint32_t nblk, uint32_t au,
                                             T eu, unsigned char *bb, const RowsLds &LL) {
    uint32_t *ut = reinterpret_cast<uint32_t *>(bb + LL.ut);
    T *uc = reinterpret_cast<T *>(bb + LL.uc);
    uint32_t *ua = reinterpret_cast<uint32_t *>(bb + LL.ua);
    T *ue = reinterpret_cast<T *>(bb + LL.ue);
    uint32_t *un = reinterpret_cast<uint32_t *>(bb + LL.un);
    const uint32_t t = threadIdx.x;
    const uint32_t g = t >> 4, b = t & 15;
    bool hop = false;
    uint32_t tgt = 0;
    T coef = 0;
    if (g < nblk) {
        if ((int)b < a.nb) {
            const uint32_t bi = a.bij[b] & 0xFF, bj = a.bij[b] >> 8;
            hop = ((au >> bi) ^ (au >> bj)) & 1;
            if (hop) {
                tgt = rank_half<0>(au ^ a.bmask[b], rt, a);
                coef = (__popc(au & a.bbetw[b]) & 1) ? (T)a.bamp[b] : -(T)a.bamp[b];
            }
        }
        if (b == 0) {
            ua[g] = au;
            ue[g] = eu;
        }
    }
    const unsigned long long bal = __ballot(hop);
    const int lane = threadIdx.x & 63;
    const unsigned long long grp = 0xFFFFull << (lane & 48);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t nu = (uint32_t)__popcll(bal & grp);
    if (hop) {
        const uint32_t pos = (uint32_t)__popcll(bal & grp & below);
        ut[g * kRowsNB + pos] = tgt;
        uc[g * kRowsNB + pos] = coef;
    }
    if (g < nblk && b >= nu) {
        // entries past the hops (every position b >= nu, written by lane b
        // whether or not it hops itself: a hop lane's own entry lies below nu):
        // block 0 of the sector with coefficient 0, so a fixed number of
        // gathers can be read and summed without a branch
        ut[g * kRowsNB + b] = 0u;
        uc[g * kRowsNB + b] = (T)0;
    }
    if (b == 0 && g < nblk) un[g] = nu;
}

// Staging of a tile's x rows: each lane loads kRowsPre rows into registers
// (a fixed number of loads, so the compiler's wait counts stay exact) while
// the previous tile computes, then stores them at the end of that tile as x
// at byte g (C_dn + 1) sizeof(T) + i sizeof(T) of the buffer for row
// g C_dn + i, as -x at cs bytes further, and a zero after every block.
constexpr int kRowsPre = (kRowsMaxX + kRowsBlock - 1) / kRowsBlock;

template <class T>
__device__ __forceinline__ void rows_pre_load(const T *src, uint32_t rows, T (&pre)[kRowsPre]) {
#pragma unroll
    for (int j = 0; j < kRowsPre; ++j) {
        const uint32_t e = threadIdx.x + j * kRowsBlock;
        pre[j] = src[e < rows ? e : 0];
    }
}

template <class T>
__device__ __forceinline__ void rows_pre_store(unsigned char *bb, size_t cs, uint32_t nblk, uint32_t cdn,
                                               const T (&pre)[kRowsPre]) {
    T *xp = reinterpret_cast<T *>(bb);
    T *xm = reinterpret_cast<T *>(bb + cs);
    const uint32_t rows = nblk * cdn;
    // block g = e / C_dn of element e = t + j 1024, stepped from j to j + 1
    // by the quotient and remainder of 1024 / C_dn
    const uint32_t qs = (uint32_t)kRowsBlock / cdn, rs = (uint32_t)kRowsBlock - qs * cdn;
    uint32_t g = threadIdx.x / cdn, rem = threadIdx.x - g * cdn;
#pragma unroll
    for (int j = 0; j < kRowsPre; ++j) {
        const uint32_t e = threadIdx.x + j * kRowsBlock;
        if (e < rows) {
            const uint32_t pos = e + g;  // g (C_dn + 1) + (e - g C_dn)
            xp[pos] = pre[j];
            xm[pos] = -pre[j];
        }
        g += qs;
        rem += rs;
        if (rem >= cdn) {
            rem -= cdn;
            ++g;
        }
    }
    if (threadIdx.x < nblk) xp[threadIdx.x * (cdn + 1) + cdn] = (T)0;
}

// Sum of the down-hop terms of one row: the list entries (byte offsets from
// xb) in groups of four; the groups past kRowsDownFixed entries are skipped
// when they are past the end of every list of the wave.  Uniform amplitude: the signed x values are summed (the
// caller scales by t); otherwise each is weighted by its bond's amplitude.
// FIX: entries summed without a branch.  The padding adds +0 to a sum that
// starts at +0 and so is never -0: FIX does not change the result.
template <class T, bool UT, int W, int FIX = kRowsDownFixed>
__device__ __forceinline__ T rows_down(const uint32_t (&hl)[W], const unsigned char *xb, const T *amp,
                                       bool valid) {
    const uint32_t n = valid ? (UT ? hl[W - 1] >> 16 : hl[W - 1]) : 0u;
    T acc = 0;
#pragma unroll
    for (int u0 = 0; u0 < kRowsNB - 1; u0 += 4) {
        // the first groups run unconditionally (padding reads the zero): a
        // branch there would let the compiler sink the list load into it
        if (u0 < FIX || (uint32_t)u0 < n) {
            constexpr int kQ = 4;
            T v[kQ];
            T c[kQ];
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int u = u0 + q;
                if (u < kRowsNB - 1) {
                    uint32_t e;
                    if constexpr (UT) e = (hl[u >> 1] >> ((u & 1) * 16)) & 0xFFFFu;
                    else e = hl[u];
                    v[q] = *reinterpret_cast<const T *>(xb + (e & 0xFFFFu));
                    if constexpr (!UT) c[q] = amp[e >> 16];
                }
            }
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                if (u0 + q < kRowsNB - 1) {
                    if constexpr (UT) acc += v[q];
                    else acc = fma_t(c[q], v[q], acc);
                }
            }
        }
    }
    return acc;
}

template <int W>
__device__ __forceinline__ void rows_load_list(const uint32_t *row, uint32_t (&hl)[W]) {
    const uint4 *p = reinterpret_cast<const uint4 *>(row);
#pragma unroll
    for (int q = 0; q < W / 4; ++q) {
        const uint4 v = p[q];
        hl[4 * q] = v.x;
        hl[4 * q + 1] = v.y;
        hl[4 * q + 2] = v.z;
        hl[4 * q + 3] = v.w;
    }
}

// Uniform copy of a rows-kernel tile descriptor (RowsTileDesc).
struct RowsTile {
    uint64_t base, soff;
    uint32_t cdn, gp, nblk, hs_up0, hs_dn, loff, sector, slot;
};

__device__ __forceinline__ void rows_desc_load(const RowsTileDesc *d, uint32_t t, uint4 (&q)[2]) {
    const uint4 *p = reinterpret_cast<const uint4 *>(d + t);
    q[0] = p[0];
    q[1] = p[1];
}

__device__ __forceinline__ RowsTile rows_desc_uniform(const uint4 (&q)[2]) {
    auto u = [](uint32_t v) { return __builtin_amdgcn_readfirstlane(v); };
    RowsTile r;
    r.base = ((uint64_t)u(q[0].y) << 32) | u(q[0].x);
    r.soff = ((uint64_t)u(q[0].w) << 32) | u(q[0].z);
    const uint32_t w0 = u(q[1].x), w1 = u(q[1].y), w2 = u(q[1].z);
    r.cdn = w0 & 0xFFF;
    r.gp = (w0 >> 12) & 0xFF;
    r.nblk = w0 >> 20;
    r.hs_up0 = w1 & 0xFFFF;
    r.hs_dn = w1 >> 16;
    r.loff = w2 & 0xFFFF;
    r.sector = w2 >> 16;
    r.slot = u(q[1].w);
    return r;
}

// Up-hop terms kUpMax .. of one row past the first batch, in groups of four:
// a group's gathers are all issued before its sums (entries past the block's
// hops are block 0 with coefficient 0, so a group needs no branch inside).
// U: the lists are the same for the whole wave (values taken from lane 0);
// otherwise a group runs when any lane of the wave needs it.
template <class T, bool U>
__device__ __forceinline__ T rows_up_tail(const T *xsec, const uint32_t *utb, const T *ucb, uint32_t cdn,
                                          uint32_t rd, uint32_t nu, T v) {
#pragma unroll
    for (int h0 = kUpMax; h0 < kRowsNB; h0 += 4) {
        const bool need = U ? nu > (uint32_t)h0 : __ballot(nu > (uint32_t)h0) != 0;
        if (!need) break;
        T g[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t t = utb[h0 + q];
            if constexpr (U) t = __builtin_amdgcn_readfirstlane(t);
            g[q] = xsec[(uint64_t)t * cdn + rd];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            T c = ucb[h0 + q];
            if constexpr (U) c = uniform_val(c);
            v = fma_t(c, g[q], v);
        }
    }
    return v;
}

template <class T, bool LZ, int R, bool UT>
__global__ void __launch_bounds__(kRowsBlock) hv_rows_kernel(HvArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const RowsLds LL = rows_lds_layout(a.rtab_entries, a.xcap, a.rgmax, sizeof(T));
    uint16_t *rt = reinterpret_cast<uint16_t *>(smem + LL.rt);
    T *amp = reinterpret_cast<T *>(smem + LL.amp);
    T *ul = reinterpret_cast<T *>(smem + LL.ul);
    double *red = reinterpret_cast<double *>(smem + LL.red);
    for (uint32_t i = threadIdx.x; i < a.rtab_entries; i += blockDim.x) rt[i] = a.rtab[i];
    if (threadIdx.x < (uint32_t)kRowsNB)
        amp[threadIdx.x] = threadIdx.x < (uint32_t)a.nb ? (T)a.bamp[threadIdx.x] : (T)0;
    if (threadIdx.x < (uint32_t)kMaxSites) ul[threadIdx.x] = (T)a.U[threadIdx.x];

    const T *x = static_cast<const T *>(a.x);
    T *out = static_cast<T *>(a.out);
    const T *p = static_cast<const T *>(a.ep.p);
    if (a.ep.basis_j) {
        const int64_t j = *a.ep.basis_j;
        x += (uint64_t)j * a.ep.basis_stride;
        p = j > 0 ? x - a.ep.basis_stride : x;
    }
    uint32_t t_cur, t_end, t_step;
    if (a.binned) {
        const uint32_t xcd = blockIdx.x % kXcd;
        t_cur = a.xoff[xcd] + blockIdx.x / kXcd;
        t_end = a.xoff[xcd + 1];
        t_step = (gridDim.x - xcd + kXcd - 1) / kXcd;
    } else {
        t_cur = blockIdx.x;
        t_end = a.n_tiles;
        t_step = gridDim.x;
    }
    if (t_cur >= t_end) return;

    const int tid = threadIdx.x;
    constexpr int kWords = UT ? kRowsNB / 2 : kRowsNB;
    const uint32_t *lists = static_cast<const uint32_t *>(a.lists);
    const RowsTileDesc *desc = a.rdesc;
    const T tu = (T)a.bamp[0];
    const uint32_t ug = (uint32_t)tid >> 4;  // block of this lane in the up-hop ranking
    const bool has_p = LZ && a.ep.c2;

    // Tile descriptors are loaded two tiles ahead and the per-tile scalars
    // (flags, epilogue coefficients, alpha_up of the ranking lanes) one tile
    // ahead, so no dependent load sits at the head of a tile.
    uint4 qc[2], qn[2];
    rows_desc_load(desc, t_cur, qc);
    rows_desc_load(desc, t_cur + t_step < t_end ? t_cur + t_step : t_cur, qn);
    int act_c;
    T c1_c, c2_c;
    __syncthreads();  // rank table, amplitudes and U in LDS
    {
        const RowsTile c = rows_desc_uniform(qc);
        unsigned char *bb = smem + LL.buf0;
        T pre[kRowsPre];
        rows_pre_load<T>(x + c.base, c.nblk * c.cdn, pre);
        const uint32_t au = ug < c.nblk ? a.hs_states[c.hs_up0 + ug] : 0u;
        const T eu = ug < c.nblk ? (T)a.hs_energy[c.hs_up0 + ug] : (T)0;
        act_c = a.ep.active ? a.ep.active[c.sector] : 1;
        c1_c = LZ ? (T)a.ep.c1[c.sector] : (T)1;
        c2_c = has_p ? (T)a.ep.c2[c.sector] : (T)0;
        rows_uplists<T>(a, rt, c.nblk, au, eu, bb, LL);
        rows_pre_store<T>(bb, LL.cs, c.nblk, c.cdn, pre);
    }
    __syncthreads();

    // One alpha_up block per tile: the spin-down side of a row slot (its
    // down-hop list, half state and energy) is the same in every tile of a
    // sector, so a lane keeps its slots' copies in registers until the tile's
    // sector changes, where registers allow: at most 32 list words, and in
    // fp64 only the short lists of uniform hopping and at most two slots (the
    // other fp64 shapes already fill the 128 registers of a 1024-lane
    // workgroup).
    constexpr bool kKeepDn = R * kWords <= 32 && (sizeof(T) == 4 || (UT && R <= 2));
    constexpr bool kKeepHs = kKeepDn || UT;  // the half states and energies alone
    uint32_t hlc[kKeepDn ? R : 1][kWords], gac[kKeepHs ? R : 1];
    T gec[kKeepHs ? R : 1];
    uint32_t kept_loff = 0xFFFFFFFFu, kept_hs = 0xFFFFFFFFu;

    for (int buf = 0; t_cur < t_end; t_cur += t_step, buf ^= 1) {
        const RowsTile c = rows_desc_uniform(qc);
        const uint32_t t_next = t_cur + t_step;
        const bool has_next = t_next < t_end;
        uint4 qnn[2];
        rows_desc_load(desc, t_next + t_step < t_end ? t_next + t_step : t_cur, qnn);
        const bool active = __builtin_amdgcn_readfirstlane(act_c) != 0;
        const T c1 = uniform_val(c1_c), c2 = uniform_val(c2_c);

        // the next tile's x rows are loaded into registers while this tile
        // computes, and so are its scalars
        unsigned char *nb2 = smem + LL.buf0 + (size_t)(buf ^ 1) * LL.bstride;
        RowsTile n{};
        uint32_t au_n = 0;
        T eu_n = 0;
        T pre[kRowsPre];
        if (has_next) {
            n = rows_desc_uniform(qn);
            rows_pre_load<T>(x + n.base, n.nblk * n.cdn, pre);
            if (ug < n.nblk) {
                au_n = a.hs_states[n.hs_up0 + ug];
                eu_n = (T)a.hs_energy[n.hs_up0 + ug];
            }
            act_c = a.ep.active ? a.ep.active[n.sector] : 1;
            c1_c = LZ ? (T)a.ep.c1[n.sector] : (T)1;
            c2_c = has_p ? (T)a.ep.c2[n.sector] : (T)0;
        }

        const uint32_t cdn = c.cdn;
        const uint64_t base = c.base;
        const unsigned char *bb = smem + LL.buf0 + (size_t)buf * LL.bstride;
        const uint32_t *ut = reinterpret_cast<const uint32_t *>(bb + LL.ut);
        const T *uc = reinterpret_cast<const T *>(bb + LL.uc);
        const uint32_t *ua = reinterpret_cast<const uint32_t *>(bb + LL.ua);
        const T *ue = reinterpret_cast<const T *>(bb + LL.ue);
        const uint32_t *un = reinterpret_cast<const uint32_t *>(bb + LL.un);
        const uint32_t *slists = lists + (size_t)c.loff * kWords;
        const T *xsec = x + c.soff;
        double dot = 0.0;
        if (active) {
            if (c.gp == 1) {
                // One alpha_up block per tile: its data is uniform, held in scalars.
                const uint32_t nu = __builtin_amdgcn_readfirstlane(un[0]);
                const uint32_t au = __builtin_amdgcn_readfirstlane(ua[0]);
                const T eu = uniform_val(ue[0]);
                const T *src[kUpMax];
                T cf[kUpMax];
                // entries past nu are block 0 with coefficient 0: read without a branch
#pragma unroll
                for (int h = 0; h < kUpMax; ++h) {
                    src[h] = xsec + (uint64_t)__builtin_amdgcn_readfirstlane(ut[h]) * cdn;
                    cf[h] = uniform_val(uc[h]);
                }
                T gx[2][kUpMax], gp_[2], ge[2];
                uint32_t ga[2];
                uint32_t hl[2][kWords];
                // a fixed batch of loads per row slot (lanes past C_dn read row 0,
                // hops past nu read row 0 of the sector with coefficient 0), so
                // the wait for slot r leaves slot r + 1 in flight
                const T *pp = has_p ? p : x;
                if constexpr (kKeepHs) {
                    if (c.loff != kept_loff || c.hs_dn != kept_hs) {
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const int rd = tid + r * kRowsBlock;
                            const int rc = rd < (int)cdn ? rd : 0;
                            if constexpr (kKeepDn) rows_load_list(slists + (size_t)rc * kWords, hlc[r]);
                            gac[r] = a.hs_states[c.hs_dn + rc];
                            gec[r] = (T)a.hs_energy[c.hs_dn + rc];
                        }
                        kept_loff = c.loff;
                        kept_hs = c.hs_dn;
                    }
                }
                auto gather = [&](int r, int s) {
                    const int rd = tid + r * kRowsBlock;
                    const int rc = rd < (int)cdn ? rd : 0;
#pragma unroll
                    for (int h = 0; h < kUpMax; ++h) gx[s][h] = src[h][rc];
                    if constexpr (!kKeepDn) rows_load_list(slists + (size_t)rc * kWords, hl[s]);
                    if constexpr (!kKeepHs) {
                        ga[s] = a.hs_states[c.hs_dn + rc];
                        ge[s] = (T)a.hs_energy[c.hs_dn + rc];
                    }
                    if constexpr (LZ) gp_[s] = pp[base + rc];
                };
                gather(0, 0);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int s = r & 1;
                    if (r + 1 < R) gather(r + 1, s ^ 1);
                    const int rd = tid + r * kRowsBlock;
                    const uint32_t(&hlr)[kWords] = kKeepDn ? hlc[kKeepDn ? r : 0] : hl[s];
                    const uint32_t gar = kKeepHs ? gac[kKeepHs ? r : 0] : ga[s];
                    const T ger = kKeepHs ? gec[kKeepHs ? r : 0] : ge[s];
                    const T acc = rows_down<T, UT>(hlr, bb, amp, rd < (int)cdn);
                    if (rd < (int)cdn) {
                        const T xv = reinterpret_cast<const T *>(bb)[rd];
                        const T dg = eu + ger + rows_u_energy<T>(au & gar, a, ul);
                        T v = fma_t(dg, xv, UT ? tu * acc : acc);
                        // cf = 0 and gx = x[row 0] past nu: those terms add an exact zero
#pragma unroll
                        for (int h = 0; h < kUpMax; ++h) v = fma_t(cf[h], gx[s][h], v);
                        v = rows_up_tail<T, true>(xsec, ut, uc, cdn, (uint32_t)rd, nu, v);
                        const uint64_t row = base + rd;
                        if constexpr (LZ) {
                            const T uu = lz_out(v, c1, c2, gp_[s], has_p);
                            out[row] = uu;
                            dot = __builtin_fma((double)xv, (double)uu, dot);
                        } else {
                            out[row] = v;
                        }
                    }
                }
            } else if (sizeof(T) == 4 && R <= (int)rows_slots(UT) && c.gp == 0) {
                // Several alpha_up blocks per tile (C_dn <= 1024), one per row
                // slot: lane tid owns alpha_dn = tid in every block, so its
                // down-hop list, half state and energy serve all of them, and
                // the up-hop gathers of block r + 1 are in flight while block r
                // computes.  Same sums as the one-block path.
                const int rd = tid;
                const bool valid = rd < (int)cdn;
                const int rc = valid ? rd : 0;
                T gx[2][kUpMax], cfs[2][kUpMax], gp_[2];
                uint32_t hl1[kWords];
                uint32_t ga1 = 0;
                T ge1 = 0;
                const T *pp = has_p ? p : x;
                if constexpr (kKeepHs) {
                    // only slot 0's copies: tagged so that the one-block path reloads all
                    const uint32_t tag = c.loff | 0x80000000u;
                    if (tag != kept_loff || c.hs_dn != kept_hs) {
                        if constexpr (kKeepDn) rows_load_list(slists + (size_t)rc * kWords, hlc[0]);
                        gac[0] = a.hs_states[c.hs_dn + rc];
                        gec[0] = (T)a.hs_energy[c.hs_dn + rc];
                        kept_loff = tag;
                        kept_hs = c.hs_dn;
                    }
                }
                if constexpr (!kKeepDn) rows_load_list(slists + (size_t)rc * kWords, hl1);
                if constexpr (!kKeepHs) {
                    ga1 = a.hs_states[c.hs_dn + rc];
                    ge1 = (T)a.hs_energy[c.hs_dn + rc];
                }
                const uint32_t(&hld)[kWords] = kKeepDn ? hlc[0] : hl1;
                const uint32_t gad = kKeepHs ? gac[0] : ga1;
                const T ged = kKeepHs ? gec[0] : ge1;
                const int nblk = (int)c.nblk;
                auto gather = [&](int g, int sl) {
                    // entries past the block's hops are block 0 with coefficient 0
#pragma unroll
                    for (int h = 0; h < kUpMax; ++h) {
                        const uint32_t t = __builtin_amdgcn_readfirstlane(ut[g * kRowsNB + h]);
                        gx[sl][h] = xsec[(uint64_t)t * cdn + rc];
                        cfs[sl][h] = uniform_val(uc[g * kRowsNB + h]);
                    }
                    if constexpr (LZ) gp_[sl] = pp[base + (uint64_t)g * cdn + rc];
                };
                gather(0, 0);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (r >= nblk) break;
                    const int sl = r & 1;
                    if (r + 1 < R && r + 1 < nblk) gather(r + 1, sl ^ 1);
                    const unsigned char *xb = bb + (size_t)r * (cdn + 1) * sizeof(T);
                    const T acc = rows_down<T, UT>(hld, xb, amp, valid);
                    if (valid) {
                        const uint32_t nu = __builtin_amdgcn_readfirstlane(un[r]);
                        const uint32_t au = __builtin_amdgcn_readfirstlane(ua[r]);
                        const T eu = uniform_val(ue[r]);
                        const T xv = reinterpret_cast<const T *>(xb)[rd];
                        const T dg = eu + ged + rows_u_energy<T>(au & gad, a, ul);
                        T v = fma_t(dg, xv, UT ? tu * acc : acc);
#pragma unroll
                        for (int h = 0; h < kUpMax; ++h) v = fma_t(cfs[sl][h], gx[sl][h], v);
                        v = rows_up_tail<T, true>(xsec, ut + r * kRowsNB, uc + r * kRowsNB, cdn, (uint32_t)rd,
                                                  nu, v);
                        const uint64_t row = base + (uint64_t)r * cdn + rd;
                        if constexpr (LZ) {
                            const T uu = lz_out(v, c1, c2, gp_[sl], has_p);
                            out[row] = uu;
                            dot = __builtin_fma((double)xv, (double)uu, dot);
                        } else {
                            out[row] = v;
                        }
                    }
                }
            } else {
                // several small blocks per tile: block data per lane from LDS; the
                // first kUpMax up-hop gathers are issued before the LDS work
                const int g = tid / (int)cdn;
                if (g < (int)c.nblk && g < (int)c.gp) {
                    const int rd = tid - g * (int)cdn;
                    const uint64_t row = base + (uint64_t)g * cdn + rd;
                    const uint32_t nu = un[g];
                    // entries past nu are block 0 with coefficient 0: no branch
                    T gx[kUpMax];
#pragma unroll
                    for (int h = 0; h < kUpMax; ++h) gx[h] = xsec[(uint64_t)ut[g * kRowsNB + h] * cdn + rd];
                    uint32_t hl[kWords];
                    rows_load_list(slists + (size_t)rd * kWords, hl);
                    const T pv = has_p ? p[row] : (T)0;
                    const uint32_t adr = a.hs_states[c.hs_dn + rd];
                    const T edr = (T)a.hs_energy[c.hs_dn + rd];
                    const unsigned char *xb = bb + (size_t)g * (cdn + 1) * sizeof(T);
                    const T acc = rows_down<T, UT>(hl, xb, amp, true);
                    const T xv = reinterpret_cast<const T *>(xb)[rd];
                    const T dg = ue[g] + edr + rows_u_energy<T>(ua[g] & adr, a, ul);
                    T v = fma_t(dg, xv, UT ? tu * acc : acc);
#pragma unroll
                    for (int h = 0; h < kUpMax; ++h) v = fma_t(uc[g * kRowsNB + h], gx[h], v);
                    v = rows_up_tail<T, false>(xsec, ut + g * kRowsNB, uc + g * kRowsNB, cdn, (uint32_t)rd, nu, v);
                    if constexpr (LZ) {
                        const T uu = lz_out(v, c1, c2, pv, has_p);
                        out[row] = uu;
                        dot = __builtin_fma((double)xv, (double)uu, dot);
                    } else {
                        out[row] = v;
                    }
                }
            }
        }
        // tile partial of <q_j, u>: each wave leaves its sum in this tile's half
        // of red; after the barrier below wave 0 adds the 16 of them (a fixed
        // tree) while the other waves go on, so the tile costs no extra barrier
        if (a.ep.partial) {
            double v = dot;
            for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
            if ((tid & 63) == 0) red[buf * kRowsWaves + (tid >> 6)] = v;
        }
        // next tile: up-hop targets, negated copy of the staged rows, zeros
        if (has_next) {
            rows_uplists<T>(a, rt, n.nblk, au_n, eu_n, nb2, LL);
            rows_pre_store<T>(nb2, LL.cs, n.nblk, n.cdn, pre);
        }
        __syncthreads();
        if (a.ep.partial && tid < 64) {
            // red[buf] is rewritten two tiles on, after the next barrier
            double v = tid < kRowsWaves ? red[buf * kRowsWaves + tid] : 0.0;
            for (int o = kRowsWaves / 2; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
            if (tid == 0) a.ep.partial[c.slot] = active ? v : 0.0;
        }
        qc[0] = qn[0];
        qc[1] = qn[1];
        qn[0] = qnn[0];
        qn[1] = qnn[1];
    }
}

// ------------------------------------------------------------------------
// Block kernel (launch shape G = -2) for sectors with C_dn > 512.  One
// alpha_up block per 1024-lane workgroup and no loop over tiles: a workgroup
// stages its block of x in LDS (x and -x, the layout the down-hop lists
// address), sums its rows and exits, so a CU holds two of them, each with its
// own loads in flight, where the rows kernel holds one that sweeps tile after
// tile behind a barrier.  The up-hop targets and signed amplitudes of every
// half state are listed once per launch shape (hv_uplists_kernel) and read
// as scalars.  The workgroups of an XCD take one contiguous, cost-balanced
// range of tiles, so the neighbouring alpha_up blocks that the up-hops gather
// meet in that XCD's L2.  Terms are summed in the order of the rows kernel
// (down-hops in list order, the diagonal, up-hops in bond order) with the same
// fused operations, so the products are bitwise equal.
// ------------------------------------------------------------------------
constexpr int kBlockLanes = 1024;
constexpr uint32_t kBlockMin = kBlockLanes / 2;  // C_dn above which a sector takes this kernel

template <class T>
struct BlockUpLists {
    const uint32_t *tgt;  // [half state][kRowsNB]: target ranks in bond order, 0 past the hops
    const T *coef;        // [half state][kRowsNB]: signed amplitudes, 0 past the hops
    const uint32_t *n;    // [half state]: number of hops
};

// Up-hop lists of every half state (one lane each), with the ranks and signed
// amplitudes that rows_uplists computes for a tile's blocks.
template <class T>
__global__ void __launch_bounds__(256) hv_uplists_kernel(HvArgs a, uint32_t n_hs, uint32_t *tgt, T *coef,
                                                         uint32_t *cnt) {
    const uint32_t hs = blockIdx.x * blockDim.x + threadIdx.x;
    if (hs >= n_hs) return;
    const uint32_t au = a.hs_states[hs];
    uint32_t n = 0;
    for (int b = 0; b < a.nb; ++b) {
        const uint32_t bi = a.bij[b] & 0xFF, bj = a.bij[b] >> 8;
        if (!(((au >> bi) ^ (au >> bj)) & 1)) continue;
        tgt[(size_t)hs * kRowsNB + n] = rank_half<0>(au ^ a.bmask[b], a.rtab, a);
        coef[(size_t)hs * kRowsNB + n] = (__popc(au & a.bbetw[b]) & 1) ? (T)a.bamp[b] : -(T)a.bamp[b];
        ++n;
    }
    for (uint32_t u = n; u < (uint32_t)kRowsNB; ++u) {
        tgt[(size_t)hs * kRowsNB + u] = 0u;
        coef[(size_t)hs * kRowsNB + u] = (T)0;
    }
    cnt[hs] = n;
}

// LDS of the block kernel: x at byte 0 and -x at byte cs (cs = the down-hop
// lists' offset of the negated copy), bond amplitudes, on-site U, reduction,
// then alpha_up's up-hop targets and coefficients.
__host__ __device__ inline size_t block_lds_bytes(uint32_t xcap, size_t tsz) {
    const size_t cs = ((size_t)xcap * tsz + 15) & ~(size_t)15;
    return 2 * cs + (size_t)(kRowsNB + kMaxSites) * tsz + kRowsWaves * sizeof(double) + (size_t)kRowsNB * (4 + tsz);
}

template <class T, bool LZ, bool UT>
__global__ void __launch_bounds__(kBlockLanes) hv_block_kernel(HvArgs a, BlockUpLists<T> up) {
    extern __shared__ __align__(16) unsigned char smem[];
    const size_t cs = ((size_t)a.xcap * sizeof(T) + 15) & ~(size_t)15;
    T *xp = reinterpret_cast<T *>(smem);
    T *xm = reinterpret_cast<T *>(smem + cs);
    T *amp = reinterpret_cast<T *>(smem + 2 * cs);
    T *ul = amp + kRowsNB;
    double *red = reinterpret_cast<double *>(smem + 2 * cs + (size_t)(kRowsNB + kMaxSites) * sizeof(T));
    uint32_t *lt = reinterpret_cast<uint32_t *>(red + kRowsWaves);
    T *lc = reinterpret_cast<T *>(lt + kRowsNB);
    uint32_t ti;
    if (a.binned) {
        const uint32_t xcd = blockIdx.x % kXcd;
        ti = a.xoff[xcd] + blockIdx.x / kXcd;
        if (ti >= a.xoff[xcd + 1]) return;  // whole workgroup: no barrier is skipped by part of it
    } else {
        ti = blockIdx.x;
        if (ti >= a.n_tiles) return;
    }
    const int tid = threadIdx.x;
    uint4 q[2];
    rows_desc_load(a.rdesc, ti, q);
    const RowsTile c = rows_desc_uniform(q);
    const T *x = static_cast<const T *>(a.x);
    T *out = static_cast<T *>(a.out);
    const T *p = static_cast<const T *>(a.ep.p);
    if (a.ep.basis_j) {
        const int64_t j = *a.ep.basis_j;
        x += (uint64_t)j * a.ep.basis_stride;
        p = j > 0 ? x - a.ep.basis_stride : x;
    }
    const uint32_t cdn = c.cdn;
    // Every load the workgroup needs before its barrier is issued first, so
    // that they are in flight together: the block of x (vector), alpha_up's
    // pattern, energy and up-hop lists (scalar).
    const T *xs = x + c.base;
    T pre[kRowsMaxR];
#pragma unroll
    for (int r = 0; r < kRowsMaxR; ++r) {
        const uint32_t e = tid + r * kBlockLanes;
        pre[r] = xs[e < cdn ? e : 0];
    }
    const uint32_t hsu = c.hs_up0;
    // the 16-bit pattern from its aligned 32-bit word (a scalar load)
    const uint32_t hw = reinterpret_cast<const uint32_t *>(a.hs_states)[hsu >> 1];
    const uint32_t au = __builtin_amdgcn_readfirstlane((hw >> ((hsu & 1) * 16)) & 0xFFFFu);
    const T eu = uniform_val((T)a.hs_energy[hsu]);
    const uint32_t nu = __builtin_amdgcn_readfirstlane(up.n[hsu]);
    const uint32_t *utb = up.tgt + (size_t)hsu * kRowsNB;
    const T *ucb = up.coef + (size_t)hsu * kRowsNB;
    const T *xsec = x + c.soff;
    // the first kUpMax entries in scalar registers; all of them in LDS for
    // the tail (reloading them from memory inside the row loop, past the
    // stores to out, costs a round trip per row; holding all sixteen in
    // scalar registers leaves too few of those for two workgroups per CU)
    // (sources as 32-bit byte offsets in the sector, which configure keeps
    // below 4 GiB: one scalar register each instead of a pointer's two)
    T cf[kUpMax];
    uint32_t sob[kUpMax];
#pragma unroll
    for (int h = 0; h < kUpMax; ++h) {
        sob[h] = __builtin_amdgcn_readfirstlane(utb[h]) * cdn * (uint32_t)sizeof(T);
        cf[h] = uniform_val(ucb[h]);
    }
    const unsigned char *xsb = reinterpret_cast<const unsigned char *>(xsec);
    if (tid < kRowsNB) {
        lt[tid] = utb[tid];
        lc[tid] = ucb[tid];
    }
    // the block of x, its negation, and a zero after it; amplitudes and U
    // only where the sums read them (bond-dependent hopping, site-dependent U)
#pragma unroll
    for (int r = 0; r < kRowsMaxR; ++r) {
        const uint32_t e = tid + r * kBlockLanes;
        if (e < cdn) {
            xp[e] = pre[r];
            xm[e] = -pre[r];
        }
    }
    if (tid == 0) xp[cdn] = (T)0;
    if (!UT && tid < kRowsNB) amp[tid] = tid < a.nb ? (T)a.bamp[tid] : (T)0;
    if (!a.U_uniform && tid < kMaxSites) ul[tid] = (T)a.U[tid];
    const bool active = !a.ep.active || __builtin_amdgcn_readfirstlane(a.ep.active[c.sector]) != 0;
    const bool has_p = LZ && a.ep.c2;
    const T c1 = LZ ? uniform_val((T)a.ep.c1[c.sector]) : (T)1;
    const T c2 = has_p ? uniform_val((T)a.ep.c2[c.sector]) : (T)0;
    const T tu = (T)a.bamp[0];
    constexpr int kWords = UT ? kRowsNB / 2 : kRowsNB;
    const uint32_t *slists = static_cast<const uint32_t *>(a.lists) + (size_t)c.loff * kWords;
    __syncthreads();
    double dot = 0.0;
    if (active) {
#pragma unroll
        for (int r = 0; r < kRowsMaxR; ++r) {
            const int rd = tid + r * kBlockLanes;
            if (rd >= (int)cdn) break;
            // the first kUpMax up-hop sources (past the hops: block 0 with
            // coefficient 0) are in flight during the down-hop work
            T g[kUpMax];
#pragma unroll
            for (int h = 0; h < kUpMax; ++h)
                g[h] = *reinterpret_cast<const T *>(xsb + (sob[h] + (uint32_t)rd * (uint32_t)sizeof(T)));
            // up-hops kUpMax .. kUpMax + 3 (a fifth of the chain's blocks have
            // them) are in flight with the first batch, where the registers
            // allow (fp64 with bond amplitudes would drop to seven waves a SIMD)
            constexpr bool kEarlyTail = UT || sizeof(T) == 4;
            const bool tail = nu > (uint32_t)kUpMax;
            T g2[4];
            if (kEarlyTail && tail) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t t = __builtin_amdgcn_readfirstlane(lt[kUpMax + q]);
                    g2[q] = *reinterpret_cast<const T *>(xsb + (t * cdn + (uint32_t)rd) * (uint32_t)sizeof(T));
                }
            }
            uint32_t hl[kWords];
            rows_load_list(slists + (size_t)rd * kWords, hl);
            const uint64_t row = c.base + (uint32_t)rd;
            const T pv = has_p ? p[row] : (T)0;
            const uint32_t adr = a.hs_states[c.hs_dn + rd];
            const T edr = (T)a.hs_energy[c.hs_dn + rd];
            const T acc = rows_down<T, UT, kWords, 8>(hl, smem, amp, true);
            const T xv = xp[rd];
            const T dg = eu + edr + rows_u_energy<T>(au & adr, a, ul);
            T v = fma_t(dg, xv, UT ? tu * acc : acc);
#pragma unroll
            for (int h = 0; h < kUpMax; ++h) v = fma_t(cf[h], g[h], v);
            // the rest in groups of four, in the order rows_up_tail sums them
            if (!kEarlyTail) {
                v = rows_up_tail<T, true>(xsec, lt, lc, cdn, (uint32_t)rd, nu, v);
            } else if (tail) {
#pragma unroll
                for (int q = 0; q < 4; ++q) v = fma_t(uniform_val(lc[kUpMax + q]), g2[q], v);
                if (nu > (uint32_t)kUpMax + 4) {
                    T g3[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const uint32_t t = __builtin_amdgcn_readfirstlane(lt[kUpMax + 4 + q]);
                        g3[q] = *reinterpret_cast<const T *>(xsb + (t * cdn + (uint32_t)rd) * (uint32_t)sizeof(T));
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) v = fma_t(uniform_val(lc[kUpMax + 4 + q]), g3[q], v);
                }
            }
            if constexpr (LZ) {
                const T uu = lz_out(v, c1, c2, pv, has_p);
                out[row] = uu;
                dot = __builtin_fma((double)xv, (double)uu, dot);
            } else {
                out[row] = v;
            }
        }
    }
    // the tile's partial of <x, u>: per wave, then wave 0 adds the 16 (the
    // rows kernel's order for a one-block tile)
    if (a.ep.partial) {
        double v = dot;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if ((tid & 63) == 0) red[tid >> 6] = v;
        __syncthreads();
        if (tid < 64) {
            double w = tid < kRowsWaves ? red[tid] : 0.0;
            for (int o = kRowsWaves / 2; o > 0; o >>= 1) w += __shfl_down(w, o, 64);
            if (tid == 0) a.ep.partial[c.slot] = active ? w : 0.0;
        }
    }
}

// ------------------------------------------------------------------------
// Flat kernel.  Every row is independent work for one lane: no staged x, no
// down-hop lists, no barrier between rows, so a CU holds as many waves as its
// registers allow and their gathers overlap.  A 256-lane workgroup takes one
// tile (a few alpha_up blocks of one sector, about kFlatRows rows); lane t
// handles rows t, t + 256, ... of the tile, splitting each into (alpha_up,
// alpha_dn) with the sector's reciprocal multiplier.  Both halves' hops are
// ranked on the LDS table (Fig. fastrank) for every bond, branch-free: a bond
// that does not hop gets coefficient 0 and the row's own x.  Down-hop
// sources lie in the row's own alpha_up block (3.7 KB in fp32 for the
// 12-site impurity model, L1/L2 resident), up-hop sources in the same
// alpha_dn column of other blocks (contiguous across lanes).  The terms are
// summed in the order of the rows kernel (down-hops in bond order, the
// diagonal, up-hops in bond order) with the same fused operations, so both
// give bitwise identical products.  Tiles are binned by XCD like the other
// kernels, so a sector's x is gathered through one L2.
// ------------------------------------------------------------------------
constexpr int kFlatBlock = 256;
constexpr uint32_t kFlatRows = 1024;  // rows per tile (whole alpha_up blocks; at least one)

template <class T, int NCH, bool LZ>
__global__ void __launch_bounds__(kFlatBlock) hv_flat_kernel(HvArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t *rt = reinterpret_cast<uint16_t *>(smem);
    double *red = reinterpret_cast<double *>(smem + ((a.rtab_entries * 2 + 15) & ~15u));
    for (uint32_t i = threadIdx.x; i < a.rtab_entries; i += blockDim.x) rt[i] = a.rtab[i];

    uint32_t ti;
    if (a.binned) {
        const uint32_t xcd = blockIdx.x % kXcd;
        ti = a.xoff[xcd] + blockIdx.x / kXcd;
        if (ti >= a.xoff[xcd + 1]) return;  // whole workgroup: no barrier is skipped by part of it
    } else {
        ti = blockIdx.x;
        if (ti >= a.n_tiles) return;
    }
    const T *x = static_cast<const T *>(a.x);
    T *out = static_cast<T *>(a.out);
    const T *p = static_cast<const T *>(a.ep.p);
    if (a.ep.basis_j) {
        const int64_t j = *a.ep.basis_j;
        x += (uint64_t)j * a.ep.basis_stride;
        p = j > 0 ? x - a.ep.basis_stride : x;
    }
    const HvTile tl = a.tiles[ti];
    const HvSector sc = a.secs[tl.sector];
    __syncthreads();  // rank table in LDS
    const bool active = !a.ep.active || a.ep.active[tl.sector];
    double dot = 0.0;
    if (active) {
        const uint32_t cdn = sc.cdn;
        const uint32_t rows = tl.nblk * cdn;
        const T *xs = x + sc.off;
        const uint64_t base = sc.off + (uint64_t)tl.rup0 * cdn;
        const int nb = a.nb;
        const bool has_p = LZ && a.ep.c2 != nullptr;
        const T c1 = LZ ? (T)a.ep.c1[tl.sector] : (T)1;
        const T c2 = has_p ? (T)a.ep.c2[tl.sector] : (T)0;
        const T tu = (T)a.bamp[0];
        for (uint32_t e = threadIdx.x; e < rows; e += blockDim.x) {
            uint32_t g = __umulhi(e, sc.magic);
            uint32_t rd = e - g * cdn;
            if (rd >= cdn) {
                rd -= cdn;
                ++g;
            }
            const uint32_t ru = tl.rup0 + g;
            const uint32_t au = a.hs_states[sc.hs_up + ru], ad = a.hs_states[sc.hs_dn + rd];
            const T eu = (T)a.hs_energy[sc.hs_up + ru], ed = (T)a.hs_energy[sc.hs_dn + rd];
            const uint64_t ubase = (uint64_t)ru * cdn;  // row of this alpha_up block, in the sector
            const T xv = xs[ubase + rd];
            T pv = 0;
            if constexpr (LZ) {
                if (has_p) pv = p[base + e];
            }
            T acc = 0;
#pragma unroll 4
            for (int b = 0; b < nb; ++b) {
                const uint32_t bi = a.bij[b] & 0xFF, bj = a.bij[b] >> 8;
                const bool hop = ((ad >> bi) ^ (ad >> bj)) & 1;
                uint32_t rr = rank_half<NCH>(ad ^ a.bmask[b], rt, a);
                rr = hop ? rr : rd;
                const T mag = a.t_uniform ? (T)1 : (T)a.bamp[b];
                T c = (__popc(ad & a.bbetw[b]) & 1) ? mag : -mag;
                c = hop ? c : (T)0;
                acc = fma_t(c, xs[ubase + rr], acc);
            }
            const T dg = eu + ed + u_energy<T>(au & ad, a);
            T v = fma_t(dg, xv, a.t_uniform ? tu * acc : acc);
#pragma unroll 4
            for (int b = 0; b < nb; ++b) {
                const uint32_t bi = a.bij[b] & 0xFF, bj = a.bij[b] >> 8;
                const bool hop = ((au >> bi) ^ (au >> bj)) & 1;
                uint32_t rr = rank_half<NCH>(au ^ a.bmask[b], rt, a);
                rr = hop ? rr : ru;
                T c = (__popc(au & a.bbetw[b]) & 1) ? (T)a.bamp[b] : -(T)a.bamp[b];
                c = hop ? c : (T)0;
                v = fma_t(c, xs[(uint64_t)rr * cdn + rd], v);
            }
            if constexpr (LZ) {
                const T uu = lz_out(v, c1, c2, pv, has_p);
                out[base + e] = uu;
                dot = __builtin_fma((double)xv, (double)uu, dot);
            } else {
                out[base + e] = v;
            }
        }
    }
    if (a.ep.partial) {
        double v = dot;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < kFlatBlock / 64; ++w) s += red[w];
            a.ep.partial[tl.slot] = active ? s : 0.0;
        }
    }
}

// Trie-ranked product (the plain trie method of Sec. IV inside H·x, which
// Sec. V.B compares with staggered lookup): the flat kernel's tiles and sums,
// but the row's pattern is read from the sector's list and every hop
// target's full 2L-bit pattern is ranked by a walk through the sector's
// packed trie, its top levels staged in LDS.  Every hop target of a spin
// sector is a member, so the walk's value is its rank (no membership read).
// Terms are summed in the order of the other kernels, so the products are
// bitwise equal to theirs.
template <class T, bool LZ>
__global__ void __launch_bounds__(kFlatBlock) hv_trie_kernel(HvArgs a, const HvTrieDesc *__restrict__ tries,
                                                             uint32_t lds_cap) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *top = reinterpret_cast<uint32_t *>(smem);
    double *red = reinterpret_cast<double *>(smem + (size_t)lds_cap * 4);
    uint32_t ti;
    if (a.binned) {
        const uint32_t xcd = blockIdx.x % kXcd;
        ti = a.xoff[xcd] + blockIdx.x / kXcd;
        if (ti >= a.xoff[xcd + 1]) return;
    } else {
        ti = blockIdx.x;
        if (ti >= a.n_tiles) return;
    }
    const HvTile tl = a.tiles[ti];
    const HvSector sc = a.secs[tl.sector];
    const HvTrieDesc td = tries[tl.sector];
    stage_to_lds(top, td.tab, (uint64_t)td.lds_entries * 4);
    const T *x = static_cast<const T *>(a.x);
    T *out = static_cast<T *>(a.out);
    const T *p = static_cast<const T *>(a.ep.p);
    if (a.ep.basis_j) {
        const int64_t j = *a.ep.basis_j;
        x += (uint64_t)j * a.ep.basis_stride;
        p = j > 0 ? x - a.ep.basis_stride : x;
    }
    __syncthreads();  // staged levels in LDS
    const bool active = !a.ep.active || a.ep.active[tl.sector];
    double dot = 0.0;
    if (active) {
        const int L = a.Lsites;
        const uint32_t lo_mask = (1u << L) - 1;
        const uint32_t cdn = sc.cdn;
        const uint32_t rows = tl.nblk * cdn;
        const T *xs = x + sc.off;
        const uint64_t base = sc.off + (uint64_t)tl.rup0 * cdn;
        const uint32_t lbase = tl.rup0 * cdn;  // first row of the tile within the sector
        const int nb = a.nb;
        const bool has_p = LZ && a.ep.c2 != nullptr;
        const T c1 = LZ ? (T)a.ep.c1[tl.sector] : (T)1;
        const T c2 = has_p ? (T)a.ep.c2[tl.sector] : (T)0;
        const T tu = (T)a.bamp[0];
        auto walk = [&](uint32_t alpha) {
            uint32_t node = 0;
            uint32_t l = 0;
            for (; l < td.lds_levels; ++l) node = top[td.off[l] + node + ((alpha >> td.shift[l]) & td.wmask[l])];
            for (; l < td.H; ++l) node = td.tab[td.off[l] + node + ((alpha >> td.shift[l]) & td.wmask[l])];
            return node;
        };
        for (uint32_t e = threadIdx.x; e < rows; e += blockDim.x) {
            uint32_t g = __umulhi(e, sc.magic);
            uint32_t rd = e - g * cdn;
            if (rd >= cdn) {
                rd -= cdn;
                ++g;
            }
            const uint32_t ru = tl.rup0 + g;
            const uint32_t own = lbase + e;
            const uint32_t alpha = td.states[own];
            const uint32_t ad = alpha & lo_mask, au = alpha >> L;
            const T eu = (T)a.hs_energy[sc.hs_up + ru], ed = (T)a.hs_energy[sc.hs_dn + rd];
            const T xv = xs[own];
            T pv = 0;
            if constexpr (LZ) {
                if (has_p) pv = p[base + e];
            }
            T acc = 0;
            for (int b = 0; b < nb; ++b) {
                const uint32_t bi = a.bij[b] & 0xFF, bj = a.bij[b] >> 8;
                const bool hop = ((ad >> bi) ^ (ad >> bj)) & 1;
                const uint32_t rr = hop ? walk(alpha ^ a.bmask[b]) : own;
                const T mag = a.t_uniform ? (T)1 : (T)a.bamp[b];
                T c = (__popc(ad & a.bbetw[b]) & 1) ? mag : -mag;
                c = hop ? c : (T)0;
                acc = fma_t(c, xs[rr], acc);
            }
            const T dg = eu + ed + u_energy<T>(au & ad, a);
            T v = fma_t(dg, xv, a.t_uniform ? tu * acc : acc);
            for (int b = 0; b < nb; ++b) {
                const uint32_t bi = a.bij[b] & 0xFF, bj = a.bij[b] >> 8;
                const bool hop = ((au >> bi) ^ (au >> bj)) & 1;
                const uint32_t rr = hop ? walk(alpha ^ (a.bmask[b] << L)) : own;
                T c = (__popc(au & a.bbetw[b]) & 1) ? (T)a.bamp[b] : -(T)a.bamp[b];
                c = hop ? c : (T)0;
                v = fma_t(c, xs[rr], v);
            }
            if constexpr (LZ) {
                const T uu = lz_out(v, c1, c2, pv, has_p);
                out[base + e] = uu;
                dot = __builtin_fma((double)xv, (double)uu, dot);
            } else {
                out[base + e] = v;
            }
        }
    }
    if (a.ep.partial) {
        double v = dot;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < kFlatBlock / 64; ++w) s += red[w];
            a.ep.partial[tl.slot] = active ? s : 0.0;
        }
    }
}

template <class T, bool LZ>
mbr_status launch_trie_hv(const mbr_hubbard *h, const HvArgs &a, unsigned grid, hipStream_t s) {
    const size_t lds = (size_t)h->trie_lds * 4 + 4 * sizeof(double);
    auto kern = hv_trie_kernel<T, LZ>;
    if (lds > 64 * 1024)
        MBR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    if (grid) kern<<<grid, kFlatBlock, lds, s>>>(a, h->d_trie.as<HvTrieDesc>(), h->trie_lds);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

template <class T, int NCH, bool LZ>
mbr_status launch_flat(const HvArgs &a, unsigned grid, hipStream_t s) {
    const size_t lds = ((a.rtab_entries * 2 + 15) & ~(size_t)15) + 4 * sizeof(double);
    auto kern = hv_flat_kernel<T, NCH, LZ>;
    if (lds > 64 * 1024)
        MBR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    if (grid) kern<<<grid, kFlatBlock, lds, s>>>(a);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

size_t lds_bytes_for(const mbr_hubbard *h, size_t tsz) {
    auto r16 = [](size_t v) { return (v + 15) & ~(size_t)15; };
    size_t o = r16(((size_t)h->tab.nrows << h->tab.k) * 2);
    o += r16((size_t)h->upcap * 4) + r16((size_t)h->upcap * tsz);
    o += 2 * r16((size_t)h->maxblk * 4) + r16((size_t)h->maxblk * tsz) + 16 * sizeof(double);
    return o + (size_t)h->xcap * tsz;
}

template <class T, int NCH, bool LZ>
mbr_status launch_g(const mbr_hubbard *h, const HvArgs &a, unsigned grid, size_t lds, hipStream_t s) {
    auto pick = [&]() {
        switch (h->G <= 0 ? 2 : h->G) {
            case 1: return hv_kernel<T, NCH, LZ, 1>;
            case 2: return hv_kernel<T, NCH, LZ, 2>;
            default: return hv_kernel<T, NCH, LZ, 4>;
        }
    };
    auto kern = pick();
    if (lds > 64 * 1024)
        MBR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    kern<<<grid, h->block, lds, s>>>(a);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

void fill_args(const mbr_hubbard *h, HvArgs &a, const void *x, void *out, const HvEpilogue &ep) {
    a.x = x;
    a.out = out;
    a.secs = h->d_secs.as<HvSector>();
    a.hs_states = h->d_hs_states.as<uint16_t>();
    a.hs_energy = h->d_hs_energy.as<double>();
    a.rtab = h->tab.table.as<uint16_t>();
    a.rtab_entries = (uint32_t)((uint64_t)h->tab.nrows << h->tab.k);
    a.nb = h->nb;
    a.Lsites = h->L;
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
    a.upcap = h->upcap;
    a.lists = h->d_lists.p;
    a.rgmax = h->rows_gmax;
    a.t_uniform = h->t_uniform ? 1 : 0;
    a.maxblk = h->maxblk;
    a.ep = ep;
}

// The rows kernel runs as many 1024-lane workgroups per CU as its registers
// and LDS allow, at most two: a CU then has a second sweep of tiles whose
// gathers are in flight while the first one waits (short spin-down blocks
// leave one tile's gathers too few to cover the latency).  cap: the number of
// tiles of a per-sector launch, 0 for a whole product.
template <class T, bool LZ, int R>
mbr_status launch_rows_r(const mbr_hubbard *h, const HvArgs &a, unsigned cap, hipStream_t s) {
    auto kern = h->t_uniform ? hv_rows_kernel<T, LZ, R, true> : hv_rows_kernel<T, LZ, R, false>;
    const size_t lds = rows_lds_layout(a.rtab_entries, a.xcap, a.rgmax, sizeof(T)).total;
    if (lds > 64 * 1024)
        MBR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kRowsBlock, lds) != hipSuccess) per_cu = 1;
    per_cu = std::max(1, std::min(per_cu, 2));
    unsigned grid = (unsigned)h->rows_grid * (unsigned)per_cu;
    if (cap) grid = std::min(grid, cap);
    kern<<<grid, kRowsBlock, lds, s>>>(a);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

template <class T, bool LZ>
mbr_status launch_rows(const mbr_hubbard *h, const HvArgs &a, unsigned cap, int R, hipStream_t s) {
    switch (R) {
        case 1: return launch_rows_r<T, LZ, 1>(h, a, cap, s);
        case 2: return launch_rows_r<T, LZ, 2>(h, a, cap, s);
        case 3: return launch_rows_r<T, LZ, 3>(h, a, cap, s);
        default: return launch_rows_r<T, LZ, 4>(h, a, cap, s);
    }
}

// Block kernel over `grid` workgroups (descriptors and ranges set in a).
template <class T, bool LZ>
mbr_status launch_block(const mbr_hubbard *h, HvArgs a, unsigned grid, hipStream_t s) {
    auto kern = h->t_uniform ? hv_block_kernel<T, LZ, true> : hv_block_kernel<T, LZ, false>;
    a.xcap = h->block_xcap;
    const size_t lds = block_lds_bytes(h->block_xcap, sizeof(T));
    if (lds > 64 * 1024)
        MBR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    BlockUpLists<T> up{h->d_up_tgt.as<uint32_t>(), h->d_up_coef.as<T>(), h->d_up_n.as<uint32_t>()};
    if (grid) kern<<<grid, kBlockLanes, lds, s>>>(a, up);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

template <class T, int NCH>
mbr_status launch_t(const mbr_hubbard *h, const void *x, void *out, const HvEpilogue &ep,
                    hipStream_t s) {
    HvArgs a{};
    fill_args(h, a, x, out, ep);
    if (ep.tiles) {
        // a tile subset of one sector (per-sector launches)
        a.tiles = ep.tiles;
        a.n_tiles = ep.n_tiles;
        a.binned = 0;
        if (ep.n_tiles == 0) return MBR_OK;
        if (h->rank_kind == MBR_HV_RANK_TRIE) {
            if (ep.c1) return launch_trie_hv<T, true>(h, a, ep.n_tiles, s);
            return launch_trie_hv<T, false>(h, a, ep.n_tiles, s);
        }
        if (!h->flat_tiles.empty()) {
            if (ep.c1) return launch_flat<T, NCH, true>(a, ep.n_tiles, s);
            return launch_flat<T, NCH, false>(a, ep.n_tiles, s);
        }
        if (h->hsec[ep.sector].blk) {
            a.rdesc = h->d_rdesc_slot.as<RowsTileDesc>() + h->hsec[ep.sector].slot0;
            if (ep.c1) return launch_block<T, true>(h, a, ep.n_tiles, s);
            return launch_block<T, false>(h, a, ep.n_tiles, s);
        }
        if (h->hsec[ep.sector].rows) {
            // the sector's tiles are the slot range starting at its first slot
            a.rdesc = h->d_rdesc_slot.as<RowsTileDesc>() + h->hsec[ep.sector].slot0;
            a.xcap = h->rows_xcap;
            if (ep.c1) return launch_rows<T, true>(h, a, ep.n_tiles, h->hsec[ep.sector].R, s);
            return launch_rows<T, false>(h, a, ep.n_tiles, h->hsec[ep.sector].R, s);
        }
        a.xcap = h->xcap;
        const size_t lds = lds_bytes_for(h, sizeof(T));
        const unsigned grid = (unsigned)std::min<uint64_t>(a.n_tiles, (uint64_t)h->grid);
        if (ep.c1) return launch_g<T, NCH, true>(h, a, grid, lds, s);
        return launch_g<T, NCH, false>(h, a, grid, lds, s);
    }
    if (!h->flat_tiles.empty()) {
        a.tiles = h->d_flat_tiles.as<HvTile>();
        a.n_tiles = (uint32_t)h->flat_tiles.size();
        a.binned = 1;
        uint32_t most = 0;
        for (int i = 0; i < kXcd; ++i) {
            a.xoff[i] = h->flat_xoff[i];
            most = std::max(most, h->flat_xoff[i + 1] - h->flat_xoff[i]);
        }
        a.xoff[kXcd] = h->flat_xoff[kXcd];
        const unsigned grid = most * kXcd;
        if (h->rank_kind == MBR_HV_RANK_TRIE) {
            if (ep.c1) return launch_trie_hv<T, true>(h, a, grid, s);
            return launch_trie_hv<T, false>(h, a, grid, s);
        }
        if (ep.c1) return launch_flat<T, NCH, true>(a, grid, s);
        return launch_flat<T, NCH, false>(a, grid, s);
    }
    if (!h->block_tiles.empty()) {
        HvArgs ab = a;
        ab.rdesc = h->d_bdesc.as<RowsTileDesc>();
        ab.n_tiles = (uint32_t)h->block_tiles.size();
        ab.binned = 1;
        uint32_t most = 0;
        for (int i = 0; i <= kXcd; ++i) ab.xoff[i] = h->block_xoff[i];
        for (int i = 0; i < kXcd; ++i) most = std::max(most, h->block_xoff[i + 1] - h->block_xoff[i]);
        const unsigned grid = most * kXcd;
        if (ep.c1) MBR_TRY((launch_block<T, true>(h, ab, grid, s)));
        else MBR_TRY((launch_block<T, false>(h, ab, grid, s)));
    }
    if (!h->rows_tiles.empty()) {
        HvArgs ar = a;
        ar.rdesc = h->d_rdesc.as<RowsTileDesc>();
        ar.n_tiles = (uint32_t)h->rows_tiles.size();
        ar.binned = 1;
        for (int i = 0; i <= kXcd; ++i) ar.xoff[i] = h->rows_xoff[i];
        ar.xcap = h->rows_xcap;
        if (ep.c1) MBR_TRY((launch_rows<T, true>(h, ar, 0, h->rows_R, s)));
        else MBR_TRY((launch_rows<T, false>(h, ar, 0, h->rows_R, s)));
    }
    if (!h->tiles_binned.empty()) {
        a.tiles = h->d_tiles.as<HvTile>();
        a.n_tiles = (uint32_t)h->tiles_binned.size();
        a.binned = 1;
        for (int i = 0; i <= kXcd; ++i) a.xoff[i] = h->xoff[i];
        a.xcap = h->xcap;
        const size_t lds = lds_bytes_for(h, sizeof(T));
        if (ep.c1) return launch_g<T, NCH, true>(h, a, (unsigned)h->grid, lds, s);
        return launch_g<T, NCH, false>(h, a, (unsigned)h->grid, lds, s);
    }
    return MBR_OK;
}

template <class T>
mbr_status launch_p(const mbr_hubbard *h, const void *x, void *out, const HvEpilogue &ep,
                    hipStream_t s) {
    switch (h->tab.nch) {
        case 1: return launch_t<T, 1>(h, x, out, ep, s);
        case 2: return launch_t<T, 2>(h, x, out, ep, s);
        case 3: return launch_t<T, 3>(h, x, out, ep, s);
        default: return launch_t<T, 0>(h, x, out, ep, s);
    }
}

// Split `tiles` (natural order) into n contiguous ranges of about equal cost.
std::vector<uint32_t> balanced_ranges(const std::vector<HvTile> &tiles, const std::vector<HvSector> &hsec,
                                      int n) {
    std::vector<double> cost(tiles.size());
    double tot = 0;
    for (size_t i = 0; i < tiles.size(); ++i) {
        cost[i] = (double)tiles[i].nblk * hsec[tiles[i].sector].cdn;
        tot += cost[i];
    }
    std::vector<uint32_t> r(n + 1, 0);
    double acc = 0;
    size_t i = 0;
    for (int b = 1; b < n; ++b) {
        const double target = tot * b / n;
        while (i < tiles.size() && acc + 0.5 * cost[i] < target) acc += cost[i++];
        r[b] = (uint32_t)i;
    }
    r[n] = (uint32_t)tiles.size();
    return r;
}

// Down-hop lists of the rows kernel, one set per n_dn it serves (lrows rows in
// all), ranked on the device with the launch shape's table.
mbr_status build_lists(mbr_hubbard *h, uint32_t lrows, hipStream_t s) {
    if (h->lists_ndn.empty()) return MBR_OK;
    const uint32_t tsz = h->precision == MBR_F64 ? 8 : 4;
    const uint32_t words = h->t_uniform ? kRowsNB / 2 : kRowsNB;
    MBR_TRY(h->d_lists.alloc((size_t)lrows * words * 4));
    HvArgs a{};
    fill_args(h, a, nullptr, nullptr, HvEpilogue{});
    const uint32_t rcs =
        (uint32_t)rows_lds_layout(a.rtab_entries, h->rows_xcap, h->rows_gmax, tsz).cs;
    const uint32_t bcs = (uint32_t)(((size_t)h->block_xcap * tsz + 15) & ~(size_t)15);
    uint32_t row0 = 0;
    for (size_t li = 0; li < h->lists_ndn.size(); ++li) {
        const uint32_t nd = h->lists_ndn[li];
        const uint32_t cs = h->lists_blk[li] ? bcs : rcs;
        const uint32_t cdn = (uint32_t)binom(h->L, (int)nd);
        uint32_t *lists = h->d_lists.as<uint32_t>() + (size_t)row0 * words;
        const unsigned grid = (cdn + 255) / 256;
        if (h->t_uniform)
            hv_lists_kernel<true><<<grid, 256, 0, s>>>(a, h->hs_off[nd], cdn, tsz, cs, lists);
        else
            hv_lists_kernel<false><<<grid, 256, 0, s>>>(a, h->hs_off[nd], cdn, tsz, cs, lists);
        MBR_HIP(hipGetLastError());
        row0 += cdn;
    }
    return MBR_OK;
}

// Up-hop lists of every half state for the block kernel.
mbr_status build_uplists(mbr_hubbard *h, hipStream_t s) {
    const uint32_t n_hs = h->hs_off[h->L + 1];
    const size_t tsz = h->precision == MBR_F64 ? 8 : 4;
    MBR_TRY(h->d_up_tgt.alloc((size_t)n_hs * kRowsNB * 4));
    MBR_TRY(h->d_up_coef.alloc((size_t)n_hs * kRowsNB * tsz));
    MBR_TRY(h->d_up_n.alloc((size_t)n_hs * 4));
    HvArgs a{};
    fill_args(h, a, nullptr, nullptr, HvEpilogue{});
    const unsigned grid = (n_hs + 255) / 256;
    if (tsz == 8)
        hv_uplists_kernel<double><<<grid, 256, 0, s>>>(a, n_hs, h->d_up_tgt.as<uint32_t>(), h->d_up_coef.as<double>(),
                                                       h->d_up_n.as<uint32_t>());
    else
        hv_uplists_kernel<float><<<grid, 256, 0, s>>>(a, n_hs, h->d_up_tgt.as<uint32_t>(), h->d_up_coef.as<float>(),
                                                      h->d_up_n.as<uint32_t>());
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

// Rebuild the rank table, tiles, work ranges and LDS budgets for (k, G, block).
// G = 0 selects the alpha_dn-stationary kernel for every sector it supports;
// G = -2 the same, but sectors with C_dn > 512 go to the block kernel.
mbr_status configure(mbr_hubbard *h, int k, int G, int block, hipStream_t s) {
    const int L = h->L;
    if (k < 1 || k > L || k > 16) MBR_FAIL(MBR_EINVAL, "k=%d outside 1..L", k);
    if (G < -2 || G > 4 || G == 3) MBR_FAIL(MBR_EINVAL, "G=%d not in {-2,-1,0,1,2,4}", G);
    const bool flat = G == -1;
    const bool rows_shape = G == 0 || G == -2;
    if (block != 256 && block != 512) MBR_FAIL(MBR_EINVAL, "block=%d not in {256,512}", block);
    StagTable tab;
    MBR_TRY(stag_build(tab, L, k, L, 2, s));
    if (tab.entry_bytes != 2) MBR_FAIL(MBR_EUNSUPPORTED, "half ranks beyond 16 bits");
    if ((((size_t)tab.nrows << k) * 2) > 64 * 1024)
        MBR_FAIL(MBR_EUNSUPPORTED, "k=%d: half table over 64 KiB", k);
    const size_t tsz = h->precision == MBR_F64 ? 8 : 4;
    const int Gt = rows_shape ? 2 : G;  // tile-kernel blocks for sectors the rows kernel does not take
    const size_t xbudget = (Gt == 4 ? 112 : 56) * 1024;
    std::vector<HvSector> hsec;
    std::vector<HvTile> tiles, rows_tiles, other_tiles, flat_tiles, block_tiles;
    uint64_t off = 0;
    uint32_t slot = 0, xcap = 0, upcap = 0, maxblk = 0, rows_xcap = 0, rows_gmax = 1, lrows = 0, block_xcap = 0;
    std::vector<uint32_t> lists_ndn, lists_rows;
    std::vector<uint8_t> lists_blk;
    int rows_R = 1;
    bool t_uniform = true;  // every bond has one amplitude (the rows kernel's uniform-hopping instances)
    for (auto &b : h->bonds) t_uniform = t_uniform && b.t == h->bonds[0].t;
    const uint32_t nbm = (uint32_t)std::max(1, h->nb);
    for (size_t si = 0; si < h->secs.size(); ++si) {
        HvSector sc{};
        sc.off = off;
        sc.cup = (uint32_t)binom(L, h->secs[si].n_up);
        sc.cdn = (uint32_t)binom(L, h->secs[si].n_dn);
        sc.hs_up = h->hs_off[h->secs[si].n_up];
        sc.hs_dn = h->hs_off[h->secs[si].n_dn];
        sc.rows = (rows_shape && sc.cdn + 1 <= kRowsMaxX && h->nb <= kRowsNB - 1) ? 1 : 0;
        // (the block kernel addresses a sector with 32-bit byte offsets)
        sc.blk = (G == -2 && sc.rows && sc.cdn > kBlockMin && (uint64_t)sc.cup * sc.cdn * tsz <= 0xFFFFFFFFull) ? 1 : 0;
        if (sc.blk) sc.rows = 0;
        sc.magic = sc.cdn == 1 ? 0xFFFFFFFFu : (uint32_t)((1ull << 32) / sc.cdn);
        uint32_t nblk;
        if (sc.blk) {
            sc.wide = 1;
            sc.x_lds = 1;
            sc.gp = 1;
            sc.R = (sc.cdn + kBlockLanes - 1) / kBlockLanes;
            nblk = 1;
        } else if (flat) {
            sc.wide = 0;
            sc.x_lds = 0;
            nblk = std::max<uint32_t>(1, kFlatRows / sc.cdn);
        } else if (sc.rows) {
            sc.wide = 1;
            sc.x_lds = 1;
            if (sc.cdn <= (uint32_t)kRowsBlock / 2) {
                // blocks across lanes
                sc.gp = std::min<uint32_t>(kRowsMaxG, kRowsBlock / sc.cdn);
                sc.R = 1;
                nblk = sc.gp;
            } else if (sc.cdn <= (uint32_t)kRowsBlock && tsz == 4) {
                // one block per row slot (gp = 0): rows_slots() blocks a tile
                // (fp32; in fp64 the extra slots would not fit the registers)
                sc.gp = 0;
                nblk = std::min<uint32_t>(rows_slots(t_uniform), kRowsMaxX / (sc.cdn + 1));
                sc.R = nblk;
            } else {
                // one block per tile, spread over ceil(C_dn / 1024) row slots
                sc.gp = 1;
                sc.R = (sc.cdn + kRowsBlock - 1) / kRowsBlock;
                nblk = 1;
            }
            rows_R = std::max(rows_R, (int)sc.R);
            rows_gmax = std::max(rows_gmax, std::max<uint32_t>(sc.gp, nblk));
        } else {
            sc.wide = sc.cdn >= kWideMin;
            if (sc.wide) {
                const uint32_t fit = (uint32_t)(xbudget / (sc.cdn * tsz));
                sc.x_lds = fit >= 1;
                nblk = sc.x_lds ? std::min<uint32_t>((uint32_t)Gt, fit) : 1;
            } else {
                sc.x_lds = 1;
                nblk = std::max<uint32_t>(1, (uint32_t)(4 * block) / sc.cdn);
                nblk = std::min<uint32_t>(nblk, 1024 / nbm);
                nblk = std::min<uint32_t>(nblk, 256);
            }
            nblk = std::max<uint32_t>(nblk, 1);
        }
        sc.slot0 = slot;
        for (uint32_t r = 0; r < sc.cup; r += nblk) {
            HvTile t{};
            t.sector = (uint32_t)si;
            t.rup0 = r;
            t.nblk = std::min(nblk, sc.cup - r);
            t.slot = slot++;
            if (sc.blk) {
                block_xcap = std::max(block_xcap, sc.cdn + 1);
                block_tiles.push_back(t);
            } else if (flat) {
                flat_tiles.push_back(t);
            } else if (sc.rows) {
                rows_xcap = std::max(rows_xcap, t.nblk * (sc.cdn + 1));
                rows_tiles.push_back(t);
            } else {
                if (sc.x_lds) xcap = std::max(xcap, t.nblk * sc.cdn);
                maxblk = std::max(maxblk, t.nblk);
                upcap = std::max(upcap, t.nblk * nbm);
                other_tiles.push_back(t);
            }
            tiles.push_back(t);
        }
        sc.nslots = slot - sc.slot0;
        if (sc.rows || sc.blk) {  // down-hop lists are shared by the sectors of one n_dn
            const uint32_t nd = (uint32_t)h->secs[si].n_dn;
            auto it = std::find(lists_ndn.begin(), lists_ndn.end(), nd);
            const size_t li = (size_t)(it - lists_ndn.begin());
            if (it == lists_ndn.end()) {
                // one n_dn is one C_dn, so its sectors all take the same kernel
                lists_ndn.push_back(nd);
                lists_rows.push_back(lrows);
                lists_blk.push_back(sc.blk ? 1 : 0);
                lrows += sc.cdn;
            }
            sc.loff = lists_rows[li];
        }
        hsec.push_back(sc);
        off += (uint64_t)sc.cup * sc.cdn;
    }
    // tile kernel: eight contiguous cost-balanced ranges, one per XCD
    const std::vector<uint32_t> xr = balanced_ranges(other_tiles, hsec, kXcd);
    // rows kernel: one workgroup per CU, the same XCD ranges
    int rows_grid = device_cu_count();
    rows_grid -= rows_grid % kXcd;
    if (rows_grid < kXcd) rows_grid = kXcd;
    const std::vector<uint32_t> rr = balanced_ranges(rows_tiles, hsec, kXcd);
    const std::vector<uint32_t> fr = balanced_ranges(flat_tiles, hsec, kXcd);
    const std::vector<uint32_t> br = balanced_ranges(block_tiles, hsec, kXcd);
    if (!block_tiles.empty() && block_lds_bytes(block_xcap, tsz) > kLdsMax)
        MBR_FAIL(MBR_EUNSUPPORTED, "block kernel needs %zu bytes of LDS", block_lds_bytes(block_xcap, tsz));
    const size_t rows_lds = rows_lds_layout((uint32_t)((uint64_t)tab.nrows << k), rows_xcap, rows_gmax, tsz).total;
    if (!rows_tiles.empty() && rows_lds > kLdsMax) MBR_FAIL(MBR_EUNSUPPORTED, "rows kernel needs %zu bytes of LDS", rows_lds);
    // commit
    h->tab = std::move(tab);
    h->k = k;
    h->G = G;
    h->block = block;
    h->hsec = hsec;
    h->total = off;
    h->n_slots = slot;
    h->tiles_by_slot = tiles;
    h->tiles_binned = other_tiles;
    h->rows_tiles = rows_tiles;
    h->flat_tiles = flat_tiles;
    for (int b = 0; b <= kXcd; ++b) h->flat_xoff[b] = fr[b];
    MBR_TRY(upload(h->d_flat_tiles, flat_tiles.data(), flat_tiles.size() * sizeof(HvTile), s));
    for (int b = 0; b <= kXcd; ++b) h->xoff[b] = xr[b];
    h->xcap = xcap;
    h->upcap = upcap;
    h->maxblk = maxblk;
    h->rows_xcap = rows_xcap;
    h->rows_R = rows_R;
    h->lists_ndn = lists_ndn;
    h->lists_blk = lists_blk;
    h->block_tiles = block_tiles;
    h->block_xcap = block_xcap;
    for (int b = 0; b <= kXcd; ++b) h->block_xoff[b] = br[b];
    h->rows_gmax = rows_gmax;
    h->rows_grid = rows_grid;
    h->t_uniform = t_uniform;
    MBR_TRY(upload(h->d_tiles, other_tiles.data(), other_tiles.size() * sizeof(HvTile), s));
    {
        auto mk = [&](const HvTile &t) {
            const HvSector &sc = hsec[t.sector];
            RowsTileDesc d{};
            d.base = sc.off + (uint64_t)t.rup0 * sc.cdn;
            d.soff = sc.off;
            d.w0 = sc.cdn | (sc.gp << 12) | (t.nblk << 20);
            d.w1 = (sc.hs_up + t.rup0) | (sc.hs_dn << 16);
            d.w2 = sc.loff | (t.sector << 16);
            d.slot = t.slot;
            return d;
        };
        for (const auto *tl : {&rows_tiles, &block_tiles})
            for (auto &t : *tl) {  // field widths of the packed descriptor
                const HvSector &sc = hsec[t.sector];
                if (sc.cdn > 0xFFF || sc.gp > 0xFF || t.nblk > 0xFFF || sc.hs_up + t.rup0 > 0xFFFF ||
                    sc.hs_dn > 0xFFFF || sc.loff > 0xFFFF || t.sector > 0xFFFF)
                    MBR_FAIL(MBR_EUNSUPPORTED, "rows-kernel tile descriptor out of range");
            }
        std::vector<RowsTileDesc> rd, rs, bd;
        for (auto &t : rows_tiles) rd.push_back(mk(t));
        for (auto &t : block_tiles) bd.push_back(mk(t));
        for (auto &t : tiles) rs.push_back(mk(t));
        MBR_TRY(upload(h->d_rdesc, rd.data(), rd.size() * sizeof(RowsTileDesc), s));
        MBR_TRY(upload(h->d_bdesc, bd.data(), bd.size() * sizeof(RowsTileDesc), s));
        MBR_TRY(upload(h->d_rdesc_slot, rs.data(), rs.size() * sizeof(RowsTileDesc), s));
    }
    for (int b = 0; b <= kXcd; ++b) h->rows_xoff[b] = rr[b];
    MBR_TRY(upload(h->d_secs, h->hsec.data(), h->hsec.size() * sizeof(HvSector), s));
    h->lds_bytes = std::max(other_tiles.empty() ? 0 : lds_bytes_for(h, tsz), rows_tiles.empty() ? 0 : rows_lds);
    if (!block_tiles.empty()) h->lds_bytes = std::max(h->lds_bytes, block_lds_bytes(block_xcap, tsz));
    if (!flat_tiles.empty())
        h->lds_bytes = std::max<size_t>(h->lds_bytes, ((((size_t)h->tab.nrows << h->tab.k) * 2 + 15) & ~(size_t)15) +
                                                          4 * sizeof(double));
    if (!other_tiles.empty() && lds_bytes_for(h, tsz) > kLdsMax)
        MBR_FAIL(MBR_EUNSUPPORTED, "tile needs %zu bytes of LDS", lds_bytes_for(h, tsz));
    const size_t tl = other_tiles.empty() ? 1 : lds_bytes_for(h, tsz);
    int per_cu = (int)std::min<size_t>(8, kLdsMax / tl);
    per_cu = std::min(per_cu, 2048 / block);
    if (per_cu < 1) per_cu = 1;
    h->grid = device_cu_count() * per_cu;
    h->grid -= h->grid % kXcd;
    if (h->grid < kXcd) h->grid = kXcd;
    MBR_TRY(build_lists(h, lrows, s));
    if (!block_tiles.empty()) MBR_TRY(build_uplists(h, s));
    h->generation++;
    return MBR_OK;
}

// Trie-ranked product: each sector's list (built once) and a packed trie of
// chunk width kt over it, replacing any earlier tries.
mbr_status build_hv_tries(mbr_hubbard *h, int kt, void *stream) {
    hipStream_t s = as_stream(stream);
    const int L = h->L;
    if (kt < 4 || kt > 16) MBR_FAIL(MBR_EINVAL, "trie chunk width k=%d outside 4..16", kt);
    if ((2 * L + kt - 1) / kt > 8) MBR_FAIL(MBR_EUNSUPPORTED, "trie of %d levels (at most 8)", (2 * L + kt - 1) / kt);
    const uint64_t lo = (1ull << L) - 1;
    if (h->tsecs.empty())
        for (auto &sc : h->secs) {
            const mbr_popc_cons cons[3] = {{(lo << L) | lo, sc.n_up + sc.n_dn, sc.n_up + sc.n_dn},
                                           {lo, sc.n_dn, sc.n_dn},
                                           {lo << L, sc.n_up, sc.n_up}};
            mbr_sector *sec = nullptr;
            MBR_TRY(mbr_sector_build(2 * L, 32, 3, cons, &sec, stream));
            h->tsecs.push_back(sec);
        }
    std::vector<mbr_ranker *> tries;
    auto drop = [&]() {
        for (auto *r : tries) mbr_ranker_destroy(r);
    };
    std::vector<HvTrieDesc> td;
    uint32_t lds = 0;
    for (mbr_sector *sec : h->tsecs) {
        mbr_ranker *tr = nullptr;
        mbr_status st = mbr_build_trie(sec, kt, &tr, stream);
        if (st != MBR_OK) {
            drop();
            return st;
        }
        tries.push_back(tr);
        const TrieLevels &t = *tr->trie;
        HvTrieDesc dd{};
        dd.tab = t.table.as<uint32_t>();
        dd.states = sec->states.as<uint32_t>();
        dd.H = (uint32_t)t.H;
        dd.lds_levels = (uint32_t)t.lds_levels;
        dd.lds_entries = (uint32_t)t.lds_entries;
        for (int l = 0; l < t.H; ++l) {
            dd.wmask[l] = (uint32_t)((1ull << t.w[l]) - 1);
            dd.shift[l] = t.shift[l];
            dd.off[l] = t.off[l];
        }
        dd.off[t.H] = t.off[t.H];
        lds = std::max(lds, dd.lds_entries);
        td.push_back(dd);
    }
    DevBuf d;
    mbr_status st = upload(d, td.data(), td.size() * sizeof(HvTrieDesc), s);
    if (st != MBR_OK) {
        drop();
        return st;
    }
    for (auto *r : h->ttries) mbr_ranker_destroy(r);
    h->ttries = std::move(tries);
    h->d_trie = std::move(d);
    h->trie_lds = (lds + 3) & ~3u;  // the partial sums after it stay 16-byte aligned
    h->trie_k = kt;
    return configure(h, (L + 1) / 2, -1, 512, s);
}

std::string tune_key(const mbr_hubbard *h) {
    hipDeviceProp_t p{};
    (void)hipGetDeviceProperties(&p, h->device);
    std::ostringstream os;
    os << p.gcnArchName << ";cu" << p.multiProcessorCount << ";L" << h->L << ";P" << h->precision << ";B";
    for (auto &b : h->bonds) os << b.i << "-" << b.j << ",";
    os << ";S";
    for (auto &s : h->secs) os << s.n_up << "." << s.n_dn << ",";
    std::string key = os.str();
    for (auto &c : key)
        if (c == ' ' || c == '\t' || c == '\n') c = '_';
    return key;
}

// Trie-ranked product: time the chunk widths that give two, three and four
// levels over the 2L-bit patterns (at least 4 bits, at most 16) and keep the
// fastest; same cache file and format as the launch-shape tuner, under the
// key with ";trie" appended (the k field holds the trie's width).
mbr_status autotune_trie_k(mbr_hubbard *h, int32_t reps, void *stream) {
    hipStream_t s = as_stream(stream);
    const int M = 2 * h->L;
    const std::string key = tune_key(h) + ";trie";
    const char *path = std::getenv("MBR_AUTOTUNE_CACHE");
    if (path && *path) {
        std::ifstream in(path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string k0;
            int kk = 0, gg = 0, bb = 0;
            double ms = 0;
            if (!(ls >> k0 >> kk >> gg >> bb >> ms) || k0 != key) continue;
            if (kk == h->trie_k || build_hv_tries(h, kk, stream) == MBR_OK) {
                h->tuned_ms = ms;
                return MBR_OK;
            }
        }
        clear_error();
    }
    std::vector<int> ks;
    for (int levels = 2; levels <= 4; ++levels) ks.push_back(std::min(16, std::max(4, (M + levels - 1) / levels)));
    std::sort(ks.begin(), ks.end());
    ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
    const size_t tsz = h->precision == MBR_F64 ? 8 : 4;
    DevBuf bx, by;
    MBR_TRY(bx.alloc(h->total * tsz));
    MBR_TRY(by.alloc(h->total * tsz));
    MBR_HIP(hipMemsetAsync(bx.p, 0, h->total * tsz, s));
    hipEvent_t e0, e1;
    MBR_HIP(hipEventCreate(&e0));
    MBR_HIP(hipEventCreate(&e1));
    int bk = h->trie_k;
    double best = 1e30;
    for (int k : ks) {
        if (k != h->trie_k && build_hv_tries(h, k, stream) != MBR_OK) continue;
        HvEpilogue ep{};
        if (hubbard_launch(h, bx.p, by.p, ep, s) != MBR_OK) continue;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps; ++r) (void)hubbard_launch(h, bx.p, by.p, ep, s);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms / reps < best) {
            best = ms / reps;
            bk = k;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    clear_error();
    if (bk != h->trie_k) MBR_TRY(build_hv_tries(h, bk, stream));
    h->tuned_ms = best < 1e30 ? best : 0.0;
    if (path && *path && best < 1e30) {
        std::ofstream outf(path, std::ios::app);
        if (outf) outf << key << " " << bk << " " << -1 << " " << 512 << " " << best << "\n";
    }
    return MBR_OK;
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
    if (d->rank_kind != MBR_HV_RANK_HALVES && d->rank_kind != MBR_HV_RANK_TRIE)
        MBR_FAIL(MBR_EINVAL, "rank_kind=%d", d->rank_kind);
    if (d->rank_kind == MBR_HV_RANK_TRIE && 2 * L > 32)
        MBR_FAIL(MBR_EUNSUPPORTED, "trie ranks need 2L <= 32 (L=%d)", L);
    if (d->rank_kind == MBR_HV_RANK_TRIE && d->k != 0 && d->k < 4)
        MBR_FAIL(MBR_EINVAL, "trie chunk width k=%d below 4", d->k);
    for (int b = 0; b < d->n_bonds; ++b) {
        const mbr_bond &bd = d->bonds[b];
        if (bd.i < 0 || bd.i >= L || bd.j < 0 || bd.j >= L || bd.i == bd.j)
            MBR_FAIL(MBR_EINVAL, "bond %d = (%d,%d)", b, bd.i, bd.j);
    }
    auto h = std::make_unique<mbr_hubbard>();
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
    h->rank_kind = d->rank_kind;
    if (h->rank_kind == MBR_HV_RANK_TRIE) {
        // each sector's ascending list of 2L-bit patterns and a packed trie on
        // it; chunk width k (0: four levels)
        MBR_TRY(build_hv_tries(h.get(), d->k > 0 ? d->k : std::max(4, (2 * L + 3) / 4), stream));
        *out = h.release();
        return MBR_OK;
    }
    // default launch shape: two lookups per half rank, two alpha_up blocks per tile
    const int k = d->k > 0 ? std::min(d->k, L) : (L + 1) / 2;
    mbr_status st = configure(h.get(), k, 0, 512, s);
    if (st != MBR_OK && d->k == 0) st = configure(h.get(), k, 1, 512, s);
    if (st != MBR_OK) return st;
    *out = h.release();
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

mbr_status mbr_hubbard_get_config(const mbr_hubbard *h, mbr_hubbard_cfg *cfg) {
    if (!h || !cfg) MBR_FAIL(MBR_EINVAL, "null argument");
    cfg->k = h->rank_kind == MBR_HV_RANK_TRIE ? h->trie_k : h->k;
    cfg->G = h->G;
    cfg->block = h->block;
    cfg->tiles = (int32_t)h->tiles_by_slot.size();
    cfg->lds_bytes = h->lds_bytes;
    cfg->tuned_ms = h->tuned_ms;
    return MBR_OK;
}

mbr_status mbr_hubbard_set_config(mbr_hubbard *h, int32_t k, int32_t G, int32_t block, void *stream) {
    if (!h) MBR_FAIL(MBR_EINVAL, "null handle");
    if (h->rank_kind == MBR_HV_RANK_TRIE) MBR_FAIL(MBR_EUNSUPPORTED, "a trie-ranked product has one launch shape");
    const int ok = h->k, oG = h->G, ob = h->block;
    mbr_status st = configure(h, k, G, block, as_stream(stream));
    if (st != MBR_OK) {
        std::string err = mbr_last_error();
        (void)configure(h, ok, oG, ob, as_stream(stream));
        set_error("%s", err.c_str());
    }
    return st;
}

mbr_status mbr_hubbard_autotune(mbr_hubbard *h, int32_t reps, void *stream) {
    if (!h) MBR_FAIL(MBR_EINVAL, "null handle");
    if (reps < 1 || reps > 1000) MBR_FAIL(MBR_EINVAL, "reps=%d", reps);
    if (h->rank_kind == MBR_HV_RANK_TRIE) return autotune_trie_k(h, reps, stream);
    hipStream_t s = as_stream(stream);
    const std::string key = tune_key(h);
    const char *path = std::getenv("MBR_AUTOTUNE_CACHE");
    if (path && *path) {
        std::ifstream in(path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string k0;
            int kk = 0, gg = 0, bb = 0;
            double ms = 0;
            if (!(ls >> k0 >> kk >> gg >> bb >> ms) || k0 != key) continue;
            if (configure(h, kk, gg, bb, s) == MBR_OK) {
                h->tuned_ms = ms;
                return MBR_OK;
            }
        }
    }
    const size_t tsz = h->precision == MBR_F64 ? 8 : 4;
    DevBuf bx, by;
    MBR_TRY(bx.alloc(h->total * tsz));
    MBR_TRY(by.alloc(h->total * tsz));
    MBR_HIP(hipMemsetAsync(bx.p, 0, h->total * tsz, s));
    hipEvent_t e0, e1;
    MBR_HIP(hipEventCreate(&e0));
    MBR_HIP(hipEventCreate(&e1));
    std::vector<int> ks = {(h->L + 1) / 2, h->L, (h->L + 2) / 3};
    std::sort(ks.begin(), ks.end());
    ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
    int bk = h->k, bG = h->G, bb = h->block;
    double best = 1e30;
    for (int k : ks)
        for (int G : {-2, -1, 0, 1, 2, 4})
            for (int block : {256, 512}) {
                if (G <= 0 && block != 512) continue;  // the rows, block and flat kernels have one block size each
                if (configure(h, k, G, block, s) != MBR_OK) continue;
                HvEpilogue ep{};
                if (hubbard_launch(h, bx.p, by.p, ep, s) != MBR_OK) continue;
                (void)hipEventRecord(e0, s);
                for (int r = 0; r < reps; ++r) (void)hubbard_launch(h, bx.p, by.p, ep, s);
                (void)hipEventRecord(e1, s);
                (void)hipEventSynchronize(e1);
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                const double per = ms / reps;
                if (per < best) {
                    best = per;
                    bk = k;
                    bG = G;
                    bb = block;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    clear_error();
    MBR_TRY(configure(h, bk, bG, bb, s));
    h->tuned_ms = best;
    if (path && *path) {
        std::ofstream outf(path, std::ios::app);
        if (outf) outf << key << " " << bk << " " << bG << " " << bb << " " << best << "\n";
    }
    return MBR_OK;
}

}  // extern "C"
