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

using namespace mbr;

namespace {
constexpr int kXcd = 8;
}

struct mbr_hubbard {
    int32_t L = 0, nb = 0, precision = MBR_F64;
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
    DevBuf d_rows_tiles;
    uint32_t rows_xoff[kXcd + 1] = {0};
    uint32_t rows_xcap = 0;
    int rows_R = 1, rows_grid = 0;
    bool t_uniform = true;              // all bonds share one amplitude
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
            T c = (__popc(ad & a.bbetw[b]) & 1) ? (T)a.bamp[b] : -(T)a.bamp[b];
            c = hop ? c : (T)0;
#pragma unroll
            for (int g = 0; g < G; ++g)
                if (g < nblk) acc[g] += c * xsrc[g * cdn + rr];
        }
        // 3. diagonal, up-hops, epilogue
#pragma unroll
        for (int g = 0; g < G; ++g) {
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
    for (uint32_t ti = t_begin; ti < t_end; ti += t_step) {
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
                T v = (up_e[g] + ed + u_energy<T>(au & ad, a)) * xv;
                for (int b = 0; b < nb; ++b) {
                    const uint32_t bi = a.bij[b] & 0xFF, bj = a.bij[b] >> 8;
                    if (((ad >> bi) ^ (ad >> bj)) & 1) {
                        const uint32_t rr = rank_half<NCH>(ad ^ a.bmask[b], rt, a);
                        const T c = (__popc(ad & a.bbetw[b]) & 1) ? (T)a.bamp[b] : -(T)a.bamp[b];
                        v += c * xs[g * cdn + rr];
                    }
                }
#pragma unroll
                for (int u = 0; u < kUpPre; ++u)
                    if (u < (int)n) v += up_coef[g * nb + u] * upv[u];
                for (uint32_t h = kUpPre; h < n; ++h)
                    v += up_coef[g * nb + h] * x[sc.off + (uint64_t)up_tgt[g * nb + h] * cdn + rd];
                if constexpr (LZ) {
                    T u = (T)a.ep.c1[tl.sector] * v;
                    if (a.ep.c2) u -= (T)a.ep.c2[tl.sector] * pv;
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

// ------------------------------------------------------------------------
// alpha_dn-stationary kernel.  A workgroup of kRowsBlock lanes sweeps a
// contiguous run of tiles of one sector (or a few small sectors).  Each lane
// owns fixed spin-down configurations (R of them, or one per (block, alpha_dn)
// pair when C_dn is small); their down-hop targets are ranked once per run
// (staggered lookup) and kept in registers as a compacted list in bond order,
// so every alpha_up block of the run reuses them: per row and hop only one LDS
// gather and one FMA remain.  The x rows of the next tile are loaded into
// registers while the current tile computes and then written to the other
// half of a double-buffered LDS tile; the next tile's up-hop targets are
// ranked by 16-lane groups (one lane per bond, ballot compaction in bond
// order).  Summation order per row is the same as in the tile kernel.
// ------------------------------------------------------------------------
// alpha_dn-stationary kernel.  Each lane owns fixed spin-down configurations
// of the sector (R of them, or one (block, alpha_dn) pair when C_dn is small)
// and ranks their down-hop targets once (staggered lookup); the targets stay
// in registers as a list in bond order, padded with a pointer to a zero in
// LDS, so every alpha_up block the workgroup visits reuses them: per row and
// hop one LDS gather and one FMA remain, with no branches.  Up-hop targets
// of a block are uniform: they are ranked once per tile (one lane per bond,
// ballot compaction in bond order) and read into scalar registers, so each
// up-hop gather is a scalar base plus the lane's offset.  The next tile's x
// rows are loaded into registers while the current tile computes and then
// stored to the other half of a double-buffered LDS tile.  Tiles are visited
// in the XCD-binned order of the tile kernel.  Per row the terms are summed in
// the same order as in the tile kernel, so both give identical results.
constexpr int kRowsBlock = 1024;
constexpr int kRowsNB = 16;    // bonds
constexpr int kRowsMaxG = 64;  // alpha_up blocks per tile when C_dn is small
constexpr int kRowsMaxR = 4;   // alpha_dn per lane, so C_dn <= 4096
constexpr int kUpMax = 8;      // up-hop gathers in flight per row (more run in a tail loop)

// LDS layout: rank table | amplitudes | reduction scratch | two buffers, each
// x rows (+ one zero) | up-hop targets | coefficients | alpha_up | energies |
// counts.  Buffer b starts at buf0 + b * bstride.
struct RowsLds {
    size_t rt, amp, red, buf0, bstride, xs, ut, uc, ua, ue, un, total;
};

__host__ __device__ inline RowsLds rows_lds_layout(uint32_t rtab_entries, uint32_t xcap, size_t tsz) {
    auto r16 = [](size_t v) { return (v + 15) & ~(size_t)15; };
    RowsLds L{};
    size_t o = 0;
    L.rt = o;
    o += r16((size_t)rtab_entries * 2);
    L.amp = o;
    o += r16(2 * kRowsNB * tsz);
    L.red = o;
    o += 32 * sizeof(double);
    L.buf0 = o;
    size_t b = 0;
    L.xs = b;
    b += r16((size_t)(xcap + 1) * tsz);
    L.ut = b;
    b += r16((size_t)kRowsMaxG * kRowsNB * 4);
    L.uc = b;
    b += r16((size_t)kRowsMaxG * kRowsNB * tsz);
    L.ua = b;
    b += r16(kRowsMaxG * 4);
    L.ue = b;
    b += r16(kRowsMaxG * tsz);
    L.un = b;
    b += r16(kRowsMaxG * 4);
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

template <class T>
__device__ __forceinline__ void rows_uplists(const HvArgs &a, const uint16_t *rt, const HvTile &tl,
                                             const HvSector &sc, unsigned char *bb, const RowsLds &LL) {
    uint32_t *ut = reinterpret_cast<uint32_t *>(bb + LL.ut);
    T *uc = reinterpret_cast<T *>(bb + LL.uc);
    uint32_t *ua = reinterpret_cast<uint32_t *>(bb + LL.ua);
    T *ue = reinterpret_cast<T *>(bb + LL.ue);
    uint32_t *un = reinterpret_cast<uint32_t *>(bb + LL.un);
    // lane t: block g = t / 16, bond b = t % 16 (16-lane groups stay inside a wave)
    const uint32_t t = threadIdx.x;
    const uint32_t g = t >> 4, b = t & 15;
    bool hop = false;
    uint32_t tgt = 0;
    T coef = 0;
    if (g < tl.nblk) {
        const uint32_t hi = sc.hs_up + tl.rup0 + g;
        const uint32_t au = a.hs_states[hi];
        if ((int)b < a.nb) {
            const uint32_t bi = a.bij[b] & 0xFF, bj = a.bij[b] >> 8;
            hop = ((au >> bi) ^ (au >> bj)) & 1;
            if (hop) {
                const uint32_t beta = au ^ a.bmask[b];
                uint32_t r = 0;
                int np = 0;
                const uint32_t cm = (1u << a.k) - 1;
                for (int c = 0; c < a.nch; ++c) {
                    const uint32_t ch = (beta >> (c * a.k)) & cm;
                    r += rt[((uint32_t)(a.rowoff[c] + np) << a.k) + ch];
                    np += __popc(ch);
                }
                tgt = r;
                coef = (__popc(au & a.bbetw[b]) & 1) ? (T)a.bamp[b] : -(T)a.bamp[b];
            }
        }
        if (b == 0) {
            ua[g] = au;
            ue[g] = (T)a.hs_energy[hi];
        }
    }
    const unsigned long long bal = __ballot(hop);
    const int lane = threadIdx.x & 63;
    const unsigned long long grp = 0xFFFFull << (lane & 48);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (hop) {
        const uint32_t pos = (uint32_t)__popcll(bal & grp & below);
        ut[g * kRowsNB + pos] = tgt;
        uc[g * kRowsNB + pos] = coef;
    }
    if (b == 0 && g < tl.nblk) un[g] = (uint32_t)__popcll(bal & grp);
}

template <class T, bool LZ, int R, bool UT>
__global__ void __launch_bounds__(kRowsBlock) hv_rows_kernel(HvArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const RowsLds LL = rows_lds_layout(a.rtab_entries, a.xcap, sizeof(T));
    uint16_t *rt = reinterpret_cast<uint16_t *>(smem + LL.rt);
    T *amp = reinterpret_cast<T *>(smem + LL.amp);
    double *red = reinterpret_cast<double *>(smem + LL.red);
    for (uint32_t i = threadIdx.x; i < a.rtab_entries; i += blockDim.x) rt[i] = a.rtab[i];
    if (threadIdx.x < 2 * (uint32_t)a.nb) {
        const int b = threadIdx.x >> 1;
        amp[threadIdx.x] = (threadIdx.x & 1) ? (T)a.bamp[b] : -(T)a.bamp[b];
    }
    if (threadIdx.x < 2) {  // the zero every non-hop entry points at
        T *xz = reinterpret_cast<T *>(smem + LL.buf0 + threadIdx.x * LL.bstride + LL.xs);
        xz[a.xcap] = (T)0;
    }

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
    constexpr int kPer = UT ? 2 : 1;  // entries per register
    constexpr int kWords = kRowsNB / kPer;
    uint32_t hl[R][kWords];
    uint32_t ad[R];
    T ed[R];
    int wmax = 0;
    uint32_t cur_sector = 0xFFFFFFFFu;

    __syncthreads();  // rank table, amplitudes and zeros in LDS
    {
        const HvTile tl = a.tiles[t_cur];
        const HvSector sc = a.secs[tl.sector];
        unsigned char *bb = smem + LL.buf0;
        T *xs = reinterpret_cast<T *>(bb + LL.xs);
        const uint64_t base = sc.off + (uint64_t)tl.rup0 * sc.cdn;
        const uint32_t rows = tl.nblk * sc.cdn;
        for (uint32_t e = threadIdx.x; e < rows; e += blockDim.x) xs[e] = x[base + e];
        rows_uplists<T>(a, rt, tl, sc, bb, LL);
    }
    __syncthreads();

    for (int buf = 0; t_cur < t_end; t_cur += t_step, buf ^= 1) {
        const HvTile tl = a.tiles[t_cur];
        const HvSector sc = a.secs[tl.sector];
        const uint32_t cdn = sc.cdn;
        const uint64_t base = sc.off + (uint64_t)tl.rup0 * cdn;
        unsigned char *bb = smem + LL.buf0 + (size_t)buf * LL.bstride;
        const T *xs = reinterpret_cast<const T *>(bb + LL.xs);
        const uint32_t *ut = reinterpret_cast<const uint32_t *>(bb + LL.ut);
        const T *uc = reinterpret_cast<const T *>(bb + LL.uc);
        const uint32_t *ua = reinterpret_cast<const uint32_t *>(bb + LL.ua);
        const T *ue = reinterpret_cast<const T *>(bb + LL.ue);
        const uint32_t *un = reinterpret_cast<const uint32_t *>(bb + LL.un);

        // new sector: this lane's alpha_dn and their down-hop targets
        if (tl.sector != cur_sector) {
            cur_sector = tl.sector;
            int mx = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                int g, rd;
                if (sc.gp > 1) {
                    g = tid / (int)cdn;
                    rd = tid - g * (int)cdn;
                } else {
                    g = 0;
                    rd = tid + r * kRowsBlock;
                }
                const bool ok = (r == 0 || sc.gp == 1) && rd < (int)cdn && g < (int)sc.gp;
                ad[r] = ok ? a.hs_states[sc.hs_dn + rd] : 0u;
                ed[r] = ok ? (T)a.hs_energy[sc.hs_dn + rd] : (T)0;
                // index of the LDS zero relative to this lane's block rows
                const uint32_t zero = ok ? a.xcap - (uint32_t)g * cdn : 0u;
                uint32_t cnt = 0;
#pragma unroll
                for (int u = 0; u < kWords; ++u) hl[r][u] = UT ? (zero | (zero << 16)) : zero;
#pragma unroll
                for (int b = 0; b < kRowsNB; ++b) {
                    const uint32_t bi = a.bij[b] & 0xFF, bj = a.bij[b] >> 8;
                    const bool hop = ok && b < a.nb && (((ad[r] >> bi) ^ (ad[r] >> bj)) & 1);
                    uint32_t e = 0;
                    if (hop) {
                        const uint32_t beta = ad[r] ^ a.bmask[b];
                        uint32_t rr = 0;
                        int np = 0;
                        const uint32_t cm = (1u << a.k) - 1;
                        for (int c = 0; c < a.nch; ++c) {
                            const uint32_t ch = (beta >> (c * a.k)) & cm;
                            rr += rt[((uint32_t)(a.rowoff[c] + np) << a.k) + ch];
                            np += __popc(ch);
                        }
                        const uint32_t sg = __popc(ad[r] & a.bbetw[b]) & 1;
                        e = UT ? (rr | (sg << 15)) : (rr | ((uint32_t)b << 16) | (sg << 21));
                    }
                    // append in bond order without indexing registers by a runtime value
#pragma unroll
                    for (int u = 0; u < kRowsNB; ++u) {
                        const int wd = u / kPer, sh = (u % kPer) * 16;
                        const uint32_t put = UT ? ((hl[r][wd] & ~(0xFFFFu << sh)) | (e << sh)) : e;
                        hl[r][wd] = (hop && cnt == (uint32_t)u) ? put : hl[r][wd];
                    }
                    cnt += hop ? 1u : 0u;
                }
                mx = (int)cnt > mx ? (int)cnt : mx;
            }
            for (int o = 32; o > 0; o >>= 1) {  // wave-uniform trip count of the hop loop
                const int v = __shfl_xor(mx, o, 64);
                mx = v > mx ? v : mx;
            }
            wmax = mx;
        }

        // prefetch the next tile's x rows into registers
        constexpr int kPre = 4;
        T pre[kPre];
        uint32_t nrows_next = 0;
        const uint32_t t_next = t_cur + t_step;
        const bool has_next = t_next < t_end;
        if (has_next) {
            const HvTile tn = a.tiles[t_next];
            const HvSector sn = a.secs[tn.sector];
            nrows_next = tn.nblk * sn.cdn;
            const uint64_t nbase = sn.off + (uint64_t)tn.rup0 * sn.cdn;
#pragma unroll
            for (int j = 0; j < kPre; ++j) {
                const uint32_t e = tid + j * kRowsBlock;
                pre[j] = e < nrows_next ? x[nbase + e] : (T)0;
            }
        }

        const bool active = !a.ep.active || a.ep.active[tl.sector];
        const T c1 = LZ ? (T)a.ep.c1[tl.sector] : (T)1;
        const T c2 = (LZ && a.ep.c2) ? (T)a.ep.c2[tl.sector] : (T)0;
        const T tu = (T)a.bamp[0];
        double dot = 0.0;
        if (active) {
            if (sc.gp == 1) {
                // one alpha_up block per tile: its data is uniform, hold it in scalars
                const uint32_t nu = __builtin_amdgcn_readfirstlane(un[0]);
                const uint32_t au = __builtin_amdgcn_readfirstlane(ua[0]);
                const T eu = uniform_val(ue[0]);
                const T *src[kUpMax];
                T cf[kUpMax];
#pragma unroll
                for (int h = 0; h < kUpMax; ++h) {
                    const uint32_t tg = h < (int)nu ? __builtin_amdgcn_readfirstlane(ut[h]) : 0u;
                    cf[h] = h < (int)nu ? uniform_val(uc[h]) : (T)0;
                    src[h] = x + sc.off + (uint64_t)tg * cdn;
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int rd = tid + r * kRowsBlock;
                    if (rd >= (int)cdn) continue;
                    const uint64_t row = base + rd;
                    T upv[kUpMax];
#pragma unroll
                    for (int h = 0; h < kUpMax; ++h) upv[h] = h < (int)nu ? src[h][rd] : (T)0;
                    T pv = 0;
                    if constexpr (LZ) {
                        if (a.ep.c2) pv = p[row];
                    }
                    T acc = 0;
#pragma unroll
                    for (int u = 0; u < kRowsNB; ++u) {
                        if (u < wmax) {
                            uint32_t idx;
                            T c;
                            if constexpr (UT) {
                                const uint32_t e = (hl[r][u / kPer] >> ((u % kPer) * 16)) & 0xFFFFu;
                                idx = e & 0x7FFFu;
                                c = (e >> 15) ? tu : -tu;
                            } else {
                                const uint32_t e = hl[r][u];
                                idx = e & 0xFFFFu;
                                c = amp[((e >> 16) & 31) * 2 + (e >> 21)];
                            }
                            acc += c * xs[idx];
                        }
                    }
                    const T xv = xs[rd];
                    T v = acc + (eu + ed[r] + u_energy<T>(au & ad[r], a)) * xv;
#pragma unroll
                    for (int h = 0; h < kUpMax; ++h)
                        if (h < (int)nu) v += cf[h] * upv[h];
                    for (uint32_t h = kUpMax; h < nu; ++h) {
                        const uint32_t tg = __builtin_amdgcn_readfirstlane(ut[h]);
                        v += uniform_val(uc[h]) * x[sc.off + (uint64_t)tg * cdn + rd];
                    }
                    if constexpr (LZ) {
                        T uu = c1 * v;
                        if (a.ep.c2) uu -= c2 * pv;
                        out[row] = uu;
                        dot += (double)xv * (double)uu;
                    } else {
                        out[row] = v;
                    }
                }
            } else {
                // several small blocks per tile: block data per lane from LDS
                const int g = tid / (int)cdn;
                if (g < (int)tl.nblk && g < (int)sc.gp) {
                    const int rd = tid - g * (int)cdn;
                    const uint64_t row = base + (uint64_t)g * cdn + rd;
                    const uint32_t nu = un[g];
                    T upv[kUpMax];
#pragma unroll
                    for (int h = 0; h < kUpMax; ++h)
                        upv[h] = h < (int)nu ? x[sc.off + (uint64_t)ut[g * kRowsNB + h] * cdn + rd] : (T)0;
                    T pv = 0;
                    if constexpr (LZ) {
                        if (a.ep.c2) pv = p[row];
                    }
                    const T *xr = xs + g * cdn;
                    T acc = 0;
#pragma unroll
                    for (int u = 0; u < kRowsNB; ++u) {
                        if (u < wmax) {
                            uint32_t idx;
                            T c;
                            if constexpr (UT) {
                                const uint32_t e = (hl[0][u / kPer] >> ((u % kPer) * 16)) & 0xFFFFu;
                                idx = e & 0x7FFFu;
                                c = (e >> 15) ? tu : -tu;
                            } else {
                                const uint32_t e = hl[0][u];
                                idx = e & 0xFFFFu;
                                c = amp[((e >> 16) & 31) * 2 + (e >> 21)];
                            }
                            acc += c * xr[idx];
                        }
                    }
                    const T xv = xr[rd];
                    T v = acc + (ue[g] + ed[0] + u_energy<T>(ua[g] & ad[0], a)) * xv;
#pragma unroll
                    for (int h = 0; h < kUpMax; ++h)
                        if (h < (int)nu) v += uc[g * kRowsNB + h] * upv[h];
                    for (uint32_t h = kUpMax; h < nu; ++h)
                        v += uc[g * kRowsNB + h] * x[sc.off + (uint64_t)ut[g * kRowsNB + h] * cdn + rd];
                    if constexpr (LZ) {
                        T uu = c1 * v;
                        if (a.ep.c2) uu -= c2 * pv;
                        out[row] = uu;
                        dot += (double)xv * (double)uu;
                    } else {
                        out[row] = v;
                    }
                }
            }
        }
        if (a.ep.partial) {
            const double s = block_sum(dot, red);
            if (threadIdx.x == 0) a.ep.partial[tl.slot] = active ? s : 0.0;
        }
        // the other buffer is free (its tile finished before the last barrier):
        // store the prefetched rows and rank the next tile's up-hop targets
        if (has_next) {
            unsigned char *nb2 = smem + LL.buf0 + (size_t)(buf ^ 1) * LL.bstride;
            T *xn = reinterpret_cast<T *>(nb2 + LL.xs);
#pragma unroll
            for (int j = 0; j < kPre; ++j) {
                const uint32_t e = tid + j * kRowsBlock;
                if (e < nrows_next) xn[e] = pre[j];
            }
            const HvTile tn = a.tiles[t_next];
            const HvSector sn = a.secs[tn.sector];
            rows_uplists<T>(a, rt, tn, sn, nb2, LL);
        }
        __syncthreads();
    }
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
        switch (h->G == 0 ? 2 : h->G) {
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
    a.maxblk = h->maxblk;
    a.ep = ep;
}

template <class T, bool LZ, int R>
mbr_status launch_rows_r(const mbr_hubbard *h, const HvArgs &a, unsigned grid, hipStream_t s) {
    auto kern = h->t_uniform ? hv_rows_kernel<T, LZ, R, true> : hv_rows_kernel<T, LZ, R, false>;
    const size_t lds = rows_lds_layout(a.rtab_entries, a.xcap, sizeof(T)).total;
    if (lds > 64 * 1024)
        MBR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    kern<<<grid, kRowsBlock, lds, s>>>(a);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

template <class T, bool LZ>
mbr_status launch_rows(const mbr_hubbard *h, const HvArgs &a, unsigned grid, int R, hipStream_t s) {
    switch (R) {
        case 1: return launch_rows_r<T, LZ, 1>(h, a, grid, s);
        case 2: return launch_rows_r<T, LZ, 2>(h, a, grid, s);
        case 3: return launch_rows_r<T, LZ, 3>(h, a, grid, s);
        default: return launch_rows_r<T, LZ, 4>(h, a, grid, s);
    }
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
        if (h->hsec[ep.sector].rows) {
            a.xcap = h->rows_xcap;
            const unsigned grid = (unsigned)std::min<uint64_t>(ep.n_tiles, (uint64_t)h->rows_grid);
            if (ep.c1) return launch_rows<T, true>(h, a, grid, h->hsec[ep.sector].R, s);
            return launch_rows<T, false>(h, a, grid, h->hsec[ep.sector].R, s);
        }
        a.xcap = h->xcap;
        const size_t lds = lds_bytes_for(h, sizeof(T));
        const unsigned grid = (unsigned)std::min<uint64_t>(a.n_tiles, (uint64_t)h->grid);
        if (ep.c1) return launch_g<T, NCH, true>(h, a, grid, lds, s);
        return launch_g<T, NCH, false>(h, a, grid, lds, s);
    }
    if (!h->rows_tiles.empty()) {
        HvArgs ar = a;
        ar.tiles = h->d_rows_tiles.as<HvTile>();
        ar.n_tiles = (uint32_t)h->rows_tiles.size();
        ar.binned = 1;
        for (int i = 0; i <= kXcd; ++i) ar.xoff[i] = h->rows_xoff[i];
        ar.xcap = h->rows_xcap;
        if (ep.c1) MBR_TRY((launch_rows<T, true>(h, ar, h->rows_grid, h->rows_R, s)));
        else MBR_TRY((launch_rows<T, false>(h, ar, h->rows_grid, h->rows_R, s)));
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

// Rebuild the rank table, tiles, work ranges and LDS budgets for (k, G, block).
// G = 0 selects the alpha_dn-stationary kernel for every sector it supports.
mbr_status configure(mbr_hubbard *h, int k, int G, int block, hipStream_t s) {
    const int L = h->L;
    if (k < 1 || k > L || k > 16) MBR_FAIL(MBR_EINVAL, "k=%d outside 1..L", k);
    if (G != 0 && G != 1 && G != 2 && G != 4) MBR_FAIL(MBR_EINVAL, "G=%d not in {0,1,2,4}", G);
    if (block != 256 && block != 512) MBR_FAIL(MBR_EINVAL, "block=%d not in {256,512}", block);
    StagTable tab;
    MBR_TRY(stag_build(tab, L, k, L, 2, s));
    if (tab.entry_bytes != 2) MBR_FAIL(MBR_EUNSUPPORTED, "half ranks beyond 16 bits");
    if ((((size_t)tab.nrows << k) * 2) > 64 * 1024)
        MBR_FAIL(MBR_EUNSUPPORTED, "k=%d: half table over 64 KiB", k);
    const size_t tsz = h->precision == MBR_F64 ? 8 : 4;
    const int Gt = G == 0 ? 2 : G;  // tile-kernel blocks for sectors the rows kernel does not take
    const size_t xbudget = (Gt == 4 ? 112 : 56) * 1024;
    std::vector<HvSector> hsec;
    std::vector<HvTile> tiles, rows_tiles, other_tiles;
    uint64_t off = 0;
    uint32_t slot = 0, xcap = 0, upcap = 0, maxblk = 0, rows_xcap = 0;
    int rows_R = 1;
    const uint32_t nbm = (uint32_t)std::max(1, h->nb);
    for (size_t si = 0; si < h->secs.size(); ++si) {
        HvSector sc{};
        sc.off = off;
        sc.cup = (uint32_t)binom(L, h->secs[si].n_up);
        sc.cdn = (uint32_t)binom(L, h->secs[si].n_dn);
        sc.hs_up = h->hs_off[h->secs[si].n_up];
        sc.hs_dn = h->hs_off[h->secs[si].n_dn];
        sc.rows = (G == 0 && sc.cdn <= (uint32_t)(kRowsMaxR * kRowsBlock) && h->nb <= kRowsNB) ? 1 : 0;
        uint32_t nblk;
        if (sc.rows) {
            sc.wide = 1;
            sc.x_lds = 1;
            sc.gp = sc.cdn <= (uint32_t)kRowsBlock / 2 ? std::min<uint32_t>(kRowsMaxG, kRowsBlock / sc.cdn) : 1;
            sc.R = sc.gp > 1 ? 1 : (sc.cdn + kRowsBlock - 1) / kRowsBlock;
            rows_R = std::max(rows_R, (int)sc.R);
            nblk = sc.gp;
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
            if (sc.rows) {
                rows_xcap = std::max(rows_xcap, t.nblk * sc.cdn);
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
    const size_t rows_lds = rows_lds_layout((uint32_t)((uint64_t)tab.nrows << k), rows_xcap, tsz).total;
    if (!rows_tiles.empty() && rows_lds > kLdsMax) MBR_FAIL(MBR_EUNSUPPORTED, "rows kernel needs %zu bytes of LDS", rows_lds);
    bool t_uniform = true;
    for (auto &b : h->bonds) t_uniform = t_uniform && b.t == h->bonds[0].t;
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
    for (int b = 0; b <= kXcd; ++b) h->xoff[b] = xr[b];
    h->xcap = xcap;
    h->upcap = upcap;
    h->maxblk = maxblk;
    h->rows_xcap = rows_xcap;
    h->rows_R = rows_R;
    h->rows_grid = rows_grid;
    h->t_uniform = t_uniform;
    MBR_TRY(upload(h->d_tiles, other_tiles.data(), other_tiles.size() * sizeof(HvTile), s));
    MBR_TRY(upload(h->d_rows_tiles, rows_tiles.data(), rows_tiles.size() * sizeof(HvTile), s));
    for (int b = 0; b <= kXcd; ++b) h->rows_xoff[b] = rr[b];
    MBR_TRY(upload(h->d_secs, h->hsec.data(), h->hsec.size() * sizeof(HvSector), s));
    h->lds_bytes = std::max(other_tiles.empty() ? 0 : lds_bytes_for(h, tsz), rows_tiles.empty() ? 0 : rows_lds);
    if (!other_tiles.empty() && lds_bytes_for(h, tsz) > kLdsMax)
        MBR_FAIL(MBR_EUNSUPPORTED, "tile needs %zu bytes of LDS", lds_bytes_for(h, tsz));
    const size_t tl = other_tiles.empty() ? 1 : lds_bytes_for(h, tsz);
    int per_cu = (int)std::min<size_t>(8, kLdsMax / tl);
    per_cu = std::min(per_cu, 2048 / block);
    if (per_cu < 1) per_cu = 1;
    h->grid = device_cu_count() * per_cu;
    h->grid -= h->grid % kXcd;
    if (h->grid < kXcd) h->grid = kXcd;
    h->generation++;
    return MBR_OK;
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
    cfg->k = h->k;
    cfg->G = h->G;
    cfg->block = h->block;
    cfg->tiles = (int32_t)h->tiles_by_slot.size();
    cfg->lds_bytes = h->lds_bytes;
    cfg->tuned_ms = h->tuned_ms;
    return MBR_OK;
}

mbr_status mbr_hubbard_set_config(mbr_hubbard *h, int32_t k, int32_t G, int32_t block, void *stream) {
    if (!h) MBR_FAIL(MBR_EINVAL, "null handle");
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
        for (int G : {0, 1, 2, 4})
            for (int block : {256, 512}) {
                if (G == 0 && block != 512) continue;  // the rows kernel has one block size
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
