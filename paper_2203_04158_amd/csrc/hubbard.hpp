// Internal interface of the on-the-fly Hubbard H·x, shared with the Lanczos driver.
#pragma once

#include "common.hpp"

namespace mbr {

constexpr int kMaxBonds = 48;
constexpr int kMaxSites = 16;

// One workgroup's share of the product: nblk consecutive alpha_up blocks of
// one sector (all C(L, n_dn) spin-down configurations of each).
struct HvTile {
    uint32_t sector;
    uint32_t rup0;   // first alpha_up rank of the tile
    uint32_t nblk;   // alpha_up blocks in the tile
    uint32_t slot;   // index of this tile's partial sum (tiles of a sector are contiguous)
};

struct HvSector {
    uint64_t off;     // first row in the concatenated vector
    uint32_t cup, cdn; // C(L, n_up), C(L, n_dn)
    uint32_t hs_up, hs_dn; // offsets of the n_up / n_dn half-state lists
    uint32_t slot0, nslots; // partial-sum slots of the sector
    uint32_t wide;    // lanes over alpha_dn with blocks in registers (1) or flattened rows (0)
    uint32_t x_lds;   // x blocks staged in LDS (1) or gathered from memory (0)
    uint32_t rows;    // handled by the alpha_dn-stationary kernel (1) or the tile kernel (0)
    uint32_t gp;      // rows kernel: alpha_up blocks per tile (lanes over (block, alpha_dn))
    uint32_t R;       // rows kernel: alpha_dn values per lane
    uint32_t loff;    // rows kernel: first down-hop list row of the sector's n_dn
    uint32_t magic;   // flat kernel: floor(2^32 / C_dn), to split a row index into (alpha_up, alpha_dn)
    uint32_t blk;     // handled by the block kernel (launch shape G = -2): one alpha_up block per workgroup
};

// Epilogue: y = H x (plain), or u = c1[s] (H x)_i - c2[s] p_i written to `out`
// (which may alias p) with the per-tile partial sum of x_i u_i.
struct HvEpilogue {
    const double *c1 = nullptr;  // per-sector scale of H x (null: 1)
    const double *c2 = nullptr;  // per-sector coefficient of p (null: no p term)
    const void *p = nullptr;
    double *partial = nullptr;   // per-slot sums of x_i * u_i (null: none)
    const int32_t *active = nullptr;  // per-sector flag; inactive sectors are skipped
    // Basis mode: x and p are vectors j and j-1 of a basis with the given
    // stride (elements), j read from *basis_j on the device (p = x when j = 0).
    const int32_t *basis_j = nullptr;
    uint64_t basis_stride = 0;
    // Tile subset (by slot order) of one sector instead of the whole product.
    const HvTile *tiles = nullptr;
    uint32_t n_tiles = 0;
    uint32_t sector = 0;
};

struct HubbardImpl;

// Enqueue one product over every sector: out = epilogue(H x).
mbr_status hubbard_launch(const mbr_hubbard *h, const void *x, void *out, const HvEpilogue &ep,
                          hipStream_t s);

// Tiles in slot order (sector-contiguous), for per-sector launches and the
// elementwise Lanczos kernels.
const std::vector<HvTile> &hubbard_tiles(const mbr_hubbard *h);
// Incremented whenever the launch shape (and so the tile list) changes.
uint32_t hubbard_generation(const mbr_hubbard *h);
int hubbard_precision(const mbr_hubbard *h);
int hubbard_n_sectors(const mbr_hubbard *h);
uint64_t hubbard_total(const mbr_hubbard *h);
const std::vector<HvSector> &hubbard_sectors(const mbr_hubbard *h);
uint32_t hubbard_n_slots(const mbr_hubbard *h);

}  // namespace mbr
