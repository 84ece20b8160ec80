// Lanczos ground-state search per (N_up, N_dn) sector on the on-the-fly H·x,
// and the lowest eigenvalue of the tridiagonal matrices by Sturm bisection.
//
// Recurrence per sector: u = H v_j - beta_{j-1} v_{j-1}; alpha_j = <v_j, u>;
// w = u - alpha_j v_j; [full classical Gram-Schmidt of w against v_1..v_j];
// beta_j = |w|; v_{j+1} = w / beta_j.  All dot products accumulate in fp64 with
// fixed-order reductions (per tile, then per sector), so runs are bitwise
// repeatable.  Scalars live on the device and every kernel reads its step
// index there, so a step is a fixed launch sequence that can be captured once
// into a hipGraph and replayed; the host never waits inside a step.
//
// Plain path (no reorthogonalisation): two vectors only.  The stored q_j are
// unnormalised (q_{j+1} = w) and v_j = s_j q_j with s_j = 1/beta_{j-1} is folded
// into the kernels, so a step costs one H·x pass (which also forms u in place
// over q_{j-1} and the <q_j, u> partials) and one update pass (w and |w|^2).
// Reorthogonalising path: v_1..v_m are kept in the Hamiltonian's precision
// (fp32 in the mixed form) for the Gram-Schmidt passes; coefficients are fp64.
#include <algorithm>
#include <cmath>
#include <memory>
#include <type_traits>

#include "hubbard.hpp"

using namespace mbr;

namespace {

constexpr unsigned kBlock = 256;
constexpr int kRedWaves = kBlock / 64;

struct LzDev {
    double *alpha;   // [ns][m]
    double *beta;    // [ns][m]
    double *c1, *c2, *c3;  // per-sector step scalars
    double *pd;      // per-slot dot partials
    double *pn;      // per-slot norm partials
    double *pc;      // per-slot Gram-Schmidt partials [slot][m+1]
    double *cgs;     // per-sector Gram-Schmidt coefficients [ns][m+1]
    double *norm0;   // per-sector start norms
    int32_t *active; // per-sector flag
    int32_t *steps;  // per-sector completed steps
    int32_t *j;      // basis index of the current vector (reorthogonalising path)
};

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Fixed-order block sum; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
    return s;
}

// Sum of n partials of one sector by one workgroup, fixed order (lane t adds
// p[t], p[t + B], ... in turn; eight loads are issued before they are added).
__device__ __forceinline__ double sector_sum(const double *p, uint32_t n, double *red) {
    double v = 0;
    uint32_t i = threadIdx.x;
    for (; i + 7 * blockDim.x < n; i += 8 * blockDim.x) {
        double t[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) t[q] = p[i + q * blockDim.x];
#pragma unroll
        for (int q = 0; q < 8; ++q) v += t[q];
    }
    for (; i < n; i += blockDim.x) v += p[i];
    return block_sum(v, red);
}

// alpha_j = c1 * sum(pd); c3 = alpha_j * c1 (coefficient of the stored q_j in w).
__global__ void lz_alpha(const HvSector *secs, LzDev d, int m, uint32_t s_first) {
    __shared__ double red[kRedWaves];
    const uint32_t s = s_first + blockIdx.x;
    if (!d.active[s]) return;
    double sum = sector_sum(d.pd + secs[s].slot0, secs[s].nslots, red);
    if (threadIdx.x == 0) {
        double a = d.c1[s] * sum;
        d.alpha[(size_t)s * m + d.steps[s]] = a;
        d.c3[s] = a * d.c1[s];
    }
}

// beta_j = sqrt(sum(pn)); the sector stops at breakdown, at its dimension or at
// m steps; otherwise the scalars of the next step are prepared.
__global__ void lz_beta(const HvSector *secs, LzDev d, int m, double tol, int reorth,
                        uint32_t s_first) {
    __shared__ double red[kRedWaves];
    const uint32_t s = s_first + blockIdx.x;
    if (!d.active[s]) return;
    double sum = sector_sum(d.pn + secs[s].slot0, secs[s].nslots, red);
    if (threadIdx.x == 0) {
        const int j = d.steps[s];
        const double b = sqrt(sum);
        const double a = d.alpha[(size_t)s * m + j];
        const double bprev = j > 0 ? d.beta[(size_t)s * m + j - 1] : 0.0;
        const uint64_t dim = (uint64_t)secs[s].cup * secs[s].cdn;
        const bool stop = (b <= tol * (fabs(a) + bprev)) || (uint64_t)(j + 1) >= dim || j + 1 >= m;
        d.beta[(size_t)s * m + j] = stop ? 0.0 : b;
        d.steps[s] = j + 1;
        if (stop) {
            d.active[s] = 0;
        } else if (reorth) {
            d.c1[s] = 1.0;
            d.c2[s] = b;
            d.c3[s] = 1.0 / b;
        } else {
            d.c2[s] = b * d.c1[s];
            d.c1[s] = 1.0 / b;
        }
    }
}

// w = u - c q over elements [base, base + rows) of u (in place), returning
// this lane's share of |w|^2.  The bulk goes in 16-byte packs, four per lane
// in flight; the unaligned head and the tail element by element.  Both update
// kernels use it, so their partials agree bit for bit.
template <class T>
__device__ __forceinline__ double tile_axpy_norm(T *__restrict__ u, const T *__restrict__ q, T c, uint64_t base,
                                                 uint32_t rows) {
    constexpr uint32_t V = 16 / sizeof(T);
    using P = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
    double acc = 0;
    uint32_t head = (uint32_t)((V - base % V) % V);
    if (head > rows) head = rows;
    for (uint32_t e = threadIdx.x; e < head; e += blockDim.x) {
        const T w = u[base + e] - c * q[base + e];
        u[base + e] = w;
        acc += (double)w * (double)w;
    }
    const uint32_t np = (rows - head) / V;
    P *up = reinterpret_cast<P *>(u + base + head);
    const P *qp = reinterpret_cast<const P *>(q + base + head);
    constexpr int kU = 4;
    uint32_t pk = threadIdx.x;
    for (; pk + (kU - 1) * blockDim.x < np; pk += kU * blockDim.x) {
        P a[kU], b[kU];
#pragma unroll
        for (int i = 0; i < kU; ++i) {
            a[i] = up[pk + i * blockDim.x];
            b[i] = qp[pk + i * blockDim.x];
        }
#pragma unroll
        for (int i = 0; i < kU; ++i) {
            T *av = reinterpret_cast<T *>(&a[i]);
            const T *bv = reinterpret_cast<const T *>(&b[i]);
#pragma unroll
            for (uint32_t v = 0; v < V; ++v) {
                av[v] = av[v] - c * bv[v];
                acc += (double)av[v] * (double)av[v];
            }
            up[pk + i * blockDim.x] = a[i];
        }
    }
    for (; pk < np; pk += blockDim.x) {
        P a = up[pk];
        const P b = qp[pk];
        T *av = reinterpret_cast<T *>(&a);
        const T *bv = reinterpret_cast<const T *>(&b);
#pragma unroll
        for (uint32_t v = 0; v < V; ++v) {
            av[v] = av[v] - c * bv[v];
            acc += (double)av[v] * (double)av[v];
        }
        up[pk] = a;
    }
    for (uint32_t e = head + np * V + threadIdx.x; e < rows; e += blockDim.x) {
        const T w = u[base + e] - c * q[base + e];
        u[base + e] = w;
        acc += (double)w * (double)w;
    }
    return acc;
}

// w = u - c3 q over a tile's rows (in place in u); partial |w|^2.
template <class T>
__global__ void __launch_bounds__(kBlock) lz_update(const HvTile *tiles, uint32_t n_tiles,
                                                    const HvSector *secs, T *__restrict__ u,
                                                    const T *__restrict__ q, LzDev d) {
    __shared__ double red[kRedWaves];
    for (uint32_t ti = blockIdx.x; ti < n_tiles; ti += gridDim.x) {
        const HvTile tl = tiles[ti];
        const HvSector sc = secs[tl.sector];
        if (!d.active[tl.sector]) {
            if (threadIdx.x == 0) d.pn[tl.slot] = 0.0;
            continue;
        }
        const T c = (T)d.c3[tl.sector];
        const uint64_t base = sc.off + (uint64_t)tl.rup0 * sc.cdn;
        const uint32_t rows = tl.nblk * sc.cdn;
        const double acc = tile_axpy_norm(u, q, c, base, rows);
        double s = block_sum(acc, red);
        if (threadIdx.x == 0) d.pn[tl.slot] = s;
    }
}

// One sector per launch: lz_alpha folded into lz_update.  Every workgroup
// forms alpha_j from the sector's partials itself (the same sum in the same
// order as lz_alpha, so the same bits), workgroup 0 records it, and the
// update w = u - c3 q follows without a separate launch.
template <class T>
__global__ void __launch_bounds__(kBlock) lz_alpha_update(const HvTile *tiles, uint32_t n_tiles,
                                                          const HvSector *secs, T *__restrict__ u,
                                                          const T *__restrict__ q, LzDev d, int m,
                                                          uint32_t s) {
    __shared__ double red[kRedWaves];
    __shared__ double c3s;
    if (!d.active[s]) {
        for (uint32_t ti = blockIdx.x; ti < n_tiles; ti += gridDim.x)
            if (threadIdx.x == 0) d.pn[tiles[ti].slot] = 0.0;
        return;
    }
    const double sum = sector_sum(d.pd + secs[s].slot0, secs[s].nslots, red);
    if (threadIdx.x == 0) {
        const double a = d.c1[s] * sum;
        c3s = a * d.c1[s];
        if (blockIdx.x == 0) {
            d.alpha[(size_t)s * m + d.steps[s]] = a;
            d.c3[s] = c3s;
        }
    }
    __syncthreads();
    const T c = (T)c3s;
    for (uint32_t ti = blockIdx.x; ti < n_tiles; ti += gridDim.x) {
        const HvTile tl = tiles[ti];
        const HvSector sc = secs[tl.sector];
        const uint64_t base = sc.off + (uint64_t)tl.rup0 * sc.cdn;
        const uint32_t rows = tl.nblk * sc.cdn;
        const double acc = tile_axpy_norm(u, q, c, base, rows);
        double bs = block_sum(acc, red);
        if (threadIdx.x == 0) d.pn[tl.slot] = bs;
    }
}

// Per-slot |v|^2 of a vector (start normalisation).
template <class T>
__global__ void __launch_bounds__(kBlock) lz_norm_parts(const HvTile *tiles, uint32_t n_tiles,
                                                        const HvSector *secs, const T *__restrict__ v,
                                                        double *parts) {
    __shared__ double red[kRedWaves];
    for (uint32_t ti = blockIdx.x; ti < n_tiles; ti += gridDim.x) {
        const HvTile tl = tiles[ti];
        const HvSector sc = secs[tl.sector];
        const uint64_t base = sc.off + (uint64_t)tl.rup0 * sc.cdn;
        const uint32_t rows = tl.nblk * sc.cdn;
        double acc = 0;
        for (uint32_t e = threadIdx.x; e < rows; e += blockDim.x) {
            double w = (double)v[base + e];
            acc += w * w;
        }
        double s = block_sum(acc, red);
        if (threadIdx.x == 0) parts[tl.slot] = s;
    }
}

__global__ void lz_start_scalars(const HvSector *secs, LzDev d, int reorth) {
    __shared__ double red[kRedWaves];
    const uint32_t s = blockIdx.x;
    double sum = sector_sum(d.pn + secs[s].slot0, secs[s].nslots, red);
    if (threadIdx.x == 0) {
        double nrm = sqrt(sum);
        d.norm0[s] = nrm;
        d.active[s] = nrm > 0.0 ? 1 : 0;
        d.steps[s] = 0;
        d.c1[s] = reorth ? 1.0 : (nrm > 0 ? 1.0 / nrm : 0.0);
        d.c2[s] = 0.0;
        d.c3[s] = nrm > 0 ? 1.0 / nrm : 0.0;
        if (s == 0) *d.j = 0;
    }
}

template <class T>
__global__ void lz_convert(const double *__restrict__ v0, T *__restrict__ out, uint64_t n) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = (T)v0[i];
}

template <class T>
__global__ void lz_fill_zero(T *__restrict__ out, uint64_t n) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += stride) out[i] = (T)0;
}

// The reorthogonalising kernels move the rows of a tile (or merged group) as
// 16-byte packs: the vectors share one stride that is a multiple of 64 rows,
// so a row index decides the alignment of every vector alike.  A span is the
// unaligned head, the run of whole packs and the tail; its leftover rows (at
// most 2 (n - 1) for n elements per pack) go one to a thread.
template <class T>
struct alignas(16) Pack {
    static constexpr int n = 16 / sizeof(T);
    T e[n];
};

template <class T>
__device__ __forceinline__ Pack<T> ld_pack(const T *p) {
    return *reinterpret_cast<const Pack<T> *>(p);
}

template <class T>
__device__ __forceinline__ void st_pack(T *p, const Pack<T> &v) {
    *reinterpret_cast<Pack<T> *>(p) = v;
}

template <class T>
struct Span {
    uint64_t a0;    // first row of the first whole pack
    uint32_t nv;    // whole packs
    uint32_t head;  // rows before a0
    uint32_t left;  // head + tail rows
    uint64_t base;  // first row
    __device__ Span(uint64_t b, uint32_t rows) : base(b) {
        constexpr uint32_t n = Pack<T>::n;
        head = (uint32_t)((n - b % n) % n);
        if (head > rows) head = rows;
        a0 = b + head;
        nv = (rows - head) / n;
        left = rows - nv * n;
    }
    // row of leftover t (t < left): head rows first, then the tail
    __device__ uint64_t leftover(uint32_t t) const {
        return t < head ? base + t : a0 + (uint64_t)nv * Pack<T>::n + (t - head);
    }
};

// dst = c3 * w per sector.  With use_j the destination is basis vector j+1
// (v_{j+1} = w / beta_j, only sectors still running); otherwise vector 0.
template <class T>
__global__ void __launch_bounds__(kBlock) lz_scale_into(const HvTile *tiles, uint32_t n_tiles,
                                                        const HvSector *secs, const T *__restrict__ w,
                                                        T *__restrict__ V, uint64_t ld, LzDev d,
                                                        int use_j) {
    const int64_t j = use_j ? (int64_t)(*d.j) + 1 : 0;
    T *dst = V + (uint64_t)j * ld;
    for (uint32_t ti = blockIdx.x; ti < n_tiles; ti += gridDim.x) {
        const HvTile tl = tiles[ti];
        if (use_j && !d.active[tl.sector]) continue;
        const HvSector sc = secs[tl.sector];
        const T c = (T)d.c3[tl.sector];
        const Span<T> sp(sc.off + (uint64_t)tl.rup0 * sc.cdn, tl.nblk * sc.cdn);
        if (threadIdx.x < sp.left) {
            const uint64_t r = sp.leftover(threadIdx.x);
            dst[r] = w[r] * c;
        }
        for (uint32_t i = threadIdx.x; i < sp.nv; i += blockDim.x) {
            const uint64_t r = sp.a0 + (uint64_t)i * Pack<T>::n;
            Pack<T> v = ld_pack(w + r);
#pragma unroll
            for (int e = 0; e < Pack<T>::n; ++e) v.e[e] *= c;
            st_pack(dst + r, v);
        }
    }
}

// Reorthogonalising path: w = u - c3 v_j in place, then per-slot partials of
// <v_k, w> for k = 0..j (classical Gram-Schmidt coefficients).  The basis
// vectors are taken kKc at a time: one pass over the tile's rows loads a pack
// of each of them together (a short last chunk repeats its last vector, whose
// sums are then dropped) and one block reduction serves all kKc sums.  Each
// sum is fixed-order: per lane (its leftover row, then its packs in order,
// element by element), then across the wave, then over the waves in order.
constexpr int kKc = 8;
constexpr uint64_t kGroupRows = 4096;  // rows per merged group of the Gram-Schmidt kernels

template <class T>
__global__ void __launch_bounds__(kBlock) lz_update_dots(const HvTile *tiles, uint32_t n_tiles,
                                                         const HvSector *secs, T *__restrict__ W,
                                                         const T *__restrict__ V, uint64_t ld,
                                                         int m, LzDev d) {
    constexpr int n = Pack<T>::n;
    __shared__ double red[kKc][kRedWaves];
    const int j = *d.j;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (uint32_t ti = blockIdx.x; ti < n_tiles; ti += gridDim.x) {
        const HvTile tl = tiles[ti];
        if (!d.active[tl.sector]) continue;
        double *pc = d.pc + (size_t)tl.slot * (m + 1);
        const HvSector sc = secs[tl.sector];
        const Span<T> sp(sc.off + (uint64_t)tl.rup0 * sc.cdn, tl.nblk * sc.cdn);
        const T c = (T)d.c3[tl.sector];
        const T *vj = V + (uint64_t)j * ld;
        const bool has_left = threadIdx.x < sp.left;
        const uint64_t rl = has_left ? sp.leftover(threadIdx.x) : 0;
        if (has_left) W[rl] = W[rl] - c * vj[rl];
        for (uint32_t i = threadIdx.x; i < sp.nv; i += blockDim.x) {
            const uint64_t r = sp.a0 + (uint64_t)i * n;
            Pack<T> x = ld_pack(W + r);
            const Pack<T> y = ld_pack(vj + r);
#pragma unroll
            for (int e = 0; e < n; ++e) x.e[e] = x.e[e] - c * y.e[e];
            st_pack(W + r, x);
        }
        __syncthreads();
        for (int k0 = 0; k0 <= j; k0 += kKc) {
            const int nk = (j + 1 - k0) < kKc ? (j + 1 - k0) : kKc;
            const T *vk[kKc];
#pragma unroll
            for (int q = 0; q < kKc; ++q) vk[q] = V + (uint64_t)(k0 + (q < nk ? q : nk - 1)) * ld;
            double acc[kKc];
#pragma unroll
            for (int q = 0; q < kKc; ++q) acc[q] = 0.0;
            if (has_left) {
                const double x = (double)W[rl];
#pragma unroll
                for (int q = 0; q < kKc; ++q) acc[q] += (double)vk[q][rl] * x;
            }
            for (uint32_t i = threadIdx.x; i < sp.nv; i += blockDim.x) {
                const uint64_t r = sp.a0 + (uint64_t)i * n;
                const Pack<T> x = ld_pack(W + r);
                Pack<T> v[kKc];
#pragma unroll
                for (int q = 0; q < kKc; ++q) v[q] = ld_pack(vk[q] + r);
#pragma unroll
                for (int q = 0; q < kKc; ++q)
#pragma unroll
                    for (int e = 0; e < n; ++e) acc[q] += (double)v[q].e[e] * (double)x.e[e];
            }
#pragma unroll
            for (int q = 0; q < kKc; ++q) acc[q] = wave_sum(acc[q]);
            __syncthreads();  // the previous chunk's readers of red are done
            if (lane == 0)
#pragma unroll
                for (int q = 0; q < kKc; ++q) red[q][wv] = acc[q];
            __syncthreads();
            if ((int)threadIdx.x < nk) {
                double sum = 0;
                for (int w2 = 0; w2 < (int)(blockDim.x >> 6); ++w2) sum += red[threadIdx.x][w2];
                pc[k0 + threadIdx.x] = sum;
            }
        }
    }
}

// Per-sector Gram-Schmidt coefficients.  Lanes take consecutive k (so the
// slot rows are read coalesced) and the 16 waves split the slots: wave v adds
// slots v, v + 16, ... (eight loads in flight), then thread k of wave 0 adds the
// wave sums in wave order.  The order is fixed for a given slot count.
constexpr unsigned kCgsBlock = 1024;

__global__ void __launch_bounds__(kCgsBlock) lz_reduce_cgs(const HvSector *secs, LzDev d, int m,
                                                           uint32_t s_first) {
    constexpr int nw = kCgsBlock / 64;
    __shared__ double part[nw][64];
    const uint32_t s = s_first + blockIdx.x;
    if (!d.active[s]) return;
    const int j = *d.j;
    const HvSector sc = secs[s];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const size_t ldp = (size_t)m + 1;
    const double *p = d.pc + (size_t)sc.slot0 * ldp;
    for (int k0 = 0; k0 <= j; k0 += 64) {
        const int k = k0 + lane;
        double v = 0;
        if (k <= j) {
            uint32_t i = wv;
            for (; i + 7 * nw < sc.nslots; i += 8 * nw) {
                double t[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) t[q] = p[(size_t)(i + q * nw) * ldp + k];
#pragma unroll
                for (int q = 0; q < 8; ++q) v += t[q];
            }
            for (; i < sc.nslots; i += nw) v += p[(size_t)i * ldp + k];
        }
        part[wv][lane] = v;
        __syncthreads();
        if (wv == 0 && k <= j) {
            double sum = 0;
            for (int w2 = 0; w2 < nw; ++w2) sum += part[w2][lane];
            d.cgs[(size_t)s * ldp + k] = sum;
        }
        __syncthreads();
    }
}

// w -= sum_k c_k v_k (fp64 accumulation, k in order), then partial |w|^2.  The
// block stages c_0..c_j in LDS followed by kKc - 1 zeros, so every chunk of kKc
// basis vectors is whole: a vector past j is read at index j and subtracted
// with coefficient 0, which leaves w unchanged.  Dynamic LDS: (m + kKc) doubles.
template <class T>
__global__ void __launch_bounds__(kBlock) lz_subtract(const HvTile *tiles, uint32_t n_tiles,
                                                      const HvSector *secs, T *__restrict__ W,
                                                      const T *__restrict__ V, uint64_t ld, int m,
                                                      LzDev d) {
    constexpr int n = Pack<T>::n;
    __shared__ double red[kRedWaves];
    extern __shared__ double cs[];
    const int j = *d.j;
    const int kend = j + 1 + kKc - 1;  // staged coefficients (c_0..c_j, then zeros)
    for (uint32_t ti = blockIdx.x; ti < n_tiles; ti += gridDim.x) {
        const HvTile tl = tiles[ti];
        if (!d.active[tl.sector]) {
            if (threadIdx.x == 0) d.pn[tl.slot] = 0.0;
            continue;
        }
        const HvSector sc = secs[tl.sector];
        const Span<T> sp(sc.off + (uint64_t)tl.rup0 * sc.cdn, tl.nblk * sc.cdn);
        const double *c = d.cgs + (size_t)tl.sector * (m + 1);
        __syncthreads();  // the previous tile's readers of cs are done
        for (int k = threadIdx.x; k < kend; k += blockDim.x) cs[k] = k <= j ? c[k] : 0.0;
        __syncthreads();
        double acc = 0;
        if (threadIdx.x < sp.left) {
            const uint64_t r = sp.leftover(threadIdx.x);
            double w = (double)W[r];
            for (int k = 0; k <= j; ++k) w -= cs[k] * (double)V[(uint64_t)k * ld + r];
            const T wt = (T)w;
            W[r] = wt;
            acc += (double)wt * (double)wt;
        }
        for (uint32_t i = threadIdx.x; i < sp.nv; i += blockDim.x) {
            const uint64_t r = sp.a0 + (uint64_t)i * n;
            const Pack<T> x = ld_pack(W + r);
            double w[n];
#pragma unroll
            for (int e = 0; e < n; ++e) w[e] = (double)x.e[e];
            for (int k0 = 0; k0 <= j; k0 += kKc) {
                Pack<T> v[kKc];
#pragma unroll
                for (int q = 0; q < kKc; ++q) {
                    const int k = k0 + q <= j ? k0 + q : j;
                    v[q] = ld_pack(V + (uint64_t)k * ld + r);
                }
#pragma unroll
                for (int q = 0; q < kKc; ++q)
#pragma unroll
                    for (int e = 0; e < n; ++e) w[e] -= cs[k0 + q] * (double)v[q].e[e];
            }
            Pack<T> o;
#pragma unroll
            for (int e = 0; e < n; ++e) {
                o.e[e] = (T)w[e];
                acc += (double)o.e[e] * (double)o.e[e];
            }
            st_pack(W + r, o);
        }
        const double s = block_sum(acc, red);
        if (threadIdx.x == 0) d.pn[tl.slot] = s;
    }
}

__global__ void lz_advance(LzDev d, int m) {
    if (*d.j < m) *d.j += 1;
}

// ---------------------------------------------------------------- tridiagonal
// Number of eigenvalues below x: negative pivots of the LDL^T factorisation of
// T - x I (Sturm sequence).
__device__ __forceinline__ int sturm_count(const double *a, const double *b, int n, double x) {
    int c = 0;
    double q = a[0] - x;
    if (q < 0) ++c;
    for (int i = 1; i < n; ++i) {
        const double qq = (q == 0.0) ? -1e-300 : q;
        q = (a[i] - x) - b[i - 1] * b[i - 1] / qq;
        if (q < 0) ++c;
    }
    return c;
}

// One wave per matrix: 64-way multisection of the Gershgorin interval, keeping
// the sub-interval where the Sturm count first reaches one.
__global__ void tridiag_lowest_kernel(const double *alpha, const double *beta, const int32_t *len,
                                      int ld, int nb, double *e0) {
    const int bi = blockIdx.x;
    if (bi >= nb) return;
    const int lane = threadIdx.x;
    int n = len[bi];
    if (n > ld) n = ld;
    const double *a = alpha + (size_t)bi * ld;
    const double *b = beta + (size_t)bi * ld;
    if (n <= 0) {
        if (lane == 0) e0[bi] = 0.0;
        return;
    }
    double lo = a[0], hi = a[0];
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < n ? fabs(b[i]) : 0.0);
        lo = fmin(lo, a[i] - r);
        hi = fmax(hi, a[i] + r);
    }
    const double pad = 1e-12 * fmax(1.0, fmax(fabs(lo), fabs(hi)));
    lo -= pad;
    hi += pad;
    for (int it = 0; it < 40; ++it) {
        if (!(hi - lo > 4.5e-16 * fmax(fabs(lo), fabs(hi)) + 1e-300)) break;
        const double h = (hi - lo) / 65.0;
        const double x = lo + h * (double)(lane + 1);
        const int c = sturm_count(a, b, n, x);
        const unsigned long long ball = __ballot(c >= 1);
        const int first = ball ? (__ffsll((long long)ball) - 1) : 64;
        const double nlo = lo + h * (double)first;
        const double nhi = (first == 64) ? hi : lo + h * (double)(first + 1);
        lo = nlo;
        hi = nhi;
    }
    if (lane == 0) e0[bi] = 0.5 * (lo + hi);
}

}  // namespace

// ---------------------------------------------------------------- handle
struct mbr_lanczos {
    const mbr_hubbard *h = nullptr;
    mbr_lanczos_opts o{};
    int ns = 0, m = 0, prec = MBR_F64;
    size_t tsz = 8;
    uint64_t total = 0;
    uint64_t ld = 0;  // stride of the stored basis vectors (total rounded up to 64 rows)
    uint32_t n_slots = 0;
    std::vector<HvSector> secs;
    DevBuf d_tiles_slot, d_secs;
    // reorthogonalising path: consecutive tiles of a sector merged into groups
    // of at least kGroupRows rows, with their own slot numbering (rsecs holds
    // the sectors with slot0/nslots over those slots); rt0/rnt per sector
    DevBuf d_rtiles, d_rsecs;
    std::vector<uint32_t> rt0, rnt;
    uint32_t n_rtiles = 0;
    DevBuf bufA, bufB, basis, work;
    DevBuf alpha, beta, c1, c2, c3, pd, pn, pc, cgs, norm0, active, steps, jcount, e0;
    LzDev dev{};
    int parity = 0;  // plain path: 0 -> q_j in A, 1 -> q_j in B
    bool started = false;
    uint32_t generation = 0;  // Hamiltonian launch shape the tiles were taken from
    unsigned grid = 0;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    hipStream_t cap_stream = nullptr;
    ~mbr_lanczos() {
        for (auto &g : graph)
            if (g) (void)hipGraphExecDestroy(g);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

namespace {

double default_tol(const mbr_lanczos *lz) {
    if (lz->o.breakdown_tol > 0) return lz->o.breakdown_tol;
    return lz->prec == MBR_F64 ? 1e-12 : 1e-6;
}

// Kernels of one step for sectors [s0, s0 + nsec) whose tiles are the slot
// range [t0, t0 + nt).
template <class T>
mbr_status enqueue_plain(mbr_lanczos *lz, int par, uint32_t s0, uint32_t nsec, uint32_t t0,
                         uint32_t nt, bool all, hipStream_t s) {
    T *X = par ? lz->bufB.as<T>() : lz->bufA.as<T>();
    T *P = par ? lz->bufA.as<T>() : lz->bufB.as<T>();
    const HvSector *secs = lz->d_secs.as<HvSector>();
    const HvTile *tiles = lz->d_tiles_slot.as<HvTile>() + t0;
    HvEpilogue ep{};
    ep.c1 = lz->dev.c1;
    ep.c2 = lz->dev.c2;
    ep.p = P;
    ep.partial = lz->dev.pd;
    ep.active = lz->dev.active;
    if (!all) {
        ep.tiles = tiles;
        ep.n_tiles = nt;
        ep.sector = s0;
    }
    MBR_TRY(hubbard_launch(lz->h, X, P, ep, s));
    const unsigned g = std::min<unsigned>(lz->grid, nt);
    if (nsec == 1) {
        lz_alpha_update<T><<<g, kBlock, 0, s>>>(tiles, nt, secs, P, X, lz->dev, lz->m, s0);
    } else {
        lz_alpha<<<nsec, kBlock, 0, s>>>(secs, lz->dev, lz->m, s0);
        lz_update<T><<<g, kBlock, 0, s>>>(tiles, nt, secs, P, X, lz->dev);
    }
    lz_beta<<<nsec, kBlock, 0, s>>>(secs, lz->dev, lz->m, default_tol(lz), 0, s0);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

template <class T>
mbr_status enqueue_reorth(mbr_lanczos *lz, uint32_t s0, uint32_t nsec, uint32_t t0, uint32_t nt,
                          bool all, hipStream_t s) {
    T *V = lz->basis.as<T>();
    T *W = lz->work.as<T>();
    const HvSector *secs = lz->d_secs.as<HvSector>();
    const HvTile *tiles = lz->d_tiles_slot.as<HvTile>() + t0;
    HvEpilogue ep{};
    ep.c1 = lz->dev.c1;
    ep.c2 = lz->dev.c2;
    ep.p = V;
    ep.partial = lz->dev.pd;
    ep.active = lz->dev.active;
    ep.basis_j = lz->dev.j;
    ep.basis_stride = lz->ld;
    if (!all) {
        ep.tiles = tiles;
        ep.n_tiles = nt;
        ep.sector = s0;
    }
    MBR_TRY(hubbard_launch(lz->h, V, W, ep, s));
    // the Gram-Schmidt kernels run over the merged groups of these sectors
    const uint32_t g0 = all ? 0 : lz->rt0[s0], gn = all ? lz->n_rtiles : lz->rnt[s0];
    const HvTile *groups = lz->d_rtiles.as<HvTile>() + g0;
    const HvSector *rsecs = lz->d_rsecs.as<HvSector>();
    // batched: one workgroup per group, so the dispatcher balances groups of
    // unequal size; per sector: the tile grid of the other kernels
    const unsigned g = all ? std::max<unsigned>(1, std::min<unsigned>(gn, 1u << 20))
                           : std::min<unsigned>(lz->grid, gn);
    lz_alpha<<<nsec, kBlock, 0, s>>>(secs, lz->dev, lz->m, s0);
    lz_update_dots<T><<<g, kBlock, 0, s>>>(groups, gn, rsecs, W, V, lz->ld, lz->m, lz->dev);
    lz_reduce_cgs<<<nsec, kCgsBlock, 0, s>>>(rsecs, lz->dev, lz->m, s0);
    lz_subtract<T><<<g, kBlock, (size_t)(lz->m + kKc) * sizeof(double), s>>>(groups, gn, rsecs, W, V, lz->ld,
                                                                           lz->m, lz->dev);
    lz_beta<<<nsec, kBlock, 0, s>>>(rsecs, lz->dev, lz->m, default_tol(lz), 1, s0);
    lz_scale_into<T><<<g, kBlock, 0, s>>>(groups, gn, rsecs, W, V, lz->ld, lz->dev, 1);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

// One full step (all sectors), batched or one launch set per sector.
template <class T>
mbr_status enqueue_step(mbr_lanczos *lz, int par, hipStream_t s) {
    const bool reorth = lz->o.reorth != 0;
    if (lz->o.batched) {
        if (reorth) MBR_TRY(enqueue_reorth<T>(lz, 0, lz->ns, 0, lz->n_slots, true, s));
        else MBR_TRY(enqueue_plain<T>(lz, par, 0, lz->ns, 0, lz->n_slots, true, s));
    } else {
        for (int si = 0; si < lz->ns; ++si) {
            const HvSector &sc = lz->secs[si];
            if (reorth) MBR_TRY(enqueue_reorth<T>(lz, si, 1, sc.slot0, sc.nslots, false, s));
            else MBR_TRY(enqueue_plain<T>(lz, par, si, 1, sc.slot0, sc.nslots, false, s));
        }
    }
    if (reorth) {
        lz_advance<<<1, 1, 0, s>>>(lz->dev, lz->m);
        MBR_HIP(hipGetLastError());
    }
    return MBR_OK;
}

mbr_status step_any(mbr_lanczos *lz, int par, hipStream_t s) {
    return lz->prec == MBR_F64 ? enqueue_step<double>(lz, par, s) : enqueue_step<float>(lz, par, s);
}

mbr_status capture(mbr_lanczos *lz, int par) {
    if (!lz->cap_stream) MBR_HIP(hipStreamCreateWithFlags(&lz->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    MBR_HIP(hipStreamBeginCapture(lz->cap_stream, hipStreamCaptureModeThreadLocal));
    mbr_status st = step_any(lz, par, lz->cap_stream);
    hipError_t e = hipStreamEndCapture(lz->cap_stream, &g);
    if (st != MBR_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) MBR_FAIL(MBR_EHIP, "graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&lz->graph[par], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) MBR_FAIL(MBR_EHIP, "graph instantiate: %s", hipGetErrorString(e));
    return MBR_OK;
}

template <class T>
mbr_status lz_start_t(mbr_lanczos *lz, const double *v0, hipStream_t s) {
    const HvSector *secs = lz->d_secs.as<HvSector>();
    const HvTile *tiles = lz->d_tiles_slot.as<HvTile>();
    const unsigned eg = (unsigned)std::min<uint64_t>((lz->total + kBlock - 1) / kBlock, 8192);
    const bool reorth = lz->o.reorth != 0;
    T *X = reorth ? lz->work.as<T>() : lz->bufA.as<T>();
    lz_convert<T><<<eg, kBlock, 0, s>>>(v0, X, lz->total);
    if (!reorth) lz_fill_zero<T><<<eg, kBlock, 0, s>>>(lz->bufB.as<T>(), lz->total);
    lz_norm_parts<T><<<lz->grid, kBlock, 0, s>>>(tiles, lz->n_slots, secs, X, lz->dev.pn);
    lz_start_scalars<<<lz->ns, kBlock, 0, s>>>(secs, lz->dev, reorth ? 1 : 0);
    if (reorth)
        lz_scale_into<T><<<lz->grid, kBlock, 0, s>>>(tiles, lz->n_slots, secs, X, lz->basis.as<T>(),
                                                      lz->ld, lz->dev, 0);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

}  // namespace

extern "C" {

mbr_status mbr_lanczos_create(const mbr_hubbard *h, const mbr_lanczos_opts *o, mbr_lanczos **out) {
    if (!out) MBR_FAIL(MBR_EINVAL, "null output handle");
    *out = nullptr;
    if (!h || !o) MBR_FAIL(MBR_EINVAL, "null Hamiltonian or options");
    if (o->max_steps < 1 || o->max_steps > 4096) MBR_FAIL(MBR_EINVAL, "max_steps=%d outside 1..4096", o->max_steps);
    if (o->breakdown_tol < 0) MBR_FAIL(MBR_EINVAL, "negative breakdown tolerance");
    auto lz = std::make_unique<mbr_lanczos>();
    lz->h = h;
    lz->o = *o;
    lz->ns = hubbard_n_sectors(h);
    lz->m = o->max_steps;
    lz->prec = hubbard_precision(h);
    lz->tsz = lz->prec == MBR_F64 ? 8 : 4;
    lz->total = hubbard_total(h);
    lz->ld = (lz->total + 63) / 64 * 64;
    lz->n_slots = hubbard_n_slots(h);
    lz->secs = hubbard_sectors(h);
    lz->generation = hubbard_generation(h);
    const auto &tiles = hubbard_tiles(h);
    hipStream_t s = nullptr;
    MBR_TRY(upload(lz->d_tiles_slot, tiles.data(), tiles.size() * sizeof(HvTile), s));
    MBR_TRY(upload(lz->d_secs, lz->secs.data(), lz->secs.size() * sizeof(HvSector), s));
    if (o->reorth) {
        // batched steps: merge a sector's tiles (contiguous rows, slot order)
        // into groups of at least kGroupRows rows, so there is one block
        // reduction per group and basis vector instead of one per tile.
        // Per-sector launches keep the tiles (a lone sector needs them all to
        // fill the GPU).
        const uint64_t grow = o->batched ? kGroupRows : 0;
        std::vector<HvTile> groups;
        std::vector<HvSector> rsecs = lz->secs;
        lz->rt0.assign(lz->ns, 0);
        lz->rnt.assign(lz->ns, 0);
        for (int si = 0; si < lz->ns; ++si) {
            const HvSector &sc = lz->secs[si];
            lz->rt0[si] = (uint32_t)groups.size();
            rsecs[si].slot0 = (uint32_t)groups.size();
            for (uint32_t t = sc.slot0; t < sc.slot0 + sc.nslots;) {
                HvTile g = tiles[t];
                g.slot = (uint32_t)groups.size();
                uint64_t rows = (uint64_t)g.nblk * sc.cdn;
                for (++t; t < sc.slot0 + sc.nslots && rows < grow; ++t) {
                    g.nblk += tiles[t].nblk;  // tiles[t] starts where the group ends
                    rows += (uint64_t)tiles[t].nblk * sc.cdn;
                }
                groups.push_back(g);
            }
            lz->rnt[si] = (uint32_t)groups.size() - lz->rt0[si];
            rsecs[si].nslots = lz->rnt[si];
        }
        lz->n_rtiles = (uint32_t)groups.size();
        MBR_TRY(upload(lz->d_rtiles, groups.data(), groups.size() * sizeof(HvTile), s));
        MBR_TRY(upload(lz->d_rsecs, rsecs.data(), rsecs.size() * sizeof(HvSector), s));
    }
    const size_t ns = lz->ns, m = lz->m, nsl = lz->n_slots;
    if (o->reorth) {
        const double bytes = (double)lz->ld * lz->tsz * (m + 2);
        if (bytes > 250e9) MBR_FAIL(MBR_ENOMEM, "basis of %.1f GB", bytes / 1e9);
        MBR_TRY(lz->basis.alloc(lz->ld * lz->tsz * (m + 1)));
        MBR_TRY(lz->work.alloc(lz->total * lz->tsz));
        MBR_TRY(lz->pc.alloc(nsl * (m + 1) * 8));
        MBR_TRY(lz->cgs.alloc(ns * (m + 1) * 8));
    } else {
        MBR_TRY(lz->bufA.alloc(lz->total * lz->tsz));
        MBR_TRY(lz->bufB.alloc(lz->total * lz->tsz));
    }
    MBR_TRY(lz->alpha.alloc(ns * m * 8));
    MBR_TRY(lz->beta.alloc(ns * m * 8));
    MBR_TRY(lz->c1.alloc(ns * 8));
    MBR_TRY(lz->c2.alloc(ns * 8));
    MBR_TRY(lz->c3.alloc(ns * 8));
    MBR_TRY(lz->pd.alloc(nsl * 8));
    MBR_TRY(lz->pn.alloc(nsl * 8));
    MBR_TRY(lz->norm0.alloc(ns * 8));
    MBR_TRY(lz->active.alloc(ns * 4));
    MBR_TRY(lz->steps.alloc(ns * 4));
    MBR_TRY(lz->jcount.alloc(8));
    MBR_TRY(lz->e0.alloc(ns * 8));
    MBR_HIP(hipMemset(lz->alpha.p, 0, ns * m * 8));
    MBR_HIP(hipMemset(lz->beta.p, 0, ns * m * 8));
    MBR_HIP(hipMemset(lz->active.p, 0, ns * 4));
    MBR_HIP(hipMemset(lz->steps.p, 0, ns * 4));
    MBR_HIP(hipMemset(lz->jcount.p, 0, 8));
    LzDev &d = lz->dev;
    d.alpha = lz->alpha.as<double>();
    d.beta = lz->beta.as<double>();
    d.c1 = lz->c1.as<double>();
    d.c2 = lz->c2.as<double>();
    d.c3 = lz->c3.as<double>();
    d.pd = lz->pd.as<double>();
    d.pn = lz->pn.as<double>();
    d.pc = lz->pc.as<double>();
    d.cgs = lz->cgs.as<double>();
    d.norm0 = lz->norm0.as<double>();
    d.active = lz->active.as<int32_t>();
    d.steps = lz->steps.as<int32_t>();
    d.j = lz->jcount.as<int32_t>();
    lz->grid = (unsigned)std::min<uint64_t>(lz->n_slots, (uint64_t)device_cu_count() * 8);
    *out = lz.release();
    return MBR_OK;
}

mbr_status mbr_lanczos_start(mbr_lanczos *lz, const double *d_v0, void *stream) {
    if (!lz || !d_v0) MBR_FAIL(MBR_EINVAL, "null argument");
    hipStream_t s = as_stream(stream);
    lz->parity = 0;
    lz->started = true;
    if (lz->prec == MBR_F64) return lz_start_t<double>(lz, d_v0, s);
    return lz_start_t<float>(lz, d_v0, s);
}

mbr_status mbr_lanczos_step(mbr_lanczos *lz, int32_t nsteps, void *stream) {
    if (!lz) MBR_FAIL(MBR_EINVAL, "null handle");
    if (!lz->started) MBR_FAIL(MBR_EINVAL, "mbr_lanczos_start has not been called");
    if (nsteps < 0) MBR_FAIL(MBR_EINVAL, "nsteps=%d", nsteps);
    if (lz->generation != hubbard_generation(lz->h))
        MBR_FAIL(MBR_EINVAL, "the Hamiltonian's launch shape changed after this Lanczos handle was created");
    hipStream_t s = as_stream(stream);
    const bool reorth = lz->o.reorth != 0;
    for (int i = 0; i < nsteps; ++i) {
        const int par = reorth ? 0 : lz->parity;
        if (lz->o.use_graph) {
            if (!lz->graph[par]) MBR_TRY(capture(lz, par));
            MBR_HIP(hipGraphLaunch(lz->graph[par], s));
        } else {
            MBR_TRY(step_any(lz, par, s));
        }
        if (!reorth) lz->parity ^= 1;
    }
    return MBR_OK;
}

mbr_status mbr_lanczos_result(mbr_lanczos *lz, double *e0, int32_t *steps_done, void *stream) {
    if (!lz) MBR_FAIL(MBR_EINVAL, "null handle");
    hipStream_t s = as_stream(stream);
    tridiag_lowest_kernel<<<lz->ns, 64, 0, s>>>(lz->dev.alpha, lz->dev.beta, lz->dev.steps, lz->m,
                                                lz->ns, lz->e0.as<double>());
    MBR_HIP(hipGetLastError());
    if (e0) MBR_HIP(hipMemcpyAsync(e0, lz->e0.p, lz->ns * 8, hipMemcpyDeviceToHost, s));
    if (steps_done) MBR_HIP(hipMemcpyAsync(steps_done, lz->dev.steps, lz->ns * 4, hipMemcpyDeviceToHost, s));
    MBR_HIP(hipStreamSynchronize(s));
    return MBR_OK;
}

mbr_status mbr_lanczos_coeffs(mbr_lanczos *lz, double *alpha, double *beta, void *stream) {
    if (!lz) MBR_FAIL(MBR_EINVAL, "null handle");
    hipStream_t s = as_stream(stream);
    const size_t n = (size_t)lz->ns * lz->m * 8;
    if (alpha) MBR_HIP(hipMemcpyAsync(alpha, lz->dev.alpha, n, hipMemcpyDeviceToHost, s));
    if (beta) MBR_HIP(hipMemcpyAsync(beta, lz->dev.beta, n, hipMemcpyDeviceToHost, s));
    MBR_HIP(hipStreamSynchronize(s));
    return MBR_OK;
}

mbr_status mbr_lanczos_destroy(mbr_lanczos *lz) {
    delete lz;
    return MBR_OK;
}

mbr_status mbr_tridiag_lowest(const double *d_alpha, const double *d_beta, const int32_t *d_len,
                              int32_t ld, int32_t n_batch, double *d_e0, void *stream) {
    if (n_batch < 0 || ld < 1) MBR_FAIL(MBR_EINVAL, "ld=%d n_batch=%d", ld, n_batch);
    if (n_batch == 0) return MBR_OK;
    if (!d_alpha || !d_beta || !d_len || !d_e0) MBR_FAIL(MBR_EINVAL, "null pointer");
    tridiag_lowest_kernel<<<n_batch, 64, 0, as_stream(stream)>>>(d_alpha, d_beta, d_len, ld, n_batch,
                                                                 d_e0);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

}  // extern "C"
