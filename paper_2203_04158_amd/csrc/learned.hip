// Learned index for ranking (an extension; the paper has none), in two
// stages as a recursive model index (Kraska et al., "The Case for Learned
// Index Structures", 2018):
//  * stage 1: a per-sector network 32 bit features -> 64 -> 64 -> 1 (ReLU)
//    predicts y ~ rank / N_s;
//  * stage 2: y selects one of n_leaves = 2^b leaves, leaf floor(y 2^b); each
//    leaf records the smallest and largest rank of the members the network
//    sends to it, measured with the query kernel's own arithmetic.
// A query is answered by the lower bound of the pattern in states[lo .. hi] of
// its leaf, so answers are exact: a member always lies inside its leaf's window
// and a non-member is never found.  The lower bound is found level by level
// over copies of every kSample^l-th state, l = H..1: a bisection over the top
// copy (at most kTopMax entries, staged in LDS), then at each level one over
// the at most kSample entries the level above leaves open (one 64-byte line),
// then one inside a block of kSample states, so below the top each level
// costs one line per query.  The recorded error e is the widest leaf window (hi - lo); when
// e exceeds the caller's bound the fallback ranker answers instead.  The
// single-window error max |rint(N_s y) - i| of stage 1 alone is kept as a
// statistic.
//
// Parameters (6337 fp32 masters): W1[64][32], b1[64], W2[64][64], b2[64],
// w3[64], b3.  Queries use their bf16 roundings with fp32 accumulation.
//
// Inference runs on the matrix cores, v_mfma_f32_16x16x32_bf16 (wave64, the
// gfx950 form with 32 products per lane pair and instruction): a wave
// evaluates 16 queries per product chain.  Layers are computed transposed,
// D = W * H^T (features x queries): the 16x16 fp32 output fragment of one
// layer (lane l holds features 4*(l/16)+r of query l%16 of a 16-feature
// tile) feeds the next product's B operand (K = features, N = queries)
// without shuffles, because the order in which a product sums over K is
// free: the K slot (g, j) of lane group g = l/16 and element j < 8 of a
// 32-feature chunk c takes feature 16 (2c + j/4) + 4 g + j%4, i.e. the two
// output fragments of tiles 2c and 2c+1 side by side, and the weights are
// loaded in that order.  Activations go from fp32 to bf16 in registers
// (rounded, then ReLU as a packed 16-bit integer maximum).  Training runs in
// fp32 on the vector ALUs (forward with the bf16 weights, backward,
// fixed-order batch reductions, Adam).
#include <cmath>
#include <memory>
#include <mutex>

#include "common.hpp"

namespace {

constexpr int kIn = 32, kH = 64;
constexpr int P_W1 = 0, P_B1 = 2048, P_W2 = 2112, P_B2 = 6208, P_W3 = 6272, P_B3 = 6336;
constexpr int kParams = 6337;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 mfma_bf16x8 __attribute__((ext_vector_type(8)));

__host__ __device__ inline uint16_t f2bf(float f) {
    // round to nearest even (finite inputs)
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf2f(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// Per-lane weight fragments of the three products (A operands), biases in the
// output-fragment layout.
struct MlpFrags {
    bf16x8 w1[4];     // tile t: one 32-input chunk
    bf16x8 w2[4][2];  // tile t, 32-feature chunk c
    bf16x8 w3[2];
    f32x4 b1[4];  // the accumulators start from the biases
    f32x4 b2[4];
    f32x4 b3;
};

// Hidden feature of K slot (lane group g, element j) of 32-feature chunk c.
__device__ __forceinline__ int kslot_feature(int c, int g, int j) { return 16 * (2 * c + (j >> 2)) + 4 * g + (j & 3); }

// bf16 bits of parameter i: stored as bf16, or rounded from fp32 as the
// training kernels round them (mlp_round_kernel).
__device__ __forceinline__ uint16_t wbits(const uint16_t *__restrict__ w, int i) { return w[i]; }
__device__ __forceinline__ uint16_t wbits(const float *__restrict__ w, int i) { return f2bf(w[i]); }

// wb: bf16 weights (or fp32 parameters) in parameter order.
template <class W>
__device__ __forceinline__ void load_frags(MlpFrags &f, const W *__restrict__ wb) {
    const int l = threadIdx.x & 63;
    const int row = l & 15, g = l >> 4, kg = g * 4;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        // layer 1: K slot (g, j) is input bit 8 g + j
#pragma unroll
        for (int j = 0; j < 8; ++j) f.w1[t][j] = (short)wbits(wb, P_W1 + (16 * t + row) * kIn + 8 * g + j);
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int j = 0; j < 8; ++j)
                f.w2[t][c][j] = (short)wbits(wb, P_W2 + (16 * t + row) * kH + kslot_feature(c, g, j));
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            f.b1[t][r] = bf2f(wbits(wb, P_B1 + 16 * t + kg + r));
            f.b2[t][r] = bf2f(wbits(wb, P_B2 + 16 * t + kg + r));
        }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int j = 0; j < 8; ++j)
            f.w3[c][j] = row == 0 ? (short)wbits(wb, P_W3 + kslot_feature(c, g, j)) : (short)0;
    const float b3 = bf2f(wbits(wb, P_B3));
    f.b3 = (f32x4){b3, b3, b3, b3};
}

// ReLU(acc) rounded to bf16: the hardware conversion (nearest even, the
// rounding of f2bf for finite values, two values per instruction), then the
// ReLU as a packed signed 16-bit maximum with 0 on the bf16 bit patterns
// (every negative value, -0 included, has the sign bit set; rounding keeps
// the sign, so this equals rounding the ReLU).  acc already holds the bias.
typedef __bf16 bf16v2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ bf16x4 relu_bf16(const f32x4 &acc) {
    s16x2 h0 = __builtin_bit_cast(s16x2, __builtin_convertvector((f32x2){acc[0], acc[1]}, bf16v2));
    s16x2 h1 = __builtin_bit_cast(s16x2, __builtin_convertvector((f32x2){acc[2], acc[3]}, bf16v2));
    h0 = __builtin_elementwise_max(h0, (s16x2){0, 0});
    h1 = __builtin_elementwise_max(h1, (s16x2){0, 0});
    return (bf16x4){h0[0], h0[1], h1[0], h1[1]};
}

__device__ __forceinline__ f32x4 mfma32(const bf16x8 &a, const bf16x8 &b, const f32x4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(mfma_bf16x8, a),
                                                   __builtin_bit_cast(mfma_bf16x8, b), c, 0, 0, 0);
}

// Network output for the 16 queries held by lanes 16*grp .. 16*grp+15 of the
// wave (pattern in `q` of each lane).  The result is valid in lanes 0..15,
// lane n holding the output of query 16*grp + n.  All 64 lanes must call.
__device__ __forceinline__ float mlp16(const MlpFrags &f, uint32_t q, int grp) {
    const int l = threadIdx.x & 63;
    const uint32_t a = (uint32_t)__shfl((int)q, 16 * grp + (l & 15), 64);
    const uint32_t bits = (a >> (8 * (l >> 4))) & 0xFFu;  // inputs 8 g .. 8 g + 7
    bf16x8 xb;
#pragma unroll
    for (int j = 0; j < 8; ++j) xb[j] = ((bits >> j) & 1u) ? (short)0x3F80 : (short)0;
    bf16x4 h1[4], h2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) h1[t] = relu_bf16(mfma32(f.w1[t], xb, f.b1[t]));
    const bf16x8 k1[2] = {__builtin_shufflevector(h1[0], h1[1], 0, 1, 2, 3, 4, 5, 6, 7),
                          __builtin_shufflevector(h1[2], h1[3], 0, 1, 2, 3, 4, 5, 6, 7)};
#pragma unroll
    for (int t = 0; t < 4; ++t) h2[t] = relu_bf16(mfma32(f.w2[t][1], k1[1], mfma32(f.w2[t][0], k1[0], f.b2[t])));
    const bf16x8 k2[2] = {__builtin_shufflevector(h2[0], h2[1], 0, 1, 2, 3, 4, 5, 6, 7),
                          __builtin_shufflevector(h2[2], h2[3], 0, 1, 2, 3, 4, 5, 6, 7)};
    const f32x4 acc = mfma32(f.w3[1], k2[1], mfma32(f.w3[0], k2[0], f.b3));
    return acc[0];
}

// Network outputs for the 64 queries of a wave, each lane receiving its own.
// The four groups run one after another: going through each layer with all
// four together hides the latency of the dependent products but needs about
// 180 registers, which costs the ranking kernel more occupancy than it gains.
__device__ __forceinline__ float mlp64(const MlpFrags &f, uint32_t q) {
    const int l = threadIdx.x & 63;
    const float y0 = mlp16(f, q, 0), y1 = mlp16(f, q, 1), y2 = mlp16(f, q, 2), y3 = mlp16(f, q, 3);
    const float s0 = __shfl(y0, l & 15, 64), s1 = __shfl(y1, l & 15, 64);
    const float s2 = __shfl(y2, l & 15, 64), s3 = __shfl(y3, l & 15, 64);
    const int g = l >> 4;
    return g == 0 ? s0 : g == 1 ? s1 : g == 2 ? s2 : s3;
}

__device__ __forceinline__ int64_t predict_rank(float y, uint64_t n) {
    double p = rint((double)n * (double)y);
    if (!(p >= 0.0)) p = 0.0;  // also NaN
    if (p > (double)(n - 1)) p = (double)(n - 1);
    return (int64_t)p;
}

// ---------------------------------------------------------------- inference
template <class W>
__global__ void __launch_bounds__(256) mlp_forward_kernel(const W *__restrict__ wb,
                                                          const uint32_t *__restrict__ q, int B,
                                                          float *__restrict__ out) {
    MlpFrags f;
    load_frags(f, wb);
    const int waves = gridDim.x * (blockDim.x >> 6);
    for (int base = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64; base < B; base += waves * 64) {
        const int i = base + (threadIdx.x & 63);
        const uint32_t a = i < B ? q[i] : 0u;
        const float y = mlp64(f, a);
        if (i < B) out[i] = y;
    }
}

// Largest |p(alpha_i) - i| over the sector (the query kernel's arithmetic).
__global__ void __launch_bounds__(256) mlp_maxerr_kernel(const uint16_t *__restrict__ wb,
                                                         const uint32_t *__restrict__ states,
                                                         uint64_t n, unsigned long long *emax) {
    MlpFrags f;
    load_frags(f, wb);
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    unsigned long long e = 0;
    for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64; base < n;
         base += waves * 64) {
        const uint64_t i = base + (threadIdx.x & 63);
        const uint32_t a = i < n ? states[i] : 0u;
        const float y = mlp64(f, a);
        if (i < n) {
            const int64_t p = predict_rank(y, n);
            const unsigned long long d = (unsigned long long)(p > (int64_t)i ? p - (int64_t)i : (int64_t)i - p);
            e = d > e ? d : e;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long v = __shfl_down(e, o, 64);
        e = v > e ? v : e;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(emax, e);
}

// Leaf of a network output: floor(y n_leaves) clamped to the leaves (n_leaves
// is a power of two, so the product is exact in fp32); NaN and y <= 0 go to
// leaf 0.
__device__ __forceinline__ uint32_t leaf_of(float y, uint32_t nleaf) {
    if (!(y > 0.f)) return 0u;
    if (y >= 1.f) return nleaf - 1u;
    return (uint32_t)(y * (float)nleaf);
}

// Empty leaves: lo = all ones, hi = 0 (an empty window).
__global__ void leaf_clear_kernel(uint2 *leaf, uint32_t nleaf) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nleaf) leaf[i] = make_uint2(0xFFFFFFFFu, 0u);
}

// Stage-2 windows: every member i widens the window of its leaf to include i.
__global__ void __launch_bounds__(256) leaf_build_kernel(const uint16_t *__restrict__ wb,
                                                         const uint32_t *__restrict__ states, uint64_t n,
                                                         uint32_t nleaf, uint2 *__restrict__ leaf) {
    MlpFrags f;
    load_frags(f, wb);
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64; base < n;
         base += waves * 64) {
        const uint64_t i = base + (threadIdx.x & 63);
        const uint32_t a = i < n ? states[i] : 0u;
        const float y = mlp64(f, a);
        if (i < n) {
            uint32_t *w = reinterpret_cast<uint32_t *>(leaf + leaf_of(y, nleaf));
            atomicMin(w, (uint32_t)i);
            atomicMax(w + 1, (uint32_t)i);
        }
    }
}

// Window statistics over the members: acc[0] += hi - lo + 1 of each member's
// leaf (the mean window is acc[0] / n), acc[1] = max (hi - lo).
__global__ void __launch_bounds__(256) leaf_stats_kernel(const uint16_t *__restrict__ wb,
                                                         const uint32_t *__restrict__ states, uint64_t n,
                                                         uint32_t nleaf, const uint2 *__restrict__ leaf,
                                                         unsigned long long *acc) {
    MlpFrags f;
    load_frags(f, wb);
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    unsigned long long sum = 0, mx = 0;
    for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64; base < n;
         base += waves * 64) {
        const uint64_t i = base + (threadIdx.x & 63);
        const uint32_t a = i < n ? states[i] : 0u;
        const float y = mlp64(f, a);
        if (i < n) {
            const uint2 w = leaf[leaf_of(y, nleaf)];
            const unsigned long long d = (unsigned long long)(w.y - w.x);
            sum += d + 1;
            mx = d > mx ? d : mx;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        sum += __shfl_down(sum, o, 64);
        const unsigned long long v = __shfl_down(mx, o, 64);
        mx = v > mx ? v : mx;
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(acc, sum);
        atomicMax(acc + 1, mx);
    }
}

constexpr uint32_t kSample = 16;     // states per sampled block (64 bytes)
constexpr uint32_t kTopMax = 8192;   // entries of the top copy (32 KB of LDS)
constexpr int kMaxLevels = 8;        // kSample^8 = 2^32 states

struct SampleLevels {
    const uint32_t *lv[kMaxLevels];  // lv[l]: states[b kSample^(l+1)]
    int32_t H;                       // copies; lv[H-1] is the top
    uint32_t top_n;                  // entries of the top copy
    uint64_t n;                      // states
};

// sample[b] = states[b stride] for b < nb, all ones up to the padded length
// npad (a multiple of kSample, so every aligned line of the copy can be read
// whole).
__global__ void sample_kernel(const uint32_t *__restrict__ states, uint32_t stride,
                              uint32_t *__restrict__ sample, uint64_t nb, uint64_t npad) {
    for (uint64_t b = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; b < npad; b += (uint64_t)gridDim.x * blockDim.x)
        sample[b] = b < nb ? states[b * stride] : 0xFFFFFFFFu;
}

// Entries [lo, hi) of v lie in the aligned line of kSample entries at base;
// their lower bound for a is lo plus the number below a (they are sorted).
// The line is read as four 16-byte loads in one round trip.
__device__ __forceinline__ uint32_t line_lower_bound(const uint32_t *__restrict__ v, uint32_t base,
                                                     uint32_t lo, uint32_t hi, uint32_t a) {
    const uint4 *p = reinterpret_cast<const uint4 *>(v + base);
    const uint4 q0 = p[0], q1 = p[1], q2 = p[2], q3 = p[3];
    const uint32_t e[kSample] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w,
                                 q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w};
    uint32_t c = 0;
#pragma unroll
    for (uint32_t i = 0; i < kSample; ++i) c += (base + i >= lo && base + i < hi && e[i] < a) ? 1u : 0u;
    return lo + c;
}

// narrow() for a copy below the top: the blocks it considers are the at most
// kSample children of the block the level above left open, one aligned line.
__device__ __forceinline__ void narrow_line(const uint32_t *__restrict__ smp, uint32_t stride, uint32_t a,
                                            uint32_t &L, uint32_t &H1) {
    const uint32_t b0 = L / stride + 1, b1 = (H1 - 1) / stride + 1;
    const uint32_t bl = b1 > b0 ? line_lower_bound(smp, (b0 - 1) & ~(kSample - 1), b0, b1, a) : b0;
    const uint32_t lo = (bl - 1) * stride, hi = bl * stride;
    L = lo > L ? lo : L;
    H1 = hi < H1 ? hi : H1;
}

// Narrow [L, H1), which holds the lower bound of a among the states of the
// window (H1 when none is >= a), to the blocks of `stride` states: among the
// blocks b with b stride in (L, H1 - 1], the first whose sampled state is not
// below a bounds the answer from above and the block before it from below.
template <class PTR>
__device__ __forceinline__ void narrow(PTR smp, uint32_t stride, uint32_t a, uint32_t &L, uint32_t &H1) {
    uint32_t bl = L / stride + 1, br = (H1 - 1) / stride + 1;
    while (bl < br) {
        const uint32_t mid = bl + ((br - bl) >> 1);
        if (smp[mid] < a) bl = mid + 1;
        else br = mid;
    }
    const uint32_t lo = (bl - 1) * stride, hi = bl * stride;
    L = lo > L ? lo : L;
    H1 = hi < H1 ? hi : H1;
}

// NET: the window comes from the network and its leaf; without it the window
// is the whole list and the search alone ranks (a static 16-ary search over
// the sampled copies).
template <bool NET>
__global__ void __launch_bounds__(256) learned_rank_kernel(const uint16_t *__restrict__ wb,
                                                           const uint32_t *__restrict__ states,
                                                           SampleLevels sl,
                                                           const uint2 *__restrict__ leaf, uint32_t nleaf,
                                                           int M, const uint32_t *__restrict__ q,
                                                           uint64_t nq, uint32_t *__restrict__ out) {
    __shared__ uint32_t top[kTopMax];
    for (uint32_t i = threadIdx.x; i < sl.top_n; i += blockDim.x) top[i] = sl.lv[sl.H - 1][i];
    __syncthreads();
    MlpFrags f;
    if constexpr (NET) load_frags(f, wb);
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64; base < nq;
         base += waves * 64) {
        const uint64_t j = base + (threadIdx.x & 63);
        const uint32_t a = j < nq ? q[j] : 0u;
        uint2 w = make_uint2(0u, (uint32_t)(sl.n - 1));
        if constexpr (NET) {
            const float y = mlp64(f, a);  // every lane of the wave takes part
            if (j < nq) w = leaf[leaf_of(y, nleaf)];
        }
        if (j >= nq) continue;
        const bool in_width = M >= 32 || (a >> M) == 0;
        // lower bound of a in states[lo .. hi] (empty when lo > hi)
        uint32_t L = w.x, R = w.y + 1u;
        bool hit = false;
        if (in_width && w.x <= w.y) {
            uint32_t stride = 1;
            for (int l = 0; l < sl.H; ++l) stride *= kSample;
            narrow(top, stride, a, L, R);
            for (int l = sl.H - 2; l >= 0; --l) {
                stride /= kSample;
                narrow_line(sl.lv[l], stride, a, L, R);
            }
            // [L, R) lies in one aligned block of kSample states
            const uint32_t base = L & ~(kSample - 1);
            if ((uint64_t)base + kSample <= sl.n) {
                L = line_lower_bound(states, base, L, R, a);
            } else {
                while (L < R) {
                    const uint32_t mid = L + ((R - L) >> 1);
                    if (states[mid] < a) L = mid + 1;
                    else R = mid;
                }
            }
            hit = L <= w.y && states[L] == a;
        }
        out[j] = hit ? L : MBR_NOT_FOUND;
    }
}

// ---------------------------------------------------------------- training
// SplitMix64, element k of the stream of `seed` (the generator the sample
// draws are defined by).
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Scratch of one batch, feature-major ([feature][sample]) so that the
// per-sample threads write and the reduction reads contiguous rows.
struct TrainScratch {
    float *h1, *h2, *dz1, *dz2;  // [64][B]
    float *dy;                   // [B]
    uint32_t *x;                 // [B] patterns
    float *loss_part;            // [B / 64]
};

// One thread per sample: forward with bf16-rounded weights in fp32, loss,
// backward to dz2 and dz1.  Samples come from (q, tgt) when given, else are
// drawn from the sector: idx = splitmix64(seed, step*B + s) mod n.
__global__ void __launch_bounds__(64) mlp_fwd_bwd_kernel(const float *__restrict__ wr, int B,
                                                         const uint32_t *__restrict__ q,
                                                         const float *__restrict__ tgt,
                                                         const uint32_t *__restrict__ states,
                                                         uint64_t n, uint64_t seed, uint64_t step,
                                                         TrainScratch S) {
    __shared__ float w1[kH * kIn], w2[kH * kH], b1[kH], b2[kH], w3[kH];
    __shared__ float sh1[kH][64], sdz2[kH][64];  // per-thread vectors, [feature][thread]
    const int tid = threadIdx.x;
    for (int i = threadIdx.x; i < kH * kIn; i += blockDim.x) w1[i] = wr[P_W1 + i];
    for (int i = threadIdx.x; i < kH * kH; i += blockDim.x) w2[i] = wr[P_W2 + i];
    for (int i = threadIdx.x; i < kH; i += blockDim.x) {
        b1[i] = wr[P_B1 + i];
        b2[i] = wr[P_B2 + i];
        w3[i] = wr[P_W3 + i];
    }
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    float sq = 0.f;
    if (s < B) {
        uint32_t a;
        float t;
        if (q) {
            a = q[s];
            t = tgt[s];
        } else {
            const uint64_t idx = splitmix64_at(seed, step * (uint64_t)B + (uint64_t)s) % n;
            a = states[idx];
            t = (float)((double)idx / (double)n);
        }
        S.x[s] = a;
        for (int i = 0; i < kH; ++i) {
            float z = b1[i];
            uint32_t m = a;
            while (m) {
                const int k = __ffs(m) - 1;
                m &= m - 1;
                z += w1[i * kIn + k];
            }
            const float h = z > 0.f ? z : 0.f;
            sh1[i][tid] = h;
            S.h1[(size_t)i * B + s] = h;
        }
        float y = wr[P_B3];
        for (int j = 0; j < kH; ++j) {
            float z = b2[j];
#pragma unroll 16
            for (int i = 0; i < kH; ++i) z += w2[j * kH + i] * sh1[i][tid];
            const float h = z > 0.f ? z : 0.f;
            S.h2[(size_t)j * B + s] = h;
            y += w3[j] * h;
            sdz2[j][tid] = z > 0.f ? 1.f : 0.f;  // ReLU mask, scaled below
        }
        const float d = 2.f * (y - t) / (float)B;
        sq = (y - t) * (y - t);
        S.dy[s] = d;
        for (int j = 0; j < kH; ++j) {
            const float g = sdz2[j][tid] * d * w3[j];
            sdz2[j][tid] = g;
            S.dz2[(size_t)j * B + s] = g;
        }
        for (int i = 0; i < kH; ++i) {
            float g = 0.f;
#pragma unroll 16
            for (int j = 0; j < kH; ++j) g += w2[j * kH + i] * sdz2[j][tid];
            S.dz1[(size_t)i * B + s] = sh1[i][tid] > 0.f ? g : 0.f;
        }
    }
    // per-wave partial of the squared error
    for (int o = 32; o > 0; o >>= 1) sq += __shfl_down(sq, o, 64);
    if ((threadIdx.x & 63) == 0) S.loss_part[s >> 6] = sq;
}

constexpr int kChunk = 64;  // samples per gradient-partial workgroup

// Gradient partials of one chunk of kChunk samples, all 6337 parameters.
__global__ void __launch_bounds__(256) mlp_grad_part_kernel(int B, TrainScratch S, float *__restrict__ part) {
    __shared__ float ta[kH][kChunk + 1];
    __shared__ float tb[kH][kChunk + 1];
    __shared__ uint32_t xs[kChunk];
    __shared__ float dys[kChunk];
    const int c0 = blockIdx.x * kChunk;
    const int cn = min(kChunk, B - c0);
    float *out = part + (size_t)blockIdx.x * kParams;
    // phase A: dz2 (ta) and h1 (tb): gW2[j][i] = sum_s dz2[j][s] h1[i][s], gb2
    for (int e = threadIdx.x; e < kH * kChunk; e += blockDim.x) {
        const int f = e / kChunk, s = e % kChunk;
        ta[f][s] = s < cn ? S.dz2[(size_t)f * B + c0 + s] : 0.f;
        tb[f][s] = s < cn ? S.h1[(size_t)f * B + c0 + s] : 0.f;
    }
    for (int s = threadIdx.x; s < kChunk; s += blockDim.x) {
        xs[s] = s < cn ? S.x[c0 + s] : 0u;
        dys[s] = s < cn ? S.dy[c0 + s] : 0.f;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kH * kH; e += blockDim.x) {
        const int j = e / kH, i = e % kH;
        float g = 0.f;
        for (int s = 0; s < kChunk; ++s) g += ta[j][s] * tb[i][s];
        out[P_W2 + e] = g;
    }
    for (int j = threadIdx.x; j < kH; j += blockDim.x) {
        float g = 0.f;
        for (int s = 0; s < kChunk; ++s) g += ta[j][s];
        out[P_B2 + j] = g;
    }
    __syncthreads();
    // phase B: dz1 (ta) and h2 (tb): gW1[i][k] = sum_s dz1[i][s] x_k(s), gb1, gw3, gb3
    for (int e = threadIdx.x; e < kH * kChunk; e += blockDim.x) {
        const int f = e / kChunk, s = e % kChunk;
        ta[f][s] = s < cn ? S.dz1[(size_t)f * B + c0 + s] : 0.f;
        tb[f][s] = s < cn ? S.h2[(size_t)f * B + c0 + s] : 0.f;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kH * kIn; e += blockDim.x) {
        const int i = e / kIn, k = e % kIn;
        float g = 0.f;
        for (int s = 0; s < kChunk; ++s) g += ((xs[s] >> k) & 1u) ? ta[i][s] : 0.f;
        out[P_W1 + e] = g;
    }
    for (int i = threadIdx.x; i < kH; i += blockDim.x) {
        float g1 = 0.f, g3 = 0.f;
        for (int s = 0; s < kChunk; ++s) {
            g1 += ta[i][s];
            g3 += dys[s] * tb[i][s];
        }
        out[P_B1 + i] = g1;
        out[P_W3 + i] = g3;
    }
    if (threadIdx.x == 0) {
        float g = 0.f;
        for (int s = 0; s < kChunk; ++s) g += dys[s];
        out[P_B3] = g;
    }
}

// Sum the chunk partials in chunk order; optionally apply one Adam step to the
// fp32 masters and refresh the rounded copies (fp32 value and bf16 bits).
__global__ void mlp_reduce_adam_kernel(const float *__restrict__ part, int nchunk, float *grad,
                                       float *w, float *m, float *v, float *wr, uint16_t *wb,
                                       float lr, float b1c, float b2c, int adam) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    float g = 0.f;
    for (int c = 0; c < nchunk; ++c) g += part[(size_t)c * kParams + p];
    if (grad) grad[p] = g;
    if (!adam) return;
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    const float mm = beta1 * m[p] + (1.f - beta1) * g;
    const float vv = beta2 * v[p] + (1.f - beta2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / b1c, vh = vv / b2c;
    const float nw = w[p] - lr * mh / (sqrtf(vh) + eps);
    w[p] = nw;
    const uint16_t b = f2bf(nw);
    wb[p] = b;
    wr[p] = bf2f(b);
}

__global__ void mlp_round_kernel(const float *__restrict__ w, float *wr, uint16_t *wb) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    const uint16_t b = f2bf(w[p]);
    wb[p] = b;
    wr[p] = bf2f(b);
}

__global__ void mlp_loss_kernel(const float *__restrict__ lp, int nparts, int B, float *loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float s = 0.f;
    for (int i = 0; i < nparts; ++i) s += lp[i];
    *loss = s / (float)B;
}

// Bytes of a batch's activation scratch and of its chunk partials.
constexpr size_t act_bytes(size_t b) { return b * 4 * (4 * kH + 2) + (b / 64 + 1) * 4; }
constexpr size_t part_bytes(size_t b) { return (b + kChunk - 1) / kChunk * kParams * 4; }

// Activation scratch of B samples laid out in the memory at f.
TrainScratch carve(float *f, size_t n) {
    TrainScratch S{};
    S.h1 = f;
    S.h2 = f + n * kH;
    S.dz1 = f + 2 * n * kH;
    S.dz2 = f + 3 * n * kH;
    S.dy = f + 4 * n * kH;
    S.x = reinterpret_cast<uint32_t *>(f + 4 * n * kH + n);
    S.loss_part = f + 4 * n * kH + 2 * n;
    return S;
}

// Batch scratch of B samples.
struct TrainBufs {
    mbr::DevBuf scratch, part;
    TrainScratch S{};
    int B = 0;
    mbr_status alloc(int b) {
        B = b;
        MBR_TRY(scratch.alloc(act_bytes((size_t)b)));
        S = carve(scratch.as<float>(), (size_t)b);
        MBR_TRY(part.alloc(part_bytes((size_t)b)));
        return MBR_OK;
    }
};

// Scratch of mbr_mlp_gradients_noalloc in one file-scope device array: the
// rounded weights (fp32 and bf16), then the activations and the chunk
// partials of a batch of up to kStaticBatch samples.  Each device holds its
// own copy for the life of the process; host code uses only the address
// hipGetSymbolAddress returns for the current device (static_scratch).
constexpr int kStaticBatch = 8192;
constexpr size_t kAl = 256;
constexpr size_t al256(size_t v) { return (v + kAl - 1) / kAl * kAl; }
constexpr size_t kStWr = 0;
constexpr size_t kStWb = al256(kStWr + (size_t)kParams * 4);
constexpr size_t kStAct = al256(kStWb + (size_t)kParams * 2);
constexpr size_t kStPart = al256(kStAct + act_bytes(kStaticBatch));
constexpr size_t kStaticBytes = al256(kStPart + part_bytes(kStaticBatch));
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices] = {nullptr};

// Device address of `scratch` on the current device, looked up once per device.
mbr_status static_scratch(unsigned char **out) {
    int dev = 0;
    MBR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) MBR_FAIL(MBR_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            MBR_FAIL(MBR_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_static_ptr[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_static_ptr[dev]);
    return MBR_OK;
}

// Forward/backward and chunk partials of one batch.
mbr_status batch_grad(TrainBufs &T, const float *wr, const uint32_t *q, const float *tgt,
                      const uint32_t *states, uint64_t n, uint64_t seed, uint64_t step, hipStream_t s) {
    const int B = T.B;
    mlp_fwd_bwd_kernel<<<(B + 63) / 64, 64, 0, s>>>(wr, B, q, tgt, states, n, seed, step, T.S);
    mlp_grad_part_kernel<<<(B + kChunk - 1) / kChunk, 256, 0, s>>>(B, T.S, T.part.as<float>());
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

}  // namespace

struct LearnedModel {
    bool net = true;              // false: sampled-copy search over the whole list
    uint64_t n = 0;
    int32_t M = 0;
    mbr::DevBuf w, m, v, wr, wb;  // masters, Adam moments, rounded fp32, bf16
    mbr::DevBuf leaf;             // stage-2 windows, uint2 {lo, hi} per leaf
    mbr::DevBuf sample[kMaxLevels];  // copy l: every kSample^(l+1)-th state of the sector
    int32_t n_sample = 0;
    uint32_t n_leaves = 0;
    uint64_t e = 0;               // widest leaf window, hi - lo
    uint64_t e_single = 0;        // max |rint(N_s y) - i| of stage 1 alone
    double mean_window = 0;       // member-weighted mean of hi - lo + 1
    int32_t uses_window = 0;
    double last_loss = 0;
};

void learned_free(LearnedModel *m) { delete m; }
int32_t learned_levels(const LearnedModel *m) { return m ? m->n_sample + 1 : 0; }
uint64_t learned_bytes(const LearnedModel *m) {
    if (!m) return 0;
    uint64_t b = m->net ? (uint64_t)kParams * 2 + (uint64_t)m->n_leaves * 8 : 0;
    for (int l = 0; l < m->n_sample; ++l) b += m->sample[l].bytes;
    return b;
}

// Sampled copies of the sector list, every kSample^l-th state, until the
// top one fits kTopMax.
static mbr_status build_samples(LearnedModel &lm, const mbr_sector *sec, hipStream_t s) {
    using namespace mbr;
    uint64_t stride = 1, nb = sec->n;
    lm.n_sample = 0;
    do {
        stride *= kSample;
        nb = (sec->n + stride - 1) / stride;
        const uint64_t npad = (nb + kSample - 1) / kSample * kSample;
        DevBuf &d = lm.sample[lm.n_sample++];
        MBR_TRY(d.alloc(npad * 4));
        sample_kernel<<<grid_for(npad, 256, device_cu_count() * 8), 256, 0, s>>>(
            sec->states.as<uint32_t>(), (uint32_t)stride, d.as<uint32_t>(), nb, npad);
    } while (nb > kTopMax && lm.n_sample < kMaxLevels);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

mbr_status rank_learned_launch(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out,
                               hipStream_t s) {
    const LearnedModel &lm = *r->learned;
    if (lm.net && !lm.uses_window) {
        if (!r->fallback) MBR_FAIL(MBR_EINVAL, "learned ranker without window or fallback");
        return mbr_rank_batch(r->fallback, q, n, out, s);
    }
    const unsigned grid = mbr::grid_for(n, 256, mbr::device_cu_count() * 8);
    SampleLevels sl{};
    sl.H = lm.n_sample;
    uint64_t stride = 1;
    for (int l = 0; l < lm.n_sample; ++l) {
        sl.lv[l] = lm.sample[l].as<uint32_t>();
        stride *= kSample;
    }
    sl.top_n = (uint32_t)((lm.n + stride - 1) / stride);
    sl.n = lm.n;
    auto kernel = lm.net ? learned_rank_kernel<true> : learned_rank_kernel<false>;
    kernel<<<grid, 256, 0, s>>>(lm.wb.as<uint16_t>(), r->sector->states.as<uint32_t>(), sl,
                                lm.leaf.as<uint2>(), lm.n_leaves, lm.M, static_cast<const uint32_t *>(q), n,
                                out);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

namespace {

// He-uniform initialisation from SplitMix64 (host), biases zero.
std::vector<float> init_params(uint64_t seed) {
    std::vector<float> p(kParams, 0.f);
    uint64_t k = 0;
    auto u01 = [&]() {
        uint64_t z = seed + (++k) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double)(z >> 11) * (1.0 / 9007199254740992.0);
    };
    const double a1 = std::sqrt(6.0 / kIn), a2 = std::sqrt(6.0 / kH), a3 = std::sqrt(3.0 / kH);
    for (int i = 0; i < kH * kIn; ++i) p[P_W1 + i] = (float)((2 * u01() - 1) * a1);
    for (int i = 0; i < kH * kH; ++i) p[P_W2 + i] = (float)((2 * u01() - 1) * a2);
    for (int i = 0; i < kH; ++i) p[P_W3 + i] = (float)((2 * u01() - 1) * a3);
    p[P_B3] = 0.5f;
    return p;
}

}  // namespace

extern "C" {

mbr_status mbr_learned_train(const mbr_sector *sec, const mbr_learned_opts *o,
                             const mbr_ranker *fallback, mbr_ranker **out, void *stream) {
    using namespace mbr;
    if (!out) MBR_FAIL(MBR_EINVAL, "null output handle");
    *out = nullptr;
    if (!sec || !o) MBR_FAIL(MBR_EINVAL, "null sector or options");
    if (sec->width_bits != 32) MBR_FAIL(MBR_EUNSUPPORTED, "learned ranking needs 32-bit patterns");
    if (sec->n < 2) MBR_FAIL(MBR_EINVAL, "sector of %llu states", (unsigned long long)sec->n);
    if (sec->n >= MBR_NOT_FOUND) MBR_FAIL(MBR_ERANGE, "ranks of %llu states do not fit below MBR_NOT_FOUND",
                                          (unsigned long long)sec->n);
    if (o->epochs < 0 || o->batch < 256 || o->batch % 256 != 0 || o->batch > (1 << 20))
        MBR_FAIL(MBR_EINVAL, "epochs=%d batch=%d (batch: multiple of 256 up to 2^20)", o->epochs, o->batch);
    if (!(o->lr > 0.f)) MBR_FAIL(MBR_EINVAL, "lr must be positive");
    if (o->log2_leaves != 0 && (o->log2_leaves < 8 || o->log2_leaves > 28))
        MBR_FAIL(MBR_EINVAL, "log2_leaves=%d (0, or 8 to 28)", o->log2_leaves);
    if (fallback && fallback->n_states != sec->n) MBR_FAIL(MBR_EINVAL, "fallback ranks a different sector");
    hipStream_t s = as_stream(stream);
    auto lm = std::make_unique<LearnedModel>();
    lm->n = sec->n;
    lm->M = sec->M;
    std::vector<float> p0 = init_params(o->seed);
    MBR_TRY(upload(lm->w, p0.data(), kParams * 4, s));
    MBR_TRY(lm->m.alloc(kParams * 4));
    MBR_TRY(lm->v.alloc(kParams * 4));
    MBR_TRY(lm->wr.alloc(kParams * 4));
    MBR_TRY(lm->wb.alloc(kParams * 2));
    MBR_HIP(hipMemsetAsync(lm->m.p, 0, kParams * 4, s));
    MBR_HIP(hipMemsetAsync(lm->v.p, 0, kParams * 4, s));
    mlp_round_kernel<<<(kParams + 255) / 256, 256, 0, s>>>(lm->w.as<float>(), lm->wr.as<float>(), lm->wb.as<uint16_t>());
    TrainBufs T;
    MBR_TRY(T.alloc(o->batch));
    const uint64_t per_epoch = o->samples_per_epoch ? o->samples_per_epoch : sec->n;
    const uint64_t steps_per_epoch = (per_epoch + o->batch - 1) / o->batch;
    const uint64_t total = steps_per_epoch * (uint64_t)o->epochs;
    const int nchunk = (o->batch + kChunk - 1) / kChunk;
    double b1p = 1.0, b2p = 1.0;
    for (uint64_t st = 0; st < total; ++st) {
        MBR_TRY(batch_grad(T, lm->wr.as<float>(), nullptr, nullptr, sec->states.as<uint32_t>(), sec->n,
                           o->seed, st, s));
        b1p *= 0.9;
        b2p *= 0.999;
        // cosine decay of the step size over the run
        const double lr = o->lr * 0.5 * (1.0 + std::cos(3.14159265358979323846 * (double)st / (double)total));
        mlp_reduce_adam_kernel<<<(kParams + 255) / 256, 256, 0, s>>>(
            T.part.as<float>(), nchunk, nullptr, lm->w.as<float>(), lm->m.as<float>(), lm->v.as<float>(),
            lm->wr.as<float>(), lm->wb.as<uint16_t>(), (float)lr, (float)(1.0 - b1p), (float)(1.0 - b2p), 1);
        MBR_HIP(hipGetLastError());
    }
    // maximum error with the query kernel's own arithmetic
    DevBuf d_e;
    MBR_TRY(d_e.alloc(8));
    MBR_HIP(hipMemsetAsync(d_e.p, 0, 8, s));
    const unsigned grid = grid_for(sec->n, 256, device_cu_count() * 8);
    mlp_maxerr_kernel<<<grid, 256, 0, s>>>(lm->wb.as<uint16_t>(), sec->states.as<uint32_t>(), sec->n,
                                           d_e.as<unsigned long long>());
    MBR_HIP(hipGetLastError());
    // stage 2: leaf windows (about four members per leaf), then their statistics
    // Automatic: about four members per leaf, at most 2^12 leaves.  The table
    // (32 KB) then stays in every L2; with many more leaves the leaf read
    // becomes a gather from HBM that costs more than the narrower windows
    // save (2^26 leaves: 13.0 against 16.3 Granks/s on a 165.6 M sector).
    uint64_t nl = 256;
    if (o->log2_leaves) nl = 1ull << o->log2_leaves;
    else
        while (nl < sec->n / 4 && nl < (1ull << 12)) nl <<= 1;
    lm->n_leaves = (uint32_t)nl;
    MBR_TRY(lm->leaf.alloc(nl * 8));
    MBR_TRY(build_samples(*lm, sec, s));
    leaf_clear_kernel<<<(unsigned)((nl + 255) / 256), 256, 0, s>>>(lm->leaf.as<uint2>(), (uint32_t)nl);
    leaf_build_kernel<<<grid, 256, 0, s>>>(lm->wb.as<uint16_t>(), sec->states.as<uint32_t>(), sec->n,
                                           (uint32_t)nl, lm->leaf.as<uint2>());
    DevBuf d_acc;
    MBR_TRY(d_acc.alloc(16));
    MBR_HIP(hipMemsetAsync(d_acc.p, 0, 16, s));
    leaf_stats_kernel<<<grid, 256, 0, s>>>(lm->wb.as<uint16_t>(), sec->states.as<uint32_t>(), sec->n,
                                           (uint32_t)nl, lm->leaf.as<uint2>(), d_acc.as<unsigned long long>());
    MBR_HIP(hipGetLastError());
    unsigned long long e = 0, acc[2] = {0, 0};
    MBR_HIP(hipMemcpyAsync(&e, d_e.p, 8, hipMemcpyDeviceToHost, s));
    MBR_HIP(hipMemcpyAsync(acc, d_acc.p, 16, hipMemcpyDeviceToHost, s));
    MBR_HIP(hipStreamSynchronize(s));
    lm->e_single = e;
    lm->e = acc[1];
    lm->mean_window = (double)acc[0] / (double)sec->n;
    lm->uses_window = (lm->e <= o->max_window) ? 1 : 0;
    if (!lm->uses_window && !fallback)
        MBR_FAIL(MBR_ERANGE, "widest leaf window %llu exceeds max_window and no fallback was given",
                 (unsigned long long)lm->e);
    auto *r = new (std::nothrow) mbr_ranker;
    if (!r) MBR_FAIL(MBR_ENOMEM, "host allocation");
    r->kind = MBR_RANKER_LEARNED;
    r->M = sec->M;
    r->k = 0;
    r->width_bits = 32;
    r->n_states = sec->n;
    r->sector = sec;
    r->fallback = fallback;
    (void)hipGetDevice(&r->device);
    r->learned = lm.release();
    *out = r;
    return MBR_OK;
}

mbr_status mbr_build_sampled_ranker(const mbr_sector *sec, mbr_ranker **out, void *stream) {
    using namespace mbr;
    if (!out) MBR_FAIL(MBR_EINVAL, "null output handle");
    *out = nullptr;
    if (!sec) MBR_FAIL(MBR_EINVAL, "null sector");
    if (sec->width_bits != 32) MBR_FAIL(MBR_EUNSUPPORTED, "the sampled search needs 32-bit patterns");
    if (sec->n == 0) MBR_FAIL(MBR_EINVAL, "empty sector");
    if (sec->n >= MBR_NOT_FOUND) MBR_FAIL(MBR_ERANGE, "ranks of %llu states do not fit below MBR_NOT_FOUND",
                                          (unsigned long long)sec->n);
    hipStream_t s = as_stream(stream);
    auto lm = std::make_unique<LearnedModel>();
    lm->net = false;
    lm->n = sec->n;
    lm->M = sec->M;
    lm->uses_window = 1;
    MBR_TRY(build_samples(*lm, sec, s));
    MBR_HIP(hipStreamSynchronize(s));
    auto r = std::make_unique<mbr_ranker>();
    r->kind = MBR_RANKER_SAMPLED;
    r->M = sec->M;
    r->k = 0;
    r->width_bits = 32;
    r->n_states = sec->n;
    r->sector = sec;
    (void)hipGetDevice(&r->device);
    r->learned = lm.release();
    *out = r.release();
    return MBR_OK;
}

mbr_status mbr_learned_max_error(const mbr_ranker *r, uint64_t *e, int32_t *uses_window) {
    if (!r || r->kind != MBR_RANKER_LEARNED) MBR_FAIL(MBR_EINVAL, "not a learned ranker");
    if (e) *e = r->learned->e;
    if (uses_window) *uses_window = r->learned->uses_window;
    return MBR_OK;
}

mbr_status mbr_learned_autotune(mbr_ranker *r, const void *d_q, uint64_t n, int32_t reps, double *ms_window,
                                double *ms_fallback, void *stream) {
    using namespace mbr;
    if (!r || r->kind != MBR_RANKER_LEARNED || !r->learned) MBR_FAIL(MBR_EINVAL, "not a learned ranker");
    if (!r->fallback) MBR_FAIL(MBR_EINVAL, "learned ranker without a fallback");
    if (!d_q || n == 0) MBR_FAIL(MBR_EINVAL, "no queries");
    if (reps < 1 || reps > 1000) MBR_FAIL(MBR_EINVAL, "reps=%d outside 1..1000", reps);
    hipStream_t s = as_stream(stream);
    LearnedModel &lm = *r->learned;
    const int32_t keep = lm.uses_window;
    DevBuf ranks;
    MBR_TRY(ranks.alloc(n * 4));
    hipEvent_t e0, e1;
    MBR_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        MBR_FAIL(MBR_EHIP, "hipEventCreate failed");
    }
    double t[2] = {0, 0};
    mbr_status st = MBR_OK;
    for (int path = 0; path < 2 && st == MBR_OK; ++path) {
        lm.uses_window = path == 0 ? 1 : 0;  // 0: window search, 1: fallback
        st = rank_learned_launch(r, d_q, n, ranks.as<uint32_t>(), s);
        if (st != MBR_OK) break;
        (void)hipEventRecord(e0, s);
        for (int i = 0; i < reps && st == MBR_OK; ++i) st = rank_learned_launch(r, d_q, n, ranks.as<uint32_t>(), s);
        (void)hipEventRecord(e1, s);
        float ms = 0;
        hipError_t he = hipEventSynchronize(e1);
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (st == MBR_OK && he != hipSuccess) {
            set_error("timing failed: %s", hipGetErrorString(he));
            st = MBR_EHIP;
        }
        t[path] = ms / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != MBR_OK) {
        lm.uses_window = keep;
        return st;
    }
    lm.uses_window = t[0] <= t[1] ? 1 : 0;
    if (ms_window) *ms_window = t[0];
    if (ms_fallback) *ms_fallback = t[1];
    return MBR_OK;
}

mbr_status mbr_learned_stats(const mbr_ranker *r, mbr_learned_info *info) {
    if (!r || r->kind != MBR_RANKER_LEARNED || !info) MBR_FAIL(MBR_EINVAL, "not a learned ranker");
    const LearnedModel &lm = *r->learned;
    info->n_leaves = lm.n_leaves;
    info->max_window = lm.e;
    info->mean_window = lm.mean_window;
    info->single_window_error = lm.e_single;
    info->uses_window = lm.uses_window;
    return MBR_OK;
}

mbr_status mbr_learned_params(const mbr_ranker *r, float *host_out, void *stream) {
    if (!r || r->kind != MBR_RANKER_LEARNED || !host_out) MBR_FAIL(MBR_EINVAL, "bad argument");
    hipStream_t s = mbr::as_stream(stream);
    MBR_HIP(hipMemcpyAsync(host_out, r->learned->wr.p, kParams * 4, hipMemcpyDeviceToHost, s));
    MBR_HIP(hipStreamSynchronize(s));
    return MBR_OK;
}

mbr_status mbr_mlp_forward(const float *d_params, const uint32_t *d_q, int32_t B, float *d_pred,
                           void *stream) {
    using namespace mbr;
    if (!d_params || !d_q || !d_pred) MBR_FAIL(MBR_EINVAL, "null pointer");
    if (B <= 0 || B % 64 != 0) MBR_FAIL(MBR_EINVAL, "B=%d must be a positive multiple of 64", B);
    hipStream_t s = as_stream(stream);
    // each workgroup rounds the fp32 parameters to bf16 as it loads them
    mlp_forward_kernel<float><<<grid_for((uint64_t)B, 256, 4096), 256, 0, s>>>(d_params, d_q, B, d_pred);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

mbr_status mbr_mlp_gradients(const float *d_params, const uint32_t *d_q, const float *d_tgt, int32_t B,
                             float *d_grad, float *d_loss, void *stream) {
    using namespace mbr;
    if (!d_params || !d_q || !d_tgt || !d_grad) MBR_FAIL(MBR_EINVAL, "null pointer");
    if (B <= 0 || B % 64 != 0) MBR_FAIL(MBR_EINVAL, "B=%d must be a positive multiple of 64", B);
    hipStream_t s = as_stream(stream);
    DevBuf wr, wb;
    MBR_TRY(wr.alloc(kParams * 4));
    MBR_TRY(wb.alloc(kParams * 2));
    mlp_round_kernel<<<(kParams + 255) / 256, 256, 0, s>>>(d_params, wr.as<float>(), wb.as<uint16_t>());
    TrainBufs T;
    MBR_TRY(T.alloc(B));
    MBR_TRY(batch_grad(T, wr.as<float>(), d_q, d_tgt, nullptr, 0, 0, 0, s));
    mlp_reduce_adam_kernel<<<(kParams + 255) / 256, 256, 0, s>>>(T.part.as<float>(), (B + kChunk - 1) / kChunk,
                                                                 d_grad, nullptr, nullptr, nullptr, nullptr,
                                                                 nullptr, 0.f, 1.f, 1.f, 0);
    if (d_loss) mlp_loss_kernel<<<1, 1, 0, s>>>(T.S.loss_part, B / 64, B, d_loss);
    MBR_HIP(hipGetLastError());
    MBR_HIP(hipStreamSynchronize(s));
    return MBR_OK;
}

mbr_status mbr_mlp_gradients_noalloc(const float *d_params, const uint32_t *d_q, const float *d_tgt, int32_t B,
                                     float *d_grad, float *d_loss, void *stream) {
    using namespace mbr;
    if (!d_params || !d_q || !d_tgt || !d_grad) MBR_FAIL(MBR_EINVAL, "null pointer");
    if (B <= 0 || B % 64 != 0) MBR_FAIL(MBR_EINVAL, "B=%d must be a positive multiple of 64", B);
    if (B > kStaticBatch)
        MBR_FAIL(MBR_ERANGE, "B=%d exceeds the %d samples of the static scratch", B, kStaticBatch);
    unsigned char *base = nullptr;
    MBR_TRY(static_scratch(&base));
    hipStream_t s = as_stream(stream);
    float *wr = reinterpret_cast<float *>(base + kStWr);
    uint16_t *wb = reinterpret_cast<uint16_t *>(base + kStWb);
    const TrainScratch S = carve(reinterpret_cast<float *>(base + kStAct), (size_t)B);
    float *part = reinterpret_cast<float *>(base + kStPart);
    // every scratch word the kernels read is written first in this call
    mlp_round_kernel<<<(kParams + 255) / 256, 256, 0, s>>>(d_params, wr, wb);
    mlp_fwd_bwd_kernel<<<(B + 63) / 64, 64, 0, s>>>(wr, B, d_q, d_tgt, nullptr, 0, 0, 0, S);
    mlp_grad_part_kernel<<<(B + kChunk - 1) / kChunk, 256, 0, s>>>(B, S, part);
    mlp_reduce_adam_kernel<<<(kParams + 255) / 256, 256, 0, s>>>(part, (B + kChunk - 1) / kChunk, d_grad, nullptr,
                                                                 nullptr, nullptr, nullptr, nullptr, 0.f, 1.f, 1.f,
                                                                 0);
    if (d_loss) mlp_loss_kernel<<<1, 1, 0, s>>>(S.loss_part, B / 64, B, d_loss);
    MBR_HIP(hipGetLastError());
    return MBR_OK;
}

}  // extern "C"
