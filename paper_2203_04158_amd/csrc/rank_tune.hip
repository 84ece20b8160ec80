// Rank-side autotuner: the chunk width k of a ranker kind for one sector, and
// the learned index's choice between its window search and its fallback.
//
// The best k depends on the sector and the machine (Sec. V.A finds R = 8
// fastest on its CPU for staggered lookup; on the GPU the answer moves with
// what fits LDS and how many dependent far reads a walk takes), so it is
// measured: every candidate is built, timed on the caller's own queries with
// HIP events on the caller's stream, and the fastest kept.  Host code only.
#include <algorithm>
#include <cstdlib>
#include <fstream>
#include <sstream>

#include "common.hpp"

namespace {

using namespace mbr;

// Particle number of a sector that is exactly C(M, N): one window over all M
// bits with lo == hi, no modular weight, not adopted from a list.  -1 otherwise.
int plain_particle_number(const mbr_sector *s) {
    if (s->from_list || s->modulus != 0 || s->cons.size() != 1) return -1;
    const mbr_popc_cons &c = s->cons[0];
    const uint64_t all = s->M >= 64 ? ~0ull : (1ull << s->M) - 1;
    if ((c.mask & all) != all || c.lo != c.hi) return -1;
    return c.lo;
}

std::string rank_key(const mbr_sector *s, int32_t kind) {
    hipDeviceProp_t p{};
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipGetDeviceProperties(&p, dev);
    std::ostringstream os;
    os << "rank;" << p.gcnArchName << ";cu" << p.multiProcessorCount << ";kind" << kind << ";M" << s->M << ";W"
       << s->width_bits << ";n" << s->n << ";C";
    for (auto &c : s->cons) os << std::hex << c.mask << std::dec << ":" << c.lo << "-" << c.hi << ",";
    os << ";mod" << s->modulus << "." << s->residue;
    for (int32_t w : s->weights) os << "," << w;
    std::string key = os.str();
    for (auto &ch : key)
        if (ch == ' ' || ch == '\t' || ch == '\n') ch = '_';
    return key;
}

mbr_status build_kind(const mbr_sector *s, int32_t kind, int32_t N, int32_t k, mbr_ranker **r, void *stream) {
    switch (kind) {
    case MBR_RANKER_STAGGERED:
        return mbr_build_staggered_tables(s->M, N, k, s->width_bits, r, stream);
    case MBR_RANKER_TRIE:
        return mbr_build_trie(s, k, r, stream);
    default:
        return mbr_build_bitmap_trie(s, k, r, stream);
    }
}

// Average time of `reps` launches after one untimed launch.
mbr_status time_ranker(const mbr_ranker *r, const void *q, uint64_t n, uint32_t *out, int32_t reps,
                       hipStream_t s, double *ms) {
    hipEvent_t e0, e1;
    MBR_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        MBR_FAIL(MBR_EHIP, "hipEventCreate failed");
    }
    mbr_status st = mbr_rank_batch(r, q, n, out, s);
    if (st == MBR_OK) {
        (void)hipEventRecord(e0, s);
        for (int i = 0; i < reps && st == MBR_OK; ++i) st = mbr_rank_batch(r, q, n, out, s);
        (void)hipEventRecord(e1, s);
    }
    hipError_t he = hipEventSynchronize(e1);
    float t = 0;
    if (st == MBR_OK && he == hipSuccess) he = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != MBR_OK) return st;
    if (he != hipSuccess) MBR_FAIL(MBR_EHIP, "timing failed: %s", hipGetErrorString(he));
    *ms = t / reps;
    return MBR_OK;
}

}  // namespace

extern "C" {

mbr_status mbr_rank_autotune(const mbr_sector *s, int32_t kind, const int32_t *ks, int32_t n_ks, const void *d_q,
                             uint64_t n, int32_t reps, mbr_rank_tuning *res, mbr_ranker **out, void *stream) {
    if (!out || !res) MBR_FAIL(MBR_EINVAL, "null output");
    *out = nullptr;
    if (!s) MBR_FAIL(MBR_EINVAL, "null sector");
    if (kind != MBR_RANKER_STAGGERED && kind != MBR_RANKER_TRIE && kind != MBR_RANKER_BITMAP_TRIE)
        MBR_FAIL(MBR_EINVAL, "kind=%d (staggered, trie or bitmap trie)", kind);
    if (!d_q || n == 0) MBR_FAIL(MBR_EINVAL, "no queries");
    if (reps < 1 || reps > 1000) MBR_FAIL(MBR_EINVAL, "reps=%d outside 1..1000", reps);
    if (n_ks < 0 || n_ks > 64 || (n_ks > 0 && !ks)) MBR_FAIL(MBR_EINVAL, "n_ks=%d", n_ks);
    if (s->n == 0) MBR_FAIL(MBR_EINVAL, "empty sector");
    const int32_t N = plain_particle_number(s);
    if (kind == MBR_RANKER_STAGGERED && N < 0)
        MBR_FAIL(MBR_EINVAL, "staggered tables rank C(M, N): the sector must be one fixed particle number");
    const int kmax = kind == MBR_RANKER_BITMAP_TRIE ? 8 : 16;
    std::vector<int32_t> cand;
    if (n_ks > 0) {
        cand.assign(ks, ks + n_ks);
    } else if (kind == MBR_RANKER_STAGGERED) {
        cand = {3, 4, 5, 6, 7, 8, 10, 12, 14, 16};
    } else if (kind == MBR_RANKER_TRIE) {
        cand = {4, 6, 8, 10, 12};
    } else {
        cand = {4, 5, 6, 7, 8};
    }
    for (int32_t k : cand)
        if (k < 1 || k > kmax) MBR_FAIL(MBR_EINVAL, "candidate k=%d outside 1..%d", k, kmax);
    // widths beyond M add nothing: one chunk already covers the pattern
    for (auto &k : cand) k = std::min(k, s->M);
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    hipStream_t hs = as_stream(stream);

    *res = mbr_rank_tuning{};
    res->kind = kind;
    const std::string key = s->from_list ? std::string() : rank_key(s, kind);
    const char *path = std::getenv("MBR_AUTOTUNE_CACHE");
    if (!key.empty() && path && *path) {
        std::ifstream in(path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string k0;
            int kk = 0;
            double ms = 0;
            if (!(ls >> k0 >> kk >> ms) || k0 != key) continue;
            if (kk < 1 || kk > kmax || !(ms >= 0)) continue;
            mbr_ranker *r = nullptr;
            if (build_kind(s, kind, N, kk, &r, stream) != MBR_OK) continue;
            res->k = kk;
            res->ms = ms;
            res->from_cache = 1;
            clear_error();
            *out = r;
            return MBR_OK;
        }
    }

    DevBuf ranks;
    MBR_TRY(ranks.alloc(n * 4));
    mbr_ranker *best = nullptr;
    double best_ms = 0;
    std::string first_err;
    mbr_status first_st = MBR_OK;
    for (int32_t k : cand) {
        mbr_ranker *r = nullptr;
        mbr_status st = build_kind(s, kind, N, k, &r, stream);
        double ms = 0;
        if (st == MBR_OK) st = time_ranker(r, d_q, n, ranks.as<uint32_t>(), reps, hs, &ms);
        if (st != MBR_OK) {
            // a candidate that cannot be built or run here (memory, table
            // size, ranks beyond 32 bits) is skipped
            if (first_st == MBR_OK) {
                first_st = st;
                first_err = mbr_last_error();
            }
            if (r) mbr_ranker_destroy(r);
            continue;
        }
        ++res->tried;
        if (!best || ms < best_ms) {
            if (best) mbr_ranker_destroy(best);
            best = r;
            best_ms = ms;
            res->k = k;
        } else {
            mbr_ranker_destroy(r);
        }
    }
    if (!best) {
        set_error("no candidate k could be built and timed (first failure: %s)", first_err.c_str());
        return first_st;
    }
    clear_error();
    res->ms = best_ms;
    if (!key.empty() && path && *path) {
        std::ofstream of(path, std::ios::app);
        if (of) of << key << " " << res->k << " " << best_ms << "\n";
    }
    *out = best;
    return MBR_OK;
}

}  // extern "C"
